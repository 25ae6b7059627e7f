"""The CCD step bound over caller-given pairs, through the C ABI: the entry
point that allocates nothing (bal_pairs_ccd_bound_noalloc, file-scope device
scratch) against the one that allocates its partials (bal_pairs_ccd_bound),
and both against the oracle's CCD over the same pairs (Sec. 5.3)."""
import ctypes as C

import numpy as np
import pytest

import scenes
from oracle import OracleScene
from oracle.bal_oracle import Pairs

pytestmark = pytest.mark.gpu


def swept_pairs(seed):
    """Swept candidate pairs of the tiny cube pressed to 0.4 mm above its plane
    (inside dhat), along a downward displacement with noise."""
    from paper_2407_00046_amd import Scene
    sc = scenes.tiny_cube()
    o = OracleScene(sc)
    x = o.x.copy()
    x[: o.n_body, 1] -= x[: o.n_body, 1].min() - 4e-4
    rng = np.random.default_rng(seed)
    p = np.zeros_like(x)
    p[: o.n_body, 1] = -1.5e-3
    p[: o.n_body] += rng.normal(scale=3e-4, size=(o.n_body, 3))
    g = Scene(sc)
    kind, nodes, _ = g.candidates(x, p)
    g.close()
    return o, x, p, kind.astype(np.int32), nodes.astype(np.int32)


def entry(name):
    from paper_2407_00046_amd import bal
    return getattr(bal, name)


def call(fn, x, p, kind, nodes, n, dhat, rule=0):
    import torch
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    ptr = lambda t: C.c_void_p(t.data_ptr())
    st = torch.cuda.current_stream().cuda_stream
    rc = fn(0, ptr(x), ptr(p), int(x.shape[0]), ptr(kind), ptr(nodes), int(n), float(dhat), int(rule), ptr(out),
            C.c_void_p(st))
    torch.cuda.synchronize()
    return rc, float(out.item())


def test_no_alloc_matches_allocating_and_oracle():
    import torch
    from paper_2407_00046_amd import bal
    o, x, p, kind, nodes = swept_pairs(6)
    dev = lambda a: torch.tensor(a, device="cuda")
    xd, pd, kd, nd = dev(x), dev(p), dev(kind), dev(nodes)
    n = len(kind)
    assert n > 100
    # two calls in a row, the second on fewer pairs (a prefix, so its partials cover fewer blocks)
    for m in (n, n // 3):
        rc1, a_alloc = call(entry('bal_pairs_ccd_bound'), xd, pd, kd, nd, m, o.dhat)
        rc2, a_none = call(entry('bal_pairs_ccd_bound_noalloc'), xd, pd, kd, nd, m, o.dhat)
        assert rc1 == 0 and rc2 == 0
        pr = Pairs(kind[:m].astype(np.int64), np.zeros(m, np.int64), np.zeros(m, np.int64),
                   nodes[:m].astype(np.int64))
        a_ora = o.ccd(x, p, pr)
        print(f"{m} pairs: alpha_max allocating {a_alloc!r}, no-alloc {a_none!r}, oracle {a_ora!r}")
        assert a_none == a_alloc
        assert abs(a_none - a_ora) <= 1e-9
        assert a_none < 1.0
    # no pairs: alpha_max = 1
    assert call(entry('bal_pairs_ccd_bound_noalloc'), xd, pd, kd, nd, 0, o.dhat) == (0, 1.0)


def test_no_alloc_limits_and_bad_indices():
    import torch
    from paper_2407_00046_amd import bal
    o, x, p, kind, nodes = swept_pairs(7)
    dev = lambda a: torch.tensor(a, device="cuda")
    xd, pd, kd = dev(x), dev(p), dev(kind)
    bad = nodes.copy()
    bad[len(bad) // 2, 2] = x.shape[0]  # one node index past the vertex array
    bd = dev(bad)
    for fn in (entry('bal_pairs_ccd_bound'), entry('bal_pairs_ccd_bound_noalloc')):
        rc, a = call(fn, xd, pd, kd, bd, len(bad), o.dhat)
        assert rc == 0 and np.isnan(a)
        assert call(fn, xd, pd, kd, bd, 10, -1.0)[0] == bal.BAL_E_INVALID_ARG
    # beyond the scratch's 2^26 pairs: refused before any GPU work
    rc, _ = call(entry('bal_pairs_ccd_bound_noalloc'), xd, pd, kd, bd, (1 << 26) + 1, o.dhat)
    assert rc == bal.BAL_E_CAPACITY
