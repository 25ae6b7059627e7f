"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Kernel-level checks evaluate both sides at the same iterate and state;
step-level checks run both through whole time steps.  Tolerances:
FP64 kernels 1e-9 relative (rounding of different but exact algorithms),
FP64 trajectories 1e-6 of the bounding-box diagonal, mixed precision 1e-4.
"""
import numpy as np
import pytest

import scenes
from oracle import ALState, OracleScene, Pairs, Params

pytestmark = pytest.mark.gpu


def lib_scene(sc, **kw):
    from paper_2407_00046_amd import Scene
    return Scene(sc, **kw)


def contact_state(sc, depth=4e-4, seed=7, every=3):
    """Cube pressed to `depth` above the plane with a hand-made augmentation set."""
    o = OracleScene(sc)
    x = o.x.copy()
    x[: o.n_body, 1] -= x[: o.n_body, 1].min() - depth
    rng = np.random.default_rng(seed)
    x[: o.n_body] += rng.uniform(-2e-5, 2e-5, size=(o.n_body, 3))
    pairs = o.all_pairs()
    d, _ = o.distances(x, pairs)
    act = np.nonzero(d < o.dhat)[0]
    aug = pairs.take(act[::every])
    st = ALState(sigma=3e4, sigma0=3e4, aug=aug, mu=rng.uniform(0, 50, len(aug)), s=rng.uniform(0, 2e-4, len(aug)))
    y = o.predictor(o.x, o.v)
    return o, x, y, pairs, st


def map_aug(g, aug: Pairs):
    """Oracle pairs -> (kind, library primitive ids)."""
    sv, st, se = g.surface()
    vpos = {int(v): i for i, v in enumerate(sv)}
    tpos = {tuple(sorted(map(int, t))): i for i, t in enumerate(st)}
    epos = {tuple(sorted(map(int, e))): i for i, e in enumerate(se)}
    kind = aug.kind.astype(np.int32)
    prims = np.zeros((len(aug), 2), np.int32)
    for j in range(len(aug)):
        nd = aug.nodes[j]
        if aug.kind[j] == 0:
            prims[j] = (vpos[int(nd[0])], tpos[tuple(sorted(map(int, nd[1:])))])
        else:
            prims[j] = (epos[tuple(sorted(map(int, nd[:2])))], epos[tuple(sorted(map(int, nd[2:])))])
    return kind, prims


def free_rows(o, a):
    return a[o.free_idx].reshape(-1)


@pytest.fixture(scope="module")
def contact_case():
    sc = scenes.tiny_cube()
    o, x, y, pairs, st = contact_state(sc)
    return sc, o, x, y, pairs, st


@pytest.mark.parametrize("project", [True, False])
def test_linearize_energy_gradient_hessian(contact_case, project):
    sc, o, x, y, pairs, st = contact_case
    g = lib_scene(sc)
    kind, prims = map_aug(g, st.aug)
    E, grad, nact = g.linearize(x, st.sigma, kind, prims, st.mu, st.s, project=project)
    L, gref = o.lagrangian(x, y, pairs, st, with_grad=True)
    d, _ = o.distances(x, pairs)
    print(f"pairs active {nact} (oracle {(d < o.dhat).sum()}), |A'| = {len(st.aug)}, E = {E:.12e} vs {L:.12e}")
    assert nact == int((d < o.dhat).sum())
    assert abs(E - L) <= 1e-10 * abs(L)
    gf, rf = free_rows(o, grad), free_rows(o, gref)
    assert np.abs(gf - rf).max() <= 1e-9 * np.abs(rf).max()
    H = o.hessian(x, pairs, st, project=project)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.normal(size=(o.N, 3))
        hv = H @ free_rows(o, v)
        lv = free_rows(o, g.hessian_apply(v))
        assert np.linalg.norm(lv - hv) <= 1e-9 * np.linalg.norm(hv)


def test_element_projection_at_a_crushed_twisted_state():
    """Projected element Hessians where the projection matters: the cube
    squashed to 55% of its height, twisted by 40 degrees about its vertical
    axis and sheared, so that many element Hessians have clearly negative
    eigenvalues (counted on the oracle's 12x12 blocks).  The library's
    projection (9x9 reduced eigenproblem per element) must give the oracle's
    assembled projected H v (12x12 eigendecomposition per element), and the
    unprojected one must differ from it."""
    sc = scenes.tiny_cube()
    o = OracleScene(sc)
    x = o.x.copy()
    nb = o.n_body
    c = x[:nb].mean(0)
    r = x[:nb] - c
    h = (r[:, 1] - r[:, 1].min()) / np.ptp(r[:, 1])
    ang = np.deg2rad(40.0) * h
    xr = np.cos(ang) * r[:, 0] - np.sin(ang) * r[:, 2]
    zr = np.sin(ang) * r[:, 0] + np.cos(ang) * r[:, 2]
    x[:nb] = c + np.stack([xr + 0.08 * h, 0.55 * r[:, 1], zr], axis=1)
    x[:nb, 1] += 0.05 - x[:nb, 1].min()   # keep clear of the plane: elements only
    tets = o.tets
    e = x[tets[:, 1:]] - x[tets[:, :1]]
    assert np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])).min() > 0.0
    He = o.element_hessians(x, False)
    lam_min = np.linalg.eigvalsh(He).min(axis=1) / np.abs(np.linalg.eigvalsh(He)).max(axis=1)
    n_neg = int((lam_min < -1e-3).sum())
    print(f"elements with an eigenvalue below -1e-3 of their largest: {n_neg} of {len(tets)}")
    assert n_neg >= len(tets) // 10
    g = lib_scene(sc)
    pairs = o.all_pairs()
    st = ALState()
    rng = np.random.default_rng(8)
    for project in (True, False):
        g.linearize(x, 0.0, project=project)
        H = o.hessian(x, pairs, st, project=project)
        for _ in range(3):
            v = rng.normal(size=(o.N, 3))
            hv = H @ free_rows(o, v)
            lv = free_rows(o, g.hessian_apply(v))
            assert np.linalg.norm(lv - hv) <= 1e-9 * np.linalg.norm(hv)
    Hp = o.hessian(x, pairs, st, project=True)
    Hu = o.hessian(x, pairs, st, project=False)
    assert abs(Hp - Hu).max() > 1e-3 * abs(Hu).max()


def test_stiffness_groups(contact_case):
    sc, o, x, y, pairs, st = contact_case
    g = lib_scene(sc)
    kind, prims = map_aug(g, st.aug)
    g.linearize(x, st.sigma, kind, prims, st.mu, st.s)
    e, grp = g.stiffness()
    _, eref = o.hessian(x, pairs, st, with_lambda=True)
    fi = o.free_idx
    assert np.abs(e[fi] - eref[fi]).max() <= 1e-9 * eref[fi].max()
    lg = np.log10(eref[fi])
    clear = np.abs(lg - np.round(lg)) > 1e-9
    assert (grp[fi][clear] == np.floor(lg[clear]).astype(int)).all()
    assert np.unique(grp[fi]).size >= 2


def test_pcg_and_warm_start_against_direct_solves(contact_case):
    sc, o, x, y, pairs, st = contact_case
    g = lib_scene(sc)
    kind, prims = map_aug(g, st.aug)
    g.linearize(x, st.sigma, kind, prims, st.mu, st.s)
    H, eref = o.hessian(x, pairs, st, with_lambda=True)
    rng = np.random.default_rng(4)
    b = rng.normal(size=(o.N, 3))
    z, it, rel = g.solve(b, mode=0, rtol=1e-13, max_iters=20000)
    zref = o.solve(H, free_rows(o, b))
    print(f"global PCG: {it} iterations, rel residual {rel:.2e}")
    assert np.linalg.norm(free_rows(o, z) - zref) <= 1e-8 * np.linalg.norm(zref)
    groups = o.stiffness_groups(eref[o.free_idx])
    zw, itw, _ = g.solve(b, mode=1, rtol=1e-14, max_iters=20000)
    zwref = o.groupwise_solve(H, free_rows(o, b), groups)
    print(f"warm start: {itw} iterations")
    assert np.linalg.norm(free_rows(o, zw) - zwref) <= 1e-7 * np.linalg.norm(zwref)
    z2, it2, rel2 = g.solve(b, mode=2, rtol=1e-13, max_iters=20000)
    assert np.linalg.norm(free_rows(o, z2) - zref) <= 1e-8 * np.linalg.norm(zref)


def test_candidates_cover_active_pairs(contact_case):
    sc, o, x, y, pairs, st = contact_case
    g = lib_scene(sc)
    kind, nodes, dist = g.candidates(x)
    d, _ = o.distances(x, pairs)
    act = np.nonzero(d < o.dhat)[0]

    def key(k, nd):
        nd = list(map(int, nd))
        return (int(k), nd[0], tuple(sorted(nd[1:]))) if k == 0 else \
            (int(k), tuple(sorted([tuple(sorted(nd[:2])), tuple(sorted(nd[2:]))])))
    got = {key(k, nd): dd for k, nd, dd in zip(kind, nodes, dist)}
    for i in act:
        kk = key(pairs.kind[i], pairs.nodes[i])
        assert kk in got
        assert abs(got[kk] - d[i]) <= 1e-12 * max(1.0, d[i]) + 1e-15
    # swept pass along a displacement covers every pair the oracle finds within dhat along the path
    rng = np.random.default_rng(5)
    p = np.zeros_like(x)
    p[: o.n_body] = rng.normal(scale=2e-3, size=(o.n_body, 3))
    kind2, nodes2, _ = g.candidates(x, p)
    got2 = {key(k, nd) for k, nd in zip(kind2, nodes2)}
    for t in np.linspace(0, 1, 5):
        dt, _ = o.distances(x + t * p, pairs)
        for i in np.nonzero(dt < o.dhat)[0]:
            assert key(pairs.kind[i], pairs.nodes[i]) in got2


def box_overlap_candidates(x, p, sv, st, se, free, n_body, dhat):
    """The candidate set by its definition, brute force: every point-triangle
    and edge-edge pair of surface primitives with no shared vertex, some free
    vertex and not both on obstacles, whose boxes over [x, x + p] overlap once
    one of the two is inflated by dhat (the same FP64 operations as the
    library's box test, so the set is exact)."""
    e = x if p is None else x + p
    lo_v, hi_v = np.minimum(x, e), np.maximum(x, e)

    def boxes(prims, infl):
        return lo_v[prims].min(axis=1) - infl, hi_v[prims].max(axis=1) + infl

    out = set()
    # point-triangle: vertex box against the inflated triangle box
    vlo, vhi = boxes(sv[:, None], 0.0)
    tlo, thi = boxes(st, dhat)
    ov = np.all((tlo[None] <= vhi[:, None]) & (vlo[:, None] <= thi[None]), axis=2)
    for i, j in zip(*np.nonzero(ov)):
        v, tri = int(sv[i]), tuple(sorted(map(int, st[j])))
        if v in tri or not (free[v] or any(free[t] for t in tri)) or (v >= n_body and tri[0] >= n_body):
            continue
        out.add((0, v, tri))
    # edge-edge: first edge's box against the second's inflated box
    alo, ahi = boxes(se, 0.0)
    blo, bhi = boxes(se, dhat)
    ov = np.all((blo[None] <= ahi[:, None]) & (alo[:, None] <= bhi[None]), axis=2)
    for i, j in zip(*np.nonzero(np.triu(ov, 1))):
        a, b = tuple(sorted(map(int, se[i]))), tuple(sorted(map(int, se[j])))
        if set(a) & set(b) or not any(free[v] for v in a + b) or (min(a) >= n_body and min(b) >= n_body):
            continue
        out.add((1, tuple(sorted([a, b]))))
    return out


def candidate_keys(kind, nodes):
    keys = []
    for k, nd in zip(kind, nodes):
        nd = list(map(int, nd))
        keys.append((0, nd[0], tuple(sorted(nd[1:]))) if k == 0 else
                    (1, tuple(sorted([tuple(sorted(nd[:2])), tuple(sorted(nd[2:]))]))))
    return keys


@pytest.mark.parametrize("broad", ["hash", "lbvh"])
@pytest.mark.parametrize("case", ["tiny_cube", "two_boxes"])
def test_candidates_equal_box_overlap_set(case, broad):
    """Either broad phase (spatial hash, or the paper's LBVH) returns exactly
    the box-overlap candidate set, each pair once, at rest and along swept
    displacements.  At rest every hash query lane finds a few partners and
    the keys it keeps in its slots are compacted into place; the 6 cm sweep
    spans whole cubes, so lanes find more partners than their slots hold and
    the pass traverses a second time to write them."""
    if case == "tiny_cube":
        sc = scenes.tiny_cube()
        o, x, _, _, _ = contact_state(sc)
        x = np.concatenate([x[: o.n_body], np.asarray(sc["obs_pos"]).reshape(-1, 3)])
    else:
        sc = scenes.stacked_boxes(n_cubes=2, cells=6, seed=0)
        x = np.concatenate([sc["x0"], np.asarray(sc["obs_pos"]).reshape(-1, 3)])
    nb = sc["rest_pos"].shape[0]
    g = lib_scene(sc, broad_phase=broad)
    sv, st, se = g.surface()
    free = np.concatenate([sc["fixed"] == 0, np.zeros(x.shape[0] - nb, bool)])
    rng = np.random.default_rng(9)
    for scale in (0.0, 2e-3, 2e-2, 6e-2):
        p = None
        if scale > 0:
            p = np.zeros_like(x)
            p[:nb] = rng.normal(scale=scale, size=(nb, 3))
            p[:nb, 1] -= scale
        kind, nodes, _ = g.candidates(x, p)
        got = candidate_keys(kind, nodes)
        ref = box_overlap_candidates(x, p, sv, st, se, free, nb, sc["dhat"])
        print(f"{case} sweep {scale}: {len(got)} candidates, {len(ref)} by definition")
        assert len(set(got)) == len(got)
        assert set(got) == ref


def test_ccd_bound(contact_case):
    sc, o, x, y, pairs, st = contact_case
    g = lib_scene(sc)
    rng = np.random.default_rng(6)
    for trial in range(4):
        p = np.zeros_like(x)
        p[: o.n_body, 1] = -1.5e-3 * (1 + trial)
        p[: o.n_body] += rng.normal(scale=3e-4, size=(o.n_body, 3))
        a_gpu = g.ccd_bound(x, p)
        a_ora = o.ccd(x, p, pairs)
        print(f"trial {trial}: alpha_max gpu {a_gpu:.15f} oracle {a_ora:.15f}")
        assert abs(a_gpu - a_ora) <= 1e-9


def first_divergence(gt, tr, dhat, e0, rtol=1e-6, e_rtol=1e-6, newton_rtol=None, state_err=0.0):
    """First Newton iteration where the GPU trace row and the oracle trace
    entry disagree, or None.  |A|, |A'| must agree exactly; sigma, min d,
    alpha_max and alpha to rtol relative (widened to 1e3 x the relative
    position difference the step started from, state_err; min d also to
    1e-6 dhat absolute); |e| to e_rtol relative.  The library's PCG stops at
    1e-12 of the residual where the oracle solves exactly, and the barrier's
    conditioning (up to ~1e6 here) carries that difference into the next
    iterates, so the real-valued decisions agree to ~1e-6 rather than to the
    1e-8 of two exact solves (measured: a time of coplanarity 21 iterations
    into a step, 2.6e-8 apart).  The iteration counts must agree, except that
    a step whose convergence test is decided near its threshold (the last
    common |e| within a factor 10 of it: with friction frames updated per
    iteration the last iterations contract linearly) may take one iteration
    more on one side (newton_rtol given).  The step length of the last
    (converged) iteration, and of iterations whose |e| is within 100x of the
    Newton threshold, is not compared: its line search weighs energy changes
    at the rounding level of L, where either halving is a correct outcome,
    and its step is below the Newton tolerance."""
    rt = max(rtol, 1e3 * state_err)
    n = min(len(gt), len(tr))
    if len(gt) != len(tr):
        thr = None if newton_rtol is None else newton_rtol * e0
        e_last = [r[6] for r in gt[n - 1:]] + [t["enorm"] for t in tr[n - 1:]]
        if thr is None or abs(len(gt) - len(tr)) > 1 or not any(0.1 * thr <= e <= 10.0 * thr for e in e_last):
            return f"iteration counts differ: gpu {len(gt)}, oracle {len(tr)}"
        n -= 1
    for i, (r, t) in enumerate(zip(gt[:n], tr[:n])):
        if int(r[0]) != t["n_active"] or int(r[1]) != t["n_aug"]:
            return f"iteration {i}: |A|, |A'| gpu {int(r[0])}, {int(r[1])} oracle {t['n_active']}, {t['n_aug']}"
        reals = [("sigma", r[2], t["sigma"] or 0.0, 0.0), ("min d", r[3], min(t["min_d"], dhat), 1e-6 * dhat),
                 ("alpha_max", r[4], t["alpha_max"], 0.0)]
        # a step length is a rounding-level decision once |e| is within 100x of
        # the Newton threshold (the energy decrease is then ~1e-16 of L)
        near_floor = newton_rtol is not None and max(r[6], t["enorm"]) <= 100.0 * newton_rtol * e0
        if i + 1 < len(gt) and not near_floor:
            reals.append(("alpha", r[5], t["alpha"], 0.0))
        for name, a, b, floor in reals:
            if abs(a - b) > rt * max(abs(a), abs(b)) + floor:
                return f"iteration {i}: {name} gpu {a!r} oracle {b!r}"
        if abs(r[6] - t["enorm"]) > e_rtol * max(e0, abs(r[6]), abs(t["enorm"])):
            return f"iteration {i}: |e| gpu {r[6]!r} oracle {t['enorm']!r}"
    return None


def run_both(sc, n_steps, precision="fp64", newton_rtol=1e-7, pcg_rtol=1e-12, check_trace=True, **kw):
    """Steps the library and the oracle side by side from the same state.  Both
    must converge; with check_trace the per-iteration decision traces must
    agree (integers exactly, reals to 1e-6, see first_divergence).  Returns eps_x per step and the
    largest |A'| seen."""
    g = lib_scene(sc, precision=precision, newton_rtol=newton_rtol, pcg_rtol=pcg_rtol, max_newton=200, **kw)
    o = OracleScene(sc, Params(newton_rtol=newton_rtol, max_newton=200, use_al=kw.get("use_al", True),
                               sigma_fixed=kw.get("sigma_fixed", 0.0),
                               ccd_rule=kw.get("ccd_rule", "printed")))
    n = sc["rest_pos"].shape[0]
    L = np.linalg.norm(sc["x0"].max(0) - sc["x0"].min(0))
    errs, aug_max = [], 0
    err = 0.0
    for k in range(n_steps):
        err_prev = err
        st = g.step(allow=(0, -7))
        tr = []
        so = o.step(trace=tr)
        xg, vg = g.get_state()
        err = np.linalg.norm(xg - o.x[:n], axis=1).max() / L
        gt = g.trace()
        print(f"step {k}: gpu status {st['status']} iters {st['newton_iters']} pcg {st['pcg_iters']} | "
              f"oracle iters {len(tr)} converged {so['converged']} | eps_x {err:.3e}")
        print("   gpu   |A| |A'| alpha |e|:", [(int(r[0]), int(r[1]), round(r[5], 6), float(f"{r[6]:.3e}")) for r in gt])
        print("   oracle|A| |A'| alpha |e|:", [(t['n_active'], t['n_aug'], round(t['alpha'], 6), float(f"{t['enorm']:.3e}")) for t in tr])
        assert st["converged"] == 1 and so["converged"], (st["status"], so["converged"])
        if check_trace:
            div = first_divergence(gt, tr, sc["dhat"], tr[0]["enorm"], newton_rtol=newton_rtol, state_err=err_prev)
            assert div is None, f"step {k}: {div}"
        aug_max = max(aug_max, max((t["n_aug"] for t in tr), default=0))
        errs.append(err)
    return errs, aug_max


def test_tiny_cube_steps_fp64():
    errs, _ = run_both(scenes.tiny_cube(), 3)
    assert max(errs) <= 1e-6


def test_tiny_cube_steps_fixed_sigma_plain_barrier():
    """The differentiable-rollout configuration: sigma held fixed, no A'."""
    errs, _ = run_both(scenes.tiny_cube(), 3, use_al=False, sigma_fixed=1e3)
    assert max(errs) <= 1e-6


def test_tiny_cube_steps_mixed():
    """Mixed precision against the FP64 oracle: the FP32 products change the
    PCG iterates, so the decision traces are not compared, only positions."""
    errs, _ = run_both(scenes.tiny_cube(), 3, precision="mixed", newton_rtol=1e-6, pcg_rtol=1e-6, check_trace=False)
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tiny_cube_steps_production_tolerance(precision):
    """Newton and PCG tolerances of the paper (1e-4, Alg. 1 and App. B) on the
    library, against the lockstep oracle (1e-7): the positions differ by the
    Newton stopping error, estimated at ~1e-4 (g + v/h) h^2 / L of the scene
    size, so the bound is the mixed-precision target, 1e-4."""
    sc = scenes.tiny_cube()
    g = lib_scene(sc, precision=precision, newton_rtol=1e-4, pcg_rtol=1e-4)
    o = OracleScene(sc, Params(newton_rtol=1e-7, max_newton=200))
    n = sc["rest_pos"].shape[0]
    L = np.linalg.norm(sc["x0"].max(0) - sc["x0"].min(0))
    for k in range(3):
        st = g.step()
        o.step()
        xg, _ = g.get_state()
        err = np.linalg.norm(xg - o.x[:n], axis=1).max() / L
        print(f"step {k}: {st['newton_iters']} Newton, {st['pcg_iters']} PCG iterations, eps_x {err:.3e}")
        assert st["converged"] == 1
        assert err <= 1e-4


def test_small_stacked_boxes_fp64():
    sc = scenes.stacked_boxes(n_cubes=2, cells=3, seed=0, n_steps=2)
    errs, _ = run_both(sc, 2, newton_rtol=1e-5)
    assert max(errs) <= 1e-6


def test_small_stacked_boxes_no_warm_start():
    """The warm-start ablation (plain block-Jacobi PCG from zero) takes the
    same decisions: with exact-enough solves the direction does not depend on
    the initial guess."""
    sc = scenes.stacked_boxes(n_cubes=2, cells=3, seed=0, n_steps=2)
    errs, _ = run_both(sc, 2, newton_rtol=1e-5, warm_start=False)
    assert max(errs) <= 1e-6


def test_augmented_set_lockstep():
    """The augmentation machinery over many iterations: with sigma held at 30
    the resting cube's barrier lets pairs come within 1e-2 dhat, so A' holds
    10-36 pairs through the second step while the multipliers and slacks are
    updated every iteration (Alg. 1 lines 3-6 and 12-14).  That step does not
    reach the gradient test quickly (a fixed sigma makes the dual ascent
    slow), so both sides stop at a 40-iteration cap; their traces (|A|, |A'|
    exactly, reals as in first_divergence) and end positions must agree."""
    sc = scenes.tiny_cube()
    kw = dict(newton_rtol=1e-7, max_newton=40, sigma_fixed=30.0)
    g = lib_scene(sc, pcg_rtol=1e-12, **kw)
    o = OracleScene(sc, Params(**kw))
    n = sc["rest_pos"].shape[0]
    L = np.linalg.norm(sc["x0"].max(0) - sc["x0"].min(0))
    err = 0.0
    for k in range(2):
        err_prev = err
        st = g.step(allow=(0, -7))
        tr = []
        so = o.step(trace=tr)
        xg, _ = g.get_state()
        err = np.linalg.norm(xg - o.x[:n], axis=1).max() / L
        augs = [t["n_aug"] for t in tr]
        print(f"step {k}: gpu status {st['status']} iters {st['newton_iters']} | oracle iters {len(tr)} "
              f"converged {so['converged']} | max |A'| {max(augs)}, iterations with |A'| > 1: "
              f"{sum(a > 1 for a in augs)} | eps_x {err:.3e}")
        assert (st["status"] == 0) == bool(so["converged"])
        div = first_divergence(g.trace(), tr, sc["dhat"], tr[0]["enorm"], state_err=err_prev)
        assert div is None, f"step {k}: {div}"
        assert err <= 1e-6
    assert max(augs) >= 10 and sum(a > 1 for a in augs) >= 20


def test_lbvh_steps_equal_hash_steps():
    """Both broad phases hand the step the same sorted candidate lists, so a
    rollout with the LBVH takes bitwise the hash's steps."""
    sc = scenes.stacked_boxes(n_cubes=2, cells=4, seed=0, n_steps=3)
    runs = []
    for broad in ("hash", "lbvh"):
        g = lib_scene(sc, broad_phase=broad, newton_rtol=1e-6, pcg_rtol=1e-6)
        stats = [g.step(allow=(0, -7)) for _ in range(3)]
        x, v = g.get_state()
        g.close()
        runs.append((x, [(s["newton_iters"], s["pcg_iters"], s["n_active_max"]) for s in stats]))
    print("iterations per step:", runs[0][1])
    assert runs[0][1] == runs[1][1]
    assert np.array_equal(runs[0][0], runs[1][0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_steps_are_bitwise_repeatable(precision):
    """Two scenes built from the same inputs take bitwise the same steps: every
    reduction sums in a fixed order and the candidate lists are sorted, so a
    checkpointed rollout recomputes exactly the trajectory it stored."""
    sc = scenes.stacked_boxes(n_cubes=2, cells=4, seed=0, n_steps=3)
    runs = []
    for _ in range(2):
        g = lib_scene(sc, precision=precision, newton_rtol=1e-6, pcg_rtol=1e-6)
        stats = [g.step(allow=(0, -7)) for _ in range(3)]
        x, v = g.get_state()
        g.close()
        runs.append((x, v, [(s["newton_iters"], s["pcg_iters"], s["warm_iters"]) for s in stats]))
    (x0, v0, s0), (x1, v1, s1) = runs
    print(f"{precision}: iterations per step {s0}")
    assert s0 == s1
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
