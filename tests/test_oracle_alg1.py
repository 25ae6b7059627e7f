"""Pins of the oracle's Algorithm 1 bookkeeping, line search, contact share
of the stiffness estimate and CCD activation rule.

Every expected value here comes from a hand evaluation of the paper's
printed rule on a hand-built state (closed forms such as b(dhat/2, dhat) =
dhat^2 ln(2) / 4), from the defining optimisation problem solved by a
library minimiser, from eigenvalues computed by a library routine, or from
dense time scans of the geometry; none retypes the oracle's arithmetic.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import scenes
from oracle import (ALState, OracleScene, Pairs, Params, classify_ee, dual_update, line_search,
                    rebuild_aug_set, sigma_update, slack_update)

DH = 1e-3


def pairs_of(n):
    k = np.zeros(n, np.int64)
    return Pairs(k, np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64) + 100,
                 np.tile(np.arange(4, dtype=np.int64), (n, 1)) + 4 * np.arange(n)[:, None])


# ------------------------------------------------------------------ slack, mu, sigma
def test_slack_is_the_minimiser_of_the_slack_problem():
    """s_i minimises mu (dhat + s - d) + sigma/2 (dhat + s - d)^2 over s >= 0 (eq. problem-s)."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        mu = rng.uniform(0.0, 50.0)
        sigma = 10.0 ** rng.uniform(1, 6)
        d = rng.uniform(0.0, 4.0 * DH)
        f = lambda s: mu * (DH + s - d) + 0.5 * sigma * (DH + s - d) ** 2
        r = scipy.optimize.minimize_scalar(f, bounds=(0.0, 10.0 * DH), method="bounded",
                                           options=dict(xatol=1e-14))
        s_ref = r.x if f(r.x) < f(0.0) else 0.0
        s = float(slack_update(np.array([mu]), np.array([d]), sigma, DH)[0])
        assert s >= 0.0
        assert abs(s - s_ref) <= 1e-9 * DH + 1e-6 * s_ref, (mu, sigma, d, s, s_ref)


def test_dual_update_closed_forms():
    """Alg. 1 lines 12-14 by hand: s first, then mu += sigma b(d, dhat + s) with the new s.

    (a) mu = 0, d = dhat/2, sigma = 2: s = 0, mu' = 2 b(dhat/2, dhat) = dhat^2 ln(2) / 2.
    (b) mu = 3 sigma dhat, d = dhat/2, sigma = 5: s = 0, mu' = mu + 5 dhat^2 ln(2) / 4.
    (c) mu = 0.2 sigma dhat, d = 2 dhat, sigma = 7: s = 0.8 dhat, dhat + s = 1.8 dhat < d, mu' = mu.
    (d) mu = 0, d = dhat: s = 0 and b(dhat, dhat) = 0, mu' = 0.
    (e) mu = 0, d = dhat/4, sigma = 1: mu' = b(dhat/4, dhat) = (9/16) dhat^2 ln 4.
    """
    cases = [  # mu, d, sigma, s expected, mu expected
        (0.0, DH / 2, 2.0, 0.0, DH * DH * math.log(2.0) / 2.0),
        (3 * 5.0 * DH, DH / 2, 5.0, 0.0, 3 * 5.0 * DH + 5.0 * DH * DH * math.log(2.0) / 4.0),
        (0.2 * 7.0 * DH, 2 * DH, 7.0, 0.8 * DH, 0.2 * 7.0 * DH),
        (0.0, DH, 3.0, 0.0, 0.0),
        (0.0, DH / 4, 1.0, 0.0, 9.0 / 16.0 * DH * DH * math.log(4.0)),
    ]
    for mu, d, sigma, s_ex, mu_ex in cases:
        mu_new, s_new = dual_update(np.array([mu]), np.array([d]), sigma, DH)
        assert abs(s_new[0] - s_ex) <= 1e-15, (mu, d, sigma)
        assert abs(mu_new[0] - mu_ex) <= 1e-13 * max(abs(mu_ex), 1e-12), (mu, d, sigma, mu_new[0], mu_ex)


def test_sigma_growth_rule():
    """Alg. 1 lines 15-17: sigma <- max(1.2 sigma, 100 sigma^0) when min d < 1e-2 dhat (strict)."""
    assert sigma_update(1.0, 1.0, 0.5e-2 * DH, DH) == 100.0        # jump to 100 sigma^0
    assert sigma_update(200.0, 1.0, 0.5e-2 * DH, DH) == 240.0      # then x 1.2
    assert sigma_update(50.0, 1.0, 0.5e-2 * DH, DH) == 100.0
    assert sigma_update(7.0, 1.0, 2e-2 * DH, DH) == 7.0            # min d above the threshold
    assert sigma_update(7.0, 1.0, 1e-2 * DH, DH) == 7.0            # the threshold itself


def test_aug_set_rule():
    """Alg. 1 lines 3-6 (current vs previous iterate) on a hand-built sequence."""
    P = pairs_of(4)
    d = np.array([0.3e-2, 0.5e-2, 2e-2, 0.9]) * DH
    st = ALState(sigma=1.0, sigma0=1.0)
    # l = 0: min d = 0.3e-2 dhat < +inf -> A' = pairs with d < 1e-2 dhat = {0, 1}, mu = s = 0
    aug, mu, s = rebuild_aug_set(P, d, d.min(), np.inf, st, DH)
    assert list(aug.a) == [0, 1] and mu.tolist() == [0.0, 0.0] and s.tolist() == [0.0, 0.0]
    st.aug, st.mu, st.s = aug, np.array([4.0, 5.0]), np.array([1e-5, 2e-5])
    # min d increased and A' non-empty: A' unchanged
    d2 = np.array([0.4e-2, 0.2, 0.6e-2, 0.9]) * DH
    aug, mu, s = rebuild_aug_set(P, d2, d2.min(), d.min(), st, DH)
    assert list(aug.a) == [0, 1] and mu.tolist() == [4.0, 5.0]
    # min d decreased: rebuilt as {0, 2}; pair 0 keeps (mu, s), pair 2 starts at 0
    d3 = np.array([0.1e-2, 0.2, 0.6e-2, 0.9]) * DH
    aug, mu, s = rebuild_aug_set(P, d3, d3.min(), d.min(), st, DH)
    assert list(aug.a) == [0, 2] and mu.tolist() == [4.0, 0.0] and s.tolist() == [1e-5, 0.0]
    # min d above 1e-2 dhat: emptied
    d4 = np.array([2e-2, 0.2, 0.6, 0.9]) * DH
    aug, mu, s = rebuild_aug_set(P, d4, d4.min(), d3.min(), st, DH)
    assert len(aug) == 0 and mu.size == 0
    # A' empty and min d below the threshold though it increased: rebuilt
    st2 = ALState(sigma=1.0, sigma0=1.0)
    aug, mu, s = rebuild_aug_set(P, d2, d2.min(), d.min(), st2, DH)
    assert list(aug.a) == [0, 2]


# ---------------------------------------------------------------------- line search
def test_line_search_acceptance():
    """Halving from alpha_max until L <= L0 at a feasible point within capacity."""
    quad = lambda a: ((a - 0.3) ** 2 - 0.09, True, True)     # L <= 0 exactly on [0, 0.6]
    assert line_search(1.0, 0.0, quad) == 0.5
    assert line_search(0.6, 0.0, quad) == 0.6                  # equality accepted (non-increase)
    infeasible = lambda a: (-1.0, a <= 0.2, True)              # J <= 0 or d <= 0 beyond 0.2
    assert line_search(1.0, 0.0, infeasible) == 0.125
    capacity = lambda a: (-1.0, True, a <= 0.05)               # too many active pairs beyond 0.05
    assert line_search(1.0, 0.0, capacity) == 0.03125
    seen = []

    def never(a):
        seen.append(a)
        return 1.0, True, True
    assert line_search(0.75, 0.0, never, min_alpha=1e-9) == 0.0
    assert min(seen) >= 1e-9 and min(seen) < 2e-9
    assert len(seen) == math.floor(math.log2(0.75 / 1e-9)) + 1


# ----------------------------------------------------------- contact share of Lambda
def tet_above_plane(offset_xz, height):
    """One tet whose lowest vertex sits `height` above the y = 0 plane at (x, z) = offset_xz."""
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.05, 0.1], [0.1, 0.05, 0.0], [0.03, 0.12, 0.03]])
    X += np.array([offset_xz[0], height, offset_xz[1]])
    obs = np.array([[-1.0, 0.0, -1.0], [1.0, 0.0, -1.0], [1.0, 0.0, 1.0], [-1.0, 0.0, 1.0]])
    return scenes._pack(name="tet_plane", pos=X, tets=np.array([[0, 1, 2, 3]]), E=1e5, nu=0.4, rho=1000.0,
                        fixed=None, obs_pos=obs, obs_tris=np.array([[0, 2, 1], [0, 3, 2]], np.int32),
                        dt=1.0 / 30.0, dhat=DH, n_steps=1)


@pytest.mark.parametrize("where,k_expected", [((0.3, 0.2), 4), ((1.0004, 0.3), 3), ((1.0003, 1.0002), 2)])
def test_contact_contribution_to_lambda(where, k_expected):
    """Each active pair adds its stencil's mean clamped eigenvalue (over the 3k
    rows of the k nodes its distance depends on) to each of those rows: a
    node's e_j grows by 3 x that mean.  Checked with eigenvalues from a library
    eigensolver on the unprojected pair Hessian, for point-triangle (k = 4),
    point-edge (k = 3, vertex just past the plane's edge) and point-point
    (k = 2, just past its corner) cases."""
    sc = tet_above_plane(where, 4e-4)
    o = OracleScene(sc)
    x = o.x.copy()
    pairs = o.all_pairs()
    d, case = o.distances(x, pairs)
    act = np.nonzero(d < DH)[0]
    assert act.size >= 1
    st = ALState(sigma=2e3, sigma0=2e3)
    _, e_with = o.hessian(x, pairs, st, with_lambda=True)
    _, e_none = o.hessian(x, Pairs.empty(), ALState(sigma=2e3, sigma0=2e3), with_lambda=True)
    from oracle import CASE_NODES
    expect = np.zeros(o.N)
    ks = []
    for i in act:
        H = o.contact_hessians(x, pairs.take([i]), case[[i]], np.zeros(1), np.zeros(1), np.zeros(1, bool),
                               st.sigma, project=False)[0]
        nodes_local = CASE_NODES[int(case[i])]
        rows = np.concatenate([np.arange(3 * j, 3 * j + 3) for j in nodes_local])
        w = np.linalg.eigvalsh(H[np.ix_(rows, rows)])
        k = len(nodes_local)
        ks.append(k)
        mean = np.maximum(w, 0.0).sum() / (3 * k)
        for j in nodes_local:
            expect[pairs.nodes[i][j]] += 3.0 * mean
    assert k_expected in ks
    fi = o.free_idx
    got = e_with[fi] - e_none[fi]
    assert np.abs(got - expect[fi]).max() <= 1e-9 * np.abs(expect[fi]).max()
    assert expect[fi].max() > 0.0


# ------------------------------------------------------------------------ CCD rule
def pt_pair():
    return Pairs(np.array([0]), np.array([0]), np.array([0]), np.array([[0, 1, 2, 3]]))


def ee_pair():
    return Pairs(np.array([1]), np.array([0]), np.array([1]), np.array([[0, 1, 2, 3]]))


def ccd_scene(rule):
    sc = tet_above_plane((0.3, 0.2), 0.5)
    return OracleScene(sc, Params(ccd_rule=rule))


TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])


@pytest.mark.parametrize("delta,printed,half_gap", [(5e-4, 0.5, 1.0), (2e-3, 1.0, 1.0)])
def test_ccd_near_miss_activation(delta, printed, half_gap):
    """A vertex passes the triangle's plane at t = 1/2 a distance delta outside
    its edge x = 0 (point-edge case at the time of coplanarity, d_TOC = delta).
    The printed rule activates it when delta < dhat (tau = 1/2: point-edge
    cases keep tau); the half-gap departure does not, since the pair starts at
    d0 = sqrt(delta^2 + (2e-4)^2) and the margin d0 / 2 is below delta."""
    x = np.concatenate([np.array([[-delta, 2e-4, 0.5]]), TRI])
    p = np.zeros((4, 3))
    p[0, 1] = -4e-4
    for rule, want in (("printed", printed), ("half_gap", half_gap), ("literal", printed)):
        a = ccd_scene(rule).ccd(x, p, pt_pair())
        assert abs(a - want) <= 1e-12, (rule, a, want)


def test_ccd_root_at_start_frame():
    """A vertex that starts in the triangle's plane, 5e-4 outside its edge,
    and leaves it: the cubic's root at t = 0 is the start frame t0 under the
    printed reading (no bound) and a time of impact under the literal rule
    (alpha_max = 0)."""
    x = np.concatenate([np.array([[-5e-4, 0.0, 0.5]]), TRI])
    p = np.zeros((4, 3))
    p[0] = [-1e-4, 3e-4, 0.0]
    assert ccd_scene("printed").ccd(x, p, pt_pair()) == 1.0
    assert ccd_scene("literal").ccd(x, p, pt_pair()) <= 1e-12


def test_ccd_start_frame_coplanar_by_rounding():
    """A vertex left in the triangle's plane up to rounding (y = 0.1 * 3 - 0.3
    = 5.6e-17, 5e-4 outside the edge x = 0), leaving along a short direction
    (1e-9 m down): the cubic's root sits at t = 5.6e-8, far past eps, yet it is
    the start frame t0, since the start configuration is coplanar to within
    the rounding of its positions; the printed reading gives no bound there,
    the literal rule bounds the step at that root."""
    y0 = 0.1 * 3 - 0.3
    assert 0.0 < y0 < 1e-16
    x = np.concatenate([np.array([[-5e-4, y0, 0.5]]), TRI])
    p = np.zeros((4, 3))
    p[0, 1] = -1e-9
    assert ccd_scene("printed").ccd(x, p, pt_pair()) == 1.0
    a = ccd_scene("literal").ccd(x, p, pt_pair())
    assert abs(a - y0 / 1e-9) <= 1e-12 * (y0 / 1e-9)


def test_ccd_edge_edge_precedes_first_crossing():
    """alpha_max never exceeds the first time two edges pass through each
    other (dense time scan of the line-line signed distance with both
    segment parameters inside [0, 1]), and is positive for pairs that start
    farther apart than 1e-2 dhat."""
    rng = np.random.default_rng(21)
    hits = 0
    for trial in range(80):
        for rule in ("printed", "half_gap"):
            o = ccd_scene(rule)
            a0, a1 = rng.normal(size=3), rng.normal(size=3)
            mid = 0.5 * (a0 + a1) + rng.normal(size=3) * 0.3
            dirn = rng.normal(size=3)
            b0, b1 = mid - dirn, mid + dirn
            x = np.stack([a0, a1, b0, b1])
            P = rng.normal(size=(4, 3)) * 1.2
            amax = o.ccd(x, P, ee_pair())
            ts = np.linspace(0, 1, 20001)
            X = x[None] + ts[:, None, None] * P[None]
            e1, e2, w = X[:, 1] - X[:, 0], X[:, 3] - X[:, 2], X[:, 0] - X[:, 2]
            n = np.cross(e1, e2)
            sd = np.einsum("ij,ij->i", w, n)
            q, case = classify_ee(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
            inside = case == 7
            cross = np.nonzero((np.sign(sd[1:]) != np.sign(sd[:-1])) & inside[1:] & inside[:-1])[0]
            if cross.size:
                hits += 1
                assert amax <= ts[cross[0] + 1] + 1e-12, (trial, rule, amax, ts[cross[0] + 1])
            if math.sqrt(q[0]) > 1e-2 * DH:
                assert amax > 0.0
    assert hits > 10


def test_literal_rule_freezes_two_cubes_printed_reading_does_not():
    """Why the start-frame reading: on two stacked 3^3-cell cubes the second
    step of the literal rule lands an iterate on a point-edge time of
    coplanarity inside dhat; every later CCD bound of that pair is 0 and the
    step stalls unconverged.  The printed margin with the root at t = 0 read
    as the start frame converges."""
    sc = scenes.stacked_boxes(n_cubes=2, cells=3, seed=0, n_steps=2)
    res = {}
    for rule in ("literal", "printed"):
        o = OracleScene(sc, Params(newton_rtol=1e-5, max_newton=300, ccd_rule=rule))
        o.step()
        tr = []
        st = o.step(trace=tr)
        res[rule] = (st["converged"], sum(1 for t in tr if t["alpha_max"] == 0.0))
    print(res)
    assert res["literal"][0] is False and res["literal"][1] >= 1
    assert res["printed"][0] is True and res["printed"][1] == 0
