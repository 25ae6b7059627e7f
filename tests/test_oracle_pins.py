"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each test checks the oracle against something other than itself: closed
forms, textbook special cases, invariants, brute force on tiny inputs,
independent library routines, or the worked closed form of a contact-free
backward-Euler step.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import torch

import scenes
from oracle import (ALState, OracleScene, Pairs, barrier_np, barrier_torch, classify_ee, classify_pt,
                    lame, nh_density_torch, project_psd)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DT = torch.float64


def rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


# ---------------------------------------------------------------- Neo-Hookean
def test_nh_zero_energy_and_stress_at_rest():
    F = torch.eye(3, dtype=DT, requires_grad=True)
    psi = nh_density_torch(F, torch.tensor(3e5, dtype=DT), torch.tensor(7e5, dtype=DT))
    psi.backward()
    assert abs(float(psi)) < 1e-9
    assert float(F.grad.abs().max()) < 1e-9


def test_nh_rotation_invariance():
    rng = np.random.default_rng(0)
    for _ in range(5):
        F = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
        if np.linalg.det(F) <= 0:
            continue
        R = rot(rng)
        a = nh_density_torch(torch.tensor(F), 2.0, 5.0)
        b = nh_density_torch(torch.tensor(R @ F), 2.0, 5.0)
        assert abs(float(a - b)) < 1e-12 * max(1.0, abs(float(a)))


def test_nh_small_strain_limit_is_linear_elasticity():
    """Psi(I + eps G) / eps^2 -> mu |sym G|^2 + lam/2 (tr G)^2 (linear elasticity)."""
    rng = np.random.default_rng(1)
    E, nu = 1e6, 0.4
    mu, lam = lame(E, nu)
    for _ in range(3):
        G = rng.normal(size=(3, 3))
        eps = 1e-5
        psi = float(nh_density_torch(torch.tensor(np.eye(3) + eps * G), float(mu), float(lam))) / eps ** 2
        S = 0.5 * (G + G.T)
        lin = mu * np.sum(S * S) + 0.5 * lam * np.trace(G) ** 2
        assert abs(psi - lin) < 1e-4 * abs(lin)


def textbook_tet_stiffness(X, E, nu):
    """Linear-elastic stiffness of one linear tet, V B^T D B, Voigt notation (textbook FEM)."""
    Dm = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    V = np.linalg.det(Dm) / 6.0
    gradN = np.zeros((4, 3))
    gradN[1:] = np.linalg.inv(Dm)  # row k = gradient of N_{k+1}
    gradN[0] = -gradN[1:].sum(0)
    B = np.zeros((6, 12))
    for a in range(4):
        nx, ny, nz = gradN[a]
        B[:, 3 * a:3 * a + 3] = [[nx, 0, 0], [0, ny, 0], [0, 0, nz], [0, nz, ny], [nz, 0, nx], [ny, nx, 0]]
    c = E / ((1 + nu) * (1 - 2 * nu))
    D = np.zeros((6, 6))
    D[:3, :3] = c * nu
    np.fill_diagonal(D[:3, :3], c * (1 - nu))
    D[3:, 3:] = np.eye(3) * c * (1 - 2 * nu) / 2
    return V * B.T @ D @ B


def single_tet_scene(X, E=1e6, nu=0.4):
    return dict(rest_pos=X, tets=np.array([[0, 1, 2, 3]], np.int32), youngs=np.array([E]),
                poisson=np.array([nu]), density=np.array([1000.0]), fixed=np.zeros(4, np.uint8),
                obs_pos=np.zeros((0, 3)), obs_tris=np.zeros((0, 3), np.int32), x0=X.copy(),
                v0=np.zeros((4, 3)), dt=1 / 30, dhat=1e-3, gravity=np.array([0, -9.8, 0]), n_steps=1)


def test_element_hessian_at_rest_equals_linear_stiffness():
    rng = np.random.default_rng(2)
    for _ in range(4):
        X = rng.normal(size=(4, 3)) * 0.05
        if np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) < 0:
            X[[1, 2]] = X[[2, 1]]
        o = OracleScene(single_tet_scene(X))
        H = o.element_hessians(X, project=False)[0]
        K = textbook_tet_stiffness(X, 1e6, 0.4)
        assert np.abs(H - K).max() < 1e-9 * np.abs(K).max()
        Hp = o.element_hessians(X, project=True)[0]   # PSD at rest: projection is the identity
        assert np.abs(Hp - K).max() < 1e-9 * np.abs(K).max()


def test_element_forces_balance():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(4, 3)) * 0.05
    if np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) < 0:
        X[[1, 2]] = X[[2, 1]]
    o = OracleScene(single_tet_scene(X))
    x = X + 0.01 * rng.normal(size=X.shape)
    xt = torch.tensor(x, requires_grad=True)
    from oracle.bal_oracle import _tet_energy_single
    e = _tet_energy_single(xt.reshape(-1), o._t_dminv[0], o._t_vol[0], o._t_mu[0], o._t_lam[0])
    e.backward()
    f = xt.grad.numpy()
    assert np.abs(f.sum(0)).max() < 1e-9 * np.abs(f).max()            # no net force
    assert np.abs(np.cross(x, f).sum(0)).max() < 1e-9 * np.abs(f).max()  # no net torque


# -------------------------------------------------------------------- barrier
def test_barrier_clamp_and_shape():
    dh = 1e-3
    d = torch.tensor(dh, dtype=DT, requires_grad=True)
    b = barrier_torch(d, torch.tensor(dh, dtype=DT))
    (g,) = torch.autograd.grad(b, d, create_graph=True)
    (h,) = torch.autograd.grad(g, d)
    assert abs(float(b)) == 0 and abs(float(g)) < 1e-15 and abs(float(h)) < 1e-9   # C2 clamp at dhat
    # special value: d = dhat/e gives log(1/e) = -1, so b = (dhat (1 - 1/e))^2
    assert abs(barrier_np(dh / math.e, dh) - (dh * (1 - 1 / math.e)) ** 2) < 1e-20
    ds = np.linspace(1e-6, dh * 0.999, 50)
    for di in ds:
        t = torch.tensor(di, dtype=DT, requires_grad=True)
        (g,) = torch.autograd.grad(barrier_torch(t, torch.tensor(dh, dtype=DT)), t, create_graph=True)
        (h,) = torch.autograd.grad(g, t)
        assert float(g) < 0 and float(h) > 0
    assert barrier_np(0.0, dh) == np.inf
    assert barrier_np(1e-300, dh) > barrier_np(1e-12, dh) > barrier_np(1e-6, dh)  # blow-up as d -> 0+
    assert barrier_np(2 * dh, dh) == 0.0


# ------------------------------------------------------------------ distances
def brute_pt(p, a, b, c):
    """Point-triangle distance by dense sampling plus constrained local refinement."""
    n = 300
    u, v = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n))
    m = u + v <= 1
    u, v = u[m], v[m]
    pts = a + u[:, None] * (b - a) + v[:, None] * (c - a)
    k = np.argmin(np.linalg.norm(pts - p, axis=1))
    f = lambda z: np.sum((a + z[0] * (b - a) + z[1] * (c - a) - p) ** 2)
    r = scipy.optimize.minimize(f, [u[k], v[k]], method="SLSQP", bounds=[(0, 1), (0, 1)],
                                constraints=[{"type": "ineq", "fun": lambda z: 1 - z[0] - z[1]}],
                                options=dict(ftol=1e-30, maxiter=500))
    return math.sqrt(min(f(r.x), np.min(np.sum((pts - p) ** 2, 1))))


def brute_ee(a0, a1, b0, b1):
    n = 400
    s, t = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n))
    s, t = s.ravel(), t.ravel()
    P = a0 + s[:, None] * (a1 - a0)
    Q = b0 + t[:, None] * (b1 - b0)
    k = np.argmin(np.sum((P - Q) ** 2, 1))
    f = lambda z: np.sum((a0 + z[0] * (a1 - a0) - b0 - z[1] * (b1 - b0)) ** 2)
    r = scipy.optimize.minimize(f, [s[k], t[k]], method="L-BFGS-B", bounds=[(0, 1), (0, 1)],
                                options=dict(ftol=1e-30, gtol=1e-16, maxiter=500))
    return math.sqrt(min(f(r.x), np.min(np.sum((P - Q) ** 2, 1))))


def pt_cases():
    rng = np.random.default_rng(4)
    out = [rng.normal(size=(4, 3)) for _ in range(25)]
    a, b, c = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0., 1, 0])
    out += [np.array([p, a, b, c]) for p in (
        [0.2, 0.2, 0.5], [0.2, 0.2, 0.0], [0.0, 0.0, 0.3], [0.5, 0.0, 0.2], [0.5, -0.3, 0.0],
        [-0.4, -0.4, 0.1], [1.5, 0.0, 0.0], [0.5, 0.5, 0.1], [0.7, 0.7, -0.2], [0, 0, 0])]
    return out


def ee_cases():
    rng = np.random.default_rng(5)
    out = [rng.normal(size=(4, 3)) for _ in range(25)]
    out += [np.array(e, dtype=float) for e in (
        [[0, 0, 0], [1, 0, 0], [0.5, -1, 0.3], [0.5, 1, 0.3]],     # crossing, interior
        [[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]],              # parallel, overlapping
        [[0, 0, 0], [1, 0, 0], [2, 0.5, 0], [3, 0.5, 0]],          # parallel, disjoint
        [[0, 0, 0], [1, 0, 0], [1.5, 0, 0], [2.5, 0, 0]],          # collinear
        [[0, 0, 0], [1, 0, 0], [1, -1, 0.2], [1, 1, 0.2]],         # touching at an endpoint line
        [[0, 0, 0], [1, 0, 0], [2, -1, 1], [2, 1, 1]],             # endpoint-edge region
    )]
    return out


@pytest.mark.parametrize("X", pt_cases())
def test_point_triangle_distance_brute_force(X):
    q, _ = classify_pt(X[None, 0], X[None, 1], X[None, 2], X[None, 3])
    d = math.sqrt(q[0])
    ref = brute_pt(*X)
    assert abs(d - ref) <= 1e-7 * max(1.0, ref)
    assert d <= ref + 1e-12


@pytest.mark.parametrize("X", ee_cases())
def test_edge_edge_distance_brute_force(X):
    q, _ = classify_ee(X[None, 0], X[None, 1], X[None, 2], X[None, 3])
    d = math.sqrt(q[0])
    ref = brute_ee(*X)
    assert abs(d - ref) <= 1e-7 * max(1.0, ref)


def test_distance_continuity_across_regions():
    """Distance is continuous in the query point across every region boundary."""
    a, b, c = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0., 1, 0])
    ts = np.linspace(-0.5, 1.5, 2001)
    P = np.stack([ts, 0.3 * np.ones_like(ts), 0.05 * np.ones_like(ts)], 1)
    q, _ = classify_pt(P, np.broadcast_to(a, P.shape), np.broadcast_to(b, P.shape), np.broadcast_to(c, P.shape))
    d = np.sqrt(q)
    assert np.abs(np.diff(d)).max() < 2e-3


# ----------------------------------------------------------------- projection
def test_projection_matches_polar_formula():
    """Closest PSD matrix = (H + |H|)/2 with |H| = sqrtm(H^2) (polar decomposition)."""
    rng = np.random.default_rng(6)
    for n in (3, 9, 12):
        A = rng.normal(size=(n, n))
        H = A + A.T
        P = project_psd(H)
        absH = np.real(scipy.linalg.sqrtm(H @ H))
        ref = 0.5 * (H + absH)
        assert np.abs(P - ref).max() < 1e-8 * np.abs(H).max()
        assert np.linalg.eigvalsh(P).min() > -1e-10 * np.abs(H).max()
        S = A @ A.T
        assert np.abs(project_psd(S) - S).max() < 1e-10 * np.abs(S).max()


# ---------------------------------------------------------------------- steps
@pytest.fixture(scope="module")
def tiny_run():
    o = OracleScene(scenes.tiny_cube())
    x0 = o.x.copy()
    traces, states = [], []
    for _ in range(3):
        tr = []
        o.step(trace=tr)
        traces.append(tr)
        states.append((o.x.copy(), o.v.copy()))
    return o, x0, traces, states


def test_contact_free_step_closed_form(tiny_run):
    o, x0, traces, states = tiny_run
    gold = json.load(open(os.path.join(GOLDEN, "tiny_cube_step1.json")))
    x1, v1 = states[0]
    n = o.n_body
    dy = x1[:n] - x0[:n]
    assert np.abs(dy[:, 1] - gold["delta_y"]).max() < 1e-10
    assert np.abs(dy[:, [0, 2]]).max() < 1e-10
    assert np.abs(v1[:n, 1] - gold["v_y"]).max() < 1e-8
    assert len(traces[0]) == gold["newton_iterations"]
    assert abs(o.mass[:n].sum() - gold["mass_total_kg"]) < 1e-9


def test_no_interpenetration_and_no_inversion(tiny_run):
    o, x0, traces, states = tiny_run
    pairs = o.all_pairs()
    for x, _ in states:
        d, _ = o.distances(x, pairs)
        assert d.min() > 0
        e = x[o.tets[:, 1:]] - x[o.tets[:, :1]]
        J = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))
        assert J.min() > 0
    # resting on the plane at the end of step 3: lowest vertex is within dhat of it
    assert 0 < states[-1][0][: o.n_body, 1].min() < o.dhat


def test_newton_converges_each_step(tiny_run):
    o, x0, traces, states = tiny_run
    for tr in traces:
        assert tr[-1]["enorm"] <= 1e-4 * tr[0]["enorm"]


def test_momentum_free_flight():
    sc = scenes.spinning_cube()
    sc["gravity"] = np.zeros(3)
    o = OracleScene(sc)
    M = o.mass[:, None]
    p0 = (M * o.v).sum(0)
    for _ in range(3):
        o.step()
    p1 = (M * o.v).sum(0)
    assert np.abs(p1 - p0).max() < 1e-6 * np.abs(p0).max()
    sc = scenes.spinning_cube()
    o = OracleScene(sc)
    p0 = (M * o.v).sum(0)
    o.step()
    p1 = (M * o.v).sum(0)
    expect = o.h * np.array([0, -9.8, 0]) * o.mass.sum()
    assert np.abs((p1 - p0) - expect).max() < 1e-6 * np.abs(expect).max()


# ------------------------------------------------- derivatives of L_sigma (FD)
def contact_state():
    """Tiny cube pressed onto the plane with a hand-made augmentation set."""
    sc = scenes.tiny_cube()
    o = OracleScene(sc)
    x = o.x.copy()
    x[: o.n_body, 1] -= 0.02 - 4e-4
    rng = np.random.default_rng(7)
    x[: o.n_body] += rng.uniform(-2e-5, 2e-5, size=(o.n_body, 3))
    pairs = o.all_pairs()
    d, _ = o.distances(x, pairs)
    act = np.nonzero(d < o.dhat)[0]
    aug = pairs.take(act[::3])
    st = ALState(sigma=3e4, sigma0=3e4, aug=aug, mu=rng.uniform(0, 50, len(aug)),
                 s=rng.uniform(0, 2e-4, len(aug)))
    y = o.predictor(o.x, o.v)
    return o, x, y, pairs, st


def test_gradient_and_hessian_against_finite_differences():
    o, x, y, pairs, st = contact_state()
    L, g = o.lagrangian(x, y, pairs, st, with_grad=True)
    gf = o.gradient_free(g)
    H = o.hessian(x, pairs, st, project=False)
    rng = np.random.default_rng(8)
    for _ in range(3):
        dx = np.zeros_like(x)
        dx[o.free_idx] = rng.normal(size=(o.free_idx.size, 3))
        eps = 1e-7
        Lp = o.lagrangian(x + eps * dx, y, pairs, st)
        Lm = o.lagrangian(x - eps * dx, y, pairs, st)
        fd = (Lp - Lm) / (2 * eps)
        an = float(gf @ dx[o.free_idx].reshape(-1))
        assert abs(fd - an) <= 1e-6 * abs(an)
        _, gp = o.lagrangian(x + eps * dx, y, pairs, st, with_grad=True)
        _, gm = o.lagrangian(x - eps * dx, y, pairs, st, with_grad=True)
        fdh = (o.gradient_free(gp) - o.gradient_free(gm)) / (2 * eps)
        hv = H @ dx[o.free_idx].reshape(-1)
        assert np.linalg.norm(fdh - hv) <= 1e-5 * np.linalg.norm(hv)


def test_hessian_vector_product_against_finite_differences():
    """The double-backward Hessian-vector product equals central differences
    of the gradient, and the assembled unprojected Hessian times the vector."""
    o, x, y, pairs, st = contact_state()
    H = o.hessian(x, pairs, st, project=False)
    rng = np.random.default_rng(9)
    for _ in range(2):
        v = rng.normal(size=x.shape)
        hv = o.hessian_vector_product(x, y, pairs, st, v)
        dx = np.where(o.free[:, None], v, 0.0)
        eps = 1e-7
        _, gp = o.lagrangian(x + eps * dx, y, pairs, st, with_grad=True)
        _, gm = o.lagrangian(x - eps * dx, y, pairs, st, with_grad=True)
        fd = (o.gradient_free(gp) - o.gradient_free(gm)) / (2 * eps)
        an = o.gradient_free(hv)
        assert np.linalg.norm(fd - an) <= 1e-5 * np.linalg.norm(an)
        assert np.abs(H @ dx[o.free_idx].reshape(-1) - an).max() <= 1e-9 * np.abs(an).max()
        assert np.all(hv[~o.free] == 0.0)


def test_sigma0_is_least_squares_minimiser():
    """sigma0 minimises ||g_E + s g_b||^2 (checked by a scalar minimiser); else the norm-ratio fallback."""
    o, x, y_far, pairs, _ = contact_state()
    d, _ = o.distances(x, pairs)
    act = pairs.take(np.nonzero(d < o.dhat)[0])
    y_rest = o.predictor(x, np.zeros_like(x))  # resting: gravity pulls into the plane
    for y in (y_rest, y_far):
        s0 = o.sigma0(x, y, act, ALState())
        _, gE = o.lagrangian(x, y, act, ALState(sigma=0.0), with_grad=True)
        _, g1 = o.lagrangian(x, y, act, ALState(sigma=1.0), with_grad=True)
        gE, gb = o.gradient_free(gE), o.gradient_free(g1) - o.gradient_free(gE)
        r = scipy.optimize.minimize_scalar(lambda s: float(np.sum((gE + s * gb) ** 2)),
                                           bracket=(0.0, 1e3), tol=1e-14)
        if r.x > 0:
            assert abs(r.x - s0) <= 1e-6 * s0
        else:
            assert abs(s0 - np.linalg.norm(gE) / np.linalg.norm(gb)) <= 1e-9 * s0
    assert o.sigma0(x, y_rest, act, ALState()) > 0


def test_groupwise_solve_is_per_group_dense_solve():
    o, x, y, pairs, st = contact_state()
    H, e = o.hessian(x, pairs, st, with_lambda=True)
    groups = o.stiffness_groups(e[o.free_idx])
    assert (e > 0).all()
    assert np.unique(groups).size >= 2
    rng = np.random.default_rng(9)
    b = rng.normal(size=H.shape[0])
    z = o.groupwise_solve(H, b, groups)
    Hd = H.toarray()
    gd = np.repeat(groups, 3)
    for g in np.unique(groups):
        idx = np.nonzero(gd == g)[0]
        zg = np.linalg.solve(Hd[np.ix_(idx, idx)], b[idx])
        assert np.abs(zg - z[idx]).max() <= 1e-9 * np.abs(zg).max()


def test_lambda_trace_identity_single_tet():
    """Lambda per node of one tet at rest = 3 tr(K)/12 + 3 m/h^2 with K the textbook stiffness."""
    rng = np.random.default_rng(10)
    X = rng.normal(size=(4, 3)) * 0.05
    if np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) < 0:
        X[[1, 2]] = X[[2, 1]]
    o = OracleScene(single_tet_scene(X))
    _, e = o.hessian(X, Pairs.empty(), ALState(), with_lambda=True)
    K = textbook_tet_stiffness(X, 1e6, 0.4)
    V = np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) / 6
    expect = 3 * np.trace(K) / 12 + 3 * (1000 * V / 4) / o.h ** 2
    assert np.abs(e - expect).max() < 1e-9 * expect


# ------------------------------------------------------------------------ CCD
def test_cubic_roots_against_companion_eigenvalues():
    rng = np.random.default_rng(11)
    K = 300
    r = rng.uniform(-0.2, 1.2, size=(K, 3))
    c3 = rng.uniform(0.5, 2, K)
    c2 = -c3 * r.sum(1)
    c1 = c3 * (r[:, 0] * r[:, 1] + r[:, 1] * r[:, 2] + r[:, 0] * r[:, 2])
    c0 = -c3 * r.prod(1)
    got = OracleScene.cubic_roots(c3, c2, c1, c0)
    for i in range(K):
        ev = np.roots([c3[i], c2[i], c1[i], c0[i]])
        ev = np.sort(ev.real[(np.abs(ev.imag) < 1e-9) & (ev.real >= -1e-12) & (ev.real <= 1 + 1e-12)])
        g = got[i][np.isfinite(got[i])]
        if ev.size == g.size:
            if ev.size:
                assert np.abs(np.sort(g) - ev).max() < 1e-7
        else:  # near-double roots: every isolated root is a true root
            for t in g:
                assert abs(((c3[i] * t + c2[i]) * t + c1[i]) * t + c0[i]) < 1e-9


def test_ccd_bound_precedes_first_crossing():
    """alpha_max never exceeds the first time a vertex passes through a triangle (dense time scan)."""
    rng = np.random.default_rng(12)
    sc = single_tet_scene(np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]))
    o = OracleScene(sc)
    hits = 0
    for trial in range(60):
        tri = rng.normal(size=(3, 3))
        p0 = tri.mean(0) + rng.normal(size=3) * 0.5
        P = rng.normal(size=(4, 3)) * 1.5
        x = np.concatenate([p0[None], tri])
        pairs = Pairs(np.array([0]), np.array([0]), np.array([0]), np.array([[0, 1, 2, 3]]))
        amax = o.ccd(x, P, pairs)
        ts = np.linspace(0, 1, 20001)
        X = x[None] + ts[:, None, None] * P[None]
        n = np.cross(X[:, 2] - X[:, 1], X[:, 3] - X[:, 1])
        sd = np.einsum("ij,ij->i", X[:, 0] - X[:, 1], n)
        q, case = classify_pt(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
        cross = np.nonzero((np.sign(sd[1:]) != np.sign(sd[:-1])) & (case[1:] == 0) & (case[:-1] == 0))[0]
        d0 = math.sqrt(q[0])
        if cross.size:
            hits += 1
            assert amax <= ts[cross[0] + 1] + 1e-12
        if d0 > 1e-2 * o.dhat:
            assert amax > 0
    assert hits > 5


def test_kdtree_pair_superset_matches_brute_force():
    """The large-scene pair search returns every brute-force pair within reach."""
    sc = scenes.stacked_boxes(n_cubes=2, cells=3, seed=0)
    o = OracleScene(sc)
    x = o.x.copy()
    rng = np.random.default_rng(0)
    x[: o.n_body] += rng.normal(scale=2e-3, size=(o.n_body, 3))
    allp = o.all_pairs()
    d, _ = o.distances(x, allp)
    for reach in (1e-3, 5e-3, 2e-2):
        need = set(map(int, allp.keys()[d < reach]))
        have = set(map(int, o.near_pairs(x, reach).keys()))
        assert need <= have


def test_submesh_rows_equal_full_mesh_rows():
    """Rows of sampled vertices from the sub-mesh of their incident tets equal
    the full mesh's rows (the basis of the sampled full-size GPU checks)."""
    from subsets import sub_scene
    sc = scenes.spmv_grid(6)
    o = OracleScene(sc)
    x = sc["x0"]
    y = o.predictor(x, sc["v0"])
    st = ALState()
    rng = np.random.default_rng(13)
    v = rng.normal(size=x.shape)
    _, g_full = o.lagrangian(x, y, o.all_pairs(), st, with_grad=True)
    hv_full = o.hessian_vector_product(x, y, o.all_pairs(), st, v)
    pick = rng.choice(x.shape[0], size=12, replace=False)
    sub, used, remap = sub_scene(sc, pick)
    os_ = OracleScene(sub)
    ys = os_.predictor(x[used], sc["v0"][used])
    _, g_sub = os_.lagrangian(x[used], ys, os_.all_pairs(), st, with_grad=True)
    hv_sub = os_.hessian_vector_product(x[used], ys, os_.all_pairs(), st, v[used])
    assert np.abs(g_sub[remap[pick]] - g_full[pick]).max() <= 1e-12 * np.abs(g_full).max()
    assert np.abs(hv_sub[remap[pick]] - hv_full[pick]).max() <= 1e-12 * np.abs(hv_full).max()
