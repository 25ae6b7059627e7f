"""CPU pins of the oracle's friction (Sec. 4.1): the mollifier f against its
printed closed form and C1 continuation, the closest-point weights against
the distance cases, the friction potential's derivatives against central
differences and its Hessian's definiteness, and Coulomb's law in the
momentum balance of a sliding cube (an identity of any converged step)."""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import OracleScene, Params
from oracle.bal_oracle import (ALState, CASE_KIND, CASE_NODES, Pairs, classify, closest_coeffs,
                               friction_f_torch)


def f_printed(y, eh):
    return -y ** 3 / (3 * eh * eh) + y * y / eh


def test_mollifier_closed_form_and_continuity():
    eh = 1e-3 / 30.0
    for y in (0.0, 0.1 * eh, 0.5 * eh, 0.9 * eh):
        v = float(friction_f_torch(torch.tensor(y * y, dtype=torch.float64), eh))
        assert abs(v - f_printed(y, eh)) <= 1e-15 * max(1.0, f_printed(y, eh)) + 1e-20
    # C1 at y = eps h: values and slopes of the two branches meet; slope 1 beyond
    def fy(y):
        q = torch.tensor(y * y, dtype=torch.float64, requires_grad=True)
        v = friction_f_torch(q, eh)
        (g,) = torch.autograd.grad(v, q)
        return float(v), float(g) * 2 * y   # df/dy = df/dq * 2y
    lo, hi = fy(eh * (1 - 1e-9)), fy(eh * (1 + 1e-9))
    assert abs(lo[0] - hi[0]) <= 1e-8 * eh and abs(lo[1] - hi[1]) <= 1e-6
    assert abs(fy(3 * eh)[1] - 1.0) <= 1e-12
    # f'(0) = 0 and f''(0) = 2 / (eps h) (mollified start of the kinetic law)
    y = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    v = friction_f_torch(y * y, eh)
    (g,) = torch.autograd.grad(v, y, create_graph=True)
    (h2,) = torch.autograd.grad(g, y)
    assert float(g) == 0.0 and abs(float(h2) - 2.0 / eh) <= 1e-9 / eh


def random_cases(rng, n):
    X = rng.normal(size=(n, 4, 3))
    kind = rng.integers(0, 2, size=n)
    return kind, X


def test_closest_weights_give_the_case_distance():
    """n = sum beta_k X_k joins the two closest points: |n| is the case's
    distance, and n is orthogonal to the primitives' directions the case
    keeps (the edge for point-edge, the triangle for point-triangle, both
    edges for edge-edge); the weights on each side sum to +1 and -1."""
    rng = np.random.default_rng(3)
    kind, X = random_cases(rng, 400)
    q, case = classify(kind, X)
    beta = closest_coeffs(case, X)
    n = np.einsum("kj,kjc->kc", beta, X)
    assert np.allclose(np.linalg.norm(n, axis=1), np.sqrt(q), rtol=1e-9, atol=1e-12)
    seen = set()
    for i in range(len(case)):
        c = int(case[i])
        nd = CASE_NODES[c]
        k = CASE_KIND[c]
        seen.add(k)
        assert abs(beta[i].sum()) <= 1e-12   # +1 on one side, -1 on the other
        if k == 1:      # point-edge: n is orthogonal to the edge
            dirs = [X[i, nd[2]] - X[i, nd[1]]]
        elif k == 2:    # point-triangle interior: orthogonal to the triangle
            dirs = [X[i, 2] - X[i, 1], X[i, 3] - X[i, 1]]
        elif k == 3:    # edge-edge interior: orthogonal to both edges
            dirs = [X[i, 1] - X[i, 0], X[i, 3] - X[i, 2]]
        else:
            dirs = []
        for e in dirs:
            assert abs(np.dot(n[i], e)) <= 1e-9 * np.linalg.norm(e) * max(1.0, np.linalg.norm(n[i]))
    assert seen == {0, 1, 2, 3}


def resting_cube(chi, vx=1.0):
    """Tiny cube 0.4 mm above the ground (inside dhat) sliding at vx along x.
    The ground is one large triangle whose edges lie far from the cube, so
    every contact pair is a point-triangle interior pair with the normal +y
    (with the two-triangle plane, cube edges crossing its diagonal edge tilt
    a few normals by the cube's own deformation)."""
    sc = dict(scenes.tiny_cube())
    sc["obs_pos"] = np.array([[-3.0, 0.0, -3.0], [6.0, 0.0, -3.0], [-3.0, 0.0, 6.0]])
    sc["obs_tris"] = np.array([[0, 2, 1]], np.int32)
    o = OracleScene(sc, Params())
    tri = o.x[o.n_body:]
    assert np.cross(tri[2] - tri[0], tri[1] - tri[0])[1] > 0  # normal +y
    x = o.x.copy()
    x[: o.n_body, 1] -= x[: o.n_body, 1].min() - 4e-4
    sc["x0"] = x[: o.n_body].copy()
    sc["v0"] = np.zeros_like(sc["x0"])
    sc["v0"][:, 0] = vx
    return sc


def test_friction_potential_derivatives_and_definiteness():
    """With frames frozen at an iterate, the friction potential's gradient
    matches central differences and its stencil Hessians are positive
    semi-definite before any projection (the mollifier is convex on
    [0, eps h] and the kinetic branch's Hessian is f'/y times a projector)."""
    sc = resting_cube(0.4)
    o = OracleScene(sc, Params(friction=0.4))
    x_t = o.x.copy()
    rng = np.random.default_rng(4)
    x = x_t.copy()
    x[: o.n_body] += np.array([2e-3, -1e-4, 5e-4]) + rng.normal(scale=2e-6, size=(o.n_body, 3))
    pairs = o.all_pairs()
    st = ALState(sigma=1e4, sigma0=1e4)
    st.frames = o.friction_frames(x, x_t, pairs, st)
    fr = st.frames
    assert len(fr.pairs) >= 20 and (fr.lam > 0).all()
    H = o.friction_hessians(x, fr, project=False)
    ev = np.linalg.eigvalsh(H)
    assert ev.min() >= -1e-9 * np.abs(ev).max()
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    D = o.friction_energy_torch(xt, fr)
    (g,) = torch.autograd.grad(D, xt)
    g = g.numpy()
    for v, c in [(0, 0), (5, 1), (17, 2), (60, 0)]:
        h = 1e-7
        xp, xm = x.copy(), x.copy()
        xp[v, c] += h
        xm[v, c] -= h
        fd = (float(o.friction_energy_torch(torch.tensor(xp), fr)) -
              float(o.friction_energy_torch(torch.tensor(xm), fr))) / (2 * h)
        assert abs(fd - g[v, c]) <= 1e-6 * max(1.0, abs(g).max())
    # kinetic regime: each pair's force is chi lam along the sliding direction
    assert D.item() > 0


def test_sliding_cube_obeys_coulomb_in_its_momentum_balance():
    """A converged step of the sliding cube balances momentum with its contact
    forces (internal forces cancel): dp = h (-M g y + sum_j lam_j n_j - chi
    sum_j lam_j w_j), with n_j = +y for every pair (point-triangle interior on
    a flat ground) and, every pair sliding (|u h| >> eps_v h, kinetic branch
    f' = 1), w_j the unit tangential relative displacement of the step.  So
    dp_x = -chi h sum lam_j w_j,x, a little below chi times the normal impulse
    dp_y + M g h (the cube's own deformation turns some w_j off the x axis),
    and with chi = 0 the horizontal impulse vanishes."""
    for chi in (0.0, 0.5):
        sc = resting_cube(chi)
        o = OracleScene(sc, Params(newton_rtol=1e-7, max_newton=200, friction=chi))
        m = o.mass[: o.n_body][:, None]
        M = float(m.sum())
        g, h = 9.8, o.h
        for k in range(2):
            v0 = o.v[: o.n_body].copy()
            st = o.step(return_state=True)
            assert st["converged"]
            dp = (m * (o.v[: o.n_body] - v0)).sum(0)
            normal = dp[1] + M * g * h
            print(f"chi {chi} step {k}: dp {dp}, normal impulse {normal:.6f}, M g h {M * g * h:.6f}")
            assert normal > 0.1 * M * g * h
            fr = st["state"].frames
            if chi == 0.0:
                assert fr is None
                assert abs(dp[0]) <= 1e-9 * M * g * h and abs(dp[2]) <= 1e-9 * M * g * h
                continue
            x = o.x
            assert np.allclose(fr.n[:, [0, 2]], 0.0, atol=1e-15) and (fr.n[:, 1] > 0).all()
            assert abs(h * fr.lam.sum() - normal) <= 1e-5 * M * g * h
            du = np.einsum("kj,kjc->kc", fr.beta, x[fr.pairs.nodes] - fr.x_t[fr.pairs.nodes])
            w = du.copy()
            w[:, 1] = 0.0
            y = np.linalg.norm(w, axis=1)
            assert y.min() > 100 * fr.eps_h
            pred = -chi * h * (fr.lam[:, None] * w / y[:, None]).sum(0)
            assert abs(dp[0] - pred[0]) <= 1e-5 * M * g * h
            assert abs(dp[2] - pred[2]) <= 1e-5 * M * g * h
            assert 0.99 * chi * normal <= -dp[0] <= chi * normal * (1 + 1e-9)
