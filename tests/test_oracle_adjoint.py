"""Pins of the oracle's adjoint (frozen-state implicit differentiation).

Checked against central finite differences of re-solved steps and against
the closed form of rigid free flight: x_T = x_0 + h (T v_0 + h g T(T+1)/2),
so a uniform perturbation of v_0 moves every vertex of x_T by T h.
"""
import numpy as np
import pytest

import scenes
from oracle import ALState, OracleScene, Params


def small_beam():
    sc = scenes.beam(nx=6, ny=2, nz=2, cell=0.05, seed=0, n_steps=2)
    sc["obs_pos"] = np.zeros((0, 3))
    sc["obs_tris"] = np.zeros((0, 3), np.int32)
    return sc


def newton_frozen(o, x, y, st, tol=1e-11, iters=12):
    """Plain Newton on L_sigma with the augmentation state frozen (no contacts here)."""
    pairs = o.candidate_pairs(x)
    for _ in range(iters):
        _, g = o.lagrangian(x, y, pairs, st, with_grad=True)
        e = o.gradient_free(g)
        if np.linalg.norm(e) < tol:
            break
        H = o.hessian(x, pairs, st, project=True)
        dx = np.zeros_like(x)
        dx[o.free_idx] = -o.solve(H, e).reshape(-1, 3)
        x = x + dx
    return x


def loss(o, x_next, x_t, w, u):
    v_next = (x_next - x_t) / o.h
    return float(np.sum(w * x_next[: o.n_body]) + np.sum(u * v_next[: o.n_body]))


def test_adjoint_matches_central_differences():
    sc = small_beam()
    o = OracleScene(sc, Params(newton_rtol=1e-9))
    st = o.step(return_state=True)
    x_next, y, state, x_t, v_t = o.x.copy(), st["y"], st["state"], st["x_t"], st["v_t"]
    rng = np.random.default_rng(0)
    w = rng.normal(size=(o.n_body, 3))
    u = rng.normal(size=(o.n_body, 3))
    gx_t, gv_t, gE = o.adjoint_step(x_next, y, state, w, u)
    E0 = o.E.copy()
    # d loss / d E_e for a few elements
    for e in (0, 7, len(E0) - 1):
        vals = []
        for sgn in (1, -1):
            E = E0.copy()
            E[e] *= 1 + sgn * 1e-6
            o.set_youngs(E)
            xs = newton_frozen(o, x_next.copy(), y, state)
            vals.append(loss(o, xs, x_t, w, u))
        o.set_youngs(E0)
        fd = (vals[0] - vals[1]) / (2e-6 * E0[e])
        assert abs(fd - gE[e]) <= 1e-4 * max(abs(fd), 1e-8 * np.abs(gE).max())
    # d loss / d v_t along a random direction (y depends on v_t; x_t fixed)
    dv = np.zeros_like(v_t)
    dv[o.free_idx] = rng.normal(size=(o.free_idx.size, 3))
    vals = []
    for sgn in (1, -1):
        yp = o.predictor(x_t, v_t + sgn * 1e-6 * dv)
        xs = newton_frozen(o, x_next.copy(), yp, state)
        vals.append(loss(o, xs, x_t, w, u))
    fd = (vals[0] - vals[1]) / 2e-6
    an = float(np.sum(gv_t * dv[: o.n_body]))
    assert abs(fd - an) <= 1e-5 * abs(an)
    # d loss / d x_t along a random direction (x_t enters y and v_{t+1})
    dx = np.zeros_like(x_t)
    dx[o.free_idx] = rng.normal(size=(o.free_idx.size, 3))
    vals = []
    for sgn in (1, -1):
        xt2 = x_t + sgn * 1e-7 * dx
        yp = o.predictor(xt2, v_t)
        xs = newton_frozen(o, x_next.copy(), yp, state)
        vals.append(loss(o, xs, xt2, w, u))
    fd = (vals[0] - vals[1]) / 2e-7
    an = float(np.sum(gx_t * dx[: o.n_body]))
    assert abs(fd - an) <= 1e-5 * abs(an)


def test_free_flight_closed_form():
    """Uniform v0 perturbation: d x_T / d v0 = T h I; Young's moduli have no effect on rigid motion."""
    sc = scenes.spinning_cube()
    sc["v0"] = np.tile(np.array([0.3, 0.1, -0.2]), (sc["rest_pos"].shape[0], 1))
    o = OracleScene(sc, Params(newton_rtol=1e-9))
    T = 3
    hist = [o.step(return_state=True) for _ in range(T)]
    rng = np.random.default_rng(1)
    wvec = rng.normal(size=3)
    n = o.n_body
    gx = np.tile(wvec, (n, 1))
    gv = np.zeros((n, 3))
    gE = np.zeros(len(o.E))
    x_next = o.x.copy()
    for t in reversed(range(T)):
        st = hist[t]
        gx, gv, dE = o.adjoint_step(x_next, st["y"], st["state"], gx, gv)
        gE += dE
        x_next = st["x_t"]
    # x_0 perturbation moves everything rigidly: d loss / d(uniform dx0) = n w
    assert np.allclose(gv.sum(0), T * o.h * n * wvec, rtol=1e-6, atol=1e-9)
    assert np.allclose(gx.sum(0), n * wvec, rtol=1e-6, atol=1e-9)
    assert np.abs(gE).max() <= 1e-8 * np.abs(gv).max()
