"""GPU parity of fully-implicit friction (Sec. 4.1) through the C ABI: the
linearization with friction frames against the oracle's definition, and
whole steps of a sliding cube in lockstep with the oracle."""
import numpy as np
import pytest

from oracle import ALState, OracleScene, Params
from test_gpu_parity import first_divergence, free_rows
from test_oracle_friction import resting_cube

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("project", [True, False])
def test_linearize_with_friction(project):
    """At an iterate displaced along the ground from the scene's state (every
    pair sliding, some inside the mollifier's range), the library's energy,
    gradient and Hessian product equal the oracle's with the frames taken at
    that iterate."""
    from paper_2407_00046_amd import Scene
    chi = 0.4
    sc = resting_cube(chi)
    o = OracleScene(sc, Params(friction=chi))
    x_t = o.x.copy()
    rng = np.random.default_rng(4)
    x = x_t.copy()
    # most vertices slide 2 mm; a few stay within eps_v h (3.3e-5 m) of their start
    shift = np.where(rng.uniform(size=o.n_body) < 0.2, 1e-5, 2e-3)
    x[: o.n_body, 0] += shift
    x[: o.n_body] += rng.normal(scale=2e-6, size=(o.n_body, 3))
    sigma = 1e4
    g = Scene(sc, friction=chi)
    E, grad, nact = g.linearize(x, sigma, project=project)
    y = o.predictor(o.x, o.v)
    pairs = o.all_pairs()
    st = ALState(sigma=sigma, sigma0=sigma)
    st.frames = o.friction_frames(x, x_t, pairs, st)
    L, gref = o.lagrangian(x, y, pairs, st, with_grad=True)
    print(f"{len(st.frames.pairs)} friction pairs, E {E:.12e} vs {L:.12e}")
    assert len(st.frames.pairs) >= 20
    assert abs(E - L) <= 1e-10 * abs(L)
    gf, rf = free_rows(o, grad), free_rows(o, gref)
    assert np.abs(gf - rf).max() <= 1e-9 * np.abs(rf).max()
    H = o.hessian(x, pairs, st, project=project)
    for _ in range(3):
        v = rng.normal(size=(o.N, 3))
        hv = H @ free_rows(o, v)
        lv = free_rows(o, g.hessian_apply(v))
        assert np.linalg.norm(lv - hv) <= 1e-9 * np.linalg.norm(hv)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sliding_cube_steps(precision):
    """Two steps of the cube sliding at 1 m/s on the ground with chi = 0.5:
    in FP64 the decision traces and positions follow the oracle (positions to
    1e-6 of the scene size); in mixed precision the positions follow to 1e-4.
    Coulomb's law shows in the GPU step's momentum balance: the horizontal
    impulse is at most chi times the normal one and within 1% of it."""
    from paper_2407_00046_amd import Scene
    chi = 0.5
    sc = resting_cube(chi)
    rtol = 1e-7 if precision == "fp64" else 1e-6
    g = Scene(sc, precision=precision, newton_rtol=rtol, pcg_rtol=1e-12 if precision == "fp64" else 1e-6,
              max_newton=200, friction=chi)
    o = OracleScene(sc, Params(newton_rtol=rtol, max_newton=200, friction=chi))
    n = sc["rest_pos"].shape[0]
    L = np.linalg.norm(sc["x0"].max(0) - sc["x0"].min(0))
    m = o.mass[:n][:, None]
    M = float(m.sum())
    err = 0.0
    for k in range(2):
        err_prev = err
        _, v_prev = g.get_state()
        st = g.step()
        tr = []
        so = o.step(trace=tr)
        xg, vg = g.get_state()
        err = np.linalg.norm(xg - o.x[:n], axis=1).max() / L
        print(f"step {k}: gpu {st['newton_iters']} Newton, oracle {len(tr)}; eps_x {err:.3e}")
        assert st["converged"] == 1 and so["converged"]
        if precision == "fp64":
            # the frames are re-taken from every iterate and each pair's friction
            # force scales with its normal force, the barrier's stiff derivative:
            # the PCG-level iterate differences reach |e| at ~1e-5, not 1e-6
            div = first_divergence(g.trace(), tr, sc["dhat"], tr[0]["enorm"], e_rtol=1e-4, newton_rtol=rtol,
                                   state_err=err_prev)
            assert div is None, f"step {k}: {div}"
            assert err <= 1e-6
        else:
            assert err <= 1e-4
        dp = (m * (vg - v_prev)).sum(0)
        normal = dp[1] + M * 9.8 * sc["dt"]
        assert 0.99 * chi * normal <= -dp[0] <= chi * normal * (1 + 1e-6)
