"""Edge cases through the C ABI: inputs that bal_create_scene must refuse,
and degenerate scenes whose step has a closed form (one tet in free fall:
no contact candidates, a four-node system, far below one workgroup; every
vertex fixed: nothing to solve)."""
import numpy as np
import pytest

import scenes
from paper_2407_00046_amd.bal import (BAL_E_INVALID_ARG, BAL_E_INVERTED, BAL_E_PENETRATION, BalError)

pytestmark = pytest.mark.gpu

TET = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0], [0.0, 0.0, 0.1]])


def one_tet(**kw):
    args = dict(name="one_tet", pos=TET + np.array([0.0, 0.5, 0.0]), tets=np.array([[0, 1, 2, 3]]), E=1e5, nu=0.4,
                rho=1000.0, fixed=None, obs_pos=np.zeros((0, 3)), obs_tris=np.zeros((0, 3), np.int32),
                dt=1.0 / 30.0, dhat=1e-3, n_steps=1)
    args.update(kw)
    return scenes._pack(**args)


def create(sc, **kw):
    from paper_2407_00046_amd import Scene
    return Scene(sc, **kw)


def expect_refused(sc, code):
    with pytest.raises(BalError) as e:
        create(sc)
    assert e.value.code == code


def test_create_refuses_bad_inputs():
    expect_refused(one_tet(tets=np.array([[0, 1, 2, 4]])), BAL_E_INVALID_ARG)  # index out of range
    pos = TET.copy()
    pos[1, 0] = np.nan
    expect_refused(one_tet(pos=pos), BAL_E_INVALID_ARG)  # non-finite position
    expect_refused(one_tet(nu=0.5), BAL_E_INVALID_ARG)  # incompressible limit
    expect_refused(one_tet(dt=0.0), BAL_E_INVALID_ARG)
    expect_refused(one_tet(dhat=-1e-3), BAL_E_INVALID_ARG)
    # a free vertex in no tet has no mass
    pos5 = np.vstack([TET, [[1.0, 1.0, 1.0]]])
    expect_refused(one_tet(pos=pos5), BAL_E_INVALID_ARG)
    # negative rest volume
    expect_refused(one_tet(tets=np.array([[0, 2, 1, 3]])), BAL_E_INVERTED)
    # a vertex on an obstacle triangle: a pair at zero distance
    obs = np.array([[-1.0, 0.5, -1.0], [1.0, 0.5, -1.0], [1.0, 0.5, 1.0], [-1.0, 0.5, 1.0]])
    expect_refused(one_tet(obs_pos=obs, obs_tris=np.array([[0, 2, 1], [0, 3, 2]])), BAL_E_PENETRATION)


def test_one_tet_free_fall_is_the_predictor():
    """Without contact the step minimises the inertia term plus an elastic
    energy that is zero and stationary at every translation of the rest
    shape; the predictor y = x0 + h v0 + h^2 g is such a translation, so the
    step lands on it and v1 = v0 + h g."""
    v0 = np.tile([0.3, -0.2, 0.1], (4, 1))
    for prec in ("fp64", "mixed"):
        sc = one_tet(v0=v0)
        g = create(sc, precision=prec, newton_rtol=1e-8, pcg_rtol=1e-10)
        st = g.step()
        x1, v1 = g.get_state()
        g.close()
        h = sc["dt"]
        y = sc["x0"] + h * v0 + h * h * sc["gravity"]
        print(f"{prec}: {st['newton_iters']} Newton iterations, |x1 - y| = {np.abs(x1 - y).max():.2e}")
        assert st["converged"] == 1 and st["n_active_max"] == 0
        assert np.abs(x1 - y).max() <= 1e-12
        assert np.abs(v1 - (v0 + h * sc["gravity"])).max() <= 1e-10


def test_all_fixed_scene_stays_put():
    sc = one_tet(fixed=np.ones(4, np.uint8), v0=np.tile([1.0, 0.0, 0.0], (4, 1)))
    g = create(sc)
    st = g.step()
    x1, v1 = g.get_state()
    g.close()
    assert st["converged"] == 1
    assert np.array_equal(x1, sc["x0"]) and np.all(v1 == 0.0)
