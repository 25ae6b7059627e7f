"""Checks of the seeded scene generators: sizes of the workloads, positive
tets, conforming meshes with closed surfaces, and a feasible rest state
(every non-incident surface pair farther apart than d-hat)."""
from collections import Counter

import numpy as np
import pytest

import scenes


def volumes(pos, tets):
    e = pos[tets[:, 1:]] - pos[tets[:, :1]]
    return np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) / 6.0


def face_counts(tets):
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    return Counter(map(tuple, np.sort(faces, axis=1)))


def check_closed_conforming(pos, tets):
    """Every face is shared by at most two tets, the boundary faces form a
    closed surface (each boundary edge in exactly two boundary faces), and the
    tets fill the enclosed volume (divergence theorem: sum of tet volumes =
    flux of x through the outward boundary faces / 3)."""
    fc = face_counts(tets)
    assert max(fc.values()) <= 2
    bnd = [f for f, c in fc.items() if c == 1]
    ec = Counter()
    for a, b, c in bnd:
        for e in ((a, b), (b, c), (a, c)):
            ec[e] += 1
    assert set(ec.values()) == {2}
    # outward orientation of each boundary face from its tet
    owner = {}
    for t in tets:
        for drop in range(4):
            f = tuple(sorted(np.delete(t, drop)))
            if fc[f] == 1:
                owner[f] = (t, t[drop])
    flux = 0.0
    for f, (t, opp) in owner.items():
        a, b, c = pos[list(f)]
        n = np.cross(b - a, c - a)
        if np.dot(n, pos[opp] - a) > 0:
            n = -n
        flux += np.dot(a, n) / 6.0
    assert flux == pytest.approx(volumes(pos, tets).sum(), rel=1e-10)
    return len(bnd)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_icosphere_counts_and_radius(level):
    v, f = scenes.icosphere(level)
    assert v.shape[0] == 10 * 4 ** level + 2 and f.shape[0] == 20 * 4 ** level
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    # Euler characteristic of a sphere and outward (counter-clockwise) faces
    edges = {tuple(sorted(e)) for a, b, c in f for e in ((a, b), (b, c), (c, a))}
    assert v.shape[0] - len(edges) + f.shape[0] == 2
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert np.all(np.einsum("ij,ij->i", n, v[f].mean(axis=1)) > 0)


def test_prism_split_is_conforming_for_any_numbering():
    """Random global numberings of a two-layer shell: every split agrees on
    shared quads (closed boundary, no face used three times), tets positive
    after orientation, total volume unchanged."""
    rng = np.random.default_rng(3)
    pos, tets = scenes.hollow_sphere(1, 2, 0.8, 1.0)
    ref = volumes(pos, tets).sum()
    for _ in range(3):
        perm = rng.permutation(pos.shape[0])
        inv = np.argsort(perm)
        prisms = None
        v, f = scenes.icosphere(1)
        nv = v.shape[0]
        prisms = np.concatenate([np.concatenate([f + l * nv, f + (l + 1) * nv], 1) for l in range(2)])
        t = scenes.orient_positive(pos[perm], scenes.prism_to_tets(inv[prisms]))
        assert np.all(volumes(pos[perm], t) > 0)
        check_closed_conforming(pos[perm], t)
        assert volumes(pos[perm], t).sum() == pytest.approx(ref, rel=1e-12)


def test_hollow_sphere_shell_volume():
    """Shell volume converges to 4/3 pi (R^3 - r^3) from below (inscribed polyhedra)."""
    pos, tets = scenes.hollow_sphere(3, 2, 0.08, 0.1)
    vol = volumes(pos, tets)
    assert np.all(vol > 0)
    exact = 4.0 / 3.0 * np.pi * (0.1 ** 3 - 0.08 ** 3)
    assert 0.97 * exact < vol.sum() < exact
    nb = check_closed_conforming(pos, tets)
    assert nb == 2 * 20 * 4 ** 3


def test_tube_ring_is_a_closed_solid_torus():
    pos, tets = scenes.tube_ring((0, 0, 0), (1, 0, 0), (0, 0, 1), (0, 1, 0), 0.02, 0.003, 10)
    assert tets.shape[0] == 10 * 4 * 6 and pos.shape[0] == 90
    assert np.all(volumes(pos, tets) > 0)
    nb = check_closed_conforming(pos, tets)
    assert nb == 10 * 4 * 2 * 2  # 4 sides x 2 cells x 2 triangles per segment
    # volume of the polygonal square-section torus: section area x centroid path (Pappus, polygon form)
    n, R, h = 10, 0.02, 0.003
    # each segment is a frustum-like prism; exact polyhedral volume = sum over sections of
    # (2h) * integral of (2 r sin(pi/n) cos(pi/n)) dr over [R-h, R+h]
    exact = 2 * h * n * np.sin(np.pi / n) * np.cos(np.pi / n) * ((R + h) ** 2 - (R - h) ** 2)
    assert volumes(pos, tets).sum() == pytest.approx(exact, rel=1e-12)


def test_chain_net_sizes():
    sc = scenes.chain_net()
    assert sc["tets"].shape[0] == 401_280 and sc["rest_pos"].shape[0] == 135_144
    assert int(sc["fixed"].sum()) == 76 * 90
    assert np.all(volumes(sc["rest_pos"], sc["tets"].astype(np.int64)) > 0)
    net = sc["youngs"] == 1e9
    assert int(net.sum()) == 1160 * 240 and np.all(sc["youngs"][~net] == 5e5)


@pytest.mark.slow
def test_chain_net_large_sizes():
    sc = scenes.chain_net_large()
    assert sc["tets"].shape[0] == 1_762_560 and sc["rest_pos"].shape[0] == 497_160
    assert int(sc["fixed"].sum()) == 76 * 28 * 9


def test_small_chain_net_rest_state_is_feasible():
    """On a 5 x 5-site net every non-incident surface pair is farther apart
    than d-hat at rest (brute force over all pairs with the oracle's
    distances), so the threaded links start separated."""
    from oracle import OracleScene, Params
    sc = scenes.chain_net(sites=5, sphere_level=0, sphere_layers=1)
    o = OracleScene(sc, Params())
    d, _ = o.distances(o.x, o.all_pairs())
    assert d.min() > sc["dhat"]
    assert d.min() < 3e-3  # the links are threaded: the closest pairs are close
