"""Seeded synthetic scene generators for the BAL time step.

This module only builds inputs: rest geometry, tetrahedra, per-element
materials, Dirichlet masks, static obstacle triangles and the initial state.
It holds none of the method's arithmetic (no masses, volumes, surfaces,
energies or derivatives); the CPU oracle and the GPU library each derive
those on their own from what is returned here.

Every scene is a plain dict of numpy arrays and scalars:

    rest_pos  (n, 3) float64   rest positions, SI units, y up
    tets      (T, 4) int32     tetrahedra, positively oriented at rest
    youngs, poisson, density   (T,) float64 per-tet material
    fixed     (n,) uint8       Dirichlet (clamped) vertices
    obs_pos   (m, 3) float64   static obstacle vertices
    obs_tris  (k, 3) int32     static obstacle triangles (into obs_pos)
    x0, v0    (n, 3) float64   initial state
    dt, dhat  float            time step h and barrier offset d-hat
    gravity   (3,) float64
    n_steps   int              steps the workload runs

The workloads stand in for the paper's unavailable meshes (its Table of
scenarios); nothing here reproduces a published asset.
"""
from __future__ import annotations

import numpy as np

GRAVITY = np.array([0.0, -9.8, 0.0])

# Corner offsets of a hexahedral cell, keyed by the 3-bit code (a, b, c).
_CORNERS = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]


def _five_tet_split(parity: int):
    """Five tets of a unit cell as lists of corner codes (a, b, c).

    Even cells use the central tet on the even-sum corners, odd cells on the
    odd-sum corners; the four remaining tets each join one leftover corner to
    its three cell neighbours.  Alternating the parity by (i + j + k) mod 2
    makes the face diagonals of adjacent cells agree (a conforming mesh).
    """
    even = [c for c in _CORNERS if sum(c) % 2 == 0]
    odd = [c for c in _CORNERS if sum(c) % 2 == 1]
    centre, others = (even, odd) if parity == 0 else (odd, even)
    tets = [centre]
    for c in others:
        nbrs = [tuple(c[k] ^ (1 if k == ax else 0) for k in range(3)) for ax in range(3)]
        tets.append([c] + nbrs)
    return tets


def tet_grid(nx: int, ny: int, nz: int, cell: float, origin=(0.0, 0.0, 0.0)):
    """Regular grid of nx*ny*nz cells split 5 tets per cell.

    Vertex (i, j, k) has index (i*(ny+1) + j)*(nz+1) + k.  Returns
    (positions (n,3) float64, tets (T,4) int32) with every tet positively
    oriented.
    """
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    pos = np.stack([ii, jj, kk], axis=-1).reshape(-1, 3).astype(np.float64) * cell
    pos += np.asarray(origin, dtype=np.float64)

    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    parity = (ci + cj + ck) % 2
    tets = np.empty((ci.size, 5, 4), dtype=np.int64)
    for par in (0, 1):
        sel = parity == par
        for t, corners in enumerate(_five_tet_split(par)):
            for q, (a, b, c) in enumerate(corners):
                tets[sel, t, q] = vid(ci[sel] + a, cj[sel] + b, ck[sel] + c)
    tets = tets.reshape(-1, 4)
    tets = orient_positive(pos, tets)
    return pos, tets.astype(np.int32)


def orient_positive(pos, tets):
    """Swap two vertices of every negatively oriented tet (geometry only)."""
    tets = np.array(tets, dtype=np.int64, copy=True)
    e = pos[tets[:, 1:]] - pos[tets[:, :1]]
    vol6 = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    neg = vol6 < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    return tets


def random_rotation(rng: np.random.Generator):
    """Uniform random rotation from a normalised 4-normal quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ground_plane(half: float, y: float = 0.0):
    """Two-triangle square [-half, half]^2 at height y, normal +y."""
    pos = np.array([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]])
    tris = np.array([[0, 2, 1], [0, 3, 2]], dtype=np.int32)
    return pos, tris


def box_mesh(lo, hi):
    """Closed axis-aligned box: 8 vertices, 12 triangles."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    pos = np.array([[(hi if (c >> k) & 1 else lo)[k] for k in range(3)] for c in range(8)])
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    tris = []
    for a, b, c, d in quads:
        tris += [(a, b, c), (a, c, d)]
    return pos, np.array(tris, dtype=np.int32)


def _pack(name, pos, tets, E, nu, rho, fixed, obs_pos, obs_tris, dt, dhat, n_steps, v0=None, x0=None):
    n, T = pos.shape[0], tets.shape[0]
    full = lambda v: np.full(T, float(v)) if np.isscalar(v) else np.asarray(v, dtype=np.float64)
    return dict(
        name=name,
        rest_pos=np.ascontiguousarray(pos, dtype=np.float64),
        tets=np.ascontiguousarray(tets, dtype=np.int32),
        youngs=full(E), poisson=full(nu), density=full(rho),
        fixed=np.ascontiguousarray(fixed, dtype=np.uint8) if fixed is not None else np.zeros(n, np.uint8),
        obs_pos=np.ascontiguousarray(obs_pos, dtype=np.float64).reshape(-1, 3),
        obs_tris=np.ascontiguousarray(obs_tris, dtype=np.int32).reshape(-1, 3),
        x0=np.ascontiguousarray(pos if x0 is None else x0, dtype=np.float64),
        v0=np.zeros((n, 3)) if v0 is None else np.ascontiguousarray(v0, dtype=np.float64),
        dt=float(dt), dhat=float(dhat), gravity=GRAVITY.copy(), n_steps=int(n_steps),
    )


def tiny_cube():
    """4x4x4-cell cube, edge 0.4 m, dropped 0.02 m above a fixed plane.

    Cube [-0.2, 0.2]^3 shifted by +0.05 in x so that the plane's diagonal
    (x = z) passes at least 0.05 m from every cube vertex; bottom at y = 0.02.
    E = 1e5 Pa, nu = 0.4, rho = 1000, h = 1/30 s, d-hat = 1e-3 m, 3 steps.
    """
    pos, tets = tet_grid(4, 4, 4, 0.1, origin=(-0.15, 0.02, -0.2))
    obs_pos, obs_tris = ground_plane(1.0)
    return _pack("tiny_cube_320", pos, tets, 1e5, 0.4, 1000.0, None, obs_pos, obs_tris,
                 dt=1.0 / 30.0, dhat=1e-3, n_steps=3)


def stacked_boxes(n_cubes=8, cells=16, cell=0.01, gap=0.005, seed=0, E=1e6, nu=0.45, n_steps=10):
    """n_cubes randomly rotated cubes of cells^3 cells, stacked on the y axis.

    Each cube is rotated by a uniform random rotation (seeded); cube k+1's
    lowest point sits `gap` above cube k's highest point, and the bottom cube
    sits `gap` above a fixed two-triangle ground plane [-2, 2]^2.
    The default (8 cubes of 16^3 cells, 163,840 tets) is the stacked-boxes
    workload; small variants serve as parity cases.
    """
    rng = np.random.default_rng(seed)
    base, base_tets = tet_grid(cells, cells, cells, cell)
    base = base - base.mean(axis=0)
    nv = base.shape[0]
    pos_all, tets_all = [], []
    top = 0.0
    for k in range(n_cubes):
        R = random_rotation(rng)
        p = base @ R.T
        p[:, 1] += top + gap - p[:, 1].min()
        top = p[:, 1].max()
        pos_all.append(p)
        tets_all.append(base_tets + k * nv)
    pos = np.concatenate(pos_all)
    tets = np.concatenate(tets_all)
    obs_pos, obs_tris = ground_plane(2.0)
    name = f"stacked_boxes_{n_cubes}x{cells}^3"
    return _pack(name, pos, tets, E, nu, 1000.0, None, obs_pos, obs_tris,
                 dt=1.0 / 30.0, dhat=1e-3, n_steps=n_steps)


def beam(nx=128, ny=16, nz=16, cell=0.01, seed=0, sigma_logE=0.3, meanE=1e6, nu=0.4,
         n_steps=20, lognormal="mean"):
    """Cantilever beam clamped at x = 0 falling onto a fixed box.

    Beam [0, nx*cell] x [0, ny*cell] x [0, nz*cell]; the x = 0 face is
    clamped; the box top lies 5 mm below the beam's bottom face and spans
    x in [0.75*L, 1.25*L], z in [-0.3, nz*cell + 0.3] (L = nx*cell).
    Per-tet E is lognormal with arithmetic mean `meanE` (or median, with
    lognormal="median") and log-sigma `sigma_logE`; free vertices start with
    v0 = (0, -0.5, 0); h = 1/60 s.
    """
    pos, tets = tet_grid(nx, ny, nz, cell)
    rng = np.random.default_rng(seed)
    mu_log = np.log(meanE) - (0.5 * sigma_logE ** 2 if lognormal == "mean" else 0.0)
    E = np.exp(rng.normal(mu_log, sigma_logE, size=tets.shape[0]))
    fixed = (np.abs(pos[:, 0]) < 1e-12).astype(np.uint8)
    L = nx * cell
    obs_pos, obs_tris = box_mesh((0.75 * L, -0.1 - 0.005, -0.3), (1.25 * L, -0.005, nz * cell + 0.3))
    v0 = np.zeros_like(pos)
    v0[fixed == 0, 1] = -0.5
    return _pack(f"beam_{nx}x{ny}x{nz}", pos, tets, E, nu, 1000.0, fixed, obs_pos, obs_tris,
                 dt=1.0 / 60.0, dhat=1e-3, n_steps=n_steps, v0=v0)


def spmv_grid(n=128, cell=0.01, seed=2, amplitude=0.1):
    """Large regular grid for the block-SpMV roofline (no contact).

    n^3 cells x 5 tets, vertex positions perturbed by uniform noise of
    `amplitude` x cell (seeded) so that the Neo-Hookean Hessians are generic.
    """
    pos, tets = tet_grid(n, n, n, cell)
    rng = np.random.default_rng(seed)
    x0 = pos + rng.uniform(-amplitude * cell, amplitude * cell, size=pos.shape)
    return _pack(f"spmv_grid_{n}^3", pos, tets, 1e6, 0.4, 1000.0, None,
                 np.zeros((0, 3)), np.zeros((0, 3), np.int32), dt=1.0 / 30.0, dhat=1e-3,
                 n_steps=1, x0=x0)


def perturbed(scene, amplitude, seed):
    """Copy of `scene` with x0 displaced by uniform noise (parity inputs)."""
    rng = np.random.default_rng(seed)
    out = dict(scene)
    out["x0"] = scene["x0"] + rng.uniform(-amplitude, amplitude, size=scene["x0"].shape)
    return out


def spinning_cube(cells=2, size=0.2, omega=(0.0, 3.0, 1.0), v=(0.3, 0.1, -0.2)):
    """Stress-free cube in free flight (no obstacles) with rigid spin and drift."""
    pos, tets = tet_grid(cells, cells, cells, size / cells)
    c = pos.mean(axis=0)
    v0 = np.asarray(v) + np.cross(np.asarray(omega, dtype=np.float64), pos - c)
    return _pack("spinning_cube", pos, tets, 1e5, 0.4, 1000.0, None, np.zeros((0, 3)),
                 np.zeros((0, 3), np.int32), dt=1.0 / 30.0, dhat=1e-3, n_steps=3, v0=v0)


WORKLOADS = {
    "tiny_cube": tiny_cube,
    "stacked_boxes": stacked_boxes,
    "beam": beam,
    "spmv_grid": spmv_grid,
}
