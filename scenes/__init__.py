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


def stacked_boxes(n_cubes=8, cells=16, cell=0.01, gap=0.005, seed=0, E=1e6, nu=0.45, n_steps=10, rotate=True):
    """n_cubes randomly rotated cubes of cells^3 cells, stacked on the y axis.

    Each cube is rotated by a uniform random rotation (seeded); cube k+1's
    lowest point sits `gap` above cube k's highest point, and the bottom cube
    sits `gap` above a fixed two-triangle ground plane [-2, 2]^2.
    The default (8 cubes of 16^3 cells, 163,840 tets) is the stacked-boxes
    workload; small variants serve as parity cases.  With rotate=False the
    cubes stay axis-aligned (face to face; with a gap below dhat every
    interface is in contact from the start).
    """
    rng = np.random.default_rng(seed)
    base, base_tets = tet_grid(cells, cells, cells, cell)
    base = base - base.mean(axis=0)
    nv = base.shape[0]
    pos_all, tets_all = [], []
    top = 0.0
    for k in range(n_cubes):
        R = random_rotation(rng)
        p = base @ R.T if rotate else base.copy()
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


def icosphere(level: int):
    """Unit icosphere: the icosahedron with every triangle split into 4,
    `level` times, new vertices pushed to the sphere.  Returns (verts (n,3),
    faces (f,3) int64) with faces counter-clockwise seen from outside;
    n = 10 * 4^level + 2, f = 20 * 4^level."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        nxt = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nxt += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nxt
    return np.array(verts), np.array(faces, dtype=np.int64)


# Prism symmetries taking vertex k to position 0 (bottom v0 v1 v2, top v3 v4 v5,
# v_{i+3} above v_i), used by the prism split below.
_PRISM_ROT = [(0, 1, 2, 3, 4, 5), (1, 2, 0, 4, 5, 3), (2, 0, 1, 5, 3, 4),
              (3, 5, 4, 0, 2, 1), (4, 3, 5, 1, 0, 2), (5, 4, 3, 2, 1, 0)]


def prism_to_tets(prisms):
    """Split prisms (P,6) into 3 tets each so that neighbouring prisms agree.

    Every quadrilateral face is cut by the diagonal through its vertex of
    smallest global index (Dompierre et al., 1999): the prism is turned so
    that its smallest vertex is v0, which fixes the two quads through v0, and
    the third quad (v1 v2 v5 v4) is cut through min(v1, v5) vs min(v2, v4).
    """
    prisms = np.asarray(prisms, dtype=np.int64)
    rot = np.array(_PRISM_ROT)[np.argmin(prisms, axis=1)]
    v = np.take_along_axis(prisms, rot, axis=1)
    v0, v1, v2, v3, v4, v5 = v.T
    a = np.minimum(v1, v5) < np.minimum(v2, v4)
    t1 = np.where(a[:, None], np.stack([v0, v1, v2, v5], 1), np.stack([v0, v1, v2, v4], 1))
    t2 = np.where(a[:, None], np.stack([v0, v1, v5, v4], 1), np.stack([v0, v4, v2, v5], 1))
    t3 = np.stack([v0, v4, v5, v3], 1)
    return np.stack([t1, t2, t3], 1).reshape(-1, 4)


def hollow_sphere(level: int, layers: int, r_in: float, r_out: float, centre=(0.0, 0.0, 0.0)):
    """Spherical shell: icosphere `level` surface, `layers` radial layers of
    prisms between r_in and r_out, 3 tets per prism.  Vertex (l, v) of layer
    l = 0..layers has index l * n_surface + v."""
    sv, sf = icosphere(level)
    nv = sv.shape[0]
    radii = np.linspace(r_in, r_out, layers + 1)
    pos = np.concatenate([sv * r for r in radii]) + np.asarray(centre, dtype=np.float64)
    prisms = np.concatenate([np.concatenate([sf + l * nv, sf + (l + 1) * nv], axis=1) for l in range(layers)])
    tets = orient_positive(pos, prism_to_tets(prisms))
    return pos, tets.astype(np.int32)


# Kuhn split of a cube into 6 tets along the diagonal 000 -> 111: one tet per
# order in which the three axes are stepped.
_KUHN = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def tube_ring(centre, e1, e2, e3, R: float, half: float, n_u: int):
    """Closed square-section tube (a torus link) of centre-line radius R in
    the plane (e1, e2) through `centre`; the section is the square
    [-half, half]^2 in the (radial, e3) directions, split 2 x 2.  Each of the
    n_u x 2 x 2 hexahedral cells is cut into 6 tets (Kuhn split, conforming
    across cells and across the seam).  Vertex (u, a, b) has index
    (u * 3 + a) * 3 + b."""
    centre, e1, e2, e3 = (np.asarray(x, dtype=np.float64) for x in (centre, e1, e2, e3))
    u = np.arange(n_u)[:, None, None]
    a = np.arange(3)[None, :, None]
    b = np.arange(3)[None, None, :]
    th = 2.0 * np.pi * u / n_u
    rad = R + (a - 1) * half
    off = (b - 1) * half
    pos = (centre + (rad * np.cos(th))[..., None] * e1 + (rad * np.sin(th))[..., None] * e2
           + (off + 0.0 * th)[..., None] * e3).reshape(-1, 3)

    def vid(uu, aa, bb):
        return ((uu % n_u) * 3 + aa) * 3 + bb

    cu, ca, cb = (x.ravel() for x in np.meshgrid(np.arange(n_u), np.arange(2), np.arange(2), indexing="ij"))
    tets = []
    for order in _KUHN:
        step = np.zeros(3, dtype=np.int64)
        corners = [vid(cu, ca, cb)]
        for axis in order:
            step[axis] += 1
            corners.append(vid(cu + step[0], ca + step[1], cb + step[2]))
        tets.append(np.stack(corners, 1))
    tets = np.stack(tets, 1).reshape(-1, 4)
    return pos, orient_positive(pos, tets).astype(np.int32)


def chain_net(sites=40, pitch=0.025, R_flat=0.02, R_link=0.015, half=0.003, n_u=10,
              sphere_level=4, sphere_layers=2, r_in=0.08, r_out=0.1, n_steps=5,
              E_net=1e9, nu_net=0.3, E_sphere=5e5, nu_sphere=0.4):
    """Four hollow spheres falling onto a chain net of tet-meshed torus links.

    Net: a sites x sites grid of pitch `pitch` in the xz-plane (y = 0).  Flat
    rings (axis y, centre-line radius R_flat) sit at the (even, even) sites;
    connector rings (radius R_link) sit at the (odd, even) sites in the
    xy-plane and at the (even, odd) sites in the yz-plane, each threading its
    two flat neighbours.  With pitch 2.5 cm, R_flat 2 cm, R_link 1.5 cm and a
    6 mm square section the flat rings stay 5 mm apart and every threaded
    pair keeps at least 1 mm of clearance (the link crossings lie at the
    middle of the links' straight segments).  The flat rings on the border of
    the net are fixed.  Spheres: shells r_in..r_out, at (+-0.2, ., +-0.2),
    5 mm above the net's top.  The default (40 x 40 sites, 1160 links of
    n_u = 10, spheres of level 4 x 2 layers) has 401,280 tets.
    """
    ex, ey, ez = np.eye(3)
    pos_all, tets_all, E_all, nu_all, fixed_all = [], [], [], [], []
    nbase = 0

    def add(pos, tets, E, nu, fixed):
        nonlocal nbase
        pos_all.append(pos)
        tets_all.append(tets.astype(np.int64) + nbase)
        E_all.append(np.full(tets.shape[0], E))
        nu_all.append(np.full(tets.shape[0], nu))
        fixed_all.append(np.full(pos.shape[0], 1 if fixed else 0, np.uint8))
        nbase += pos.shape[0]

    c0 = -0.5 * (sites - 1) * pitch
    for i in range(sites):
        for k in range(sites):
            centre = np.array([c0 + i * pitch, 0.0, c0 + k * pitch])
            if i % 2 == 0 and k % 2 == 0:
                border = i == 0 or k == 0 or i == sites - 2 + (sites % 2) or k == sites - 2 + (sites % 2)
                p, t = tube_ring(centre, ex, ez, ey, R_flat, half, n_u)
                add(p, t, E_net, nu_net, border)
            elif i % 2 == 1 and k % 2 == 0 and i + 1 < sites:
                p, t = tube_ring(centre, ex, ey, ez, R_link, half, n_u)
                add(p, t, E_net, nu_net, False)
            elif i % 2 == 0 and k % 2 == 1 and k + 1 < sites:
                p, t = tube_ring(centre, ez, ey, ex, R_link, half, n_u)
                add(p, t, E_net, nu_net, False)
    top = R_link + half
    for sx in (-0.2, 0.2):
        for sz in (-0.2, 0.2):
            p, t = hollow_sphere(sphere_level, sphere_layers, r_in, r_out, (sx, top + 0.005 + r_out, sz))
            add(p, t, E_sphere, nu_sphere, False)
    pos = np.concatenate(pos_all)
    tets = np.concatenate(tets_all)
    name = f"chain_net_{sites}x{sites}_nu{n_u}_L{sphere_level}x{sphere_layers}"
    sc = _pack(name, pos, tets, 1.0, 0.3, 1000.0, np.concatenate(fixed_all), np.zeros((0, 3)),
               np.zeros((0, 3), np.int32), dt=1.0 / 30.0, dhat=1e-3, n_steps=n_steps)
    sc["youngs"] = np.concatenate(E_all)
    sc["poisson"] = np.concatenate(nu_all)
    return sc


def chain_net_large(E_net=1e9):
    """The chain-net scene refined: spheres of level 5 x 4 layers and links of
    n_u = 28 (1,762,560 tets), one step."""
    return chain_net(n_u=28, sphere_level=5, sphere_layers=4, n_steps=1, E_net=E_net)


def open_box(lo, hi):
    """Floor and four walls of an open box (an aquarium), inward-facing
    triangles: 8 vertices, 10 triangles."""
    pos, tris = box_mesh(lo, hi)
    top = [t for t in range(12) if all(pos[v][1] >= hi[1] for v in tris[t])]
    keep = np.array([t for t in range(12) if t not in top])
    return pos, tris[keep]


def tumbling_blocks(n_x=3, n_z=4, n_layers=5, cells=31, cell=0.01, gap=0.005, seed=0, E=5e5, nu=0.4,
                    n_steps=1):
    """The memory-limited scale-up workload: n_x * n_z * n_layers randomly
    rotated blocks of cells^3 cells x 5 tets stacked in columns (each block
    `gap` above the highest point of the one below, the lowest layer `gap`
    above the floor) inside an open box.  The default, 60 blocks of 31^3
    cells (8,937,300 tets, 1,966,080 vertices), stands in for the paper's
    tumbling-T-rex scene (its Table of scenarios: 9M tets, E = 5e5, one step
    of h = 1/30)."""
    rng = np.random.default_rng(seed)
    base, base_tets = tet_grid(cells, cells, cells, cell)
    base = base - base.mean(axis=0)
    nv = base.shape[0]
    edge = cells * cell
    pitch = 1.8 * edge
    pos_all, tets_all = [], []
    k = 0
    for i in range(n_x):
        for j in range(n_z):
            top = 0.0
            for _ in range(n_layers):
                R = random_rotation(rng)
                p = base @ R.T
                p[:, 1] += top + gap - p[:, 1].min()
                p[:, 0] += (i - 0.5 * (n_x - 1)) * pitch
                p[:, 2] += (j - 0.5 * (n_z - 1)) * pitch
                top = p[:, 1].max()
                pos_all.append(p)
                tets_all.append(base_tets + k * nv)
                k += 1
    pos = np.concatenate(pos_all)
    tets = np.concatenate(tets_all)
    half_x, half_z = 0.5 * n_x * pitch + 0.1, 0.5 * n_z * pitch + 0.1
    obs_pos, obs_tris = open_box((-half_x, 0.0, -half_z), (half_x, pos[:, 1].max() + 1.0, half_z))
    return _pack(f"tumbling_blocks_{k}x{cells}^3", pos, tets, E, nu, 1000.0, None, obs_pos, obs_tris,
                 dt=1.0 / 30.0, dhat=1e-3, n_steps=n_steps)


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
