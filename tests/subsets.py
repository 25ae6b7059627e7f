"""Sub-meshes for sampled checks: the rows of the gradient and of the
Hessian at a vertex depend only on the tets around it (and, through the
lumped mass, on the same tets), so a mesh made of every tet incident to a
set of vertices reproduces those rows exactly when no contact is active."""
import numpy as np


def sub_scene(sc, verts):
    """Every tet incident to `verts`, on the vertices they use."""
    tets = sc["tets"]
    sel = np.nonzero(np.isin(tets, verts).any(axis=1))[0]
    used = np.unique(tets[sel])
    remap = -np.ones(sc["rest_pos"].shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    sub = dict(sc)
    sub.update(rest_pos=sc["rest_pos"][used], tets=remap[tets[sel]].astype(np.int32),
               youngs=sc["youngs"][sel], poisson=sc["poisson"][sel], density=sc["density"][sel],
               fixed=sc["fixed"][used], x0=sc["x0"][used], v0=sc["v0"][used],
               obs_pos=np.zeros((0, 3)), obs_tris=np.zeros((0, 3), np.int32))
    return sub, used, remap
