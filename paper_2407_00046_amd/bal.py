"""ctypes binding of libbal.so (include/bal.h): argument marshalling only.

Every function named bal_* here calls the C entry point of the same name.
`Scene` wraps a scene handle for numpy / torch callers and `BalRollout` is a
torch.autograd.Function over multi-step rollouts whose backward pass calls
bal_step_adjoint with per-segment checkpoints.  All computation happens in
the HIP library; importing this module fails if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbal.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2407_00046_amd/build.py "
                      "(hipcc --offload-arch=gfx950); there is no fallback path")
_lib = C.CDLL(LIB_PATH)

BAL_OK, BAL_E_INVALID_ARG, BAL_E_OOM, BAL_E_HIP = 0, -1, -2, -3
BAL_E_PENETRATION, BAL_E_INVERTED, BAL_E_CAPACITY, BAL_E_NO_CONVERGENCE, BAL_E_STATE = -4, -5, -6, -7, -8
BAL_E_INDEFINITE = -9
BAL_FP64, BAL_MIXED = 0, 1
BAL_CCD_PRINTED, BAL_CCD_HALF_GAP, BAL_CCD_LITERAL = 0, 1, 2
CCD_RULES = {"printed": BAL_CCD_PRINTED, "half_gap": BAL_CCD_HALF_GAP, "literal": BAL_CCD_LITERAL}
BAL_BROAD_HASH, BAL_BROAD_LBVH = 0, 1
BROAD_PHASES = {"hash": BAL_BROAD_HASH, "lbvh": BAL_BROAD_LBVH}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


class bal_scene_desc(C.Structure):
    _fields_ = [
        ("n_verts", C.c_int32), ("n_tets", C.c_int32),
        ("rest_pos", _dp), ("tets", _ip), ("youngs", _dp), ("poisson", _dp), ("density", _dp), ("fixed", _up),
        ("n_obs_verts", C.c_int32), ("n_obs_tris", C.c_int32),
        ("obs_pos", _dp), ("obs_tris", _ip), ("x0", _dp), ("v0", _dp),
        ("dt", C.c_double), ("gravity", C.c_double * 3), ("dhat", C.c_double),
        ("newton_rtol", C.c_double), ("pcg_rtol", C.c_double), ("sigma_fixed", C.c_double),
        ("friction", C.c_double), ("eps_v", C.c_double), ("accept_rtol", C.c_double),
        ("max_newton", C.c_int32), ("max_pcg", C.c_int32), ("pcg_stall_window", C.c_int32),
        ("max_contacts", C.c_int32), ("warm_iters", C.c_int32), ("precision", C.c_int32),
        ("warm_start", C.c_int32), ("use_al", C.c_int32), ("ccd_rule", C.c_int32), ("broad_phase", C.c_int32), ("sweep_cap", C.c_int32),
        ("device", C.c_int32), ("stream", C.c_void_p),
    ]


class bal_step_stats(C.Structure):
    _fields_ = [
        ("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("warm_iters", C.c_int32),
        ("n_active_max", C.c_int32), ("n_aug_max", C.c_int32), ("converged", C.c_int32),
        ("ls_retries", C.c_int32), ("spmv_launches", C.c_int32), ("graph_launches", C.c_int32),
        ("stalled", C.c_int32),
        ("sigma", C.c_double), ("min_dist", C.c_double), ("sec_total", C.c_double), ("sec_pcg", C.c_double),
        ("sec_hessian", C.c_double), ("sec_ccd", C.c_double), ("sec_collision", C.c_double),
        ("sec_linesearch", C.c_double), ("spmv_ms", C.c_double), ("spmv_bytes", C.c_double),
        ("grad_rel", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bal_al_state(C.Structure):
    _fields_ = [("sigma", C.c_double), ("n_aug", C.c_int32), ("aug_kind", _ip), ("aug_prims", _ip),
                ("mu", _dp), ("s", _dp)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_vp = C.c_void_p
bal_desc_defaults = _sig("bal_desc_defaults", None, C.POINTER(bal_scene_desc))
bal_create_scene = _sig("bal_create_scene", C.c_int, C.POINTER(bal_scene_desc), C.POINTER(_vp))
bal_destroy_scene = _sig("bal_destroy_scene", None, _vp)
bal_step = _sig("bal_step", C.c_int, _vp, C.POINTER(bal_step_stats))
bal_get_state = _sig("bal_get_state", C.c_int, _vp, _vp, _vp, C.c_int)
bal_set_state = _sig("bal_set_state", C.c_int, _vp, _vp, _vp, C.c_int)
bal_set_youngs = _sig("bal_set_youngs", C.c_int, _vp, _vp, C.c_int)
bal_step_adjoint = _sig("bal_step_adjoint", C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int,
                        C.POINTER(bal_step_stats))
bal_status_string = _sig("bal_status_string", C.c_char_p, C.c_int)
bal_get_trace = _sig("bal_get_trace", C.c_int, _vp, _vp, C.c_int32, _ip)
bal_set_kernel_timing = _sig("bal_set_kernel_timing", C.c_int, _vp, C.c_int)
bal_get_surface = _sig("bal_get_surface", C.c_int, _vp, _ip, _vp, _ip, _vp, _ip, _vp)
bal_linearize = _sig("bal_linearize", C.c_int, _vp, _vp, C.POINTER(bal_al_state), C.c_int, _dp, _vp, _ip)
bal_hessian_apply = _sig("bal_hessian_apply", C.c_int, _vp, _vp, _vp)
bal_get_stiffness = _sig("bal_get_stiffness", C.c_int, _vp, _vp, _vp)
bal_solve = _sig("bal_solve", C.c_int, _vp, _vp, _vp, C.c_int, C.c_double, C.c_int32, _ip, _dp)
bal_ccd_bound = _sig("bal_ccd_bound", C.c_int, _vp, _vp, _vp, _dp)
bal_candidates = _sig("bal_candidates", C.c_int, _vp, _vp, _vp, C.c_int32, _vp, _vp, _vp, _ip)
bal_spmv_benchmark = _sig("bal_spmv_benchmark", C.c_int, _vp, C.c_int32, _dp, _dp)
bal_stream_benchmark = _sig("bal_stream_benchmark", C.c_int, C.c_int32, C.c_int64, C.c_int32, _dp, _dp)
_pairs_args = (C.c_int32, _vp, _vp, C.c_int32, _vp, _vp, C.c_int32, C.c_double, C.c_int32, _vp, _vp)
bal_pairs_ccd_bound = _sig("bal_pairs_ccd_bound", C.c_int, *_pairs_args)
bal_pairs_ccd_bound_noalloc = _sig("bal_pairs_ccd_bound_noalloc", C.c_int, *_pairs_args)

EXPORTED = [n for n in dir() if n.startswith("bal_") and callable(globals()[n])
            and n not in ("bal_scene_desc", "bal_step_stats", "bal_al_state")]


class BalError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {bal_status_string(code).decode()} ({code})")
        self.code = code


def _check(code, where, ok=(BAL_OK,)):
    if code not in ok:
        raise BalError(code, where)
    return code


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def stream_benchmark(device=0, n_bytes=2 << 30, reps=20):
    """(read GB/s, copy GB/s) of the library's streaming kernels (bal_stream_benchmark)."""
    r, c = C.c_double(), C.c_double()
    _check(bal_stream_benchmark(int(device), int(n_bytes), int(reps), C.byref(r), C.byref(c)),
           "bal_stream_benchmark")
    return r.value, c.value


class Scene:
    """One simulated scene on one GPU (wraps a bal_scene handle).

    `sc` is a scene dict (see scenes/); keyword arguments override the
    bal_scene_desc defaults (precision "fp64" or "mixed", warm_start, use_al,
    ccd_rule "printed", "half_gap" or "literal", broad_phase "hash" or "lbvh", sweep_cap, newton_rtol, pcg_rtol,
    max_newton, max_pcg, pcg_stall_window, max_contacts, warm_iters,
    sigma_fixed, friction, eps_v, accept_rtol, device, stream).
    """

    def __init__(self, sc, precision="fp64", **kw):
        d = bal_scene_desc()
        bal_desc_defaults(C.byref(d))
        self._keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return a

        rest = arr(sc["rest_pos"], np.float64)
        tets = arr(sc["tets"], np.int32)
        d.n_verts, d.n_tets = rest.shape[0], tets.shape[0]
        d.rest_pos = rest.ctypes.data_as(_dp)
        d.tets = tets.ctypes.data_as(_ip)
        d.youngs = arr(sc["youngs"], np.float64).ctypes.data_as(_dp)
        d.poisson = arr(sc["poisson"], np.float64).ctypes.data_as(_dp)
        d.density = arr(sc["density"], np.float64).ctypes.data_as(_dp)
        d.fixed = arr(sc["fixed"], np.uint8).ctypes.data_as(_up)
        obs = arr(np.asarray(sc["obs_pos"]).reshape(-1, 3), np.float64)
        otr = arr(np.asarray(sc["obs_tris"]).reshape(-1, 3), np.int32)
        d.n_obs_verts, d.n_obs_tris = obs.shape[0], otr.shape[0]
        d.obs_pos = obs.ctypes.data_as(_dp)
        d.obs_tris = otr.ctypes.data_as(_ip)
        d.x0 = arr(sc["x0"], np.float64).ctypes.data_as(_dp)
        d.v0 = arr(sc["v0"], np.float64).ctypes.data_as(_dp)
        d.dt = float(sc["dt"])
        for k in range(3):
            d.gravity[k] = float(sc["gravity"][k])
        d.dhat = float(sc["dhat"])
        d.precision = {"fp64": BAL_FP64, "mixed": BAL_MIXED}[precision]
        for k, v in kw.items():
            if k == "stream":
                d.stream = C.c_void_p(v)
            elif k in ("warm_start", "use_al"):
                setattr(d, k, int(bool(v)))
            elif k == "ccd_rule":
                d.ccd_rule = CCD_RULES[v] if isinstance(v, str) else int(v)
            elif k == "broad_phase":
                d.broad_phase = BROAD_PHASES[v] if isinstance(v, str) else int(v)
            else:
                setattr(d, k, v)
        self.desc = d
        self.n_verts = d.n_verts
        self.n_tets = d.n_tets
        self.n_all = d.n_verts + d.n_obs_verts
        h = C.c_void_p()
        _check(bal_create_scene(C.byref(d), C.byref(h)), "bal_create_scene")
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            bal_destroy_scene(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- stepping
    def step(self, allow=(BAL_OK,)):
        st = bal_step_stats()
        code = bal_step(self.h, C.byref(st))
        _check(code, "bal_step", ok=allow)
        out = st.as_dict()
        out["status"] = code
        return out

    def get_state(self):
        x = np.empty((self.n_verts, 3))
        v = np.empty((self.n_verts, 3))
        _check(bal_get_state(self.h, _ptr(x), _ptr(v), 0), "bal_get_state")
        return x, v

    def set_state(self, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        _check(bal_set_state(self.h, _ptr(x), _ptr(v), 0), "bal_set_state")

    def set_youngs(self, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        _check(bal_set_youngs(self.h, _ptr(E), 0), "bal_set_youngs")

    def trace(self):
        n = C.c_int32()
        _check(bal_get_trace(self.h, None, 0, C.byref(n)), "bal_get_trace")
        rows = np.zeros((max(n.value, 1), 8))
        _check(bal_get_trace(self.h, _ptr(rows), n.value, C.byref(n)), "bal_get_trace")
        return rows[: n.value]

    def set_kernel_timing(self, on=True):
        _check(bal_set_kernel_timing(self.h, int(on)), "bal_set_kernel_timing")

    # ---------------------------------------------------------- verification
    def surface(self):
        nv, nt, ne = C.c_int32(), C.c_int32(), C.c_int32()
        _check(bal_get_surface(self.h, C.byref(nv), None, C.byref(nt), None, C.byref(ne), None), "bal_get_surface")
        v = np.zeros(nv.value, np.int32)
        t = np.zeros((nt.value, 3), np.int32)
        e = np.zeros((ne.value, 2), np.int32)
        _check(bal_get_surface(self.h, C.byref(nv), _ptr(v), C.byref(nt), _ptr(t), C.byref(ne), _ptr(e)),
               "bal_get_surface")
        return v, t, e

    def linearize(self, x_all, sigma=0.0, aug_kind=None, aug_prims=None, mu=None, s=None, project=True):
        x_all = np.ascontiguousarray(x_all, dtype=np.float64)
        al = bal_al_state()
        al.sigma = float(sigma)
        keep = []
        if aug_kind is not None and len(aug_kind):
            k = np.ascontiguousarray(aug_kind, np.int32)
            p = np.ascontiguousarray(aug_prims, np.int32)
            m = np.ascontiguousarray(mu, np.float64)
            sl = np.ascontiguousarray(s, np.float64)
            keep += [k, p, m, sl]
            al.n_aug = k.shape[0]
            al.aug_kind = k.ctypes.data_as(_ip)
            al.aug_prims = p.ctypes.data_as(_ip)
            al.mu = m.ctypes.data_as(_dp)
            al.s = sl.ctypes.data_as(_dp)
        e = C.c_double()
        na = C.c_int32()
        g = np.zeros((self.n_all, 3))
        _check(bal_linearize(self.h, _ptr(x_all), C.byref(al), int(project), C.byref(e), _ptr(g), C.byref(na)),
               "bal_linearize")
        return e.value, g, na.value

    def hessian_apply(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.zeros((self.n_all, 3))
        _check(bal_hessian_apply(self.h, _ptr(v), _ptr(out)), "bal_hessian_apply")
        return out

    def stiffness(self):
        e = np.zeros(self.n_all)
        g = np.zeros(self.n_all, np.int32)
        _check(bal_get_stiffness(self.h, _ptr(e), _ptr(g)), "bal_get_stiffness")
        return e, g

    def solve(self, rhs, mode=0, rtol=1e-10, max_iters=20000):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        z = np.zeros((self.n_all, 3))
        it = C.c_int32()
        rel = C.c_double()
        _check(bal_solve(self.h, _ptr(rhs), _ptr(z), int(mode), float(rtol), int(max_iters), C.byref(it),
                         C.byref(rel)), "bal_solve", ok=(BAL_OK, BAL_E_NO_CONVERGENCE))
        return z, it.value, rel.value

    def ccd_bound(self, x_all, p_all):
        x_all = np.ascontiguousarray(x_all, dtype=np.float64)
        p_all = np.ascontiguousarray(p_all, dtype=np.float64)
        a = C.c_double()
        _check(bal_ccd_bound(self.h, _ptr(x_all), _ptr(p_all), C.byref(a)), "bal_ccd_bound")
        return a.value

    def candidates(self, x_all, p_all=None):
        x_all = np.ascontiguousarray(x_all, dtype=np.float64)
        p_all = None if p_all is None else np.ascontiguousarray(p_all, dtype=np.float64)
        n = C.c_int32()
        _check(bal_candidates(self.h, _ptr(x_all), _ptr(p_all), 0, None, None, None, C.byref(n)), "bal_candidates")
        m = n.value
        kind = np.zeros(max(m, 1), np.int32)
        nodes = np.zeros((max(m, 1), 4), np.int32)
        dist = np.zeros(max(m, 1))
        _check(bal_candidates(self.h, _ptr(x_all), _ptr(p_all), m, _ptr(kind), _ptr(nodes), _ptr(dist), C.byref(n)),
               "bal_candidates")
        return kind[:m], nodes[:m], dist[:m]

    def spmv_benchmark(self, reps=50):
        ms = C.c_double()
        by = C.c_double()
        _check(bal_spmv_benchmark(self.h, int(reps), C.byref(ms), C.byref(by)), "bal_spmv_benchmark")
        return ms.value, by.value

    def step_adjoint(self, x_t, v_t, gx_next, gv_next, gE_accum):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x_t, v_t, gx_next, gv_next)]
        gx = np.zeros((self.n_verts, 3))
        gv = np.zeros((self.n_verts, 3))
        st = bal_step_stats()
        _check(bal_step_adjoint(self.h, *[_ptr(a) for a in arrs], _ptr(gx), _ptr(gv), _ptr(gE_accum), 0,
                                C.byref(st)), "bal_step_adjoint")
        return gx, gv


def _make_rollout():
    import torch

    class BalRollout(torch.autograd.Function):
        """x_T = rollout(E, v0): T backward-Euler BAL steps from (x0, v0) with per-tet E.

        forward(E [n_tets], v0 [n_verts, 3], scene, x0 [n_verts, 3], n_steps, every)
        keeps (x_t, v_t) every `every` steps; backward re-runs each segment
        from its checkpoint and walks it in reverse through bal_step_adjoint.
        Gradients flow to E and v0 (float64 tensors).  A step that does not
        converge, in either pass, raises BalError: the gradient is that of the
        converged step map only.
        """

        @staticmethod
        def forward(ctx, E, v0, scene, x0, n_steps, every=5):
            Ed = E.detach().cpu().numpy().astype(np.float64)
            x = np.asarray(x0, dtype=np.float64).copy()
            v = v0.detach().cpu().numpy().astype(np.float64).copy()
            scene.set_youngs(Ed)
            scene.set_state(x, v)
            ckpt = {}
            for t in range(n_steps):
                if t % every == 0:
                    ckpt[t] = scene.get_state()
                scene.step()
            xT, vT = scene.get_state()
            ctx.scene, ctx.ckpt, ctx.n_steps, ctx.every, ctx.Ed = scene, ckpt, n_steps, every, Ed
            return torch.from_numpy(xT).to(v0.device)

        @staticmethod
        def backward(ctx, gxT):
            scene = ctx.scene
            scene.set_youngs(ctx.Ed)
            gx = gxT.detach().cpu().numpy().astype(np.float64).copy()
            gv = np.zeros_like(gx)
            gE = np.zeros(scene.n_tets)
            starts = sorted(ctx.ckpt.keys())
            for s0 in reversed(starts):
                s1 = min(s0 + ctx.every, ctx.n_steps)
                xs, vs = ctx.ckpt[s0]
                states = []
                scene.set_state(xs, vs)
                for _ in range(s0, s1):
                    states.append(scene.get_state())
                    scene.step()
                for t in reversed(range(s1 - s0)):
                    x_t, v_t = states[t]
                    gx, gv = scene.step_adjoint(x_t, v_t, gx, gv, gE)
            import torch
            return (torch.from_numpy(gE), torch.from_numpy(gv), None, None, None, None)

    return BalRollout


def __getattr__(name):
    if name == "BalRollout":
        return _make_rollout()
    raise AttributeError(name)
