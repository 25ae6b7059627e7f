"""Plain CPU FP64 oracle of one barrier-augmented Lagrangian (BAL) time step.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the GPU library shares no code with
this module and never imports it.

What it computes (Guo et al., "Barrier-Augmented Lagrangian for GPU-based
Elastodynamic Contact"):

* backward Euler as minimisation of the incremental potential
  E(x) = 1/(2h^2) ||x - y||_M^2 + Psi(x), y = x_t + h v_t + h^2 g
  (Sec. 3.1, problem definition and eq. problem);
* the IPC log barrier b(d, dhat) (eq. IPC-barrier) on point-triangle and
  edge-edge pairs, and the BAL objective
  L = E + sigma sum_A b(d_i, dhat) + sum_A' [mu_i (dhat + s_i - d_i) + sigma b(d_i, dhat + s_i)]
  (eq. aug-lag);
* Algorithm 1 (BAL method) with the sigma^0 least-squares initialisation and
  the sigma growth rule (Sec. 3.4), one inexact-Newton iteration per loop
  pass: projected Hessian (Sec. 4.2, stencil-wise eigen-projection), a
  direct linear solve in place of PCG, a CCD step bound (Sec. 5.3 narrow
  phase, conservative TOI) and a backtracking line search (Sec. 5.2);
* the assembled-eigenvalue stiffness Lambda and the log10 stiffness groups
  (Sec. 4.2), used to pin the warm start;
* the adjoint of a converged step (not in the paper: frozen-state implicit
  differentiation of the stationarity condition).

Method of computation, chosen to be obviously correct rather than fast:
every stencil energy is written once as its plain definition in PyTorch
(CPU, float64) and differentiated by autograd; projections clamp the
eigenvalues from numpy's symmetric eigensolver; linear systems are solved
by dense Cholesky or SuperLU; contact pairs are enumerated by brute force
(or, for large scenes, a k-d-tree superset of them); cubic roots are
isolated between the derivative's roots and refined by bisection.

Readings of points where the paper is silent or garbled are listed in the
repository's design notes and marked "reading" below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg
import torch

DT = torch.float64

# ----------------------------------------------------------------------------
# Distance cases.  A pair stencil has 4 nodes: PT = (p, a, b, c) and
# EE = (a0, a1, b0, b1).  Each case names the stencil nodes its distance
# depends on (reading: closest-point region classification, first minimum
# wins on ties, parallel edges fall back to the point-edge minimum).
# ----------------------------------------------------------------------------
PP, PE, PTK, EEK = 0, 1, 2, 3
CASE_NODES = {
    0: (0, 1, 2, 3), 1: (0, 1, 2), 2: (0, 2, 3), 3: (0, 3, 1), 4: (0, 1), 5: (0, 2), 6: (0, 3),
    7: (0, 1, 2, 3), 8: (0, 2, 3), 9: (1, 2, 3), 10: (2, 0, 1), 11: (3, 0, 1),
    12: (0, 2), 13: (0, 3), 14: (1, 2), 15: (1, 3),
}
CASE_KIND = {0: PTK, 1: PE, 2: PE, 3: PE, 4: PP, 5: PP, 6: PP, 7: EEK, 8: PE, 9: PE,
             10: PE, 11: PE, 12: PP, 13: PP, 14: PP, 15: PP}
PARALLEL_EPS = 1e-12   # ||e1 x e2||^2 < eps ||e1||^2 ||e2||^2 => parallel edges (sin < 1e-6)
CCD_EPS = 1e-12        # root interval [-eps, 1+eps] and activation d_TOC < eps + dhat
COPLANAR_ULPS = 32.0   # start frame coplanar: |det| <= 32 u max|x| (|u||v| + |v||w| + |w||u|)


def _dz_sign(v):
    """Sign with a dead zone of the CCD epsilon (reading: |sd| <= eps counts as touching)."""
    return 0 if abs(v) <= CCD_EPS else (1 if v > 0 else -1)


def _dot(a, b):
    return np.einsum("...i,...i->...", a, b)


def point_segment_sq(p, a, b):
    """Squared point-segment distance and region (0: at a, 1: interior, 2: at b)."""
    e = b - a
    t = _dot(p - a, e) / _dot(e, e)
    q_a = _dot(p - a, p - a)
    q_b = _dot(p - b, p - b)
    c = np.cross(p - a, e)
    q_e = _dot(c, c) / _dot(e, e)
    region = np.where(t <= 0.0, 0, np.where(t >= 1.0, 2, 1))
    q = np.where(region == 0, q_a, np.where(region == 2, q_b, q_e))
    return q, region


def classify_pt(P, A, B, C):
    """Squared distance and case id of point-triangle pairs (cases 0-6)."""
    e1, e2, r = B - A, C - A, P - A
    a11, a12, a22 = _dot(e1, e1), _dot(e1, e2), _dot(e2, e2)
    b1, b2 = _dot(e1, r), _dot(e2, r)
    det = a11 * a22 - a12 * a12
    beta1 = (a22 * b1 - a12 * b2) / det
    beta2 = (a11 * b2 - a12 * b1) / det
    inside = (beta1 >= 0) & (beta2 >= 0) & (beta1 + beta2 <= 1)
    n = np.cross(e1, e2)
    q_in = _dot(r, n) ** 2 / _dot(n, n)
    # the three edges (a,b), (b,c), (c,a); region -> case id
    q1, g1 = point_segment_sq(P, A, B)
    q2, g2 = point_segment_sq(P, B, C)
    q3, g3 = point_segment_sq(P, C, A)
    c1 = np.choose(g1, [4, 1, 5])
    c2 = np.choose(g2, [5, 2, 6])
    c3 = np.choose(g3, [6, 3, 4])
    qs = np.stack([q1, q2, q3], -1)
    cs = np.stack([c1, c2, c3], -1)
    k = np.argmin(qs, axis=-1)
    q_out = np.take_along_axis(qs, k[..., None], -1)[..., 0]
    c_out = np.take_along_axis(cs, k[..., None], -1)[..., 0]
    return np.where(inside, q_in, q_out), np.where(inside, 0, c_out)


def classify_ee(A0, A1, B0, B1):
    """Squared distance and case id of edge-edge pairs (cases 7-15)."""
    e1, e2, w = A1 - A0, B1 - B0, A0 - B0
    n = np.cross(e1, e2)
    nn = _dot(n, n)
    a, b, c = _dot(e1, e1), _dot(e1, e2), _dot(e2, e2)
    d, e = _dot(e1, w), _dot(e2, w)
    parallel = nn < PARALLEL_EPS * a * c
    # a c - b^2 = |e1 x e2|^2 (Lagrange identity); the cross-product form has no cancellation
    den = np.where(parallel, 1.0, nn)
    s = (b * e - c * d) / den
    t = (a * e - b * d) / den
    interior = (~parallel) & (s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)
    q_in = _dot(w, n) ** 2 / np.where(parallel, 1.0, nn)
    qa0, ga0 = point_segment_sq(A0, B0, B1)
    qa1, ga1 = point_segment_sq(A1, B0, B1)
    qb0, gb0 = point_segment_sq(B0, A0, A1)
    qb1, gb1 = point_segment_sq(B1, A0, A1)
    cs = np.stack([np.choose(ga0, [12, 8, 13]), np.choose(ga1, [14, 9, 15]),
                   np.choose(gb0, [12, 10, 14]), np.choose(gb1, [13, 11, 15])], -1)
    qs = np.stack([qa0, qa1, qb0, qb1], -1)
    k = np.argmin(qs, axis=-1)
    q_out = np.take_along_axis(qs, k[..., None], -1)[..., 0]
    c_out = np.take_along_axis(cs, k[..., None], -1)[..., 0]
    return np.where(interior, q_in, q_out), np.where(interior, 7, c_out)


def classify(kind, X4):
    """Squared distance and case for pairs of given kind (0 PT, 1 EE); X4 (K,4,3)."""
    q = np.empty(X4.shape[0])
    case = np.empty(X4.shape[0], dtype=np.int64)
    m = kind == 0
    if m.any():
        q[m], case[m] = classify_pt(X4[m, 0], X4[m, 1], X4[m, 2], X4[m, 3])
    m = kind == 1
    if m.any():
        q[m], case[m] = classify_ee(X4[m, 0], X4[m, 1], X4[m, 2], X4[m, 3])
    return q, case


def q_case_torch(case, X):
    """Squared distance of one case as a torch function of the 4 stencil nodes X (4,3)."""
    k = CASE_KIND[case]
    nd = CASE_NODES[case]
    if k == PP:
        r = X[nd[0]] - X[nd[1]]
        return (r * r).sum()
    if k == PE:
        p, a, b = X[nd[0]], X[nd[1]], X[nd[2]]
        e = b - a
        c = torch.linalg.cross(p - a, e)
        return (c * c).sum() / (e * e).sum()
    if k == PTK:
        p, a, b, c = X[0], X[1], X[2], X[3]
        n = torch.linalg.cross(b - a, c - a)
        return ((p - a) * n).sum() ** 2 / (n * n).sum()
    a0, a1, b0, b1 = X[0], X[1], X[2], X[3]
    n = torch.linalg.cross(a1 - a0, b1 - b0)
    return ((a0 - b0) * n).sum() ** 2 / (n * n).sum()


# ----------------------------------------------------------------------------
# Barrier (eq. IPC-barrier) and the Neo-Hookean energy density.
# ----------------------------------------------------------------------------
def barrier_np(d, dh):
    """b(d, dh) = -(d - dh)^2 log(d / dh) on 0 < d < dh, 0 for d >= dh, +inf for d <= 0."""
    d = np.asarray(d, dtype=np.float64)
    dh = np.broadcast_to(np.asarray(dh, dtype=np.float64), d.shape)
    out = np.zeros_like(d)
    inside = (d > 0) & (d < dh)
    out[inside] = -(d[inside] - dh[inside]) ** 2 * np.log(d[inside] / dh[inside])
    out[d <= 0] = np.inf
    return out


def barrier_torch(d, dh):
    inside = d < dh
    safe = torch.where(inside, d, dh)
    return torch.where(inside, -(safe - dh) ** 2 * torch.log(safe / dh), torch.zeros_like(d))


def barrier_d1_np(d, dh):
    """db/dd = -2 (d - dh) log(d / dh) - (d - dh)^2 / d on 0 < d < dh, 0 for d >= dh."""
    d = np.asarray(d, dtype=np.float64)
    dh = np.broadcast_to(np.asarray(dh, dtype=np.float64), d.shape)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dh)
    out[m] = -2.0 * (d[m] - dh[m]) * np.log(d[m] / dh[m]) - (d[m] - dh[m]) ** 2 / d[m]
    return out


def friction_f_torch(q, eps_h):
    """The friction mollifier f of Sec. 4.1 as a function of q = y^2, y the
    tangential relative displacement of the step:
    f(y) = -y^3 / (3 eps_v^2 h^2) + y^2 / (eps_v h) for y < eps_v h, and
    f(y) = y - eps_v h / 3 beyond (reading: the paper prints the mollified
    branch only; this is its C1 continuation, whose slope is 1, the kinetic
    regime).  Written in q so that autograd is exact at q = 0 (the y^3 term
    and its first two derivatives vanish there)."""
    small = q < eps_h * eps_h
    qs = torch.where(q > 0, q, torch.ones_like(q))
    y3 = torch.where(q > 0, qs ** 1.5, torch.zeros_like(q))
    inner = -y3 / (3.0 * eps_h * eps_h) + q / eps_h
    ql = torch.where(small, torch.full_like(q, eps_h * eps_h), q)
    outer = torch.sqrt(ql) - eps_h / 3.0
    return torch.where(small, inner, outer)


def closest_coeffs(case, X4):
    """beta (K,4): weights of the 4 stencil nodes such that sum_k beta_k X_k is
    the vector between the two closest points of each pair's distance case
    (zero on nodes the case does not use); the parameters come from the
    case's own closest-point problem (point-edge: segment parameter; point-
    triangle: barycentrics of the projection; edge-edge: the line-line
    parameters)."""
    K = X4.shape[0]
    beta = np.zeros((K, 4))
    for i in range(K):
        c = int(case[i])
        nd = CASE_NODES[c]
        k = CASE_KIND[c]
        X = X4[i]
        if k == PP:
            beta[i, nd[0]], beta[i, nd[1]] = 1.0, -1.0
        elif k == PE:
            p, a, b = X[nd[0]], X[nd[1]], X[nd[2]]
            t = float(np.dot(p - a, b - a) / np.dot(b - a, b - a))
            beta[i, nd[0]], beta[i, nd[1]], beta[i, nd[2]] = 1.0, -(1.0 - t), -t
        elif k == PTK:
            p, a, b, cc = X
            e1, e2 = b - a, cc - a
            G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
            u, v = np.linalg.solve(G, [np.dot(p - a, e1), np.dot(p - a, e2)])
            beta[i] = (1.0, -(1.0 - u - v), -u, -v)
        else:
            a0, a1, b0, b1 = X
            e1, e2, r = a1 - a0, b1 - b0, a0 - b0
            G = np.array([[e1 @ e1, -(e1 @ e2)], [-(e1 @ e2), e2 @ e2]])
            sa, sb = np.linalg.solve(G, [-(e1 @ r), e2 @ r])
            beta[i] = (1.0 - sa, sa, -(1.0 - sb), -sb)
    return beta


def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def nh_density_torch(F, mu, lam):
    """Compressible Neo-Hookean density mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2.

    Reading: the paper names the model only; this is the classic form.
    J is the triple product of F's columns.
    """
    J = (F[..., :, 0] * torch.linalg.cross(F[..., :, 1], F[..., :, 2])).sum(-1)
    I1 = (F * F).sum((-1, -2))
    lj = torch.log(J)
    return 0.5 * mu * (I1 - 3.0) - mu * lj + 0.5 * lam * lj * lj


def _tet_energy_single(x12, Dminv, vol, mu, lam):
    X = x12.reshape(4, 3)
    Ds = torch.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], dim=1)
    F = Ds @ Dminv
    return vol * nh_density_torch(F, mu, lam)


def project_psd(H):
    """Closest PSD matrix (Frobenius) of each symmetric H (..., n, n): clamp eigenvalues at 0."""
    H = 0.5 * (H + np.swapaxes(H, -1, -2))
    w, V = np.linalg.eigh(H)
    w = np.maximum(w, 0.0)
    return np.einsum("...ij,...j,...kj->...ik", V, w, V)


# ----------------------------------------------------------------------------
# Pair sets
# ----------------------------------------------------------------------------
@dataclass
class Pairs:
    """A set of contact pairs: kind (0 PT, 1 EE), primitive ids and stencil nodes."""
    kind: np.ndarray
    a: np.ndarray
    b: np.ndarray
    nodes: np.ndarray

    @staticmethod
    def empty():
        z = np.zeros(0, dtype=np.int64)
        return Pairs(z, z, z, np.zeros((0, 4), dtype=np.int64))

    def __len__(self):
        return int(self.kind.shape[0])

    def take(self, idx):
        return Pairs(self.kind[idx], self.a[idx], self.b[idx], self.nodes[idx])

    def keys(self):
        """Canonical integer key per pair: (kind, primitive a, primitive b)."""
        return (self.kind.astype(np.int64) << 60) | (self.a.astype(np.int64) << 30) | self.b.astype(np.int64)


@dataclass
class Frames:
    """Friction frames of one Newton iteration (Sec. 4.1): for each pair with
    a positive normal force at the iterate, that force's magnitude lam, the
    closest-point weights beta (K,4) and the contact normal n (K,3), held
    constant while the friction potential is differentiated and during the
    line search; x_t are the positions at the start of the time step."""
    pairs: Pairs
    lam: np.ndarray
    beta: np.ndarray
    n: np.ndarray
    x_t: np.ndarray
    chi: float
    eps_h: float


@dataclass
class ALState:
    """BAL state of one time step (Alg. 1): sigma, sigma0 and the set A' with
    mu, s; plus the friction frames of the current iterate (None: no friction)."""
    sigma: float | None = None
    sigma0: float | None = None
    aug: Pairs = field(default_factory=Pairs.empty)
    mu: np.ndarray = field(default_factory=lambda: np.zeros(0))
    s: np.ndarray = field(default_factory=lambda: np.zeros(0))
    frames: Frames | None = None

    def copy(self):
        return ALState(self.sigma, self.sigma0, self.aug, self.mu.copy(), self.s.copy(), self.frames)


@dataclass
class Params:
    newton_rtol: float = 1e-4     # ||e^l|| <= rtol ||e^0|| (Alg. 1 convergence test)
    max_newton: int = 1000        # reading: the paper states no cap
    max_contacts: int = 1 << 40   # memory-limit halving (Sec. 5.2)
    use_al: bool = True           # False: plain barrier (no A')
    min_alpha: float = 1e-9       # line-search floor (App. B)
    pair_mode: str = "brute"      # "brute" or "kdtree" (superset for large scenes)
    verbose: bool = False         # print one line per phase of each Newton iteration
    sigma_fixed: float = 0.0      # > 0: sigma held at this value (no sigma^0, no growth)
    ccd_rule: str = "printed"     # "printed" (Sec. 5.3), "half_gap" (departure) or "literal"; see ccd
    sweep_cap: float = 0.0        # > 0 (departure): CCD sweep halved while a vertex moves
                                  # more than sweep_cap mean surface edge lengths
    friction: float = 0.0         # chi (Sec. 4.1); 0: frictionless
    eps_v: float = 0.0            # mollifier threshold eps_v; <= 0: dhat
    accept_rtol: float = 0.0      # > 0: a stalled step (no measurable move) with |e| <= accept_rtol |e0|
                                  # counts as converged (the energy's FP64 rounding floor)


# ----------------------------------------------------------------------------
# Algorithm 1's bookkeeping, as functions of plain arrays.
# ----------------------------------------------------------------------------
def rebuild_aug_set(pairs: Pairs, d, min_d, prev_min, st: "ALState", dhat):
    """Alg. 1 lines 3-6 (reading: "current iterate vs previous iterate").

    Returns (aug, mu, s): A' emptied when min d exceeds 1e-2 dhat; rebuilt as
    the pairs of `pairs` with d < 1e-2 dhat when min d decreased or A' is
    empty (a pair kept across a rebuild keeps its mu and s, a new one starts
    at 0; reading); otherwise unchanged.
    """
    if min_d > 1e-2 * dhat:
        return Pairs.empty(), np.zeros(0), np.zeros(0)
    if not (min_d < prev_min or len(st.aug) == 0):
        return st.aug, st.mu, st.s
    new = pairs.take(np.nonzero(np.asarray(d) < 1e-2 * dhat)[0])
    mu = np.zeros(len(new))
    sl = np.zeros(len(new))
    if len(st.aug):
        pos = {k: i for i, k in enumerate(st.aug.keys())}
        for i, k in enumerate(new.keys()):
            j = pos.get(k)
            if j is not None:
                mu[i], sl[i] = st.mu[j], st.s[j]
    return new, mu, sl


def slack_update(mu, d, sigma, dhat):
    """Slack of each A' pair: the minimiser over s >= 0 of
    mu (dhat + s - d) + sigma/2 (dhat + s - d)^2 (eq. problem-s), in closed form."""
    return np.maximum(-np.asarray(mu) / sigma - dhat + np.asarray(d), 0.0)


def dual_update(mu, d, sigma, dhat):
    """Alg. 1 lines 12-14 for every pair of A' at distances d (at x^{l+1}):
    first s_i, then mu_i += sigma b(d_i, dhat + s_i) with the new s_i.
    Returns (mu_new, s_new)."""
    sl = slack_update(mu, d, sigma, dhat)
    return np.asarray(mu) + sigma * barrier_np(d, dhat + sl), sl


def sigma_update(sigma, sigma0, min_d_new, dhat):
    """Alg. 1 lines 15-17: sigma <- max(1.2 sigma, 100 sigma^0) when min d < 1e-2 dhat."""
    if min_d_new < 1e-2 * dhat:
        return max(1.2 * sigma, 100.0 * sigma0)
    return sigma


def line_search(alpha_max, L0, trial, min_alpha=1e-9):
    """Backtracking from alpha_max (Sec. 5.2; reading: plain non-increase).

    trial(alpha) -> (L, feasible, within_capacity).  alpha halves until
    L <= L0 at a feasible trial point (every J > 0 and d > 0) whose active
    count is within the memory limit; below min_alpha the search fails and
    returns 0.
    """
    alpha = alpha_max
    while alpha >= min_alpha:
        L, ok, cap = trial(alpha)
        if ok and cap and L <= L0:
            return alpha
        alpha *= 0.5
    return 0.0


class OracleScene:
    """Scene preprocessing (rest shape, masses, surface, pairs) and the BAL step."""

    def __init__(self, sc, params: Params | None = None):
        self.p = params or Params()
        X = np.asarray(sc["rest_pos"], dtype=np.float64)
        T = np.asarray(sc["tets"], dtype=np.int64)
        n = X.shape[0]
        obs = np.asarray(sc["obs_pos"], dtype=np.float64).reshape(-1, 3)
        m = obs.shape[0]
        self.n_body, self.n_obs, self.N = n, m, n + m
        self.tets = T
        Dm = np.stack([X[T[:, k]] - X[T[:, 0]] for k in (1, 2, 3)], axis=2)
        self.vol = np.linalg.det(Dm) / 6.0
        if not (self.vol > 0).all():
            raise ValueError("inverted or degenerate rest tetrahedron")
        self.Dm_inv = np.linalg.inv(Dm)
        self.E = np.asarray(sc["youngs"], dtype=np.float64).copy()
        self.nu = np.asarray(sc["poisson"], dtype=np.float64)
        self.rho = np.asarray(sc["density"], dtype=np.float64)
        # lumped mass: each tet gives a quarter of rho V to each of its nodes (Sec. 3.1)
        self.mass = np.zeros(self.N)
        for a in range(4):
            np.add.at(self.mass, T[:, a], self.rho * self.vol / 4.0)
        fixed = np.asarray(sc["fixed"]).astype(bool) if sc.get("fixed") is not None else np.zeros(n, bool)
        self.free = np.zeros(self.N, dtype=bool)
        self.free[:n] = ~fixed
        self.free_idx = np.nonzero(self.free)[0]
        self.dof_of = -np.ones(self.N, dtype=np.int64)
        self.dof_of[self.free_idx] = np.arange(self.free_idx.size)
        self.ndof = 3 * self.free_idx.size
        self.h = float(sc["dt"])
        self.dhat = float(sc["dhat"])
        self.g = np.asarray(sc["gravity"], dtype=np.float64)
        self.x = np.concatenate([np.asarray(sc["x0"], dtype=np.float64), obs])
        self.v = np.concatenate([np.asarray(sc["v0"], dtype=np.float64), np.zeros((m, 3))])
        self.v[~self.free] = 0.0
        self._surface(T, np.asarray(sc["obs_tris"], dtype=np.int64).reshape(-1, 3))
        # unit of the optional sweep cap: the mean body surface edge length at rest (at least 4 dhat)
        be = self.s_edges[(self.s_edges < n).all(1)]
        mean_edge = float(np.linalg.norm(X[be[:, 0]] - X[be[:, 1]], axis=1).mean()) if len(be) else 1.0
        self.mean_edge = max(mean_edge, 4.0 * self.dhat)
        self._t_dminv = torch.tensor(self.Dm_inv, dtype=DT)
        self._t_vol = torch.tensor(self.vol, dtype=DT)
        self._set_material()

    def _set_material(self):
        mu, lam = lame(self.E, self.nu)
        self.mu_l, self.lam_l = mu, lam
        self._t_mu = torch.tensor(mu, dtype=DT)
        self._t_lam = torch.tensor(lam, dtype=DT)

    def set_youngs(self, E):
        self.E = np.asarray(E, dtype=np.float64).copy()
        self._set_material()

    # ---------------------------------------------------------------- surface
    def _surface(self, T, obs_tris):
        faces = np.concatenate([T[:, [1, 2, 3]], T[:, [0, 2, 3]], T[:, [0, 1, 3]], T[:, [0, 1, 2]]])
        key = np.sort(faces, axis=1)
        uniq, cnt = np.unique(key, axis=0, return_counts=True)
        body_tris = uniq[cnt == 1]
        tris = np.concatenate([body_tris, obs_tris + self.n_body]) if obs_tris.size else body_tris
        edges = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]])
        edges = np.unique(np.sort(edges, axis=1), axis=0)
        verts = np.unique(np.concatenate([body_tris.ravel(), np.arange(self.n_body, self.N)]))
        self.s_tris, self.s_edges, self.s_verts = tris, edges, verts
        self.is_obs = np.zeros(self.N, dtype=bool)
        self.is_obs[self.n_body:] = True

    def _filter_pairs(self, kind, a, b, nodes):
        """Drop incident pairs, obstacle-only pairs and pairs with no free node (reading)."""
        incident = np.zeros(len(kind), dtype=bool)
        if len(kind):
            if (kind == 0).any():
                pt = kind == 0
                nd = nodes[pt]
                incident[pt] = (nd[:, 0:1] == nd[:, 1:]).any(1)
            if (kind == 1).any():
                ee = kind == 1
                nd = nodes[ee]
                incident[ee] = (nd[:, :2, None] == nd[:, None, 2:]).reshape(-1, 4).any(1)
        obs_only = self.is_obs[nodes].all(1) if len(kind) else incident
        # PT pairs whose point and triangle both lie on obstacles, EE pairs of two obstacle edges
        if len(kind):
            pt = kind == 0
            obs_only = np.where(pt, self.is_obs[nodes[:, 0]] & self.is_obs[nodes[:, 1]],
                                self.is_obs[nodes[:, 0]] & self.is_obs[nodes[:, 2]])
            no_free = ~self.free[nodes].any(1)
        else:
            no_free = incident
        keep = ~(incident | obs_only | no_free)
        return Pairs(kind[keep], a[keep], b[keep], nodes[keep])

    def all_pairs(self):
        """Brute-force pair set: every surface vertex x triangle and edge x edge pair."""
        V, Tr, Ed = self.s_verts, self.s_tris, self.s_edges
        vi, ti = np.meshgrid(np.arange(V.size), np.arange(Tr.shape[0]), indexing="ij")
        vi, ti = vi.ravel(), ti.ravel()
        pt_nodes = np.concatenate([V[vi][:, None], Tr[ti]], axis=1)
        ei, ej = np.triu_indices(Ed.shape[0], k=1)
        ee_nodes = np.concatenate([Ed[ei], Ed[ej]], axis=1)
        kind = np.concatenate([np.zeros(vi.size, np.int64), np.ones(ei.size, np.int64)])
        a = np.concatenate([V[vi], ei])
        b = np.concatenate([ti, ej])
        return self._filter_pairs(kind, a, b, np.concatenate([pt_nodes, ee_nodes]))

    def near_pairs(self, x, reach):
        """Superset of all pairs whose distance at x is below `reach`.

        Bounding spheres: a point is within `reach` of a triangle only if it
        lies within r_t + reach of the triangle's centroid (r_t = centroid to
        farthest vertex); two edges only if their midpoints are within
        r_1 + r_2 + reach.  Searched with k-d trees; the few edges much longer
        than the rest (large obstacle faces) are tested against every edge.
        """
        from scipy.spatial import cKDTree
        V, Tr, Ed = self.s_verts, self.s_tris, self.s_edges
        tc = x[Tr].mean(1)
        trad = np.linalg.norm(x[Tr] - tc[:, None], axis=2).max(1)
        vtree = cKDTree(x[V])
        lst = vtree.query_ball_point(tc, trad + reach)
        ti = np.repeat(np.arange(Tr.shape[0]), [len(l) for l in lst])
        vi = np.fromiter((j for l in lst for j in l), dtype=np.int64, count=ti.size)
        out = [(np.zeros(vi.size, np.int64), V[vi], ti, np.concatenate([V[vi][:, None], Tr[ti]], axis=1))]
        ec = x[Ed].mean(1)
        erad = 0.5 * np.linalg.norm(x[Ed[:, 1]] - x[Ed[:, 0]], axis=1)
        big = erad > 10.0 * np.median(erad)
        small = np.nonzero(~big)[0]
        rmax = erad[small].max() if small.size else 0.0
        etree = cKDTree(ec[small])
        lst = etree.query_ball_point(ec[small], erad[small] + rmax + reach)
        a = np.repeat(small, [len(l) for l in lst])
        b = small[np.fromiter((j for l in lst for j in l), dtype=np.int64, count=a.size)]
        keep = (a < b) & (np.linalg.norm(ec[a] - ec[b], axis=1) <= erad[a] + erad[b] + reach)
        pairs = [np.stack([a[keep], b[keep]], 1)]
        for e in np.nonzero(big)[0]:
            o = np.arange(Ed.shape[0])
            near = (o != e) & (np.linalg.norm(ec - ec[e], axis=1) <= erad + erad[e] + reach)
            o = o[near]
            pairs.append(np.stack([np.minimum(o, e), np.maximum(o, e)], 1))
        ij = np.unique(np.concatenate(pairs), axis=0) if pairs else np.zeros((0, 2), np.int64)
        out.append((np.ones(ij.shape[0], np.int64), ij[:, 0], ij[:, 1],
                    np.concatenate([Ed[ij[:, 0]], Ed[ij[:, 1]]], axis=1)))
        kind, pa, pb, nodes = (np.concatenate(z) for z in zip(*out))
        order = np.lexsort((pb, pa, kind))
        return self._filter_pairs(kind[order], pa[order], pb[order], nodes.reshape(-1, 4)[order])

    def candidate_pairs(self, x, disp=None):
        if self.p.pair_mode == "brute":
            if not hasattr(self, "_all_pairs"):
                self._all_pairs = self.all_pairs()
            return self._all_pairs
        reach = self.dhat * 1.01
        if disp is not None:
            reach += 2.0 * np.linalg.norm(disp, axis=1).max()
        return self.near_pairs(x, reach)

    # ----------------------------------------------------------- distances
    def distances(self, x, pairs: Pairs):
        q, case = classify(pairs.kind, x[pairs.nodes])
        return np.sqrt(q), case

    # -------------------------------------------------------------- energies
    def predictor(self, x_t, v_t):
        y = x_t + self.h * v_t + self.h * self.h * self.g
        y[~self.free] = x_t[~self.free]
        return y

    def _contact_energy_torch(self, xt, pairs, case, d_sel_mask, sigma, mu, s, aug_mask):
        """Sum of contact terms of `pairs` at torch positions xt (N,3)."""
        if len(pairs) == 0:
            return xt.sum() * 0.0
        X4 = xt[torch.as_tensor(pairs.nodes)]
        tot = xt.sum() * 0.0
        for c in np.unique(case):
            sel = np.nonzero(case == c)[0]
            qf = torch.vmap(lambda X: q_case_torch(int(c), X))
            d = torch.sqrt(qf(X4[sel]))
            e = sigma * barrier_torch(d, torch.full_like(d, self.dhat)) * torch.as_tensor(d_sel_mask[sel], dtype=DT)
            am = aug_mask[sel]
            if am.any():
                mu_t = torch.as_tensor(mu[sel], dtype=DT)
                s_t = torch.as_tensor(s[sel], dtype=DT)
                aug_e = mu_t * (self.dhat + s_t - d) + sigma * barrier_torch(d, self.dhat + s_t)
                e = e + aug_e * torch.as_tensor(am, dtype=DT)
            tot = tot + e.sum()
        return tot

    def _merge_pairs(self, pairs: Pairs, st: ALState):
        """Union of candidate pairs and A' pairs, with mu, s, A' mask aligned."""
        keys = pairs.keys()
        akeys = st.aug.keys()
        missing = ~np.isin(akeys, keys)
        allp = Pairs(*(np.concatenate([u, v]) for u, v in
                       zip((pairs.kind, pairs.a, pairs.b, pairs.nodes),
                           (st.aug.kind[missing], st.aug.a[missing], st.aug.b[missing], st.aug.nodes[missing]))))
        allkeys = allp.keys()
        mu = np.zeros(len(allp))
        s = np.zeros(len(allp))
        aug = np.zeros(len(allp), dtype=bool)
        if len(st.aug):
            pos = {k: i for i, k in enumerate(allkeys)}
            idx = np.array([pos[k] for k in akeys], dtype=np.int64)
            mu[idx], s[idx], aug[idx] = st.mu, st.s, True
        return allp, mu, s, aug

    def lagrangian(self, x, y, pairs: Pairs, st: ALState, with_grad=False, parts=False):
        """BAL objective L_sigma (eq. aug-lag) at x; +inf if any J <= 0 or d <= 0.

        Barrier terms run over the given candidate pairs (their support is
        d < dhat, so any superset of the active set gives the same value);
        augmentation terms run over A'.
        """
        allp, mu, s, aug = self._merge_pairs(pairs, st)
        d, case = self.distances(x, allp)
        if (d <= 0).any():
            return (np.inf, None) if with_grad else np.inf
        xt = torch.tensor(x, dtype=DT, requires_grad=with_grad)
        terms = self._objective_terms(xt, y, allp, case, d, st, mu, s, aug)
        if terms is None:
            return (np.inf, None) if with_grad else np.inf
        inertia, elastic, contact = terms
        total = inertia + elastic + contact
        if parts:
            return dict(inertia=float(inertia), elastic=float(elastic), contact=float(contact))
        if not with_grad:
            return float(total)
        total.backward()
        return float(total.detach()), xt.grad.numpy().copy()

    def _objective_terms(self, xt, y, allp, case, d, st, mu, s, aug):
        """Inertia, elastic and contact parts of L_sigma at torch positions xt
        (None if a tet is inverted)."""
        sigma = st.sigma if st.sigma is not None else 0.0
        free = torch.as_tensor(self.free)
        mass = torch.tensor(self.mass, dtype=DT)
        yt = torch.tensor(y, dtype=DT)
        diff = (xt - yt)[free]
        inertia = 0.5 / self.h ** 2 * (mass[free][:, None] * diff * diff).sum()
        X12 = xt[torch.as_tensor(self.tets)].reshape(-1, 12)
        Xr = X12.reshape(-1, 4, 3)
        Ds = torch.stack([Xr[:, 1] - Xr[:, 0], Xr[:, 2] - Xr[:, 0], Xr[:, 3] - Xr[:, 0]], dim=2)
        F = Ds @ self._t_dminv
        J = (F[..., :, 0] * torch.linalg.cross(F[..., :, 1], F[..., :, 2])).sum(-1)
        if (J <= 0).any():
            return None
        elastic = (self._t_vol * nh_density_torch(F, self._t_mu, self._t_lam)).sum()
        contact = self._contact_energy_torch(xt, allp, case, d < self.dhat, sigma, mu, s, aug)
        if st.frames is not None:
            contact = contact + self.friction_energy_torch(xt, st.frames)
        return inertia, elastic, contact

    # ------------------------------------------------------------- friction
    def friction_frames(self, x, x_t, pairs: Pairs, st: ALState):
        """Frames at iterate x (Sec. 4.1, updated per inexact Newton iteration):
        every pair of the barrier's support or of A' whose normal force
        lam = -d(pair energy)/dd is positive, with beta and n from its distance
        case at x.  None when friction is off or sigma is not yet set."""
        if not self.p.friction > 0.0 or st.sigma is None:
            return None
        allp, mu, s, aug = self._merge_pairs(pairs, st)
        d, case = self.distances(x, allp)
        sig = float(st.sigma)
        f1 = sig * barrier_d1_np(d, self.dhat) + aug * (-mu + sig * barrier_d1_np(d, self.dhat + s))
        lam = -f1
        keep = ((d < self.dhat) | aug) & (lam > 0.0)
        sel = np.nonzero(keep)[0]
        fp = allp.take(sel)
        X4 = x[fp.nodes]
        beta = closest_coeffs(case[sel], X4)
        n = np.einsum("kj,kjc->kc", beta, X4)
        eps_v = self.p.eps_v if self.p.eps_v > 0.0 else self.dhat
        return Frames(fp, lam[sel], beta, n, x_t.copy(), float(self.p.friction), eps_v * self.h)

    @staticmethod
    def _friction_pair_energy(X12, X12_t, lam, beta, n, chi, eps_h):
        """chi lam f(|P beta.(X - X_t)|) for one pair, P = I - n n^T / n.n."""
        dx = (beta[:, None] * (X12 - X12_t).reshape(4, 3)).sum(0)
        w = dx - (dx * n).sum() / (n * n).sum() * n
        return chi * lam * friction_f_torch((w * w).sum(), eps_h)

    def friction_energy_torch(self, xt, fr: Frames):
        if len(fr.pairs) == 0:
            return xt.sum() * 0.0
        nd = torch.as_tensor(fr.pairs.nodes)
        X = xt[nd].reshape(-1, 12)
        Xt = torch.tensor(fr.x_t[fr.pairs.nodes].reshape(-1, 12), dtype=DT)
        ef = torch.vmap(lambda a, b, l, be, nn: self._friction_pair_energy(a, b, l, be, nn, fr.chi, fr.eps_h))
        return ef(X, Xt, torch.tensor(fr.lam, dtype=DT), torch.tensor(fr.beta, dtype=DT),
                  torch.tensor(fr.n, dtype=DT)).sum()

    def friction_hessians(self, x, fr: Frames, project=True):
        """Per-pair 12x12 Hessians of the friction potential (PSD by
        construction; projected like every stencil)."""
        X = torch.tensor(x[fr.pairs.nodes].reshape(-1, 12), dtype=DT)
        Xt = torch.tensor(fr.x_t[fr.pairs.nodes].reshape(-1, 12), dtype=DT)
        hf = torch.vmap(torch.func.hessian(
            lambda a, b, l, be, nn: self._friction_pair_energy(a, b, l, be, nn, fr.chi, fr.eps_h)))
        H = hf(X, Xt, torch.tensor(fr.lam, dtype=DT), torch.tensor(fr.beta, dtype=DT),
               torch.tensor(fr.n, dtype=DT)).numpy()
        return project_psd(H) if project else 0.5 * (H + np.swapaxes(H, 1, 2))

    def hessian_vector_product(self, x, y, pairs: Pairs, st: ALState, v):
        """Exact (unprojected) Hessian of L_sigma at x applied to v, (N, 3):
        the gradient of the same energy definition differentiated once more
        along v.  Rows and columns of fixed and obstacle vertices are dropped
        (v is zeroed there and so is the result)."""
        allp, mu, s, aug = self._merge_pairs(pairs, st)
        d, case = self.distances(x, allp)
        xt = torch.tensor(x, dtype=DT, requires_grad=True)
        terms = self._objective_terms(xt, y, allp, case, d, st, mu, s, aug)
        total = terms[0] + terms[1] + terms[2]
        (g,) = torch.autograd.grad(total, xt, create_graph=True)
        vt = torch.tensor(np.where(self.free[:, None], v, 0.0), dtype=DT)
        (hv,) = torch.autograd.grad((g * vt).sum(), xt)
        return np.where(self.free[:, None], hv.numpy(), 0.0)

    def gradient_free(self, g_full):
        return g_full[self.free_idx].reshape(-1)

    # -------------------------------------------------------------- Hessian
    def element_hessians(self, x, project=True):
        X12 = torch.tensor(x[self.tets].reshape(-1, 12), dtype=DT)
        hf = torch.vmap(torch.func.hessian(_tet_energy_single))
        H = hf(X12, self._t_dminv, self._t_vol, self._t_mu, self._t_lam).numpy()
        return project_psd(H) if project else 0.5 * (H + np.swapaxes(H, 1, 2))

    def contact_hessians(self, x, pairs, case, mu, s, aug, sigma, project=True):
        """Per-pair 12x12 Hessians of the pair's full energy (barrier + AL terms)."""
        H = np.zeros((len(pairs), 12, 12))
        X4 = torch.tensor(x[pairs.nodes], dtype=DT)
        dh = self.dhat
        for c in np.unique(case):
            sel = np.nonzero(case == c)[0]

            def pe(X, mu_i, s_i, a_i, c=int(c)):
                d = torch.sqrt(q_case_torch(c, X.reshape(4, 3)))
                e = sigma * barrier_torch(d, torch.full_like(d, dh))
                return e + a_i * (mu_i * (dh + s_i - d) + sigma * barrier_torch(d, dh + s_i))

            hf = torch.vmap(torch.func.hessian(pe))
            H[sel] = hf(X4[sel].reshape(-1, 12), torch.tensor(mu[sel], dtype=DT),
                        torch.tensor(s[sel], dtype=DT), torch.tensor(aug[sel].astype(np.float64), dtype=DT)).numpy()
        return project_psd(H) if project else 0.5 * (H + np.swapaxes(H, 1, 2))

    def _assemble(self, blocks, nodes):
        """Sparse free-DOF matrix from stencil matrices (K,3k,3k) on nodes (K,k)."""
        K, k = nodes.shape
        dof = self.dof_of[nodes]
        rows = (3 * dof[:, :, None] + np.arange(3)).reshape(K, -1)
        ok = (dof >= 0).repeat(3, axis=1)
        R = np.broadcast_to(rows[:, :, None], (K, 3 * k, 3 * k))
        C = np.broadcast_to(rows[:, None, :], (K, 3 * k, 3 * k))
        M = ok[:, :, None] & ok[:, None, :]
        return scipy.sparse.coo_matrix((blocks[M], (R[M], C[M])), shape=(self.ndof, self.ndof)).tocsr()

    def hessian(self, x, pairs: Pairs, st: ALState, project=True, with_lambda=False):
        """Assembled free-DOF Hessian of L_sigma at x: M/h^2 + elements + active pairs.

        Every stencil (12x12 per tet, 12x12 per pair over its 4 nodes) is
        projected to its closest PSD form before assembly (Sec. 4.2); rows and
        columns of fixed nodes are then dropped (a principal submatrix stays PSD).
        With with_lambda, also returns the per-node stiffness e_j: the row sums
        over a node's 3 DOFs of Lambda = sum_i S_i [mean eigenvalue_i] S_i^T
        plus the mass term (reading: the stencil mean is tr(H_proj)/(3k) over
        the k nodes the stencil's energy depends on).
        """
        allp, mu, s, aug = self._merge_pairs(pairs, st)
        d, case = self.distances(x, allp)
        keep = (d < self.dhat) | aug
        allp, d, case, mu, s, aug = allp.take(keep), d[keep], case[keep], mu[keep], s[keep], aug[keep]
        sigma = st.sigma if st.sigma is not None else 0.0
        He = self.element_hessians(x, project)
        H = self._assemble(He, self.tets)
        Hc = None
        if len(allp):
            Hc = self.contact_hessians(x, allp, case, mu, s, aug, sigma, project)
            H = H + self._assemble(Hc, allp.nodes)
        Hf = None
        if st.frames is not None and len(st.frames.pairs):
            Hf = self.friction_hessians(x, st.frames, project)
            H = H + self._assemble(Hf, st.frames.pairs.nodes)
        md = np.repeat(self.mass[self.free_idx] / self.h ** 2, 3)
        H = (H + scipy.sparse.diags(md)).tocsr()
        if not with_lambda:
            return H
        e = np.zeros(self.N)
        tr_e = np.trace(He, axis1=1, axis2=2) / 12.0
        for a in range(4):
            np.add.at(e, self.tets[:, a], 3.0 * tr_e)
        if Hc is not None:
            for i in range(len(allp)):
                nd = [allp.nodes[i][j] for j in CASE_NODES[int(case[i])]]
                lam_bar = np.trace(Hc[i]) / (3.0 * len(nd))
                for v in nd:
                    e[v] += 3.0 * lam_bar
        if Hf is not None:
            fr = st.frames
            for i in range(len(fr.pairs)):
                nd = [fr.pairs.nodes[i][j] for j in range(4) if fr.beta[i, j] != 0.0]
                lam_bar = np.trace(Hf[i]) / (3.0 * len(nd))
                for v in nd:
                    e[v] += 3.0 * lam_bar
        e += 3.0 * self.mass / self.h ** 2
        return H, e

    @staticmethod
    def stiffness_groups(e_nodes):
        """Group label floor(log10 e_j) of each node (Sec. 4.2, algebraic decomposition)."""
        return np.floor(np.log10(e_nodes)).astype(np.int64)

    def groupwise_solve(self, H, b, groups_free):
        """Exact warm start: solve blockdiag_groups(H) z = b (blocks coupling different groups dropped)."""
        gd = np.repeat(groups_free, 3)
        Hc = H.tocoo()
        keep = gd[Hc.row] == gd[Hc.col]
        Hg = scipy.sparse.coo_matrix((Hc.data[keep], (Hc.row[keep], Hc.col[keep])), shape=H.shape).tocsc()
        return self.solve(Hg, b)

    def solve(self, H, b):
        """Direct solve: dense Cholesky for small systems, SuperLU otherwise."""
        if H.shape[0] <= 4000:
            c = scipy.linalg.cho_factor(H.toarray())
            return scipy.linalg.cho_solve(c, b)
        return scipy.sparse.linalg.splu(H.tocsc()).solve(b)

    # ------------------------------------------------------------------ CCD
    @staticmethod
    def _cubic_coeffs(u0, u1, v0, v1, w0, w1):
        """Coefficients of det[u0 + t u1, v0 + t v1, w0 + t w1] by multilinear expansion."""
        def det(a, b, c):
            return _dot(a, np.cross(b, c))
        c0 = det(u0, v0, w0)
        c1 = det(u1, v0, w0) + det(u0, v1, w0) + det(u0, v0, w1)
        c2 = det(u1, v1, w0) + det(u1, v0, w1) + det(u0, v1, w1)
        c3 = det(u1, v1, w1)
        return c3, c2, c1, c0

    @staticmethod
    def cubic_roots(c3, c2, c1, c0, lo=-CCD_EPS, hi=1.0 + CCD_EPS, iters=120):
        """Sorted real roots in [lo, hi] of c3 t^3 + c2 t^2 + c1 t + c0 (K,) -> (K,3), nan padded.

        Textbook isolation: the derivative's real roots split [lo, hi] into
        monotone pieces; each piece with a sign change is bisected.  An
        identically zero polynomial has no isolated roots and reports none.
        """
        K = c3.shape[0]
        f = lambda t: ((c3 * t + c2) * t + c1) * t + c0 if np.ndim(t) == 1 else \
            ((c3[:, None] * t + c2[:, None]) * t + c1[:, None]) * t + c0[:, None]
        A, B, C = 3 * c3, 2 * c2, c1
        disc = B * B - 4 * A * C
        crit = np.full((K, 2), np.nan)
        quad = (A != 0) & (disc > 0)
        sq = np.sqrt(np.where(quad, disc, 0.0))
        with np.errstate(divide="ignore", invalid="ignore"):
            crit[:, 0] = np.where(quad, (-B - sq) / (2 * A), np.where((A == 0) & (B != 0), -C / B, np.nan))
            crit[:, 1] = np.where(quad, (-B + sq) / (2 * A), np.nan)
        crit[(crit <= lo) | (crit >= hi)] = np.nan
        bp = np.concatenate([np.full((K, 1), lo), crit, np.full((K, 1), hi)], axis=1)
        bp = np.sort(bp, axis=1)  # nans last
        a, b = bp[:, :3], bp[:, 1:]
        valid = np.isfinite(a) & np.isfinite(b)
        fa = np.where(valid, f(np.where(valid, a, 0.0)), np.nan)
        fb = np.where(valid, f(np.where(valid, b, 0.0)), np.nan)
        has = valid & (fa * fb <= 0)
        zero_poly = (c3 == 0) & (c2 == 0) & (c1 == 0) & (c0 == 0)
        has &= ~zero_poly[:, None]
        r = np.full((K, 3), np.nan)
        ki, kj = np.nonzero(has)
        lo_, hi_, flo = a[ki, kj], b[ki, kj], fa[ki, kj]
        q3, q2, q1, q0 = c3[ki], c2[ki], c1[ki], c0[ki]
        for _ in range(iters):
            mid = 0.5 * (lo_ + hi_)
            fm = ((q3 * mid + q2) * mid + q1) * mid + q0
            left = fm * flo <= 0
            hi_ = np.where(left, mid, hi_)
            lo_ = np.where(left, lo_, mid)
            flo = np.where(left, flo, fm)
        r[ki, kj] = 0.5 * (lo_ + hi_)
        # a root on a shared breakpoint is found twice
        r = np.sort(r, axis=1)
        dup = np.abs(np.diff(r, axis=1)) <= 1e-15
        r[:, 1:][dup] = np.nan
        return np.sort(r, axis=1)

    def _signed_dist(self, kind, X4):
        """Signed point-plane (PT) or line-line (EE) distance."""
        if kind == 0:
            n = np.cross(X4[:, 2] - X4[:, 1], X4[:, 3] - X4[:, 1])
            return _dot(X4[:, 0] - X4[:, 1], n) / np.linalg.norm(n, axis=1)
        n = np.cross(X4[:, 1] - X4[:, 0], X4[:, 3] - X4[:, 2])
        return _dot(X4[:, 0] - X4[:, 2], n) / np.linalg.norm(n, axis=1)

    def ccd(self, x, p, pairs: Pairs, return_tau=False):
        """Conservative step bound alpha_max = min(1, min_i tau_i) along x + t p (Sec. 5.3).

        Per pair: roots of the coplanarity cubic in [-eps, 1+eps] (clamped to
        [0, 1]) are visited in order t1 <= t2 <= t3 with t0 = 0; the first
        root whose distance d_TOC < eps + dhat is activated, tau = t_{i+1};
        for point-triangle / edge-edge interior cases tau shrinks by 0.9
        while sign sd(tau) != sign sd((t_i + tau) / 2) (reading of the
        reference-frame rule; |sd| <= eps counts as sign 0, so a tau sitting
        on the coplanarity root always backs off); point-point / point-edge
        cases keep tau.  Edge pairs parallel at both ends of the step are
        skipped (reading: a parallel edge pair is coplanar for every t).
        A root at |t| <= eps coincides with the start frame t0 = 0 of the
        candidate times and is not a time of impact (reading: activating it
        bounds every later step of a pair that an iterate left coplanar
        inside dhat at alpha_max = 0).  So does the root of a pair whose start
        configuration is coplanar to within the rounding of its positions
        (|det| <= 32 u max|x_k| (|u||v| + |v||w| + |w||u|), u the unit
        roundoff): the cubic's constant term is then taken as 0, so its root
        at t0 is exact however short the step is (reading: a step cut at a
        coplanar time leaves the pair there, and for a short direction the
        rounding of the landing point alone moves that root past eps).

        Other rules: "literal" activates roots at |t| <= eps as well;
        "half_gap" (a departure from the printed rule) takes half the pair's
        current distance as the margin when the pair starts closer than dhat.
        """
        K = len(pairs)
        tau = np.ones(K)
        if K == 0:
            return (1.0, tau) if return_tau else 1.0
        X0 = x[pairs.nodes]
        P = p[pairs.nodes]
        pt = (pairs.kind == 0)[:, None]
        # PT: det[p - a, b - a, c - a]; EE: det[a1 - a0, b0 - a0, b1 - a0]
        u0 = np.where(pt, X0[:, 0] - X0[:, 1], X0[:, 1] - X0[:, 0])
        u1 = np.where(pt, P[:, 0] - P[:, 1], P[:, 1] - P[:, 0])
        v0 = np.where(pt, X0[:, 2] - X0[:, 1], X0[:, 2] - X0[:, 0])
        v1 = np.where(pt, P[:, 2] - P[:, 1], P[:, 2] - P[:, 0])
        w0 = np.where(pt, X0[:, 3] - X0[:, 1], X0[:, 3] - X0[:, 0])
        w1 = np.where(pt, P[:, 3] - P[:, 1], P[:, 3] - P[:, 0])
        c3, c2, c1, c0 = self._cubic_coeffs(u0, u1, v0, v1, w0, w1)
        rule = self.p.ccd_rule
        if rule != "literal":
            nu, nv, nw = (np.linalg.norm(a, axis=1) for a in (u0, v0, w0))
            xmax = np.abs(X0).max(axis=(1, 2))
            c0 = np.where(np.abs(c0) <= COPLANAR_ULPS * 2.0 ** -53 * xmax * (nu * nv + nv * nw + nw * nu), 0.0, c0)
        roots = self.cubic_roots(c3, c2, c1, c0)
        ee = pairs.kind == 1
        if ee.any():
            def par(X):
                e1 = X[:, 1] - X[:, 0]
                e2 = X[:, 3] - X[:, 2]
                n = np.cross(e1, e2)
                return _dot(n, n) < PARALLEL_EPS * _dot(e1, e1) * _dot(e2, e2)
            X1 = X0 + P
            skip = np.zeros(K, bool)
            skip[ee] = par(X0[ee]) & par(X1[ee])
            roots[skip] = np.nan
        if rule not in ("printed", "half_gap", "literal"):
            raise ValueError(rule)
        margin = np.full(K, self.dhat)
        if rule == "half_gap":
            q_start, _ = classify(pairs.kind, X0)
            d_start = np.sqrt(q_start)
            margin = np.where(d_start < self.dhat, 0.5 * d_start, self.dhat)
        done = np.zeros(K, dtype=bool)
        t_prev = np.zeros(K)
        for k in range(3):
            r = roots[:, k]
            cand = np.isfinite(r) & ~done
            if rule != "literal":
                # a root at |t| <= eps is the start frame t0 = 0 itself (reading)
                cand &= r > CCD_EPS
            if not cand.any():
                continue
            idx = np.nonzero(cand)[0]
            tk = np.clip(r[idx], 0.0, 1.0)
            Xk = X0[idx] + tk[:, None, None] * P[idx]
            q, case = classify(pairs.kind[idx], Xk)
            act = np.sqrt(q) < CCD_EPS + margin[idx]
            ai = idx[act]
            tau_a = tk[act]
            case_a = case[act]
            tp = t_prev[ai]
            for j in range(ai.size):
                i = ai[j]
                t_i = tau_a[j]
                if case_a[j] in (0, 7):
                    kd = int(pairs.kind[i])
                    for _ in range(400):
                        s1 = self._signed_dist(kd, (X0[i] + t_i * P[i])[None])[0]
                        s0 = self._signed_dist(kd, (X0[i] + 0.5 * (tp[j] + t_i) * P[i])[None])[0]
                        if _dz_sign(s1) == _dz_sign(s0):
                            break
                        t_i *= 0.9
                tau[i] = t_i
            done[ai] = True
            t_prev[idx] = tk
        amax = float(min(1.0, tau.min()))
        return (amax, tau) if return_tau else amax

    # ------------------------------------------------------------- the step
    def sigma0(self, x, y, pairs, st_empty):
        """sigma^0 = argmin_s ||g_E + s g_b||^2 = -g_b.g_E / ||g_b||^2 (reading of Sec. 3.4).

        g_E: gradient of inertia + elasticity, g_b: gradient of sum_A b(d_i, dhat),
        both over the free DOFs.  Falls back to ||g_E|| / ||g_b|| if the
        least-squares value is not positive and finite.
        """
        st0 = ALState(sigma=0.0)
        _, gE = self.lagrangian(x, y, pairs, st0, with_grad=True)
        st1 = ALState(sigma=1.0)
        _, gT = self.lagrangian(x, y, pairs, st1, with_grad=True)
        gE = self.gradient_free(gE)
        gb = self.gradient_free(gT) - gE
        nb = float(gb @ gb)
        if nb == 0.0:
            return None
        s0 = -float(gb @ gE) / nb
        if not (s0 > 0 and math.isfinite(s0)):
            s0 = math.sqrt(float(gE @ gE) / nb)
        return s0

    def _log(self, msg, t0):
        if self.p.verbose:
            import time
            print(f"[oracle] {msg} ({time.perf_counter() - t0:.1f} s)", flush=True)

    def step(self, trace=None, return_state=False):
        """Advance one time step with Algorithm 1; returns a stats dict."""
        import time
        t0 = time.perf_counter()
        p = self.p
        x_t, v_t = self.x.copy(), self.v.copy()
        y = self.predictor(x_t, v_t)
        x = x_t.copy()
        st = ALState()
        if p.sigma_fixed > 0.0:
            st.sigma = st.sigma0 = float(p.sigma_fixed)
        prev_min = np.inf
        e0 = None
        converged = False
        it = 0
        dh = self.dhat
        for it in range(p.max_newton):
            pairs = self.candidate_pairs(x)
            d, _ = self.distances(x, pairs)
            min_d = float(d.min()) if d.size else np.inf
            active = d < dh
            # A' update (Alg. 1, lines 3-6; reading: current vs previous iterate)
            if p.use_al:
                st.aug, st.mu, st.s = rebuild_aug_set(pairs, d, min_d, prev_min, st, dh)
            prev_min = min_d
            if st.sigma is None and active.any():
                s0 = self.sigma0(x, y, pairs.take(np.nonzero(active)[0]), st)
                if s0 is not None:
                    st.sigma0 = st.sigma = s0
            self._log(f"iteration {it}: {len(pairs)} candidate pairs, {int(active.sum())} active", t0)
            # friction frames at this iterate (Sec. 4.1: updated per inexact Newton iteration)
            st.frames = self.friction_frames(x, x_t, pairs, st)
            L0, g = self.lagrangian(x, y, pairs, st, with_grad=True)
            e = self.gradient_free(g)
            en = float(np.linalg.norm(e))
            if e0 is None:
                e0 = en
            self._log(f"iteration {it}: gradient, |e| = {en:.3e}", t0)
            H = self.hessian(x, pairs, st)
            self._log(f"iteration {it}: projected Hessian assembled ({H.nnz} nonzeros)", t0)
            dx = -self.solve(H, e)
            self._log(f"iteration {it}: direct solve done", t0)
            P = np.zeros_like(x)
            P[self.free_idx] = dx.reshape(-1, 3)
            sw = 1.0
            if p.sweep_cap > 0.0:
                pmax = float(np.sqrt((P * P).sum(1).max())) if len(P) else 0.0
                while sw * pmax > p.sweep_cap * self.mean_edge and sw > 1e-30:
                    sw *= 0.5
            swept = self.candidate_pairs(x, disp=sw * P)
            amax = sw * self.ccd(x, sw * P, swept)
            self._log(f"iteration {it}: CCD over {len(swept)} pairs, alpha_max = {amax:.3e}", t0)

            def trial(a):
                xa = x + a * P
                cap = True
                if p.max_contacts < (1 << 40):
                    da, _ = self.distances(xa, swept)
                    cap = int((da < dh).sum()) <= p.max_contacts
                La = self.lagrangian(xa, y, swept, st)
                return La, bool(np.isfinite(La)), cap
            alpha = line_search(amax, L0, trial, p.min_alpha)
            xn = x + alpha * P
            if trace is not None:
                trace.append(dict(it=it, n_active=int(active.sum()), n_aug=len(st.aug),
                                  sigma=st.sigma, min_d=min_d, alpha_max=amax, alpha=alpha, enorm=en))
            if en <= p.newton_rtol * e0:
                x = xn
                converged = True
                break
            moved = alpha * float(np.linalg.norm(P[self.free_idx]))
            if moved <= 1e-15 * float(np.linalg.norm(x[self.free_idx])) and len(st.aug) == 0:
                x = xn
                converged = en <= p.accept_rtol * e0
                break  # no measurable step and nothing left to update: stalled (reading)
            # dual and penalty updates (Alg. 1, lines 12-17)
            dn, _ = self.distances(xn, swept)
            if len(st.aug):
                da, _ = self.distances(xn, st.aug)
                st.mu, st.s = dual_update(st.mu, da, st.sigma, dh)
            if dn.size and st.sigma is not None and not p.sigma_fixed > 0.0:
                st.sigma = sigma_update(st.sigma, st.sigma0, float(dn.min()), dh)
            x = xn
        self.x = x
        self.v = (x - x_t) / self.h
        self.v[~self.free] = 0.0
        stats = dict(newton_iters=it + 1, converged=converged, sigma=st.sigma)
        if return_state:
            stats.update(state=st, y=y, x_t=x_t, v_t=v_t)
        return stats

    # --------------------------------------------------------------- adjoint
    def adjoint_step(self, x_next, y, st: ALState, gx_next, gv_next):
        """Frozen-state adjoint of a converged step (reading; not in the paper).

        Stationarity g(x*; x_t, v_t, E) = grad_x L = 0 with (sigma, mu, s, A')
        frozen.  With H the unprojected Hessian at x*, solve H lam = gx + gv/h
        on the free DOFs; then gx_t = (M/h^2) lam - gv/h, gv_t = (M/h) lam and
        gE_e = -lam_e . grad Psi_e / E_e (Psi is linear in E at fixed nu).
        """
        pairs = self.candidate_pairs(x_next)
        H = self.hessian(x_next, pairs, st, project=False)
        pad = lambda a: np.concatenate([np.asarray(a, dtype=np.float64), np.zeros((self.N - len(a), 3))])
        gx_next, gv_next = pad(gx_next), pad(gv_next)
        rhs = (gx_next + gv_next / self.h)[self.free_idx].reshape(-1)
        lam_f = self.solve(H, rhs) if H.shape[0] <= 4000 else scipy.sparse.linalg.spsolve(H.tocsc(), rhs)
        lam = np.zeros((self.N, 3))
        lam[self.free_idx] = lam_f.reshape(-1, 3)
        m = self.mass[:, None]
        gx_t = m / self.h ** 2 * lam - gv_next / self.h
        gv_t = m / self.h * lam
        gx_t[~self.free] = 0.0
        gv_t[~self.free] = 0.0
        X12 = torch.tensor(x_next[self.tets].reshape(-1, 12), dtype=DT)
        gf = torch.vmap(torch.func.grad(_tet_energy_single))
        gpsi = gf(X12, self._t_dminv, self._t_vol, self._t_mu, self._t_lam).numpy()
        lam_e = lam[self.tets].reshape(-1, 12)
        gE = -np.einsum("ij,ij->i", lam_e, gpsi) / self.E
        return gx_t[: self.n_body], gv_t[: self.n_body], gE

    def rollout(self, n_steps, checkpoint=None):
        """Run n_steps; returns per-step stats (states kept for the adjoint)."""
        out = []
        for _ in range(n_steps):
            out.append(self.step(return_state=True))
        return out


__all__ = [
    "OracleScene", "Params", "ALState", "Pairs", "classify", "classify_pt", "classify_ee",
    "rebuild_aug_set", "slack_update", "dual_update", "sigma_update", "line_search",
    "point_segment_sq", "q_case_torch", "barrier_np", "barrier_torch", "lame", "nh_density_torch",
    "project_psd", "CASE_NODES", "CASE_KIND", "CCD_EPS", "PARALLEL_EPS",
]
