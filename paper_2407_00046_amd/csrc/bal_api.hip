// Host side of the BAL library: scene construction, Algorithm 1 (the
// barrier-augmented Lagrangian loop with one inexact Newton-PCG iteration per
// pass), the C ABI of include/bal.h, the verification entry points and the
// frozen-state adjoint.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "bal_internal.h"

namespace bal {

int DBuf::grow(size_t need) {
  if (need <= bytes && p) return 0;
  if (p) hipFree(p);
  p = nullptr;
  bytes = 0;
  size_t n = need < 256 ? 256 : need;
  if (hipMalloc(&p, n) != hipSuccess) { p = nullptr; return 1; }
  bytes = n;
  return 0;
}
void DBuf::release() {
  if (p) hipFree(p);
  p = nullptr;
  bytes = 0;
}
int hip_ok(hipError_t e) { return e == hipSuccess ? BAL_OK : BAL_E_HIP; }

using clk = std::chrono::steady_clock;
constexpr double kWarmTol = 1e-4;  // per-group relative tolerance of the warm start
static double since(clk::time_point t0) { return std::chrono::duration<double>(clk::now() - t0).count(); }

// ---------------------------------------------------------------- small kernels
__global__ void k_mask_less(int n, const double *d, double thr, int *mask) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) mask[i] = d[i] < thr ? 1 : 0;
}

__global__ void k_compact_pairs(int n, const int *mask, const int *off, const int *kind, const int *a, const int *b,
                                const int4 *nodes, const uint64_t *key, int *okind, int *oa, int *ob, int4 *onodes,
                                uint64_t *okey) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !mask[i]) return;
  int o = off[i];
  okind[o] = kind[i];
  oa[o] = a[i];
  ob[o] = b[i];
  onodes[o] = nodes[i];
  okey[o] = key[i];
}

__device__ int find_key(const uint64_t *keys, int n, uint64_t k) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    uint64_t v = keys[mid];
    if (v == k) return mid;
    if (v < k) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// uni_aug[i] = index of pair i in A' (or -1); uni_flag[i] = barrier term on.
__global__ void k_aug_lookup(int n, const uint64_t *key, const uint64_t *akey, int naug, int *uaug, int *uflag,
                             int flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uaug[i] = naug > 0 ? find_key(akey, naug, key[i]) : -1;
  uflag[i] = flag;
}

// mask[j] = 1 if A' pair j is not among the n active pairs.
__global__ void k_aug_missing(int naug, const uint64_t *akey, const uint64_t *key, int n, int *mask) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= naug) return;
  mask[j] = (n > 0 && find_key(key, n, akey[j]) >= 0) ? 0 : 1;
}

__global__ void k_append_aug(int naug, const int *mask, const int *off, int base, const int *akind, const int *aa,
                             const int *ab, const int4 *anodes, const uint64_t *akey, int *okind, int *oa, int *ob,
                             int4 *onodes, uint64_t *okey, int *uaug, int *uflag) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= naug || !mask[j]) return;
  int o = base + off[j];
  okind[o] = akind[j];
  oa[o] = aa[j];
  ob[o] = ab[j];
  onodes[o] = anodes[j];
  okey[o] = akey[j];
  uaug[o] = j;
  uflag[o] = 0;
}

// new A' entries keep (mu, s) of the same pair in the old A' (reading: keyed by primitive pair)
__global__ void k_aug_carry(int nnew, const uint64_t *nkey, const uint64_t *okey, int nold, const double *omu,
                            const double *os, double *nmu, double *ns) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nnew) return;
  int k = nold > 0 ? find_key(okey, nold, nkey[j]) : -1;
  nmu[j] = k >= 0 ? omu[k] : 0.0;
  ns[j] = k >= 0 ? os[k] : 0.0;
}

// -|p_i|^2 per vertex (for the largest displacement of a step)
__global__ void k_neg_norm2(const double *__restrict__ p, double *__restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -(p[3 * i] * p[3 * i] + p[3 * i + 1] * p[3 * i + 1] + p[3 * i + 2] * p[3 * i + 2]);
}

__global__ void k_scale(const double *__restrict__ a, double f, double *__restrict__ b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f * a[i];
}

// With sweep_cap = n > 0 (not in the paper): the largest sweep s (a power of
// 1/2, at most 1) for which no vertex moves more than n mean surface edge
// lengths along s p.  Without it the sweep starts at the whole step and
// halves only when the candidate pass exceeds its work bound.
static double sweep_limit(Scene &s, const double *p) {
  if (s.desc.sweep_cap <= 0) return 1.0;
  if (s.tau.grow((size_t)(s.N + 1) * 8)) return 1.0;
  hipLaunchKernelGGL(k_neg_norm2, dim3(blocks_for(s.N, 256)), dim3(256), 0, s.stream, p, s.tau.as<double>(), s.N);
  double pmax = std::sqrt(std::max(0.0, -reduce_min(s, s.tau.as<double>(), s.N)));
  double sw = 1.0;
  while (sw * pmax > (double)s.desc.sweep_cap * s.cell && sw > 1e-30) sw *= 0.5;
  return sw;
}

__global__ void k_neg(const double *a, double *b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = -a[i];
}

__global__ void k_velocity(int N, const double *x, const double *xt, const uint8_t *fr, double ih, double *v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int c = 0; c < 3; ++c) v[3 * i + c] = fr[i] ? (x[3 * i + c] - xt[3 * i + c]) * ih : 0.0;
}

__global__ void k_to_float(const double *a, float *b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_to_double(const float *a, double *b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// adjoint outputs: gx_t = (M/h^2) lam - gv/h, gv_t = (M/h) lam on free nodes
__global__ void k_adjoint_state(int n, const double *lam, const double *gv, const double *m, const uint8_t *fr,
                                double h, double *gx, double *gvo) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < 3; ++c) {
    double l = lam[3 * i + c];
    gx[3 * i + c] = fr[i] ? m[i] / (h * h) * l - gv[3 * i + c] / h : 0.0;
    gvo[3 * i + c] = fr[i] ? m[i] / h * l : 0.0;
  }
}

// gE_e += -lam_e . grad Psi_e / E_e
__global__ void k_adjoint_E(int T, const int4 *tets, const double *tet_g, const double *lam, const double *E,
                            double *gE) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int4 tv = tets[t];
  int v[4] = {tv.x, tv.y, tv.z, tv.w};
  double acc = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) acc += lam[3 * v[a] + c] * tet_g[(size_t)t * 12 + 3 * a + c];
  gE[t] += -acc / E[t];
}

// ---------------------------------------------------------------- helpers
static int sync(Scene &s) { return hip_ok(hipStreamSynchronize(s.stream)); }

static int read_flags_and_clear(Scene &s) {
  int *h = s.pin.as<int>();
  hipMemcpyAsync(h, s.flags.p, sizeof(int), hipMemcpyDeviceToHost, s.stream);
  hipStreamSynchronize(s.stream);
  int f = h[0];
  hipMemsetAsync(s.flags.p, 0, sizeof(int), s.stream);
  return f;
}

static int grow_pair_list(PairList &pl, int n) {
  size_t m = (size_t)(n > 0 ? n : 1);
  if (pl.kind.grow(m * sizeof(int)) || pl.a.grow(m * sizeof(int)) || pl.b.grow(m * sizeof(int)) ||
      pl.nodes.grow(m * sizeof(int4)) || pl.d.grow(m * sizeof(double)) || pl.cs.grow(m * sizeof(int)) ||
      pl.key.grow(m * sizeof(uint64_t)))
    return BAL_E_OOM;
  return BAL_OK;
}

static int grow_aug(Scene &s, int n) {
  size_t m = (size_t)(n > 0 ? n : 1);
  if (s.aug_kind.grow(m * 4) || s.aug_a.grow(m * 4) || s.aug_b.grow(m * 4) || s.aug_nodes.grow(m * 16) ||
      s.aug_key.grow(m * 8) || s.aug_mu.grow(m * 8) || s.aug_s.grow(m * 8) || s.aug_d.grow(m * 8) ||
      s.aug_e.grow(m * 8) || s.aug_tmp_mu.grow(m * 8) || s.aug_tmp_s.grow(m * 8))
    return BAL_E_OOM;
  return BAL_OK;
}

// Rebuilds A' = {pairs of `pl` with d < thr} keeping mu, s of surviving pairs.
static int rebuild_aug(Scene &s, PairList &pl, double thr) {
  int n = pl.n;
  if (s.mask.grow((size_t)(n + 1) * 4) || s.mask_off.grow((size_t)(n + 1) * 4)) return BAL_E_OOM;
  if (n > 0)
    hipLaunchKernelGGL(k_mask_less, dim3(blocks_for(n, 256)), dim3(256), 0, s.stream, n, pl.d.as<double>(), thr,
                       s.mask.as<int>());
  int m = scan_exclusive(s, s.mask.as<int>(), s.mask_off.as<int>(), n);
  PairList &tmp = s.augtmp;
  if (grow_pair_list(tmp, m)) return BAL_E_OOM;
  if (m > 0)
    hipLaunchKernelGGL(k_compact_pairs, dim3(blocks_for(n, 256)), dim3(256), 0, s.stream, n, s.mask.as<int>(),
                       s.mask_off.as<int>(), pl.kind.as<int>(), pl.a.as<int>(), pl.b.as<int>(), pl.nodes.as<int4>(),
                       pl.key.as<uint64_t>(), tmp.kind.as<int>(), tmp.a.as<int>(), tmp.b.as<int>(),
                       tmp.nodes.as<int4>(), tmp.key.as<uint64_t>());
  DBuf nmu, ns;
  if (nmu.grow((size_t)(m + 1) * 8) || ns.grow((size_t)(m + 1) * 8)) return BAL_E_OOM;
  if (m > 0)
    hipLaunchKernelGGL(k_aug_carry, dim3(blocks_for(m, 256)), dim3(256), 0, s.stream, m, tmp.key.as<uint64_t>(),
                       s.aug_key.as<uint64_t>(), s.n_aug, s.aug_mu.as<double>(), s.aug_s.as<double>(),
                       nmu.as<double>(), ns.as<double>());
  if (grow_aug(s, m)) return BAL_E_OOM;
  if (m > 0) {
    hipMemcpyAsync(s.aug_kind.p, tmp.kind.p, (size_t)m * 4, hipMemcpyDeviceToDevice, s.stream);
    hipMemcpyAsync(s.aug_a.p, tmp.a.p, (size_t)m * 4, hipMemcpyDeviceToDevice, s.stream);
    hipMemcpyAsync(s.aug_b.p, tmp.b.p, (size_t)m * 4, hipMemcpyDeviceToDevice, s.stream);
    hipMemcpyAsync(s.aug_nodes.p, tmp.nodes.p, (size_t)m * 16, hipMemcpyDeviceToDevice, s.stream);
    hipMemcpyAsync(s.aug_key.p, tmp.key.p, (size_t)m * 8, hipMemcpyDeviceToDevice, s.stream);
    hipMemcpyAsync(s.aug_mu.p, nmu.p, (size_t)m * 8, hipMemcpyDeviceToDevice, s.stream);
    hipMemcpyAsync(s.aug_s.p, ns.p, (size_t)m * 8, hipMemcpyDeviceToDevice, s.stream);
  }
  sync(s);
  nmu.release();
  ns.release();
  s.n_aug = m;
  return BAL_OK;
}

// Union list for linearization: candidates with d < dhat (barrier on) plus
// A' pairs not among them (barrier off); each with its A' index or -1.
static int build_union(Scene &s, PairList &pl) {
  int n = pl.n;
  if (s.mask.grow((size_t)(n + s.n_aug + 1) * 4) || s.mask_off.grow((size_t)(n + s.n_aug + 1) * 4)) return BAL_E_OOM;
  if (n > 0)
    hipLaunchKernelGGL(k_mask_less, dim3(blocks_for(n, 256)), dim3(256), 0, s.stream, n, pl.d.as<double>(),
                       s.desc.dhat, s.mask.as<int>());
  int m = scan_exclusive(s, s.mask.as<int>(), s.mask_off.as<int>(), n);
  PairList &u = s.uni;
  if (grow_pair_list(u, m + s.n_aug) || s.uni_flag.grow((size_t)(m + s.n_aug + 1) * 4) ||
      s.uni_aug.grow((size_t)(m + s.n_aug + 1) * 4))
    return BAL_E_OOM;
  if (m > 0) {
    hipLaunchKernelGGL(k_compact_pairs, dim3(blocks_for(n, 256)), dim3(256), 0, s.stream, n, s.mask.as<int>(),
                       s.mask_off.as<int>(), pl.kind.as<int>(), pl.a.as<int>(), pl.b.as<int>(), pl.nodes.as<int4>(),
                       pl.key.as<uint64_t>(), u.kind.as<int>(), u.a.as<int>(), u.b.as<int>(), u.nodes.as<int4>(),
                       u.key.as<uint64_t>());
    hipLaunchKernelGGL(k_aug_lookup, dim3(blocks_for(m, 256)), dim3(256), 0, s.stream, m, u.key.as<uint64_t>(),
                       s.aug_key.as<uint64_t>(), s.n_aug, s.uni_aug.as<int>(), s.uni_flag.as<int>(), 1);
  }
  int extra = 0;
  if (s.n_aug > 0) {
    int *mk = s.mask.as<int>(), *mo = s.mask_off.as<int>();
    hipLaunchKernelGGL(k_aug_missing, dim3(blocks_for(s.n_aug, 256)), dim3(256), 0, s.stream, s.n_aug,
                       s.aug_key.as<uint64_t>(), u.key.as<uint64_t>(), m, mk);
    extra = scan_exclusive(s, mk, mo, s.n_aug);
    if (extra > 0)
      hipLaunchKernelGGL(k_append_aug, dim3(blocks_for(s.n_aug, 256)), dim3(256), 0, s.stream, s.n_aug, mk, mo, m,
                         s.aug_kind.as<int>(), s.aug_a.as<int>(), s.aug_b.as<int>(), s.aug_nodes.as<int4>(),
                         s.aug_key.as<uint64_t>(), u.kind.as<int>(), u.a.as<int>(), u.b.as<int>(), u.nodes.as<int4>(),
                         u.key.as<uint64_t>(), s.uni_aug.as<int>(), s.uni_flag.as<int>());
  }
  u.n = m + extra;
  size_t P = (size_t)(u.n > 0 ? u.n : 1);
  size_t w = s.mixed ? 4 : 8;
  if (s.pair_e.grow(P * 8) || s.pair_g.grow(P * 12 * 8) || s.pair_tr.grow(P * 8) || s.pair_blk.grow(P * 144 * w))
    return BAL_E_OOM;
  if (s.desc.friction > 0.0 && (s.fr.grow(P * 8 * 8) || s.fr_e.grow(P * 8))) return BAL_E_OOM;
  return BAL_OK;
}

// Gradient, projected (or unprojected) Hessian, stiffness groups and
// preconditioner at x for the current union list.
static int linearize_at(Scene &s, const double *x, int project, double sigma) {
  hipMemsetAsync(s.flags.p, 0, sizeof(int), s.stream);
  launch_elements(s, x, EM_HESS, project);
  launch_pair_linearize(s, x, project, sigma, 1);
  int rc = build_contact_lists(s);
  if (rc) return rc;
  launch_node_assembly(s, x, 1, 1, 1, 1, s.grad.as<double>());
  launch_offdiag_assembly(s);
  int f = read_flags_and_clear(s);
  if (f & 1) return BAL_E_INVERTED;
  if (f & 2) return BAL_E_PENETRATION;
  s.linearized = true;
  return BAL_OK;
}

// L_sigma at xp over candidate pairs pl (barrier) and A' (augmentation);
// returns BAL_OK with *L, or sets *valid = 0 if some J <= 0 or d <= 0.
// The part sums, the active count and the flags are left on the device and
// read back together: one synchronisation per evaluation.
static int energy_at(Scene &s, const double *xp, PairList &pl, double sigma, double *L, int *valid, int *nact) {
  hipMemsetAsync(s.flags.p, 0, sizeof(int), s.stream);
  launch_elements(s, xp, EM_ENERGY, 0);
  launch_inertia_energy(s, xp, s.node_e.as<double>());
  if (s.cand_e.grow((size_t)(pl.n + 1) * 8) || s.red_slots.grow(8 * sizeof(double))) return BAL_E_OOM;
  launch_pair_barrier_energy(s, pl, xp, sigma, s.cand_e.as<double>(), s.flags.as<int>());
  launch_aug_energy(s, xp, sigma, s.aug_e.as<double>(), s.aug_d.as<double>(), s.flags.as<int>());
  // slots: elements, inertia, barrier, augmentation, friction, active count, flags
  double *sl = s.red_slots.as<double>();
  hipMemsetAsync(sl, 0, 8 * sizeof(double), s.stream);
  reduce_sum_to(s, s.tet_e.as<double>(), s.T, sl);
  reduce_sum_to(s, s.node_e.as<double>(), s.N, sl + 1);
  reduce_sum_to(s, s.cand_e.as<double>(), pl.n, sl + 2);
  if (s.n_aug) reduce_sum_to(s, s.aug_e.as<double>(), s.n_aug, sl + 3);
  // friction potential with the frames of the last linearization (Sec. 4.1)
  const bool fric = s.desc.friction > 0.0 && s.uni.n > 0;
  if (fric) {
    launch_friction_energy(s, xp, s.fr_e.as<double>());
    reduce_sum_to(s, s.fr_e.as<double>(), s.uni.n, sl + 4);
  }
  count_less_to(s, pl.d.as<double>(), pl.n, s.desc.dhat, sl + 5);
  hipMemcpyAsync(sl + 6, s.flags.p, sizeof(int), hipMemcpyDeviceToDevice, s.stream);
  double *h = reinterpret_cast<double *>(static_cast<char *>(s.pin.p) + kPinEnergy);
  hipMemcpyAsync(h, sl, 7 * sizeof(double), hipMemcpyDeviceToHost, s.stream);
  if (hipStreamSynchronize(s.stream) != hipSuccess) return BAL_E_HIP;
  hipMemsetAsync(s.flags.p, 0, sizeof(int), s.stream);
  int f;
  std::memcpy(&f, h + 6, sizeof(int));
  double e = h[0] + h[1];
  e += h[2];
  if (s.n_aug) e += h[3];
  if (fric) e += h[4];
  *valid = f == 0;
  *L = e;
  *nact = (int)llround(h[5]);
  return BAL_OK;
}

// sigma^0 = -g_b.g_E / ||g_b||^2 (least-squares balance of barrier and IP gradients, Sec. 3.4;
// fallback ||g_E|| / ||g_b||), with g_b = sum over the active set of grad b(d_i, dhat).
static int compute_sigma0(Scene &s, const double *x, PairList &pl, double *out, bool *ok) {
  *ok = false;
  launch_elements(s, x, EM_GRAD, 0);
  launch_node_assembly(s, x, 0, 1, 1, 0, s.grad_b.as<double>());
  int saved_aug = s.n_aug;
  s.n_aug = 0;  // g_b from the barrier of the active set only
  int rc = build_union(s, pl);
  if (rc) { s.n_aug = saved_aug; return rc; }
  launch_pair_linearize(s, x, 0, 1.0, 0);
  rc = build_contact_lists(s);
  s.n_aug = saved_aug;
  if (rc) return rc;
  launch_node_assembly(s, x, 1, 0, 0, 0, s.rhs.as<double>());
  double bE = dot_free(s, s.rhs.as<double>(), s.grad_b.as<double>());
  double bb = dot_free(s, s.rhs.as<double>(), s.rhs.as<double>());
  double EE = dot_free(s, s.grad_b.as<double>(), s.grad_b.as<double>());
  if (!(bb > 0.0)) return BAL_OK;
  double s0 = -bE / bb;
  if (!(s0 > 0.0 && std::isfinite(s0))) s0 = std::sqrt(EE / bb);
  *out = s0;
  *ok = std::isfinite(s0) && s0 > 0.0;
  return BAL_OK;
}

static double min_or(Scene &s, PairList &pl, double fallback) {
  if (pl.n == 0) return fallback;
  double m = reduce_min(s, pl.d.as<double>(), pl.n);
  return m;
}

// min d over a pair list and the count of pairs inside dhat, read back
// together (INFINITY and 0 for an empty list)
static int min_and_count(Scene &s, PairList &pl, double dh, double *min_d, int *count) {
  *min_d = INFINITY;
  *count = 0;
  if (pl.n == 0) return BAL_OK;
  if (s.red_slots.grow(8 * sizeof(double))) return BAL_E_OOM;
  double *sl = s.red_slots.as<double>();
  reduce_min_to(s, pl.d.as<double>(), pl.n, sl);
  count_less_to(s, pl.d.as<double>(), pl.n, dh, sl + 1);
  double *h = reinterpret_cast<double *>(static_cast<char *>(s.pin.p) + kPinEnergy);
  hipMemcpyAsync(h, sl, 2 * sizeof(double), hipMemcpyDeviceToHost, s.stream);
  if (hipStreamSynchronize(s.stream) != hipSuccess) return BAL_E_HIP;
  *min_d = h[0];
  *count = (int)llround(h[1]);
  return BAL_OK;
}

static void copy3(Scene &s, double *dst, const double *src) {
  hipMemcpyAsync(dst, src, (size_t)3 * s.N * 8, hipMemcpyDeviceToDevice, s.stream);
}

// ---------------------------------------------------------------- the step
static int newton_solve(Scene &s, bal_step_stats *st, bool record) {
  auto t_start = clk::now();
  const bal_scene_desc &d = s.desc;
  const double dh = d.dhat;
  double *x = s.x.as<double>(), *dx = s.dx.as<double>(), *xtr = s.xtrial.as<double>();
  copy3(s, s.x_t.as<double>(), x);
  copy3(s, s.v_t.as<double>(), s.v.as<double>());
  launch_predictor(s);
  s.n_aug = 0;
  // a fixed barrier stiffness replaces sigma^0 and the growth rule
  s.sigma_set = d.sigma_fixed > 0.0;
  s.sigma = s.sigma0 = d.sigma_fixed > 0.0 ? d.sigma_fixed : 0.0;
  if (record) s.trace.clear();
  bal_step_stats S{};
  s.spmv_ms = 0.0;
  s.spmv_launches = 0;
  s.graph_launches = 0;
  auto tc = clk::now();
  int rc = build_candidates(s, s.cand, x, nullptr);
  if (rc) return rc;
  S.sec_collision += since(tc);
  double prev_min = INFINITY, e0 = -1.0;
  int status = BAL_E_NO_CONVERGENCE;
  // the last line search that accepted no step rejected some trial only for
  // exceeding the active-pair memory limit (Sec. 5.2)
  bool cap_blocked = false;
  for (int l = 0; l < d.max_newton; ++l) {
    tc = clk::now();
    launch_pair_distance(s, s.cand, x, s.cand.d.as<double>(), s.cand.cs.as<int>());
    double min_d = INFINITY;
    int n_active = 0;
    if ((rc = min_and_count(s, s.cand, dh, &min_d, &n_active))) return rc;
    S.sec_collision += since(tc);
    if (d.use_al) {
      if (min_d > 1e-2 * dh) {
        s.n_aug = 0;
      } else if (min_d < prev_min || s.n_aug == 0) {
        if ((rc = rebuild_aug(s, s.cand, 1e-2 * dh))) return rc;
      }
    }
    prev_min = min_d;
    if (!s.sigma_set && n_active > 0) {
      double s0;
      bool ok;
      if ((rc = compute_sigma0(s, x, s.cand, &s0, &ok))) return rc;
      if (ok) {
        s.sigma = s.sigma0 = s0;
        s.sigma_set = true;
      }
    }
    double sig = s.sigma_set ? s.sigma : 0.0;
    auto th = clk::now();
    if ((rc = build_union(s, s.cand))) return rc;
    if ((rc = linearize_at(s, x, 1, sig))) return rc;
    S.sec_hessian += since(th);
    double enorm = std::sqrt(dot_free(s, s.grad.as<double>(), s.grad.as<double>()));
    if (e0 < 0.0) e0 = enorm;
    S.n_active_max = std::max(S.n_active_max, n_active);
    S.n_aug_max = std::max(S.n_aug_max, s.n_aug);
    bool conv = enorm <= d.newton_rtol * e0;
    // search direction: warm start then global PCG on H dx = -e
    auto tp = clk::now();
    hipLaunchKernelGGL(k_neg, dim3(blocks_for(3 * s.N, 256)), dim3(256), 0, s.stream, s.grad.as<double>(),
                       s.rhs.as<double>(), 3 * s.N);
    int it_w = 0, it_g = 0;
    double rel = 0.0;
    if (d.warm_start) {
      if ((rc = warm_start_solve(s, s.rhs.as<double>(), dx, kWarmTol, d.warm_iters, &it_w))) return rc;
    }
    int prc = pcg_solve(s, s.rhs.as<double>(), dx, enorm, d.max_pcg, d.warm_start, 0, &it_g, &rel);
    if (prc != BAL_OK && prc != BAL_E_NO_CONVERGENCE) return prc;
    S.warm_iters += it_w;
    S.pcg_iters += it_g;
    S.sec_pcg += since(tp);
    // CCD bound and line search (Sec. 5.2, 5.3; App. B retry rule)
    double amax = 1.0, alpha = 0.0, L0 = 0.0;
    int retries = 0;
    for (;;) {
      auto tcc = clk::now();
      // swept candidates over [x, x + sw dx]: sw halves while the sweep is too
      // long for the hash or the pass exceeds its work bound
      double sw = sweep_limit(s, dx);
      const double *pp = dx;
      for (;;) {
        if (sw < 1.0) {
          if (s.psweep.grow(3 * (size_t)s.N * 8)) return BAL_E_OOM;
          hipLaunchKernelGGL(k_scale, dim3(blocks_for(3 * s.N, 256)), dim3(256), 0, s.stream, dx, sw,
                             s.psweep.as<double>(), 3 * s.N);
          pp = s.psweep.as<double>();
        }
        rc = build_candidates(s, s.cand2, x, pp);
        if (rc == BAL_E_CAPACITY && sw > 1e-30) {
          sw *= 0.5;
          continue;
        }
        if (rc) return rc;
        break;
      }
      if (s.tau.grow((size_t)(s.cand2.n + 1) * 8)) return BAL_E_OOM;
      launch_ccd(s, s.cand2, x, pp, s.tau.as<double>());
      amax = sw * std::min(1.0, s.cand2.n ? reduce_min(s, s.tau.as<double>(), s.cand2.n) : 1.0);
      S.sec_ccd += since(tcc);
      auto tl = clk::now();
      int valid, nact;
      if ((rc = energy_at(s, x, s.cand2, sig, &L0, &valid, &nact))) return rc;
      alpha = amax;
      bool accepted = false, over_cap = false;
      while (alpha >= 1e-9) {
        launch_axpy_state(s, xtr, x, dx, alpha, 3 * s.N);
        double L;
        if ((rc = energy_at(s, xtr, s.cand2, sig, &L, &valid, &nact))) return rc;
        if (valid && nact <= d.max_contacts && L <= L0) { accepted = true; break; }
        if (valid && L <= L0) over_cap = true;
        alpha *= 0.5;
      }
      S.sec_linesearch += since(tl);
      cap_blocked = !accepted && over_cap;
      if (accepted) break;
      if (conv || retries >= 10) {
        alpha = 0.0;
        copy3(s, xtr, x);
        break;
      }
      // resume the same PCG for 100 more iterations, then redo CCD and line search
      ++retries;
      ++S.ls_retries;
      auto tp2 = clk::now();
      int more = 0;
      prc = pcg_solve(s, s.rhs.as<double>(), dx, enorm, 100, 1, 1, &more, &rel);
      S.pcg_iters += std::max(0, more - it_g);
      it_g = more;
      S.sec_pcg += since(tp2);
    }
    if (record) {
      double row[8] = {(double)n_active, (double)s.n_aug, sig, std::min(min_d, dh), amax, alpha, enorm, (double)it_g};
      s.trace.insert(s.trace.end(), row, row + 8);
    }
    S.newton_iters = l + 1;
    S.grad_rel = e0 > 0.0 ? enorm / e0 : 0.0;
    if (s.verbose && (l % 25 == 0 || conv)) {
      std::fprintf(stderr, "[bal] Newton %d: |A| %d |A'| %d |e|/|e0| %.3e alpha_max %.3e alpha %.3e PCG %d (%.1f s)\n",
                   l, n_active, s.n_aug, S.grad_rel, amax, alpha, it_g, since(t_start));
      std::fflush(stderr);
    }
    if (conv) {
      copy3(s, x, xtr);
      status = BAL_OK;
      S.converged = 1;
      break;
    }
    if (s.n_aug == 0) {
      // no measurable step and nothing left to update: stalled
      double moved = alpha * std::sqrt(dot_free(s, dx, dx));
      if (moved <= 1e-15 * std::sqrt(dot_free(s, x, x))) {
        copy3(s, x, xtr);
        S.stalled = 1;
        if (enorm <= d.accept_rtol * e0) {
          status = BAL_OK;
          S.converged = 1;
        }
        break;
      }
    }
    // dual and penalty updates at the new iterate (Alg. 1, lines 12-17)
    if (s.n_aug) launch_aug_update(s, xtr);
    launch_pair_distance(s, s.cand2, xtr, s.cand2.d.as<double>(), s.cand2.cs.as<int>());
    double dmin_new = min_or(s, s.cand2, INFINITY);
    if (dmin_new < 1e-2 * dh && s.sigma_set && !(d.sigma_fixed > 0.0))
      s.sigma = std::max(1.2 * s.sigma, 100.0 * s.sigma0);
    copy3(s, x, xtr);
    std::swap(s.cand, s.cand2);
  }
  if (status != BAL_OK && cap_blocked) status = BAL_E_CAPACITY;
  hipLaunchKernelGGL(k_velocity, dim3(blocks_for(s.N, 256)), dim3(256), 0, s.stream, s.N, x, s.x_t.as<double>(),
                     s.freev.as<uint8_t>(), 1.0 / d.dt, s.v.as<double>());
  launch_pair_distance(s, s.cand, x, s.cand.d.as<double>(), s.cand.cs.as<int>());
  S.min_dist = std::min(dh, min_or(s, s.cand, INFINITY));
  S.sigma = s.sigma_set ? s.sigma : 0.0;
  S.spmv_ms = s.spmv_ms;
  S.spmv_launches = s.spmv_launches;
  S.graph_launches = s.graph_launches;
  S.spmv_bytes = cg_product_bytes(s);
  if ((rc = sync(s))) return rc;
  S.sec_total = since(t_start);
  s.last = S;
  if (st) *st = S;
  return status;
}

// ------------------------------------------------------------ construction
static void chol3(const double *G, double *L) {
  for (int i = 0; i < 9; ++i) L[i] = 0.0;
  for (int j = 0; j < 3; ++j) {
    double s = G[j * 3 + j];
    for (int k = 0; k < j; ++k) s -= L[j * 3 + k] * L[j * 3 + k];
    L[j * 3 + j] = std::sqrt(s);
    for (int i = j + 1; i < 3; ++i) {
      double t = G[i * 3 + j];
      for (int k = 0; k < j; ++k) t -= L[i * 3 + k] * L[j * 3 + k];
      L[i * 3 + j] = t / L[j * 3 + j];
    }
  }
}

static bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static int slot_of(int a, int b) {  // a < b
  static const int tab[4][4] = {{-1, 4, 5, 6}, {-1, -1, 7, 8}, {-1, -1, -1, 9}, {-1, -1, -1, -1}};
  return tab[a][b];
}

static int build_scene(Scene &s, const bal_scene_desc *d) {
  s.desc = *d;
  s.desc.rest_pos = nullptr; s.desc.tets = nullptr; s.desc.youngs = nullptr; s.desc.poisson = nullptr;
  s.desc.density = nullptr; s.desc.fixed = nullptr; s.desc.obs_pos = nullptr; s.desc.obs_tris = nullptr;
  s.desc.x0 = nullptr; s.desc.v0 = nullptr;
  s.dev = d->device;
  if (hipSetDevice(s.dev) != hipSuccess) return BAL_E_HIP;
  s.stream = static_cast<hipStream_t>(d->stream);
  if (s.stream == nullptr) {
    // graph capture needs a stream of our own; a blocking stream stays ordered with the NULL stream
    if (hipStreamCreateWithFlags(&s.stream, hipStreamDefault) != hipSuccess) return BAL_E_HIP;
    s.own_stream = true;
  }
  s.mixed = d->precision == BAL_MIXED;
  s.nb = d->n_verts;
  s.no = d->n_obs_verts;
  s.N = s.nb + s.no;
  s.T = d->n_tets;
  const int nb = s.nb, N = s.N, T = s.T;
  // element stencil basis
  {
    const double W[12] = {-1, 1, 0, 0, -1, 0, 1, 0, -1, 0, 0, 1};
    double G[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double t = 0.0;
        for (int k = 0; k < 4; ++k) t += W[i * 4 + k] * W[j * 4 + k];
        G[i * 3 + j] = t;
      }
    chol3(G, s.Lel);
    for (int c = 0; c < 4; ++c) {  // Q^T = L^{-1} W
      double y[3];
      for (int i = 0; i < 3; ++i) {
        double t = W[i * 4 + c];
        for (int k = 0; k < i; ++k) t -= s.Lel[i * 3 + k] * y[k];
        y[i] = t / s.Lel[i * 3 + i];
      }
      for (int i = 0; i < 3; ++i) s.Qel[c * 3 + i] = y[i];
    }
  }
  // rest data, masses
  std::vector<TetConst> tc(T);
  s.mass_h.assign(N, 0.0);
  s.youngs_h.assign(d->youngs, d->youngs + T);
  s.poisson_h.assign(d->poisson, d->poisson + T);
  const double *X = d->rest_pos;
  for (int t = 0; t < T; ++t) {
    const int *v = d->tets + 4 * t;
    double Dm[9];  // row-major, columns = edges
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) Dm[c * 3 + k] = X[3 * v[k + 1] + c] - X[3 * v[0] + c];
    double c00 = Dm[4] * Dm[8] - Dm[5] * Dm[7], c01 = Dm[5] * Dm[6] - Dm[3] * Dm[8], c02 = Dm[3] * Dm[7] - Dm[4] * Dm[6];
    double det = Dm[0] * c00 + Dm[1] * c01 + Dm[2] * c02;
    double V = det / 6.0;
    if (!(V > 0.0)) return BAL_E_INVERTED;
    double id = 1.0 / det;
    double B[9] = {c00 * id, (Dm[2] * Dm[7] - Dm[1] * Dm[8]) * id, (Dm[1] * Dm[5] - Dm[2] * Dm[4]) * id,
                   c01 * id, (Dm[0] * Dm[8] - Dm[2] * Dm[6]) * id, (Dm[2] * Dm[3] - Dm[0] * Dm[5]) * id,
                   c02 * id, (Dm[1] * Dm[6] - Dm[0] * Dm[7]) * id, (Dm[0] * Dm[4] - Dm[1] * Dm[3]) * id};
    double E = d->youngs[t], nu = d->poisson[t];
    double mu = E / (2.0 * (1.0 + nu)), lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    TetConst &k = tc[t];
    for (int i = 0; i < 9; ++i) k.B[i] = B[i];
    double BBt[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0.0;
        for (int q = 0; q < 3; ++q) a += B[i * 3 + q] * B[j * 3 + q];
        BBt[i * 3 + j] = a;
      }
    double A[9];  // L^T BB^T L
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        double a = 0.0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) a += s.Lel[i * 3 + p] * BBt[i * 3 + j] * s.Lel[j * 3 + q];
        A[p * 3 + q] = a;
      }
    k.A[0] = A[0]; k.A[1] = A[1]; k.A[2] = A[2]; k.A[3] = A[4]; k.A[4] = A[5]; k.A[5] = A[8];
    k.V = V;
    k.Vmu = V * mu;
    k.Vlam = V * lam;
    k.pad = 0.0;
    for (int a = 0; a < 4; ++a) s.mass_h[v[a]] += d->density[t] * V / 4.0;
  }
  s.free_h.assign(N, 0);
  for (int i = 0; i < nb; ++i) s.free_h[i] = d->fixed ? (d->fixed[i] ? 0 : 1) : 1;
  // a free vertex needs mass: one that belongs to no tet leaves the system singular
  for (int i = 0; i < nb; ++i)
    if (s.free_h[i] && !(s.mass_h[i] > 0.0)) return BAL_E_INVALID_ARG;
  // node -> tet incidence (tet*4 + local index), in tet order
  std::vector<int> ntp(N + 1, 0), nts(4 * (size_t)T);
  for (int t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) ntp[d->tets[4 * t + a] + 1]++;
  for (int i = 0; i < N; ++i) ntp[i + 1] += ntp[i];
  {
    std::vector<int> fill(ntp.begin(), ntp.end() - 1);
    for (int t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) nts[fill[d->tets[4 * t + a]]++] = 4 * t + a;
  }
  // surface: faces of exactly one tet (checked through the incidence of the face's first node)
  std::vector<int> tris;
  {
    const int fidx[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int t = 0; t < T; ++t) {
      const int *v = d->tets + 4 * t;
      for (int f = 0; f < 4; ++f) {
        int a = v[fidx[f][0]], b = v[fidx[f][1]], c = v[fidx[f][2]];
        bool shared = false;
        for (int k = ntp[a]; k < ntp[a + 1] && !shared; ++k) {
          int u = nts[k] >> 2;
          if (u == t) continue;
          const int *w = d->tets + 4 * u;
          bool hb = false, hc = false;
          for (int q = 0; q < 4; ++q) { hb |= w[q] == b; hc |= w[q] == c; }
          shared = hb && hc;
        }
        if (!shared) {
          int tri[3] = {a, b, c};
          std::sort(tri, tri + 3);
          tris.insert(tris.end(), tri, tri + 3);
        }
      }
    }
  }
  size_t nbt = tris.size() / 3;
  for (int k = 0; k < d->n_obs_tris; ++k)
    for (int c = 0; c < 3; ++c) tris.push_back(nb + d->obs_tris[3 * k + c]);
  s.nst = (int)(tris.size() / 3);
  std::vector<uint64_t> ekeys;
  for (int k = 0; k < s.nst; ++k) {
    int v3_[3] = {tris[3 * k], tris[3 * k + 1], tris[3 * k + 2]};
    for (int e = 0; e < 3; ++e) {
      int a = v3_[e], b = v3_[(e + 1) % 3];
      if (a > b) std::swap(a, b);
      ekeys.push_back(((uint64_t)a << 32) | (uint64_t)b);
    }
  }
  std::sort(ekeys.begin(), ekeys.end());
  ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
  s.nse = (int)ekeys.size();
  s.se_h.resize(2 * (size_t)s.nse);
  double elen = 0.0;
  for (int k = 0; k < s.nse; ++k) {
    int a = (int)(ekeys[k] >> 32), b = (int)(ekeys[k] & 0xffffffffu);
    s.se_h[2 * k] = a;
    s.se_h[2 * k + 1] = b;
  }
  std::vector<char> onsurf(N, 0);
  for (size_t k = 0; k < nbt * 3; ++k) onsurf[tris[k]] = 1;
  for (int i = nb; i < N; ++i) onsurf[i] = 1;
  s.sv_h.clear();
  for (int i = 0; i < N; ++i)
    if (onsurf[i]) s.sv_h.push_back(i);
  s.nsv = (int)s.sv_h.size();
  s.st_h = tris;
  // positions at rest for the cell size: mean body surface edge length
  std::vector<double> Xall(3 * (size_t)N);
  for (int i = 0; i < nb; ++i)
    for (int c = 0; c < 3; ++c) Xall[3 * i + c] = X[3 * i + c];
  for (int i = 0; i < s.no; ++i)
    for (int c = 0; c < 3; ++c) Xall[3 * (nb + i) + c] = d->obs_pos[3 * i + c];
  int cnt = 0;
  for (int k = 0; k < s.nse; ++k) {
    int a = s.se_h[2 * k], b = s.se_h[2 * k + 1];
    if (a >= nb || b >= nb) continue;
    double l2 = 0.0;
    for (int c = 0; c < 3; ++c) l2 += (Xall[3 * a + c] - Xall[3 * b + c]) * (Xall[3 * a + c] - Xall[3 * b + c]);
    elen += std::sqrt(l2);
    ++cnt;
  }
  s.cell = cnt ? elen / cnt : 1.0;
  if (s.cell < 4.0 * d->dhat) s.cell = 4.0 * d->dhat;
  // strictly lower block pattern over free nodes with element sources; the
  // upper triangle is read through the transposed index built below
  std::vector<int> rp(N + 1, 0), ci, bsp(1, 0), bsrc;
  {
    std::vector<std::pair<int, int>> ent;
    for (int i = 0; i < N; ++i) {
      ent.clear();
      if (s.free_h[i]) {
        for (int k = ntp[i]; k < ntp[i + 1]; ++k) {
          int t = nts[k] >> 2, a = nts[k] & 3;
          const int *v = d->tets + 4 * t;
          for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
            int j = v[b];
            if (j >= i || !s.free_h[j]) continue;
            int src = a < b ? (10 * t + slot_of(a, b)) : (int)((unsigned)(10 * t + slot_of(b, a)) | 0x80000000u);
            ent.push_back({j, src});
          }
        }
        std::sort(ent.begin(), ent.end(), [](const std::pair<int, int> &p, const std::pair<int, int> &q) {
          return p.first != q.first ? p.first < q.first : (unsigned)p.second < (unsigned)q.second;
        });
      }
      for (size_t e = 0; e < ent.size();) {
        int j = ent[e].first;
        ci.push_back(j);
        while (e < ent.size() && ent[e].first == j) bsrc.push_back(ent[e++].second);
        bsp.push_back((int)bsrc.size());
      }
      rp[i + 1] = (int)ci.size();
    }
  }
  s.nnzb = (int)ci.size();
  s.nsrc = (int)bsrc.size();
  // transposed index: row j lists the stored blocks (i, j), ascending i
  std::vector<int> upp(N + 1, 0);
  std::vector<int2> upe(s.nnzb + 1);
  for (int k = 0; k < s.nnzb; ++k) upp[ci[k] + 1]++;
  for (int i = 0; i < N; ++i) upp[i + 1] += upp[i];
  {
    std::vector<int> fill(upp.begin(), upp.end() - 1);
    for (int i = 0; i < N; ++i)
      for (int k = rp[i]; k < rp[i + 1]; ++k) upe[fill[ci[k]]++] = make_int2(i, k);
  }
  // pad entries closing both lists (lower: column 0; transposed: operand 0
  // and the spare block), read by the branch-free FP64 walk in place of an
  // entry of the other list or past the row's end
  upe[s.nnzb] = make_int2(0, s.nnzb);
  // FP32 storage also keeps one entry list per row: (column, block) of its
  // lower blocks, then (row, block) of its transposed ones; a dummy entry
  // (operand 0, the spare block) closes the list
  std::vector<int2> entl;
  if (s.mixed) {
    entl.resize((size_t)2 * s.nnzb + 1);
    size_t o = 0;
    for (int i = 0; i < N; ++i) {
      for (int k = rp[i]; k < rp[i + 1]; ++k) entl[o++] = make_int2(ci[k], k);
      for (int e = upp[i]; e < upp[i + 1]; ++e) entl[o++] = upe[e];
    }
    entl[o] = make_int2(0, s.nnzb);
  }
  ci.push_back(0);
  // device uploads
  std::vector<int4> tet4(T);
  for (int t = 0; t < T; ++t) tet4[t] = make_int4(d->tets[4 * t], d->tets[4 * t + 1], d->tets[4 * t + 2], d->tets[4 * t + 3]);
  int rc;
  if ((rc = upload(s, s.tets, tet4.data(), T)) || (rc = upload(s, s.tc, tc.data(), T)) ||
      (rc = upload(s, s.mass, s.mass_h.data(), N)) || (rc = upload(s, s.freev, s.free_h.data(), N)) ||
      (rc = upload(s, s.node_tet_ptr, ntp.data(), N + 1)) || (rc = upload(s, s.node_tet_src, nts.data(), nts.size())) ||
      (rc = upload(s, s.row_ptr, rp.data(), N + 1)) || (rc = upload(s, s.col_idx, ci.data(), ci.size())) ||
      (rc = upload(s, s.blk_src_ptr, bsp.data(), bsp.size())) || (rc = upload(s, s.blk_src, bsrc.data(), bsrc.size())) ||
      (rc = upload(s, s.up_ptr, upp.data(), N + 1)) || (rc = upload(s, s.up_ent, upe.data(), upe.size())) ||
      (s.mixed && (rc = upload(s, s.ent, entl.data(), entl.size()))) ||
      (rc = upload(s, s.sv, s.sv_h.data(), s.sv_h.size())) || (rc = upload(s, s.st, s.st_h.data(), s.st_h.size())) ||
      (rc = upload(s, s.se, s.se_h.data(), s.se_h.size())))
    return rc;
  size_t w = s.mixed ? 4 : 8;
  size_t n3 = 3 * (size_t)N;
  if (s.x.grow(n3 * 8) || s.v.grow(n3 * 8) || s.x_t.grow(n3 * 8) || s.v_t.grow(n3 * 8) || s.y.grow(n3 * 8) ||
      s.xtrial.grow(n3 * 8) || s.dx.grow(n3 * 8) || s.grad.grow(n3 * 8) || s.grad_b.grow(n3 * 8) ||
      s.rhs.grow(n3 * 8) || s.r.grow(n3 * 8) || s.z.grow(n3 * w) || s.pv.grow(n3 * w) || s.q.grow(n3 * w) ||
      s.tet_e.grow((size_t)T * 8) || s.tet_g.grow((size_t)T * 12 * 8) || s.tet_tr.grow((size_t)T * 8) ||
      s.tet_blk.grow((size_t)T * 90 * w) || s.val.grow((size_t)(s.nnzb + 1) * 9 * w) || s.Dblk.grow((size_t)N * 9 * w) ||
      s.Dinv.grow((size_t)N * 9 * w) || s.e_nodes.grow((size_t)N * 8) || s.group.grow((size_t)N * 4) ||
      s.node_e.grow((size_t)N * 8) || s.pcg_ctl.grow(4096) || s.counter.grow(64) ||
      s.red_out.grow(2048 * 8) || s.flags.grow(64) || grow_aug(s, 1) || grow_pair_list(s.uni, 1) ||
      s.uni_flag.grow(64) || s.uni_aug.grow(64) || s.pair_e.grow(64) || s.pair_g.grow(12 * 8) ||
      s.pair_tr.grow(64) || s.pair_blk.grow(144 * 8))
    return BAL_E_OOM;
  if (hipHostMalloc(&s.pin.p, 1 << 16) != hipSuccess) return BAL_E_OOM;
  for (hipEvent_t &e : s.pipe_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return BAL_E_HIP;
  s.pin.bytes = 1 << 16;
  hipMemsetAsync(s.flags.p, 0, 64, s.stream);
  hipMemsetAsync(s.counter.p, 0, 64, s.stream);
  // the spare block (read by lanes past a row's end, whose product is dropped)
  hipMemsetAsync(static_cast<char *>(s.val.p) + (size_t)s.nnzb * 9 * w, 0, 9 * w, s.stream);
  // empty contact lists
  if ((rc = build_contact_lists(s))) return rc;
  // initial state
  std::vector<double> x0(n3), v0(n3, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int c = 0; c < 3; ++c) {
      x0[3 * i + c] = d->x0 ? d->x0[3 * i + c] : X[3 * i + c];
      v0[3 * i + c] = (d->v0 && s.free_h[i]) ? d->v0[3 * i + c] : 0.0;
    }
  for (int i = 0; i < s.no; ++i)
    for (int c = 0; c < 3; ++c) x0[3 * (nb + i) + c] = d->obs_pos[3 * i + c];
  if (hipMemcpyAsync(s.x.p, x0.data(), n3 * 8, hipMemcpyHostToDevice, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.v.p, v0.data(), n3 * 8, hipMemcpyHostToDevice, s.stream) != hipSuccess)
    return BAL_E_HIP;
  // feasibility of the initial state: every tet J > 0, every pair d > 0
  launch_elements(s, s.x.as<double>(), EM_ENERGY, 0);
  if (read_flags_and_clear(s)) return BAL_E_INVERTED;
  if ((rc = build_candidates(s, s.cand, s.x.as<double>(), nullptr))) return rc;
  launch_pair_distance(s, s.cand, s.x.as<double>(), s.cand.d.as<double>(), s.cand.cs.as<int>());
  if (s.cand.n && !(reduce_min(s, s.cand.d.as<double>(), s.cand.n) > 0.0)) return BAL_E_PENETRATION;
  return sync(s);
}

static int validate_desc(const bal_scene_desc *d) {
  if (!d || d->n_verts <= 0 || d->n_tets < 0 || !d->rest_pos || (d->n_tets && (!d->tets || !d->youngs || !d->poisson || !d->density)))
    return BAL_E_INVALID_ARG;
  if (d->n_obs_verts < 0 || d->n_obs_tris < 0 || (d->n_obs_verts && !d->obs_pos) || (d->n_obs_tris && !d->obs_tris))
    return BAL_E_INVALID_ARG;
  if (!(d->dt > 0.0) || !(d->dhat > 0.0) || !std::isfinite(d->dt) || !std::isfinite(d->dhat)) return BAL_E_INVALID_ARG;
  if (!(d->sigma_fixed >= 0.0) || !std::isfinite(d->sigma_fixed)) return BAL_E_INVALID_ARG;
  if (!(d->friction >= 0.0) || !std::isfinite(d->friction) || !std::isfinite(d->eps_v)) return BAL_E_INVALID_ARG;
  if (!(d->accept_rtol >= 0.0) || !std::isfinite(d->accept_rtol)) return BAL_E_INVALID_ARG;
  if (!finite_all(d->rest_pos, 3 * (size_t)d->n_verts) || !finite_all(d->gravity, 3)) return BAL_E_INVALID_ARG;
  if (d->n_tets && (!finite_all(d->youngs, d->n_tets) || !finite_all(d->poisson, d->n_tets) ||
                    !finite_all(d->density, d->n_tets)))
    return BAL_E_INVALID_ARG;
  for (int t = 0; t < d->n_tets; ++t) {
    if (!(d->youngs[t] > 0.0) || !(d->poisson[t] > -1.0 && d->poisson[t] < 0.5) || !(d->density[t] > 0.0))
      return BAL_E_INVALID_ARG;
    for (int a = 0; a < 4; ++a)
      if (d->tets[4 * t + a] < 0 || d->tets[4 * t + a] >= d->n_verts) return BAL_E_INVALID_ARG;
  }
  if (d->x0 && !finite_all(d->x0, 3 * (size_t)d->n_verts)) return BAL_E_INVALID_ARG;
  if (d->v0 && !finite_all(d->v0, 3 * (size_t)d->n_verts)) return BAL_E_INVALID_ARG;
  if (d->n_obs_verts && !finite_all(d->obs_pos, 3 * (size_t)d->n_obs_verts)) return BAL_E_INVALID_ARG;
  for (int k = 0; k < 3 * d->n_obs_tris; ++k)
    if (d->obs_tris[k] < 0 || d->obs_tris[k] >= d->n_obs_verts) return BAL_E_INVALID_ARG;
  if (d->max_newton <= 0 || d->max_pcg <= 0 || d->precision < 0 || d->precision > 1) return BAL_E_INVALID_ARG;
  if (d->ccd_rule < BAL_CCD_PRINTED || d->ccd_rule > BAL_CCD_LITERAL || d->sweep_cap < 0) return BAL_E_INVALID_ARG;
  if (d->broad_phase != BAL_BROAD_HASH && d->broad_phase != BAL_BROAD_LBVH) return BAL_E_INVALID_ARG;
  return BAL_OK;
}

}  // namespace bal

using namespace bal;

struct bal_scene {
  Scene s;
};

extern "C" {

void bal_desc_defaults(bal_scene_desc *d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->dt = 1.0 / 30.0;
  d->gravity[1] = -9.8;
  d->dhat = 1e-3;
  d->newton_rtol = 1e-4;
  d->pcg_rtol = 1e-4;
  d->max_newton = 1000;
  d->max_pcg = 20000;
  d->pcg_stall_window = 100;
  d->max_contacts = 1 << 24;
  d->warm_iters = 100;
  d->precision = BAL_FP64;
  d->warm_start = 1;
  d->use_al = 1;
}

// ---- the caller's vertex order at the boundary
__global__ void k_gather_body3(int nb, const int *__restrict__ perm, const double *__restrict__ ext,
                               double *__restrict__ in) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int o = perm[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) in[3 * i + c] = ext[3 * o + c];
}
__global__ void k_scatter_body3(int nb, const int *__restrict__ perm, const double *__restrict__ in,
                                double *__restrict__ ext) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int o = perm[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) ext[3 * o + c] = in[3 * i + c];
}

// The caller's [rows][3] array (rows = n_verts: body; rows = N: body then
// obstacles), host or device, into the internal order at dst (device).
static int import3(Scene &s, const double *ext, double *dst, int rows, bool on_device) {
  const size_t bytes = 3 * (size_t)rows * 8;
  if (hipMemcpyAsync(s.stage.p, ext, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                     s.stream) != hipSuccess)
    return BAL_E_HIP;
  hipLaunchKernelGGL(k_gather_body3, dim3(blocks_for(s.nb, 256)), dim3(256), 0, s.stream, s.nb, s.perm_d.as<int>(),
                     s.stage.as<double>(), dst);
  if (rows > s.nb)
    hipMemcpyAsync(dst + 3 * (size_t)s.nb, s.stage.as<double>() + 3 * (size_t)s.nb, 3 * (size_t)(rows - s.nb) * 8,
                   hipMemcpyDeviceToDevice, s.stream);
  return BAL_OK;
}
// Internal device array src to the caller's order at ext (host or device);
// a host destination is complete after the stream is synchronised.
static int export3(Scene &s, const double *src, double *ext, int rows, bool on_device) {
  const size_t bytes = 3 * (size_t)rows * 8;
  hipLaunchKernelGGL(k_scatter_body3, dim3(blocks_for(s.nb, 256)), dim3(256), 0, s.stream, s.nb, s.perm_d.as<int>(),
                     src, s.stage.as<double>());
  if (rows > s.nb)
    hipMemcpyAsync(s.stage.as<double>() + 3 * (size_t)s.nb, src + 3 * (size_t)s.nb, 3 * (size_t)(rows - s.nb) * 8,
                   hipMemcpyDeviceToDevice, s.stream);
  return hip_ok(hipMemcpyAsync(ext, s.stage.p, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               s.stream));
}
static inline int ext_vertex(const Scene &s, int v) { return v < s.nb ? s.perm_h[v] : v; }

// Internal vertex order: the tet-connected pieces of the body one after the
// other (in the order of their first caller index), each in Morton order
// (10 bits per axis over the piece's own bounding box) of its rest
// positions.  Vertices close in space get close indices, so the rows that
// share matrix blocks and vector entries are processed close together and
// their second uses meet in cache; keeping a piece contiguous keeps the
// partners of its rows in the same stretch of rows (and on the same XCD,
// which takes a contiguous stretch of the product's tiles).  Returns
// internal -> caller index.
static std::vector<int> morton_order(const double *X, const int32_t *tets, int n, int T) {
  std::vector<int> root(n);
  for (int i = 0; i < n; ++i) root[i] = i;
  auto find = [&](int a) {
    while (root[a] != a) a = root[a] = root[root[a]];
    return a;
  };
  for (int t = 0; t < T; ++t)
    for (int k = 1; k < 4; ++k) {
      int a = find(tets[4 * t]), b = find(tets[4 * t + k]);
      if (a != b) root[std::max(a, b)] = std::min(a, b);  // a piece's root is its smallest index
    }
  std::vector<int> piece(n, -1), first;  // piece rank in order of first index
  for (int i = 0; i < n; ++i) {
    int r = find(i);
    if (piece[r] < 0) {
      piece[r] = (int)first.size();
      first.push_back(r);
    }
    piece[i] = piece[r];
  }
  const int np = (int)first.size();
  std::vector<double> lo(3 * (size_t)np, INFINITY), hi(3 * (size_t)np, -INFINITY);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      lo[3 * piece[i] + c] = std::min(lo[3 * piece[i] + c], X[3 * i + c]);
      hi[3 * piece[i] + c] = std::max(hi[3 * piece[i] + c], X[3 * i + c]);
    }
  auto spread = [](uint64_t v) {  // 10 bits to every third bit
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x30000ffULL;
    v = (v | (v << 8)) & 0x300f00fULL;
    v = (v | (v << 4)) & 0x30c30c3ULL;
    v = (v | (v << 2)) & 0x9249249ULL;
    return v;
  };
  std::vector<std::pair<uint64_t, int>> key(n);
  for (int i = 0; i < n; ++i) {
    uint64_t q[3];
    const int b = piece[i];
    for (int c = 0; c < 3; ++c) {
      double ext = hi[3 * b + c] - lo[3 * b + c];
      double f = ext > 0.0 ? (X[3 * i + c] - lo[3 * b + c]) / ext : 0.0;
      q[c] = (uint64_t)std::min(1023.0, std::max(0.0, std::floor(f * 1024.0)));
    }
    key[i] = {((uint64_t)b << 30) | spread(q[0]) | (spread(q[1]) << 1) | (spread(q[2]) << 2), i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = key[i].second;
  return perm;
}

int bal_create_scene(const bal_scene_desc *desc, bal_scene **out) {
  if (!out) return BAL_E_INVALID_ARG;
  *out = nullptr;
  int rc = validate_desc(desc);
  if (rc) return rc;
  bal_scene *h = new (std::nothrow) bal_scene();
  if (!h) return BAL_E_OOM;
  try {
    // the caller's arrays in the internal vertex order
    const int nb = desc->n_verts, T = desc->n_tets;
    std::vector<int> perm = morton_order(desc->rest_pos, desc->tets, nb, T), inv(nb);
    for (int i = 0; i < nb; ++i) inv[perm[i]] = i;
    std::vector<double> X(3 * (size_t)nb), x0, v0;
    std::vector<uint8_t> fx;
    std::vector<int32_t> tets(4 * (size_t)T);
    for (int i = 0; i < nb; ++i)
      for (int c = 0; c < 3; ++c) X[3 * i + c] = desc->rest_pos[3 * perm[i] + c];
    for (size_t k = 0; k < tets.size(); ++k) tets[k] = inv[desc->tets[k]];
    bal_scene_desc d = *desc;
    d.rest_pos = X.data();
    d.tets = tets.data();
    if (desc->x0) {
      x0.resize(3 * (size_t)nb);
      for (int i = 0; i < nb; ++i)
        for (int c = 0; c < 3; ++c) x0[3 * i + c] = desc->x0[3 * perm[i] + c];
      d.x0 = x0.data();
    }
    if (desc->v0) {
      v0.resize(3 * (size_t)nb);
      for (int i = 0; i < nb; ++i)
        for (int c = 0; c < 3; ++c) v0[3 * i + c] = desc->v0[3 * perm[i] + c];
      d.v0 = v0.data();
    }
    if (desc->fixed) {
      fx.resize(nb);
      for (int i = 0; i < nb; ++i) fx[i] = desc->fixed[perm[i]];
      d.fixed = fx.data();
    }
    h->s.perm_h = perm;
    // BAL_VERBOSE=1 in the environment: one progress line per 25 Newton iterations on stderr
    const char *vb = std::getenv("BAL_VERBOSE");
    h->s.verbose = vb && vb[0] == '1';
    rc = build_scene(h->s, &d);
    if (!rc) rc = upload(h->s, h->s.perm_d, perm.data(), std::max(nb, 1));
    if (!rc && h->s.stage.grow(3 * (size_t)h->s.N * 8 + 8)) rc = BAL_E_OOM;
  } catch (...) {
    rc = BAL_E_OOM;
  }
  if (rc) {
    bal_destroy_scene(h);
    return rc;
  }
  *out = h;
  return BAL_OK;
}

void bal_destroy_scene(bal_scene *h) {
  if (!h) return;
  Scene &s = h->s;
  hipSetDevice(s.dev);
  hipStreamSynchronize(s.stream);
  DBuf *bufs[] = {&s.tets, &s.tc, &s.mass, &s.freev, &s.node_tet_ptr, &s.node_tet_src, &s.row_ptr, &s.col_idx,
                  &s.blk_src_ptr, &s.blk_src, &s.up_ptr, &s.up_ent, &s.ent, &s.perm_d, &s.stage, &s.sv, &s.st, &s.se, &s.x, &s.v, &s.x_t, &s.v_t, &s.y,
                  &s.xtrial, &s.dx, &s.tet_e, &s.tet_g, &s.tet_tr, &s.tet_blk, &s.val, &s.Dblk, &s.Dinv, &s.e_nodes,
                  &s.group, &s.grad, &s.grad_b, &s.uni_flag, &s.uni_aug, &s.pair_e, &s.pair_g, &s.pair_tr,
                  &s.pair_blk, &s.cdiag_ptr, &s.cdiag_src, &s.coff_ptr, &s.coff_col, &s.coff_src, &s.cm_ptr, &s.cm_col, &s.cm_blk, &s.cm_head, &s.cm_ridx, &s.ccount,
                  &s.cfill, &s.aug_kind, &s.aug_a, &s.aug_b, &s.aug_nodes, &s.aug_key, &s.aug_mu, &s.aug_s,
                  &s.aug_d, &s.aug_e, &s.aug_tmp_mu, &s.aug_tmp_s, &s.fr, &s.fr_e, &s.hb_lo, &s.hb_hi, &s.hq_lo, &s.hq_hi,
                  &s.h_cnt, &s.h_off, &s.h_key, &s.h_prim, &s.h_bcnt, &s.h_bstart, &s.h_bfill, &s.h_skey,
                  &s.h_sprim, &s.h_large, &s.h_nlarge, &s.h_qcnt, &s.h_lcnt, &s.h_slots, &s.h_plen, &s.h_qoff, &s.h_out, &s.qoff_pt, &s.out_pt,
                  &s.qoff_ee, &s.out_ee, &s.lb_part, &s.lb_key, &s.lb_key2, &s.lb_tmp, &s.lb_prim, &s.lb_child,
                  &s.lb_parent, &s.lb_lparent, &s.lb_arrive, &s.lb_ibox, &s.h_sorted_pt, &s.h_sorted_ee, &s.r, &s.z, &s.pv, &s.pv2, &s.q, &s.pcg_ctl, &s.warm_ctl, &s.partial, &s.red_slots, &s.counter,
                  &s.scan_tmp, &s.red_out, &s.flags, &s.node_e, &s.cand_e, &s.mask, &s.mask_off, &s.tau, &s.rhs, &s.psweep};
  for (DBuf *b : bufs) b->release();
  PairList *pls[] = {&s.cand, &s.cand2, &s.uni, &s.augtmp};
  for (PairList *pl : pls) {
    DBuf *pb[] = {&pl->kind, &pl->a, &pl->b, &pl->nodes, &pl->d, &pl->cs, &pl->key};
    for (DBuf *b : pb) b->release();
  }
  if (s.pin.p) hipHostFree(s.pin.p);
  for (hipEvent_t e : s.ev_pool) hipEventDestroy(e);
  if (s.cg_exec) hipGraphExecDestroy(s.cg_exec);
  for (hipEvent_t e : s.pipe_ev)
    if (e) hipEventDestroy(e);
  if (s.warm_exec) hipGraphExecDestroy(s.warm_exec);
  if (s.own_stream && s.stream) hipStreamDestroy(s.stream);
  delete h;
}

const char *bal_status_string(int status) {
  switch (status) {
    case BAL_OK: return "ok";
    case BAL_E_INVALID_ARG: return "invalid argument";
    case BAL_E_OOM: return "out of device memory";
    case BAL_E_HIP: return "HIP runtime error";
    case BAL_E_PENETRATION: return "initial state has a pair at zero distance";
    case BAL_E_INVERTED: return "inverted or degenerate tetrahedron";
    case BAL_E_CAPACITY: return "active pairs exceed max_contacts";
    case BAL_E_NO_CONVERGENCE: return "not converged (Newton iteration cap, a stalled step, or an adjoint solve "
                                      "above its tolerance)";
    case BAL_E_INDEFINITE: return "Hessian not positive definite at the converged state (no adjoint)";
    case BAL_E_STATE: return "call out of order";
    default: return "unknown status";
  }
}

int bal_step(bal_scene *h, bal_step_stats *stats) {
  if (!h) return BAL_E_INVALID_ARG;
  hipSetDevice(h->s.dev);
  try {
    return newton_solve(h->s, stats, true);
  } catch (...) {
    return BAL_E_OOM;
  }
}

int bal_get_state(const bal_scene *h, double *x_out, double *v_out, int on_device) {
  if (!h) return BAL_E_INVALID_ARG;
  const Scene &s = h->s;
  hipSetDevice(s.dev);
  Scene &sm = const_cast<Scene &>(s);  // the staging buffer is scratch
  int rc;
  if (x_out && (rc = export3(sm, s.x.as<double>(), x_out, s.nb, on_device != 0))) return rc;
  if (v_out && (rc = export3(sm, s.v.as<double>(), v_out, s.nb, on_device != 0))) return rc;
  return hip_ok(hipStreamSynchronize(s.stream));
}

int bal_set_state(bal_scene *h, const double *x, const double *v, int on_device) {
  if (!h) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  hipSetDevice(s.dev);
  size_t bytes = (size_t)3 * s.nb * 8;
  if (!on_device) {
    if ((x && !finite_all(x, 3 * (size_t)s.nb)) || (v && !finite_all(v, 3 * (size_t)s.nb))) return BAL_E_INVALID_ARG;
  }
  (void)bytes;
  int rc;
  if (x && (rc = import3(s, x, s.x.as<double>(), s.nb, on_device != 0))) return rc;
  if (v) {
    if ((rc = import3(s, v, s.v.as<double>(), s.nb, on_device != 0))) return rc;
    // fixed vertices keep zero velocity
    const std::vector<uint8_t> &fr = s.free_h;
    std::vector<double> vh(3 * (size_t)s.N);
    hipMemcpyAsync(vh.data(), s.v.p, 3 * (size_t)s.N * 8, hipMemcpyDeviceToHost, s.stream);
    hipStreamSynchronize(s.stream);
    for (int i = 0; i < s.N; ++i)
      if (!fr[i])
        for (int c = 0; c < 3; ++c) vh[3 * i + c] = 0.0;
    hipMemcpyAsync(s.v.p, vh.data(), 3 * (size_t)s.N * 8, hipMemcpyHostToDevice, s.stream);
  }
  return hip_ok(hipStreamSynchronize(s.stream));
}

int bal_set_youngs(bal_scene *h, const double *E, int on_device) {
  if (!h || !E) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  hipSetDevice(s.dev);
  std::vector<double> Eh(s.T);
  if (on_device) {
    hipMemcpy(Eh.data(), E, (size_t)s.T * 8, hipMemcpyDeviceToHost);
  } else {
    std::copy(E, E + s.T, Eh.begin());
  }
  for (int t = 0; t < s.T; ++t)
    if (!(Eh[t] > 0.0) || !std::isfinite(Eh[t])) return BAL_E_INVALID_ARG;
  std::vector<TetConst> tc(s.T);
  hipMemcpy(tc.data(), s.tc.p, (size_t)s.T * sizeof(TetConst), hipMemcpyDeviceToHost);
  for (int t = 0; t < s.T; ++t) {
    double nu = s.poisson_h[t];
    double mu = Eh[t] / (2.0 * (1.0 + nu)), lam = Eh[t] * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    tc[t].Vmu = tc[t].V * mu;
    tc[t].Vlam = tc[t].V * lam;
  }
  s.youngs_h = Eh;
  if (hipMemcpy(s.tc.p, tc.data(), (size_t)s.T * sizeof(TetConst), hipMemcpyHostToDevice) != hipSuccess) return BAL_E_HIP;
  return BAL_OK;
}

int bal_get_trace(const bal_scene *h, double *rows, int32_t capacity, int32_t *n_rows) {
  if (!h || !n_rows) return BAL_E_INVALID_ARG;
  const Scene &s = h->s;
  int n = (int)(s.trace.size() / 8);
  *n_rows = n;
  if (rows) std::copy(s.trace.begin(), s.trace.begin() + 8 * std::min(n, (int)capacity), rows);
  return BAL_OK;
}

int bal_set_kernel_timing(bal_scene *h, int on) {
  if (!h) return BAL_E_INVALID_ARG;
  h->s.time_kernels = on != 0;
  return BAL_OK;
}

int bal_get_surface(const bal_scene *h, int32_t *n_sv, int32_t *verts, int32_t *n_st, int32_t *tris, int32_t *n_se,
                    int32_t *edges) {
  if (!h) return BAL_E_INVALID_ARG;
  const Scene &s = h->s;
  if (n_sv) *n_sv = s.nsv;
  if (n_st) *n_st = s.nst;
  if (n_se) *n_se = s.nse;
  if (verts)
    for (size_t k = 0; k < s.sv_h.size(); ++k) verts[k] = ext_vertex(s, s.sv_h[k]);
  if (tris)
    for (size_t k = 0; k < s.st_h.size(); ++k) tris[k] = ext_vertex(s, s.st_h[k]);
  if (edges)
    for (size_t k = 0; k < s.se_h.size(); ++k) edges[k] = ext_vertex(s, s.se_h[k]);
  return BAL_OK;
}

int bal_linearize(bal_scene *h, const double *x_all, const bal_al_state *al, int project, double *energy,
                  double *grad_all, int32_t *n_active) {
  if (!h || !x_all) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  hipSetDevice(s.dev);
  size_t n3 = 3 * (size_t)s.N;
  if (!finite_all(x_all, n3)) return BAL_E_INVALID_ARG;
  // predictor from the current state
  copy3(s, s.x_t.as<double>(), s.x.as<double>());
  copy3(s, s.v_t.as<double>(), s.v.as<double>());
  launch_predictor(s);
  double *x = s.xtrial.as<double>();
  int rcx = import3(s, x_all, x, s.N, false);
  if (rcx) return rcx;
  // A' from the caller: nodes and canonical keys from the surface lists, sorted by key
  int na = al ? al->n_aug : 0;
  std::vector<int> idx(na);
  std::vector<uint64_t> key(na);
  std::vector<int> kind(na), pa(na), pb(na);
  std::vector<int4> nodes(na);
  for (int j = 0; j < na; ++j) {
    int k = al->aug_kind[j], a = al->aug_prims[2 * j], b = al->aug_prims[2 * j + 1];
    if (k == 0) {
      if (a < 0 || a >= s.nsv || b < 0 || b >= s.nst) return BAL_E_INVALID_ARG;
      nodes[j] = make_int4(s.sv_h[a], s.st_h[3 * b], s.st_h[3 * b + 1], s.st_h[3 * b + 2]);
    } else {
      if (a < 0 || a >= s.nse || b < 0 || b >= s.nse || a == b) return BAL_E_INVALID_ARG;
      if (a > b) std::swap(a, b);
      nodes[j] = make_int4(s.se_h[2 * a], s.se_h[2 * a + 1], s.se_h[2 * b], s.se_h[2 * b + 1]);
    }
    kind[j] = k; pa[j] = a; pb[j] = b;
    key[j] = ((uint64_t)k << 62) | ((uint64_t)a << 31) | (uint64_t)b;
  }
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int i, int j) { return key[i] < key[j]; });
  std::vector<int> k2(na), a2(na), b2(na);
  std::vector<int4> n2(na);
  std::vector<uint64_t> key2(na);
  std::vector<double> mu2(na), s2(na);
  for (int j = 0; j < na; ++j) {
    int i = idx[j];
    k2[j] = kind[i]; a2[j] = pa[i]; b2[j] = pb[i]; n2[j] = nodes[i]; key2[j] = key[i];
    mu2[j] = al->mu[i]; s2[j] = al->s[i];
  }
  if (grow_aug(s, na)) return BAL_E_OOM;
  s.n_aug = na;
  if (na) {
    upload(s, s.aug_kind, k2.data(), na); upload(s, s.aug_a, a2.data(), na); upload(s, s.aug_b, b2.data(), na);
    upload(s, s.aug_nodes, n2.data(), na); upload(s, s.aug_key, key2.data(), na);
    upload(s, s.aug_mu, mu2.data(), na); upload(s, s.aug_s, s2.data(), na);
  }
  double sigma = al ? al->sigma : 0.0;
  int rc = build_candidates(s, s.cand, x, nullptr);
  if (rc) return rc;
  launch_pair_distance(s, s.cand, x, s.cand.d.as<double>(), s.cand.cs.as<int>());
  if ((rc = build_union(s, s.cand))) return rc;
  if ((rc = linearize_at(s, x, project, sigma))) return rc;
  int valid, nact;
  double L;
  if ((rc = energy_at(s, x, s.cand, sigma, &L, &valid, &nact))) return rc;
  if (energy) *energy = valid ? L : INFINITY;
  if (n_active) *n_active = nact;
  if (grad_all && (rc = export3(s, s.grad.as<double>(), grad_all, s.N, false))) return rc;
  return sync(s);
}

static int upload_vec_precision(Scene &s, const double *host, void *dst) {
  size_t n3 = 3 * (size_t)s.N;
  int rc = import3(s, host, s.rhs.as<double>(), s.N, false);
  if (rc) return rc;
  if (s.mixed)
    hipLaunchKernelGGL(k_to_float, dim3(blocks_for(n3, 256)), dim3(256), 0, s.stream, s.rhs.as<double>(),
                       static_cast<float *>(dst), (int)n3);
  else
    hipMemcpyAsync(dst, s.rhs.p, n3 * 8, hipMemcpyDeviceToDevice, s.stream);
  return BAL_OK;
}

int bal_hessian_apply(bal_scene *h, const double *v, double *out) {
  if (!h || !v || !out) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  if (!s.linearized) return BAL_E_STATE;
  hipSetDevice(s.dev);
  size_t n3 = 3 * (size_t)s.N;
  upload_vec_precision(s, v, s.pv.p);
  launch_spmv(s, s.pv.p, s.q.p, 0);
  if (s.mixed)
    hipLaunchKernelGGL(k_to_double, dim3(blocks_for(n3, 256)), dim3(256), 0, s.stream, static_cast<float *>(s.q.p),
                       s.rhs.as<double>(), (int)n3);
  else
    hipMemcpyAsync(s.rhs.p, s.q.p, n3 * 8, hipMemcpyDeviceToDevice, s.stream);
  int rc = export3(s, s.rhs.as<double>(), out, s.N, false);
  if (!rc) rc = sync(s);
  for (int i = 0; i < s.N; ++i)
    if (!s.free_h[i])
      for (int c = 0; c < 3; ++c) out[3 * ext_vertex(s, i) + c] = 0.0;
  return rc;
}

int bal_get_stiffness(const bal_scene *h, double *e_nodes, int32_t *groups) {
  if (!h) return BAL_E_INVALID_ARG;
  const Scene &s = h->s;
  if (!s.linearized) return BAL_E_STATE;
  hipSetDevice(s.dev);
  std::vector<double> e(s.N);
  std::vector<int32_t> gr(s.N);
  if (e_nodes) hipMemcpyAsync(e.data(), s.e_nodes.p, (size_t)s.N * 8, hipMemcpyDeviceToHost, s.stream);
  if (groups) hipMemcpyAsync(gr.data(), s.group.p, (size_t)s.N * 4, hipMemcpyDeviceToHost, s.stream);
  int rc = hip_ok(hipStreamSynchronize(s.stream));
  for (int i = 0; i < s.N; ++i) {
    if (e_nodes) e_nodes[ext_vertex(s, i)] = e[i];
    if (groups) groups[ext_vertex(s, i)] = gr[i];
  }
  return rc;
}

int bal_solve(bal_scene *h, const double *rhs, double *z, int mode, double rtol, int32_t max_iters, int32_t *iters,
              double *rel_res) {
  if (!h || !rhs || !z || mode < 0 || mode > 2 || !(rtol >= 0.0) || max_iters <= 0) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  if (!s.linearized) return BAL_E_STATE;
  hipSetDevice(s.dev);
  size_t n3 = 3 * (size_t)s.N;
  std::vector<double> b(n3);
  for (int i = 0; i < s.N; ++i)
    for (int c = 0; c < 3; ++c) b[3 * i + c] = s.free_h[i] ? rhs[3 * ext_vertex(s, i) + c] : 0.0;
  double bn = 0.0;
  for (double v : b) bn += v * v;
  bn = std::sqrt(bn);
  // the solve's right-hand side lives in grad_b (rhs is scratch for conversions)
  hipMemcpyAsync(s.grad_b.p, b.data(), n3 * 8, hipMemcpyHostToDevice, s.stream);
  double save = s.desc.pcg_rtol;
  s.desc.pcg_rtol = rtol;
  int itw = 0, itg = 0;
  double rel = 0.0;
  int rc = BAL_OK;
  double *xs = s.dx.as<double>();
  if (mode >= 1) rc = warm_start_solve(s, s.grad_b.as<double>(), xs, mode == 1 ? rtol : kWarmTol, max_iters, &itw);
  if (rc == BAL_OK && mode != 1) rc = pcg_solve(s, s.grad_b.as<double>(), xs, bn, max_iters, mode == 2, 0, &itg, &rel);
  s.desc.pcg_rtol = save;
  if (rc != BAL_OK && rc != BAL_E_NO_CONVERGENCE) return rc;
  int rc2 = export3(s, xs, z, s.N, false);
  if (!rc2) rc2 = sync(s);
  if (iters) *iters = mode == 1 ? itw : itg;
  if (rel_res) *rel_res = rel;
  return rc2 ? rc2 : rc;
}

int bal_ccd_bound(bal_scene *h, const double *x_all, const double *p_all, double *alpha_max) {
  if (!h || !x_all || !p_all || !alpha_max) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  hipSetDevice(s.dev);
  size_t n3 = 3 * (size_t)s.N;
  (void)n3;
  int rc;
  if ((rc = import3(s, x_all, s.xtrial.as<double>(), s.N, false)) || (rc = import3(s, p_all, s.rhs.as<double>(), s.N, false)))
    return rc;
  rc = build_candidates(s, s.cand2, s.xtrial.as<double>(), s.rhs.as<double>());
  if (rc) return rc;
  if (s.tau.grow((size_t)(s.cand2.n + 1) * 8)) return BAL_E_OOM;
  launch_ccd(s, s.cand2, s.xtrial.as<double>(), s.rhs.as<double>(), s.tau.as<double>());
  *alpha_max = std::min(1.0, s.cand2.n ? reduce_min(s, s.tau.as<double>(), s.cand2.n) : 1.0);
  return sync(s);
}

int bal_candidates(bal_scene *h, const double *x_all, const double *p_all, int32_t capacity, int32_t *kind,
                   int32_t *nodes, double *dist, int32_t *n_pairs) {
  if (!h || !x_all || !n_pairs) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  hipSetDevice(s.dev);
  size_t n3 = 3 * (size_t)s.N;
  (void)n3;
  int rc;
  if ((rc = import3(s, x_all, s.xtrial.as<double>(), s.N, false))) return rc;
  if (p_all && (rc = import3(s, p_all, s.rhs.as<double>(), s.N, false))) return rc;
  rc = build_candidates(s, s.cand2, s.xtrial.as<double>(), p_all ? s.rhs.as<double>() : nullptr);
  if (rc) return rc;
  launch_pair_distance(s, s.cand2, s.xtrial.as<double>(), s.cand2.d.as<double>(), s.cand2.cs.as<int>());
  int n = s.cand2.n;
  *n_pairs = n;
  int m = std::min(n, (int)capacity);
  if (m > 0) {
    if (kind) hipMemcpyAsync(kind, s.cand2.kind.p, (size_t)m * 4, hipMemcpyDeviceToHost, s.stream);
    if (nodes) hipMemcpyAsync(nodes, s.cand2.nodes.p, (size_t)m * 16, hipMemcpyDeviceToHost, s.stream);
    if (dist) hipMemcpyAsync(dist, s.cand2.d.p, (size_t)m * 8, hipMemcpyDeviceToHost, s.stream);
  }
  rc = sync(s);
  if (nodes)
    for (int k = 0; k < 4 * m; ++k) nodes[k] = ext_vertex(s, nodes[k]);
  return rc;
}

}  // extern "C"

// Streaming references for the bandwidth roofline: every thread moves four
// 16-byte words per pass with all four loads issued before any use.  The read
// kernel sums what it loads (one partial per block) so no load is dead.
__global__ void __launch_bounds__(256) k_stream_read(const double2 *__restrict__ a, long n, double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double2 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    acc += (v0.x + v0.y) + (v1.x + v1.y) + (v2.x + v2.y) + (v3.x + v3.y);
  }
  for (; i < n; i += stride) acc += a[i].x + a[i].y;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_stream_copy(const double2 *__restrict__ a, double2 *__restrict__ b, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double2 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    b[i] = v0;
    b[i + stride] = v1;
    b[i + 2 * stride] = v2;
    b[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) b[i] = a[i];
}

extern "C" {

int bal_stream_benchmark(int32_t device, int64_t n_bytes, int32_t n_reps, double *read_gbs, double *copy_gbs) {
  if (n_bytes < (1 << 20) || n_reps <= 0) return BAL_E_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return BAL_E_HIP;
  const long n = (long)(n_bytes / 16);
  const int grid = 256 * 8, bs = 256;
  void *a = nullptr, *b = nullptr, *part = nullptr;
  if (hipMalloc(&a, n * 16) != hipSuccess) return BAL_E_OOM;
  if (hipMalloc(&b, n * 16) != hipSuccess) { hipFree(a); return BAL_E_OOM; }
  if (hipMalloc(&part, grid * 8) != hipSuccess) { hipFree(a); hipFree(b); return BAL_E_OOM; }
  hipStream_t st;
  hipStreamCreate(&st);
  hipMemsetAsync(a, 0, n * 16, st);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  float ms_r = 0.f, ms_c = 0.f;
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(bs), 0, st, (const double2 *)a, n, (double *)part);
  hipEventRecord(e0, st);
  for (int k = 0; k < n_reps; ++k)
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(bs), 0, st, (const double2 *)a, n, (double *)part);
  hipEventRecord(e1, st);
  hipEventSynchronize(e1);
  hipEventElapsedTime(&ms_r, e0, e1);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(bs), 0, st, (const double2 *)a, (double2 *)b, n);
  hipEventRecord(e0, st);
  for (int k = 0; k < n_reps; ++k)
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(bs), 0, st, (const double2 *)a, (double2 *)b, n);
  hipEventRecord(e1, st);
  int rc = hip_ok(hipEventSynchronize(e1));
  hipEventElapsedTime(&ms_c, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamDestroy(st);
  hipFree(a);
  hipFree(b);
  hipFree(part);
  if (rc) return rc;
  if (read_gbs) *read_gbs = (double)n * 16 * n_reps / (ms_r * 1e-3) / 1e9;
  if (copy_gbs) *copy_gbs = 2.0 * n * 16 * n_reps / (ms_c * 1e-3) / 1e9;
  return BAL_OK;
}

int bal_spmv_benchmark(bal_scene *h, int32_t n_reps, double *ms_per_launch, double *bytes) {
  if (!h || n_reps <= 0) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  if (!s.linearized) return BAL_E_STATE;
  hipSetDevice(s.dev);
  hipMemsetAsync(s.pv.p, 0, 3 * (size_t)s.N * (s.mixed ? 4 : 8), s.stream);
  launch_spmv(s, s.pv.p, s.q.p, 0);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipEventRecord(e0, s.stream);
  for (int k = 0; k < n_reps; ++k) launch_spmv(s, s.pv.p, s.q.p, 0);
  hipEventRecord(e1, s.stream);
  hipEventSynchronize(e1);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (ms_per_launch) *ms_per_launch = ms / n_reps;
  if (bytes) *bytes = spmv_bytes(s);
  return BAL_OK;
}

int bal_step_adjoint(bal_scene *h, const double *x_t, const double *v_t, const double *gx_next,
                     const double *gv_next, double *gx_t, double *gv_t, double *gE_accum, int on_device,
                     bal_step_stats *stats) {
  if (!h || !x_t || !v_t || !gx_next || !gv_next || !gx_t || !gv_t || !gE_accum) return BAL_E_INVALID_ARG;
  Scene &s = h->s;
  if (s.desc.friction > 0.0) return BAL_E_INVALID_ARG;  // friction is not a potential: no frozen-state adjoint
  hipSetDevice(s.dev);
  int rc = bal_set_state(h, x_t, v_t, on_device);
  if (rc) return rc;
  // the frozen-state derivative exists only at a converged step
  rc = newton_solve(s, stats, false);
  if (rc != BAL_OK) return rc;
  size_t nb3 = 3 * (size_t)s.nb, n3 = 3 * (size_t)s.N;
  hipMemcpyKind kin = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipMemcpyKind kout = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  // right-hand side gx + gv / h on free body rows (grad_b holds gv, rhs holds gx + gv/h)
  hipMemsetAsync(s.grad_b.p, 0, n3 * 8, s.stream);
  hipMemsetAsync(s.rhs.p, 0, n3 * 8, s.stream);
  if ((rc = import3(s, gv_next, s.grad_b.as<double>(), s.nb, on_device != 0)) ||
      (rc = import3(s, gx_next, s.rhs.as<double>(), s.nb, on_device != 0)))
    return rc;
  launch_axpy_state(s, s.rhs.as<double>(), s.rhs.as<double>(), s.grad_b.as<double>(), 1.0 / s.desc.dt, (int)n3);
  // frozen state: sigma, A' (mu, s) and the active set at x_{t+1}; unprojected Hessian
  double *x = s.x.as<double>();
  if ((rc = build_candidates(s, s.cand, x, nullptr))) return rc;
  launch_pair_distance(s, s.cand, x, s.cand.d.as<double>(), s.cand.cs.as<int>());
  if ((rc = build_union(s, s.cand))) return rc;
  double sig = s.sigma_set ? s.sigma : 0.0;
  if ((rc = linearize_at(s, x, 0, sig))) return rc;
  double bn = std::sqrt(dot_free(s, s.rhs.as<double>(), s.rhs.as<double>()));
  // the adjoint system is solved to 1e-10 without the stagnation exit (an
  // early stop here is an error in the gradient, not a cheaper Newton step)
  const double save = s.desc.pcg_rtol;
  const int save_stall = s.desc.pcg_stall_window;
  const int cap = std::max(s.desc.max_pcg, 200000);
  s.desc.pcg_rtol = 1e-10;
  s.desc.pcg_stall_window = 0;
  int it = 0;
  double rel = 0.0;
  double *lam = s.dx.as<double>();
  rc = pcg_solve(s, s.rhs.as<double>(), lam, bn, cap, 0, 0, &it, &rel);
  s.desc.pcg_rtol = save;
  s.desc.pcg_stall_window = save_stall;
  if (stats) stats->pcg_iters = it;
  // p.q <= 0: the unprojected Hessian is not positive definite at x_{t+1}, so
  // x_{t+1} is no strict minimiser and the step map has no derivative there
  if (rc == BAL_E_NO_CONVERGENCE) return BAL_E_INDEFINITE;
  if (rc != BAL_OK) return rc;
  if (rel > 1e-10) return BAL_E_NO_CONVERGENCE;
  // tet_g holds grad Psi_e at x_{t+1} from the linearization
  DBuf gEd, gxo, gvo, Ed;
  if (gEd.grow((size_t)s.T * 8) || gxo.grow(n3 * 8) || gvo.grow(n3 * 8) || Ed.grow((size_t)s.T * 8)) return BAL_E_OOM;
  hipMemcpyAsync(gEd.p, gE_accum, (size_t)s.T * 8, kin, s.stream);
  hipMemcpyAsync(Ed.p, s.youngs_h.data(), (size_t)s.T * 8, hipMemcpyHostToDevice, s.stream);
  hipLaunchKernelGGL(k_adjoint_E, dim3(blocks_for(s.T, 256)), dim3(256), 0, s.stream, s.T, s.tets.as<int4>(),
                     s.tet_g.as<double>(), lam, Ed.as<double>(), gEd.as<double>());
  hipLaunchKernelGGL(k_adjoint_state, dim3(blocks_for(s.N, 256)), dim3(256), 0, s.stream, s.N, lam,
                     s.grad_b.as<double>(), s.mass.as<double>(), s.freev.as<uint8_t>(), s.desc.dt, gxo.as<double>(),
                     gvo.as<double>());
  hipMemcpyAsync(gE_accum, gEd.p, (size_t)s.T * 8, kout, s.stream);
  rc = export3(s, gxo.as<double>(), gx_t, s.nb, on_device != 0);
  if (!rc) rc = export3(s, gvo.as<double>(), gv_t, s.nb, on_device != 0);
  int rs = sync(s);
  rc = rc ? rc : rs;
  gEd.release(); gxo.release(); gvo.release(); Ed.release();
  return rc;
}

}  // extern "C"
