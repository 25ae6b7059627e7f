// Contact-pair kernels: distances (closest-point case classification),
// barrier and augmentation energies (eq. IPC-barrier, eq. aug-lag), the
// per-pair gradient and projected Hessian of the summed pair energy
// (Sec. 4.2), the multiplier / slack update (Alg. 1 lines 12-14), and the
// conservative CCD step bound (Sec. 5.3 narrow phase).  One thread per pair.
#include "bal_internal.h"

namespace bal {

__device__ __forceinline__ void load_pair(const double *x, int4 nd, v3 *X) {
  X[0] = ld3(x, nd.x);
  X[1] = ld3(x, nd.y);
  X[2] = ld3(x, nd.z);
  X[3] = ld3(x, nd.w);
}

__global__ void k_pair_distance(int n, const int *__restrict__ kind, const int4 *__restrict__ nodes,
                                const double *__restrict__ x, double *__restrict__ d, int *__restrict__ cs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 X[4];
  load_pair(x, nodes[i], X);
  int c;
  double q = pair_classify(kind[i], X, &c);
  d[i] = sqrt(q);
  if (cs) cs[i] = c;
}

void launch_pair_distance(Scene &s, const PairList &pl, const double *x, double *d, int *cs) {
  if (pl.n == 0) return;
  hipLaunchKernelGGL(k_pair_distance, dim3(blocks_for(pl.n, 256)), dim3(256), 0, s.stream, pl.n, pl.kind.as<int>(),
                     pl.nodes.as<int4>(), x, d, cs);
}

// sigma b(d, dhat) per pair; flags bit 2 if some d <= 0.
__global__ void k_pair_barrier_energy(int n, const int *__restrict__ kind, const int4 *__restrict__ nodes,
                                      const double *__restrict__ x, double sigma, double dhat,
                                      double *__restrict__ e, double *__restrict__ dout, int *__restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 X[4];
  load_pair(x, nodes[i], X);
  int c;
  double d = sqrt(pair_classify(kind[i], X, &c));
  dout[i] = d;
  if (!(d > 0.0)) {
    e[i] = 0.0;
    atomicOr(flags, 2);
    return;
  }
  e[i] = sigma * barrier(d, dhat);
}

void launch_pair_barrier_energy(Scene &s, const PairList &pl, const double *x, double sigma, double *e, int *flags) {
  if (pl.n == 0) return;
  hipLaunchKernelGGL(k_pair_barrier_energy, dim3(blocks_for(pl.n, 256)), dim3(256), 0, s.stream, pl.n,
                     pl.kind.as<int>(), pl.nodes.as<int4>(), x, sigma, s.desc.dhat, e, pl.d.as<double>(), flags);
}

// Augmentation terms mu (dhat + s - d) + sigma b(d, dhat + s) for each pair of A'.
__global__ void k_aug_energy(int n, const int *__restrict__ kind, const int4 *__restrict__ nodes,
                             const double *__restrict__ mu, const double *__restrict__ sl, const double *__restrict__ x,
                             double sigma, double dhat, double *__restrict__ e, double *__restrict__ dout,
                             int *__restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 X[4];
  load_pair(x, nodes[i], X);
  int c;
  double d = sqrt(pair_classify(kind[i], X, &c));
  if (dout) dout[i] = d;
  if (!(d > 0.0)) {
    e[i] = 0.0;
    atomicOr(flags, 2);
    return;
  }
  e[i] = mu[i] * (dhat + sl[i] - d) + sigma * barrier(d, dhat + sl[i]);
}

void launch_aug_energy(Scene &s, const double *x, double sigma, double *e, double *d, int *flags) {
  if (s.n_aug == 0) return;
  hipLaunchKernelGGL(k_aug_energy, dim3(blocks_for(s.n_aug, 256)), dim3(256), 0, s.stream, s.n_aug,
                     s.aug_kind.as<int>(), s.aug_nodes.as<int4>(), s.aug_mu.as<double>(), s.aug_s.as<double>(), x,
                     sigma, s.desc.dhat, e, d, flags);
}

// Dual update on A' at the new iterate: s_i = max(-mu_i/sigma - dhat + d_i, 0),
// then mu_i += sigma b(d_i, dhat + s_i)  (Alg. 1, lines 12-14; sec. 3.2 slack formula).
__global__ void k_aug_update(int n, const int *__restrict__ kind, const int4 *__restrict__ nodes,
                             double *__restrict__ mu, double *__restrict__ sl, const double *__restrict__ x,
                             double sigma, double dhat) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 X[4];
  load_pair(x, nodes[i], X);
  int c;
  double d = sqrt(pair_classify(kind[i], X, &c));
  double si = -mu[i] / sigma - dhat + d;
  si = si > 0.0 ? si : 0.0;
  sl[i] = si;
  mu[i] = mu[i] + sigma * barrier(d, dhat + si);
}

void launch_aug_update(Scene &s, const double *x) {
  if (s.n_aug == 0) return;
  hipLaunchKernelGGL(k_aug_update, dim3(blocks_for(s.n_aug, 256)), dim3(256), 0, s.stream, s.n_aug,
                     s.aug_kind.as<int>(), s.aug_nodes.as<int4>(), s.aug_mu.as<double>(), s.aug_s.as<double>(), x,
                     s.sigma, s.desc.dhat);
}

// ------------------------------------------------------------ linearize
// Per pair of the union list (active candidates plus A'): energy, gradient
// on the 4 stencil slots, the projected Hessian blocks between the case's
// nodes (stencil-slot 4x4 grid of 3x3 blocks) and the mean projected
// eigenvalue tr / (3k).
// Friction of one pair (Sec. 4.1) at the iterate: the 3x3 tangent stiffness S,
// the force direction times magnitude gf and the closest-point weights beta of
// the 4 stencil slots; the stencil's blocks get beta_a beta_b S and its
// gradient slots beta_a gf (S is positive semi-definite by construction).
struct PairFriction {
  bool on;
  double beta[4], gf[3], S[9];
};

template <int R, int K>
__device__ __forceinline__ void finish_pair(double *Hu, const double *gu, const double *W, int cs, int project,
                                            double *gout, double *blk_out, double *tr_out, bool fp32,
                                            float *blk_out_f, const PairFriction &fr) {
  constexpr int n = 3 * R;
  double L[R * R], Q[K * R];
  reduced_basis<R, K>(W, L, Q);
  reduce_hessian<R>(Hu, L);
  double P[n * (n + 1) / 2];
  pack_sym<n>(Hu, P);
  double tr;
  if (project) {
    tr = project_psd<n>(P);
  } else {
    tr = 0.0;
#pragma unroll
    for (int i = 0; i < n; ++i) tr += P[pk<n>(i, i)];
  }
  double trf = 0.0;
  if (fr.on) {
    double sb2 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) sb2 += fr.beta[j] * fr.beta[j];
    trf = sb2 * (fr.S[0] + fr.S[4] + fr.S[8]);
  }
  *tr_out = tr / (3.0 * K) + trf / (3.0 * K);
  // gradient on the case's local nodes
#pragma unroll
  for (int j = 0; j < K; ++j) {
    int slot = kCaseNodes[cs][j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) s += W[i * K + j] * gu[3 * i + c];
      if (fr.on) s += fr.beta[slot] * fr.gf[c];
      gout[3 * slot + c] = s;
    }
  }
#pragma unroll
  for (int a = 0; a < K; ++a)
#pragma unroll
    for (int b = 0; b < K; ++b) {
      double blk[9];
      expand_block<R>(P, Q, a, b, blk);
      int sa = kCaseNodes[cs][a], sb = kCaseNodes[cs][b];
      if (fr.on) {
        const double ww = fr.beta[sa] * fr.beta[sb];
#pragma unroll
        for (int e = 0; e < 9; ++e) blk[e] += ww * fr.S[e];
      }
      size_t off = (size_t)(sa * 4 + sb) * 9;
      if (fp32) {
#pragma unroll
        for (int e = 0; e < 9; ++e) blk_out_f[off + e] = (float)blk[e];
      } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) blk_out[off + e] = blk[e];
      }
    }
}

// Closest-point weights of the 4 stencil slots for distance case cs: sum_k
// beta_k X_k joins the case's two closest points (the barycentric
// coordinates of the contact stencil, Sec. 4.1).  Point-edge: the segment
// parameter; point-triangle interior: the barycentrics of the projection;
// edge-edge interior: the line-line parameters (Gram systems solved with the
// squared cross product as determinant).
__device__ void closest_beta(int cs, const v3 *X, double *beta) {
  beta[0] = beta[1] = beta[2] = beta[3] = 0.0;
  const int k = kCaseK[cs];
  if (k == 2) {
    beta[kCaseNodes[cs][0]] = 1.0;
    beta[kCaseNodes[cs][1]] = -1.0;
  } else if (k == 3) {
    const int n0 = kCaseNodes[cs][0], n1 = kCaseNodes[cs][1], n2 = kCaseNodes[cs][2];
    const v3 e = X[n2] - X[n1];
    const double t = dot(X[n0] - X[n1], e) / dot(e, e);
    beta[n0] = 1.0;
    beta[n1] = -(1.0 - t);
    beta[n2] = -t;
  } else if (cs == 0) {
    const v3 e1 = X[2] - X[1], e2 = X[3] - X[1], r = X[0] - X[1];
    const v3 c = cross(e1, e2);
    const double det = dot(c, c), g11 = dot(e1, e1), g12 = dot(e1, e2), g22 = dot(e2, e2);
    const double r1 = dot(r, e1), r2 = dot(r, e2);
    const double u = (r1 * g22 - r2 * g12) / det, v = (g11 * r2 - g12 * r1) / det;
    beta[0] = 1.0;
    beta[1] = -(1.0 - u - v);
    beta[2] = -u;
    beta[3] = -v;
  } else {
    const v3 e1 = X[1] - X[0], e2 = X[3] - X[2], r = X[0] - X[2];
    const v3 c = cross(e1, e2);
    const double det = dot(c, c), g11 = dot(e1, e1), g12 = dot(e1, e2), g22 = dot(e2, e2);
    const double r1 = -dot(e1, r), r2 = dot(e2, r);
    // [g11 -g12; -g12 g22] [sa; sb] = [r1; r2]
    const double sa = (r1 * g22 + g12 * r2) / det, sb = (g11 * r2 + g12 * r1) / det;
    beta[0] = 1.0 - sa;
    beta[1] = sa;
    beta[2] = -(1.0 - sb);
    beta[3] = -sb;
  }
}

// Tangential relative displacement of the step, w = P sum_k beta_k (X_k - X_k^t)
// with P = I - n n^T / n.n (Sec. 4.1: u h), and the mollifier f of |w|
// (f(y) = -y^3/(3 eps_v^2 h^2) + y^2/(eps_v h) below eps_v h, its C1
// continuation y - eps_v h / 3 above) with f'(y)/y and f''(y).
__device__ __forceinline__ void friction_w(const v3 *X, const v3 *Xt, const double *beta, v3 n, double eh, v3 *w,
                                           double *f, double *fp_y, double *fpp) {
  v3 du{0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) du = du + beta[k] * (X[k] - Xt[k]);
  *w = du - (dot(du, n) / dot(n, n)) * n;
  const double q = dot(*w, *w), y = sqrt(q);
  if (y < eh) {
    *f = -q * y / (3.0 * eh * eh) + q / eh;
    *fp_y = -y / (eh * eh) + 2.0 / eh;
    *fpp = -2.0 * y / (eh * eh) + 2.0 / eh;
  } else {
    *f = y - eh / 3.0;
    *fp_y = 1.0 / y;
    *fpp = 0.0;
  }
}

__global__ void k_friction_energy(int n, const int4 *__restrict__ nodes, const double *__restrict__ fr,
                                  const double *__restrict__ x, const double *__restrict__ xt, double chi, double eh,
                                  double *__restrict__ e) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *F = fr + (size_t)i * 8;
  const double lam = F[0];
  if (!(lam > 0.0)) {
    e[i] = 0.0;
    return;
  }
  v3 X[4], Xt[4];
  load_pair(x, nodes[i], X);
  load_pair(xt, nodes[i], Xt);
  v3 w;
  double f, fp_y, fpp;
  friction_w(X, Xt, F + 1, v3{F[5], F[6], F[7]}, eh, &w, &f, &fp_y, &fpp);
  e[i] = chi * lam * f;
}

void launch_friction_energy(Scene &s, const double *x, double *e) {
  if (s.uni.n == 0) return;
  hipLaunchKernelGGL(k_friction_energy, dim3(blocks_for(s.uni.n, 256)), dim3(256), 0, s.stream, s.uni.n,
                     s.uni.nodes.as<int4>(), s.fr.as<double>(), x, s.x_t.as<double>(), s.desc.friction,
                     friction_eps_h(s), e);
}

__global__ __launch_bounds__(64) void k_pair_linearize(
    int n, const int *__restrict__ kind, const int4 *__restrict__ nodes, const int *__restrict__ bar_on,
    const int *__restrict__ aug_idx, const double *__restrict__ mu, const double *__restrict__ sl,
    const double *__restrict__ x, double sigma, double dhat, int project, int fp32, double *__restrict__ pe,
    double *__restrict__ pg, void *__restrict__ pblk, double *__restrict__ ptr, int *__restrict__ pcase,
    int *__restrict__ flags, double chi, double eh, const double *__restrict__ xt, double *__restrict__ fr_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v3 X[4];
  load_pair(x, nodes[i], X);
  int cs;
  double q = pair_classify(kind[i], X, &cs);
  double d = sqrt(q);
  pcase[i] = cs;
  double *gout = pg + (size_t)i * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) gout[k] = 0.0;
  if (!(d > 0.0)) {
    pe[i] = 0.0;
    ptr[i] = 0.0;
    atomicOr(flags, 2);
    return;
  }
  double fb = bar_on[i] ? sigma : 0.0;
  int ai = aug_idx[i];
  double e = fb * barrier(d, dhat);
  double f1 = fb * barrier_d1(d, dhat);
  double f2 = fb * barrier_d2(d, dhat);
  if (ai >= 0) {
    double m = mu[ai], s = sl[ai];
    e += m * (dhat + s - d) + sigma * barrier(d, dhat + s);
    f1 += -m + sigma * barrier_d1(d, dhat + s);
    f2 += sigma * barrier_d2(d, dhat + s);
  }
  // friction frame at this iterate (lam, beta, n held constant while D is
  // differentiated and during the line search, Sec. 4.1)
  PairFriction pf;
  pf.on = false;
  if (chi > 0.0) {
    const double lam = -f1;
    double *F = fr_out + (size_t)i * 8;
    F[0] = 0.0;
    if (lam > 0.0) {
      v3 Xt[4];
      load_pair(xt, nodes[i], Xt);
      closest_beta(cs, X, pf.beta);
      v3 nv{0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) nv = nv + pf.beta[k] * X[k];
      v3 w;
      double f, fp_y, fpp;
      friction_w(X, Xt, pf.beta, nv, eh, &w, &f, &fp_y, &fpp);
      const double cl = chi * lam;
      e += cl * f;
      pf.gf[0] = cl * fp_y * w.x;
      pf.gf[1] = cl * fp_y * w.y;
      pf.gf[2] = cl * fp_y * w.z;
      // S = chi lam P [f'/y (I - w^ w^T) + f'' w^ w^T] P = chi lam [f'/y (P - w^ w^T) + f'' w^ w^T]
      const double nn = dot(nv, nv), q = dot(w, w);
      const double nc[3] = {nv.x, nv.y, nv.z}, wc[3] = {w.x, w.y, w.z};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const double Pab = (a == b ? 1.0 : 0.0) - nc[a] * nc[b] / nn;
          const double ww = q > 0.0 ? wc[a] * wc[b] / q : 0.0;
          pf.S[3 * a + b] = cl * (fp_y * (Pab - ww) + fpp * ww);
        }
      pf.on = true;
      F[0] = lam;
#pragma unroll
      for (int k = 0; k < 4; ++k) F[1 + k] = pf.beta[k];
      F[5] = nv.x;
      F[6] = nv.y;
      F[7] = nv.z;
    }
  }
  pe[i] = e;
  // chain rule through d = sqrt(q): grad f = f1/(2d) grad q,
  // Hess f = (f2/(4 d^2) - f1/(4 d^3)) grad q grad q^T + f1/(2d) Hess q
  double c1 = f2 / (4.0 * d * d) - f1 / (4.0 * d * d * d);
  double c2 = f1 / (2.0 * d);
  double *bd = fp32 ? nullptr : static_cast<double *>(pblk) + (size_t)i * 144;
  float *bf = fp32 ? static_cast<float *>(pblk) + (size_t)i * 144 : nullptr;
  int k = kCaseK[cs];
  if (k == 4) {
    v3 r, e1, e2;
    if (cs == 0) { r = X[0] - X[1]; e1 = X[2] - X[1]; e2 = X[3] - X[1]; }
    else { r = X[0] - X[2]; e1 = X[1] - X[0]; e2 = X[3] - X[2]; }
    double qq, g[9], H[81];
    q9_derivs(r, e1, e2, &qq, g, H);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = 0; b < 9; ++b) H[a * 9 + b] = c1 * g[a] * g[b] + c2 * H[a * 9 + b];
#pragma unroll
    for (int a = 0; a < 9; ++a) g[a] *= c2;
    double W[12];
    case_W(cs, W);
    finish_pair<3, 4>(H, g, W, cs, project, gout, bd, ptr + i, fp32, bf, pf);
  } else if (k == 3) {
    int n0 = kCaseNodes[cs][0], n1 = kCaseNodes[cs][1], n2 = kCaseNodes[cs][2];
    double qq, g[6], H[36];
    q6_derivs(X[n0] - X[n1], X[n2] - X[n1], &qq, g, H);
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) H[a * 6 + b] = c1 * g[a] * g[b] + c2 * H[a * 6 + b];
#pragma unroll
    for (int a = 0; a < 6; ++a) g[a] *= c2;
    double W[6];
    case_W(cs, W);
    finish_pair<2, 3>(H, g, W, cs, project, gout, bd, ptr + i, fp32, bf, pf);
  } else {
    int n0 = kCaseNodes[cs][0], n1 = kCaseNodes[cs][1];
    v3 r = X[n0] - X[n1];
    double g[3] = {2.0 * r.x, 2.0 * r.y, 2.0 * r.z}, H[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) H[a * 3 + b] = c1 * g[a] * g[b] + c2 * (a == b ? 2.0 : 0.0);
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] *= c2;
    double W[2];
    case_W(cs, W);
    finish_pair<1, 2>(H, g, W, cs, project, gout, bd, ptr + i, fp32, bf, pf);
  }
}

void launch_pair_linearize(Scene &s, const double *x, int project, double sigma, int with_friction) {
  if (s.uni.n == 0) return;
  const double chi = with_friction ? s.desc.friction : 0.0;
  hipLaunchKernelGGL(k_pair_linearize, dim3(blocks_for(s.uni.n, 64)), dim3(64), 0, s.stream, s.uni.n,
                     s.uni.kind.as<int>(), s.uni.nodes.as<int4>(), s.uni_flag.as<int>(), s.uni_aug.as<int>(),
                     s.aug_mu.as<double>(), s.aug_s.as<double>(), x, sigma, s.desc.dhat, project, s.mixed ? 1 : 0,
                     s.pair_e.as<double>(), s.pair_g.as<double>(), s.pair_blk.p, s.pair_tr.as<double>(),
                     s.uni.cs.as<int>(), s.flags.as<int>(), chi, friction_eps_h(s), s.x_t.as<double>(),
                     chi > 0.0 ? s.fr.as<double>() : nullptr);
}

// ------------------------------------------------------------------- CCD
constexpr double kCcdEps = 1e-12;
constexpr double kCoplanarUlps = 32.0;

__device__ __forceinline__ double cubic(double c3, double c2, double c1, double c0, double t) {
  return ((c3 * t + c2) * t + c1) * t + c0;
}

// Safeguarded Newton iteration on a bracket [a, b] with f(a) f(b) <= 0.
__device__ double newton_bisect(double c3, double c2, double c1, double c0, double a, double b) {
  double fa = cubic(c3, c2, c1, c0, a);
  if (fa == 0.0) return a;
  double t = 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double f = cubic(c3, c2, c1, c0, t);
    if (f == 0.0) return t;
    if ((f < 0.0) == (fa < 0.0)) { a = t; fa = f; } else { b = t; }
    double df = (3.0 * c3 * t + 2.0 * c2) * t + c1;
    double tn = df != 0.0 ? t - f / df : 0.5 * (a + b);
    if (!(tn > a && tn < b)) tn = 0.5 * (a + b);
    if (fabs(tn - t) <= 1e-16 * fmax(1.0, fabs(t)) || b - a <= 4e-16 * fmax(1.0, fabs(b))) return tn;
    t = tn;
  }
  return t;
}

// Real roots of the cubic in [lo, hi], ascending (at most 3).  The smallest
// root comes from Newton-bisection on the first monotone piece with a sign
// change; the cubic is then deflated, c(t) = (t - r)(A t^2 + B t + C) with
// A = c3, B = c2 + A r, C = c1 + B r, and the quadratic gives the rest.
__device__ int cubic_roots(double c3, double c2, double c1, double c0, double lo, double hi, double *roots) {
  if (c3 == 0.0 && c2 == 0.0 && c1 == 0.0 && c0 == 0.0) return 0;
  // monotone pieces from the derivative's roots
  double br[4];
  int nb = 0;
  br[nb++] = lo;
  double A = 3.0 * c3, B = 2.0 * c2, C = c1;
  if (A != 0.0) {
    double disc = B * B - 4.0 * A * C;
    if (disc > 0.0) {
      double sq = sqrt(disc);
      double qv = -0.5 * (B + (B >= 0.0 ? sq : -sq));
      double t1 = qv / A, t2 = qv != 0.0 ? C / qv : t1;
      if (t1 > t2) { double tmp = t1; t1 = t2; t2 = tmp; }
      if (t1 > lo && t1 < hi) br[nb++] = t1;
      if (t2 > lo && t2 < hi && t2 != t1) br[nb++] = t2;
    }
  } else if (B != 0.0) {
    double t1 = -C / B;
    if (t1 > lo && t1 < hi) br[nb++] = t1;
  }
  br[nb++] = hi;
  double first = 0.0;
  bool found = false;
  for (int k = 0; k + 1 < nb && !found; ++k) {
    double fa = cubic(c3, c2, c1, c0, br[k]), fb = cubic(c3, c2, c1, c0, br[k + 1]);
    if (fa * fb <= 0.0) {
      first = newton_bisect(c3, c2, c1, c0, br[k], br[k + 1]);
      found = true;
    }
  }
  if (!found) return 0;
  int n = 0;
  roots[n++] = first;
  if (c3 != 0.0) {
    double qa = c3, qb = c2 + qa * first, qc = c1 + qb * first;
    double disc = qb * qb - 4.0 * qa * qc;
    if (disc >= 0.0) {
      double sq = sqrt(disc);
      double qv = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
      double r1 = qv / qa, r2 = qv != 0.0 ? qc / qv : r1;
      if (r1 > r2) { double tmp = r1; r1 = r2; r2 = tmp; }
      if (r1 > first && r1 >= lo && r1 <= hi) roots[n++] = r1;
      if (r2 > first && r2 >= lo && r2 <= hi && (n == 1 || r2 != roots[n - 1])) roots[n++] = r2;
    }
  } else if (c2 != 0.0) {
    // quadratic c2 t^2 + c1 t + c0 = (t - first)(c2 t + c1 + c2 first)
    double r1 = -(c1 + c2 * first) / c2;
    if (r1 > first && r1 >= lo && r1 <= hi) roots[n++] = r1;
  }
  return n;
}

__device__ __forceinline__ double signed_dist(int kind, const v3 *X) {
  if (kind == 0) {
    v3 nn = cross(X[2] - X[1], X[3] - X[1]);
    return dot(X[0] - X[1], nn) / sqrt(dot(nn, nn));
  }
  v3 nn = cross(X[1] - X[0], X[3] - X[2]);
  return dot(X[0] - X[2], nn) / sqrt(dot(nn, nn));
}

// Sign with a dead zone of the CCD epsilon: |sd| <= eps counts as touching (sign 0).
__device__ __forceinline__ double sgn(double v) { return v > kCcdEps ? 1.0 : (v < -kCcdEps ? -1.0 : 0.0); }

// Conservative time of impact of one candidate pair along x + t p, t in [0, 1]
// (Sec. 5.3 narrow phase).  The roots of the coplanarity cubic in
// [-eps, 1+eps] (clamped into [0, 1]) are the times of coplanarity t1 <= t2 <=
// t3 after t0 = 0; the first whose distance there is below eps + margin is
// activated, tau = that time.  For a point-triangle or edge-edge interior
// case tau shrinks by 0.9 while the signed distance at tau and at the
// reference time (t_prev + tau) / 2 differ in sign (|sd| <= eps counts as
// sign 0, so tau never rests on the coplanarity itself); point-point and
// point-edge cases keep tau.  Rules (bal_ccd_rule): printed, margin = dhat
// and a root at |t| <= eps is the start frame t0 = 0, not a time of impact,
// as is the root of a start frame coplanar to within the rounding of its
// positions (|det| <= 32 u max|x| (|u||v| + |v||w| + |w||u|): constant
// term taken as 0);
// half-gap (not in the paper), margin = d0 / 2 for a pair that starts closer
// than dhat; literal, margin = dhat with roots at |t| <= eps activated.
__device__ double pair_toi(int kd, const v3 *X0, const v3 *P, double dhat, int rule) {
  v3 u0, u1, v0, v1, w0, w1;
  if (kd == 0) {
    u0 = X0[0] - X0[1]; u1 = P[0] - P[1];
    v0 = X0[2] - X0[1]; v1 = P[2] - P[1];
    w0 = X0[3] - X0[1]; w1 = P[3] - P[1];
  } else {
    u0 = X0[1] - X0[0]; u1 = P[1] - P[0];
    v0 = X0[2] - X0[0]; v1 = P[2] - P[0];
    w0 = X0[3] - X0[0]; w1 = P[3] - P[0];
    v3 X1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) X1[k] = X0[k] + P[k];
    if (ee_parallel(X0[1] - X0[0], X0[3] - X0[2]) && ee_parallel(X1[1] - X1[0], X1[3] - X1[2])) return 1.0;
  }
  // det[u0 + t u1, v0 + t v1, w0 + t w1] expanded by multilinearity
  double c0 = dot(u0, cross(v0, w0));
  double c1 = dot(u1, cross(v0, w0)) + dot(u0, cross(v1, w0)) + dot(u0, cross(v0, w1));
  double c2 = dot(u1, cross(v1, w0)) + dot(u1, cross(v0, w1)) + dot(u0, cross(v1, w1));
  double c3 = dot(u1, cross(v1, w1));
  if (rule != BAL_CCD_LITERAL) {
    // a start frame coplanar to within the rounding of the positions has its
    // root at t0 exactly (however short p is)
    double xm = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) xm = fmax(xm, fmax(fabs(X0[m].x), fmax(fabs(X0[m].y), fabs(X0[m].z))));
    const double nu = sqrt(dot(u0, u0)), nv = sqrt(dot(v0, v0)), nw = sqrt(dot(w0, w0));
    if (fabs(c0) <= kCoplanarUlps * 0x1p-53 * xm * (nu * nv + nv * nw + nw * nu)) c0 = 0.0;
  }
  double roots[3];
  int nr = cubic_roots(c3, c2, c1, c0, -kCcdEps, 1.0 + kCcdEps, roots);
  double margin = dhat;
  if (rule == BAL_CCD_HALF_GAP) {
    int cs0;
    const double d0 = sqrt(pair_classify(kd, X0, &cs0));
    if (d0 < dhat) margin = 0.5 * d0;
  }
  double tprev = 0.0;
  for (int k = 0; k < nr; ++k) {
    if (rule != BAL_CCD_LITERAL && roots[k] <= kCcdEps) continue;
    double tk = fmin(fmax(roots[k], 0.0), 1.0);
    v3 Xt[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) Xt[m] = X0[m] + tk * P[m];
    int cs;
    double dt = sqrt(pair_classify(kd, Xt, &cs));
    if (dt < kCcdEps + margin) {
      double t = tk;
      if (cs == 0 || cs == 7) {
        for (int it = 0; it < 400; ++it) {
          v3 A[4], Bm[4];
          double tm = 0.5 * (tprev + t);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            A[m] = X0[m] + t * P[m];
            Bm[m] = X0[m] + tm * P[m];
          }
          if (sgn(signed_dist(kd, A)) == sgn(signed_dist(kd, Bm))) break;
          t *= 0.9;
        }
      }
      return t;
    }
    tprev = tk;
  }
  return 1.0;
}

__global__ void k_ccd(int n, const int *__restrict__ kind, const int4 *__restrict__ nodes, const double *__restrict__ x,
                      const double *__restrict__ p, double dhat, int rule, double *__restrict__ tau) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int4 nd = nodes[i];
  v3 X0[4], P[4];
  load_pair(x, nd, X0);
  load_pair(p, nd, P);
  tau[i] = pair_toi(kind[i], X0, P, dhat, rule);
}

void launch_ccd(Scene &s, const PairList &pl, const double *x, const double *p, double *tau) {
  if (pl.n == 0) return;
  hipLaunchKernelGGL(k_ccd, dim3(blocks_for(pl.n, 128)), dim3(128), 0, s.stream, pl.n, pl.kind.as<int>(),
                     pl.nodes.as<int4>(), x, p, s.desc.dhat, s.desc.ccd_rule, tau);
}

}  // namespace bal

// ------------------------------------------------- CCD bound over given pairs
// Stateless step bound over pairs the caller supplies (no scene): pass 1 takes
// four pairs per thread and writes one partial minimum of tau per block; pass
// 2 folds the partials into alpha_max = min(1, min tau).  A node index outside
// [0, n_verts) turns the result into NaN (no host round trip, so the whole
// call stays asynchronous on the caller's stream).
#include <cmath>
#include <mutex>

namespace bal {

constexpr int kPairsPerThread = 4;
constexpr int kPairBlock = 256;
constexpr int kPairsPerBlock = kPairsPerThread * kPairBlock;
// partials of the scratch-array entry point: one double per block of pass 1
constexpr int kPairScratchDoubles = 1 << 16;  // 512 KiB per device
constexpr long kPairsMaxNoAlloc = (long)kPairScratchDoubles * kPairsPerBlock;

__global__ void __launch_bounds__(kPairBlock) k_pairs_toi_min(int n, int n_verts, const int *__restrict__ kind,
                                                              const int4 *__restrict__ nodes,
                                                              const double *__restrict__ x,
                                                              const double *__restrict__ p, double dhat, int rule,
                                                              double *__restrict__ part) {
  __shared__ double red[kPairBlock / 64];
  double m = 1.0;
  const int base = blockIdx.x * kPairsPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    const int i = base + k * kPairBlock;
    if (i < n) {
      const int4 nd = nodes[i];
      const bool ok = nd.x >= 0 && nd.x < n_verts && nd.y >= 0 && nd.y < n_verts && nd.z >= 0 && nd.z < n_verts &&
                      nd.w >= 0 && nd.w < n_verts && (kind[i] == 0 || kind[i] == 1);
      if (!ok) {
        m = NAN;
      } else {
        v3 X0[4], P[4];
        load_pair(x, nd, X0);
        load_pair(p, nd, P);
        const double t = pair_toi(kind[i], X0, P, dhat, rule);
        m = (m != m) ? m : fmin(m, t);  // NaN sticks
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(m, off, 64);
    m = (m != m || o != o) ? NAN : fmin(m, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < kPairBlock / 64; ++w) r = (r != r || red[w] != red[w]) ? NAN : fmin(r, red[w]);
    part[blockIdx.x] = r;
  }
}

__global__ void __launch_bounds__(1024) k_pairs_min_final(int nb, const double *__restrict__ part,
                                                          double *__restrict__ out) {
  __shared__ double red[16];
  double m = 1.0;
  for (int i = threadIdx.x; i < nb; i += 1024) {
    const double v = part[i];
    m = (m != m || v != v) ? NAN : fmin(m, v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(m, off, 64);
    m = (m != m || o != o) ? NAN : fmin(m, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < 16; ++w) r = (r != r || red[w] != red[w]) ? NAN : fmin(r, red[w]);
    *out = r;
  }
}

static int pairs_args_ok(const double *x, const double *p, int32_t n_verts, const int32_t *kind,
                         const int32_t *nodes, int32_t n_pairs, double dhat, int32_t rule, const double *out) {
  if (!x || !p || !out || n_verts < 0 || n_pairs < 0 || !(dhat > 0.0) || !std::isfinite(dhat)) return 0;
  if (n_pairs > 0 && (!kind || !nodes)) return 0;
  return rule == BAL_CCD_PRINTED || rule == BAL_CCD_HALF_GAP || rule == BAL_CCD_LITERAL;
}

static void launch_pairs_ccd(const double *x, const double *p, int32_t n_verts, const int32_t *kind,
                             const int32_t *nodes, int32_t n_pairs, double dhat, int32_t rule, double *part,
                             double *alpha_max, hipStream_t st) {
  const int nb = n_pairs > 0 ? (int)((n_pairs + kPairsPerBlock - 1) / kPairsPerBlock) : 0;
  if (nb > 0)
    hipLaunchKernelGGL(k_pairs_toi_min, dim3(nb), dim3(kPairBlock), 0, st, n_pairs, n_verts, kind,
                       (const int4 *)nodes, x, p, dhat, rule, part);
  hipLaunchKernelGGL(k_pairs_min_final, dim3(1), dim3(1024), 0, st, nb, part, alpha_max);
}

// The scratch of bal_pairs_ccd_bound_noalloc: file-scope device memory, one
// copy per GPU.  Host code never passes this name to a kernel; it uses the
// device address looked up once per device (pair_scratch_ptr).
static __device__ __align__(256) double scratch[kPairScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once).
static int pair_scratch_ptr(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return BAL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BAL_E_HIP;
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return BAL_OK;
}

}  // namespace bal

extern "C" {

int bal_pairs_ccd_bound(int32_t device, const double *x, const double *p, int32_t n_verts, const int32_t *kind,
                        const int32_t *nodes, int32_t n_pairs, double dhat, int32_t ccd_rule, double *alpha_max,
                        void *stream) {
  using namespace bal;
  if (!pairs_args_ok(x, p, n_verts, kind, nodes, n_pairs, dhat, ccd_rule, alpha_max)) return BAL_E_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return BAL_E_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t nb = n_pairs > 0 ? (size_t)((n_pairs + kPairsPerBlock - 1) / kPairsPerBlock) : 1;
  void *part = nullptr;
  if (hipMallocAsync(&part, nb * sizeof(double), st) != hipSuccess) return BAL_E_OOM;
  launch_pairs_ccd(x, p, n_verts, kind, nodes, n_pairs, dhat, ccd_rule, static_cast<double *>(part), alpha_max, st);
  int rc = hip_ok(hipGetLastError());
  if (hipFreeAsync(part, st) != hipSuccess && rc == BAL_OK) rc = BAL_E_HIP;
  return rc;
}

int bal_pairs_ccd_bound_noalloc(int32_t device, const double *x, const double *p, int32_t n_verts,
                                const int32_t *kind, const int32_t *nodes, int32_t n_pairs, double dhat,
                                int32_t ccd_rule, double *alpha_max, void *stream) {
  using namespace bal;
  if (!pairs_args_ok(x, p, n_verts, kind, nodes, n_pairs, dhat, ccd_rule, alpha_max)) return BAL_E_INVALID_ARG;
  if ((long)n_pairs > kPairsMaxNoAlloc) return BAL_E_CAPACITY;
  if (hipSetDevice(device) != hipSuccess) return BAL_E_INVALID_ARG;
  double *part = nullptr;
  int rc = pair_scratch_ptr(device, &part);
  if (rc) return rc;
  launch_pairs_ccd(x, p, n_verts, kind, nodes, n_pairs, dhat, ccd_rule, part, alpha_max,
                   static_cast<hipStream_t>(stream));
  return hip_ok(hipGetLastError());
}

}  // extern "C"
