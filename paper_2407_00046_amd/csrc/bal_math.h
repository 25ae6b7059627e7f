// Device math for the BAL time step: Neo-Hookean element terms, barrier,
// pair distances with their derivatives, and stencil projection.
//
// Projection without a 12x12 eigensolve.  Every stencil energy here is a
// function of a few difference vectors u = (W (x) I3) x, where W is a small
// constant matrix with rows orthogonal to (1,...,1) (translations).  With
// W W^T = L L^T (Cholesky) and Q = W^T L^{-T} (orthonormal columns), the
// stencil Hessian is H_x = (Q (x) I3) M (Q (x) I3)^T with M = (L^T (x) I3)
// H_u (L (x) I3).  The nonzero eigenvalues of H_x are those of M, so the
// closest PSD matrix to H_x (eigenvalues clamped at zero, Sec. 4.2) is
// (Q (x) I3) proj(M) (Q (x) I3)^T, and tr(proj H_x) = tr(proj M).  Elements
// and point-triangle / edge-edge pairs need a 9x9 eigenproblem, point-edge a
// 6x6 and point-point a 3x3, instead of 12x12.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define BAL_DEV __device__ __forceinline__

namespace bal {

// ---------------------------------------------------------------- 3-vectors
struct v3 { double x, y, z; };
BAL_DEV v3 mk(double a, double b, double c) { return v3{a, b, c}; }
BAL_DEV v3 operator+(v3 a, v3 b) { return v3{a.x + b.x, a.y + b.y, a.z + b.z}; }
BAL_DEV v3 operator-(v3 a, v3 b) { return v3{a.x - b.x, a.y - b.y, a.z - b.z}; }
BAL_DEV v3 operator*(double s, v3 a) { return v3{s * a.x, s * a.y, s * a.z}; }
BAL_DEV double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
BAL_DEV v3 cross(v3 a, v3 b) { return v3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
BAL_DEV double comp(v3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
BAL_DEV v3 ld3(const double *p, int i) { return v3{p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }

// ------------------------------------------------------------------ barrier
// b(d, dh) = -(d - dh)^2 ln(d / dh) on 0 < d < dh, zero beyond (eq. IPC-barrier).
BAL_DEV double barrier(double d, double dh) {
  if (d >= dh) return 0.0;
  double t = d - dh;
  return -t * t * log(d / dh);
}
BAL_DEV double barrier_d1(double d, double dh) {
  if (d >= dh) return 0.0;
  double t = d - dh;
  return -2.0 * t * log(d / dh) - t * t / d;
}
BAL_DEV double barrier_d2(double d, double dh) {
  if (d >= dh) return 0.0;
  double t = d - dh;
  return -2.0 * log(d / dh) - 4.0 * t / d + t * t / (d * d);
}

// ------------------------------------------------------- symmetric projection
// Packed upper-triangular index of (i, j), i <= j, in an N x N symmetric matrix.
template <int N>
BAL_DEV constexpr int pk(int i, int j) {
  return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
}

// Cyclic Jacobi on a symmetric N x N matrix held packed (upper triangle,
// N(N+1)/2 doubles) in registers; on return P holds V diag(max(lambda, 0)) V^T
// and the function returns the sum of the clamped eigenvalues (the trace of
// the projection).  Rotations use the symmetric two-sided update.
template <int N>
BAL_DEV double project_psd(double *P) {
  double V[N * N];
#pragma unroll
  for (int i = 0; i < N * N; ++i) V[i] = (i / N == i % N) ? 1.0 : 0.0;
  double fro = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) fro += (i == j ? 1.0 : 2.0) * P[pk<N>(i, j)] * P[pk<N>(i, j)];
  const double tol = 1e-30 * fro;
  for (int sweep = 0; sweep < 24; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int q = p + 1; q < N; ++q) off += P[pk<N>(p, q)] * P[pk<N>(p, q)];
    if (off <= tol) break;
#pragma unroll
    for (int p = 0; p < N; ++p) {
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        double apq = P[pk<N>(p, q)];
        if (apq * apq <= 1e-36 * fro) continue;
        double theta = (P[pk<N>(q, q)] - P[pk<N>(p, p)]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0);
        double s = t * c;
        P[pk<N>(p, p)] -= t * apq;
        P[pk<N>(q, q)] += t * apq;
        P[pk<N>(p, q)] = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          if (k == p || k == q) continue;
          double akp = P[pk<N>(k, p)], akq = P[pk<N>(k, q)];
          P[pk<N>(k, p)] = c * akp - s * akq;
          P[pk<N>(k, q)] = s * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
          double vkp = V[k * N + p], vkq = V[k * N + q];
          V[k * N + p] = c * vkp - s * vkq;
          V[k * N + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  double lam[N];
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    lam[i] = P[pk<N>(i, i)] > 0.0 ? P[pk<N>(i, i)] : 0.0;
    tr += lam[i];
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += V[i * N + k] * lam[k] * V[j * N + k];
      P[pk<N>(i, j)] = acc;
    }
  return tr;
}

// Reduced basis of a stencil: W is R x K (R difference vectors over K nodes,
// row-major, small integers).  Computes the lower Cholesky factor L of W W^T
// (R x R) and Q = W^T L^{-T} (K x R).
template <int R, int K>
BAL_DEV void reduced_basis(const double *W, double *L, double *Q) {
  double G[R * R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) s += W[i * K + k] * W[j * K + k];
      G[i * R + j] = s;
    }
#pragma unroll
  for (int i = 0; i < R * R; ++i) L[i] = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double s = G[j * R + j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j * R + k] * L[j * R + k];
    L[j * R + j] = sqrt(s);
#pragma unroll
    for (int i = j + 1; i < R; ++i) {
      double t = G[i * R + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i * R + k] * L[j * R + k];
      L[i * R + j] = t / L[j * R + j];
    }
  }
  // Q^T = L^{-1} W  (forward substitution per column of W)
#pragma unroll
  for (int c = 0; c < K; ++c) {
    double y[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double t = W[i * K + c];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i * R + k] * y[k];
      y[i] = t / L[i * R + i];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) Q[c * R + i] = y[i];
  }
}

// M = (L^T (x) I3) Hu (L (x) I3) for Hu of size 3R x 3R (blocks indexed by
// difference vector), in place.
template <int R>
BAL_DEV void reduce_hessian(double *Hu, const double *L) {
  constexpr int n = 3 * R;
  double T[n * n];
  // T = Hu (L (x) I3): column block q = sum_l Hu[:, block l] L[l][q]
#pragma unroll
  for (int r = 0; r < n; ++r)
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
#pragma unroll
        for (int l = q; l < R; ++l) s += Hu[r * n + 3 * l + c] * L[l * R + q];
        T[r * n + 3 * q + c] = s;
      }
#pragma unroll
  for (int p = 0; p < R; ++p)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int col = 0; col < n; ++col) {
        double s = 0.0;
#pragma unroll
        for (int k = p; k < R; ++k) s += L[k * R + p] * T[(3 * k + a) * n + col];
        Hu[(3 * p + a) * n + col] = s;
      }
}

// 3x3 block (a, b) of (Q (x) I3) Mp (Q (x) I3)^T for packed symmetric Mp
// (3R x 3R), written row-major to out[9].
template <int R>
BAL_DEV void expand_block(const double *Mp, const double *Q, int a, int b, double *out) {
  constexpr int n = 3 * R;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < R; ++p)
#pragma unroll
        for (int q = 0; q < R; ++q) s += Q[a * R + p] * Mp[pk<n>(3 * p + i, 3 * q + j)] * Q[b * R + q];
      out[3 * i + j] = s;
    }
}

// Packs the upper triangle of a full n x n matrix.
template <int n>
BAL_DEV void pack_sym(const double *F, double *P) {
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = i; j < n; ++j) P[pk<n>(i, j)] = 0.5 * (F[i * n + j] + F[j * n + i]);
}

// ------------------------------------------------------------ element terms
// Per-tet constants: B = Dm^{-1} (row-major 3x3), A = L^T B B^T L (symmetric
// 3x3 with L = chol(W W^T) of the element stencil), V mu, V lam.
struct TetConst {
  double B[9];
  double A[6];  // a00 a01 a02 a11 a12 a22
  double Vmu, Vlam, V, pad;
};

// Stencil of an element: u_k = x_{k+1} - x_0.
BAL_DEV void element_W(double *W) {
  const double w[12] = {-1, 1, 0, 0, -1, 0, 1, 0, -1, 0, 0, 1};
#pragma unroll
  for (int i = 0; i < 12; ++i) W[i] = w[i];
}

// Inverse and determinant of a 3x3 matrix given by its columns c0, c1, c2.
// Returns rows of the inverse (r_k = row k of Ds^{-1} = column k of Ds^{-T}).
BAL_DEV double inv_cols(v3 c0, v3 c1, v3 c2, v3 *r0, v3 *r1, v3 *r2) {
  v3 x12 = cross(c1, c2), x20 = cross(c2, c0), x01 = cross(c0, c1);
  double det = dot(c0, x12);
  double id = 1.0 / det;
  *r0 = id * x12;
  *r1 = id * x20;
  *r2 = id * x01;
  return det;
}

// ------------------------------------------------------------ distance cases
// Pair stencil nodes: PT = (p, a, b, c), EE = (a0, a1, b0, b1).
// Cases: 0 PT interior; 1 PE(p;a,b); 2 PE(p;b,c); 3 PE(p;c,a); 4 PP(p,a);
// 5 PP(p,b); 6 PP(p,c); 7 EE interior; 8 PE(a0;b0,b1); 9 PE(a1;b0,b1);
// 10 PE(b0;a0,a1); 11 PE(b1;a0,a1); 12 PP(a0,b0); 13 PP(a0,b1);
// 14 PP(a1,b0); 15 PP(a1,b1).
// Node slots of each case (distance depends on these stencil slots, in order).
__constant__ const int8_t kCaseNodes[16][4] = {
    {0, 1, 2, 3}, {0, 1, 2, -1}, {0, 2, 3, -1}, {0, 3, 1, -1}, {0, 1, -1, -1}, {0, 2, -1, -1},
    {0, 3, -1, -1}, {0, 1, 2, 3}, {0, 2, 3, -1}, {1, 2, 3, -1}, {2, 0, 1, -1}, {3, 0, 1, -1},
    {0, 2, -1, -1}, {0, 3, -1, -1}, {1, 2, -1, -1}, {1, 3, -1, -1}};
__constant__ const int8_t kCaseK[16] = {4, 3, 3, 3, 2, 2, 2, 4, 3, 3, 3, 3, 2, 2, 2, 2};
constexpr double kParallelEps = 1e-12;  // sin^2 of the angle between edges

// Squared point-segment distance; region 0 (at a), 1 (interior), 2 (at b).
BAL_DEV double pseg(v3 p, v3 a, v3 b, int *region) {
  v3 e = b - a, r = p - a;
  double ee = dot(e, e);
  double t = dot(r, e) / ee;
  if (t <= 0.0) { *region = 0; return dot(r, r); }
  if (t >= 1.0) { *region = 2; v3 rb = p - b; return dot(rb, rb); }
  *region = 1;
  v3 c = cross(r, e);
  return dot(c, c) / ee;
}

// Squared distance and case of a point-triangle pair.
BAL_DEV double pt_classify(v3 p, v3 a, v3 b, v3 c, int *cs) {
  v3 e1 = b - a, e2 = c - a, r = p - a;
  double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
  double b1 = dot(e1, r), b2 = dot(e2, r);
  double det = a11 * a22 - a12 * a12;
  double be1 = (a22 * b1 - a12 * b2) / det;
  double be2 = (a11 * b2 - a12 * b1) / det;
  if (be1 >= 0.0 && be2 >= 0.0 && be1 + be2 <= 1.0) {
    v3 n = cross(e1, e2);
    double s = dot(r, n);
    *cs = 0;
    return s * s / dot(n, n);
  }
  int g;
  double best = pseg(p, a, b, &g);
  int bc = g == 0 ? 4 : (g == 1 ? 1 : 5);
  double q = pseg(p, b, c, &g);
  if (q < best) { best = q; bc = g == 0 ? 5 : (g == 1 ? 2 : 6); }
  q = pseg(p, c, a, &g);
  if (q < best) { best = q; bc = g == 0 ? 6 : (g == 1 ? 3 : 4); }
  *cs = bc;
  return best;
}

BAL_DEV bool ee_parallel(v3 e1, v3 e2) {
  v3 n = cross(e1, e2);
  return dot(n, n) < kParallelEps * dot(e1, e1) * dot(e2, e2);
}

// Squared distance and case of an edge-edge pair.
BAL_DEV double ee_classify(v3 a0, v3 a1, v3 b0, v3 b1, int *cs) {
  v3 e1 = a1 - a0, e2 = b1 - b0, w = a0 - b0;
  v3 n = cross(e1, e2);
  double nn = dot(n, n);
  double a = dot(e1, e1), b = dot(e1, e2), c = dot(e2, e2);
  bool par = nn < kParallelEps * a * c;
  if (!par) {
    double d = dot(e1, w), e = dot(e2, w);
    double den = nn;  // equals a c - b^2 without its cancellation
    double s = (b * e - c * d) / den;
    double t = (a * e - b * d) / den;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      double sw = dot(w, n);
      *cs = 7;
      return sw * sw / nn;
    }
  }
  int g;
  double best = pseg(a0, b0, b1, &g);
  int bc = g == 0 ? 12 : (g == 1 ? 8 : 13);
  double q = pseg(a1, b0, b1, &g);
  if (q < best) { best = q; bc = g == 0 ? 14 : (g == 1 ? 9 : 15); }
  q = pseg(b0, a0, a1, &g);
  if (q < best) { best = q; bc = g == 0 ? 12 : (g == 1 ? 10 : 14); }
  q = pseg(b1, a0, a1, &g);
  if (q < best) { best = q; bc = g == 0 ? 13 : (g == 1 ? 11 : 15); }
  *cs = bc;
  return best;
}

BAL_DEV double pair_classify(int kind, const v3 *X, int *cs) {
  return kind == 0 ? pt_classify(X[0], X[1], X[2], X[3], cs) : ee_classify(X[0], X[1], X[2], X[3], cs);
}

// ------------------------------------------- squared distance derivatives
// For the 9-dim cases (PT interior, EE interior) u = (r, e1, e2) and
// q = s^2 / m with s = r . (e1 x e2), m = |e1 x e2|^2.
// PT: r = p - a, e1 = b - a, e2 = c - a.  EE: r = a0 - b0, e1 = a1 - a0, e2 = b1 - b0.
// Writes q, grad (9) and Hessian (81, row-major).
BAL_DEV void skew_add(double *H, int n, int r0, int c0, v3 v, double s) {
  // H[r0+i][c0+j] += s * [v]x_ij, [v]x = [[0,-vz,vy],[vz,0,-vx],[-vy,vx,0]]
  H[(r0 + 0) * n + c0 + 1] += -s * v.z;
  H[(r0 + 0) * n + c0 + 2] += s * v.y;
  H[(r0 + 1) * n + c0 + 0] += s * v.z;
  H[(r0 + 1) * n + c0 + 2] += -s * v.x;
  H[(r0 + 2) * n + c0 + 0] += -s * v.y;
  H[(r0 + 2) * n + c0 + 1] += s * v.x;
}

BAL_DEV void q9_derivs(v3 r, v3 e1, v3 e2, double *qo, double *g, double *H) {
  v3 n = cross(e1, e2);
  double s = dot(r, n), m = dot(n, n);
  double gs[9], gm[9], Hs[81], Hm[81];
#pragma unroll
  for (int i = 0; i < 81; ++i) { Hs[i] = 0.0; Hm[i] = 0.0; }
  v3 gs1 = cross(e2, r), gs2 = cross(r, e1);
  v3 gm1 = 2.0 * cross(e2, n), gm2 = 2.0 * cross(n, e1);
  const v3 gsb[3] = {n, gs1, gs2};
  const v3 gmb[3] = {mk(0, 0, 0), gm1, gm2};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) { gs[3 * b + i] = comp(gsb[b], i); gm[3 * b + i] = comp(gmb[b], i); }
  // Hessian of s: (r,e1) = -[e2]x, (r,e2) = [e1]x, (e1,e2) = -[r]x, plus transposes
  skew_add(Hs, 9, 0, 3, e2, -1.0);
  skew_add(Hs, 9, 3, 0, e2, 1.0);
  skew_add(Hs, 9, 0, 6, e1, 1.0);
  skew_add(Hs, 9, 6, 0, e1, -1.0);
  skew_add(Hs, 9, 3, 6, r, -1.0);
  skew_add(Hs, 9, 6, 3, r, 1.0);
  // Hessian of m: (e1,e1) = 2(|e2|^2 I - e2 e2^T), (e2,e2) = 2(|e1|^2 I - e1 e1^T),
  // (e1,e2) = 2(e1 e2^T - (e1.e2) I) - 2[n]x, (e2,e1) its transpose
  double d12 = dot(e1, e2), s22 = dot(e2, e2), s11 = dot(e1, e1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double dij = i == j ? 1.0 : 0.0;
      Hm[(3 + i) * 9 + 3 + j] = 2.0 * (s22 * dij - comp(e2, i) * comp(e2, j));
      Hm[(6 + i) * 9 + 6 + j] = 2.0 * (s11 * dij - comp(e1, i) * comp(e1, j));
      double x = 2.0 * (comp(e1, i) * comp(e2, j) - d12 * dij);
      Hm[(3 + i) * 9 + 6 + j] = x;
      Hm[(6 + j) * 9 + 3 + i] = x;
    }
  skew_add(Hm, 9, 3, 6, n, -2.0);
  skew_add(Hm, 9, 6, 3, n, 2.0);
  double im = 1.0 / m;
  *qo = s * s * im;
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = 2.0 * s * im * gs[i] - s * s * im * im * gm[i];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j)
      H[i * 9 + j] = 2.0 * im * gs[i] * gs[j] + 2.0 * s * im * Hs[i * 9 + j] -
                     2.0 * s * im * im * (gs[i] * gm[j] + gm[i] * gs[j]) - s * s * im * im * Hm[i * 9 + j] +
                     2.0 * s * s * im * im * im * gm[i] * gm[j];
}

// Point-edge: u = (r, e), r = p - a, e = b - a, q = |r x e|^2 / |e|^2.
BAL_DEV void q6_derivs(v3 r, v3 e, double *qo, double *g, double *H) {
  v3 w = cross(r, e);
  double W = dot(w, w), E = dot(e, e);
  double gW[6], gE[6];
  v3 gWr = 2.0 * cross(e, w), gWe = 2.0 * cross(w, r);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gW[i] = comp(gWr, i); gW[3 + i] = comp(gWe, i);
    gE[i] = 0.0; gE[3 + i] = 2.0 * comp(e, i);
  }
  double HW[36];
  double ee = dot(e, e), rr = dot(r, r), er = dot(e, r);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double dij = i == j ? 1.0 : 0.0;
      HW[i * 6 + j] = 2.0 * (ee * dij - comp(e, i) * comp(e, j));
      HW[(3 + i) * 6 + 3 + j] = 2.0 * (rr * dij - comp(r, i) * comp(r, j));
      double x = 2.0 * (comp(r, i) * comp(e, j) - er * dij);
      HW[i * 6 + 3 + j] = x;
      HW[(3 + j) * 6 + i] = x;
    }
  skew_add(HW, 6, 0, 3, w, -2.0);
  skew_add(HW, 6, 3, 0, w, 2.0);
  double iE = 1.0 / E;
  *qo = W * iE;
#pragma unroll
  for (int i = 0; i < 6; ++i) g[i] = gW[i] * iE - W * iE * iE * gE[i];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double HE = (i >= 3 && i == j) ? 2.0 : 0.0;
      H[i * 6 + j] = HW[i * 6 + j] * iE - (gW[i] * gE[j] + gE[i] * gW[j]) * iE * iE - W * iE * iE * HE +
                     2.0 * W * iE * iE * iE * gE[i] * gE[j];
    }
}

// Difference-vector matrices W (rows over the case's local nodes, as listed in kCaseNodes).
// 9-dim PT: r = p - a, e1 = b - a, e2 = c - a.
// 9-dim EE: r = a0 - b0, e1 = a1 - a0, e2 = b1 - b0.
// 6-dim PE (nodes p, a, b): r = p - a, e = b - a.   3-dim PP (nodes p, a): r = p - a.
BAL_DEV void case_W(int cs, double *W) {
  if (cs == 0) {
    const double w[12] = {1, -1, 0, 0, 0, -1, 1, 0, 0, -1, 0, 1};
    for (int i = 0; i < 12; ++i) W[i] = w[i];
  } else if (cs == 7) {
    const double w[12] = {1, 0, -1, 0, -1, 1, 0, 0, 0, 0, -1, 1};
    for (int i = 0; i < 12; ++i) W[i] = w[i];
  } else if (kCaseK[cs] == 3) {
    const double w[6] = {1, -1, 0, 0, -1, 1};
    for (int i = 0; i < 6; ++i) W[i] = w[i];
  } else {
    W[0] = 1; W[1] = -1;
  }
}

}  // namespace bal
