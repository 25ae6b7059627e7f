// Neo-Hookean element kernels: energy, gradient and the projected 12x12
// element Hessian (Sec. 4.2, stencil-wise projection), one thread per tet.
//
// With Ds = [x1-x0, x2-x0, x3-x0], F = Ds B (B = Dm^{-1}), C = Ds^{-T} (its
// columns r_k are the rows of Ds^{-1}) and c' = lam ln J - mu:
//   Psi      = V [mu/2 (|F|^2 - 3) - mu ln J + lam/2 (ln J)^2]
//   dPsi/du_k = V [mu sum_j B_kj F_j + c' r_k]          (u_k = x_{k+1} - x_0)
//   M_pq     = V [mu A_pq I + lam d_p d_q^T - c' d_q d_p^T],  d_p = sum_k L_kp r_k,
// where A = L^T B B^T L and L = chol(W W^T) of the element stencil; M is the
// 9x9 reduced Hessian whose clamped eigen-reconstruction gives the exact
// closest-PSD 12x12 element Hessian (see bal_math.h).
#include "bal_internal.h"

namespace bal {

struct ElemBasis {
  double L[9];
  double Q[12];
};

// MODE is a template argument: the energy and gradient launches (line
// search, gradient) then get registers for what they compute, not the
// Hessian's eigen-solve footprint, and run at full occupancy
template <typename MT, int MODE>
__global__ __launch_bounds__(128) void k_elements(int T, const int4 *__restrict__ tets,
                                                  const TetConst *__restrict__ tc, const double *__restrict__ x,
                                                  int project, ElemBasis eb, double *__restrict__ tet_e,
                                                  double *__restrict__ tet_g, MT *__restrict__ tet_blk,
                                                  double *__restrict__ tet_tr, int *__restrict__ flags) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int4 tv = tets[t];
  v3 x0 = ld3(x, tv.x), x1 = ld3(x, tv.y), x2 = ld3(x, tv.z), x3 = ld3(x, tv.w);
  v3 c0 = x1 - x0, c1 = x2 - x0, c2 = x3 - x0;
  const TetConst k = tc[t];
  v3 rr[3];
  double detDs = inv_cols(c0, c1, c2, &rr[0], &rr[1], &rr[2]);
  double J = detDs / (6.0 * k.V);
  if (!(J > 0.0)) {
    tet_e[t] = 0.0;
    atomicOr(flags, 1);
    return;
  }
  const double *B = k.B;
  v3 F0 = B[0] * c0 + B[3] * c1 + B[6] * c2;
  v3 F1 = B[1] * c0 + B[4] * c1 + B[7] * c2;
  v3 F2 = B[2] * c0 + B[5] * c1 + B[8] * c2;
  double I1 = dot(F0, F0) + dot(F1, F1) + dot(F2, F2);
  double lj = log(J);
  tet_e[t] = 0.5 * k.Vmu * (I1 - 3.0) - k.Vmu * lj + 0.5 * k.Vlam * lj * lj;
  if constexpr (MODE == EM_ENERGY) return;
  double Vc = k.Vlam * lj - k.Vmu;
  v3 gu[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) gu[q] = k.Vmu * (B[3 * q] * F0 + B[3 * q + 1] * F1 + B[3 * q + 2] * F2) + Vc * rr[q];
  v3 g0 = -1.0 * (gu[0] + gu[1] + gu[2]);
  double *gt = tet_g + (size_t)t * 12;
  gt[0] = g0.x; gt[1] = g0.y; gt[2] = g0.z;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    gt[3 + 3 * q] = gu[q].x;
    gt[4 + 3 * q] = gu[q].y;
    gt[5 + 3 * q] = gu[q].z;
  }
  if constexpr (MODE == EM_GRAD) return;
  const double *L = eb.L;
  v3 d[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) d[p] = L[0 * 3 + p] * rr[0] + L[1 * 3 + p] * rr[1] + L[2 * 3 + p] * rr[2];
  const double A[9] = {k.A[0], k.A[1], k.A[2], k.A[1], k.A[3], k.A[4], k.A[2], k.A[4], k.A[5]};
  double M[45];  // packed upper triangle of the 9x9 reduced Hessian
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = p; q < 3; ++q)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (3 * p + i > 3 * q + j) continue;
          M[pk<9>(3 * p + i, 3 * q + j)] = (i == j ? k.Vmu * A[3 * p + q] : 0.0) +
                                           k.Vlam * comp(d[p], i) * comp(d[q], j) -
                                           Vc * comp(d[q], i) * comp(d[p], j);
        }
  double tr;
  if (project) {
    tr = project_psd<9>(M);
  } else {
    tr = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) tr += M[pk<9>(i, i)];
  }
  tet_tr[t] = tr / 12.0;
  const int sa[10] = {0, 1, 2, 3, 0, 0, 0, 1, 1, 2};
  const int sb[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
  MT *out = tet_blk + (size_t)t * 90;
#pragma unroll
  for (int s = 0; s < 10; ++s) {
    double blk[9];
    expand_block<3>(M, eb.Q, sa[s], sb[s], blk);
#pragma unroll
    for (int e = 0; e < 9; ++e) out[s * 9 + e] = (MT)blk[e];
  }
}

template <typename MT, int MODE>
static void launch_elements_t(Scene &s, const double *x, int project, const ElemBasis &eb) {
  dim3 grid(blocks_for(s.T, 128)), block(128);
  hipLaunchKernelGGL((k_elements<MT, MODE>), grid, block, 0, s.stream, s.T, s.tets.as<int4>(), s.tc.as<TetConst>(),
                     x, project, eb, s.tet_e.as<double>(), s.tet_g.as<double>(), static_cast<MT *>(s.tet_blk.p),
                     s.tet_tr.as<double>(), s.flags.as<int>());
}

template <typename MT>
static void launch_elements_m(Scene &s, const double *x, int mode, int project, const ElemBasis &eb) {
  if (mode == EM_ENERGY) launch_elements_t<MT, EM_ENERGY>(s, x, project, eb);
  else if (mode == EM_GRAD) launch_elements_t<MT, EM_GRAD>(s, x, project, eb);
  else launch_elements_t<MT, EM_HESS>(s, x, project, eb);
}

void launch_elements(Scene &s, const double *x, int mode, int project) {
  ElemBasis eb;
  for (int i = 0; i < 9; ++i) eb.L[i] = s.Lel[i];
  for (int i = 0; i < 12; ++i) eb.Q[i] = s.Qel[i];
  if (s.T == 0) return;
  if (s.mixed) launch_elements_m<float>(s, x, mode, project, eb);
  else launch_elements_m<double>(s, x, mode, project, eb);
}

}  // namespace bal
