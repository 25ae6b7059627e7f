// Assembly, block SpMV and PCG (Sec. 5.1 sparse storage and SpMV, Sec. 4.2
// block-Jacobi warm start, App. B stopping rules), plus deterministic
// reductions and scans.
//
// Storage.  The static element part is a full (both triangles) 3x3 block
// CSR over free nodes, gathered per block from per-tet blocks through a
// static source list, so assembly and SpMV need no atomics and are
// bit-reproducible.  Contact blocks stay in per-pair buffers; per Newton
// iteration each row gets a sorted list of the contact blocks it reads.
// Diagonal blocks (mass + elements + contacts) form the dense block
// diagonal D that also feeds the block-Jacobi preconditioner.
#include "bal_internal.h"

namespace bal {

constexpr int kBS = 256;

// ------------------------------------------------------------ reductions
template <typename Op>
__device__ double block_reduce(double v, Op op, double ident) {
  __shared__ double sh[kBS / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_down(v, o, 64));
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = op(r, sh[i]);
    sh[0] = r;
  }
  __syncthreads();
  double r = sh[0];
  __syncthreads();
  return r;
}

struct OpSum { __device__ double operator()(double a, double b) const { return a + b; } };
struct OpMin { __device__ double operator()(double a, double b) const { return a < b ? a : b; } };

template <typename Op>
__global__ void k_reduce_stage(const double *__restrict__ in, long n, double *__restrict__ out, Op op,
                               double ident) {
  double acc = ident;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc = op(acc, in[i]);
  acc = block_reduce(acc, op, ident);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

__global__ void k_count_less(const double *__restrict__ in, long n, double thr, double *__restrict__ out) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += in[i] < thr ? 1.0 : 0.0;
  acc = block_reduce(acc, OpSum(), 0.0);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

static double read_scalar(Scene &s, const double *dptr) {
  double *h = s.pin.as<double>();
  hipMemcpyAsync(h, dptr, sizeof(double), hipMemcpyDeviceToHost, s.stream);
  hipStreamSynchronize(s.stream);
  return h[0];
}

template <typename Op>
static double reduce_op(Scene &s, const double *in, int n, Op op, double ident) {
  if (n <= 0) return ident;
  int nb = blocks_for(n, kBS);
  if (nb > 1024) nb = 1024;
  double *part = s.red_out.as<double>();
  hipLaunchKernelGGL(k_reduce_stage<Op>, dim3(nb), dim3(kBS), 0, s.stream, in, (long)n, part + 1, op, ident);
  hipLaunchKernelGGL(k_reduce_stage<Op>, dim3(1), dim3(kBS), 0, s.stream, part + 1, (long)nb, part, op, ident);
  return read_scalar(s, part);
}

double reduce_sum(Scene &s, const double *in, int n) { return reduce_op(s, in, n, OpSum(), 0.0); }
double reduce_min(Scene &s, const double *in, int n) { return reduce_op(s, in, n, OpMin(), INFINITY); }
int reduce_count_less(Scene &s, const double *in, int n, double thr) {
  if (n <= 0) return 0;
  int nb = blocks_for(n, kBS);
  if (nb > 1024) nb = 1024;
  double *part = s.red_out.as<double>();
  hipLaunchKernelGGL(k_count_less, dim3(nb), dim3(kBS), 0, s.stream, in, (long)n, thr, part + 1);
  hipLaunchKernelGGL(k_reduce_stage<OpSum>, dim3(1), dim3(kBS), 0, s.stream, part + 1, (long)nb, part, OpSum(), 0.0);
  return (int)llround(read_scalar(s, part));
}

__global__ void k_dot_free(const double *__restrict__ a, const double *__restrict__ b, int n3,
                           double *__restrict__ out) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  acc = block_reduce(acc, OpSum(), 0.0);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

double dot_free(Scene &s, const double *a, const double *b) {
  int n3 = 3 * s.N;
  int nb = blocks_for(n3, kBS);
  if (nb > 1024) nb = 1024;
  double *part = s.red_out.as<double>();
  hipLaunchKernelGGL(k_dot_free, dim3(nb), dim3(kBS), 0, s.stream, a, b, n3, part + 1);
  hipLaunchKernelGGL(k_reduce_stage<OpSum>, dim3(1), dim3(kBS), 0, s.stream, part + 1, (long)nb, part, OpSum(), 0.0);
  return read_scalar(s, part);
}

// ------------------------------------------------------------------ scan
constexpr int kScanItems = 4;
__global__ void k_scan_block(const int *__restrict__ in, int *__restrict__ out, int n, int *__restrict__ sums) {
  __shared__ int sh[kBS];
  int base = blockIdx.x * kBS * kScanItems + threadIdx.x * kScanItems;
  int v[kScanItems];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    tot += v[k];
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < kBS; o <<= 1) {
    int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tot;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kBS - 1) sums[blockIdx.x] = sh[kBS - 1];
}

__global__ void k_scan_sums(int *__restrict__ sums, int nb, int *__restrict__ total) {
  __shared__ int sh[kBS];
  int carry = 0;
  for (int base = 0; base < nb; base += kBS) {
    int i = base + threadIdx.x;
    int v = i < nb ? sums[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBS; o <<= 1) {
      int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + sh[threadIdx.x] - v;
    int blocktot = sh[kBS - 1];
    __syncthreads();
    carry += blocktot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int *__restrict__ out, int n, const int *__restrict__ sums) {
  int i = blockIdx.x * kBS * kScanItems + threadIdx.x;
  int add = sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int j = i + k * kBS;
    if (j < n) out[j] += add;
  }
}

int scan_exclusive(Scene &s, const int *in, int *out, int n) {
  if (n <= 0) return 0;
  int nb = blocks_for(n, kBS * kScanItems);
  if (s.scan_tmp.grow((size_t)(nb + 2) * sizeof(int))) return -1;
  int *sums = s.scan_tmp.as<int>() + 1;
  int *total = s.scan_tmp.as<int>();
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kBS), 0, s.stream, in, out, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBS), 0, s.stream, sums, nb, total);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kBS), 0, s.stream, out, n, sums);
  int *h = s.pin.as<int>();
  hipMemcpyAsync(h, total, sizeof(int), hipMemcpyDeviceToHost, s.stream);
  hipStreamSynchronize(s.stream);
  return h[0];
}

// ------------------------------------------------------------ vectors
__global__ void k_predictor(int N, const double *__restrict__ xt, const double *__restrict__ vt,
                            const uint8_t *__restrict__ fr, double h, double gx, double gy, double gz,
                            double *__restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double g[3] = {gx, gy, gz};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double xv = xt[3 * i + c];
    y[3 * i + c] = fr[i] ? xv + h * vt[3 * i + c] + h * h * g[c] : xv;
  }
}

void launch_predictor(Scene &s) {
  hipLaunchKernelGGL(k_predictor, dim3(blocks_for(s.N, kBS)), dim3(kBS), 0, s.stream, s.N, s.x_t.as<double>(),
                     s.v_t.as<double>(), s.freev.as<uint8_t>(), s.desc.dt, s.desc.gravity[0], s.desc.gravity[1],
                     s.desc.gravity[2], s.y.as<double>());
}

__global__ void k_axpy(double *__restrict__ out, const double *__restrict__ a, const double *__restrict__ b,
                       double alpha, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + alpha * b[i];
}

void launch_axpy_state(Scene &s, double *out, const double *a, const double *b, double alpha, int n3) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n3, kBS)), dim3(kBS), 0, s.stream, out, a, b, alpha, n3);
}

// 1/(2h^2) m |x - y|^2 per free node (inertia term of the incremental potential, Sec. 3.1).
__global__ void k_inertia(int N, const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ m, const uint8_t *__restrict__ fr, double ih2,
                          double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double e = 0.0;
  if (fr[i]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double d = x[3 * i + c] - y[3 * i + c];
      e += d * d;
    }
    e *= 0.5 * ih2 * m[i];
  }
  out[i] = e;
}

void launch_inertia_energy(Scene &s, const double *x, double *out) {
  hipLaunchKernelGGL(k_inertia, dim3(blocks_for(s.N, kBS)), dim3(kBS), 0, s.stream, s.N, x, s.y.as<double>(),
                     s.mass.as<double>(), s.freev.as<uint8_t>(), 1.0 / (s.desc.dt * s.desc.dt), out);
}

// ------------------------------------------------------ contact lists
// Per union pair, for the case's nodes a, b (both free): a diagonal source
// (node_a; pair*4 + slot_a) and off-diagonal sources (node_a, node_b;
// pair*16 + slot_a*4 + slot_b).
__global__ void k_contact_count(int n, const int4 *__restrict__ nodes, const int *__restrict__ pcase,
                                const uint8_t *__restrict__ fr, int *__restrict__ dcnt, int *__restrict__ ocnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int4 nd = nodes[i];
  int idx[4] = {nd.x, nd.y, nd.z, nd.w};
  int cs = pcase[i];
  int k = kCaseK[cs];
  for (int a = 0; a < k; ++a) {
    int na = idx[kCaseNodes[cs][a]];
    if (!fr[na]) continue;
    atomicAdd(&dcnt[na], 1);
    for (int b = 0; b < k; ++b) {
      if (b == a) continue;
      int nbv = idx[kCaseNodes[cs][b]];
      if (fr[nbv]) atomicAdd(&ocnt[na], 1);
    }
  }
}

__global__ void k_contact_fill(int n, const int4 *__restrict__ nodes, const int *__restrict__ pcase,
                               const uint8_t *__restrict__ fr, const int *__restrict__ dptr,
                               const int *__restrict__ optr, int *__restrict__ dfill, int *__restrict__ ofill,
                               int *__restrict__ dsrc, int *__restrict__ ocol, int *__restrict__ osrc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int4 nd = nodes[i];
  int idx[4] = {nd.x, nd.y, nd.z, nd.w};
  int cs = pcase[i];
  int k = kCaseK[cs];
  for (int a = 0; a < k; ++a) {
    int sa = kCaseNodes[cs][a];
    int na = idx[sa];
    if (!fr[na]) continue;
    int pos = dptr[na] + atomicAdd(&dfill[na], 1);
    dsrc[pos] = i * 4 + sa;
    for (int b = 0; b < k; ++b) {
      if (b == a) continue;
      int sb = kCaseNodes[cs][b];
      int nbv = idx[sb];
      if (!fr[nbv]) continue;
      int p2 = optr[na] + atomicAdd(&ofill[na], 1);
      ocol[p2] = nbv;
      osrc[p2] = i * 16 + sa * 4 + sb;
    }
  }
}

// Insertion sort of each node's sources (deterministic order).
__global__ void k_contact_sort(int N, const int *__restrict__ dptr, int *__restrict__ dsrc,
                               const int *__restrict__ optr, int *__restrict__ ocol, int *__restrict__ osrc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int a = dptr[i] + 1; a < dptr[i + 1]; ++a) {
    int v = dsrc[a], b = a - 1;
    while (b >= dptr[i] && dsrc[b] > v) { dsrc[b + 1] = dsrc[b]; --b; }
    dsrc[b + 1] = v;
  }
  for (int a = optr[i] + 1; a < optr[i + 1]; ++a) {
    int v = osrc[a], c = ocol[a], b = a - 1;
    while (b >= optr[i] && osrc[b] > v) { osrc[b + 1] = osrc[b]; ocol[b + 1] = ocol[b]; --b; }
    osrc[b + 1] = v;
    ocol[b + 1] = c;
  }
}

int build_contact_lists(Scene &s) {
  int N = s.N;
  if (s.cdiag_ptr.grow((N + 1) * sizeof(int)) || s.coff_ptr.grow((N + 1) * sizeof(int)) ||
      s.ccount.grow(2 * (size_t)(N + 1) * sizeof(int)) || s.cfill.grow(2 * (size_t)(N + 1) * sizeof(int)))
    return BAL_E_OOM;
  int *dcnt = s.ccount.as<int>(), *ocnt = dcnt + (N + 1);
  int *dfill = s.cfill.as<int>(), *ofill = dfill + (N + 1);
  hipMemsetAsync(dcnt, 0, 2 * (size_t)(N + 1) * sizeof(int), s.stream);
  hipMemsetAsync(dfill, 0, 2 * (size_t)(N + 1) * sizeof(int), s.stream);
  int n = s.uni.n;
  if (n > 0)
    hipLaunchKernelGGL(k_contact_count, dim3(blocks_for(n, kBS)), dim3(kBS), 0, s.stream, n, s.uni.nodes.as<int4>(),
                       s.uni.cs.as<int>(), s.freev.as<uint8_t>(), dcnt, ocnt);
  s.n_cdiag = scan_exclusive(s, dcnt, s.cdiag_ptr.as<int>(), N + 1);
  s.n_coff = scan_exclusive(s, ocnt, s.coff_ptr.as<int>(), N + 1);
  if (s.n_cdiag < 0 || s.n_coff < 0) return BAL_E_OOM;
  if (s.cdiag_src.grow((size_t)(s.n_cdiag + 1) * sizeof(int)) || s.coff_col.grow((size_t)(s.n_coff + 1) * sizeof(int)) ||
      s.coff_src.grow((size_t)(s.n_coff + 1) * sizeof(int)))
    return BAL_E_OOM;
  if (n > 0) {
    hipLaunchKernelGGL(k_contact_fill, dim3(blocks_for(n, kBS)), dim3(kBS), 0, s.stream, n, s.uni.nodes.as<int4>(),
                       s.uni.cs.as<int>(), s.freev.as<uint8_t>(), s.cdiag_ptr.as<int>(), s.coff_ptr.as<int>(), dfill,
                       ofill, s.cdiag_src.as<int>(), s.coff_col.as<int>(), s.coff_src.as<int>());
    hipLaunchKernelGGL(k_contact_sort, dim3(blocks_for(N, kBS)), dim3(kBS), 0, s.stream, N, s.cdiag_ptr.as<int>(),
                       s.cdiag_src.as<int>(), s.coff_ptr.as<int>(), s.coff_col.as<int>(), s.coff_src.as<int>());
  }
  return BAL_OK;
}

// ------------------------------------------------------------ assembly
// Per node: gradient (inertia + elements + contacts), the diagonal block D
// (mass/h^2 + element and contact diagonal blocks), the stiffness estimate
// e_j (Sec. 4.2: 3 m/h^2 plus 3 x the mean projected eigenvalue of every
// stencil touching the node), its group floor(log10 e_j), and D^{-1}.
template <typename MT>
__global__ void k_node_assembly(int N, const double *__restrict__ x, const double *__restrict__ y,
                                const double *__restrict__ m, const uint8_t *__restrict__ fr, double ih2,
                                const int *__restrict__ ntp, const int *__restrict__ nts,
                                const double *__restrict__ tet_g, const MT *__restrict__ tet_blk,
                                const double *__restrict__ tet_tr, const int *__restrict__ dptr,
                                const int *__restrict__ dsrc, const double *__restrict__ pg,
                                const MT *__restrict__ pblk, const double *__restrict__ ptr, int with_contacts,
                                int with_inertia, int with_elements, int want_hess, double *__restrict__ grad,
                                MT *__restrict__ Dblk, MT *__restrict__ Dinv, double *__restrict__ e_nodes,
                                int *__restrict__ group) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (!fr[i]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) grad[3 * i + c] = 0.0;
    if (want_hess) {
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        Dblk[9 * i + e] = (MT)(e % 4 == 0 ? 1.0 : 0.0);
        Dinv[9 * i + e] = (MT)(e % 4 == 0 ? 1.0 : 0.0);
      }
      e_nodes[i] = 0.0;
      group[i] = -1000;
    }
    return;
  }
  double g[3] = {0.0, 0.0, 0.0};
  double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double est = 0.0;
  double mi = m[i] * ih2;
  if (with_inertia) {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = mi * (x[3 * i + c] - y[3 * i + c]);
  }
  if (with_elements) {
    for (int k = ntp[i]; k < ntp[i + 1]; ++k) {
      int src = nts[k];
      int t = src >> 2, a = src & 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] += tet_g[(size_t)t * 12 + 3 * a + c];
      if (want_hess) {
        const MT *b = tet_blk + (size_t)t * 90 + a * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) D[e] += (double)b[e];
        est += tet_tr[t];
      }
    }
  }
  if (with_contacts) {
    for (int k = dptr[i]; k < dptr[i + 1]; ++k) {
      int src = dsrc[k];
      int p = src >> 2, sa = src & 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] += pg[(size_t)p * 12 + 3 * sa + c];
      if (want_hess) {
        const MT *b = pblk + (size_t)p * 144 + (sa * 5) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) D[e] += (double)b[e];
        est += ptr[p];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) grad[3 * i + c] = g[c];
  if (!want_hess) return;
  D[0] += mi;
  D[4] += mi;
  D[8] += mi;
  double en = 3.0 * (mi + est);
  e_nodes[i] = en;
  group[i] = (int)floor(log10(en));
  double c00 = D[4] * D[8] - D[5] * D[7], c01 = D[5] * D[6] - D[3] * D[8], c02 = D[3] * D[7] - D[4] * D[6];
  double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
  double id = 1.0 / det;
  double inv[9] = {c00 * id, (D[2] * D[7] - D[1] * D[8]) * id, (D[1] * D[5] - D[2] * D[4]) * id,
                   c01 * id, (D[0] * D[8] - D[2] * D[6]) * id, (D[2] * D[3] - D[0] * D[5]) * id,
                   c02 * id, (D[1] * D[6] - D[0] * D[7]) * id, (D[0] * D[4] - D[1] * D[3]) * id};
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Dblk[9 * i + e] = (MT)D[e];
    Dinv[9 * i + e] = (MT)inv[e];
  }
}

void launch_node_assembly(Scene &s, const double *x, int with_contacts, int with_inertia, int with_elements,
                          int want_hess, double *grad_out) {
  double ih2 = 1.0 / (s.desc.dt * s.desc.dt);
  dim3 g(blocks_for(s.N, kBS)), b(kBS);
  if (s.mixed)
    hipLaunchKernelGGL(k_node_assembly<float>, g, b, 0, s.stream, s.N, x, s.y.as<double>(), s.mass.as<double>(),
                       s.freev.as<uint8_t>(), ih2, s.node_tet_ptr.as<int>(), s.node_tet_src.as<int>(),
                       s.tet_g.as<double>(), s.tet_blk.as<float>(), s.tet_tr.as<double>(), s.cdiag_ptr.as<int>(),
                       s.cdiag_src.as<int>(), s.pair_g.as<double>(), s.pair_blk.as<float>(), s.pair_tr.as<double>(),
                       with_contacts, with_inertia, with_elements, want_hess, grad_out, s.Dblk.as<float>(),
                       s.Dinv.as<float>(), s.e_nodes.as<double>(), s.group.as<int>());
  else
    hipLaunchKernelGGL(k_node_assembly<double>, g, b, 0, s.stream, s.N, x, s.y.as<double>(), s.mass.as<double>(),
                       s.freev.as<uint8_t>(), ih2, s.node_tet_ptr.as<int>(), s.node_tet_src.as<int>(),
                       s.tet_g.as<double>(), s.tet_blk.as<double>(), s.tet_tr.as<double>(), s.cdiag_ptr.as<int>(),
                       s.cdiag_src.as<int>(), s.pair_g.as<double>(), s.pair_blk.as<double>(), s.pair_tr.as<double>(),
                       with_contacts, with_inertia, with_elements, want_hess, grad_out, s.Dblk.as<double>(),
                       s.Dinv.as<double>(), s.e_nodes.as<double>(), s.group.as<int>());
}

// Off-diagonal block b of the static pattern: sum of its element sources
// (tet*10 + slot, bit 31 = transposed).
template <typename MT>
__global__ void k_offdiag_assembly(int nnzb, const int *__restrict__ sp, const int *__restrict__ src,
                                   const MT *__restrict__ tet_blk, MT *__restrict__ val) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = sp[b]; k < sp[b + 1]; ++k) {
    unsigned s = (unsigned)src[k];
    bool tr = (s >> 31) != 0;
    unsigned ts = s & 0x7fffffffu;
    const MT *blk = tet_blk + (size_t)(ts / 10) * 90 + (ts % 10) * 9;
    if (tr) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[3 * i + j] += (double)blk[3 * j + i];
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) acc[e] += (double)blk[e];
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) val[(size_t)b * 9 + e] = (MT)acc[e];
}

void launch_offdiag_assembly(Scene &s) {
  if (s.nnzb == 0) return;
  dim3 g(blocks_for(s.nnzb, kBS)), b(kBS);
  if (s.mixed)
    hipLaunchKernelGGL(k_offdiag_assembly<float>, g, b, 0, s.stream, s.nnzb, s.blk_src_ptr.as<int>(),
                       s.blk_src.as<int>(), s.tet_blk.as<float>(), s.val.as<float>());
  else
    hipLaunchKernelGGL(k_offdiag_assembly<double>, g, b, 0, s.stream, s.nnzb, s.blk_src_ptr.as<int>(),
                       s.blk_src.as<int>(), s.tet_blk.as<double>(), s.val.as<double>());
}

// ---------------------------------------------------------------- SpMV
// y_i = D_i v_i + sum_static A_ij v_j + sum_contact C_ij v_j; with masked,
// blocks whose row and column lie in different stiffness groups are skipped
// (the warm start's domain-decomposed product, Sec. 4.2).
template <typename MT, typename VT>
__device__ __forceinline__ void spmv_row(int i, const int *__restrict__ rp, const int *__restrict__ ci,
                                         const MT *__restrict__ val, const MT *__restrict__ D,
                                         const int *__restrict__ cp, const int *__restrict__ cc,
                                         const int *__restrict__ cs, const MT *__restrict__ pblk,
                                         const int *__restrict__ grp, int masked, const VT *__restrict__ v,
                                         VT *acc) {
  VT v0 = v[3 * i], v1 = v[3 * i + 1], v2 = v[3 * i + 2];
  const MT *d = D + (size_t)9 * i;
  acc[0] = (VT)d[0] * v0 + (VT)d[1] * v1 + (VT)d[2] * v2;
  acc[1] = (VT)d[3] * v0 + (VT)d[4] * v1 + (VT)d[5] * v2;
  acc[2] = (VT)d[6] * v0 + (VT)d[7] * v1 + (VT)d[8] * v2;
  int gi = masked ? grp[i] : 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    int j = ci[k];
    if (masked && grp[j] != gi) continue;
    const MT *a = val + (size_t)9 * k;
    VT w0 = v[3 * j], w1 = v[3 * j + 1], w2 = v[3 * j + 2];
    acc[0] += (VT)a[0] * w0 + (VT)a[1] * w1 + (VT)a[2] * w2;
    acc[1] += (VT)a[3] * w0 + (VT)a[4] * w1 + (VT)a[5] * w2;
    acc[2] += (VT)a[6] * w0 + (VT)a[7] * w1 + (VT)a[8] * w2;
  }
  for (int k = cp[i]; k < cp[i + 1]; ++k) {
    int j = cc[k];
    if (masked && grp[j] != gi) continue;
    const MT *a = pblk + (size_t)9 * cs[k];
    VT w0 = v[3 * j], w1 = v[3 * j + 1], w2 = v[3 * j + 2];
    acc[0] += (VT)a[0] * w0 + (VT)a[1] * w1 + (VT)a[2] * w2;
    acc[1] += (VT)a[3] * w0 + (VT)a[4] * w1 + (VT)a[5] * w2;
    acc[2] += (VT)a[6] * w0 + (VT)a[7] * w1 + (VT)a[8] * w2;
  }
}

template <typename MT, typename VT>
__global__ __launch_bounds__(kBS) void k_spmv(int N, const int *__restrict__ rp, const int *__restrict__ ci,
                                              const MT *__restrict__ val, const MT *__restrict__ D,
                                              const int *__restrict__ cp, const int *__restrict__ cc,
                                              const int *__restrict__ cs, const MT *__restrict__ pblk,
                                              const int *__restrict__ grp, int masked, const VT *__restrict__ v,
                                              VT *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  VT acc[3];
  spmv_row<MT, VT>(i, rp, ci, val, D, cp, cc, cs, pblk, grp, masked, v, acc);
  out[3 * i] = acc[0];
  out[3 * i + 1] = acc[1];
  out[3 * i + 2] = acc[2];
}

void launch_spmv(Scene &s, const void *vin, void *vout, int masked) {
  dim3 g(blocks_for(s.N, kBS)), b(kBS);
  if (s.mixed)
    hipLaunchKernelGGL((k_spmv<float, float>), g, b, 0, s.stream, s.N, s.row_ptr.as<int>(), s.col_idx.as<int>(),
                       s.val.as<float>(), s.Dblk.as<float>(), s.coff_ptr.as<int>(), s.coff_col.as<int>(),
                       s.coff_src.as<int>(), s.pair_blk.as<float>(), s.group.as<int>(), masked,
                       static_cast<const float *>(vin), static_cast<float *>(vout));
  else
    hipLaunchKernelGGL((k_spmv<double, double>), g, b, 0, s.stream, s.N, s.row_ptr.as<int>(), s.col_idx.as<int>(),
                       s.val.as<double>(), s.Dblk.as<double>(), s.coff_ptr.as<int>(), s.coff_col.as<int>(),
                       s.coff_src.as<int>(), s.pair_blk.as<double>(), s.group.as<int>(), masked,
                       static_cast<const double *>(vin), static_cast<double *>(vout));
}

double spmv_bytes(const Scene &s) {
  // the paper's symmetric storage: each off-diagonal pair of blocks once
  double w = s.mixed ? 4.0 : 8.0;
  double nL = 0.5 * (double)s.nnzb, nC = 0.5 * (double)s.n_coff;
  double N = (double)s.N;
  return (nL + nC) * (9.0 * w + 4.0) + N * 9.0 * w + 4.0 * N + 3.0 * N * w + 3.0 * N * w;
}

// ----------------------------------------------------------------- PCG
// Bins: bin(i) = 0 for the global solve; for the warm start the node's
// stiffness group + 32 clamped to [0, 63].  Each bin carries its own
// alpha, beta (segmented dot products).  The last block to finish a
// reduction (ticket counter) combines the per-block partials in block
// order, so the scalars are bit-reproducible.
template <int NB>
__device__ __forceinline__ int bin_of(const int *grp, int i) {
  if (NB == 1) return 0;
  int b = grp[i] + kGroupOffset;
  return b < 0 ? 0 : (b >= NB ? NB - 1 : b);
}

template <int NB, int NV>
__device__ bool block_partials_and_ticket(int bin, const double *vals, double *partial, unsigned *counter) {
  // Each thread contributes vals[0..NV) to one bin (bin < 0: nothing).  The
  // block's per-bin sums go to partial[block][v][bin]; returns true in the
  // last block to finish (after a fence), which may then read all partials.
  __shared__ double sh[NV][NB];
  __shared__ bool last;
  if (NB == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = block_reduce(bin >= 0 ? vals[v] : 0.0, OpSum(), 0.0);
      if (threadIdx.x == 0) sh[v][0] = r;
    }
  } else {
    __shared__ int sbin[kBS];
    __shared__ double sval[NV][kBS];
    sbin[threadIdx.x] = bin;
#pragma unroll
    for (int v = 0; v < NV; ++v) sval[v][threadIdx.x] = bin >= 0 ? vals[v] : 0.0;
    __syncthreads();
    for (int b = threadIdx.x; b < NB; b += blockDim.x) {
      double acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0.0;
      for (int t = 0; t < (int)blockDim.x; ++t)
        if (sbin[t] == b) {
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] += sval[v][t];
        }
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][b] = acc[v];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV * NB; k += blockDim.x)
    partial[(size_t)blockIdx.x * NV * NB + k] = sh[k / NB][k % NB];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(counter, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

template <int NB, int NV>
__device__ void combine_partials(const double *partial, double (*out)[NB]) {
  // out[v][bin] = sum over blocks in order (thread k handles entry k)
  for (int k = threadIdx.x; k < NV * NB; k += blockDim.x) {
    double acc = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) acc += partial[(size_t)b * NV * NB + k];
    out[k / NB][k % NB] = acc;
  }
  __syncthreads();
}

// q = A p ; partial p.q ; last block: alpha
template <typename MT, typename VT, int NB>
__global__ __launch_bounds__(kBS) void k_pcg_spmv(int N, const int *__restrict__ rp, const int *__restrict__ ci,
                                                  const MT *__restrict__ val, const MT *__restrict__ D,
                                                  const int *__restrict__ cp, const int *__restrict__ cc,
                                                  const int *__restrict__ cs, const MT *__restrict__ pblk,
                                                  const int *__restrict__ grp, const VT *__restrict__ p,
                                                  VT *__restrict__ q, PcgCtl *ctl, double *partial,
                                                  unsigned *counter) {
  if (ctl->done) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double vals[1] = {0.0};
  int bin = -1;
  if (i < N) {
    VT acc[3];
    spmv_row<MT, VT>(i, rp, ci, val, D, cp, cc, cs, pblk, grp, NB > 1, p, acc);
    q[3 * i] = acc[0];
    q[3 * i + 1] = acc[1];
    q[3 * i + 2] = acc[2];
    bin = bin_of<NB>(grp, i);
    vals[0] = (double)p[3 * i] * (double)acc[0] + (double)p[3 * i + 1] * (double)acc[1] +
              (double)p[3 * i + 2] * (double)acc[2];
  }
  if (!block_partials_and_ticket<NB, 1>(bin, vals, partial, counter)) return;
  __shared__ double tot[1][NB];
  combine_partials<NB, 1>(partial, tot);
  if (threadIdx.x == 0) {
    *counter = 0u;
    bool breakdown = false;
    for (int b = 0; b < NB; ++b) {
      double pq = tot[0][b];
      ctl->pq[b] = pq;
      if (!ctl->active[b]) { ctl->alpha[b] = 0.0; continue; }
      if (!(pq > 0.0)) {
        ctl->alpha[b] = 0.0;
        if (NB == 1) breakdown = true; else ctl->active[b] = 0;
        continue;
      }
      ctl->alpha[b] = ctl->rz[b] / pq;
    }
    if (breakdown) ctl->done = PCG_BREAKDOWN;
    __threadfence();
  }
}

// x += alpha p ; r -= alpha q ; z = Dinv r ; partials r.z, r.r ; last block: beta, stopping rules
template <typename MT, typename VT, int NB>
__global__ __launch_bounds__(kBS) void k_pcg_update(int N, const uint8_t *__restrict__ fr,
                                                    const MT *__restrict__ Dinv, const int *__restrict__ grp,
                                                    const VT *__restrict__ p, const VT *__restrict__ q,
                                                    double *__restrict__ x, double *__restrict__ r,
                                                    VT *__restrict__ z, PcgCtl *ctl, double *partial,
                                                    unsigned *counter) {
  if (ctl->done) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double vals[2] = {0.0, 0.0};
  int bin = -1;
  if (i < N && fr[i]) {
    int b = bin_of<NB>(grp, i);
    bin = b;
    double al = ctl->alpha[b];
    double rr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] += al * (double)p[3 * i + c];
      rr[c] = r[3 * i + c] - al * (double)q[3 * i + c];
      r[3 * i + c] = rr[c];
    }
    const MT *d = Dinv + (size_t)9 * i;
    double zz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      zz[c] = (double)d[3 * c] * rr[0] + (double)d[3 * c + 1] * rr[1] + (double)d[3 * c + 2] * rr[2];
      z[3 * i + c] = (VT)zz[c];
    }
    vals[0] = rr[0] * (double)(VT)zz[0] + rr[1] * (double)(VT)zz[1] + rr[2] * (double)(VT)zz[2];
    vals[1] = rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2];
  }
  if (!block_partials_and_ticket<NB, 2>(bin, vals, partial, counter)) return;
  __shared__ double tot[2][NB];
  combine_partials<NB, 2>(partial, tot);
  if (threadIdx.x == 0) {
    *counter = 0u;
    ctl->it += 1;
    double rrsum = 0.0;
    int any = 0;
    for (int b = 0; b < NB; ++b) {
      rrsum += tot[1][b];
      if (!ctl->active[b]) { ctl->beta[b] = 0.0; continue; }
      ctl->beta[b] = ctl->rz[b] != 0.0 ? tot[0][b] / ctl->rz[b] : 0.0;
      ctl->rz[b] = tot[0][b];
      ctl->rr[b] = tot[1][b];
      if (NB > 1 && tot[1][b] <= ctl->tol2 * ctl->ref2[b]) ctl->active[b] = 0;
      any |= ctl->active[b];
    }
    double rn = sqrt(rrsum);
    ctl->rnorm = rn;
    if (NB == 1) {
      if (rrsum <= ctl->tol2 * ctl->ref2[0]) ctl->done = PCG_CONVERGED;
      if (rn < ctl->rmin) { ctl->rmin = rn; ctl->it_min = ctl->it; }
      if (!ctl->done && ctl->stall_window > 0 && ctl->it - ctl->it_min >= ctl->stall_window) ctl->done = PCG_STALLED;
    } else if (!any) {
      ctl->done = PCG_CONVERGED;
    }
    if (!ctl->done && ctl->it >= ctl->max_it) ctl->done = PCG_CAPPED;
    __threadfence();
  }
}

template <typename VT, int NB>
__global__ void k_pcg_dir(int N, const int *__restrict__ grp, const VT *__restrict__ z, VT *__restrict__ p,
                          const PcgCtl *ctl) {
  if (ctl->done) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double be = ctl->beta[bin_of<NB>(grp, i)];
#pragma unroll
  for (int c = 0; c < 3; ++c) p[3 * i + c] = (VT)((double)z[3 * i + c] + be * (double)p[3 * i + c]);
}

// r = b - q (q = A x0 or zero), z = Dinv r, p = z; partials r.z, r.r, b.b per bin
template <typename MT, typename VT, int NB>
__global__ void k_pcg_init(int N, const uint8_t *__restrict__ fr, const MT *__restrict__ Dinv,
                           const int *__restrict__ grp, const double *__restrict__ bvec, const VT *__restrict__ q,
                           int use_q, double *__restrict__ r, VT *__restrict__ z, VT *__restrict__ p,
                           double *__restrict__ part3) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (!fr[i]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) { r[3 * i + c] = 0.0; z[3 * i + c] = (VT)0; p[3 * i + c] = (VT)0; }
    part3[3 * (size_t)i] = 0.0; part3[3 * (size_t)i + 1] = 0.0; part3[3 * (size_t)i + 2] = 0.0;
    return;
  }
  double rr[3], bb = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double bv = bvec[3 * i + c];
    bb += bv * bv;
    rr[c] = bv - (use_q ? (double)q[3 * i + c] : 0.0);
    r[3 * i + c] = rr[c];
  }
  const MT *d = Dinv + (size_t)9 * i;
  double rz = 0.0, r2 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double zz = (double)d[3 * c] * rr[0] + (double)d[3 * c + 1] * rr[1] + (double)d[3 * c + 2] * rr[2];
    VT zv = (VT)zz;
    z[3 * i + c] = zv;
    p[3 * i + c] = zv;
    rz += rr[c] * (double)zv;
    r2 += rr[c] * rr[c];
  }
  part3[3 * (size_t)i] = rz;
  part3[3 * (size_t)i + 1] = r2;
  part3[3 * (size_t)i + 2] = bb;
}

// Per-bin sums of part3 (single block, fixed order) into the control block.
template <int NB>
__global__ void k_pcg_init_finish(int N, const uint8_t *__restrict__ fr, const int *__restrict__ grp,
                                  const double *__restrict__ part3, PcgCtl *ctl, double tol2, double ref2_global,
                                  int max_it, int stall) {
  __shared__ double sh[3][NB];
  for (int k = threadIdx.x; k < 3 * NB; k += blockDim.x) sh[k / NB][k % NB] = 0.0;
  __syncthreads();
  // each thread owns a contiguous chunk of nodes; chunks are combined in thread order
  int chunk = (N + blockDim.x - 1) / blockDim.x;
  int lo = threadIdx.x * chunk, hi = min(N, lo + chunk);
  double loc[3][NB];
  for (int v = 0; v < 3; ++v)
    for (int b = 0; b < NB; ++b) loc[v][b] = 0.0;
  for (int i = lo; i < hi; ++i) {
    if (!fr[i]) continue;
    int b = bin_of<NB>(grp, i);
    for (int v = 0; v < 3; ++v) loc[v][b] += part3[3 * (size_t)i + v];
  }
  for (int t = 0; t < (int)blockDim.x; ++t) {
    if ((int)threadIdx.x == t)
      for (int v = 0; v < 3; ++v)
        for (int b = 0; b < NB; ++b) sh[v][b] += loc[v][b];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double rrs = 0.0;
    for (int b = 0; b < NB; ++b) {
      ctl->rz[b] = sh[0][b];
      ctl->rr[b] = sh[1][b];
      rrs += sh[1][b];
      ctl->ref2[b] = NB == 1 ? ref2_global : sh[2][b];
      ctl->active[b] = (NB == 1) ? 1 : (sh[2][b] > 0.0 && sh[1][b] > tol2 * sh[2][b]);
      ctl->alpha[b] = 0.0;
      ctl->beta[b] = 0.0;
      ctl->pq[b] = 0.0;
    }
    for (int b = NB; b < kGroups; ++b) ctl->active[b] = 0;
    ctl->tol2 = tol2;
    ctl->rnorm = sqrt(rrs);
    ctl->rmin = ctl->rnorm;
    ctl->it = 0;
    ctl->it_min = 0;
    ctl->max_it = max_it;
    ctl->stall_window = stall;
    ctl->nbins = NB;
    int any = 0;
    for (int b = 0; b < NB; ++b) any |= ctl->active[b];
    ctl->done = PCG_RUN;
    if (NB == 1 && rrs <= tol2 * ref2_global) ctl->done = PCG_CONVERGED;
    if (NB > 1 && !any) ctl->done = PCG_CONVERGED;
    if (max_it <= 0) ctl->done = PCG_CAPPED;
  }
}

__global__ void k_to_vt_f(const double *__restrict__ a, float *__restrict__ b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_copy_d(const double *__restrict__ a, double *__restrict__ b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

static hipEvent_t take_event(Scene &s) {
  if (s.ev_used >= (int)s.ev_pool.size()) {
    hipEvent_t e;
    hipEventCreate(&e);
    s.ev_pool.push_back(e);
  }
  return s.ev_pool[s.ev_used++];
}

static void harvest_events(Scene &s) {
  for (int k = 0; k + 1 < s.ev_used; k += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s.ev_pool[k], s.ev_pool[k + 1]) == hipSuccess) {
      s.spmv_ms += ms;
      s.spmv_launches += 1;
    }
  }
  s.ev_used = 0;
}

template <typename MT, typename VT, int NB>
static int pcg_run(Scene &s, const double *rhs, double *xsol, double tol, double ref2, int max_iters, bool start,
                   bool resume, int *iters_out, double *rnorm_out) {
  int N = s.N, n3 = 3 * N;
  PcgCtl *ctl = s.pcg_ctl.as<PcgCtl>();
  int nb = blocks_for(N, kBS);
  size_t need = (size_t)nb * 2 * NB * sizeof(double);
  if (s.partial.grow(need < (size_t)3 * N * sizeof(double) ? (size_t)3 * N * sizeof(double) : need)) return BAL_E_OOM;
  double *partial = s.partial.as<double>();
  unsigned *counter = s.counter.as<unsigned>();
  VT *p = static_cast<VT *>(s.pv.p), *q = static_cast<VT *>(s.q.p), *z = static_cast<VT *>(s.z.p);
  double *r = s.r.as<double>();
  const MT *val = static_cast<const MT *>(s.val.p), *D = static_cast<const MT *>(s.Dblk.p);
  const MT *Dinv = static_cast<const MT *>(s.Dinv.p), *pblk = static_cast<const MT *>(s.pair_blk.p);
  const int *grp = s.group.as<int>();
  if (resume) {
    // continue the same Krylov sequence for max_iters more iterations, tolerance off
    PcgCtl *h = s.pin.as<PcgCtl>();
    hipMemcpyAsync(h, ctl, sizeof(PcgCtl), hipMemcpyDeviceToHost, s.stream);
    hipStreamSynchronize(s.stream);
    h->max_it = h->it + max_iters;
    h->tol2 = 0.0;
    h->done = h->done == PCG_BREAKDOWN ? PCG_BREAKDOWN : PCG_RUN;
    h->it_min = h->it;
    hipMemcpyAsync(ctl, h, sizeof(PcgCtl), hipMemcpyHostToDevice, s.stream);
  } else {
    hipMemsetAsync(counter, 0, sizeof(unsigned), s.stream);
    bool use_q = false;
    if (!start) {
      hipMemsetAsync(xsol, 0, n3 * sizeof(double), s.stream);
    } else {
      // x0 given in xsol: q = A x0
      if (sizeof(VT) == 4)
        hipLaunchKernelGGL(k_to_vt_f, dim3(blocks_for(n3, kBS)), dim3(kBS), 0, s.stream, xsol, (float *)p, n3);
      else
        hipLaunchKernelGGL(k_copy_d, dim3(blocks_for(n3, kBS)), dim3(kBS), 0, s.stream, xsol, (double *)p, n3);
      hipLaunchKernelGGL((k_spmv<MT, VT>), dim3(nb), dim3(kBS), 0, s.stream, N, s.row_ptr.as<int>(),
                         s.col_idx.as<int>(), val, D, s.coff_ptr.as<int>(), s.coff_col.as<int>(), s.coff_src.as<int>(),
                         pblk, grp, NB > 1 ? 1 : 0, p, q);
      use_q = true;
    }
    hipLaunchKernelGGL((k_pcg_init<MT, VT, NB>), dim3(nb), dim3(kBS), 0, s.stream, N, s.freev.as<uint8_t>(), Dinv, grp,
                       rhs, q, use_q ? 1 : 0, r, z, p, partial);
    hipLaunchKernelGGL((k_pcg_init_finish<NB>), dim3(1), dim3(kBS), 0, s.stream, N, s.freev.as<uint8_t>(), grp,
                       partial, ctl, tol * tol, ref2, max_iters, NB == 1 ? s.desc.pcg_stall_window : 0);
  }
  const int chunk = 16;
  PcgCtl *h = s.pin.as<PcgCtl>();
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (s.time_kernels) { e0 = take_event(s); hipEventRecord(e0, s.stream); }
      hipLaunchKernelGGL((k_pcg_spmv<MT, VT, NB>), dim3(nb), dim3(kBS), 0, s.stream, N, s.row_ptr.as<int>(),
                         s.col_idx.as<int>(), val, D, s.coff_ptr.as<int>(), s.coff_col.as<int>(), s.coff_src.as<int>(),
                         pblk, grp, p, q, ctl, partial, counter);
      if (s.time_kernels) { e1 = take_event(s); hipEventRecord(e1, s.stream); }
      hipLaunchKernelGGL((k_pcg_update<MT, VT, NB>), dim3(nb), dim3(kBS), 0, s.stream, N, s.freev.as<uint8_t>(), Dinv,
                         grp, p, q, xsol, r, z, ctl, partial, counter);
      hipLaunchKernelGGL((k_pcg_dir<VT, NB>), dim3(nb), dim3(kBS), 0, s.stream, N, grp, z, p, ctl);
    }
    hipMemcpyAsync(h, ctl, sizeof(PcgCtl), hipMemcpyDeviceToHost, s.stream);
    if (hipStreamSynchronize(s.stream) != hipSuccess) return BAL_E_HIP;
    if (s.time_kernels) harvest_events(s);
    if (h->done) break;
  }
  *iters_out = h->it;
  *rnorm_out = h->rnorm;
  return h->done == PCG_BREAKDOWN ? BAL_E_NO_CONVERGENCE : BAL_OK;
}

int pcg_solve(Scene &s, const double *rhs, double *xsol, double rtol_ref, int max_iters, int warm, int resume,
              int *iters_out, double *rel_out) {
  // rtol_ref: ||r|| <= pcg_rtol * rtol_ref is the stopping rule (reading: zero-guess residual)
  double rn = 0.0;
  int rc;
  double ref2 = rtol_ref * rtol_ref;
  if (s.mixed)
    rc = pcg_run<float, float, 1>(s, rhs, xsol, s.desc.pcg_rtol, ref2, max_iters, warm != 0, resume != 0, iters_out, &rn);
  else
    rc = pcg_run<double, double, 1>(s, rhs, xsol, s.desc.pcg_rtol, ref2, max_iters, warm != 0, resume != 0, iters_out,
                                    &rn);
  *rel_out = rtol_ref > 0 ? rn / rtol_ref : rn;
  return rc;
}

int warm_start_solve(Scene &s, const double *rhs, double *xsol, double wtol, int max_iters, int *iters_out) {
  double rn = 0.0;
  if (s.mixed) return pcg_run<float, float, kGroups>(s, rhs, xsol, wtol, 0.0, max_iters, false, false, iters_out, &rn);
  return pcg_run<double, double, kGroups>(s, rhs, xsol, wtol, 0.0, max_iters, false, false, iters_out, &rn);
}

}  // namespace bal
