// Assembly, block SpMV and PCG (Sec. 5.1 sparse storage and SpMV, Sec. 4.2
// block-Jacobi warm start, App. B stopping rules), plus deterministic
// reductions and scans.
//
// Storage.  The static element part is the strictly lower triangle of a 3x3
// block CSR over free nodes (plus a transposed index for the upper half; with
// FP32 blocks also one (operand, block) entry list per row), gathered per
// block from per-tet blocks through a static source list, so assembly and
// SpMV need no atomics and are bit-reproducible.  Contact blocks stay in
// per-pair buffers; per Newton iteration each row gets a sorted list of the
// contact blocks it reads.
// Diagonal blocks (mass + elements + contacts) form the dense block
// diagonal D that also feeds the block-Jacobi preconditioner.
#include <hip/hip_ext.h>

#include <algorithm>

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

// The same sums and counts left on the device in *dst (stream-ordered, no
// synchronisation), so that a caller can read several at once: the partial
// area is reused, which the stream order makes safe.  n <= 0 writes nothing.
template <typename Op>
static void reduce_op_to(Scene &s, const double *in, int n, Op op, double ident, double *dst) {
  if (n <= 0) return;
  int nb = blocks_for(n, kBS);
  if (nb > 1024) nb = 1024;
  double *part = s.red_out.as<double>() + 1;
  hipLaunchKernelGGL(k_reduce_stage<Op>, dim3(nb), dim3(kBS), 0, s.stream, in, (long)n, part, op, ident);
  hipLaunchKernelGGL(k_reduce_stage<Op>, dim3(1), dim3(kBS), 0, s.stream, part, (long)nb, dst, op, ident);
}
void reduce_sum_to(Scene &s, const double *in, int n, double *dst) { reduce_op_to(s, in, n, OpSum(), 0.0, dst); }
void reduce_min_to(Scene &s, const double *in, int n, double *dst) {
  reduce_op_to(s, in, n, OpMin(), INFINITY, dst);
}
void count_less_to(Scene &s, const double *in, int n, double thr, double *dst) {
  if (n <= 0) return;
  int nb = blocks_for(n, kBS);
  if (nb > 1024) nb = 1024;
  double *part = s.red_out.as<double>() + 1;
  hipLaunchKernelGGL(k_count_less, dim3(nb), dim3(kBS), 0, s.stream, in, (long)n, thr, part);
  hipLaunchKernelGGL(k_reduce_stage<OpSum>, dim3(1), dim3(kBS), 0, s.stream, part, (long)nb, dst, OpSum(), 0.0);
}
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

int scan_exclusive_async(Scene &s, const int *in, int *out, int n) {
  if (n <= 0) return 0;
  int nb = blocks_for(n, kBS * kScanItems);
  if (s.scan_tmp.grow((size_t)(nb + 2) * sizeof(int))) return -1;
  int *sums = s.scan_tmp.as<int>() + 1;
  int *total = s.scan_tmp.as<int>();
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kBS), 0, s.stream, in, out, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBS), 0, s.stream, sums, nb, total);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kBS), 0, s.stream, out, n, sums);
  return 0;
}

int scan_exclusive(Scene &s, const int *in, int *out, int n) {
  if (n <= 0) return 0;
  if (scan_exclusive_async(s, in, out, n)) return -1;
  int *total = s.scan_tmp.as<int>();
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

// Each node's sources in ascending order (a deterministic order; the sources
// are distinct).  One wave per node: a list of up to kRankSort entries is
// staged in LDS and every entry goes to its rank (the number of smaller
// sources); a longer list is insertion-sorted by one lane.
constexpr int kRankSort = 256;
__device__ void rank_sort(int lo, int hi, int *__restrict__ key, int *__restrict__ pay, int *sk, int *sp) {
  const int m = hi - lo, lane = threadIdx.x;
  if (m <= 1) return;
  if (m > kRankSort) {
    if (lane == 0)
      for (int a = lo + 1; a < hi; ++a) {
        const int v = key[a], c = pay ? pay[a] : 0;
        int b = a - 1;
        while (b >= lo && key[b] > v) {
          key[b + 1] = key[b];
          if (pay) pay[b + 1] = pay[b];
          --b;
        }
        key[b + 1] = v;
        if (pay) pay[b + 1] = c;
      }
    return;
  }
  for (int e = lane; e < m; e += blockDim.x) {
    sk[e] = key[lo + e];
    if (pay) sp[e] = pay[lo + e];
  }
  __syncthreads();
  for (int e = lane; e < m; e += blockDim.x) {
    const int v = sk[e];
    int r = 0;
    for (int f = 0; f < m; ++f) r += sk[f] < v;
    key[lo + r] = v;
    if (pay) pay[lo + r] = sp[e];
  }
  __syncthreads();
}

// The same for (column, source) pairs in lexicographic order: the entries of
// one column become adjacent, in source order (sources are distinct).
__device__ void rank_sort2(int lo, int hi, int *__restrict__ col, int *__restrict__ src, int *sk, int *sp) {
  const int m = hi - lo, lane = threadIdx.x;
  if (m <= 1) return;
  auto less = [](int c0, int s0, int c1, int s1) { return c0 < c1 || (c0 == c1 && s0 < s1); };
  if (m > kRankSort) {
    if (lane == 0)
      for (int a = lo + 1; a < hi; ++a) {
        const int c = col[a], v = src[a];
        int b = a - 1;
        while (b >= lo && less(c, v, col[b], src[b])) {
          col[b + 1] = col[b];
          src[b + 1] = src[b];
          --b;
        }
        col[b + 1] = c;
        src[b + 1] = v;
      }
    return;
  }
  for (int e = lane; e < m; e += blockDim.x) {
    sk[e] = col[lo + e];
    sp[e] = src[lo + e];
  }
  __syncthreads();
  for (int e = lane; e < m; e += blockDim.x) {
    const int c = sk[e], v = sp[e];
    int r = 0;
    for (int f = 0; f < m; ++f) r += less(sk[f], sp[f], c, v);
    col[lo + r] = c;
    src[lo + r] = v;
  }
  __syncthreads();
}

__global__ void k_contact_sort(const int *__restrict__ dptr, int *__restrict__ dsrc, const int *__restrict__ optr,
                               int *__restrict__ ocol, int *__restrict__ osrc) {
  __shared__ int sk[kRankSort], sp[kRankSort];
  const int i = blockIdx.x;
  rank_sort(dptr[i], dptr[i + 1], dsrc, nullptr, sk, sp);
  rank_sort2(optr[i], optr[i + 1], ocol, osrc, sk, sp);
}

// Merged contact blocks: every row's off-diagonal contact sources with the
// same column are summed (in source order, in FP64, rounded once to the
// storage precision) into one block, so the products read one block per
// distinct (row, column) instead of one per pair that touches it.  A run is
// a maximal stretch of one row's sorted entries with one column: its first
// entry is flagged, the flags are scanned into run indices, and one thread
// per run sums it.
__global__ void k_run_rows(int N, const int *__restrict__ optr, int *__restrict__ head) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && optr[i] < optr[i + 1]) head[optr[i]] = 1;
}

__global__ void k_run_cols(int n, const int *__restrict__ ocol, int *__restrict__ head) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && e > 0 && ocol[e] != ocol[e - 1]) head[e] = 1;
}

template <typename MT>
__global__ void k_merge_runs(int n, const int *__restrict__ head, const int *__restrict__ ridx,
                             const int *__restrict__ ocol, const int *__restrict__ osrc, const MT *__restrict__ pblk,
                             int *__restrict__ mcol, MT *__restrict__ mblk) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n || !head[e]) return;
  double acc[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int f = e;
  do {
    const MT *b = pblk + (size_t)9 * osrc[f];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] += (double)b[k];
    ++f;
  } while (f < n && !head[f]);
  const int m = ridx[e];
  mcol[m] = ocol[e];
#pragma unroll
  for (int k = 0; k < 9; ++k) mblk[(size_t)9 * m + k] = (MT)acc[k];
}

__global__ void k_run_ptr(int N, const int *__restrict__ optr, const int *__restrict__ ridx, int *__restrict__ mptr) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= N) mptr[i] = ridx[optr[i]];
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
    if (N > 0)
      hipLaunchKernelGGL(k_contact_sort, dim3(N), dim3(64), 0, s.stream, s.cdiag_ptr.as<int>(), s.cdiag_src.as<int>(),
                         s.coff_ptr.as<int>(), s.coff_col.as<int>(), s.coff_src.as<int>());
  }
  // merged off-diagonal contact blocks (one per distinct row, column)
  const int nc = s.n_coff;
  if (s.cm_ptr.grow((N + 1) * sizeof(int)) || s.cm_head.grow((size_t)(nc + 1) * sizeof(int)) ||
      s.cm_ridx.grow((size_t)(nc + 1) * sizeof(int)))
    return BAL_E_OOM;
  int *head = s.cm_head.as<int>(), *ridx = s.cm_ridx.as<int>();
  hipMemsetAsync(head, 0, (size_t)(nc + 1) * sizeof(int), s.stream);
  if (nc > 0) {
    hipLaunchKernelGGL(k_run_rows, dim3(blocks_for(N, kBS)), dim3(kBS), 0, s.stream, N, s.coff_ptr.as<int>(), head);
    hipLaunchKernelGGL(k_run_cols, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, s.stream, nc, s.coff_col.as<int>(), head);
  }
  s.n_cm = scan_exclusive(s, head, ridx, nc + 1);
  if (s.n_cm < 0) return BAL_E_OOM;
  hipLaunchKernelGGL(k_run_ptr, dim3(blocks_for(N + 1, kBS)), dim3(kBS), 0, s.stream, N, s.coff_ptr.as<int>(), ridx,
                     s.cm_ptr.as<int>());
  const size_t w = s.mixed ? 4 : 8;
  if (s.cm_col.grow((size_t)(s.n_cm + 1) * sizeof(int)) || s.cm_blk.grow((size_t)(s.n_cm + 1) * 9 * w))
    return BAL_E_OOM;
  if (nc > 0) {
    if (s.mixed)
      hipLaunchKernelGGL((k_merge_runs<float>), dim3(blocks_for(nc, kBS)), dim3(kBS), 0, s.stream, nc, head, ridx,
                         s.coff_col.as<int>(), s.coff_src.as<int>(), s.pair_blk.as<float>(), s.cm_col.as<int>(),
                         s.cm_blk.as<float>());
    else
      hipLaunchKernelGGL((k_merge_runs<double>), dim3(blocks_for(nc, kBS)), dim3(kBS), 0, s.stream, nc, head, ridx,
                         s.coff_col.as<int>(), s.coff_src.as<int>(), s.pair_blk.as<double>(), s.cm_col.as<int>(),
                         s.cm_blk.as<double>());
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
// y_i = D_i v_i + sum_{j<i} L_ij v_j + sum_{m>i} L_mi^T v_m + sum_contact C_ij v_j.
// The element part is stored once, as its strictly lower triangle L (block
// CSR by row, the paper's symmetric storage, Sec. 5.1); row i reads its own
// blocks directly and the blocks of column i through the transposed index
// (row m, block position), so every block is fetched from HBM once and its
// second use is served from cache.  Row-gather only: no atomics, and the
// summation order is fixed.  With masked, blocks whose row and column lie in
// different stiffness groups are skipped (the warm start's domain-decomposed
// product, Sec. 4.2).
// One block row is computed by a group of kG consecutive lanes: lane g takes
// entries g, g + kG, ... of the row's concatenated lower and transposed lists
// (then of its contact list), partial products are summed with shuffles, and
// lane 0 of the group adds D_i v_i and holds the result.
constexpr int kG = 4;

template <typename MT>
struct BsrView {
  const int *rp, *ci;   // lower rows: row_ptr, column
  const MT *val;        // 9 scalars per stored block
  const int *up;        // transposed rows: pointer
  const int2 *ue;       // (row m, block position) of the blocks (m, j), m > j
  const MT *D;          // diagonal blocks
  const int *cp, *cc;   // contact rows: pointer, column of the merged blocks
  const MT *pblk;       // merged contact blocks
  const int2 *ent;      // FP32 storage: per row, lower then transposed entries (operand, block)
  int ndummy;           // index of the closing dummy entry
  int npad;             // index of the pad entries closing ci and ue (and of the spare block)
};

template <typename MT>
static BsrView<MT> bsr_view(const Scene &s) {
  return BsrView<MT>{s.row_ptr.as<int>(), s.col_idx.as<int>(), static_cast<const MT *>(s.val.p), s.up_ptr.as<int>(),
                     s.up_ent.as<int2>(), static_cast<const MT *>(s.Dblk.p), s.cm_ptr.as<int>(),
                     s.cm_col.as<int>(), static_cast<const MT *>(s.cm_blk.p),
                     s.ent.as<int2>(), 2 * s.nnzb, s.nnzb};
}

template <typename MT>
static std::vector<uintptr_t> bsr_sig(const BsrView<MT> &B) {
  return {(uintptr_t)B.rp, (uintptr_t)B.ci, (uintptr_t)B.val, (uintptr_t)B.up, (uintptr_t)B.ue, (uintptr_t)B.D,
          (uintptr_t)B.cp, (uintptr_t)B.cc, (uintptr_t)B.pblk, (uintptr_t)B.ent};
}

// Workgroups are handed to the 8 XCDs round-robin; this permutation gives
// each XCD one contiguous range of tiles, so that the rows sharing a block or
// a vector entry mostly run on the same XCD and meet in its L2.  The grid
// must be a multiple of 8 (spmv_grid).
__device__ __forceinline__ int xcd_tile() {
  return (int)((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3));
}
inline int spmv_grid(int N) {
  int nb = blocks_for((long)N * kG, kBS);
  return (nb + 7) & ~7;
}

// Vector operand of the product: read as stored, or (the CG direction)
// formed as p = z + beta p_old where it is read, in the same expression as
// the row owner uses to store it, so every reader sees identical values.
template <typename VT>
struct VecPlain {
  const VT *__restrict__ v;
  __device__ __forceinline__ void load(int j, VT *w) const {
    w[0] = v[3 * j];
    w[1] = v[3 * j + 1];
    w[2] = v[3 * j + 2];
  }
};
template <typename VT>
struct VecDir {
  const VT *__restrict__ z;
  const VT *__restrict__ p;
  double beta;
  // the two halves of load(): the raw entries (issued before beta is
  // known) and the combination
  __device__ __forceinline__ void raw(int j, VT *zr, VT *pr) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      zr[c] = z[3 * j + c];
      pr[c] = p[3 * j + c];
    }
  }
  __device__ __forceinline__ void form(const VT *zr, const VT *pr, VT *w) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = (VT)((double)zr[c] + beta * (double)pr[c]);
  }
  __device__ __forceinline__ void load(int j, VT *w) const {
    VT zr[3], pr[3];
    raw(j, zr, pr);
    form(zr, pr, w);
  }
};

template <typename MT, typename VT>
__device__ __forceinline__ void blk_mv(const MT *__restrict__ a, const VT *w, VT *acc) {
  acc[0] += (VT)a[0] * w[0] + (VT)a[1] * w[1] + (VT)a[2] * w[2];
  acc[1] += (VT)a[3] * w[0] + (VT)a[4] * w[1] + (VT)a[5] * w[2];
  acc[2] += (VT)a[6] * w[0] + (VT)a[7] * w[1] + (VT)a[8] * w[2];
}
template <typename MT, typename VT>
__device__ __forceinline__ void blk_mtv(const MT *__restrict__ a, const VT *w, VT *acc) {
  acc[0] += (VT)a[0] * w[0] + (VT)a[3] * w[1] + (VT)a[6] * w[2];
  acc[1] += (VT)a[1] * w[0] + (VT)a[4] * w[1] + (VT)a[7] * w[2];
  acc[2] += (VT)a[2] * w[0] + (VT)a[5] * w[1] + (VT)a[8] * w[2];
}

// Row i of the product into acc (complete on lane g == 0, which also
// returns the row's own operand entries in own).  The row's own blocks and
// the transposed blocks of its column form one list of nl + nu entries; a
// lane takes entries g, g + kG, ... and handles kU of them per pass: first
// all their indices, then all their blocks and operand entries, then the
// arithmetic, so that a typical row costs two rounds of memory latency.
// `pre` runs (on every thread of the block) after the first pass's index
// and block loads and the diagonal block load are issued and before any
// operand entry is read; it returns false to abandon the product.  (The PCG
// product launch has its own copy of this loop, which also issues the first
// pass's raw operand entries before its scalars are known.)
constexpr int kU = 3;
// entries per pass of the PCG product's branch-free FP64 walk: its batch's
// loads are all in flight together, and two per pass keep the registers
// within three waves per SIMD (three per pass need 204)
constexpr int kUSplit = 2;

template <typename MT, int U = kU>
struct RowBatch {
  int j[U], k[U];
  bool tr[U], on[U];
  MT a[U][9];
};

template <typename MT>
__device__ __forceinline__ void row_fetch(int i, int t, int l0, int nl, int u0, int nt, const BsrView<MT> &B,
                                          RowBatch<MT> &rb) {
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int tt = t + u * kG;
    rb.on[u] = tt < nt;
    rb.tr[u] = tt >= nl;
    rb.j[u] = i;
    rb.k[u] = 0;
    if (rb.on[u]) {
      if (!rb.tr[u]) {
        rb.k[u] = l0 + tt;
        rb.j[u] = B.ci[rb.k[u]];
      } else {
        const int2 e = B.ue[u0 + tt - nl];
        rb.j[u] = e.x;
        rb.k[u] = e.y;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u)
    if (rb.on[u]) {
      const MT *src = B.val + (size_t)9 * rb.k[u];
#pragma unroll
      for (int c = 0; c < 9; ++c) rb.a[u][c] = src[c];
    }
}

// FP32 storage walks the row's single entry list in branch-free batches:
// lanes past the row's end read the dummy entry and drop their product by a
// select, so the compiler keeps every batch's loads in flight together
// (measured: the 128^3-grid product 246 -> 238 us, a PCG iteration on the
// stacked boxes 15.8 -> 15.3 us).  The plain and warm-start products with
// FP64 storage keep the predicated walk of the lower and transposed lists,
// whose 4-byte lower-entry index matters more there than the branches (the
// single list made the grid product 392 -> 403 us); the FP64 PCG product
// walks the two lists without branches (row_fetch_split).
template <typename MT>
constexpr bool kUnifiedWalk = sizeof(MT) == 4;

template <typename MT, int U>
__device__ __forceinline__ void row_fetch_unified(int t, int ep, int nl, int nt, const BsrView<MT> &B,
                                                  RowBatch<MT, U> &rb) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int tt = t + u * kG;
    rb.on[u] = tt < nt;
    rb.tr[u] = tt >= nl;
    const int2 e = B.ent[rb.on[u] ? ep + tt : B.ndummy];
    rb.j[u] = e.x;
    rb.k[u] = e.y;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const MT *src = B.val + (size_t)9 * rb.k[u];
#pragma unroll
    for (int c = 0; c < 9; ++c) rb.a[u][c] = src[c];
  }
}

// FP64 storage, branch-free: each of a lane's kU entries reads both of its
// candidate index entries, the lower list's (l0 + tt while tt < nl, else
// the pad entry) and the transposed list's (u0 + tt - nl while nl <= tt <
// nt, else the pad entry), and keeps the one its position selects; past
// the row's end that is the transposed pad (operand 0, the spare block),
// whose product the caller drops by a select.  With no branch among them,
// a batch's index loads, then its block loads, stay in flight together
// (the predicated walk waited for every earlier load at each branch join).
template <typename MT, int U>
__device__ __forceinline__ void row_fetch_split(int t, int l0, int nl, int u0, int nt, const BsrView<MT> &B,
                                                RowBatch<MT, U> &rb) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int tt = t + u * kG;
    rb.on[u] = tt < nt;
    rb.tr[u] = tt >= nl;
    const int kl = tt < nl ? l0 + tt : B.npad;
    const int ku = rb.tr[u] && rb.on[u] ? u0 + tt - nl : B.npad;
    const int cj = B.ci[kl];
    const int2 e = B.ue[ku];
    rb.j[u] = rb.tr[u] ? e.x : cj;
    rb.k[u] = rb.tr[u] ? e.y : kl;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const MT *src = B.val + (size_t)9 * rb.k[u];
#pragma unroll
    for (int c = 0; c < 9; ++c) rb.a[u][c] = src[c];
  }
}

// acc += A w (tr false) or A^T w (tr true) when on; nothing otherwise
template <typename MT, typename VT>
__device__ __forceinline__ void blk_sel(const MT *a, const VT *w, bool tr, bool on, VT *acc) {
  const VT d0 = (VT)a[0] * w[0] + (VT)a[1] * w[1] + (VT)a[2] * w[2];
  const VT d1 = (VT)a[3] * w[0] + (VT)a[4] * w[1] + (VT)a[5] * w[2];
  const VT d2 = (VT)a[6] * w[0] + (VT)a[7] * w[1] + (VT)a[8] * w[2];
  const VT t0 = (VT)a[0] * w[0] + (VT)a[3] * w[1] + (VT)a[6] * w[2];
  const VT t1 = (VT)a[1] * w[0] + (VT)a[4] * w[1] + (VT)a[7] * w[2];
  const VT t2 = (VT)a[2] * w[0] + (VT)a[5] * w[1] + (VT)a[8] * w[2];
  acc[0] += on ? (tr ? t0 : d0) : (VT)0;
  acc[1] += on ? (tr ? t1 : d1) : (VT)0;
  acc[2] += on ? (tr ? t2 : d2) : (VT)0;
}

// The same with the block's transpose taken by selecting its elements
// (FP64 storage: one product instead of two keeps the registers of a
// batch's blocks and operands, all in flight together, within three waves
// per SIMD)
template <typename MT, typename VT>
__device__ __forceinline__ void blk_sel_t(const MT *a, const VT *w, bool tr, bool on, VT *acc) {
  MT b[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) b[3 * r + c] = r == c ? a[3 * r + c] : (tr ? a[3 * c + r] : a[3 * r + c]);
  const VT d0 = (VT)b[0] * w[0] + (VT)b[1] * w[1] + (VT)b[2] * w[2];
  const VT d1 = (VT)b[3] * w[0] + (VT)b[4] * w[1] + (VT)b[5] * w[2];
  const VT d2 = (VT)b[6] * w[0] + (VT)b[7] * w[1] + (VT)b[8] * w[2];
  acc[0] += on ? d0 : (VT)0;
  acc[1] += on ? d1 : (VT)0;
  acc[2] += on ? d2 : (VT)0;
}

// The row's merged contact blocks (one per distinct column, stored in row
// order), kC entries per lane per pass: all their indices and blocks, then
// all operand entries, then the arithmetic, so that a row with many
// contacts costs a few rounds of memory latency rather than two per entry.
// Lanes past the row's end reread a valid entry and drop it.
constexpr int kC = 4;
template <typename MT, typename VT, bool MASK, typename F>
__device__ __forceinline__ void contact_rows(int c0, int c1, int g, const BsrView<MT> &B, const int *__restrict__ grp,
                                             int gi, const F &v, VT *acc) {
  for (int c = c0 + g; c < c1; c += kC * kG) {
    int j[kC];
    const MT *a[kC];
    bool on[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int cu = c + u * kG;
      on[u] = cu < c1;
      const int ce = on[u] ? cu : c;
      j[u] = B.cc[ce];
      a[u] = B.pblk + (size_t)9 * ce;
    }
    MT blk[kC][9];
    VT w[kC][3];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
#pragma unroll
      for (int e = 0; e < 9; ++e) blk[u][e] = a[u][e];
      v.load(j[u], w[u]);
    }
#pragma unroll
    for (int u = 0; u < kC; ++u) blk_sel<MT, VT>(blk[u], w[u], false, on[u] && (!MASK || grp[j[u]] == gi), acc);
  }
}

template <typename MT, typename VT, bool MASK, typename F, typename Pre>
__device__ __forceinline__ bool spmv_row_pre(int i, int g, const BsrView<MT> &B, const int *__restrict__ grp, F &v,
                                             Pre &&pre, VT *acc, VT *own) {
  acc[0] = acc[1] = acc[2] = (VT)0;
  int l0 = 0, nl = 0, u0 = 0, nt = 0, c0 = 0, c1 = 0, gi = 0;
  RowBatch<MT> rb;
  MT dblk[9];
  if (i >= 0) {
    l0 = B.rp[i];
    nl = B.rp[i + 1] - l0;
    u0 = B.up[i];
    nt = nl + B.up[i + 1] - u0;
    c0 = B.cp[i];
    c1 = B.cp[i + 1];
    if (MASK) gi = grp[i];
    if constexpr (kUnifiedWalk<MT>) row_fetch_unified<MT, kU>(g, l0 + u0, nl, nt, B, rb);
    else row_fetch<MT>(i, g, l0, nl, u0, nt, B, rb);
    if (g == 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) dblk[c] = B.D[(size_t)9 * i + c];
    }
  }
  if (!pre()) return false;
  if (i >= 0) {
    for (int t = g;;) {
      VT w[kU][3];
      if constexpr (kUnifiedWalk<MT>) {
#pragma unroll
        for (int u = 0; u < kU; ++u) v.load(rb.j[u], w[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u)
          blk_sel<MT, VT>(rb.a[u], w[u], rb.tr[u], rb.on[u] && (!MASK || grp[rb.j[u]] == gi), acc);
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (rb.on[u]) v.load(rb.j[u], w[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (rb.on[u] && (!MASK || grp[rb.j[u]] == gi)) {
            if (rb.tr[u]) blk_mtv<MT, VT>(rb.a[u], w[u], acc);
            else blk_mv<MT, VT>(rb.a[u], w[u], acc);
          }
        }
      }
      t += kU * kG;
      if (t >= nt) break;
      if constexpr (kUnifiedWalk<MT>) row_fetch_unified<MT, kU>(t, l0 + u0, nl, nt, B, rb);
      else row_fetch<MT>(i, t, l0, nl, u0, nt, B, rb);
    }
    if constexpr (kUnifiedWalk<MT>) {
      contact_rows<MT, VT, MASK>(c0, c1, g, B, grp, gi, v, acc);
    } else {
      // FP64 storage: the batched walk changed the plain product's code
      // enough to cost the 128^3-grid product 392 -> 421 us
      for (int c = c0 + g; c < c1; c += kG) {
        const int j = B.cc[c];
        VT w0[3];
        v.load(j, w0);
        if (!MASK || grp[j] == gi) blk_mv<MT, VT>(B.pblk + (size_t)9 * c, w0, acc);
      }
    }
  }
#pragma unroll
  for (int o = kG / 2; o > 0; o >>= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], o, kG);
  if (i >= 0 && g == 0) {
    v.load(i, own);
    blk_mv<MT, VT>(dblk, own, acc);
  }
  return true;
}

template <typename MT, typename VT, bool MASK, typename F>
__device__ __forceinline__ void spmv_row(int i, int g, const BsrView<MT> &B, const int *__restrict__ grp, F v,
                                         VT *acc, VT *own) {
  spmv_row_pre<MT, VT, MASK>(i, g, B, grp, v, [] { return true; }, acc, own);
}

template <typename MT, typename VT, bool MASK>
__global__ __launch_bounds__(kBS) void k_spmv(int N, BsrView<MT> B, const int *__restrict__ grp,
                                              const VT *__restrict__ v, VT *__restrict__ out) {
  long t = (long)xcd_tile() * blockDim.x + threadIdx.x;
  int i = (int)(t / kG), g = (int)(t % kG);
  VT acc[3], own[3];
  spmv_row<MT, VT, MASK>(i < N ? i : -1, g, B, grp, VecPlain<VT>{v}, acc, own);
  if (i < N && g == 0) {
    out[3 * i] = acc[0];
    out[3 * i + 1] = acc[1];
    out[3 * i + 2] = acc[2];
  }
}

template <typename MT, typename VT>
static void launch_spmv_t(Scene &s, const void *vin, void *vout, int masked) {
  dim3 g(spmv_grid(s.N)), b(kBS);
  if (masked)
    hipLaunchKernelGGL((k_spmv<MT, VT, true>), g, b, 0, s.stream, s.N, bsr_view<MT>(s), s.group.as<int>(),
                       static_cast<const VT *>(vin), static_cast<VT *>(vout));
  else
    hipLaunchKernelGGL((k_spmv<MT, VT, false>), g, b, 0, s.stream, s.N, bsr_view<MT>(s), s.group.as<int>(),
                       static_cast<const VT *>(vin), static_cast<VT *>(vout));
}

void launch_spmv(Scene &s, const void *vin, void *vout, int masked) {
  if (s.mixed)
    launch_spmv_t<float, float>(s, vin, vout, masked);
  else
    launch_spmv_t<double, double>(s, vin, vout, masked);
}

double spmv_bytes(const Scene &s) {
  // the paper's symmetric storage: each off-diagonal pair of blocks once
  double w = s.mixed ? 4.0 : 8.0;
  double nL = (double)s.nnzb, nC = 0.5 * (double)s.n_cm;
  double N = (double)s.N;
  return (nL + nC) * (9.0 * w + 4.0) + N * 9.0 * w + 4.0 * N + 3.0 * N * w + 3.0 * N * w;
}

double cg_product_bytes(const Scene &s) {
  // the PCG product launch also reads z and writes the new direction p
  double w = s.mixed ? 4.0 : 8.0;
  return spmv_bytes(s) + 6.0 * (double)s.N * w;
}

// ----------------------------------------------------------------- PCG
// No kernel here fences or counts tickets: a kernel writes per-block
// partial sums, and the next kernel (a kernel boundary orders the writes)
// re-sums them in a fixed order, so every scalar is bit-reproducible.
//
// Global solve, two launches per iteration k:
//   cg_dir_spmv  state after iteration k from the previous partials
//                (beta_k = rz_k / rz_{k-1}, stopping rules; block 0 writes
//                it), p_k = z + beta_k p_{k-1} formed where it is read,
//                q = A p_k, partial p_k.q
//   cg_update    alpha = rz_k / sum(p.q) in every block; x += alpha p_k,
//                r -= alpha q, z = D^{-1} r, partials r.z, r.r
// The state after iteration k lives in slot k & 1 (the host passes k), so
// the slot being written is never the slot being read.
//
// Warm start (per stiffness group, 64 bins): per-block per-bin partials;
// the p.q sums are formed by each update block for the bins it holds, the
// r.z and r.r sums by one block per bin.
template <int NB>
__device__ __forceinline__ int bin_of(const int *grp, int i) {
  if (NB == 1) return 0;
  int b = grp[i] + kGroupOffset;
  return b < 0 ? 0 : (b >= NB ? NB - 1 : b);
}

// Per-bin sums of one value per lane inside a wave: lanes are grouped by bin
// with ballots (one pass per distinct bin in the wave, usually one or two),
// each group reduced with a fixed shuffle tree.  Deterministic.
template <int NB>
__device__ __forceinline__ void wave_bin_sums(int bin, double v, double *wave_out /* [NB], zeroed */) {
  const int lane = threadIdx.x & 63;
  bool pending = bin >= 0;
  while (__ballot(pending) != 0ull) {
    unsigned long long act = __ballot(pending);
    int leader = __ffsll((long long)act) - 1;
    int b = __shfl(bin, leader, 64);
    bool mine = pending && bin == b;
    double x = mine ? v : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) wave_out[b] = x;
    if (mine) pending = false;
  }
}

// Block per-bin sums written bin-major, part[(v * NB + bin) * nbk + blk] with
// nbk = gridDim.x, so that one bin's partials are contiguous.
template <int NB, int NV>
__device__ void block_partials(int bin, const double *vals, double *part, int blk) {
  constexpr int W = kBS / 64;
  __shared__ double wsum[W][NV][NB];
  const int w = threadIdx.x >> 6;
  if (NB > 1) {
    for (int k = threadIdx.x; k < W * NV * NB; k += blockDim.x) (&wsum[0][0][0])[k] = 0.0;
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double x = bin >= 0 ? vals[v] : 0.0;
    if (NB == 1) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
      if ((threadIdx.x & 63) == 0) wsum[w][v][0] = x;
    } else {
      wave_bin_sums<NB>(bin, x, wsum[w][v]);
    }
  }
  __syncthreads();
  const int nbk = gridDim.x;
  for (int k = threadIdx.x; k < NV * NB; k += blockDim.x) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) acc += (&wsum[q][0][0])[k];
    part[(size_t)k * nbk + blk] = acc;
  }
}

// tot[v][b] = sum over nbk blocks of part[(v * NB + b) * nbk + block]; one
// wave per entry, lanes striding over blocks, fixed shuffle tree.  All
// threads of the calling block see the result (after the barrier).
template <int NB, int NV>
__device__ void sum_blocks(const double *part, int nbk, double (*tot)[NB]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = w; k < NV * NB; k += nw) {
    int v = k / NB, b = k % NB;
    double acc = 0.0;
    for (int j = lane; j < nbk; j += 64) acc += part[(size_t)k * nbk + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) tot[v][b] = acc;
  }
  __syncthreads();
}

struct CgSlot {
  double rz, rr, rmin, rnorm;
  int it, it_min, done, pad;
};
struct CgCtl {
  CgSlot slot[2];
  double tol2, ref2;
  int max_it, stall;
  int stop;  // raised with the final state: every later launch exits at once
  int pad;
};
// pinned-buffer offset of the pipelined chunks' control-block copies
constexpr size_t kPinPipe = 32768;
static_assert(kPinPipe + 2 * sizeof(CgCtl) <= 65536, "pinned scratch is 64 KiB");
struct WarmCtl {
  double rz[kGroups], alpha[kGroups], beta[kGroups], rr[kGroups], ref2[kGroups];
  int active[kGroups];
  double tol2, rnorm;
  int it, max_it, done, pad;
};

// ---- shared pieces
// x += al p ; r -= al q ; z = Dinv r ; partial r.z and r.r
template <typename MT, typename VT, int NB>
__device__ __forceinline__ void update_partial(int N, int i, const uint8_t *fr, const MT *Dinv, const int *grp,
                                               const VT *p, const VT *q, double *x, double *r, VT *z,
                                               const double *alpha_bins, double *part) {
  double vals[2] = {0.0, 0.0};
  int bin = -1;
  if (i < N && fr[i]) {
    int b = bin_of<NB>(grp, i);
    bin = b;
    double al = alpha_bins[b];
    double rr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] += al * (double)p[3 * i + c];
      rr[c] = r[3 * i + c] - al * (double)q[3 * i + c];
      r[3 * i + c] = rr[c];
    }
    const MT *d = Dinv + (size_t)9 * i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double zz = (double)d[3 * c] * rr[0] + (double)d[3 * c + 1] * rr[1] + (double)d[3 * c + 2] * rr[2];
      VT zv = (VT)zz;
      z[3 * i + c] = zv;
      vals[0] += rr[c] * (double)zv;
      vals[1] += rr[c] * rr[c];
    }
  }
  block_partials<NB, 2>(bin, vals, part, blockIdx.x);
}

// ---- global solve
// Sums of up to three partial arrays with every thread of the block, in two
// halves so that a kernel can issue the loads early: sums_load issues the
// first round (four per thread per array), sums_finish adds them in a fixed
// order (and any further rounds), then a fixed shuffle tree per wave and the
// waves in order.  The partial arrays here hold a few hundred entries, so one
// round of loads covers them.
template <int NS>
__device__ __forceinline__ void sums_load(const double *const *src, const int *n, double (&v)[NS][4]) {
#pragma unroll
  for (int m = 0; m < NS; ++m)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = threadIdx.x + u * kBS;
      v[m][u] = j < n[m] ? src[m][j] : 0.0;
    }
}

template <int NS>
__device__ void sums_finish(const double *const *src, const int *n, const double (&v)[NS][4], double *out) {
  __shared__ double sh[NS][kBS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    acc[m] = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[m] += v[m][u];
    for (int j0 = threadIdx.x + 4 * kBS; j0 < n[m]; j0 += 4 * kBS) {
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = j0 + u * kBS < n[m] ? src[m][j0 + u * kBS] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[m] += x[u];
    }
  }
#pragma unroll
  for (int m = 0; m < NS; ++m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[m] += __shfl_down(acc[m], o, 64);
    if (lane == 0) sh[m][w] = acc[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBS / 64; ++q) t += sh[m][q];
    out[m] = t;
  }
  __syncthreads();  // sh is reused by the next call
}

template <int NS>
__device__ void block_sums(const double *const *src, const int *n, double *out) {
  double v[NS][4];
  sums_load<NS>(src, n, v);
  sums_finish<NS>(src, n, v, out);
}

// Iteration k, first launch.  Unless this is the first iteration (previous
// slot marked it = -1, state 0 written by the initialisation), forms the
// state after iteration k from the previous partials and applies the
// stopping rules (App. B: relative residual, stagnation over the window, cap;
// p.q <= 0 is a breakdown); block 0 stores it in slot k & 1.  Then
// p_k = z + beta_k p_{k-1} (the row owner stores it), q = A p_k and the
// partial p_k.q.  The row's extents are loaded with the control block, then
// the previous partials, then the first pass's indices, blocks and raw z and
// p_{k-1} entries; beta is formed while these are in flight.  p is
// double-buffered (p_new never aliases p_old) and so is the p.q partial
// array (this launch reads one and writes the other).
template <typename MT, typename VT>
__global__ __launch_bounds__(kBS) void k_cg_dir_spmv(int N, int k, BsrView<MT> B, const VT *__restrict__ z,
                                                     const VT *__restrict__ p_old, VT *__restrict__ p_new,
                                                     VT *__restrict__ q, CgCtl *ctl, const double *part, int nb,
                                                     const double *part_pq_prev, double *part_pq) {
  const int tile = xcd_tile();
  const long t = (long)tile * blockDim.x + threadIdx.x;
  const int i = t / kG < N ? (int)(t / kG) : -1, g = (int)(t % kG);
  // The row's extents depend on nothing in the control block, so their
  // loads are issued with the control block's, before the first wait.  One
  // exit test covers every control word, so no load waits for another.
  // Lanes past the last row read row 0's extents and ignore them: with no
  // branch there is no copy of a loaded register that would wait for it.
  const int ir = i >= 0 ? i : 0;
  const int rp0 = B.rp[ir], rp1 = B.rp[ir + 1], up0 = B.up[ir], up1 = B.up[ir + 1];
  const int c0 = i >= 0 ? B.cp[ir] : 0, c1 = i >= 0 ? B.cp[ir + 1] : 0;
  const CgSlot prev = ctl->slot[(k - 1) & 1];
  const int stop = ctl->stop, cur_done = ctl->slot[k & 1].done;
  const bool first = prev.it < 0;
  if (stop | (first ? cur_done : prev.done)) return;
  const int l0 = rp0, nl = rp1 - rp0, u0 = up0, nt = nl + up1 - up0;
  const double *src[3] = {part, part + nb, part_pq_prev};
  const int cnt[3] = {nb, nb, (int)gridDim.x};
  double pv[3][4];
  if (!first) sums_load<3>(src, cnt, pv);
  VecDir<VT> dir{z, first ? z : p_old, 0.0};  // p_0 = z_0: beta = 0 must not meet an unset buffer
  VT acc[3] = {(VT)0, (VT)0, (VT)0};
  constexpr int U = kUnifiedWalk<MT> ? kU : kUSplit;
  RowBatch<MT, U> rb;
  VT zr[U][3], pr[U][3];
  if (i >= 0) {
    if constexpr (kUnifiedWalk<MT>) row_fetch_unified<MT, U>(g, l0 + u0, nl, nt, B, rb);
    else row_fetch_split<MT, U>(g, l0, nl, u0, nt, B, rb);
#pragma unroll
    for (int u = 0; u < U; ++u) dir.raw(rb.j[u], zr[u], pr[u]);
  }
  if (!first) {
    // the state after iteration k and beta_k
    double tv[3];
    sums_finish<3>(src, cnt, pv, tv);
    const double rz = tv[0], rr = tv[1], pq = tv[2];
    const int it = prev.it + 1;
    const double rn = sqrt(rr);
    int done = PCG_RUN;
    double rmin = prev.rmin;
    int it_min = prev.it_min;
    if (!(pq > 0.0)) done = PCG_BREAKDOWN;
    else if (rr <= ctl->tol2 * ctl->ref2) done = PCG_CONVERGED;
    if (rn < rmin) { rmin = rn; it_min = it; }
    if (!done && ctl->stall > 0 && it - it_min >= ctl->stall) done = PCG_STALLED;
    if (!done && it >= ctl->max_it) done = PCG_CAPPED;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      CgSlot &o = ctl->slot[k & 1];
      o.rz = rz;
      o.rr = rr;
      o.rmin = rmin;
      o.rnorm = rn;
      o.it = it;
      o.it_min = it_min;
      o.done = done;
      if (done) ctl->stop = 1;  // later launches exit at once
    }
    if (done) return;
    dir.beta = prev.rz != 0.0 ? rz / prev.rz : 0.0;
  }
  if (i >= 0) {
    for (int tt = g;;) {
      VT w[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) dir.form(zr[u], pr[u], w[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (kUnifiedWalk<MT>) blk_sel<MT, VT>(rb.a[u], w[u], rb.tr[u], rb.on[u], acc);
        else blk_sel_t<MT, VT>(rb.a[u], w[u], rb.tr[u], rb.on[u], acc);
      }
      tt += U * kG;
      if (tt >= nt) break;
      if constexpr (kUnifiedWalk<MT>) row_fetch_unified<MT, U>(tt, l0 + u0, nl, nt, B, rb);
      else row_fetch_split<MT, U>(tt, l0, nl, u0, nt, B, rb);
#pragma unroll
      for (int u = 0; u < U; ++u) dir.raw(rb.j[u], zr[u], pr[u]);
    }
    contact_rows<MT, VT, false>(c0, c1, g, B, nullptr, 0, dir, acc);
  }
#pragma unroll
  for (int o = kG / 2; o > 0; o >>= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], o, kG);
  double vals[1] = {0.0};
  int bin = -1;
  if (i >= 0 && g == 0) {
    // the diagonal block and the row's own operand entries are read here,
    // in one round, rather than held in registers through the walk
    VT own[3];
    MT dblk[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) dblk[c] = B.D[(size_t)9 * i + c];
    dir.load(i, own);
    blk_mv<MT, VT>(dblk, own, acc);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p_new[3 * i + c] = own[c];
      q[3 * i + c] = acc[c];
    }
    bin = 0;
    vals[0] = (double)own[0] * (double)acc[0] + (double)own[1] * (double)acc[1] + (double)own[2] * (double)acc[2];
  }
  block_partials<1, 1>(bin, vals, part_pq, tile);
}

// Iteration k, second launch: alpha = rz_k / sum(p.q); x += alpha p,
// r -= alpha q, z = D^{-1} r, partials r.z and r.r.
template <typename MT, typename VT>
__global__ __launch_bounds__(kBS) void k_cg_update(int N, int k, const uint8_t *__restrict__ fr,
                                                   const MT *__restrict__ Dinv, const VT *__restrict__ p,
                                                   const VT *__restrict__ q, double *__restrict__ x,
                                                   double *__restrict__ r, VT *__restrict__ z, const CgCtl *ctl,
                                                   const double *part_pq, int nb_pq, double *part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // the node's operands (whether or not the node is free) are loaded with
  // its free flag and the control block, and are in flight while the p.q
  // partials are summed
  const bool in = i < N;
  double pv[3] = {0.0, 0.0, 0.0}, qv[3] = {0.0, 0.0, 0.0}, xv[3] = {0.0, 0.0, 0.0}, rv[3] = {0.0, 0.0, 0.0};
  MT d[9];
  bool act = false;
  if (in) {
    act = fr[i] != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv[c] = (double)p[3 * i + c];
      qv[c] = (double)q[3 * i + c];
      xv[c] = x[3 * i + c];
      rv[c] = r[3 * i + c];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) d[c] = Dinv[(size_t)9 * i + c];
  }
  const int stop = ctl->stop, done = ctl->slot[k & 1].done;
  const double rz = ctl->slot[k & 1].rz;
  if (stop || done) return;
  double pq;
  const double *src[1] = {part_pq};
  const int cnt[1] = {nb_pq};
  block_sums<1>(src, cnt, &pq);
  const double al = pq > 0.0 ? rz / pq : 0.0;  // a breakdown is recorded by the next launch
  double vals[2] = {0.0, 0.0};
  int bin = -1;
  if (act) {
    bin = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] = xv[c] + al * pv[c];
      rv[c] = rv[c] - al * qv[c];
      r[3 * i + c] = rv[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double zz = (double)d[3 * c] * rv[0] + (double)d[3 * c + 1] * rv[1] + (double)d[3 * c + 2] * rv[2];
      VT zv = (VT)zz;
      z[3 * i + c] = zv;
      vals[0] += rv[c] * (double)zv;
      vals[1] += rv[c] * rv[c];
    }
  }
  block_partials<1, 2>(bin, vals, part, blockIdx.x);
}

// ---- warm start (per-group bins), three launches per iteration
//   k_w_dir_spmv  the stop decision from the per-bin state of the previous
//                 iteration (every block, same inputs; block 0 records it),
//                 then p = z + beta_bin p_old formed where it is read (the
//                 row owner stores p; p is double-buffered), q = the
//                 group-masked product and the per-bin partials p.q
//   k_w_update    alpha of every bin present in the block, summed from that
//                 bin's p.q partials; x += alpha p, r -= alpha q,
//                 z = D^{-1} r, per-bin partials r.z and r.r
//   k_w_beta      one block per bin: beta, rz, rr and the bin's tolerance
//                 test; block 0 also counts the iteration
template <typename MT, typename VT>
__global__ __launch_bounds__(kBS) void k_w_dir_spmv(int N, BsrView<MT> B, const int *__restrict__ grp,
                                                    const VT *__restrict__ z, const VT *__restrict__ p_old,
                                                    VT *__restrict__ p_new, VT *__restrict__ q, WarmCtl *ctl,
                                                    double *part_pq) {
  if (ctl->done) return;
  int any = 0;
  for (int b = 0; b < kGroups; ++b) any |= ctl->active[b];
  const int it = ctl->it;
  const int done = !any ? PCG_CONVERGED : (it >= ctl->max_it ? PCG_CAPPED : PCG_RUN);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double rr = 0.0;
    for (int b = 0; b < kGroups; ++b) rr += ctl->rr[b];
    ctl->rnorm = sqrt(rr);
    if (done) ctl->done = done;
  }
  if (done) return;
  const int tile = xcd_tile();
  const long t = (long)tile * blockDim.x + threadIdx.x;
  const int i = t / kG < N ? (int)(t / kG) : -1, g = (int)(t % kG);
  // p_0 = z_0: beta = 0 must not meet an unset buffer
  const bool first = it == 0;
  VecDir<VT> dir{z, first ? z : p_old, (i >= 0 && !first) ? ctl->beta[bin_of<kGroups>(grp, i)] : 0.0};
  double vals[1] = {0.0};
  int bin = -1;
  VT acc[3], own[3];
  spmv_row<MT, VT, true>(i, g, B, grp, dir, acc, own);
  if (i >= 0 && g == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p_new[3 * i + c] = own[c];
      q[3 * i + c] = acc[c];
    }
    bin = bin_of<kGroups>(grp, i);
    vals[0] = (double)own[0] * (double)acc[0] + (double)own[1] * (double)acc[1] + (double)own[2] * (double)acc[2];
  }
  block_partials<kGroups, 1>(bin, vals, part_pq, tile);
}

template <typename MT, typename VT>
__global__ __launch_bounds__(kBS) void k_w_update(int N, int nbs, const uint8_t *__restrict__ fr,
                                                  const MT *__restrict__ Dinv, const int *__restrict__ grp,
                                                  const VT *__restrict__ p, const VT *__restrict__ q,
                                                  double *__restrict__ x, double *__restrict__ r, VT *__restrict__ z,
                                                  WarmCtl *ctl, const double *part_pq, double *part) {
  if (ctl->done) return;
  __shared__ unsigned present[kGroups / 32];
  __shared__ double alpha_sh[kGroups];
  if (threadIdx.x < kGroups / 32) present[threadIdx.x] = 0u;
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && fr[i]) {
    const int b = bin_of<kGroups>(grp, i);
    atomicOr(&present[b >> 5], 1u << (b & 31));
  }
  __syncthreads();
  // alpha of each bin present here, from that bin's p.q partials (the same
  // sums, in the same order, in every block that holds the bin)
  for (int w = 0; w < kGroups / 32; ++w) {
    unsigned m = present[w];
    while (m) {
      const int b = 32 * w + __builtin_ctz(m);
      m &= m - 1;
      const double *src[1] = {part_pq + (size_t)b * nbs};
      double pq;
      block_sums<1>(src, &nbs, &pq);
      if (threadIdx.x == 0) {
        const bool act = ctl->active[b] != 0, ok = pq > 0.0;
        alpha_sh[b] = act && ok ? ctl->rz[b] / pq : 0.0;
        if (act && !ok) ctl->active[b] = 0;  // breakdown: the bin stops (same value from every block)
      }
    }
  }
  __syncthreads();
  update_partial<MT, VT, kGroups>(N, i, fr, Dinv, grp, p, q, x, r, z, alpha_sh, part);
}

// One block per group bin: the sum of that bin's partials (bin-major
// layout, contiguous), reduced in a fixed order and seen by every thread.
__device__ double bin_sum(const double *part, int nbk, int k) {
  const double *src[1] = {part + (size_t)k * nbk};
  double out;
  block_sums<1>(src, &nbk, &out);
  return out;
}

__global__ void k_w_beta(int nbk, WarmCtl *ctl, const double *part) {
  const int b = blockIdx.x;
  if (ctl->done) return;
  if (b == 0 && threadIdx.x == 0) ctl->it += 1;  // read by the next launch only
  if (!ctl->active[b]) {
    if (threadIdx.x == 0) ctl->beta[b] = 0.0;
    return;
  }
  double rz = bin_sum(part, nbk, b), rr = bin_sum(part, nbk, kGroups + b);
  if (threadIdx.x == 0) {
    ctl->beta[b] = ctl->rz[b] != 0.0 ? rz / ctl->rz[b] : 0.0;
    ctl->rz[b] = rz;
    ctl->rr[b] = rr;
    if (rr <= ctl->tol2 * ctl->ref2[b]) ctl->active[b] = 0;
  }
}

// ---- initialisation: r = b - q (q = A x0 or zero), z = Dinv r, p = z;
// partials r.z, r.r, b.b per bin; a single block then fills the control block.
template <typename MT, typename VT, int NB>
__global__ __launch_bounds__(kBS) void k_pcg_init(int N, const uint8_t *__restrict__ fr, const MT *__restrict__ Dinv,
                                                  const int *__restrict__ grp, const double *__restrict__ bvec,
                                                  const VT *__restrict__ q, int use_q, double *__restrict__ r,
                                                  VT *__restrict__ z, VT *__restrict__ p, double *part) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double vals[3] = {0.0, 0.0, 0.0};
  int bin = -1;
  if (i < N) {
    if (!fr[i]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) { r[3 * i + c] = 0.0; z[3 * i + c] = (VT)0; p[3 * i + c] = (VT)0; }
    } else {
      bin = bin_of<NB>(grp, i);
      double rr[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double bv = bvec[3 * i + c];
        vals[2] += bv * bv;
        rr[c] = bv - (use_q ? (double)q[3 * i + c] : 0.0);
        r[3 * i + c] = rr[c];
      }
      const MT *d = Dinv + (size_t)9 * i;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double zz = (double)d[3 * c] * rr[0] + (double)d[3 * c + 1] * rr[1] + (double)d[3 * c + 2] * rr[2];
        VT zv = (VT)zz;
        z[3 * i + c] = zv;
        p[3 * i + c] = zv;
        vals[0] += rr[c] * (double)zv;
        vals[1] += rr[c] * rr[c];
      }
    }
  }
  block_partials<NB, 3>(bin, vals, part, blockIdx.x);
}

__global__ void k_cg_init_finish(int nbk, CgCtl *ctl, const double *part, double tol2, double ref2, int max_it,
                                 int stall) {
  __shared__ double tot[3][1];
  sum_blocks<1, 3>(part, nbk, tot);
  if (threadIdx.x == 0) {
    ctl->tol2 = tol2;
    ctl->ref2 = ref2;
    ctl->max_it = max_it;
    ctl->stall = stall;
    CgSlot &s = ctl->slot[0];
    s.rz = tot[0][0];
    s.rr = tot[1][0];
    s.rnorm = sqrt(tot[1][0]);
    s.rmin = s.rnorm;
    s.it = 0;
    s.it_min = 0;
    s.done = PCG_RUN;
    if (tot[1][0] <= tol2 * ref2) s.done = PCG_CONVERGED;
    if (max_it <= 0) s.done = PCG_CAPPED;
    ctl->slot[1] = s;
    ctl->slot[1].it = -1;
    ctl->stop = s.done ? 1 : 0;
  }
}

__global__ void k_w_init_bins(int nbk, WarmCtl *ctl, const double *part, double tol2) {
  const int b = blockIdx.x;
  double rz = bin_sum(part, nbk, b), rr = bin_sum(part, nbk, kGroups + b), bb = bin_sum(part, nbk, 2 * kGroups + b);
  if (threadIdx.x == 0) {
    ctl->rz[b] = rz;
    ctl->rr[b] = rr;
    ctl->ref2[b] = bb;
    ctl->active[b] = bb > 0.0 && rr > tol2 * bb;
    ctl->alpha[b] = 0.0;
    ctl->beta[b] = 0.0;
  }
}

__global__ void k_w_init_done(WarmCtl *ctl, double tol2, int max_it) {
  if (threadIdx.x != 0) return;
  double rr = 0.0;
  int any = 0;
  for (int b = 0; b < kGroups; ++b) {
    rr += ctl->rr[b];
    any |= ctl->active[b];
  }
  ctl->tol2 = tol2;
  ctl->rnorm = sqrt(rr);
  ctl->it = 0;
  ctl->max_it = max_it;
  ctl->done = any ? (max_it > 0 ? PCG_RUN : PCG_CAPPED) : PCG_CONVERGED;
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

// Adds the timed SpMV launches of one chunk that did work: pair c brackets
// iteration first + c, and only iterations below n_real ran (later launches
// of the chunk exit at once).
static void harvest_events(Scene &s, int first, int n_real) {
  for (int k = 0; k + 1 < s.ev_used; k += 2) {
    float ms = 0.f;
    if (first + k / 2 < n_real && hipEventElapsedTime(&ms, s.ev_pool[k], s.ev_pool[k + 1]) == hipSuccess) {
      s.spmv_ms += ms;
      s.spmv_launches += 1;
    }
  }
  s.ev_used = 0;
}

// r = b - A x0 with x0 given in xsol (start) or zero; leaves r, z, p and the partials.
template <typename MT, typename VT, int NB>
static int pcg_start(Scene &s, const double *rhs, double *xsol, bool start, double *part) {
  int N = s.N, n3 = 3 * N, nb = blocks_for(N, kBS);
  VT *p = static_cast<VT *>(s.pv.p), *q = static_cast<VT *>(s.q.p), *z = static_cast<VT *>(s.z.p);
  const MT *Dinv = static_cast<const MT *>(s.Dinv.p);
  const int *grp = s.group.as<int>();
  bool use_q = false;
  if (!start) {
    hipMemsetAsync(xsol, 0, n3 * sizeof(double), s.stream);
  } else {
    if (sizeof(VT) == 4)
      hipLaunchKernelGGL(k_to_vt_f, dim3(blocks_for(n3, kBS)), dim3(kBS), 0, s.stream, xsol, (float *)p, n3);
    else
      hipLaunchKernelGGL(k_copy_d, dim3(blocks_for(n3, kBS)), dim3(kBS), 0, s.stream, xsol, (double *)p, n3);
    launch_spmv_t<MT, VT>(s, p, q, NB > 1 ? 1 : 0);
    use_q = true;
  }
  hipLaunchKernelGGL((k_pcg_init<MT, VT, NB>), dim3(nb), dim3(kBS), 0, s.stream, N, s.freev.as<uint8_t>(), Dinv, grp,
                     rhs, q, use_q ? 1 : 0, s.r.as<double>(), z, p, part);
  return BAL_OK;
}

// Graph replay: a chunk of PCG iterations is captured once and replayed;
// any change of a buffer address or size invalidates the capture.
static bool graph_current(const std::vector<uintptr_t> &have, const std::vector<uintptr_t> &want,
                          hipGraphExec_t exec) {
  return exec != nullptr && have == want;
}

static void drop_graph(hipGraphExec_t &exec) {
  if (exec) hipGraphExecDestroy(exec);
  exec = nullptr;
}

template <typename F>
static bool capture_graph(Scene &s, hipGraphExec_t &exec, F launches) {
  drop_graph(exec);
  if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  launches();
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s.stream, &g);
  if (e != hipSuccess || g == nullptr) {
    (void)hipGetLastError();
    if (g) hipGraphDestroy(g);
    return false;
  }
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    exec = nullptr;
    return false;
  }
  return true;
}

template <typename MT, typename VT>
static int cg_run(Scene &s, const double *rhs, double *xsol, double tol, double ref2, int max_iters, bool start,
                  bool resume, int *iters_out, double *rnorm_out) {
  int N = s.N, nb = blocks_for(N, kBS), nbs = spmv_grid(N);
  if (s.partial.grow((size_t)(2 * nbs + 3 * nb) * sizeof(double)) || s.pcg_ctl.grow(sizeof(CgCtl)) ||
      s.pv2.grow((size_t)3 * N * sizeof(VT)))
    return BAL_E_OOM;
  double *pq0 = s.partial.as<double>(), *pq1 = pq0 + (size_t)nbs, *part = pq1 + (size_t)nbs;
  CgCtl *ctl = s.pcg_ctl.as<CgCtl>();
  CgCtl *h = s.pin.as<CgCtl>();
  VT *p0 = static_cast<VT *>(s.pv.p), *p1 = static_cast<VT *>(s.pv2.p), *q = static_cast<VT *>(s.q.p),
     *z = static_cast<VT *>(s.z.p);
  const BsrView<MT> B = bsr_view<MT>(s);
  const MT *Dinv = static_cast<const MT *>(s.Dinv.p);
  double *r = s.r.as<double>();
  int k;
  if (resume) {
    // continue the same Krylov sequence for max_iters more iterations, tolerance off:
    // the stopped state k is recomputed from the partials it was made of, with the
    // stagnation window restarted
    hipMemcpyAsync(h, ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, s.stream);
    hipStreamSynchronize(s.stream);
    int cur = h->slot[0].it >= h->slot[1].it ? 0 : 1;
    CgSlot sl = h->slot[cur];
    k = sl.it;
    if (sl.done == PCG_BREAKDOWN) { *iters_out = k; *rnorm_out = sl.rnorm; return BAL_E_NO_CONVERGENCE; }
    if (k == 0) {
      h->slot[0].done = PCG_RUN;
      h->slot[0].it_min = 0;
      h->slot[0].rmin = h->slot[0].rnorm;
    } else {
      CgSlot &pv = h->slot[(k - 1) & 1];
      pv.done = PCG_RUN;
      pv.rmin = INFINITY;
    }
    h->max_it = k + max_iters;
    h->tol2 = 0.0;
    h->stop = 0;
    hipMemcpyAsync(ctl, h, sizeof(CgCtl), hipMemcpyHostToDevice, s.stream);
  } else {
    pcg_start<MT, VT, 1>(s, rhs, xsol, start, part);
    hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kBS), 0, s.stream, nb, ctl, part, tol * tol, ref2, max_iters,
                       s.desc.pcg_stall_window);
    k = 0;
  }
  const int chunk = 16;
  auto launch_iter = [&](int kk, hipEvent_t e0, hipEvent_t e1) {
    VT *pnew = (kk & 1) ? p1 : p0, *pold = (kk & 1) ? p0 : p1;
    double *ppq = (kk & 1) ? pq1 : pq0, *ppq_prev = (kk & 1) ? pq0 : pq1;
    // timed launches carry their own start/stop events (kernel execution only)
    if (e0)
      hipExtLaunchKernelGGL((k_cg_dir_spmv<MT, VT>), dim3(nbs), dim3(kBS), 0, s.stream, e0, e1, 0, N, kk, B, z, pold,
                            pnew, q, ctl, part, nb, ppq_prev, ppq);
    else
      hipLaunchKernelGGL((k_cg_dir_spmv<MT, VT>), dim3(nbs), dim3(kBS), 0, s.stream, N, kk, B, z, pold, pnew, q, ctl,
                         part, nb, ppq_prev, ppq);
    hipLaunchKernelGGL((k_cg_update<MT, VT>), dim3(nb), dim3(kBS), 0, s.stream, N, kk, s.freev.as<uint8_t>(), Dinv,
                       pnew, q, xsol, r, z, ctl, ppq, nbs, part);
  };
  // the kernels use only k & 1, so one capture serves every chunk that starts
  // at an even k.  Kernel timing brackets every product with events, which a
  // captured graph does not time: timed solves launch eagerly.
  std::vector<uintptr_t> sig = bsr_sig(B);
  sig.insert(sig.end(), {(uintptr_t)p0, (uintptr_t)p1, (uintptr_t)q, (uintptr_t)ctl, (uintptr_t)pq0,
                         (uintptr_t)s.freev.p, (uintptr_t)Dinv, (uintptr_t)xsol, (uintptr_t)r, (uintptr_t)z,
                         (uintptr_t)N});
  // Graph chunks are pipelined: chunk c + 1 is queued before the host waits
  // for chunk c's control block, so the stop test leaves the GPU no idle
  // gap, and after the stop the one queued chunk's launches exit at once.
  // The control-block copies go to a pinned area of their own (two slots):
  // the queued chunk's copy may land after this call returns.
  if (s.use_graphs && !s.time_kernels && (k & 1) == 0 && s.pipe_ev[0] && s.pipe_ev[1]) {
    if (!graph_current(s.cg_sig, sig, s.cg_exec)) {
      bool ok = capture_graph(s, s.cg_exec, [&]() {
        for (int c = 0; c < chunk; ++c) launch_iter(c, nullptr, nullptr);
      });
      if (ok) s.cg_sig = sig; else { s.use_graphs = false; s.cg_sig.clear(); }
    }
    if (s.use_graphs) {
      CgCtl *hb = reinterpret_cast<CgCtl *>(static_cast<char *>(s.pin.p) + kPinPipe);
      auto enqueue = [&](int slot) {
        if (hipGraphLaunch(s.cg_exec, s.stream) != hipSuccess) return false;
        ++s.graph_launches;
        k += chunk;
        return hipMemcpyAsync(&hb[slot], ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, s.stream) == hipSuccess &&
               hipEventRecord(s.pipe_ev[slot], s.stream) == hipSuccess;
      };
      if (!enqueue(0)) return BAL_E_HIP;
      for (int c = 0;; ++c) {
        if (!enqueue((c + 1) & 1)) return BAL_E_HIP;
        if (hipEventSynchronize(s.pipe_ev[c & 1]) != hipSuccess) return BAL_E_HIP;
        const CgCtl &hc = hb[c & 1];
        const CgSlot &sl = hc.slot[hc.slot[0].it >= hc.slot[1].it ? 0 : 1];
        if (sl.done) {
          *iters_out = sl.it;
          *rnorm_out = sl.rnorm;
          return sl.done == PCG_BREAKDOWN ? BAL_E_NO_CONVERGENCE : BAL_OK;
        }
      }
    }
  }
  for (;;) {
    bool graphed = false;
    const int first = k;
    if (s.use_graphs && !s.time_kernels && (k & 1) == 0) {
      if (!graph_current(s.cg_sig, sig, s.cg_exec)) {
        bool ok = capture_graph(s, s.cg_exec, [&]() {
          for (int c = 0; c < chunk; ++c) launch_iter(c, nullptr, nullptr);
        });
        if (ok) s.cg_sig = sig; else { s.use_graphs = false; s.cg_sig.clear(); }
      }
      if (s.use_graphs && hipGraphLaunch(s.cg_exec, s.stream) == hipSuccess) {
        graphed = true;
        ++s.graph_launches;
      }
    }
    if (graphed) {
      k += chunk;
    } else {
      for (int c = 0; c < chunk; ++c, ++k) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (s.time_kernels) { e0 = take_event(s); e1 = take_event(s); }
        launch_iter(k, e0, e1);
      }
    }
    hipMemcpyAsync(h, ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, s.stream);
    if (hipStreamSynchronize(s.stream) != hipSuccess) return BAL_E_HIP;
    const CgSlot &sl = h->slot[h->slot[0].it >= h->slot[1].it ? 0 : 1];
    if (s.time_kernels) harvest_events(s, first, sl.it);
    if (sl.done) {
      *iters_out = sl.it;
      *rnorm_out = sl.rnorm;
      return sl.done == PCG_BREAKDOWN ? BAL_E_NO_CONVERGENCE : BAL_OK;
    }
  }
}

template <typename MT, typename VT>
static int warm_run(Scene &s, const double *rhs, double *xsol, double tol, int max_iters, int *iters_out) {
  int N = s.N, nb = blocks_for(N, kBS), nbs = spmv_grid(N);
  // per-bin partials: r.z, r.r, b.b of the update (and the initialisation),
  // then p.q of the product
  if (s.partial.grow(((size_t)3 * kGroups * nb + (size_t)kGroups * nbs) * sizeof(double)) ||
      s.warm_ctl.grow(sizeof(WarmCtl)) || s.pv2.grow((size_t)3 * N * sizeof(VT)))
    return BAL_E_OOM;
  double *part = s.partial.as<double>(), *part_pq = part + (size_t)3 * kGroups * nb;
  WarmCtl *ctl = s.warm_ctl.as<WarmCtl>();
  VT *pb[2] = {static_cast<VT *>(s.pv.p), static_cast<VT *>(s.pv2.p)};
  VT *q = static_cast<VT *>(s.q.p), *z = static_cast<VT *>(s.z.p);
  const BsrView<MT> B = bsr_view<MT>(s);
  const MT *Dinv = static_cast<const MT *>(s.Dinv.p);
  const int *grp = s.group.as<int>();
  double *r = s.r.as<double>();
  pcg_start<MT, VT, kGroups>(s, rhs, xsol, false, part);
  hipLaunchKernelGGL(k_w_init_bins, dim3(kGroups), dim3(kBS), 0, s.stream, nb, ctl, part, tol * tol);
  hipLaunchKernelGGL(k_w_init_done, dim3(1), dim3(64), 0, s.stream, ctl, tol * tol, max_iters);
  WarmCtl *h = s.pin.as<WarmCtl>();
  // iterations go in whole chunks of an even count, so iteration c of a
  // chunk has the parity of c
  const int chunk = 8;
  auto launch_iter = [&](int c) {
    VT *pnew = pb[c & 1], *pold = pb[(c & 1) ^ 1];
    hipLaunchKernelGGL((k_w_dir_spmv<MT, VT>), dim3(nbs), dim3(kBS), 0, s.stream, N, B, grp, z, pold, pnew, q, ctl,
                       part_pq);
    hipLaunchKernelGGL((k_w_update<MT, VT>), dim3(nb), dim3(kBS), 0, s.stream, N, nbs, s.freev.as<uint8_t>(), Dinv,
                       grp, pnew, q, xsol, r, z, ctl, part_pq, part);
    hipLaunchKernelGGL(k_w_beta, dim3(kGroups), dim3(kBS), 0, s.stream, nb, ctl, part);
  };
  std::vector<uintptr_t> sig = bsr_sig(B);
  sig.insert(sig.end(), {(uintptr_t)grp, (uintptr_t)pb[0], (uintptr_t)pb[1], (uintptr_t)q, (uintptr_t)ctl,
                         (uintptr_t)part, (uintptr_t)s.freev.p, (uintptr_t)Dinv, (uintptr_t)xsol, (uintptr_t)r,
                         (uintptr_t)z, (uintptr_t)N});
  for (;;) {
    bool graphed = false;
    if (s.use_graphs) {
      if (!graph_current(s.warm_sig, sig, s.warm_exec)) {
        bool ok = capture_graph(s, s.warm_exec, [&]() {
          for (int c = 0; c < chunk; ++c) launch_iter(c);
        });
        if (ok) s.warm_sig = sig; else { s.use_graphs = false; s.warm_sig.clear(); }
      }
      if (s.use_graphs && hipGraphLaunch(s.warm_exec, s.stream) == hipSuccess) {
        graphed = true;
        ++s.graph_launches;
      }
    }
    if (!graphed)
      for (int c = 0; c < chunk; ++c) launch_iter(c);
    hipMemcpyAsync(h, ctl, sizeof(WarmCtl), hipMemcpyDeviceToHost, s.stream);
    if (hipStreamSynchronize(s.stream) != hipSuccess) return BAL_E_HIP;
    if (h->done) break;
  }
  *iters_out = h->it;
  return BAL_OK;
}

int pcg_solve(Scene &s, const double *rhs, double *xsol, double rtol_ref, int max_iters, int warm, int resume,
              int *iters_out, double *rel_out) {
  // ||r|| <= pcg_rtol * rtol_ref is the stopping rule (reading: zero-guess residual)
  double rn = 0.0;
  int rc;
  double ref2 = rtol_ref * rtol_ref;
  if (s.mixed)
    rc = cg_run<float, float>(s, rhs, xsol, s.desc.pcg_rtol, ref2, max_iters, warm != 0, resume != 0, iters_out, &rn);
  else
    rc = cg_run<double, double>(s, rhs, xsol, s.desc.pcg_rtol, ref2, max_iters, warm != 0, resume != 0, iters_out, &rn);
  *rel_out = rtol_ref > 0 ? rn / rtol_ref : rn;
  return rc;
}

int warm_start_solve(Scene &s, const double *rhs, double *xsol, double wtol, int max_iters, int *iters_out) {
  if (s.mixed) return warm_run<float, float>(s, rhs, xsol, wtol, max_iters, iters_out);
  return warm_run<double, double>(s, rhs, xsol, wtol, max_iters, iters_out);
}

}  // namespace bal
