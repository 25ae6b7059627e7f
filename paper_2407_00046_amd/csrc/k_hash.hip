// Spatial-hash candidate pass (supporting kernel; replaces the paper's two
// LBVHs of Sec. 5.3 broad phase).
//
// Entry primitives (triangles for point-triangle, edges for edge-edge) are
// inserted into every grid cell their dhat-inflated box (optionally swept
// over [x, x + p]) overlaps; cells hash into a bucket table built by a
// counting sort.  The cell is the mean surface edge length, widened in a
// swept pass by twice the mean sweep length.  Each query primitive (surface
// vertex, surface edge) scans the cells of its own box; a pair is reported
// only in the lowest cell of the overlap of the two cell ranges, so it is
// found once.  Primitives whose box spans more than kLargeCells cells (big
// obstacle faces) are kept out of the grid and tested directly.  Each query
// is served by kQG lanes that split its cells' bucket entries (and its
// direct tests) between them; one traversal counts each lane's partners
// and keeps the first few in the lane's slots, which are compacted at
// scanned offsets (a second traversal writes them when a lane found more),
// and one radix sort of the (query, partner) keys per half puts the list in
// canonical (kind, a, b) order with no atomics in the output.
#include <hipcub/hipcub.hpp>

#include "bal_internal.h"

namespace bal {

constexpr int kHB = 256;
constexpr long kLargeCells = 64;
constexpr long kQueryCells = 4096;
constexpr int kOff = 1 << 20;
constexpr int kQG = 8;  // lanes per query (a power of two dividing the wave)
constexpr int kQSlots = 8;  // keys a query lane keeps from the counting traversal
// Bound on the box tests of one pass (direct tests of large entries and of
// large queries); beyond it the pass reports BAL_E_CAPACITY and the caller
// shortens the sweep.
constexpr double kWorkCap = (double)(1 << 28);

struct Box { double lo[3], hi[3]; };

__device__ __forceinline__ uint64_t cell_key(int ix, int iy, int iz) {
  return ((uint64_t)(ix + kOff) << 42) | ((uint64_t)(iy + kOff) << 21) | (uint64_t)(iz + kOff);
}
__device__ __forceinline__ uint32_t hash64(uint64_t k, uint32_t mask) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return (uint32_t)k & mask;
}
// Cell coordinate, clamped so that the integer conversion is always defined.
__device__ __forceinline__ int cellc(double v, double ih) {
  double c = floor(v * ih);
  c = c > (double)(kOff - 2) ? (double)(kOff - 2) : (c < -(double)(kOff - 2) ? -(double)(kOff - 2) : c);
  return (int)c;
}
// Number of grid cells a box spans (a huge value for non-finite boxes).
__device__ __forceinline__ double box_cells(const double *lo, const double *hi, double ih) {
  double n = 1.0;
  for (int c = 0; c < 3; ++c) {
    if (!(lo[c] <= hi[c]) || !isfinite(lo[c]) || !isfinite(hi[c])) return 1e300;
    n *= floor(hi[c] * ih) - floor(lo[c] * ih) + 1.0;
  }
  return n;
}

// primitive types: 0 vertex (sv), 1 triangle (st), 2 edge (se)
__device__ __forceinline__ int prim_verts(int type, int i, const int *sv, const int *st, const int *se, int *v) {
  if (type == 0) { v[0] = sv[i]; return 1; }
  if (type == 1) { v[0] = st[3 * i]; v[1] = st[3 * i + 1]; v[2] = st[3 * i + 2]; return 3; }
  v[0] = se[2 * i]; v[1] = se[2 * i + 1]; return 2;
}

__device__ Box prim_box(int type, int i, const int *sv, const int *st, const int *se, const double *x,
                        const double *p, double infl) {
  int v[3];
  int nv = prim_verts(type, i, sv, st, se, v);
  Box b;
#pragma unroll
  for (int c = 0; c < 3; ++c) { b.lo[c] = INFINITY; b.hi[c] = -INFINITY; }
  for (int k = 0; k < nv; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double a = x[3 * v[k] + c];
      double e = p ? a + p[3 * v[k] + c] : a;
      double lo = a < e ? a : e, hi = a < e ? e : a;
      b.lo[c] = lo < b.lo[c] ? lo : b.lo[c];
      b.hi[c] = hi > b.hi[c] ? hi : b.hi[c];
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) { b.lo[c] -= infl; b.hi[c] += infl; }
  return b;
}

// Entry boxes (inflated), cell counts, large flags.
__global__ void k_entry_boxes(int n, int type, const int *sv, const int *st, const int *se, const double *x,
                              const double *p, double infl, double ih, Box *boxes, int *cnt, int *large_list,
                              int *nlarge) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Box b = prim_box(type, i, sv, st, se, x, p, infl);
  boxes[i] = b;
  double nc = box_cells(b.lo, b.hi, ih);
  if (nc > (double)kLargeCells) {
    cnt[i] = 0;
    int k = atomicAdd(nlarge, 1);
    large_list[k] = i;
  } else {
    cnt[i] = (int)nc;
  }
}

__global__ void k_entry_write(int n, const Box *boxes, const int *cnt, const int *off, double ih, uint32_t mask,
                              uint64_t *ekey, int *eprim, int *bcnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || cnt[i] == 0) return;
  Box b = boxes[i];
  int l[3], h[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) { l[c] = cellc(b.lo[c], ih); h[c] = cellc(b.hi[c], ih); }
  int o = off[i];
  for (int ix = l[0]; ix <= h[0]; ++ix)
    for (int iy = l[1]; iy <= h[1]; ++iy)
      for (int iz = l[2]; iz <= h[2]; ++iz) {
        uint64_t k = cell_key(ix, iy, iz);
        ekey[o] = k;
        eprim[o] = i;
        atomicAdd(&bcnt[hash64(k, mask)], 1);
        ++o;
      }
}

__global__ void k_entry_scatter(int E, const uint64_t *ekey, const int *eprim, uint32_t mask, const int *bstart,
                                int *bfill, uint64_t *skey, int *sprim) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  uint32_t b = hash64(ekey[e], mask);
  int pos = bstart[b] + atomicAdd(&bfill[b], 1);
  skey[pos] = ekey[e];
  sprim[pos] = eprim[e];
}

struct QueryArgs {
  int qtype, etype, nq, ne;
  const int *sv, *st, *se;
  const uint8_t *fr;
  int nbody;
  const double *x, *p;
  const Box *ebox;
  double ih;
  uint32_t mask;
  const int *bstart;
  const uint64_t *skey;
  const int *sprim;
  const int *large_list;
  int nlarge;
  const uint8_t *qlarge;  // EE: query edge is large (brute-force role)
};

__device__ __forceinline__ bool boxes_overlap(const Box &a, const Box &b) {
  return a.lo[0] <= b.hi[0] && b.lo[0] <= a.hi[0] && a.lo[1] <= b.hi[1] && b.lo[1] <= a.hi[1] &&
         a.lo[2] <= b.hi[2] && b.lo[2] <= a.hi[2];
}

// Pair filters (reading): no shared vertex, not obstacle-only, some free node.
__device__ bool pair_ok(const QueryArgs &A, int q, int t) {
  int vq[3], vt[3];
  int nq = prim_verts(A.qtype, q, A.sv, A.st, A.se, vq);
  int nt = prim_verts(A.etype, t, A.sv, A.st, A.se, vt);
  bool anyfree = false;
  for (int a = 0; a < nq; ++a) {
    anyfree |= A.fr[vq[a]] != 0;
    for (int b = 0; b < nt; ++b)
      if (vq[a] == vt[b]) return false;
  }
  for (int b = 0; b < nt; ++b) anyfree |= A.fr[vt[b]] != 0;
  if (!anyfree) return false;
  bool qobs = vq[0] >= A.nbody, tobs = vt[0] >= A.nbody;
  return !(qobs && tobs);
}

// Visits the candidate partners of query q that fall to lane `lane` of the
// query's kQG lanes; emit(t) for each.  For edge-edge only partners t > q
// are reported (each unordered pair once, in the segment of its smaller edge).
template <typename F>
__device__ void visit_query(const QueryArgs &A, int q, int lane, F emit) {
  Box qb = prim_box(A.qtype, q, A.sv, A.st, A.se, A.x, A.p, 0.0);
  bool ee = A.qtype == 2;
  if ((ee && A.qlarge[q]) || box_cells(qb.lo, qb.hi, A.ih) > (double)kQueryCells) {
    // large query (big obstacle edge, or a box spanning too many cells):
    // direct test against every entry (every later edge for edge-edge)
    for (int t = (ee ? q + 1 : 0) + lane; t < A.ne; t += kQG)
      if (boxes_overlap(qb, A.ebox[t]) && pair_ok(A, q, t)) emit(t);
    return;
  }
  int l[3], h[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) { l[c] = cellc(qb.lo[c], A.ih); h[c] = cellc(qb.hi[c], A.ih); }
  for (int ix = l[0]; ix <= h[0]; ++ix)
    for (int iy = l[1]; iy <= h[1]; ++iy)
      for (int iz = l[2]; iz <= h[2]; ++iz) {
        uint64_t k = cell_key(ix, iy, iz);
        uint32_t b = hash64(k, A.mask);
        for (int e = A.bstart[b] + lane; e < A.bstart[b + 1]; e += kQG) {
          if (A.skey[e] != k) continue;
          int t = A.sprim[e];
          if (ee && t <= q) continue;
          const Box &tb = A.ebox[t];
          // canonical cell: lowest cell of the overlap of the two cell ranges
          int c0 = max(l[0], cellc(tb.lo[0], A.ih)), c1 = max(l[1], cellc(tb.lo[1], A.ih)),
              c2 = max(l[2], cellc(tb.lo[2], A.ih));
          if (c0 != ix || c1 != iy || c2 != iz) continue;
          if (boxes_overlap(qb, tb) && pair_ok(A, q, t)) emit(t);
        }
      }
  for (int k = lane; k < A.nlarge; k += kQG) {
    int t = A.large_list[k];
    if (ee && t <= q) continue;
    if (boxes_overlap(qb, A.ebox[t]) && pair_ok(A, q, t)) emit(t);
  }
}

// One thread per (query, lane); the kQG lanes of a query are consecutive
// lanes of one wave.  Writes the lane's count and the query's total, and
// keeps the lane's first ks keys in its own slots.  A lane with more
// raises the overflow flag (a plain store of 1) and the pass traverses
// again with k_query_write; otherwise k_query_compact moves the slots into
// place, so that one traversal serves both count and write.
__global__ void k_query_count_keep(QueryArgs A, int ks, int *lcnt, int *qcnt, uint64_t *slots, int *ovf) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int q = gid / kQG, lane = gid % kQG;
  if (q >= A.nq) return;  // whole groups leave together
  uint64_t *mine = slots + (size_t)gid * ks;
  int c = 0;
  visit_query(A, q, lane, [&](int t) {
    if (c < ks) mine[c] = ((uint64_t)q << 32) | (uint32_t)t;
    ++c;
  });
  lcnt[gid] = c;
  if (c > ks) *ovf = 1;
#pragma unroll
  for (int m = kQG / 2; m > 0; m >>= 1) c += __shfl_xor(c, m, kQG);
  if (lane == 0) qcnt[q] = c;
}

__global__ void k_query_compact(int nq, int ks, const int *lcnt, const int *qoff, const uint64_t *slots,
                                uint64_t *outb) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int q = gid / kQG, lane = gid % kQG;
  if (q >= nq) return;
  int o = qoff[q];
  const int *lc = lcnt + (size_t)q * kQG;
  for (int k = 0; k < lane; ++k) o += lc[k];
  const int c = lc[lane];  // <= ks: no lane overflowed
  const uint64_t *mine = slots + (size_t)gid * ks;
  for (int m = 0; m < c; ++m) outb[o + m] = mine[m];
}

// Same traversal; each lane writes at the query's offset plus the counts of
// the lanes before it.  The segment is sorted by the emit pass.
__global__ void k_query_write(QueryArgs A, const int *lcnt, const int *qoff, uint64_t *outb) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int q = gid / kQG, lane = gid % kQG;
  if (q >= A.nq) return;
  int o = qoff[q];
  const int *lc = lcnt + (size_t)q * kQG;
  for (int k = 0; k < lane; ++k) o += lc[k];
  visit_query(A, q, lane, [&](int t) { outb[o++] = ((uint64_t)q << 32) | (uint32_t)t; });
}

// Queries whose box is tested directly against every entry.
__global__ void k_big_queries(QueryArgs A, int *nbig) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  Box qb = prim_box(A.qtype, q, A.sv, A.st, A.se, A.x, A.p, 0.0);
  if ((A.qtype == 2 && A.qlarge[q]) || box_cells(qb.lo, qb.hi, A.ih) > (double)kQueryCells) atomicAdd(nbig, 1);
}

__global__ void k_large_flag(int n, const Box *ebox, double ih, uint8_t *fl) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Box b = ebox[i];
  fl[i] = box_cells(b.lo, b.hi, ih) > (double)kLargeCells ? 1 : 0;
}

// Pairs from their (query, partner) keys, already radix-sorted into the
// canonical (query, partner) order: one thread per pair.
__global__ void k_emit_sorted(int P, int kind, const uint64_t *__restrict__ keys, const int *sv, const int *st,
                              const int *se, int base, int *okind, int *oa, int *ob, int4 *onodes, uint64_t *okey) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint64_t key = keys[k];
  const int q = (int)(key >> 32), t = (int)(uint32_t)key;
  const int o = base + k;
  okind[o] = kind;
  oa[o] = q;
  ob[o] = t;
  int4 nd;
  if (kind == 0) nd = make_int4(sv[q], st[3 * t], st[3 * t + 1], st[3 * t + 2]);
  else nd = make_int4(se[2 * q], se[2 * q + 1], se[2 * t], se[2 * t + 1]);
  onodes[o] = nd;
  okey[o] = ((uint64_t)kind << 62) | ((uint64_t)q << 31) | (uint64_t)t;
}

static int grow_pairs(PairList &pl, int n) {
  size_t m = (size_t)(n > 0 ? n : 1);
  if (pl.kind.grow(m * sizeof(int)) || pl.a.grow(m * sizeof(int)) || pl.b.grow(m * sizeof(int)) ||
      pl.nodes.grow(m * sizeof(int4)) || pl.d.grow(m * sizeof(double)) || pl.cs.grow(m * sizeof(int)) ||
      pl.key.grow(m * sizeof(uint64_t)))
    return BAL_E_OOM;
  return BAL_OK;
}

// One half of the pass (point-triangle or edge-edge); returns the pair count
// (negative on error) and leaves per-query offsets in qoff_buf and the
// (query, partner) keys, grouped by query, in out_buf.  Two host synchronisations: the entry
// count (with the large-entry and large-query counts of the work bound) and
// the pair count.
static int hash_half(Scene &s, int qtype, int etype, const double *x, const double *p, double cell,
                     int *qoff_out_n, DBuf &qoff_buf, DBuf &out_buf) {
  int nq = qtype == 0 ? s.nsv : s.nse;
  int ne = etype == 1 ? s.nst : s.nse;
  double ih = 1.0 / cell;
  double infl = s.desc.dhat;
  if (s.hb_lo.grow((size_t)(ne + 1) * sizeof(Box)) || s.h_cnt.grow((size_t)(ne + 1) * sizeof(int)) ||
      s.h_off.grow((size_t)(ne + 1) * sizeof(int)) || s.h_large.grow((size_t)(ne + 1) * sizeof(int)) ||
      s.h_nlarge.grow(3 * sizeof(int)) || s.hq_lo.grow((size_t)(nq + 1) * sizeof(uint8_t)) ||
      s.h_lcnt.grow(((size_t)nq * kQG + 1) * sizeof(int)) ||
      s.h_slots.grow(((size_t)nq * kQG * kQSlots + 1) * sizeof(uint64_t)))
    return BAL_E_OOM;
  const int ks = kQSlots;
  Box *ebox = s.hb_lo.as<Box>();
  int *nlarge_d = s.h_nlarge.as<int>();  // [0] large entries, [1] large queries, [2] slot overflow
  hipMemsetAsync(nlarge_d, 0, 3 * sizeof(int), s.stream);
  if (ne > 0)
    hipLaunchKernelGGL(k_entry_boxes, dim3(blocks_for(ne, kHB)), dim3(kHB), 0, s.stream, ne, etype, s.sv.as<int>(),
                       s.st.as<int>(), s.se.as<int>(), x, p, infl, ih, ebox, s.h_cnt.as<int>(), s.h_large.as<int>(),
                       nlarge_d);
  uint8_t *qlarge = s.hq_lo.as<uint8_t>();
  if (qtype == 2 && ne > 0)
    hipLaunchKernelGGL(k_large_flag, dim3(blocks_for(ne, kHB)), dim3(kHB), 0, s.stream, ne, ebox, ih, qlarge);
  QueryArgs A{};
  A.qtype = qtype; A.etype = etype; A.nq = nq; A.ne = ne;
  A.sv = s.sv.as<int>(); A.st = s.st.as<int>(); A.se = s.se.as<int>();
  A.fr = s.freev.as<uint8_t>(); A.nbody = s.nb; A.x = x; A.p = p; A.ebox = ebox; A.ih = ih;
  A.large_list = s.h_large.as<int>(); A.qlarge = qlarge;
  if (nq > 0)
    hipLaunchKernelGGL(k_big_queries, dim3(blocks_for(nq, 128)), dim3(128), 0, s.stream, A, nlarge_d + 1);
  int *hn = s.pin.as<int>() + 1024;  // clear of the slot the scan reads back
  hipMemcpyAsync(hn, nlarge_d, 2 * sizeof(int), hipMemcpyDeviceToHost, s.stream);
  int E = scan_exclusive(s, s.h_cnt.as<int>(), s.h_off.as<int>(), ne);  // synchronises
  if (E < 0) return BAL_E_OOM;
  if (ne <= 0 && hipStreamSynchronize(s.stream) != hipSuccess) return BAL_E_HIP;  // the scan returned at once
  const int nlarge = hn[0], nbig = hn[1];
  if ((double)nq * nlarge + (double)nbig * ne > kWorkCap) return BAL_E_CAPACITY;
  uint32_t M = 1024;
  while ((long)M < 2L * E) M <<= 1;
  if (s.h_key.grow((size_t)(E + 1) * sizeof(uint64_t)) || s.h_prim.grow((size_t)(E + 1) * sizeof(int)) ||
      s.h_skey.grow((size_t)(E + 1) * sizeof(uint64_t)) || s.h_sprim.grow((size_t)(E + 1) * sizeof(int)) ||
      s.h_bcnt.grow((size_t)(M + 1) * sizeof(int)) || s.h_bstart.grow((size_t)(M + 1) * sizeof(int)) ||
      s.h_bfill.grow((size_t)(M + 1) * sizeof(int)))
    return BAL_E_OOM;
  hipMemsetAsync(s.h_bcnt.p, 0, (M + 1) * sizeof(int), s.stream);
  hipMemsetAsync(s.h_bfill.p, 0, (M + 1) * sizeof(int), s.stream);
  if (ne > 0)
    hipLaunchKernelGGL(k_entry_write, dim3(blocks_for(ne, kHB)), dim3(kHB), 0, s.stream, ne, ebox, s.h_cnt.as<int>(),
                       s.h_off.as<int>(), ih, M - 1, s.h_key.as<uint64_t>(), s.h_prim.as<int>(), s.h_bcnt.as<int>());
  if (scan_exclusive_async(s, s.h_bcnt.as<int>(), s.h_bstart.as<int>(), (int)M + 1)) return BAL_E_OOM;
  if (E > 0)
    hipLaunchKernelGGL(k_entry_scatter, dim3(blocks_for(E, kHB)), dim3(kHB), 0, s.stream, E, s.h_key.as<uint64_t>(),
                       s.h_prim.as<int>(), M - 1, s.h_bstart.as<int>(), s.h_bfill.as<int>(), s.h_skey.as<uint64_t>(),
                       s.h_sprim.as<int>());
  A.mask = M - 1;
  A.bstart = s.h_bstart.as<int>(); A.skey = s.h_skey.as<uint64_t>(); A.sprim = s.h_sprim.as<int>();
  A.nlarge = nlarge;
  if (s.h_qcnt.grow((size_t)(nq + 1) * sizeof(int)) || qoff_buf.grow((size_t)(nq + 1) * sizeof(int))) return BAL_E_OOM;
  hipMemsetAsync(s.h_qcnt.p, 0, (nq + 1) * sizeof(int), s.stream);
  const int qthreads = nq * kQG;  // nq * kQG < 2^31: nq is a surface count
  if (nq > 0)
    hipLaunchKernelGGL(k_query_count_keep, dim3(blocks_for(qthreads, kHB)), dim3(kHB), 0, s.stream, A, ks,
                       s.h_lcnt.as<int>(), s.h_qcnt.as<int>(), s.h_slots.as<uint64_t>(), nlarge_d + 2);
  hipMemcpyAsync(hn + 2, nlarge_d + 2, sizeof(int), hipMemcpyDeviceToHost, s.stream);
  int P = scan_exclusive(s, s.h_qcnt.as<int>(), qoff_buf.as<int>(), nq + 1);  // synchronises
  if (P < 0) return BAL_E_OOM;
  if (out_buf.grow((size_t)(P + 1) * sizeof(uint64_t))) return BAL_E_OOM;
  if (nq > 0 && P > 0) {
    if (hn[2])  // some lane found more than its slots hold: traverse again
      hipLaunchKernelGGL(k_query_write, dim3(blocks_for(qthreads, kHB)), dim3(kHB), 0, s.stream, A,
                         s.h_lcnt.as<int>(), qoff_buf.as<int>(), out_buf.as<uint64_t>());
    else
      hipLaunchKernelGGL(k_query_compact, dim3(blocks_for(qthreads, kHB)), dim3(kHB), 0, s.stream, nq, ks,
                         s.h_lcnt.as<int>(), qoff_buf.as<int>(), s.h_slots.as<uint64_t>(), out_buf.as<uint64_t>());
  }
  *qoff_out_n = nq;
  return P;
}

// ------------------------------------------------------------------- LBVH
// The paper's own broad phase (Sec. 5.3), selectable in place of the hash:
// one linear BVH per half over the entry primitives (triangles for
// point-triangle, edges for edge-edge), their boxes inflated by dhat (and
// swept for CCD) exactly as the hash's.  Each entry gets a 64-bit key, the
// 30-bit Morton code of its box centre (10 bits per axis over the centres'
// bounding box) in the high word and its index in the low word, so keys are
// distinct; a radix sort orders them; the binary radix tree over the sorted
// keys is built one internal node per thread (split at the highest differing
// key bit), and boxes are fitted bottom up, each internal node completed by
// the second of its two children to arrive.  Queries then descend the tree
// with a stack and report the same pairs, through the same filters, as the
// hash; the emit pass sorts each query's segment, so both broad phases return
// the same canonical list.
constexpr int kLbvhStack = 72;  // tree depth <= key length (64) + 1

struct LbvhView {
  int n;                   // leaves
  const int *leaf_prim;    // entry index of each leaf (sorted order)
  const int2 *child;       // internal node children: >= 0 internal, < 0 leaf ~c
  const Box *ibox;         // internal node boxes
};

__device__ __forceinline__ uint32_t morton30(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 10; ++b)
    m |= (((x >> b) & 1u) << (3 * b + 2)) | (((y >> b) & 1u) << (3 * b + 1)) | (((z >> b) & 1u) << (3 * b));
  return m;
}

// Entry boxes and per-block bounds of their centres (lo, hi of 3 axes).
__global__ void k_lbvh_boxes(int n, int type, const int *sv, const int *st, const int *se, const double *x,
                             const double *p, double infl, Box *boxes, double *part) {
  __shared__ double red[6][kHB];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double c[3] = {INFINITY, INFINITY, INFINITY}, d[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (i < n) {
    Box b = prim_box(type, i, sv, st, se, x, p, infl);
    boxes[i] = b;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = d[k] = 0.5 * (b.lo[k] + b.hi[k]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) { red[k][threadIdx.x] = c[k]; red[3 + k][threadIdx.x] = d[k]; }
  __syncthreads();
  for (int w = kHB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[(size_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_lbvh_bounds(int nb, const double *part, double *bounds) {
  __shared__ double red[6][kHB];
  double c[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c[k] = fmin(c[k], part[(size_t)b * 6 + k]);
      c[3 + k] = fmax(c[3 + k], part[(size_t)b * 6 + 3 + k]);
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = c[k];
  __syncthreads();
  for (int w = kHB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) bounds[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_lbvh_keys(int n, const Box *boxes, const double *bounds, uint64_t *keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Box b = boxes[i];
  uint32_t q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ext = bounds[3 + k] - bounds[k];
    double t = ext > 0.0 ? (0.5 * (b.lo[k] + b.hi[k]) - bounds[k]) / ext : 0.0;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    q[k] = (uint32_t)fmin(t * 1024.0, 1023.0);
  }
  keys[i] = ((uint64_t)morton30(q[0], q[1], q[2]) << 32) | (uint64_t)(uint32_t)i;
}

// common prefix length of sorted keys i and j (-1 outside [0, n))
__device__ __forceinline__ int lbvh_delta(const uint64_t *k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  return __clzll(k[i] ^ k[j]);
}

// Internal node i of the radix tree over n sorted (distinct) keys: the range
// of leaves it covers extends from i in the direction of the neighbour with
// the longer common prefix; it splits where the common prefix of the range
// ends.  Also the leaves' entry indices and every node's parent.
__global__ void k_lbvh_tree(int n, const uint64_t *keys, int *leaf_prim, int2 *child, int *parent,
                            int *leaf_parent) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) leaf_prim[i] = (int)(uint32_t)(keys[i] & 0xffffffffu);
  if (i >= n - 1) return;
  const int d = lbvh_delta(keys, n, i, i + 1) - lbvh_delta(keys, n, i, i - 1) >= 0 ? 1 : -1;
  const int dmin = lbvh_delta(keys, n, i, i - d);
  int lmax = 2;
  while (lbvh_delta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
  int l = 0;
  for (int t = lmax / 2; t >= 1; t /= 2)
    if (lbvh_delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = lbvh_delta(keys, n, i, j);
  int sp = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (lbvh_delta(keys, n, i, i + (sp + t) * d) > dnode) sp += t;
  } while (t > 1);
  const int gamma = i + sp * d + (d < 0 ? d : 0);
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  const int left = lo == gamma ? ~gamma : gamma;
  const int right = hi == gamma + 1 ? ~(gamma + 1) : gamma + 1;
  child[i] = make_int2(left, right);
  if (left < 0) leaf_parent[~left] = i; else parent[left] = i;
  if (right < 0) leaf_parent[~right] = i; else parent[right] = i;
  if (i == 0) parent[0] = -1;
}

__device__ __forceinline__ double ld_acq(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bottom-up fit: one thread per leaf walks to the root; at each internal node
// the first arrival stops and the second (whose sibling subtree is complete)
// writes the node's box.  Node boxes go through device-scope atomic loads and
// stores with a fence before each arrival count, so the second arrival reads
// the boxes the first one wrote.  Every thread stops after at most depth steps.
__global__ void k_lbvh_refit(int n, const Box *ebox, const int *leaf_prim, const int2 *child, const int *parent,
                             const int *leaf_parent, int *arrive, Box *ibox) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int node = leaf_parent[i];
  for (int step = 0; step < kLbvhStack && node >= 0; ++step) {
    __threadfence();
    if (atomicAdd(&arrive[node], 1) == 0) return;
    __threadfence();
    const int2 c = child[node];
    double lo[3], hi[3];
    const int cc[2] = {c.x, c.y};
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double *src = cc[h] < 0 ? (const double *)&ebox[leaf_prim[~cc[h]]] : (const double *)&ibox[cc[h]];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lo[k] = fmin(lo[k], ld_acq(src + k));
        hi[k] = fmax(hi[k], ld_acq(src + 3 + k));
      }
    }
    double *dst = (double *)&ibox[node];
#pragma unroll
    for (int k = 0; k < 3; ++k) { st_rel(dst + k, lo[k]); st_rel(dst + 3 + k, hi[k]); }
    node = parent[node];
  }
}

// Partners of query q in the tree (edge-edge: only partners t > q); emit(t).
// Returns false if the descent stack overflowed (cannot happen for a tree of
// depth <= 64, which the 64-bit keys guarantee).
template <typename F>
__device__ bool lbvh_visit(const QueryArgs &A, const LbvhView &T, int q, F emit) {
  const Box qb = prim_box(A.qtype, q, A.sv, A.st, A.se, A.x, A.p, 0.0);
  const bool ee = A.qtype == 2;
  auto leaf = [&](int lf) {
    const int t = T.leaf_prim[lf];
    if ((!ee || t > q) && boxes_overlap(qb, A.ebox[t]) && pair_ok(A, q, t)) emit(t);
  };
  if (T.n == 0) return true;
  if (T.n == 1) { leaf(0); return true; }
  int stack[kLbvhStack];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const int2 c = T.child[stack[--sp]];
    const int cc[2] = {c.x, c.y};
    for (int h = 0; h < 2; ++h) {
      if (cc[h] < 0) {
        leaf(~cc[h]);
      } else if (boxes_overlap(qb, T.ibox[cc[h]])) {
        if (sp >= kLbvhStack) return false;
        stack[sp++] = cc[h];
      }
    }
  }
  return true;
}

__global__ void k_lbvh_count(QueryArgs A, LbvhView T, int *qcnt, int *flags) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  int c = 0;
  if (!lbvh_visit(A, T, q, [&](int) { ++c; })) atomicOr(flags, 4);
  qcnt[q] = c;
}

__global__ void k_lbvh_write(QueryArgs A, LbvhView T, const int *qoff, uint64_t *outb) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.nq) return;
  int o = qoff[q];
  lbvh_visit(A, T, q, [&](int t) { outb[o++] = ((uint64_t)q << 32) | (uint32_t)t; });
}

static int lbvh_half(Scene &s, int qtype, int etype, const double *x, const double *p, double /*cell*/,
                     int *qoff_out_n, DBuf &qoff_buf, DBuf &out_buf) {
  const int nq = qtype == 0 ? s.nsv : s.nse;
  const int ne = etype == 1 ? s.nst : s.nse;
  const int nbk = blocks_for(ne > 0 ? ne : 1, kHB);
  const size_t E1 = (size_t)(ne > 0 ? ne : 1);
  if (s.hb_lo.grow((E1 + 1) * sizeof(Box)) || s.lb_part.grow((size_t)nbk * 6 * 8 + 6 * 8) ||
      s.lb_key.grow(E1 * 8) || s.lb_key2.grow(E1 * 8) || s.lb_prim.grow(E1 * 4) ||
      s.lb_child.grow(E1 * sizeof(int2)) || s.lb_parent.grow(E1 * 4) || s.lb_lparent.grow(E1 * 4) ||
      s.lb_arrive.grow(E1 * 4) || s.lb_ibox.grow(E1 * sizeof(Box)))
    return BAL_E_OOM;
  Box *ebox = s.hb_lo.as<Box>();
  double *bounds = s.lb_part.as<double>() + (size_t)nbk * 6;
  if (ne > 0) {
    hipLaunchKernelGGL(k_lbvh_boxes, dim3(nbk), dim3(kHB), 0, s.stream, ne, etype, s.sv.as<int>(), s.st.as<int>(),
                       s.se.as<int>(), x, p, s.desc.dhat, ebox, s.lb_part.as<double>());
    hipLaunchKernelGGL(k_lbvh_bounds, dim3(1), dim3(kHB), 0, s.stream, nbk, s.lb_part.as<double>(), bounds);
    hipLaunchKernelGGL(k_lbvh_keys, dim3(nbk), dim3(kHB), 0, s.stream, ne, ebox, bounds, s.lb_key.as<uint64_t>());
    size_t tmp = 0;
    if (hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, s.lb_key.as<uint64_t>(), s.lb_key2.as<uint64_t>(), ne, 0, 64,
                                          s.stream) != hipSuccess)
      return BAL_E_HIP;
    if (s.lb_tmp.grow(tmp + 16)) return BAL_E_OOM;
    if (hipcub::DeviceRadixSort::SortKeys(s.lb_tmp.p, tmp, s.lb_key.as<uint64_t>(), s.lb_key2.as<uint64_t>(), ne, 0,
                                          64, s.stream) != hipSuccess)
      return BAL_E_HIP;
    hipMemsetAsync(s.lb_arrive.p, 0, E1 * 4, s.stream);
    hipLaunchKernelGGL(k_lbvh_tree, dim3(nbk), dim3(kHB), 0, s.stream, ne, s.lb_key2.as<uint64_t>(),
                       s.lb_prim.as<int>(), s.lb_child.as<int2>(), s.lb_parent.as<int>(), s.lb_lparent.as<int>());
    if (ne > 1)
      hipLaunchKernelGGL(k_lbvh_refit, dim3(nbk), dim3(kHB), 0, s.stream, ne, ebox, s.lb_prim.as<int>(),
                         s.lb_child.as<int2>(), s.lb_parent.as<int>(), s.lb_lparent.as<int>(), s.lb_arrive.as<int>(),
                         s.lb_ibox.as<Box>());
  }
  QueryArgs A{};
  A.qtype = qtype; A.etype = etype; A.nq = nq; A.ne = ne;
  A.sv = s.sv.as<int>(); A.st = s.st.as<int>(); A.se = s.se.as<int>();
  A.fr = s.freev.as<uint8_t>(); A.nbody = s.nb; A.x = x; A.p = p; A.ebox = ebox;
  LbvhView T{ne, s.lb_prim.as<int>(), s.lb_child.as<int2>(), s.lb_ibox.as<Box>()};
  if (s.h_qcnt.grow((size_t)(nq + 1) * sizeof(int)) || qoff_buf.grow((size_t)(nq + 1) * sizeof(int))) return BAL_E_OOM;
  hipMemsetAsync(s.h_qcnt.p, 0, (nq + 1) * sizeof(int), s.stream);
  hipMemsetAsync(s.flags.p, 0, sizeof(int), s.stream);
  if (nq > 0)
    hipLaunchKernelGGL(k_lbvh_count, dim3(blocks_for(nq, 128)), dim3(128), 0, s.stream, A, T, s.h_qcnt.as<int>(),
                       s.flags.as<int>());
  int *fl = s.pin.as<int>() + 1024;
  hipMemcpyAsync(fl, s.flags.p, sizeof(int), hipMemcpyDeviceToHost, s.stream);
  int P = scan_exclusive(s, s.h_qcnt.as<int>(), qoff_buf.as<int>(), nq + 1);  // synchronises
  if (P < 0) return BAL_E_OOM;
  if (*fl & 4) return BAL_E_CAPACITY;  // descent stack overflow (not reachable for 64-bit keys)
  if (out_buf.grow((size_t)(P + 1) * sizeof(uint64_t))) return BAL_E_OOM;
  if (nq > 0 && P > 0)
    hipLaunchKernelGGL(k_lbvh_write, dim3(blocks_for(nq, 128)), dim3(128), 0, s.stream, A, T, qoff_buf.as<int>(),
                       out_buf.as<uint64_t>());
  *qoff_out_n = nq;
  return P;
}

static int bits_for(int n) {
  int b = 1;
  while (b < 31 && (1 << b) < n) ++b;
  return b;
}

// The half's keys radix-sorted into (query, partner) order (query in bits
// 32.., partner in bits 0..31: only the bits in use are sorted), in `sorted`.
static int sort_half(Scene &s, int P, int nq, DBuf &keys, DBuf &sorted) {
  if (P <= 0) return BAL_OK;
  if (sorted.grow((size_t)P * sizeof(uint64_t))) return BAL_E_OOM;
  const int end_bit = 32 + bits_for(nq + 1);
  size_t tmp = 0;
  if (hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, keys.as<uint64_t>(), sorted.as<uint64_t>(), P, 0, end_bit,
                                        s.stream) != hipSuccess)
    return BAL_E_HIP;
  if (s.lb_tmp.grow(tmp + 16)) return BAL_E_OOM;
  if (hipcub::DeviceRadixSort::SortKeys(s.lb_tmp.p, tmp, keys.as<uint64_t>(), sorted.as<uint64_t>(), P, 0, end_bit,
                                        s.stream) != hipSuccess)
    return BAL_E_HIP;
  return BAL_OK;
}

// |p_i| per vertex, summed for the pass's mean sweep length
__global__ void k_sweep_len(const double *__restrict__ p, double *__restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt(p[3 * i] * p[3 * i] + p[3 * i + 1] * p[3 * i + 1] + p[3 * i + 2] * p[3 * i + 2]);
}

// Hash cell of a pass.  At rest the cell is the mean surface edge length; a
// swept pass widens it by twice the mean sweep length: swept boxes cover a
// few cells instead of dozens (each of which also holds dozens of swept
// entries), and few entries or queries pass the large-box thresholds.  The
// candidate set is the box-overlap set whatever the cell.
static double pass_cell(Scene &s, const double *p) {
  if (p == nullptr || s.N <= 0 || s.h_plen.grow((size_t)(s.N + 1) * sizeof(double))) return s.cell;
  hipLaunchKernelGGL(k_sweep_len, dim3(blocks_for(s.N, kHB)), dim3(kHB), 0, s.stream, p, s.h_plen.as<double>(), s.N);
  const double mean = reduce_sum(s, s.h_plen.as<double>(), s.N) / s.N;
  return std::isfinite(mean) ? s.cell + 2.0 * mean : s.cell;
}

int build_candidates(Scene &s, PairList &out, const double *x, const double *p) {
  out.n = 0;
  if (s.nsv == 0 && s.nse == 0) return BAL_OK;
  const bool lbvh = s.desc.broad_phase == BAL_BROAD_LBVH;
  auto half = lbvh ? lbvh_half : hash_half;
  const double cell = lbvh ? s.cell : pass_cell(s, p);
  int nq_pt = 0, nq_ee = 0;
  const int Ppt = half(s, 0, 1, x, p, cell, &nq_pt, s.qoff_pt, s.out_pt);
  if (Ppt < 0) return Ppt;
  int rc = sort_half(s, Ppt, nq_pt, s.out_pt, s.h_sorted_pt);
  if (rc) return rc;
  const int Pee = half(s, 2, 2, x, p, cell, &nq_ee, s.qoff_ee, s.out_ee);
  if (Pee < 0) return Pee;
  if ((rc = sort_half(s, Pee, nq_ee, s.out_ee, s.h_sorted_ee))) return rc;
  const int total = Ppt + Pee;
  if (grow_pairs(out, total)) return BAL_E_OOM;
  if (Ppt > 0)
    hipLaunchKernelGGL(k_emit_sorted, dim3(blocks_for(Ppt, kHB)), dim3(kHB), 0, s.stream, Ppt, 0,
                       s.h_sorted_pt.as<uint64_t>(), s.sv.as<int>(), s.st.as<int>(), s.se.as<int>(), 0,
                       out.kind.as<int>(), out.a.as<int>(), out.b.as<int>(), out.nodes.as<int4>(),
                       out.key.as<uint64_t>());
  if (Pee > 0)
    hipLaunchKernelGGL(k_emit_sorted, dim3(blocks_for(Pee, kHB)), dim3(kHB), 0, s.stream, Pee, 1,
                       s.h_sorted_ee.as<uint64_t>(), s.sv.as<int>(), s.st.as<int>(), s.se.as<int>(), Ppt,
                       out.kind.as<int>(), out.a.as<int>(), out.b.as<int>(), out.nodes.as<int4>(),
                       out.key.as<uint64_t>());
  out.n = total;
  return BAL_OK;
}

}  // namespace bal
