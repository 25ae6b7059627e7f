// Internal declarations shared by the library's translation units: the scene
// object, device buffers and the host-side kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bal.h"
#include "bal_math.h"

namespace bal {

// Growable device buffer (bytes); grow() never shrinks and drops contents.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  int grow(size_t need);
  void release();
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

// byte offset of the energy evaluation's readback slots in the pinned scratch
constexpr size_t kPinEnergy = 16384;

// Stiffness-group bins of the warm start: group label + 32 clamped to [0, 63].
constexpr int kGroups = 64;
constexpr int kGroupOffset = 32;
// done codes
enum { PCG_RUN = 0, PCG_CONVERGED = 1, PCG_STALLED = 2, PCG_CAPPED = 3, PCG_BREAKDOWN = 4 };


struct PairList {            // candidate pairs (sorted by (kind, a, b))
  int n = 0;
  DBuf kind, a, b, nodes, d, cs;  // int, int, int, int4, double, int
  DBuf key;                       // uint64 key
};

struct Scene {
  int dev = 0;
  hipStream_t stream = nullptr;
  bal_scene_desc desc;  // scalar parameters (pointers cleared)
  int nb = 0, no = 0, N = 0, T = 0;
  int nsv = 0, nst = 0, nse = 0;
  double cell = 0.0;    // spatial-hash cell size
  bool mixed = false;
  // Body vertices are numbered internally in Morton order of the rest shape;
  // perm_h[internal] = caller's index.  Obstacle vertices keep their slots.
  std::vector<int> perm_h;
  DBuf perm_d, stage;
  std::vector<double> mass_h;
  std::vector<uint8_t> free_h;
  std::vector<int> sv_h, st_h, se_h;
  std::vector<double> youngs_h, poisson_h;
  // static device data
  DBuf tets, tc, mass, freev, node_tet_ptr, node_tet_src, row_ptr, col_idx, blk_src_ptr, blk_src;
  DBuf up_ptr, up_ent;   // per row j: (i, block index) of the stored blocks (i, j), i > j, ascending i
  DBuf sv, st, se;
  int nnzb = 0;          // stored off-diagonal element blocks: strictly lower triangle (i > j)
  int nsrc = 0;
  // state
  DBuf x, v, x_t, v_t, y, xtrial, dx;
  // per-iteration element data
  DBuf tet_e, tet_g, tet_tr, tet_blk;
  // assembled matrix
  DBuf val, Dblk, Dinv, e_nodes, group;
  DBuf grad, grad_b;  // gradient, barrier-only gradient
  // contacts
  PairList cand, cand2, uni, augtmp;
  DBuf uni_flag, uni_aug;  // barrier on (int), aug index (int)
  DBuf pair_e, pair_g, pair_tr, pair_blk;
  DBuf fr, fr_e;  // friction frame per union pair: lam, beta[4], n[3] (8 doubles); friction energies
  DBuf cdiag_ptr, cdiag_src, coff_ptr, coff_col, coff_src, ccount, cfill;
  DBuf cm_ptr, cm_col, cm_blk;  // merged off-diagonal contact blocks per row (one per distinct column)
  DBuf cm_head, cm_ridx;        // run flags and run indices of the sorted off-diagonal entries
  int n_cdiag = 0, n_coff = 0, n_cm = 0;
  // augmentation set A' (sorted by key)
  int n_aug = 0;
  DBuf aug_kind, aug_a, aug_b, aug_nodes, aug_key, aug_mu, aug_s, aug_d, aug_e;
  DBuf aug_tmp_mu, aug_tmp_s;
  double sigma = 0.0, sigma0 = 0.0;
  bool sigma_set = false;
  // hash scratch
  DBuf hb_lo, hb_hi, hq_lo, hq_hi, h_cnt, h_off, h_key, h_prim, h_bcnt, h_bstart, h_bfill, h_skey, h_sprim,
      h_large, h_nlarge, h_qcnt, h_lcnt, h_slots, h_plen, h_qoff, h_out, qoff_pt, out_pt, qoff_ee, out_ee;
  // LBVH scratch
  DBuf lb_part, lb_key, lb_key2, lb_tmp, lb_prim, lb_child, lb_parent, lb_lparent, lb_arrive, lb_ibox;
  DBuf h_sorted_pt, h_sorted_ee;  // candidate keys of each half in canonical order
  // PCG
  DBuf ent;  // FP32 storage: per row its lower then transposed entries (operand, block), one dummy at the end
  DBuf r, z, pv, pv2, q, pcg_ctl, warm_ctl, partial, counter, scan_tmp, red_out, red_slots, flags;
  DBuf node_e, cand_e, mask, mask_off, tau, rhs, psweep;
  DBuf pin;     // pinned host scratch (hipHostMalloc, 64 KiB): bytes 0-4095 scalar and
                // control-block readbacks, 4096- candidate-pass counts, kPinEnergy- the
                // energy readback, 32768- the pipelined PCG chunks' control-block copies
  // graph replay of PCG chunks (re-captured when a buffer moves)
  bool use_graphs = true;
  bool own_stream = false;
  hipGraphExec_t cg_exec = nullptr, warm_exec = nullptr;
  hipEvent_t pipe_ev[2] = {nullptr, nullptr};  // pipelined PCG chunks: one per control-block copy
  std::vector<uintptr_t> cg_sig, warm_sig;
  // timing
  bool time_kernels = false;
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  double spmv_ms = 0.0;
  int spmv_launches = 0;
  int graph_launches = 0;
  // trace of the last step
  std::vector<double> trace;
  bool linearized = false;
  bool verbose = false;  // progress lines on stderr (BAL_VERBOSE=1)
  bal_step_stats last{};
  // cached element stencil reduction
  double Lel[9], Qel[12];
};

// ----- launchers (k_elem.hip)
enum ElemMode { EM_ENERGY = 0, EM_GRAD = 1, EM_HESS = 2 };
void launch_elements(Scene &s, const double *x, int mode, int project);
// ----- launchers (k_contact.hip)
void launch_pair_distance(Scene &s, const PairList &pl, const double *x, double *d, int *cs);
void launch_pair_barrier_energy(Scene &s, const PairList &pl, const double *x, double sigma, double *e, int *flags);
void launch_aug_energy(Scene &s, const double *x, double sigma, double *e, double *d, int *flags);
void launch_pair_linearize(Scene &s, const double *x, int project, double sigma, int with_friction);
void launch_friction_energy(Scene &s, const double *x, double *e);
void launch_aug_update(Scene &s, const double *x);
void launch_ccd(Scene &s, const PairList &pl, const double *x, const double *p, double *tau);
// ----- launchers (k_hash.hip)
int build_candidates(Scene &s, PairList &out, const double *x, const double *p);
// ----- launchers (k_linalg.hip)
int scan_exclusive(Scene &s, const int *in, int *out, int n);  // returns total (synchronises), -1 on OOM
int scan_exclusive_async(Scene &s, const int *in, int *out, int n);  // 0, or -1 on OOM
double reduce_sum(Scene &s, const double *in, int n);
double reduce_min(Scene &s, const double *in, int n);
int reduce_count_less(Scene &s, const double *in, int n, double thr);
void reduce_sum_to(Scene &s, const double *in, int n, double *dst);
void reduce_min_to(Scene &s, const double *in, int n, double *dst);
void count_less_to(Scene &s, const double *in, int n, double thr, double *dst);
void launch_predictor(Scene &s);
void launch_axpy_state(Scene &s, double *out, const double *a, const double *b, double alpha, int n3);
void launch_inertia_energy(Scene &s, const double *x, double *out_per_node);
int build_contact_lists(Scene &s);
void launch_node_assembly(Scene &s, const double *x, int with_contacts, int with_inertia, int with_elements,
                          int want_hess, double *grad_out);
void launch_offdiag_assembly(Scene &s);
void launch_spmv(Scene &s, const void *vin, void *vout, int masked);
int pcg_solve(Scene &s, const double *rhs, double *xsol, double rtol_ref, int max_iters, int warm,
              int resume, int *iters_out, double *rel_out);
int warm_start_solve(Scene &s, const double *rhs, double *xsol, double tol, int max_iters, int *iters_out);
double spmv_bytes(const Scene &s);
double cg_product_bytes(const Scene &s);
double dot_free(Scene &s, const double *a, const double *b);

// helpers
int hip_ok(hipError_t e);
// eps_v h of the friction mollifier (eps_v <= 0 in the description: dhat)
inline double friction_eps_h(const Scene &s) {
  return (s.desc.eps_v > 0.0 ? s.desc.eps_v : s.desc.dhat) * s.desc.dt;
}
template <typename T> int upload(Scene &s, DBuf &b, const T *src, size_t n) {
  if (b.grow(n * sizeof(T))) return BAL_E_OOM;
  if (n && hipMemcpyAsync(b.p, src, n * sizeof(T), hipMemcpyHostToDevice, s.stream) != hipSuccess) return BAL_E_HIP;
  return BAL_OK;
}
inline int blocks_for(long n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace bal
