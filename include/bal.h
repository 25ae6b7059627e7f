/*
 * bal.h -- C ABI of the MI355X (gfx950) barrier-augmented Lagrangian library.
 *
 * One call of bal_step advances one backward-Euler time step: it minimises
 * the incremental potential E(x) = 1/(2h^2)||x - y||_M^2 + Psi(x) with
 * y = x_t + h v_t + h^2 g (Sec. 3.1, problem definition, eq. problem) under
 * the non-penetration constraints d_i(x) > dhat on point-triangle and
 * edge-edge pairs, through the barrier-augmented Lagrangian
 *   L_sigma = E + sigma sum_A b(d_i, dhat)
 *               + sum_A' [mu_i (dhat + s_i - d_i) + sigma b(d_i, dhat + s_i)]
 * (eq. aug-lag, eq. IPC-barrier) and Algorithm 1, each loop pass being one
 * inexact Newton-PCG iteration (Sec. 4) with a CCD step bound and a line
 * search (Sec. 5).  Material: Neo-Hookean tetrahedra; friction is not
 * modelled (frictionless contact).
 *
 * Conventions
 *  - Every call returns an int status (BAL_OK = 0, negative on error) except
 *    bal_destroy_scene / bal_desc_defaults (void) and bal_status_string.
 *    No C++ exception crosses this boundary.
 *  - Positions and vectors at the boundary are row-major [n][3] float64 in
 *    SI units, whatever the precision used inside.
 *  - Vertex numbering: body vertices 0..n_verts-1, then the static obstacle
 *    vertices n_verts..n_verts+n_obs_verts-1 ("all vertices", N_all).
 *  - on_device = 0: pointers are host memory, copied synchronously.
 *    on_device = 1: pointers are device memory of the scene's device; the
 *    call is ordered on the scene's stream (e.g. torch tensors' data_ptr()
 *    with the stream from torch.cuda.current_stream()).
 *  - A scene owns all of its device memory.  Input pointers are read during
 *    the call only.  Output buffers are allocated by the caller.
 *  - One scene must not be used from two host threads at once; calls on one
 *    scene are ordered on its stream.
 */
#ifndef BAL_H
#define BAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bal_status {
  BAL_OK = 0,
  BAL_E_INVALID_ARG = -1,     /* bad size, index, NaN/Inf input, null pointer */
  BAL_E_OOM = -2,             /* device allocation failed */
  BAL_E_HIP = -3,             /* a HIP runtime call failed */
  BAL_E_PENETRATION = -4,     /* initial state has a pair with d <= 0 */
  BAL_E_INVERTED = -5,        /* a tetrahedron with non-positive volume */
  BAL_E_CAPACITY = -6,        /* active pairs exceed max_contacts at every step length */
  BAL_E_NO_CONVERGENCE = -7,  /* max_newton reached; the last iterate is kept */
  BAL_E_STATE = -8,           /* call out of order (e.g. solve before linearize) */
  BAL_E_INDEFINITE = -9       /* bal_step_adjoint: the unprojected Hessian at x_{t+1} is not
                                 positive definite (PCG met p.q <= 0); no gradient is returned */
};

enum bal_precision {
  BAL_FP64 = 0,   /* every step in float64 */
  BAL_MIXED = 1   /* float32 Hessian storage, SpMV, preconditioner and PCG directions;
                     float64 distances, barrier, CCD, residual, dot products,
                     Newton check and multiplier updates */
};

/* Activation rule of the CCD step bound (Sec. 5.3, narrow phase).  The roots of
 * the coplanarity cubic are sought in [-eps, 1+eps] (eps = 1e-12) and clamped
 * into [0, 1]; a time of coplanarity is activated when the pair's distance
 * there is below eps + margin. */
enum bal_ccd_rule {
  BAL_CCD_PRINTED = 0,  /* margin dhat, as printed; a root at |t| <= eps coincides with the
                           start frame t0 = 0 of the paper's candidate times and is not a time
                           of impact (reading: activating it stops every later step of a pair
                           that an iterate left coplanar inside dhat) */
  BAL_CCD_HALF_GAP = 1, /* departure (not in the paper): margin d0 / 2 for a pair that starts
                           closer than dhat (d0 its distance at t = 0), dhat otherwise */
  BAL_CCD_LITERAL = 2   /* margin dhat and roots at |t| <= eps activated too (the literal
                           reading; an iterate left on a point-edge coplanarity inside dhat
                           then bounds every later step at alpha_max = 0) */
};

/* Broad phase of the candidate pass (Sec. 5.3). */
enum bal_broad_phase {
  BAL_BROAD_HASH = 0,  /* spatial hash over dhat-inflated (and swept) boxes (default) */
  BAL_BROAD_LBVH = 1   /* the paper's linear BVH: 64-bit Morton/index keys, radix sort, radix tree,
                          bottom-up box fit; the same candidate set as the hash */
};

typedef struct bal_scene bal_scene;

/* Scene description (read once by bal_create_scene; defaults from bal_desc_defaults). */
typedef struct bal_scene_desc {
  int32_t n_verts, n_tets;
  const double *rest_pos;      /* [n_verts][3] rest positions */
  const int32_t *tets;         /* [n_tets][4] positively oriented at rest */
  const double *youngs;        /* [n_tets] E (Pa) */
  const double *poisson;       /* [n_tets] nu */
  const double *density;       /* [n_tets] rho (kg/m^3) */
  const uint8_t *fixed;        /* [n_verts] 1 = clamped (Dirichlet), or NULL */
  int32_t n_obs_verts, n_obs_tris;
  const double *obs_pos;       /* [n_obs_verts][3] static obstacle vertices */
  const int32_t *obs_tris;     /* [n_obs_tris][3] indices into obs_pos */
  const double *x0, *v0;       /* [n_verts][3] initial state (NULL: rest, zero) */
  double dt;                   /* time step h */
  double gravity[3];
  double dhat;                 /* barrier offset dhat (eq. IPC-barrier) */
  double newton_rtol;          /* ||e^l|| <= rtol ||e^0|| (Alg. 1), default 1e-4 */
  double pcg_rtol;             /* ||r^k|| <= rtol ||r^0|| (App. B), default 1e-4 */
  double sigma_fixed;          /* 0: adaptive barrier stiffness (sigma^0 and growth rule, Sec. 3.4);
                                  > 0: sigma held at this value in every step, so that a step is
                                  the minimiser of one smooth energy (differentiable rollouts) */
  double friction;             /* friction coefficient chi (Sec. 4.1), default 0 (frictionless):
                                  D_j = chi lam_j f(|u_j h|) on every pair with a positive normal force,
                                  its frame (lam_j, normal, barycentric weights) updated per Newton
                                  iteration (fully-implicit friction) */
  double eps_v;                /* mollifier threshold eps_v of f (Sec. 4.1); <= 0: dhat (default) */
  double accept_rtol;          /* 0 (default): a step converges only by the Newton test.  > 0: a step
                                  whose line search finds no decrease of L at FP64 resolution (no
                                  measurable move and A' empty) also counts as converged when its
                                  gradient is within accept_rtol ||e^0|| (the energy's rounding floor
                                  lies above tight Newton tolerances; see bal_step_stats.stalled) */
  int32_t max_newton;          /* default 1000 */
  int32_t max_pcg;             /* PCG iteration cap per Newton iteration, default 20000 */
  int32_t pcg_stall_window;    /* stop PCG when no new minimum of ||r|| in this many
                                  iterations (App. B), default 100 */
  int32_t max_contacts;        /* active-pair memory limit (Sec. 5.2), default 1<<24 */
  int32_t warm_iters;          /* warm-start PCG iteration cap, default 100 */
  int32_t precision;           /* bal_precision */
  int32_t warm_start;          /* 1: stiffness-grouped block-Jacobi warm start (Sec. 4.2) */
  int32_t use_al;              /* 1: augmentation set A' (BAL); 0: plain barrier */
  int32_t ccd_rule;            /* bal_ccd_rule, default BAL_CCD_PRINTED */
  int32_t broad_phase;         /* bal_broad_phase, default BAL_BROAD_HASH */
  int32_t sweep_cap;           /* 0 (default): the swept candidate pass halves its sweep only when it
                                  would exceed its work bound (2^28 direct box tests, the memory
                                  limit of Sec. 5.2); n > 0 (departure, not in the paper): also while
                                  some vertex would move more than n mean surface edge lengths.
                                  alpha_max is then at most the swept fraction of the step */
  int32_t device;              /* HIP device ordinal */
  void *stream;                /* hipStream_t, or NULL for the default stream */
} bal_scene_desc;

/* Statistics of the last bal_step (or the solve inside bal_step_adjoint). */
typedef struct bal_step_stats {
  int32_t newton_iters;        /* loop passes of Alg. 1 */
  int32_t pcg_iters;           /* global PCG iterations, summed */
  int32_t warm_iters;          /* warm-start PCG iterations, summed */
  int32_t n_active_max;        /* max |A| over the step */
  int32_t n_aug_max;           /* max |A'| over the step */
  int32_t converged;           /* 1 if the Newton test passed */
  int32_t ls_retries;          /* line searches that fell below alpha 1e-9 and resumed PCG */
  int32_t spmv_launches;       /* PCG product launches timed (when kernel timing is on) */
  int32_t graph_launches;      /* PCG chunks replayed as HIP graphs (0: launched one by one) */
  int32_t stalled;             /* 1 if the step ended with no measurable move (see accept_rtol) */
  double sigma;                /* final penalty sigma (0 if never initialised) */
  double min_dist;             /* min pair distance at the end of the step (dhat if none closer) */
  double sec_total, sec_pcg, sec_hessian, sec_ccd, sec_collision, sec_linesearch;
  double spmv_ms;              /* summed PCG product kernel time (hipEvents; kernel timing on) */
  double spmv_bytes;           /* algorithmic bytes of one PCG product launch at the last matrix:
                                  the symmetric block SpMV plus reading z and writing the new direction */
  double grad_rel;             /* ||e^l|| / ||e^0|| at the last Newton iterate of the step */
} bal_step_stats;

/* Fills *d with defaults (all pointers NULL, sizes 0). */
void bal_desc_defaults(bal_scene_desc *d);

/* Builds a scene: validates (finite inputs, indices in range, every free
 * vertex in some tet, else BAL_E_INVALID_ARG; positive rest volumes and x0
 * volumes -> BAL_E_INVERTED, every pair at x0 with d > 0 -> BAL_E_PENETRATION),
 * derives masses, rest shape matrices, the surface and the block-sparse
 * pattern, and allocates device memory.  *out is NULL on error. */
int bal_create_scene(const bal_scene_desc *desc, bal_scene **out);

void bal_destroy_scene(bal_scene *s);

/* One time step (Alg. 1).  The state stays on the device.  On
 * BAL_E_NO_CONVERGENCE or BAL_E_CAPACITY the scene still advances to its
 * last feasible iterate.  stats may be NULL. */
int bal_step(bal_scene *s, bal_step_stats *stats);

/* Current positions / velocities of the body vertices, [n_verts][3].
 * Either pointer may be NULL.  Synchronises the stream. */
int bal_get_state(const bal_scene *s, double *x_out, double *v_out, int on_device);

/* Replaces the body state (checkpoint restore).  Fixed vertices keep their
 * given positions and get zero velocity. */
int bal_set_state(bal_scene *s, const double *x, const double *v, int on_device);

/* Replaces per-tet Young's moduli [n_tets] (Poisson ratios unchanged). */
int bal_set_youngs(bal_scene *s, const double *youngs, int on_device);

/* Adjoint of one converged step (not in the paper; frozen-state implicit
 * differentiation of grad_x L_sigma(x*) = 0 with sigma, mu, s, A, A' held at
 * their final values).  Restores (x_t, v_t), re-solves the step to x_{t+1},
 * then solves H lam = gx_next + gv_next / h with the unprojected Hessian H at
 * x_{t+1} by PCG and returns
 *   gx_t = (M/h^2) lam - gv_next / h,   gv_t = (M/h) lam,
 *   gE_accum[e] += -lam_e . grad Psi_e(x_{t+1}) / E_e.
 * All arrays body-vertex sized [n_verts][3] except gE_accum [n_tets].
 * The scene's state is left at (x_{t+1}, v_{t+1}).
 * Friction (chi > 0) has no adjoint here: BAL_E_INVALID_ARG.
 * Errors: BAL_E_NO_CONVERGENCE if the re-solved step does not converge or the
 * adjoint PCG stays above 1e-10 relative residual, BAL_E_INDEFINITE if H is
 * not positive definite; in either case no output (gE_accum included) is
 * written. */
int bal_step_adjoint(bal_scene *s, const double *x_t, const double *v_t,
                     const double *gx_next, const double *gv_next,
                     double *gx_t, double *gv_t, double *gE_accum,
                     int on_device, bal_step_stats *stats);

const char *bal_status_string(int status);

/* Per-iteration decision trace of the last bal_step: *n_rows rows of 8
 * doubles (|A|, |A'|, sigma, min d, alpha_max, alpha, ||e||, PCG iterations).
 * rows may be NULL to query the count; capacity in rows. */
int bal_get_trace(const bal_scene *s, double *rows, int32_t capacity, int32_t *n_rows);

/* Turns per-launch SpMV timing with hipEvents on (1) or off (0). */
int bal_set_kernel_timing(bal_scene *s, int on);

/* ------------------------------------------------------------------------
 * Verification entry points: evaluate the pieces of one Newton iteration at
 * a given iterate, so each can be compared with an independent evaluation.
 * Host pointers only (copies are synchronous).
 * ---------------------------------------------------------------------- */

/* Augmentation state used by bal_linearize (A' with multipliers and slacks). */
typedef struct bal_al_state {
  double sigma;                /* penalty sigma (0: barrier terms off) */
  int32_t n_aug;
  const int32_t *aug_kind;     /* [n_aug] 0 = point-triangle, 1 = edge-edge */
  const int32_t *aug_prims;    /* [n_aug][2] (surface vertex id, surface triangle id) or
                                  (surface edge id, surface edge id), ids as in bal_get_surface */
  const double *mu, *s;        /* [n_aug] multipliers and slacks */
} bal_al_state;

/* Surface primitives in the library's numbering (all-vertex ids):
 * verts [n_sv], tris [n_st][3], edges [n_se][2]; any output may be NULL to
 * query the counts. */
int bal_get_surface(const bal_scene *s, int32_t *n_sv, int32_t *verts, int32_t *n_st,
                    int32_t *tris, int32_t *n_se, int32_t *edges);

/* At iterate x_all [N_all][3] with the scene's predictor y (from its current
 * state) and the given A' state: candidate pairs within dhat, L_sigma
 * (*energy), its gradient grad_all [N_all][3] (zero rows for fixed and
 * obstacle vertices), and the assembled, stencil-projected (project = 1) or
 * unprojected (project = 0) Hessian kept for bal_hessian_apply / bal_solve.
 * *n_active = number of pairs with d < dhat. */
int bal_linearize(bal_scene *s, const double *x_all, const bal_al_state *al, int project,
                  double *energy, double *grad_all, int32_t *n_active);

/* out = H v for the Hessian of the last bal_linearize, [N_all][3] host arrays
 * (fixed / obstacle rows of v are ignored and of out are zero). */
int bal_hessian_apply(bal_scene *s, const double *v, double *out);

/* Stiffness estimate of the last linearize: e_nodes[N_all] (sum over a
 * node's 3 rows of Lambda plus 3 m/h^2, 0 for non-free nodes) and group
 * labels floor(log10 e) (Sec. 4.2).  Either output may be NULL. */
int bal_get_stiffness(const bal_scene *s, double *e_nodes, int32_t *groups);

/* Solves H z = rhs for the last linearize (rows of non-free vertices are
 * ignored).  mode 0: block-Jacobi PCG from zero; mode 1: stiffness-grouped
 * warm start only (blocks coupling different groups skipped, per-group
 * scalars); mode 2: warm start then global PCG.  rtol relative to ||rhs||,
 * max_iters caps each phase.  *iters and *rel_res report the result. */
int bal_solve(bal_scene *s, const double *rhs, double *z, int mode, double rtol,
              int32_t max_iters, int32_t *iters, double *rel_res);

/* CCD step bound alpha_max = min(1, min_i tau_i) along x + t p, t in [0,1],
 * over the candidate pairs of the swept spatial-hash pass (Sec. 5.3). */
int bal_ccd_bound(bal_scene *s, const double *x_all, const double *p_all, double *alpha_max);

/* Candidate pairs of the spatial-hash pass for positions x_all swept along
 * p_all (p_all may be NULL for a proximity pass), sorted canonically:
 * kind[k] (0 PT, 1 EE), nodes[k][4] (PT: p,a,b,c; EE: a0,a1,b0,b1), and the
 * distance dist[k] at x_all.  capacity bounds the outputs; *n_pairs is the
 * full count. */
int bal_candidates(bal_scene *s, const double *x_all, const double *p_all, int32_t capacity,
                   int32_t *kind, int32_t *nodes, double *dist, int32_t *n_pairs);

/* Times n_reps back-to-back SpMV launches on the Hessian of the last
 * linearize (or bal_step) with hipEvents; returns *ms_per_launch and the
 * algorithmic bytes of one launch (*bytes) under the paper's symmetric
 * storage (Sec. 5.1): each lower-triangular or contact off-diagonal block
 * once (9 scalars + a 4-byte index), the N diagonal blocks, a 4-byte row
 * offset per row, one read of the input and one write of the output. */
int bal_spmv_benchmark(bal_scene *s, int32_t n_reps, double *ms_per_launch, double *bytes);

/* CCD step bound over caller-given pairs, no scene (Sec. 5.3 narrow phase,
 * with the scene's rules): alpha_max = min(1, min_i tau_i) along x + t p,
 * t in [0, 1], for pairs (kind[i] 0 point-triangle / 1 edge-edge,
 * nodes[i][4] = p,a,b,c or a0,a1,b0,b1 indexing x and p) with barrier offset
 * dhat and rule ccd_rule (bal_ccd_rule).  Every pointer is device memory of
 * `device`: x, p [n_verts][3] float64, kind [n_pairs], nodes [n_pairs][4]
 * int32, alpha_max one float64.  The call is asynchronous on `stream`
 * (hipStream_t, NULL for the default stream); *alpha_max is written when the
 * stream reaches it.  A node index outside [0, n_verts) or a kind other than
 * 0/1 makes *alpha_max NaN.  Scratch: one float64 per 1024 pairs, allocated
 * and freed on the stream (hipMallocAsync / hipFreeAsync).
 * Returns BAL_E_INVALID_ARG for null pointers, negative sizes, dhat <= 0 or
 * an unknown rule; BAL_E_OOM if the scratch cannot be allocated. */
int bal_pairs_ccd_bound(int32_t device, const double *x, const double *p, int32_t n_verts, const int32_t *kind,
                        const int32_t *nodes, int32_t n_pairs, double dhat, int32_t ccd_rule, double *alpha_max,
                        void *stream);

/* bal_pairs_ccd_bound for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result, with the scratch in a file-scope device array of
 * 2^16 float64 (512 KiB) that each GPU the library runs on holds until the
 * process ends.  At most 2^26 pairs per call (BAL_E_CAPACITY beyond, before
 * any GPU work).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two host threads) race.  Nothing needs
 * clearing between calls (each call writes every partial it reads).  Other
 * errors as bal_pairs_ccd_bound. */
int bal_pairs_ccd_bound_noalloc(int32_t device, const double *x, const double *p, int32_t n_verts,
                                const int32_t *kind, const int32_t *nodes, int32_t n_pairs, double dhat,
                                int32_t ccd_rule, double *alpha_max, void *stream);

/* Streaming-bandwidth reference for the rooflines above: on device `device`,
 * times n_reps launches of a read of n_bytes (summed, so every load is used)
 * and of a copy of n_bytes into a second buffer; reports bytes moved per
 * second in GB/s (the copy counts its reads and writes).  Allocates and frees
 * its own two buffers of n_bytes (n_bytes >= 1 MiB). */
int bal_stream_benchmark(int32_t device, int64_t n_bytes, int32_t n_reps, double *read_gbs, double *copy_gbs);

#ifdef __cplusplus
}
#endif

#endif /* BAL_H */
