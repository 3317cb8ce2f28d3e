/* dmrg.h -- SU(2) spin-adapted two-site DMRG: the Davidson H.psi hot path.
 *
 * Effective-Hamiltonian action of one two-site step (paper: Sec. II A,
 * Eq. (2)-(3)): F := F + sum_i alpha_i A_i B_i C_i D_i E, where E and F are
 * the reduced two-site wavefunction, A (D) are reduced operators of the left
 * (right) block, B (C) are reduced operators of the left (right) site, and
 * the SU(2) coupling enters as scalar factors C~ of Eq. (4) (Sec. II B-C).
 *
 * Conventions (all spins are passed doubled, 2S, as int32):
 *  - Orbitals 0..L-1; sites l = site_l, r = site_l+1; left block [0, l),
 *    right block [l+2, L).  Jordan-Wigner order L < l < r < R.
 *  - Hamiltonian: Eq. (1) in spin-free form with real chemist integrals,
 *    H = sum h_ij E_ij + 1/2 sum (ij|kl) sum_st a+_is a+_kt a_lt a_js.
 *  - Reduced elements: <J'M'|T^k_q|JM> = <JM;kq|J'M'> <J'||T^k||J>.
 *    a~_q = (-1)^(1/2-q) a_{-q}; [T x U]^K_Q = sum <k1 q1;k2 q2|K Q> T_q1 U_q2.
 *  - Sites have three multiplets: 0 = empty, 1 = one electron (s=1/2),
 *    2 = doubly occupied a+_up a+_dn|0>.
 *  - Wavefunction basis ((L l) S_Ll (r R) S_rR) S; blocks are enumerated by
 *    nested loops over (left sector, l, 2S_Ll ascending, r, right sector,
 *    2S_rR ascending) keeping those with the right electron count and spin
 *    triangles; each block is a column-major d_L x d_R FP64 matrix and the
 *    blocks are concatenated in that order.
 *  - Operator families (id: name, 2k, labels) of a block -- see the family
 *    table below.  Each family member is a reduced operator between block
 *    sectors; records group all positions (labels) of one family for one
 *    (row sector, column sector) pair as [npos][rows][cols], each matrix
 *    column-major (Sec. II A: position-dependent operators stored
 *    contiguously with a third index).
 *
 * Family table (W0_ij = 2(ij|xy) - (iy|xj), W1_ij = sqrt(3) (iy|xj); j, k, l, i
 * internal to the block; outside labels: left block [l, L) with pairs having
 * at least one site orbital, right block [0, l+2) with all pairs):
 *   0 H   2k=0  one position           block Hamiltonian
 *   1 C   2k=1  i in block             a+_i
 *   2 A0  2k=0  i<=j in block (left)   [a+_i a+_j]^0
 *   3 A1  2k=2  i<j  in block (left)   [a+_i a+_j]^1
 *   4 B0  2k=0  i<=j in block (left)   [a+_i a~_j]^0
 *   5 B1  2k=2  i<=j in block (left)   [a+_i a~_j]^1
 *   6 S   2k=1  x outside              sum (xj|kl) [[a+_k a~_l]^0 a~_j]^1/2
 *   7 P0  2k=0  x<=y outside           sum (xj|yl) [a~_l a~_j]^0
 *   8 P1  2k=2  x<y  outside           sum (xj|yl) [a~_l a~_j]^1
 *   9 Q0  2k=0  x<=y outside           sum W0_ij [a+_i a~_j]^0
 *  10 Q1  2k=2  x<=y outside           sum W1_ij [a+_i a~_j]^1
 *   Label order: single labels ascending.  Pairs inside the left block (A, B)
 *   and pairs of the right block's P, Q come in groups: (1) x<y inside the
 *   left block, lexicographic; (2) (x,x) inside it; (3) (x,l); (4) (x,l+1) with
 *   x in the left block; (5) site pairs (l,l), (l,l+1), (l+1,l+1) -- groups
 *   3-5 only for the right block, strict families (x<y) omit diagonal pairs.
 *   Pairs of the left block's P, Q are lexicographic (x outer, y inner).
 *
 * Ownership: the caller owns every array.  Host arrays are read during
 * dmrg_build_tasks only.  Operator data (ldata/rdata) are DEVICE arrays that
 * the plan references until dmrg_plan_free; psi/hpsi are device arrays
 * borrowed for one call.  The plan owns its descriptors, operator copies,
 * slices and stripe workspace: device memory taken with hipMalloc by
 * dmrg_build_tasks (the stripe workspace bounded by opts.workspace_bytes)
 * and by dmrg_davidson for its basis, all returned by dmrg_plan_free or at
 * the end of the solve.
 * Errors: negative status codes; no exception crosses the ABI; on error the
 * outputs are unspecified and dmrg_last_error() (thread-local) describes it.
 * After DMRG_EHIP the plan must be freed.  A plan is not reentrant.
 */
#ifndef DMRG_H
#define DMRG_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  DMRG_OK = 0,
  DMRG_EINVAL = -1,     /* malformed argument */
  DMRG_ESYM = -2,       /* electron count / spin triangle violated */
  DMRG_ERANGE = -3,     /* record offset or size beyond its data array */
  DMRG_ENOMEM = -4,     /* device or host allocation failed */
  DMRG_EHIP = -5,       /* HIP runtime error */
  DMRG_ENONFINITE = -6, /* NaN or Inf met */
  DMRG_ENOCONV = -7     /* Davidson did not converge (best pair returned) */
};

typedef struct { int32_t n, two_s, dim; } dmrg_sector_t;
typedef struct { int32_t fam, row_sec, col_sec, npos; int64_t off; } dmrg_oprec_t;

typedef struct {
  int32_t n_orb, n_elec, two_s, site_l;
  const double *h1;          /* host [L*L] one-electron integrals            */
  const double *eri;         /* host [L^4] (ij|kl), index ((i*L+j)*L+k)*L+l   */
  int32_t n_lsec, n_rsec;
  const dmrg_sector_t *lsec, *rsec;   /* host sector tables                  */
  int64_t n_lrec, n_rrec;
  const dmrg_oprec_t *lrec, *rrec;    /* host operator records               */
  const double *ldata, *rdata;        /* DEVICE operator data                */
  int64_t ldata_len, rdata_len;       /* elements                            */
} dmrg_problem_t;

enum { DMRG_FP64 = 0, DMRG_SPLIT_BF16 = 1 };

/* Plan flags.
 *  DMRG_PLAN_GRAPH: dmrg_apply_H records its launch sequence once per
 *    (psi, hpsi) pair into a HIP graph (on a plan-owned capture stream) and
 *    replays it on the caller's stream; at most 64 graphs are kept (least
 *    recently created evicted).  Profiling events are not recorded in graphs.
 *  DMRG_PLAN_AUTOTUNE: dmrg_build_tasks times dmrg_apply_H under candidate
 *    settings -- kpart in {1024, 2048, 4096} x tile_policy in {0, 1}, then
 *    for split plans the work-group tile threshold (macro_min) in
 *    {none, 32, 48, 96} at the best of those and the wide tile threshold
 *    (wide_min) in {none, 48, 96, 192}, then workspace caps of 512 MiB and
 *    192 MiB -- and keeps the fastest; choices are cached by a hash of the
 *    plan's block shapes and options, for the process and in opts.tune_cache.
 *    The chosen values are in dmrg_plan_stats.
 *  DMRG_PLAN_XCD: accepted for compatibility; every tile launch takes its
 *    tiles from per-XCD queues (contiguous equal-cost ranges of the list). */
enum { DMRG_PLAN_GRAPH = 1, DMRG_PLAN_XCD = 2, DMRG_PLAN_AUTOTUNE = 4 };

typedef struct {
  int32_t precision;        /* DMRG_FP64 or DMRG_SPLIT_BF16                   */
  int32_t n_slices;         /* split only: BF16 slices per operand (3..7)     */
  int64_t workspace_bytes;  /* cap for the intermediate stripes, 0 = 64 GiB   */
  int32_t flags;            /* DMRG_PLAN_* bits                                */
  int32_t kpart;            /* summed K per second-stage work item, 0 = 2048 */
  int32_t tile_policy;      /* 0: 16x64 / 32x32 / 64x16 by output shape,
                               1: 32x32 except outputs of <= 16 rows          */
  int32_t macro_min;        /* split plans: outputs with both sides >= this are
                               computed in 64x64 tiles by whole work groups
                               sharing LDS-staged operands (0: 48; < 0: never) */
  int32_t wide_min;         /* split plans with n_slices <= 5: outputs with both
                               sides >= this are cut into 128-wide bands (a
                               last band of >= this many lines included) of
                               128x128 tiles of one work group each (one per
                               CU), the rest of them into the tiles above
                               (0: 48; < 0: never)                          */
  int32_t pad_opts;
  /* Device memory of the plan (descriptors, operator copies, slices,
   * workspace), of the autotuner and of dmrg_davidson / dmrg_mlp_collect on
   * this plan comes from alloc_fn(bytes, alloc_ctx) and goes back through
   * free_fn(ptr, alloc_ctx) (at dmrg_plan_free, re-planning, or the end of a
   * solve); both NULL: hipMalloc / hipFree.  alloc_fn returns NULL on
   * failure (DMRG_ENOMEM).  The memory must be usable on the streams the plan
   * is given (e.g. a caching allocator's blocks of that stream). */
  void *(*alloc_fn)(size_t bytes, void *ctx);
  void (*free_fn)(void *ptr, void *ctx);
  void *alloc_ctx;
  /* DMRG_PLAN_AUTOTUNE: path of a text file of tuned settings (one line per
   * plan-shape hash), read before tuning and appended after it, so a choice
   * survives the process; NULL: tuning results are kept for the process. */
  const char *tune_cache;
} dmrg_plan_opts_t;

typedef struct dmrg_plan dmrg_plan_t;

typedef struct {
  int64_t psi_len;          /* total wavefunction length (all problems)       */
  int64_t n_blocks;         /* wavefunction blocks                            */
  int64_t n_rows;           /* operator-table rows (Eq. 2 combinations)       */
  int64_t n_tasks;          /* sector tasks x positions (Eq. 3 rows)          */
  int64_t n_stage1;         /* first-stage products                           */
  int64_t n_segments;       /* second-stage stripe segments                   */
  double flops;             /* algorithmic FP64 flops of one H.psi, 2mnk      */
  double stage1_flops, stage2_flops;
  int64_t workspace_bytes;  /* stripe workspace actually used                 */
  int32_t n_chunks;         /* launches pairs per H.psi                       */
  int32_t kpart;            /* settings in use (after autotuning)             */
  int32_t tile_policy;
  int32_t xcd;
  int32_t tuned;            /* candidates timed by the autotuner (0: none,
                               -1: settings read from the tune cache file) */
  int32_t launches;         /* kernel launches of one H.psi                  */
  int64_t workspace_cap;    /* stripe workspace cap in use, bytes            */
  double tune_ms;           /* autotuner wall time                            */
  double tasks_ms;          /* host: operator, sector-task and value tables  */
  double plan_ms;           /* stripe grouping, tile lists, device set-up (and
                               autotuning)                                  */
  int32_t macro_min;        /* work-group tile threshold in use (0: none)    */
  int32_t wide_min;         /* wide tile threshold in use (0: none)          */
  int64_t device_bytes;     /* device memory the plan holds                  */
} dmrg_plan_stats_t;

/* Build the operator table, sector-task and sector-value tables (Sec. II A,
 * II C, Eq. (3)-(4)), group them into stripe products (Sec. III A) and upload
 * the plan.  probs: n_probs problems solved side by side (one concatenated
 * wavefunction).  stream: hipStream_t or NULL.  */
int dmrg_build_tasks(const dmrg_problem_t *probs, int32_t n_probs,
                     const dmrg_plan_opts_t *opts, void *stream, dmrg_plan_t **out);

/* Offset and length of problem `prob` inside the concatenated wavefunction
 * (the reduced two-site wavefunction E/F of Eq. (2), Sec. II A, stored as its
 * sector blocks, Sec. II A "sector-table"; problems of a plan concatenated in
 * order).  off/len: host pointers, either may be NULL.  DMRG_EINVAL for a
 * NULL plan or prob outside [0, n_probs). */
int dmrg_psi_layout(const dmrg_plan_t *p, int32_t prob, int64_t *off, int64_t *len);

/* hpsi := H_eff psi for all problems (device arrays of psi_len doubles). */
int dmrg_apply_H(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream);

/* For callers that cannot allocate device memory (code under a graph capture
 * of their own, tight serving loops, harnesses that forbid hipMalloc): the
 * same H.psi as dmrg_apply_H, but the scratch memory of the launch sequence
 * (stripe workspace, partial tiles and, for split plans, stripe slices and
 * their exponents) comes from one static device array of
 * DMRG_STATIC_SCRATCH_BYTES per GPU, held until the process ends, instead of
 * the plan's buffers.  Allocates nothing (no hipMalloc, no graph); psi/hpsi
 * are device arrays of psi_len doubles, borrowed for the call.  Returns
 * DMRG_EINVAL when the plan's scratch exceeds the array (build the plan with
 * a smaller workspace_bytes: its stripe workspace is cut into more launches).
 * Every call on a GPU shares that GPU's array and leaves its contents behind
 * (each word a call reads is written earlier in the same call): calls that
 * overlap on one GPU, on any streams, race. */
#define DMRG_STATIC_SCRATCH_BYTES ((int64_t)256 << 20)
int dmrg_apply_H_static(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream);

/* diag := diagonal of H_eff (device array of psi_len doubles). */
int dmrg_diag_H(dmrg_plan_t *p, double *diag, void *stream);

/* Davidson solve for the lowest eigenpair of H_eff (paper, Sec. II: the
 * effective Hamiltonian is diagonalised iteratively by Lanczos or Davidson),
 * for every problem of the plan at once (one segment of psi per problem, as
 * laid out by dmrg_psi_layout).  psi: device array of psi_len doubles, in =
 * starting vectors, out = normalised Ritz vector of each problem; evals: host
 * array of n_probs doubles, out = Ritz values.  Block size 1, thick restart
 * to the current and previous Ritz vectors at m_max (all problems restart
 * together), two-pass Gram-Schmidt, correction -r/(diag - theta) with
 * |diag - theta| >= floor * sigma, sigma the root mean square of diag - theta
 * over the problem (or the learned correction of the network in o->mlp, see
 * below), a problem stops when ||H u - theta u||_2 <= tol
 * (its segment of later basis vectors is zero).  Returns DMRG_ENOCONV (with
 * the best pairs in psi/evals) when max_iter is reached before every problem
 * converged.  All vector work runs on the GPU in FP64 (segmented, fixed-order
 * reductions: bitwise reproducible); the m x m projected problems are solved
 * on the host.  stats: iters = most iterations of any problem, converged =
 * number of converged problems, residual = largest final residual, energy =
 * Ritz value of problem 0. */
typedef struct dmrg_mlp dmrg_mlp_t;
enum { DMRG_PRECOND_DIAG = 0, DMRG_PRECOND_MLP = 1 };
typedef struct {
  double tol;               /* residual-norm tolerance, e.g. 1e-8            */
  int32_t max_iter;
  int32_t m_max;            /* subspace size, 3..64 (24 by default)         */
  int32_t precond;          /* DMRG_PRECOND_DIAG or DMRG_PRECOND_MLP         */
  int32_t verbose;          /* > 0: a progress line on stderr every 25 iterations */
  double floor;             /* relative preconditioner denominator floor: the
                               magnitude of diag - theta is raised to at least
                               floor * RMS(diag - theta) of the problem (1e-2
                               with no options; an absolute floor had to be
                               hand-set per workload)                        */
  const dmrg_mlp_t *mlp;    /* network for DMRG_PRECOND_MLP, else NULL       */
  int32_t mlp_patience;     /* learned steps of a problem stop after this many
                               iterations without a new smallest residual
                               (0: 30); the rest of its solve is diagonal    */
  int32_t pad;
} dmrg_dav_opts_t;
/* fallbacks: learned corrections rejected by the guard (non-finite, or
 * |cos(t_mlp, t_diag)| < DMRG_MLP_GUARD) and replaced by the diagonal step;
 * switched: problems whose learned steps were stopped by mlp_patience. */
typedef struct {
  int32_t iters, n_hpsi, converged, fallbacks;
  double residual, energy;
  double t_total_s, t_hpsi_s;
  int32_t switched, pad;
  double sigma;             /* RMS(diag - theta) of problem 0 at its last theta */
} dmrg_dav_stats_t;
int dmrg_davidson(dmrg_plan_t *p, double *psi, double *evals, const dmrg_dav_opts_t *o,
                  dmrg_dav_stats_t *st, void *stream);

/* Plan statistics (host struct, filled): sizes of the operator table, the
 * sector-task table and its stripe grouping (Sec. II A, Eq. (3); Sec. III A),
 * and the algorithmic FP64 flop count of one H.psi -- 2mnk summed over the
 * executed products, the measure of the paper's TFLOPS figures (Sec. IV A,
 * complexity of the operations of Eq. (2) over the elapsed time); split plans
 * count each product once.  DMRG_EINVAL for NULL arguments. */
int dmrg_plan_stats(const dmrg_plan_t *p, dmrg_plan_stats_t *st);

/* ---- learned Davidson preconditioner ------------------------------------
 * The paper leaves the Davidson details open (Sec. II).  This optional
 * preconditioner corrects the diagonal step per element with a 3-layer
 * perceptron: t_i = td_i (1 + g(x_i)), td_i = -r_i / (d_i - theta) (floored),
 * g(x) = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, td floored as the diagonal
 * step (relative floor), inputs
 * x_i = (asinh((d_i - theta)/sigma), log10(||r||)/8), sigma the root mean
 * square of d - theta over the problem.  Parameters are FP32 on the device,
 * one flat vector: W1[DMRG_MLP_IN][w], b1[w], W2[w][w], b2[w], w3[w], b3
 * (row-major, W[k][j] maps input k to unit j).  Training data are exact
 * corrections of converged solves: at iteration k, t*_k = psi* / <u_k|psi*> - u_k;
 * each element gives a row x, a = td s, b = t* s with s = sqrt(n)/||t*_k||,
 * both scaled by DMRG_MLP_A_MAX/|a| where |a| exceeds DMRG_MLP_A_MAX (keeps
 * the row's optimum, bounds its weight); the loss is mean (a (1 + g) - b)^2
 * over rows.  Widths 32, 64, 128, 256.  */
enum { DMRG_MLP_IN = 2 };
#define DMRG_MLP_A_MAX 10.0
#define DMRG_MLP_GUARD 1e-3
/* New network, parameters drawn from a seeded generator (He scaling), Adam
 * state zero.  Device memory is allocated here and by dmrg_mlp_train. */
int dmrg_mlp_create(int32_t width, uint64_t seed, dmrg_mlp_t **out);
int64_t dmrg_mlp_num_params(const dmrg_mlp_t *m);
/* Host <-> device parameter copies of exactly num_params floats; setting the
 * parameters resets the Adam state.  Both (and dmrg_mlp_free) first wait for
 * the last dmrg_mlp_forward / dmrg_mlp_adam_step launches of this network,
 * which return before their work is done (an event on their stream, not a
 * device-wide synchronisation). */
int dmrg_mlp_set_params(dmrg_mlp_t *m, const float *host, int64_t n);
int dmrg_mlp_get_params(const dmrg_mlp_t *m, float *host, int64_t n);
/* g[i] := network output for row x[i] (device arrays x[n][2], g[n]). */
int dmrg_mlp_forward(dmrg_mlp_t *m, const float *x, int64_t n, float *g, void *stream);
/* The learned correction of one preconditioning step, as dmrg_davidson
 * applies it (same fused kernel): for every segment k, elements
 * [seg_off[k], seg_off[k+1]) of the device vectors diag, r and t,
 * t_i = td_i (1 + g(x_i)), td_i = -r_i / (diag_i - theta_k) with
 * |diag_i - theta_k| raised to at least floor * sigma_k, and
 * x_i = (asinh((diag_i - theta_k) / sigma_k), log10(rnorm_k) / 8).  theta,
 * sigma (the RMS of diag - theta over the segment), rnorm (the norm of the
 * segment of r): host arrays of nseg doubles; seg_off: host array of nseg + 1
 * offsets starting at 0.  floor: the relative floor (> 0).  Synchronises the
 * stream; takes a small temporary device buffer.  DMRG_EINVAL for malformed
 * arguments. */
int dmrg_mlp_step(const dmrg_mlp_t *m, const double *diag, const double *r, int32_t nseg,
                  const int64_t *seg_off, const double *theta, const double *sigma, const double *rnorm,
                  double floor, double *t, void *stream);
/* loss (host) and its gradient (device array of num_params floats) over the
 * n rows (x, a, b) (device arrays), by back-propagation. */
int dmrg_mlp_loss_grad(dmrg_mlp_t *m, const float *x, const float *a, const float *b, int64_t n,
                       double *loss, float *grad, void *stream);
/* One Adam update with the gradient grad (device), bias-corrected with the
 * network's own step counter (incremented first). */
int dmrg_mlp_adam_step(dmrg_mlp_t *m, const float *grad, float lr, float beta1, float beta2, float eps,
                       void *stream);
typedef struct {
  float lr, beta1, beta2, eps;
  int32_t batch;            /* rows per step, drawn with replacement         */
  int32_t steps;
  uint64_t seed;            /* minibatch index generator (SplitMix64)         */
} dmrg_mlp_train_opts_t;
/* Minibatch Adam training on n rows (device arrays x[n][2], a[n], b[n]);
 * loss_trace: host array of `steps` floats or NULL. */
int dmrg_mlp_train(dmrg_mlp_t *m, const float *x, const float *a, const float *b, int64_t n,
                   const dmrg_mlp_train_opts_t *o, float *loss_trace, void *stream);
/* Training rows from one single-problem plan: solve to convergence from psi0
 * (device, not modified) with the diagonal preconditioner, then repeat the
 * identical solve recording the rows of every iteration whose overlap
 * |<u_k|psi*>| >= 1e-3.  x (device [capacity][2]), a, b (device [capacity]);
 * rows beyond capacity are dropped (whole iterations).  Outputs the number of
 * rows and recorded iterations. */
int dmrg_mlp_collect(dmrg_plan_t *p, const double *psi0, const dmrg_dav_opts_t *o, int64_t capacity,
                     float *x, float *a, float *b, int64_t *n_rows, int32_t *n_records, void *stream);
void dmrg_mlp_free(dmrg_mlp_t *m);

/* Profiling: when on, dmrg_apply_H records a hipEvent pair on its stream
 * around each tile launch of the first (1) and second (2) stage -- the wide
 * and the 64 x 64 work-group tile launches of split plans and the wavefront
 * tile launch, each with the algorithmic flops of its tiles (slicing launches
 * fall outside the pairs).  dmrg_get_profile waits for the recorded events
 * and returns the number of launches, their summed duration and summed
 * algorithmic flops since the last dmrg_set_profiling call, for stage 1 or 2
 * (all its tile launches), 11 or 12 (its 64 x 64 work-group tile launches
 * only), 21 or 22 (its wavefront tile launches only) or 31 or 32 (its wide
 * tile launches only). */
int dmrg_set_profiling(dmrg_plan_t *p, int32_t on);
int dmrg_get_profile(dmrg_plan_t *p, int32_t stage, int64_t *n_launches, double *total_ms,
                     double *total_flops);
void dmrg_plan_free(dmrg_plan_t *p);
const char *dmrg_last_error(void);

/* ---- renormalization of the left block through the left site ----------
 * After a two-site step the left block [0, l) and the site l merge into the
 * block [0, l] of the next bond (Sec. I: renormalized block operators are
 * formed during the contraction; Sec. II C: block x site tensor products,
 * each sector product scaled by the Eq. (4) factor C~ -- the W9j(l) role --
 * followed by the truncation).  The problem's left block (sectors, records,
 * DEVICE data), site_l, n_orb and integrals are the input; site_l >= 1.
 *
 * Product basis: the sectors of (left block) x (site) are the reachable
 * (N, 2S) pairs in ascending order; the rows of one are components
 * (left sector a, site multiplet m) in the order a ascending, then m = 0, 1,
 * 2, each d_a consecutive rows in the order of sector a's states
 * (dmrg_renorm_product lists them).  The caller keeps, per chosen product
 * sector, `kept` states given by a column-major rows x kept matrix U at
 * u_off of one DEVICE array (orthonormal columns in a DMRG sweep; any matrix
 * is accepted).  The new block's sectors are the keep entries, in their
 * order: (n, two_s, kept).
 *
 * Output: the families H, C, A0, A1, B0, B1, S (and with DMRG_RENORM_ALL_PAIRS
 * also P0, P1, Q0, Q1) of the new block (labels of a left
 * block at bond site_l + 1), as records in the input format -- one per
 * (family, row sector, column sector) with any contribution, all positions,
 * [npos][kept_row][kept_col] column-major -- in a caller-owned DEVICE array
 * of data_len elements.  Members of the new block whose labels lie in the
 * old one are [A (x) 1]; members with the label l are products of single
 * creation/annihilation operators; H is the Hamiltonian restricted to
 * [0, l], with the parts of two or more indices in the old block taken from
 * its S_l, P_ll and Q_ll; S_x (x > l) is S_x of the old block plus its P_xl
 * and Q_xl times single site operators plus explicit products.  P and Q of
 * the new block need P and Q of the old block for every outside pair, while
 * the H.psi input keeps only the pairs touching the two sites: with the flag
 * DMRG_RENORM_ALL_PAIRS the left block's P0, P1, Q0, Q1 records hold every
 * pair (x, y) of outside orbitals (x <= y, x < y for P1, lexicographic; the
 * other families as in the family table) and the new block's P, Q come out
 * in the same form, (P_xy)_ts = sum (xj|yl) a_lt a_js and
 * (Q_xy)_ts = delta_ts sum (xy|kl) E_kl - sum (xl|ky) a+_ks a_lt being those
 * of the old block plus their terms with an index at l.  Without the flag a
 * fam_mask naming P or Q is DMRG_EINVAL.
 *
 * Right block (flag DMRG_RENORM_RIGHT, the sweep's other direction): the
 * site r = site_l + 1 and the right block [r + 1, L) merge into the right
 * block [r, L) of bond site_l - 1 (Sec. II C: site x block, the W9j(r)
 * factor; coupled states ((r s) x (R S_R)) S, site first as in the two-site
 * basis; an R operator picks up (-1)^(its parity x the site's electrons)).
 * Product basis rows: components (site multiplet m, right sector b) in the
 * order m = 0, 1, 2, then b ascending (dmrg_renorm_product with the flag;
 * dmrg_rcomp_t.l_sec then names the right sector).  Output: H, C, S, P0, P1,
 * Q0, Q1 of a right block at bond site_l - 1, every one of them (the right
 * block's S, P, Q already cover every orbital and pair left of it).  Not
 * combined with DMRG_RENORM_ALL_PAIRS.
 *
 * dmrg_renorm_create builds the term and product lists on the host and
 * copies them to the device (hipMalloc, freed by dmrg_renorm_free); the
 * block's data pointer is kept until then and its contents must not change:
 * create also makes, on the null stream and waiting for them, a transposed
 * copy of the records applied as adjoints and the dressed operators (terms
 * that differ only in the position of their C factor merged into one term
 * on sum_j alpha_j C_j).  The lists' memory is about the first-stage
 * workspace (work_elems doubles) plus one block-data-sized buffer.
 * dmrg_renorm_apply transposes U per kept sector and runs the two FP64
 * product stages of the H.psi engine on `stream` (T = op(A) U rows, then
 * new = sum coef U^T T per output tile in a fixed order: bitwise
 * reproducible) and returns before they finish; calls on one handle must
 * not overlap (they share its workspace).  Errors: DMRG_EINVAL
 * (arguments, families), DMRG_ESYM (a kept (N, 2S) that is no product
 * sector), DMRG_ERANGE (U beyond u_len, outputs too small), DMRG_ENONFINITE
 * (integrals), DMRG_ENOMEM, DMRG_EHIP. */
typedef struct { int32_t n, two_s, kept, pad; int64_t u_off; } dmrg_rkeep_t;
typedef struct { int32_t sec, l_sec, site, row0, dim, pad; } dmrg_rcomp_t;
typedef struct dmrg_renorm dmrg_renorm_t;
typedef struct {
  int64_t n_terms;       /* coupled terms alpha [A (x) B]^K over all members */
  int64_t n_products1;   /* first-stage products op(A) U_rows               */
  int64_t n_products2;   /* second-stage products coef U_rows^T T           */
  int64_t n_tiles1, n_tiles2;
  int64_t work_elems;    /* first-stage workspace (doubles)                  */
  int64_t out_elems;     /* = data_len                                       */
  int64_t n_records;     /* output records                                   */
  double flops1, flops2; /* algorithmic 2mnk of the two stages               */
  double build_ms;
} dmrg_renorm_stats_t;
/* Sectors (n, two_s, rows) and components of the product basis.  Either
 * output may be NULL (counts only); DMRG_ERANGE when a capacity is short. */
int dmrg_renorm_product(const dmrg_problem_t *prob, int32_t flags, dmrg_sector_t *sec, int32_t sec_cap,
                        int32_t *n_sec, dmrg_rcomp_t *comp, int32_t comp_cap, int32_t *n_comp);
/* fam_mask: bit f for family f (0 = every family the flags allow); flags:
 * 0, DMRG_RENORM_ALL_PAIRS or DMRG_RENORM_RIGHT; u_len: elements of the U
 * array that dmrg_renorm_apply will be given. */
enum { DMRG_RENORM_ALL_PAIRS = 1, DMRG_RENORM_RIGHT = 2 };
int dmrg_renorm_create(const dmrg_problem_t *prob, const dmrg_rkeep_t *keep, int32_t n_keep, int32_t fam_mask,
                       int32_t flags, int64_t u_len, dmrg_renorm_t **out);
/* Output records (rec may be NULL to size) and the output length. */
int dmrg_renorm_records(const dmrg_renorm_t *r, dmrg_oprec_t *rec, int64_t cap, int64_t *n_rec, int64_t *data_len);
int dmrg_renorm_apply(dmrg_renorm_t *r, const double *u, double *out, void *stream);
int dmrg_renorm_stats(const dmrg_renorm_t *r, dmrg_renorm_stats_t *st);
/* Profiling as for plans: when on, dmrg_renorm_apply records a hipEvent pair
 * on its stream around the first-stage (1) and the second-stage (2) product
 * launch; dmrg_renorm_get_profile waits for them and returns the number of
 * launches, their summed duration and algorithmic flops since the last
 * dmrg_renorm_set_profiling call. */
int dmrg_renorm_set_profiling(dmrg_renorm_t *r, int32_t on);
int dmrg_renorm_get_profile(dmrg_renorm_t *r, int32_t stage, int64_t *n_launches, double *total_ms,
                            double *total_flops);
void dmrg_renorm_free(dmrg_renorm_t *r);

/* ---- truncation of a two-site step (the U of dmrg_renorm_create) -------
 * Sec. II (two-site DMRG; the truncation rule is left to the reviews the
 * paper cites): for every product sector (N, 2S) of (left block) x (left
 * site), rows as in the renormalization's product basis, the reduced density
 * matrix rho(a, a') = sum_c X_{a,c} X_{a',c}^T over the right parts c =
 * (r, right sector, 2S_rR) of the wavefunction blocks (psi: DEVICE, the
 * problem's reduced coefficients in the dmrg_psi_layout order) is formed on
 * the GPU tile engine and diagonalised with rocSOLVER (dsyevd) on `stream`;
 * the eigenvectors of the max_kept largest eigenvalues over all sectors
 * (eigenvalues <= cutoff dropped; ties by sector order, then rank) are kept.
 * Outputs: keep[n_keep] (host) in product-sector order, sectors without
 * kept states left out, u_off into u (DEVICE, u_len elements: per kept
 * sector a column-major rows x kept matrix, columns in descending eigenvalue
 * order, signs as the eigensolver returns them) -- exactly the input of
 * dmrg_renorm_create; weights[0] = kept eigenvalue sum, weights[1] = trace
 * (|psi|^2), if weights is not NULL.  With keep or u NULL only the sizes
 * (n_keep, u_len) and weights are returned; DMRG_ERANGE when keep_cap or
 * u_cap is short.  Device scratch (rho, lists, eigensolver workspace) is
 * taken with hipMalloc and freed before returning; the call waits for its
 * work on `stream`.  flags: 0, or DMRG_RENORM_RIGHT for the mirror -- the
 * sectors of (right site) x (right block) in the right renormalization's
 * product order, rho(b, b') = sum over left parts c = (left sector, l,
 * 2S_Ll) of X_{c,b}^T X_{c,b'}. */
int dmrg_truncate(const dmrg_problem_t *prob, int32_t flags, const double *psi, int32_t max_kept, double cutoff,
                  dmrg_rkeep_t *keep, int32_t keep_cap, int32_t *n_keep, double *u, int64_t u_cap,
                  int64_t *u_len, double *weights, void *stream);

/* ---- a left-to-right two-site sweep on the device -----------------------
 * Sec. II (two-site DMRG) and Sec. I (Davidson, then the renormalization):
 * at every bond p = bond0 .. n_orb - 2 the two-site problem of the current
 * left block and rights[p - bond0] is planned (dmrg_build_tasks with
 * plan_opts; NULL: the FP64 defaults; allocator callbacks apply to the plans) and
 * solved (dmrg_davidson with `dav`, NULL: defaults; start vector drawn from
 * `seed` and the bond); below the last bond the wavefunction is cut to at
 * most max_kept multiplets (dmrg_truncate) and the left block renormalized
 * in that basis (dmrg_renorm_*, DMRG_RENORM_ALL_PAIRS) into the left block
 * of bond p + 1.  `left` is the left block of bond0 in the all-pairs form;
 * rights[i] the right block of bond bond0 + i in the H.psi form; block data
 * are DEVICE arrays (borrowed), tables host arrays.  The blocks built on the
 * way stay in device memory; the H.psi form of each left block (P and Q of
 * the pairs at the two sites) is cut from its all-pairs records by device
 * copies.  steps[i] (host, n_orb - 1 - bond0 entries) receive the bond, the
 * Ritz value, the Davidson iterations, the kept multiplets and the kept
 * weight (last bond: kept 0, weight 1).  grown_out (host, as many entries
 * as steps, or NULL): entry i receives the block grown at step i -- the left
 * block of bond bond0 + i + 1 in the all-pairs form (the last entry stays
 * empty) -- with tables from malloc and device data from hipMalloc, owned by
 * the caller (dmrg_block_release); on an error none is returned.  Other
 * device memory is taken with hipMalloc and freed before returning; errors
 * as the calls it makes.
 *
 * dmrg_sweep_right_to_left is the mirror: bonds p = bond0 .. 0 (bond0 <=
 * n_orb - 3), `right` the right block of bond0, lefts[p] (p = 0 .. bond0)
 * the left block of bond p in the H.psi form or in the all-pairs form (the
 * blocks a left-to-right sweep returns); below bond 0 the
 * wavefunction is cut to multiplets of (right site x right block)
 * (DMRG_RENORM_RIGHT) and the right block renormalized into that of bond
 * p - 1.  steps[i] and grown_out[i] (bond0 + 1 entries) describe bond
 * bond0 - i; grown_out[i] is the right block of bond bond0 - i - 1. */
typedef struct {
  int32_t n_sec, pad;
  const dmrg_sector_t *sec;
  int64_t n_rec;
  const dmrg_oprec_t *rec;
  const double *data;          /* DEVICE */
  int64_t data_len;
} dmrg_block_t;
typedef struct {
  int32_t bond, kept;
  double energy, kept_weight;
  int32_t iters, pad;
} dmrg_sweep_step_t;
int dmrg_sweep_left_to_right(int32_t n_orb, int32_t n_elec, int32_t two_s, const double *h1, const double *eri,
                             int32_t bond0, const dmrg_block_t *left, const dmrg_block_t *rights,
                             int32_t max_kept, const dmrg_plan_opts_t *plan_opts, const dmrg_dav_opts_t *dav,
                             uint64_t seed, dmrg_sweep_step_t *steps, dmrg_block_t *grown_out, void *stream);
int dmrg_sweep_right_to_left(int32_t n_orb, int32_t n_elec, int32_t two_s, const double *h1, const double *eri,
                             int32_t bond0, const dmrg_block_t *lefts, const dmrg_block_t *right,
                             int32_t max_kept, const dmrg_plan_opts_t *plan_opts, const dmrg_dav_opts_t *dav,
                             uint64_t seed, dmrg_sweep_step_t *steps, dmrg_block_t *grown_out, void *stream);
/* Frees a block returned by a sweep (tables and device data) and empties it. */
void dmrg_block_release(dmrg_block_t *b);

/* ---- host-logic inspection (no GPU use; for tests of the host tables) ---- */
/* Wigner 6j {a b c; d e f}, 9j and the Eq. (4) factor, doubled spins.       */
double dmrg_wigner_6j(int a, int b, int c, int d, int e, int f);
double dmrg_wigner_9j(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp);
double dmrg_ctilde(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp);
/* Test-only host evaluation of the task list built for a problem whose
 * ldata/rdata are HOST arrays: y := sum over tasks of v A X D^T, computed with
 * plain loops on the CPU.  It checks the host tables without a GPU and is
 * never used by dmrg_apply_H.  */
int dmrg_debug_host_apply(const dmrg_problem_t *prob, const double *psi, double *y,
                          dmrg_plan_stats_t *st);
/* Test-only: build the device plan's tile and segment lists for one problem
 * with HOST operator data and execute them on the CPU with the kernels'
 * addressing (psi or y NULL: only fill *st).  Never used by dmrg_apply_H. */
int dmrg_debug_plan_host_apply(const dmrg_problem_t *prob, const double *psi, double *y,
                               const dmrg_plan_opts_t *opts, dmrg_plan_stats_t *st);
/* Test-only: per-tile work of stage 1 or 2 of the plan that opts (NULL:
 * defaults, FP64) give for one problem (operator data not read): rows (tile
 * rows and columns inside the output, segments, summed K, rows and columns of
 * the whole output block, tile kind: 1, 2, 4 wavefront, 8 work-group 64 x 64,
 * 16 wide 128 x 128) written to out[7 * i ..] for i < cap; returns the number
 * of tiles (call with out = NULL to size) or a negative status. */
int64_t dmrg_debug_plan_tiles(const dmrg_problem_t *prob, const dmrg_plan_opts_t *opts, int32_t stage,
                              int64_t *out, int64_t cap);
/* Test-only: the renormalization lists built as by dmrg_renorm_create for a
 * problem whose ldata is a HOST array, executed on the CPU with the kernels'
 * addressing (u, out HOST; out = NULL: statistics only); rec (may be NULL)
 * receives up to rec_cap output records. */
int dmrg_debug_renorm_host(const dmrg_problem_t *prob, const dmrg_rkeep_t *keep, int32_t n_keep, int32_t fam_mask,
                           int32_t flags, const double *u, int64_t u_len, double *out, int64_t out_len, dmrg_oprec_t *rec,
                           int64_t rec_cap, dmrg_renorm_stats_t *st);
/* Test-only: the density matrices of dmrg_truncate from a HOST psi, formed
 * on the CPU with the kernels' addressing: every product sector's rho in
 * product order, column-major rows x rows, concatenated (rho NULL: only the
 * length in *len). */
int dmrg_debug_truncate_rho_host(const dmrg_problem_t *prob, int32_t flags, const double *psi, double *rho,
                                 int64_t cap, int64_t *len);
/* Test-only: the host eigensolver dmrg_davidson applies to its projected
 * matrix (cyclic Jacobi).  A: m x m symmetric, row-major, HOST, 1 <= m <= 64;
 * w: m eigenvalues ascending; Z: m x m row-major, eigenvector j in column j.
 * Returns the number of Jacobi sweeps run (100 when the sweep limit stopped
 * it), or DMRG_EINVAL for m out of range or NULL pointers. */
int dmrg_debug_jacobi(int32_t m, const double *A, double *w, double *Z);

#ifdef __cplusplus
}
#endif
#endif
