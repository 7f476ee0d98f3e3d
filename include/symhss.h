/*
 * symhss: symmetric Muller-like HSS direct solver for 2-D Helmholtz
 * transmission scattering, on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper Section 2): find u (boundary trace of the field) and
 * q = (1/eps) du/dnu on a closed C^2 curve Gamma between an exterior medium
 * (k0, eps0) and an interior one (k1, eps1), for an incident wave u_in.
 * The discretisation (Section 3.1) is the N-point trapezoidal Nystrom rule
 * in the 2 pi-periodic parameter with one-point corrected diagonals; the
 * system (Section 3.2, eq. symmetric_muller) has 2N unknowns [q; u] and is
 * complex symmetric up to its free terms.  The solver (Section 4) compresses
 * every off-diagonal block with the proxy method and an interpolative
 * decomposition; with symmetry one ID per half-box serves as left and right
 * basis (eq. low-rank_R).
 *
 * A context may also hold a batch of boundaries (symhss_assemble_batch): the
 * boundaries are independent problems, each with its own medium, and every
 * tree level of all of them is compressed and factored in the same launches.
 * The unknowns of boundary t then occupy [2 B_t, 2 B_t + 2 N_t), with
 * B_t = N_0 + ... + N_{t-1}, each block in the order [q; u].
 *
 * Calling order: create -> assemble -> compress -> factor -> solve (any
 * number of times).  assemble invalidates later stages; calls out of order
 * return SYMHSS_ESTATE.  Every call returns a status and never aborts; the
 * message of the last failure is symhss_last_error().  A context is not
 * thread-safe: use one per host thread.  The context owns every device
 * allocation; the caller owns all arrays it passes, which are only read or
 * written during the call.
 */
#ifndef SYMHSS_H
#define SYMHSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct symhss_ctx symhss_ctx;

/* complex FP64, layout-compatible with C99 double _Complex and torch.complex128 */
typedef struct {
  double re, im;
} symhss_z;

typedef enum {
  SYMHSS_OK = 0,
  SYMHSS_EINVAL = 1,    /* bad argument: sizes, non-finite geometry, zero speed, k <= 0 */
  SYMHSS_ENOMEM = 2,    /* device or host allocation failed */
  SYMHSS_EDEVICE = 3,   /* HIP runtime error */
  SYMHSS_ESTATE = 4,    /* call out of order */
  SYMHSS_ESINGULAR = 5, /* zero pivot in a diagonal-block LU */
  SYMHSS_ERANK = 6,     /* proxy matrix beyond the ID kernel's limits */
  SYMHSS_ENOTCONV = 7   /* mixed-precision refinement reached its iteration limit above its
                           target; the outputs hold the last iterate */
} symhss_status;

typedef enum {
  /* eq. symmetric_muller, one-sided ID: L_i = R_i^T (the paper's method) */
  SYMHSS_MULLER_SYM = 0,
  /* eq. naive_muller (unscaled), two-sided ID of M_R and M_L (the paper's Base) */
  SYMHSS_MULLER_BASE = 1,
  /* ablation: the symmetric matrix compressed two-sided, symmetry unused */
  SYMHSS_MULLER_SYM_TWOSIDED = 2,
  /* eq. symmetric_pmchwt (row-scaled, exactly symmetric), one-sided ID.  Its
     N_k0, N_k1 are hypersingular: the one-point rule converges at O(h) */
  SYMHSS_PMCHWT_SYM = 3,
  /* eq. naive_pmchwt (unscaled), two-sided ID */
  SYMHSS_PMCHWT_BASE = 4,
  /* eq. bm (Section 6.1, alpha = i/k0), unscaled, two-sided ID.  Unknowns in
     the same [q; u] order as the other systems (the paper writes [u; q]);
     rows: exterior equation minus alpha times its normal derivative, then
     the interior equation; right-hand side [-(u_in + alpha q_in); 0] */
  SYMHSS_BURTON_MILLER = 5
} symhss_form;

/* Materials: k_i = omega sqrt(eps_i) > 0 (Section 2); eps_i > 0. */
typedef struct {
  double k0, k1, eps0, eps1;
} symhss_medium;

typedef struct {
  int32_t leaf;        /* points per leaf box (>= 8); tree levels L = ceil(log2(N/leaf)) */
  int32_t form;        /* symhss_form */
  double tol;          /* relative ID tolerance: rank = #{j : |R_jj| > tol |R_00|}, > 0 */
  int32_t n_proxy;     /* minimum proxy points per circle (e.g. 64) */
  int32_t root_max;    /* top of the tree: compression stops at the first level (from the
                          leaves) whose boxes' ranks sum to at most root_max, and that level's
                          compressed system is factored densely; 0: default 2048; < 0: compress
                          every level down to level 1 (two boxes at the root) */
  double proxy_ratio;  /* proxy radius / box radius (e.g. 1.5) */
} symhss_opts;

/* Flag for solve/rhs/matvec: arrays are device pointers (HBM) rather than host. */
#define SYMHSS_DEVICE_PTRS 1

/* Create a context on HIP device `device`; `hip_stream` (a hipStream_t) may
 * be NULL, in which case the context creates its own stream. */
symhss_status symhss_create(symhss_ctx **out, int device, void *hip_stream);
void symhss_destroy(symhss_ctx *ctx);
/* Message of the last failed call on ctx; with ctx == NULL, of the last failed
 * symhss_create on this thread. */
const char *symhss_last_error(const symhss_ctx *ctx);
/* The stream all work is queued on (a hipStream_t). */
void *symhss_stream(symhss_ctx *ctx);

/* Discretisation (Section 3.1).  theta_j = 2 pi j / N, j = 0..N-1, counter-
 * clockwise.  x, dx, ddx: host arrays of N x 2 interleaved doubles holding
 * x(theta_j), x'(theta_j), x''(theta_j); copied to the device.  Computes the
 * normals (into the exterior), curvature and weights w_j = |x'_j| 2 pi / N on
 * the GPU and builds the box tree.  EINVAL for N < 2 leaf, non-finite values,
 * |x'| = 0, k or eps <= 0, tol <= 0. */
symhss_status symhss_assemble(symhss_ctx *ctx, int64_t n, const double *x, const double *dx, const double *ddx,
                              const symhss_medium *medium, const symhss_opts *opts);

/* Batch of `count` independent boundaries (Section 4.1's partition per
 * boundary; the boundaries do not interact).  n[t]: nodes of boundary t;
 * x, dx, ddx: the boundaries' node arrays (as for symhss_assemble) one after
 * another, sum(n) x 2 doubles each; media[t]: its materials.  One option set
 * for all.  Levels are counted from the leaves of the deepest boundary.
 * EINVAL as for symhss_assemble, per boundary. */
symhss_status symhss_assemble_batch(symhss_ctx *ctx, int32_t count, const int64_t *n, const double *x,
                                    const double *dx, const double *ddx, const symhss_medium *media,
                                    const symhss_opts *opts);

/* Proxy-method compression (Section 4.1), levels L..1: generates M_R (and
 * M_L for the two-sided forms) on the GPU and computes the column-pivoted
 * QR IDs of their halves.  A compress that fails leaves the context
 * assembled only (factor and solve return SYMHSS_ESTATE until a compress
 * succeeds). */
symhss_status symhss_compress(symhss_ctx *ctx);

/* Compressed-equation factorisation (Section 4.2): per box LU of the
 * diagonal block D, X = D^{-1} L, A~ = (R X)^{-1}; parent blocks
 * [[A~_c1, S_c1c2], [S_c2c1, A~_c2]]; dense LU at the root.  ESINGULAR on a
 * zero pivot.  A factor that fails leaves the context compressed (solve
 * returns SYMHSS_ESTATE until a factor succeeds). */
symhss_status symhss_factor(symhss_ctx *ctx);

/* symhss_factor followed by symhss_solve, with the same results and errors
 * (ESINGULAR on a zero pivot is reported after x was written).  With the
 * factorisation pipelined during compress (SYMHSS_OPT_PIPELINE, FP64, no
 * graphs) the solve's sweep up the levels runs while the top-level LU
 * (Section 4.2, the dense root system) is still being computed, and waits
 * for it only before its top-level part; otherwise the two calls run one
 * after the other.  Arguments as for symhss_solve. */
symhss_status symhss_factor_solve(symhss_ctx *ctx, const symhss_z *b, symhss_z *x, int32_t nrhs, int32_t flags);

/* Solve A x = b for nrhs right-hand sides.  b and x are 2N x nrhs column-
 * major in the block order [q; u] and the scaling of the chosen form (row-
 * scaled for SYMHSS_MULLER_SYM* and SYMHSS_PMCHWT_SYM, unscaled for the
 * others).  Host
 * pointers unless flags has SYMHSS_DEVICE_PTRS.  b and x may not overlap. */
symhss_status symhss_solve(symhss_ctx *ctx, const symhss_z *b, symhss_z *x, int32_t nrhs, int32_t flags);

/* Physical interface (Section 2, the transmission conditions that close the
 * exterior and interior problems): from the incident field's boundary data
 * u_in and q_in = du_in/dnu at the nodes, solve the chosen form's system and
 * return the boundary traces q and u of the solution (the unknowns [q; u]).
 * The result does not depend on the form beyond its discretisation error.
 * uin, qin, q, u: N x nrhs column-major (N = all nodes of a batch, boundary t
 * at rows [B_t, B_t + N_t)); host pointers unless flags has
 * SYMHSS_DEVICE_PTRS.  Inputs and outputs may not overlap.  ESTATE before
 * factor; ENOTCONV as for symhss_solve. */
symhss_status symhss_solve_incident(symhss_ctx *ctx, const symhss_z *uin, const symhss_z *qin, symhss_z *q,
                                    symhss_z *u, int32_t nrhs, int32_t flags);

/* Incident plane wave at the nodes: u_in = exp(i k0 (cos a x1 + sin a x2)) and
 * q_in = du_in/dnu, with a = angles[t] on boundary t (one angle for a single
 * boundary); uin, qin: N values each (host pointers unless
 * SYMHSS_DEVICE_PTRS).  Valid after assemble. */
symhss_status symhss_plane_wave(symhss_ctx *ctx, const double *angles, symhss_z *uin, symhss_z *qin,
                                int32_t flags);

/* Right-hand side of the chosen form for the plane wave
 * u_in = exp(i k0 (cos a x1 + sin a x2)), q_in = du_in/dnu:
 * b = [-eps0 W u_in; W q_in] (eq. symmetric_muller) or [-eps0 u_in; q_in];
 * PMCHWT [-W u_in; W q_in / eps0] (W = I unscaled); Burton-Miller
 * [-(u_in + alpha q_in); 0]. */
symhss_status symhss_rhs_plane_wave(symhss_ctx *ctx, double angle, symhss_z *b, int32_t flags);

/* Plane-wave right-hand sides of a batch: angles[t] for boundary t (the
 * layout of symhss_solve).  symhss_rhs_plane_wave uses one angle for all. */
symhss_status symhss_rhs_plane_wave_batch(symhss_ctx *ctx, const double *angles, symhss_z *b, int32_t flags);

/* Verification: entries A[rows][:, cols] of the 2N x 2N system (indices
 * < N: first equation / q unknown of node i; N + i: second equation / u
 * unknown), out is nr x nc column-major, host memory.  Valid after assemble.
 * For a batch, indices are global unknowns and entries that couple two
 * boundaries are zero. */
symhss_status symhss_eval_entries(symhss_ctx *ctx, int64_t nr, const int64_t *rows, int64_t nc,
                                  const int64_t *cols, symhss_z *out);

/* Verification: J0, Y0, J1, Y1, Y1 + 2/(pi z) at n points z > 0 (out: 5n
 * doubles), evaluated by the device code used for the kernel entries. */
symhss_status symhss_eval_bessel(symhss_ctx *ctx, int64_t n, const double *z, double *out);

/* y = A x with every entry generated on the fly in FP64 (no storage; O(N^2)
 * work per boundary; block-diagonal for a batch).  x, y: 2N complex; host
 * pointers unless SYMHSS_DEVICE_PTRS. */
symhss_status symhss_matvec_direct(symhss_ctx *ctx, const symhss_z *x, symhss_z *y, int32_t flags);

/* Execution options; value in brackets is the default.
 *  SYMHSS_OPT_GRAPHS      [0] 1: the second time a compressed structure is
 *       factored (with SYMHSS_OPT_PIPELINE off), its launch sequence is
 *       captured as a HIP graph and every later factorisation of the same
 *       structure replays it; likewise a
 *       device-pointer solve repeated with the same vectors and nrhs.  Kernel
 *       timings in the statistics are not collected for replays.
 *  SYMHSS_OPT_AUTOTUNE    [0] 1: the first ID and LU launch of each size bucket
 *       (count, rows, columns), and the first product of the solve sweeps with
 *       at most four right-hand sides in each bucket (64 x 64 matrix-core tile
 *       or the skinny 64-row kernel), times every launch variant on the real
 *       data (restored between trials) and keeps the fastest.  The variants
 *       compute the same pivoted QR with different summation orders (the
 *       ID also as a blocked QR followed by the pivoted QR of its triangle),
 *       so ranks and skeletons agree up to rounding.
 *  SYMHSS_OPT_PERSISTENT [-1] ID kernel: -1 automatic (the blocked QR and
 *       the pivoted QR of its triangle in registers for proxy matrices of at
 *       most 512 rows and 128 columns, else the one-stage kernel); 0 the
 *       one-stage kernel with one workgroup per matrix, 1 the one-stage
 *       kernel as a persistent grid taking matrices from a work queue.
 *  SYMHSS_OPT_PREDICTOR   [0] 1: proxy counts from the rank predictor (below).
 *  SYMHSS_OPT_PROXY_MARGIN [16] proxy points added to the predicted rank.
 *  SYMHSS_OPT_PRECISION   [0] 1: mixed precision.  The IDs and every kernel
 *       block stay FP64; the generated blocks are kept, and with the FP64
 *       interpolation matrices form the FP64 HSS representation.  The
 *       factorisation (diagonal-block LUs, X, A~, top-level systems) and the
 *       solve sweeps run in complex FP32 on the FP32 roundings, and
 *       symhss_solve refines: x += FP32 solve of r, r = b - A_HSS x in FP64,
 *       until |r| / |b| <= 10^-digits (every right-hand side) or the
 *       iteration limit.  Changing it requires a new symhss_factor.
 *  SYMHSS_OPT_REFINE_DIGITS [10] the refinement target 10^-digits (1..15).
 *  SYMHSS_OPT_REFINE_MAXIT  [10] the refinement iteration limit (1..100).  A
 *       solve whose residual is still above the target after the last
 *       iteration (or not finite) returns SYMHSS_ENOTCONV with x holding the
 *       last iterate.
 *  SYMHSS_OPT_RANK_LEAF    [0] k_L > 0: fixed-rank schedule (Section 4.3):
 *       every ID of a box at level l of its boundary's tree (leaves at level
 *       L) has rank min(round(k_L a^(L - l)), columns, rows) per half, instead
 *       of the tolerance rule; 0: tolerance mode.
 *  SYMHSS_OPT_RANK_SCALE [1000] the growth a per level, times 1000 (1000..4000).
 *       Both require a new symhss_compress.
 *  SYMHSS_OPT_PIPELINE    [1] 1: (either precision) symhss_compress already queues
 *       each level's factorisation on a second stream as soon as the level's
 *       IDs are known (it overlaps the planning of the next level);
 *       symhss_factor then adds the top-level systems and waits.  Such a
 *       factorisation is not captured as a graph (solves still are).
 * EINVAL for an unknown option or value. */
#define SYMHSS_OPT_GRAPHS 0
#define SYMHSS_OPT_AUTOTUNE 1
#define SYMHSS_OPT_PERSISTENT 2
#define SYMHSS_OPT_PREDICTOR 3
#define SYMHSS_OPT_PROXY_MARGIN 4
#define SYMHSS_OPT_PRECISION 5
#define SYMHSS_OPT_REFINE_DIGITS 6
#define SYMHSS_OPT_REFINE_MAXIT 7
#define SYMHSS_OPT_RANK_LEAF 8
#define SYMHSS_OPT_RANK_SCALE 9
#define SYMHSS_OPT_PIPELINE 10
/*  SYMHSS_OPT_DEVICE_LIMIT [0] bytes of device memory the context's work
 *       buffers may hold (0: no limit).  A call that would allocate beyond it
 *       fails with SYMHSS_ENOMEM; a compress or factor that fails leaves the
 *       context assembled (resp. compressed), so that later stages return
 *       SYMHSS_ESTATE until it is run again.  Small staging chunks for launch
 *       descriptors are not counted. */
#define SYMHSS_OPT_DEVICE_LIMIT 11
symhss_status symhss_configure(symhss_ctx *ctx, int32_t option, int64_t value);

/* Rank predictor (sizes fixed before the factorisation runs, Section 4.3):
 * a 6 -> 64 -> 64 -> 64 -> 1 ReLU network in FP32 predicting log(rank) of a
 * box, the larger of its two halves' ranks, from its features
 *   (k_out d, k_in d, mean |kappa| d, max |kappa| d, level, log10 tol),
 * d = box diameter (twice the largest distance of its nodes from the
 * bounding-box midpoint), kappa = curvature at its nodes, level = the box's
 * level in its boundary's tree.  Features are float, 6 per sample, row-major.
 *
 * Weights: SYMHSS_PREDICTOR_WEIGHTS floats = the 8833 network parameters
 * (W1 64x6 row-major, b1, W2 64x64, b2, W3 64x64, b3, W4 1x64, b4) followed
 * by the 6 feature means and 6 feature scales used to normalise inputs.
 *
 * With SYMHSS_OPT_PREDICTOR = 1 (weights loaded or trained), compress sizes
 * each box's proxy circle from its predicted rank k^:
 *   n_p = min(rule, roundup16(max(32, ceil(k^) + margin))),
 * margin = SYMHSS_OPT_PROXY_MARGIN [16], rule = the count used without the
 * predictor; a box whose measured rank exceeds k^ is compressed again with
 * the rule's count (the adaptive column-pivoted QR stays the judge). */
#define SYMHSS_PREDICTOR_WEIGHTS 8845
typedef struct {
  int32_t epochs;  /* passes over the samples (>= 1) */
  int32_t batch;   /* mini-batch size (>= 1) */
  float lr;        /* Adam step size (> 0); beta1 0.9, beta2 0.999, eps 1e-8 */
  float alpha;     /* weight of under-predicted samples in the loss (>= 1) */
  uint64_t seed;   /* initialisation and shuffling */
} symhss_train_params;

/* Train on the GPU from n samples (feat: n x 6, rank: n values >= 1); the
 * loss is (1/B) sum c_s (yhat_s - log rank_s)^2 per mini-batch of B, with
 * c_s = alpha for under-predictions and 1 otherwise.  history (may be NULL):
 * epochs floats, the mean mini-batch loss of each epoch.  The trained
 * weights stay in the context. */
symhss_status symhss_predictor_train(symhss_ctx *ctx, const float *feat, const float *rank, int64_t n,
                                     const symhss_train_params *hp, float *history);
/* Load / read SYMHSS_PREDICTOR_WEIGHTS floats (host memory). */
symhss_status symhss_predictor_load(symhss_ctx *ctx, const float *weights, int64_t count);
symhss_status symhss_predictor_get(symhss_ctx *ctx, float *weights, int64_t count);
/* rank_out[s] = exp(network(feat[s])) for n samples (host memory). */
symhss_status symhss_predictor_predict(symhss_ctx *ctx, const float *feat, int64_t n, float *rank_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): symhss_predictor_predict with device
 * pointers (feat: n x 6 floats, rank_out: n floats, both in HBM), queued on
 * the context's stream and returning without waiting for it.  The network's
 * activations live in a fixed scratch array in the library's device memory
 * (SYMHSS_PREDICT_NOALLOC_MAX samples, about 6.5 MB per device, held until
 * the process ends); nothing is allocated, copied to the host or
 * synchronised.  EINVAL for n < 0 or n > SYMHSS_PREDICT_NOALLOC_MAX; n = 0 does
 * nothing.  Features are not checked: a non-finite feature gives a
 * non-finite rank.  Every context on a device shares that device's scratch:
 * calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race and must be ordered by the caller. */
#define SYMHSS_PREDICT_NOALLOC_MAX 8192
symhss_status symhss_predictor_predict_noalloc(symhss_ctx *ctx, const float *feat, int64_t n, float *rank_out);
/* Training data after compress: for every compressed box (heights from the
 * leaves up, boundaries in order within a height) its 6 predictor features
 * (feat, count x 6), its measured rank, the larger of its halves' ranks
 * (rank), and info (count x 6 int32: boundary, level in its boundary's tree,
 * first node, one past the last node, proxy count used, predicted rank or 0).
 * Any output may be NULL; with all NULL only *count is set, otherwise *count
 * must hold the capacity (EINVAL if too small) and receives the count. */
symhss_status symhss_box_table(symhss_ctx *ctx, int64_t *count, float *feat, int32_t *rank, int32_t *info);

/* Verification: loss and its gradient (8833 floats) over all n samples as one
 * batch, for the given weights (SYMHSS_PREDICTOR_WEIGHTS floats); replaces the
 * context's weights with them. */
symhss_status symhss_predictor_grad(symhss_ctx *ctx, const float *weights, const float *feat, const float *rank,
                                    int64_t n, float alpha, float *grad, float *loss);

/* Verification (mixed precision, after factor): y = A_HSS x, the FP64
 * product of the compressed representation that drives the refinement;
 * x, y: 2N complex, host pointers unless SYMHSS_DEVICE_PTRS.  ESTATE in FP64
 * mode (the generators are not kept there). */
symhss_status symhss_hss_matvec(symhss_ctx *ctx, const symhss_z *x, symhss_z *y, int32_t flags);

/* Statistics of the last assemble/compress/factor/solve. */
typedef struct {
  int32_t levels;            /* L */
  int32_t leaf_boxes;        /* 2^L */
  int32_t root_size;         /* order of the dense top-level system (largest of a batch) */
  int32_t form;
  int64_t entries_compress;  /* matrix entries generated by compress */
  int64_t entries_factor;    /* matrix entries generated by factor */
  double t_compress, t_factor, t_solve;          /* seconds, host wall clock incl. sync */
  double t_kblock_compress, t_kblock_factor;     /* seconds in the kernel-block generator (HIP events) */
  double t_id, t_lu;                             /* seconds in ID and LU kernels (HIP events) */
  int64_t device_bytes;
  int32_t rank_min[32], rank_max[32]; /* per level (index = level), q + u rank of a box */
  double rank_mean[32];
  int32_t proxy_max[32];     /* largest proxy count per level */
  int32_t n_kblock, n_id, n_lu;  /* timed launches behind t_kblock_*, t_id, t_lu */
  int32_t root_level;        /* level whose boxes form the dense top-level system (batch: the
                                highest such level) */
  /* algorithmic work of the timed launches (FP64 real flops; bytes written) */
  double flops_id;           /* pivoted QR steps and T = R11^-1 R12 of the IDs */
  double flops_lu_batched;   /* one-workgroup-per-block LU launches (k_lu_fused) */
  double flops_lu_multi;     /* multi-workgroup LU (top levels and the dense top system) */
  double t_lu_batched, t_lu_multi;  /* seconds, HIP events; t_lu = their sum */
  int32_t n_lu_batched, n_lu_multi;
  double bytes_kblock;       /* 16 bytes per generated entry (compress + factor) */
  int32_t graph_replays;     /* factorisations and solves served by a HIP graph since assemble */
  int32_t tuned_buckets;     /* size buckets the autotuner has settled */
  /* predictor-sized compression (last compress) */
  int32_t pred_boxes;        /* boxes whose proxy count came from the predictor */
  int32_t pred_fallbacks;    /* of those, compressed again with the rule's count */
  int64_t proxy_rows;        /* proxy-matrix rows generated (all passes) */
  int64_t proxy_rows_rule;   /* rows the rule's counts would have generated */
  double proxy_bytes;        /* bytes of the proxy matrices generated (all passes) */
  double proxy_bytes_rule;   /* bytes with the rule's counts */
  /* mixed precision (last solve) */
  int32_t refine_iters;      /* FP32 solves performed */
  int32_t pad0;
  double fp32_residual;      /* |b - A_HSS x| / |b| after the first FP32 solve */
  double refine_residual;    /* the same after the last one */
  double t_compress_wait;    /* of t_compress, seconds the host waited for the GPU */
  /* host-side work of the last compress (seconds, wall clock, waits excluded) */
  double t_host_plan;        /* active sets, proxy circles, near fields, next level's boxes */
  double t_host_ids;         /* proxy points, index unions, kernel-block and ID descriptors */
  double t_host_post;        /* skeletons, interpolation descriptors, child maps */
  double t_host_factor;      /* queueing each level's factorisation (pipelined factor) */
} symhss_stats;

symhss_status symhss_get_stats(const symhss_ctx *ctx, symhss_stats *out);

/* Verification: data of one box after compress.  The box is the box-th of
 * all boxes at `level` (boundaries of a batch one after another, each in
 * curve order).  `what` selects:
 *  0/1  active column node ids (q / u half)      2/3  active row node ids (eq 1 / eq 2)
 *  4/5  column skeleton, local indices (q / u)    6/7  row skeleton, local indices
 *  8    dense column interpolation R (kc x sc, complex, column-major)
 *  9    dense row interpolation L (sr x kr)
 *  10   proxy circle: centre x, centre y, radius, count (4 doubles)
 *  11/12 near row node ids (eq 1 / eq 2)          13/14 near column node ids (q / u)
 *  15   ranks kc_q, kc_u, kr_q, kr_u (4 int32)
 *  16   boundary, index within the boundary's boxes at this level, first node,
 *       one past the last node, 1 if the box is part of its boundary's dense
 *       top-level system (5 int32)
 * Element type: int32 for ids/indices/ranks, symhss_z for 8/9, double for 10.
 * With out == NULL only *count is set; otherwise out must hold *count elements. */
symhss_status symhss_box_query(symhss_ctx *ctx, int32_t level, int32_t box, int32_t what, int64_t *count,
                               void *out);

#ifdef __cplusplus
}
#endif

#endif /* SYMHSS_H */
