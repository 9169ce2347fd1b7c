/*
 * fmm.h -- C ABI of the MI355X 3-D Laplace fast multipole library.
 *
 * The operation (Yokota, Ibeid, Keyes, "Fast Multipole Method as a Matrix-Free
 * Hierarchical Low-Rank Approximation", Sec. 1): for N points x_i that are both
 * sources and targets, with charges q_i,
 *
 *     phi_i  = sum_{j != i, x_j != x_i} q_j / |x_i - x_j|        (no 4*pi)
 *     grad_i = d phi / d x_i  (the gradient of phi, not the field -grad phi)
 *
 * approximated by the FMM: a hierarchical octree decomposition with multipole
 * and local expansions of order p for the far field, and a direct sum over
 * neighbouring leaves for the near field.  The paper treats the FMM as a
 * matrix-free H^2 mat-vec whose set-up and application are timed separately
 * (Sec. 1; Sec. 4.1), and asks for a split between the hierarchical structure
 * and the inner kernels (Sec. 5); hence a plan (octree + interaction lists,
 * Sec. 2.2) built once per point set and applied to any number of charge
 * vectors.
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers on the current HIP device, owned by
 *     the caller, FP32, contiguous, row-major.  points/gradients are [n][3].
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *     is asynchronous on that stream except fmm_plan, which synchronises the
 *     stream a few times to read counts back to the host.
 *   - Errors are returned as fmm_status; nothing crosses the ABI as an
 *     exception.  fmm_last_error() gives a thread-local message for the last
 *     failing call on the calling thread.
 *   - Results are deterministic: the same inputs give bit-identical outputs.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s *fmm_plan_t;

typedef enum {
    FMM_OK = 0,
    FMM_EINVAL = 1,       /* bad argument (n < 1, ncrit < 1, p outside [0,16], theta outside (0, 1/sqrt 3), NULL pointer) */
    FMM_ENOMEM = 2,       /* the allocator returned NULL */
    FMM_EDEVICE = 3,      /* a HIP runtime call failed */
    FMM_ENONFINITE = 4,   /* a coordinate is NaN or infinite */
    FMM_EUNSUPPORTED = 5  /* geometry outside the library's limits (e.g. an M2L offset too large to key) */
} fmm_status;

typedef enum {
    FMM_PREC_FP32 = 0,    /* FP32 everywhere (M2L on FP32 MFMA) */
    FMM_PREC_MIXED = 1    /* split-FP16 M2L on MFMA with FP32 accumulation, compensated FP32 P2P,
                             FP64 coefficient accumulation at the root levels */
} fmm_precision;

/* Phase mask for fmm_eval_ex */
#define FMM_NEAR 1        /* near field only: P2P over neighbouring leaves */
#define FMM_FAR 2         /* far field only: P2M, M2M, M2L, L2L, L2P */
#define FMM_ALL 3

/*
 * Device allocator used for every plan workspace (the paper stresses that the FMM's memory
 * is O(N), Sec. 4.1: all of it is workspace of the plan, obtained here).  alloc returns
 * NULL on failure (the call then fails with FMM_ENOMEM); release takes back a pointer
 * that alloc returned.  `stream` is the stream the block is first used on, and the block
 * may be reused by its owner in that stream's order once released:
 *   - fmm_plan and its variants: the plan call's stream, except the near-field lists,
 *     which are built on the library's own per-device side stream and allocated (and,
 *     when they are temporaries, released) with that stream;
 *   - the scratch that the adjoint and Hessian calls add to a plan on first use: the
 *     stream of that call.
 * Blocks still held by a plan are released by fmm_plan_destroy after every stream the
 * plan was used on has been synchronised.  Passing NULL for both restores the default: a
 * process-wide caching allocator over hipMalloc (blocks are kept for reuse and not
 * returned to the driver).  Plans keep the allocator that was current when they were
 * built.  The Python binding installs PyTorch's caching allocator here.  The operator
 * tables (a process-wide cache per expansion order) and the pinned host mailboxes are
 * the library's own and do not go through this allocator.
 */
typedef void *(*fmm_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*fmm_free_fn)(void *ptr, void *stream, void *ctx);
fmm_status fmm_set_allocator(fmm_alloc_fn alloc, fmm_free_fn release, void *ctx);

/*
 * Build a plan for `n` points (device [n][3] FP32).
 *   ncrit  >= 1   a cell is split while it holds more than ncrit points (and is above level 21)
 *   p in [0, 16]  expansion order: spherical harmonics of degree 0..p, (p+1)^2 coefficients
 *   theta         opening angle of the multipole acceptance criterion: the pair (A <- B) is
 *                 far iff A != B and theta*|c_A - c_B| >= R_A + R_B (R = half box side);
 *                 0 < theta < 1/sqrt(3) so that accepted pairs are always convergent
 *   prec          FMM_PREC_FP32 or FMM_PREC_MIXED
 * On success *out owns all plan memory (allocated through the current allocator on
 * `stream`).  The plan copies what it needs from `points`; the buffer may be reused
 * after the call returns.
 */
fmm_status fmm_plan(const float *points, int64_t n, int ncrit, int p, float theta,
                    fmm_precision prec, void *stream, fmm_plan_t *out);

/*
 * fmm_plan with a variable-order M2L (the paper notes that expansions whose order varies
 * with the separation, or low-rank (SVD) operators, cut the M2L work; Sec. 2.2).
 *   m2l_tol >= 0  every M2L operator is applied in 16 x 16 blocks; a block is left out
 *                 when it is among the smallest blocks of that operator whose summed
 *                 size stays within m2l_tol, the size of a block being what it can add to
 *                 a potential (entries weighted by the bounds h^n / sqrt((n+m)!(n-m)!) of
 *                 the source's multipole and the target's local coefficients, h = sqrt(3)/2)
 *                 relative to the interaction's monopole-to-monopole term.  So every M2L
 *                 pair's potential changes by at most m2l_tol of its monopole term.
 *                 0 keeps every block (same result as fmm_plan).  FP32 precision only.
 *   lists         FMM_LISTS_DUAL: the dual traversal of fmm_plan (a pair of cells at the same
 *                 level that fails the MAC is replaced by all pairs of their children);
 *                 FMM_LISTS_LEVEL_SKIP: only the cell with the smaller Morton prefix is split,
 *                 so that distant members of a list can be served by their parent (the
 *                 paper's level-skip remark, Sec. 2.2); fewer M2L pairs, same MAC, pair sets
 *                 still symmetric.
 * Other arguments, ownership and errors as fmm_plan; EINVAL for a negative, NaN or
 * infinite m2l_tol, m2l_tol > 0 with FMM_PREC_MIXED, or an unknown lists value.
 */
/*
 * fmm_plan with SVD-compressed M2L operators (the paper: an SVD of the translation matrices
 * gives what expansions of varying order give, systematically; Sec. 2.2, Sec. 5).  Every
 * operator A (one per relative offset) is replaced by a rank-r product Pf Qf from the SVD of
 * W A W, W = diag(h^n / sqrt((n+m)!(n-m)!)) with h = sqrt(3)/2 (the bounds of a multipole
 * coefficient of degree n per unit charge, and of a local coefficient's reach on the
 * potential): singular values at or below svd_tol times the largest are dropped.  M2L then
 * applies two products per pair, Qf (r x (p+1)^2) and Pf ((p+1)^2 x r), r rounded up to a
 * multiple of 16.  0 < svd_tol < 1; FP32 precision; other arguments, ownership and errors
 * as fmm_plan (EINVAL for svd_tol outside [0, 1)).  svd_tol = 0 is fmm_plan.  The factors
 * are computed on the host (all cores) on first use of a (p, key, svd_tol) and cached for
 * the life of the process.
 */
fmm_status fmm_plan_svd(const float *points, int64_t n, int ncrit, int p, float theta, double svd_tol,
                        void *stream, fmm_plan_t *out);

#define FMM_LISTS_DUAL 0
#define FMM_LISTS_LEVEL_SKIP 1
fmm_status fmm_plan_ex(const float *points, int64_t n, int ncrit, int p, float theta,
                       fmm_precision prec, double m2l_tol, int lists, void *stream, fmm_plan_t *out);

/*
 * Apply the plan to charges q (device [n]): potential (device [n]) and, when
 * `gradient` is not NULL, grad phi (device [n][3]).  Outputs are in input order.
 * Calls that share one plan must not overlap (the plan holds the work buffers).
 */
fmm_status fmm_eval(fmm_plan_t plan, const float *charges, float *potential, float *gradient, void *stream);

/* As fmm_eval, restricted to the phases in `phases` (FMM_NEAR | FMM_FAR). */
fmm_status fmm_eval_ex(fmm_plan_t plan, const float *charges, float *potential, float *gradient,
                       int phases, void *stream);

/*
 * Adjoint of L = sum_i w_i phi_i with w = dL_dphi (device [n]), for the frozen plan.  The
 * paper treats the FMM as a matrix-free application of a fixed (H^2) matrix (Sec. 1); for a
 * fixed plan that matrix A is symmetric (symmetric pair sets, symmetric truncation), so
 * its transpose is applied by the same FMM, and the plan is recomputed in the backward
 * pass rather than stored (the compute-over-memory argument of Sec. 1):
 *   dL_dq[i]  = sum_k w_k A_ki  = (A w)_i            (A is symmetric: the same FMM with charges w)
 *   dL_dx[i]  = w_i grad phi(x_i) + q_i grad psi(x_i),  psi = A w
 * gradient_fwd is grad phi from fmm_eval with `charges` ([n][3]); when NULL it is recomputed.
 * dL_dq is [n], dL_dx is [n][3]; either may be NULL to skip it.
 */
fmm_status fmm_adjoint(fmm_plan_t plan, const float *charges, const float *gradient_fwd,
                       const float *dL_dphi, float *dL_dq, float *dL_dx, void *stream);

/*
 * fmm_adjoint for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same arguments,
 * results and errors as fmm_adjoint, but the call allocates nothing: the adjoint's
 * scratch (psi when dL_dq is NULL, grad psi, and grad phi when gradient_fwd is NULL; 7
 * floats per point) lives in a static device array of the library, FMM_NOALLOC_MAX_N * 7
 * floats (28 MiB), that each GPU the library runs on holds until the process ends; its
 * address is looked up once per device on the first call there.  The plan must have been
 * built beforehand (fmm_plan allocates).  FMM_EINVAL when the plan has more than
 * FMM_NOALLOC_MAX_N points, or when the current device is not the plan's.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (on different streams,
 * from different threads or for different plans) race.  Nothing in the array has to start
 * at zero (every value is written before it is read).
 */
#define FMM_NOALLOC_MAX_N ((int64_t)1 << 20)
fmm_status fmm_adjoint_noalloc(fmm_plan_t plan, const float *charges, const float *gradient_fwd,
                               const float *dL_dphi, float *dL_dq, float *dL_dx, void *stream);

/*
 * Potential, gradient and Hessian of the potential at every point (the Hessian is what
 * the adjoint of a loss through grad phi needs).  hessian: device [n][6], order xx, yy,
 * zz, xy, xz, yz (symmetric); potential and gradient may be NULL.  The second derivatives
 * come from the same tree and lists: L2P differentiates the local expansions twice
 * (degree <= p-2 terms), the near field uses the exact kernel q (3 d d^T/r^5 - I/r^3).
 * FP32 near field for both precisions.
 */
fmm_status fmm_eval_hessian(fmm_plan_t plan, const float *charges, float *potential, float *gradient, float *hessian,
                            void *stream);

/*
 * Field of charges and dipoles (Sec. 1, with the source positions as variables: a dipole
 * g at x_j is the derivative of a unit charge's field as x_j moves along g):
 *   phi_i  = sum_{j != i, x_j != x_i} q_j / |d| + g_j . d / |d|^3,   d = x_i - x_j,
 *   grad_i = its gradient in x_i.
 * charges [n], dipoles [n][3] (device, FP32, input order); potential [n] and gradient
 * [n][3] as in fmm_eval (either may be NULL, not both).  Same plan, tree and lists: P2M
 * adds each dipole's multipole (the derivative of its charge's), the near field the exact
 * dipole kernel.  EINVAL for NULL pointers or a plan made by fmm_plan_targets.
 */
fmm_status fmm_eval_dipoles(fmm_plan_t plan, const float *charges, const float *dipoles, float *potential,
                            float *gradient, void *stream);

/*
 * Adjoint of a loss L(phi, grad phi) (fmm_adjoint extended to losses through the gradient
 * output): given w = dL/dphi [n] and g = dL/d(grad phi) [n][3],
 *   dL/dq = Psi,   dL/dx_k = w_k grad phi_k + H_k g_k + q_k grad Psi_k,
 * where grad phi and H are the gradient and Hessian of the FMM of the charges q, and Psi the
 * FMM of the charges w with the dipoles g (fmm_eval_dipoles).  Because the plan's pair
 * kernel is symmetric, this is the exact gradient of the loss of the frozen-plan
 * approximation.  Two evaluations on the plan.  dL_dq [n] and dL_dx [n][3] may each be NULL.
 */
fmm_status fmm_adjoint_ex(fmm_plan_t plan, const float *charges, const float *dL_dphi, const float *dL_dgrad,
                          float *dL_dq, float *dL_dx, void *stream);

/*
 * Separate target set: the field of ns charged sources at nt target points that need not
 * be sources (the potential evaluation of Sec. 1 with distinct source and target sets).
 *
 * fmm_plan_targets: sources [ns][3], targets [nt][3] (device, FP32); other arguments as
 * in fmm_plan.  The plan is built over the union of the two sets (sources first): a
 * target carries zero charge, so it adds nothing to the field, and a source and a target
 * at the same position do not interact (the coincident-point rule).  Plans built this way
 * are used only with the two calls below (FMM_EINVAL otherwise, and for plain plans).
 *
 * fmm_eval_targets: charges [ns] -> potential [nt], gradient [nt][3] (either may be NULL,
 * not both).
 *
 * fmm_adjoint_targets: the exact adjoint of L(phi, grad phi at the targets) for the frozen
 * plan, with dL_dphi [nt] and, optionally, dL_dgrad [nt][3] (NULL: L depends on phi only).
 * Outputs dL_dq [ns], dL_dx_src [ns][3] (source positions) and dL_dx_tgt [nt][3] (target
 * positions); each may be NULL.  gradient_fwd [nt][3] is the forward gradient at the
 * targets (NULL: recomputed); it is not used when dL_dgrad is given.  On the union the
 * loss weights of the sources are zero, so these are fmm_adjoint and fmm_adjoint_ex of
 * the union problem restricted to the two sets: two evaluations, or five with dL_dgrad.
 */
fmm_status fmm_plan_targets(const float *sources, int64_t ns, const float *targets, int64_t nt, int ncrit, int p,
                            float theta, fmm_precision prec, void *stream, fmm_plan_t *out);
fmm_status fmm_eval_targets(fmm_plan_t plan, const float *charges, float *potential, float *gradient, void *stream);
fmm_status fmm_adjoint_targets(fmm_plan_t plan, const float *charges, const float *gradient_fwd, const float *dL_dphi,
                               const float *dL_dgrad, float *dL_dq, float *dL_dx_src, float *dL_dx_tgt, void *stream);

/* Plan statistics (host struct, filled synchronously from host-side copies). */
#define FMM_MAX_LEVELS 22
struct fmm_stats {
    int64_t n;
    int32_t p, ncrit, precision, max_level;
    float theta;
    int32_t root_exponent;                  /* root side = 2^root_exponent */
    double root_corner[3];
    int64_t ncells, nleaves;
    int64_t cells_per_level[FMM_MAX_LEVELS];
    int64_t leaves_per_level[FMM_MAX_LEVELS];
    int64_t m2l_pairs, m2l_pairs_same_level;
    int64_t m2l_keys, m2l_keys_same_level;  /* distinct (level difference, offset) operators */
    int64_t m2l_targets, m2l_tiles, m2l_entries, m2l_work_items;
    int64_t p2p_pairs;                      /* (target leaf, source leaf) pairs */
    int64_t p2p_interactions;               /* ordered (target, source) point pairs, self excluded */
    int64_t ncoef, ncoef_padded;            /* (p+1)^2 and its padded length */
    double m2l_flops;                       /* 2 (p+1)^4 per M2L pair */
    double p2p_flops;                       /* 20 per interaction (stated convention) */
    int64_t workspace_bytes;                /* device bytes the plan holds from the allocator now (its
                                               workspace, and scratch added on first use by an adjoint or
                                               Hessian call) */
    double m2l_tol;                         /* variable-order tolerance (0: every block) */
    double m2l_kept_fraction;               /* pair-weighted fraction of operator blocks applied */
    int64_t lists;                          /* FMM_LISTS_DUAL or FMM_LISTS_LEVEL_SKIP */
    int64_t p2p_work_items;                 /* near-field workgroups per evaluation: one per target
                                               leaf, more for leaves split into pieces */
    int64_t p2p_split_pieces;               /* pieces of split leaves (0: no leaf is split) */
    int64_t m2l_pool_pairs;                 /* M2L pairs of sparse (tile, key) cells, regrouped into slots */
    int64_t m2l_slots;                      /* slots: (target, source-side cell of the split that produced
                                               the pairs), one partial column each */
    int64_t m2l_slot_tiles;                 /* tiles of 64 slots with one key sequence */
    double svd_tol;                         /* SVD-compressed M2L tolerance (0: dense operators) */
    double m2l_svd_rank_mean;               /* pair-weighted mean rank of the compressed operators */
};
/* Host copy of the plan's statistics: tree shape, interaction-list sizes (the paper's
 * list-size count of Sec. 2.2 is m2l_pairs per target box in a uniform region), the work
 * of one application (M2L and P2P flops) and the memory it holds (O(N), Sec. 4.1). */
fmm_status fmm_plan_stats(fmm_plan_t plan, struct fmm_stats *out);

/*
 * Copies of the plan's tree and lists into HOST arrays (sizes from fmm_plan_stats),
 * for checking the plan against an independent construction.  Cells are numbered
 * level by level, Morton order inside a level.  Any pointer may be NULL.
 *   level[ncells], prefix[ncells] (Morton prefix: key >> 3*(21-level)), start[ncells],
 *   count[ncells] (range in the sorted order), leaf[ncells] (0/1)
 *   order[n]: sorted position -> input index
 *   m2l[m2l_pairs][2], p2p[p2p_pairs][2]: (target cell, source cell)
 */
fmm_status fmm_plan_export(fmm_plan_t plan, int32_t *level, uint64_t *prefix, int64_t *start,
                           int64_t *count, int32_t *leaf, int64_t *order, int64_t *m2l, int64_t *p2p);

/*
 * Per-phase device time of the most recent fmm_eval / fmm_adjoint on this plan, measured
 * with HIP events on the stream each phase ran on, when timing is enabled (fmm_plan_set_timing).
 * ms[] order: 0 permute, 1 P2M, 2 M2M, 3 M2L, 4 L2L, 5 L2P, 6 P2P, 7 combine, 8 total.
 * Synchronises the plan's events.
 */
#define FMM_NUM_PHASES 9
fmm_status fmm_plan_set_timing(fmm_plan_t plan, int enable);
fmm_status fmm_plan_phase_times(fmm_plan_t plan, float *ms);

void fmm_plan_destroy(fmm_plan_t plan);
const char *fmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
