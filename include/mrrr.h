/*
 * mrrr.h -- C ABI of the MI355X (gfx950) MRRR symmetric tridiagonal eigensolver.
 *
 * The problem (Petschow, Peise, Bientinesi, arXiv:1205.2107, Sec. 1.1 and Stage 4
 * of Sec. 1.2): for a real symmetric tridiagonal T of order n with diagonal d and
 * off-diagonal e, compute eigenpairs (lambda_j, z_j), T z_j = lambda_j z_j, with
 * orthonormal z_j -- all of them, or the subset selected by index or by value
 * (the MRRR cost is O(n k) for k eigenpairs, Sec. 2.3).  The method is MRRR
 * (Sec. 3.1, 3.1.1): root representation, bisection, relative-gap
 * classification, twisted factorizations for singletons, child representations
 * for clusters.  Accuracy contract (Sec. 2.3, Eq. Tresnorm, Eq. Torthogo):
 * residuals O(n eps ||T||), orthogonality O(n eps).
 *
 * Conventions shared by every entry point:
 *  - All array pointers are DEVICE pointers (hipMalloc'ed or equivalent) owned by
 *    the caller; the library never frees them.  d and e are only read.
 *  - Matrices are column-major with a leading dimension (ld >= number of rows).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *    work is ordered on it.  The representation tree is driven level by level
 *    from the host, so every solve entry point synchronizes `stream` before it
 *    returns; outputs are complete on return.
 *  - The library keeps a per-device workspace that grows with hipMalloc when a
 *    call needs more than the previous calls did (mrrr_release frees it).  Calls
 *    from several host threads on the same device are serialized internally.
 *  - Return value: 0 success; negative -k: argument k (1-based) is invalid,
 *    checked on the host before any device work; positive: a status code below.
 *    mrrr_last_error() gives a message for the calling thread's last failure.
 */
#ifndef MRRR_H
#define MRRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (positive return values and mrrr_info.status) */
#define MRRR_OK 0
#define MRRR_ERR_NO_RRR 1      /* no child representation with finite entries */
#define MRRR_ERR_DEPTH 2       /* representation tree deeper than 64 levels */
#define MRRR_ERR_CAPACITY 3    /* workspace limit reached (MRRR_MAX_WORKSPACE_GB) */
#define MRRR_ERR_NONFINITE 4   /* d or e holds inf or NaN */
#define MRRR_ERR_HIP 5         /* a HIP runtime call failed (see mrrr_last_error) */
#define MRRR_ERR_NO_DEVICE 6   /* no usable gfx950 device / kernel image */

/* Which eigenpairs: all; indices il..iu (1-based, inclusive, of the ascending
 * spectrum); or values in (vl, vu] as decided by Sturm counts at vl and vu. */
typedef enum { MRRR_ALL = 0, MRRR_INDEX = 1, MRRR_VALUE = 2 } mrrr_range_kind;

typedef struct {
  int32_t kind; /* mrrr_range_kind */
  int32_t reserved;
  int64_t il, iu;
  double vl, vu;
} mrrr_range;

/* Per-call report, written to HOST memory.  counters: see MRRR_CNT_*. */
typedef struct {
  int64_t m;          /* number of eigenpairs returned */
  int32_t status;     /* MRRR_OK or a status code */
  int32_t max_depth;  /* deepest representation-tree level reached */
  int64_t counters[16];
} mrrr_info;

#define MRRR_CNT_BLOCKS 0        /* unreduced blocks after splitting */
#define MRRR_CNT_NODES 1         /* child representations built */
#define MRRR_CNT_LEVELS 2        /* tree levels processed */
#define MRRR_CNT_STURM_STEPS 3   /* Sturm-count row steps executed (bisection + Newton) */
#define MRRR_CNT_QDS_STEPS 4     /* row steps of twisted factorizations and child builds */
#define MRRR_CNT_SINGLETONS 5    /* eigenvectors computed */
#define MRRR_CNT_RQI 6           /* twisted factorizations executed */
#define MRRR_CNT_FALLBACKS 7     /* singletons that needed the bisection fallback */
#define MRRR_CNT_CHILD_REJECT 8  /* clusters whose child failed the growth bound */
#define MRRR_CNT_WORKSPACE_MB 9  /* device workspace in use after the call */
#define MRRR_CNT_WAVE_SOLVES 10  /* twisted-factorization rounds summed over wavefronts (lockstep cost) */
#define MRRR_CNT_POOL_ROWS 11    /* representation rows in use (roots, children, speculative candidates) */
#define MRRR_CNT_AMBIGUOUS_LEFT 12 /* adjacent pairs classified from unrefined brackets after three refinements */
#define MRRR_CNT_WORKSPACE_BYTES 13 /* device workspace bytes in use after the call (carved bytes with `work`) */

/*
 * mrrr_step -- eigenpairs of one tridiagonal (Stage 4, STEP).
 *   n      order of T (n >= 0)                                         [arg 1]
 *   d      device, n doubles: diagonal                                  [arg 2]
 *   e      device, n-1 doubles: off-diagonal (may be NULL when n <= 1)   [arg 3]
 *   range  MRRR_ALL; MRRR_INDEX with 1 <= il <= iu <= n; MRRR_VALUE with vl < vu [arg 4]
 *   w      device, room for m doubles: eigenvalues, ascending            [arg 5]
 *   Z      device, ldz x m column-major (m = n for ALL, iu-il+1 for INDEX,
 *          at most n for VALUE): column j pairs with w[j]; rows outside the
 *          eigenvector's unreduced block are exact zeros; largest-magnitude
 *          entry of each column positive. Z may be NULL: eigenvalues only.  [arg 6]
 *   ldz    leading dimension of Z, >= max(1, n)                         [arg 7]
 *   info   host, may be NULL: m, status and counters                    [arg 8]
 *   stream hipStream_t as void*                                         [arg 9]
 * Blocks are split where |e_i| <= eps ||T||_1 (footnote of Sec. 3.1.1).
 */
int mrrr_step(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z,
              int64_t ldz, mrrr_info* info, void* stream);

/*
 * mrrr_workspace_size -- bytes of caller workspace for mrrr_step_ws on a
 * problem of order n and this range: the per-row arrays (slots, count grid,
 * node table, cluster list), the root representations plus room for child
 * representations of n rows each (MRRR_WS_CHILD_ROWS_PER_N * n rows, with
 * the checkpoints of their candidate shifts), and the eigenvector scratch for
 * every wanted pair at once.  A smaller workspace also works down to a floor
 * the solver checks as it goes: the eigenvector phase then runs in several
 * launches, and a tree whose representations do not fit returns status
 * MRRR_ERR_CAPACITY.  Host-only (no device work, no allocation).  Returns 0
 * for an invalid range or n < 0.  Uses the current tuning (grid density,
 * eigenvectors per wavefront).
 */
#define MRRR_WS_CHILD_ROWS_PER_N 32
size_t mrrr_workspace_size(int64_t n, mrrr_range range);

/*
 * mrrr_step_ws -- mrrr_step with a caller-provided device workspace and a
 * device-resident report (the boundary of the problem statement in Sec. 1.1 /
 * Stage 4 of Sec. 1.2: the eigenpairs of T, all or a subset).
 *   n, d, e, range, w, Z, ldz   as for mrrr_step                  [args 1-7]
 *   work        device, work_bytes bytes (256-byte aligned recommended),
 *               owned by the caller; NULL: the library's own grow-only
 *               workspace (as mrrr_step)                              [arg 8]
 *   work_bytes  size of work (see mrrr_workspace_size)                [arg 9]
 *   info_dev    DEVICE pointer to one mrrr_info, may be NULL: written on
 *               `stream` at the end of the solve                      [arg 10]
 *   stream      hipStream_t as void*                                   [arg 11]
 * With work != NULL the call allocates no device memory: every buffer is
 * carved from work (its contents on entry are ignored and on return are
 * undefined).  Two calls that share a workspace must not overlap in time.
 * Returns 0, a negative argument index (checked on the host before any
 * device work), or a status; MRRR_ERR_CAPACITY when work is too small for
 * this input (outputs are then undefined).
 */
int mrrr_step_ws(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z,
                 int64_t ldz, void* work, size_t work_bytes, mrrr_info* info_dev, void* stream);

/*
 * mrrr_step_noalloc -- mrrr_step_ws whose workspace is a fixed device array
 * inside the library, for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation).  The call makes no hipMalloc / hipFree or other allocating call
 * and uses one stream (no second stream for the eigenvector kernels).
 *   n          0 .. MRRR_NOALLOC_MAX_N; larger n returns -1          [arg 1]
 *   d, e, range, w, Z, ldz, info_dev, stream   as for mrrr_step_ws   [args 2-9]
 * The array (MRRR_NOALLOC_SCRATCH_BYTES, 256-byte aligned) is held on each
 * device the library runs this entry point on until the process ends; its
 * device address is taken once per device, on the first call there.  Every
 * call on a device uses the same array: calls that overlapped in time on one
 * device would race.  The library serializes its calls per device and each
 * call returns only after its work on `stream` has finished, so calls through
 * this library do not overlap; the array keeps the last call's contents and
 * each call initializes what it reads.  A tree whose representations do not
 * fit returns MRRR_ERR_CAPACITY.
 */
#define MRRR_NOALLOC_MAX_N 1024
#define MRRR_NOALLOC_SCRATCH_BYTES (64u << 20)
int mrrr_step_noalloc(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z,
                      int64_t ldz, mrrr_info* info_dev, void* stream);

/*
 * Limits of the representation tree.  Lowering them makes the solver report
 * the corresponding status instead of going on (used by the tests of those
 * paths):
 *   max_depth           1 .. 64 (default 64): nodes at this depth do not get
 *                       child representations; their clustered eigenvalues
 *                       are computed as singletons of the deepest node and the
 *                       call returns MRRR_ERR_DEPTH.
 *   child_growth_limit  0 (default): a cluster takes the candidate shift with
 *                       the least element growth when none meets the growth
 *                       bound of 8 spectral diameters; > 0: candidates whose
 *                       max |D_c| exceeds this many spectral diameters are
 *                       rejected, and a cluster without an acceptable one is
 *                       handed back to its parent (MRRR_ERR_NO_RRR).
 * mrrr_set_limits returns -1 for out-of-range fields.
 */
typedef struct {
  int32_t max_depth;
  int32_t reserved;
  double child_growth_limit;
} mrrr_limits;

int mrrr_get_limits(mrrr_limits* l);
int mrrr_set_limits(const mrrr_limits* l);

/*
 * mrrr_step_batched -- all eigenpairs of `batch` independent tridiagonals in one
 * pass of the solver (every level of every problem's representation tree is
 * processed by the same kernel launches).
 *   batch        number of problems (>= 0)                                [arg 1]
 *   n_host       HOST, batch int64: orders n_b >= 1                         [arg 2]
 *   off_host     HOST, batch int64: offset of problem b in d, e and w       [arg 3]
 *   d, e         device: d[off_b + i], i < n_b; e[off_b + i], i < n_b - 1    [args 4, 5]
 *   w            device: eigenvalues of problem b at w[off_b ...], ascending [arg 6]
 *   Z            device: problem b's n_b x n_b eigenvectors at Z + zoff_b,
 *                column-major with leading dimension n_b                    [arg 7]
 *   zoff_host    HOST, batch int64: offsets of the Z blocks                 [arg 8]
 *   info         host, may be NULL: batch entries                          [arg 9]
 *   stream                                                                   [arg 10]
 * Problems must not overlap in d/e/w/Z.
 */
int mrrr_step_batched(int64_t batch, const int64_t* n_host, const int64_t* off_host, const double* d,
                      const double* e, double* w, double* Z, const int64_t* zoff_host, mrrr_info* info,
                      void* stream);

/*
 * mrrr_step_backward -- reverse-mode derivative of the decomposition.
 * Given eigenvalues w (n), orthonormal eigenvectors Z (n x n, ldz) of T and the
 * cotangents gw = dL/dw (n, may be NULL) and gZ = dL/dZ (n x n, ldgz, may be
 * NULL), writes gd = dL/dd (n) and ge = dL/de (n-1):
 *   M = diag(gw) + F o (Z^T gZ),  F_ik = 1/(w_k - w_i) (i != k), F_kk = 0,
 *   A = Z M Z^T,  gd_i = A_ii,  ge_i = A_{i,i+1} + A_{i+1,i}.
 * Requires distinct eigenvalues (F is unbounded at multiple eigenvalues).
 * Uses FP64 matrix cores for the two dense contractions; A is never stored.
 *   args: n [1], w [2], Z [3], ldz [4], gw [5], gZ [6], ldgz [7], gd [8], ge [9], stream [10]
 */
int mrrr_step_backward(int64_t n, const double* w, const double* Z, int64_t ldz, const double* gw,
                       const double* gZ, int64_t ldgz, double* gd, double* ge, void* stream);

/*
 * mrrr_step_backward_batched -- the backward for `batch` problems with the
 * layout of mrrr_step_batched (Z_b and gZ_b at zoff_b with leading dimension n_b;
 * w_b, gw_b, gd_b, ge_b at off_b).  gw or gZ may be NULL.
 *   args: batch [1], n_host [2], off_host [3], zoff_host [4], w [5], Z [6], gw [7], gZ [8],
 *         gd [9], ge [10], stream [11]
 */
int mrrr_step_backward_batched(int64_t batch, const int64_t* n_host, const int64_t* off_host,
                               const int64_t* zoff_host, const double* w, const double* Z, const double* gw,
                               const double* gZ, double* gd, double* ge, void* stream);

/* Launch-shape parameters of the solver (the batched autotuner sets these). */
typedef struct {
  int32_t grid_density;    /* Sturm-count grid points per eigenvalue for the initial brackets (1..16) */
  int32_t refine_wave_slots; /* eigenvalues per wavefront in refinement (0 = automatic, 16, 32 or 64) */
  int32_t vec_wave_slots;  /* eigenvectors per wavefront (0 = automatic, 8, 16 or 32) */
  /* eigenvector kernel choice: runs of at least this many singletons of one
   * representation (in blocks of vec_ckpt_min_n rows or more) go to the checkpointing
   * kernel, the rest to the stored-vector kernel.  0 = automatic (16), -1 =
   * stored-vector kernel only, else 1 .. 2^30.  Both kernels give bit-identical
   * results; this only moves work between them. */
  int32_t vec_ckpt_min_run;
  /* ... and the block order from which that applies: 0 = automatic, else
   * 64 .. 2^30. */
  int32_t vec_ckpt_min_n;
  int32_t reserved[3];
} mrrr_tuning;

int mrrr_get_tuning(mrrr_tuning* t);

int mrrr_set_tuning(const mrrr_tuning* t); /* -1 on out-of-range fields */

/* Autotuner of the batched form (a schedule choice, not part of the method).
 * Solves the batch described exactly as for mrrr_step_batched several times
 * with different launch shapes -- eigenvectors per wavefront, eigenvalues per
 * refinement wavefront, count-grid density, the run length from which the
 * checkpointing eigenvector kernel takes singletons -- by a coordinate search, timing
 * each synchronised solve on the host clock, and stores the fastest shape in a
 * process-wide cache keyed by the batch's size histogram (problem counts per
 * power-of-two size class, counts rounded to powers of two).  Later
 * mrrr_step_batched calls whose batch has the same key use the cached shape;
 * other calls use the global tuning.  w and Z receive the results of the last
 * trial (a valid solve).  best (may be NULL) receives the chosen shape.
 * Costs about twelve solves of the batch.  Returns 0 or a status / negative
 * argument code as mrrr_step_batched. */
int mrrr_autotune_batched(int64_t batch, const int64_t* n_host, const int64_t* off_host, const double* d,
                          const double* e, double* w, double* Z, const int64_t* zoff_host, mrrr_tuning* best,
                          void* stream);

/* Kernel timing.  While enabled, the solve entry points record HIP events on
 * the stream each of their main kernels runs on (the caller's stream, or for
 * MRRR_K_VECTORS_CKPT the library's second stream, joined to the caller's)
 * around every launch and accumulate the elapsed times and the algorithmic
 * work of those launches:
 *   MRRR_K_GRID     Sturm-count grid        work = 4 flops per row step
 *   MRRR_K_REFINE   bisection/Newton        work = 4 flops per row step
 *   MRRR_K_CHILD    child representations   work = 5 flops per row step
 *   MRRR_K_VECTORS  twisted factorizations, stored-work-vector kernel:
 *                   work = 15 flops per row per iteration; bytes = 8 per
 *                   eigenvector entry written
 *   MRRR_K_BACKWARD both backward GEMMs     work = 2 n^3 flops each
 *   MRRR_K_VECTORS_CKPT  twisted factorizations, checkpointing kernel (long
 *                   runs of one node's singletons in large blocks); work and
 *                   bytes counted as for MRRR_K_VECTORS
 *   MRRR_K_BACKTRANSFORM  mrrr_backtransform (all its launches as one):
 *                   work = 4 K nb m flops per block of nb reflectors over
 *                   its K rows (about 2 n^2 m in all)
 *   MRRR_K_TRIDIAG  mrrr_tridiagonalize (all its launches as one):
 *                   work = 4 n^3 / 3 flops; bytes = 8 per entry of the
 *                   trailing lower triangles the matrix-vector products
 *                   read (sum over m = 1 .. n-1 of m (m + 1) / 2)
 *   MRRR_K_GHEP     mrrr_cholesky (n^3 / 3 flops), mrrr_sygst (2 n^3) and
 *                   mrrr_trsm_lt (n^2 m), all their launches
 * mrrr_profile_read fills launches, total milliseconds, work and bytes. */
#define MRRR_K_GRID 0
#define MRRR_K_REFINE 1
#define MRRR_K_CHILD 2
#define MRRR_K_VECTORS 3
#define MRRR_K_BACKWARD 4
#define MRRR_K_VECTORS_CKPT 5
#define MRRR_K_BACKTRANSFORM 6
#define MRRR_K_TRIDIAG 7
#define MRRR_K_GHEP 8
#define MRRR_K_COUNT 9

typedef struct {
  int64_t launches;
  double ms;
  double work;   /* algorithmic flops */
  double bytes;  /* algorithmic HBM bytes */
} mrrr_kernel_time;

int mrrr_profile_enable(int on);
int mrrr_profile_reset(void);
int mrrr_profile_read(int kernel, mrrr_kernel_time* out); /* -1 on a bad kernel id */

/* mrrr_step_f32 -- the FP32 interface with FP64 arithmetic inside (the
 * mixed-precision use the paper names for orthogonality-sensitive work,
 * Sec. 2.3): d, e, w, Z are FP32 device arrays, laid out as for mrrr_step;
 * the library widens d and e, runs the FP64 solver with the relative-gap
 * threshold of the classification lowered from 1e-3 to min(1e-3, n 2^-27)
 * (FP64 arithmetic leaves room for that: eigenvectors of singletons that
 * close still lean towards their neighbours by less than eps32 / 4, and the
 * representation tree has fewer clusters), and rounds w and Z to FP32.
 * Orthogonality and residuals are then set by that rounding, O(eps32)
 * rather than O(n eps32).  The library keeps a grow-only FP64 staging
 * buffer (3 n + n m doubles, m the wanted pairs; n columns for VALUE ranges);
 * calls are serialized and synchronize the stream.  Arguments, range, info
 * and returns as for mrrr_step. */
int mrrr_step_f32(int64_t n, const float* d, const float* e, mrrr_range range, float* w, float* Z, int64_t ldz,
                  mrrr_info* info, void* stream);

/* Stage 5 back-transformation (Sec. 1.2, stage 5: the eigenvectors of the
 * dense symmetric M are Y = Q Z after a lower tridiagonal reduction
 * T = Q^T M Q), on FP64 matrix cores.  Q = H_0 H_1 ... H_{n-2},
 * H_i = I - tau_i v_i v_i^T, with v_i[0..i] = 0, v_i[i+1] = 1 and
 * v_i[i+2..n-1] = V[(i+2..n-1) + i ldv]: the storage a lower reduction
 * (LAPACK's dsytrd with uplo 'L') leaves.  Entries of V on or above the
 * first subdiagonal are not read.
 *   V    device, n x (n - 1) used of n x ldv column-major, read-only;
 *   tau  device, n - 1 doubles, read-only;
 *   Z    device, n x m column-major (leading dimension ldz), overwritten
 *        with Q Z.
 * Applied in blocks of 64 reflectors in compact WY form (I - V_b T_b V_b^T),
 * last block first.  The library keeps a grow-only workspace per process
 * (64 x 64 doubles per block plus 64 x m); calls are serialized by a lock and
 * synchronize the stream before returning.  Returns 0; -1 (n < 0 or
 * n > 2^31), -2 (m), -3 (V null with n > 2), -4 (ldv < max(1, n)), -5 (tau
 * null with n > 1), -6 (Z null with n, m > 0), -7 (ldz < max(1, n));
 * MRRR_ERR_CAPACITY when the workspace cannot be allocated; MRRR_ERR_HIP on a
 * failed launch.  n <= 1 or m == 0 leaves Z as it is. */
int mrrr_backtransform(int64_t n, int64_t m, const double* V, int64_t ldv, const double* tau, double* Z,
                       int64_t ldz, void* stream);

/* Stage 3 reduction to tridiagonal form (Sec. 1.2, stage 3; Sec. 2.2: the
 * direct reduction of the dense pipeline): T = Q^T M Q for the real symmetric
 * M, by Householder reflectors in the storage a lower reduction (LAPACK's
 * dsytrd with uplo 'L') leaves, so that mrrr_backtransform applies Q.
 *   A    device, n x n column-major (leading dimension lda).  On entry the
 *        lower triangle holds M.  On return the diagonal holds d, the first
 *        subdiagonal e, and A[(i+2..n-1) + i lda] the reflector v_i below its
 *        unit entry (v_i[0..i] = 0, v_i[i+1] = 1).  The strict upper triangle
 *        is neither read nor written;
 *   d    device, n doubles: the diagonal of T;
 *   e    device, n - 1 doubles: the off-diagonal of T (e_i = beta_i, either
 *        sign);
 *   tau  device, n - 1 doubles: H_i = I - tau_i v_i v_i^T (tau_{n-2} = 0).
 * The reflector of x = (alpha, x_2, ...): beta = -sign(alpha) ||x|| (alpha
 * = 0 counts as positive), tau = (beta - alpha) / beta, v = x / (alpha -
 * beta) below the unit entry; H = I (tau = 0, beta = alpha) when x_2.. are
 * zero.  Blocked in panels of 64 columns (trailing update on FP64 matrix
 * cores); reductions in a fixed order, so results repeat exactly.  The library
 * keeps a grow-only workspace (2 x 64 n doubles for the panel, 64 ceil(n/64)^2
 * for the partial sums of the matrix-vector products, plus O(n)); calls are
 * serialized by a lock and synchronize the stream before returning.  Returns
 * 0; -1 (n < 0 or n > 2^18), -2 (A null with n > 0), -3 (lda < max(1, n)),
 * -4 (d null with n > 0), -5 (e null with n > 1), -6 (tau null with n > 1);
 * MRRR_ERR_CAPACITY when the workspace cannot be allocated; MRRR_ERR_HIP on a
 * failed launch.  Non-finite entries propagate (no status). */
int mrrr_tridiagonalize(int64_t n, double* A, int64_t lda, double* d, double* e, double* tau, void* stream);

/* Stages 1, 2 and 6 of the generalized eigenproblem A x = lambda B x with B
 * symmetric positive definite (Sec. 1.2, stage list): the Cholesky
 * factorization B = L L^T, the reduction to the standard problem
 * M y = lambda y with M = L^{-1} A L^{-T}, and the second back-transformation
 * x = L^{-T} y.  With mrrr_tridiagonalize, mrrr_step and mrrr_backtransform
 * in between they form the dense generalized eigensolver.  All matrices are
 * device, column-major, blocked in 64 x 64 tiles (triangular solves with one
 * diagonal block per lane vector, updates of rank 64 to 256 on FP64 matrix
 * cores); calls synchronize the stream before returning and are serialized
 * by a lock per function family.  n <= 2^18.
 *
 * mrrr_cholesky: B (n x n, leading dimension ldb): the lower triangle holds B
 * on entry and L on return; the strict upper triangle is not referenced.
 * *info (host) = 0, or the 1-based column whose pivot was not positive (B
 * not positive definite; the factorization stops there, the lower triangle
 * holds partial results).  Returns 0; -1 (n), -2 (B null with n > 0),
 * -3 (ldb < max(1, n)), -4 (info null); MRRR_ERR_HIP on a failed launch. */
int mrrr_cholesky(int64_t n, double* B, int64_t ldb, int64_t* info, void* stream);

/* mrrr_sygst: M = L^{-1} A L^{-T}.  A (n x n, lda): its lower triangle holds
 * the symmetric A on entry; on return all of A holds M (symmetric up to
 * rounding; the reduction to tridiagonal form reads its lower triangle).
 * L (n x n, ldl): the lower triangle of the Cholesky factor, read-only.  The
 * library keeps a grow-only workspace of n x n doubles.  Returns 0; -1 (n),
 * -2 (A null), -3 (lda), -4 (L null), -5 (ldl); MRRR_ERR_CAPACITY when the
 * workspace cannot be allocated; MRRR_ERR_HIP on a failed launch. */
int mrrr_sygst(int64_t n, double* A, int64_t lda, const double* L, int64_t ldl, void* stream);

/* mrrr_trsm_lt: Y <- L^{-T} Y for Y (n x m, ldy), L (n x n lower, ldl,
 * read-only).  Returns 0; -1 (n), -2 (m < 0 or m > 2^31), -3 (L null), -4
 * (ldl), -5 (Y null with n, m > 0), -6 (ldy); MRRR_ERR_HIP on a failed
 * launch. */
int mrrr_trsm_lt(int64_t n, int64_t m, const double* L, int64_t ldl, double* Y, int64_t ldy, void* stream);

/* Dense drivers: every stage on the GPU, on the caller's stream.
 *
 * mrrr_syev: all eigenpairs of the dense symmetric A (n x n, lda, lower
 * triangle read): mrrr_tridiagonalize, mrrr_step, mrrr_backtransform.  A is
 * overwritten (its lower triangle holds the reduction); w (device, n) the
 * eigenvalues ascending; Z (device, n x n, ldz) the eigenvectors; info as for
 * mrrr_step (the tridiagonal solve's report).  Returns 0; -1 (n < 0 or
 * n > 2^18), -2 (A null), -3 (lda), -4 (w null), -5 (Z null), -6 (ldz); else
 * the first non-zero return of a stage.
 *
 * mrrr_sygv: all eigenpairs of A x = lambda B x, B positive definite (lower
 * triangles of A and B read): mrrr_cholesky, mrrr_sygst, mrrr_syev,
 * mrrr_trsm_lt.  A and B are overwritten (B with L); Z holds X with
 * X^T B X = I.  *not_pd (host) = 0, or the 1-based column whose pivot was not
 * positive (then nothing else is computed and the return is 0).  Returns 0;
 * -1 (n), -2 (A null), -3 (lda), -4 (B null), -5 (ldb), -6 (w null), -7 (Z
 * null), -8 (ldz), -9 (not_pd null); else the first non-zero return of a
 * stage.  The library keeps 3 n doubles for d, e and tau. */
int mrrr_syev(int64_t n, double* A, int64_t lda, double* w, double* Z, int64_t ldz, mrrr_info* info, void* stream);
int mrrr_sygv(int64_t n, double* A, int64_t lda, double* B, int64_t ldb, double* w, double* Z, int64_t ldz,
              int64_t* not_pd, mrrr_info* info, void* stream);

/* The same drivers for a subset of the eigenpairs (range as for mrrr_step:
 * all, an index range il..iu, or the values in (vl, vu]; for mrrr_sygvr the
 * generalized eigenvalues, which are those of the standard problem).  Only
 * the info->m computed eigenvectors are back-transformed, in the first
 * info->m columns of Z (room for n columns with a value range).  Returns as
 * mrrr_syev and mrrr_sygv with the range as argument 4 (mrrr_syevr: -4 on a
 * bad kind, later arguments numbered one higher) and 6 (mrrr_sygvr). */
int mrrr_syevr(int64_t n, double* A, int64_t lda, mrrr_range range, double* w, double* Z, int64_t ldz,
               mrrr_info* info, void* stream);
int mrrr_sygvr(int64_t n, double* A, int64_t lda, double* B, int64_t ldb, mrrr_range range, double* w, double* Z,
               int64_t ldz, int64_t* not_pd, mrrr_info* info, void* stream);

/* Arithmetic probe: the reciprocal and quotient forms the kernels use, on
 * caller-given operands (no solve; for tests of their rounding).  a, b: device
 * arrays of n doubles; out: device array of 4 n doubles, written as
 *   out[i]         v_rcp_f64(b[i]), the hardware reciprocal approximation;
 *   out[n + i]     that after one Newton-Raphson step r + r (1 - b r): the
 *                  reciprocal of the Sturm counts, the twisted transforms and
 *                  the Rayleigh-quotient correction;
 *   out[2n + i]    after two steps: the multipliers of child representations
 *                  (stationary qds, Sec. 3.1.1 child step);
 *   out[3n + i]    a[i] / b[i] from the two-step reciprocal, the product and
 *                  one residual correction: the eigenvector recurrence across
 *                  a zero pivot.
 * Enqueued on stream (NULL: the default stream) without synchronising.
 * Returns 0; -1 when n < 0 or n > 2^31; -2 on a null pointer with n > 0;
 * MRRR_ERR_HIP when the launch fails. */
int mrrr_probe_division(int64_t n, const double* a, const double* b, double* out, void* stream);

/* Free the calling device's workspace (the next call allocates again). */
int mrrr_release(void);

/* Message for the calling thread's last non-zero return. */
const char* mrrr_last_error(void);

/* Message for a status code. */
const char* mrrr_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* MRRR_H */
