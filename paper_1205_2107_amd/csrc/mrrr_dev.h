// Device-side data layout and arithmetic of the MI355X MRRR solver (gfx950, FP64).
//
// Layout in HBM (one workspace per device, grown on demand):
//   * "slots": one per matrix row of every problem; slot s of a block holds the
//     eigenvalue with local index j = s - row0 + 1 of that block: its bracket
//     [lo, hi] in the frame of node snode[s], Sturm counts at the bracket ends,
//     flags, output column.
//   * "rep pool": representations L D L^T as an array of Rep rows (32 bytes,
//     {D, L, LD, LLD}); roots occupy pool rows [0, Ntot) aligned with the slots,
//     children are appended (4 candidates per cluster, one of which is kept).
//   * nodes: one per representation (roots first), clusters: per tree level.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrrr {

constexpr double kEps = 2.220446049250313080847e-16;      // 2^-52
constexpr double kSafmin = 2.2250738585072013830903e-308; // smallest normal
constexpr double kRelgapTol = 1.0e-3;                     // Sec. 3.1.1 footnote
constexpr int kMaxDepth = 64;
constexpr double kGrowthBound = 8.0;   // child accepted outright if max|D_c| <= 8 spdiam
constexpr double kPertScale = 4.0;     // root perturbation 4 eps u, u in [-1, 1)
constexpr int kMaxRqi = 5;              // Rayleigh-quotient solves per singleton (one more to repeat the best)
constexpr int kMaxSweeps = 200;        // refinement sweeps per eigenvalue (cap)
constexpr int kSeg = 8;                 // eigenvector solves: rows per recomputed segment
// pool rows a child build takes beyond the child's own n rows: the s_i
// checkpoints of its 16 candidate shifts every 64 rows (4 doubles per row of
// the pool)
__host__ __device__ inline int64_t child_ck_rows(int64_t n) { return 4 * ((n + 63) / 64); }
constexpr int kCkptMinRun = 16;          // checkpointing eigenvector kernel: equal-node run length ...
constexpr int kCkptMinN = 256;           // ... and block order from which it is used

// slot flags
constexpr uint32_t F_NEEDS_REFINE = 1u;   // bracket must be (re)validated/refined
constexpr uint32_t F_SINGLETON = 2u;      // eigenvector to be computed from snode
constexpr uint32_t F_ACTIVE = 4u;         // slot belongs to a node of the current level
constexpr uint32_t F_RUNSTART = 8u;       // first index of a run (classification)
constexpr uint32_t F_DONE = 16u;          // eigenvector written
constexpr uint32_t F_ACCURATE = 32u;      // bracket validated and at full relative accuracy
constexpr uint32_t F_CKPT = 64u;          // eigenvector by the checkpointing kernel (long runs, large blocks)

struct Rep {
  double D, L, LD, LLD;
};

struct Problem {
  int64_t off;     // first row in packed d/e/w
  int64_t n;
  int64_t zoff;    // offset of Z block
  int64_t ldz;
  int64_t il, iu;  // INDEX range (1-based)
  double vl, vu;   // VALUE range (unscaled)
  int32_t kind;
  int32_t nblk;
  int64_t m;       // eigenpairs returned (filled on device for VALUE)
  uint64_t tmax_bits;   // max |entry| (bits of a non-negative double)
  uint64_t tnorm_bits;  // ||T||_1 after scaling
  double scale;         // power of two applied to d and e
  int32_t status;
  int32_t first_blk;    // first block id of the problem
  int64_t below;        // VALUE: eigenvalues at or below vl over all blocks
  double gaptol;        // relative-gap threshold of the classification (0: kRelgapTol)
};

struct Block {
  int64_t row0;    // global first row
  int64_t lrow0;   // first row inside its problem
  int32_t n;
  int32_t prob;
  double gl, gu, pivmin, sigma;
  int32_t wl, wu;  // wanted local range (1-based, inclusive)
  int32_t left;    // root shift at the left end of the spectrum
  int32_t gP;      // grid intervals
  int64_t goff;    // first grid point
  double glo, ghi; // grid end points (root frame)
  double gaptol;   // relative-gap threshold of the classification
};

struct Node {
  int64_t rep;     // first pool row
  double acc;      // shifts summed root to leaf
  double sigma;    // this node's shift relative to its parent (0 for roots)
  double gapl, gapr;
  int32_t blk;
  int32_t depth;
  int32_t f, l;    // local index range (1-based)
  int32_t parent;
  int32_t pad;
  double growth;   // max |D| of the representation / spectral diameter of the block
};

struct Cluster {
  int32_t node;    // parent node
  int32_t f, l;
  int32_t pad;
  double gapl, gapr;
};

// device-wide counters and status of one solve
struct Counters {
  unsigned long long sturm_steps;
  unsigned long long qds_steps;
  unsigned long long rqi;
  unsigned long long fallbacks;
  unsigned long long singletons;
  unsigned long long child_reject;
  unsigned long long pool_used;   // pool rows in use
  int32_t nclusters;              // clusters produced by the last classification
  int32_t status;                 // first non-zero device status
  int32_t grid_fail;              // grid end points did not bracket the spectrum
  int32_t unsorted;               // some problem's w is not ascending
  int32_t max_depth;
  int32_t pad;
  unsigned long long cluster_rows; // sum of cluster block sizes (pool demand)
  unsigned long long child_steps;  // row steps of child factorizations
  unsigned long long vec_rows;     // rows of twisted factorizations (per iteration)
  unsigned long long z_entries;    // eigenvector entries written
  int32_t ambiguous;               // classifications that need refined brackets
  int32_t pad2;
  unsigned long long wave_solves;  // twisted-factorization rounds summed over wavefronts
  unsigned long long ckpt_vec_rows;   // vec_rows of the checkpointing eigenvector kernel
  unsigned long long ckpt_z_entries;  // z_entries of the checkpointing eigenvector kernel
};

// ---------------------------------------------------------------------------
// counter-based random numbers: SplitMix64 output function (Steele, Lea, Flood
// 2014), evaluated at state seed + (counter + 1) * golden gamma.

__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline double unit_sym(uint64_t seed, uint64_t counter) {
  double u = (double)(splitmix64_at(seed, counter) >> 11) * (1.0 / 9007199254740992.0);
  return 2.0 * u - 1.0;
}

// grid point k of block b (identical arithmetic wherever it is evaluated)
__device__ inline double grid_point(double glo, double ghi, int k, int P) {
  if (k == 0) return glo;
  if (k == P) return ghi;
  return glo + (ghi - glo) * ((double)k / (double)P);
}

// ---------------------------------------------------------------------------
// Reciprocal: v_rcp_f64 approximates 1/x to a relative error of about 2^-24
// (measured 4.6e-8); each Newton-Raphson step r <- r + r (1 - x r) doubles the
// correct bits.  One step leaves at most 11 ulp (measured; enough for Sturm
// counts, whose backward error analysis only needs O(eps) relative error per
// operation); two steps, and the quotient below, gave the correctly rounded
// result on all of about 2.9 million operands across the normal range
// (tests/test_gpu_division.py through mrrr_probe_division).  A subnormal x
// has no finite reciprocal here (the steps give NaN): callers guard pivots to
// at least pivmin, a normal number, or test the result for finiteness.
__device__ __forceinline__ double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rcp_nr2(double x) {
  const double r = rcp_nr1(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// a / b with two Newton steps on the reciprocal and a final residual correction
__device__ __forceinline__ double div_nr(double a, double b) {
  const double r = rcp_nr2(b);
  const double q = a * r;
  const double res = fma(-b, q, a);
  return fma(res, r, q);
}

// ---------------------------------------------------------------------------
// Sturm count of L D L^T - tau I (negative pivots of the stationary qds
// transform s_1 = -tau, D+_i = D_i + s_i, s_{i+1} = (s_i / D+_i) LLD_i - tau).
// Tiny pivots become -pivmin; inf/inf ratios count as 1.
__device__ inline int sturm_count(const Rep* __restrict__ R, int n, double tau, double pivmin) {
  double s = -tau;
  int c = 0;
  for (int i = 0; i < n - 1; ++i) {
    const double D = R[i].D;
    const double LLD = R[i].LLD;
    double dp = D + s;
    dp = (fabs(dp) < pivmin) ? -pivmin : dp;
    c += (dp < 0.0) ? 1 : 0;
    double t = s * rcp_nr1(dp);
    t = (t != t) ? 1.0 : t;
    s = fma(t, LLD, -tau);
  }
  double dp = R[n - 1].D + s;
  dp = (fabs(dp) < pivmin) ? -pivmin : dp;
  c += (dp < 0.0) ? 1 : 0;
  return c;
}

// Sturm count plus the log-derivative g = d/dtau log|det(L D L^T - tau I)| =
// sum_i (ds_i/dtau) / D+_i, with ds_1 = -1 and
// ds_{i+1} = LLD_i D_i ds_i / D+_i^2 - 1.  A Newton step on the determinant is
// tau - 1/g.  The loop carries no NaN test; a NaN at the end (only possible
// after an overflow) is answered by the guarded recount of sturm_count.
__device__ inline int sturm_count_deriv(const Rep* __restrict__ R, int n, double tau, double pivmin, double* g_out) {
  double s = -tau, ds = -1.0, g = 0.0;
  int c = 0;
#pragma unroll 4
  for (int i = 0; i < n - 1; ++i) {
    const double D = R[i].D;
    const double LLD = R[i].LLD;
    double dp = D + s;
    dp = (fabs(dp) < pivmin) ? -pivmin : dp;
    c += (dp < 0.0) ? 1 : 0;
    const double inv = rcp_nr1(dp);
    const double dsi = ds * inv;
    g += dsi;
    ds = fma(LLD * D, dsi * inv, -1.0);
    s = fma(s * inv, LLD, -tau);
  }
  double dp = R[n - 1].D + s;
  dp = (fabs(dp) < pivmin) ? -pivmin : dp;
  c += (dp < 0.0) ? 1 : 0;
  g += ds * rcp_nr1(dp);
  if (!(s == s)) {
    c = sturm_count(R, n, tau, pivmin);
    g = NAN;
  }
  *g_out = g;
  return c;
}

// Sturm count on T itself (d, squared off-diagonals computed on the fly).
__device__ inline int sturm_count_T(const double* __restrict__ d, const double* __restrict__ e, int n, double tau,
                                    double pivmin) {
  double q = d[0] - tau;
  q = (fabs(q) < pivmin) ? -pivmin : q;
  int c = (q < 0.0) ? 1 : 0;
  for (int i = 1; i < n; ++i) {
    const double ee = e[i - 1];
    q = (d[i] - tau) - (ee * ee) / q;
    q = (fabs(q) < pivmin) ? -pivmin : q;
    c += (q < 0.0) ? 1 : 0;
  }
  return c;
}

}  // namespace mrrr
