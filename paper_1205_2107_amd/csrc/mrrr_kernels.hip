// HIP kernels of the MRRR tridiagonal eigensolver for gfx950 (MI355X), FP64.
//
// Steps (Petschow, Peise, Bientinesi, arXiv:1205.2107, Sec. 3.1.1):
//   split            k_prep_max, k_prep_scale, k_split_flags, k_blocks*
//   root RRR         k_root           L0 D0 L0^T = T - sigma I, T - sigma I definite
//   bisection        k_grid, k_assign, k_refine   Sturm counts on L D L^T (one lane per
//                    eigenvalue), accelerated by safeguarded Newton steps on det
//   classification   k_cls_flags, k_cls_compact, k_cls_runs   relative gaps, tol 1e-3
//   clusters         k_child, k_shift L_c D_c L_c^T = L D L^T - sigma_c I (stationary qds)
//   singletons       k_vectors        twisted factorization + Rayleigh correction,
//                    z written to column-major Z through an LDS transpose
#include <map>
#include <mutex>
#include <type_traits>

#include "mrrr_dev.h"
#include "mrrr_launch.h"

namespace mrrr {

// ---------------------------------------------------------------------------
// helpers

__device__ inline int find_segment(const int64_t* __restrict__ off, int count, int64_t x) {
  // largest k in [0, count) with off[k] <= x (off ascending, off[0] = 0)
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline void atomic_max_nonneg(uint64_t* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

__device__ inline void set_status(Counters* C, int code) { atomicCAS(&C->status, 0, code); }

__device__ __forceinline__ int first_lane(uint64_t mask) { return __ffsll((unsigned long long)mask) - 1; }


// ---------------------------------------------------------------------------
// 1. input checks, scaling, 1-norm, split points

__global__ void k_prep_max(Problem* __restrict__ P, int nprob, const int64_t* __restrict__ poff, int64_t ntot,
                           const double* __restrict__ d, const double* __restrict__ e, int32_t* __restrict__ sprob) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  int p = find_segment(poff, nprob, s);
  sprob[s] = p;
  const int64_t i = s - poff[p];
  const int64_t n = P[p].n;
  const double dv = d[P[p].off + i];
  const double ev = (i + 1 < n) ? e[P[p].off + i] : 0.0;
  if (!isfinite(dv) || !isfinite(ev)) {
    atomicCAS(&P[p].status, 0, 4);
    return;
  }
  atomic_max_nonneg(&P[p].tmax_bits, fmax(fabs(dv), fabs(ev)));
}

__global__ void k_prep_scale(Problem* __restrict__ P, const int64_t* __restrict__ poff, int64_t ntot,
                             const double* __restrict__ d, const double* __restrict__ e,
                             const int32_t* __restrict__ sprob, double* __restrict__ ds, double* __restrict__ es) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int p = sprob[s];
  const int64_t i = s - poff[p];
  const int64_t n = P[p].n;
  const double tmax = __longlong_as_double((long long)P[p].tmax_bits);
  double scale = 1.0;
  if (tmax > 0.0 && (tmax < 0x1p-500 || tmax > 0x1p500)) scale = ldexp(1.0, -ilogb(tmax));
  if (i == 0) P[p].scale = scale;
  // a problem with a non-finite entry is solved as the zero matrix (status 4)
  const bool bad = P[p].status == 4;
  const double dv = bad ? 0.0 : d[P[p].off + i] * scale;
  const double ev = (!bad && i + 1 < n) ? e[P[p].off + i] * scale : 0.0;
  const double evm = (!bad && i > 0) ? e[P[p].off + i - 1] * scale : 0.0;
  ds[s] = dv;
  es[s] = ev;
  atomic_max_nonneg(&P[p].tnorm_bits, fabs(evm) + fabs(dv) + fabs(ev));
}

__global__ void k_split_flags(const Problem* __restrict__ P, const int64_t* __restrict__ poff, int64_t ntot,
                              const int32_t* __restrict__ sprob, double* __restrict__ es, int32_t* __restrict__ flag) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int p = sprob[s];
  const int64_t i = s - poff[p];
  int start = (i == 0);
  if (!start) {
    const double tnorm = __longlong_as_double((long long)P[p].tnorm_bits);
    if (fabs(es[s - 1]) <= kEps * tnorm) {
      es[s - 1] = 0.0;
      start = 1;
    }
  }
  flag[s] = start;
}

// exclusive scan of int32 flags: per-workgroup pass, top-level pass, fix-up
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int wg_inclusive_scan(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int r = sh[t];
  __syncthreads();
  return r;
}

__global__ void k_scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out, int32_t* __restrict__ tile_sum,
                             int64_t n) {
  __shared__ int sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    sum += v[k];
  }
  int incl = wg_inclusive_scan(sum, sh);
  int run = incl - sum;
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = incl;
}

__global__ void k_scan_top(int32_t* __restrict__ tile_sum, int64_t ntiles, int32_t* __restrict__ total) {
  __shared__ int sh[kScanThreads];
  __shared__ int s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < ntiles; base += kScanThreads) {
    const int64_t k = base + threadIdx.x;
    const int v = (k < ntiles) ? tile_sum[k] : 0;
    const int incl = wg_inclusive_scan(v, sh);
    const int carry = s_carry;
    if (k < ntiles) tile_sum[k] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) s_carry = carry + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = s_carry;
}

__global__ void k_scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ tile_sum, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  const int add = tile_sum[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] += add;
}

// block table from the split flags and their exclusive scan
__global__ void k_blocks(const int32_t* __restrict__ flag, const int32_t* __restrict__ excl, int64_t ntot,
                         int64_t* __restrict__ bstart, int32_t* __restrict__ sblk) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int f = flag[s];
  const int b = excl[s] + f - 1;
  sblk[s] = b;
  if (f) bstart[b] = s;
}

__global__ void k_blocks2(Problem* __restrict__ P, const int64_t* __restrict__ poff, const int64_t* __restrict__ bstart,
                          int nblk, int64_t ntot, const int32_t* __restrict__ sprob, Block* __restrict__ B) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int64_t r0 = bstart[b];
  const int64_t r1 = (b + 1 < nblk) ? bstart[b + 1] : ntot;
  const int p = sprob[r0];
  Block blk;
  blk.row0 = r0;
  blk.lrow0 = r0 - poff[p];
  blk.n = (int32_t)(r1 - r0);
  blk.prob = p;
  blk.gl = blk.gu = blk.pivmin = blk.sigma = 0.0;
  blk.wl = 1;
  blk.wu = blk.n;
  blk.left = 1;
  blk.gP = 0;
  blk.goff = 0;
  blk.glo = blk.ghi = 0.0;
  blk.gaptol = P[p].gaptol > 0.0 ? P[p].gaptol : kRelgapTol;
  B[b] = blk;
  atomicAdd(&P[p].nblk, 1);
  if (blk.lrow0 == 0) P[p].first_blk = b;
}

// ---------------------------------------------------------------------------
// 2. root representation per block (one workgroup of 256 threads per block)

__device__ inline double wg_reduce(double v, double* sh, int op) {  // op 0 min, 1 max
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] = op ? fmax(sh[t], sh[t + off]) : fmin(sh[t], sh[t + off]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

constexpr int kRootChunk = 1024;  // rows of the root factorization staged at a time

__global__ void __launch_bounds__(256) k_root(Problem* __restrict__ P, Block* __restrict__ B, Node* __restrict__ N,
                                              const double* __restrict__ ds, const double* __restrict__ es,
                                              Rep* __restrict__ pool, Counters* __restrict__ C, int grid_density) {
  __shared__ double sh[256];
  __shared__ double s_d[kRootChunk + 1], s_e[kRootChunk + 1], s_D[kRootChunk], s_L[kRootChunk];
  __shared__ int s_ok;
  __shared__ int s_cnt[2];
  const int b = blockIdx.x;
  Block blk = B[b];
  const int n = blk.n;
  const int p = blk.prob;
  const double* d = ds + blk.row0;
  const double* e = es + blk.row0;
  double gl = INFINITY, gu = -INFINITY, em = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double r = 0.0;
    if (i > 0) r += fabs(e[i - 1]);
    if (i + 1 < n) {
      r += fabs(e[i]);
      em = fmax(em, e[i] * e[i]);
    }
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
  }
  gl = wg_reduce(gl, sh, 0);
  gu = wg_reduce(gu, sh, 1);
  em = wg_reduce(em, sh, 1);
  const double pivmin = kSafmin * fmax(1.0, em);
  const Problem pr = P[p];
  int wl = 1, wu = n;
  if (pr.kind == 1 && pr.nblk == 1) {
    wl = (int)pr.il;
    wu = (int)pr.iu;
  }
  // VALUE ranges: local index range from Sturm counts on T (two waves)
  if (pr.kind == 2) {
    if (threadIdx.x == 64 || threadIdx.x == 128) {
      const double v = (threadIdx.x == 64 ? pr.vl : pr.vu) * pr.scale;
      s_cnt[threadIdx.x == 128] = sturm_count_T(d, e, n, v, pivmin);
    }
    __syncthreads();
    wl = s_cnt[0] + 1;
    wu = s_cnt[1];
  }
  const int left = (pr.kind == 0) || (pr.kind == 1 && pr.nblk > 1) || (wl + wu <= n + 1);
  Rep* R = pool + blk.row0;
  // L0 D0 L0^T = T - sigma I, one row after the other (thread 0), on chunks
  // of kRootChunk rows that the whole workgroup stages through LDS: the
  // serial chain then waits on LDS, not on a memory round trip per row
  double delta = 4.0 * (double)n * kEps * fmax(fabs(gl), fabs(gu));
  if (!(delta > 0.0)) delta = pivmin;
  double sigma = 0.0;
  for (int tries = 0; tries < 64; ++tries) {
    sigma = left ? gl - delta : gu + delta;
    // the pivots must keep the sign of the definite side and stay finite;
    // sgn * Dp is exact, and a NaN fails the comparison
    const double sgn = left ? 1.0 : -1.0;
    int ok = 1;
    double Dp = 0.0;
    for (int c0 = 0; c0 < n; c0 += kRootChunk) {
      // rows c0 .. c0 + m - 1, plus the next chunk's first diagonal entry
      const int m = min(kRootChunk, n - c0);
      for (int i = threadIdx.x; i <= m; i += blockDim.x) {
        s_d[i] = (c0 + i < n) ? d[c0 + i] : 0.0;
        s_e[i] = (c0 + i + 1 < n) ? e[c0 + i] : 0.0;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        if (c0 == 0) Dp = s_d[0] - sigma;
        const int mi = (c0 + m < n) ? m : m - 1;  // rows with an off-diagonal entry
#pragma unroll 4
        for (int i = 0; i < mi; ++i) {
          const double L = s_e[i] / Dp;
          s_D[i] = Dp;
          s_L[i] = L;
          ok &= (int)isfinite(Dp) & (int)isfinite(L) & (int)(sgn * Dp > 0.0);
          Dp = (s_d[i + 1] - sigma) - L * s_e[i];
        }
        if (mi < m) {  // the last row of the block
          s_D[mi] = Dp;
          s_L[mi] = 0.0;
          ok &= (int)isfinite(Dp) & (int)(sgn * Dp > 0.0);
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        R[c0 + i].D = s_D[i];
        R[c0 + i].L = s_L[i];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) s_ok = ok;
    __syncthreads();
    delta *= 2.0;
    if (s_ok) break;
  }
  if (!s_ok) set_status(C, 1);
  // deterministic relative perturbation of the root, then the products
  const uint64_t seed = (uint64_t)blk.lrow0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double D = R[i].D * (1.0 + kPertScale * kEps * unit_sym(seed, 2u * (uint64_t)i));
    double L = (i + 1 < n) ? R[i].L * (1.0 + kPertScale * kEps * unit_sym(seed, 2u * (uint64_t)i + 1u)) : 0.0;
    double LD = L * D;
    R[i].D = D;
    R[i].L = L;
    R[i].LD = LD;
    R[i].LLD = LD * L;
  }
  if (threadIdx.x == 0) {
    const double pad = 8.0 * (double)n * kEps * fmax(fabs(gl), fabs(gu)) + 4.0 * pivmin;
    blk.gl = gl;
    blk.gu = gu;
    blk.pivmin = pivmin;
    blk.sigma = sigma;
    blk.wl = wl;
    blk.wu = wu;
    blk.left = left;
    blk.glo = (gl - sigma) - pad;
    blk.ghi = (gu - sigma) + pad;
    blk.gP = grid_density * n;
    B[b] = blk;
    Node nd;
    nd.rep = blk.row0;
    nd.acc = sigma;
    nd.sigma = 0.0;
    nd.gapl = INFINITY;
    nd.gapr = INFINITY;
    nd.blk = b;
    nd.depth = 0;
    nd.f = 1;
    nd.l = n;
    nd.parent = -1;
    nd.pad = 0;
    nd.growth = 0.0;
    N[b] = nd;
    if (pr.kind == 2) {
      atomicAdd((unsigned long long*)&P[p].m, (unsigned long long)(wu >= wl ? wu - wl + 1 : 0));
      atomicAdd((unsigned long long*)&P[p].below, (unsigned long long)(wl - 1));
    }
  }
}

// ---------------------------------------------------------------------------
// 3. eigenvalue brackets: a grid of Sturm counts per block, then one lane per
//    eigenvalue picks its grid cell

__global__ void k_assign(const Block* __restrict__ B, const int64_t* __restrict__ goff, int64_t ntot,
                         const int32_t* __restrict__ sblk, const int32_t* __restrict__ gcnt, double* __restrict__ lo,
                         double* __restrict__ hi, int32_t* __restrict__ clo, int32_t* __restrict__ chi,
                         int32_t* __restrict__ snode, uint32_t* __restrict__ sflag, Counters* __restrict__ C) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int b = sblk[s];
  const Block blk = B[b];
  const int j = (int)(s - blk.row0) + 1;
  const int32_t* c = gcnt + goff[b];
  const int P = blk.gP;
  int a = 0, z = P;
  if (c[0] > j - 1 || c[P] < j) atomicExch(&C->grid_fail, 1);
  while (z - a > 1) {
    const int mid = (a + z) >> 1;
    if (c[mid] <= j - 1)
      a = mid;
    else
      z = mid;
  }
  lo[s] = grid_point(blk.glo, blk.ghi, a, P);
  hi[s] = grid_point(blk.glo, blk.ghi, z, P);
  clo[s] = c[a];
  chi[s] = c[z];
  snode[s] = b;
  sflag[s] = F_NEEDS_REFINE | F_ACTIVE;
}

// ---------------------------------------------------------------------------
// 4. refinement.  L lanes serve one eigenvalue and evaluate L shifts per sweep
//    (Sturm count plus log-derivative of the determinant each); the group then
//    shares the results and every lane updates the same state:
//      validation   the bracket ends (and widened ends) until cnt(lo) <= j-1 < cnt(hi)
//      section      L equispaced interior points while the bracket holds more
//                   than one eigenvalue (or no Newton estimate lies inside)
//      Newton       tau_N = tau - 1/g from the bracket end with the smaller
//                   step, plus probes tau_N -+ delta that certify the bracket
//    until the bracket is 4 eps relative wide (bisection's guarantee of high
//    relative accuracy, reached with far fewer sweeps).

struct EigState {
  double lo, hi;    // bracket (w.r.t. the slot's node)
  double glo, ghi;  // log-derivative at lo / hi (NaN: unknown)
  double pad;       // widening step while validating
  int clo, chi;     // counts at lo / hi, -1 when not validated
  int j;            // 1-based index in the block
  int done;
};

__device__ inline bool bracket_converged(double lo, double hi) {
  const double mid = 0.5 * (lo + hi);
  return hi - lo <= 4.0 * kEps * fmax(fabs(lo), fabs(hi)) || mid <= lo || mid >= hi;
}

// r, nr: this eigenvalue's place among the nr eigenvalues of its wavefront
// that share its bracket (a cell holding several eigenvalues): their points
// interleave, nr L of them over the cell
template <int L>
__device__ inline double next_point(const EigState& S, int k, int r, int nr) {
  const bool vl = S.clo >= 0, vh = S.chi >= 0;
  if (!vl || !vh) {
    if (!vl && !vh) {
      if (L == 1) return S.lo;
      if (L == 2) return k == 0 ? S.lo : S.hi;
      const double pts[4] = {S.lo, S.hi, S.lo - S.pad, S.hi + S.pad};
      return pts[k & 3];
    }
    const double x = vl ? S.hi : S.lo;
    const double dir = vl ? 1.0 : -1.0;
    const double mult[4] = {0.0, 1.0, 4.0, 16.0};
    return x + dir * S.pad * mult[k & 3];
  }
  const double mid = 0.5 * (S.lo + S.hi);
  if (S.chi - S.clo == 1) {
    // Newton estimates from both ends; keep the shorter step that stays inside
    double tn = NAN, step = INFINITY;
    if (isfinite(S.glo) && S.glo != 0.0) {
      const double st = 1.0 / S.glo;
      const double c = S.lo - st;
      if (c > S.lo && c < S.hi && fabs(st) < step) { tn = c; step = fabs(st); }
    }
    if (isfinite(S.ghi) && S.ghi != 0.0) {
      const double st = 1.0 / S.ghi;
      const double c = S.hi - st;
      if (c > S.lo && c < S.hi && fabs(st) < step) { tn = c; step = fabs(st); }
    }
    if (tn == tn) {
      const double delta = fmax(2.0 * kEps * fabs(tn), 1e-3 * step);
      const bool far_hi = (S.hi - tn) > (tn - S.lo);
      double p;
      if (L == 1) {
        p = (step <= 2.0 * kEps * fabs(tn)) ? (far_hi ? tn + delta : tn - delta) : tn;
      } else if (L == 2) {
        p = (k == 0) ? tn : (far_hi ? tn + delta : tn - delta);
      } else {
        const double pts[4] = {tn, tn - delta, tn + delta, mid};
        p = pts[k & 3];
      }
      return (p > S.lo && p < S.hi) ? p : mid;
    }
  }
  return S.lo + (S.hi - S.lo) * ((double)(r * L + k + 1) / (double)(nr * L + 1));
}

// a count only moves a validated end inward, and never past the other
// validated end: counts from rounded arithmetic need not be monotone in the
// shift, and a bracket must not invert
__device__ __forceinline__ void apply_point(EigState& S, double p, int c, double g) {
  if (c <= S.j - 1) {
    if ((S.clo < 0 || p > S.lo) && (S.chi < 0 || p < S.hi)) { S.lo = p; S.clo = c; S.glo = g; }
  } else {
    if ((S.chi < 0 || p < S.hi) && (S.clo < 0 || p > S.lo)) { S.hi = p; S.chi = c; S.ghi = g; }
  }
}

template <int L>
__device__ inline void update_state(EigState& S, const double* p, const int* c, const double* g, bool vonly) {
  double pmin = INFINITY, pmax = -INFINITY;
  for (int q = 0; q < L; ++q) {
    pmin = fmin(pmin, p[q]);
    pmax = fmax(pmax, p[q]);
    if (c[q] <= S.j - 1) {
      if ((S.clo < 0 || p[q] > S.lo) && (S.chi < 0 || p[q] < S.hi)) { S.lo = p[q]; S.clo = c[q]; S.glo = g[q]; }
    } else {
      if ((S.chi < 0 || p[q] < S.hi) && (S.clo < 0 || p[q] > S.lo)) { S.hi = p[q]; S.chi = c[q]; S.ghi = g[q]; }
    }
  }
  if (S.clo < 0) { S.lo = fmin(pmin, S.hi) - S.pad; S.pad *= 4.0; }
  if (S.chi < 0) { S.hi = fmax(pmax, S.lo) + S.pad; S.pad *= 4.0; }
  S.done = (S.clo >= 0 && S.chi >= 0 && (vonly || bracket_converged(S.lo, S.hi))) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// rows of a representation shared by a whole wavefront, staged through LDS in
// groups of kSG rows: while one group is consumed (LDS broadcast reads), lane
// l already holds doubles l, l + 64, l + 128, l + 192 of the next one, loaded
// with four coalesced 512-byte wavefront loads -- one wait per group instead
// of one per row.  body(i, D, L, LD, LLD) runs for i = 0 .. n - 1 in order.
// st: 2 * 4 * kSG doubles of LDS; every lane of the wavefront must call.

constexpr int kSG = 64;

// as staged_rows, for the first nrow <= n rows, with group(g0) called at the
// start of every group (before its rows) and body(i, j, D, L, LD, LLD) given
// the row's position j = i - g0 inside its group
template <class Group, class Body>
__device__ inline void staged_rows_g(const double* __restrict__ Rd, int n, int nrow, double* __restrict__ st,
                                     Group&& group, Body&& body) {
  const int lane = threadIdx.x & 63;
  const int64_t n4 = 4 * (int64_t)n;
  double q[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t idx = lane + 64 * k;
    q[k] = (idx < n4) ? Rd[idx] : 0.0;
  }
  for (int g0 = 0; g0 < nrow; g0 += kSG) {
    double* buf = st + ((g0 / kSG) & 1) * (4 * kSG);
#pragma unroll
    for (int k = 0; k < 4; ++k) buf[lane + 64 * k] = q[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t idx = (int64_t)(g0 + kSG) * 4 + lane + 64 * k;
      q[k] = (idx < n4) ? Rd[idx] : 0.0;
    }
    group(g0);
    const int m = min(kSG, nrow - g0);
#pragma unroll 8
    for (int j = 0; j < m; ++j) body(g0 + j, j, buf[4 * j], buf[4 * j + 1], buf[4 * j + 2], buf[4 * j + 3]);
  }
}

template <class Body>
__device__ inline void staged_rows(const double* __restrict__ Rd, int n, double* __restrict__ st, Body&& body) {
  staged_rows_g(Rd, n, n, st, [](int) {},
                [&](int i, int, double D, double L, double LD, double LLD) { body(i, D, L, LD, LLD); });
}

// a value equal in every lane, made visibly wave-uniform (scalar registers)
__device__ __forceinline__ long long uniform_ll(long long x) {
  const unsigned long long u = (unsigned long long)x;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Sturm count plus log-derivative (as sturm_count_deriv) for a wavefront
// whose lanes share the representation
__device__ inline int staged_count_deriv(const double* __restrict__ Rd, int n, double tau, double pivmin,
                                         double* __restrict__ st, double* g_out) {
  double s = -tau, ds = -1.0, g = 0.0;
  int c = 0;
  // no zero-pivot guard in this pass: a zero or tiny pivot ends in a
  // non-finite s, answered by the guarded recount below
  staged_rows(Rd, n, st, [&](int, double D, double, double, double LLD) {
    const double dp = D + s;
    c += (dp < 0.0) ? 1 : 0;
    const double inv = rcp_nr1(dp);
    const double dsi = ds * inv;
    g += dsi;
    // the last row has LLD = 0; its update is harmless
    ds = fma(LLD * D, dsi * inv, -1.0);
    s = fma(s * inv, LLD, -tau);
  });
  if (!isfinite(s) || !isfinite(g)) {
    c = sturm_count(reinterpret_cast<const Rep*>(Rd), n, tau, pivmin);
    g = NAN;
  }
  *g_out = g;
  return c;
}

// Sturm count as sturm_count (same arithmetic, bit for bit) for a wavefront
// whose lanes share the representation; the last row's LLD is 0, so its
// update of s is harmless
__device__ inline int staged_count(const double* __restrict__ Rd, int n, double tau, double pivmin,
                                   double* __restrict__ st) {
  double s = -tau;
  int c = 0;
  staged_rows(Rd, n, st, [&](int, double D, double, double, double LLD) {
    double dp = D + s;
    dp = (fabs(dp) < pivmin) ? -pivmin : dp;
    c += (dp < 0.0) ? 1 : 0;
    double t = s * rcp_nr1(dp);
    t = (t != t) ? 1.0 : t;
    s = fma(t, LLD, -tau);
  });
  return c;
}

// ---------------------------------------------------------------------------
// 3. eigenvalue brackets (continued): the grid of Sturm counts per block

__global__ void __launch_bounds__(64) k_grid(const Block* __restrict__ B, int nblk, const int64_t* __restrict__ goff,
                                             int64_t gtot, const Rep* __restrict__ pool, int32_t* __restrict__ gcnt) {
  const int64_t t0 = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t t = t0 < gtot ? t0 : gtot - 1;  // tail lanes repeat the last point
  const int b = find_segment(goff, nblk, t);
  const Block blk = B[b];
  const int k = (int)(t - goff[b]);
  const double x = grid_point(blk.glo, blk.ghi, k, blk.gP);
  const int b0 = __shfl(b, 0, 64);
  int c;
  if (__ballot(b != b0) == 0) {
    __shared__ double st[2 * 4 * kSG];
    c = staged_count(reinterpret_cast<const double*>(pool + blk.row0), __builtin_amdgcn_readfirstlane(blk.n), x,
                     blk.pivmin, st);
  } else {
    c = sturm_count(pool + blk.row0, blk.n, x, blk.pivmin);
  }
  if (t0 < gtot) gcnt[t0] = c;
}

template <int L>
__device__ inline long long refine_sweeps(EigState& S, bool act, const Rep* __restrict__ R, int n, double pivmin,
                                          int k, int gbase, double* __restrict__ st, bool vonly, bool share_ok) {
  // with one representation for the whole wavefront (st), every count is
  // valid for every eigenvalue of it: with share_ok, the groups that share a
  // bracket holding several eigenvalues spread their points over it, and
  // every group takes all 64 counts of the sweep
  constexpr int G = 64 / L;  // eigenvalue groups per wavefront
  const bool share = share_ok && st != nullptr;
  const int lane = threadIdx.x & 63;
  const int g = gbase / L;
  long long steps = 0;
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    const bool need = act && !S.done;
    if (__ballot(need) == 0) break;
    int r = 0, nr = 1;
    if (share) {
      // groups with the same validated multi-eigenvalue bracket are adjacent
      // (consecutive indices): rank r in their run of nr groups
      const bool cell = need && S.clo >= 0 && S.chi >= 0 && S.chi - S.clo > 1;
      const int src = g > 0 ? lane - L : lane;
      const double plo = __shfl(S.lo, src, 64), phi = __shfl(S.hi, src, 64);
      const int pclo = __shfl(S.clo, src, 64), pchi = __shfl(S.chi, src, 64);
      const bool pcell = __shfl(cell ? 1 : 0, src, 64) != 0;
      const bool same = g > 0 && cell && pcell && plo == S.lo && phi == S.hi && pclo == S.clo && pchi == S.chi;
      int head = same ? 0 : g;  // index of the run's first group (prefix max)
      int next = same ? G : g;  // first run start at or after a group (suffix min)
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const int hb = __shfl(head, max(lane - d * L, 0), 64);
        const int na = __shfl(next, min(lane + d * L, 63), 64);
        if (g >= d) head = max(head, hb);
        if (g + d < G) next = min(next, na);
      }
      // the run ends where the next group starts a new run
      int end = __shfl(next, min(lane + L, 63), 64);
      if (g + 1 >= G) end = G;
      r = g - head;
      nr = end - head;
    }
    const double p = need ? next_point<L>(S, k, r, nr) : 0.0;
    double gv;
    const int c = st ? staged_count_deriv(reinterpret_cast<const double*>(R), n, p, pivmin, st, &gv)
                     : sturm_count_deriv(R, n, p, pivmin, &gv);
    if (need) steps += n;
    if (share) {
      // own points bound an unvalidated end; every point of the wavefront
      // moves a validated one
      double pmin = INFINITY, pmax = -INFINITY;
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const double pq = __shfl(p, gbase + q, 64);
        pmin = fmin(pmin, pq);
        pmax = fmax(pmax, pq);
      }
      for (int q = 0; q < 64; ++q) {
        const double pq = __shfl(p, q, 64);
        const int cq = __shfl(c, q, 64);
        const double gq = __shfl(gv, q, 64);
        if (need) apply_point(S, pq, cq, gq);
      }
      if (need) {
        if (S.clo < 0) { S.lo = fmin(pmin, S.hi) - S.pad; S.pad *= 4.0; }
        if (S.chi < 0) { S.hi = fmax(pmax, S.lo) + S.pad; S.pad *= 4.0; }
        S.done = (S.clo >= 0 && S.chi >= 0 && (vonly || bracket_converged(S.lo, S.hi))) ? 1 : 0;
      }
    } else {
      double pq[L], gq[L];
      int cq[L];
#pragma unroll
      for (int q = 0; q < L; ++q) {
        pq[q] = __shfl(p, gbase + q, 64);
        cq[q] = __shfl(c, gbase + q, 64);
        gq[q] = __shfl(gv, gbase + q, 64);
      }
      if (need) update_state<L>(S, pq, cq, gq, vonly);
    }
  }
  return steps;
}

template <int L>
__global__ void __launch_bounds__(64) k_refine(const Block* __restrict__ B, const Node* __restrict__ N,
                                               int64_t ntot, const int32_t* __restrict__ sblk,
                                               const int32_t* __restrict__ snode, const Rep* __restrict__ pool,
                                               double* __restrict__ lo_a, double* __restrict__ hi_a,
                                               int32_t* __restrict__ clo_a, int32_t* __restrict__ chi_a,
                                               uint32_t* __restrict__ sflag, Counters* __restrict__ C, int vonly,
                                               const int64_t* __restrict__ cstart, const int32_t* __restrict__ rid,
                                               int nchunks, int share) {
  const int lane = threadIdx.x;
  const int k = lane % L, gbase = lane - k;
  // eigenvalues of the wavefront: 64 / L consecutive slots, or (cstart) the
  // slots of one chunk of equal-node slots needing refinement
  int64_t s;
  bool act;
  if (cstart != nullptr) {
    if ((int)blockIdx.x >= nchunks) return;
    const int64_t first = cstart[blockIdx.x];
    s = first + lane / L;
    act = s < ntot && rid[s] == rid[first];
  } else {
    s = (int64_t)blockIdx.x * (64 / L) + lane / L;
    act = (s < ntot) && (sflag[s] & F_NEEDS_REFINE);
  }
  const uint64_t am = __ballot(act);
  if (am == 0) return;
  const int64_t sf = __shfl(s, first_lane(am), 64);
  const int64_t ss = act ? s : sf;  // idle lanes shadow a valid slot
  const Block blk = B[sblk[ss]];
  const Node nd = N[snode[ss]];
  EigState S;
  S.lo = lo_a[ss];
  S.hi = hi_a[ss];
  S.clo = clo_a[ss];
  S.chi = chi_a[ss];
  S.glo = NAN;
  S.ghi = NAN;
  S.j = (int)(ss - blk.row0) + 1;
  S.pad = fmax(fmax(S.hi - S.lo, 4.0 * kEps * fmax(fabs(S.lo), fabs(S.hi))), blk.pivmin);
  S.done = (S.clo >= 0 && S.chi >= 0 && (vonly || bracket_converged(S.lo, S.hi))) ? 1 : 0;
  const int64_t rep0 = __shfl(nd.rep, first_lane(am), 64);
  long long steps;
  if (__ballot(nd.rep != rep0) == 0) {
    __shared__ double st[2 * 4 * kSG];
    // per-lane copy of the (equal) pointer keeps the staged loads global
    steps = refine_sweeps<L>(S, act, pool + nd.rep, __builtin_amdgcn_readfirstlane(blk.n), blk.pivmin, k, gbase,
                             st, vonly != 0, share != 0);
  } else {
    steps = refine_sweeps<L>(S, act, pool + nd.rep, blk.n, blk.pivmin, k, gbase, nullptr, vonly != 0, false);
  }
  if (act && k == 0) {
    lo_a[s] = S.lo;
    hi_a[s] = S.hi;
    clo_a[s] = S.clo;
    chi_a[s] = S.chi;
    uint32_t fl = sflag[s] & ~F_NEEDS_REFINE;
    if (S.clo >= 0 && S.chi >= 0 && bracket_converged(S.lo, S.hi)) fl |= F_ACCURATE;
    sflag[s] = fl;
  }
  // each lane evaluated its own points: count all of them
  if (act) atomicAdd(&C->sturm_steps, (unsigned long long)steps);
}

// Refinement by persistent wavefronts over node runs (maximal runs of
// flagged slots of one node; at the root level, whole blocks).  A wavefront
// starts on the run of its chunk; its lane groups claim that run's eigenvalues
// one at a time from the run's counter, and a group whose eigenvalue has
// converged writes it back and claims the next.  Once the run has nothing
// left to claim and every group is idle, the wavefront takes the next chunk
// from a global cursor and moves to its run.  Every eigenvalue is refined on
// its own L points exactly as in k_refine without shared points (the same
// points, counts and updates in the same order), so its result does not
// depend on which wavefront or group took it; only the load balance differs.
// claim: one counter per run, zero on entry; cursor: gridDim.x on entry.
template <int L>
__global__ void __launch_bounds__(64) k_refine_fill(const Block* __restrict__ B, const Node* __restrict__ N,
                                                    int64_t ntot, const int32_t* __restrict__ sblk,
                                                    const int32_t* __restrict__ snode, const Rep* __restrict__ pool,
                                                    double* __restrict__ lo_a, double* __restrict__ hi_a,
                                                    int32_t* __restrict__ clo_a, int32_t* __restrict__ chi_a,
                                                    uint32_t* __restrict__ sflag, Counters* __restrict__ C,
                                                    const int64_t* __restrict__ cstart, const int32_t* __restrict__ rid,
                                                    const int64_t* __restrict__ rstart, int nchunks,
                                                    int32_t* __restrict__ claim, int32_t* __restrict__ cursor) {
  __shared__ double st[2 * 4 * kSG];
  const int lane = threadIdx.x;
  const int k = lane % L, gbase = lane - k;
  long long steps = 0;
  int c = blockIdx.x;
  while (c < nchunks) {
    const int q = __builtin_amdgcn_readfirstlane(rid[cstart[c]]);
    const int64_t r0 = rstart[q];
    const Block blk = B[sblk[r0]];
    const Node nd = N[snode[r0]];
    const Rep* R = pool + nd.rep;
    const int n = __builtin_amdgcn_readfirstlane(blk.n);
    EigState S;
    int64_t s = -1;        // this group's slot, -1 when idle
    bool open = true;      // the run may still hold unclaimed eigenvalues
    int sweeps = 0;
    for (;;) {
      // settle (every lane runs this loop; the groups diverge only inside):
      // write back converged eigenvalues (or those at the sweep cap) and claim
      // the run's next ones until every group holds one that needs a sweep or
      // the run has none left for it
      for (;;) {
        if (s >= 0 && (S.done || sweeps >= kMaxSweeps)) {
          if (k == 0) {
            lo_a[s] = S.lo;
            hi_a[s] = S.hi;
            clo_a[s] = S.clo;
            chi_a[s] = S.chi;
            uint32_t fl = sflag[s] & ~F_NEEDS_REFINE;
            if (S.clo >= 0 && S.chi >= 0 && bracket_converged(S.lo, S.hi)) fl |= F_ACCURATE;
            sflag[s] = fl;
          }
          s = -1;
        }
        const bool want = s < 0 && open;
        if (__ballot(want) == 0) break;
        if (want) {
          int idx = 0;
          if (k == 0) idx = atomicAdd(&claim[q], 1);
          idx = __shfl(idx, gbase, 64);
          const int64_t t = r0 + idx;
          if (t < ntot && rid[t] == q) {
            s = t;
            S.lo = lo_a[s];
            S.hi = hi_a[s];
            S.clo = clo_a[s];
            S.chi = chi_a[s];
            S.glo = NAN;
            S.ghi = NAN;
            S.j = (int)(s - blk.row0) + 1;
            S.pad = fmax(fmax(S.hi - S.lo, 4.0 * kEps * fmax(fabs(S.lo), fabs(S.hi))), blk.pivmin);
            S.done = (S.clo >= 0 && S.chi >= 0 && bracket_converged(S.lo, S.hi)) ? 1 : 0;
            sweeps = 0;
          } else {
            open = false;
          }
        }
      }
      if (__ballot(s >= 0) == 0) break;
      const bool need = s >= 0;
      const double p = need ? next_point<L>(S, k, 0, 1) : 0.0;
      double gv;
      const int cnt = staged_count_deriv(reinterpret_cast<const double*>(R), n, p, blk.pivmin, st, &gv);
      if (need) steps += n;
      double pq[L], gq[L];
      int cq[L];
#pragma unroll
      for (int u = 0; u < L; ++u) {
        pq[u] = __shfl(p, gbase + u, 64);
        cq[u] = __shfl(cnt, gbase + u, 64);
        gq[u] = __shfl(gv, gbase + u, 64);
      }
      if (need) {
        update_state<L>(S, pq, cq, gq, false);
        ++sweeps;
      }
    }
    // the run is exhausted for this wavefront: the next chunk's run
    int nc = 0;
    if (lane == 0) nc = atomicAdd(cursor, 1);
    c = __shfl(nc, 0, 64);
  }
  if (steps) atomicAdd(&C->sturm_steps, (unsigned long long)steps);
}

// claim counters of k_refine_fill cleared, its cursor set to the grid size
__global__ void k_fill_init(int64_t nclaim, int32_t* __restrict__ claim, int32_t* __restrict__ cursor, int grid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nclaim) claim[i] = 0;
  if (i == 0) *cursor = grid;
}

// singletons whose bracket is not at full accuracy in their leaf's frame
__global__ void k_mark_leaf(int64_t ntot, const int64_t* __restrict__ scol, uint32_t* __restrict__ sflag) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const uint32_t fl = sflag[s];
  if ((fl & F_SINGLETON) && scol[s] >= 0 && !(fl & F_ACCURATE)) sflag[s] = fl | F_NEEDS_REFINE;
}

// ---------------------------------------------------------------------------
// 5. output columns: single-block problems map local indices directly; with
//    several blocks the rank of each eigenvalue in its problem is found by
//    binary search in the (running-maximum) value lists of the other blocks.

__global__ void k_cummax(const Block* __restrict__ B, int nblk, const Node* __restrict__ N,
                         const double* __restrict__ lo, const double* __restrict__ hi, const Problem* __restrict__ P,
                         double* __restrict__ val) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const Block blk = B[b];
  if (P[blk.prob].nblk <= 1) return;
  const double acc = N[b].acc;
  double run = -INFINITY;
  for (int i = 0; i < blk.n; ++i) {
    const int64_t s = blk.row0 + i;
    run = fmax(run, acc + 0.5 * (lo[s] + hi[s]));
    val[s] = run;
  }
}

__device__ inline int count_below(const double* v, int n, double x, bool inclusive) {
  // number of entries < x (or <= x when inclusive) in ascending v[0..n)
  int a = 0, z = n;
  while (a < z) {
    const int mid = (a + z) >> 1;
    const bool below = inclusive ? (v[mid] <= x) : (v[mid] < x);
    if (below)
      a = mid + 1;
    else
      z = mid;
  }
  return a;
}

__global__ void k_columns(const Problem* __restrict__ P, Block* __restrict__ B, int64_t ntot,
                          const int32_t* __restrict__ sblk, const double* __restrict__ val, int64_t* __restrict__ scol) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int b = sblk[s];
  const Block blk = B[b];
  const Problem pr = P[blk.prob];
  const int j = (int)(s - blk.row0) + 1;
  int64_t col = -1;
  if (pr.nblk <= 1) {
    if (j >= blk.wl && j <= blk.wu) col = j - blk.wl;
  } else {
    const double x = val[s];
    int64_t rank = j - 1;
    for (int bb = pr.first_blk; bb < pr.first_blk + pr.nblk; ++bb) {
      if (bb == b) continue;
      const Block o = B[bb];
      rank += count_below(val + o.row0, o.n, x, bb < b);
    }
    if (pr.kind == 0) {
      col = rank;
    } else if (pr.kind == 1) {
      if (rank >= pr.il - 1 && rank <= pr.iu - 1) col = rank - (pr.il - 1);
    } else {
      if (j >= blk.wl && j <= blk.wu) {
        col = rank - pr.below;
        if (col < 0 || col >= pr.m) col = -1;
      }
    }
  }
  scol[s] = col;
}

// for multi-block INDEX problems: the wanted local range of each block
__global__ void k_block_wanted(Block* __restrict__ B, int nblk, const Problem* __restrict__ P,
                               const int64_t* __restrict__ scol) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  Block blk = B[b];
  if (!(P[blk.prob].kind == 1 && P[blk.prob].nblk > 1)) return;
  int wl = blk.n + 1, wu = 0;
  for (int i = 0; i < blk.n; ++i)
    if (scol[blk.row0 + i] >= 0) {
      wl = min(wl, i + 1);
      wu = max(wu, i + 1);
    }
  B[b].wl = wl;
  B[b].wu = wu;
}

// ---------------------------------------------------------------------------
// 6. classification of the active nodes' indices into runs

__device__ inline bool rel_break(double lo_j, double hi_j, double lo_k, double hi_k, double gaptol) {
  const double mj = 0.5 * (lo_j + hi_j);
  const double mk = 0.5 * (lo_k + hi_k);
  return (lo_k - hi_j) >= gaptol * fmax(fabs(mj), fabs(mk));
}

// absolute gap of slot s to its neighbours within node nd (the node's outer gaps
// at its ends), from the brackets of the node's frame
__device__ inline double slot_gap(const Node& nd, int64_t row0, int64_t s, const double* __restrict__ lo,
                                  const double* __restrict__ hi) {
  const int j = (int)(s - row0) + 1;
  const double gl = (j == nd.f) ? nd.gapl : lo[s] - hi[s - 1];
  const double gr = (j == nd.l) ? nd.gapr : lo[s + 1] - hi[s];
  return fmax(fmin(gl, gr), 0.0);
}

__global__ void k_cls_flags(const Block* __restrict__ B, const Node* __restrict__ N, int64_t ntot,
                            const int32_t* __restrict__ sblk, const int32_t* __restrict__ snode,
                            const double* __restrict__ lo, const double* __restrict__ hi,
                            uint32_t* __restrict__ sflag, int32_t* __restrict__ runflag, Counters* __restrict__ C) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const uint32_t fl = sflag[s];
  int start = 0;
  if (fl & F_ACTIVE) {
    const Block blk = B[sblk[s]];
    const Node nd = N[snode[s]];
    const int j = (int)(s - blk.row0) + 1;
    if (j == nd.f) {
      start = 1;
    } else {
      const double l0 = lo[s - 1], h0 = hi[s - 1], l1 = lo[s], h1 = hi[s];
      start = rel_break(l0, h0, l1, h1, blk.gaptol);
      // the decision is ambiguous when the bracket widths could flip it
      const uint32_t fp = sflag[s - 1];
      if (!((fp & F_ACCURATE) && (fl & F_ACCURATE))) {
        const double m0 = 0.5 * (l0 + h0), m1 = 0.5 * (l1 + h1);
        const double margin = (l1 - h0) - blk.gaptol * fmax(fabs(m0), fabs(m1));
        const double unc = 2.0 * ((h0 - l0) + (h1 - l1));
        if (fabs(margin) <= unc) {
          if (!(fp & F_ACCURATE)) atomicOr(&sflag[s - 1], F_NEEDS_REFINE);
          if (!(fl & F_ACCURATE)) atomicOr(&sflag[s], F_NEEDS_REFINE);
          atomicAdd(&C->ambiguous, 1);
        }
      }
    }
  }
  runflag[s] = start;
}

__global__ void k_cls_compact(int64_t ntot, const int32_t* __restrict__ runflag, const int32_t* __restrict__ runid,
                              int64_t* __restrict__ runs) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  if (runflag[s]) runs[runid[s]] = s;
}

__global__ void k_cls_runs(const Block* __restrict__ B, const Node* __restrict__ N, int nruns,
                           const int64_t* __restrict__ runs, const int32_t* __restrict__ sblk,
                           const int32_t* __restrict__ snode, const double* __restrict__ lo,
                           const double* __restrict__ hi, const int64_t* __restrict__ scol,
                           uint32_t* __restrict__ sflag, double* __restrict__ sgap, Cluster* __restrict__ clusters,
                           int max_clusters, Counters* __restrict__ C, int max_depth) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nruns) return;
  const int64_t s = runs[r];
  const int b = sblk[s];
  const Block blk = B[b];
  const int node = snode[s];
  const Node nd = N[node];
  const int64_t last = blk.row0 + nd.l - 1;
  int64_t e = last;
  if (r + 1 < nruns) e = min(e, runs[r + 1] - 1);
  const int a = (int)(s - blk.row0) + 1;
  const int z = (int)(e - blk.row0) + 1;
  const bool overlap = !(z < blk.wl || a > blk.wu);
  if (!overlap) return;
  if (a == z) {
    if (scol[s] >= 0) {
      sflag[s] |= F_SINGLETON;
      sgap[s] = slot_gap(nd, blk.row0, s, lo, hi);
    }
    return;
  }
  if (nd.depth + 1 > max_depth) {
    set_status(C, 2);
    for (int64_t q = s; q <= e; ++q)
      if (scol[q] >= 0) {
        sflag[q] |= F_SINGLETON;
        sgap[q] = slot_gap(nd, blk.row0, q, lo, hi);
      }
    return;
  }
  const int k = atomicAdd(&C->nclusters, 1);
  if (k >= max_clusters) {
    set_status(C, 3);
    return;
  }
  Cluster cl;
  cl.node = node;
  cl.f = a;
  cl.l = z;
  cl.pad = 0;
  cl.gapl = (a == nd.f) ? nd.gapl : lo[s] - hi[s - 1];
  cl.gapr = (z == nd.l) ? nd.gapr : lo[e + 1] - hi[e];
  clusters[k] = cl;
  atomicAdd(&C->cluster_rows, (unsigned long long)blk.n);
}

// ---------------------------------------------------------------------------
// 7. child representations: one wavefront per cluster.  Pass 1: lanes evaluate
//    kChildCand candidate shifts -- both ends of the cluster, each with margins
//    growing geometrically from the end eigenvalue's bracket to half the outer
//    gap -- by the stationary qds
//      s_1 = -sigma, D+_i = D_i + s_i, L+_i = LD_i / D+_i, s_{i+1} = L+_i L_i s_i - sigma
//    over LDS-staged parent rows, keeping the element growth max|D+_i| and
//    the value of s_i every kSG rows (checkpoints).  The closest shift whose
//    growth is within the bound wins (ties between the two ends: the smaller
//    growth); without one, the least growth.  Pass 2 writes the winner's
//    rows: every lane recomputes the segments of kSG rows that start at its
//    checkpoints (the same arithmetic from the same s_i, so the rows equal a
//    sequential pass bit for bit), which takes a 64th of the sequential
//    chain.

constexpr int kChildLevels = 8;
constexpr int kChildCand = 2 * kChildLevels;
static_assert(kChildCand == 16 && kSG == 64, "child checkpoints: 16 candidates every 64 rows (child_ck_rows)");

__device__ inline double child_sigma(const Cluster& cl, const Block& blk, const double* __restrict__ lo,
                                     const double* __restrict__ hi, int cand, bool* valid) {
  const int64_t sa = blk.row0 + cl.f - 1, sb = blk.row0 + cl.l - 1;
  const int side = cand & 1, lev = cand >> 1;
  const int64_t se = side ? sb : sa;
  const double l0 = lo[se], h0 = hi[se];
  const double d0 = fmax(4.0 * kEps * fabs(0.5 * (l0 + h0)), h0 - l0);
  const double avgap = (hi[sb] - lo[sa]) / (double)(cl.l - cl.f);
  const double gside = side ? cl.gapr : cl.gapl;
  const double dmax = fmin(0.5 * gside, fmax(2.0 * avgap, d0));
  double delta = d0;
  *valid = true;
  if (lev > 0) {
    if (!(dmax > d0)) {
      *valid = false;
    } else {
      delta = d0 * pow(dmax / d0, (double)lev / (double)(kChildLevels - 1));
    }
  }
  return side ? h0 + delta : l0 - delta;
}

// one row of the stationary qds transform of a child candidate: the pivot,
// multiplier and products of row i from the parent row (D, L, LD) and s_i;
// returns s_{i+1}.  Both passes of k_child use it, so pass 2 repeats pass 1
// bit for bit.
__device__ __forceinline__ double child_row(double D, double L, double LD, double sv, double sigma, double& dp,
                                            double& lp, double& ld, double& lld) {
  dp = D + sv;
  lp = LD * rcp_nr2(dp);
  ld = lp * dp;
  lld = ld * lp;
  return fma(lp * L, sv, -sigma);
}

// One wavefront per cluster: lanes 0 .. kChildCand-1 evaluate the candidate
// shifts (pass 1), then all 64 lanes write the winner's rows from its
// checkpoints (pass 2).  Pool use per cluster: the child's n rows and, after
// them, the checkpoints of every candidate (kChildCand x ceil(n / kSG)
// doubles).
__global__ void __launch_bounds__(64) k_child(const Block* __restrict__ B, Node* __restrict__ N, int nclusters,
                                              int node_base, const Cluster* __restrict__ clusters,
                                              const double* __restrict__ lo, const double* __restrict__ hi,
                                              Rep* __restrict__ pool, unsigned long long pool_cap,
                                              Counters* __restrict__ C, double growth_limit) {
  __shared__ double st[2 * 4 * kSG];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const Cluster cl = clusters[c];
  const Node par = N[cl.node];
  const Block blk = B[par.blk];
  const int n = __builtin_amdgcn_readfirstlane(blk.n);
  const int nseg = (n + kSG - 1) / kSG;
  const double* Rd = reinterpret_cast<const double*>(pool + par.rep);
  const unsigned long long rows = (unsigned long long)n + (unsigned long long)child_ck_rows(n);
  long long base = -1;
  if (lane == 0) {
    base = (long long)atomicAdd(&C->pool_used, rows);
    if ((unsigned long long)base + rows > pool_cap) {
      set_status(C, 3);
      base = -1;
    }
  }
  base = uniform_ll(__shfl(base, 0, 64));
  // checkpoints: ck[cand * nseg + g] = s at row g kSG of candidate cand
  double* const ck = reinterpret_cast<double*>(pool + (base >= 0 ? base + n : 0));
  const bool cand_lane = lane < kChildCand;
  bool valid = false;
  double sigma = 0.0;
  if (cand_lane) sigma = child_sigma(cl, blk, lo, hi, lane, &valid);
  // pass 1: growth and checkpoints of every candidate (rows 0 .. n-2; the last row has no L)
  double sv = -sigma, gmax = 0.0, chk = 0.0;
  // chk: x * 0 is NaN exactly when x is infinite or NaN, so chk stays 0
  // while every pivot and multiplier is finite (a check kept off the
  // recurrence's dependency chain)
  staged_rows_g(
      Rd, n, n - 1, st,
      [&](int g0) {
        if (cand_lane && base >= 0) ck[lane * nseg + g0 / kSG] = sv;
      },
      [&](int, int, double D, double L, double LD, double) {
        double dp, lp, ld, lld;
        sv = child_row(D, L, LD, sv, sigma, dp, lp, ld, lld);
        gmax = fmax(gmax, fabs(dp));
        chk = fma(dp, 0.0, chk);
        chk = fma(lp, 0.0, chk);
      });
  bool fin = isfinite(chk);
  const double dlast = Rd[4 * (int64_t)(n - 1)] + sv;
  gmax = fmax(gmax, fabs(dlast));
  fin = fin && isfinite(dlast);
  const double growth = (valid && fin) ? gmax : INFINITY;
  double gr[kChildCand];
#pragma unroll
  for (int k = 0; k < kChildCand; ++k) gr[k] = __shfl(growth, k, 64);
  // the same decision in every lane (identical inputs)
  const double bound = kGrowthBound * (blk.gu - blk.gl);
  int pick = -1;
  for (int lev = 0; lev < kChildLevels && pick < 0; ++lev) {
    const double a = gr[2 * lev], b = gr[2 * lev + 1];
    if (a <= bound || b <= bound) pick = (a <= b) ? 2 * lev : 2 * lev + 1;
  }
  const bool forced = pick < 0;
  if (forced) {
    double best = INFINITY;
    for (int k = 0; k < kChildCand; ++k)
      if (gr[k] < best) {
        best = gr[k];
        pick = k;
      }
  }
  // optional hard limit on the element growth (caller's setting): without an
  // acceptable candidate the cluster gets no child (status 1)
  if (pick >= 0 && growth_limit > 0.0 && !(gr[pick] <= growth_limit * (blk.gu - blk.gl))) pick = -1;
  const long long off = uniform_ll((pick < 0 || base < 0) ? -1 : base);
  bool v;
  const double sg = (pick >= 0) ? child_sigma(cl, blk, lo, hi, pick, &v) : 0.0;
  const double dl = __shfl(dlast, pick >= 0 ? pick : 0, 64);
  if (lane == 0) {
    if (forced) atomicAdd(&C->child_reject, 1ull);
    Node nd;
    nd.blk = par.blk;
    nd.parent = cl.node;
    nd.f = cl.f;
    nd.l = cl.l;
    nd.gapl = cl.gapl;
    nd.gapr = cl.gapr;
    nd.pad = 0;
    if (off < 0) {
      if (pick < 0) set_status(C, 1);
      nd.growth = INFINITY;
      nd.rep = -1;
      nd.acc = par.acc;
      nd.sigma = 0.0;
      nd.depth = -1;
    } else {
      nd.rep = off;
      nd.growth = gr[pick] / (blk.gu - blk.gl);
      nd.acc = par.acc + sg;
      nd.sigma = sg;
      nd.depth = par.depth + 1;
      atomicMax(&C->max_depth, nd.depth);
      atomicAdd(&C->qds_steps, (unsigned long long)n);
      atomicAdd(&C->child_steps, (unsigned long long)n);
    }
    N[node_base + c] = nd;
  }
  if (off < 0) return;
  // pass 2: lane l writes segments l, l + 64, ... of the winner, each from its checkpoint
  double* const Q = reinterpret_cast<double*>(pool + off);
  for (int g = lane; g < nseg; g += 64) {
    double s2 = ck[pick * nseg + g];
    const int i0 = g * kSG, i1 = min(i0 + kSG, n - 1);
#pragma unroll 4
    for (int i = i0; i < i1; ++i) {
      const double* row = Rd + 4 * (int64_t)i;
      double dp, lp, ld, lld;
      s2 = child_row(row[0], row[1], row[2], s2, sg, dp, lp, ld, lld);
      double* q = Q + 4 * (int64_t)i;
      q[0] = dp;
      q[1] = lp;
      q[2] = ld;
      q[3] = lld;
    }
  }
  if (lane == 0) {
    double* q = Q + 4 * (int64_t)(n - 1);
    q[0] = dl;
    q[1] = 0.0;
    q[2] = 0.0;
    q[3] = 0.0;
  }
}

// move the cluster's brackets into the child's frame (or, without a child,
// hand its wanted eigenvalues to the parent as singletons)
__global__ void k_shift(const Block* __restrict__ B, const Node* __restrict__ N, int node_base,
                        const Cluster* __restrict__ clusters, const int64_t* __restrict__ scol,
                        double* __restrict__ lo, double* __restrict__ hi, int32_t* __restrict__ clo,
                        int32_t* __restrict__ chi, int32_t* __restrict__ snode, uint32_t* __restrict__ sflag,
                        double* __restrict__ sgap) {
  const int c = blockIdx.x;
  const Node nd = N[node_base + c];
  const Block blk = B[nd.blk];
  for (int j = nd.f + (int)threadIdx.x; j <= nd.l; j += blockDim.x) {
    const int64_t s = blk.row0 + j - 1;
    uint32_t fl = sflag[s] & ~(F_ACTIVE | F_RUNSTART);
    if (nd.depth < 0) {
      if (scol[s] >= 0) {
        fl |= F_SINGLETON;
        sgap[s] = slot_gap(nd, blk.row0, s, lo, hi);
      }
      sflag[s] = fl;
      continue;
    }
    // the child's eigenvalue is the parent's minus sigma up to the effect of the
    // relative perturbations of the mixed stable transform (at most O(n eps)
    // relative to the parent's eigenvalue): a generous pad.  Classification
    // refines (validates by counts) every pair whose decision the pads could
    // flip, so the unrefined brackets only decide clear cases -- and pairs
    // near the gap threshold stay together, which keeps borderline
    // eigenvalues off poorly conditioned representations.
    const double l0 = lo[s], h0 = hi[s];
    const double pad = 4.0 * (double)blk.n * kEps * (fabs(l0) + fabs(h0)) + 4.0 * kEps * fabs(nd.sigma);
    lo[s] = (l0 - nd.sigma) - pad;
    hi[s] = (h0 - nd.sigma) + pad;
    clo[s] = -1;
    chi[s] = -1;
    snode[s] = node_base + c;
    sflag[s] = (fl & ~(F_ACCURATE | F_NEEDS_REFINE)) | F_ACTIVE;
  }
}

__global__ void k_clear_active(int64_t ntot, uint32_t* __restrict__ sflag) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  sflag[s] &= ~(F_ACTIVE | F_RUNSTART);
}

// ---------------------------------------------------------------------------
// 8. eigenvectors of singletons (Sec. 3.1.1, eq. errorangle): twisted
//    factorization of L D L^T - lam I, one solve per Rayleigh-quotient step.
//    Two lanes serve one eigenvector, up to 32 consecutive slots per wavefront:
//      lane 2c     top-down stationary transform
//                  s_1 = -lam,  s_{i+1} = s_i LLD_i / (D_i + s_i) - lam
//      lane 2c+1   bottom-up progressive transform
//                  p_n = D_n - lam,  p_i = p_{i+1} D_i / (LLD_i + p_{i+1}) - lam
//    Both are x' = x f / (b + x) - lam with (b, f) chosen by the lane's role;
//    a step also gives the quotient the solve needs, L+_i = LD_i / (D_i + s_i)
//    or U-_i = L_i D_i / (LLD_i + p_{i+1}).  Then
//      twist   gamma_k = s_k + p_k + lam, r = argmin |gamma_k| (ties: smallest k)
//      solve   z_r = 1; z_i = -L+_i z_{i+1} above the twist (lane 2c),
//              z_{i+1} = -U-_i z_i below it (lane 2c+1)
//      then    lam <- lam + gamma_r / ||z||^2 until the stopping rule holds.
//    Nothing of length n is stored per eigenvector: the transforms keep their
//    variable at the first row of every segment of kSeg rows (checkpoints), and
//    the twist search and the solve recompute one segment at a time from its
//    checkpoint, in registers, with the same operations and therefore the same
//    values.  After the last solve the vector is recomputed once more and
//    written to Z already normalized.  A solve reads the representation about
//    three times per lane and writes 2 n / kSeg doubles per lane pair.

// angle accepted for a singleton's vector: eps * max(n / 8, 4 log2 n), a
// small fraction of the O(n eps) orthogonality the method guarantees
__device__ inline double rqi_angle_tol(int n) {
  return kEps * fmax((double)n * 0.125, 4.0 * fmax(1.0, log2((double)n)));
}
struct VecState {
  double lam, lo, hi;
  double gap;    // absolute gap to the nearest other eigenvalue of the leaf
  double resid;  // smallest residual norm so far
  double best;   // lambda of that solve
  int stall;     // solves without a smaller residual
  double lam_out;
  double nrm;    // ||z||^2 of the committed solve
  double zmaxv;  // signed largest-magnitude entry of the committed solve
  long long qsteps;
  int rq;
  bool fallback;
};

// bookkeeping after one twisted solve of a lane still iterating: Rayleigh
// correction, stopping rule, next shift
__device__ inline void rqi_commit(VecState& V, bool& conv, bool& last, int it, int n, double gmin, double nrm,
                                  double zmaxv, double lam) {
  V.qsteps += 4ll * n;
  V.rq++;
  V.nrm = nrm;
  V.zmaxv = zmaxv;
  const double corr = gmin / nrm;
  const double resid = fabs(gmin) / sqrt(nrm);
  const double lamc = lam + corr;
  // the bracket comes from Sturm counts whose rounding differs from the
  // twisted factorization's; within a quarter of the gap of the bracket the
  // nearest eigenvalue is still this one
  const double slack = 0.25 * V.gap;
  const bool inside = (lamc >= V.lo - slack && lamc <= V.hi + slack);
  // resid / gap bounds the sine of the angle between z and the eigenvector
  // (gap theorem): such a solve is kept.  Once the correction is within
  // 2 eps |lambda| (two to four ulps, LAPACK's dlarrv tolerance) lambda cannot
  // improve, but z was solved at the uncorrected lambda and leans towards the
  // nearest other eigenvector by about |corr| / gap -- up to 2 eps / relgap,
  // a few thousand ulps for singletons near the classification threshold --
  // so one more solve at the corrected lambda is kept instead.  The floor
  // test: the first correction must halve the residual and every later one
  // cut the smallest residual so far by 32 (Rayleigh quotient iteration
  // converges cubically above the rounding floor, so a smaller cut means the
  // floor is reached).  There, or at the iteration cap, the solve with the
  // smallest residual is kept: the current one if it is that, else it is
  // repeated.
  const bool fine = resid <= rqi_angle_tol(n) * V.gap;
  const bool flat = fabs(corr) <= 2.0 * kEps * fabs(lam);
  const bool progress = resid < (it >= 1 ? 0.03125 : 0.5) * V.resid;
  const bool improved = resid < V.resid;
  if (improved) {
    V.resid = resid;
    V.best = lam;
  } else {
    V.stall++;
  }
  if (last || fine || (flat && (corr == 0.0 || !inside || it >= kMaxRqi))) {
    conv = true;
    V.lam_out = inside ? lamc : lam;
  } else if (flat) {
    V.lam = lamc;
    last = true;
  } else if (!progress || it + 1 >= kMaxRqi) {
    V.fallback = true;
    if (improved) {
      conv = true;
      V.lam_out = inside ? lamc : lam;
    } else {
      V.lam = V.best;
      last = true;
    }
  } else if (!inside) {
    // correction leaves the bracket: one last pass at the midpoint
    V.lam = 0.5 * (V.lo + V.hi);
    last = true;
    V.fallback = true;
  } else {
    V.lam = lamc;
  }
}

// compiler-only barrier: memory operations are not moved across it
__device__ __forceinline__ void ring_fence() { asm volatile("" ::: "memory"); }

// One step of the unified transform x' = x f / (b + x) - lam: role 0
// (stationary, top-down) b = D, f = LLD; role 1 (progressive, bottom-up)
// b = LLD, f = D.  Also sets w = LD / (b + x); quotients to about one ulp
// (reciprocal with one Newton step, then one Newton correction of the
// quotient).  The fast form divides the product x f, which overflows once a
// near-zero pivot has made x huge; the guarded form (`guard`, kMayGuard
// instantiations only) takes the ratio first, x (f / (b + x)), as the qds
// transforms do, replaces a pivot below pivmin by -pivmin, and gives f - lam
// where the ratio vanishes (b + x infinite).
template <bool kMayGuard>
__device__ __forceinline__ double xstep_bf(double b, double f, double LD, double x, double lam, double pivmin,
                                           bool guard, double& w) {
  double den = b + x;
  if (kMayGuard) den = (guard && fabs(den) < pivmin) ? -pivmin : den;
  const double rc = rcp_nr1(den);
  const double xf = x * f;
  const double q0 = xf * rc;
  const double q = fma(rc, fma(-den, q0, xf), q0);
  double xn = q - lam;
  if (kMayGuard) {
    const double t0 = f * rc;
    const double tc = fma(rc, fma(-den, t0, f), t0);
    // the quotient's correction is NaN where the ratio is infinite (a pivot
    // of -pivmin under a large f) and where b + x is infinite (rc is NaN):
    // the uncorrected ratio there, and a vanishing one for an infinite
    // b + x, so the transform goes on past a zero pivot
    const double t = (tc == tc) ? tc : (isinf(den) ? 0.0 : t0);
    // one rounding in every inlining context (no contraction left to the compiler)
    const double xs = (t == 0.0) ? f - lam : fma(x, t, -lam);
    xn = guard ? xs : xn;
  }
  const double w0 = LD * rc;
  w = fma(rc, fma(-den, w0, LD), w0);
  return xn;
}

// Derivative of the transform variable with respect to lam along the same
// step: d x' = (f b / (b + x)^2) d x - 1 = w^2 d x - 1 (f b = (L D)^2), from
// d x = -1 at the start.  Accumulated this way, -d s_r and -d p_r are the
// sums of the squared entries of the twisted solve's z (z_r = 1) above and
// below the twist, in Horner form, so ||z||^2 = -(d s_r + d p_r + 1) =
// -d gamma_r / d lam comes with the transforms and no solve is needed.
__device__ __forceinline__ double dstep(double w, double dx) { return fma(w * w, dx, -1.0); }

// LDS hand-off between the lanes of a workgroup of one wavefront: its LDS
// operations complete in order, so waiting for them and keeping the compiler
// from moving memory operations across is enough; unlike __syncthreads this
// does not wait for the wavefront's outstanding global stores
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited for
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// staged eigenvector entries: entry o of lane l at zt[o * kZtStride + l]; the
// stride keeps both the lane-wise writes and the segment-wise reads free of
// bank conflicts
constexpr int kZtStride = 68;

// the write-back address and entry mask of a lane's segment, parked in LDS
__device__ __forceinline__ void zp_lds_store(double** zp, uint32_t* zm, int lane, double* p, uint32_t m) {
  zp[lane] = p;
  zm[lane] = m;
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

constexpr int kSB = 64;           // representation rows per staged group
constexpr int kGS = kSB / kSeg;   // segments per staged group

// Segment iterations j = 0 .. J - 1 (J wave-uniform) for a wavefront whose
// lanes share one representation R of n rows.  Lanes of role q visit segment
// k0 + dir * j, with k0 and dir equal across the role.  The rows of kGS
// consecutive segments of each role are staged through LDS one group ahead
// (lanes 0-31 load the role-0 rows, lanes 32-63 the role-1 rows, 64 bytes per
// lane per group); kNck per-lane checkpoint values per segment, ck(k, which),
// are loaded one group ahead as well and parked in LDS.  fn(j, k, rows, c0,
// c1) runs per iteration, rows pointing at the LDS copy of segment k (row u:
// rows[4u .. 4u+3] = D, L, LD, LLD).  With kRoleOrder the copy is in the
// order of the lane's role instead: role-1 lanes see the segment's rows
// descending and each row as (LLD, L, LD, D), so that field 0 is b and field
// 3 is f of the unified step for either role.  lds: kStageLds doubles.  Rows
// outside [0, n) are clamped; every lane must call.
constexpr int kStageLds = 2 * 2 * kSB * 4 + 2 * kGS * 64;

template <int kNck, class Ck>
__device__ __forceinline__ void stage_load(const double* __restrict__ Rd, int n, int b, int li, int k0, int dir, int g,
                                           Ck& ck, double2& q0, double2& q1, double2& q2, double2& q3,
                                           double (&c0)[kGS], double (&c1)[kGS]) {
  const double2* s0 = reinterpret_cast<const double2*>(Rd + 4 * (int64_t)min(max(b + li, 0), n - 1));
  const double2* s1 = reinterpret_cast<const double2*>(Rd + 4 * (int64_t)min(max(b + li + 1, 0), n - 1));
  q0 = s0[0];
  q1 = s0[1];
  q2 = s1[0];
  q3 = s1[1];
#pragma unroll
  for (int m = 0; m < kGS; ++m) {
    const int k = k0 + dir * (g * kGS + m);
    if (kNck > 0) c0[m] = ck(k, 0);
    if (kNck > 1) c1[m] = ck(k, 1);
  }
}

__device__ __forceinline__ int stage_first_seg(int k0, int dir, int g) {
  return dir > 0 ? k0 + g * kGS : k0 - g * kGS - (kGS - 1);
}

template <int kNck, bool kRoleOrder, class Ck, class Fn>
__device__ inline void staged_segments(const Rep* __restrict__ R, int n, int J, int k0, int dir,
                                       double* __restrict__ lds, Ck&& ck, Fn&& fn) {
  const int lane = threadIdx.x & 63;
  const int role = lane & 1;
  const int lrole = lane >> 5;
  const int k0l = __shfl(k0, lrole, 64);  // lane 0 has role 0, lane 1 role 1
  const int dirl = __shfl(dir, lrole, 64);
  const int li = (lane & 31) * 2;
  J = __builtin_amdgcn_readfirstlane(J);
  const int ng = (J + kGS - 1) / kGS;
  const double* Rd = reinterpret_cast<const double*>(R);
  double* cks = lds + 2 * 2 * kSB * 4;  // [which][m][lane]
  // LDS positions of this lane's two rows (reversed inside the segment and
  // with D and LLD swapped for role-1 streams with kRoleOrder)
  const bool rev = kRoleOrder && lrole == 1;
  const int p0 = rev ? (li & ~(kSeg - 1)) + kSeg - 1 - (li & (kSeg - 1)) : li;
  const int p1 = rev ? p0 - 1 : li + 1;
  double2 q0, q1, q2, q3;
  double c0[kGS], c1[kGS];
#pragma unroll
  for (int m = 0; m < kGS; ++m) c0[m] = c1[m] = 0.0;
  stage_load<kNck>(Rd, n, stage_first_seg(k0l, dirl, 0) * kSeg, li, k0, dir, 0, ck, q0, q1, q2, q3, c0, c1);
  for (int g = 0; g < ng; ++g) {
    double* buf = lds + (g & 1) * (2 * kSB * 4);
    double2* d0 = reinterpret_cast<double2*>(buf + lrole * kSB * 4 + p0 * 4);
    double2* d1 = reinterpret_cast<double2*>(buf + lrole * kSB * 4 + p1 * 4);
    if (rev) {
      d0[0] = make_double2(q1.y, q0.y);
      d0[1] = make_double2(q1.x, q0.x);
      d1[0] = make_double2(q3.y, q2.y);
      d1[1] = make_double2(q3.x, q2.x);
    } else {
      d0[0] = q0;
      d0[1] = q1;
      d1[0] = q2;
      d1[1] = q3;
    }
#pragma unroll
    for (int m = 0; m < kGS; ++m) {
      if (kNck > 0) cks[m * 64 + lane] = c0[m];
      if (kNck > 1) cks[(kGS + m) * 64 + lane] = c1[m];
    }
    __syncthreads();
    if (g + 1 < ng)
      stage_load<kNck>(Rd, n, stage_first_seg(k0l, dirl, g + 1) * kSeg, li, k0, dir, g + 1, ck, q0, q1, q2, q3, c0,
                       c1);
    const int b = stage_first_seg(k0, dir, g) * kSeg;
    const double* mine = buf + role * kSB * 4;
#pragma unroll 1
    for (int m = 0; m < kGS; ++m) {
      const int j = g * kGS + m;
      if (j < J) {
        const int k = k0 + dir * j;
        const double v0 = (kNck > 0) ? cks[m * 64 + lane] : 0.0;
        const double v1 = (kNck > 1) ? cks[(kGS + m) * 64 + lane] : 0.0;
        fn(j, k, mine + (k * kSeg - b) * 4, v0, v1);
      }
    }
  }
}

// 1-2. the two transforms and the twist index in one pass.  First half: lane
//    2c runs the stationary transform over the segments above the middle one
//    (hs = nseg / 2 segments), lane 2c+1 the progressive transform over the
//    others.  Second half: each lane continues its transform into the other
//    half, segment by segment, and recomputes there the partner's variable
//    from the partner's checkpoints of the first half, so gamma_k = s_k + p_k
//    + lam is formed on the way; the smallest |gamma| wins, ties to the
//    smaller index.  Each lane carries the derivative of its own variable
//    along and stores checkpoints of both at every segment it passes (SC[k],
//    DS[k] = s, d s at row k kSeg; PC[k], DP[k] = p, d p there, k >= 1).
//    Returns the lane's last transform value (s_n or p_1) for the finiteness
//    test.
template <int kPairSlots, bool kMayGuard>
__device__ inline double transform_twist(bool go, int role, const Rep* __restrict__ R, int n, double pivmin,
                                         bool guard, double lam, double x0, double xlast, double* __restrict__ SC,
                                         double* __restrict__ PC, double* __restrict__ DS, double* __restrict__ DP,
                                         int c, double* __restrict__ lds, double& gmin_out, int& r_out) {
  const int nseg = (n + kSeg - 1) / kSeg;
  const int hs = nseg >> 1;
  const int cnt1 = role ? nseg - hs : hs;  // first-half segments of the lane
  double x = x0, dx = -1.0;
  // first half: the lane's own transform, rows in its role's order
  staged_segments<0, true>(
      R, n, nseg - hs, role ? nseg - 1 : 0, role ? -1 : 1, lds, [](int, int) { return 0.0; },
      [&](int j, int k, const double* rows, double, double) {
        const bool on = j < cnt1;
        if (go && on && !role) {
          SC[(int64_t)k * kPairSlots + c] = x;
          DS[(int64_t)k * kPairSlots + c] = dx;
        }
        if (__ballot(k == nseg - 1) == 0) {
#pragma unroll
          for (int u = 0; u < kSeg; ++u) {
            const double f = rows[4 * u + 3], LD = rows[4 * u + 2];
            double w;
            const double xn = xstep_bf<kMayGuard>(rows[4 * u], f, LD, x, lam, pivmin, guard, w);
            const double dxn = dstep(w, dx);
            x = on ? xn : x;
            dx = on ? dxn : dx;
          }
        } else {
          // the last segment: no step at row n-1 and beyond
#pragma unroll
          for (int u = 0; u < kSeg; ++u) {
            const int o = role ? kSeg - 1 - u : u;
            const double f = rows[4 * u + 3], LD = rows[4 * u + 2];
            double w;
            const double xn = xstep_bf<kMayGuard>(rows[4 * u], f, LD, x, lam, pivmin, guard, w);
            const double dxn = dstep(w, dx);
            const bool st = on && k * kSeg + o <= n - 2;
            x = st ? xn : x;
            dx = st ? dxn : dx;
          }
        }
        if (go && on && role && k >= 1) {
          PC[(int64_t)k * kPairSlots + c] = x;
          DP[(int64_t)k * kPairSlots + c] = dx;
        }
      });
  __syncthreads();  // first-half checkpoints complete and visible to the partner lane
  // second half: lane 2c over segments hs .. nseg-1 (ascending), lane 2c+1
  // over hs-1 .. 0 (descending); both walk a segment's rows upward for s and
  // downward for p
  const int cnt2 = role ? hs : nseg - hs;
  double gbest = INFINITY;
  int rbest = -1;
  staged_segments<1, false>(
      R, n, nseg - hs, role ? hs - 1 : hs, role ? -1 : 1, lds,
      [&](int k, int) {
        const int kk = min(max(role ? k : k + 1, 0), nseg - 1);
        return (role ? SC : PC)[(int64_t)kk * kPairSlots + c];
      },
      [&](int j, int k, const double* rows, double ck, double) {
        const bool on = j < cnt2;
        if (go && on && !role) {
          SC[(int64_t)k * kPairSlots + c] = x;
          DS[(int64_t)k * kPairSlots + c] = dx;
        }
        auto seg = [&](auto E) {
          constexpr bool kEdge = decltype(E)::value;
          // s_i at the rows of the segment: lane 2c continues its transform
          // (and its derivative), lane 2c+1 recomputes from the partner's
          // checkpoint
          double sv[kSeg];
          double xs = role ? ck : x, dxs = dx;
#pragma unroll
          for (int u = 0; u < kSeg; ++u) {
            sv[u] = xs;
            double w;
            const double LD = rows[4 * u + 2];
            const double xn = xstep_bf<kMayGuard>(rows[4 * u], rows[4 * u + 3], LD, xs, lam, pivmin, guard, w);
            const bool st = !kEdge || k * kSeg + u <= n - 2;
            xs = st ? xn : xs;
            if (!role) dxs = st ? dstep(w, dxs) : dxs;
          }
          // p_i downward from the first row of the next segment (or p_n): lane
          // 2c+1 continues its transform (and its derivative), lane 2c
          // recomputes from a checkpoint
          const int rs = min((k + 1) * kSeg, n - 1);
          double xp = role ? x : ((kEdge && rs == n - 1) ? xlast : ck);
          double dxp = dx;
          double gseg = INFINITY;
          int rseg = -1;
#pragma unroll
          for (int u = kSeg - 1; u >= 0; --u) {
            const int row = k * kSeg + u;
            double w;
            const double D = rows[4 * u];
            const double xpn =
                xstep_bf<kMayGuard>(rows[4 * u + 3], D, rows[4 * u + 2], xp, lam, pivmin, guard, w);
            const bool st = !kEdge || row < rs;
            xp = st ? xpn : xp;
            if (role) dxp = st ? dstep(w, dxp) : dxp;
            const double g = sv[u] + xp + lam;
            const bool take = (!kEdge || row <= rs) && isfinite(g) && fabs(g) <= fabs(gseg);
            gseg = take ? g : gseg;
            rseg = take ? row : rseg;
          }
          if (on) {
            // segments come in ascending order on lane 2c and descending on
            // lane 2c+1: ties go to the smaller index either way
            const bool better = role ? fabs(gseg) <= fabs(gbest) && rseg >= 0 : fabs(gseg) < fabs(gbest);
            if (better) {
              gbest = gseg;
              rbest = rseg;
            }
            x = role ? xp : xs;
            dx = role ? dxp : dxs;
          }
        };
        if (__ballot(k >= nseg - 1) != 0)
          seg(std::true_type{});
        else
          seg(std::false_type{});
        if (go && on && role && k >= 1) {
          PC[(int64_t)k * kPairSlots + c] = x;
          DP[(int64_t)k * kPairSlots + c] = dx;
        }
      });
  // the partner's candidate; lane 2c+1 searched the smaller indices
  const double go_g = __shfl_xor(gbest, 1, 64);
  const int go_r = __shfl_xor(rbest, 1, 64);
  const double gt = role ? gbest : go_g, gb = role ? go_g : gbest;  // gt: lane 2c+1 (rows below the middle)
  const int rt = role ? rbest : go_r, rb = role ? go_r : rbest;
  const bool take_b = (rb >= 0) && (rt < 0 || fabs(gb) < fabs(gt));
  double gmin = take_b ? gb : gt;
  int r = take_b ? rb : rt;
  if (r < 0) {
    r = 0;
    gmin = NAN;  // no finite gamma: marks the round for the solve
  }
  gmin_out = gmin;
  r_out = r;
  return x;
}

// d s_r (lane 2c: from the checkpoint of r's segment up to row r) and d p_r
// (lane 2c+1: from the checkpoint of the next segment, or p_n, down to row
// r), the same steps as the transforms, so the same bits; returns
// d s_r + d p_r for both lanes of the pair.
template <int kPairSlots, bool kMayGuard>
__device__ inline double twist_derivative(bool go, int role, const Rep* __restrict__ R, int n, double pivmin,
                                          bool guard, double lam, double xlast, int r,
                                          const double* __restrict__ SC, const double* __restrict__ PC,
                                          const double* __restrict__ DS, const double* __restrict__ DP, int c) {
  const int nseg = (n + kSeg - 1) / kSeg;
  const int kr = r / kSeg;
  double x = 0.0, dx = 0.0;
  int start;  // first row stepped: lane 2c upward from kr kSeg, lane 2c+1 downward from start
  if (!role) {
    start = kr * kSeg;
    x = go ? SC[(int64_t)kr * kPairSlots + c] : 0.0;
    dx = go ? DS[(int64_t)kr * kPairSlots + c] : 0.0;
  } else {
    const int ke = kr + 1;
    const bool at_end = ke >= nseg || ke * kSeg >= n - 1;
    start = at_end ? n - 1 : ke * kSeg;
    x = at_end ? xlast : (go ? PC[(int64_t)ke * kPairSlots + c] : 0.0);
    dx = at_end ? -1.0 : (go ? DP[(int64_t)ke * kPairSlots + c] : 0.0);
  }
#pragma unroll
  for (int t = 0; t < kSeg; ++t) {
    // lane 2c: step at row start + t while it is below r; lane 2c+1: step at
    // row start - 1 - t while it is at or above r
    const int row = role ? start - 1 - t : start + t;
    const bool st = go && (role ? row >= r : row < r);
    const Rep q = R[min(max(row, 0), n - 1)];
    double w;
    const double b = role ? q.LLD : q.D, f = role ? q.D : q.LLD;
    const double xn = xstep_bf<kMayGuard>(b, f, q.LD, x, lam, pivmin, guard, w);
    const double dxn = dstep(w, dx);
    x = st ? xn : x;
    dx = st ? dxn : dx;
  }
  const double o = __shfl_xor(dx, 1, 64);
  return role ? o + dx : dx + o;  // d s_r + d p_r
}

// 3. the solve outward from the twist r: lane 2c from row r-1 up to row 0,
//    lane 2c+1 from row r down to row n-1, segment by segment in one order per
//    role (role 0 from the highest segment any of its lanes needs, role 1 from
//    the lowest), each lane working from its own twist on.  A segment's
//    quotients are recomputed from its checkpoint, then z walks through it;
//    where a z is zero the row of L D L^T - lam I gives the next one from the
//    one before.  Accumulates ||z||^2 and the signed entry of largest
//    magnitude (ties: smaller row) of the lane's half; with kWrite, stores
//    z * scale into Zc (z_r by the caller): each lane parks the (up to) 8
//    entries of its segment in LDS (zt, with the address of the segment's
//    first entry in zaddr and a mask of the entries it owns in zm), and the
//    wavefront writes them back column segment by column segment, 8 lanes
//    per segment (64 contiguous bytes each, 8 segments per store).
template <int kPairSlots, bool kMayGuard, bool kWrite>
__device__ inline void solve_pass(bool go, int role, const Rep* __restrict__ R, int n, double pivmin, bool guard,
                                  double lam, double xlast, int r, const double* __restrict__ SC,
                                  const double* __restrict__ PC, int c, double* __restrict__ lds,
                                  double* __restrict__ Zc, double scale, double& nrm_out, double& zbest_out,
                                  double* __restrict__ zt = nullptr, double** __restrict__ zaddr = nullptr,
                                  uint32_t* __restrict__ zm = nullptr) {
  const int nseg = (n + kSeg - 1) / kSeg;
  const int klast = (n - 2) / kSeg;  // segment of row n-2
  const bool has = go && (role ? r <= n - 2 : r >= 1);
  const int kown = role ? r / kSeg : (r - 1) / kSeg;
  const int kT = wave_max((has && !role) ? kown : -1);
  const int kB = wave_min((has && role) ? kown : INT_MAX);
  const int JT = kT + 1;
  const int JB = (kB == INT_MAX) ? 0 : klast - kB + 1;
  const int J = max(JT, JB);
  double nrm = (go && role) ? 1.0 : 0.0;
  double zbest = (go && role) ? 1.0 : 0.0;
  double zc = 1.0, zp = 0.0;
  const int dir = role ? 1 : -1;
  staged_segments<1, true>(
      R, n, J, role ? (kB == INT_MAX ? 0 : kB) : max(kT, 0), dir, lds,
      [&](int k, int) {
        const int kk = min(max(role ? k + 1 : k, 0), nseg - 1);
        return (role ? PC : SC)[(int64_t)kk * kPairSlots + c];
      },
      [&](int, int k, const double* rows, double c0, double) {
        const bool seg_on = has && (role ? (k >= kown && k <= klast) : (k <= kown && k >= 0));
        const int rs = min((k + 1) * kSeg, n - 1);
        double x = (role && rs == n - 1) ? xlast : c0;
        double wb[kSeg];
        auto quotients = [&](auto E) {
          constexpr bool kEdge = decltype(E)::value;
#pragma unroll
          for (int u = 0; u < kSeg; ++u) {
            const int o = role ? kSeg - 1 - u : u;
            const int row = k * kSeg + o;
            const double f = rows[4 * u + 3], LD = rows[4 * u + 2];
            const double xn = xstep_bf<kMayGuard>(rows[4 * u], f, LD, x, lam, pivmin, guard, wb[u]);
            x = (!kEdge || (role ? row < rs : row <= n - 2)) ? xn : x;
          }
        };
        if (__ballot(k >= nseg - 1) != 0)
          quotients(std::true_type{});
        else
          quotients(std::false_type{});
        // rows in solve order: descending (role 0), ascending (role 1)
        double zv[kSeg];
        uint32_t msk = 0;
#pragma unroll
        for (int u = kSeg - 1; u >= 0; --u) {
          const int o = role ? kSeg - 1 - u : u;
          const int row = k * kSeg + o;
          const bool act = seg_on && (role ? (row >= r && row <= n - 2) : (row <= r - 1));
          const bool first = role ? (row == r) : (row == r - 1);
          double zn = -wb[u] * zc;
          const bool slow = act && !(zc != 0.0 || first);
          if (__ballot(slow) != 0) {
            if (slow) {
              if (zp != 0.0) {
                const double ldi = R[row].LD;
                const double ldn = R[row - dir].LD;
                zn = (ldi != 0.0) ? -div_nr(ldn, ldi) * zp : 0.0;
              } else {
                zn = 0.0;  // an underflowed tail stays zero
              }
            }
          }
          zn = isfinite(zn) ? zn : 0.0;
          zv[o] = zn * scale;
          if (act) {
            msk |= 1u << o;
            zp = zc;
            zc = zn;
            nrm += zn * zn;
            if (role ? fabs(zn) > fabs(zbest) : fabs(zn) >= fabs(zbest)) zbest = zn;
          }
        }
        if (kWrite) {
          // entry o of the lane's segment is row k kSeg + o (role 0) or
          // k kSeg + o + 1 (role 1) of its column
          const int lane = threadIdx.x & 63;
#pragma unroll
          for (int o = 0; o < kSeg; ++o) zt[o * kZtStride + lane] = zv[o];
          zp_lds_store(zaddr, zm, lane, Zc + k * kSeg + role, msk);
          wave_lds_sync();
#pragma unroll
          for (int i = 0; i < 64 / kSeg; ++i) {
            const int q = i * kSeg + (lane >> 3), u = lane & (kSeg - 1);
            if ((zm[q] >> u) & 1u) zaddr[q][u] = zt[u * kZtStride + q];
          }
          wave_lds_sync();
        }
      });
  nrm_out = nrm;
  zbest_out = zbest;
}

// Rayleigh-quotient iteration for the eigenvector of lane pair c (role 0 =
// top-down / upward lane, role 1 = bottom-up / downward lane) over
// checkpoints SC, PC, DS, DP ([segment][kPairSlots] each).  Every round is one
// pass of the transforms with the twist search; ||z||^2 comes from the
// derivative of gamma_r (a solve runs only where that is not finite).
// Returns the twist index of the last round, with its shift in lam_last and
// its guard flag in g_last.
template <int kPairSlots>
__device__ inline int pair_rqi(bool solve, int role, const Rep* __restrict__ R, int n, double pivmin,
                               double* __restrict__ SC, double* __restrict__ PC, double* __restrict__ DS,
                               double* __restrict__ DP, int c, double* __restrict__ lds, VecState& V,
                               double& lam_last, bool& g_last) {
  bool conv = !solve;
  bool last = false;
  bool sticky = false;  // the pair needed the guarded form in an earlier round
  int rout = 0;
  const double dn = R[n - 1].D;
  for (int it = 0; it <= kMaxRqi; ++it) {
    const bool go = solve && !conv;
    if (__ballot(go) == 0) break;
    const double lam = V.lam;
    const double xlast = dn - lam;  // p_n
    // 1-2. the two transforms, concurrently, with the twist search.  Without
    //    a zero or overflowing pivot (the usual case) the guard and the
    //    special-case rule are no-ops, so the first pass runs without them; a
    //    lane that ends with a non-finite value makes the wavefront repeat the
    //    pass with both, and the recomputations of this round follow the pass
    //    that was kept.  A pair that needed the guard once (a shift at an
    //    eigenvalue of a leading or trailing submatrix) keeps it: its later
    //    rounds start in the guarded form, in which the other pairs' steps
    //    are the fast ones.
    const double x0 = role ? xlast : -lam;
    bool any_guard = false, gl = false;  // the lane's kept pass is the guarded form
    double gmin;
    int r;
    {
      const bool gs = go && sticky;
      const bool pre = __ballot(gs) != 0;
      const double x =
          pre ? transform_twist<kPairSlots, true>(go, role, R, n, pivmin, gs, lam, x0, xlast, SC, PC, DS, DP, c, lds,
                                                  gmin, r)
              : transform_twist<kPairSlots, false>(go, role, R, n, pivmin, false, lam, x0, xlast, SC, PC, DS, DP, c,
                                                   lds, gmin, r);
      bool gn = go && !gs && !isfinite(x);
      // the pair's two lanes share the guard: the checkpoints of both are
      // recomputed; every lane reads its partner's flag (a cross-lane read
      // under the short circuit would run with the flagged lanes switched off)
      const bool gp = __shfl_xor(gn ? 1 : 0, 1, 64) != 0;
      gn = gn || gp;
      gl = gs || gn;
      any_guard = __ballot(gl) != 0;
      if (__ballot(gn) != 0) {
        __syncthreads();  // the first pass's checkpoints are read before they are rewritten
        transform_twist<kPairSlots, true>(go, role, R, n, pivmin, gl, lam, x0, xlast, SC, PC, DS, DP, c, lds, gmin,
                                          r);
      }
      sticky = sticky || gl;
    }
    __syncthreads();  // checkpoints complete and visible to the partner lane
    // 3. ||z||^2 = -(d s_r + d p_r + 1); a pair without a finite value solves
    const double dg = any_guard ? twist_derivative<kPairSlots, true>(go, role, R, n, pivmin, gl, lam, xlast, r, SC,
                                                                     PC, DS, DP, c)
                                : twist_derivative<kPairSlots, false>(go, role, R, n, pivmin, false, lam, xlast, r,
                                                                      SC, PC, DS, DP, c);
    double nrm = -(dg + 1.0);
    const bool need = go && !(nrm < INFINITY && gmin == gmin);
    gmin = (gmin == gmin) ? gmin : 0.0;
    if (__ballot(need) != 0) {
      double ns, zb;
      if (any_guard)
        solve_pass<kPairSlots, true, false>(need, role, R, n, pivmin, gl, lam, xlast, r, SC, PC, c, lds, nullptr,
                                            1.0, ns, zb);
      else
        solve_pass<kPairSlots, false, false>(need, role, R, n, pivmin, false, lam, xlast, r, SC, PC, c, lds,
                                             nullptr, 1.0, ns, zb);
      const double ns_o = __shfl_xor(ns, 1, 64);  // combine the halves
      ns += ns_o;
      nrm = need ? ns : nrm;
      __syncthreads();
    }
    if (go) {
      rout = r;
      lam_last = lam;
      g_last = gl;
      rqi_commit(V, conv, last, it, n, gmin, nrm, 1.0, lam);
    }
  }
  if (solve && !conv) V.lam_out = V.lam;
  return rout;
}

// One wavefront per chunk: up to kPairSlots consecutive singletons of one
// node (cstart[ci] is the chunk's first slot; rid: run of equal-node
// singletons per slot, -1 elsewhere), so every lane works on the same
// representation.  Checkpoints of chunk ci at scratch + ci * stride.
template <int kPairSlots, int kWavesPerSimd>
__global__ void __launch_bounds__(64, kWavesPerSimd) k_vectors(
    const Problem* __restrict__ P, const Block* __restrict__ B, const Node* __restrict__ N,
    const int64_t* __restrict__ cstart, int nchunks, int64_t ntot, const int32_t* __restrict__ rid,
    const int32_t* __restrict__ sblk, const int32_t* __restrict__ snode, const int64_t* __restrict__ scol,
    const double* __restrict__ lo_a, const double* __restrict__ hi_a, const double* __restrict__ sgap,
    const Rep* __restrict__ pool, const double* __restrict__ ds, double* __restrict__ scratch, int64_t stride,
    double* __restrict__ w_out, double* __restrict__ Z, Counters* __restrict__ C) {
  __shared__ double lds[kStageLds];
  __shared__ int64_t s_col[kPairSlots];
  __shared__ int64_t s_zoff[kPairSlots];
  __shared__ int s_n[kPairSlots];
  __shared__ int64_t s_lrow0[kPairSlots];
  __shared__ int64_t s_pn[kPairSlots];
  __shared__ double s_zt[kSeg * kZtStride];  // staged eigenvector entries of the write pass
  __shared__ double* s_zp[64];
  __shared__ uint32_t s_zm[64];
  const int lane = threadIdx.x;
  const int c = lane >> 1;
  const int role = lane & 1;
  const int ci = blockIdx.x;
  if (ci >= nchunks) return;
  const int64_t first = cstart[ci];
  const int64_t s = first + c;
  const bool lane_slot = c < kPairSlots;  // lanes beyond 2 * kPairSlots idle
  const int run = rid[first];
  const bool act = lane_slot && s < ntot && rid[s] == run;
  const int64_t ss = act ? s : first;  // idle lanes shadow the chunk's first slot
  const int64_t col = act ? scol[s] : -1;
  // one node per chunk: block, node and representation are the same in every lane
  const Block blk = B[sblk[first]];
  const Node nd = N[snode[first]];
  const int n = __builtin_amdgcn_readfirstlane(blk.n);
  double* SC = scratch + (int64_t)ci * stride;
  double* PC = SC + (int64_t)((n + kSeg - 1) / kSeg) * kPairSlots;
  double* DS = PC + (int64_t)((n + kSeg - 1) / kSeg) * kPairSlots;
  double* DP = DS + (int64_t)((n + kSeg - 1) / kSeg) * kPairSlots;
  const int cs = lane_slot ? c : 0;  // checkpoint column (idle lanes never store)
  VecState V;
  V.lo = lo_a[ss];
  V.hi = hi_a[ss];
  V.gap = sgap[ss];
  V.resid = INFINITY;
  V.stall = 0;
  V.lam = 0.5 * (V.lo + V.hi);
  V.best = V.lam;
  V.lam_out = V.lam;
  V.nrm = 1.0;
  V.zmaxv = 1.0;
  V.qsteps = 0;
  V.rq = 0;
  V.fallback = false;
  const bool solve = act && n > 1;
  double lam_last = V.lam;
  bool g_last = false;
  const Rep* R = pool + uniform_ll(nd.rep);
  const double pivmin = __longlong_as_double(uniform_ll(__double_as_longlong(blk.pivmin)));
  const int r = pair_rqi<kPairSlots>(solve, role, R, n, pivmin, SC, PC, DS, DP, cs, lds, V, lam_last, g_last);
  // the sign (largest entry positive) is known once the vector is written
  const double scale = solve ? 1.0 / sqrt(V.nrm) : 1.0;
  const Problem pr = P[blk.prob];
  // eigenvalue (once per pair)
  if (act && !role) {
    const double wv = (n == 1) ? ds[s] / pr.scale : (nd.acc + V.lam_out) / pr.scale;
    w_out[pr.off + col] = wv;
    s_col[c] = col;
    s_zoff[c] = pr.zoff + col * pr.ldz;
    s_n[c] = n;
    s_lrow0[c] = blk.lrow0;
    s_pn[c] = pr.n;
  } else if (!role && lane_slot) {
    s_col[c] = -1;
    s_n[c] = 0;
    s_pn[c] = 0;
  }
  __syncthreads();
  if (Z != nullptr) {
    // the last solve once more, z * scale straight into the lane's column
    double* Zc = Z + (act ? pr.zoff + col * pr.ldz + blk.lrow0 : 0);
    double nrm_d, zb_d;
    if (n > 1)
      solve_pass<kPairSlots, true, true>(solve, role, R, n, pivmin, g_last, lam_last, R[n - 1].D - lam_last, r, SC,
                                         PC, cs, lds, Zc, scale, nrm_d, zb_d, s_zt, s_zp, s_zm);
    if (act && role) Zc[solve ? r : 0] = scale;  // z_r = 1 (n = 1: the unit vector)
    if (n > 1) {
      // the signed entry of largest magnitude (ties: smaller row) decides the
      // sign; its twist row holds z_r = 1 > 0, so a flip is rare.  A pair
      // whose entry is negative negates its rows: lane 2c rows 0 .. r-1, lane
      // 2c+1 rows r .. n-1 (the values -(z s) equal z (-s) bit for bit).
      const double zb_o = __shfl_xor(zb_d, 1, 64);
      const double zt = role ? zb_o : zb_d, zb = role ? zb_d : zb_o;
      const double zmax = (fabs(zt) >= fabs(zb) && zt != 0.0) ? zt : zb;
      const bool flip = solve && zmax < 0.0;
      if (__ballot(flip) != 0) {
        const int a = role ? r : 0;
        const int len = flip ? (role ? n - r : r) : 0;
        const int T = wave_max(len);
        for (int t0 = 0; t0 < T; t0 += 8) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = (t0 + u < len) ? Zc[a + t0 + u] : 0.0;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (t0 + u < len) Zc[a + t0 + u] = -v[u];
        }
      }
    }
    // rows of the problem outside the block are exact zeros
    for (int cl = 0; cl < kPairSlots; ++cl) {
      if (s_col[cl] < 0) continue;
      const int64_t pn = s_pn[cl];
      const int64_t r0 = s_lrow0[cl];
      const int64_t r1 = r0 + s_n[cl];
      if (r0 == 0 && r1 == pn) continue;
      for (int64_t i = lane; i < pn; i += 64)
        if (i < r0 || i >= r1) Z[s_zoff[cl] + i] = 0.0;
    }
  }
  if (act && !role) {
    atomicAdd(&C->qds_steps, (unsigned long long)V.qsteps);
    atomicAdd(&C->vec_rows, (unsigned long long)(V.qsteps / 4));
    atomicAdd(&C->ckpt_vec_rows, (unsigned long long)(V.qsteps / 4));
    if (Z != nullptr) {
      atomicAdd(&C->z_entries, (unsigned long long)s_pn[c]);
      atomicAdd(&C->ckpt_z_entries, (unsigned long long)s_pn[c]);
    }
    atomicAdd(&C->rqi, (unsigned long long)V.rq);
    atomicAdd(&C->singletons, 1ull);
    if (V.fallback) atomicAdd(&C->fallbacks, 1ull);
  }
  {
    const int rqm = wave_max(V.rq);
    if (lane == 0) atomicAdd(&C->wave_solves, (unsigned long long)rqm);
  }
}

// ---- stored work vectors: the variant for small blocks and small nodes ----
// Work vectors per wavefront: S, P, W0 (L+, then z above the twist), W1 (U-,
// then z from the twist down), each [row][slots], written by the transforms
// and read back by the twist scan, the solve and the Z write.  For blocks
// whose work vectors stay in the caches this costs less than recomputing
// segments, and a wavefront may mix nodes (32 consecutive slots).

constexpr int kZRows = 32;      // rows per LDS transpose tile

__device__ __forceinline__ int clamp_row(int i, int n) { return min(max(i, 0), n - 1); }

// the three fields of a representation row the transforms use
struct Row3 {
  double D, LD, LLD;
};
__device__ __forceinline__ Row3 load_row3(const Rep* __restrict__ R, int i) {
  Row3 r;
  r.D = R[i].D;
  r.LD = R[i].LD;
  r.LLD = R[i].LLD;
  return r;
}

constexpr int kHB = 8;  // steps per half of a double buffer

// software pipeline over steps t = 0 .. T - 1 (T wave-uniform): the loads of
// one half of kHB steps are issued while the other half is consumed, so every
// value arrives kHB .. 2 kHB - 1 steps after its load was issued.  load(t)
// must be in bounds for any t >= 0; step(t, v) sees steps in order.
template <int kH = kHB, class Ld, class St>
__device__ __forceinline__ void pipelined(int T, Ld&& load, St&& step) {
  constexpr int kHB = kH;  // this pipeline's half depth
  using V = decltype(load(0));
  V a[kHB], b[kHB];
#pragma unroll
  for (int k = 0; k < kHB; ++k) a[k] = load(k);
  for (int t0 = 0; t0 < T; t0 += 2 * kHB) {
#pragma unroll
    for (int k = 0; k < kHB; ++k) b[k] = load(t0 + kHB + k);
    ring_fence();
#pragma unroll
    for (int k = 0; k < kHB; ++k) step(t0 + k, a[k]);
    ring_fence();
#pragma unroll
    for (int k = 0; k < kHB; ++k) a[k] = load(t0 + 2 * kHB + k);
    ring_fence();
#pragma unroll
    for (int k = 0; k < kHB; ++k) step(t0 + kHB + k, b[k]);
    ring_fence();
  }
}

struct Quad {
  double s, p, ds, dp;
};
struct Row2x {
  double x, b, LD;
};

// The quotient of the step at one row, as the transform step computes it
// (same operations, so the same bits): w = LD / (b + x), the pivot replaced
// by -pivmin below pivmin in the guarded form.
__device__ __forceinline__ double step_w(double b, double x, double LD, double pivmin, bool guard) {
  double den = b + x;
  den = (guard && fabs(den) < pivmin) ? -pivmin : den;
  const double rc = rcp_nr1(den);
  const double w0 = LD * rc;
  return fma(rc, fma(-den, w0, LD), w0);
}

// Solve outward from the twist r of every lane with `on_lane`: z_i = -L+_i
// z_{i+1} upward (lane 2c), z_{i+1} = -U-_i z_i downward (lane 2c+1), the
// quotients recomputed from the stored s (top) or p (bottom) and the
// representation row; where a z is zero the row of L D L^T - lam I gives the
// next one from the one before.  z goes to the lane's work vector Wr (rows
// < r in W0, rows >= r in W1, z_r = 1); returns ||z||^2 and the signed entry
// of largest magnitude (ties: smaller row) over both halves.  Rows are
// visited in a wave-uniform order per role (top lanes from the largest twist
// index of the wave down, bottom lanes from the smallest up), each lane
// active on its own side of its twist, so every access is one coalesced row
// of the work vector.
template <int kPairSlots>
__device__ inline void solve_stored(bool on_lane, int role, const Rep* __restrict__ R, int n, double pivmin,
                                    bool guard, int r, const double* __restrict__ S, const double* __restrict__ P,
                                    double* __restrict__ Wr, int c, double& nrm_out, double& zbest_out) {
  double nrm = 0.0, zbest = 0.0;
  if (on_lane && role) {
    nrm = 1.0;
    zbest = 1.0;
  }
  int rmax = (on_lane && !role) ? r : 0;        // top lanes: rows rmax-1 .. 0
  int rmin = (on_lane && role) ? r : INT_MAX;   // bottom lanes: rows rmin .. n-2
  for (int o = 32; o > 0; o >>= 1) {
    rmax = max(rmax, __shfl_xor(rmax, o, 64));
    rmin = min(rmin, __shfl_xor(rmin, o, 64));
  }
  if (rmin == INT_MAX) rmin = 0;  // no lane iterating: nothing to visit
  int nb = (on_lane && role) ? n - 1 - rmin : 0;
  for (int o = 32; o > 0; o >>= 1) nb = max(nb, __shfl_xor(nb, o, 64));
  const int T3 = max(rmax, nb);
  const int base = role ? rmin : rmax - 1;
  const int dir = role ? 1 : -1;
  double zc = 1.0, zp = 0.0;
  pipelined<4>(
      T3,
      [&](int t) {
        // top: s_i with D_i; bottom: p_{i+1} with LLD_i
        const int row = clamp_row(base + dir * t, n);
        const int xr = role ? min(row + 1, n - 1) : row;
        Row2x v;
        v.x = (role ? P : S)[(int64_t)xr * kPairSlots + c];
        v.b = role ? R[row].LLD : R[row].D;
        v.LD = R[row].LD;
        return v;
      },
      [&](int t, const Row2x& v) {
        const int row = base + dir * t;
        const bool on = role ? (row >= r && row < n - 1) : (row < r && row >= 0);
        if (t < T3 && on_lane && on) {
          const bool first = role ? (row == r) : (row == r - 1);
          double zn;
          if (zc != 0.0 || first) {
            zn = -step_w(v.b, v.x, v.LD, pivmin, guard) * zc;
          } else if (zp != 0.0) {
            const double ldi = R[row].LD;
            const double ldn = R[row - dir].LD;
            zn = (ldi != 0.0) ? -div_nr(ldn, ldi) * zp : 0.0;
          } else {
            zn = 0.0;  // an underflowed tail stays zero
          }
          zn = isfinite(zn) ? zn : 0.0;
          const int zrow = role ? row + 1 : row;
          Wr[(int64_t)zrow * kPairSlots + c] = zn;
          zp = zc;
          zc = zn;
          nrm += zn * zn;
          // largest magnitude, ties to the smaller row
          if (role ? fabs(zn) > fabs(zbest) : fabs(zn) >= fabs(zbest)) zbest = zn;
        }
      });
  if (on_lane && role) Wr[(int64_t)r * kPairSlots + c] = 1.0;
  // combine the halves: rows < r (lane 2c) and rows >= r (lane 2c+1)
  const double nrm_o = __shfl_xor(nrm, 1, 64);
  const double zb_o = __shfl_xor(zbest, 1, 64);
  nrm += nrm_o;
  const double zt = role ? zb_o : zbest, zb = role ? zbest : zb_o;
  nrm_out = nrm;
  zbest_out = (fabs(zt) >= fabs(zb) && zt != 0.0) ? zt : zb;
}

// one Rayleigh-quotient iteration sequence for the eigenvector of lane pair c;
// role 0 = top-down / upward lane, role 1 = bottom-up / downward lane.  Work
// vectors, each [row][kPairSlots]: S = s_i, P = p_i, W0 = d s_i / d lam (then
// z above the twist), W1 = d p_i / d lam (then z from the twist down).  Every
// round is the two transforms and the twist scan; ||z||^2 comes from the
// derivatives at the twist (a solve runs only where that is not finite).
// Returns the twist index of the last round, with its shift in lam_last and
// its guard flag in g_last.
template <int kPairSlots>
__device__ inline int pair_rqi_stored(bool solve, int role, const Rep* __restrict__ R, int n, int nmax, double pivmin,
                                      double* __restrict__ S, double* __restrict__ P, double* __restrict__ W0,
                                      double* __restrict__ W1, int c, VecState& V, double& lam_last, bool& g_last) {
  bool conv = !solve;
  bool last = false;
  bool sticky = false;  // the pair needed the guarded form in an earlier round
  int rout = 0;
  // wave-uniform trip counts
  int T = n - 1;
  for (int o = 32; o > 0; o >>= 1) T = max(T, __shfl_xor(T, o, 64));
  double* const X = role ? P : S;    // this lane's transform variable
  double* const Wr = role ? W1 : W0;  // this lane's derivatives, then z
  for (int it = 0; it <= kMaxRqi; ++it) {
    const bool go = solve && !conv;
    if (__ballot(go) == 0) break;
    const double lam = V.lam;
    // 1. the two transforms, concurrently, each with its derivative
    double x, dx = -1.0;
    if (role) {
      x = R[n - 1].D - lam;
      if (go) {
        P[(int64_t)(n - 1) * kPairSlots + c] = x;
        W1[(int64_t)(n - 1) * kPairSlots + c] = dx;
      }
    } else {
      x = -lam;
    }
    bool gl;
    {
      // rows in two buffers of kHB: one is consumed while the other's loads
      // are in flight (prefetch distance kHB .. 2 kHB - 1 steps)
      // The first pass runs the fast form of the step; a lane that ends
      // with a non-finite value (a zero or overflowing pivot) repeats its
      // transform in the guarded form, the other lanes repeat theirs
      // unchanged, so each eigenvector's values do not depend on its
      // wavefront.  A pair that needed the guard once starts its later
      // rounds in the guarded form.
      auto rowof = [&](int t) { return clamp_row(role ? n - 2 - t : t, n); };
      const double x0 = x;
      auto pass = [&](auto G, bool glp) {
        constexpr bool kG = decltype(G)::value;
        x = x0;
        dx = -1.0;
        auto step = [&](int t, const Row3& rr) {
          if (t < T && go && t < n - 1) {
            const int row = role ? n - 2 - t : t;
            const double b = role ? rr.LLD : rr.D;
            const double f = role ? rr.D : rr.LLD;
            double w;
            const double xn = xstep_bf<kG>(b, f, rr.LD, x, lam, pivmin, glp, w);
            const double dxn = dstep(w, dx);
            const int64_t o = (int64_t)row * kPairSlots + c;
            X[o] = role ? xn : x;
            Wr[o] = role ? dxn : dx;
            x = xn;
            dx = dxn;
          }
        };
        pipelined(T, [&](int t) { return load_row3(R, rowof(t)); }, step);
      };
      const bool gs = go && sticky;
      if (__ballot(gs) != 0)
        pass(std::true_type{}, gs);
      else
        pass(std::false_type{}, false);
      bool gn = go && !gs && !isfinite(x);
      // both transforms of a pair in one form; every lane reads its partner's
      // flag (a cross-lane read under the short circuit would run with the
      // flagged lanes switched off)
      const bool gp = __shfl_xor(gn ? 1 : 0, 1, 64) != 0;
      gn = gn || gp;
      gl = gs || gn;
      if (__ballot(gn) != 0) pass(std::true_type{}, gl);
      sticky = sticky || gl;
    }
    if (go && !role) {
      S[(int64_t)(n - 1) * kPairSlots + c] = x;
      W0[(int64_t)(n - 1) * kPairSlots + c] = dx;
    }
    __syncthreads();  // S, P and the derivatives complete and visible to the partner lane
    // 2. twist index: lane 2c scans k < h, lane 2c+1 scans k >= h
    const int h = n >> 1;
    double gmin = INFINITY, dg = 0.0;
    int r = -1;
    {
      const int kb = role ? h : 0;
      const int kc = role ? n - h : h;
      int T2 = kc;
      for (int o = 32; o > 0; o >>= 1) T2 = max(T2, __shfl_xor(T2, o, 64));
      pipelined<4>(
          T2,
          [&](int t) {
            const int64_t o = (int64_t)clamp_row(kb + t, n) * kPairSlots + c;
            Quad v;
            v.s = S[o];
            v.p = P[o];
            v.ds = W0[o];
            v.dp = W1[o];
            return v;
          },
          [&](int t, const Quad& v) {
            if (t < T2 && go && t < kc) {
              const double g = v.s + v.p + lam;
              if (isfinite(g) && fabs(g) < fabs(gmin)) {
                gmin = g;
                dg = v.ds + v.dp;
                r = kb + t;
              }
            }
          });
      // the partner's candidate; ties go to the smaller index (the upper half)
      const double go_g = __shfl_xor(gmin, 1, 64);
      const double go_d = __shfl_xor(dg, 1, 64);
      const int go_r = __shfl_xor(r, 1, 64);
      const double gt = role ? go_g : gmin, gb = role ? gmin : go_g;
      const double dt = role ? go_d : dg, db = role ? dg : go_d;
      const int rt = role ? go_r : r, rb = role ? r : go_r;
      const bool take_b = (rb >= 0) && (rt < 0 || fabs(gb) < fabs(gt));
      gmin = take_b ? gb : gt;
      dg = take_b ? db : dt;
      r = take_b ? rb : rt;
      if (r < 0) {
        // no finite gamma: no norm either (the solve supplies it)
        r = 0;
        gmin = 0.0;
        dg = NAN;
      }
    }
    // 3. ||z||^2 = -(d s_r + d p_r + 1); a pair without a finite value solves
    double nrm = -(dg + 1.0);
    const bool need = go && !(nrm < INFINITY);
    if (__ballot(need) != 0) {
      __syncthreads();  // the derivatives are read before z overwrites them
      double ns, zb;
      solve_stored<kPairSlots>(need, role, R, n, pivmin, gl, r, S, P, Wr, c, ns, zb);
      nrm = need ? ns : nrm;
    }
    __syncthreads();  // the work vectors are read before the next transform overwrites them
    if (go) {
      rout = r;
      lam_last = lam;
      g_last = gl;
      rqi_commit(V, conv, last, it, n, gmin, nrm, 1.0, lam);
    }
  }
  if (solve && !conv) V.lam_out = V.lam;
  return rout;
}

template <int kPairSlots>
__global__ void __launch_bounds__(64, 2) k_vectors_stored(
    const Problem* __restrict__ P, const Block* __restrict__ B, const Node* __restrict__ N,
    const int32_t* __restrict__ chunks, const int64_t* __restrict__ chunk_off, int nchunks, int64_t ntot,
    const int32_t* __restrict__ sblk, const int32_t* __restrict__ snode, const uint32_t* __restrict__ sflag,
    const int64_t* __restrict__ scol, const double* __restrict__ lo_a, const double* __restrict__ hi_a,
    const double* __restrict__ sgap, const Rep* __restrict__ pool, const double* __restrict__ ds,
    double* __restrict__ scratch, double* __restrict__ w_out, double* __restrict__ Z, Counters* __restrict__ C) {
  __shared__ double tile[kPairSlots][kZRows + 1];
  __shared__ int64_t s_col[kPairSlots];
  __shared__ int64_t s_zoff[kPairSlots];
  __shared__ int s_n[kPairSlots];
  __shared__ int64_t s_lrow0[kPairSlots];
  __shared__ int64_t s_pn[kPairSlots];
  const int lane = threadIdx.x;
  const int c = lane >> 1;
  const int role = lane & 1;
  const int ci = blockIdx.x;
  if (ci >= nchunks) return;
  const int64_t chunk = chunks[ci];
  const int64_t s = chunk * kPairSlots + c;
  double* S = scratch + chunk_off[ci];
  const bool lane_slot = c < kPairSlots;  // lanes beyond 2 * kPairSlots idle
  bool act = false;
  if (lane_slot && s < ntot) act = (sflag[s] & (F_SINGLETON | F_CKPT)) == F_SINGLETON && scol[s] >= 0;
  const uint64_t am = __ballot(act);
  if (am == 0) return;
  const int64_t sf = __shfl(s, first_lane(am), 64);
  const int64_t ss = act ? s : sf;  // idle lanes shadow a valid slot
  const int64_t col = act ? scol[s] : -1;
  const Block blk = B[sblk[ss]];
  const Node nd = N[snode[ss]];
  const int n = blk.n;
  int nmax = act ? n : 0;
  for (int o = 32; o > 0; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, 64));
  double* Pv = S + (int64_t)nmax * kPairSlots;
  double* W0 = Pv + (int64_t)nmax * kPairSlots;
  double* W1 = W0 + (int64_t)nmax * kPairSlots;
  const int cs = lane_slot ? c : 0;  // scratch column (idle lanes never store)
  VecState V;
  V.lo = lo_a[ss];
  V.hi = hi_a[ss];
  V.gap = sgap[ss];
  V.resid = INFINITY;
  V.stall = 0;
  V.lam = 0.5 * (V.lo + V.hi);
  V.best = V.lam;
  V.lam_out = V.lam;
  V.nrm = 1.0;
  V.zmaxv = 1.0;
  V.qsteps = 0;
  V.rq = 0;
  V.fallback = false;
  const bool solve = act && n > 1;
  int r = 0;
  if (act && n == 1 && role) W1[c] = 1.0;
  double lam_last = V.lam;
  bool g_last = false;
  r = pair_rqi_stored<kPairSlots>(solve, role, pool + nd.rep, n, nmax, blk.pivmin, S, Pv, W0, W1, cs, V, lam_last,
                                  g_last);
  // the vector of the last round: z into W0 / W1, its largest entry for the sign
  {
    double nz, zb;
    solve_stored<kPairSlots>(solve, role, pool + nd.rep, n, blk.pivmin, g_last, r, S, Pv, role ? W1 : W0, cs, nz,
                             zb);
    if (solve) V.zmaxv = zb;
  }
  __syncthreads();  // z complete before the transposed write reads it
  double scale = 1.0;
  if (solve) {
    scale = 1.0 / sqrt(V.nrm);
    if (V.zmaxv < 0.0) scale = -scale;
  }
  // eigenvalue (once per pair)
  if (act && !role) {
    const Problem pr = P[blk.prob];
    const double wv = (n == 1) ? ds[s] / pr.scale : (nd.acc + V.lam_out) / pr.scale;
    w_out[pr.off + col] = wv;
    s_col[c] = col;
    s_zoff[c] = pr.zoff + col * pr.ldz;
    s_n[c] = n;
    s_lrow0[c] = blk.lrow0;
    s_pn[c] = pr.n;
  } else if (!role && lane_slot) {
    s_col[c] = -1;
    s_n[c] = 0;
    s_pn[c] = 0;
  }
  __syncthreads();
  if (Z != nullptr) {
    // z * scale into column-major Z through an LDS transpose: each pass stages
    // 32 rows x 32 columns (lane 2c rows 0-15 of column c, lane 2c+1 rows
    // 16-31), then every column gets one contiguous 256-byte segment
    for (int r0 = 0; r0 < nmax; r0 += kZRows) {
      double v[kZRows / 2];
#pragma unroll
      for (int k = 0; k < kZRows / 2; ++k) {
        const int row = r0 + role * (kZRows / 2) + k;
        const double* src = (row < r) ? W0 : W1;
        v[k] = (row < nmax) ? src[(int64_t)row * kPairSlots + cs] : 0.0;
      }
      if (lane_slot) {
#pragma unroll
        for (int k = 0; k < kZRows / 2; ++k) {
          const int row = r0 + role * (kZRows / 2) + k;
          tile[c][role * (kZRows / 2) + k] = (act && row < n) ? v[k] * scale : 0.0;
        }
      }
      __syncthreads();
      const int rr = lane & (kZRows - 1);
      for (int cg = 0; cg < kPairSlots; cg += 2) {
        const int cl = cg + (lane >> 5);
        const int i = r0 + rr;
        if (s_col[cl] >= 0 && i < s_n[cl]) Z[s_zoff[cl] + s_lrow0[cl] + i] = tile[cl][rr];
      }
      __syncthreads();
    }
    // rows of the problem outside the block are exact zeros
    for (int cl = 0; cl < kPairSlots; ++cl) {
      if (s_col[cl] < 0) continue;
      const int64_t pn = s_pn[cl];
      const int64_t r0 = s_lrow0[cl];
      const int64_t r1 = r0 + s_n[cl];
      if (r0 == 0 && r1 == pn) continue;
      for (int64_t i = lane; i < pn; i += 64)
        if (i < r0 || i >= r1) Z[s_zoff[cl] + i] = 0.0;
    }
  }
  if (act && !role) {
    atomicAdd(&C->qds_steps, (unsigned long long)V.qsteps);
    atomicAdd(&C->vec_rows, (unsigned long long)(V.qsteps / 4));
    if (Z != nullptr) atomicAdd(&C->z_entries, (unsigned long long)s_pn[c]);
    atomicAdd(&C->rqi, (unsigned long long)V.rq);
    atomicAdd(&C->singletons, 1ull);
    if (V.fallback) atomicAdd(&C->fallbacks, 1ull);
  }
  {
    int rqm = V.rq;
    for (int o = 32; o > 0; o >>= 1) rqm = max(rqm, __shfl_xor(rqm, o, 64));
    if (lane == 0) atomicAdd(&C->wave_solves, (unsigned long long)rqm);
  }
}

// scratch rows each chunk of `slots` consecutive slots needs for the stored
// variant (0: no singleton of that variant to compute)
__global__ void k_chunk_rows(const Block* __restrict__ B, int64_t ntot, const int32_t* __restrict__ sblk,
                             const uint32_t* __restrict__ sflag, const int64_t* __restrict__ scol, int slots,
                             int32_t* __restrict__ rows) {
  const int64_t s = (int64_t)blockIdx.x * slots + (threadIdx.x & (slots - 1));
  int v = 0;
  if ((int)threadIdx.x < slots && s < ntot && (sflag[s] & (F_SINGLETON | F_CKPT)) == F_SINGLETON && scol[s] >= 0)
    v = B[sblk[s]].n;
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  if (threadIdx.x == 0) rows[blockIdx.x] = v;
}

// singletons in runs of at least min_run equal-node slots of blocks of order
// min_n or more go to the checkpointing kernel (rid, rstart: equal-node runs)
__global__ void k_mark_ckpt(int64_t ntot, const Block* __restrict__ B, const int32_t* __restrict__ sblk,
                            const int32_t* __restrict__ rid, const int64_t* __restrict__ rstart, int min_run,
                            int min_n, uint32_t* __restrict__ sflag) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int q = rid[s];
  if (q < 0) return;
  const int64_t t = rstart[q] + min_run - 1;
  if (t < ntot && rid[t] == q && B[sblk[s]].n >= min_n) sflag[s] |= F_CKPT;
}

// chunks of slots of one node: runs of consecutive slots that have every
// flag of `need` (and, with need_col, an output column) and the same node,
// cut into pieces of at most `slots`
__device__ __forceinline__ bool chunk_slot(const uint32_t* __restrict__ sflag, const int64_t* __restrict__ scol,
                                          uint32_t need, bool need_col, int64_t s) {
  return (sflag[s] & need) == need && (!need_col || scol[s] >= 0);
}

__global__ void k_vec_runs(int64_t ntot, const uint32_t* __restrict__ sflag, const int64_t* __restrict__ scol,
                           uint32_t need, int need_col, const int32_t* __restrict__ snode,
                           int32_t* __restrict__ runflag) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  int f = 0;
  if (chunk_slot(sflag, scol, need, need_col, s))
    f = (s == 0 || !chunk_slot(sflag, scol, need, need_col, s - 1) || snode[s - 1] != snode[s]) ? 1 : 0;
  runflag[s] = f;
}

__global__ void k_vec_rid(int64_t ntot, const uint32_t* __restrict__ sflag, const int64_t* __restrict__ scol,
                          uint32_t need, int need_col, const int32_t* __restrict__ runflag,
                          const int32_t* __restrict__ runid, int32_t* __restrict__ rid, int64_t* __restrict__ rstart) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const bool v = chunk_slot(sflag, scol, need, need_col, s);
  rid[s] = v ? runid[s] + runflag[s] - 1 : -1;
  if (runflag[s]) rstart[runid[s]] = s;
}

__global__ void k_vec_cflags(int64_t ntot, const int32_t* __restrict__ rid, const int64_t* __restrict__ rstart,
                             int slots, int32_t* __restrict__ cflag) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int q = rid[s];
  cflag[s] = (q >= 0 && (s - rstart[q]) % slots == 0) ? 1 : 0;
}

__global__ void k_vec_cstart(int64_t ntot, const int32_t* __restrict__ cflag, const int32_t* __restrict__ cid,
                             int64_t* __restrict__ cstart) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  if (cflag[s]) cstart[cid[s]] = s;
}


// ---------------------------------------------------------------------------
// 9. output order: eigenvalues ascending within each problem (swaps are only
//    ever needed between near-equal values from different leaves or blocks)

__global__ void k_check_sorted(const Problem* __restrict__ P, int nprob, const double* __restrict__ w,
                               int32_t* __restrict__ bad, Counters* __restrict__ C) {
  const int p = blockIdx.x;
  if (p >= nprob) return;
  const Problem pr = P[p];
  int flag = 0;
  for (int64_t c = threadIdx.x; c + 1 < pr.m; c += blockDim.x)
    if (w[pr.off + c] > w[pr.off + c + 1]) flag = 1;
  if (flag) {
    bad[p] = 1;
    atomicExch(&C->unsorted, 1);
  }
}

// insertion sort of one problem's w with the matching column permutation; the
// columns are then moved through a scratch copy
__global__ void k_sort_problem(const Problem* __restrict__ P, const int32_t* __restrict__ bad, double* __restrict__ w,
                               int64_t* __restrict__ perm) {
  const int p = blockIdx.x;
  if (!bad[p] || threadIdx.x != 0) return;
  const Problem pr = P[p];
  double* wv = w + pr.off;
  int64_t* pm = perm + pr.off;
  for (int64_t c = 0; c < pr.m; ++c) pm[c] = c;
  for (int64_t c = 1; c < pr.m; ++c) {
    const double x = wv[c];
    const int64_t px = pm[c];
    int64_t k = c - 1;
    while (k >= 0 && wv[k] > x) {
      wv[k + 1] = wv[k];
      pm[k + 1] = pm[k];
      --k;
    }
    wv[k + 1] = x;
    pm[k + 1] = px;
  }
}

// Z_new[:, c] = Z_old[:, perm[c]], following the permutation's cycles with one
// temporary column (tmp, n doubles at the problem's slot offset)
__global__ void k_permute_cols(const Problem* __restrict__ P, const int32_t* __restrict__ bad,
                               int64_t* __restrict__ perm, double* __restrict__ tmp, double* __restrict__ Z) {
  const int p = blockIdx.x;
  if (!bad[p]) return;
  const Problem pr = P[p];
  int64_t* pm = perm + pr.off;
  double* t = tmp + pr.off;
  __shared__ int64_t s_next;
  for (int64_t c0 = 0; c0 < pr.m; ++c0) {
    if (pm[c0] < 0 || pm[c0] == c0) continue;  // uniform: every thread reads the same value
    for (int64_t i = threadIdx.x; i < pr.n; i += blockDim.x) t[i] = Z[pr.zoff + c0 * pr.ldz + i];
    int64_t c = c0;
    for (int64_t guard = 0; guard <= pr.m; ++guard) {
      __syncthreads();
      if (threadIdx.x == 0) s_next = pm[c];
      __syncthreads();
      const int64_t src = s_next;
      if (threadIdx.x == 0) pm[c] = -1 - pm[c];
      if (src == c0) {
        for (int64_t i = threadIdx.x; i < pr.n; i += blockDim.x) Z[pr.zoff + c * pr.ldz + i] = t[i];
        break;
      }
      for (int64_t i = threadIdx.x; i < pr.n; i += blockDim.x)
        Z[pr.zoff + c * pr.ldz + i] = Z[pr.zoff + src * pr.ldz + i];
      c = src;
    }
    __syncthreads();
  }
}

// eigenvalues only: the root-level values
__global__ void k_values_only(const Problem* __restrict__ P, const Block* __restrict__ B, const Node* __restrict__ N,
                              int64_t ntot, const int32_t* __restrict__ sblk, const int32_t* __restrict__ snode,
                              const int64_t* __restrict__ scol, const double* __restrict__ lo,
                              const double* __restrict__ hi, const double* __restrict__ ds, double* __restrict__ w) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntot) return;
  const int64_t col = scol[s];
  if (col < 0) return;
  const Block blk = B[sblk[s]];
  const Problem pr = P[blk.prob];
  const double v = (blk.n == 1) ? ds[s] : N[snode[s]].acc + 0.5 * (lo[s] + hi[s]);
  w[pr.off + col] = v / pr.scale;
}

// ---------------------------------------------------------------------------
// launch wrappers

#define GRID1(n, t) dim3((unsigned)(((n) + (t)-1) / (t))), dim3(t)

// SIMDs of the current device (four per compute unit on CDNA), cached per device
static int simd_count() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
  cache[dev] = 4 * cu;
  return 4 * cu;
}


void launch_prep(hipStream_t st, Problem* P, int nprob, const int64_t* poff, int64_t ntot, const double* d,
                 const double* e, int32_t* sprob, double* ds, double* es, int32_t* flag) {
  if (ntot == 0) return;
  hipLaunchKernelGGL(k_prep_max, GRID1(ntot, 256), 0, st, P, nprob, poff, ntot, d, e, sprob);
  hipLaunchKernelGGL(k_prep_scale, GRID1(ntot, 256), 0, st, P, poff, ntot, d, e, sprob, ds, es);
  hipLaunchKernelGGL(k_split_flags, GRID1(ntot, 256), 0, st, P, poff, ntot, sprob, es, flag);
}

void launch_scan(hipStream_t st, const int32_t* in, int32_t* out, int32_t* tile_sum, int64_t n, int32_t* total) {
  if (n == 0) {
    (void)hipMemsetAsync(total, 0, sizeof(int32_t), st);
    return;
  }
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, in, out, tile_sum, n);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, tile_sum, ntiles, total);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, out, tile_sum, n);
}

void launch_blocks(hipStream_t st, Problem* P, const int64_t* poff, const int32_t* flag, const int32_t* excl,
                   int64_t ntot, int nblk, const int32_t* sprob, int64_t* bstart, int32_t* sblk, Block* B) {
  hipLaunchKernelGGL(k_blocks, GRID1(ntot, 256), 0, st, flag, excl, ntot, bstart, sblk);
  hipLaunchKernelGGL(k_blocks2, GRID1(nblk, 64), 0, st, P, poff, bstart, nblk, ntot, sprob, B);
}

void launch_root(hipStream_t st, Problem* P, Block* B, Node* N, int nblk, const double* ds, const double* es,
                 Rep* pool, Counters* C, int grid_density) {
  hipLaunchKernelGGL(k_root, dim3(nblk), dim3(256), 0, st, P, B, N, ds, es, pool, C, grid_density);
}

void launch_grid(hipStream_t st, const Block* B, int nblk, const int64_t* goff, int64_t gtot, const Rep* pool,
                 int32_t* gcnt) {
  hipLaunchKernelGGL(k_grid, GRID1(gtot, 64), 0, st, B, nblk, goff, gtot, pool, gcnt);
}

void launch_assign(hipStream_t st, const Block* B, const int64_t* goff, int64_t ntot, const int32_t* sblk,
                   const int32_t* gcnt, double* lo, double* hi, int32_t* clo, int32_t* chi, int32_t* snode,
                   uint32_t* sflag, Counters* C) {
  hipLaunchKernelGGL(k_assign, GRID1(ntot, 256), 0, st, B, goff, ntot, sblk, gcnt, lo, hi, clo, chi, snode, sflag,
                     C);
}

void launch_refine(hipStream_t st, const Block* B, const Node* N, int64_t ntot, const int32_t* sblk,
                   const int32_t* snode, const Rep* pool, double* lo, double* hi, int32_t* clo, int32_t* chi,
                   uint32_t* sflag, Counters* C, int lanes, bool validate_only, const int64_t* cstart,
                   const int32_t* rid, int nchunks, bool share) {
  // `lanes` lanes per eigenvalue: 64 / lanes eigenvalues per wavefront
  const unsigned g4 = (unsigned)((ntot + 15) / 16), g2 = (unsigned)((ntot + 31) / 32),
                 g1 = (unsigned)((ntot + 63) / 64);
  const int v = validate_only ? 1 : 0;
  const bool ch = cstart != nullptr;
  if (ch && nchunks == 0) return;
  if (lanes >= 4)
    hipLaunchKernelGGL(k_refine<4>, dim3(ch ? (unsigned)nchunks : g4), dim3(64), 0, st, B, N, ntot, sblk, snode, pool,
                       lo, hi, clo, chi, sflag, C, v, cstart, rid, nchunks, share ? 1 : 0);
  else if (lanes == 2)
    hipLaunchKernelGGL(k_refine<2>, dim3(ch ? (unsigned)nchunks : g2), dim3(64), 0, st, B, N, ntot, sblk, snode, pool,
                       lo, hi, clo, chi, sflag, C, v, cstart, rid, nchunks, share ? 1 : 0);
  else
    hipLaunchKernelGGL(k_refine<1>, dim3(ch ? (unsigned)nchunks : g1), dim3(64), 0, st, B, N, ntot, sblk, snode, pool,
                       lo, hi, clo, chi, sflag, C, v, cstart, rid, nchunks, share ? 1 : 0);
}

void launch_refine_fill(hipStream_t st, const Block* B, const Node* N, int64_t ntot, const int32_t* sblk,
                        const int32_t* snode, const Rep* pool, double* lo, double* hi, int32_t* clo, int32_t* chi,
                        uint32_t* sflag, Counters* C, int lanes, const int64_t* cstart, const int32_t* rid,
                        const int64_t* rstart, int nchunks, int32_t* claim, int32_t* cursor, int max_waves) {
  if (nchunks <= 0 || ntot <= 0) return;
  const int grid = std::max(1, std::min(nchunks, max_waves));
  hipLaunchKernelGGL(k_fill_init, GRID1(ntot, 256), 0, st, ntot, claim, cursor, grid);
  if (lanes >= 4)
    hipLaunchKernelGGL(k_refine_fill<4>, dim3(grid), dim3(64), 0, st, B, N, ntot, sblk, snode, pool, lo, hi, clo, chi,
                       sflag, C, cstart, rid, rstart, nchunks, claim, cursor);
  else if (lanes == 2)
    hipLaunchKernelGGL(k_refine_fill<2>, dim3(grid), dim3(64), 0, st, B, N, ntot, sblk, snode, pool, lo, hi, clo, chi,
                       sflag, C, cstart, rid, rstart, nchunks, claim, cursor);
  else
    hipLaunchKernelGGL(k_refine_fill<1>, dim3(grid), dim3(64), 0, st, B, N, ntot, sblk, snode, pool, lo, hi, clo, chi,
                       sflag, C, cstart, rid, rstart, nchunks, claim, cursor);
}

int device_simds() { return simd_count(); }

void launch_mark_leaf(hipStream_t st, int64_t ntot, const int64_t* scol, uint32_t* sflag) {
  hipLaunchKernelGGL(k_mark_leaf, GRID1(ntot, 256), 0, st, ntot, scol, sflag);
}

void launch_columns(hipStream_t st, const Problem* P, Block* B, int nblk, const Node* N, int64_t ntot,
                    const int32_t* sblk, const double* lo, const double* hi, double* val, int64_t* scol,
                    bool multi) {
  if (multi) hipLaunchKernelGGL(k_cummax, GRID1(nblk, 64), 0, st, B, nblk, N, lo, hi, P, val);
  hipLaunchKernelGGL(k_columns, GRID1(ntot, 256), 0, st, P, B, ntot, sblk, val, scol);
  if (multi) hipLaunchKernelGGL(k_block_wanted, GRID1(nblk, 64), 0, st, B, nblk, P, scol);
}

void launch_cls_flags(hipStream_t st, const Block* B, const Node* N, int64_t ntot, const int32_t* sblk,
                      const int32_t* snode, const double* lo, const double* hi, uint32_t* sflag, int32_t* runflag,
                      Counters* C) {
  hipLaunchKernelGGL(k_cls_flags, GRID1(ntot, 256), 0, st, B, N, ntot, sblk, snode, lo, hi, sflag, runflag, C);
}

void launch_cls_compact(hipStream_t st, int64_t ntot, const int32_t* runflag, const int32_t* runid, int64_t* runs) {
  hipLaunchKernelGGL(k_cls_compact, GRID1(ntot, 256), 0, st, ntot, runflag, runid, runs);
}

void launch_cls_runs(hipStream_t st, const Block* B, const Node* N, int nruns, const int64_t* runs,
                     const int32_t* sblk, const int32_t* snode, const double* lo, const double* hi,
                     const int64_t* scol, uint32_t* sflag, double* sgap, Cluster* clusters, int max_clusters,
                     Counters* C, int max_depth) {
  if (nruns == 0) return;
  hipLaunchKernelGGL(k_cls_runs, GRID1(nruns, 64), 0, st, B, N, nruns, runs, sblk, snode, lo, hi, scol, sflag,
                     sgap, clusters, max_clusters, C, max_depth);
}

void launch_child(hipStream_t st, const Block* B, Node* N, int nclusters, int node_base, const Cluster* clusters,
                  const double* lo, const double* hi, Rep* pool, unsigned long long pool_cap, Counters* C,
                  double growth_limit) {
  hipLaunchKernelGGL(k_child, dim3(nclusters), dim3(64), 0, st, B, N, nclusters, node_base, clusters, lo, hi, pool,
                     pool_cap, C, growth_limit);
}

void launch_shift(hipStream_t st, const Block* B, const Node* N, int nclusters, int node_base,
                  const Cluster* clusters, const int64_t* scol, double* lo, double* hi, int32_t* clo, int32_t* chi,
                  int32_t* snode, uint32_t* sflag, double* sgap) {
  hipLaunchKernelGGL(k_shift, dim3(nclusters), dim3(256), 0, st, B, N, node_base, clusters, scol, lo, hi, clo, chi,
                     snode, sflag, sgap);
}

void launch_clear_active(hipStream_t st, int64_t ntot, uint32_t* sflag) {
  hipLaunchKernelGGL(k_clear_active, GRID1(ntot, 256), 0, st, ntot, sflag);
}

void launch_node_chunks(hipStream_t st, int64_t ntot, const uint32_t* sflag, const int64_t* scol, uint32_t need,
                        bool need_col, const int32_t* snode, int slots, int32_t* runflag, int32_t* runid,
                        int32_t* tiles, int32_t* total, int32_t* rid, int64_t* rstart, int32_t* cflag, int32_t* cid,
                        int64_t* cstart) {
  if (ntot == 0) return;
  const int nc = need_col ? 1 : 0;
  hipLaunchKernelGGL(k_vec_runs, GRID1(ntot, 256), 0, st, ntot, sflag, scol, need, nc, snode, runflag);
  launch_scan(st, runflag, runid, tiles, ntot, total);
  hipLaunchKernelGGL(k_vec_rid, GRID1(ntot, 256), 0, st, ntot, sflag, scol, need, nc, runflag, runid, rid, rstart);
  hipLaunchKernelGGL(k_vec_cflags, GRID1(ntot, 256), 0, st, ntot, rid, rstart, slots, cflag);
  launch_scan(st, cflag, cid, tiles, ntot, total);
  hipLaunchKernelGGL(k_vec_cstart, GRID1(ntot, 256), 0, st, ntot, cflag, cid, cstart);
}

// the reciprocal and quotient forms of the kernels on caller-given operands
__global__ void k_probe_division(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                 double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = b[i];
  out[i] = __builtin_amdgcn_rcp(x);
  out[n + i] = rcp_nr1(x);
  out[2 * n + i] = rcp_nr2(x);
  out[3 * n + i] = div_nr(a[i], x);
}

void launch_probe_division(hipStream_t st, int64_t n, const double* a, const double* b, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_probe_division, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, b, out);
}

void launch_vectors(hipStream_t st, const Problem* P, const Block* B, const Node* N, const int64_t* cstart,
                    int nchunks, int64_t ntot, const int32_t* rid, const int32_t* sblk, const int32_t* snode,
                    const int64_t* scol, const double* lo, const double* hi, const double* sgap, const Rep* pool,
                    const double* ds, double* scratch, int64_t stride, double* w, double* Z, Counters* C, int slots) {
  if (nchunks == 0) return;
  // the kernel's full register budget (one wavefront per SIMD) while the
  // launch has no more wavefronts than the device has SIMDs; half of it (two
  // per SIMD, some spilling) once wavefronts would otherwise wait for a SIMD
  const bool wide = nchunks > simd_count();
#define MRRR_VEC(SL)                                                                                              \
  do {                                                                                                            \
    if (wide)                                                                                                     \
      hipLaunchKernelGGL((k_vectors<SL, 2>), dim3(nchunks), dim3(64), 0, st, P, B, N, cstart, nchunks, ntot, rid,   \
                         sblk, snode, scol, lo, hi, sgap, pool, ds, scratch, stride, w, Z, C);                        \
    else                                                                                                          \
      hipLaunchKernelGGL((k_vectors<SL, 1>), dim3(nchunks), dim3(64), 0, st, P, B, N, cstart, nchunks, ntot, rid,   \
                         sblk, snode, scol, lo, hi, sgap, pool, ds, scratch, stride, w, Z, C);                        \
  } while (0)
  if (slots == 8)
    MRRR_VEC(8);
  else if (slots == 16)
    MRRR_VEC(16);
  else
    MRRR_VEC(32);
#undef MRRR_VEC
}

void launch_vectors_stored(hipStream_t st, const Problem* P, const Block* B, const Node* N, const int32_t* chunks,
                           const int64_t* chunk_off, int nchunks, int64_t ntot, const int32_t* sblk,
                           const int32_t* snode, const uint32_t* sflag, const int64_t* scol, const double* lo,
                           const double* hi, const double* sgap, const Rep* pool, const double* ds, double* scratch,
                           double* w, double* Z, Counters* C, int slots) {
  if (nchunks == 0) return;
#define MRRR_VEC(SL)                                                                                              \
  hipLaunchKernelGGL(k_vectors_stored<SL>, dim3(nchunks), dim3(64), 0, st, P, B, N, chunks, chunk_off, nchunks, ntot, \
                     sblk, snode, sflag, scol, lo, hi, sgap, pool, ds, scratch, w, Z, C)
  if (slots == 8)
    MRRR_VEC(8);
  else if (slots == 16)
    MRRR_VEC(16);
  else
    MRRR_VEC(32);
#undef MRRR_VEC
}

void launch_chunk_rows(hipStream_t st, const Block* B, int64_t ntot, const int32_t* sblk, const uint32_t* sflag,
                       const int64_t* scol, int slots, int32_t* rows) {
  const int64_t nch = (ntot + slots - 1) / slots;
  if (nch == 0) return;
  hipLaunchKernelGGL(k_chunk_rows, dim3((unsigned)nch), dim3(64), 0, st, B, ntot, sblk, sflag, scol, slots, rows);
}

void launch_mark_ckpt(hipStream_t st, int64_t ntot, const Block* B, const int32_t* sblk, const int32_t* rid,
                      const int64_t* rstart, int min_run, int min_n, uint32_t* sflag) {
  if (ntot == 0) return;
  hipLaunchKernelGGL(k_mark_ckpt, GRID1(ntot, 256), 0, st, ntot, B, sblk, rid, rstart, min_run, min_n, sflag);
}

void launch_check_sorted(hipStream_t st, const Problem* P, int nprob, const double* w, int32_t* bad, Counters* C) {
  hipLaunchKernelGGL(k_check_sorted, dim3(nprob), dim3(256), 0, st, P, nprob, w, bad, C);
}

void launch_sort_fix(hipStream_t st, const Problem* P, int nprob, const int32_t* bad, double* w, int64_t* perm,
                     double* tmp, double* Z) {
  hipLaunchKernelGGL(k_sort_problem, dim3(nprob), dim3(64), 0, st, P, bad, w, perm);
  if (Z != nullptr) hipLaunchKernelGGL(k_permute_cols, dim3(nprob), dim3(256), 0, st, P, bad, perm, tmp, Z);
}

__global__ void k_store_info(InfoWords* __restrict__ dst, InfoWords v) {
  if (threadIdx.x < 18) dst->w[threadIdx.x] = v.w[threadIdx.x];
}

void launch_store_info(InfoWords* dst, InfoWords v, hipStream_t st) {
  hipLaunchKernelGGL(k_store_info, dim3(1), dim3(64), 0, st, dst, v);
}

void launch_values_only(hipStream_t st, const Problem* P, const Block* B, const Node* N, int64_t ntot,
                        const int32_t* sblk, const int32_t* snode, const int64_t* scol, const double* lo,
                        const double* hi, const double* ds, double* w) {
  hipLaunchKernelGGL(k_values_only, GRID1(ntot, 256), 0, st, P, B, N, ntot, sblk, snode, scol, lo, hi, ds, w);
}

}  // namespace mrrr
