// Stage 3 reduction to tridiagonal form T = Q^T M Q (arXiv:1205.2107
// Sec. 1.2, stage 3; Sec. 2.2: the direct reduction of the paper's dense
// pipeline), gfx950, FP64.
//
// Lower Householder reduction: column i = 0 .. n-2 in turn, the reflector
// H_i = I - tau_i v_i v_i^T (v_i[:i+1] = 0, v_i[i+1] = 1) maps the column's
// entries below the diagonal onto beta_i e_1, and the trailing matrix becomes
// H_i A H_i = A - v w^T - w v^T, y = tau A v, w = y - (tau/2)(v^T y) v.
//
// Blocked in panels of NBR columns (the panel form of LAPACK's dsytrd): the
// trailing matrix is updated once per panel, A <- A - V W^T - W V^T with the
// panel's reflectors V and vectors W (k_tr_syr2k, FP64 matrix cores).  Inside
// the panel the current matrix is A - V_j W_j^T - W_j V_j^T for the first j
// columns, so per column
//   column update   a = A[:, i] - V_j W_j[i, :]^T - W_j V_j[i, :]^T
//   reflector       from a[i+1:]
//   product         y = tau (A v - V_j (W_j^T v) - W_j (V_j^T v))
//   correction      w = y - (tau/2)(v^T y) v.
// The product's A v reads the panel-start trailing matrix, its lower
// triangle only, in 64 x 64 tiles: a workgroup takes up to kStrip tiles of
// one column strip J, accumulates A_IJ^T v_I for the strip's columns over its
// tiles and forms A_IJ v_J for each tile's rows; these partial sums go to one
// slot per (row block, contributor), and k_tr_ysum adds each row's slots in a
// fixed order (k_tr_symv, k_tr_ysum).  The strict upper triangle is neither
// read nor written.  The column work is spread so that only the reflector
// itself runs in one workgroup:
//   k_tr_col   (one workgroup)  finishes the previous column's w (its
//              (tau/2)(v^T y) term needs the global sum of k_tr_w's
//              partials), the rest of the column update, the reflector;
//   k_tr_symv  the partial sums of A v; W_j^T v and V_j^T v;
//   k_tr_ysum  A v from the partial sums;
//   k_tr_w     (one row per thread) w before its correction, the partial
//              sums of v^T w, and the next column's update by every pair
//              but the correction term.
// Reductions run in a fixed order: results are the same from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "mrrr.h"
#include "mrrr_prof.h"

namespace mrrr_tr {

constexpr int NBR = 64;         // panel width (reflectors per trailing update)
constexpr int TK = 16;          // reduction step of the panel update staged in LDS
constexpr int NT = 256;         // threads per workgroup (panel update, w, mirror)
constexpr int NTC = 1024;       // threads of the reflector workgroup
constexpr int kStrip = 8;       // tiles of one column strip per workgroup of the product
constexpr int kSW = 8;          // wavefronts per workgroup of the product
constexpr int kCPT = NBR / kSW; // tile columns per thread in the product
constexpr int kYW = 8;          // wavefronts per workgroup adding the product's slots

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// sum (or max) over the workgroup in a fixed order; every thread gets it
template <bool kMax>
__device__ double block_reduce(double x, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  x = kMax ? wave_max(x) : wave_sum(x);
  __syncthreads();
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  double r = sh[0];
  for (int k = 1; k < nw; ++k) r = kMax ? fmax(r, sh[k]) : r + sh[k];
  return r;
}

// the sum of the partials S[0 .. nS) by the first wavefront (every lane
// gets it): lane l adds S[l], S[l + 64], ... in order, then the lanes in a
// fixed tree
__device__ __forceinline__ double sum_partials(const double* __restrict__ S, int nS) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nS; b += 64) s += S[b];
  return wave_sum(s);
}

// two maxima over the workgroup with one pair of barriers; every thread gets both
__device__ void block_max2(double& x, double& y, double* sh, double* sh2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  x = wave_max(x);
  y = wave_max(y);
  __syncthreads();
  if (lane == 0) {
    sh[wave] = x;
    sh2[wave] = y;
  }
  __syncthreads();
  x = sh[0];
  y = sh2[0];
  for (int k = 1; k < nw; ++k) {
    x = fmax(x, sh[k]);
    y = fmax(y, sh2[k]);
  }
}

// ---------------------------------------------------------------------------
// the column update and reflector of column i (j = i - k within the panel).
// A[r, i] for r >= i holds the column updated by every pair of the panel but
// the correction term of pair j - 1, which is applied here together with
// finishing that pair's w: W[r, j-1] += alpha v_{j-1}[r], a[r] -= 2 alpha
// v_{j-1}[r] (v_{j-1}[i] = 1), alpha = -(tau_{i-1}/2) sum(S).
// last: i = n - 1, no reflector (only d).
__global__ void __launch_bounds__(NTC) k_tr_col(int64_t n, double* __restrict__ A, int64_t lda, int64_t i, int j,
                                                double* __restrict__ Vp, double* __restrict__ Wp,
                                                const double* __restrict__ S, int nS, double* __restrict__ d,
                                                double* __restrict__ e, double* __restrict__ tau, int last) {
  __shared__ double sh[NTC / 64], sh2[NTC / 64];
  __shared__ double s_alpha;
  const int t = threadIdx.x;
  double* col = A + i * lda;
  // the column update (j > 0) and the largest magnitudes of the entries below
  // the diagonal (mx) and below the subdiagonal (mt) in one pass
  double mx = 0.0, mt = 0.0;
  if (j > 0) {
    if (t < 64) {
      const double s = sum_partials(S, nS);
      if (t == 0) s_alpha = -0.5 * tau[i - 1] * s;
    }
    __syncthreads();
    const double al = s_alpha;
    double* vp = Vp + (int64_t)(j - 1) * n;
    double* wp = Wp + (int64_t)(j - 1) * n;
    for (int64_t r = i + t; r < n; r += NTC) {
      const double v = vp[r];
      wp[r] = fma(al, v, wp[r]);
      const double c = fma(-2.0 * al, v, col[r]);
      col[r] = c;
      if (r >= i + 1) mx = fmax(mx, fabs(c));
      if (r >= i + 2) mt = fmax(mt, fabs(c));
    }
  } else {
    for (int64_t r = i + 1 + t; r < n; r += NTC) {
      const double a = fabs(col[r]);
      mx = fmax(mx, a);
      if (r >= i + 2) mt = fmax(mt, a);
    }
  }
  if (last) {
    __syncthreads();
    if (t == 0) d[i] = col[i];
    return;
  }
  // reflector of x = col[i+1 ..]: scale by a power of two near max |x|
  block_max2(mx, mt, sh, sh2);
  const double alpha = col[i + 1];
  double beta = alpha, tu = 0.0, scale = 0.0;
  if (mt > 0.0) {
    int ex;
    (void)frexp(mx, &ex);
    double ss = 0.0;
    for (int64_t r = i + 2 + t; r < n; r += NTC) {
      const double a = ldexp(col[r], -ex);
      ss = fma(a, a, ss);
    }
    ss = block_reduce<false>(ss, sh);
    const double sa = ldexp(alpha, -ex);
    const double norm = ldexp(sqrt(fma(sa, sa, ss)), ex);
    beta = alpha >= 0.0 ? -norm : norm;
    tu = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  double* vj = Vp + (int64_t)j * n;
  for (int64_t r = i + 2 + t; r < n; r += NTC) {
    const double v = col[r] * scale;
    col[r] = v;
    vj[r] = v;
  }
  if (t == 0) {
    d[i] = col[i];
    e[i] = beta;
    tau[i] = tu;
    col[i + 1] = beta;
    vj[i + 1] = 1.0;
  }
}

// group g of column strip J of the product -> linear index: the groups are
// numbered by g, then J; group g of every strip J < Tn - g kStrip exists
__device__ __forceinline__ int64_t strip_offset(int64_t g, int64_t Tn) { return g * Tn - kStrip * g * (g - 1) / 2; }
__device__ __forceinline__ void strip_group(int64_t l, int64_t Tn, int64_t* g, int64_t* J) {
  const double b = (double)Tn + 0.5 * kStrip;
  int64_t x = (int64_t)((b - sqrt(fmax(0.0, b * b - 2.0 * kStrip * (double)l))) / kStrip);
  x = x < 0 ? 0 : x;
  while (x > 0 && strip_offset(x, Tn) > l) --x;
  while (strip_offset(x + 1, Tn) <= l && (x + 1) * kStrip < Tn) ++x;
  *g = x;
  *J = l - strip_offset(x, Tn);
}

// Partial sums of y = A v over the trailing matrix (rows and columns
// o = i+1 .. n-1, lower triangle), v = V[:, j].  Blocks of 64 rows are counted
// from T0 = o / 64 (absolute alignment; rows and columns below o masked), Tn
// of them; P holds Tn slots of 64 doubles per block:
//   slot J < K of block K:            A_KJ v_J              (tile (K, J))
//   slot K + g kStrip of block K:     sum over the tiles I of group g of
//                                     strip K of A_IK^T v_I, plus for g = 0
//                                     the strict lower part of A_KK v_K.
// Workgroup (g, J) takes tiles I = J + g kStrip .. of strip J: thread (a, w)
// holds row a of the tile in its 16 columns b = w + 4k, forms its share of
// A_IJ v_J (the four wavefronts' shares added in LDS) and accumulates
// A_IJ^T v_I over its tiles; at the end each wavefront reduces its 16 column
// sums across its lanes (halving exchanges).  The next tile is fetched while
// the current one is used.  Workgroups past ntask form pq[j'] = W[:, j'] . v
// and pq[NBR + j'] = V[:, j'] . v, j' < j.
__global__ void __launch_bounds__(64 * kSW) k_tr_symv(int64_t n, const double* __restrict__ A, int64_t lda, int64_t i,
                                                int j, const double* __restrict__ Vp, const double* __restrict__ Wp,
                                                double* __restrict__ P, double* __restrict__ pq, int64_t ntask) {
  __shared__ double vJs[NBR];
  __shared__ double rs[2][kSW][NBR];
  __shared__ double us[NBR];
  __shared__ double sh[kSW];
  const int t = threadIdx.x, lane = t & 63, part = t >> 6;
  const int64_t o = i + 1;
  const int64_t T0 = o >> 6, Tn = ((n + 63) >> 6) - T0;
  const double* v = Vp + (int64_t)j * n;
  if ((int64_t)blockIdx.x >= ntask) {
    const int jj = (int)(blockIdx.x - ntask);
    const double* w = Wp + (int64_t)jj * n;
    const double* u = Vp + (int64_t)jj * n;
    double sp = 0.0, sq = 0.0;
    for (int64_t r = o + t; r < n; r += 64 * kSW) {
      const double vr = v[r];
      sp = fma(w[r], vr, sp);
      sq = fma(u[r], vr, sq);
    }
    sp = block_reduce<false>(sp, sh);
    sq = block_reduce<false>(sq, sh);
    if (t == 0) {
      pq[jj] = sp;
      pq[NBR + jj] = sq;
    }
    return;
  }
  int64_t g, Jr;
  strip_group(blockIdx.x, Tn, &g, &Jr);
  const int64_t Ib = Jr + g * kStrip, Ie = std::min<int64_t>(Tn, Ib + kStrip);
  const int64_t cJ = (T0 + Jr) * NBR;
  if (t < NBR) {
    const int64_t c = cJ + t;
    vJs[t] = (c >= o && c < n) ? v[c] : 0.0;
  }
  __syncthreads();
  double vj[kCPT], u[kCPT], cur[kCPT], nxt[kCPT];
#pragma unroll
  for (int k = 0; k < kCPT; ++k) {
    vj[k] = vJs[part + kSW * k];
    u[k] = 0.0;
  }
  auto fetch = [&](int64_t I, double* dst) {
    const int64_t r = (T0 + I) * NBR + lane;
    const bool rin = r >= o && r < n;
    const bool diag = I == Jr;
#pragma unroll
    for (int k = 0; k < kCPT; ++k) {
      const int b = part + kSW * k;
      const int64_t c = cJ + b;
      const bool in = rin && c >= o && c < n && (!diag || lane >= b);
      dst[k] = in ? A[c * lda + r] : 0.0;
    }
  };
  fetch(Ib, nxt);
  double xdiag = 0.0;
  for (int64_t I = Ib; I < Ie; ++I) {
#pragma unroll
    for (int k = 0; k < kCPT; ++k) cur[k] = nxt[k];
    if (I + 1 < Ie) fetch(I + 1, nxt);
    const int64_t r = (T0 + I) * NBR + lane;
    const double vi = (r >= o && r < n) ? v[r] : 0.0;
    const bool diag = I == Jr;
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < kCPT; ++k) {
      const int b = part + kSW * k;
      const double a = (diag && b == lane) ? 0.0 : cur[k];  // the row sums take the strict lower part
      x = fma(a, vj[k], x);
      u[k] = fma(cur[k], vi, u[k]);
    }
    // two buffers: the barrier of the next tile orders this tile's readers
    // before the writers of the tile after it
    const int buf = (int)((I - Ib) & 1);
    rs[buf][part][lane] = x;
    __syncthreads();
    if (t < NBR) {
      double xs = rs[buf][0][t];
#pragma unroll
      for (int w = 1; w < kSW; ++w) xs += rs[buf][w][t];
      if (diag)
        xdiag = xs;
      else
        P[(I * Tn + Jr) * NBR + t] = xs;
    }
  }
  // column sums: log2(kCPT) halving exchanges leave lane l with column index
  // k(l) (the top bits of l) summed over the lanes that differ in those
  // bits; exchanges over the remaining bits complete it
  constexpr int kSteps = kCPT == 16 ? 4 : (kCPT == 8 ? 3 : (kCPT == 4 ? 2 : (kCPT == 2 ? 1 : 0)));
  static_assert((1 << kSteps) == kCPT, "columns per thread must be a power of two up to 16");
#pragma unroll
  for (int step = 0; step < kSteps; ++step) {
    const int off = 32 >> step, half = (kCPT / 2) >> step;
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int k = 0; k < kCPT / 2; ++k) {
      if (k < half) {
        const double lo = u[k], hi = u[k + half];
        const double send = up ? lo : hi;
        const double keep = up ? hi : lo;
        u[k] = keep + __shfl_xor(send, off, 64);
      }
    }
  }
  double cs = u[0];
#pragma unroll
  for (int off = 32 >> kSteps; off >= 1; off >>= 1) cs += __shfl_xor(cs, off, 64);
  if ((lane & ((32 >> kSteps) * 2 - 1)) == 0) {
    int k = 0;
#pragma unroll
    for (int step = 0; step < kSteps; ++step) k = 2 * k + ((lane >> (5 - step)) & 1);
    us[part + kSW * k] = cs;
  }
  __syncthreads();
  if (t < NBR) P[(Jr * Tn + Ib) * NBR + t] = (g == 0) ? us[t] + xdiag : us[t];
}

// y[r] = (A v)[r] for rows o .. n-1: block K's slots added in a fixed order
// (each of the four wavefronts a quarter of them, then the four in order)
__global__ void __launch_bounds__(64 * kYW) k_tr_ysum(int64_t n, int64_t i, const double* __restrict__ P,
                                                      double* __restrict__ y) {
  __shared__ double rs[kYW][NBR];
  const int t = threadIdx.x, a = t & 63, part = t >> 6;
  const int64_t o = i + 1;
  const int64_t T0 = o >> 6, Tn = ((n + 63) >> 6) - T0;
  const int64_t K = blockIdx.x;
  const double* p = P + (K * Tn) * NBR + a;
  double s0 = 0.0, s1 = 0.0;
  int64_t s = part;
  for (; s + kYW < K; s += 2 * kYW) {
    s0 += p[s * NBR];
    s1 += p[(s + kYW) * NBR];
  }
  for (; s < K; s += kYW) s0 += p[s * NBR];
  for (int64_t gg = part; K + gg * kStrip < Tn; gg += kYW) s1 += p[(K + gg * kStrip) * NBR];
  rs[part][a] = s0 + s1;
  __syncthreads();
  if (t < NBR) {
    const int64_t r = (T0 + K) * NBR + t;
    double acc = rs[0][t];
#pragma unroll
    for (int w = 1; w < kYW; ++w) acc += rs[w][t];
    if (r >= o && r < n) y[r] = acc;
  }
}

// w before its correction, one row per thread over rows i+1 .. n-1:
// w[r] = tau (y[r] - sum_{j'<j} (V[r,j'] p[j'] + W[r,j'] q[j'])), stored in
// W[:, j]; S[block] = sum of w[r] v[r] over the block's rows.  With next
// (column i+1 belongs to the panel): A[r, i+1] -= sum_{j'<j} (V[r,j'] W[i+1,j']
// + W[r,j'] V[i+1,j']) + v[r] w[i+1] + w[r] (v[i+1] = 1), i.e. every pair's
// share of the next column's update but pair j's correction term.
__device__ __forceinline__ double w_row(double yr, const double* vrow, const double* wrow, int64_t ldp,
                                        const double* p, const double* q, int j, double tu) {
  double acc = yr;
  for (int jj = 0; jj < j; ++jj) {
    acc = fma(-vrow[(int64_t)jj * ldp], p[jj], acc);
    acc = fma(-wrow[(int64_t)jj * ldp], q[jj], acc);
  }
  return tu * acc;
}

__global__ void __launch_bounds__(NT) k_tr_w(int64_t n, double* __restrict__ A, int64_t lda, int64_t i, int j,
                                             double* __restrict__ Vp, double* __restrict__ Wp,
                                             const double* __restrict__ y, const double* __restrict__ pq,
                                             const double* __restrict__ tau, double* __restrict__ S, int next) {
  __shared__ double p[NBR], q[NBR], vn[NBR], wn[NBR];
  __shared__ double sh[NT / 64];
  __shared__ double s_w1;
  const int t = threadIdx.x;
  const double tu = tau[i];
  if (t < j) {
    p[t] = pq[t];
    q[t] = pq[NBR + t];
    vn[t] = Vp[(int64_t)t * n + i + 1];
    wn[t] = Wp[(int64_t)t * n + i + 1];
  }
  __syncthreads();
  if (t == 0 && next) s_w1 = w_row(y[i + 1], Vp + i + 1, Wp + i + 1, n, p, q, j, tu);
  __syncthreads();
  const int64_t r = i + 1 + (int64_t)blockIdx.x * NT + t;
  double part = 0.0;
  if (r < n) {
    const double wr = w_row(y[r], Vp + r, Wp + r, n, p, q, j, tu);
    const double vr = Vp[(int64_t)j * n + r];
    Wp[(int64_t)j * n + r] = wr;
    part = wr * vr;
    if (next) {
      double a = A[(i + 1) * lda + r];
      for (int jj = 0; jj < j; ++jj) {
        a = fma(-Vp[(int64_t)jj * n + r], wn[jj], a);
        a = fma(-Wp[(int64_t)jj * n + r], vn[jj], a);
      }
      a = fma(-vr, s_w1, a);
      a -= wr;
      A[(i + 1) * lda + r] = a;
    }
  }
  part = block_reduce<false>(part, sh);
  if (t == 0) S[blockIdx.x] = part;
}

// the last panel column's w: W[r, j] += alpha v[r], alpha = -(tau_i/2) sum(S)
__global__ void __launch_bounds__(NT) k_tr_wfin(int64_t n, int64_t i, int j, const double* __restrict__ Vp,
                                                double* __restrict__ Wp, const double* __restrict__ S, int nS,
                                                const double* __restrict__ tau) {
  __shared__ double s_alpha;
  if (threadIdx.x < 64) {
    const double s = sum_partials(S, nS);
    if (threadIdx.x == 0) s_alpha = -0.5 * tau[i] * s;
  }
  __syncthreads();
  const int64_t r = i + 1 + (int64_t)blockIdx.x * NT + threadIdx.x;
  if (r < n) Wp[(int64_t)j * n + r] = fma(s_alpha, Vp[(int64_t)j * n + r], Wp[(int64_t)j * n + r]);
}

// lower 64 x 64 tile number tl -> (I, J), I >= J
__device__ __forceinline__ void lower_tile(int64_t tl, int64_t* I, int64_t* J) {
  int64_t a = (int64_t)((sqrt(8.0 * (double)tl + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > tl) --a;
  while ((a + 1) * (a + 2) / 2 <= tl) ++a;
  *I = a;
  *J = tl - a * (a + 1) / 2;
}

// writes the lower part of tile L (L[b][a] = entry (a, b) of block (I, J),
// padded) to block (I, J): all of it below the diagonal blocks, the lower
// triangle of a diagonal block.  Rows and columns at or beyond mt (the
// trailing order) are skipped.
__device__ void store_lower_tile(double* __restrict__ A, int64_t lda, int64_t o, int64_t mt, int64_t I, int64_t J,
                                 const double (*L)[NBR + 1]) {
  const int t = threadIdx.x;
  const int64_t oi = o + I * NBR, oj = o + J * NBR;
  const int64_t ri = std::min<int64_t>(NBR, mt - I * NBR), rj = std::min<int64_t>(NBR, mt - J * NBR);
  for (int e = t; e < NBR * NBR; e += NT) {
    const int a = e & (NBR - 1), b = e >> 6;
    if (a < ri && b < rj && (I != J || a >= b)) A[(oj + b) * lda + oi + a] = L[b][a];
  }
}

__device__ void load_tile(const double* __restrict__ A, int64_t lda, int64_t o, int64_t mt, int64_t I, int64_t J,
                          double (*L)[NBR + 1]) {
  const int t = threadIdx.x;
  const int64_t oi = o + I * NBR, oj = o + J * NBR;
  const int64_t ri = std::min<int64_t>(NBR, mt - I * NBR), rj = std::min<int64_t>(NBR, mt - J * NBR);
  for (int e = t; e < NBR * NBR; e += NT) {
    const int a = e & (NBR - 1), b = e >> 6;
    L[b][a] = (a < ri && b < rj) ? A[(oj + b) * lda + oi + a] : 0.0;
  }
}

// One 64 x 64 x 16 step: P[a][k], Q[b][k] in LDS; each wave accumulates a
// 32 x 32 quadrant as 2 x 2 MFMA 16x16 blocks over four K-chunks of 4.
// v_mfma_f64_16x16x4f64: lane l supplies P[l % 16][l / 16] and Q[l / 16][l % 16].
__device__ inline void mma_step(const double (*P)[TK + 1], const double (*Q)[TK + 1], v4d acc[2][2], int wr, int wc,
                                int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kc = 0; kc < TK / 4; ++kc) {
    double a[2], b[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) a[m] = P[wr * 32 + m * 16 + li][kc * 4 + lk];
#pragma unroll
    for (int q = 0; q < 2; ++q) b[q] = Q[wc * 32 + q * 16 + li][kc * 4 + lk];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
  }
}

// the accumulator's (row, column) inside the 64 x 64 tile for lane, block (m, q), element v
__device__ __forceinline__ int acc_row(int wr, int m, int lane, int v) { return wr * 32 + m * 16 + (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_col(int wc, int q, int lane) { return wc * 32 + q * 16 + (lane & 15); }

// trailing update A[o:, o:] -= V W^T + W V^T over the panel's NBR pairs
// (rows o .. n-1 of Vp, Wp), one lower 64 x 64 tile per workgroup, written to
// both triangles.  The product [V_I | W_I] [W_J | V_J]^T runs over K = 2 NBR
// in steps of TK, the next step's operands fetched into registers while the
// matrix cores work.
__global__ void __launch_bounds__(NT) k_tr_syr2k(int64_t n, double* __restrict__ A, int64_t lda, int64_t o,
                                                 const double* __restrict__ Vp, const double* __restrict__ Wp) {
  __shared__ double Ps[NBR][TK + 1];
  __shared__ double Qs[NBR][TK + 1];
  __shared__ double L[NBR][NBR + 1];
  const int64_t mt = n - o;
  int64_t I, J;
  lower_tile(blockIdx.x, &I, &J);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // loader: thread t fetches tile row t % 64, K entries 4 (t / 64) .. +3
  const int la = t & 63, lk = (t >> 6) * 4;
  const int64_t gi = o + I * NBR + la, gj = o + J * NBR + la;
  const bool ini = gi < n, inj = gj < n;
  double rp[4], rq[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + lk + u;
      const double* pa = k < NBR ? Vp + (int64_t)k * n : Wp + (int64_t)(k - NBR) * n;
      const double* qa = k < NBR ? Wp + (int64_t)k * n : Vp + (int64_t)(k - NBR) * n;
      rp[u] = ini ? pa[gi] : 0.0;
      rq[u] = inj ? qa[gj] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < 2 * NBR; k0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Ps[la][lk + u] = rp[u];
      Qs[la][lk + u] = rq[u];
    }
    __syncthreads();
    if (k0 + TK < 2 * NBR) fetch(k0 + TK);
    mma_step(Ps, Qs, acc, wr, wc, lane);
    __syncthreads();
  }
  load_tile(A, lda, o, mt, I, J, L);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) L[acc_col(wc, q, lane)][acc_row(wr, m, lane, v)] -= acc[m][q][v];
  __syncthreads();
  store_lower_tile(A, lda, o, mt, I, J, L);
}

// ---------------------------------------------------------------------------
// host side

static std::mutex g_mu;
static void* g_ws = nullptr;
static size_t g_ws_bytes = 0;
static int g_ws_dev = -1;

static int grow(size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    mrrr::set_last_error("hipGetDevice failed");
    return MRRR_ERR_HIP;
  }
  if (bytes <= g_ws_bytes && g_ws && dev == g_ws_dev) return 0;
  if (g_ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g_ws);
  }
  g_ws = nullptr;
  g_ws_bytes = 0;
  const size_t nb = std::max(bytes, (size_t)1 << 20);
  if (hipMalloc(&g_ws, nb) != hipSuccess) {
    mrrr::set_last_error("hipMalloc failed for the tridiagonal reduction workspace");
    return MRRR_ERR_CAPACITY;
  }
  g_ws_bytes = nb;
  g_ws_dev = dev;
  return 0;
}

static unsigned lower_tiles(int64_t m) {
  const int64_t T = (m + NBR - 1) / NBR;
  return (unsigned)(T * (T + 1) / 2);
}

}  // namespace mrrr_tr

using namespace mrrr_tr;

extern "C" {

int mrrr_tridiagonalize(int64_t n, double* A, int64_t lda, double* d, double* e, double* tau, void* stream) {
  if (n < 0 || n > (int64_t)1 << 18) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (n > 0 && !d) return -4;
  if (n > 1 && !e) return -5;
  if (n > 1 && !tau) return -6;
  if (n == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t nS_max = (n + NT - 1) / NT;
  const int64_t nb_max = (n + NBR - 1) / NBR;  // row blocks of the product's partial sums
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t pbytes = al(sizeof(double) * (size_t)(n * NBR));
  const size_t ybytes = al(sizeof(double) * (size_t)n);
  const size_t Pbytes = al(sizeof(double) * (size_t)(nb_max * nb_max * NBR));
  const size_t qbytes = al(sizeof(double) * 2 * NBR);
  const size_t sbytes = al(sizeof(double) * (size_t)nS_max);
  int rc = grow(2 * pbytes + ybytes + Pbytes + qbytes + sbytes);
  if (rc) return rc;
  char* base = (char*)g_ws;
  double* Vp = (double*)base;
  double* Wp = (double*)(base + pbytes);
  double* y = (double*)(base + 2 * pbytes);
  double* Py = (double*)(base + 2 * pbytes + ybytes);
  double* pq = (double*)(base + 2 * pbytes + ybytes + Pbytes);
  double* S = (double*)(base + 2 * pbytes + ybytes + Pbytes + qbytes);
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_TRIDIAG);
  int64_t launches = 0;
  int nS = 0;
  for (int64_t k = 0; k < n - 1; k += NBR) {
    const int pw = (int)std::min<int64_t>(NBR, n - 1 - k);
    for (int j = 0; j < pw; ++j) {
      const int64_t i = k + j;
      hipLaunchKernelGGL(k_tr_col, dim3(1), dim3(NTC), 0, st, n, A, lda, i, j, Vp, Wp, (const double*)S, nS, d, e,
                         tau, 0);
      const int64_t m = n - i - 1;
      const int64_t T0 = (i + 1) / NBR, Tn = (n + NBR - 1) / NBR - T0;
      const int64_t G = (Tn + kStrip - 1) / kStrip;
      const int64_t ntask = G * Tn - (int64_t)kStrip * G * (G - 1) / 2;
      hipLaunchKernelGGL(k_tr_symv, dim3((unsigned)(ntask + j)), dim3(64 * kSW), 0, st, n, (const double*)A, lda, i, j,
                         (const double*)Vp, (const double*)Wp, Py, pq, ntask);
      hipLaunchKernelGGL(k_tr_ysum, dim3((unsigned)Tn), dim3(64 * kYW), 0, st, n, i, (const double*)Py, y);
      nS = (int)((m + NT - 1) / NT);
      const int next = (j + 1 < pw) || (i + 1 == n - 1);
      hipLaunchKernelGGL(k_tr_w, dim3((unsigned)nS), dim3(NT), 0, st, n, A, lda, i, j, Vp, Wp, (const double*)y,
                         (const double*)pq, (const double*)tau, S, next);
      launches += 4;
    }
    if (k + pw == n - 1) {
      // the last column: its update by the final panel, then d
      hipLaunchKernelGGL(k_tr_col, dim3(1), dim3(NTC), 0, st, n, A, lda, n - 1, pw, Vp, Wp, (const double*)S, nS, d,
                         e, tau, 1);
      ++launches;
    } else {
      const int64_t i = k + pw - 1;
      hipLaunchKernelGGL(k_tr_wfin, dim3((unsigned)nS), dim3(NT), 0, st, n, i, pw - 1, (const double*)Vp, Wp,
                         (const double*)S, nS, (const double*)tau);
      const int64_t o = k + pw;
      hipLaunchKernelGGL(k_tr_syr2k, dim3(lower_tiles(n - o)), dim3(NT), 0, st, n, A, lda, o, (const double*)Vp,
                         (const double*)Wp);
      launches += 2;
    }
  }
  if (n == 1) {
    hipLaunchKernelGGL(k_tr_col, dim3(1), dim3(NTC), 0, st, n, A, lda, (int64_t)0, 0, Vp, Wp, (const double*)S, 0, d,
                       e, tau, 1);
    ++launches;
  }
  prof.end();
  hipError_t er = hipStreamSynchronize(st);
  if (er == hipSuccess) er = hipGetLastError();
  if (er != hipSuccess) {
    mrrr::set_last_error((std::string("tridiagonal reduction kernels failed: ") + hipGetErrorString(er)).c_str());
    return MRRR_ERR_HIP;
  }
  if (prof.on) {
    double ms;
    int64_t l;
    prof.total(MRRR_K_TRIDIAG, &ms, &l);
    // 4/3 n^3 flops; bytes: the product's reads of the trailing lower
    // triangles, sum over m = 1 .. n-1 of m (m + 1) / 2 entries
    const double nn = (double)n;
    const double work = 4.0 / 3.0 * nn * nn * nn;
    const double bytes = 8.0 * (nn - 1.0) * nn * (nn + 1.0) / 6.0;
    mrrr::prof_add(MRRR_K_TRIDIAG, launches, ms, work, bytes);
  }
  return 0;
}

}  // extern "C"
