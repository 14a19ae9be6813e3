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
// The product's A v reads the panel-start trailing matrix; A is kept with
// both triangles (mirrored from the lower one at the start, the panel
// updates write both), so (A v)[c] = A[:, c] . v reads one contiguous column
// per output entry (k_tr_symv).  The column work is spread so that only the
// reflector itself runs in one workgroup:
//   k_tr_col   (one workgroup)  finishes the previous column's w (its
//              (tau/2)(v^T y) term needs the global sum of k_tr_w's
//              partials), the rest of the column update, the reflector;
//   k_tr_symv  (one wavefront per two columns) A v, W_j^T v, V_j^T v;
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
constexpr int kSymvWaves = 4;   // wavefronts per workgroup of the product
constexpr int kUnroll = 4;      // row loads in flight per lane in the product

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
  __shared__ double sh[NTC / 64];
  __shared__ double s_alpha;
  const int t = threadIdx.x;
  double* col = A + i * lda;
  if (j > 0) {
    if (t == 0) {
      double s = 0.0;
      for (int b = 0; b < nS; ++b) s += S[b];
      s_alpha = -0.5 * tau[i - 1] * s;
    }
    __syncthreads();
    const double al = s_alpha;
    double* vp = Vp + (int64_t)(j - 1) * n;
    double* wp = Wp + (int64_t)(j - 1) * n;
    for (int64_t r = i + t; r < n; r += NTC) {
      const double v = vp[r];
      wp[r] = fma(al, v, wp[r]);
      col[r] = fma(-2.0 * al, v, col[r]);
    }
    __syncthreads();
  }
  if (last) {
    if (t == 0) d[i] = col[i];
    return;
  }
  // reflector of x = col[i+1 ..]: scale by a power of two near max |x|
  double mx = 0.0, mt = 0.0;
  for (int64_t r = i + 1 + t; r < n; r += NTC) {
    const double a = fabs(col[r]);
    mx = fmax(mx, a);
    if (r >= i + 2) mt = fmax(mt, a);
  }
  mx = block_reduce<true>(mx, sh);
  mt = block_reduce<true>(mt, sh);
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

// y[c] = A[i+1:, c] . v for c = i+1 .. n-1 (one wavefront per two columns),
// then pq[j'] = W[:, j'] . v and pq[NBR + j'] = V[:, j'] . v for j' < j
// (one wavefront per j'), all over rows i+1 .. n-1.
__global__ void __launch_bounds__(64 * kSymvWaves) k_tr_symv(int64_t n, const double* __restrict__ A, int64_t lda,
                                                             int64_t i, int j, const double* __restrict__ Vp,
                                                             const double* __restrict__ Wp, double* __restrict__ y,
                                                             double* __restrict__ pq) {
  const int lane = threadIdx.x & 63;
  const int64_t task = (int64_t)blockIdx.x * kSymvWaves + (threadIdx.x >> 6);
  const int64_t m = n - i - 1;
  const int64_t ncol = (m + 1) / 2;
  if (task >= ncol + j) return;
  const double* v = Vp + (int64_t)j * n;
  const double *c0, *c1;
  bool two = true;
  if (task < ncol) {
    const int64_t c = i + 1 + 2 * task;
    c0 = A + c * lda;
    two = c + 1 < n;
    c1 = two ? c0 + lda : c0;
  } else {
    const int jj = (int)(task - ncol);
    c0 = Wp + (int64_t)jj * n;
    c1 = Vp + (int64_t)jj * n;
  }
  // rows from i+1, loads aligned to 64-row groups
  const int64_t r0 = (i + 1) & ~(int64_t)63;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t rb = r0; rb < n; rb += 64 * kUnroll) {
    double a0[kUnroll], a1[kUnroll], vv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t rr = rb + 64 * u + lane;
      const bool in = rr > i && rr < n;
      vv[u] = in ? v[rr] : 0.0;
      a0[u] = in ? c0[rr] : 0.0;
      a1[u] = in ? c1[rr] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      s0 = fma(a0[u], vv[u], s0);
      s1 = fma(a1[u], vv[u], s1);
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    if (task < ncol) {
      const int64_t c = i + 1 + 2 * task;
      y[c] = s0;
      if (two) y[c + 1] = s1;
    } else {
      const int jj = (int)(task - ncol);
      pq[jj] = s0;
      pq[NBR + jj] = s1;
    }
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
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nS; ++b) s += S[b];
    s_alpha = -0.5 * tau[i] * s;
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

// writes the tile L (L[b][a] = entry (a, b) of block (I, J), padded) to block
// (I, J) and its transpose to block (J, I); a diagonal block takes its lower
// triangle mirrored.  Rows and columns at or beyond mt (the trailing order)
// are skipped.
__device__ void store_sym_tile(double* __restrict__ A, int64_t lda, int64_t o, int64_t mt, int64_t I, int64_t J,
                               const double (*L)[NBR + 1]) {
  const int t = threadIdx.x;
  const int64_t oi = o + I * NBR, oj = o + J * NBR;
  const int64_t ri = std::min<int64_t>(NBR, mt - I * NBR), rj = std::min<int64_t>(NBR, mt - J * NBR);
  for (int e = t; e < NBR * NBR; e += NT) {
    const int a = e & (NBR - 1), b = e >> 6;
    if (a < ri && b < rj) {
      const double x = (I != J || a >= b) ? L[b][a] : L[a][b];
      A[(oj + b) * lda + oi + a] = x;
    }
  }
  if (I != J)
    for (int e = t; e < NBR * NBR; e += NT) {
      const int b = e & (NBR - 1), a = e >> 6;  // entry (b, a) of block (J, I)
      if (a < ri && b < rj) A[(oi + a) * lda + oj + b] = L[b][a];
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

// upper triangle <- lower triangle, one lower tile per workgroup
__global__ void __launch_bounds__(NT) k_tr_mirror(int64_t n, double* __restrict__ A, int64_t lda) {
  __shared__ double L[NBR][NBR + 1];
  int64_t I, J;
  lower_tile(blockIdx.x, &I, &J);
  load_tile(A, lda, 0, n, I, J, L);
  __syncthreads();
  store_sym_tile(A, lda, 0, n, I, J, L);
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
  store_sym_tile(A, lda, o, mt, I, J, L);
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
  if (n < 0 || n > (int64_t)1 << 20) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (n > 0 && !d) return -4;
  if (n > 1 && !e) return -5;
  if (n > 1 && !tau) return -6;
  if (n == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t nS_max = (n + NT - 1) / NT;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t pbytes = al(sizeof(double) * (size_t)(n * NBR));
  const size_t ybytes = al(sizeof(double) * (size_t)n);
  const size_t qbytes = al(sizeof(double) * 2 * NBR);
  const size_t sbytes = al(sizeof(double) * (size_t)nS_max);
  int rc = grow(2 * pbytes + ybytes + qbytes + sbytes);
  if (rc) return rc;
  char* base = (char*)g_ws;
  double* Vp = (double*)base;
  double* Wp = (double*)(base + pbytes);
  double* y = (double*)(base + 2 * pbytes);
  double* pq = (double*)(base + 2 * pbytes + ybytes);
  double* S = (double*)(base + 2 * pbytes + ybytes + qbytes);
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_TRIDIAG);
  int64_t launches = 0;
  if (n > 1) {
    hipLaunchKernelGGL(k_tr_mirror, dim3(lower_tiles(n)), dim3(NT), 0, st, n, A, lda);
    ++launches;
  }
  int nS = 0;
  for (int64_t k = 0; k < n - 1; k += NBR) {
    const int pw = (int)std::min<int64_t>(NBR, n - 1 - k);
    for (int j = 0; j < pw; ++j) {
      const int64_t i = k + j;
      hipLaunchKernelGGL(k_tr_col, dim3(1), dim3(NTC), 0, st, n, A, lda, i, j, Vp, Wp, (const double*)S, nS, d, e,
                         tau, 0);
      const int64_t m = n - i - 1;
      const int64_t tasks = (m + 1) / 2 + j;
      hipLaunchKernelGGL(k_tr_symv, dim3((unsigned)((tasks + kSymvWaves - 1) / kSymvWaves)), dim3(64 * kSymvWaves),
                         0, st, n, (const double*)A, lda, i, j, (const double*)Vp, (const double*)Wp, y, pq);
      nS = (int)((m + NT - 1) / NT);
      const int next = (j + 1 < pw) || (i + 1 == n - 1);
      hipLaunchKernelGGL(k_tr_w, dim3((unsigned)nS), dim3(NT), 0, st, n, A, lda, i, j, Vp, Wp, (const double*)y,
                         (const double*)pq, (const double*)tau, S, next);
      launches += 3;
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
    // 4/3 n^3 flops; bytes: the product's reads of the trailing columns,
    // sum over i of (n - i - 1)^2 entries
    const double nn = (double)n;
    const double work = 4.0 / 3.0 * nn * nn * nn;
    const double bytes = 8.0 * (nn - 1.0) * nn * (2.0 * nn - 1.0) / 6.0;
    mrrr::prof_add(MRRR_K_TRIDIAG, launches, ms, work, bytes);
  }
  return 0;
}

}  // extern "C"
