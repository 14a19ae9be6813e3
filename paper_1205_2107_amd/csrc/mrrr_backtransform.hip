// Stage 5 back-transformation Y = Q Z on FP64 matrix cores
// (v_mfma_f64_16x16x4f64), gfx950.
//
// After a lower tridiagonal reduction T = Q^T M Q (Stage 3, arXiv:1205.2107
// Sec. 1.2), the eigenvectors of M are Y = Q Z for the tridiagonal
// eigenvectors Z (Sec. 1.2, stage 5).  Q = H_0 H_1 ... H_{n-2} with
// H_i = I - tau_i v_i v_i^T, v_i[:i+1] = 0, v_i[i+1] = 1, v_i[i+2:] stored in
// V[i+2:, i] (column-major, leading dimension ldv).
//
// Blocked form (compact WY): reflectors j0 .. j0+nb-1 form
//   H_j0 ... H_{j0+nb-1} = I - V_b T_b V_b^T,
// T_b upper triangular with T_ii = tau_i and
//   T[0:i, i] = -tau_i T[0:i, 0:i] (V_b[:, 0:i]^T v_i).
// Q Z applies the blocks last to first; per block
//   W = T_b (V_b^T Z)          (k_bt_wpart: partial products over chunks of
//                               the block's rows; k_bt_wsum: their sum, times T_b)
//   Z <- Z - V_b W             (k_bt_update: a rank-nb update)
// on rows j0+1 .. n-1 of Z.  The T factors of all blocks come first
// (k_bt_tfactor: the Gram matrix V_b^T V_b on matrix cores, then the
// triangular recurrence).  The unit and zero entries of v_i are formed on the
// fly, so V's entries on and above the first subdiagonal are never read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "mrrr.h"
#include "mrrr_prof.h"

namespace mrrr_bt {

constexpr int NB = 64;   // reflectors per block = tile size
constexpr int TK = 16;   // reduction step staged in LDS
constexpr int NT = 256;  // threads per workgroup (4 waves, 2 x 2 quadrants of 32 x 32)
constexpr int kXcds = 8;             // XCDs of the MI355X (workgroups are dispatched round-robin over them)
constexpr int kUpdCols = 4;          // column tiles per workgroup of the update
constexpr int64_t kMinChunk = 1024;  // rows per chunk of the partial products, at least
constexpr int64_t kMaxChunks = 16;   // chunks per block, at most

typedef double v4d __attribute__((ext_vector_type(4)));

// One 64 x 64 x 16 step: A[i][r], B[j][r] in LDS; each wave accumulates a
// 32 x 32 quadrant as 2 x 2 MFMA 16x16 blocks over four K-chunks of 4.
// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[l / 16 + 4 v][l % 16], v = 0..3.
__device__ inline void mma_step(const double (*As)[TK + 1], const double (*Bs)[TK + 1], v4d acc[2][2], int wr,
                                int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kc = 0; kc < TK / 4; ++kc) {
    double a[2], b[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) a[m] = As[wr * 32 + m * 16 + li][kc * 4 + lk];
#pragma unroll
    for (int q = 0; q < 2; ++q) b[q] = Bs[wc * 32 + q * 16 + li][kc * 4 + lk];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
  }
}

// entry (r, c) of the explicit reflector matrix: v_c[r]
__device__ __forceinline__ double vref(const double* __restrict__ V, int64_t ldv, int64_t r, int64_t c) {
  return (r == c + 1) ? 1.0 : ((r > c + 1) ? V[c * ldv + r] : 0.0);
}

// the accumulator's (row, column) inside the 64 x 64 tile for lane, block (m, q), element v
__device__ __forceinline__ int acc_row(int wr, int m, int lane, int v) { return wr * 32 + m * 16 + (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_col(int wc, int q, int lane) { return wc * 32 + q * 16 + (lane & 15); }

// T factor of every block (grid: one workgroup per block).  Tws[b] is 64 x 64
// row-major, zero outside the block's upper triangle.
__global__ void __launch_bounds__(NT) k_bt_tfactor(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ tau, double* __restrict__ Tws) {
  __shared__ double As[NB][TK + 1];
  __shared__ double G[NB][NB + 1];
  __shared__ double Ts[NB][NB + 1];
  const int b = blockIdx.x;
  const int64_t nref = n - 1;
  const int64_t j0 = (int64_t)b * NB;
  const int nbk = (int)std::min<int64_t>(NB, nref - j0);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // G = V_b^T V_b over rows j0 + 1 .. n - 1; thread t loads column t / 4, rows 4 (t % 4) .. +3
  const int lc = t >> 2, lr = (t & 3) * 4;
  for (int64_t r0 = j0 + 1; r0 < n; r0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + lr + u;
      As[lc][lr + u] = (r < n && lc < nbk) ? vref(V, ldv, r, j0 + lc) : 0.0;
    }
    __syncthreads();
    mma_step(As, As, acc, wr, wc, lane);
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) G[acc_row(wr, m, lane, v)][acc_col(wc, q, lane)] = acc[m][q][v];
  for (int e = t; e < NB * NB; e += NT) Ts[e / NB][e % NB] = 0.0;
  __syncthreads();
  // T[i][i] = tau_i; T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i], column by column
  for (int i = 0; i < nbk; ++i) {
    const double ti = tau[j0 + i];
    double s = 0.0;
    if (t < i)
      for (int k = t; k < i; ++k) s += Ts[t][k] * G[k][i];
    __syncthreads();
    if (t < i) Ts[t][i] = -ti * s;
    if (t == i) Ts[i][i] = ti;
    __syncthreads();
  }
  double* Tb = Tws + (int64_t)b * NB * NB;
  for (int e = t; e < NB * NB; e += NT) Tb[e] = Ts[e / NB][e % NB];
}

// Partial products P_s = Z[rows_s, c0 : c0 + 64]^T V_b[rows_s, :] over the
// s-th chunk of kc rows of block b (rows j0 + 1 + s kc ..), grid (column
// tiles, chunks).  The accumulator holds D[j][c] (Z column j, reflector c),
// so the 16 lanes of an MFMA row group write 16 consecutive reflectors.
// The next chunk's operands are fetched into registers while the matrix
// cores work on the current one.  P_s is stored as 64 x m (ld 64) at
// P + s 64 m.
__global__ void __launch_bounds__(NT) k_bt_wpart(int64_t n, int64_t m, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ Z, int64_t ldz, int b, int64_t kc,
                                                 double* __restrict__ P) {
  __shared__ double As[NB][TK + 1];  // Z^T: As[j][k] = Z[r0 + k, c0 + j]
  __shared__ double Bs[NB][TK + 1];  // V_b: Bs[c][k] = v_{j0 + c}[r0 + k]
  const int64_t j0 = (int64_t)b * NB;
  const int nbk = (int)std::min<int64_t>(NB, n - 1 - j0);
  const int64_t c0 = (int64_t)blockIdx.x * NB;
  const int64_t rb = j0 + 1 + (int64_t)blockIdx.y * kc;
  const int64_t re = std::min<int64_t>(n, rb + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[mm][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // thread t loads column / reflector t / 4, rows 4 (t % 4) .. +3 of the chunk
  const int lc = t >> 2, lr = (t & 3) * 4;
  const int64_t cz = c0 + lc;
  const bool zcol = cz < m, vcol = lc < nbk;
  double ra[4], rv[4];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + lr + u;
      ra[u] = (r < re && zcol) ? Z[cz * ldz + r] : 0.0;
      rv[u] = (r < re && vcol) ? vref(V, ldv, r, j0 + lc) : 0.0;
    }
  };
  fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[lc][lr + u] = ra[u];
      Bs[lc][lr + u] = rv[u];
    }
    __syncthreads();
    if (r0 + TK < re) fetch(r0 + TK);
    mma_step(As, Bs, acc, wr, wc, lane);
    __syncthreads();
  }
  double* Ps = P + (int64_t)blockIdx.y * NB * m;
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = c0 + acc_row(wr, mm, lane, v);
        const int c = acc_col(wc, q, lane);
        if (j < m) Ps[j * NB + c] = acc[mm][q][v];
      }
}

// W[:, c0 : c0 + 64] = T_b (sum_s P_s) for block b (chunks summed in order);
// W is 64 x m column-major (ld 64).  Thread t forms column t / 4, rows
// 16 (t % 4) .. +15 (T upper triangular, read from global memory where it is
// cached for every workgroup of the block).
__global__ void __launch_bounds__(NT) k_bt_wsum(int64_t m, const double* __restrict__ Tws, int b, int nchunk,
                                                const double* __restrict__ P, double* __restrict__ W) {
  __shared__ double Xs[NB][NB + 1];  // Xs[k][j] = sum_s P_s[k, c0 + j]
  const int64_t c0 = (int64_t)blockIdx.x * NB;
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += NT) {
    const int k = e % NB, j = e / NB;
    const int64_t cz = c0 + j;
    double x = 0.0;
    if (cz < m)
      for (int s = 0; s < nchunk; ++s) x += P[(int64_t)s * NB * m + cz * NB + k];
    Xs[k][j] = x;
  }
  __syncthreads();
  const double* Tb = Tws + (int64_t)b * NB * NB;
  const int oc = t >> 2, or0 = (t & 3) * 16;
  const int64_t cz = c0 + oc;
  for (int i = or0; i < or0 + 16; ++i) {
    double x = 0.0;
    for (int k = i; k < NB; ++k) x += Tb[i * NB + k] * Xs[k][oc];
    if (cz < m) W[cz * NB + i] = x;
  }
}

// One 64 x 64 x 64 product from operands held whole in LDS in k-major
// layout (A[k][i], B[k][j], no padding: the 16 lanes of an operand read touch
// consecutive entries): each wave accumulates its 32 x 32 quadrant.
__device__ inline void mma_tile64(const double (*At)[NB], const double (*Bt)[NB], v4d acc[2][2], int wr, int wc,
                                  int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kc = 0; kc < NB / 4; ++kc) {
    double a[2], bb[2];
#pragma unroll
    for (int mm = 0; mm < 2; ++mm) a[mm] = At[kc * 4 + lk][wr * 32 + mm * 16 + li];
#pragma unroll
    for (int q = 0; q < 2; ++q) bb[q] = Bt[kc * 4 + lk][wc * 32 + q * 16 + li];
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[mm][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mm], bb[q], acc[mm][q], 0, 0, 0);
  }
}

// Z[i0 .., :] -= V_b W for a tile of 64 rows and a group of kUpdCols column
// tiles of 64.  The tile's V_b rows are staged in LDS once; per column tile
// the W block is staged and the Z entries this lane updates are fetched
// before the products (the next tile's W and Z are fetched into registers
// while the matrix cores work).  The accumulator holds D[j][i] (Z column j,
// row i), so the 16 lanes of an MFMA row group update 16 consecutive rows of
// one column.  Workgroup L runs on XCD L mod 8 (round-robin dispatch); each
// XCD takes its own contiguous share of the column groups, so the slice of W
// its tiles read stays in that XCD's L2.  ncx column groups per XCD.
__global__ void __launch_bounds__(NT) k_bt_update(int64_t n, int64_t m, const double* __restrict__ V, int64_t ldv,
                                                  double* __restrict__ Z, int64_t ldz, int b,
                                                  const double* __restrict__ W, int ncx, int ngroups) {
  __shared__ double Vt[NB][NB];  // Vt[k][i] = v_{j0 + k}[i0 + i]
  __shared__ double Wt[NB][NB];  // Wt[k][j] = W[k, c0 + j]
  const int xcd = (int)(blockIdx.x % kXcds), local = (int)(blockIdx.x / kXcds);
  const int grp = xcd * ncx + local % ncx, rtile = local / ncx;
  if (grp >= ngroups) return;
  const int64_t j0 = (int64_t)b * NB;
  const int nbk = (int)std::min<int64_t>(NB, n - 1 - j0);
  const int64_t i0 = j0 + 1 + (int64_t)rtile * NB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // V_b rows: thread t stages reflector t / 4, rows 16 (t % 4) .. +15
  {
    const int k = t >> 2, ib = (t & 3) * 16;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t r = i0 + ib + u;
      Vt[k][ib + u] = (r < n && k < nbk) ? vref(V, ldv, r, j0 + k) : 0.0;
    }
  }
  // W block: thread t reads column t / 4, reflectors 16 (t % 4) .. +15
  const int wj = t >> 2, wk = (t & 3) * 16;
  double wr_[16], zr[2][2][4];
  const int64_t cbeg = (int64_t)grp * kUpdCols * NB;
  auto fetch = [&](int64_t c0) {
    const int64_t cz = c0 + wj;
#pragma unroll
    for (int u = 0; u < 16; ++u) wr_[u] = (cz < m && wk + u < nbk) ? W[cz * NB + wk + u] : 0.0;
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = c0 + acc_row(wr, mm, lane, v);
          const int64_t r = i0 + acc_col(wc, q, lane);
          zr[mm][q][v] = (r < n && j < m) ? Z[j * ldz + r] : 0.0;
        }
  };
  fetch(cbeg);
  for (int g = 0; g < kUpdCols; ++g) {
    const int64_t c0 = cbeg + (int64_t)g * NB;
    if (c0 >= m) break;
#pragma unroll
    for (int u = 0; u < 16; ++u) Wt[wk + u][wj] = wr_[u];
    double zc[2][2][4];
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) zc[mm][q][v] = zr[mm][q][v];
    __syncthreads();
    if (g + 1 < kUpdCols && c0 + NB < m) fetch(c0 + NB);
    v4d acc[2][2];
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[mm][q] = v4d{0.0, 0.0, 0.0, 0.0};
    mma_tile64(Wt, Vt, acc, wr, wc, lane);
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = c0 + acc_row(wr, mm, lane, v);
          const int64_t r = i0 + acc_col(wc, q, lane);
          if (r < n && j < m) Z[j * ldz + r] = zc[mm][q][v] - acc[mm][q][v];
        }
    __syncthreads();
  }
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
    mrrr::set_last_error("hipMalloc failed for the back-transformation workspace");
    return MRRR_ERR_CAPACITY;
  }
  g_ws_bytes = nb;
  g_ws_dev = dev;
  return 0;
}

}  // namespace mrrr_bt

using namespace mrrr_bt;

extern "C" {

int mrrr_backtransform(int64_t n, int64_t m, const double* V, int64_t ldv, const double* tau, double* Z,
                       int64_t ldz, void* stream) {
  if (n < 0 || n > (int64_t)1 << 31) return -1;
  if (m < 0 || m > (int64_t)1 << 31) return -2;
  if (n > 2 && !V) return -3;
  if (ldv < std::max<int64_t>(1, n)) return -4;
  if (n > 1 && !tau) return -5;
  if (n > 0 && m > 0 && !Z) return -6;
  if (ldz < std::max<int64_t>(1, n)) return -7;
  if (n <= 1 || m == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t nref = n - 1;
  const int64_t nblk = (nref + NB - 1) / NB;
  // rows per chunk of the partial products: at least kMinChunk, at most
  // kMaxChunks chunks per block, a multiple of TK
  const int64_t kc = std::max<int64_t>(kMinChunk, ((nref + kMaxChunks - 1) / kMaxChunks + TK - 1) / TK * TK);
  const int64_t maxch = (nref + kc - 1) / kc;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t tbytes = al(sizeof(double) * (size_t)(nblk * NB * NB));
  const size_t wbytes = al(sizeof(double) * (size_t)(NB * m));
  const size_t pbytes = sizeof(double) * (size_t)(maxch * NB * m);
  int rc = grow(tbytes + wbytes + pbytes);
  if (rc) return rc;
  double* Tws = (double*)g_ws;
  double* W = (double*)((char*)g_ws + tbytes);
  double* P = (double*)((char*)g_ws + tbytes + wbytes);
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_BACKTRANSFORM);
  hipLaunchKernelGGL(k_bt_tfactor, dim3((unsigned)nblk), dim3(NT), 0, st, n, V, ldv, tau, Tws);
  const unsigned ct = (unsigned)((m + NB - 1) / NB);
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t rows = n - 1 - b * NB;
    const int64_t nch = (rows + kc - 1) / kc;
    hipLaunchKernelGGL(k_bt_wpart, dim3(ct, (unsigned)nch), dim3(NT), 0, st, n, m, V, ldv, (const double*)Z, ldz,
                       (int)b, kc, P);
    hipLaunchKernelGGL(k_bt_wsum, dim3(ct), dim3(NT), 0, st, m, (const double*)Tws, (int)b, (int)nch,
                       (const double*)P, W);
    const int64_t rt = (rows + NB - 1) / NB;
    const int ngroups = (int)((ct + kUpdCols - 1) / kUpdCols);
    const int ncx = (ngroups + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(k_bt_update, dim3((unsigned)(kXcds * ncx * rt)), dim3(NT), 0, st, n, m, V, ldv, Z, ldz, (int)b,
                       (const double*)W, ncx, ngroups);
  }
  prof.end();
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    mrrr::set_last_error((std::string("back-transformation kernels failed: ") + hipGetErrorString(e)).c_str());
    return MRRR_ERR_HIP;
  }
  if (prof.on) {
    double ms;
    int64_t l;
    prof.total(MRRR_K_BACKTRANSFORM, &ms, &l);
    // two products of 2 K nb m flops per block over its K = n - 1 - j0 rows
    double work = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
      const double nbk = (double)std::min<int64_t>(NB, nref - b * NB);
      work += 4.0 * (double)(n - 1 - b * NB) * nbk * (double)m;
    }
    mrrr::prof_add(MRRR_K_BACKTRANSFORM, l, ms, work, 0.0);
  }
  return 0;
}

}  // extern "C"
