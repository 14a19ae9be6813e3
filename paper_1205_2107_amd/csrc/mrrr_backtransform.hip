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

// Partial products P_s = Z[rows_s, c0 : c0 + 64]^T [V_b .. V_{b+kH-1}][rows_s, :]
// over the s-th chunk of kc rows from the first block's first row (rows
// j0 + 1 + s kc ..), grid (column tiles, chunks): kH = 1 one block of 64
// reflectors, kH = 2 two adjacent blocks read with one pass over Z.  The
// accumulator holds D[j][c] (Z column j, reflector c), so the 16 lanes of an
// MFMA row group write 16 consecutive reflectors.  The next chunk's operands
// are fetched into registers while the matrix cores work on the current one.
// P_s is stored as 64 kH x m (ld 64 kH) at P + s 64 kH m.
template <int kH>
__global__ void __launch_bounds__(NT) k_bt_wpart(int64_t n, int64_t m, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ Z, int64_t ldz, int b, int64_t kc,
                                                 double* __restrict__ P) {
  __shared__ double As[NB][TK + 1];       // Z^T: As[j][k] = Z[r0 + k, c0 + j]
  __shared__ double Bs[kH][NB][TK + 1];   // V: Bs[h][c][k] = v_{j0 + 64 h + c}[r0 + k]
  const int64_t j0 = (int64_t)b * NB;
  const int64_t c0 = (int64_t)blockIdx.x * NB;
  const int64_t rb = j0 + 1 + (int64_t)blockIdx.y * kc;
  const int64_t re = std::min<int64_t>(n, rb + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[kH][2][2];
#pragma unroll
  for (int h = 0; h < kH; ++h)
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[h][mm][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // thread t loads column / reflector t / 4, rows 4 (t % 4) .. +3 of the chunk
  const int lc = t >> 2, lr = (t & 3) * 4;
  const int64_t cz = c0 + lc;
  const bool zcol = cz < m;
  bool vcol[kH];
#pragma unroll
  for (int h = 0; h < kH; ++h) vcol[h] = j0 + NB * h + lc < n - 1;
  double ra[4], rv[kH][4];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + lr + u;
      ra[u] = (r < re && zcol) ? Z[cz * ldz + r] : 0.0;
#pragma unroll
      for (int h = 0; h < kH; ++h) rv[h][u] = (r < re && vcol[h]) ? vref(V, ldv, r, j0 + NB * h + lc) : 0.0;
    }
  };
  fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[lc][lr + u] = ra[u];
#pragma unroll
      for (int h = 0; h < kH; ++h) Bs[h][lc][lr + u] = rv[h][u];
    }
    __syncthreads();
    if (r0 + TK < re) fetch(r0 + TK);
#pragma unroll
    for (int h = 0; h < kH; ++h) mma_step(As, Bs[h], acc[h], wr, wc, lane);
    __syncthreads();
  }
  double* Ps = P + (int64_t)blockIdx.y * kH * NB * m;
#pragma unroll
  for (int h = 0; h < kH; ++h)
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = c0 + acc_row(wr, mm, lane, v);
          const int c = acc_col(wc, q, lane);
          if (j < m) Ps[j * (kH * NB) + NB * h + c] = acc[h][mm][q][v];
        }
}

// W[:, c0 : c0 + 64] = T_b (sum_s P_s) for block b (chunks summed in order);
// W is 64 x m column-major (ld 64).  Thread t forms column t / 4, rows
// 16 (t % 4) .. +15 (T upper triangular, read from global memory where it is
// cached for every workgroup of the block).
__global__ void __launch_bounds__(NT) k_bt_wsum(int64_t m, const double* __restrict__ Tws, int b, int nchunk,
                                                const double* __restrict__ P, double* __restrict__ W, int64_t ldw) {
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
    if (cz < m) W[cz * ldw + i] = x;
  }
}

// Two adjacent blocks b, b + 1 applied as one block of 128 reflectors:
// I - [V0 V1] T [V0 V1]^T with T = [[T0, -T0 C T1], [0, T1]], C = V0^T V1, so
// W = T X for X = [V0 V1]^T Z is W1 = T1 X1 and W0 = T0 (X0 - C W1).
// X = the sum of the chunks of the two-block partial products (P_s 128 x m,
// ld 128); W is 128 x m (ld 128).  32 columns per workgroup, eight threads a
// column.
__global__ void __launch_bounds__(NT) k_bt_wsum2(int64_t m, const double* __restrict__ Tws, int b, int nchunk,
                                                 const double* __restrict__ P, const double* __restrict__ Cws,
                                                 double* __restrict__ W) {
  __shared__ double Xs[2 * NB][33];  // Xs[k][j] = sum_s P_s[k, c0 + j]; rows 0..63 later hold X0 - C W1
  __shared__ double W1s[NB][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32;
  const int t = threadIdx.x;
  for (int e = t; e < 2 * NB * 32; e += NT) {
    const int k = e % (2 * NB), j = e / (2 * NB);
    const int64_t cz = c0 + j;
    double x = 0.0;
    if (cz < m)
      for (int s = 0; s < nchunk; ++s) x += P[(int64_t)s * 2 * NB * m + cz * 2 * NB + k];
    Xs[k][j] = x;
  }
  __syncthreads();
  const double* T0 = Tws + (int64_t)b * NB * NB;
  const double* T1 = Tws + (int64_t)(b + 1) * NB * NB;
  const double* C = Cws + (int64_t)b * NB * NB;
  // eight threads a column, each eight rows of every step
  const int oc = t >> 3, r0 = (t & 7) * 8;
  const int64_t cz = c0 + oc;
  for (int i = r0; i < r0 + 8; ++i) {  // W1 = T1 X1
    double x = 0.0;
    for (int k = i; k < NB; ++k) x += T1[i * NB + k] * Xs[NB + k][oc];
    W1s[i][oc] = x;
    if (cz < m) W[cz * 2 * NB + NB + i] = x;
  }
  __syncthreads();
  for (int i = r0; i < r0 + 8; ++i) {  // X0 - C W1
    double x = Xs[i][oc];
    for (int k = 0; k < NB; ++k) x -= C[i * NB + k] * W1s[k][oc];
    Xs[i][oc] = x;
  }
  __syncthreads();
  for (int i = r0; i < r0 + 8; ++i) {  // W0 = T0 (X0 - C W1)
    double x = 0.0;
    for (int k = i; k < NB; ++k) x += T0[i * NB + k] * Xs[k][oc];
    if (cz < m) W[cz * 2 * NB + i] = x;
  }
}

// C_b = V_b^T V_{b+1} (64 x 64 row-major, rows of V_{b+1}'s nonzero part) for
// every adjacent pair of blocks, one workgroup per pair
__global__ void __launch_bounds__(NT) k_bt_cross(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                 double* __restrict__ Cws) {
  __shared__ double As[NB][TK + 1];
  __shared__ double Bs[NB][TK + 1];
  const int b = blockIdx.x;
  const int64_t nref = n - 1;
  const int64_t j0 = (int64_t)b * NB, j1 = j0 + NB;
  const int nb0 = (int)std::min<int64_t>(NB, nref - j0), nb1 = (int)std::min<int64_t>(NB, nref - j1);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[mm][q] = v4d{0.0, 0.0, 0.0, 0.0};
  const int lc = t >> 2, lr = (t & 3) * 4;
  for (int64_t r0 = j1 + 1; r0 < n; r0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + lr + u;
      As[lc][lr + u] = (r < n && lc < nb0) ? vref(V, ldv, r, j0 + lc) : 0.0;
      Bs[lc][lr + u] = (r < n && lc < nb1) ? vref(V, ldv, r, j1 + lc) : 0.0;
    }
    __syncthreads();
    mma_step(As, Bs, acc, wr, wc, lane);
    __syncthreads();
  }
  double* Cb = Cws + (int64_t)b * NB * NB;
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cb[acc_row(wr, mm, lane, v) * NB + acc_col(wc, q, lane)] = acc[mm][q][v];
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
// its tiles read stays in that XCD's L2.  ncx column groups per XCD; rows at
// or beyond rend are left alone; W has leading dimension ldw.
__global__ void __launch_bounds__(NT) k_bt_update(int64_t n, int64_t m, const double* __restrict__ V, int64_t ldv,
                                                  double* __restrict__ Z, int64_t ldz, int b,
                                                  const double* __restrict__ W, int64_t ldw, int64_t rend, int ncx,
                                                  int ngroups) {
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
      Vt[k][ib + u] = (r < rend && k < nbk) ? vref(V, ldv, r, j0 + k) : 0.0;
    }
  }
  // W block: thread t reads column t / 4, reflectors 16 (t % 4) .. +15
  const int wj = t >> 2, wk = (t & 3) * 16;
  double wr_[16], zr[2][2][4];
  const int64_t cbeg = (int64_t)grp * kUpdCols * NB;
  auto fetch = [&](int64_t c0) {
    const int64_t cz = c0 + wj;
#pragma unroll
    for (int u = 0; u < 16; ++u) wr_[u] = (cz < m && wk + u < nbk) ? W[cz * ldw + wk + u] : 0.0;
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = c0 + acc_row(wr, mm, lane, v);
          const int64_t r = i0 + acc_col(wc, q, lane);
          zr[mm][q][v] = (r < rend && j < m) ? Z[j * ldz + r] : 0.0;
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
          if (r < rend && j < m) Z[j * ldz + r] = zc[mm][q][v] - acc[mm][q][v];
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

// Z[r, :] -= V[r, j0 : j0 + 128] W (W 128 x m, ld 128) for the rows r >= rb
// where both blocks' reflectors are stored entries of V (no unit or zero
// entries formed), one 64 x 64 tile of Z per workgroup (grid x column tiles,
// y row tiles); K = 128 in steps of TK with the next step's operands fetched
// into registers while the matrix cores work, the lane's Z entries fetched
// before the products; 16 lanes of an MFMA row group update 16 consecutive
// rows of one column.
__global__ void __launch_bounds__(NT) k_bt_rank128(int64_t n, int64_t m, const double* __restrict__ V, int64_t ldv,
                                                   int64_t j0, int64_t rb, const double* __restrict__ W,
                                                   double* __restrict__ Z, int64_t ldz) {
  __shared__ double Ps[NB][TK + 1];  // Ps[i][k] = V[rb + I 64 + i, j0 + k0 + k]
  __shared__ double Qs[NB][TK + 1];  // Qs[j][k] = W[k0 + k, c0 + j]
  const int64_t i0 = rb + (int64_t)blockIdx.y * NB, c0 = (int64_t)blockIdx.x * NB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[mm][q] = v4d{0.0, 0.0, 0.0, 0.0};
  double zc[2][2][4];
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = c0 + acc_row(wr, mm, lane, v);
        const int64_t r = i0 + acc_col(wc, q, lane);
        zc[mm][q][v] = (r < n && j < m) ? Z[j * ldz + r] : 0.0;
      }
  // loaders: V rows contiguous over threads; W reflectors contiguous over threads
  double rp[4], rq[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ia = t & 63, ka = (t >> 6) * 4 + u;
      const int kb = t & 15, jb = (t >> 4) + 16 * u;
      const int64_t r = i0 + ia, c = c0 + jb;
      rp[u] = r < n ? V[(j0 + k0 + ka) * ldv + r] : 0.0;
      rq[u] = c < m ? W[c * 2 * NB + k0 + kb] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < 2 * NB; k0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Ps[t & 63][(t >> 6) * 4 + u] = rp[u];
      Qs[(t >> 4) + 16 * u][t & 15] = rq[u];
    }
    __syncthreads();
    if (k0 + TK < 2 * NB) fetch(k0 + TK);
    mma_step(Qs, Ps, acc, wr, wc, lane);  // D[j][i]: Z column j, row i
    __syncthreads();
  }
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
}

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
  const size_t cbytes = al(sizeof(double) * (size_t)(std::max<int64_t>(nblk - 1, 1) * NB * NB));
  const size_t wbytes = al(sizeof(double) * (size_t)(2 * NB * m));
  const size_t pbytes = sizeof(double) * (size_t)(maxch * 2 * NB * m);
  int rc = grow(tbytes + cbytes + wbytes + pbytes);
  if (rc) return rc;
  double* Tws = (double*)g_ws;
  double* Cws = (double*)((char*)g_ws + tbytes);
  double* W = (double*)((char*)g_ws + tbytes + cbytes);
  double* P = (double*)((char*)g_ws + tbytes + cbytes + wbytes);
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_BACKTRANSFORM);
  hipLaunchKernelGGL(k_bt_tfactor, dim3((unsigned)nblk), dim3(NT), 0, st, n, V, ldv, tau, Tws);
  if (nblk > 1) hipLaunchKernelGGL(k_bt_cross, dim3((unsigned)(nblk - 1)), dim3(NT), 0, st, n, V, ldv, Cws);
  const unsigned ct = (unsigned)((m + NB - 1) / NB);
  const int ngroups = (int)((ct + kUpdCols - 1) / kUpdCols);
  const int ncx = (ngroups + kXcds - 1) / kXcds;
  // the update of block b over rows j0 + 1 .. rend - 1 (W with leading dimension ldw)
  auto update = [&](int64_t b, const double* Wb, int64_t ldw, int64_t rend) {
    const int64_t rows = rend - (b * NB + 1);
    if (rows <= 0) return;
    const int64_t rt = (rows + NB - 1) / NB;
    hipLaunchKernelGGL(k_bt_update, dim3((unsigned)(kXcds * ncx * rt)), dim3(NT), 0, st, n, m, V, ldv, Z, ldz, (int)b,
                       Wb, ldw, rend, ncx, ngroups);
  };
  // one block of 64 reflectors: three passes over its rows of Z
  auto single = [&](int64_t b) {
    const int64_t rows = n - 1 - b * NB;
    const int64_t nch = (rows + kc - 1) / kc;
    hipLaunchKernelGGL(k_bt_wpart<1>, dim3(ct, (unsigned)nch), dim3(NT), 0, st, n, m, V, ldv, (const double*)Z, ldz,
                       (int)b, kc, P);
    hipLaunchKernelGGL(k_bt_wsum, dim3(ct), dim3(NT), 0, st, m, (const double*)Tws, (int)b, (int)nch,
                       (const double*)P, W, (int64_t)NB);
    update(b, W, NB, n);
  };
  // blocks b, b + 1 (both full) as one block of 128: the same three passes
  // for both; the first 128 rows (unit and zero entries of the reflectors)
  // by the one-block update, the rows below by one rank-128 update
  auto pair = [&](int64_t b) {
    const int64_t j0 = b * NB;
    const int64_t rows = n - 1 - j0;
    const int64_t nch = (rows + kc - 1) / kc;
    hipLaunchKernelGGL(k_bt_wpart<2>, dim3(ct, (unsigned)nch), dim3(NT), 0, st, n, m, V, ldv, (const double*)Z, ldz,
                       (int)b, kc, P);
    hipLaunchKernelGGL(k_bt_wsum2, dim3((unsigned)((m + 31) / 32)), dim3(NT), 0, st, m, (const double*)Tws, (int)b,
                       (int)nch, (const double*)P, (const double*)Cws, W);
    const int64_t rtop = std::min<int64_t>(n, j0 + 1 + 2 * NB);
    update(b, W, 2 * NB, rtop);
    update(b + 1, W + NB, 2 * NB, rtop);
    if (rtop < n)
      hipLaunchKernelGGL(k_bt_rank128, dim3(ct, (unsigned)((n - rtop + NB - 1) / NB)), dim3(NT), 0, st, n, m, V, ldv,
                         j0, rtop, (const double*)W, Z, ldz);
  };
  // last block first; pairs of full blocks, a ragged last block and an odd
  // first block alone
  int64_t b = nblk - 1;
  if (nref - b * NB < NB) single(b--);
  for (; b >= 1; b -= 2) pair(b - 1);
  if (b == 0) single(0);
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
