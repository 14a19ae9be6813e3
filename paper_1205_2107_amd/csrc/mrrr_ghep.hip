// Stages 1, 2 and 6 of the generalized eigenproblem A x = lambda B x
// (arXiv:1205.2107 Sec. 1.2, stage list), gfx950, FP64:
//   Cholesky factorization   B = L L^T                      (mrrr_cholesky)
//   reduction to standard    M = L^{-1} A L^{-T}             (mrrr_sygst)
//   second back-transform    X = L^{-T} Y                    (mrrr_trsm_lt)
// The stages in between (reduction to tridiagonal form, the tridiagonal
// eigensolver, the first back-transformation) are mrrr_tridiagonalize,
// mrrr_step and mrrr_backtransform.
//
// All three are blocked in 64 x 64 tiles: a triangular solve with one
// diagonal block of L, one RHS vector per lane, the block staged in LDS
// (k_trsm_tile), and updates of everything below (or above) it on FP64
// matrix cores (k_gemm_sub; the triangular solves and the Cholesky
// factorization work in panels of four tiles, so the large updates are of
// rank 256).  The Cholesky factorization adds the factorization of its
// diagonal blocks (k_chol_diag, one wavefront).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "mrrr.h"
#include "mrrr_prof.h"

namespace mrrr_gh {

constexpr int NB = 64;  // tile order
constexpr int TK = 16;  // reduction step of the updates staged in LDS
constexpr int NT = 256; // threads per workgroup of the updates
constexpr int kPanel = 4; // diagonal blocks per step of the triangular solves

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Cholesky factorization of one diagonal block (kb <= 64 rows) in place, one
// wavefront, lane = row: column j takes l_jj = sqrt(a_jj), l_ij = a_ij / l_jj
// and updates the columns to its right by the rank-one term.  A pivot that is
// not positive (or not finite) writes its global column (1-based) to *fail
// and leaves the block as it is.  Skips when *fail is already set.
__global__ void __launch_bounds__(64) k_chol_diag(double* __restrict__ B, int64_t ldb, int kb, int64_t k0,
                                                  int* __restrict__ fail) {
  __shared__ double T[NB][NB + 1];  // T[c][r] = block entry (r, c)
  __shared__ int s_bad;
  if (*fail) return;
  const int lane = threadIdx.x;
  for (int c = 0; c < kb; ++c) T[c][lane] = (lane < kb && lane >= c) ? B[(int64_t)c * ldb + lane] : 0.0;
  if (lane == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    const double piv = T[j][j];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (lane == 0) s_bad = j + 1;
      break;
    }
    const double ljj = sqrt(piv);
    const double lij = (lane > j && lane < kb) ? T[j][lane] / ljj : 0.0;
    __syncthreads();
    if (lane == j) T[j][j] = ljj;
    if (lane > j && lane < kb) T[j][lane] = lij;
    __syncthreads();
    // trailing columns c > j: a_rc -= l_rj l_cj (rows r >= c)
    for (int c = j + 1; c < kb; ++c) {
      const double lcj = T[j][c];
      if (lane >= c && lane < kb) T[c][lane] = fma(-lij, lcj, T[c][lane]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_bad) {
    if (lane == 0) atomicCAS(fail, 0, (int)(k0 + s_bad));
    return;
  }
  for (int c = 0; c < kb; ++c)
    if (lane >= c && lane < kb) B[(int64_t)c * ldb + lane] = T[c][lane];
}

// Triangular solves with the diagonal block Lkk (order kb <= 64, lower,
// leading dimension ldl), one right-hand side per lane, 64 per workgroup:
//   kRows = false: the RHS are the columns of the kb-row block R (columns
//                  blockIdx.x * 64 .. of nv, leading dimension ldr), lane =
//                  column;
//   kRows = true:  the RHS are the rows of the nv x kb block R (rows
//                  blockIdx.x * 64 ..), lane = row.
//   kTrans = false: x <- Lkk^{-1} x (forward); true: x <- Lkk^{-T} x (back).
// The tile is read and written coalesced through LDS; each lane's vector is
// solved in registers.  Skips when *fail is set.
template <bool kRows, bool kTrans>
__global__ void __launch_bounds__(64) k_trsm_tile(const double* __restrict__ Lkk, int64_t ldl, int kb,
                                                  double* __restrict__ R, int64_t ldr, int64_t nv,
                                                  const int* __restrict__ fail) {
  __shared__ double Ls[NB][NB + 1];  // Ls[c][r] = Lkk(r, c)
  __shared__ double S[NB][NB + 1];   // S[q][e] = element e of vector q
  if (fail && *fail) return;
  const int lane = threadIdx.x;
  const int64_t q0 = (int64_t)blockIdx.x * NB;
  for (int c = 0; c < NB; ++c)
    Ls[c][lane] = (c < kb && lane < kb) ? Lkk[(int64_t)c * ldl + lane] : (lane == c ? 1.0 : 0.0);
  if (kRows) {
    // element e = column of R, vector q = row: lanes read consecutive rows
    const int64_t r = q0 + lane;
    for (int e = 0; e < NB; ++e) S[lane][e] = (r < nv && e < kb) ? R[(int64_t)e * ldr + r] : 0.0;
  } else {
    // element e = row of R, vector q = column: lanes read consecutive rows of one column
    for (int q = 0; q < NB; ++q) {
      const int64_t c = q0 + q;
      S[q][lane] = (c < nv && lane < kb) ? R[c * ldr + lane] : 0.0;
    }
  }
  __syncthreads();
  double x[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) x[e] = S[lane][e];
  if (!kTrans) {
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      double acc = x[r];
#pragma unroll
      for (int c = 0; c < r; ++c) acc = fma(-Ls[c][r], x[c], acc);
      x[r] = acc / Ls[r][r];
    }
  } else {
#pragma unroll
    for (int r = NB - 1; r >= 0; --r) {
      double acc = x[r];
#pragma unroll
      for (int c = r + 1; c < NB; ++c) acc = fma(-Ls[r][c], x[c], acc);
      x[r] = acc / Ls[r][r];
    }
  }
#pragma unroll
  for (int e = 0; e < NB; ++e) S[lane][e] = x[e];
  __syncthreads();
  if (kRows) {
    const int64_t r = q0 + lane;
    for (int e = 0; e < kb; ++e)
      if (r < nv) R[(int64_t)e * ldr + r] = S[lane][e];
  } else {
    for (int q = 0; q < NB; ++q) {
      const int64_t c = q0 + q;
      if (c < nv && lane < kb) R[c * ldr + lane] = S[q][lane];
    }
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

// lower 64 x 64 tile number tl -> (I, J), I >= J
__device__ __forceinline__ void lower_tile(int64_t tl, int64_t* I, int64_t* J) {
  int64_t a = (int64_t)((sqrt(8.0 * (double)tl + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > tl) --a;
  while ((a + 1) * (a + 2) / 2 <= tl) ++a;
  *I = a;
  *J = tl - a * (a + 1) / 2;
}

// C (M x N, leading dimension ldc) -= op(A) op(B) with K = kk (in steps of 16):
//   op(A)[i][k] = kTA ? A[k + i lda] : A[i + k lda]
//   op(B)[k][j] = kTB ? B[j + k ldb] : B[k + j ldb]
// one 64 x 64 tile of C per workgroup (grid x = tiles over N, y = tiles over
// M), or with kLower (M = N) the lower tiles only (grid x = their number),
// the lower triangle of a diagonal tile only.  The next 16-step of both
// operands is fetched into registers while the matrix cores work.
template <bool kTA, bool kTB, bool kLower>
__global__ void __launch_bounds__(NT) k_gemm_sub(int64_t M, int64_t N, int kk, const double* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                 double* __restrict__ C, int64_t ldc, const int* __restrict__ fail) {
  __shared__ double Ps[NB][TK + 1];
  __shared__ double Qs[NB][TK + 1];
  if (fail && *fail) return;
  int64_t I, J;
  if (kLower) {
    lower_tile(blockIdx.x, &I, &J);
  } else {
    I = blockIdx.y;
    J = blockIdx.x;
  }
  const int64_t i0 = I * NB, j0 = J * NB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // loaders: the index that is contiguous in memory varies fastest over threads
  double ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int ia, ka, jb, kb_;
      if (kTA) {  // contiguous in k
        ka = t & 15;
        ia = (t >> 4) + 16 * u;
      } else {  // contiguous in i
        ia = t & 63;
        ka = (t >> 6) * 4 + u;
      }
      if (kTB) {  // contiguous in j
        jb = t & 63;
        kb_ = (t >> 6) * 4 + u;
      } else {  // contiguous in k
        kb_ = t & 15;
        jb = (t >> 4) + 16 * u;
      }
      const int64_t gi = i0 + ia, gj = j0 + jb;
      const int gka = k0 + ka, gkb = k0 + kb_;
      ra[u] = (gi < M && gka < kk) ? (kTA ? A[gka + gi * lda] : A[gi + (int64_t)gka * lda]) : 0.0;
      rb[u] = (gj < N && gkb < kk) ? (kTB ? B[gj + (int64_t)gkb * ldb] : B[gkb + gj * ldb]) : 0.0;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int ia, ka, jb, kb_;
      if (kTA) {
        ka = t & 15;
        ia = (t >> 4) + 16 * u;
      } else {
        ia = t & 63;
        ka = (t >> 6) * 4 + u;
      }
      if (kTB) {
        jb = t & 63;
        kb_ = (t >> 6) * 4 + u;
      } else {
        kb_ = t & 15;
        jb = (t >> 4) + 16 * u;
      }
      Ps[ia][ka] = ra[u];
      Qs[jb][kb_] = rb[u];
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < kk; k0 += TK) {
    stage();
    __syncthreads();
    if (k0 + TK < kk) fetch(k0 + TK);
    mma_step(Qs, Ps, acc, wr, wc, lane);  // D[b][a]: the 16 lanes of a row group hold 16 consecutive rows of C
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = acc_row(wr, m, lane, v), a = acc_col(wc, q, lane);
        const int64_t gi = i0 + a, gj = j0 + b;
        if (gi < M && gj < N && (!kLower || I != J || a >= b)) {
          double* c = C + gi + gj * ldc;
          *c = *c - acc[m][q][v];
        }
      }
}

// X (n x n, full) from the lower triangle of A
__global__ void __launch_bounds__(NT) k_sym_full(int64_t n, const double* __restrict__ A, int64_t lda,
                                                 double* __restrict__ X, int64_t ldx) {
  __shared__ double T[NB][NB + 1];
  const int64_t I = blockIdx.y, J = blockIdx.x;  // tile of X
  const int t = threadIdx.x;
  // source tile: (I, J) if I >= J else the transpose of (J, I)
  const bool low = I >= J;
  const int64_t si = low ? I : J, sj = low ? J : I;
  for (int e = t; e < NB * NB; e += NT) {
    const int a = e & 63, b = e >> 6;
    const int64_t r = si * NB + a, c = sj * NB + b;
    T[b][a] = (r < n && c < n) ? A[r + c * lda] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += NT) {
    const int a = e & 63, b = e >> 6;  // entry (a, b) of tile (I, J) of X
    const int64_t r = I * NB + a, c = J * NB + b;
    if (r >= n || c >= n) continue;
    double x;
    if (low)
      x = (I != J || a >= b) ? T[b][a] : T[a][b];
    else
      x = T[a][b];
    X[r + c * ldx] = x;
  }
}

// Y = X^T (n x n)
__global__ void __launch_bounds__(NT) k_transpose(int64_t n, const double* __restrict__ X, int64_t ldx,
                                                  double* __restrict__ Y, int64_t ldy) {
  __shared__ double T[NB][NB + 1];
  const int64_t I = blockIdx.y, J = blockIdx.x;  // tile of Y
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += NT) {
    const int a = e & 63, b = e >> 6;  // X tile (J, I) entry (a, b)
    const int64_t r = J * NB + a, c = I * NB + b;
    T[b][a] = (r < n && c < n) ? X[r + c * ldx] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += NT) {
    const int a = e & 63, b = e >> 6;  // Y tile (I, J) entry (a, b) = X (J b, I a)
    const int64_t r = I * NB + a, c = J * NB + b;
    if (r < n && c < n) Y[r + c * ldy] = T[a][b];
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
    mrrr::set_last_error("hipMalloc failed for the generalized-problem workspace");
    return MRRR_ERR_CAPACITY;
  }
  g_ws_bytes = nb;
  g_ws_dev = dev;
  return 0;
}

static int finish(hipStream_t st, const char* what) {
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    mrrr::set_last_error((std::string(what) + " kernels failed: " + hipGetErrorString(e)).c_str());
    return MRRR_ERR_HIP;
  }
  return 0;
}

static unsigned tiles(int64_t m) { return (unsigned)((m + NB - 1) / NB); }

// R (n x nv) <- L^{-1} R, L lower n x n
static void trsm_lower_left(hipStream_t st, int64_t n, int64_t nv, const double* L, int64_t ldl, double* R,
                            int64_t ldr) {
  // kPanel diagonal blocks per step: each block's solve is followed by the
  // update of the panel's remaining rows, and the rows below the panel take
  // one update of rank 64 kPanel, so the large updates pass over R
  // 1 / kPanel as often
  for (int64_t k0 = 0; k0 < n; k0 += kPanel * NB) {
    const int64_t kend = std::min<int64_t>(n, k0 + kPanel * NB);
    for (int64_t kb0 = k0; kb0 < kend; kb0 += NB) {
      const int kb = (int)std::min<int64_t>(NB, kend - kb0);
      hipLaunchKernelGGL((k_trsm_tile<false, false>), dim3(tiles(nv)), dim3(64), 0, st, L + kb0 + kb0 * ldl, ldl, kb,
                         R + kb0, ldr, nv, (const int*)nullptr);
      const int64_t rest = kend - kb0 - kb;
      if (rest > 0)
        hipLaunchKernelGGL((k_gemm_sub<false, false, false>), dim3(tiles(nv), tiles(rest)), dim3(NT), 0, st, rest, nv,
                           kb, L + (kb0 + kb) + kb0 * ldl, ldl, (const double*)(R + kb0), ldr, R + kb0 + kb, ldr,
                           (const int*)nullptr);
    }
    const int64_t below = n - kend;
    if (below > 0)
      hipLaunchKernelGGL((k_gemm_sub<false, false, false>), dim3(tiles(nv), tiles(below)), dim3(NT), 0, st, below, nv,
                         (int)(kend - k0), L + kend + k0 * ldl, ldl, (const double*)(R + k0), ldr, R + kend, ldr,
                         (const int*)nullptr);
  }
}

}  // namespace mrrr_gh

using namespace mrrr_gh;

extern "C" {

int mrrr_cholesky(int64_t n, double* B, int64_t ldb, int64_t* info, void* stream) {
  if (n < 0 || n > (int64_t)1 << 18) return -1;
  if (n > 0 && !B) return -2;
  if (ldb < std::max<int64_t>(1, n)) return -3;
  if (!info) return -4;
  *info = 0;
  if (n == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = grow(256);
  if (rc) return rc;
  int* fail = (int*)g_ws;
  if (hipMemsetAsync(fail, 0, sizeof(int), st) != hipSuccess) {
    mrrr::set_last_error("hipMemsetAsync failed");
    return MRRR_ERR_HIP;
  }
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_GHEP);
  // panels of kPanel tile columns: each tile column is first brought up to
  // date by the panel's earlier columns (its diagonal tile's lower triangle
  // and the rows below), then factored and solved; the trailing matrix takes
  // one update of rank 64 kPanel per panel
  for (int64_t k0 = 0; k0 < n; k0 += kPanel * NB) {
    const int64_t kend = std::min<int64_t>(n, k0 + kPanel * NB);
    for (int64_t t0 = k0; t0 < kend; t0 += NB) {
      const int kb = (int)std::min<int64_t>(NB, n - t0);
      const int64_t below = n - t0 - kb;
      if (t0 > k0) {
        const int kk = (int)(t0 - k0);
        const double* Pt = B + t0 + k0 * ldb;  // rows t0 .. t0 + kb of the panel's earlier columns
        hipLaunchKernelGGL((k_gemm_sub<false, true, true>), dim3(1), dim3(NT), 0, st, (int64_t)kb, (int64_t)kb, kk,
                           Pt, ldb, Pt, ldb, B + t0 + t0 * ldb, ldb, (const int*)fail);
        if (below > 0)
          hipLaunchKernelGGL((k_gemm_sub<false, true, false>), dim3(1, tiles(below)), dim3(NT), 0, st, below,
                             (int64_t)kb, kk, (const double*)(B + (t0 + kb) + k0 * ldb), ldb, Pt, ldb,
                             B + (t0 + kb) + t0 * ldb, ldb, (const int*)fail);
      }
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, B + t0 + t0 * ldb, ldb, kb, t0, fail);
      if (below > 0)
        // X L_tt^T = A21, row by row: L_tt x^T = a^T (forward)
        hipLaunchKernelGGL((k_trsm_tile<true, false>), dim3(tiles(below)), dim3(64), 0, st,
                           (const double*)(B + t0 + t0 * ldb), ldb, kb, B + (t0 + kb) + t0 * ldb, ldb, below,
                           (const int*)fail);
    }
    const int64_t below = n - kend;
    if (below > 0) {
      const double* X = B + kend + k0 * ldb;  // the panel's rows below it
      const int64_t T = tiles(below);
      hipLaunchKernelGGL((k_gemm_sub<false, true, true>), dim3((unsigned)(T * (T + 1) / 2)), dim3(NT), 0, st, below,
                         below, (int)(kend - k0), X, ldb, X, ldb, B + kend + kend * ldb, ldb, (const int*)fail);
    }
  }
  prof.end();
  int f = 0;
  if (hipMemcpyAsync(&f, fail, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) {
    mrrr::set_last_error("hipMemcpyAsync failed");
    return MRRR_ERR_HIP;
  }
  rc = finish(st, "Cholesky");
  if (rc) return rc;
  *info = f;
  if (prof.on) {
    double ms;
    int64_t l;
    prof.total(MRRR_K_GHEP, &ms, &l);
    const double nn = (double)n;
    mrrr::prof_add(MRRR_K_GHEP, l, ms, nn * nn * nn / 3.0, 0.0);
  }
  return 0;
}

int mrrr_sygst(int64_t n, double* A, int64_t lda, const double* L, int64_t ldl, void* stream) {
  if (n < 0 || n > (int64_t)1 << 18) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (n > 0 && !L) return -4;
  if (ldl < std::max<int64_t>(1, n)) return -5;
  if (n == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  const size_t xbytes = sizeof(double) * (size_t)n * (size_t)n;
  int rc = grow(256 + xbytes);
  if (rc) return rc;
  double* X = (double*)((char*)g_ws + 256);
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_GHEP);
  const unsigned T = tiles(n);
  hipLaunchKernelGGL(k_sym_full, dim3(T, T), dim3(NT), 0, st, n, (const double*)A, lda, X, n);
  trsm_lower_left(st, n, n, L, ldl, X, n);  // X = L^{-1} A
  hipLaunchKernelGGL(k_transpose, dim3(T, T), dim3(NT), 0, st, n, (const double*)X, n, A, lda);  // A = X^T
  trsm_lower_left(st, n, n, L, ldl, A, lda);  // A = L^{-1} A L^{-T}
  prof.end();
  rc = finish(st, "reduction to standard form");
  if (rc) return rc;
  if (prof.on) {
    double ms;
    int64_t l;
    prof.total(MRRR_K_GHEP, &ms, &l);
    const double nn = (double)n;
    mrrr::prof_add(MRRR_K_GHEP, l, ms, 2.0 * nn * nn * nn, 0.0);
  }
  return 0;
}

int mrrr_trsm_lt(int64_t n, int64_t m, const double* L, int64_t ldl, double* Y, int64_t ldy, void* stream) {
  if (n < 0 || n > (int64_t)1 << 18) return -1;
  if (m < 0 || m > (int64_t)1 << 31) return -2;
  if (n > 0 && !L) return -3;
  if (ldl < std::max<int64_t>(1, n)) return -4;
  if (n > 0 && m > 0 && !Y) return -5;
  if (ldy < std::max<int64_t>(1, n)) return -6;
  if (n == 0 || m == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_GHEP);
  // kPanel diagonal blocks per step, last first (as in the forward solve):
  // after each block's solve the panel's blocks above it are updated, and
  // the rows above the panel take one update of rank up to 64 kPanel
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t bt = nblk - 1; bt >= 0; bt -= kPanel) {
    const int64_t bb = std::max<int64_t>(0, bt - kPanel + 1);  // the panel's first block
    const int64_t p0 = bb * NB, pend = std::min<int64_t>(n, (bt + 1) * NB);
    for (int64_t b = bt; b >= bb; --b) {
      const int64_t k0 = b * NB;
      const int kb = (int)std::min<int64_t>(NB, n - k0);
      hipLaunchKernelGGL((k_trsm_tile<false, true>), dim3(tiles(m)), dim3(64), 0, st, L + k0 + k0 * ldl, ldl, kb,
                         Y + k0, ldy, m, (const int*)nullptr);
      const int64_t up = k0 - p0;  // panel rows above this block
      if (up > 0)
        // Y[p0:k0, :] -= L[k0:k0+kb, p0:k0]^T Y[k0:k0+kb, :]
        hipLaunchKernelGGL((k_gemm_sub<true, false, false>), dim3(tiles(m), tiles(up)), dim3(NT), 0, st, up, m, kb,
                           L + k0 + p0 * ldl, ldl, (const double*)(Y + k0), ldy, Y + p0, ldy, (const int*)nullptr);
    }
    if (p0 > 0)
      // rows above: Y[0:p0, :] -= L[p0:pend, 0:p0]^T Y[p0:pend, :]
      hipLaunchKernelGGL((k_gemm_sub<true, false, false>), dim3(tiles(m), tiles(p0)), dim3(NT), 0, st, p0, m,
                         (int)(pend - p0), L + p0, ldl, (const double*)(Y + p0), ldy, Y, ldy, (const int*)nullptr);
  }
  prof.end();
  int rc = finish(st, "triangular solve");
  if (rc) return rc;
  if (prof.on) {
    double ms;
    int64_t l;
    prof.total(MRRR_K_GHEP, &ms, &l);
    const double nn = (double)n;
    mrrr::prof_add(MRRR_K_GHEP, l, ms, nn * nn * (double)m, 0.0);
  }
  return 0;
}

// the dense drivers: every stage in turn on the caller's stream, through
// the entry points above (their workspaces, locks and synchronisation)
static std::mutex g_drv_mu;
static void* g_drv = nullptr;
static size_t g_drv_bytes = 0;
static int g_drv_dev = -1;

static int drv_buffers(int64_t n, double** d, double** e, double** tau) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    mrrr::set_last_error("hipGetDevice failed");
    return MRRR_ERR_HIP;
  }
  const size_t one = ((sizeof(double) * (size_t)std::max<int64_t>(n, 1)) + 255) & ~(size_t)255;
  if (!g_drv || g_drv_bytes < 3 * one || g_drv_dev != dev) {
    if (g_drv) {
      (void)hipDeviceSynchronize();
      (void)hipFree(g_drv);
    }
    g_drv = nullptr;
    g_drv_bytes = 0;
    if (hipMalloc(&g_drv, 3 * one) != hipSuccess) {
      mrrr::set_last_error("hipMalloc failed for the dense driver");
      return MRRR_ERR_CAPACITY;
    }
    g_drv_bytes = 3 * one;
    g_drv_dev = dev;
  }
  *d = (double*)g_drv;
  *e = (double*)((char*)g_drv + one);
  *tau = (double*)((char*)g_drv + 2 * one);
  return 0;
}

int mrrr_syevr(int64_t n, double* A, int64_t lda, mrrr_range range, double* w, double* Z, int64_t ldz,
                mrrr_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (n < 0 || n > (int64_t)1 << 18) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (range.kind < MRRR_ALL || range.kind > MRRR_VALUE) return -4;
  if (n > 0 && !w) return -5;
  if (n > 0 && !Z) return -6;
  if (ldz < std::max<int64_t>(1, n)) return -7;
  if (n == 0) return 0;
  std::lock_guard<std::mutex> lk(g_drv_mu);
  double *d, *e, *tau;
  int rc = drv_buffers(n, &d, &e, &tau);
  if (rc) return rc;
  rc = mrrr_tridiagonalize(n, A, lda, d, e, tau, stream);
  if (rc) return rc;
  mrrr_info inf;
  rc = mrrr_step(n, d, e, range, w, Z, ldz, &inf, stream);
  if (info) *info = inf;
  if (rc) return rc;
  // only the m computed eigenvectors are transformed
  return mrrr_backtransform(n, inf.m, A, lda, tau, Z, ldz, stream);
}

int mrrr_syev(int64_t n, double* A, int64_t lda, double* w, double* Z, int64_t ldz, mrrr_info* info, void* stream) {
  mrrr_range all;
  memset(&all, 0, sizeof(all));
  all.kind = MRRR_ALL;
  const int rc = mrrr_syevr(n, A, lda, all, w, Z, ldz, info, stream);
  return rc <= -5 ? rc + 1 : rc;  // argument numbers without the range
}

int mrrr_sygvr(int64_t n, double* A, int64_t lda, double* B, int64_t ldb, mrrr_range range, double* w, double* Z,
               int64_t ldz, int64_t* not_pd, mrrr_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  if (n < 0 || n > (int64_t)1 << 18) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (n > 0 && !B) return -4;
  if (ldb < std::max<int64_t>(1, n)) return -5;
  if (range.kind < MRRR_ALL || range.kind > MRRR_VALUE) return -6;
  if (n > 0 && !w) return -7;
  if (n > 0 && !Z) return -8;
  if (ldz < std::max<int64_t>(1, n)) return -9;
  if (!not_pd) return -10;
  *not_pd = 0;
  if (n == 0) return 0;
  int rc = mrrr_cholesky(n, B, ldb, not_pd, stream);
  if (rc || *not_pd) return rc;
  rc = mrrr_sygst(n, A, lda, B, ldb, stream);
  if (rc) return rc;
  mrrr_info inf;
  rc = mrrr_syevr(n, A, lda, range, w, Z, ldz, &inf, stream);
  if (info) *info = inf;
  if (rc) return rc;
  return mrrr_trsm_lt(n, inf.m, B, ldb, Z, ldz, stream);
}

int mrrr_sygv(int64_t n, double* A, int64_t lda, double* B, int64_t ldb, double* w, double* Z, int64_t ldz,
              int64_t* not_pd, mrrr_info* info, void* stream) {
  mrrr_range all;
  memset(&all, 0, sizeof(all));
  all.kind = MRRR_ALL;
  const int rc = mrrr_sygvr(n, A, lda, B, ldb, all, w, Z, ldz, not_pd, info, stream);
  return rc <= -7 ? rc + 1 : rc;  // argument numbers without the range
}

}  // extern "C"
