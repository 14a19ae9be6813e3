// Reverse-mode derivative of the tridiagonal eigendecomposition on FP64 matrix
// cores (v_mfma_f64_16x16x4f64), gfx950.
//
// For T = V diag(w) V^T and cotangents gw, gV (first-order perturbation theory):
//   M = diag(gw) + F o (V^T gV),  F_ik = 1/(w_k - w_i) (i != k), F_kk = 0
//   A = V M V^T,  grad_d_i = A_ii,  grad_e_i = A_{i,i+1} + A_{i+1,i}.
// GEMM 1 (k_bwd_c): C = V^T gV with the F epilogue, M stored column-major.
// GEMM 2 (k_bwd_band): W = V M tile by tile; the epilogue forms, per row i of
// the tile, sum_k W_ik V_ik, sum_k W_ik V_{i+1,k} and sum_k W_ik V_{i-1,k};
// W itself is never stored.  Row partials per column tile are reduced by
// k_bwd_reduce (deterministic order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "mrrr.h"
#include "mrrr_prof.h"

namespace mrrr_bwd {

constexpr int TM = 64;  // tile rows
constexpr int TN = 64;  // tile columns
constexpr int TK = 16;  // reduction step staged in LDS
constexpr int NT = 256; // threads per workgroup (4 waves, 2 x 2 quadrants of 32 x 32)

typedef double v4d __attribute__((ext_vector_type(4)));

struct Prob {
  int64_t n;
  int64_t ldv;    // leading dimension of V and gV
  const double* V;
  const double* G;  // gV (may be null)
  const double* w;
  const double* gw; // may be null
  double* M;        // n x n, column-major, ld n
  double* part;     // 3 * ntiles * n partial row sums
  double* gd;
  double* ge;
};

struct Tile {
  int32_t prob;
  int32_t ti;  // row tile
  int32_t tk;  // column tile
  int32_t pad;
};

// One 64 x 64 x 16 step: As[i][r] and Bs[j][r] in LDS; each wave accumulates a
// 32 x 32 quadrant as 2 x 2 MFMA 16x16 blocks over four K-chunks of 4.
// Operand layout of v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; it receives D[l / 16 + 4 v][l % 16], v = 0..3.
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

// GEMM 1: C = V^T G (both operands read along the reduction index r), epilogue
// M_ik = [i == k] gw_i + [i != k] C_ik / (w_k - w_i).
__global__ void __launch_bounds__(NT) k_bwd_c(const Prob* __restrict__ probs, const Tile* __restrict__ tiles) {
  __shared__ double As[TM][TK + 1];
  __shared__ double Bs[TN][TK + 1];
  const Tile tl = tiles[blockIdx.x];
  const Prob pb = probs[tl.prob];
  const int64_t n = pb.n, ld = pb.ldv;
  const int64_t i0 = (int64_t)tl.ti * TM, k0 = (int64_t)tl.tk * TN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // loader: thread t fetches column (t / 4) rows r0 + 4 (t % 4) .. +3; the
  // next step's operands are fetched into registers while the matrix cores
  // work on the current ones
  const int lc = t >> 2, lr = (t & 3) * 4;
  const int64_t ci = i0 + lc, ck = k0 + lc;
  double ra[4], rb[4];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + lr + u;
      ra[u] = (r < n && ci < n) ? pb.V[ci * ld + r] : 0.0;
      rb[u] = (r < n && ck < n) ? pb.G[ck * ld + r] : 0.0;
    }
  };
  fetch(0);
  for (int64_t r0 = 0; r0 < n; r0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[lc][lr + u] = ra[u];
      Bs[lc][lr + u] = rb[u];
    }
    __syncthreads();
    if (r0 + TK < n) fetch(r0 + TK);
    mma_step(As, Bs, acc, wr, wc, lane);
    __syncthreads();
  }
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wr * 32 + m * 16 + lk + 4 * v;
        const int64_t k = k0 + wc * 32 + q * 16 + li;
        if (i < n && k < n) {
          double val;
          if (i == k)
            val = pb.gw ? pb.gw[i] : 0.0;
          else
            val = acc[m][q][v] / (pb.w[k] - pb.w[i]);
          pb.M[k * n + i] = val;
        }
      }
}

// diag(gw) alone (no eigenvector cotangent)
__global__ void k_bwd_diag(const Prob* __restrict__ probs, const Tile* __restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const Prob pb = probs[tl.prob];
  const int64_t n = pb.n;
  const int64_t i0 = (int64_t)tl.ti * TM, k0 = (int64_t)tl.tk * TN;
  for (int e = threadIdx.x; e < TM * TN; e += blockDim.x) {
    const int64_t i = i0 + (e % TM), k = k0 + (e / TM);
    if (i < n && k < n) pb.M[k * n + i] = (i == k && pb.gw) ? pb.gw[i] : 0.0;
  }
}

// GEMM 2: W = V M and the band epilogue
__global__ void __launch_bounds__(NT) k_bwd_band(const Prob* __restrict__ probs, const Tile* __restrict__ tiles) {
  __shared__ double As[TM][TK + 1];
  __shared__ double Bs[TN][TK + 1];
  __shared__ double Vs[TM + 2][TN + 1];  // V rows i0-1 .. i0+64 of the tile's columns
  __shared__ double red[3][2][TM];       // per column half: row partials
  const Tile tl = tiles[blockIdx.x];
  const Prob pb = probs[tl.prob];
  const int64_t n = pb.n, ld = pb.ldv;
  const int64_t i0 = (int64_t)tl.ti * TM, k0 = (int64_t)tl.tk * TN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // A = V[i0.., r0..]: thread t reads column r0 + t / 16, rows i0 + 4 (t % 16) .. +3
  const int ar = t >> 4, ai = (t & 15) * 4;
  // B = M[r0.., k0..]: thread t reads column k0 + t / 4, rows r0 + 4 (t % 4) .. +3
  const int bc = t >> 2, brr = (t & 3) * 4;
  double ra[4], rm[4];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + ai + u, r = r0 + ar;
      ra[u] = (i < n && r < n) ? pb.V[r * ld + i] : 0.0;
      const int64_t rb = r0 + brr + u, kb = k0 + bc;
      rm[u] = (rb < n && kb < n) ? pb.M[kb * n + rb] : 0.0;
    }
  };
  fetch(0);
  for (int64_t r0 = 0; r0 < n; r0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[ai + u][ar] = ra[u];
      Bs[bc][brr + u] = rm[u];
    }
    __syncthreads();
    if (r0 + TK < n) fetch(r0 + TK);
    mma_step(As, Bs, acc, wr, wc, lane);
    __syncthreads();
  }
  // stage V rows i0-1 .. i0+TM (columns k0 .. k0+TN-1)
  for (int e = t; e < (TM + 2) * TN; e += NT) {
    const int rr = e % (TM + 2), cc = e / (TM + 2);
    const int64_t i = i0 - 1 + rr, k = k0 + cc;
    Vs[rr][cc] = (i >= 0 && i < n && k < n) ? pb.V[k * ld + i] : 0.0;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  // each lane: rows wr*32 + m*16 + lk + 4 v, column wc*32 + q*16 + li
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rl = wr * 32 + m * 16 + lk + 4 * v;  // tile-local row
      double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int cl = wc * 32 + q * 16 + li;
        const double wv = acc[m][q][v];
        sa += wv * Vs[rl + 1][cl];
        sb += wv * Vs[rl + 2][cl];
        sc += wv * Vs[rl][cl];
      }
      // sum over the 16 lanes that share this row (lane bits 0..3)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        sa += __shfl_xor(sa, o, 64);
        sb += __shfl_xor(sb, o, 64);
        sc += __shfl_xor(sc, o, 64);
      }
      if (li == 0) {
        red[0][wc][rl] = sa;
        red[1][wc][rl] = sb;
        red[2][wc][rl] = sc;
      }
    }
  __syncthreads();
  if (t < TM) {
    const int64_t i = i0 + t;
    if (i < n) {
      const int64_t ntk = (n + TN - 1) / TN;
      double* P = pb.part;
      P[(0 * ntk + tl.tk) * n + i] = red[0][0][t] + red[0][1][t];
      P[(1 * ntk + tl.tk) * n + i] = red[1][0][t] + red[1][1][t];
      P[(2 * ntk + tl.tk) * n + i] = red[2][0][t] + red[2][1][t];
    }
  }
}

// gd_i = sum_kt Pa[kt][i];  ge_i = sum_kt (Pb[kt][i] + Pc[kt][i+1])
__global__ void k_bwd_reduce(const Prob* __restrict__ probs, int nprob, const int64_t* __restrict__ rowoff,
                             int64_t rows) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows) return;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rowoff[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const Prob pb = probs[lo];
  const int64_t i = g - rowoff[lo];
  const int64_t n = pb.n;
  const int64_t ntk = (n + TN - 1) / TN;
  const double* P = pb.part;
  double a = 0.0, b = 0.0;
  for (int64_t kt = 0; kt < ntk; ++kt) {
    a += P[(0 * ntk + kt) * n + i];
    if (i + 1 < n) b += P[(1 * ntk + kt) * n + i] + P[(2 * ntk + kt) * n + i + 1];
  }
  pb.gd[i] = a;
  if (i + 1 < n) pb.ge[i] = b;
}

// ---------------------------------------------------------------------------
// host side

static std::mutex g_mu;
static void* g_ws = nullptr;
static size_t g_ws_bytes = 0;

static int grow(size_t bytes) {
  if (bytes <= g_ws_bytes && g_ws) return 0;
  if (g_ws) (void)hipFree(g_ws);
  g_ws = nullptr;
  g_ws_bytes = 0;
  size_t nb = std::max(bytes, (size_t)1 << 20);
  if (hipMalloc(&g_ws, nb) != hipSuccess) {
    mrrr::set_last_error("hipMalloc failed for the backward workspace");
    return MRRR_ERR_CAPACITY;
  }
  g_ws_bytes = nb;
  return 0;
}

static int run(std::vector<Prob>& probs, hipStream_t st) {
  const int np = (int)probs.size();
  // workspace: M and partials per problem, then the problem and tile tables
  size_t bytes = 0;
  std::vector<size_t> moff(np), poff(np);
  std::vector<Tile> tiles;
  std::vector<int64_t> rowoff(np + 1, 0);
  for (int p = 0; p < np; ++p) {
    const int64_t n = probs[p].n;
    const int64_t nt = (n + TM - 1) / TM;
    moff[p] = bytes;
    bytes += sizeof(double) * (size_t)(n * n);
    poff[p] = bytes;
    bytes += sizeof(double) * (size_t)(3 * nt * n);
    for (int64_t a = 0; a < nt; ++a)
      for (int64_t b = 0; b < nt; ++b) tiles.push_back(Tile{p, (int32_t)a, (int32_t)b, 0});
    rowoff[p + 1] = rowoff[p] + n;
  }
  bytes = (bytes + 255) & ~(size_t)255;
  const size_t prob_off = bytes;
  bytes += sizeof(Prob) * np;
  bytes = (bytes + 255) & ~(size_t)255;
  const size_t tile_off = bytes;
  bytes += sizeof(Tile) * tiles.size();
  bytes = (bytes + 255) & ~(size_t)255;
  const size_t row_off = bytes;
  bytes += sizeof(int64_t) * (np + 1);
  int rc = grow(bytes);
  if (rc) return rc;
  char* base = (char*)g_ws;
  bool anyG = false;
  for (int p = 0; p < np; ++p) {
    probs[p].M = (double*)(base + moff[p]);
    probs[p].part = (double*)(base + poff[p]);
    anyG = anyG || probs[p].G != nullptr;
  }
  Prob* dP = (Prob*)(base + prob_off);
  Tile* dT = (Tile*)(base + tile_off);
  int64_t* dR = (int64_t*)(base + row_off);
  if (hipMemcpyAsync(dP, probs.data(), sizeof(Prob) * np, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dT, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dR, rowoff.data(), sizeof(int64_t) * (np + 1), hipMemcpyHostToDevice, st) != hipSuccess) {
    mrrr::set_last_error("hipMemcpyAsync failed");
    return MRRR_ERR_HIP;
  }
  const unsigned nt = (unsigned)tiles.size();
  mrrr::ProfEvents prof(st);
  prof.begin(MRRR_K_BACKWARD);
  // problems without gV take the diagonal path; GEMM 1 is only launched when
  // every problem has gV (mixed batches are rejected by the caller)
  if (anyG)
    hipLaunchKernelGGL(k_bwd_c, dim3(nt), dim3(NT), 0, st, dP, dT);
  else
    hipLaunchKernelGGL(k_bwd_diag, dim3(nt), dim3(256), 0, st, dP, dT);
  hipLaunchKernelGGL(k_bwd_band, dim3(nt), dim3(NT), 0, st, dP, dT);
  prof.end();
  const int64_t rows = rowoff[np];
  hipLaunchKernelGGL(k_bwd_reduce, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, dP, np, dR, rows);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    mrrr::set_last_error((std::string("backward kernels failed: ") + hipGetErrorString(e)).c_str());
    return MRRR_ERR_HIP;
  }
  if (prof.on) {
    double ms, work = 0.0;
    int64_t l;
    prof.total(MRRR_K_BACKWARD, &ms, &l);
    for (auto& p : probs) work += (anyG ? 4.0 : 2.0) * (double)p.n * (double)p.n * (double)p.n;
    mrrr::prof_add(MRRR_K_BACKWARD, l, ms, work, 0.0);
  }
  return 0;
}

}  // namespace mrrr_bwd

using namespace mrrr_bwd;

extern "C" {

int mrrr_step_backward(int64_t n, const double* w, const double* Z, int64_t ldz, const double* gw,
                       const double* gZ, int64_t ldgz, double* gd, double* ge, void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !w) return -2;
  if (n > 0 && !Z) return -3;
  if (ldz < std::max<int64_t>(1, n)) return -4;
  if (gZ && ldgz != ldz) return -7;  // one leading dimension for V and gV
  if (n > 0 && !gd) return -8;
  if (n > 1 && !ge) return -9;
  if (n > 46340) return -1;
  if (n == 0) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<Prob> probs(1);
  probs[0] = Prob{n, ldz, Z, gZ, w, gw, nullptr, nullptr, gd, ge};
  return run(probs, (hipStream_t)stream);
}

int mrrr_step_backward_batched(int64_t batch, const int64_t* n_host, const int64_t* off_host,
                               const int64_t* zoff_host, const double* w, const double* Z, const double* gw,
                               const double* gZ, double* gd, double* ge, void* stream) {
  if (batch < 0) return -1;
  if (batch == 0) return 0;
  if (!n_host) return -2;
  if (!off_host) return -3;
  if (!zoff_host) return -4;
  if (!w) return -5;
  if (!Z) return -6;
  if (!gd) return -9;
  if (!ge) return -10;
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<Prob> probs(batch);
  for (int64_t b = 0; b < batch; ++b) {
    const int64_t n = n_host[b];
    if (n < 1 || n > 46340) return -2;
    const int64_t o = off_host[b], zo = zoff_host[b];
    probs[b] = Prob{n, n, Z + zo, gZ ? gZ + zo : nullptr, w + o, gw ? gw + o : nullptr,
                    nullptr, nullptr, gd + o, ge + o};
  }
  return run(probs, (hipStream_t)stream);
}

}  // extern "C"
