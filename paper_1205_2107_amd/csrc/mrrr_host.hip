// Host runtime and C ABI of the MI355X MRRR solver: workspace management, the
// level-by-level drive of the representation tree, argument checking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mrrr.h"
#include "mrrr_dev.h"
#include "mrrr_launch.h"
#include "mrrr_prof.h"

namespace mrrr {

static thread_local std::string g_err;
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static mrrr_kernel_time g_prof[MRRR_K_COUNT];

bool prof_enabled() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

void prof_add(int kernel, int64_t launches, double ms, double work, double bytes) {
  if (kernel < 0 || kernel >= MRRR_K_COUNT) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof[kernel].launches += launches;
  g_prof[kernel].ms += ms;
  g_prof[kernel].work += work;
  g_prof[kernel].bytes += bytes;
}

static mrrr_tuning g_tune = {4, 0, 0, 0, 0, {0, 0, 0}};
static std::mutex g_tune_mu;

void set_last_error(const char* msg) { g_err = msg ? msg : ""; }

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(x)                                                                                   \
  do {                                                                                               \
    hipError_t _e = (x);                                                                             \
    if (_e != hipSuccess) return fail(MRRR_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(_e));     \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Workspace {
  std::mutex mu;
  DevBuf problems, poff, sprob, ds, es, flag, excl, tiles, total, bstart, sblk, blocks, goff, nodes, pool, gcnt, lo,
      hi, clo, chi, snode, sflag, scol, val, runflag, runid, runs, clusters, counters, vrid, cflag, cid, cstart,
      scratch, ckscratch, chunkrows, chunks, chunkoff, bad, perm, tmp, sgap;
  // second stream (default priority) for the checkpointing eigenvector kernel,
  // which runs beside the stored-vector kernel; fork and join events
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // arena mode: every buffer is carved from one caller-provided region
  // [abase, abase + acap) by a bump pointer; nothing is allocated.  The most
  // recently carved buffer can grow in place.
  char* abase = nullptr;
  size_t acap = 0, aused = 0;
  void* alast = nullptr;
  bool no_fork = false;  // run both eigenvector kernels on the caller's stream
  size_t total_bytes() const {
    const DevBuf* all[] = {&problems, &poff, &sprob, &ds, &es, &flag, &excl, &tiles, &total, &bstart, &sblk, &blocks,
                           &goff, &nodes, &pool, &gcnt, &lo, &hi, &clo, &chi, &snode, &sflag, &scol, &val, &runflag,
                           &runid, &runs, &clusters, &counters, &vrid, &cflag, &cid, &cstart, &scratch, &ckscratch,
                           &chunkrows, &chunks, &chunkoff, &bad, &perm, &tmp, &sgap};
    size_t t = 0;
    for (auto* b : all) t += b->bytes;
    return t;
  }
  void release() {
    DevBuf* all[] = {&problems, &poff, &sprob, &ds, &es, &flag, &excl, &tiles, &total, &bstart, &sblk, &blocks,
                     &goff, &nodes, &pool, &gcnt, &lo, &hi, &clo, &chi, &snode, &sflag, &scol, &val, &runflag,
                     &runid, &runs, &clusters, &counters, &vrid, &cflag, &cid, &cstart, &scratch, &ckscratch,
                     &chunkrows, &chunks, &chunkoff, &bad, &perm, &tmp, &sgap};
    for (auto* b : all) {
      if (b->p) (void)hipFree(b->p);
      b->p = nullptr;
      b->bytes = 0;
    }
    if (aux) (void)hipStreamDestroy(aux);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    aux = nullptr;
    ev_fork = ev_join = nullptr;
  }
};

static std::mutex g_ws_mu;
static std::map<int, Workspace*> g_ws;

static Workspace* workspace_for_current_device(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_ws.find(dev);
  if (it == g_ws.end()) it = g_ws.emplace(dev, new Workspace()).first;
  *dev_out = dev;
  return it->second;
}

constexpr size_t kAlign = 256;
static size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// arena mode: a region of the caller's workspace (no allocation); keep copies
// the old contents into a new region unless the buffer is the last one carved,
// which grows in place
static int carve(Workspace& W, DevBuf& b, size_t bytes, hipStream_t st, bool keep) {
  bytes = align_up(std::max<size_t>(bytes, 1));
  if (b.p && b.p == W.alast) {
    const size_t start = (size_t)((char*)b.p - W.abase);
    if (start + bytes > W.acap)
      return fail(MRRR_ERR_CAPACITY, "workspace of %zu bytes exhausted (needs at least %zu)", W.acap, start + bytes);
    W.aused = start + bytes;
    b.bytes = bytes;
    return 0;
  }
  const size_t start = align_up(W.aused);
  if (start + bytes > W.acap)
    return fail(MRRR_ERR_CAPACITY, "workspace of %zu bytes exhausted (needs at least %zu)", W.acap, start + bytes);
  void* p = W.abase + start;
  if (keep && b.p && b.bytes) {
    hipError_t e = hipMemcpyAsync(p, b.p, b.bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(MRRR_ERR_HIP, "workspace copy failed: %s", hipGetErrorString(e));
  }
  b.p = p;
  b.bytes = bytes;
  W.aused = start + bytes;
  W.alast = p;
  return 0;
}

// bytes still free in the arena
static size_t arena_free(const Workspace& W) {
  const size_t u = align_up(W.aused);
  return u < W.acap ? W.acap - u : 0;
}

// grow-only device buffer; contents are not preserved unless keep is set
static int ensure(Workspace& W, DevBuf& b, size_t bytes, hipStream_t st, bool keep = false) {
  if (bytes <= b.bytes && b.p) return 0;
  if (W.abase) return carve(W, b, bytes, st, keep);
  size_t nb = std::max(bytes, b.bytes + b.bytes / 4);
  nb = std::max<size_t>(nb, 256);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) return fail(MRRR_ERR_CAPACITY, "hipMalloc(%zu bytes) failed: %s", nb, hipGetErrorString(e));
  if (keep && b.p && b.bytes) {
    e = hipMemcpyAsync(p, b.p, b.bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return fail(MRRR_ERR_HIP, "workspace copy failed: %s", hipGetErrorString(e));
    }
  }
  if (b.p) (void)hipFree(b.p);
  b.p = p;
  b.bytes = nb;
  return 0;
}

template <class T>
static T* P_(DevBuf& b) {
  return static_cast<T*>(b.p);
}

// scratch budget for the eigenvector kernel (bytes): a quarter of the device
constexpr bool kShareLevels = true, kShareLeaf = true;
constexpr int64_t kFillMinBlock = 4096;  // mean block size from which the root refinement is persistent

static size_t scratch_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess || tot == 0) return size_t(8) << 30;
  return std::max<size_t>(size_t(1) << 30, tot / 4);
}

struct Report {
  Counters c;
  int nblk = 0;
  int levels = 0;
  int nodes = 0;
  size_t ws_bytes = 0;
  int64_t ambiguous_left = 0;  // pairs classified from unrefined brackets after three refinements
  int depth_stop = 0;          // the level loop stopped at its depth guard
};

// limits the caller may lower (tests use them to force the status paths)
static mrrr_limits g_limits = {kMaxDepth, 0, 0.0};
static std::mutex g_limits_mu;

// Solve a list of problems (packed into slot space) on one stream.
static int solve(Workspace& W, std::vector<Problem>& probs, const double* d, const double* e, double* w, double* Z,
                 hipStream_t st, Report* rep, const mrrr_tuning* use = nullptr) {
  const int nprob = (int)probs.size();
  mrrr_tuning tune;
  if (use) {
    tune = *use;
  } else {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune = g_tune;
  }
  const int G = tune.grid_density;
  mrrr_limits lim;
  {
    std::lock_guard<std::mutex> lk(g_limits_mu);
    lim = g_limits;
  }
  std::vector<int64_t> poff(nprob + 1, 0);
  for (int p = 0; p < nprob; ++p) poff[p + 1] = poff[p] + probs[p].n;
  const int64_t ntot = poff[nprob];
  memset(rep, 0, sizeof(*rep));
  if (ntot == 0) return 0;
  int rc;
  ProfEvents prof(st);
  // lanes per eigenvalue in refinement: spread small problems over more lanes
  int slots = tune.refine_wave_slots;
  if (slots == 0) slots = (ntot <= 32768) ? 16 : (ntot <= 131072 ? 32 : 64);
  const int lanes = 64 / slots;
  double grid_work = 0.0;
#define ENS(buf, bytes)                                             \
  do {                                                              \
    if ((rc = ensure(W, W.buf, (size_t)(bytes), st)) != 0) return rc; \
  } while (0)
  ENS(problems, sizeof(Problem) * nprob);
  ENS(poff, sizeof(int64_t) * (nprob + 1));
  ENS(sprob, sizeof(int32_t) * ntot);
  ENS(ds, sizeof(double) * ntot);
  ENS(es, sizeof(double) * ntot);
  ENS(flag, sizeof(int32_t) * ntot);
  ENS(excl, sizeof(int32_t) * ntot);
  ENS(tiles, sizeof(int32_t) * ((ntot + 1023) / 1024 + 1));
  ENS(total, sizeof(int32_t) * 4);
  ENS(counters, sizeof(Counters));
  for (auto& p : probs) {
    p.tmax_bits = 0;
    p.tnorm_bits = 0;
    p.scale = 1.0;
    p.status = 0;
    p.nblk = 0;
    p.first_blk = 0;
    p.below = 0;
    if (p.kind == MRRR_ALL) p.m = p.n;
    if (p.kind == MRRR_INDEX) p.m = p.iu - p.il + 1;
    if (p.kind == MRRR_VALUE) p.m = 0;
  }
  HIP_TRY(hipMemcpyAsync(W.problems.p, probs.data(), sizeof(Problem) * nprob, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(W.poff.p, poff.data(), sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(W.counters.p, 0, sizeof(Counters), st));
  Problem* dP = P_<Problem>(W.problems);
  Counters* dC = P_<Counters>(W.counters);

  // 1. scale, norms, split
  launch_prep(st, dP, nprob, P_<int64_t>(W.poff), ntot, d, e, P_<int32_t>(W.sprob), P_<double>(W.ds),
              P_<double>(W.es), P_<int32_t>(W.flag));
  launch_scan(st, P_<int32_t>(W.flag), P_<int32_t>(W.excl), P_<int32_t>(W.tiles), ntot, P_<int32_t>(W.total));
  int32_t nblk = 0;
  HIP_TRY(hipMemcpyAsync(&nblk, W.total.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipGetLastError());
  rep->nblk = nblk;
  const bool arena = W.abase != nullptr;
  ENS(bstart, sizeof(int64_t) * (nblk + 1));
  ENS(sblk, sizeof(int32_t) * ntot);
  ENS(blocks, sizeof(Block) * nblk);
  ENS(goff, sizeof(int64_t) * (nblk + 1));
  // node table: roots first; grows per level (in arena mode sized once for
  // nblk + ntot nodes: every child holds at least two eigenvalues of its parent)
  ENS(nodes, sizeof(Node) * (size_t)(arena ? (int64_t)nblk + ntot + 16
                                           : std::max<int64_t>(nblk + 16, 2 * (int64_t)nblk)));
  // per-slot arrays, the count grid and the cluster list: sizes known now
  const int64_t gtot = (int64_t)G * ntot + nblk;
  ENS(gcnt, sizeof(int32_t) * gtot);
  ENS(lo, sizeof(double) * ntot);
  ENS(hi, sizeof(double) * ntot);
  ENS(clo, sizeof(int32_t) * ntot);
  ENS(chi, sizeof(int32_t) * ntot);
  ENS(snode, sizeof(int32_t) * ntot);
  ENS(sflag, sizeof(uint32_t) * ntot);
  ENS(scol, sizeof(int64_t) * ntot);
  ENS(val, sizeof(double) * ntot);
  ENS(sgap, sizeof(double) * ntot);
  ENS(runflag, sizeof(int32_t) * ntot);
  ENS(runid, sizeof(int32_t) * ntot);
  ENS(runs, sizeof(int64_t) * (ntot + 1));
  ENS(vrid, sizeof(int32_t) * ntot);
  ENS(cflag, sizeof(int32_t) * ntot);
  ENS(cid, sizeof(int32_t) * ntot);
  ENS(cstart, sizeof(int64_t) * (ntot + 1));
  const int max_clusters = (int)std::min<int64_t>(ntot / 2 + 1, INT32_MAX / 2);
  if (Z != nullptr) ENS(clusters, sizeof(Cluster) * (size_t)max_clusters);
  int64_t nmax_prob = 1;
  for (auto& p : probs) nmax_prob = std::max<int64_t>(nmax_prob, p.n);
  int vslots = tune.vec_wave_slots;
  if (vslots == 0) vslots = 32;
  // arena mode: what the eigenvector phase needs at least after the tree
  // (chunk lists, one chunk of each kernel's scratch, the sort fix-up), kept
  // free while the pool grows
  const int64_t nch_all = (ntot + vslots - 1) / vslots;
  const size_t vec_reserve =
      (Z == nullptr) ? align_up(sizeof(int32_t) * nprob)
                     : 8 * kAlign + align_up(sizeof(int32_t) * nch_all) + align_up(sizeof(int32_t) * (nch_all + 1)) +
                           align_up(sizeof(int64_t) * (nch_all + 1)) +
                           align_up(sizeof(double) * 4 * (size_t)vslots * (size_t)nmax_prob) +
                           align_up(sizeof(double) * 4 * (size_t)vslots * (size_t)((nmax_prob + kSeg - 1) / kSeg)) +
                           align_up(sizeof(int32_t) * nprob) + 2 * align_up(sizeof(int64_t) * ntot);
  // pool: roots aligned with slots plus room for children (grown on demand;
  // in arena mode it is carved last, so it grows in place)
  size_t pool_rows = (size_t)ntot + (size_t)std::max<int64_t>(4 * 1024, ntot / 2);
  if (arena) {
    pool_rows = (size_t)ntot + (Z != nullptr ? (size_t)2 * (size_t)nmax_prob : 0);
    const size_t room = arena_free(W) > vec_reserve ? arena_free(W) - vec_reserve : 0;
    pool_rows = std::max<size_t>((size_t)ntot, std::min(pool_rows, room / sizeof(Rep)));
  } else if (W.pool.bytes / sizeof(Rep) > pool_rows) {
    pool_rows = W.pool.bytes / sizeof(Rep);
  }
  ENS(pool, sizeof(Rep) * pool_rows);
  launch_blocks(st, dP, P_<int64_t>(W.poff), P_<int32_t>(W.flag), P_<int32_t>(W.excl), ntot, nblk,
                P_<int32_t>(W.sprob), P_<int64_t>(W.bstart), P_<int32_t>(W.sblk), P_<Block>(W.blocks));
  // grid offsets: block b owns G * n_b + 1 points starting at G * row0_b + b
  {
    std::vector<int64_t> bst(nblk);
    HIP_TRY(hipMemcpyAsync(bst.data(), W.bstart.p, sizeof(int64_t) * nblk, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> go(nblk + 1);
    for (int b = 0; b < nblk; ++b) {
      go[b] = (int64_t)G * bst[b] + b;
      const int64_t nb = ((b + 1 < nblk) ? bst[b + 1] : ntot) - bst[b];
      grid_work += 4.0 * (double)(G * nb + 1) * (double)nb;
    }
    go[nblk] = (int64_t)G * ntot + nblk;
    HIP_TRY(hipMemcpyAsync(W.goff.p, go.data(), sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice, st));
  }
  Block* dB = P_<Block>(W.blocks);
  Rep* dpool = P_<Rep>(W.pool);

  // 2. root representations, 3. brackets from the count grid, 4. refinement
  launch_root(st, dP, dB, P_<Node>(W.nodes), nblk, P_<double>(W.ds), P_<double>(W.es), dpool, dC, G);
  prof.begin(MRRR_K_GRID);
  launch_grid(st, dB, nblk, P_<int64_t>(W.goff), gtot, dpool, P_<int32_t>(W.gcnt));
  prof.end();
  launch_assign(st, dB, P_<int64_t>(W.goff), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.gcnt), P_<double>(W.lo),
                P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi), P_<int32_t>(W.snode),
                P_<uint32_t>(W.sflag), dC);
  // the refinements of child frames work on chunks of one node's flagged
  // slots (64 / lanes per wavefront): a wavefront counts with one
  // representation, so its eigenvalues share their counts, and its make-up
  // depends only on the node, not on the other problems of a batch.  The root
  // level refines each eigenvalue on its own points (shared points there
  // changed the geometric matrix's tree for the worse), so it needs no chunks.
  auto refine_flagged = [&](bool need_col, bool share) -> int {
    launch_node_chunks(st, ntot, P_<uint32_t>(W.sflag), P_<int64_t>(W.scol), F_NEEDS_REFINE, need_col,
                       P_<int32_t>(W.snode), 64 / lanes, P_<int32_t>(W.runflag), P_<int32_t>(W.runid),
                       P_<int32_t>(W.tiles), P_<int32_t>(W.total), P_<int32_t>(W.vrid), P_<int64_t>(W.runs),
                       P_<int32_t>(W.cflag), P_<int32_t>(W.cid), P_<int64_t>(W.cstart));
    int32_t nrc = 0;
    HIP_TRY(hipMemcpyAsync(&nrc, W.total.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    prof.begin(MRRR_K_REFINE);
    launch_refine(st, dB, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode), dpool,
                  P_<double>(W.lo), P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi),
                  P_<uint32_t>(W.sflag), dC, lanes, false, P_<int64_t>(W.cstart), P_<int32_t>(W.vrid), nrc,
                  share);
    prof.end();
    return 0;
  };
  // root level: every slot is flagged, so the node runs are the blocks.  With
  // large blocks and more chunks than SIMDs the refinement runs as persistent
  // wavefronts (one per SIMD) whose lane groups claim the eigenvalues of their
  // block one at a time (the split buffers, free since the blocks were formed,
  // hold the claim counters and cursor); small blocks (a batch of small
  // problems) keep one wavefront per chunk, which hides latency better there.
  // Both give the same values.
  const int simds = device_simds();
  if (ntot < (int64_t)kFillMinBlock * nblk || ntot / (64 / lanes) <= simds) {
    prof.begin(MRRR_K_REFINE);
    launch_refine(st, dB, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode), dpool,
                  P_<double>(W.lo), P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi),
                  P_<uint32_t>(W.sflag), dC, lanes);
    prof.end();
  } else {
    launch_node_chunks(st, ntot, P_<uint32_t>(W.sflag), P_<int64_t>(W.scol), F_NEEDS_REFINE, false,
                       P_<int32_t>(W.snode), 64 / lanes, P_<int32_t>(W.runflag), P_<int32_t>(W.runid),
                       P_<int32_t>(W.tiles), P_<int32_t>(W.total), P_<int32_t>(W.vrid), P_<int64_t>(W.runs),
                       P_<int32_t>(W.cflag), P_<int32_t>(W.cid), P_<int64_t>(W.cstart));
    int32_t nrc = 0;
    HIP_TRY(hipMemcpyAsync(&nrc, W.total.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    prof.begin(MRRR_K_REFINE);
    launch_refine_fill(st, dB, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode), dpool,
                       P_<double>(W.lo), P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi),
                       P_<uint32_t>(W.sflag), dC, lanes, P_<int64_t>(W.cstart), P_<int32_t>(W.vrid),
                       P_<int64_t>(W.runs), nrc, P_<int32_t>(W.flag), P_<int32_t>(W.excl), simds);
    prof.end();
  }
  // problem table after the root pass: VALUE counts, block counts
  HIP_TRY(hipMemcpyAsync(probs.data(), W.problems.p, sizeof(Problem) * nprob, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipGetLastError());
  bool multi = false;
  for (auto& p : probs) multi = multi || p.nblk > 1;
  // 5. output columns
  launch_columns(st, dP, dB, nblk, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<double>(W.lo),
                 P_<double>(W.hi), P_<double>(W.val), P_<int64_t>(W.scol), multi);
  if (Z == nullptr) {
    launch_values_only(st, dP, dB, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode),
                       P_<int64_t>(W.scol), P_<double>(W.lo), P_<double>(W.hi), P_<double>(W.ds), w);
  } else {
    // 6-7. representation tree, level by level
    int node_base = nblk;
    const size_t node_cap = W.nodes.bytes / sizeof(Node);
    for (int level = 0;; ++level) {
      // classification; pairs whose decision the bracket widths could flip are
      // refined (validated, full accuracy) and classified again
      int32_t nruns = 0;
      for (int round = 0;; ++round) {
        HIP_TRY(hipMemsetAsync((char*)W.counters.p + offsetof(Counters, ambiguous), 0, sizeof(int32_t), st));
        launch_cls_flags(st, dB, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode),
                         P_<double>(W.lo), P_<double>(W.hi), P_<uint32_t>(W.sflag), P_<int32_t>(W.runflag), dC);
        launch_scan(st, P_<int32_t>(W.runflag), P_<int32_t>(W.runid), P_<int32_t>(W.tiles), ntot,
                    P_<int32_t>(W.total));
        int32_t amb = 0;
        HIP_TRY(hipMemcpyAsync(&nruns, W.total.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&amb, (char*)W.counters.p + offsetof(Counters, ambiguous), sizeof(int32_t),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (amb == 0) break;
        if (round >= 3) {
          // still ambiguous after three refinements: classified from the
          // brackets as they are (counted, not an error)
          rep->ambiguous_left += amb;
          break;
        }
        if ((rc = refine_flagged(false, kShareLevels)) != 0) return rc;
      }
      launch_cls_compact(st, ntot, P_<int32_t>(W.runflag), P_<int32_t>(W.runid), P_<int64_t>(W.runs));
      launch_cls_runs(st, dB, P_<Node>(W.nodes), nruns, P_<int64_t>(W.runs), P_<int32_t>(W.sblk),
                      P_<int32_t>(W.snode), P_<double>(W.lo), P_<double>(W.hi), P_<int64_t>(W.scol),
                      P_<uint32_t>(W.sflag), P_<double>(W.sgap), P_<Cluster>(W.clusters), max_clusters, dC,
                      lim.max_depth);
      launch_clear_active(st, ntot, P_<uint32_t>(W.sflag));
      Counters hc;
      HIP_TRY(hipMemcpyAsync(&hc, W.counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipGetLastError());
      rep->levels = level + 1;
      const int ncl = std::min(hc.nclusters, max_clusters);
      if (ncl == 0) break;
      if (level > lim.max_depth + 2) {
        // the depth test of the classification makes this unreachable; kept
        // as a guard so the loop always ends
        rep->depth_stop = 1;
        break;
      }
      // capacity for the new nodes and the speculative child regions of every
      // cluster (two with masked stores, four in the branch-free form, every
      // candidate's when the regions stay small: no second pass)
      if (arena && (size_t)(node_base + ncl) > node_cap)
        return fail(MRRR_ERR_CAPACITY, "node table of %zu entries exhausted", node_cap);
      if ((rc = ensure(W, W.nodes, sizeof(Node) * (size_t)(node_base + ncl), st, true)) != 0) return rc;
      // pool demand of the level: each cluster's child (its block's n rows)
      // and the checkpoints of its candidates (child_ck_rows, n / 16 rows)
      const size_t used_rows = (size_t)std::max<unsigned long long>(hc.pool_used, (unsigned long long)ntot);
      const size_t level_rows = (size_t)hc.cluster_rows + (size_t)hc.cluster_rows / 16 + (size_t)8 * (size_t)ncl;
      if (arena) {
        // the pool grows in place up to what the eigenvector phase must keep free
        const size_t pool_start = (size_t)((char*)W.pool.p - W.abase);
        const size_t room_rows =
            (W.acap > vec_reserve + pool_start) ? (W.acap - vec_reserve - pool_start) / sizeof(Rep) : 0;
        if (used_rows + level_rows > room_rows)
          return fail(MRRR_ERR_CAPACITY, "workspace of %zu bytes too small for the representation tree", W.acap);
      }
      const size_t need_rows = used_rows + level_rows;
      if (need_rows * sizeof(Rep) > W.pool.bytes) {
        if ((rc = ensure(W, W.pool, need_rows * sizeof(Rep) + (arena ? 0 : W.pool.bytes / 2), st, true)) != 0)
          return rc;
        dpool = P_<Rep>(W.pool);
      }
      const unsigned long long pool_cap = W.pool.bytes / sizeof(Rep);
      // children are appended after the root rows
      if (hc.pool_used < (unsigned long long)ntot) {
        unsigned long long pu = (unsigned long long)ntot;
        HIP_TRY(hipMemcpyAsync((char*)W.counters.p + offsetof(Counters, pool_used), &pu, sizeof(pu),
                               hipMemcpyHostToDevice, st));
      }
      prof.begin(MRRR_K_CHILD);
      launch_child(st, dB, P_<Node>(W.nodes), ncl, node_base, P_<Cluster>(W.clusters), P_<double>(W.lo),
                   P_<double>(W.hi), dpool, pool_cap, dC, lim.child_growth_limit);
      prof.end();
      launch_shift(st, dB, P_<Node>(W.nodes), ncl, node_base, P_<Cluster>(W.clusters), P_<int64_t>(W.scol),
                   P_<double>(W.lo), P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi),
                   P_<int32_t>(W.snode), P_<uint32_t>(W.sflag), P_<double>(W.sgap));
      HIP_TRY(hipMemsetAsync((char*)W.counters.p + offsetof(Counters, nclusters), 0, sizeof(int32_t), st));
      HIP_TRY(hipMemsetAsync((char*)W.counters.p + offsetof(Counters, cluster_rows), 0, sizeof(unsigned long long),
                             st));
      node_base += ncl;
    }
    rep->nodes = node_base - nblk;
    // singletons of child nodes: validated, full-accuracy brackets in their
    // leaf's frame; each wavefront takes eigenvalues of one node (chunks of
    // equal-node slots) so that it reads one representation through LDS
    launch_mark_leaf(st, ntot, P_<int64_t>(W.scol), P_<uint32_t>(W.sflag));
    if ((rc = refine_flagged(false, kShareLeaf)) != 0) return rc;
    // 8. eigenvectors of all singletons.  Long runs of singletons of one node
    //    in large blocks go to the checkpointing kernel (one node per
    //    wavefront, representation staged through LDS, nothing of length n
    //    stored per eigenvector); the rest to the stored-vector kernel (32
    //    consecutive slots per wavefront, four work vectors in memory).  Both
    //    compute the same values.  Eigenvectors per wavefront: tuning, 32 by
    //    default.
    launch_node_chunks(st, ntot, P_<uint32_t>(W.sflag), P_<int64_t>(W.scol), F_SINGLETON, true,
                       P_<int32_t>(W.snode), vslots, P_<int32_t>(W.runflag), P_<int32_t>(W.runid),
                       P_<int32_t>(W.tiles), P_<int32_t>(W.total), P_<int32_t>(W.vrid), P_<int64_t>(W.runs),
                       P_<int32_t>(W.cflag), P_<int32_t>(W.cid), P_<int64_t>(W.cstart));
    const int min_run = tune.vec_ckpt_min_run == 0 ? kCkptMinRun
                        : (tune.vec_ckpt_min_run < 0 ? INT_MAX : tune.vec_ckpt_min_run);
    const int min_n = tune.vec_ckpt_min_n > 0 ? tune.vec_ckpt_min_n : kCkptMinN;
    launch_mark_ckpt(st, ntot, dB, P_<int32_t>(W.sblk), P_<int32_t>(W.vrid), P_<int64_t>(W.runs), min_run,
                     min_n, P_<uint32_t>(W.sflag));
    launch_node_chunks(st, ntot, P_<uint32_t>(W.sflag), P_<int64_t>(W.scol), F_SINGLETON | F_CKPT, true,
                       P_<int32_t>(W.snode), vslots, P_<int32_t>(W.runflag), P_<int32_t>(W.runid),
                       P_<int32_t>(W.tiles), P_<int32_t>(W.total), P_<int32_t>(W.vrid), P_<int64_t>(W.runs),
                       P_<int32_t>(W.cflag), P_<int32_t>(W.cid), P_<int64_t>(W.cstart));
    int32_t nchunks = 0;
    HIP_TRY(hipMemcpyAsync(&nchunks, W.total.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int64_t nmax_all = 1;
    for (auto& p : probs) nmax_all = std::max<int64_t>(nmax_all, p.n);
    // checkpoints per chunk: s, p and their derivatives, [segment][slot] each
    const int64_t stride = 4 * (int64_t)vslots * ((nmax_all + kSeg - 1) / kSeg);
    // the stored-vector kernel's chunks (32 consecutive slots, scratch sized
    // by their largest block), planned and uploaded before either kernel
    // starts: a transfer queued while the checkpointing kernel fills the chip
    // would wait for free compute units
    const int64_t nch = nch_all;
    ENS(chunkrows, sizeof(int32_t) * nch);
    if (arena) {
      ENS(chunks, sizeof(int32_t) * (nch + 1));
      ENS(chunkoff, sizeof(int64_t) * (nch + 1));
    }
    launch_chunk_rows(st, dB, ntot, P_<int32_t>(W.sblk), P_<uint32_t>(W.sflag), P_<int64_t>(W.scol), vslots,
                      P_<int32_t>(W.chunkrows));
    std::vector<int32_t> rows(nch);
    HIP_TRY(hipMemcpyAsync(rows.data(), W.chunkrows.p, sizeof(int32_t) * nch, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int32_t> act;
    int64_t maxper = 0;
    for (int64_t c = 0; c < nch; ++c)
      if (rows[c] > 0) {
        act.push_back((int32_t)c);
        maxper = std::max<int64_t>(maxper, 4 * vslots * (int64_t)rows[c]);
      }
    // scratch budgets: a quarter of the device each, or in arena mode what is
    // left of the workspace (less the sort fix-up), shared by the two kernels
    size_t sbudget = scratch_budget(), ckbudget = scratch_budget();
    if (arena) {
      const size_t tail = 4 * kAlign + align_up(sizeof(int32_t) * nprob) + 2 * align_up(sizeof(int64_t) * ntot);
      const size_t fr = arena_free(W) > tail ? arena_free(W) - tail : 0;
      const size_t sb = (size_t)stride * sizeof(double);
      const size_t stneed = act.empty() ? 0 : align_up((size_t)maxper * sizeof(double)) + kAlign;
      if (fr < stneed + (nchunks > 0 ? sb + kAlign : 0))
        return fail(MRRR_ERR_CAPACITY, "workspace of %zu bytes too small for the eigenvector scratch", W.acap);
      // the checkpointing kernel takes up to half of what is left (at least
      // one chunk's checkpoints), the stored-vector kernel the rest
      size_t ck = 0;
      if (nchunks > 0) {
        const size_t cap = fr - stneed - kAlign;
        const size_t want = act.empty() ? cap : std::min(cap, std::max(sb, fr / 2));
        ck = std::min<size_t>((size_t)nchunks, std::max<size_t>(1, want / sb)) * sb;
      }
      ckbudget = ck;
      sbudget = fr - (ck ? align_up(ck) + kAlign : 0);
    }
    // batches of chunks whose scratch fits the budget; offsets relative to
    // the scratch base, which every batch reuses
    const size_t budget = std::max(sbudget, (size_t)maxper * sizeof(double));
    std::vector<int64_t> aoff(act.size());
    std::vector<size_t> bstart_h{0};
    int64_t used = 0, used_max = 0;
    for (size_t i = 0; i < act.size(); ++i) {
      const int64_t need = 4 * vslots * (int64_t)rows[act[i]];
      if ((size_t)(used + need) * sizeof(double) > budget && i > bstart_h.back()) {
        bstart_h.push_back(i);
        used = 0;
      }
      aoff[i] = used;
      used += need;
      used_max = std::max(used_max, used);
    }
    bstart_h.push_back(act.size());
    ENS(chunks, sizeof(int32_t) * (act.size() + 1));
    ENS(chunkoff, sizeof(int64_t) * (act.size() + 1));
    if (!act.empty()) {
      ENS(scratch, sizeof(double) * (size_t)used_max);
      HIP_TRY(hipMemcpyAsync(W.chunks.p, act.data(), sizeof(int32_t) * act.size(), hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(W.chunkoff.p, aoff.data(), sizeof(int64_t) * act.size(), hipMemcpyHostToDevice, st));
    }
    const int64_t cmax = std::max<int64_t>(
        1, (int64_t)(std::max(ckbudget, (size_t)stride * sizeof(double)) / (sizeof(double) * (size_t)stride)));
    if (nchunks > 0) ENS(ckscratch, sizeof(double) * (size_t)(std::min<int64_t>(nchunks, cmax) * stride));
    HIP_TRY(hipStreamSynchronize(st));  // the uploads have read the host vectors
    bool forked = false;
    if (nchunks > 0 && W.no_fork) {
      prof.begin(MRRR_K_VECTORS_CKPT);
      for (int64_t c0 = 0; c0 < nchunks; c0 += cmax) {
        const int64_t nc = std::min<int64_t>(cmax, nchunks - c0);
        launch_vectors(st, dP, dB, P_<Node>(W.nodes), P_<int64_t>(W.cstart) + c0, (int)nc, ntot, P_<int32_t>(W.vrid),
                       P_<int32_t>(W.sblk), P_<int32_t>(W.snode), P_<int64_t>(W.scol), P_<double>(W.lo),
                       P_<double>(W.hi), P_<double>(W.sgap), dpool, P_<double>(W.ds), P_<double>(W.ckscratch),
                       stride, w, Z, dC, vslots);
      }
      prof.end();
    } else if (nchunks > 0) {
      if (!W.aux) HIP_TRY(hipStreamCreateWithFlags(&W.aux, hipStreamNonBlocking));
      if (!W.ev_fork) HIP_TRY(hipEventCreateWithFlags(&W.ev_fork, hipEventDisableTiming));
      if (!W.ev_join) HIP_TRY(hipEventCreateWithFlags(&W.ev_join, hipEventDisableTiming));
      HIP_TRY(hipEventRecord(W.ev_fork, st));
      HIP_TRY(hipStreamWaitEvent(W.aux, W.ev_fork, 0));
      forked = true;
      prof.begin_on(MRRR_K_VECTORS_CKPT, W.aux);
      for (int64_t c0 = 0; c0 < nchunks; c0 += cmax) {
        const int64_t nc = std::min<int64_t>(cmax, nchunks - c0);
        launch_vectors(W.aux, dP, dB, P_<Node>(W.nodes), P_<int64_t>(W.cstart) + c0, (int)nc, ntot,
                       P_<int32_t>(W.vrid), P_<int32_t>(W.sblk), P_<int32_t>(W.snode), P_<int64_t>(W.scol),
                       P_<double>(W.lo), P_<double>(W.hi), P_<double>(W.sgap), dpool, P_<double>(W.ds),
                       P_<double>(W.ckscratch), stride, w, Z, dC, vslots);
      }
      prof.end_on(W.aux);
      HIP_TRY(hipEventRecord(W.ev_join, W.aux));
    }
    for (size_t bi = 0; bi + 1 < bstart_h.size(); ++bi) {
      const size_t i0 = bstart_h[bi], i1 = bstart_h[bi + 1];
      if (i1 == i0) continue;
      prof.begin(MRRR_K_VECTORS);
      launch_vectors_stored(st, dP, dB, P_<Node>(W.nodes), P_<int32_t>(W.chunks) + i0, P_<int64_t>(W.chunkoff) + i0,
                            (int)(i1 - i0), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode), P_<uint32_t>(W.sflag),
                            P_<int64_t>(W.scol), P_<double>(W.lo), P_<double>(W.hi), P_<double>(W.sgap), dpool,
                            P_<double>(W.ds), P_<double>(W.scratch), w, Z, dC, vslots);
      prof.end();
    }
    if (forked) HIP_TRY(hipStreamWaitEvent(st, W.ev_join, 0));
  }
  // 9. ascending order within each problem
  ENS(bad, sizeof(int32_t) * nprob);
  HIP_TRY(hipMemsetAsync(W.bad.p, 0, sizeof(int32_t) * nprob, st));
  launch_check_sorted(st, dP, nprob, w, P_<int32_t>(W.bad), dC);
  Counters hc;
  HIP_TRY(hipMemcpyAsync(&hc, W.counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hc.unsorted) {
    ENS(perm, sizeof(int64_t) * ntot);
    ENS(tmp, sizeof(double) * ntot);
    launch_sort_fix(st, dP, nprob, P_<int32_t>(W.bad), w, P_<int64_t>(W.perm), P_<double>(W.tmp), Z);
  }
  HIP_TRY(hipMemcpyAsync(probs.data(), W.problems.p, sizeof(Problem) * nprob, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&hc, W.counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipGetLastError());
  rep->c = hc;
  rep->ws_bytes = W.abase ? W.aused : W.total_bytes();
  if (prof.on) {
    const double vr = (double)(hc.vec_rows - hc.ckpt_vec_rows), ze = (double)(hc.z_entries - hc.ckpt_z_entries);
    const double work[MRRR_K_COUNT] = {grid_work, 4.0 * (double)hc.sturm_steps, 5.0 * (double)hc.child_steps,
                                       15.0 * vr, 0.0, 15.0 * (double)hc.ckpt_vec_rows};
    const double bytes[MRRR_K_COUNT] = {0.0, 0.0, 32.0 * (double)hc.child_steps, 8.0 * ze, 0.0,
                                        8.0 * (double)hc.ckpt_z_entries};
    for (int k = 0; k < MRRR_K_COUNT; ++k) {
      if (k == MRRR_K_BACKWARD || k == MRRR_K_BACKTRANSFORM || k == MRRR_K_TRIDIAG || k == MRRR_K_GHEP) continue;
      double ms;
      int64_t l;
      prof.total(k, &ms, &l);
      if (l) prof_add(k, l, ms, work[k], bytes[k]);
    }
  }
  if (hc.grid_fail) return fail(MRRR_ERR_HIP, "internal: Sturm grid did not bracket the spectrum");
  if (rep->depth_stop && hc.status == 0) rep->c.status = MRRR_ERR_DEPTH;
  return 0;
#undef ENS
}

static void fill_info(mrrr_info* info, const Problem& p, const Report& r) {
  memset(info, 0, sizeof(*info));
  info->m = p.m;
  info->status = p.status ? p.status : r.c.status;
  info->max_depth = r.c.max_depth;
  info->counters[MRRR_CNT_BLOCKS] = r.nblk;
  info->counters[MRRR_CNT_NODES] = r.nodes;
  info->counters[MRRR_CNT_LEVELS] = r.levels;
  info->counters[MRRR_CNT_STURM_STEPS] = (int64_t)r.c.sturm_steps;
  info->counters[MRRR_CNT_QDS_STEPS] = (int64_t)r.c.qds_steps;
  info->counters[MRRR_CNT_SINGLETONS] = (int64_t)r.c.singletons;
  info->counters[MRRR_CNT_RQI] = (int64_t)r.c.rqi;
  info->counters[MRRR_CNT_FALLBACKS] = (int64_t)r.c.fallbacks;
  info->counters[MRRR_CNT_CHILD_REJECT] = (int64_t)r.c.child_reject;
  info->counters[MRRR_CNT_WORKSPACE_MB] = (int64_t)(r.ws_bytes >> 20);
  info->counters[MRRR_CNT_WAVE_SOLVES] = (int64_t)r.c.wave_solves;
  info->counters[MRRR_CNT_POOL_ROWS] = (int64_t)r.c.pool_used;
  info->counters[MRRR_CNT_AMBIGUOUS_LEFT] = r.ambiguous_left;
  info->counters[MRRR_CNT_WORKSPACE_BYTES] = (int64_t)r.ws_bytes;
}

static_assert(sizeof(mrrr_info) == sizeof(InfoWords), "mrrr_info is stored as 18 words");

static int check_step_args(int64_t n, const double* d, const double* e, mrrr_range range, const double* w,
                           const double* Z, int64_t ldz) {
  if (n < 0) return fail(-1, "n < 0");
  if (n > 0 && !d) return fail(-2, "d is NULL");
  if (n > 1 && !e) return fail(-3, "e is NULL");
  if (range.kind < 0 || range.kind > 2) return fail(-4, "bad range kind");
  if (range.kind == MRRR_INDEX && n > 0 && (range.il < 1 || range.il > range.iu || range.iu > n))
    return fail(-4, "index range must satisfy 1 <= il <= iu <= n");
  if (range.kind == MRRR_VALUE && !(range.vl < range.vu)) return fail(-4, "value range must satisfy vl < vu");
  if (n > 0 && !w) return fail(-5, "w is NULL");
  if (Z && ldz < std::max<int64_t>(1, n)) return fail(-7, "ldz < max(1, n)");
  if (n > INT32_MAX / 8) return fail(-1, "n too large");
  return 0;
}

// one problem; arena (may be NULL): carve every buffer from [work, work +
// work_bytes) instead of the library's workspace
static int step_impl(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z,
                     int64_t ldz, void* work, size_t work_bytes, bool no_fork, mrrr_info* info, hipStream_t stream,
                     double gaptol = 0.0) {
  if (info) memset(info, 0, sizeof(*info));
  if (n == 0) return 0;
  int dev = 0;
  Workspace* W = workspace_for_current_device(&dev);
  if (!W) return fail(MRRR_ERR_NO_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(W->mu);
  std::vector<Problem> probs(1);
  Problem& p = probs[0];
  memset(&p, 0, sizeof(p));
  p.off = 0;
  p.n = n;
  p.zoff = 0;
  p.ldz = Z ? ldz : n;
  p.kind = range.kind;
  p.il = range.il;
  p.iu = range.iu;
  p.vl = range.vl;
  p.vu = range.vu;
  p.gaptol = gaptol;
  Report r;
  int rc;
  if (work) {
    // a workspace of this call only; the library's second stream and events
    // are borrowed for the concurrent eigenvector kernels
    Workspace A;
    A.abase = static_cast<char*>(work);
    A.acap = work_bytes;
    A.no_fork = no_fork;
    A.aux = W->aux;
    A.ev_fork = W->ev_fork;
    A.ev_join = W->ev_join;
    rc = solve(A, probs, d, e, w, Z, stream, &r);
    W->aux = A.aux;
    W->ev_fork = A.ev_fork;
    W->ev_join = A.ev_join;
  } else {
    rc = solve(*W, probs, d, e, w, Z, stream, &r);
  }
  if (rc != 0) return rc;
  if (info) fill_info(info, probs[0], r);
  const int st = probs[0].status ? probs[0].status : r.c.status;
  if (st) fail(st, "%s", mrrr_status_string(st));
  return st;
}

// the per-row buffers of one problem of order n as solve() carves them (nblk
// taken as n), the eigenvector phase's minimum, and the pool and scratch
// allowances of mrrr_workspace_size
static size_t workspace_bytes(int64_t n, int64_t m, bool vectors, const mrrr_tuning& t) {
  const int G = t.grid_density;
  const int vs = t.vec_wave_slots ? t.vec_wave_slots : 32;
  const int64_t nb = n;
  size_t b = 0;
  auto add = [&](size_t x) { b += align_up(std::max<size_t>(x, 1)) + kAlign; };
  add(sizeof(Problem));
  add(sizeof(int64_t) * 2);
  add(sizeof(int32_t) * n);                   // sprob
  add(sizeof(double) * n);                    // ds
  add(sizeof(double) * n);                    // es
  add(sizeof(int32_t) * n);                   // flag
  add(sizeof(int32_t) * n);                   // excl
  add(sizeof(int32_t) * (n / 1024 + 2));      // tiles
  add(sizeof(int32_t) * 4);                   // total
  add(sizeof(Counters));
  add(sizeof(int64_t) * (nb + 1));            // bstart
  add(sizeof(int32_t) * n);                   // sblk
  add(sizeof(Block) * nb);
  add(sizeof(int64_t) * (nb + 1));            // goff
  add(sizeof(Node) * (size_t)(nb + n + 16));  // nodes
  add(sizeof(int32_t) * (size_t)(G * n + nb));  // count grid
  add(sizeof(double) * n * 2);                // lo, hi
  add(sizeof(int32_t) * n * 2);               // clo, chi
  add(sizeof(int32_t) * n);                   // snode
  add(sizeof(uint32_t) * n);                  // sflag
  add(sizeof(int64_t) * n);                   // scol
  add(sizeof(double) * n * 2);                // val, sgap
  add(sizeof(int32_t) * n * 2);               // runflag, runid
  add(sizeof(int64_t) * (n + 1));             // runs
  add(sizeof(int32_t) * n * 3);               // vrid, cflag, cid
  add(sizeof(int64_t) * (n + 1));             // cstart
  if (vectors) add(sizeof(Cluster) * (size_t)(n / 2 + 1));
  // pool: roots, speculative candidates of one level, children
  const size_t rows =
      (size_t)n + (vectors ? (size_t)MRRR_WS_CHILD_ROWS_PER_N * (size_t)n + (size_t)child_ck_rows(n) * 32 : 0);
  add(sizeof(Rep) * rows);
  if (vectors) {
    const int64_t nch = (n + vs - 1) / vs;
    add(sizeof(int32_t) * nch);
    add(sizeof(int32_t) * (nch + 1));
    add(sizeof(int64_t) * (nch + 1));
    // every wanted pair's checkpoints at once (checkpointing kernel) and the
    // stored work vectors of up to 4096 pairs
    add(sizeof(double) * 4 * (size_t)(m + vs) * (size_t)((n + kSeg - 1) / kSeg));
    add(sizeof(double) * 4 * (size_t)std::min<int64_t>(m + vs, 4096) * (size_t)n);
  }
  add(sizeof(int32_t));  // sort check
  add(sizeof(int64_t) * n);
  add(sizeof(double) * n);
  return b;
}

// ---------------------------------------------------------------------------
// the FP32 interface (mrrr_step_f32): FP32 data in and out, the solver in
// FP64 with the classification threshold relaxed to what FP32 results need

__global__ void k_f32_to_f64(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

// y[:, c] = x[:, c] rounded, columns of n rows (leading dimensions ldx, ldy)
__global__ void k_f64_to_f32(int64_t n, int64_t m, const double* __restrict__ x, int64_t ldx, float* __restrict__ y,
                             int64_t ldy) {
  for (int64_t c = blockIdx.y; c < m; c += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      y[c * ldy + i] = (float)x[c * ldx + i];
}

// Relative-gap threshold for FP32 results computed in FP64: a singleton's
// vector leans towards its neighbours by about eps64 / relgap, the pairs
// of a node by about n eps64 / gaptol; with gaptol = 4 n eps64 / eps32 =
// n 2^-27 that stays below eps32 / 4, so singletons may be much closer than
// the FP64 threshold of 1e-3 allows (fewer clusters, a shallower tree).
static double mixed_gaptol(int64_t n) {
  return std::min(kRelgapTol, std::max(1.0, (double)n) * std::ldexp(1.0, -27));
}

static std::mutex g_mixed_mu;
static void* g_mixed = nullptr;
static size_t g_mixed_bytes = 0;
static int g_mixed_dev = -1;

}  // namespace mrrr

using namespace mrrr;

extern "C" {

int mrrr_step(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z, int64_t ldz,
              mrrr_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  int rc = check_step_args(n, d, e, range, w, Z, ldz);
  if (rc != 0) return rc;
  return step_impl(n, d, e, range, w, Z, ldz, nullptr, 0, false, info, (hipStream_t)stream);
}

int mrrr_step_f32(int64_t n, const float* d, const float* e, mrrr_range range, float* w, float* Z, int64_t ldz,
                  mrrr_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
  int rc = check_step_args(n, (const double*)d, (const double*)e, range, (const double*)w, (const double*)Z, ldz);
  if (rc != 0) return rc;
  if (n == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const int64_t mmax = range.kind == MRRR_INDEX ? range.iu - range.il + 1 : n;
  std::lock_guard<std::mutex> lk(g_mixed_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MRRR_ERR_NO_DEVICE, "no HIP device");
  const size_t zb = Z ? sizeof(double) * (size_t)n * (size_t)mmax : 0;
  const size_t need = align_up(sizeof(double) * (size_t)n) * 3 + align_up(std::max<size_t>(zb, 1));
  if (!g_mixed || g_mixed_bytes < need || g_mixed_dev != dev) {
    if (g_mixed) {
      (void)hipDeviceSynchronize();
      (void)hipFree(g_mixed);
    }
    g_mixed = nullptr;
    g_mixed_bytes = 0;
    if (hipMalloc(&g_mixed, need) != hipSuccess) return fail(MRRR_ERR_CAPACITY, "hipMalloc failed for the FP32 interface");
    g_mixed_bytes = need;
    g_mixed_dev = dev;
  }
  char* base = (char*)g_mixed;
  double* d64 = (double*)base;
  double* e64 = (double*)(base + align_up(sizeof(double) * (size_t)n));
  double* w64 = (double*)(base + 2 * align_up(sizeof(double) * (size_t)n));
  double* Z64 = Z ? (double*)(base + 3 * align_up(sizeof(double) * (size_t)n)) : nullptr;
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_f32_to_f64, dim3(g), dim3(256), 0, st, n, d, d64);
  if (n > 1) hipLaunchKernelGGL(k_f32_to_f64, dim3(g), dim3(256), 0, st, n - 1, e, e64);
  mrrr_info inf;
  rc = step_impl(n, d64, e64, range, w64, Z64, n, nullptr, 0, false, &inf, st, mixed_gaptol(n));
  if (info) *info = inf;
  if (rc < 0) return rc;
  const int64_t m = inf.m;
  if (m > 0) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 65535), 1), dim3(256), 0, st,
                       m, (int64_t)1, (const double*)w64, m, w, m);
    if (Z)
      hipLaunchKernelGGL(k_f64_to_f32,
                         dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), (unsigned)std::min<int64_t>(m, 65535)),
                         dim3(256), 0, st, n, m, (const double*)Z64, n, Z, ldz);
  }
  hipError_t er = hipStreamSynchronize(st);
  if (er == hipSuccess) er = hipGetLastError();
  if (er != hipSuccess) return fail(MRRR_ERR_HIP, "FP32 conversion failed: %s", hipGetErrorString(er));
  return rc;
}

size_t mrrr_workspace_size(int64_t n, mrrr_range range) {
  if (n < 0 || n > INT32_MAX / 8 || range.kind < 0 || range.kind > 2) return 0;
  if (range.kind == MRRR_INDEX && n > 0 && (range.il < 1 || range.il > range.iu || range.iu > n)) return 0;
  if (n == 0) return kAlign;
  mrrr_tuning t;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    t = g_tune;
  }
  const int64_t m = range.kind == MRRR_INDEX ? range.iu - range.il + 1 : n;
  return workspace_bytes(n, m, true, t);
}

int mrrr_step_ws(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z, int64_t ldz,
                 void* work, size_t work_bytes, mrrr_info* info_dev, void* stream) {
  int rc = check_step_args(n, d, e, range, w, Z, ldz);
  if (rc != 0) return rc;
  if (work && work_bytes < kAlign) return fail(-9, "work_bytes too small");
  mrrr_info info;
  rc = step_impl(n, d, e, range, w, Z, ldz, work, work_bytes, false, &info, (hipStream_t)stream);
  if (rc < 0) return rc;
  if (info_dev) {
    if (rc != 0 && info.status == 0) info.status = rc;
    launch_store_info(reinterpret_cast<InfoWords*>(info_dev), *reinterpret_cast<const InfoWords*>(&info),
                      (hipStream_t)stream);
    const hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return fail(MRRR_ERR_HIP, "info store failed: %s", hipGetErrorString(e2));
  }
  return rc;
}

int mrrr_probe_division(int64_t n, const double* a, const double* b, double* out, void* stream) {
  if (n < 0 || n > ((int64_t)1 << 31)) return fail(-1, "n out of range");
  if (n == 0) return 0;
  if (!a || !b || !out) return fail(-2, "null pointer");
  launch_probe_division((hipStream_t)stream, n, a, b, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MRRR_ERR_HIP, "probe launch failed: %s", hipGetErrorString(e));
  return 0;
}

int mrrr_get_limits(mrrr_limits* l) {
  if (!l) return -1;
  std::lock_guard<std::mutex> lk(g_limits_mu);
  *l = g_limits;
  return 0;
}

int mrrr_set_limits(const mrrr_limits* l) {
  if (!l) return -1;
  if (l->max_depth < 1 || l->max_depth > kMaxDepth) return -1;
  if (!(l->child_growth_limit >= 0.0) || !std::isfinite(l->child_growth_limit)) return -1;
  std::lock_guard<std::mutex> lk(g_limits_mu);
  g_limits = *l;
  return 0;
}

// ---------------------------------------------------------------------------
// tuning cache of the batched form, keyed by the batch's size histogram
// (problem counts per power-of-two size class, each count rounded to a power
// of two)

static std::mutex g_cache_mu;
static std::map<uint64_t, mrrr_tuning> g_cache;

static uint64_t size_key(int64_t batch, const int64_t* n_host) {
  int64_t hist[64] = {0};
  for (int64_t b = 0; b < batch; ++b) {
    int c = 0;
    for (int64_t v = n_host[b]; v > 1; v >>= 1) ++c;
    hist[c]++;
  }
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  for (int c = 0; c < 64; ++c) {
    int q = 0;
    for (int64_t v = hist[c]; v > 0; v >>= 1) ++q;
    h = (h ^ (uint64_t)(c * 64 + q)) * 1099511628211ull;
  }
  return h;
}

static bool cache_lookup(uint64_t key, mrrr_tuning* t) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *t = it->second;
  return true;
}

int mrrr_step_batched(int64_t batch, const int64_t* n_host, const int64_t* off_host, const double* d,
                      const double* e, double* w, double* Z, const int64_t* zoff_host, mrrr_info* info,
                      void* stream) {
  if (batch < 0) return fail(-1, "batch < 0");
  if (batch == 0) return 0;
  if (!n_host) return fail(-2, "n_host is NULL");
  if (!off_host) return fail(-3, "off_host is NULL");
  if (!d) return fail(-4, "d is NULL");
  if (!e) return fail(-5, "e is NULL");
  if (!w) return fail(-6, "w is NULL");
  if (Z && !zoff_host) return fail(-8, "zoff_host is NULL");
  int64_t tot = 0;
  for (int64_t b = 0; b < batch; ++b) {
    if (n_host[b] < 1 || n_host[b] > INT32_MAX / 8) return fail(-2, "n_host[%lld] out of range", (long long)b);
    if (off_host[b] < 0) return fail(-3, "off_host[%lld] < 0", (long long)b);
    tot += n_host[b];
  }
  if (tot > INT32_MAX / 2) return fail(-2, "total order too large");
  int dev = 0;
  Workspace* W = workspace_for_current_device(&dev);
  if (!W) return fail(MRRR_ERR_NO_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(W->mu);
  std::vector<Problem> probs(batch);
  for (int64_t b = 0; b < batch; ++b) {
    Problem& p = probs[b];
    memset(&p, 0, sizeof(p));
    p.off = off_host[b];
    p.n = n_host[b];
    p.zoff = Z ? zoff_host[b] : 0;
    p.ldz = n_host[b];
    p.kind = MRRR_ALL;
  }
  Report r;
  mrrr_tuning cached;
  const bool have = cache_lookup(size_key(batch, n_host), &cached);
  int rc = solve(*W, probs, d, e, w, Z, (hipStream_t)stream, &r, have ? &cached : nullptr);
  if (rc != 0) return rc;
  int st = 0;
  for (int64_t b = 0; b < batch; ++b) {
    if (info) fill_info(&info[b], probs[b], r);
    if (!st && probs[b].status) st = probs[b].status;
  }
  if (!st) st = r.c.status;
  if (st) fail(st, "%s", mrrr_status_string(st));
  return st;
}

// coordinate search over the launch shapes: eigenvectors per wavefront,
// eigenvalues per refinement wavefront, count-grid density; each candidate is
// timed (host clock around a whole synchronised solve) on the caller's batch
int mrrr_autotune_batched(int64_t batch, const int64_t* n_host, const int64_t* off_host, const double* d,
                          const double* e, double* w, double* Z, const int64_t* zoff_host, mrrr_tuning* best,
                          void* stream) {
  if (batch < 1) return fail(-1, "batch < 1");
  if (!n_host) return fail(-2, "n_host is NULL");
  if (!off_host) return fail(-3, "off_host is NULL");
  if (!d) return fail(-4, "d is NULL");
  if (!e) return fail(-5, "e is NULL");
  if (!w) return fail(-6, "w is NULL");
  if (Z && !zoff_host) return fail(-8, "zoff_host is NULL");
  int64_t tot = 0;
  for (int64_t b = 0; b < batch; ++b) {
    if (n_host[b] < 1 || n_host[b] > INT32_MAX / 8) return fail(-2, "n_host[%lld] out of range", (long long)b);
    if (off_host[b] < 0) return fail(-3, "off_host[%lld] < 0", (long long)b);
    tot += n_host[b];
  }
  if (tot > INT32_MAX / 2) return fail(-2, "total order too large");
  int dev = 0;
  Workspace* W = workspace_for_current_device(&dev);
  if (!W) return fail(MRRR_ERR_NO_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(W->mu);
  std::vector<Problem> tmpl(batch);
  for (int64_t b = 0; b < batch; ++b) {
    Problem& p = tmpl[b];
    memset(&p, 0, sizeof(p));
    p.off = off_host[b];
    p.n = n_host[b];
    p.zoff = Z ? zoff_host[b] : 0;
    p.ldz = n_host[b];
    p.kind = MRRR_ALL;
  }
  auto run = [&](const mrrr_tuning& t, double* ms) -> int {
    std::vector<Problem> probs = tmpl;
    Report r;
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = solve(*W, probs, d, e, w, Z, (hipStream_t)stream, &r, &t);
    const auto t1 = std::chrono::steady_clock::now();
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return rc;
  };
  mrrr_tuning cur;
  {
    std::lock_guard<std::mutex> lk2(g_tune_mu);
    cur = g_tune;
  }
  if (cur.refine_wave_slots == 0) cur.refine_wave_slots = (tot <= 32768) ? 16 : (tot <= 131072 ? 32 : 64);
  if (cur.vec_wave_slots == 0) cur.vec_wave_slots = 32;
  if (cur.vec_ckpt_min_run == 0) cur.vec_ckpt_min_run = kCkptMinRun;
  double best_ms = 0.0;
  int rc = run(cur, &best_ms);  // grows the workspace
  if (rc != 0) return rc;
  if ((rc = run(cur, &best_ms)) != 0) return rc;
  const int vec_c[] = {32, 16, 8};
  const int ref_c[] = {16, 32, 64};
  const int grid_c[] = {2, 4, 8};
  const int run_c[] = {16, 8, 4};  // equal-node run length for the checkpointing eigenvector kernel
  for (int param = 0; param < 4; ++param) {
    const int* cand = param == 0 ? vec_c : (param == 1 ? ref_c : (param == 2 ? grid_c : run_c));
    for (int k = 0; k < 3; ++k) {
      mrrr_tuning t = cur;
      int* field = param == 0   ? &t.vec_wave_slots
                   : param == 1 ? &t.refine_wave_slots
                   : param == 2 ? &t.grid_density
                                : &t.vec_ckpt_min_run;
      if (*field == cand[k]) continue;
      *field = cand[k];
      double ms = 0.0;
      if ((rc = run(t, &ms)) != 0) return rc;
      if (ms < best_ms) {
        best_ms = ms;
        cur = t;
      }
    }
  }
  {
    std::lock_guard<std::mutex> lk3(g_cache_mu);
    g_cache[size_key(batch, n_host)] = cur;
  }
  if (best) *best = cur;
  return 0;
}

int mrrr_get_tuning(mrrr_tuning* t) {
  if (!t) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *t = g_tune;
  return 0;
}

int mrrr_set_tuning(const mrrr_tuning* t) {
  if (!t) return -1;
  if (t->grid_density < 1 || t->grid_density > 16) return -1;
  if (!(t->refine_wave_slots == 0 || t->refine_wave_slots == 16 || t->refine_wave_slots == 32 ||
        t->refine_wave_slots == 64))
    return -1;
  if (!(t->vec_wave_slots == 0 || t->vec_wave_slots == 8 || t->vec_wave_slots == 16 || t->vec_wave_slots == 32))
    return -1;
  if (t->vec_ckpt_min_run < -1 || t->vec_ckpt_min_run > (1 << 30)) return -1;
  if (t->vec_ckpt_min_n != 0 && (t->vec_ckpt_min_n < 64 || t->vec_ckpt_min_n > (1 << 30))) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = *t;
  return 0;
}

int mrrr_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return 0;
}

int mrrr_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  memset(g_prof, 0, sizeof(g_prof));
  return 0;
}

int mrrr_profile_read(int kernel, mrrr_kernel_time* out) {
  if (kernel < 0 || kernel >= MRRR_K_COUNT || !out) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  *out = g_prof[kernel];
  return 0;
}

int mrrr_release(void) {
  int dev = 0;
  Workspace* W = workspace_for_current_device(&dev);
  if (!W) return fail(MRRR_ERR_NO_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(W->mu);
  W->release();
  return 0;
}

const char* mrrr_last_error(void) { return g_err.c_str(); }

const char* mrrr_status_string(int code) {
  switch (code) {
    case MRRR_OK: return "ok";
    case MRRR_ERR_NO_RRR: return "no child representation with finite entries";
    case MRRR_ERR_DEPTH: return "representation tree deeper than 64 levels";
    case MRRR_ERR_CAPACITY: return "workspace capacity exhausted";
    case MRRR_ERR_NONFINITE: return "non-finite entry in d or e";
    case MRRR_ERR_HIP: return "HIP runtime error";
    case MRRR_ERR_NO_DEVICE: return "no usable device";
    default: return code < 0 ? "invalid argument" : "unknown status";
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free entry point: the workspace is a file-scope device array.  In
// host code the array's name is only a host-side stand-in; its device address
// on each GPU is taken once, with that device current, by hipGetSymbolAddress,
// and only that address is passed to the solver.

namespace mrrr {

static __device__ __align__(256) unsigned char scratch[MRRR_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static std::map<int, void*> g_noalloc_ptr;

// device address of `scratch` on the current device (set up on the first call
// on each device)
static int noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(MRRR_ERR_NO_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(dev);
  if (it == g_noalloc_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(MRRR_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    it = g_noalloc_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return 0;
}

}  // namespace mrrr

extern "C" int mrrr_step_noalloc(int64_t n, const double* d, const double* e, mrrr_range range, double* w,
                                 double* Z, int64_t ldz, mrrr_info* info_dev, void* stream) {
  int rc = check_step_args(n, d, e, range, w, Z, ldz);
  if (rc != 0) return rc;
  if (n > MRRR_NOALLOC_MAX_N)
    return fail(-1, "n = %lld exceeds the allocation-free limit of %d rows", (long long)n, MRRR_NOALLOC_MAX_N);
  void* ptr = nullptr;
  if (n > 0 && (rc = noalloc_scratch(&ptr)) != 0) return rc;
  mrrr_info info;
  // one stream (no second stream for the eigenvector kernels), every buffer
  // carved from the array
  rc = step_impl(n, d, e, range, w, Z, ldz, ptr, MRRR_NOALLOC_SCRATCH_BYTES, true, &info, (hipStream_t)stream);
  if (rc < 0) return rc;
  if (info_dev) {
    if (rc != 0 && info.status == 0) info.status = rc;
    launch_store_info(reinterpret_cast<InfoWords*>(info_dev), *reinterpret_cast<const InfoWords*>(&info),
                      (hipStream_t)stream);
    const hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return fail(MRRR_ERR_HIP, "info store failed: %s", hipGetErrorString(e2));
  }
  return rc;
}
