// Host runtime and C ABI of the MI355X MRRR solver: workspace management, the
// level-by-level drive of the representation tree, argument checking.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// grow-only device buffer; contents are not preserved unless keep is set
static int ensure(DevBuf& b, size_t bytes, hipStream_t st, bool keep = false) {
  if (bytes <= b.bytes && b.p) return 0;
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
};

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
#define ENS(buf, bytes)                                          \
  do {                                                           \
    if ((rc = ensure(W.buf, (size_t)(bytes), st)) != 0) return rc; \
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
  ENS(bstart, sizeof(int64_t) * (nblk + 1));
  ENS(sblk, sizeof(int32_t) * ntot);
  ENS(blocks, sizeof(Block) * nblk);
  ENS(goff, sizeof(int64_t) * (nblk + 1));
  // node table: roots first; grows per level
  ENS(nodes, sizeof(Node) * (size_t)std::max<int64_t>(nblk + 16, 2 * (int64_t)nblk));
  // pool: roots aligned with slots plus room for children (grown on demand)
  size_t pool_rows = (size_t)ntot + (size_t)std::max<int64_t>(4 * 1024, ntot / 2);
  if (W.pool.bytes / sizeof(Rep) > pool_rows) pool_rows = W.pool.bytes / sizeof(Rep);
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
  ENS(vrid, sizeof(int32_t) * ntot);
  ENS(cflag, sizeof(int32_t) * ntot);
  ENS(cid, sizeof(int32_t) * ntot);
  ENS(cstart, sizeof(int64_t) * (ntot + 1));
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
  prof.begin(MRRR_K_REFINE);
  launch_refine(st, dB, P_<Node>(W.nodes), ntot, P_<int32_t>(W.sblk), P_<int32_t>(W.snode), dpool, P_<double>(W.lo),
                P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi), P_<uint32_t>(W.sflag), dC, lanes);
  prof.end();
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
    int64_t nmax_prob = 1;
    for (auto& p : probs) nmax_prob = std::max<int64_t>(nmax_prob, p.n);
    int max_clusters = (int)std::min<int64_t>(ntot / 2 + 1, INT32_MAX / 2);
    ENS(clusters, sizeof(Cluster) * (size_t)max_clusters);
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
        if (amb == 0 || round >= 3) break;
        if ((rc = refine_flagged(false, kShareLevels)) != 0) return rc;
      }
      launch_cls_compact(st, ntot, P_<int32_t>(W.runflag), P_<int32_t>(W.runid), P_<int64_t>(W.runs));
      launch_cls_runs(st, dB, P_<Node>(W.nodes), nruns, P_<int64_t>(W.runs), P_<int32_t>(W.sblk),
                      P_<int32_t>(W.snode), P_<double>(W.lo), P_<double>(W.hi), P_<int64_t>(W.scol),
                      P_<uint32_t>(W.sflag), P_<double>(W.sgap), P_<Cluster>(W.clusters), max_clusters, dC);
      launch_clear_active(st, ntot, P_<uint32_t>(W.sflag));
      Counters hc;
      HIP_TRY(hipMemcpyAsync(&hc, W.counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipGetLastError());
      rep->levels = level + 1;
      const int ncl = std::min(hc.nclusters, max_clusters);
      if (ncl == 0) break;
      // capacity for the new nodes and the speculative child regions of every
      // cluster (two with masked stores, four in the branch-free form, every
      // candidate's when the regions stay small: no second pass)
      if ((rc = ensure(W.nodes, sizeof(Node) * (size_t)(node_base + ncl), st, true)) != 0) return rc;
      const bool masked = ncl >= kChildMaskedFrom || nmax_prob >= kChildFewMaxN;
      const bool all = !masked && nmax_prob < kChildAllMaxN &&
                       (size_t)kChildSpecAll * (size_t)hc.cluster_rows <= (size_t)kChildAllMaxRows;
      const int spec = masked ? kChildSpecMany : (all ? kChildSpecAll : kChildSpecFew);
      const size_t need_rows = (size_t)hc.pool_used + (size_t)ntot + (size_t)spec * (size_t)hc.cluster_rows;
      if (need_rows * sizeof(Rep) > W.pool.bytes) {
        if ((rc = ensure(W.pool, need_rows * sizeof(Rep) + (W.pool.bytes / 2), st, true)) != 0) return rc;
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
                   P_<double>(W.hi), dpool, pool_cap, dC, spec);
      prof.end();
      launch_shift(st, dB, P_<Node>(W.nodes), ncl, node_base, P_<Cluster>(W.clusters), P_<int64_t>(W.scol),
                   P_<double>(W.lo), P_<double>(W.hi), P_<int32_t>(W.clo), P_<int32_t>(W.chi),
                   P_<int32_t>(W.snode), P_<uint32_t>(W.sflag), P_<double>(W.sgap));
      HIP_TRY(hipMemsetAsync((char*)W.counters.p + offsetof(Counters, nclusters), 0, sizeof(int32_t), st));
      HIP_TRY(hipMemsetAsync((char*)W.counters.p + offsetof(Counters, cluster_rows), 0, sizeof(unsigned long long),
                             st));
      node_base += ncl;
      if (level > kMaxDepth + 2) break;
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
    int vslots = tune.vec_wave_slots;
    if (vslots == 0) vslots = 32;
    ENS(vrid, sizeof(int32_t) * ntot);
    ENS(cflag, sizeof(int32_t) * ntot);
    ENS(cid, sizeof(int32_t) * ntot);
    ENS(cstart, sizeof(int64_t) * (ntot + 1));
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
    const int64_t nch = (ntot + vslots - 1) / vslots;
    ENS(chunkrows, sizeof(int32_t) * nch);
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
    // batches of chunks whose scratch fits the budget; offsets relative to
    // the scratch base, which every batch reuses
    const size_t budget = std::max(scratch_budget(), (size_t)maxper * sizeof(double));
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
    const size_t ckbudget = std::max(scratch_budget(), (size_t)stride * sizeof(double));
    const int64_t cmax = std::max<int64_t>(1, (int64_t)(ckbudget / (sizeof(double) * (size_t)stride)));
    if (nchunks > 0) ENS(ckscratch, sizeof(double) * (size_t)(std::min<int64_t>(nchunks, cmax) * stride));
    HIP_TRY(hipStreamSynchronize(st));  // the uploads have read the host vectors
    bool forked = false;
    if (nchunks > 0) {
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
  rep->ws_bytes = W.total_bytes();
  // diagnostics: MRRR_DEBUG_DUMP=<file> writes the per-slot tree state
  if (const char* path = getenv("MRRR_DEBUG_DUMP")) {
    const int nnodes = nblk + rep->nodes;
    std::vector<int32_t> hn(ntot);
    std::vector<uint32_t> hf(ntot);
    std::vector<double> hl(ntot), hh(ntot), hg(ntot);
    std::vector<Node> nodes(nnodes);
    HIP_TRY(hipMemcpy(hg.data(), W.sgap.p, sizeof(double) * ntot, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hn.data(), W.snode.p, sizeof(int32_t) * ntot, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hf.data(), W.sflag.p, sizeof(uint32_t) * ntot, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hl.data(), W.lo.p, sizeof(double) * ntot, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hh.data(), W.hi.p, sizeof(double) * ntot, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(nodes.data(), W.nodes.p, sizeof(Node) * nnodes, hipMemcpyDeviceToHost));
    if (FILE* f = fopen(path, "wb")) {
      const int64_t hdr[3] = {ntot, nnodes, (int64_t)sizeof(Node)};
      fwrite(hdr, sizeof(hdr), 1, f);
      fwrite(hn.data(), sizeof(int32_t), ntot, f);
      fwrite(hf.data(), sizeof(uint32_t), ntot, f);
      fwrite(hl.data(), sizeof(double), ntot, f);
      fwrite(hh.data(), sizeof(double), ntot, f);
      fwrite(nodes.data(), sizeof(Node), nnodes, f);
      fwrite(hg.data(), sizeof(double), ntot, f);
      // representation rows (D, L, LD, LLD) of the leaf nodes of the slots
      // listed in MRRR_DEBUG_DUMP_SLOTS (comma separated)
      std::vector<int> want;
      if (const char* nl = getenv("MRRR_DEBUG_DUMP_SLOTS")) {
        for (const char* q = nl; *q;) {
          const long long sl = atoll(q);
          if (sl >= 0 && sl < ntot) want.push_back(hn[sl]);
          while (*q && *q != ',') ++q;
          if (*q == ',') ++q;
        }
      }
      std::sort(want.begin(), want.end());
      want.erase(std::unique(want.begin(), want.end()), want.end());
      for (int k : want) {
        if (k < 0 || k >= nnodes || nodes[k].rep < 0) continue;
        Block hb;
        HIP_TRY(hipMemcpy(&hb, (Block*)W.blocks.p + nodes[k].blk, sizeof(Block), hipMemcpyDeviceToHost));
        std::vector<Rep> rows(hb.n);
        HIP_TRY(hipMemcpy(rows.data(), (Rep*)W.pool.p + nodes[k].rep, sizeof(Rep) * hb.n, hipMemcpyDeviceToHost));
        const int64_t h2[2] = {k, hb.n};
        fwrite(h2, sizeof(h2), 1, f);
        fwrite(rows.data(), sizeof(Rep), hb.n, f);
      }
      fclose(f);
    }
  }
  if (prof.on) {
    const double vr = (double)(hc.vec_rows - hc.ckpt_vec_rows), ze = (double)(hc.z_entries - hc.ckpt_z_entries);
    const double work[MRRR_K_COUNT] = {grid_work, 4.0 * (double)hc.sturm_steps, 5.0 * (double)hc.child_steps,
                                       15.0 * vr, 0.0, 15.0 * (double)hc.ckpt_vec_rows};
    const double bytes[MRRR_K_COUNT] = {0.0, 0.0, 32.0 * (double)hc.child_steps, 8.0 * ze, 0.0,
                                        8.0 * (double)hc.ckpt_z_entries};
    for (int k = 0; k < MRRR_K_COUNT; ++k) {
      if (k == MRRR_K_BACKWARD) continue;
      double ms;
      int64_t l;
      prof.total(k, &ms, &l);
      if (l) prof_add(k, l, ms, work[k], bytes[k]);
    }
  }
  if (hc.grid_fail) return fail(MRRR_ERR_HIP, "internal: Sturm grid did not bracket the spectrum");
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
}

}  // namespace mrrr

using namespace mrrr;

extern "C" {

int mrrr_step(int64_t n, const double* d, const double* e, mrrr_range range, double* w, double* Z, int64_t ldz,
              mrrr_info* info, void* stream) {
  if (info) memset(info, 0, sizeof(*info));
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
  Report r;
  int rc = solve(*W, probs, d, e, w, Z, (hipStream_t)stream, &r);
  if (rc != 0) return rc;
  if (info) fill_info(info, probs[0], r);
  const int st = probs[0].status ? probs[0].status : r.c.status;
  if (st) fail(st, "%s", mrrr_status_string(st));
  return st;
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
