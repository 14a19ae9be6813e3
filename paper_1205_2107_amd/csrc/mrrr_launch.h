// Host-callable launch wrappers of the solver kernels (defined in mrrr_kernels.hip).
#pragma once
#include "mrrr_dev.h"

namespace mrrr {

void launch_prep(hipStream_t st, Problem* P, int nprob, const int64_t* poff, int64_t ntot, const double* d,
                 const double* e, int32_t* sprob, double* ds, double* es, int32_t* flag);
void launch_scan(hipStream_t st, const int32_t* in, int32_t* out, int32_t* tile_sum, int64_t n, int32_t* total);
void launch_blocks(hipStream_t st, Problem* P, const int64_t* poff, const int32_t* flag, const int32_t* excl,
                   int64_t ntot, int nblk, const int32_t* sprob, int64_t* bstart, int32_t* sblk, Block* B);
void launch_root(hipStream_t st, Problem* P, Block* B, Node* N, int nblk, const double* ds, const double* es,
                 Rep* pool, Counters* C, int grid_density);
void launch_grid(hipStream_t st, const Block* B, int nblk, const int64_t* goff, int64_t gtot, const Rep* pool,
                 int32_t* gcnt);
void launch_assign(hipStream_t st, const Block* B, const int64_t* goff, int64_t ntot, const int32_t* sblk,
                   const int32_t* gcnt, double* lo, double* hi, int32_t* clo, int32_t* chi, int32_t* snode,
                   uint32_t* sflag, Counters* C);
void launch_refine(hipStream_t st, const Block* B, const Node* N, int64_t ntot, const int32_t* sblk,
                   const int32_t* snode, const Rep* pool, double* lo, double* hi, int32_t* clo, int32_t* chi,
                   uint32_t* sflag, Counters* C, int lanes, bool validate_only = false,
                   const int64_t* cstart = nullptr, const int32_t* rid = nullptr, int nchunks = 0,
                   bool share = false);
void launch_mark_leaf(hipStream_t st, int64_t ntot, const int64_t* scol, uint32_t* sflag);
void launch_columns(hipStream_t st, const Problem* P, Block* B, int nblk, const Node* N, int64_t ntot,
                    const int32_t* sblk, const double* lo, const double* hi, double* val, int64_t* scol, bool multi);
void launch_cls_flags(hipStream_t st, const Block* B, const Node* N, int64_t ntot, const int32_t* sblk,
                      const int32_t* snode, const double* lo, const double* hi, uint32_t* sflag, int32_t* runflag,
                      Counters* C);
void launch_cls_compact(hipStream_t st, int64_t ntot, const int32_t* runflag, const int32_t* runid, int64_t* runs);
void launch_cls_runs(hipStream_t st, const Block* B, const Node* N, int nruns, const int64_t* runs,
                     const int32_t* sblk, const int32_t* snode, const double* lo, const double* hi,
                     const int64_t* scol, uint32_t* sflag, double* sgap, Cluster* clusters, int max_clusters,
                     Counters* C, int max_depth);
void launch_child(hipStream_t st, const Block* B, Node* N, int nclusters, int node_base, const Cluster* clusters,
                  const double* lo, const double* hi, Rep* pool, unsigned long long pool_cap, Counters* C,
                  double growth_limit);
void launch_shift(hipStream_t st, const Block* B, const Node* N, int nclusters, int node_base,
                  const Cluster* clusters, const int64_t* scol, double* lo, double* hi, int32_t* clo, int32_t* chi,
                  int32_t* snode, uint32_t* sflag, double* sgap);
void launch_clear_active(hipStream_t st, int64_t ntot, uint32_t* sflag);
void launch_node_chunks(hipStream_t st, int64_t ntot, const uint32_t* sflag, const int64_t* scol, uint32_t need,
                        bool need_col, const int32_t* snode, int slots, int32_t* runflag, int32_t* runid,
                        int32_t* tiles, int32_t* total, int32_t* rid, int64_t* rstart, int32_t* cflag, int32_t* cid,
                        int64_t* cstart);
void launch_vectors(hipStream_t st, const Problem* P, const Block* B, const Node* N, const int64_t* cstart,
                    int nchunks, int64_t ntot, const int32_t* rid, const int32_t* sblk, const int32_t* snode,
                    const int64_t* scol, const double* lo, const double* hi, const double* sgap, const Rep* pool,
                    const double* ds, double* scratch, int64_t stride, double* w, double* Z, Counters* C, int slots);
void launch_vectors_stored(hipStream_t st, const Problem* P, const Block* B, const Node* N, const int32_t* chunks,
                           const int64_t* chunk_off, int nchunks, int64_t ntot, const int32_t* sblk,
                           const int32_t* snode, const uint32_t* sflag, const int64_t* scol, const double* lo,
                           const double* hi, const double* sgap, const Rep* pool, const double* ds, double* scratch,
                           double* w, double* Z, Counters* C, int slots);
void launch_chunk_rows(hipStream_t st, const Block* B, int64_t ntot, const int32_t* sblk, const uint32_t* sflag,
                       const int64_t* scol, int slots, int32_t* rows);
void launch_mark_ckpt(hipStream_t st, int64_t ntot, const Block* B, const int32_t* sblk, const int32_t* rid,
                      const int64_t* rstart, int min_run, int min_n, uint32_t* sflag);
void launch_check_sorted(hipStream_t st, const Problem* P, int nprob, const double* w, int32_t* bad, Counters* C);
void launch_sort_fix(hipStream_t st, const Problem* P, int nprob, const int32_t* bad, double* w, int64_t* perm,
                     double* tmp, double* Z);
void launch_values_only(hipStream_t st, const Problem* P, const Block* B, const Node* N, int64_t ntot,
                        const int32_t* sblk, const int32_t* snode, const int64_t* scol, const double* lo,
                        const double* hi, const double* ds, double* w);

// the report of a call (mrrr_info, 18 words) stored to device memory by a
// kernel that takes it by value
struct InfoWords {
  int64_t w[18];
};
void launch_refine_fill(hipStream_t st, const Block* B, const Node* N, int64_t ntot, const int32_t* sblk,
                        const int32_t* snode, const Rep* pool, double* lo, double* hi, int32_t* clo, int32_t* chi,
                        uint32_t* sflag, Counters* C, int lanes, const int64_t* cstart, const int32_t* rid,
                        const int64_t* rstart, int nchunks, int32_t* claim, int32_t* cursor, int max_waves);
int device_simds();
void launch_probe_division(hipStream_t st, int64_t n, const double* a, const double* b, double* out);
void launch_store_info(InfoWords* dst, InfoWords v, hipStream_t st);

}  // namespace mrrr
