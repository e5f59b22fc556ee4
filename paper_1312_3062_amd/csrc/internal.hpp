// Internal declarations shared by the library's translation units.
#pragma once

#include "common.hpp"

struct ann_index {
    int64_t n = 0;
    int32_t d = 0;
    int32_t dtype = 0;
    int32_t P = 0, K = 0, R = 0;
    int64_t nb = 0;  // K^P bridge vectors
    int64_t E = 0;   // total length of the bridge lists
    int device = 0;
    int64_t row_bytes = 0;  // d (u8) or 4d (f32)
    uint8_t* X = nullptr;           // n x row_bytes
    uint16_t* Xbf16 = nullptr;      // n x d bf16 copy (f32 indexes, made on first use)
    void* codebooks = nullptr;      // P x K x (d/P), dtype of X
    uint32_t* G = nullptr;          // n x R
    uint32_t* boff = nullptr;       // nb + 1
    uint32_t* bids = nullptr;       // E
    int64_t bytes = 0;
};

namespace ann {

struct SearchLaunch {
    const ann_index* idx;
    const void* d_q;
    int64_t nq;
    int kmax, Tmax;
    const int32_t* d_k;
    const int32_t* d_T;
    int L;
    int precision;
    int rerank_k;
    int32_t* d_ids;
    void* d_dists;
    int32_t* d_stats;
    int32_t* d_trace;
    hipStream_t stream;
    // launch tuning (never changes results)
    int lookahead = 0;      // queue entries whose rows are loaded together (0: as many as fit)
    int persistent = 0;     // resident grid draining a work counter
    int waves_per_cu = 0;   // persistent: resident workgroups per CU (0: all that fit)
    int order = 0;          // persistent with per-query budgets: longest first
    void* workspace = nullptr;  // caller-provided workspace (null: allocated on the stream)
    // neighborhood-graph search without bridges: seed ids measured first
    bool graph_only = false;
    const uint32_t* d_seeds = nullptr;
    int n_seeds = 0;
    int64_t workspace_bytes = 0;
};

int launch_search(const SearchLaunch& a);
int search_workspace_bytes(const SearchLaunch& a, int64_t* bytes, bool minimum = false);
// LDS one query of this launch occupies on a compute unit (allocation
// granules included), the largest over the launch's budget classes.
int search_lds_per_query(const SearchLaunch& a, int64_t* bytes);
int search_min_workspace(const ann_index* idx, int64_t nq, int32_t k, int32_t budget, const ann_search_params* sp,
                         int64_t* bytes);
int launch_tables(const ann_index* idx, const void* d_q, int64_t nq, void* d_sorted, int32_t* d_perm,
                  hipStream_t s);
int launch_knn(const void* d_x, int64_t n, int d, int dtype, const void* d_q, int64_t nq, int k, int exclude_self,
               int32_t* d_ids, void* d_dists, hipStream_t s);
int build_codebooks(ann_index* idx, int iters, int fx_log2, hipStream_t s);
int build_bridge_graph(ann_index* idx, int t, int b, hipStream_t s);
// the k-means assignment step for subspace p alone (nearest of K codewords,
// ties to the smaller one): cb_p holds that subspace's K x ds codewords
int kmeans_assign_subspace(const uint8_t* X, int64_t n, int d, bool f32, int ds, int p, int K, const void* cb_p,
                           int32_t* assign, hipStream_t s);
int make_bf16_copy(ann_index* idx, hipStream_t s);

// SplitMix64 and the seeded choice of the initial k-means rows (host side).
void kmeans_init_rows(int64_t n, int K, uint64_t seed, int64_t* rows);

// Device allocation tracked in the index's byte count.
int dalloc(ann_index* idx, void** p, size_t bytes);

}  // namespace ann
