// Search over the augmented neighborhood graph (Sec. 4.2, Alg. 1) on gfx950.
//
// One wavefront (64 lanes, one workgroup) serves one query at a time:
//   1. query tables: P x K squared subspace distances, each subspace sorted
//      by (value, codeword)                                        (Sec. 4.2)
//   2. multi-sequence extraction of bridge vectors in (distance, lid) order
//      (Sec. 3.3).  The frontier is a binary heap driven by one lane; the
//      bridge order does not depend on the traversal, so bridges are
//      extracted ahead in batches and their CSR offsets read by all lanes at
//      once.  Empty bridges are dropped there: expanding one changes nothing.
//   3. best-first expansion (Alg. 1).  The adjacency row of a reference and
//      its distance to the query are pure functions of ids, so the wave works
//      ahead of the exact order: it loads the kNN rows of the S best queue
//      entries together and gathers every neighbour that is neither visited
//      nor already measured, all in one memory round trip.  Rows and
//      distances stay in registers (lane s*R + j holds neighbour j of the
//      s-th entry) and in an LDS distance cache.  The exact loop then pops in
//      Alg. 1's order; a popped reference whose row is held is expanded with
//      no memory access: its white neighbours are marked in the exact visited
//      set, the first (T - t) of them in adjacency order are evaluated, and
//      the results are merged into the bounded main queue and the result
//      set.  Look-ahead never changes which vectors are evaluated, nor their
//      order.
//
// Register layout: the main queue (L <= 64) is one key per lane, sorted,
// with a head offset for pops; the result set is KPL keys per lane, sorted
// (element e in lane e % 64, register e / 64).  A merge of m new keys costs
// m scalar steps of ballots and one LDS scatter.
//
// The visited set and the distance cache are open-addressing tables of
// 16-byte buckets (four 32-bit ids), probed a bucket at a time.
//
// The multi-sequence heap lives in LDS with a small capacity.  A query whose
// frontier outgrows it is recorded and the same search is run again by a
// second kernel that keeps the heap in global memory.
#include "internal.hpp"
#include "mseq.hpp"

namespace ann {
namespace {

enum { MODE_U8 = 0, MODE_F32 = 1, MODE_BF16 = 2 };

constexpr int GEN_BATCH = 32;  // most bridges extracted per refill (ring capacity above T = 2048)
constexpr int MAX_SPEC = 8;    // references whose rows are loaded ahead together
constexpr int PRE_LIST = 8;    // bridge lists up to this length are fetched with the bridge

struct SearchArgs {
    const uint8_t* X;     // rows that drive the search (u8, f32 or bf16)
    const uint8_t* Xf32;  // fp32 rows for the final re-rank (bf16 mode)
    int64_t row_bytes;
    int64_t row_bytes_f32;
    int64_t n;
    int d, P, K, ds;
    const void* cb;
    const uint32_t* G;
    int R;
    const uint32_t* boff;
    const uint32_t* bids;
    const void* Q;
    int64_t nq;
    const int32_t* ks;
    const int32_t* Ts;
    int kmax, Tmax, L, rerank_k;
    int32_t* out_ids;
    void* out_d;
    int32_t* stats;
    int32_t* trace;
    uint32_t hash_buckets;  // visited set: buckets of 4 slots
    uint32_t dc_buckets;    // distance cache: buckets of 4 slots
    int spec;               // S, references loaded ahead (S * R <= 64)
    int ms_cap;             // multi-sequence: materialised side and outer frontier capacity
    int gen_batch;          // ring capacity: most bridges extracted per refill
    int prefetch;           // fetch short bridge lists (and distances) with the bridges
    uint32_t* ovf_list;  // queries whose LDS heap overflowed
    uint32_t* ovf_count;
    uint8_t* gheap;      // multi-sequence state in global memory: nslots slots of gms_cap
    int gms_cap;         // capacity of a slot
    int nslots;          // slots; the re-run kernel's workgroup b owns slot b
    uint32_t* slot_bits; // main kernel: bitmap of the slots in use (cleared at launch)
    int t_lo, t_hi;          // budget class served by this launch (inclusive); t_hi = Tmax
    int Tall;                // largest budget of the whole request: clamp and trace row stride
    uint32_t* work_counter;  // persistent launch: next work item (null: grid-stride)
    const uint32_t* perm;    // optional serving order of the queries
    int graph_only;          // neighborhood-graph search without bridges
    const uint32_t* seeds;   // its seed ids, measured first
    int nseeds;
    // budgets whose visited set does not fit LDS: a bitmap over the n vectors
    // per workgroup in global memory (workgroup b owns bitmap b; null: the
    // LDS set)
    uint32_t* gvis;
    int64_t gvis_words;      // 32-bit words of a bitmap
    int gvis_slots;          // bitmaps (the grids are capped to it)
    // LDS layout (byte offsets)
    int o_mrg;  // merge buffer of the register queues
    int o_q, o_sv, o_perm, o_ms, o_rk, o_ro, o_rl, o_sk, o_pid, o_pd, o_hash, o_dck, o_dcv, o_scr, o_gid, o_gd,
        o_sc;
};

template <int MODE>
struct Traits;
template <>
struct Traits<MODE_U8> {
    static constexpr int LPR = 1;  // lanes per gathered row
    static constexpr bool FLOAT = false;
};
template <>
struct Traits<MODE_F32> {
    static constexpr int LPR = 16;
    static constexpr bool FLOAT = true;
};
template <>
struct Traits<MODE_BF16> {
    static constexpr int LPR = 8;
    static constexpr bool FLOAT = true;
};

// ------------------------------------------------------------------
// squared distance of one gathered row; `part` of `lpr` lanes
// ------------------------------------------------------------------
template <int MODE, int NC16>
__device__ inline uint32_t row_partial(const uint8_t* row, const uint8_t* qv, int nc16, int part, int lpr);

// sum of squares of the query's bytes (u8 rows of 128 bytes take it precomputed)
__device__ inline uint32_t query_norm_u8(const uint8_t* qv, int d) {
    uint32_t qq = 0;
    for (int c = 0; c < d / 4; ++c) {
        const uint32_t w = reinterpret_cast<const uint32_t*>(qv)[c];
        qq = __builtin_amdgcn_udot4(w, w, qq, false);
    }
    return qq;
}

// d = 128: the whole 128-byte row in one lane, all loads in flight at once.
// sum (q-x)^2 = sum q^2 + sum x^2 - 2 sum q*x, every term an exact integer;
// qq = sum q^2 is the query's, computed once
__device__ inline uint32_t row_dist_u8_128(const uint8_t* row, const uint8_t* qv, uint32_t qq) {
    uint4 x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = reinterpret_cast<const uint4*>(row)[c];
    uint32_t xx = 0, qx = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint4 q = *reinterpret_cast<const uint4*>(qv + c * 16);
        xx = __builtin_amdgcn_udot4(x[c].x, x[c].x, xx, false);
        xx = __builtin_amdgcn_udot4(x[c].y, x[c].y, xx, false);
        xx = __builtin_amdgcn_udot4(x[c].z, x[c].z, xx, false);
        xx = __builtin_amdgcn_udot4(x[c].w, x[c].w, xx, false);
        qx = __builtin_amdgcn_udot4(q.x, x[c].x, qx, false);
        qx = __builtin_amdgcn_udot4(q.y, x[c].y, qx, false);
        qx = __builtin_amdgcn_udot4(q.z, x[c].z, qx, false);
        qx = __builtin_amdgcn_udot4(q.w, x[c].w, qx, false);
    }
    return xx + qq - 2u * qx;
}

template <>
__device__ inline uint32_t row_partial<MODE_U8, 0>(const uint8_t* row, const uint8_t* qv, int nc16, int part,
                                                   int lpr) {
    uint32_t xx = 0, qq = 0, qx = 0;
#pragma unroll 4
    for (int c = part; c < nc16; c += lpr) {
        const uint4 x = *reinterpret_cast<const uint4*>(row + c * 16);
        const uint4 q = *reinterpret_cast<const uint4*>(qv + c * 16);
        xx = __builtin_amdgcn_udot4(x.x, x.x, xx, false);
        xx = __builtin_amdgcn_udot4(x.y, x.y, xx, false);
        xx = __builtin_amdgcn_udot4(x.z, x.z, xx, false);
        xx = __builtin_amdgcn_udot4(x.w, x.w, xx, false);
        qq = __builtin_amdgcn_udot4(q.x, q.x, qq, false);
        qq = __builtin_amdgcn_udot4(q.y, q.y, qq, false);
        qq = __builtin_amdgcn_udot4(q.z, q.z, qq, false);
        qq = __builtin_amdgcn_udot4(q.w, q.w, qq, false);
        qx = __builtin_amdgcn_udot4(q.x, x.x, qx, false);
        qx = __builtin_amdgcn_udot4(q.y, x.y, qx, false);
        qx = __builtin_amdgcn_udot4(q.z, x.z, qx, false);
        qx = __builtin_amdgcn_udot4(q.w, x.w, qx, false);
    }
    return xx + qq - 2u * qx;  // modulo 2^32; the group total is exact
}

template <>
__device__ inline uint32_t row_partial<MODE_F32, 0>(const uint8_t* row, const uint8_t* qv, int nc16, int part,
                                                    int lpr) {
    float acc = 0.f;
#pragma unroll 4
    for (int c = part; c < nc16; c += lpr) {
        const float4 x = *reinterpret_cast<const float4*>(row + c * 16);
        const float4 q = *reinterpret_cast<const float4*>(qv + c * 16);
        float t0 = q.x - x.x, t1 = q.y - x.y, t2 = q.z - x.z, t3 = q.w - x.w;
        acc = fmaf(t0, t0, acc);
        acc = fmaf(t1, t1, acc);
        acc = fmaf(t2, t2, acc);
        acc = fmaf(t3, t3, acc);
    }
    return f_bits(acc);
}

template <>
__device__ inline uint32_t row_partial<MODE_BF16, 0>(const uint8_t* row, const uint8_t* qv, int nc16, int part,
                                                     int lpr) {
    // row chunk c holds bf16 dims [8c, 8c+8); the query stays fp32
    float acc = 0.f;
#pragma unroll 4
    for (int c = part; c < nc16; c += lpr) {
        const uint4 x = *reinterpret_cast<const uint4*>(row + c * 16);
        const float4 qa = *reinterpret_cast<const float4*>(qv + c * 32);
        const float4 qb = *reinterpret_cast<const float4*>(qv + c * 32 + 16);
        float t;
        t = qa.x - bf16_lo(x.x); acc = fmaf(t, t, acc);
        t = qa.y - bf16_hi(x.x); acc = fmaf(t, t, acc);
        t = qa.z - bf16_lo(x.y); acc = fmaf(t, t, acc);
        t = qa.w - bf16_hi(x.y); acc = fmaf(t, t, acc);
        t = qb.x - bf16_lo(x.z); acc = fmaf(t, t, acc);
        t = qb.y - bf16_hi(x.z); acc = fmaf(t, t, acc);
        t = qb.z - bf16_lo(x.w); acc = fmaf(t, t, acc);
        t = qb.w - bf16_hi(x.w); acc = fmaf(t, t, acc);
    }
    return f_bits(acc);
}

// total over the lpr lanes of a row group (fixed butterfly order)
template <int MODE>
__device__ inline uint32_t group_sum(uint32_t v, int lpr) {
    if constexpr (!Traits<MODE>::FLOAT) {
        for (int m = 1; m < lpr; m <<= 1) v += __shfl_xor(v, m);
        return v;
    } else {
        float f = bits_f(v);
        for (int m = 1; m < lpr; m <<= 1) f += __shfl_xor(f, m);
        return f_bits(f);
    }
}

// Float rows of a size fixed at compile time (NC16 16-byte chunks): 8 lanes
// per row, every chunk of a lane (chunks part, part + 8, ...) loaded before
// any is used, so a pass over 8 rows is one memory round trip.
constexpr int FIXED_LPR = 8;

template <int MODE, int NC16>
__device__ inline uint32_t row_partial_fixed(const uint8_t* row, const uint8_t* qv, int part) {
    constexpr int CPL = NC16 / FIXED_LPR;
    float acc = 0.f;
    if constexpr (MODE == MODE_F32) {
        float4 x[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) x[u] = reinterpret_cast<const float4*>(row)[part + u * FIXED_LPR];
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const float4 q = reinterpret_cast<const float4*>(qv)[part + u * FIXED_LPR];
            float t0 = q.x - x[u].x, t1 = q.y - x[u].y, t2 = q.z - x[u].z, t3 = q.w - x[u].w;
            acc = fmaf(t0, t0, acc);
            acc = fmaf(t1, t1, acc);
            acc = fmaf(t2, t2, acc);
            acc = fmaf(t3, t3, acc);
        }
    } else {
        uint4 x[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) x[u] = reinterpret_cast<const uint4*>(row)[part + u * FIXED_LPR];
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int c = part + u * FIXED_LPR;  // bf16 dims [8c, 8c + 8); the query stays fp32
            const float4 qa = *reinterpret_cast<const float4*>(qv + c * 32);
            const float4 qb = *reinterpret_cast<const float4*>(qv + c * 32 + 16);
            float t;
            t = qa.x - bf16_lo(x[u].x); acc = fmaf(t, t, acc);
            t = qa.y - bf16_hi(x[u].x); acc = fmaf(t, t, acc);
            t = qa.z - bf16_lo(x[u].y); acc = fmaf(t, t, acc);
            t = qa.w - bf16_hi(x[u].y); acc = fmaf(t, t, acc);
            t = qb.x - bf16_lo(x[u].z); acc = fmaf(t, t, acc);
            t = qb.y - bf16_hi(x[u].z); acc = fmaf(t, t, acc);
            t = qb.z - bf16_lo(x[u].w); acc = fmaf(t, t, acc);
            t = qb.w - bf16_hi(x[u].w); acc = fmaf(t, t, acc);
        }
    }
    return f_bits(acc);
}

// lanes that share a gathered row
template <int MODE, int NC16>
__host__ __device__ constexpr int gather_lpr() {
    return Traits<MODE>::LPR == 1 ? 1 : (NC16 > 0 ? FIXED_LPR : Traits<MODE>::LPR);
}

// Distance of the row `id` for every lane with `need`, returned in that lane.
// One lane per row (u8); otherwise the rows are listed in LDS and groups of
// LPR lanes gather them, RPP rows per pass.
template <int MODE, int NC16>
__device__ inline uint32_t gather_need(const SearchArgs& a, const uint8_t* qv, uint32_t qq, uint32_t id, bool need,
                                       uint32_t* gid, uint32_t* gd, int lane) {
    constexpr int LPR = gather_lpr<MODE, NC16>();
    if constexpr (LPR == 1) {
        uint32_t d = 0;
        if (need) {
            if constexpr (MODE == MODE_U8 && NC16 == 8)
                d = row_dist_u8_128(a.X + int64_t(id) * a.row_bytes, qv, qq);
            else
                d = row_partial<MODE, NC16>(a.X + int64_t(id) * a.row_bytes, qv, int(a.row_bytes / 16), 0, 1);
        }
        return d;
    } else {
        constexpr int RPP = WAVE / LPR;
        const uint64_t nm = __ballot(need);
        const int m = __popcll(nm);
        const int pos = lanes_below(nm);
        if (need) gid[pos] = id;
        __syncthreads();
        const int part = lane % LPR, grp = lane / LPR;
        const int nc16 = int(a.row_bytes / 16);
        for (int p0 = 0; p0 < m; p0 += RPP) {
            const int row = p0 + grp;
            uint32_t ps = 0;
            if (row < m) {
                const uint8_t* src = a.X + int64_t(gid[row]) * a.row_bytes;
                if constexpr (NC16 > 0)
                    ps = row_partial_fixed<MODE, NC16>(src, qv, part);
                else
                    ps = row_partial<MODE, 0>(src, qv, nc16, part, LPR);
            }
            const uint32_t dsum = group_sum<MODE>(ps, LPR);
            if (part == 0 && row < m) gd[row] = dsum;
        }
        __syncthreads();
        return need ? gd[pos] : 0u;
    }
}

// ------------------------------------------------------------------
// Exact sets of 32-bit ids: open addressing over 16-byte buckets of four
// slots, linear probing bucket by bucket.  A bucket is read with one LDS
// access; a slot is claimed with compare-and-swap.
// ------------------------------------------------------------------
__device__ inline uint32_t home_bucket(uint32_t id, uint32_t nbk) {
    return uint32_t((uint64_t(id * 0x9E3779B1u) * nbk) >> 32);
}

// A bucket's slots fill in order: a slot is claimed only as the bucket's
// first empty one, and slots are emptied only all at once (a clear of the
// whole table).  So a bucket with room has an empty last slot, and its
// first empty slot is the number of ids it holds.
__device__ inline bool bucket_open(uint4 v) { return v.w == ID_EMPTY; }
__device__ inline bool bucket_has(uint4 v, uint32_t id) {
    return min(min(v.x ^ id, v.y ^ id), min(v.z ^ id, v.w ^ id)) == 0u;
}
__device__ inline uint32_t bucket_fill(uint4 v) {
    return min(v.x + 1u, 1u) + min(v.y + 1u, 1u) + min(v.z + 1u, 1u) + min(v.w + 1u, 1u);
}
__device__ inline uint32_t bucket_index(uint4 v, uint32_t id) {  // v holds id
    return v.x == id ? 0u : v.y == id ? 1u : v.z == id ? 2u : 3u;
}

// Slot of id, inserting it if absent.  fresh = it was absent.  Returns -1
// (fresh = false) only if the table is full, which the callers' sizing rules
// out; the probe count is bounded so that a wave can never spin here.
__device__ inline int set_insert(uint32_t* T, uint32_t nbk, uint32_t id, bool& fresh) {
    uint32_t b = home_bucket(id, nbk);
    for (uint32_t step = 0; step < 5 * nbk + 4; ++step) {
        const uint4 v = reinterpret_cast<const uint4*>(T)[b];
        if (bucket_has(v, id)) {
            fresh = false;
            return int(b * 4 + bucket_index(v, id));
        }
        if (!bucket_open(v)) {
            b = (b + 1 == nbk) ? 0 : b + 1;
            continue;
        }
        const uint32_t f = bucket_fill(v);
        const uint32_t old = atomicCAS(&T[b * 4 + f], ID_EMPTY, id);
        if (old == ID_EMPTY || old == id) {
            fresh = old == ID_EMPTY;
            return int(b * 4 + f);
        }
        // another lane took the slot for a different id: read the bucket again
    }
    fresh = false;
    return -1;
}

// Atomic OR on a word known to be in global memory (a generic pointer would
// make the compiler test at run time whether it addresses LDS).
typedef __attribute__((address_space(1))) uint32_t global_u32;
__device__ inline uint32_t global_or(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_or((global_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The distance cache's values carry a visited flag in their top bit (u8
// distances stay below 2^31 for d <= 512; fp32 distances are non-negative).
constexpr uint32_t VISITED_FLAG = 0x80000000u;
constexpr uint32_t DIST_BITS = 0x7FFFFFFFu;

// Lookups read two consecutive buckets at once (one LDS round trip); the
// second counts only when the first is full, so the probe order is that of
// bucket-by-bucket linear probing.  Slot of id, or -1.
__device__ inline int set_find(const uint32_t* T, uint32_t nbk, uint32_t id) {
    uint32_t b = home_bucket(id, nbk);
    for (uint32_t step = 0; step < nbk; step += 2) {
        const uint32_t b2 = (b + 1 == nbk) ? 0 : b + 1;
        const uint4 v = reinterpret_cast<const uint4*>(T)[b];
        const uint4 w = reinterpret_cast<const uint4*>(T)[b2];
        if (bucket_has(v, id)) return int(b * 4 + bucket_index(v, id));
        if (bucket_open(v)) return -1;
        if (bucket_has(w, id)) return int(b2 * 4 + bucket_index(w, id));
        if (bucket_open(w)) return -1;
        b = (b2 + 1 == nbk) ? 0 : b2 + 1;
    }
    return -1;
}

// Whether the set holds id (the same probes, no slot).
__device__ inline bool set_has(const uint32_t* T, uint32_t nbk, uint32_t id) {
    uint32_t b = home_bucket(id, nbk);
    for (uint32_t step = 0; step < nbk; step += 2) {
        const uint32_t b2 = (b + 1 == nbk) ? 0 : b + 1;
        const uint4 v = reinterpret_cast<const uint4*>(T)[b];
        const uint4 w = reinterpret_cast<const uint4*>(T)[b2];
        if (bucket_has(v, id)) return true;
        if (bucket_open(v)) return false;
        if (bucket_has(w, id)) return true;
        if (bucket_open(w)) return false;
        b = (b2 + 1 == nbk) ? 0 : b2 + 1;
    }
    return false;
}

// ------------------------------------------------------------------
// Sorted key arrays held in registers
// ------------------------------------------------------------------
__device__ inline uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l));
    return (uint64_t(hi) << 32) | lo;
}

template <int KPL>
__device__ inline uint64_t reg_get(const uint64_t (&v)[KPL], int e) {
    uint64_t r = 0;
#pragma unroll
    for (int u = 0; u < KPL; ++u)
        if (e / WAVE == u) r = readlane64(v[u], e % WAVE);
    return r;
}

// Whole-wave lane shifts of a 64-bit value (DPP wave_shr:1 / wave_shl:1).
// shr: lane i receives lane i-1, lane 0 receives `fill`.
// shl: lane i receives lane i+1, lane 63 receives `fill`.
__device__ inline uint64_t wave_shr1(uint64_t v, uint64_t fill) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(fill)), int(uint32_t(v)), 0x138, 0xF, 0xF, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(fill >> 32)), int(uint32_t(v >> 32)), 0x138, 0xF, 0xF, false));
    return (uint64_t(hi) << 32) | lo;
}
__device__ inline uint64_t wave_shl1(uint64_t v, uint64_t fill) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(fill)), int(uint32_t(v)), 0x130, 0xF, 0xF, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(fill >> 32)), int(uint32_t(v >> 32)), 0x130, 0xF, 0xF, false));
    return (uint64_t(hi) << 32) | lo;
}

// v with lane l replaced by the wave-uniform value x (v_writelane_b32, its
// lane select in m0: two scalar operands would exceed the constant bus)
__device__ inline int write_lane(int v, int x, int l) {
    asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "{m0}"(l));
    return v;
}

// Offer the keys of the lanes with `isnew` (distinct, none present) to the
// sorted array v[0..n) of capacity cap <= 64 (one key per lane), all new keys
// at once: the result is the smallest min(cap, n + m) of the old and new
// keys, sorted, which is what offering them one at a time to a bounded set
// that evicts its largest key leaves.  Each key's place is its rank among old and
// new keys, counted in one pass over the new keys; the keys are written to
// their places in LDS (buf: 64 keys for this wavefront) and read back.
__device__ inline void reg_merge1(uint64_t& v, int& n, int cap, uint64_t x, bool isnew, int lane, uint64_t* buf) {
    uint64_t nm = __ballot(isnew);
    const int m = __popcll(nm);
    const bool old = lane < n;
    // lanes at or past n hold KEY_EMPTY, above every key offered, so the
    // counts below need no mask of old lanes: the number of old keys below
    // x_j is 64 minus the lanes whose key lies above x_j
    int above = 0;      // old key: new keys below it
    int new_below = 0;  // new key: new keys below it
    int old_below = 0;  // new key: old keys below it
    while (nm) {
        const int j = __builtin_ctzll(nm);
        nm &= nm - 1;
        const uint64_t xj = readlane64(x, j);
        above += xj < v ? 1 : 0;
        new_below += xj < x ? 1 : 0;
        const int ob = WAVE - __popcll(__ballot(xj < v));  // keys are distinct
        old_below = write_lane(old_below, ob, j);
    }
    const int po = lane + above, pn = old_below + new_below;
    if (old && po < cap) buf[po] = v;
    if (isnew && pn < cap) buf[pn] = x;
    lds_wave_order();
    const int total = min(cap, n + m);
    v = lane < total ? buf[lane] : KEY_EMPTY;
    n = total;
    lds_wave_order();
}

// reg_merge1 for a sorted array of KPL keys per lane (element e in lane
// e % 64, register e / 64; elements at or past n hold KEY_EMPTY): each key's
// place is its rank among old and new keys, counted in one pass over the new
// keys; buf holds KPL * 64 keys.  A new key costs KPL compares and ballots
// instead of a shift of the whole array.
template <int KPL>
__device__ inline void reg_mergeN(uint64_t (&v)[KPL], int& n, int cap, uint64_t x, bool isnew, int lane,
                                  uint64_t* buf) {
    uint64_t nm = __ballot(isnew);
    const int m = __popcll(nm);
    int above[KPL];
#pragma unroll
    for (int u = 0; u < KPL; ++u) above[u] = 0;
    int new_below = 0, old_below = 0;
    while (nm) {
        const int j = __builtin_ctzll(nm);
        nm &= nm - 1;
        const uint64_t xj = readlane64(x, j);
        int ob = KPL * WAVE;  // old elements below x_j: all but those above it (keys are distinct)
#pragma unroll
        for (int u = 0; u < KPL; ++u) {
            const bool lt = xj < v[u];
            above[u] += lt ? 1 : 0;
            ob -= __popcll(__ballot(lt));
        }
        new_below += xj < x ? 1 : 0;
        old_below = write_lane(old_below, ob, j);
    }
#pragma unroll
    for (int u = 0; u < KPL; ++u) {
        const int e = lane + u * WAVE;
        const int po = e + above[u];
        if (e < n && po < cap) buf[po] = v[u];
    }
    const int pn = old_below + new_below;
    if (isnew && pn < cap) buf[pn] = x;
    lds_wave_order();
    const int total = min(cap, n + m);
#pragma unroll
    for (int u = 0; u < KPL; ++u) {
        const int e = lane + u * WAVE;
        v[u] = e < total ? buf[e] : KEY_EMPTY;
    }
    n = total;
    lds_wave_order();
}

// remove and return the smallest key (n > 0)
__device__ inline uint64_t reg_pop_front(uint64_t (&v)[1], int& n) {
    const uint64_t x = readlane64(v[0], 0);
    v[0] = wave_shl1(v[0], KEY_EMPTY);
    --n;
    return x;
}

// ------------------------------------------------------------------
// Pairwise multi-sequence (Sec. 3.3), driven by one lane.
//
// The P sorted subspace lists are split into two sides: X = lists {0} or
// {0,1}, Y = the rest ({}, {1}, {2} or {2,3}).  A side of two lists is
// enumerated lazily by its own 2-list multi-sequence and its elements kept in
// order ("materialised"); a side of one list is that list.  The outer 2-list
// enumeration over (X, Y) yields the bridges in (sum, lid) order: every list
// is sorted by (value, codeword), each side by (sum, lid) with lid the
// concatenated codewords, and a tuple's unique parent -- (i, j-1), or (i-1, 0)
// when j = 0 -- always precedes it in that order.  The outer frontier holds
// at most one entry per row of X, so it grows with the square root of the
// bridges extracted, not with their number.
// ------------------------------------------------------------------
struct MSeqMem {
    uint64_t* mx;  // materialised X elements: sum << 32 | lid
    uint64_t* my;  // materialised Y elements
    hent_t* ho;    // outer heap: keys sum << 32 | n + lid, positions i << 16 | j
    hent_t* hx;    // inner heap of X: keys, ranks ra << 8 | rb
    hent_t* hy;    // inner heap of Y
    int cap;       // capacity of mx and my
    int ocap;      // of the outer heap
};


// Capacities.  A frontier holds at most one entry per started row, and a row
// is started only once the element heading it is known: the outer frontier
// never exceeds the X elements materialised (K when X is one list), and an
// inner frontier never exceeds one more than the elements it has produced.
struct MSeqCaps {
    int cap, ocap, icap;
};
__host__ __device__ inline MSeqCaps mseq_caps(int cap, int K, int P) {
    MSeqCaps c;
    c.cap = cap;
    c.ocap = P >= 3 ? cap + 2 : K + 1;
    c.icap = cap + 2 < K + 1 ? cap + 2 : K + 1;
    return c;
}

__host__ __device__ inline int mseq_bytes(int cap, int K, int P) {
    const MSeqCaps c = mseq_caps(cap, K, P);
    return c.cap * 8 * 2 + (c.ocap + c.icap * 2) * int(sizeof(hent_t)) + 64;
}

// a global slot: mseq_bytes rounded up so that every slot starts 64-byte aligned
__host__ __device__ inline int mseq_slot_bytes(int cap, int K, int P) { return (mseq_bytes(cap, K, P) + 63) & ~63; }

__device__ inline MSeqMem mseq_carve(uint8_t* base, int cap, int K, int P) {
    const MSeqCaps c = mseq_caps(cap, K, P);
    MSeqMem m;
    m.mx = reinterpret_cast<uint64_t*>(base);  // 16-byte aligned
    m.my = m.mx + c.cap;
    m.ho = reinterpret_cast<hent_t*>(m.my + c.cap);  // 16 * cap bytes in: still aligned
    m.hx = m.ho + c.ocap;
    m.hy = m.hx + c.icap;
    m.cap = c.cap;
    m.ocap = c.ocap;
    return m;
}

// Constant part of the enumeration (the same in every lane).
struct MSeqConf {
    const uint32_t* sv;
    const uint8_t* perm;
    int K;
    uint32_t n;
    int nx, ny;           // lists on each side
    int ax, bx, ay, by;   // their subspaces
    uint32_t sizeX, sizeY;
    MSeqMem m;
};

__device__ inline MSeqConf mseq_conf(const uint32_t* sv, const uint8_t* perm, int P, int K, uint32_t n, MSeqMem m) {
    MSeqConf c;
    c.sv = sv;
    c.perm = perm;
    c.K = K;
    c.n = n;
    c.m = m;
    c.nx = P >= 3 ? 2 : 1;
    c.ny = P - c.nx;
    c.ax = 0;
    c.bx = 1;
    c.ay = c.nx;
    c.by = c.nx + 1;
    c.sizeX = c.nx == 2 ? uint32_t(K * K) : uint32_t(K);
    c.sizeY = c.ny == 2 ? uint32_t(K * K) : (c.ny == 1 ? uint32_t(K) : 1u);
    return c;
}

// Changing part, driven by one lane.
template <bool FLOAT>
struct PairMSeq {
    int cx, cy, hxn, hyn, hon, maxf;
    bool of;  // a structure outgrew its capacity

    __device__ static uint32_t add(uint32_t s1, uint32_t s2) {
        if constexpr (FLOAT)
            return f_bits(bits_f(s1) + bits_f(s2));
        else
            return s1 + s2;
    }
    __device__ static uint64_t inner_key(const MSeqConf& c, int a, int b, uint32_t ra, uint32_t rb) {
        const uint32_t sum = add(c.sv[a * c.K + ra], c.sv[b * c.K + rb]);
        return make_key(sum, uint32_t(c.perm[a * c.K + ra]) * uint32_t(c.K) + c.perm[b * c.K + rb]);
    }
    // element e of a side, materialising it if needed
    __device__ bool elem(const MSeqConf& c, bool isx, uint32_t e, uint32_t& sum, uint32_t& lid) {
        const int nl = isx ? c.nx : c.ny;
        const int la = isx ? c.ax : c.ay, lb = isx ? c.bx : c.by;
        if (nl == 0) {
            sum = 0;
            lid = 0;
            return true;
        }
        if (nl == 1) {
            sum = c.sv[la * c.K + e];
            lid = c.perm[la * c.K + e];
            return true;
        }
        int& cnt = isx ? cx : cy;
        int& hn = isx ? hxn : hyn;
        uint64_t* M = isx ? c.m.mx : c.m.my;
        hent_t* hp = isx ? c.m.hx : c.m.hy;
        while (uint32_t(cnt) <= e) {
            if (hn == 0) return false;
            if (cnt >= c.m.cap) {
                of = true;
                return false;
            }
            if constexpr (FLOAT) {
                const hent_t top = hp[0];
                const uint64_t key = hkey(top);
                const uint32_t rk = top.z;
                M[cnt++] = key;
                const uint32_t ra = rk >> 8, rb = rk & 0xFF;
                // the successor in the row takes the top's place (none: the
                // last entry does); a row's first element also starts the next row
                uint64_t nk;
                uint32_t nr;
                if (rb + 1 < uint32_t(c.K)) {
                    nk = inner_key(c, la, lb, ra, rb + 1);
                    nr = (ra << 8) | (rb + 1);
                } else {
                    const hent_t last = hp[--hn];
                    nk = hkey(last);
                    nr = last.z;
                }
                heap_replace_top(hp, hn, nk, nr);
                if (rb == 0 && ra + 1 < uint32_t(c.K)) heap_push(hp, hn, inner_key(c, la, lb, ra + 1, 0), (ra + 1) << 8);
            } else {
                uint64_t key;
                uint32_t rk;
                heap_pop(hp, hn, key, rk);
                M[cnt++] = key;
                const uint32_t ra = rk >> 8, rb = rk & 0xFF;
                if (rb + 1 < uint32_t(c.K)) heap_push(hp, hn, inner_key(c, la, lb, ra, rb + 1), (ra << 8) | (rb + 1));
                if (rb == 0 && ra + 1 < uint32_t(c.K)) heap_push(hp, hn, inner_key(c, la, lb, ra + 1, 0), (ra + 1) << 8);
            }
        }
        sum = key_dist(M[e]);
        lid = key_id(M[e]);
        return true;
    }
    // element e of a side that is already materialised
    __device__ static void known(const MSeqConf& c, bool isx, uint32_t e, uint32_t& sum, uint32_t& lid) {
        const int nl = isx ? c.nx : c.ny;
        const int la = isx ? c.ax : c.ay;
        if (nl == 0) {
            sum = 0;
            lid = 0;
        } else if (nl == 1) {
            sum = c.sv[la * c.K + e];
            lid = c.perm[la * c.K + e];
        } else {
            const uint64_t v = (isx ? c.m.mx : c.m.my)[e];
            sum = key_dist(v);
            lid = key_id(v);
        }
    }
    // start row i of the outer frontier at (i, 0); Y[0] is materialised
    __device__ void start_row(const MSeqConf& c, uint32_t i) {
        uint32_t sx, lx, sy, ly;
        if (!elem(c, true, i, sx, lx)) return;
        known(c, false, 0, sy, ly);
        if (hon >= c.m.ocap) {
            of = true;
            return;
        }
        heap_push(c.m.ho, hon, make_key(add(sx, sy), c.n + lx * c.sizeY + ly), i << 16);
        maxf = max(maxf, hon);
    }
    __device__ void outer_push(const MSeqConf& c, uint32_t i, uint32_t j) {
        uint32_t sx, lx, sy, ly;
        if (!elem(c, true, i, sx, lx) || !elem(c, false, j, sy, ly)) return;
        if (hon >= c.m.ocap) {
            of = true;
            return;
        }
        heap_push(c.m.ho, hon, make_key(add(sx, sy), c.n + lx * c.sizeY + ly), (i << 16) | j);
        maxf = max(maxf, hon);
    }
    // the next call of next() may need an element or frontier entry beyond
    // the capacity (it adds at most one element to each side and one entry to
    // the frontier: a pushed position is at most one past the elements its
    // parent used)
    __device__ bool tight(const MSeqConf& c) const {
        const bool x = c.nx == 2 && cx >= c.m.cap && uint32_t(cx) < c.sizeX;
        const bool y = c.ny == 2 && cy >= c.m.cap && uint32_t(cy) < c.sizeY;
        return x || y || hon + 2 > c.m.ocap;
    }
    __device__ void init(const MSeqConf& c) {
        cx = cy = hxn = hyn = hon = maxf = 0;
        of = false;
        if (c.nx == 2) heap_push(c.m.hx, hxn, inner_key(c, c.ax, c.bx, 0, 0), 0u);
        if (c.ny == 2) heap_push(c.m.hy, hyn, inner_key(c, c.ay, c.by, 0, 0), 0u);
        if constexpr (FLOAT) {
            uint32_t s0, l0;
            if (elem(c, false, 0, s0, l0)) start_row(c, 0);
        } else {
            outer_push(c, 0, 0);
        }
    }
    // The next bridge in (distance, lid) order; false when exhausted or
    // overflowed.  Float tables: the taken tuple's successor in its row
    // replaces it at the top of the heap (one sift-down that stops where the
    // successor belongs); the bridge-heavy float indexes spend their longest
    // queries here.  Integer tables keep a pop and pushes: in the u8 kernels
    // the other form cost the search loop registers.
    __device__ bool next(const MSeqConf& c, uint64_t& key) {
        if (hon == 0 || of) return false;
        if constexpr (FLOAT) {
            const hent_t top = c.m.ho[0];
            key = hkey(top);
            const uint32_t pos = top.z;
            const uint32_t i = pos >> 16, j = pos & 0xFFFF;
            // (i, j + 1) takes the top's place (none, or no room for its
            // elements: the last entry does)
            uint32_t sx, lx, sy, ly;
            uint64_t nk;
            uint32_t np;
            if (j + 1 < c.sizeY && elem(c, false, j + 1, sy, ly)) {
                known(c, true, i, sx, lx);  // row i started with X[i]
                nk = make_key(add(sx, sy), c.n + lx * c.sizeY + ly);
                np = (i << 16) | (j + 1);
            } else {
                const hent_t last = c.m.ho[--hon];
                nk = hkey(last);
                np = last.z;
            }
            heap_replace_top(c.m.ho, hon, nk, np);
            if (j == 0 && i + 1 < c.sizeX) start_row(c, i + 1);
        } else {
            uint32_t pos;
            heap_pop(c.m.ho, hon, key, pos);
            const uint32_t i = pos >> 16, j = pos & 0xFFFF;
            if (j + 1 < c.sizeY) outer_push(c, i, j + 1);
            if (j == 0 && i + 1 < c.sizeX) outer_push(c, i + 1, 0);
        }
        return true;
    }
};

// COUNT: per-query counters and the evaluation trace are recorded (when the
// caller asked for either); without them fewer scalars stay live.
template <int MODE, int NC16, int KPL, bool RERUN, bool COUNT>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(MODE == MODE_U8 && KPL <= 2 ? 4 : 1, 8)))
k_search(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr bool FLOAT = Traits<MODE>::FLOAT;

    uint8_t* qv = lds + a.o_q;
    uint32_t* sv = reinterpret_cast<uint32_t*>(lds + a.o_sv);
    uint8_t* perm = lds + a.o_perm;
    uint64_t* ring_key = reinterpret_cast<uint64_t*>(lds + a.o_rk);
    uint32_t* ring_off = reinterpret_cast<uint32_t*>(lds + a.o_ro);
    uint32_t* ring_len = reinterpret_cast<uint32_t*>(lds + a.o_rl);
    uint64_t* stage = reinterpret_cast<uint64_t*>(lds + a.o_sk);
    uint32_t* pre_id = reinterpret_cast<uint32_t*>(lds + a.o_pid);  // prefetched bridge lists, 8 per entry
    uint32_t* pre_d = reinterpret_cast<uint32_t*>(lds + a.o_pd);    // and their distances
    uint32_t* H = reinterpret_cast<uint32_t*>(lds + a.o_hash);
    // budgets beyond LDS: this workgroup's visited bitmap in global memory
    // (its address is formed where used, never kept live across the search)
    const bool gvis = a.gvis != nullptr;
    uint32_t* DK = reinterpret_cast<uint32_t*>(lds + a.o_dck);
    uint32_t* DV = reinterpret_cast<uint32_t*>(lds + a.o_dcv);
    uint64_t* scratch = reinterpret_cast<uint64_t*>(lds + a.o_scr);
    uint32_t* gid = reinterpret_cast<uint32_t*>(lds + a.o_gid);
    uint32_t* gd = reinterpret_cast<uint32_t*>(lds + a.o_gd);
    int* sc = reinterpret_cast<int*>(lds + a.o_sc);
    uint64_t* mrg = reinterpret_cast<uint64_t*>(lds + a.o_mrg);  // merge buffer, 64 keys a result register


    const int lane = lane_id();
    const int64_t n = a.n;
    const int P = a.P, K = a.K, R = a.R;
    const int HW = int(a.hash_buckets) * 4;
    const int DW = int(a.dc_buckets) * 4;
    const int dc_limit = DW * 5 / 8 - WAVE;  // keeps the cache at most about 5/8 full
    const int qbytes = FLOAT ? a.d * 4 : a.d;
    const int S = a.spec;
    const int row_lane_slot = R > 0 ? lane / R : 0;  // which look-ahead entry this lane serves
    const int row_lane_j = R > 0 ? lane % R : 0;

    const int64_t nwork = RERUN ? int64_t(*a.ovf_count) : a.nq;
    // persistent launch: every workgroup takes the next item of a device
    // counter until the batch is drained; otherwise grid-stride
    const bool persistent = !RERUN && a.work_counter != nullptr;
    auto grab = [&]() -> int64_t {
        if (lane == 0) sc[3] = int(atomicAdd(a.work_counter, 1u));
        __syncthreads();
        const int64_t v = sc[3];
        __syncthreads();
        return v;
    };
    for (int64_t wi = persistent ? grab() : int64_t(blockIdx.x); wi < nwork;
         wi = persistent ? grab() : wi + gridDim.x) {
        const int64_t qi = RERUN ? int64_t(a.ovf_list[wi]) : (a.perm ? int64_t(a.perm[wi]) : wi);
        // per-query values are clamped to the launch maxima that sized the buffers
        const int k = a.ks ? min(max(a.ks[qi], 1), a.kmax) : a.kmax;
        const int T = a.Ts ? min(max(a.Ts[qi], 0), a.Tall) : a.Tall;
        if (!RERUN && (T < a.t_lo || T > a.t_hi)) continue;  // another budget class's query
        const int rcap = (MODE == MODE_BF16) ? max(k, a.rerank_k) : k;

        // ---- load the query, clear the distance cache
        {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(a.Q) + qi * qbytes);
            uint32_t* dst = reinterpret_cast<uint32_t*>(qv);
            for (int i = lane; i < qbytes / 4; i += WAVE) dst[i] = src[i];
            for (int i = lane; i < DW; i += WAVE) DK[i] = ID_EMPTY;
        }
        __syncthreads();
        const uint32_t qq = (MODE == MODE_U8 && NC16 == 8) ? query_norm_u8(qv, 128) : 0u;

        // ---- tables and their sort (the raw tables use the visited set's
        //      memory, cleared afterwards); the nearest bridge seeds the frontier
        const bool graph_only = a.graph_only != 0;  // neighborhood-graph search, no bridges
        if (!graph_only) compute_tables<FLOAT>(qv, a.cb, P, K, a.ds, H, sv, perm, lane);
        for (int i = lane; i < HW; i += WAVE) H[i] = ID_EMPTY;
        if (gvis) {
            global_u32* gv = (global_u32*)(a.gvis + int64_t(blockIdx.x) * a.gvis_words);
            for (int64_t i = lane; i < a.gvis_words; i += WAVE) gv[i] = 0u;
        }
        __syncthreads();
        int slot = -1;  // global slot the enumeration moved to (main kernel)
        // where the enumeration state lives: LDS, or a global slot (the re-run
        // kernel's workgroup b owns slot b); rebuilt where used rather than kept
        // in registers across the search
        auto ms_conf = [&]() {
            const int64_t slot_bytes = mseq_slot_bytes(a.gms_cap, K, P);
            MSeqMem m;
            if (RERUN)
                m = mseq_carve(a.gheap + int64_t(blockIdx.x) * slot_bytes, a.gms_cap, K, P);
            else if (slot >= 0)
                m = mseq_carve(a.gheap + int64_t(slot) * slot_bytes, a.gms_cap, K, P);
            else
                m = mseq_carve(lds + a.o_ms, a.ms_cap, K, P);
            return mseq_conf(sv, perm, P, K, uint32_t(n), m);
        };
        PairMSeq<FLOAT> ms;
        if (lane == 0 && !graph_only) ms.init(ms_conf());
        bool ms_alive = !graph_only;  // the enumeration can still yield bridges
        int heap_max = 1;
        int flags = 0;
        int ring_h = 0, ring_n = 0;
        int refills = 0;
        uint32_t ids_mask = 0, dist_mask = 0;  // ring entries with prefetched ids / distances
        uint64_t bkey = KEY_EMPTY;  // next non-empty bridge (ring head)
        if (graph_only && a.nseeds > 0) {
            // the seed list is expanded before anything else, like the list
            // of a bridge at distance 0 walked from memory (key 0 is below
            // every queue key); no bridge follows it
            if (lane == 0) {
                ring_key[0] = 0;
                ring_off[0] = 0;
                ring_len[0] = uint32_t(a.nseeds);
            }
            __syncthreads();
            ring_n = 1;
            bkey = 0;
        }
        uint64_t Qv[1] = {KEY_EMPTY};
        int qn = 0;
        uint64_t Rv[KPL];
#pragma unroll
        for (int u = 0; u < KPL; ++u) Rv[u] = KEY_EMPTY;
        int rn = 0;
        // look-ahead rows: lane l holds neighbour (l % R) of entry (l / R)
        uint32_t acn = ID_EMPTY;  // lane s < S: node id of entry s
        uint32_t ac_id = ID_EMPTY, ac_d = 0;
        // Visits: an id is visited if the visited set H holds it, or if the
        // distance cache holds it with its visited flag set; for an id in the
        // cache the flag decides.  A lane's neighbour that was unvisited when
        // its row was loaded keeps its distance-cache slot (ac_slot) until its
        // row is expanded: expanding the row marks the visit with one atomic
        // on that slot's flag, and so does a bridge that visits an id the
        // cache holds (the row then finds the flag set).  A visit of an id
        // outside the cache goes to H; when the cache is cleared, its flagged
        // ids move to H first.
        int ac_slot = -1;
        int t = 0;
        int dc_fill = 0;
        int st_rpop = 0, st_bpop = 0, st_bids = 0, st_gen = 0, st_rows = 0, st_spec = 0;
        int r = 0;

        // the lanes with `ev` hold evaluated keys (rank r in adjacency order):
        // record them and offer them to the result set and the main queue
        auto offer = [&](uint64_t key, bool ev) {
            if (COUNT && a.trace && ev) a.trace[qi * a.Tall + t + r] = int32_t(key_id(key));
            const uint64_t rworst = rn < rcap ? KEY_EMPTY : reg_get<KPL>(Rv, rn - 1);
            const bool ra = ev && key < rworst;
            if (__ballot(ra)) {
                if constexpr (KPL == 1)
                    reg_merge1(Rv[0], rn, rcap, key, ra, lane, mrg);
                else
                    reg_mergeN<KPL>(Rv, rn, rcap, key, ra, lane, mrg);
            }
            const uint64_t qworst = qn < a.L ? KEY_EMPTY : readlane64(Qv[0], qn - 1);
            const bool qa = ev && key < qworst;
            if (__ballot(qa)) reg_merge1(Qv[0], qn, a.L, key, qa, lane, mrg);
        };

        // the visited set: the LDS table, or the global bitmap (atomics at L2:
        // a lane reads what the wave's other lanes set)
        auto vis_insert = [&](uint32_t vid, bool& fresh) -> bool {
            if (gvis) {
                const uint32_t bit = 1u << (vid & 31u);
                uint32_t* w = a.gvis + int64_t(blockIdx.x) * a.gvis_words + (vid >> 5);
                fresh = (global_or(w, bit) & bit) == 0u;
                return true;
            }
            return set_insert(H, a.hash_buckets, vid, fresh) >= 0;
        };
        auto vis_has = [&](uint32_t vid) -> bool {
            if (gvis) {
                uint32_t* w = a.gvis + int64_t(blockIdx.x) * a.gvis_words + (vid >> 5);
                return (global_or(w, 0u) >> (vid & 31u)) & 1u;
            }
            return set_has(H, a.hash_buckets, vid);
        };

        // a bridge's list entry: visited unless the cache flags it or H holds
        // it, marked visited either way; `cached` gets the distance the cache
        // holds for it, or ID_EMPTY
        auto visit_listed = [&](uint32_t vid, bool& full, uint32_t& cached) -> bool {
            cached = ID_EMPTY;
            if (vid == ID_EMPTY) return false;
            const int ds = set_find(DK, a.dc_buckets, vid);
            if (ds >= 0) {
                const uint32_t old = atomicOr(&DV[ds], VISITED_FLAG);
                cached = old & DIST_BITS;
                return (old & VISITED_FLAG) == 0u;
            }
            bool fresh = false;
            if (!vis_insert(vid, fresh)) full = true;
            return fresh;
        };

        while (t < T) {
            bool full = false;
            // ---- look-ahead extraction of the next non-empty bridges; their
            //      lists (and, once bridges are in use, their distances) are
            //      fetched with them: the bridge order does not depend on the
            //      traversal
            if (ring_h == ring_n) {
                while (ring_h == ring_n && ms_alive && flags == 0) {
                    if (lane == 0) {
                        // batches of 4, 8, 16, then 32 bridges: at small budgets a
                        // query expands about one bridge
                        const int gb = min(a.gen_batch, 4 << min(refills, 3));
                        const MSeqConf msc = ms_conf();
                        int g = 0;
                        uint64_t key;
                        bool move = false;
                        while (g < gb) {
                            if (!RERUN && slot < 0 && ms.tight(msc)) {
                                move = true;  // continue from a global slot
                                break;
                            }
                            if (!ms.next(msc, key)) break;
                            stage[g++] = key;
                        }
                        sc[0] = (ms.hon > 0 && !ms.of) ? 1 : 0;
                        sc[1] = ms.of ? 1 : 0;
                        sc[2] = g;
                        sc[4] = ms.maxf;
                        sc[5] = move ? 1 : 0;
                    }
                    __syncthreads();
                    const bool move = sc[5] != 0;
                    ms_alive = sc[0] != 0;
                    if constexpr (COUNT) heap_max = sc[4];
                    const int g = sc[2];
                    if (sc[1]) flags = ANN_ERESOURCE;
                    if constexpr (COUNT) st_gen += g;
                    bool ne = false;
                    uint64_t key = 0;
                    uint32_t o0 = 0, o1 = 0;
                    if (lane < g) {
                        key = stage[lane];
                        const uint32_t lid = key_id(key) - uint32_t(n);
                        o0 = a.boff[lid];
                        o1 = a.boff[lid + 1];
                        ne = o1 > o0;
                    }
                    const uint64_t mask = __ballot(ne);
                    const int pos = lanes_below(mask);
                    if (ne) {
                        ring_key[pos] = key;
                        ring_off[pos] = o0;
                        ring_len[pos] = o1 - o0;
                    }
                    ring_h = 0;
                    ring_n = __popcll(mask);
                    // short lists: ids now, from the second refill on also distances
                    if (a.prefetch) {
                        // bit e: ring entry e (rank of its lane among the non-empty ones) is short
                        const uint64_t sm = __ballot(ne && o1 - o0 <= uint32_t(PRE_LIST));
                        uint32_t mk = 0;
                        uint64_t bits = sm;
                        while (bits) {
                            const int l = __builtin_ctzll(bits);
                            bits &= bits - 1;
                            mk |= 1u << __popcll(mask & ((uint64_t(1) << l) - 1));
                        }
                        ids_mask = mk;
                    }
                    __syncthreads();
                    ++refills;
                    const bool with_dist = refills >= 2;
#pragma unroll 1
                    for (int u = 0; a.prefetch && u < GEN_BATCH * PRE_LIST / WAVE; ++u) {
                        const int sl = lane + u * WAVE;
                        const int e = sl / PRE_LIST, x = sl % PRE_LIST;
                        uint32_t pid = ID_EMPTY;
                        if (e < ring_n && ((ids_mask >> e) & 1u) && uint32_t(x) < ring_len[e])
                            pid = a.bids[ring_off[e] + x];
                        pre_id[sl] = pid;
                        if (with_dist) {
                            bool need = false;
                            uint32_t d = 0;
                            if (pid != ID_EMPTY && !vis_has(pid)) {
                                const int ds = set_find(DK, a.dc_buckets, pid);
                                if (ds >= 0)
                                    d = DV[ds] & DIST_BITS;
                                else
                                    need = true;
                            }
                            const uint32_t gdist = gather_need<MODE, NC16>(a, qv, qq, pid, need, gid, gd, lane);
                            if constexpr (COUNT) st_rows += __popcll(__ballot(need));
                            pre_d[sl] = need ? gdist : d;
                        }
                    }
                    dist_mask = with_dist ? ids_mask : 0u;
                    __syncthreads();
                    if constexpr (!RERUN) {
                        if (move) {
                            // the LDS state is full: claim a free global slot and
                            // carry on there (no free slot: the re-run kernel
                            // redoes the query)
                            if (lane == 0) {
                                int got = -1;
                                for (int tries = 0; tries < 4 * a.nslots && got < 0; ++tries) {
                                    const int w = (int(blockIdx.x) + tries) % ((a.nslots + 31) / 32);
                                    const uint32_t used = __hip_atomic_load(a.slot_bits + w, __ATOMIC_RELAXED,
                                                                            __HIP_MEMORY_SCOPE_AGENT);
                                    const int nb = min(32, a.nslots - 32 * w);
                                    const uint32_t freeb = ~used & (nb == 32 ? ~0u : ((1u << nb) - 1u));
                                    if (freeb == 0) continue;
                                    const uint32_t bit = freeb & (0u - freeb);
                                    const uint32_t old = __hip_atomic_fetch_or(a.slot_bits + w, bit, __ATOMIC_ACQUIRE,
                                                                               __HIP_MEMORY_SCOPE_AGENT);
                                    if (!(old & bit)) got = 32 * w + __builtin_ctz(bit);
                                }
                                sc[6] = got;
                                sc[7] = ms.cx;
                                sc[8] = ms.cy;
                                sc[9] = ms.hxn;
                                sc[10] = ms.hyn;
                                sc[11] = ms.hon;
                            }
                            __syncthreads();
                            const int got = sc[6];
                            if (got < 0) {
                                flags = ANN_ERESOURCE;
                            } else {
                                const MSeqMem l = ms_conf().m;  // the LDS state (no slot yet)
                                slot = got;
                                const MSeqMem g = ms_conf().m;
                                for (int i = lane; i < sc[7]; i += WAVE) g.mx[i] = l.mx[i];
                                for (int i = lane; i < sc[8]; i += WAVE) g.my[i] = l.my[i];
                                for (int i = lane; i < sc[9]; i += WAVE) g.hx[i] = l.hx[i];
                                for (int i = lane; i < sc[10]; i += WAVE) g.hy[i] = l.hy[i];
                                for (int i = lane; i < sc[11]; i += WAVE) g.ho[i] = l.ho[i];
                            }
                            __syncthreads();
                        }
                    }
                }
                bkey = ring_h < ring_n ? ring_key[ring_h] : KEY_EMPTY;
            }
            if (flags) break;

            // ---- which vertex Alg. 1 pops next: the queue head or the next bridge
            const uint64_t qkey = qn > 0 ? readlane64(Qv[0], 0) : KEY_EMPTY;
            const bool use_bridge = ring_h < ring_n && bkey < qkey;
            if (!use_bridge && qn == 0) break;  // queue empty and every bridge consumed
            if (!use_bridge && key_id(qkey) >= uint32_t(n)) {  // never happens: keys hold evaluated ids
                flags = ANN_ERESOURCE;
                break;
            }

            bool ev = false;
            uint32_t id = ID_EMPTY, dist = 0;
            int take = 0;
            if (!use_bridge) {
                // ---- a reference: find its row among the rows loaded ahead
                const uint32_t node = key_id(qkey);
                uint64_t hit = __ballot(lane < S && acn == node);
                if (!hit) {
                    // work ahead: rows of the S best queue entries, distances of
                    // their unvisited neighbours not yet in the cache
                    if constexpr (COUNT) ++st_spec;
                    const int ns = min(S, qn);
                    acn = lane < ns ? key_id(Qv[0]) : ID_EMPTY;  // lane s holds queue entry s
                    const uint32_t nd_l = uint32_t(__shfl(int(acn), row_lane_slot));
                    // the lane's column is re-stated here so that no per-lane row
                    // pointer is kept (and spilled) across the search
                    int col = row_lane_j;
                    asm("" : "+v"(col));
                    uint32_t nid = ID_EMPTY;
                    if (R > 0 && lane < ns * R) nid = a.G[int64_t(nd_l) * R + col];
                    // while the rows load: the distance cache is cleared when 5/8
                    // full, its visit marks moving to the visited set first
                    if (dc_fill > dc_limit) {
                        for (int c0 = 0; c0 < DW; c0 += WAVE) {
                            const int i = c0 + lane;
                            uint32_t vid = ID_EMPTY;
                            if (i < DW && (DV[i] & VISITED_FLAG)) vid = DK[i];
                            bool fresh = false;
                            if (vid != ID_EMPTY && !vis_insert(vid, fresh)) full = true;
                        }
                        for (int i = lane; i < DW; i += WAVE) DK[i] = ID_EMPTY;
                        dc_fill = 0;
                        lds_wave_order();
                    }
                    ac_id = nid;
                    bool need = false, known = false;
                    int slot = 0;
                    if (ac_id != ID_EMPTY && !vis_has(ac_id)) {
                        known = true;
                        slot = set_insert(DK, a.dc_buckets, ac_id, need);
                        if (slot < 0) {
                            full = true;
                            slot = 0;
                            known = false;
                        }
                    }
                    const uint32_t gdist = gather_need<MODE, NC16>(a, qv, qq, ac_id, need, gid, gd, lane);
                    if (need) DV[slot] = gdist;
                    const int m = __popcll(__ballot(need));
                    dc_fill += m;
                    if constexpr (COUNT) st_rows += m;
                    __syncthreads();
                    // an id the cache already held may have been visited since
                    const uint32_t dv = known && !need ? DV[slot] : 0u;
                    if (dv & VISITED_FLAG) known = false;
                    ac_d = known ? (need ? gdist : (dv & DIST_BITS)) : 0u;
                    ac_slot = known ? slot : -1;
                    hit = 1;  // entry 0 is the queue head
                }
                const int s = __builtin_ctzll(hit);
                reg_pop_front(Qv, qn);
                if constexpr (COUNT) ++st_rpop;
                // ---- expand: the row sits in lanes [s*R, s*R + R)
                const bool inrow = R > 0 && row_lane_slot == s && lane < (s + 1) * R;
                // unvisited when the row was loaded, and not visited since unless
                // a pop or a bridge of this window set the slot's flag
                bool white = false;
                if (inrow && ac_slot >= 0) white = (atomicOr(&DV[ac_slot], VISITED_FLAG) & VISITED_FLAG) == 0u;
                if (inrow) ac_slot = -1;  // the row is expanded
                const uint64_t wm = __ballot(white);
                take = min(int(__popcll(wm)), T - t);
                r = lanes_below(wm);
                ev = white && r < take;
                id = ac_id;
                dist = ac_d;
            } else if ((ids_mask >> ring_h) & 1u) {
                // ---- a bridge whose short list was fetched ahead (Sec. 4.1 bridge graph)
                const int e = ring_h;
                const int len = int(ring_len[e]);
                ++ring_h;
                bkey = ring_h < ring_n ? ring_key[ring_h] : KEY_EMPTY;
                if constexpr (COUNT) {
                    ++st_bpop;
                    st_bids += len;
                }
                id = lane < len ? pre_id[e * PRE_LIST + lane] : ID_EMPTY;
                uint32_t cached = ID_EMPTY;
                const bool white = visit_listed(id, full, cached);
                const uint64_t wm = __ballot(white);
                take = min(int(__popcll(wm)), T - t);
                r = lanes_below(wm);
                ev = white && r < take;
                if ((dist_mask >> e) & 1u) {
                    dist = pre_d[e * PRE_LIST + lane];  // measured ahead: white then, so not visited then
                } else {
                    const bool miss = ev && cached == ID_EMPTY;
                    const uint32_t gdist = gather_need<MODE, NC16>(a, qv, qq, id, miss, gid, gd, lane);
                    if constexpr (COUNT) st_rows += __popcll(__ballot(miss));
                    dist = cached != ID_EMPTY ? cached : gdist;
                }
            } else {
                // ---- a bridge with a long list: walked from global memory
                const int64_t base = ring_off[ring_h];
                const int len = int(ring_len[ring_h]);
                ++ring_h;
                bkey = ring_h < ring_n ? ring_key[ring_h] : KEY_EMPTY;
                if constexpr (COUNT) {
                    ++st_bpop;
                    st_bids += len;
                }
                // lists longer than a wave are walked in chunks; every chunk but
                // the one that ends the list or the budget is merged here, that
                // one below
                const uint32_t* list = graph_only ? a.seeds : a.bids;
                for (int c0 = 0;; c0 += WAVE) {
                    const int j = c0 + lane;
                    id = j < len ? list[base + j] : ID_EMPTY;
                    if (id >= uint32_t(n)) id = ID_EMPTY;  // a seed outside [0, n) is skipped
                    uint32_t cached = ID_EMPTY;
                    const bool white = visit_listed(id, full, cached);
                    const uint64_t wm = __ballot(white);
                    take = min(int(__popcll(wm)), T - t);
                    r = lanes_below(wm);
                    ev = white && r < take;
                    const bool miss = ev && cached == ID_EMPTY;
                    const uint32_t gdist = gather_need<MODE, NC16>(a, qv, qq, id, miss, gid, gd, lane);
                    if constexpr (COUNT) st_rows += __popcll(__ballot(miss));
                    dist = cached != ID_EMPTY ? cached : gdist;
                    if (c0 + WAVE >= len || t + take >= T) break;
                    offer(make_key(dist, id), ev);
                    t += take;
                }
            }

            if (__ballot(full)) {  // a table outgrew its sizing: give up on this query
                flags = ANN_ERESOURCE;
                break;
            }
            // ---- evaluated vectors enter the result set and the main queue
            if (take > 0) {
                offer(make_key(dist, id), ev);
                t += take;
            }
        }

        if (!RERUN && slot >= 0) {
            // give the slot back once this wave's last write to it is done
            if (lane == 0) {
                __threadfence();
                __hip_atomic_fetch_and(a.slot_bits + slot / 32, ~(1u << (slot % 32)), __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (!RERUN && flags) {
            // no room for the multi-sequence state: the re-run kernel redoes this query
            if (lane == 0) a.ovf_list[atomicAdd(a.ovf_count, 1u)] = uint32_t(qi);
            __syncthreads();
            continue;
        }

        // ---- bf16 mode: re-rank the kept candidates with fp32 rows
        if constexpr (MODE == MODE_BF16) {
#pragma unroll
            for (int u = 0; u < KPL; ++u) {
                const int e = lane + u * WAVE;
                if (e < rn) scratch[e] = Rv[u];
            }
            __syncthreads();
            constexpr int LPR = 16, RPP = WAVE / LPR;
            const int part = lane % LPR, grp = lane / LPR;
            const int nc16f = int(a.row_bytes_f32 / 16);
            uint64_t* rr = reinterpret_cast<uint64_t*>(gid);  // rn <= rcap keys (sized by the host)
            for (int p0 = 0; p0 < rn; p0 += RPP) {
                const int row = p0 + grp;
                uint32_t part_sum = 0, rid = 0;
                if (row < rn) {
                    rid = key_id(scratch[row]);
                    part_sum = row_partial<MODE_F32, 0>(a.Xf32 + int64_t(rid) * a.row_bytes_f32, qv, nc16f, part, LPR);
                }
                const uint32_t dsum = group_sum<MODE_F32>(part_sum, LPR);
                if (part == 0 && row < rn) rr[row] = make_key(dsum, rid);
            }
            __syncthreads();
            for (int i = lane; i < rn; i += WAVE) {
                const uint64_t v = rr[i];
                int rk = 0;
                for (int jj = 0; jj < rn; ++jj) rk += rr[jj] < v;
                scratch[rk] = v;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < KPL; ++u) {
                const int e = lane + u * WAVE;
                Rv[u] = e < rn ? scratch[e] : KEY_EMPTY;
            }
            __syncthreads();
        }

        // ---- results, ascending by (distance, id), padded
#pragma unroll
        for (int u = 0; u < KPL; ++u) {
            const int i = lane + u * WAVE;
            if (i < a.kmax) {
                const int64_t o = qi * a.kmax + i;
                if (flags == 0 && i < k && i < rn) {
                    a.out_ids[o] = int32_t(key_id(Rv[u]));
                    static_cast<uint32_t*>(a.out_d)[o] = key_dist(Rv[u]);
                } else {
                    a.out_ids[o] = -1;
                    static_cast<uint32_t*>(a.out_d)[o] = FLOAT ? 0x7F800000u : 0x7FFFFFFFu;
                }
            }
        }
        if (COUNT && a.trace)
            for (int i = t + lane; i < a.Tall; i += WAVE) a.trace[qi * a.Tall + i] = -1;
        if (COUNT && a.stats && lane == 0) {
            int32_t* s = a.stats + qi * ANN_NSTATS;
            s[ANN_STAT_EVALS] = t;
            s[ANN_STAT_REF_POPS] = st_rpop;
            s[ANN_STAT_BRIDGE_POPS] = st_bpop;
            s[ANN_STAT_BRIDGE_IDS] = st_bids;
            s[ANN_STAT_BRIDGES_GEN] = st_gen;
            s[ANN_STAT_HEAP_MAX] = heap_max;
            s[ANN_STAT_FLAGS] = flags;
            s[ANN_STAT_ROWS] = st_rows;
            s[ANN_STAT_LOOKAHEADS] = st_spec;
            s[ANN_STAT_RERUN] = RERUN ? 1 : 0;
            s[ANN_STAT_MOVED] = slot >= 0 ? 1 : 0;
            s[ANN_STAT_MOVED + 1] = 0;
        }
        __syncthreads();
    }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Serving order for uneven budgets: queries bucketed by descending budget
// (powers of two), so the longest ones start first.  Any order gives the same
// results; this one shortens the tail of a persistent launch.
__device__ inline int budget_bucket(int T) { return 20 - min(20, 31 - __clz(max(T, 1))); }

__global__ void k_order_count(const int32_t* Ts, int64_t nq, uint32_t* counts) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nq) atomicAdd(&counts[budget_bucket(Ts[i])], 1u);
}

__global__ void k_order_scan(uint32_t* counts) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int b = 0; b < 32; ++b) {
        const uint32_t c = counts[b];
        counts[b] = run;
        run += c;
    }
}

__global__ void k_order_scatter(const int32_t* Ts, int64_t nq, const uint32_t* start, uint32_t* cursor,
                                uint32_t* perm) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nq) {
        const int b = budget_bucket(Ts[i]);
        perm[start[b] + atomicAdd(&cursor[b], 1u)] = uint32_t(i);
    }
}

// standalone tables kernel (query preprocessing only)
template <bool FLOAT>
__global__ void __launch_bounds__(WAVE) k_tables(const void* Q, int64_t nq, int d, const void* cb, int P, int K,
                                                  int ds, uint32_t* out_sorted, int32_t* out_perm) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int qbytes = FLOAT ? d * 4 : d;
    const int PK = P * K;
    uint8_t* qv = lds;
    uint32_t* tab = reinterpret_cast<uint32_t*>(lds + ((qbytes + 15) & ~15));
    uint32_t* sv = tab + PK;
    uint8_t* perm = reinterpret_cast<uint8_t*>(sv + PK);
    const int lane = lane_id();
    for (int64_t qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(Q) + qi * qbytes);
        for (int i = lane; i < qbytes / 4; i += WAVE) reinterpret_cast<uint32_t*>(qv)[i] = src[i];
        __syncthreads();
        compute_tables<FLOAT>(qv, cb, P, K, ds, tab, sv, perm, lane);
        for (int e = lane; e < PK; e += WAVE) {
            out_sorted[qi * PK + e] = sv[e];
            out_perm[qi * PK + e] = perm[e];
        }
        __syncthreads();
    }
}

int align_up(int v, int a) { return (v + a - 1) / a * a; }

// LDS layout of one query's state; the heap is left out for the re-run kernel
int layout(SearchArgs& a, int qbytes, int PK, int rcap, bool with_heap, bool bf16, int lpr) {
    int off = 0;
    auto take = [&](int bytes, int al) {
        off = align_up(off, al);
        int o = off;
        off += bytes;
        return o;
    };
    a.o_q = take(align_up(qbytes, 16), 16);
    a.o_sv = take(PK * 4, 8);
    a.o_perm = take(PK, 8);
    a.o_ms = with_heap ? take(mseq_bytes(a.ms_cap, a.K, a.P), 16) : 0;
    a.o_rk = take(a.gen_batch * 8, 8);
    a.o_ro = take(a.gen_batch * 4, 8);
    a.o_rl = take(a.gen_batch * 4, 8);
    a.o_sk = a.o_rk;  // a batch is staged where it is compacted into the ring
    a.o_pid = a.prefetch ? take(GEN_BATCH * PRE_LIST * 4, 16) : 0;
    a.o_pd = a.prefetch ? take(GEN_BATCH * PRE_LIST * 4, 16) : 0;
    // the visited set also holds the raw distance tables before the search
    a.o_hash = take(std::max(int(a.hash_buckets) * 16, PK * 4), 16);
    a.o_dck = take(int(a.dc_buckets) * 16, 16);
    a.o_dcv = take(int(a.dc_buckets) * 16, 16);
    // re-rank keys (bf16) and the row list of multi-lane gathers (fp32, bf16)
    a.o_scr = take(bf16 ? rcap * 8 : 8, 8);
    a.o_gid = take(bf16 ? std::max(WAVE * 4, rcap * 8) : (lpr > 1 ? WAVE * 4 : 8), 8);
    a.o_gd = take(lpr > 1 ? WAVE * 4 : 8, 8);
    a.o_sc = take(16 * 4, 8);
    a.o_mrg = take(align_up(std::max(rcap, WAVE), WAVE) * 8, 8);
    return align_up(off, 16);
}

struct Grid {
    int64_t grid;     // workgroups of the main launch (0: derive from occupancy)
    int waves_per_cu; // persistent: cap on resident workgroups per CU (0: all that fit)
    int cus;
};

template <int MODE, int NC16, int KPL, bool COUNT>
int launch_mode_c(const SearchArgs& a1, const SearchArgs& a2, int lds1, int lds2, Grid g, int grid2, hipStream_t st) {
    auto* k1 = k_search<MODE, NC16, KPL, false, COUNT>;
    int64_t grid = g.grid;
    if (a1.work_counter) {
        int per_cu = 0;
        ANN_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k1, WAVE, lds1));
        per_cu = std::max(1, per_cu);
        if (g.waves_per_cu > 0) per_cu = std::min(per_cu, g.waves_per_cu);
        grid = std::min<int64_t>(a1.nq, int64_t(per_cu) * g.cus);
    }
    if (a1.gvis) grid = std::min<int64_t>(grid, a1.gvis_slots);  // workgroup b owns visited bitmap b
    hipLaunchKernelGGL(k1, dim3(unsigned(grid)), dim3(WAVE), lds1, st, a1);
    hipLaunchKernelGGL((k_search<MODE, NC16, KPL, true, COUNT>), dim3(unsigned(grid2)), dim3(WAVE), lds2, st, a2);
    return ANN_OK;
}

template <int MODE, int NC16, int KPL>
int launch_mode(const SearchArgs& a1, const SearchArgs& a2, int lds1, int lds2, Grid g, int grid2,
                hipStream_t st) {
    if (a1.stats || a1.trace) return launch_mode_c<MODE, NC16, KPL, true>(a1, a2, lds1, lds2, g, grid2, st);
    return launch_mode_c<MODE, NC16, KPL, false>(a1, a2, lds1, lds2, g, grid2, st);
}

template <int MODE, int NC16>
int launch_kpl(int rcap, const SearchArgs& a1, const SearchArgs& a2, int lds1, int lds2, Grid g, int grid2,
               hipStream_t st) {
    if (rcap <= 64) return launch_mode<MODE, NC16, 1>(a1, a2, lds1, lds2, g, grid2, st);
    if (rcap <= 128) return launch_mode<MODE, NC16, 2>(a1, a2, lds1, lds2, g, grid2, st);
    return launch_mode<MODE, NC16, 16>(a1, a2, lds1, lds2, g, grid2, st);
}

}  // namespace

// Everything about a search launch that follows from the index and the
// request: kernel arguments, LDS layout and the workspace it needs.
struct Plan {
    SearchArgs a, a2;
    int lds1 = 0, lds2 = 0, rcap = 0;
    bool bf16 = false, is_f32 = false;
    int grid2 = 128;
    int64_t gcap = 0;
    size_t slot_bytes = 0;
    int max_slots = 0;
    bool gvis = false;       // the visited set is a global bitmap (budget beyond LDS)
    int64_t gvis_words = 0;  // words of one bitmap
    int gvis_slots = 0;      // bitmaps wanted (one per workgroup of the grid)
};

static size_t round16(size_t v) { return (v + 15) & ~size_t(15); }
constexpr int kLdsGranule = 2560;  // LDS allocation granule of a workgroup (160 KB / 64)

// Global slots for multi-sequence state that outgrows LDS: one for every
// workgroup that can be resident, so a query never finds them all taken
// (such a query is redone by the second kernel, at many times the cost: on
// an index whose queries expand tens to hundreds of bridges most queries
// move, at any budget).  At most 512 MiB of slots.  A workspace smaller
// than the full size gets fewer slots (at least one).
constexpr size_t kMaxSlotBytes = size_t(512) << 20;
// Visited bitmaps of budgets beyond LDS: at most 1 GiB of them (the grid of
// such a class is capped to the bitmaps; each workgroup clears its own per
// query, n / 8 bytes, against the T rows of at least 100 bytes it gathers).
constexpr size_t kMaxBitmapBytes = size_t(1) << 30;

static int make_plan(const SearchLaunch& s, Plan& pl) {
    const ann_index* idx = s.idx;
    ANN_REQUIRE(idx->R <= WAVE, "search: graph out-degree above 64 is not supported");
    SearchArgs& a = pl.a;
    a = SearchArgs{};
    pl.is_f32 = idx->dtype == ANN_F32;
    pl.bf16 = pl.is_f32 && s.precision == ANN_PRECISION_BF16_RERANK;
    if (pl.bf16) {
        ANN_REQUIRE(idx->Xbf16 != nullptr, "bf16 copy of the vectors is missing");
        ANN_REQUIRE(idx->d % 8 == 0, "bf16 precision needs d divisible by 8");
    }
    a.X = pl.bf16 ? reinterpret_cast<const uint8_t*>(idx->Xbf16) : idx->X;
    a.Xf32 = idx->X;
    a.row_bytes = pl.bf16 ? int64_t(idx->d) * 2 : idx->row_bytes;
    a.row_bytes_f32 = idx->row_bytes;
    a.n = idx->n;
    a.d = idx->d;
    a.P = idx->P;
    a.K = idx->K;
    a.ds = idx->d / idx->P;
    a.cb = idx->codebooks;
    a.G = idx->G;
    a.R = idx->R;
    a.boff = idx->boff;
    a.bids = idx->bids;
    a.Q = s.d_q;
    a.nq = s.nq;
    a.ks = s.d_k;
    a.Ts = s.d_T;
    a.kmax = s.kmax;
    a.Tmax = s.Tmax;
    a.Tall = s.Tmax;
    a.t_lo = 0;
    a.t_hi = s.Tmax;
    a.L = s.L;
    a.rerank_k = s.rerank_k;  // 0: each query's own k
    a.out_ids = s.d_ids;
    a.out_d = s.d_dists;
    a.stats = s.d_stats;
    a.trace = s.d_trace;
    a.graph_only = s.graph_only ? 1 : 0;
    a.seeds = s.d_seeds;
    a.nseeds = s.graph_only ? s.n_seeds : 0;

    // visited set: at most T + 64 ids (the last adjacency chunk may mark more
    // than it evaluates), buckets for a final load of about 0.8 (its lookups
    // sit on the look-ahead's critical path: at 0.92 the 1M x 128 search took
    // 15% longer), or 0.9 where residency is chosen over latency (below).
    // The distance cache (cleared when 5/8 full) gets at least 56 buckets and
    // grows into the slack of the last LDS granule (below).
    const int64_t visit_ids = int64_t(s.Tmax) + WAVE;
    auto visited_buckets = [&](bool dense) {
        return uint32_t(std::max<int64_t>(4, (dense ? visit_ids * 10 / 9 : visit_ids * 5 / 4) / 4 + 1));
    };
    a.dc_buckets = 56;
    const int max_spec = idx->R > 0 ? std::min(MAX_SPEC, WAVE / idx->R) : 1;
    a.spec = s.lookahead > 0 ? std::min(s.lookahead, max_spec) : max_spec;
    // multi-sequence capacity in LDS (materialised side elements and outer
    // frontier), by budget; a query that outgrows it moves its state to a
    // global slot and carries on.  Up to T = 2048 the kNN graph does almost
    // all the work (one bridge per query on the 1M workload); beyond it
    // bridges take over and their lists are fetched ahead.
    const int64_t side = int64_t(idx->K) * idx->K;
    // The state is only fast in LDS: a query that outgrows it continues at L2
    // latency, one lane at a time.  With four lists of at most 64 codewords
    // a query at T <= 2048 expands about one bridge and 8 elements per side
    // suffice.  Between 2048 and 4096 residency wins: 64 elements and the
    // visited set at load 0.9 keep one more query per CU than 256 at 0.8
    // (1M x 128 at T = 3072: 43.5 -> 34.0 ms; 10M x 128 uneven batch:
    // 31.6 -> 28.1 ms).  Above 4096 bridges take over and a state that moves
    // out of LDS makes its query the slowest of its launch: 256 at 0.8 (a
    // mixed request stream on the 10M index served 98K queries/s against
    // 83K), unless the launch has one budget and more queries than fit the
    // chip at that size, where residency wins again (1M x 128 at T = 8192:
    // 310 against 398 ms).  With three lists or K >= 100 (fewer, larger
    // sides, and tens to hundreds of bridges expanded per query) the state
    // gets 256, or 512 when the whole batch is still resident at that size
    // (below), and the short bridge lists are fetched ahead at every budget.
    const bool few_bridges = idx->P >= 4 && idx->K <= 64;
    const bool mid_budget = s.Tmax > 2048 && s.Tmax <= 4096;
    a.hash_buckets = visited_buckets(mid_budget);
    a.ms_cap = int(std::min<int64_t>(side, few_bridges ? (s.Tmax <= 2048 ? 8 : (mid_budget ? 64 : 256)) : 256));
    a.prefetch = (s.Tmax > 2048 || !few_bridges) ? 1 : 0;
    a.gen_batch = s.Tmax <= 2048 ? 16 : GEN_BATCH;

    const int qbytes = pl.is_f32 ? idx->d * 4 : idx->d;
    const int PK = idx->P * idx->K;
    pl.rcap = pl.bf16 ? std::max(s.kmax, a.rerank_k) : s.kmax;
    ANN_REQUIRE(pl.rcap <= 1024, "search: k (or rerank_k) above 1024");
    const int lpr = pl.is_f32 ? (pl.bf16 ? Traits<MODE_BF16>::LPR : Traits<MODE_F32>::LPR) : Traits<MODE_U8>::LPR;
    int cus = 0, lds_cu = 0;
    ANN_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, idx->device));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, idx->device));
    if (few_bridges && s.Tmax > 4096 && !s.d_T && a.ms_cap > 64) {
        // one budget for the whole launch: throughput first when the batch
        // does not fit the chip at the larger state
        const int lds_lat = layout(a, qbytes, PK, pl.rcap, true, pl.bf16, lpr);
        const int64_t granules = ceil_div(lds_lat, kLdsGranule);
        if (int64_t(cus) * (lds_cu / (granules * kLdsGranule)) < s.nq) {
            a.ms_cap = int(std::min<int64_t>(side, 64));
            a.hash_buckets = visited_buckets(true);
        }
    }
    if (!few_bridges && a.ms_cap < side) {
        // a batch that fits on the chip either way: the larger state keeps
        // the bridge-heavy queries (the launch's slowest) in LDS
        SearchArgs big = a;
        big.ms_cap = int(std::min<int64_t>(side, 512));
        const int lds_big = layout(big, qbytes, PK, pl.rcap, true, pl.bf16, lpr);
        const int64_t granules = ceil_div(lds_big, kLdsGranule);
        if (int64_t(cus) * (lds_cu / (granules * kLdsGranule)) >= s.nq) a.ms_cap = big.ms_cap;
    }
    pl.lds1 = layout(a, qbytes, PK, pl.rcap, true, pl.bf16, lpr);
    {
        // LDS is allocated to a workgroup in granules of 2.5 KB: a larger
        // distance cache that stays within the same granules costs no
        // residency (a bucket of keys and values is 32 bytes)
        const int slack = int(ceil_div(pl.lds1, kLdsGranule) * kLdsGranule) - pl.lds1;
        a.dc_buckets = uint32_t(std::min(128, 56 + slack / 32));
        pl.lds1 = layout(a, qbytes, PK, pl.rcap, true, pl.bf16, lpr);
    }
    int max_lds = 0;
    ANN_HIP_CHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, idx->device));
    if (pl.lds1 > max_lds) {
        // the visited set for this budget does not fit a workgroup's LDS: a
        // bitmap over the vectors in global memory takes its place (the LDS
        // table's memory still holds the raw distance tables first)
        pl.gvis = true;
        pl.gvis_words = ceil_div(idx->n, 32);
        a.hash_buckets = 4;
        a.dc_buckets = 56;
        pl.lds1 = layout(a, qbytes, PK, pl.rcap, true, pl.bf16, lpr);
        const int slack = int(ceil_div(pl.lds1, kLdsGranule) * kLdsGranule) - pl.lds1;
        a.dc_buckets = uint32_t(std::min(128, 56 + slack / 32));
        pl.lds1 = layout(a, qbytes, PK, pl.rcap, true, pl.bf16, lpr);
    }
    pl.a2 = a;
    pl.lds2 = layout(pl.a2, qbytes, PK, pl.rcap, false, pl.bf16, lpr);

    // workspace: counters | slot bitmap | overflow list | order buckets |
    // order | global multi-sequence slots (a side holds at most K^2 elements)
    pl.gcap = std::min<int64_t>(int64_t(idx->K) * idx->K, 8192);
    pl.slot_bytes = size_t(mseq_slot_bytes(int(pl.gcap), idx->K, idx->P));
    const int64_t resident = int64_t(cus) * std::max(1, std::min(32, lds_cu / std::max(1, pl.lds1)));
    int64_t slots = resident;
    slots = std::min<int64_t>(slots, int64_t(kMaxSlotBytes / pl.slot_bytes));
    pl.max_slots = int(std::max<int64_t>(1, std::min<int64_t>(slots, s.nq)));
    if (pl.gvis) {
        const int64_t fit = std::max<int64_t>(1, int64_t(kMaxBitmapBytes / (size_t(pl.gvis_words) * 4)));
        pl.gvis_slots = int(std::max<int64_t>(1, std::min(std::min<int64_t>(resident, s.nq), fit)));
    }
    return ANN_OK;
}

// Budget classes.  With per-query budgets a launch serves up to four classes
// (T <= 512, T <= 2048, T <= 4096, larger) by one kernel each, in turn on the
// stream, each sized (LDS, multi-sequence capacity, slots) by its own largest
// budget: a few long queries then do not shrink the residency of the many
// short ones, and the longest class keeps the larger state it needs.
struct ClassPlan {
    Plan pl;
    int t_lo, t_hi;
};

// at most four classes, held in place (a search launch allocates nothing on
// the host either)
struct ClassPlans {
    ClassPlan c[4];
    int n = 0;
    ClassPlan* begin() { return c; }
    ClassPlan* end() { return c + n; }
    const ClassPlan* begin() const { return c; }
    const ClassPlan* end() const { return c + n; }
};

static int make_class_plans(const SearchLaunch& s, ClassPlans& out) {
    out.n = 0;
    int ranges[4][2];
    int nr = 0;
    if (!s.d_T || s.Tmax <= 512) {
        ranges[nr][0] = 0;
        ranges[nr++][1] = s.Tmax;
    } else {
        if (s.Tmax > 4096) {
            ranges[nr][0] = 4097;
            ranges[nr++][1] = s.Tmax;
        }
        if (s.Tmax > 2048) {
            ranges[nr][0] = 2049;
            ranges[nr++][1] = std::min(s.Tmax, 4096);
        }
        ranges[nr][0] = 513;
        ranges[nr++][1] = std::min(s.Tmax, 2048);
        ranges[nr][0] = 0;
        ranges[nr++][1] = 512;
    }
    for (int i = 0; i < nr; ++i) {
        SearchLaunch sc = s;
        sc.Tmax = ranges[i][1];
        ClassPlan& c = out.c[out.n];
        int rc = make_plan(sc, c.pl);
        if (rc) return rc;
        c.pl.a.Tall = c.pl.a2.Tall = s.Tmax;
        c.pl.a.t_lo = c.pl.a2.t_lo = ranges[i][0];
        c.pl.a.t_hi = c.pl.a2.t_hi = ranges[i][1];
        c.t_lo = ranges[i][0];
        c.t_hi = ranges[i][1];
        ++out.n;
    }
    return ANN_OK;
}

// workspace: counters | slot bitmap | overflow list | order buckets | order |
// global multi-sequence slots (the largest count any class uses)
struct WsLayout {
    int max_slots = 0, bit_words = 0;
    size_t slot_bytes = 0, fixed = 0, total = 0;
    int gvis_max = 0;        // visited bitmaps (0: every class keeps its set in LDS)
    size_t gvis_each = 0;    // bytes of one bitmap
};

static WsLayout ws_layout(const ClassPlans& cl, int64_t nq) {
    WsLayout L;
    for (const auto& c : cl) L.max_slots = std::max(L.max_slots, c.pl.max_slots);
    L.slot_bytes = cl.c[0].pl.slot_bytes;
    L.bit_words = int(ceil_div(L.max_slots, 32));
    L.fixed = (256 + round16(size_t(L.bit_words) * 4) + round16(size_t(nq) * 4) + 256 + round16(size_t(nq) * 4) + 63) &
              ~size_t(63);
    for (const auto& c : cl)
        if (c.pl.gvis) {
            L.gvis_max = std::max(L.gvis_max, c.pl.gvis_slots);
            L.gvis_each = (size_t(c.pl.gvis_words) * 4 + 255) & ~size_t(255);
        }
    L.total = L.fixed + size_t(L.gvis_max) * L.gvis_each + size_t(L.max_slots) * L.slot_bytes;
    return L;
}

// smallest workspace: one visited bitmap (if any class needs them) and one
// multi-sequence slot
static size_t ws_minimum(const WsLayout& L) { return L.fixed + (L.gvis_max > 0 ? L.gvis_each : 0) + L.slot_bytes; }

int search_workspace_bytes(const SearchLaunch& s, int64_t* bytes, bool minimum) {
    ClassPlans cl;
    int rc = make_class_plans(s, cl);
    if (rc) return rc;
    const WsLayout L = ws_layout(cl, s.nq);
    *bytes = int64_t(minimum ? ws_minimum(L) : L.total);
    return ANN_OK;
}

int search_lds_per_query(const SearchLaunch& s, int64_t* bytes) {
    ClassPlans cl;
    int rc = make_class_plans(s, cl);
    if (rc) return rc;
    int64_t most = 0;
    for (const auto& c : cl) most = std::max<int64_t>(most, ceil_div(c.pl.lds1, kLdsGranule) * kLdsGranule);
    *bytes = most;
    return ANN_OK;
}

int launch_search(const SearchLaunch& s) {
    if (s.nq == 0) return ANN_OK;
    ClassPlans cl;
    int rc = make_class_plans(s, cl);
    if (rc) return rc;
    const WsLayout L = ws_layout(cl, s.nq);

    int dev = 0, max_lds = 0, cus = 0;
    ANN_HIP_CHECK(hipGetDevice(&dev));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (const auto& c : cl)
        if (c.pl.lds1 > max_lds)
            return set_error(ANN_EUNSUPPORTED, "search needs " + std::to_string(c.pl.lds1) +
                                                   " bytes of LDS per query, more than the device's " +
                                                   std::to_string(max_lds) + " (lower budget or k)");

    uint8_t* w = static_cast<uint8_t*>(s.workspace);
    const bool own = w == nullptr;
    int avail = L.max_slots;
    int gv_avail = L.gvis_max;
    if (own) {
        ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&w), L.total, s.stream));
    } else {
        const size_t least = ws_minimum(L);
        ANN_REQUIRE(s.workspace_bytes >= int64_t(least),
                    "search: workspace too small (" + std::to_string(s.workspace_bytes) + " bytes, at least " +
                        std::to_string(least) + " needed)");
        ANN_REQUIRE((reinterpret_cast<uintptr_t>(w) & 15) == 0, "search: workspace must be 16-byte aligned");
        // bitmaps first (at least one each way), then multi-sequence slots
        const int64_t spare = s.workspace_bytes - int64_t(L.fixed);
        if (L.gvis_max > 0)
            gv_avail = int(std::max<int64_t>(
                1, std::min<int64_t>(L.gvis_max, (spare - int64_t(L.slot_bytes)) / int64_t(L.gvis_each))));
        avail = int(std::min<int64_t>(L.max_slots,
                                      (spare - int64_t(gv_avail) * int64_t(L.gvis_each)) / int64_t(L.slot_bytes)));
    }
    // [0] overflow count, [1] work counter
    uint32_t* counters = reinterpret_cast<uint32_t*>(w);
    size_t o = 256;
    uint32_t* slot_bits = reinterpret_cast<uint32_t*>(w + o);  // global slots in use
    o += round16(size_t(L.bit_words) * 4);
    uint32_t* ovf_list = reinterpret_cast<uint32_t*>(w + o);
    o += round16(size_t(s.nq) * 4);
    uint32_t* buckets = reinterpret_cast<uint32_t*>(w + o);  // 32 starts + 32 cursors
    o += 256;
    uint32_t* perm = reinterpret_cast<uint32_t*>(w + o);
    o += round16(size_t(s.nq) * 4);
    o = (o + 63) & ~size_t(63);  // == L.fixed
    uint32_t* gvis = reinterpret_cast<uint32_t*>(w + o);  // visited bitmaps
    o += size_t(gv_avail) * L.gvis_each;
    uint8_t* gheap = w + o;

    // the serving order (longest budgets first) is shared by the classes;
    // buffers are cleared by a kernel (no memset nodes in captured graphs)
    const uint32_t* order = nullptr;
    if (s.persistent && s.order && s.d_T) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(WAVE), 0, s.stream, buckets, 64);
        const unsigned gb = unsigned(ceil_div(s.nq, 256));
        hipLaunchKernelGGL(k_order_count, dim3(gb), dim3(256), 0, s.stream, s.d_T, s.nq, buckets);
        hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(WAVE), 0, s.stream, buckets);
        hipLaunchKernelGGL(k_order_scatter, dim3(gb), dim3(256), 0, s.stream, s.d_T, s.nq, buckets, buckets + 32,
                           perm);
        order = perm;
    }

    const Grid g{std::min<int64_t>(s.nq, int64_t(1) << 30), s.waves_per_cu, cus};
    const ann_index* idx = s.idx;
    for (auto& c : cl) {
        Plan& pl = c.pl;
        SearchArgs& a = pl.a;
        SearchArgs& a2 = pl.a2;
        const int nslots = std::min(pl.max_slots, avail);
        pl.grid2 = std::min(pl.grid2, nslots);
        if (pl.gvis) {
            a.gvis = a2.gvis = gvis;
            a.gvis_words = a2.gvis_words = pl.gvis_words;
            a.gvis_slots = a2.gvis_slots = std::min(pl.gvis_slots, gv_avail);
            pl.grid2 = std::min(pl.grid2, a.gvis_slots);
        } else {
            a.gvis = a2.gvis = nullptr;
        }
        a.ovf_count = a2.ovf_count = counters;
        a.ovf_list = a2.ovf_list = ovf_list;
        a.gheap = a2.gheap = gheap;
        a.gms_cap = a2.gms_cap = int(pl.gcap);
        a.nslots = a2.nslots = nslots;
        a.slot_bits = a2.slot_bits = slot_bits;
        a2.ms_cap = a.ms_cap;
        a.work_counter = s.persistent ? counters + 1 : nullptr;
        a2.work_counter = nullptr;
        a.perm = order;
        a2.perm = nullptr;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(WAVE), 0, s.stream, counters, 64);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(WAVE), 0, s.stream, slot_bits, L.bit_words);
        if (!pl.is_f32) {
            if (idx->row_bytes == 128)
                rc = launch_kpl<MODE_U8, 8>(pl.rcap, a, a2, pl.lds1, pl.lds2, g, pl.grid2, s.stream);
            else
                rc = launch_kpl<MODE_U8, 0>(pl.rcap, a, a2, pl.lds1, pl.lds2, g, pl.grid2, s.stream);
        } else if (pl.bf16) {
            if (idx->d == 384)
                rc = launch_kpl<MODE_BF16, 48>(pl.rcap, a, a2, pl.lds1, pl.lds2, g, pl.grid2, s.stream);
            else
                rc = launch_kpl<MODE_BF16, 0>(pl.rcap, a, a2, pl.lds1, pl.lds2, g, pl.grid2, s.stream);
        } else {
            if (idx->d == 384)
                rc = launch_kpl<MODE_F32, 96>(pl.rcap, a, a2, pl.lds1, pl.lds2, g, pl.grid2, s.stream);
            else
                rc = launch_kpl<MODE_F32, 0>(pl.rcap, a, a2, pl.lds1, pl.lds2, g, pl.grid2, s.stream);
        }
        if (rc) return rc;
        ANN_HIP_CHECK(hipGetLastError());
    }
    if (own) ANN_HIP_CHECK(hipFreeAsync(w, s.stream));
    return ANN_OK;
}

int launch_tables(const ann_index* idx, const void* d_q, int64_t nq, void* d_sorted, int32_t* d_perm,
                  hipStream_t s) {
    if (nq == 0) return ANN_OK;
    const bool is_f32 = idx->dtype == ANN_F32;
    const int qbytes = is_f32 ? idx->d * 4 : idx->d;
    const int PK = idx->P * idx->K;
    const int lds = align_up(qbytes, 16) + PK * 4 * 2 + PK + 16;
    const int64_t grid = std::min<int64_t>(nq, int64_t(1) << 30);
    if (is_f32)
        hipLaunchKernelGGL(k_tables<true>, dim3(unsigned(grid)), dim3(WAVE), lds, s, d_q, nq, idx->d,
                           idx->codebooks, idx->P, idx->K, idx->d / idx->P, static_cast<uint32_t*>(d_sorted),
                           d_perm);
    else
        hipLaunchKernelGGL(k_tables<false>, dim3(unsigned(grid)), dim3(WAVE), lds, s, d_q, nq, idx->d,
                           idx->codebooks, idx->P, idx->K, idx->d / idx->P, static_cast<uint32_t*>(d_sorted),
                           d_perm);
    ANN_HIP_CHECK(hipGetLastError());
    return ANN_OK;
}

}  // namespace ann
