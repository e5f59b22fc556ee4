// Search over the augmented neighborhood graph (Sec. 4.2, Alg. 1) on gfx950.
//
// One wavefront (64 lanes, one workgroup) serves one query at a time:
//   1. query tables: P x K squared subspace distances, each subspace sorted
//      by (value, codeword)                                   (Sec. 4.2)
//   2. multi-sequence extraction of bridge vectors in (distance, lid) order;
//      the frontier is a binary heap in LDS driven by one lane.  Because the
//      bridge order does not depend on the traversal, bridges are extracted
//      ahead in batches and their CSR offsets are read by all lanes at once;
//      empty bridges are dropped there (expanding one changes nothing).
//                                                            (Sec. 3.3)
//   3. best-first expansion: the smaller of the main-queue head and the
//      next bridge is expanded; white neighbours are marked in an exact
//      open-addressing hash in LDS, the first (T - t) of them in adjacency
//      order are evaluated; each row is gathered by a group of lanes and
//      reduced across the group; the results are merged into the bounded
//      main queue and the result set, both sorted arrays in LDS. (Alg. 1)
#include "internal.hpp"
#include "mseq.hpp"

namespace ann {
namespace {

enum { MODE_U8 = 0, MODE_F32 = 1, MODE_BF16 = 2 };

constexpr int GEN_BATCH = 32;  // bridges extracted per look-ahead step

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
    int hash_bits;
    int heap_cap;
    // LDS layout (byte offsets)
    int o_q, o_tab, o_sv, o_perm, o_hk, o_hr, o_rk, o_ro, o_rl, o_sk, o_hash, o_qa, o_qb, o_ra, o_rb, o_ek,
        o_eid, o_sc;
};

template <int MODE>
struct Traits;
template <>
struct Traits<MODE_U8> {
    static constexpr int LPR = 4;  // lanes per gathered row
    static constexpr bool FLOAT = false;
};
template <>
struct Traits<MODE_F32> {
    static constexpr int LPR = 16;
    static constexpr bool FLOAT = true;
};
template <>
struct Traits<MODE_BF16> {
    static constexpr int LPR = 16;
    static constexpr bool FLOAT = true;
};

// ------------------------------------------------------------------
// squared distance of one gathered row, partial sum of this lane
// ------------------------------------------------------------------
template <int MODE>
__device__ inline uint32_t row_partial(const uint8_t* row, const uint8_t* qv, int nc16, int part);

template <>
__device__ inline uint32_t row_partial<MODE_U8>(const uint8_t* row, const uint8_t* qv, int nc16, int part) {
    // sum (q-x)^2 = sum q^2 + sum x^2 - 2 sum q*x, every term an exact integer
    uint32_t xx = 0, qq = 0, qx = 0;
    for (int c = part; c < nc16; c += 4) {
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
    return xx + qq - 2u * qx;  // modulo 2^32; the 4-lane total is exact
}

template <>
__device__ inline uint32_t row_partial<MODE_F32>(const uint8_t* row, const uint8_t* qv, int nc16, int part) {
    float acc = 0.f;
    for (int c = part; c < nc16; c += 16) {
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
__device__ inline uint32_t row_partial<MODE_BF16>(const uint8_t* row, const uint8_t* qv, int nc16, int part) {
    // row chunk c holds bf16 dims [8c, 8c+8); the query stays fp32
    float acc = 0.f;
    for (int c = part; c < nc16; c += 16) {
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

// total over the LPR lanes of a row group (fixed butterfly order)
template <int MODE>
__device__ inline uint32_t group_sum(uint32_t v) {
    if constexpr (!Traits<MODE>::FLOAT) {
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        return v;
    } else {
        float f = bits_f(v);
#pragma unroll
        for (int m = 1; m < Traits<MODE>::LPR; m <<= 1) f += __shfl_xor(f, m);
        return f_bits(f);
    }
}

// ------------------------------------------------------------------
// visited set: open addressing with linear probing, exact
// ------------------------------------------------------------------
__device__ inline bool hash_insert(uint32_t* H, int bits, uint32_t id) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t s = (id * 0x9E3779B1u) >> (32 - bits);
    for (;;) {
        const uint32_t old = atomicCAS(&H[s], ID_EMPTY, id);
        if (old == ID_EMPTY) return true;
        if (old == id) return false;
        s = (s + 1u) & mask;
    }
}

// ------------------------------------------------------------------
// Merge m new keys nk[0..m) (distinct, not present) into the sorted live
// range src[h .. h+n), keep the `cap` smallest, write them to dst[0..).
// Returns the new size.  Equivalent to offering the keys one by one to a
// bounded set that evicts its largest key when full.
// ------------------------------------------------------------------
__device__ int merge_keep(const uint64_t* src, int h, int n, uint64_t* dst, int cap, const uint64_t* nk, int m,
                          int lane) {
    const int total = min(cap, n + m);
    for (int i = lane; i < n; i += WAVE) {
        const uint64_t v = src[h + i];
        int c = 0;
        for (int j = 0; j < m; ++j) c += nk[j] < v;
        const int pos = i + c;
        if (pos < total) dst[pos] = v;
    }
    if (lane < m) {
        const uint64_t v = nk[lane];
        int c = 0;
        for (int j = 0; j < m; ++j) c += nk[j] < v;
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (src[h + mid] < v)
                lo = mid + 1;
            else
                hi = mid;
        }
        const int pos = c + lo;
        if (pos < total) dst[pos] = v;
    }
    __syncthreads();
    return total;
}

// true if any of the m new keys would enter a set of capacity cap
__device__ inline bool any_admitted(const uint64_t* src, int h, int n, int cap, const uint64_t* nk, int m, int lane) {
    if (m == 0 || cap == 0) return false;
    if (n < cap) return true;
    const uint64_t worst = src[h + n - 1];
    return __ballot(lane < m && nk[lane] < worst) != 0;
}

template <int MODE>
__global__ void __launch_bounds__(WAVE) k_search(SearchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr bool FLOAT = Traits<MODE>::FLOAT;
    constexpr int LPR = Traits<MODE>::LPR;
    constexpr int RPP = WAVE / LPR;  // rows per gather pass

    uint8_t* qv = lds + a.o_q;
    uint32_t* tab = reinterpret_cast<uint32_t*>(lds + a.o_tab);
    uint32_t* sv = reinterpret_cast<uint32_t*>(lds + a.o_sv);
    uint8_t* perm = lds + a.o_perm;
    uint64_t* hk = reinterpret_cast<uint64_t*>(lds + a.o_hk);
    uint32_t* hr = reinterpret_cast<uint32_t*>(lds + a.o_hr);
    uint64_t* ring_key = reinterpret_cast<uint64_t*>(lds + a.o_rk);
    uint32_t* ring_off = reinterpret_cast<uint32_t*>(lds + a.o_ro);
    uint32_t* ring_len = reinterpret_cast<uint32_t*>(lds + a.o_rl);
    uint64_t* stage = reinterpret_cast<uint64_t*>(lds + a.o_sk);
    uint32_t* H = reinterpret_cast<uint32_t*>(lds + a.o_hash);
    uint64_t* QA = reinterpret_cast<uint64_t*>(lds + a.o_qa);
    uint64_t* QB = reinterpret_cast<uint64_t*>(lds + a.o_qb);
    uint64_t* RA = reinterpret_cast<uint64_t*>(lds + a.o_ra);
    uint64_t* RB = reinterpret_cast<uint64_t*>(lds + a.o_rb);
    uint64_t* ek = reinterpret_cast<uint64_t*>(lds + a.o_ek);
    uint32_t* eid = reinterpret_cast<uint32_t*>(lds + a.o_eid);
    int* sc = reinterpret_cast<int*>(lds + a.o_sc);

    const int lane = lane_id();
    const int part = lane % LPR;
    const int grp = lane / LPR;
    const int64_t n = a.n;
    const int P = a.P, K = a.K;
    const int HS = 1 << a.hash_bits;
    const int qbytes = FLOAT ? a.d * 4 : a.d;
    const int nc16 = int(a.row_bytes / 16);

    for (int64_t qi = blockIdx.x; qi < a.nq; qi += gridDim.x) {
        // per-query values are clamped to the launch maxima that sized the buffers
        const int k = a.ks ? min(max(a.ks[qi], 1), a.kmax) : a.kmax;
        const int T = a.Ts ? min(max(a.Ts[qi], 0), a.Tmax) : a.Tmax;
        const int rcap = (MODE == MODE_BF16) ? max(k, a.rerank_k) : k;

        // ---- load the query, clear the visited set
        {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(a.Q) + qi * qbytes);
            uint32_t* dst = reinterpret_cast<uint32_t*>(qv);
            for (int i = lane; i < qbytes / 4; i += WAVE) dst[i] = src[i];
            for (int i = lane; i < HS; i += WAVE) H[i] = ID_EMPTY;
        }
        __syncthreads();

        // ---- tables and their sort; the nearest bridge seeds the frontier
        compute_tables<FLOAT>(qv, a.cb, P, K, a.ds, tab, sv, perm, lane);
        if (lane == 0) {
            int hn = 0;
            heap_push(hk, hr, hn, tuple_key<FLOAT>(0u, sv, perm, P, K, n), 0u);
            sc[0] = hn;
            sc[1] = 0;  // overflow flag
        }
        __syncthreads();

        int heap_n = sc[0];
        int heap_max = heap_n;
        int flags = 0;
        int ring_h = 0, ring_n = 0;
        int qh = 0, qn = 0, rn = 0;
        uint64_t* Qc = QA;
        uint64_t* Qn = QB;
        uint64_t* Rc = RA;
        uint64_t* Rn = RB;
        int t = 0;
        int st_rpop = 0, st_bpop = 0, st_bids = 0, st_gen = 0;

        while (t < T) {
            // ---- look-ahead extraction of the next non-empty bridges
            while (ring_h == ring_n && heap_n > 0 && flags == 0) {
                if (lane == 0) {
                    int hn = heap_n, g = 0, of = 0;
                    for (; g < GEN_BATCH && hn > 0; ++g) {
                        uint64_t key;
                        uint32_t rk;
                        heap_pop(hk, hr, hn, key, rk);
                        stage[g] = key;
                        // unique-parent rule: raise one rank at or after the last non-zero one
                        int last = 0;
                        for (int p = 0; p < P; ++p)
                            if ((rk >> (8 * p)) & 0xFF) last = p;
                        for (int b = last; b < P; ++b) {
                            const int r = (rk >> (8 * b)) & 0xFF;
                            if (r + 1 >= K) continue;
                            if (hn >= a.heap_cap) {
                                of = 1;
                                break;
                            }
                            const uint32_t crk = rk + (1u << (8 * b));
                            heap_push(hk, hr, hn, tuple_key<FLOAT>(crk, sv, perm, P, K, n), crk);
                        }
                        if (of) {
                            ++g;
                            break;
                        }
                    }
                    sc[0] = hn;
                    sc[1] = of;
                    sc[2] = g;
                }
                __syncthreads();
                heap_n = sc[0];
                heap_max = max(heap_max, heap_n);
                const int g = sc[2];
                if (sc[1]) flags = ANN_ERESOURCE;
                st_gen += g;
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
                if (ne) {
                    const int pos = lanes_below(mask);
                    ring_key[pos] = key;
                    ring_off[pos] = o0;
                    ring_len[pos] = o1 - o0;
                }
                ring_h = 0;
                ring_n = __popcll(mask);
                __syncthreads();
            }
            if (flags) break;

            // ---- pop the best of the queue head and the next bridge
            const uint64_t bkey = ring_h < ring_n ? ring_key[ring_h] : KEY_EMPTY;
            const uint64_t qkey = qn > 0 ? Qc[qh] : KEY_EMPTY;
            const uint32_t* src;
            int64_t base;
            int len;
            if (ring_h < ring_n && bkey < qkey) {
                src = a.bids;
                base = ring_off[ring_h];
                len = int(ring_len[ring_h]);
                ++ring_h;
                ++st_bpop;
                st_bids += len;
            } else if (qn > 0) {
                src = a.G;
                base = int64_t(key_id(qkey)) * a.R;
                len = a.R;
                ++qh;
                --qn;
                ++st_rpop;
            } else {
                break;  // queue empty and every bridge consumed
            }

            // ---- expand: 64 adjacency entries at a time
            for (int c0 = 0; c0 < len && t < T; c0 += WAVE) {
                const int j = c0 + lane;
                const uint32_t id = j < len ? src[base + j] : ID_EMPTY;
                const bool white = id != ID_EMPTY && hash_insert(H, a.hash_bits, id);
                const uint64_t wm = __ballot(white);
                const int take = min(int(__popcll(wm)), T - t);
                const int r = lanes_below(wm);
                if (white && r < take) eid[r] = id;
                __syncthreads();

                // gather and distance, RPP rows per pass
                for (int p0 = 0; p0 < take; p0 += RPP) {
                    const int row = p0 + grp;
                    uint32_t part_sum = 0;
                    uint32_t rid = 0;
                    if (row < take) {
                        rid = eid[row];
                        part_sum = row_partial<MODE>(a.X + int64_t(rid) * a.row_bytes, qv, nc16, part);
                    }
                    const uint32_t dsum = group_sum<MODE>(part_sum);
                    if (part == 0 && row < take) ek[row] = make_key(dsum, rid);
                }
                __syncthreads();
                if (a.trace && lane < take) a.trace[qi * a.Tmax + t + lane] = int32_t(eid[lane]);

                if (any_admitted(Rc, 0, rn, rcap, ek, take, lane)) {
                    rn = merge_keep(Rc, 0, rn, Rn, rcap, ek, take, lane);
                    uint64_t* tmp = Rc;
                    Rc = Rn;
                    Rn = tmp;
                }
                if (any_admitted(Qc, qh, qn, a.L, ek, take, lane)) {
                    qn = merge_keep(Qc, qh, qn, Qn, a.L, ek, take, lane);
                    qh = 0;
                    uint64_t* tmp = Qc;
                    Qc = Qn;
                    Qn = tmp;
                }
                t += take;
            }
        }

        // ---- bf16 mode: re-rank the kept candidates with fp32 rows
        if constexpr (MODE == MODE_BF16) {
            const int nc16f = int(a.row_bytes_f32 / 16);
            for (int p0 = 0; p0 < rn; p0 += RPP) {
                const int row = p0 + grp;
                uint32_t part_sum = 0, rid = 0;
                if (row < rn) {
                    rid = key_id(Rc[row]);
                    part_sum = row_partial<MODE_F32>(a.Xf32 + int64_t(rid) * a.row_bytes_f32, qv, nc16f, part);
                }
                const uint32_t dsum = group_sum<MODE_F32>(part_sum);
                if (part == 0 && row < rn) Rn[row] = make_key(dsum, rid);
            }
            __syncthreads();
            for (int i = lane; i < rn; i += WAVE) {
                const uint64_t v = Rn[i];
                int r = 0;
                for (int jj = 0; jj < rn; ++jj) r += Rn[jj] < v;
                Rc[r] = v;
            }
            __syncthreads();
        }

        // ---- results, ascending by (distance, id), padded
        for (int i = lane; i < a.kmax; i += WAVE) {
            const int64_t o = qi * a.kmax + i;
            if (flags == 0 && i < k && i < rn) {
                const uint64_t v = Rc[i];
                a.out_ids[o] = int32_t(key_id(v));
                static_cast<uint32_t*>(a.out_d)[o] = key_dist(v);
            } else {
                a.out_ids[o] = -1;
                static_cast<uint32_t*>(a.out_d)[o] = FLOAT ? 0x7F800000u : 0x7FFFFFFFu;
            }
        }
        if (a.trace)
            for (int i = t + lane; i < T; i += WAVE) a.trace[qi * a.Tmax + i] = -1;
        if (a.trace)
            for (int i = T + lane; i < a.Tmax; i += WAVE) a.trace[qi * a.Tmax + i] = -1;
        if (a.stats && lane == 0) {
            int32_t* s = a.stats + qi * ANN_NSTATS;
            s[ANN_STAT_EVALS] = t;
            s[ANN_STAT_REF_POPS] = st_rpop;
            s[ANN_STAT_BRIDGE_POPS] = st_bpop;
            s[ANN_STAT_BRIDGE_IDS] = st_bids;
            s[ANN_STAT_BRIDGES_GEN] = st_gen;
            s[ANN_STAT_HEAP_MAX] = heap_max;
            s[ANN_STAT_FLAGS] = flags;
            s[ANN_STAT_RESERVED] = 0;
        }
        __syncthreads();
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

}  // namespace

int launch_search(const SearchLaunch& s) {
    const ann_index* idx = s.idx;
    if (s.nq == 0) return ANN_OK;
    SearchArgs a{};
    const bool is_f32 = idx->dtype == ANN_F32;
    const bool bf16 = is_f32 && s.precision == ANN_PRECISION_BF16_RERANK;
    if (bf16) {
        ANN_REQUIRE(idx->Xbf16 != nullptr, "bf16 copy of the vectors is missing");
        ANN_REQUIRE(idx->d % 8 == 0, "bf16 precision needs d divisible by 8");
    }
    a.X = bf16 ? reinterpret_cast<const uint8_t*>(idx->Xbf16) : idx->X;
    a.Xf32 = idx->X;
    a.row_bytes = bf16 ? int64_t(idx->d) * 2 : idx->row_bytes;
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
    a.L = s.L;
    a.rerank_k = s.rerank_k > 0 ? s.rerank_k : s.kmax;
    a.out_ids = s.d_ids;
    a.out_d = s.d_dists;
    a.stats = s.d_stats;
    a.trace = s.d_trace;

    // visited set: >= 1.5 x (budget + one adjacency chunk) slots, a power of two
    int bits = 6;
    while ((1 << bits) < (3 * (s.Tmax + WAVE)) / 2) ++bits;
    a.hash_bits = bits;
    // multi-sequence frontier: one pop adds at most P - 1 entries; it never
    // holds more than the K^P tuples
    a.heap_cap = int(std::min<int64_t>(idx->nb, std::max(256, s.Tmax + 64 * idx->P)));

    const int qbytes = is_f32 ? idx->d * 4 : idx->d;
    const int PK = idx->P * idx->K;
    const int rcap = bf16 ? std::max(s.kmax, a.rerank_k) : s.kmax;
    int off = 0;
    auto take = [&](int bytes, int al) {
        off = align_up(off, al);
        int o = off;
        off += bytes;
        return o;
    };
    a.o_q = take(align_up(qbytes, 16), 16);
    a.o_tab = take(PK * 4, 8);
    a.o_sv = take(PK * 4, 8);
    a.o_perm = take(PK, 8);
    a.o_hk = take(a.heap_cap * 8, 8);
    a.o_hr = take(a.heap_cap * 4, 8);
    a.o_rk = take(WAVE * 8, 8);
    a.o_ro = take(WAVE * 4, 8);
    a.o_rl = take(WAVE * 4, 8);
    a.o_sk = take(WAVE * 8, 8);
    a.o_hash = take((1 << bits) * 4, 8);
    a.o_qa = take(s.L * 8, 8);
    a.o_qb = take(s.L * 8, 8);
    a.o_ra = take(rcap * 8, 8);
    a.o_rb = take(rcap * 8, 8);
    a.o_ek = take(WAVE * 8, 8);
    a.o_eid = take(WAVE * 4, 8);
    a.o_sc = take(16 * 4, 8);
    const int lds_bytes = align_up(off, 16);

    int dev = 0, max_lds = 0;
    ANN_HIP_CHECK(hipGetDevice(&dev));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds_bytes > max_lds)
        return set_error(ANN_EUNSUPPORTED, "search needs " + std::to_string(lds_bytes) +
                                               " bytes of LDS per query, more than the device's " +
                                               std::to_string(max_lds) + " (lower budget or k)");
    const int64_t grid = std::min<int64_t>(s.nq, int64_t(1) << 30);
    if (!is_f32) {
        hipLaunchKernelGGL(k_search<MODE_U8>, dim3(unsigned(grid)), dim3(WAVE), lds_bytes, s.stream, a);
    } else if (bf16) {
        hipLaunchKernelGGL(k_search<MODE_BF16>, dim3(unsigned(grid)), dim3(WAVE), lds_bytes, s.stream, a);
    } else {
        hipLaunchKernelGGL(k_search<MODE_F32>, dim3(unsigned(grid)), dim3(WAVE), lds_bytes, s.stream, a);
    }
    ANN_HIP_CHECK(hipGetLastError());
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
