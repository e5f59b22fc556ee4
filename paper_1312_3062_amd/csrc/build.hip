// Index build on the GPU (Sec. 4.1): product-quantisation codebooks by
// k-means per subspace, and the bridge graph linking bridge vectors
// (Cartesian concatenations of codewords) to reference vectors.
#include <algorithm>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "mseq.hpp"

namespace ann {

// ----------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, 2014): add the golden-ratio increment,
// then two xor-shift-multiply rounds and a final xor-shift.
// ----------------------------------------------------------------------
static uint64_t splitmix64(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// First K positions of a Fisher-Yates shuffle of [0, n): the initial rows.
// Only the positions a swap has touched are stored (a vocabulary of millions
// of rows is drawn in time linear in K).
void kmeans_init_rows(int64_t n, int K, uint64_t seed, int64_t* rows) {
    std::unordered_map<int64_t, int64_t> moved;  // position -> value, where it differs from the position
    moved.reserve(size_t(2) * size_t(K));
    auto value_at = [&](int64_t i) {
        const auto it = moved.find(i);
        return it == moved.end() ? i : it->second;
    };
    uint64_t st = seed;
    for (int i = 0; i < K; ++i) {
        const int64_t j = i + int64_t(splitmix64(st) % uint64_t(n - i));
        const int64_t vi = value_at(i), vj = value_at(j);
        moved[i] = vj;
        moved[j] = vi;
        rows[i] = vj;
    }
}

namespace {

constexpr int KM_THREADS = 256;

// ----------------------------------------------------------------------
// k-means (Sec. 3.2 product quantisation, per subspace), one subspace at a
// time.
//   assign: one thread per point; the subspace's codewords stream through
//     LDS in chunks, every thread reading the same codeword at once.
//     u8: nearest by |c|^2 - 2 x.c (|x|^2 is common), exact ints;
//     f32: nearest by the fp32 sum of (x - c)^2.  Ties go to the smaller j.
//   accum: member sums over a slice of at most 64 dimensions; lanes cover
//     consecutive dimensions of one point (coalesced rows, distinct LDS
//     addresses), per-workgroup sums in LDS, then global atomics.  u8 sums
//     are exact integers; f32 values enter as int64 fixed point
//     (x * 2^scale rounded), so the order of the additions does not matter.
// ----------------------------------------------------------------------
template <bool FLOAT>
using lsum_t = typename std::conditional<FLOAT, unsigned long long, unsigned int>::type;

constexpr int KM_CHUNK_BYTES = 32768;  // codewords staged in LDS per pass
constexpr int KM_SLICE = 64;           // dimensions summed by one workgroup
constexpr int KM_POINTS = 2048;        // points per accumulation workgroup

// MAXDS > 0: the point's subvector (ds <= MAXDS dims, a multiple of 4 for
// u8) is held in registers for the whole codeword loop; MAXDS = 0 reads it
// again for every codeword (any ds; used above 128 dims).  The arithmetic and its order are the
// same either way.
template <bool FLOAT, int MAXDS>
__global__ void __launch_bounds__(KM_THREADS) k_kmeans_assign(const uint8_t* X, int64_t n, int d, int ds, int p, int K,
                                                              const void* cb_p, int kc, int32_t* assign) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int esz = FLOAT ? 4 : 1;
    uint8_t* c_l = lds;                                                  // kc codewords
    uint32_t* cnorm = reinterpret_cast<uint32_t*>(lds + ((kc * ds * esz + 15) & ~15));  // u8: |c|^2
    const int64_t i = int64_t(blockIdx.x) * KM_THREADS + threadIdx.x;
    const bool live = i < n;
    constexpr int RW = MAXDS > 0 ? (FLOAT ? MAXDS : MAXDS / 4) : 1;  // register words of the subvector
    float xf[FLOAT ? RW : 1];
    uint32_t xu[FLOAT ? 1 : RW];
    if constexpr (MAXDS > 0) {
        if (live) {
            if constexpr (FLOAT) {
                const float* x = reinterpret_cast<const float*>(X) + i * d + int64_t(p) * ds;
#pragma unroll
                for (int e = 0; e < RW; ++e) xf[e] = e < ds ? x[e] : 0.f;
            } else {
                const uint8_t* x = X + i * d + int64_t(p) * ds;
#pragma unroll
                for (int w = 0; w < RW; ++w) {
                    uint32_t v = 0;
                    if (4 * w < ds) __builtin_memcpy(&v, x + 4 * w, 4);
                    xu[w] = v;
                }
            }
        }
    }
    int best = 0;
    uint32_t bd = 0;
    for (int j0 = 0; j0 < K; j0 += kc) {
        const int m = min(kc, K - j0);
        __syncthreads();
        const int words = (m * ds * esz) / 4;
        const uint8_t* src = static_cast<const uint8_t*>(cb_p) + int64_t(j0) * ds * esz;
        for (int w = threadIdx.x; w < words; w += KM_THREADS)
            reinterpret_cast<uint32_t*>(c_l)[w] = reinterpret_cast<const uint32_t*>(src)[w];
        for (int w = words * 4 + threadIdx.x; w < m * ds * esz; w += KM_THREADS) c_l[w] = src[w];
        __syncthreads();
        if constexpr (!FLOAT) {
            for (int e = threadIdx.x; e < m; e += KM_THREADS) {
                uint32_t s2 = 0;
                for (int q = 0; q < ds; ++q) s2 += uint32_t(c_l[e * ds + q]) * c_l[e * ds + q];
                cnorm[e] = s2;
            }
            __syncthreads();
        }
        if (!live) continue;
        for (int jj = 0; jj < m; ++jj) {
            const int j = j0 + jj;
            uint32_t dist;
            if constexpr (!FLOAT) {
                const uint8_t* c = c_l + jj * ds;
                uint32_t dot = 0;
                if constexpr (MAXDS > 0) {
#pragma unroll
                    for (int w = 0; w < RW; ++w) {
                        if (4 * w < ds) {
                            uint32_t cw;
                            __builtin_memcpy(&cw, c + 4 * w, 4);
                            dot = __builtin_amdgcn_udot4(xu[w], cw, dot, false);
                        }
                    }
                } else {
                    const uint8_t* x = X + i * d + int64_t(p) * ds;
                    int e = 0;
                    if ((ds & 3) == 0) {
                        for (; e < ds; e += 4) {
                            uint32_t xw, cw;
                            __builtin_memcpy(&xw, x + e, 4);
                            __builtin_memcpy(&cw, c + e, 4);
                            dot = __builtin_amdgcn_udot4(xw, cw, dot, false);
                        }
                    }
                    for (; e < ds; ++e) dot += uint32_t(x[e]) * c[e];
                }
                dist = cnorm[jj] - 2u * dot + 0x80000000u;  // order-preserving bias (value may be negative)
            } else {
                const float* c = reinterpret_cast<const float*>(c_l) + jj * ds;
                float acc = 0.f;
                if constexpr (MAXDS > 0) {
#pragma unroll
                    for (int e = 0; e < RW; ++e) {
                        if (e < ds) {
                            const float t = xf[e] - c[e];
                            acc = fmaf(t, t, acc);
                        }
                    }
                } else {
                    const float* x = reinterpret_cast<const float*>(X) + i * d + int64_t(p) * ds;
                    for (int e = 0; e < ds; ++e) {
                        const float t = x[e] - c[e];
                        acc = fmaf(t, t, acc);
                    }
                }
                dist = __float_as_uint(acc);
            }
            if (j == 0 || dist < bd) {
                bd = dist;
                best = j;
            }
        }
    }
    if (live) assign[i] = best;
}

// ----------------------------------------------------------------------
// u8 assignment on matrix cores.  With u = x - 128 and v = c - 128 as int8,
// |x - c|^2 = |u|^2 + |v|^2 - 2 u.v, so a point's nearest codeword minimises
// w = |v|^2 - 2 u.v (exact in int32, |u|^2 being common to its codewords),
// and u.v comes from v_mfma_i32_16x16x64_i8.  The subspace's codewords (at
// most 256, ds <= 128 dimensions, a multiple of 16) sit in LDS shifted and
// zero-padded to 64-byte k-slices (rows padded by 16 bytes for distinct
// banks).  Four wavefronts of 64 points each keep their operands in
// registers: lane l holds point l % 16 of each 16-point block (bytes
// 16 (l / 16) .. +15 of a k-slice) and, per block of 16 codewords, the
// results of points 4 (l / 16) .. +3 against codeword l % 16 of the block.
// A key (w + 2^23) << 8 | j orders by w, then by the smaller j (the tie rule
// of the scalar form: |w| < 2^23 at ds <= 128); the minimum over the 16 lanes
// of a row (DPP) is the point's codeword.
// ----------------------------------------------------------------------
typedef int km_v4i32 __attribute__((ext_vector_type(4)));
constexpr int KMM_MAXK = 256;

template <int CTRL>
__device__ inline uint32_t row_min_step(uint32_t v) {
    const uint32_t o = uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), CTRL, 0xF, 0xF, false));
    return o < v ? o : v;
}

template <int KS>
__global__ void __launch_bounds__(256) k_kmeans_assign_mfma(const uint8_t* X, int64_t n, int d, int ds, int p, int K,
                                                           const uint8_t* cb, int32_t* assign) {
    constexpr int STRIDE = KS * 64 + 16;
    constexpr int C16 = KS * 4;  // 16-byte chunks of a padded codeword
    __shared__ __align__(16) uint8_t cw[KMM_MAXK * STRIDE];
    __shared__ int vn[KMM_MAXK];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    for (int i = threadIdx.x; i < K * C16; i += 256) {
        const int j = i / C16, c = i - j * C16;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (c * 16 < ds) {
            v = *reinterpret_cast<const uint4*>(cb + int64_t(j) * ds + c * 16);
            v.x ^= 0x80808080u;
            v.y ^= 0x80808080u;
            v.z ^= 0x80808080u;
            v.w ^= 0x80808080u;
        }
        *reinterpret_cast<uint4*>(cw + j * STRIDE + c * 16) = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < K; j += 256) {
        int sq = 0;
        for (int e = 0; e < ds; ++e) {
            const int v = int(int8_t(cw[j * STRIDE + e]));
            sq += v * v;
        }
        vn[j] = sq;
    }
    const int64_t row0 = int64_t(blockIdx.x) * 256 + wv * 64;
    km_v4i32 a[4][KS];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t r = min<int64_t>(row0 + rb * 16 + col, n - 1);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int off = s * 64 + kq * 16;
            uint4 v = make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u);  // 0 once shifted
            if (off < ds) v = *reinterpret_cast<const uint4*>(X + r * d + int64_t(p) * ds + off);
            a[rb][s] = km_v4i32{int(v.x ^ 0x80808080u), int(v.y ^ 0x80808080u), int(v.z ^ 0x80808080u),
                                int(v.w ^ 0x80808080u)};
        }
    }
    __syncthreads();
    uint32_t best[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int t = 0; t < 4; ++t) best[rb][t] = 0xFFFFFFFFu;
    for (int c0 = 0; c0 < K; c0 += 16) {
        const int j = c0 + col;  // this lane's codeword; past K: read, then ignored
        km_v4i32 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = km_v4i32{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const km_v4i32 b = *reinterpret_cast<const km_v4i32*>(cw + j * STRIDE + s * 64 + kq * 16);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rb][s], b, acc[rb], 0, 0, 0);
        }
        if (j < K) {
            const int vj = vn[j];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t key = (uint32_t(vj - 2 * acc[rb][t] + (1 << 23)) << 8) | uint32_t(j);
                    best[rb][t] = key < best[rb][t] ? key : best[rb][t];
                }
        }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t v = best[rb][t];
            v = row_min_step<0xB1>(v);   // quad_perm 1,0,3,2
            v = row_min_step<0x4E>(v);   // quad_perm 2,3,0,1
            v = row_min_step<0x141>(v);  // row_half_mirror
            v = row_min_step<0x140>(v);  // row_mirror: the row's minimum in all 16 lanes
            const int64_t r = row0 + rb * 16 + 4 * kq + t;
            if (col == 0 && r < n) assign[r] = int32_t(v & 0xFFu);
        }
}

// one assignment launch for subspace p, the register form when ds allows
template <bool FLOAT>
void launch_kmeans_assign(const uint8_t* X, int64_t n, int d, int ds, int p, int K, const void* cb_p, int kc,
                          int lds, int32_t* assign, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(ceil_div(n, KM_THREADS)));
    if constexpr (!FLOAT) {
        // matrix cores: subvectors of 16..128 bytes in 16-byte steps, rows of
        // 16-byte multiples, at most 256 codewords
        if (ds % 16 == 0 && ds >= 16 && ds <= 128 && d % 16 == 0 && K >= 1 && K <= KMM_MAXK) {
            if (ds <= 64)
                hipLaunchKernelGGL(k_kmeans_assign_mfma<1>, grid, dim3(256), 0, s, X, n, d, ds, p, K,
                                   static_cast<const uint8_t*>(cb_p), assign);
            else
                hipLaunchKernelGGL(k_kmeans_assign_mfma<2>, grid, dim3(256), 0, s, X, n, d, ds, p, K,
                                   static_cast<const uint8_t*>(cb_p), assign);
            return;
        }
    }
    const bool words = FLOAT || (ds & 3) == 0;
    if (words && ds <= 16)
        hipLaunchKernelGGL((k_kmeans_assign<FLOAT, 16>), grid, dim3(KM_THREADS), lds, s, X, n, d, ds, p, K, cb_p, kc,
                           assign);
    else if (words && ds <= 64)
        hipLaunchKernelGGL((k_kmeans_assign<FLOAT, 64>), grid, dim3(KM_THREADS), lds, s, X, n, d, ds, p, K, cb_p, kc,
                           assign);
    else if (words && ds <= 128)
        hipLaunchKernelGGL((k_kmeans_assign<FLOAT, 128>), grid, dim3(KM_THREADS), lds, s, X, n, d, ds, p, K, cb_p, kc,
                           assign);
    else
        hipLaunchKernelGGL((k_kmeans_assign<FLOAT, 0>), grid, dim3(KM_THREADS), lds, s, X, n, d, ds, p, K, cb_p, kc,
                           assign);
}

template <bool FLOAT>
__global__ void __launch_bounds__(KM_THREADS) k_kmeans_accum(const uint8_t* X, int64_t n, int d, int ds, int p, int K,
                                                             const int32_t* assign, float fx_scale, uint64_t* sums_p,
                                                             uint32_t* counts_p) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int e0 = blockIdx.y * KM_SLICE;
    const int sw = min(KM_SLICE, ds - e0);                 // dimensions in this slice
    lsum_t<FLOAT>* lsum = reinterpret_cast<lsum_t<FLOAT>*>(lds);  // K x sw
    uint32_t* lcnt = reinterpret_cast<uint32_t*>(lds + ((K * sw * int(sizeof(lsum_t<FLOAT>)) + 15) & ~15));
    for (int w = threadIdx.x; w < K * sw; w += KM_THREADS) lsum[w] = 0;
    for (int w = threadIdx.x; w < K; w += KM_THREADS) lcnt[w] = 0;
    __syncthreads();
    const int per = KM_THREADS / sw;  // points per pass (sw divides neither? then some lanes idle)
    const int e = threadIdx.x % sw, r = threadIdx.x / sw;
    const int64_t p0 = int64_t(blockIdx.x) * KM_POINTS;
    const int64_t p1 = min<int64_t>(n, p0 + KM_POINTS);
    if (r < per) {
        for (int64_t i = p0 + r; i < p1; i += per) {
            const int a = assign[i];
            lsum_t<FLOAT> v;
            if constexpr (!FLOAT)
                v = X[i * d + int64_t(p) * ds + e0 + e];
            else
                v = static_cast<unsigned long long>(
                    __float2ll_rn(reinterpret_cast<const float*>(X)[i * d + int64_t(p) * ds + e0 + e] * fx_scale));
            atomicAdd(&lsum[a * sw + e], v);
            if (blockIdx.y == 0 && e == 0) atomicAdd(&lcnt[a], 1u);
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < K * sw; w += KM_THREADS)
        if (lsum[w])
            atomicAdd(reinterpret_cast<unsigned long long*>(&sums_p[(w / sw) * ds + e0 + w % sw]),
                      static_cast<unsigned long long>(lsum[w]));
    if (blockIdx.y == 0)
        for (int w = threadIdx.x; w < K; w += KM_THREADS)
            if (lcnt[w]) atomicAdd(&counts_p[w], lcnt[w]);
}

// update: member mean, u8 rounded half up in exact integers; empty keeps
template <bool FLOAT>
__global__ void k_kmeans_update(void* cb, const uint64_t* sums, const uint32_t* counts, int P, int K, int ds,
                                float inv_fx_scale) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * K * ds) return;
    const uint32_t cnt = counts[e / ds];
    if (cnt == 0) return;
    if constexpr (!FLOAT) {
        const uint64_t s = sums[e];
        static_cast<uint8_t*>(cb)[e] = uint8_t((2 * s + cnt) / (2 * uint64_t(cnt)));
    } else {
        const int64_t s = int64_t(sums[e]);
        static_cast<float*>(cb)[e] = float(s) * inv_fx_scale / float(cnt);
    }
}

// ----------------------------------------------------------------------
// Bridge graph, step 1: for every reference vector its top-t bridges by
// (distance, lid), from the reference's own subspace tables and the
// multi-sequence heap.  One wavefront per reference vector.
// Output key = (distance bits << 32 | reference id), lid alongside.
// ----------------------------------------------------------------------
__host__ __device__ inline int topt_layout(int rowb, int PK, int heap_cap, int& o_tab, int& o_sv, int& o_heap,
                                           int& o_perm) {
    o_tab = (rowb + 15) & ~15;
    o_sv = o_tab + PK * 4;
    o_heap = (o_sv + PK * 4 + 15) & ~15;
    o_perm = o_heap + heap_cap * int(sizeof(hent_t));
    return (o_perm + PK + 15) & ~15;
}

template <bool FLOAT>
__global__ void __launch_bounds__(WAVE) k_bridge_topt(const uint8_t* X, int64_t n, int d, int P, int K,
                                                       const void* cb, int t, int heap_cap, uint32_t* out_lid,
                                                       uint64_t* out_key, uint32_t* counts) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int ds = d / P;
    const int PK = P * K;
    const int rowb = FLOAT ? d * 4 : d;
    int o_tab, o_sv, o_heap, o_perm;
    topt_layout(rowb, PK, heap_cap, o_tab, o_sv, o_heap, o_perm);
    uint8_t* qv = lds;
    uint32_t* tab = reinterpret_cast<uint32_t*>(lds + o_tab);
    uint32_t* sv = reinterpret_cast<uint32_t*>(lds + o_sv);
    hent_t* heap = reinterpret_cast<hent_t*>(lds + o_heap);
    uint8_t* perm = lds + o_perm;
    const int lane = lane_id();
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        for (int w = lane; w < rowb / 4; w += WAVE)
            reinterpret_cast<uint32_t*>(qv)[w] = reinterpret_cast<const uint32_t*>(X + i * rowb)[w];
        __syncthreads();
        compute_tables<FLOAT>(qv, cb, P, K, ds, tab, sv, perm, lane);
        if (lane == 0) {
            // keys carry n + lid like the search; strip n when writing
            int hn = 0;
            heap_push(heap, hn, tuple_key<FLOAT>(0u, sv, perm, P, K, 0), 0u);
            for (int j = 0; j < t; ++j) {
                uint64_t key;
                uint32_t rk;
                heap_pop(heap, hn, key, rk);
                out_lid[i * t + j] = key_id(key);
                out_key[i * t + j] = make_key(key_dist(key), uint32_t(i));
                atomicAdd(&counts[key_id(key)], 1u);
                int last = 0;
                for (int p = 0; p < P; ++p)
                    if ((rk >> (8 * p)) & 0xFF) last = p;
                for (int b = last; b < P; ++b) {
                    const int r = (rk >> (8 * b)) & 0xFF;
                    if (r + 1 >= K) continue;
                    const uint32_t crk = rk + (1u << (8 * b));
                    heap_push(heap, hn, tuple_key<FLOAT>(crk, sv, perm, P, K, 0), crk);
                }
            }
        }
        __syncthreads();
    }
}

// step 2: scatter each (bridge, key) into its bridge's bucket
__global__ void k_bridge_scatter(const uint32_t* lid, const uint64_t* key, int64_t m, const uint32_t* start,
                                 uint32_t* cursor, uint64_t* bucket) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t b = lid[i];
    const uint32_t pos = start[b] + atomicAdd(&cursor[b], 1u);
    bucket[pos] = key[i];
}

// step 3: order each bucket by (distance, id); keep the first b (0 = all)
__global__ void k_bridge_sort(uint64_t* bucket, const uint32_t* start, const uint32_t* count, int64_t nb, int b,
                              uint32_t* kept) {
    const int64_t lid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lid >= nb) return;
    uint64_t* v = bucket + start[lid];
    const int m = int(count[lid]);
    const int keep = (b > 0 && b < m) ? b : m;
    // selection of the `keep` smallest, in order (in place)
    for (int i = 0; i < keep; ++i) {
        int best = i;
        uint64_t bv = v[i];
        for (int j = i + 1; j < m; ++j) {
            const uint64_t x = v[j];
            if (x < bv) {
                bv = x;
                best = j;
            }
        }
        v[best] = v[i];
        v[i] = bv;
    }
    kept[lid] = uint32_t(keep);
}

// step 4: CSR ids
__global__ void k_bridge_emit(const uint64_t* bucket, const uint32_t* start, const uint32_t* off, int64_t nb,
                              uint32_t* ids) {
    const int64_t lid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lid >= nb) return;
    const uint32_t o = off[lid], e = off[lid + 1], s = start[lid];
    for (uint32_t i = 0; i < e - o; ++i) ids[o + i] = key_id(bucket[s + i]);
}

// ----------------------------------------------------------------------
// exclusive scan of uint32 counts (n + 1 outputs, last = total)
// ----------------------------------------------------------------------
constexpr int SCAN_BLOCK = 1024;

__global__ void k_scan_block(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* block_sums) {
    __shared__ uint32_t s[SCAN_BLOCK];
    const int64_t i = int64_t(blockIdx.x) * SCAN_BLOCK + threadIdx.x;
    const uint32_t v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
        const uint32_t add = threadIdx.x >= unsigned(o) ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;  // exclusive
    if (threadIdx.x == SCAN_BLOCK - 1) block_sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_sums(uint32_t* block_sums, int64_t nblocks, uint32_t* total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t run = 0;
    for (int64_t b = 0; b < nblocks; ++b) {
        const uint32_t v = block_sums[b];
        block_sums[b] = run;
        run += v;
    }
    *total = run;
}

__global__ void k_scan_add(uint32_t* out, int64_t n, const uint32_t* block_sums) {
    const int64_t i = int64_t(blockIdx.x) * SCAN_BLOCK + threadIdx.x;
    if (i < n) out[i] += block_sums[blockIdx.x];
}

int exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out /* n + 1 */, hipStream_t s) {
    const int64_t nbk = ceil_div(n, SCAN_BLOCK);
    uint32_t* bs = nullptr;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&bs), size_t(nbk) * 4, s));
    hipLaunchKernelGGL(k_scan_block, dim3(unsigned(nbk)), dim3(SCAN_BLOCK), 0, s, in, n, out, bs);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, s, bs, nbk, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nbk)), dim3(SCAN_BLOCK), 0, s, out, n, bs);
    ANN_HIP_CHECK(hipGetLastError());
    ANN_HIP_CHECK(hipFreeAsync(bs, s));
    return ANN_OK;
}

__global__ void k_to_bf16(const float* x, int64_t m, uint16_t* y) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) y[i] = f32_to_bf16_rne(x[i]);
}

}  // namespace

// ----------------------------------------------------------------------
// host orchestration
// ----------------------------------------------------------------------
int build_codebooks(ann_index* idx, int iters, int fx_log2, hipStream_t s) {
    // the initial codewords are already in idx->codebooks
    const bool f = idx->dtype == ANN_F32;
    const int P = idx->P, K = idx->K, ds = idx->d / idx->P;
    const int PKd = P * K * ds;
    uint64_t* sums = nullptr;
    uint32_t* counts = nullptr;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&sums), size_t(PKd) * 8, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&counts), size_t(P * K) * 4, s));
    // f32 sums in fixed point x * 2^fx_log2 (the caller bounds n * max|x| * 2^fx_log2 by 2^62)
    const float fx = f ? ldexpf(1.f, fx_log2) : 1.f;
    const float inv_fx = f ? ldexpf(1.f, -fx_log2) : 1.f;
    const int esz = f ? 4 : 1;
    const int kc = std::max(1, std::min(K, KM_CHUNK_BYTES / (ds * esz)));
    const int lds_assign = ((kc * ds * esz + 15) & ~15) + kc * 4;
    const int slices = int(ceil_div(ds, KM_SLICE));
    const int sw0 = std::min(KM_SLICE, ds);
    const int lds_accum = ((K * sw0 * (f ? 8 : 4) + 15) & ~15) + K * 4;
    int dev = 0, max_lds = 0;
    ANN_HIP_CHECK(hipGetDevice(&dev));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds_accum > max_lds || lds_assign > max_lds)
        return set_error(ANN_EUNSUPPORTED, "codebooks too large for the k-means kernels");
    int32_t* assign = nullptr;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&assign), size_t(idx->n) * 4, s));
    const dim3 agrid(unsigned(ceil_div(idx->n, KM_POINTS)), unsigned(slices));
    for (int it = 0; it < iters; ++it) {
        ANN_HIP_CHECK(hipMemsetAsync(sums, 0, size_t(PKd) * 8, s));
        ANN_HIP_CHECK(hipMemsetAsync(counts, 0, size_t(P * K) * 4, s));
        for (int p = 0; p < P; ++p) {
            const uint8_t* cb_p = static_cast<const uint8_t*>(idx->codebooks) + int64_t(p) * K * ds * esz;
            uint64_t* sums_p = sums + int64_t(p) * K * ds;
            uint32_t* counts_p = counts + p * K;
            if (f) {
                launch_kmeans_assign<true>(idx->X, idx->n, idx->d, ds, p, K, cb_p, kc, lds_assign, assign, s);
                hipLaunchKernelGGL(k_kmeans_accum<true>, agrid, dim3(KM_THREADS), lds_accum, s, idx->X, idx->n,
                                   idx->d, ds, p, K, assign, fx, sums_p, counts_p);
            } else {
                launch_kmeans_assign<false>(idx->X, idx->n, idx->d, ds, p, K, cb_p, kc, lds_assign, assign, s);
                hipLaunchKernelGGL(k_kmeans_accum<false>, agrid, dim3(KM_THREADS), lds_accum, s, idx->X, idx->n,
                                   idx->d, ds, p, K, assign, fx, sums_p, counts_p);
            }
            ANN_HIP_CHECK(hipGetLastError());
        }
        const int ub = (PKd + 255) / 256;
        if (f)
            hipLaunchKernelGGL(k_kmeans_update<true>, dim3(ub), dim3(256), 0, s, idx->codebooks, sums, counts, P, K,
                               ds, inv_fx);
        else
            hipLaunchKernelGGL(k_kmeans_update<false>, dim3(ub), dim3(256), 0, s, idx->codebooks, sums, counts, P,
                               K, ds, inv_fx);
        ANN_HIP_CHECK(hipGetLastError());
    }
    ANN_HIP_CHECK(hipFreeAsync(sums, s));
    ANN_HIP_CHECK(hipFreeAsync(counts, s));
    ANN_HIP_CHECK(hipFreeAsync(assign, s));
    return ANN_OK;
}

int kmeans_assign_subspace(const uint8_t* X, int64_t n, int d, bool f32, int ds, int p, int K, const void* cb_p,
                           int32_t* assign, hipStream_t s) {
    const int esz = f32 ? 4 : 1;
    const int kc = std::max(1, std::min(K, KM_CHUNK_BYTES / (ds * esz)));
    const int lds_assign = ((kc * ds * esz + 15) & ~15) + kc * 4;
    if (f32)
        launch_kmeans_assign<true>(X, n, d, ds, p, K, cb_p, kc, lds_assign, assign, s);
    else
        launch_kmeans_assign<false>(X, n, d, ds, p, K, cb_p, kc, lds_assign, assign, s);
    ANN_HIP_CHECK(hipGetLastError());
    return ANN_OK;
}

int build_bridge_graph(ann_index* idx, int t, int b, hipStream_t s) {
    const bool f = idx->dtype == ANN_F32;
    const int64_t n = idx->n, nb = idx->nb;
    if (t > nb) t = int(nb);
    const int64_t m = n * t;
    if (m >= (int64_t(1) << 32)) return set_error(ANN_EUNSUPPORTED, "n * bridge_t must stay below 2^32");
    uint32_t *lid = nullptr, *counts = nullptr, *start = nullptr, *cursor = nullptr, *kept = nullptr;
    uint64_t *key = nullptr, *bucket = nullptr;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&lid), size_t(m) * 4, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&key), size_t(m) * 8, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&counts), size_t(nb) * 4, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&start), size_t(nb + 1) * 4, s));
    ANN_HIP_CHECK(hipMemsetAsync(counts, 0, size_t(nb) * 4, s));

    const int heap_cap = 1 + (idx->P - 1) * t + idx->P;
    const int rowb = f ? idx->d * 4 : idx->d;
    const int PK = idx->P * idx->K;
    int o1, o2, o3, o4;
    const int lds = topt_layout(rowb, PK, heap_cap, o1, o2, o3, o4);
    int dev = 0, max_lds = 0;
    ANN_HIP_CHECK(hipGetDevice(&dev));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds > max_lds) return set_error(ANN_EUNSUPPORTED, "bridge_t too large for the bridge-graph kernel");
    const int64_t grid = std::min<int64_t>(n, 1 << 20);
    if (f)
        hipLaunchKernelGGL(k_bridge_topt<true>, dim3(unsigned(grid)), dim3(WAVE), lds, s, idx->X, n, idx->d, idx->P,
                           idx->K, idx->codebooks, t, heap_cap, lid, key, counts);
    else
        hipLaunchKernelGGL(k_bridge_topt<false>, dim3(unsigned(grid)), dim3(WAVE), lds, s, idx->X, n, idx->d,
                           idx->P, idx->K, idx->codebooks, t, heap_cap, lid, key, counts);
    ANN_HIP_CHECK(hipGetLastError());
    int rc = exclusive_scan(counts, nb, start, s);
    if (rc) return rc;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&cursor), size_t(nb) * 4, s));
    ANN_HIP_CHECK(hipMemsetAsync(cursor, 0, size_t(nb) * 4, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&bucket), size_t(m) * 8, s));
    hipLaunchKernelGGL(k_bridge_scatter, dim3(unsigned(ceil_div(m, 256))), dim3(256), 0, s, lid, key, m, start,
                       cursor, bucket);
    ANN_HIP_CHECK(hipGetLastError());
    ANN_HIP_CHECK(hipFreeAsync(lid, s));
    ANN_HIP_CHECK(hipFreeAsync(key, s));
    ANN_HIP_CHECK(hipFreeAsync(cursor, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&kept), size_t(nb) * 4, s));
    hipLaunchKernelGGL(k_bridge_sort, dim3(unsigned(ceil_div(nb, 256))), dim3(256), 0, s, bucket, start, counts, nb,
                       b, kept);
    ANN_HIP_CHECK(hipGetLastError());
    int rc2 = dalloc(idx, reinterpret_cast<void**>(&idx->boff), size_t(nb + 1) * 4);
    if (rc2) return rc2;
    rc = exclusive_scan(kept, nb, idx->boff, s);
    if (rc) return rc;
    uint32_t E = 0;
    ANN_HIP_CHECK(hipMemcpyAsync(&E, idx->boff + nb, 4, hipMemcpyDeviceToHost, s));
    ANN_HIP_CHECK(hipStreamSynchronize(s));
    idx->E = E;
    rc2 = dalloc(idx, reinterpret_cast<void**>(&idx->bids), size_t(std::max<int64_t>(E, 1)) * 4);
    if (rc2) return rc2;
    hipLaunchKernelGGL(k_bridge_emit, dim3(unsigned(ceil_div(nb, 256))), dim3(256), 0, s, bucket, start, idx->boff,
                       nb, idx->bids);
    ANN_HIP_CHECK(hipGetLastError());
    ANN_HIP_CHECK(hipFreeAsync(bucket, s));
    ANN_HIP_CHECK(hipFreeAsync(counts, s));
    ANN_HIP_CHECK(hipFreeAsync(start, s));
    ANN_HIP_CHECK(hipFreeAsync(kept, s));
    ANN_HIP_CHECK(hipStreamSynchronize(s));
    return ANN_OK;
}

int make_bf16_copy(ann_index* idx, hipStream_t s) {
    if (idx->dtype != ANN_F32 || idx->Xbf16) return ANN_OK;
    const int64_t m = idx->n * idx->d;
    int rc = dalloc(idx, reinterpret_cast<void**>(&idx->Xbf16), size_t(m) * 2);
    if (rc) return rc;
    hipLaunchKernelGGL(k_to_bf16, dim3(unsigned(ceil_div(m, 256))), dim3(256), 0, s,
                       reinterpret_cast<const float*>(idx->X), m, idx->Xbf16);
    ANN_HIP_CHECK(hipGetLastError());
    return ANN_OK;
}

}  // namespace ann
