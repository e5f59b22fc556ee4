// Exact k nearest neighbours by linear scan: the ground truth of Sec. 5.1
// and the exact kNN graph of Sec. 4.1 (each vector's R nearest others).
//
// One thread owns one query row and keeps its best k (distance, id) keys in
// registers, sorted.  Candidate rows stream through LDS in tiles shared by
// the 256 queries of a workgroup; every lane reads the same candidate chunk
// at the same time (an LDS broadcast).
//   u8:  |q - x|^2 = |q|^2 + |x|^2 - 2 q.x with packed 4 x u8 dot products,
//        exact in int32 (d <= 512 keeps every term below 2^31).
//   f32: sum of (q - x)^2 in fp32, fixed order.
#include "internal.hpp"

namespace ann {
namespace {

constexpr int KNN_THREADS = 256;

template <int KMAX>
__device__ inline void topk_offer(uint64_t (&top)[KMAX], uint64_t c) {
    if (c >= top[KMAX - 1]) return;
    top[KMAX - 1] = c;
#pragma unroll
    for (int i = KMAX - 1; i > 0; --i) {
        const uint64_t a = top[i - 1], b = top[i];
        const bool sw = b < a;
        top[i - 1] = sw ? b : a;
        top[i] = sw ? a : b;
    }
}

// blockIdx.y selects a contiguous slice of the candidates; with more than one
// slice the kernel writes each slice's sorted best-k keys to `partial`
// (nq x slices x k) and k_knn_merge combines them.
template <bool FLOAT, int KMAX, int TJ>
__global__ void __launch_bounds__(KNN_THREADS) k_knn(const uint8_t* X, int64_t n, int64_t row_bytes,
                                                      const uint8_t* Q, int64_t nq, int k, int exclude_self,
                                                      int32_t* out_ids, uint32_t* out_d, uint64_t* partial) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t* tile = lds;                                                    // TJ x row_bytes
    uint32_t* xnorm = reinterpret_cast<uint32_t*>(lds + TJ * row_bytes);   // TJ (u8 only)
    const int nc16 = int(row_bytes / 16);
    const int64_t qi = int64_t(blockIdx.x) * KNN_THREADS + threadIdx.x;
    const bool active = qi < nq;
    const uint4* qrow = reinterpret_cast<const uint4*>(Q + (active ? qi : 0) * row_bytes);

    uint32_t qnorm = 0;
    if constexpr (!FLOAT) {
        for (int c = 0; c < nc16; ++c) {
            const uint4 q = qrow[c];
            qnorm = __builtin_amdgcn_udot4(q.x, q.x, qnorm, false);
            qnorm = __builtin_amdgcn_udot4(q.y, q.y, qnorm, false);
            qnorm = __builtin_amdgcn_udot4(q.z, q.z, qnorm, false);
            qnorm = __builtin_amdgcn_udot4(q.w, q.w, qnorm, false);
        }
    }
    uint64_t top[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) top[i] = KEY_EMPTY;

    const int64_t per = (n + gridDim.y - 1) / gridDim.y;
    const int64_t jbeg = int64_t(blockIdx.y) * per;
    const int64_t jend = min<int64_t>(n, jbeg + per);
    for (int64_t j0 = jbeg; j0 < jend; j0 += TJ) {
        const int tj = int(min<int64_t>(TJ, jend - j0));
        __syncthreads();
        {
            const uint4* src = reinterpret_cast<const uint4*>(X + j0 * row_bytes);
            uint4* dst = reinterpret_cast<uint4*>(tile);
            for (int i = threadIdx.x; i < tj * nc16; i += KNN_THREADS) dst[i] = src[i];
        }
        __syncthreads();
        if constexpr (!FLOAT) {
            for (int r = threadIdx.x; r < tj; r += KNN_THREADS) {
                const uint4* row = reinterpret_cast<const uint4*>(tile + r * row_bytes);
                uint32_t s = 0;
                for (int c = 0; c < nc16; ++c) {
                    const uint4 x = row[c];
                    s = __builtin_amdgcn_udot4(x.x, x.x, s, false);
                    s = __builtin_amdgcn_udot4(x.y, x.y, s, false);
                    s = __builtin_amdgcn_udot4(x.z, x.z, s, false);
                    s = __builtin_amdgcn_udot4(x.w, x.w, s, false);
                }
                xnorm[r] = s;
            }
            __syncthreads();
        }
        // chunk-major accumulation: one query chunk in registers, TJ partial sums
        uint32_t acc[TJ];
        float facc[TJ];
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            acc[j] = 0;
            facc[j] = 0.f;
        }
        for (int c = 0; c < nc16; ++c) {
            const uint4 q = qrow[c];
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const uint4 x = *reinterpret_cast<const uint4*>(tile + j * row_bytes + c * 16);
                if constexpr (!FLOAT) {
                    uint32_t a = acc[j];
                    a = __builtin_amdgcn_udot4(q.x, x.x, a, false);
                    a = __builtin_amdgcn_udot4(q.y, x.y, a, false);
                    a = __builtin_amdgcn_udot4(q.z, x.z, a, false);
                    a = __builtin_amdgcn_udot4(q.w, x.w, a, false);
                    acc[j] = a;
                } else {
                    float f = facc[j];
                    float t;
                    t = __uint_as_float(q.x) - __uint_as_float(x.x); f = fmaf(t, t, f);
                    t = __uint_as_float(q.y) - __uint_as_float(x.y); f = fmaf(t, t, f);
                    t = __uint_as_float(q.z) - __uint_as_float(x.z); f = fmaf(t, t, f);
                    t = __uint_as_float(q.w) - __uint_as_float(x.w); f = fmaf(t, t, f);
                    facc[j] = f;
                }
            }
        }
        if (active) {
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                if (j < tj) {
                    const int64_t id = j0 + j;
                    if (!(exclude_self && id == qi)) {
                        const uint32_t dist = FLOAT ? __float_as_uint(facc[j]) : qnorm + xnorm[j] - 2u * acc[j];
                        topk_offer<KMAX>(top, make_key(dist, uint32_t(id)));
                    }
                }
            }
        }
    }
    if (active && partial) {
        uint64_t* dst = partial + (qi * gridDim.y + blockIdx.y) * k;
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) dst[i] = top[i];
    } else if (active) {
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                const uint64_t v = top[i];
                const bool ok = v != KEY_EMPTY;
                out_ids[qi * k + i] = ok ? int32_t(key_id(v)) : -1;
                out_d[qi * k + i] = ok ? key_dist(v) : (FLOAT ? 0x7F800000u : 0x7FFFFFFFu);
            }
        }
    }
}

template <bool FLOAT, int KMAX>
__global__ void __launch_bounds__(KNN_THREADS) k_knn_merge(const uint64_t* partial, int64_t nq, int slices, int k,
                                                            int32_t* out_ids, uint32_t* out_d) {
    const int64_t qi = int64_t(blockIdx.x) * KNN_THREADS + threadIdx.x;
    if (qi >= nq) return;
    uint64_t top[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) top[i] = KEY_EMPTY;
    const uint64_t* src = partial + qi * int64_t(slices) * k;
    for (int i = 0; i < slices * k; ++i) topk_offer<KMAX>(top, src[i]);
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (i < k) {
            const uint64_t v = top[i];
            const bool ok = v != KEY_EMPTY;
            out_ids[qi * k + i] = ok ? int32_t(key_id(v)) : -1;
            out_d[qi * k + i] = ok ? key_dist(v) : (FLOAT ? 0x7F800000u : 0x7FFFFFFFu);
        }
    }
}

// ----------------------------------------------------------------------
// u8 on matrix cores.  With u = x - 128 as int8 (x xor 0x80),
//   |x - y|^2 = |u|^2 + |v|^2 - 2 u.v, exact in int32,
// and u.v comes from v_mfma_i32_16x16x64_i8.  A workgroup of four wavefronts
// owns 256 query rows, 64 per wavefront, whose operands stay in registers
// for the whole scan; 64-candidate tiles stream through LDS (rows padded by
// 16 bytes so that the 16 lanes reading one k-slice of 16 rows hit distinct
// banks).  Lane l holds row l % 16 of a 16 x 64 operand block (bytes
// 16 (l / 16) .. +15) and result rows 4 (l / 16) .. +3 of column l % 16.
// The epilogue is two VALU operations per value: |v|^2 - 2 u.v against the
// row's threshold (k-th best distance minus |u|^2).  The rare survivors go
// through per-row LDS buckets to the lane that owns the row, which keeps its
// best k keys sorted in registers.
// ----------------------------------------------------------------------
typedef int v4i32 __attribute__((ext_vector_type(4)));

constexpr int MQ_ROWS = 256;  // query rows per workgroup
constexpr int MC_TILE = 64;   // candidates per LDS tile

// |x - 128|^2 per row: sum x^2 - 256 sum x + 128^2 d
__global__ void k_shifted_norms(const uint8_t* X, int64_t n, int d, uint32_t* out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4* r = reinterpret_cast<const uint4*>(X + i * d);
    uint32_t sq = 0, sm = 0;
    for (int c = 0; c < d / 16; ++c) {
        const uint4 x = r[c];
        sq = __builtin_amdgcn_udot4(x.x, x.x, sq, false);
        sq = __builtin_amdgcn_udot4(x.y, x.y, sq, false);
        sq = __builtin_amdgcn_udot4(x.z, x.z, sq, false);
        sq = __builtin_amdgcn_udot4(x.w, x.w, sq, false);
        sm = __builtin_amdgcn_udot4(x.x, 0x01010101u, sm, false);
        sm = __builtin_amdgcn_udot4(x.y, 0x01010101u, sm, false);
        sm = __builtin_amdgcn_udot4(x.z, 0x01010101u, sm, false);
        sm = __builtin_amdgcn_udot4(x.w, 0x01010101u, sm, false);
    }
    out[i] = sq - 256u * sm + 16384u * uint32_t(d);
}

template <int KS, int KMAX>
__global__ void __launch_bounds__(256) k_knn_mfma(const uint8_t* X, const uint32_t* xn, int64_t n, const uint8_t* Q,
                                                  const uint32_t* qn_g, int64_t nq, int k, int excl,
                                                  int32_t* out_ids, uint32_t* out_d, uint64_t* partial) {
    constexpr int D = KS * 64;
    constexpr int STRIDE = D + 16;
    constexpr int C16 = D / 16;                       // 16-byte chunks per row
    constexpr int PER = MC_TILE * C16 / 256;          // chunks per thread per tile
    __shared__ __align__(16) uint8_t tile[2][MC_TILE * STRIDE];  // double buffer
    __shared__ int cn_l[2][MC_TILE];
    __shared__ uint64_t bucket[4][64][16];
    __shared__ int bcnt[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * MQ_ROWS + w * 64;

    v4i32 a[4][KS];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t r = min<int64_t>(row0 + rb * 16 + col, nq - 1);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const uint4 v = *reinterpret_cast<const uint4*>(Q + r * D + s * 64 + kq * 16);
            a[rb][s] = v4i32{int(v.x ^ 0x80808080u), int(v.y ^ 0x80808080u), int(v.z ^ 0x80808080u),
                             int(v.w ^ 0x80808080u)};
        }
    }
    // this lane's result rows: rb * 16 + 4 kq + t of the wavefront's 64.  A
    // candidate passes when 2 u.v - |v|^2 >= nt = |u|^2 - (k-th best distance)
    auto qnorm = [&](int wr) { return row0 + wr < nq ? int(qn_g[row0 + wr]) : 0; };
    int nt[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int t = 0; t < 4; ++t) nt[rb][t] = qnorm(rb * 16 + 4 * kq + t) - 0x7FFFFFFF;
    const int qn_own = qnorm(lane);  // |u|^2 of the row this lane keeps
    uint64_t top[KMAX];  // row row0 + lane, ascending
#pragma unroll
    for (int i = 0; i < KMAX; ++i) top[i] = KEY_EMPTY;
    bcnt[w][lane] = 0;

    const int64_t per = (n + gridDim.y - 1) / gridDim.y;
    const int64_t jbeg = int64_t(blockIdx.y) * per;
    const int64_t jend = min<int64_t>(n, jbeg + per);
    // the next tile is loaded into registers while the current one is used
    uint4 pre[PER];
    int pcn = 0;
    auto fetch = [&](int64_t j0) {
        const int tj = int(min<int64_t>(MC_TILE, jend - j0));
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * 256;
            const int rr = i / C16, c = i - rr * C16;
            pre[u] = rr < tj ? *reinterpret_cast<const uint4*>(X + (j0 + rr) * D + c * 16) : make_uint4(0, 0, 0, 0);
        }
        if (threadIdx.x < MC_TILE) pcn = int(threadIdx.x) < tj ? int(xn[j0 + threadIdx.x]) : 0x3FFFFFFF;
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * 256;
            const int rr = i / C16, c = i - rr * C16;
            uint4 v = pre[u];
            v.x ^= 0x80808080u;
            v.y ^= 0x80808080u;
            v.z ^= 0x80808080u;
            v.w ^= 0x80808080u;
            *reinterpret_cast<uint4*>(tile[buf] + rr * STRIDE + c * 16) = v;
        }
        if (threadIdx.x < MC_TILE) cn_l[buf][threadIdx.x] = pcn;
    };
    if (jbeg < jend) {
        fetch(jbeg);
        stash(0);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t j0 = jbeg; j0 < jend; j0 += MC_TILE, cur ^= 1) {
        const int tj = int(min<int64_t>(MC_TILE, jend - j0));
        const bool more = j0 + MC_TILE < jend;
        if (more) fetch(j0 + MC_TILE);
        const uint8_t* tl = tile[cur];
        const bool self_tile = excl && j0 < row0 + 64 && j0 + MC_TILE > row0;
#pragma unroll
        for (int cb = 0; cb < MC_TILE / 16; ++cb) {
            v4i32 acc[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = v4i32{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const v4i32 b = *reinterpret_cast<const v4i32*>(tl + (cb * 16 + col) * STRIDE + s * 64 + kq * 16);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rb][s], b, acc[rb], 0, 0, 0);
            }
            const int jj = cb * 16 + col;
            const int64_t j = j0 + jj;
            int ncn = -cn_l[cur][jj];  // past the tile's end: too small to pass
            // opaque to the compiler, so that 2 u.v - |v|^2 is one shift-add
            // per value rather than a shift and a subtraction of |v|^2
            asm volatile("" : "+v"(ncn));
            bool any = false;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int t = 0; t < 4; ++t) any |= (acc[rb][t] << 1) + ncn >= nt[rb][t];
            if (__ballot(any) == 0) continue;
            // ---- slow path: survivors to their rows' buckets, owners merge
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int wv = (acc[rb][t] << 1) + ncn;
                    const int wr = rb * 16 + 4 * kq + t;
                    const bool me = self_tile && j == row0 + wr;
                    if (wv >= nt[rb][t] && jj < tj && !me) {
                        const int slot = atomicAdd(&bcnt[w][wr], 1);
                        bucket[w][wr][slot] = make_key(uint32_t(wv), uint32_t(j));  // the owner adds |u|^2
                    }
                }
            lds_wave_order();
            const int c = bcnt[w][lane];
            for (int e = 0; e < c; ++e) {
                const uint64_t b = bucket[w][lane][e];
                topk_offer<KMAX>(top, make_key(uint32_t(qn_own - int(key_dist(b))), key_id(b)));
            }
            bcnt[w][lane] = 0;
            uint64_t th = top[0];
#pragma unroll
            for (int i = 1; i < KMAX; ++i)
                if (i == k - 1) th = top[i];
            const int nthr = qn_own - (th == KEY_EMPTY ? 0x7FFFFFFF : int(key_dist(th)));
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int t = 0; t < 4; ++t) nt[rb][t] = __shfl(nthr, rb * 16 + 4 * kq + t);
            lds_wave_order();
        }
        if (more) stash(cur ^ 1);
        __syncthreads();
    }
    const int64_t qi = row0 + lane;
    if (qi >= nq) return;
    if (partial) {
        uint64_t* dst = partial + (qi * gridDim.y + blockIdx.y) * k;
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) dst[i] = top[i];
    } else {
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                const uint64_t v = top[i];
                const bool ok = v != KEY_EMPTY;
                out_ids[qi * k + i] = ok ? int32_t(key_id(v)) : -1;
                out_d[qi * k + i] = ok ? key_dist(v) : 0x7FFFFFFFu;
            }
        }
    }
}

template <int KS, int KMAX>
int launch_knn_mfma(const void* d_x, int64_t n, const void* d_q, int64_t nq, int k, int excl, int32_t* d_ids,
                    void* d_dists, hipStream_t s) {
    const int64_t grid = ceil_div(nq, MQ_ROWS);
    int slices = 1;
    while (grid * slices < 1024 && slices < 256 && n / (slices * 2) >= MC_TILE * 16) slices *= 2;
    uint32_t* norms = nullptr;
    const bool same = d_q == d_x;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&norms), size_t(n + (same ? 0 : nq)) * 4, s));
    uint32_t* qn = same ? norms : norms + n;
    hipLaunchKernelGGL(k_shifted_norms, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s,
                       static_cast<const uint8_t*>(d_x), n, KS * 64, norms);
    if (!same)
        hipLaunchKernelGGL(k_shifted_norms, dim3(unsigned(ceil_div(nq, 256))), dim3(256), 0, s,
                           static_cast<const uint8_t*>(d_q), nq, KS * 64, qn);
    uint64_t* partial = nullptr;
    if (slices > 1)
        ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial), size_t(nq) * slices * k * sizeof(uint64_t), s));
    hipLaunchKernelGGL((k_knn_mfma<KS, KMAX>), dim3(unsigned(grid), unsigned(slices)), dim3(256), 0, s,
                       static_cast<const uint8_t*>(d_x), norms, n, static_cast<const uint8_t*>(d_q), qn, nq, k, excl,
                       d_ids, static_cast<uint32_t*>(d_dists), partial);
    ANN_HIP_CHECK(hipGetLastError());
    if (slices > 1) {
        hipLaunchKernelGGL((k_knn_merge<false, KMAX>), dim3(unsigned(ceil_div(nq, KNN_THREADS))), dim3(KNN_THREADS),
                           0, s, partial, nq, slices, k, d_ids, static_cast<uint32_t*>(d_dists));
        ANN_HIP_CHECK(hipGetLastError());
        ANN_HIP_CHECK(hipFreeAsync(partial, s));
    }
    ANN_HIP_CHECK(hipFreeAsync(norms, s));
    return ANN_OK;
}

template <int KMAX>
int launch_knn_mfma_d(int d, const void* d_x, int64_t n, const void* d_q, int64_t nq, int k, int excl, int32_t* d_ids,
                      void* d_dists, hipStream_t s) {
    switch (d) {
        case 64: return launch_knn_mfma<1, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
        case 128: return launch_knn_mfma<2, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
        case 192: return launch_knn_mfma<3, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
        default: return launch_knn_mfma<4, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
    }
}

// ----------------------------------------------------------------------
// fp32 on matrix cores (v_mfma_f32_16x16x4f32).  Candidates are selected by
// |q|^2 + |x|^2 - 2 q.x in fp32; the k kept per row are then measured again
// as the fp32 sum of (q - x)^2 and re-sorted, so returned distances carry no
// cancellation error.  A wavefront owns 16 query rows whose operands stay in
// registers (lane l: row l % 16, dimensions 4 s + l / 16); 64-candidate
// tiles stream through LDS in stages of 128 dimensions, rows padded by four
// floats so that the 64 lanes of one step hit distinct banks.
// ----------------------------------------------------------------------
typedef float v4f32 __attribute__((ext_vector_type(4)));

constexpr int FQ_ROWS = 64;   // query rows per workgroup, 16 per wavefront

__global__ void k_sq_norms_f32(const float* X, int64_t n, int d, float* out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4* r = reinterpret_cast<const float4*>(X + i * d);
    float s = 0.f;
    for (int c = 0; c < d / 4; ++c) {
        const float4 x = r[c];
        s = fmaf(x.x, x.x, s);
        s = fmaf(x.y, x.y, s);
        s = fmaf(x.z, x.z, s);
        s = fmaf(x.w, x.w, s);
    }
    out[i] = s;
}

template <int KS4, int KMAX>
__global__ void __launch_bounds__(256) k_knn_mfma_f32(const float* X, const float* xn, int64_t n, const float* Q,
                                                      const float* qn_g, int64_t nq, int k, int excl,
                                                      int32_t* out_ids, uint32_t* out_d, uint64_t* partial) {
    constexpr int D = KS4 * 4;
    constexpr int CH = D < 128 ? D : 128;  // dimensions per LDS stage
    constexpr int NCH = D / CH;
    constexpr int STRIDE = CH + 4;
    __shared__ __align__(16) float tile[MC_TILE * STRIDE];
    __shared__ float cn_l[MC_TILE];
    __shared__ uint64_t bucket[4][16][MC_TILE];
    __shared__ int bcnt[4][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * FQ_ROWS + w * 16;

    float a[KS4];
    {
        const float* q = Q + min<int64_t>(row0 + col, nq - 1) * D + kq;
#pragma unroll
        for (int s = 0; s < KS4; ++s) a[s] = q[4 * s];
    }
    float qn[4], tq[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t r = row0 + 4 * kq + t;
        qn[t] = r < nq ? qn_g[r] : 0.f;
        tq[t] = __builtin_inff();
    }
    uint64_t top[KMAX];  // lanes 0..15: row row0 + lane, ascending
#pragma unroll
    for (int i = 0; i < KMAX; ++i) top[i] = KEY_EMPTY;
    if (lane < 16) bcnt[w][lane] = 0;

    const int64_t per = (n + gridDim.y - 1) / gridDim.y;
    const int64_t jbeg = int64_t(blockIdx.y) * per;
    const int64_t jend = min<int64_t>(n, jbeg + per);
    for (int64_t j0 = jbeg; j0 < jend; j0 += MC_TILE) {
        const int tj = int(min<int64_t>(MC_TILE, jend - j0));
        v4f32 acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            __syncthreads();
            constexpr int C4 = CH / 4;
            for (int i = threadIdx.x; i < MC_TILE * C4; i += 256) {
                const int rr = i / C4, c = i - rr * C4;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (rr < tj) v = *reinterpret_cast<const float4*>(X + (j0 + rr) * D + ch * CH + c * 4);
                *reinterpret_cast<float4*>(tile + rr * STRIDE + c * 4) = v;
            }
            if (ch == 0 && threadIdx.x < MC_TILE)
                cn_l[threadIdx.x] = int(threadIdx.x) < tj ? xn[j0 + threadIdx.x] : __builtin_inff();
            __syncthreads();
#pragma unroll
            for (int s = 0; s < C4; ++s) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const float b = tile[(cb * 16 + col) * STRIDE + 4 * s + kq];
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ch * C4 + s], b, acc[cb], 0, 0, 0);
                }
            }
        }
        bool any = false;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const float cn = cn_l[cb * 16 + col];
#pragma unroll
            for (int t = 0; t < 4; ++t) any |= fmaf(-2.f, acc[cb][t], cn) <= tq[t];
        }
        if (__ballot(any) == 0) continue;
        const bool self_tile = excl && j0 < row0 + 16 && j0 + MC_TILE > row0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int jj = cb * 16 + col;
            const int64_t j = j0 + jj;
            const float cn = cn_l[jj];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float v = fmaf(-2.f, acc[cb][t], cn);
                const int wr = 4 * kq + t;
                const bool me = self_tile && j == row0 + wr;
                if (v <= tq[t] && jj < tj && !me) {
                    const int slot = atomicAdd(&bcnt[w][wr], 1);
                    bucket[w][wr][slot] = make_key(__float_as_uint(fmaxf(v + qn[t], 0.f)), uint32_t(j));
                }
            }
        }
        lds_wave_order();
        float thr = __builtin_inff();
        if (lane < 16) {
            const int c = bcnt[w][lane];
            for (int e = 0; e < c; ++e) topk_offer<KMAX>(top, bucket[w][lane][e]);
            bcnt[w][lane] = 0;
            uint64_t th = top[0];
#pragma unroll
            for (int i = 1; i < KMAX; ++i)
                if (i == k - 1) th = top[i];
            if (th != KEY_EMPTY) thr = __uint_as_float(key_dist(th));
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) tq[t] = __shfl(thr, 4 * kq + t) - qn[t];
        lds_wave_order();
    }
    const int64_t qi = row0 + lane;
    if (lane >= 16 || qi >= nq) return;
    // the kept keys measured again as sum (q - x)^2, then sorted
    uint64_t fin[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) fin[i] = KEY_EMPTY;
    const float4* qr = reinterpret_cast<const float4*>(Q + qi * D);
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (i < k && top[i] != KEY_EMPTY) {
            const uint32_t j = key_id(top[i]);
            const float4* xr = reinterpret_cast<const float4*>(X + int64_t(j) * D);
            float e = 0.f;
            for (int c = 0; c < D / 4; ++c) {
                const float4 q = qr[c], x = xr[c];
                float t;
                t = q.x - x.x; e = fmaf(t, t, e);
                t = q.y - x.y; e = fmaf(t, t, e);
                t = q.z - x.z; e = fmaf(t, t, e);
                t = q.w - x.w; e = fmaf(t, t, e);
            }
            topk_offer<KMAX>(fin, make_key(__float_as_uint(e), j));
        }
    }
    if (partial) {
        uint64_t* dst = partial + (qi * gridDim.y + blockIdx.y) * k;
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) dst[i] = fin[i];
    } else {
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                const uint64_t v = fin[i];
                const bool ok = v != KEY_EMPTY;
                out_ids[qi * k + i] = ok ? int32_t(key_id(v)) : -1;
                out_d[qi * k + i] = ok ? key_dist(v) : 0x7F800000u;
            }
        }
    }
}

template <int KS4, int KMAX>
int launch_knn_mfma_f32(const void* d_x, int64_t n, const void* d_q, int64_t nq, int k, int excl, int32_t* d_ids,
                        void* d_dists, hipStream_t s) {
    const int64_t grid = ceil_div(nq, FQ_ROWS);
    int slices = 1;
    while (grid * slices < 1024 && slices < 256 && n / (slices * 2) >= MC_TILE * 16) slices *= 2;
    float* norms = nullptr;
    const bool same = d_q == d_x;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&norms), size_t(n + (same ? 0 : nq)) * 4, s));
    float* qn = same ? norms : norms + n;
    hipLaunchKernelGGL(k_sq_norms_f32, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s,
                       static_cast<const float*>(d_x), n, KS4 * 4, norms);
    if (!same)
        hipLaunchKernelGGL(k_sq_norms_f32, dim3(unsigned(ceil_div(nq, 256))), dim3(256), 0, s,
                           static_cast<const float*>(d_q), nq, KS4 * 4, qn);
    uint64_t* partial = nullptr;
    if (slices > 1)
        ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial), size_t(nq) * slices * k * sizeof(uint64_t), s));
    hipLaunchKernelGGL((k_knn_mfma_f32<KS4, KMAX>), dim3(unsigned(grid), unsigned(slices)), dim3(256), 0, s,
                       static_cast<const float*>(d_x), norms, n, static_cast<const float*>(d_q), qn, nq, k, excl,
                       d_ids, static_cast<uint32_t*>(d_dists), partial);
    ANN_HIP_CHECK(hipGetLastError());
    if (slices > 1) {
        hipLaunchKernelGGL((k_knn_merge<true, KMAX>), dim3(unsigned(ceil_div(nq, KNN_THREADS))), dim3(KNN_THREADS),
                           0, s, partial, nq, slices, k, d_ids, static_cast<uint32_t*>(d_dists));
        ANN_HIP_CHECK(hipGetLastError());
        ANN_HIP_CHECK(hipFreeAsync(partial, s));
    }
    ANN_HIP_CHECK(hipFreeAsync(norms, s));
    return ANN_OK;
}

template <int KMAX>
int launch_knn_mfma_f32_d(int d, const void* d_x, int64_t n, const void* d_q, int64_t nq, int k, int excl,
                          int32_t* d_ids, void* d_dists, hipStream_t s) {
    switch (d) {
        case 128: return launch_knn_mfma_f32<32, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
        case 256: return launch_knn_mfma_f32<64, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
        default: return launch_knn_mfma_f32<96, KMAX>(d_x, n, d_q, nq, k, excl, d_ids, d_dists, s);
    }
}

template <bool FLOAT, int KMAX>
int launch_knn_t(const void* d_x, int64_t n, int64_t row_bytes, const void* d_q, int64_t nq, int k, int excl,
                 int32_t* d_ids, void* d_dists, hipStream_t s) {
    constexpr int TJ = FLOAT ? 8 : 32;
    const int lds = int(TJ * row_bytes + TJ * 4);
    const int64_t grid = ceil_div(nq, KNN_THREADS);
    // enough workgroups to fill the chip: split the candidates when queries are few
    int slices = 1;
    while (grid * slices < 2048 && slices < 256 && n / (slices * 2) >= TJ * 8) slices *= 2;
    uint64_t* partial = nullptr;
    if (slices > 1) ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial),
                                                 size_t(nq) * slices * k * sizeof(uint64_t), s));
    hipLaunchKernelGGL((k_knn<FLOAT, KMAX, TJ>), dim3(unsigned(grid), unsigned(slices)), dim3(KNN_THREADS), lds, s,
                       static_cast<const uint8_t*>(d_x), n, row_bytes, static_cast<const uint8_t*>(d_q), nq, k,
                       excl, d_ids, static_cast<uint32_t*>(d_dists), partial);
    ANN_HIP_CHECK(hipGetLastError());
    if (slices > 1) {
        hipLaunchKernelGGL((k_knn_merge<FLOAT, KMAX>), dim3(unsigned(grid)), dim3(KNN_THREADS), 0, s, partial, nq,
                           slices, k, d_ids, static_cast<uint32_t*>(d_dists));
        ANN_HIP_CHECK(hipGetLastError());
        ANN_HIP_CHECK(hipFreeAsync(partial, s));
    }
    return ANN_OK;
}

}  // namespace

int launch_knn(const void* d_x, int64_t n, int d, int dtype, const void* d_q, int64_t nq, int k, int exclude_self,
               int32_t* d_ids, void* d_dists, hipStream_t s) {
    ANN_REQUIRE(k >= 1 && k <= 32, "ann_knn_device: k must be in [1, 32]");
    ANN_REQUIRE(n >= 1 && nq >= 0, "ann_knn_device: bad sizes");
    const bool f = dtype == ANN_F32;
    const int64_t row_bytes = f ? int64_t(d) * 4 : d;
    ANN_REQUIRE(row_bytes % 16 == 0, "ann_knn_device: rows must be a multiple of 16 bytes");
    ANN_REQUIRE(f || d <= 512, "ann_knn_device: u8 dimension above 512");
    if (nq == 0) return ANN_OK;
    if (f) {
        if (d == 128 || d == 256 || d == 384) {  // matrix cores
            if (k <= 16) return launch_knn_mfma_f32_d<16>(d, d_x, n, d_q, nq, k, exclude_self, d_ids, d_dists, s);
            return launch_knn_mfma_f32_d<32>(d, d_x, n, d_q, nq, k, exclude_self, d_ids, d_dists, s);
        }
        if (k <= 16) return launch_knn_t<true, 16>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
        return launch_knn_t<true, 32>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
    }
    if (d % 64 == 0 && d <= 256) {  // matrix cores
        if (k <= 16) return launch_knn_mfma_d<16>(d, d_x, n, d_q, nq, k, exclude_self, d_ids, d_dists, s);
        return launch_knn_mfma_d<32>(d, d_x, n, d_q, nq, k, exclude_self, d_ids, d_dists, s);
    }
    if (k <= 16) return launch_knn_t<false, 16>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
    return launch_knn_t<false, 32>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
}

}  // namespace ann
