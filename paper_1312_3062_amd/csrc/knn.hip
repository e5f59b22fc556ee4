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
        if (k <= 16) return launch_knn_t<true, 16>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
        return launch_knn_t<true, 32>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
    }
    if (k <= 16) return launch_knn_t<false, 16>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
    return launch_knn_t<false, 32>(d_x, n, row_bytes, d_q, nq, k, exclude_self, d_ids, d_dists, s);
}

}  // namespace ann
