// Graph-D-ADC (the paper's billion-scale system, Sec. 5): the search over the
// augmented neighborhood graph, run on a vocabulary of coarse centres, finds
// the inverted lists nearest to a vector or a query; each vector's residual
// to its list's centre is encoded by product quantisation (m bytes, 256
// codewords per subspace), and the candidates of the nearest lists are
// re-ranked by their asymmetric (ADC) distances.
//
// ADC distance of a query q and a vector x of list l with centre c and
// quantised residual r (the concatenated codewords of its code):
//     |q - c - r|^2 = |q - c|^2 + beta(x) - 2 <q, r>,
//     beta(x) = |r|^2 + 2 <c, r>           (per vector, at build)
//     <q, r>  = sum_j table[j][code_j],  table[j][w] = <q_j, codeword_jw>
// |q - c|^2 is the centre distance the list search returns; the table is one
// per query.  The candidates are scanned in list order (lists by increasing
// centre distance, a list in increasing vector id) and the scan stops after
// `candidates` of them, mid-list if need be.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

struct ann_ivf {
    ann_index* centres = nullptr;  // augmented index over the C centres (their vectors in centres->X)
    int64_t n = 0;
    int32_t d = 0, C = 0, m = 0, ds = 0;
    int device = 0;
    uint32_t* list_off = nullptr;  // C + 1
    uint32_t* list_ids = nullptr;  // n vector ids, list order
    uint8_t* codes = nullptr;      // n x m, list order
    float* beta = nullptr;         // n, list order
    float* pq = nullptr;           // m x 256 x ds codewords
    int64_t bytes = 0;
};

namespace ann {
namespace {

constexpr int PQ_K = 256;        // codewords per subspace
constexpr int ADC_THREADS = 1024;  // one workgroup per query: 16 waves, two workgroups per CU by LDS
constexpr int ADC_BUF = 2048;    // candidate keys buffered before a merge
constexpr int ADC_SORT = 4096;   // merge sort width (buffer + kept keys, padded)
constexpr int ADC_KMAX = 1024;
constexpr int ADC_WMAX = 1024;   // lists per query
constexpr int ADC_RMAX = 256;    // rounds whose first candidate's list is found once, up front

__global__ void k_ivf_residual(const uint8_t* X, int64_t n, int d, const uint8_t* centres, const int32_t* assign,
                               float* resid) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t i = e / d;
    const int j = int(e % d);
    resid[e] = float(int(X[e]) - int(centres[int64_t(assign[i]) * d + j]));
}

// initial codewords: the rows' residual subvectors, per subspace
__global__ void k_pq_init(const float* resid, int d, int m, int ds, const int64_t* rows, float* pq) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * PQ_K * ds) return;
    const int p = e / (PQ_K * ds), w = (e / ds) % PQ_K, q = e % ds;
    pq[e] = resid[rows[w] * d + p * ds + q];
}

__global__ void k_pq_pack(const int32_t* a, int64_t n, int m, int p, uint8_t* codes) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) codes[i * m + p] = uint8_t(a[i]);
}

// per vector (vector order): its code and beta in list order
__global__ void k_ivf_place(const uint8_t* codes_v, const uint8_t* centres, const int32_t* assign, const float* pq,
                            const uint32_t* list_ids, int64_t n, int d, int m, int ds, uint8_t* codes_l,
                            float* beta_l) {
    const int64_t pos = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const int64_t i = list_ids[pos];
    const uint8_t* c = centres + int64_t(assign[i]) * d;
    float rr = 0.f, cr = 0.f;
    for (int p = 0; p < m; ++p) {
        const int w = codes_v[i * m + p];
        codes_l[pos * m + p] = uint8_t(w);
        const float* cw = pq + (int64_t(p) * PQ_K + w) * ds;
        for (int q = 0; q < ds; ++q) {
            rr = fmaf(cw[q], cw[q], rr);
            cr = fmaf(float(c[p * ds + q]), cw[q], cr);
        }
    }
    beta_l[pos] = rr + 2.f * cr;
}

// key of a candidate: its non-negative float distance bits, then the vector id
// sort the first `cnt` keys of buf ascending (bitonic over ADC_SORT entries,
// the tail padded with empty keys)
__device__ inline void adc_sort(uint64_t* buf, int cnt) {
    for (int i = cnt + int(threadIdx.x); i < ADC_SORT; i += ADC_THREADS) buf[i] = KEY_EMPTY;
    __syncthreads();
    for (int size = 2; size <= ADC_SORT; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < ADC_SORT / 2; i += ADC_THREADS) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = buf[lo], b = buf[hi];
                if ((a > b) == up) {
                    buf[lo] = b;
                    buf[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

template <int M>
__global__ void __launch_bounds__(ADC_THREADS) k_ivf_adc(const uint8_t* Q, int d, const int32_t* cid,
                                                         const int32_t* cdist, int W, const uint32_t* off,
                                                         const uint32_t* ids, const uint8_t* codes,
                                                         const float* beta, const float* pq, int ds, int L, int k,
                                                         int32_t* out_ids, float* out_d) {
    extern __shared__ __align__(16) uint8_t lds[];
    float* table = reinterpret_cast<float*>(lds);                      // M x 256
    uint64_t* buf = reinterpret_cast<uint64_t*>(table + M * PQ_K);     // ADC_SORT keys
    uint64_t* thresh = buf + ADC_SORT;                                 // the k-th best kept key
    int* sc = reinterpret_cast<int*>(thresh + 1);                      // [0] buffered keys, [1] kept keys
    uint32_t* pre = reinterpret_cast<uint32_t*>(sc + 4);               // W + 1 prefix of list lengths
    uint32_t* lstart = pre + ADC_WMAX + 4;                             // W list starts
    float* ldist = reinterpret_cast<float*>(lstart + ADC_WMAX);        // W centre distances
    uint32_t* rlo = reinterpret_cast<uint32_t*>(ldist + ADC_WMAX);     // ADC_RMAX: list of a round's first candidate
    float* qf = reinterpret_cast<float*>(rlo + ADC_RMAX);              // d
    const int64_t qi = blockIdx.x;
    const int t = threadIdx.x;

    for (int e = t; e < d; e += ADC_THREADS) qf[e] = float(Q[qi * d + e]);
    for (int w = t; w < W; w += ADC_THREADS) {
        const int l = cid[qi * W + w];
        uint32_t len = 0, st = 0;
        if (l >= 0) {
            st = off[l];
            len = off[l + 1] - st;
        }
        lstart[w] = st;
        pre[w + 1] = len;
        ldist[w] = l >= 0 ? float(cdist[qi * W + w]) : 0.f;
    }
    if (t == 0) {
        pre[0] = 0;
        sc[0] = 0;
        sc[1] = 0;
        *thresh = KEY_EMPTY;
    }
    __syncthreads();
    for (int e = t; e < M * PQ_K; e += ADC_THREADS) {
        const int j = e / PQ_K;
        const float* cw = pq + int64_t(e) * ds;
        float acc = 0.f;
        for (int q = 0; q < ds; ++q) acc = fmaf(qf[j * ds + q], cw[q], acc);
        table[e] = acc;
    }
    // prefix sums of the list lengths (W <= 1024: one per thread): scans
    // within each wavefront, then the wavefront totals (staged in rlo, which
    // is filled only afterwards)
    {
        static_assert(ADC_WMAX <= ADC_THREADS && ADC_THREADS / WAVE <= ADC_RMAX, "one list per thread");
        const int lane = t % WAVE, wv = t / WAVE;
        uint32_t v = t < W ? pre[t + 1] : 0u;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t y = __shfl_up(v, o, WAVE);
            if (lane >= o) v += y;
        }
        if (lane == WAVE - 1) rlo[wv] = v;
        __syncthreads();
        uint32_t before = 0;
        for (int i = 0; i < wv; ++i) before += rlo[i];
        if (t < W) pre[t + 1] = v + before;
        __syncthreads();
    }
    const int64_t total = min(int64_t(pre[W]), int64_t(L));
    // list of candidate g: the last w in [lo, hi] with pre[w] <= g (pre[lo] <= g)
    auto list_of = [&](int64_t g, int lo, int hi) {
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (int64_t(pre[mid]) <= g)
                lo = mid;
            else
                hi = mid - 1;
        }
        return lo;
    };
    // the lists of the rounds' first candidates bound every search to the
    // few lists a round spans
    const int64_t rounds = (total + ADC_THREADS - 1) / ADC_THREADS;
    const int known = int(min(rounds, int64_t(ADC_RMAX)));
    for (int r = t; r < known; r += ADC_THREADS) rlo[r] = uint32_t(list_of(int64_t(r) * ADC_THREADS, 0, W - 1));
    __syncthreads();

    // merge the buffered keys with the kept ones and keep the best k
    auto merge = [&]() {
        const int nb = min(sc[0], ADC_BUF), nk = sc[1];
        __syncthreads();
        // kept keys sit after the buffer
        adc_sort(buf, nb + nk);
        const int keep = min(k, nb + nk);
        // move the best `keep` to the tail region and reset the buffer
        __syncthreads();
        uint64_t v[ADC_KMAX / ADC_THREADS];
#pragma unroll
        for (int u = 0; u < ADC_KMAX / ADC_THREADS; ++u) {
            const int i = t + u * ADC_THREADS;
            v[u] = i < keep ? buf[i] : KEY_EMPTY;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < ADC_KMAX / ADC_THREADS; ++u) {
            const int i = t + u * ADC_THREADS;
            if (i < keep) buf[ADC_BUF + i] = v[u];
        }
        __syncthreads();
        if (t == 0) {
            sc[0] = 0;
            sc[1] = keep;
            *thresh = keep == k ? buf[ADC_BUF + k - 1] : KEY_EMPTY;
        }
        __syncthreads();
    };
    // buf[0 .. ADC_BUF): new keys; buf[ADC_BUF .. ADC_BUF + kept): the best so far.
    // Before a sort the kept keys are moved next to the buffered ones.
    auto compact = [&]() {
        const int nb = sc[0], nk = sc[1];
        __syncthreads();
        uint64_t v[ADC_KMAX / ADC_THREADS];
#pragma unroll
        for (int u = 0; u < ADC_KMAX / ADC_THREADS; ++u) {
            const int i = t + u * ADC_THREADS;
            v[u] = i < nk ? buf[ADC_BUF + i] : KEY_EMPTY;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < ADC_KMAX / ADC_THREADS; ++u) {
            const int i = t + u * ADC_THREADS;
            if (i < nk) buf[nb + i] = v[u];
        }
        __syncthreads();
    };

    // a round measures one candidate per thread and adds at most ADC_BUF / 2 keys
    for (int64_t g0 = 0, r = 0; g0 < total; g0 += ADC_THREADS, ++r) {
        const uint64_t th = *thresh;
        const int64_t g = g0 + t;
        if (g < total) {
            const int lo = list_of(g, r < known ? int(rlo[r]) : 0, r + 1 < known ? int(rlo[r + 1]) : W - 1);
            const int64_t pos = int64_t(lstart[lo]) + (g - pre[lo]);
            const uint8_t* cw = codes + pos * M;
            float acc = 0.f;
            if constexpr (M == 8) {
                const uint2 c = *reinterpret_cast<const uint2*>(cw);
#pragma unroll
                for (int j = 0; j < 4; ++j) acc += table[j * PQ_K + ((c.x >> (8 * j)) & 255u)];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc += table[(4 + j) * PQ_K + ((c.y >> (8 * j)) & 255u)];
            } else {
                const uint4 c = *reinterpret_cast<const uint4*>(cw);
                const uint32_t w4[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc += table[(4 * h + j) * PQ_K + ((w4[h] >> (8 * j)) & 255u)];
            }
            const uint32_t db = f_bits(fmaxf(ldist[lo] + beta[pos] - 2.f * acc, 0.f));
            // the id is read only for a candidate that can enter
            if (db <= key_dist(th)) {
                const uint64_t key = make_key(db, ids[pos]);
                if (key < th) {
                    const int slot = atomicAdd(&sc[0], 1);
                    buf[slot] = key;
                }
            }
        }
        __syncthreads();
        if (sc[0] > ADC_BUF / 2) {
            compact();
            merge();
        }
    }
    if (sc[0] > 0) {
        compact();
        merge();
    }
    const int kept = sc[1];
    for (int i = t; i < k; i += ADC_THREADS) {
        const int64_t o = qi * k + i;
        if (i < kept) {
            const uint64_t key = buf[ADC_BUF + i];
            out_ids[o] = int32_t(key_id(key));
            out_d[o] = bits_f(key_dist(key));
        } else {
            out_ids[o] = -1;
            out_d[o] = INFINITY;
        }
    }
}

int adc_lds_bytes(int M, int d) {
    return M * PQ_K * 4 + ADC_SORT * 8 + 8 + 16 + (ADC_WMAX + 4) * 4 + ADC_WMAX * 4 + ADC_WMAX * 4 + ADC_RMAX * 4 +
           d * 4;
}

void free_ivf(ann_ivf* v) {
    if (!v) return;
    if (v->centres) ann_index_free(v->centres);
    for (void* p : {static_cast<void*>(v->list_off), static_cast<void*>(v->list_ids), static_cast<void*>(v->codes),
                    static_cast<void*>(v->beta), static_cast<void*>(v->pq)})
        if (p) (void)hipFree(p);
    delete v;
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" {

int ann_ivf_build(const void* data, int64_t n, int32_t d, const ann_ivf_params* ip, ann_ivf** out) {
    ANN_REQUIRE(data && ip && out, "ann_ivf_build: null argument");
    ANN_REQUIRE(ip->struct_size == sizeof(ann_ivf_params), "ann_ivf_params.struct_size mismatch");
    ANN_REQUIRE(ip->lists >= 1 && ip->lists <= n, "ann_ivf_build: lists must be in [1, n]");
    ANN_REQUIRE(n >= PQ_K && n < (int64_t(1) << 31), "ann_ivf_build: n must be in [256, 2^31)");
    ANN_REQUIRE(ip->pq_m == 8 || ip->pq_m == 16, "ann_ivf_build: pq_m must be 8 or 16");
    ANN_REQUIRE(d > 0 && d % ip->pq_m == 0, "ann_ivf_build: pq_m must divide d");
    ANN_REQUIRE(ip->pq_iters >= 0 && ip->assign_budget >= 1, "ann_ivf_build: pq_iters >= 0, assign_budget >= 1");
    ANN_REQUIRE(ip->reserved == 0, "ann_ivf_params.reserved must be 0");
    ANN_REQUIRE(ip->centres.struct_size == sizeof(ann_build_params), "ann_ivf_build: centre index parameters");
    hipStream_t s = nullptr;
    auto v = new (std::nothrow) ann_ivf();
    if (!v) return set_error(ANN_ENOMEM, "ann_ivf_build: out of host memory");
    struct Guard {
        ann_ivf* v;
        std::vector<void*> tmp;
        ~Guard() {
            for (void* p : tmp)
                if (p) (void)hipFree(p);
            if (v) free_ivf(v);
        }
    } g{v, {}};
    v->n = n;
    v->d = d;
    v->C = ip->lists;
    v->m = ip->pq_m;
    v->ds = d / ip->pq_m;
    ANN_HIP_CHECK(hipGetDevice(&v->device));
    const uint8_t* X = static_cast<const uint8_t*>(data);

    // vocabulary: a seeded sample of the vectors (the first C entries of a
    // Fisher-Yates shuffle driven by SplitMix64), indexed by the augmented graph
    std::vector<int64_t> rows(size_t(v->C));
    kmeans_init_rows(n, v->C, ip->seed, rows.data());
    std::vector<uint8_t> cent(size_t(v->C) * d);
    for (int j = 0; j < v->C; ++j) std::copy_n(X + rows[j] * d, d, cent.data() + size_t(j) * d);
    int rc = ann_build_index(cent.data(), v->C, d, ANN_U8, &ip->centres, nullptr, nullptr, &v->centres);
    if (rc) return rc;

    // each vector to its list: the search over the centres, k = 1
    auto dmal = [&](void** p, size_t bytes) -> int {
        ANN_HIP_CHECK(hipMalloc(p, bytes));
        g.tmp.push_back(*p);
        return ANN_OK;
    };
    uint8_t* dX = nullptr;
    int32_t *assign = nullptr, *adist = nullptr;
    if ((rc = dmal(reinterpret_cast<void**>(&dX), size_t(n) * d))) return rc;
    if ((rc = dmal(reinterpret_cast<void**>(&assign), size_t(n) * 4))) return rc;
    if ((rc = dmal(reinterpret_cast<void**>(&adist), size_t(n) * 4))) return rc;
    ANN_HIP_CHECK(hipMemcpy(dX, X, size_t(n) * d, hipMemcpyHostToDevice));
    ann_search_params sp{};
    sp.struct_size = sizeof(ann_search_params);
    sp.queue_len = 64;
    if ((rc = ann_search_device(v->centres, dX, n, 1, ip->assign_budget, nullptr, nullptr, &sp, assign, adist, nullptr,
                                nullptr, s)))
        return rc;
    std::vector<int32_t> a_host(static_cast<size_t>(n));
    ANN_HIP_CHECK(hipMemcpy(a_host.data(), assign, size_t(n) * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i)
        if (a_host[size_t(i)] < 0) return set_error(ANN_ERESOURCE, "ann_ivf_build: a vector found no list");

    // residual product quantisation: k-means per subspace on the residuals
    float* resid = nullptr;
    if ((rc = dmal(reinterpret_cast<void**>(&resid), size_t(n) * d * 4))) return rc;
    const int64_t ne = n * d;
    hipLaunchKernelGGL(k_ivf_residual, dim3(unsigned(ceil_div(ne, 256))), dim3(256), 0, s, dX, n, d,
                       v->centres->X, assign, resid);
    ANN_HIP_CHECK(hipGetLastError());
    std::vector<int64_t> prow(PQ_K);
    kmeans_init_rows(n, PQ_K, ip->seed + 1, prow.data());
    int64_t* d_prow = nullptr;
    if ((rc = dmal(reinterpret_cast<void**>(&d_prow), PQ_K * 8))) return rc;
    ANN_HIP_CHECK(hipMemcpy(d_prow, prow.data(), PQ_K * 8, hipMemcpyHostToDevice));
    ANN_HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&v->pq), size_t(v->m) * PQ_K * v->ds * 4));
    hipLaunchKernelGGL(k_pq_init, dim3(unsigned(ceil_div(v->m * PQ_K * v->ds, 256))), dim3(256), 0, s, resid, d,
                       v->m, v->ds, d_prow, v->pq);
    ANN_HIP_CHECK(hipGetLastError());
    ann_index tmp;  // the residuals seen as an fp32 index, for the k-means kernels
    tmp.n = n;
    tmp.d = d;
    tmp.dtype = ANN_F32;
    tmp.P = v->m;
    tmp.K = PQ_K;
    tmp.device = v->device;
    tmp.row_bytes = int64_t(d) * 4;
    tmp.X = reinterpret_cast<uint8_t*>(resid);
    tmp.codebooks = v->pq;
    // residual components lie in [-255, 255]: member sums in int64 fixed point stay exact
    const int fx = std::max(0, std::min(40, int(std::floor(62.0 - std::log2(double(n)) - 8.0 - 2.0))));
    rc = build_codebooks(&tmp, ip->pq_iters, fx, s);
    tmp.X = nullptr;
    tmp.codebooks = nullptr;
    if (rc) return rc;

    // codes: the nearest codeword of each residual subvector (fp32, ties to
    // the smaller codeword), by the k-means assignment step
    uint8_t* codes_v = nullptr;
    int32_t* ca = nullptr;
    if ((rc = dmal(reinterpret_cast<void**>(&codes_v), size_t(n) * v->m))) return rc;
    if ((rc = dmal(reinterpret_cast<void**>(&ca), size_t(n) * 4))) return rc;
    for (int p = 0; p < v->m; ++p) {
        if ((rc = kmeans_assign_subspace(reinterpret_cast<const uint8_t*>(resid), n, d, true, v->ds, p, PQ_K,
                                         v->pq + int64_t(p) * PQ_K * v->ds, ca, s)))
            return rc;
        hipLaunchKernelGGL(k_pq_pack, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s, ca, n, v->m, p, codes_v);
        ANN_HIP_CHECK(hipGetLastError());
    }

    // inverted lists in increasing vector id (a counting sort on the host)
    std::vector<uint32_t> off(size_t(v->C) + 1, 0), ids(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) ++off[size_t(a_host[size_t(i)]) + 1];
    for (int j = 0; j < v->C; ++j) off[size_t(j) + 1] += off[size_t(j)];
    {
        std::vector<uint32_t> cur(off.begin(), off.end() - 1);
        for (int64_t i = 0; i < n; ++i) ids[cur[size_t(a_host[size_t(i)])]++] = uint32_t(i);
    }
    ANN_HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&v->list_off), off.size() * 4));
    ANN_HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&v->list_ids), ids.size() * 4));
    ANN_HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&v->codes), size_t(n) * v->m));
    ANN_HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&v->beta), size_t(n) * 4));
    ANN_HIP_CHECK(hipMemcpy(v->list_off, off.data(), off.size() * 4, hipMemcpyHostToDevice));
    ANN_HIP_CHECK(hipMemcpy(v->list_ids, ids.data(), ids.size() * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_ivf_place, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s, codes_v, v->centres->X, assign,
                       v->pq, v->list_ids, n, d, v->m, v->ds, v->codes, v->beta);
    ANN_HIP_CHECK(hipGetLastError());
    ANN_HIP_CHECK(hipDeviceSynchronize());
    v->bytes = int64_t(off.size()) * 4 + n * 4 + n * v->m + n * 4 + int64_t(v->m) * PQ_K * v->ds * 4;
    g.v = nullptr;
    *out = v;
    return ANN_OK;
}

int ann_ivf_get_info(const ann_ivf* v, ann_ivf_info* info) {
    ANN_REQUIRE(v && info, "ann_ivf_get_info: null argument");
    info->n = v->n;
    info->d = v->d;
    info->lists = v->C;
    info->pq_m = v->m;
    info->device_bytes = v->bytes;
    return ANN_OK;
}

int ann_ivf_export(const ann_ivf* v, uint8_t* centres, uint32_t* list_off, uint32_t* list_ids, uint8_t* codes,
                   float* pq_codebooks) {
    ANN_REQUIRE(v, "ann_ivf_export: null ivf");
    if (centres) ANN_HIP_CHECK(hipMemcpy(centres, v->centres->X, size_t(v->C) * v->d, hipMemcpyDeviceToHost));
    if (list_off) ANN_HIP_CHECK(hipMemcpy(list_off, v->list_off, size_t(v->C + 1) * 4, hipMemcpyDeviceToHost));
    if (list_ids) ANN_HIP_CHECK(hipMemcpy(list_ids, v->list_ids, size_t(v->n) * 4, hipMemcpyDeviceToHost));
    if (codes) ANN_HIP_CHECK(hipMemcpy(codes, v->codes, size_t(v->n) * v->m, hipMemcpyDeviceToHost));
    if (pq_codebooks)
        ANN_HIP_CHECK(hipMemcpy(pq_codebooks, v->pq, size_t(v->m) * PQ_K * v->ds * 4, hipMemcpyDeviceToHost));
    return ANN_OK;
}

const ann_index* ann_ivf_centres(const ann_ivf* v) { return v ? v->centres : nullptr; }

int ann_ivf_search_device(const ann_ivf* v, const void* d_queries, int64_t nq, int32_t k, int32_t lists,
                          int32_t centre_budget, int32_t candidates, int32_t* d_ids, float* d_dists, void* stream) {
    ANN_REQUIRE(v, "ann_ivf_search_device: null ivf");
    ANN_REQUIRE(nq >= 0 && k >= 1 && k <= ADC_KMAX, "ann_ivf_search_device: k must be in [1, 1024]");
    ANN_REQUIRE(lists >= 1 && lists <= ADC_WMAX, "ann_ivf_search_device: lists must be in [1, 1024]");
    ANN_REQUIRE(centre_budget >= 0 && candidates >= 0, "ann_ivf_search_device: negative budget");
    ANN_REQUIRE(nq == 0 || (d_queries && d_ids && d_dists), "ann_ivf_search_device: null buffer");
    if (nq == 0) return ANN_OK;
    int max_lds = 0;
    ANN_HIP_CHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, v->device));
    if (adc_lds_bytes(v->m, v->d) > max_lds)
        return set_error(ANN_EUNSUPPORTED, "ann_ivf_search_device: the distance tables of this d and m exceed LDS");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *cid = nullptr, *cd = nullptr;
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&cid), size_t(nq) * lists * 4, s));
    ANN_HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&cd), size_t(nq) * lists * 4, s));
    ann_search_params sp{};
    sp.struct_size = sizeof(ann_search_params);
    sp.queue_len = 64;
    int rc = ann_search_device(v->centres, d_queries, nq, lists, centre_budget, nullptr, nullptr, &sp, cid, cd, nullptr,
                               nullptr, stream);
    if (rc == ANN_OK) {
        const int lds = adc_lds_bytes(v->m, v->d);
        const dim3 grid(static_cast<unsigned>(nq));
        if (v->m == 8)
            hipLaunchKernelGGL(k_ivf_adc<8>, grid, dim3(ADC_THREADS), lds, s, static_cast<const uint8_t*>(d_queries),
                               v->d, cid, cd, lists, v->list_off, v->list_ids, v->codes, v->beta, v->pq, v->ds,
                               candidates, k, d_ids, d_dists);
        else
            hipLaunchKernelGGL(k_ivf_adc<16>, grid, dim3(ADC_THREADS), lds, s, static_cast<const uint8_t*>(d_queries),
                               v->d, cid, cd, lists, v->list_off, v->list_ids, v->codes, v->beta, v->pq, v->ds,
                               candidates, k, d_ids, d_dists);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = set_error(ANN_EDEVICE, std::string("k_ivf_adc: ") + hipGetErrorString(e));
    }
    (void)hipFreeAsync(cid, s);
    (void)hipFreeAsync(cd, s);
    return rc;
}

void ann_ivf_free(ann_ivf* v) { free_ivf(v); }

}  // extern "C"
