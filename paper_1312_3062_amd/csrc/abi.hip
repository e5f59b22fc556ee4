// C ABI of the library (include/ann.h): argument checks, the index object,
// build orchestration, import / export / save / load, search wrappers.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "internal.hpp"

namespace ann {

static thread_local std::string g_last_error;

int set_error(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int dalloc(ann_index* idx, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return set_error(ANN_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                         hipGetErrorString(e));
    }
    idx->bytes += int64_t(bytes);
    return ANN_OK;
}

static void free_index(ann_index* idx) {
    if (!idx) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(idx->device);
    for (void* p : {static_cast<void*>(idx->X), static_cast<void*>(idx->Xbf16), idx->codebooks,
                    static_cast<void*>(idx->G), static_cast<void*>(idx->boff), static_cast<void*>(idx->bids)})
        if (p) (void)hipFree(p);
    (void)hipSetDevice(cur);
    delete idx;
}

struct IndexGuard {
    ann_index* p;
    ~IndexGuard() { free_index(p); }
    ann_index* release() {
        ann_index* r = p;
        p = nullptr;
        return r;
    }
};

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// shape checks shared by build and import
static int check_shape(int64_t n, int32_t d, int32_t dtype, int32_t P, int32_t K, int32_t R) {
    ANN_REQUIRE(dtype == ANN_U8 || dtype == ANN_F32, "dtype must be ANN_U8 or ANN_F32");
    ANN_REQUIRE(n >= 1, "n must be >= 1");
    ANN_REQUIRE(n < (int64_t(1) << 31), "n must be below 2^31");
    ANN_REQUIRE(d >= 1, "d must be >= 1");
    ANN_REQUIRE(P >= 1 && P <= 4, "P must be in [1, 4]");
    ANN_REQUIRE(d % P == 0, "P must divide d");
    ANN_REQUIRE(K >= 1 && K <= 256, "K must be in [1, 256]");
    ANN_REQUIRE(n + ipow(K, P) < (int64_t(1) << 32), "n + K^P must stay below 2^32");
    ANN_REQUIRE(R >= 0 && (R < n || R == 0), "graph_k must be in [0, n)");
    if (dtype == ANN_U8) {
        ANN_REQUIRE(d % 16 == 0, "u8 vectors must be a multiple of 16 bytes");
        ANN_REQUIRE(d <= 512, "u8 dimension above 512 is not supported");
    } else {
        ANN_REQUIRE(d % 4 == 0, "f32 dimension must be a multiple of 4");
    }
    return ANN_OK;
}

static ann_index* new_index(int64_t n, int32_t d, int32_t dtype, int32_t P, int32_t K, int32_t R) {
    ann_index* idx = new (std::nothrow) ann_index();
    if (!idx) return nullptr;
    idx->n = n;
    idx->d = d;
    idx->dtype = dtype;
    idx->P = P;
    idx->K = K;
    idx->R = R;
    idx->nb = ipow(K, P);
    idx->row_bytes = dtype == ANN_F32 ? int64_t(d) * 4 : d;
    (void)hipGetDevice(&idx->device);
    return idx;
}

static int upload(ann_index* idx, void** dst, const void* src, size_t bytes) {
    int rc = dalloc(idx, dst, bytes);
    if (rc) return rc;
    if (src && bytes) ANN_HIP_CHECK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return ANN_OK;
}

static int check_graph_rows(const uint32_t* g, int64_t n, int R) {
    std::vector<uint32_t> row(R);
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < R; ++j) {
            const uint32_t v = g[i * R + j];
            if (v >= uint64_t(n)) return set_error(ANN_EINVAL, "graph id out of range in row " + std::to_string(i));
            row[j] = v;
        }
        std::sort(row.begin(), row.end());
        if (std::adjacent_find(row.begin(), row.end()) != row.end())
            return set_error(ANN_EINVAL, "graph row " + std::to_string(i) + " repeats an id");
    }
    return ANN_OK;
}

static int check_bridge_lists(const uint32_t* off, const uint32_t* ids, int64_t nb, int64_t n) {
    if (off[0] != 0) return set_error(ANN_EINVAL, "bridge_off[0] must be 0");
    std::vector<uint32_t> lst;
    for (int64_t b = 0; b < nb; ++b) {
        if (off[b + 1] < off[b]) return set_error(ANN_EINVAL, "bridge_off must be non-decreasing");
        const uint32_t len = off[b + 1] - off[b];
        if (len == 0) continue;
        lst.assign(ids + off[b], ids + off[b + 1]);
        for (uint32_t v : lst)
            if (v >= uint64_t(n)) return set_error(ANN_EINVAL, "bridge id out of range in list " + std::to_string(b));
        if (len > 1) {
            std::sort(lst.begin(), lst.end());
            if (std::adjacent_find(lst.begin(), lst.end()) != lst.end())
                return set_error(ANN_EINVAL, "bridge list " + std::to_string(b) + " repeats an id");
        }
    }
    return ANN_OK;
}

static int fixed_point_log2(const float* x, int64_t m, int64_t n) {
    float mx = 0.f;
    for (int64_t i = 0; i < m; ++i) mx = std::max(mx, std::fabs(x[i]));
    if (!(mx > 0.f)) return 30;
    const int e = int(std::floor(62.0 - std::log2(double(n)) - std::log2(double(mx)) - 2.0));
    return std::max(-60, std::min(100, e));
}

}  // namespace ann

using namespace ann;

extern "C" {

const char* ann_last_error(void) { return g_last_error.c_str(); }

int ann_version(void) { return 10000; }

int ann_build_index(const void* data, int64_t n, int32_t d, int32_t dtype, const ann_build_params* bp,
                    const void* codebooks, const uint32_t* graph, ann_index** out) {
    ANN_REQUIRE(data && bp && out, "ann_build_index: null data, params or out");
    ANN_REQUIRE(bp->struct_size == sizeof(ann_build_params), "ann_build_params.struct_size mismatch");
    int rc = check_shape(n, d, dtype, bp->P, bp->K, bp->graph_k);
    if (rc) return rc;
    ANN_REQUIRE(bp->kmeans_iters >= 0, "kmeans_iters must be >= 0");
    ANN_REQUIRE(bp->bridge_t >= 1, "bridge_t must be >= 1");
    ANN_REQUIRE(bp->bridge_b >= 0, "bridge_b must be >= 0");
    ANN_REQUIRE(bp->reserved == 0, "reserved must be 0");
    ANN_REQUIRE(codebooks || bp->K <= n, "K must not exceed n when training codebooks");
    if (graph) {
        rc = check_graph_rows(graph, n, bp->graph_k);
        if (rc) return rc;
    }
    IndexGuard g{new_index(n, d, dtype, bp->P, bp->K, bp->graph_k)};
    if (!g.p) return set_error(ANN_ENOMEM, "host allocation failed");
    ann_index* idx = g.p;
    hipStream_t s = nullptr;
    const size_t xbytes = size_t(n) * idx->row_bytes;
    rc = upload(idx, reinterpret_cast<void**>(&idx->X), data, xbytes);
    if (rc) return rc;

    // codebooks: given, or k-means from seeded initial rows
    const int ds = d / bp->P;
    const size_t esz = dtype == ANN_F32 ? 4 : 1;
    const size_t cbytes = size_t(bp->P) * bp->K * ds * esz;
    if (codebooks) {
        rc = upload(idx, &idx->codebooks, codebooks, cbytes);
        if (rc) return rc;
    } else {
        std::vector<int64_t> rows(bp->K);
        kmeans_init_rows(n, bp->K, bp->seed, rows.data());
        std::vector<uint8_t> init(cbytes);
        for (int p = 0; p < bp->P; ++p)
            for (int j = 0; j < bp->K; ++j)
                std::memcpy(&init[(size_t(p) * bp->K + j) * ds * esz],
                            static_cast<const uint8_t*>(data) + size_t(rows[j]) * idx->row_bytes + size_t(p) * ds * esz,
                            ds * esz);
        rc = upload(idx, &idx->codebooks, init.data(), cbytes);
        if (rc) return rc;
        const int fx = dtype == ANN_F32
                           ? fixed_point_log2(static_cast<const float*>(data), n * int64_t(d), n)
                           : 0;
        rc = build_codebooks(idx, bp->kmeans_iters, fx, s);
        if (rc) return rc;
    }

    // exact kNN graph (Sec. 4.1; each row the R nearest others)
    if (bp->graph_k > 0) {
        if (graph) {
            rc = upload(idx, reinterpret_cast<void**>(&idx->G), graph, size_t(n) * bp->graph_k * 4);
            if (rc) return rc;
        } else {
            rc = dalloc(idx, reinterpret_cast<void**>(&idx->G), size_t(n) * bp->graph_k * 4);
            if (rc) return rc;
            void* tmp = nullptr;
            ANN_HIP_CHECK(hipMalloc(&tmp, size_t(n) * bp->graph_k * 4));
            rc = launch_knn(idx->X, n, d, dtype, idx->X, n, bp->graph_k, 1, reinterpret_cast<int32_t*>(idx->G), tmp,
                            s);
            hipError_t e = hipStreamSynchronize(s);
            (void)hipFree(tmp);
            if (rc) return rc;
            if (e != hipSuccess) return set_error(ANN_EDEVICE, std::string("kNN graph: ") + hipGetErrorString(e));
        }
    }

    // bridge graph (Sec. 4.1)
    rc = build_bridge_graph(idx, bp->bridge_t, bp->bridge_b, s);
    if (rc) return rc;
    if (dtype == ANN_F32) {
        rc = make_bf16_copy(idx, s);
        if (rc) return rc;
    }
    ANN_HIP_CHECK(hipStreamSynchronize(s));
    *out = g.release();
    return ANN_OK;
}

int ann_index_import(const void* data, int64_t n, int32_t d, int32_t dtype, int32_t P, int32_t K,
                     const void* codebooks, int32_t graph_k, const uint32_t* graph, const uint32_t* bridge_off,
                     const uint32_t* bridge_ids, ann_index** out) {
    ANN_REQUIRE(data && codebooks && bridge_off && out, "ann_index_import: null argument");
    ANN_REQUIRE(graph_k == 0 || graph, "ann_index_import: graph is null but graph_k > 0");
    int rc = check_shape(n, d, dtype, P, K, graph_k);
    if (rc) return rc;
    const int64_t nb = ipow(K, P);
    const int64_t E = bridge_off[nb];
    ANN_REQUIRE(E == 0 || bridge_ids, "ann_index_import: bridge_ids is null");
    rc = check_bridge_lists(bridge_off, bridge_ids, nb, n);
    if (rc) return rc;
    if (graph_k > 0) {
        rc = check_graph_rows(graph, n, graph_k);
        if (rc) return rc;
    }
    IndexGuard g{new_index(n, d, dtype, P, K, graph_k)};
    if (!g.p) return set_error(ANN_ENOMEM, "host allocation failed");
    ann_index* idx = g.p;
    idx->E = E;
    const size_t esz = dtype == ANN_F32 ? 4 : 1;
    if ((rc = upload(idx, reinterpret_cast<void**>(&idx->X), data, size_t(n) * idx->row_bytes))) return rc;
    if ((rc = upload(idx, &idx->codebooks, codebooks, size_t(P) * K * (d / P) * esz))) return rc;
    if (graph_k > 0 &&
        (rc = upload(idx, reinterpret_cast<void**>(&idx->G), graph, size_t(n) * graph_k * 4)))
        return rc;
    if ((rc = upload(idx, reinterpret_cast<void**>(&idx->boff), bridge_off, size_t(nb + 1) * 4))) return rc;
    if ((rc = upload(idx, reinterpret_cast<void**>(&idx->bids), bridge_ids, size_t(E) * 4))) return rc;
    if (dtype == ANN_F32) {
        if ((rc = make_bf16_copy(idx, nullptr))) return rc;
        ANN_HIP_CHECK(hipStreamSynchronize(nullptr));
    }
    *out = g.release();
    return ANN_OK;
}

int ann_index_get_info(const ann_index* idx, ann_index_info* info) {
    ANN_REQUIRE(idx && info, "ann_index_get_info: null argument");
    info->n = idx->n;
    info->d = idx->d;
    info->dtype = idx->dtype;
    info->P = idx->P;
    info->K = idx->K;
    info->graph_k = idx->R;
    info->reserved = 0;
    info->n_bridges = idx->nb;
    info->n_bridge_entries = idx->E;
    info->device_bytes = idx->bytes;
    return ANN_OK;
}

int ann_index_export(const ann_index* idx, void* codebooks, uint32_t* graph, uint32_t* bridge_off,
                     uint32_t* bridge_ids) {
    ANN_REQUIRE(idx, "ann_index_export: null index");
    const size_t esz = idx->dtype == ANN_F32 ? 4 : 1;
    if (codebooks)
        ANN_HIP_CHECK(hipMemcpy(codebooks, idx->codebooks, size_t(idx->P) * idx->K * (idx->d / idx->P) * esz,
                                hipMemcpyDeviceToHost));
    if (graph && idx->R > 0)
        ANN_HIP_CHECK(hipMemcpy(graph, idx->G, size_t(idx->n) * idx->R * 4, hipMemcpyDeviceToHost));
    if (bridge_off) ANN_HIP_CHECK(hipMemcpy(bridge_off, idx->boff, size_t(idx->nb + 1) * 4, hipMemcpyDeviceToHost));
    if (bridge_ids && idx->E > 0)
        ANN_HIP_CHECK(hipMemcpy(bridge_ids, idx->bids, size_t(idx->E) * 4, hipMemcpyDeviceToHost));
    return ANN_OK;
}

// ---- save / load: "ANNMI\0\0\1", then the header, then the arrays
struct FileHeader {
    char magic[8];
    int32_t version, dtype, d, P, K, R;
    int64_t n, nb, E;
};

static const char kMagic[8] = {'A', 'N', 'N', 'M', 'I', 0, 0, 1};

int ann_index_save(const ann_index* idx, const char* path) {
    ANN_REQUIRE(idx && path, "ann_index_save: null argument");
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "wb"), std::fclose);
    if (!f) return set_error(ANN_EIO, std::string("cannot open ") + path);
    FileHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = 1;
    h.dtype = idx->dtype;
    h.d = idx->d;
    h.P = idx->P;
    h.K = idx->K;
    h.R = idx->R;
    h.n = idx->n;
    h.nb = idx->nb;
    h.E = idx->E;
    if (std::fwrite(&h, sizeof h, 1, f.get()) != 1) return set_error(ANN_EIO, "write failed");
    const size_t esz = idx->dtype == ANN_F32 ? 4 : 1;
    struct Part {
        const void* dev;
        size_t bytes;
    } parts[] = {{idx->X, size_t(idx->n) * idx->row_bytes},
                 {idx->codebooks, size_t(idx->P) * idx->K * (idx->d / idx->P) * esz},
                 {idx->G, size_t(idx->n) * idx->R * 4},
                 {idx->boff, size_t(idx->nb + 1) * 4},
                 {idx->bids, size_t(idx->E) * 4}};
    std::vector<uint8_t> buf;
    for (const Part& p : parts) {
        const size_t chunk = size_t(64) << 20;
        for (size_t o = 0; o < p.bytes; o += chunk) {
            const size_t m = std::min(chunk, p.bytes - o);
            buf.resize(m);
            ANN_HIP_CHECK(hipMemcpy(buf.data(), static_cast<const uint8_t*>(p.dev) + o, m, hipMemcpyDeviceToHost));
            if (std::fwrite(buf.data(), 1, m, f.get()) != m) return set_error(ANN_EIO, "write failed");
        }
    }
    return ANN_OK;
}

int ann_index_load(const char* path, ann_index** out) {
    ANN_REQUIRE(path && out, "ann_index_load: null argument");
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "rb"), std::fclose);
    if (!f) return set_error(ANN_EIO, std::string("cannot open ") + path);
    FileHeader h{};
    if (std::fread(&h, sizeof h, 1, f.get()) != 1 || std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1)
        return set_error(ANN_EIO, "not an index file of this version");
    int rc = check_shape(h.n, h.d, h.dtype, h.P, h.K, h.R);
    if (rc) return rc;
    if (h.nb != ipow(h.K, h.P) || h.E < 0) return set_error(ANN_EIO, "corrupt index header");
    const size_t esz = h.dtype == ANN_F32 ? 4 : 1;
    auto rd = [&](std::vector<uint8_t>& v, size_t bytes) {
        v.resize(bytes);
        return bytes == 0 || std::fread(v.data(), 1, bytes, f.get()) == bytes;
    };
    std::vector<uint8_t> X, cb, G, off, ids;
    if (!rd(X, size_t(h.n) * h.d * esz) || !rd(cb, size_t(h.P) * h.K * (h.d / h.P) * esz) ||
        !rd(G, size_t(h.n) * h.R * 4) || !rd(off, size_t(h.nb + 1) * 4) || !rd(ids, size_t(h.E) * 4))
        return set_error(ANN_EIO, "truncated index file");
    if (reinterpret_cast<const uint32_t*>(off.data())[h.nb] != uint64_t(h.E))
        return set_error(ANN_EIO, "corrupt bridge offsets");
    return ann_index_import(X.data(), h.n, h.d, h.dtype, h.P, h.K, cb.data(), h.R,
                            reinterpret_cast<const uint32_t*>(G.data()), reinterpret_cast<const uint32_t*>(off.data()),
                            reinterpret_cast<const uint32_t*>(ids.data()), out);
}

void ann_index_free(ann_index* idx) { free_index(idx); }

// struct_size of the first version of ann_search_params (no tuning fields)
static constexpr uint32_t kSearchParamsV1 = 16;

static int check_search(const ann_index* idx, int64_t nq, int32_t k, int32_t budget, const ann_search_params* sp) {
    ANN_REQUIRE(idx, "search: null index");
    ANN_REQUIRE(nq >= 0, "search: nq must be >= 0");
    ANN_REQUIRE(k >= 1 && k <= 1024, "search: k must be in [1, 1024]");
    ANN_REQUIRE(budget >= 0, "search: budget must be >= 0");
    ANN_REQUIRE(budget <= (1 << 20), "search: budget above 2^20");
    if (sp) {
        ANN_REQUIRE(sp->struct_size == sizeof(ann_search_params) || sp->struct_size == kSearchParamsV1,
                    "ann_search_params.struct_size mismatch");
        ANN_REQUIRE(sp->queue_len >= 1 && sp->queue_len <= 64, "queue_len must be in [1, 64]");
        ANN_REQUIRE(sp->precision == ANN_PRECISION_EXACT || sp->precision == ANN_PRECISION_BF16_RERANK,
                    "unknown precision");
        ANN_REQUIRE(sp->rerank_k >= 0 && sp->rerank_k <= 1024, "rerank_k must be in [0, 1024]");
        if (sp->struct_size == sizeof(ann_search_params)) {
            ANN_REQUIRE(sp->lookahead >= 0 && sp->lookahead <= 8, "lookahead must be in [0, 8]");
            ANN_REQUIRE(sp->persistent == 0 || sp->persistent == 1, "persistent must be 0 or 1");
            ANN_REQUIRE(sp->waves_per_cu >= 0 && sp->waves_per_cu <= 64, "waves_per_cu must be in [0, 64]");
            ANN_REQUIRE(sp->order == 0 || sp->order == 1, "order must be 0 or 1");
        }
    }
    return ANN_OK;
}

static SearchLaunch make_launch(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                                const int32_t* d_k, const int32_t* d_budget, const ann_search_params* sp,
                                int32_t* d_ids, void* d_dists, int32_t* d_stats, int32_t* d_trace, void* stream) {
    SearchLaunch a{};
    a.idx = idx;
    a.d_q = d_queries;
    a.nq = nq;
    a.kmax = k;
    a.Tmax = budget;
    a.d_k = d_k;
    a.d_T = d_budget;
    a.L = sp ? sp->queue_len : 64;
    a.precision = (sp && idx->dtype == ANN_F32) ? sp->precision : ANN_PRECISION_EXACT;
    a.rerank_k = sp ? sp->rerank_k : 0;
    a.d_ids = d_ids;
    a.d_dists = d_dists;
    a.d_stats = d_stats;
    a.d_trace = d_trace;
    a.stream = static_cast<hipStream_t>(stream);
    if (sp && sp->struct_size == sizeof(ann_search_params)) {
        a.lookahead = sp->lookahead;
        a.persistent = sp->persistent;
        a.waves_per_cu = sp->waves_per_cu;
        a.order = sp->order;
    }
    return a;
}

}  // extern "C"

namespace ann {
// Smallest workspace ann_search_device_ws accepts for this request: the
// per-query lists plus one global multi-sequence slot.  Arguments are
// checked as ann_search_device checks them.
int search_min_workspace(const ann_index* idx, int64_t nq, int32_t k, int32_t budget, const ann_search_params* sp,
                         int64_t* bytes) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    return search_workspace_bytes(
        make_launch(idx, nullptr, nq, k, budget, nullptr, nullptr, sp, nullptr, nullptr, nullptr, nullptr, nullptr),
        bytes, true);
}
}  // namespace ann

extern "C" {

int ann_search_device(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                      const int32_t* d_k, const int32_t* d_budget, const ann_search_params* sp, int32_t* d_ids,
                      void* d_dists, int32_t* d_stats, int32_t* d_trace, void* stream) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    ANN_REQUIRE(nq == 0 || (d_queries && d_ids && d_dists), "search: null device buffer");
    return launch_search(make_launch(idx, d_queries, nq, k, budget, d_k, d_budget, sp, d_ids, d_dists, d_stats,
                                     d_trace, stream));
}

int ann_search_workspace_size(const ann_index* idx, int64_t nq, int32_t k, int32_t budget,
                              const ann_search_params* sp, int64_t* bytes) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    ANN_REQUIRE(bytes, "ann_search_workspace_size: null output");
    return search_workspace_bytes(
        make_launch(idx, nullptr, nq, k, budget, nullptr, nullptr, sp, nullptr, nullptr, nullptr, nullptr, nullptr),
        bytes);
}

int ann_search_device_ws(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                         const int32_t* d_k, const int32_t* d_budget, const ann_search_params* sp, int32_t* d_ids,
                         void* d_dists, int32_t* d_stats, int32_t* d_trace, void* workspace, int64_t workspace_bytes,
                         void* stream) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    ANN_REQUIRE(nq == 0 || (d_queries && d_ids && d_dists), "search: null device buffer");
    ANN_REQUIRE(nq == 0 || workspace, "ann_search_device_ws: null workspace");
    ANN_REQUIRE((reinterpret_cast<uintptr_t>(workspace) & 15) == 0, "ann_search_device_ws: workspace not 16-byte aligned");
    SearchLaunch a =
        make_launch(idx, d_queries, nq, k, budget, d_k, d_budget, sp, d_ids, d_dists, d_stats, d_trace, stream);
    a.workspace = workspace;
    a.workspace_bytes = workspace_bytes;
    return launch_search(a);
}

int ann_search_graph_device(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                            const int32_t* d_seeds, int32_t n_seeds, const ann_search_params* sp, int32_t* d_ids,
                            void* d_dists, int32_t* d_stats, int32_t* d_trace, void* stream) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    ANN_REQUIRE(nq == 0 || (d_queries && d_ids && d_dists), "search: null device buffer");
    ANN_REQUIRE(n_seeds >= 0 && n_seeds <= (1 << 20), "ann_search_graph_device: n_seeds must be in [0, 2^20]");
    ANN_REQUIRE(n_seeds == 0 || d_seeds, "ann_search_graph_device: null seeds");
    ANN_REQUIRE(!sp || sp->precision == ANN_PRECISION_EXACT || idx->dtype == ANN_U8,
                "ann_search_graph_device: exact precision only");
    SearchLaunch a =
        make_launch(idx, d_queries, nq, k, budget, nullptr, nullptr, sp, d_ids, d_dists, d_stats, d_trace, stream);
    a.precision = ANN_PRECISION_EXACT;
    a.graph_only = true;
    a.d_seeds = reinterpret_cast<const uint32_t*>(d_seeds);
    a.n_seeds = n_seeds;
    return launch_search(a);
}

int ann_autotune(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                 const int32_t* d_k, const int32_t* d_budget, ann_search_params* sp, void* stream) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    ANN_REQUIRE(sp && sp->struct_size == sizeof(ann_search_params), "ann_autotune: params of the current version");
    ANN_REQUIRE(nq > 0 && d_queries, "ann_autotune: empty batch");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t ob = size_t(nq) * k * 4;
    void *di = nullptr, *dd = nullptr;
    ANN_HIP_CHECK(hipMalloc(&di, ob));
    ANN_HIP_CHECK(hipMalloc(&dd, ob));
    struct Free {
        void** p[2];
        ~Free() {
            for (void** q : p)
                if (*q) (void)hipFree(*q);
        }
    } guard{{&di, &dd}};
    hipEvent_t e0, e1;
    ANN_HIP_CHECK(hipEventCreate(&e0));
    ANN_HIP_CHECK(hipEventCreate(&e1));
    std::vector<int32_t> ref(size_t(nq) * k), got(size_t(nq) * k);
    const int max_spec = idx->R > 0 ? std::min(8, 64 / idx->R) : 1;
    std::vector<int> specs = {max_spec};
    for (int v : {1, 2, 4})
        if (v < max_spec) specs.push_back(v);
    std::vector<ann_search_params> cands;
    for (int spec : specs) {
        ann_search_params c = *sp;
        c.lookahead = spec;
        c.persistent = 0;
        c.waves_per_cu = 0;
        c.order = 0;
        cands.push_back(c);
        for (int wpc : {0, 8, 4}) {
            for (int ord : {0, 1}) {
                if (ord && !d_budget) continue;
                ann_search_params p = c;
                p.persistent = 1;
                p.waves_per_cu = wpc;
                p.order = ord;
                cands.push_back(p);
            }
        }
    }
    auto time_one = [&](const ann_search_params& c, float& t) -> int {
        ANN_HIP_CHECK(hipEventRecord(e0, st));
        const int r = ann_search_device(idx, d_queries, nq, k, budget, d_k, d_budget, &c, static_cast<int32_t*>(di),
                                        dd, nullptr, nullptr, stream);
        if (r) return r;
        ANN_HIP_CHECK(hipEventRecord(e1, st));
        ANN_HIP_CHECK(hipEventSynchronize(e1));
        ANN_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
        return ANN_OK;
    };
    // first pass: every candidate twice (the better run counts), results
    // checked against the default launch's
    std::vector<float> first(cands.size(), 1e30f);
    for (size_t i = 0; i < cands.size(); ++i) {
        for (int rep = 0; rep < 2; ++rep) {
            float t = 0.f;
            if ((rc = time_one(cands[i], t))) return rc;
            first[i] = std::min(first[i], t);
        }
        ANN_HIP_CHECK(hipMemcpy(i == 0 ? ref.data() : got.data(), di, ob, hipMemcpyDeviceToHost));
        if (i > 0 && got != ref)
            return set_error(ANN_ESTATE, "ann_autotune: a launch setting changed the results (candidate " +
                                             std::to_string(i) + ")");
    }
    // finals: the three fastest and the default, timed in turn five times
    // each; the lowest median wins (a single lucky run cannot)
    std::vector<size_t> fin(cands.size());
    for (size_t i = 0; i < fin.size(); ++i) fin[i] = i;
    std::sort(fin.begin(), fin.end(), [&](size_t x, size_t y) { return first[x] < first[y]; });
    fin.resize(std::min<size_t>(3, fin.size()));
    if (std::find(fin.begin(), fin.end(), size_t(0)) == fin.end()) fin.push_back(0);
    std::vector<std::vector<float>> runs(fin.size());
    for (int rep = 0; rep < 5; ++rep)
        for (size_t f = 0; f < fin.size(); ++f) {
            float t = 0.f;
            if ((rc = time_one(cands[fin[f]], t))) return rc;
            runs[f].push_back(t);
        }
    float best = 1e30f;
    ann_search_params best_p = cands[0];
    for (size_t f = 0; f < fin.size(); ++f) {
        std::sort(runs[f].begin(), runs[f].end());
        const float med = runs[f][runs[f].size() / 2];
        if (med < best) {
            best = med;
            best_p = cands[fin[f]];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    sp->lookahead = best_p.lookahead;
    sp->persistent = best_p.persistent;
    sp->waves_per_cu = best_p.waves_per_cu;
    sp->order = best_p.order;
    return ANN_OK;
}

int ann_search(const ann_index* idx, const void* queries, int64_t nq, int32_t k, int32_t budget,
               const ann_search_params* sp, int32_t* ids, void* dists) {
    int rc = check_search(idx, nq, k, budget, sp);
    if (rc) return rc;
    if (nq == 0) return ANN_OK;
    ANN_REQUIRE(queries && ids && dists, "ann_search: null host buffer");
    const size_t qb = size_t(nq) * idx->row_bytes, ob = size_t(nq) * k * 4, sb = size_t(nq) * ANN_NSTATS * 4;
    void *dq = nullptr, *di = nullptr, *dd = nullptr, *dst = nullptr;
    struct Free {
        void** p[4];
        ~Free() {
            for (void** q : p)
                if (*q) (void)hipFree(*q);
        }
    } guard{{&dq, &di, &dd, &dst}};
    ANN_HIP_CHECK(hipMalloc(&dq, qb));
    ANN_HIP_CHECK(hipMalloc(&di, ob));
    ANN_HIP_CHECK(hipMalloc(&dd, ob));
    ANN_HIP_CHECK(hipMalloc(&dst, sb));
    ANN_HIP_CHECK(hipMemcpy(dq, queries, qb, hipMemcpyHostToDevice));
    rc = ann_search_device(idx, dq, nq, k, budget, nullptr, nullptr, sp, static_cast<int32_t*>(di), dd,
                           static_cast<int32_t*>(dst), nullptr, nullptr);
    if (rc) return rc;
    ANN_HIP_CHECK(hipStreamSynchronize(nullptr));
    ANN_HIP_CHECK(hipMemcpy(ids, di, ob, hipMemcpyDeviceToHost));
    ANN_HIP_CHECK(hipMemcpy(dists, dd, ob, hipMemcpyDeviceToHost));
    std::vector<int32_t> st(size_t(nq) * ANN_NSTATS);
    ANN_HIP_CHECK(hipMemcpy(st.data(), dst, sb, hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < nq; ++q)
        if (st[size_t(q) * ANN_NSTATS + ANN_STAT_FLAGS])
            return set_error(ANN_ERESOURCE, "query " + std::to_string(q) +
                                                ": multi-sequence frontier outgrew its capacity");
    return ANN_OK;
}

int ann_query_tables_device(const ann_index* idx, const void* d_queries, int64_t nq, void* d_sorted, int32_t* d_perm,
                            void* stream) {
    ANN_REQUIRE(idx && nq >= 0, "ann_query_tables_device: bad argument");
    ANN_REQUIRE(nq == 0 || (d_queries && d_sorted && d_perm), "ann_query_tables_device: null buffer");
    return launch_tables(idx, d_queries, nq, d_sorted, d_perm, static_cast<hipStream_t>(stream));
}

int ann_knn_device(const void* d_x, int64_t n, int32_t d, int32_t dtype, const void* d_q, int64_t nq, int32_t k,
                   int32_t exclude_self, int32_t* d_ids, void* d_dists, void* stream) {
    ANN_REQUIRE(d_x && (nq == 0 || (d_q && d_ids && d_dists)), "ann_knn_device: null buffer");
    ANN_REQUIRE(dtype == ANN_U8 || dtype == ANN_F32, "ann_knn_device: bad dtype");
    ANN_REQUIRE(!exclude_self || nq <= n, "ann_knn_device: exclude_self needs nq <= n");
    return launch_knn(d_x, n, d, dtype, d_q, nq, k, exclude_self, d_ids, d_dists, static_cast<hipStream_t>(stream));
}

}  // extern "C"
