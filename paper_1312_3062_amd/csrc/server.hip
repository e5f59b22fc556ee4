// Continuous-batching request server over a device-resident index.
//
// Requests (a batch of query vectors with their own k and budget) are queued
// by ann_server_submit and served by micro-batch launches on a few streams
// ("slots").  Whenever a slot is free, the server takes pending requests in
// arrival order into one micro-batch for as long as their footprint fits:
//   - device memory: the micro-batch's query rows, per-query k and budget,
//     its result rows and its search workspace form one chunk of the
//     server's device arena; the chunk must fit a free gap of the arena,
//     beside the chunks of the micro-batches still in flight;
//   - LDS: each query occupies, while resident on a compute unit, the LDS
//     layout of its budget class; the LDS of all queries in flight stays
//     within `lds_rounds` times the chip's LDS, so a launch is not queued
//     behind more resident rounds than that.
// Requests that arrive while others are on the GPU are admitted as slots and
// memory free up, and their launches overlap on the device.  A query's result
// depends only on (index, query, k, budget, queue length, precision), so it is
// the same alone and in any mix.
//
// Host side only: everything on the device is the library's search.
#include <algorithm>
#include <deque>
#include <memory>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

using namespace ann;

namespace {

struct Request {
    int64_t ticket = 0;
    int32_t nq = 0, k = 0, T = 0;
    int64_t lds = 0;             // LDS while resident (all its queries)
    std::vector<uint8_t> q;      // query rows, copied at submission
    std::vector<int32_t> ids;    // nq x k, filled on completion
    std::vector<uint8_t> dists;  // nq x k x 4
    bool done = false;
};

struct Chunk {
    int64_t off = 0, bytes = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t* h_q = nullptr;      // pinned: slot_queries x row_bytes
    int32_t* h_kt = nullptr;     // pinned: 2 x slot_queries (k, then budget)
    int32_t* h_ids = nullptr;    // pinned: slot_queries x kmax
    uint8_t* h_dists = nullptr;  // pinned: slot_queries x kmax x 4
    bool busy = false;
    int kb = 0;                  // row stride of this launch's results
    Chunk chunk;
    int64_t lds = 0;
    std::vector<Request*> reqs;
};

}  // namespace

struct ann_server {
    const ann_index* idx = nullptr;
    ann_server_params p{};
    int64_t lds_limit = 0;
    uint8_t* arena = nullptr;
    std::vector<Chunk> used;  // chunks of the micro-batches in flight
    std::vector<Slot> slots;
    std::deque<Request*> pending;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    std::vector<int64_t> finished;  // completed tickets not yet reported
    int64_t next_ticket = 1;
    int64_t lds_in_flight = 0;
    int64_t launches = 0;
};

namespace {

// Switches to the index's device for the duration of a call and back.
struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define SERVER_DEVICE(srv)                                                                           \
    DeviceScope scope_((srv)->idx->device);                                                          \
    if (scope_.err != hipSuccess)                                                                    \
        return set_error(ANN_EDEVICE, std::string("server: device switch failed: ") + hipGetErrorString(scope_.err))

int64_t round256(int64_t v) { return (v + 255) & ~int64_t(255); }

// Plans of a micro-batch.  The launch passes per-query k and budgets, so its
// plan splits budget classes; the plan code only tests the budget pointer
// for null, and this stand-in (never read) gets the same split.
const int32_t kPerQueryBudgets = 0;

SearchLaunch launch_of(const ann_server* s, int64_t nq, int k, int T) {
    SearchLaunch a{};
    a.idx = s->idx;
    a.d_T = &kPerQueryBudgets;
    a.nq = nq;
    a.kmax = k;
    a.Tmax = T;
    a.L = s->p.search.queue_len;
    a.precision = s->idx->dtype == ANN_F32 ? s->p.search.precision : ANN_PRECISION_EXACT;
    a.rerank_k = s->p.search.rerank_k;
    a.lookahead = s->p.search.lookahead;
    a.persistent = s->p.search.persistent;
    a.waves_per_cu = s->p.search.waves_per_cu;
    a.order = s->p.search.order;
    return a;
}

// budget class bound a query of budget T is laid out for inside a launch
int class_budget(const ann_server* s, int T) {
    if (T <= 512) return 512;
    if (T <= 2048) return 2048;
    return T <= 4096 ? std::min(4096, s->p.max_budget) : s->p.max_budget;
}

// device bytes of a micro-batch: query rows, k and budget, results, workspace
int batch_bytes(const ann_server* s, int64_t nq, int kb, int Tb, int64_t* bytes) {
    int64_t ws = 0;
    int rc = search_workspace_bytes(launch_of(s, nq, kb, Tb), &ws);
    if (rc) return rc;
    int64_t ws_min = 0;
    if ((rc = search_workspace_bytes(launch_of(s, nq, kb, Tb), &ws_min, true))) return rc;
    // global multi-sequence slots beyond 64 MiB are not taken: queries that
    // find none free are searched again, with the same results
    ws = std::max(ws_min, std::min<int64_t>(ws, int64_t(64) << 20));
    *bytes = round256(nq * s->idx->row_bytes) + round256(nq * 8) + 2 * round256(nq * kb * 4) + round256(ws);
    return ANN_OK;
}

// first gap of the arena that holds `bytes`, or -1
int64_t find_gap(const ann_server* s, int64_t bytes) {
    std::vector<Chunk> u = s->used;
    std::sort(u.begin(), u.end(), [](const Chunk& a, const Chunk& b) { return a.off < b.off; });
    int64_t at = 0;
    for (const Chunk& c : u) {
        if (c.off - at >= bytes) return at;
        at = c.off + c.bytes;
    }
    return s->p.device_bytes - at >= bytes ? at : -1;
}

int retire(ann_server* s) {
    for (Slot& sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return set_error(ANN_EDEVICE, std::string("server: launch failed: ") + hipGetErrorString(q));
        int64_t row = 0;
        for (Request* r : sl.reqs) {
            r->ids.resize(size_t(r->nq) * r->k);
            r->dists.resize(size_t(r->nq) * r->k * 4);
            for (int32_t i = 0; i < r->nq; ++i, ++row) {
                std::copy_n(sl.h_ids + row * sl.kb, r->k, r->ids.data() + size_t(i) * r->k);
                std::copy_n(sl.h_dists + row * sl.kb * 4, size_t(r->k) * 4, r->dists.data() + size_t(i) * r->k * 4);
            }
            r->done = true;
            std::vector<uint8_t>().swap(r->q);
            s->finished.push_back(r->ticket);
        }
        sl.reqs.clear();
        s->lds_in_flight -= sl.lds;
        for (size_t i = 0; i < s->used.size(); ++i)
            if (s->used[i].off == sl.chunk.off) {
                s->used.erase(s->used.begin() + i);
                break;
            }
        sl.busy = false;
    }
    return ANN_OK;
}

int admit(ann_server* s) {
    for (Slot& sl : s->slots) {
        if (s->pending.empty()) return ANN_OK;
        if (sl.busy) continue;
        // take pending requests in arrival order while the micro-batch fits
        std::vector<Request*> take;
        int64_t nq = 0, lds = 0, off = -1, bytes = 0;
        int kb = 1, Tb = 0;
        for (Request* r : s->pending) {
            const int64_t nq2 = nq + r->nq;
            const int kb2 = std::max(kb, r->k), Tb2 = std::max(Tb, r->T);
            if (nq2 > s->p.slot_queries) break;
            if (s->lds_in_flight + lds + r->lds > s->lds_limit) break;
            int64_t b = 0;
            int rc = batch_bytes(s, nq2, kb2, Tb2, &b);
            if (rc) return rc;
            const int64_t at = find_gap(s, b);
            if (at < 0) break;
            take.push_back(r);
            nq = nq2;
            kb = kb2;
            Tb = Tb2;
            lds += r->lds;
            off = at;
            bytes = b;
        }
        if (take.empty()) return ANN_OK;  // the head request waits for memory to free up
        s->pending.erase(s->pending.begin(), s->pending.begin() + int64_t(take.size()));
        // stage the queries, k and budget of every query
        int64_t row = 0;
        for (Request* r : take) {
            std::copy(r->q.begin(), r->q.end(), sl.h_q + row * s->idx->row_bytes);
            std::fill_n(sl.h_kt + row, r->nq, r->k);
            std::fill_n(sl.h_kt + s->p.slot_queries + row, r->nq, r->T);
            row += r->nq;
        }
        uint8_t* base = s->arena + off;
        uint8_t* d_q = base;
        int32_t* d_kt = reinterpret_cast<int32_t*>(base + round256(nq * s->idx->row_bytes));
        int32_t* d_ids = reinterpret_cast<int32_t*>(reinterpret_cast<uint8_t*>(d_kt) + round256(nq * 8));
        uint8_t* d_dists = reinterpret_cast<uint8_t*>(d_ids) + round256(nq * kb * 4);
        uint8_t* d_ws = d_dists + round256(nq * kb * 4);
        const int64_t ws_bytes = bytes - (d_ws - base);
        ANN_HIP_CHECK(hipMemcpyAsync(d_q, sl.h_q, size_t(nq * s->idx->row_bytes), hipMemcpyHostToDevice, sl.stream));
        ANN_HIP_CHECK(hipMemcpyAsync(d_kt, sl.h_kt, size_t(nq) * 4, hipMemcpyHostToDevice, sl.stream));
        ANN_HIP_CHECK(hipMemcpyAsync(d_kt + nq, sl.h_kt + s->p.slot_queries, size_t(nq) * 4, hipMemcpyHostToDevice,
                                     sl.stream));
        int rc = ann_search_device_ws(s->idx, d_q, nq, kb, Tb, d_kt, d_kt + nq, &s->p.search, d_ids, d_dists, nullptr,
                                      nullptr, d_ws, ws_bytes, sl.stream);
        if (rc) return rc;
        ANN_HIP_CHECK(hipMemcpyAsync(sl.h_ids, d_ids, size_t(nq * kb) * 4, hipMemcpyDeviceToHost, sl.stream));
        ANN_HIP_CHECK(hipMemcpyAsync(sl.h_dists, d_dists, size_t(nq * kb) * 4, hipMemcpyDeviceToHost, sl.stream));
        ANN_HIP_CHECK(hipEventRecord(sl.done, sl.stream));
        sl.busy = true;
        sl.kb = kb;
        sl.chunk = Chunk{off, bytes};
        sl.lds = lds;
        sl.reqs = take;
        s->used.push_back(sl.chunk);
        s->lds_in_flight += lds;
        ++s->launches;
    }
    return ANN_OK;
}

void release(ann_server* s) {
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_q) (void)hipHostFree(sl.h_q);
        if (sl.h_kt) (void)hipHostFree(sl.h_kt);
        if (sl.h_ids) (void)hipHostFree(sl.h_ids);
        if (sl.h_dists) (void)hipHostFree(sl.h_dists);
    }
    if (s->arena) (void)hipFree(s->arena);
}

}  // namespace

extern "C" {

int ann_server_create(const ann_index* idx, const ann_server_params* params, ann_server** out) {
    ANN_REQUIRE(idx && params && out, "ann_server_create: null argument");
    ANN_REQUIRE(params->struct_size == sizeof(ann_server_params), "ann_server_params.struct_size mismatch");
    const ann_server_params& p = *params;
    ANN_REQUIRE(p.slots >= 1 && p.slots <= 16, "server: slots must be in [1, 16]");
    ANN_REQUIRE(p.slot_queries >= 1 && p.slot_queries <= (1 << 20), "server: slot_queries must be in [1, 2^20]");
    ANN_REQUIRE(p.kmax >= 1 && p.kmax <= 1024, "server: kmax must be in [1, 1024]");
    ANN_REQUIRE(p.max_budget >= 0 && p.max_budget <= (1 << 20), "server: max_budget must be in [0, 2^20]");
    ANN_REQUIRE(p.lds_rounds >= 0, "server: lds_rounds must be >= 0");
    ANN_REQUIRE(p.device_bytes >= 0, "server: device_bytes must be >= 0");
    ANN_REQUIRE(p.search.struct_size == sizeof(ann_search_params), "server: search params of the current version");
    ANN_REQUIRE(p.search.queue_len >= 1 && p.search.queue_len <= 64, "server: queue_len must be in [1, 64]");
    auto s = std::make_unique<ann_server>();
    s->idx = idx;
    s->p = p;
    if (s->p.lds_rounds == 0) s->p.lds_rounds = 2;
    DeviceScope scope(idx->device);
    if (scope.err != hipSuccess) return set_error(ANN_EDEVICE, "server: device switch failed");
    int cus = 0, lds_cu = 0;
    ANN_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, idx->device));
    ANN_HIP_CHECK(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, idx->device));
    s->lds_limit = int64_t(cus) * lds_cu * s->p.lds_rounds;
    // the largest single micro-batch must fit: a full slot at the largest k and budget
    int64_t full = 0;
    int rc = batch_bytes(s.get(), p.slot_queries, p.kmax, p.max_budget, &full);
    if (rc) return rc;
    if (s->p.device_bytes == 0) s->p.device_bytes = full * p.slots;
    ANN_REQUIRE(s->p.device_bytes >= full, "server: device_bytes (" + std::to_string(s->p.device_bytes) +
                                               ") below one full slot (" + std::to_string(full) + ")");
    int64_t lds_one = 0;
    if ((rc = search_lds_per_query(launch_of(s.get(), 1, p.kmax, p.max_budget), &lds_one))) return rc;
    ANN_REQUIRE(lds_one <= s->lds_limit, "server: one query at max_budget needs more LDS than the chip holds");
    struct Undo {
        ann_server* s;
        ~Undo() {
            if (s) release(s);
        }
    } undo{s.get()};
    ANN_HIP_CHECK(hipMalloc(reinterpret_cast<void**>(&s->arena), size_t(s->p.device_bytes)));
    s->slots.resize(size_t(p.slots));
    for (Slot& sl : s->slots) {
        ANN_HIP_CHECK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
        ANN_HIP_CHECK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        ANN_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&sl.h_q), size_t(p.slot_queries) * idx->row_bytes));
        ANN_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&sl.h_kt), size_t(p.slot_queries) * 8));
        ANN_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&sl.h_ids), size_t(p.slot_queries) * p.kmax * 4));
        ANN_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&sl.h_dists), size_t(p.slot_queries) * p.kmax * 4));
    }
    undo.s = nullptr;
    *out = s.release();
    return ANN_OK;
}

int ann_server_footprint(const ann_server* s, int32_t nq, int32_t k, int32_t budget, int64_t* lds_bytes,
                         int64_t* device_bytes) {
    ANN_REQUIRE(s && nq >= 1 && k >= 1 && budget >= 0, "ann_server_footprint: bad argument");
    ANN_REQUIRE(k <= s->p.kmax && budget <= s->p.max_budget, "ann_server_footprint: k or budget above the server's");
    SERVER_DEVICE(s);
    int64_t per = 0;
    int rc = search_lds_per_query(launch_of(s, 1, k, class_budget(s, budget)), &per);
    if (rc) return rc;
    if (lds_bytes) *lds_bytes = per * nq;
    int64_t b = 0;
    if ((rc = batch_bytes(s, nq, k, budget, &b))) return rc;
    if (device_bytes) *device_bytes = b;
    return ANN_OK;
}

int ann_server_submit(ann_server* s, const void* queries, int32_t nq, int32_t k, int32_t budget, int64_t* ticket) {
    ANN_REQUIRE(s && queries && ticket, "ann_server_submit: null argument");
    ANN_REQUIRE(nq >= 1 && nq <= s->p.slot_queries,
                "ann_server_submit: a request holds 1.." + std::to_string(s->p.slot_queries) + " queries");
    ANN_REQUIRE(k >= 1 && k <= s->p.kmax, "ann_server_submit: k above the server's kmax");
    ANN_REQUIRE(budget >= 0 && budget <= s->p.max_budget, "ann_server_submit: budget above the server's max_budget");
    SERVER_DEVICE(s);
    auto r = std::make_unique<Request>();
    r->ticket = s->next_ticket++;
    r->nq = nq;
    r->k = k;
    r->T = budget;
    int64_t per = 0;
    int rc = search_lds_per_query(launch_of(s, 1, k, class_budget(s, budget)), &per);
    if (rc) return rc;
    r->lds = per * nq;
    ANN_REQUIRE(r->lds <= s->lds_limit, "ann_server_submit: the request's LDS footprint (" + std::to_string(r->lds) +
                                            " bytes) exceeds what the server admits at once (" +
                                            std::to_string(s->lds_limit) + ")");
    const uint8_t* src = static_cast<const uint8_t*>(queries);
    r->q.assign(src, src + size_t(nq) * s->idx->row_bytes);
    s->pending.push_back(r.get());
    *ticket = r->ticket;
    s->reqs.emplace(r->ticket, std::move(r));
    return admit(s);
}

int ann_server_progress(ann_server* s, int64_t* done, int32_t cap, int32_t* n_done) {
    ANN_REQUIRE(s && n_done && (cap == 0 || done) && cap >= 0, "ann_server_progress: bad argument");
    SERVER_DEVICE(s);
    int rc = retire(s);
    if (rc) return rc;
    if ((rc = admit(s))) return rc;
    const int32_t m = int32_t(std::min<size_t>(size_t(cap), s->finished.size()));
    std::copy_n(s->finished.begin(), m, done);
    s->finished.erase(s->finished.begin(), s->finished.begin() + m);
    *n_done = m;
    return ANN_OK;
}

int ann_server_result(ann_server* s, int64_t ticket, int32_t* ids, void* dists) {
    ANN_REQUIRE(s && ids && dists, "ann_server_result: null argument");
    auto it = s->reqs.find(ticket);
    ANN_REQUIRE(it != s->reqs.end(), "ann_server_result: unknown ticket " + std::to_string(ticket));
    if (!it->second->done) return set_error(ANN_ESTATE, "ann_server_result: request not completed yet");
    Request& r = *it->second;
    std::copy(r.ids.begin(), r.ids.end(), ids);
    std::copy(r.dists.begin(), r.dists.end(), static_cast<uint8_t*>(dists));
    s->reqs.erase(it);
    return ANN_OK;
}

int ann_server_drain(ann_server* s) {
    ANN_REQUIRE(s, "ann_server_drain: null server");
    SERVER_DEVICE(s);
    for (;;) {
        int rc = retire(s);
        if (rc) return rc;
        if ((rc = admit(s))) return rc;
        bool busy = false;
        for (Slot& sl : s->slots) busy = busy || sl.busy;
        if (!busy && s->pending.empty()) return ANN_OK;
        for (Slot& sl : s->slots)
            if (sl.busy) {
                ANN_HIP_CHECK(hipEventSynchronize(sl.done));
                break;
            }
    }
}

int ann_server_get_info(const ann_server* s, ann_server_info* info) {
    ANN_REQUIRE(s && info, "ann_server_get_info: null argument");
    info->pending = int64_t(s->pending.size());
    int64_t busy = 0;
    for (const Slot& sl : s->slots) busy += sl.busy ? 1 : 0;
    info->busy_slots = busy;
    info->launches = s->launches;
    info->lds_in_flight = s->lds_in_flight;
    info->lds_limit = s->lds_limit;
    int64_t dev = 0;
    for (const Chunk& c : s->used) dev += c.bytes;
    info->device_in_flight = dev;
    info->device_bytes = s->p.device_bytes;
    return ANN_OK;
}

void ann_server_destroy(ann_server* s) {
    if (!s) return;
    DeviceScope scope(s->idx->device);
    release(s);
    delete s;
}

}  // extern "C"
