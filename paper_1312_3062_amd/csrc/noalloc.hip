// Search that allocates nothing: its workspace is a buffer compiled into the
// library, one copy per GPU.
//
// The array below exists once on every device the library's code object is
// loaded on, from load until the process ends.  In host code its name is only
// a stand-in symbol, not a device address: the address a kernel may use is the
// one hipGetSymbolAddress returns with that device current, looked up once per
// device and kept.  Every call on a device shares that device's copy, and the
// copy keeps the last call's contents; the launch clears what must start at
// zero (its counters and slot bitmap) with a kernel of its own.  Calls that
// overlap in time on one device race on the buffer.
#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(ANN_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of its alignment");

__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

int scratch_address(void** out) {
    int dev = 0;
    ANN_HIP_CHECK(hipGetDevice(&dev));
    ANN_REQUIRE(dev >= 0 && dev < kMaxDevices, "ann_search_device_noalloc: device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        ANN_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        ANN_REQUIRE(p != nullptr && (reinterpret_cast<uintptr_t>(p) & 255) == 0,
                    "ann_search_device_noalloc: scratch symbol has no aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ANN_OK;
}

}  // namespace

extern "C" int ann_search_device_noalloc(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k,
                                         int32_t budget, const int32_t* d_k, const int32_t* d_budget,
                                         const ann_search_params* sp, int32_t* d_ids, void* d_dists,
                                         int32_t* d_stats, int32_t* d_trace, void* stream) {
    if (nq == 0) return ann_search_device(idx, d_queries, nq, k, budget, d_k, d_budget, sp, d_ids, d_dists, d_stats,
                                          d_trace, stream);
    int64_t need = 0;
    int rc = ann::search_min_workspace(idx, nq, k, budget, sp, &need);
    if (rc) return rc;
    if (need > int64_t(kScratchBytes))
        return ann::set_error(ANN_EINVAL, "ann_search_device_noalloc: the request needs " + std::to_string(need) +
                                              " bytes of workspace, more than the library's fixed " +
                                              std::to_string(kScratchBytes) + " (search fewer queries per call)");
    void* ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    return ann_search_device_ws(idx, d_queries, nq, k, budget, d_k, d_budget, sp, d_ids, d_dists, d_stats, d_trace,
                                ws, int64_t(kScratchBytes), stream);
}
