// Shared device and host helpers of the HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ann.h"

namespace ann {

constexpr int WAVE = 64;
constexpr uint64_t KEY_EMPTY = ~0ull;
constexpr uint32_t ID_EMPTY = 0xFFFFFFFFu;

// ---------------------------------------------------------------------
// Errors: a thread-local message plus a status code.
// ---------------------------------------------------------------------
int set_error(int status, const std::string& msg);

#define ANN_HIP_CHECK(expr)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::ann::set_error(ANN_EDEVICE, std::string(#expr " failed: ") +            \
                                                     hipGetErrorString(e_));                 \
    } while (0)

#define ANN_REQUIRE(cond, msg)                                                               \
    do {                                                                                     \
        if (!(cond)) return ::ann::set_error(ANN_EINVAL, (msg));                             \
    } while (0)

// ---------------------------------------------------------------------
// (distance, id) keys packed in 64 bits.  Squared distances are
// non-negative: int32 values and float bit patterns both order like
// unsigned 32-bit integers, so (bits << 32 | id) orders as (distance, id).
// ---------------------------------------------------------------------
__host__ __device__ inline uint64_t make_key(uint32_t dist_bits, uint32_t id) {
    return (uint64_t(dist_bits) << 32) | id;
}
__host__ __device__ inline uint32_t key_dist(uint64_t k) { return uint32_t(k >> 32); }
__host__ __device__ inline uint32_t key_id(uint64_t k) { return uint32_t(k); }

__device__ inline float bits_f(uint32_t b) { return __uint_as_float(b); }
__device__ inline uint32_t f_bits(float f) { return __float_as_uint(f); }

// ---------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

// number of set bits of `mask` below this lane
// Order LDS accesses of one wavefront around a cross-lane exchange through
// LDS.  A wavefront's LDS instructions execute in issue order, so it only has
// to keep the compiler from moving memory operations across this point; it
// does not wait for outstanding global loads (a fence would).
__device__ inline void lds_wave_order() {
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

__device__ inline int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0));
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = __shfl_xor(uint32_t(v), m);
    uint32_t hi = __shfl_xor(uint32_t(v >> 32), m);
    return (uint64_t(hi) << 32) | lo;
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl(uint32_t(v), src);
    uint32_t hi = __shfl(uint32_t(v >> 32), src);
    return (uint64_t(hi) << 32) | lo;
}

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
        uint64_t o = shfl_xor_u64(v, m);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------
// bf16 helpers (round to nearest even; inputs are finite)
// ---------------------------------------------------------------------
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return uint16_t(u >> 16);
}

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace ann
