// Device code shared by the search and the bridge-graph build: subspace
// distance tables with their per-subspace sort (Sec. 4.2) and the
// multi-sequence frontier (Sec. 3.3), a binary min-heap of bridge keys.
#pragma once

#include "common.hpp"

namespace ann {

// ------------------------------------------------------------------
// query tables (Sec. 4.2): tab[p*K + j] = |q^p - c_pj|^2, then per
// subspace the ranks by (value, j): sv[p*K + r] value, perm[p*K + r] = j
// ------------------------------------------------------------------
template <bool FLOAT>
__device__ inline void compute_tables(const uint8_t* qv, const void* cb, int P, int K, int ds, uint32_t* tab, uint32_t* sv,
                               uint8_t* perm, int lane) {
    const int PK = P * K;
    for (int e = lane; e < PK; e += WAVE) {
        const int p = e / K;
        if constexpr (!FLOAT) {
            const uint8_t* c = static_cast<const uint8_t*>(cb) + int64_t(e) * ds;
            const uint8_t* q = qv + p * ds;
            uint32_t acc = 0;
            for (int i = 0; i < ds; ++i) {
                int t = int(q[i]) - int(c[i]);
                acc += uint32_t(t * t);
            }
            tab[e] = acc;
        } else {
            const float* c = static_cast<const float*>(cb) + int64_t(e) * ds;
            const float* q = reinterpret_cast<const float*>(qv) + p * ds;
            float acc = 0.f;
            for (int i = 0; i < ds; ++i) {
                float t = q[i] - c[i];
                acc = fmaf(t, t, acc);
            }
            tab[e] = f_bits(acc);
        }
    }
    __syncthreads();
    for (int e = lane; e < PK; e += WAVE) {
        const int p = e / K, j = e - p * K;
        const uint64_t mine = make_key(tab[e], uint32_t(j));
        int r = 0;
        for (int jj = 0; jj < K; ++jj) r += make_key(tab[p * K + jj], uint32_t(jj)) < mine;
        sv[p * K + r] = tab[e];
        perm[p * K + r] = uint8_t(j);
    }
    __syncthreads();
}

// ------------------------------------------------------------------
// multi-sequence frontier: binary min-heap of (sum << 32 | n + lid) keys
// with the packed rank tuple (8 bits per subspace) alongside
// ------------------------------------------------------------------
template <bool FLOAT>
__device__ inline uint64_t tuple_key(uint32_t rk, const uint32_t* sv, const uint8_t* perm, int P, int K, int64_t n) {
    uint32_t s = 0;
    float fs = 0.f;
    uint32_t lid = 0;
    for (int p = 0; p < P; ++p) {
        const int r = (rk >> (8 * p)) & 0xFF;
        const uint32_t v = sv[p * K + r];
        if constexpr (FLOAT)
            fs = (p == 0) ? bits_f(v) : fs + bits_f(v);
        else
            s += v;
        lid = lid * uint32_t(K) + perm[p * K + r];
    }
    return make_key(FLOAT ? f_bits(fs) : s, uint32_t(n) + lid);
}

__device__ inline void heap_push(uint64_t* hk, uint32_t* hr, int& hn, uint64_t key, uint32_t rk) {
    int i = hn++;
    while (i > 0) {
        const int par = (i - 1) >> 1;
        const uint64_t pk = hk[par];
        if (pk <= key) break;
        hk[i] = pk;
        hr[i] = hr[par];
        i = par;
    }
    hk[i] = key;
    hr[i] = rk;
}

__device__ inline void heap_pop(uint64_t* hk, uint32_t* hr, int& hn, uint64_t& key, uint32_t& rk) {
    key = hk[0];
    rk = hr[0];
    --hn;
    const uint64_t lk = hk[hn];
    const uint32_t lr = hr[hn];
    int i = 0;
    for (;;) {
        int c = 2 * i + 1;
        if (c >= hn) break;
        uint64_t ck = hk[c];
        if (c + 1 < hn) {
            const uint64_t ck2 = hk[c + 1];
            if (ck2 < ck) {
                ck = ck2;
                ++c;
            }
        }
        if (lk <= ck) break;
        hk[i] = ck;
        hr[i] = hr[c];
        i = c;
    }
    hk[i] = lk;
    hr[i] = lr;
}

}  // namespace ann
