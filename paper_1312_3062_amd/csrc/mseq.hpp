// Device code shared by the search and the bridge-graph build: subspace
// distance tables with their per-subspace sort (Sec. 4.2) and the
// multi-sequence frontier (Sec. 3.3), a 4-ary min-heap of bridge keys.
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
            // u8 subvectors are a multiple of 4 bytes (d % 16 == 0, P <= 4):
            // |q - c|^2 = q.q + c.c - 2 q.c by 4-byte dot products, exact
            const uint32_t* c = reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(cb) + int64_t(e) * ds);
            const uint32_t* q = reinterpret_cast<const uint32_t*>(qv + p * ds);
            uint32_t qq = 0, cc = 0, qc = 0;
            for (int i = 0; i < ds / 4; ++i) {
                const uint32_t qw = q[i], cw = c[i];
                qq = __builtin_amdgcn_udot4(qw, qw, qq, false);
                cc = __builtin_amdgcn_udot4(cw, cw, cc, false);
                qc = __builtin_amdgcn_udot4(qw, cw, qc, false);
            }
            tab[e] = qq + cc - 2u * qc;
        } else {
            const float* c = static_cast<const float*>(cb) + int64_t(e) * ds;
            const float* q = reinterpret_cast<const float*>(qv) + p * ds;
            float acc = 0.f;
            int i = 0;
            if (ds % 4 == 0) {
                // 16-byte loads, the same order of operations as one at a time
                for (; i < ds; i += 4) {
                    const float4 cv = *reinterpret_cast<const float4*>(c + i);
                    const float4 qv4 = *reinterpret_cast<const float4*>(q + i);
                    float t = qv4.x - cv.x;
                    acc = fmaf(t, t, acc);
                    t = qv4.y - cv.y;
                    acc = fmaf(t, t, acc);
                    t = qv4.z - cv.z;
                    acc = fmaf(t, t, acc);
                    t = qv4.w - cv.w;
                    acc = fmaf(t, t, acc);
                }
            }
            for (; i < ds; ++i) {
                const float t = q[i] - c[i];
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
// multi-sequence frontier: min-heap of (sum << 32 | n + lid) keys with the
// packed rank tuple (8 bits per subspace) alongside
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

// A frontier entry: key (low, high word) and packed ranks side by side in
// one 16-byte vector, so that one access moves both.
typedef uint32_t hent_t __attribute__((ext_vector_type(4)));
__device__ inline uint64_t hkey(hent_t e) { return (uint64_t(e.y) << 32) | e.x; }
__device__ inline hent_t hmake(uint64_t key, uint32_t rk) {
    hent_t e;
    e.x = uint32_t(key);
    e.y = uint32_t(key >> 32);
    e.z = rk;
    e.w = 0u;
    return e;
}

// 4-ary min-heap: half the levels of a binary heap, and the four children of
// a node are read together, so a level costs one memory round trip.  Keys
// are distinct, so the order of extraction is the keys' order whatever the
// heap's shape.  HP is a pointer to hent_t in any address space (LDS, global
// or generic).
template <typename HP>
__device__ inline void heap_push(HP h, int& hn, uint64_t key, uint32_t rk) {
    int i = hn++;
    while (i > 0) {
        const int par = (i - 1) >> 2;
        const hent_t pe = h[par];
        if (hkey(pe) <= key) break;
        h[i] = pe;
        i = par;
    }
    h[i] = hmake(key, rk);
}

template <typename HP>
__device__ inline void heap_pop(HP h, int& hn, uint64_t& key, uint32_t& rk) {
    const hent_t top = h[0];
    key = hkey(top);
    rk = top.z;
    --hn;
    const hent_t last = h[hn];
    const uint64_t lk = hkey(last);
    int i = 0;
    for (;;) {
        const int c = 4 * i + 1;
        if (c >= hn) break;
        // children past the end are read at a valid index and ignored; the
        // ranks are read with the keys (one round trip), not after the choice
        hent_t e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = h[min(c + q, hn - 1)];
        asm volatile("" ::"v"(e[0].z), "v"(e[1].z), "v"(e[2].z), "v"(e[3].z));
        int bc = c;
        hent_t b = e[0];
#pragma unroll
        for (int q = 1; q < 4; ++q)
            if (c + q < hn && hkey(e[q]) < hkey(b)) {
                b = e[q];
                bc = c + q;
            }
        if (lk <= hkey(b)) break;
        h[i] = b;
        i = bc;
    }
    h[i] = last;
}

// Replace the smallest entry by (key, rk) and restore the order: one
// sift-down from the root.  Taking the smallest key and inserting its
// successor this way costs one pass that stops where the successor belongs,
// where a pop and a push cost a pass that sinks the last entry to the bottom
// and a second pass up.
template <typename HP>
__device__ inline void heap_replace_top(HP h, int hn, uint64_t key, uint32_t rk) {
    int i = 0;
    for (;;) {
        const int c = 4 * i + 1;
        if (c >= hn) break;
        hent_t e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = h[min(c + q, hn - 1)];
        asm volatile("" ::"v"(e[0].z), "v"(e[1].z), "v"(e[2].z), "v"(e[3].z));
        int bc = c;
        hent_t b = e[0];
#pragma unroll
        for (int q = 1; q < 4; ++q)
            if (c + q < hn && hkey(e[q]) < hkey(b)) {
                b = e[q];
                bc = c + q;
            }
        if (key <= hkey(b)) break;
        h[i] = b;
        i = bc;
    }
    h[i] = hmake(key, rk);
}

}  // namespace ann
