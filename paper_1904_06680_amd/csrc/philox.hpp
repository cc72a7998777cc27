// Philox4x32-10 counter-based generator (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
// "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11), device side, and the map from one
// 32-bit word to a controller parameter.
//
// The planner's parameter vectors theta (Sect. II-E, Step 5: theta and the random seed are what
// the host hands to the GPU each sampling time) are drawn from this generator so that every
// sample's parameters are a pure function of (seed, inst, sample, parameter index) and can be
// regenerated anywhere without storing them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnp {

struct PhiloxKey {
    uint32_t k0, k1;
};

// Ten rounds; each round multiplies counter words 0 and 2 by the Philox constants, mixes the
// high halves with words 1, 3 and the round key, and the key advances by the Weyl increments
// between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, PhiloxKey key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// theta = (2m + 1 - 2^24) * 2^-24 with m the top 24 bits: an odd multiple of 2^-24 in (-1, 1),
// exactly representable in float, uniform on (-1, 1).
__device__ __forceinline__ float theta_from_word(uint32_t w)
{
    const int m = (int)(w >> 8);
    return (float)(2 * m + 1 - 16777216) * 5.9604644775390625e-8f;
}

__device__ __forceinline__ uint32_t word_of(uint4 w, int j)
{
    return j == 0 ? w.x : j == 1 ? w.y : j == 2 ? w.z : w.w;
}

// Counter layout: (k / 4, sample, stream, inst); stream 0 is the uniform parameter draw.
struct ThetaSource {
    const float *explicit_theta;   // row of this sample in an explicit [N][n_theta] array, or null
    PhiloxKey key;
    uint32_t sample, inst;

    __device__ __forceinline__ uint4 block4(int c) const
    {
        return philox4x32_10(make_uint4((uint32_t)c, sample, 0u, inst), key);
    }

    // dst[e] = theta[base + e] for a base that is a multiple of 4. Long slices are generated
    // in chunks of STAGE values through a per-lane LDS staging area (stage[e * BLOCK + tid]) so
    // that the Philox loop can stay rolled while every register of dst is written with a
    // compile-time index.
    static constexpr int STAGE = 32;

    template <int COUNT>
    __device__ __forceinline__ void fill_aligned(float (&dst)[COUNT], int base, float *stage,
                                                 int tid, int block) const
    {
        if (explicit_theta) {
#pragma unroll
            for (int e = 0; e < COUNT; ++e) dst[e] = explicit_theta[base + e];
            return;
        }
        if constexpr (COUNT <= STAGE) {
#pragma unroll
            for (int c = 0; c < (COUNT + 3) / 4; ++c) {
                const uint4 w = block4((base >> 2) + c);
                if (4 * c + 0 < COUNT) dst[4 * c + 0] = theta_from_word(w.x);
                if (4 * c + 1 < COUNT) dst[4 * c + 1] = theta_from_word(w.y);
                if (4 * c + 2 < COUNT) dst[4 * c + 2] = theta_from_word(w.z);
                if (4 * c + 3 < COUNT) dst[4 * c + 3] = theta_from_word(w.w);
            }
        } else {
            static_assert(COUNT % 4 == 0, "aligned slices come in whole Philox blocks");
            constexpr int NCH = (COUNT + STAGE - 1) / STAGE;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int len = ch + 1 < NCH ? STAGE : COUNT - (NCH - 1) * STAGE;
#pragma unroll 1
                for (int c = 0; c < len / 4; ++c) {
                    const uint4 w = block4((base >> 2) + ch * (STAGE / 4) + c);
                    stage[(4 * c + 0) * block + tid] = theta_from_word(w.x);
                    stage[(4 * c + 1) * block + tid] = theta_from_word(w.y);
                    stage[(4 * c + 2) * block + tid] = theta_from_word(w.z);
                    stage[(4 * c + 3) * block + tid] = theta_from_word(w.w);
                }
#pragma unroll
                for (int e = 0; e < STAGE; ++e)
                    if (ch * STAGE + e < COUNT) dst[ch * STAGE + e] = stage[e * block + tid];
            }
        }
    }

    // dst[e] = theta[base + e] for a short slice (COUNT even) whose base is even: its pairs never
    // straddle a Philox block.
    template <int COUNT>
    __device__ __forceinline__ void fill_even(float (&dst)[COUNT], int base) const
    {
        static_assert(COUNT % 2 == 0, "pairs of parameters");
        if (explicit_theta) {
#pragma unroll
            for (int e = 0; e < COUNT; ++e) dst[e] = explicit_theta[base + e];
            return;
        }
#pragma unroll
        for (int e = 0; e < COUNT; e += 2) {
            const int k = base + e;
            const uint4 w = block4(k >> 2);
            const bool hi = (k & 2) != 0;
            dst[e] = theta_from_word(hi ? w.z : w.x);
            dst[e + 1] = theta_from_word(hi ? w.w : w.y);
        }
    }

    // dst[e] = theta[BASE + e] for a compile-time base of any alignment.
    template <int BASE, int COUNT>
    __device__ __forceinline__ void fill_const(float (&dst)[COUNT]) const
    {
        if (explicit_theta) {
#pragma unroll
            for (int e = 0; e < COUNT; ++e) dst[e] = explicit_theta[BASE + e];
            return;
        }
        constexpr int c0 = BASE >> 2, c1 = (BASE + COUNT - 1) >> 2;
#pragma unroll
        for (int c = c0; c <= c1; ++c) {
            const uint4 w = block4(c);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = 4 * c + j - BASE;
                if (e >= 0 && e < COUNT) dst[e] = theta_from_word(word_of(w, j));
            }
        }
    }

    // theta[k] for any k.
    __device__ __forceinline__ float one(int k) const
    {
        if (explicit_theta) return explicit_theta[k];
        return theta_from_word(word_of(block4(k >> 2), k & 3));
    }
};

}  // namespace nnp
