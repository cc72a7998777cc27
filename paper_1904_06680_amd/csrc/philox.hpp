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

// Standard normal pair from two Philox words by the Box-Muller transform (G. E. P. Box and
// M. E. Muller, 1958): u = (m + 1/2) 2^-23 with m the top 23 bits of a word, so u and 2u are exact
// floats in (0, 1) and (0, 2); z0 = sqrt(-2 ln u_a) cos(2 pi u_b), z1 = the sine.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float &z0, float &z1)
{
    const float ua = (float)(2 * (int)(wa >> 9) + 1) * 5.9604644775390625e-8f;     // 2^-24
    const float two_ub = (float)(2 * (int)(wb >> 9) + 1) * 1.1920928955078125e-7f;  // 2^-23
    const float r = sqrtf(-2.0f * logf(ua));
    float sn, cs;
    sincospif(two_ub, &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
}

// Counter layout: (k / 4, sample, stream, inst). Stream 0 is the uniform parameter draw; stream 1
// the Gaussian proposal theta_k = mu_k + exp(s_k) z_k, whose normals come from block k / 4: words
// (0, 1) for k mod 4 in {0, 1}, words (2, 3) for {2, 3}, cosine for even k, sine for odd k.
struct ThetaSource {
    const float *explicit_theta;   // row of this sample in an explicit [N][n_theta] array, or null
    const float *mu, *log_sigma;   // Gaussian proposal of this sample's problem, or null (uniform)
    int n_theta;                   // length of mu / log_sigma
    PhiloxKey key;
    uint32_t sample, inst;         // Philox sample word (index within the sample's own stream)

    __device__ __forceinline__ uint4 block4(int c, uint32_t stream) const
    {
        return philox4x32_10(make_uint4((uint32_t)c, sample, stream, inst), key);
    }

    __device__ __forceinline__ float gauss(int k, float z) const
    {
        return k < n_theta ? fmaf(expf(log_sigma[k]), z, mu[k]) : 0.0f;
    }

    // theta[k], theta[k + 1] for even k.
    __device__ __forceinline__ float2 pair(int k) const
    {
        if (!mu) {
            const uint4 w = block4(k >> 2, 0u);
            return (k & 2) ? make_float2(theta_from_word(w.z), theta_from_word(w.w))
                           : make_float2(theta_from_word(w.x), theta_from_word(w.y));
        }
        const uint4 w = block4(k >> 2, 1u);
        float z0, z1;
        if (k & 2) box_muller(w.z, w.w, z0, z1);
        else box_muller(w.x, w.y, z0, z1);
        return make_float2(gauss(k, z0), gauss(k + 1, z1));
    }

    // theta[4c .. 4c + 3].
    __device__ __forceinline__ float4 value4(int c) const
    {
        if (!mu) {
            const uint4 w = block4(c, 0u);
            return make_float4(theta_from_word(w.x), theta_from_word(w.y), theta_from_word(w.z),
                               theta_from_word(w.w));
        }
        const uint4 w = block4(c, 1u);
        float z0, z1, z2, z3;
        box_muller(w.x, w.y, z0, z1);
        box_muller(w.z, w.w, z2, z3);
        return make_float4(gauss(4 * c, z0), gauss(4 * c + 1, z1), gauss(4 * c + 2, z2),
                           gauss(4 * c + 3, z3));
    }

    // dst[e] = theta[base + e] for a base that is a multiple of 4. Long slices are generated
    // in chunks of STAGE values through a per-lane LDS staging area (stage[e * BLOCK + tid]) so
    // that the generator loop can stay rolled while every register of dst is written with a
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
                const float4 w = value4((base >> 2) + c);
                if (4 * c + 0 < COUNT) dst[4 * c + 0] = w.x;
                if (4 * c + 1 < COUNT) dst[4 * c + 1] = w.y;
                if (4 * c + 2 < COUNT) dst[4 * c + 2] = w.z;
                if (4 * c + 3 < COUNT) dst[4 * c + 3] = w.w;
            }
        } else {
            static_assert(COUNT % 4 == 0, "aligned slices come in whole Philox blocks");
            constexpr int NCH = (COUNT + STAGE - 1) / STAGE;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int len = ch + 1 < NCH ? STAGE : COUNT - (NCH - 1) * STAGE;
#pragma unroll 1
                for (int c = 0; c < len / 4; ++c) {
                    const float4 w = value4((base >> 2) + ch * (STAGE / 4) + c);
                    stage[(4 * c + 0) * block + tid] = w.x;
                    stage[(4 * c + 1) * block + tid] = w.y;
                    stage[(4 * c + 2) * block + tid] = w.z;
                    stage[(4 * c + 3) * block + tid] = w.w;
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
            const float2 w = pair(base + e);
            dst[e] = w.x;
            dst[e + 1] = w.y;
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
            const float4 w = value4(c);
            const float v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = 4 * c + j - BASE;
                if (e >= 0 && e < COUNT) dst[e] = v[j];
            }
        }
    }

    // theta[k] for any k.
    __device__ __forceinline__ float one(int k) const
    {
        if (explicit_theta) return explicit_theta[k];
        const float2 w = pair(k & ~1);
        return (k & 1) ? w.y : w.x;
    }
};

}  // namespace nnp
