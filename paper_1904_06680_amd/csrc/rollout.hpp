// Device side of one planner sample: controller weights in registers, the closed loop of
// Sect. II-E (features eq. (3) -> MLP eq. (4) -> control map and kinematic model of Sect. II-F),
// the per-point rectangle test of eq. (2) and the cost.
//
// Lane layout: a sample occupies K adjacent lanes of a wavefront (K in {1, 2, 4, 8, 16}). Each
// lane holds H/K rows of every hidden layer plus the output-layer weights of its own share of the
// last hidden layer, so the 1410-parameter 8-32-32-2 network fits in registers at K = 8 (178
// per lane). The K lanes split the obstacle points of every step and keep identical copies of
// the state; the first hidden layer's outputs reach the second by lane broadcasts (DPP, swizzle)
// or, for K >= 8 in the rollout kernels, through a per-sample LDS slot, and the output layer's
// chunk sums meet in a pairwise tree across the lanes. Every hidden-layer dot product runs over
// its inputs in index order and the output layer uses the same tree whatever K is, so results
// are bit-identical for every K.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "philox.hpp"

namespace nnp {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr float PI_F = 3.14159274101257324f;        // smallest float above pi
constexpr float TWO_PI_HI = 6.28318548202514648f;   // float nearest 2 pi (above it)
constexpr float TWO_PI_LO = -1.74845553e-7f;         // 2 pi - TWO_PI_HI

// One +-2 pi correction of an angle at or beyond +-PI_F: the wrap of the heading after a step and
// of heading errors. In the per-sample code the correction is a branch that the wavefront skips
// when none of its lanes needs it (the usual case).
__device__ __forceinline__ float wrap_pi(float a)
{
    if (a >= PI_F) a = (a - TWO_PI_HI) - TWO_PI_LO;
    else if (a <= -PI_F) a = (a + TWO_PI_HI) + TWO_PI_LO;
    return a;
}

// The same bits without a branch, for a chain of dependent steps in one lane: (a - s1) - s2 with
// (s1, s2) = (HI, LO), (-HI, -LO) or (+0, +0) selected by the same tests is (a - HI) - LO,
// (a + HI) + LO (subtracting -x is adding x), or a itself (subtracting +0 keeps a, -0 included).
__device__ __forceinline__ float wrap_pi_select(float a)
{
    const bool up = a >= PI_F, dn = a <= -PI_F;
    const float s1 = up ? TWO_PI_HI : (dn ? -TWO_PI_HI : 0.0f);
    const float s2 = up ? TWO_PI_LO : (dn ? -TWO_PI_LO : 0.0f);
    return (a - s1) - s2;
}

// Constants derived from nnp_model on the host (Table I, Table II and the cost weights).
struct DevModel {
    float dt;
    float lr_over_L, inv_L;            // l_r / (l_f + l_r), 1 / (l_f + l_r)
    float ihl, ihw, oc;                // 1/half-length, 1/half-width, centre offset along xi
    float delta_max, rate;             // rate: max |a0 - a0_prev| per step, 0 = off
    float u_min, u_half_range;         // u = u_min + (a1 + 1) * u_half_range
    float v_min, v_max;
    float inv_nxi, inv_neta, inv_nphi, inv_nv;
    float d_cap, inv_dcap;
    float effort_scale;                // effort_weight * dt
    float w_phi, w_v;                  // terminal heading / speed weights (0 = off)
    float eps_xi, eps_eta, eps_phi, eps_v;
};

// tanh in binary32 for the controller's units, about 3 ulp worst case:
//  |x| <  0.4: the odd Maclaurin series x + c3 x^3 + ... + c13 x^13, c_{2n-1} =
//              B_{2n} 4^n (4^n - 1) / (2n)! (B: Bernoulli numbers); the first omitted term is
//              below 4e-9 relative on this interval;
//  |x| >= 0.4: (1 - e) / (1 + e) with e = exp(-2|x|) from the hardware base-2 exponential and
//              reciprocal (1 ulp each); 1 - e loses at most a factor e / (1 - e) < 0.82 of the
//              exponential's error, and large |x| gives e = 0 and exactly +-1.
__device__ __forceinline__ float tanh_f32(float x)
{
    const float s = x * x;
    float p = 3.59212803657248e-3f;                  // 21844 / 6081075
    p = fmaf(p, s, -8.86323552990220e-3f);           // -1382 / 155925
    p = fmaf(p, s, 2.18694885361552e-2f);            // 62 / 2835
    p = fmaf(p, s, -5.39682539682540e-2f);           // -17 / 315
    p = fmaf(p, s, 1.33333333333333e-1f);            // 2 / 15
    p = fmaf(p, s, -3.33333333333333e-1f);           // -1 / 3
    const float small = fmaf(x * s, p, x);
    const float a = fabsf(x);
    const float e = __builtin_amdgcn_exp2f(a * -2.88539008177793f);   // -2 / ln 2
    const float big = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
    return a < 0.4f ? small : copysignf(big, x);
}

// MLP shape: NIN inputs, hidden widths H1 and H2 (H2 = 0: one hidden layer), 2 tanh outputs.
// Parameters are stored layer by layer, W_l row-major [n_l][n_{l-1}] followed by b_l.
template <int NIN_, int H1_, int H2_, int FEAT_>
struct Net {
    static constexpr int NIN = NIN_, H1 = H1_, H2 = H2_, FEAT = FEAT_;
    static constexpr int HL = H2 ? H2 : H1;     // width feeding the output layer
    static constexpr int OFF_W1 = 0;
    static constexpr int OFF_B1 = H1 * NIN;
    static constexpr int OFF_W2 = OFF_B1 + H1;
    static constexpr int OFF_B2 = OFF_W2 + H2 * H1;
    static constexpr int OFF_WO = H2 ? OFF_B2 + H2 : OFF_W2;
    static constexpr int OFF_BO = OFF_WO + 2 * HL;
    static constexpr int NTHETA = OFF_BO + 2;
};

// ---------------------------------------------------------------------------------------------
// Lane exchanges within a sample's K lanes: DPP quad permutations for K <= 4 (a quad), plus the
// half-row mirror (lane i <-> 7 - i) and swizzle broadcasts for K = 8, row mirror and row
// broadcasts for K = 16 (one DPP row per sample).
// ---------------------------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int K>
__device__ __forceinline__ float group_min(float v)
{
    if constexpr (K >= 2) v = fminf(v, dpp_f<0xB1>(v));   // quad_perm [1,0,3,2]: lane ^ 1
    if constexpr (K >= 4) v = fminf(v, dpp_f<0x4E>(v));   // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (K >= 8) v = fminf(v, dpp_f<0x141>(v));  // row_half_mirror: the other quad
    if constexpr (K >= 16) v = fminf(v, dpp_f<0x140>(v)); // row_mirror: the other half-row
    return v;
}

// Value of sub-lane B of the caller's group.
template <int K, int B>
__device__ __forceinline__ float group_bcast(float v)
{
    if constexpr (K == 1) return v;
    else if constexpr (K == 2) return dpp_f<(B | (B << 2) | ((2 + B) << 4) | ((2 + B) << 6))>(v);
    else if constexpr (K == 4) return dpp_f<(B * 0x55)>(v);
    else if constexpr (K == 8)   // swizzle bit mode: lane = (lane & 0b11000) | B within 32 lanes
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x18 | (B << 5)));
    else                         // K = 16, one DPP row: row_newbcast of lane B
        return dpp_f<0x150 + B>(v);
}

// ---------------------------------------------------------------------------------------------
// Controller a = X(s, theta), eq. (4): tanh MLP, weights resident in registers.
// ---------------------------------------------------------------------------------------------
template <class NetT, int K>
struct Controller {
    static constexpr int NIN = NetT::NIN, H1 = NetT::H1, H2 = NetT::H2, HL = NetT::HL;
    static constexpr int U1 = H1 / K;
    static constexpr int U2 = H2 ? H2 / K : 1;
    static constexpr int UL = HL / K;               // inputs of the output layer held by a lane
    // Output layer: when HL is a multiple of 4, each output is summed in chunks of four inputs
    // (a multiply and three fused multiply-adds in index order), and the HL / 4 chunk sums are
    // added pairwise as a balanced tree (chunks 2c and 2c+1 first, then pairs of pairs, ...),
    // then the bias. A lane holds the output weights of the chunks it covers (one chunk per pair
    // of lanes at K = 16), computes both outputs, and the tree's upper levels run across lanes;
    // every lane layout K adds the same numbers in the same tree, so all K give the same bits.
    // Other widths (K = 1 only) sum in index order starting from the bias.
    static constexpr bool CHUNKED = HL % 4 == 0;
    static constexpr int LW = K == 1 ? HL : (UL >= 4 ? UL : 4);   // weights per output per lane
    static constexpr int NCH = LW / 4;              // chunks summed by one lane (CHUNKED)
    static constexpr int LPC = UL >= 4 ? 1 : 4 / UL;   // lanes sharing one chunk (K = 16: 2)
    static_assert(H1 % K == 0 && (H2 == 0 || H2 % K == 0), "hidden widths must split over K");
    static_assert(K == 1 || CHUNKED, "lane layouts need output-layer widths divisible by 4");
    static_assert(K == 1 || ((U1 * NIN) % 4 == 0 && NetT::OFF_B1 % 4 == 0 && U1 % 2 == 0 &&
                             NetT::OFF_WO % 4 == 0 && HL % 4 == 0 &&
                             (H2 == 0 || ((U2 * H1) % 4 == 0 && NetT::OFF_W2 % 4 == 0 &&
                                          NetT::OFF_B2 % 4 == 0 && U2 % 2 == 0))),
                  "weight slices of a lane must start on Philox blocks, bias slices on pairs");

    float w1[U1 * NIN], b1[U1];
    float w2[H2 ? U2 * H1 : 1], b2[U2];
    float wo[2][LW], bo[2];

    // stage: LDS scratch of ThetaSource::STAGE * block floats shared by the workgroup, each
    // lane using its own column.
    __device__ __forceinline__ void load(const ThetaSource &src, int q, float *stage, int tid,
                                         int block)
    {
        if constexpr (K == 1) {
            src.template fill_const<NetT::OFF_W1, U1 * NIN>(w1);
            src.template fill_const<NetT::OFF_B1, U1>(b1);
            if constexpr (H2) {
                src.template fill_const<NetT::OFF_W2, U2 * H1>(w2);
                src.template fill_const<NetT::OFF_B2, U2>(b2);
            }
            src.template fill_const<NetT::OFF_WO, HL>(wo[0]);
            src.template fill_const<NetT::OFF_WO + HL, HL>(wo[1]);
            src.template fill_const<NetT::OFF_BO, 2>(bo);
        } else {
            src.fill_aligned(w1, NetT::OFF_W1 + q * U1 * NIN, stage, tid, block);
            src.fill_even(b1, NetT::OFF_B1 + q * U1);
            if constexpr (H2) {
                src.fill_aligned(w2, NetT::OFF_W2 + q * U2 * H1, stage, tid, block);
                src.fill_even(b2, NetT::OFF_B2 + q * U2);
            }
            const int e0 = (q / LPC) * LW;          // first output-layer input covered
            src.fill_aligned(wo[0], NetT::OFF_WO + e0, stage, tid, block);
            src.fill_aligned(wo[1], NetT::OFF_WO + HL + e0, stage, tid, block);
            src.fill_even(bo, NetT::OFF_BO);
        }
    }

    // Sub-lane B's value of a per-lane array element, as a compile-time selected broadcast.
    template <int B>
    __device__ __forceinline__ static float bcast(float v)
    {
        return group_bcast<K, B>(v);
    }

    // acc[o] += sum_j W[o][j] x[j] over the full input vector x of width U * K, whose element
    // j = b * U + u lives in sub-lane b as own[u]. Elements are broadcast one at a time and
    // consumed in index order (so no gathered copy of x is kept and the summation order is
    // the same for every K).
    template <int NOUT, int U, int B = 0>
    __device__ __forceinline__ static void accumulate(const float *W, const float (&own)[U],
                                                      float (&acc)[NOUT])
    {
        constexpr int NINP = U * K;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float x = bcast<B>(own[u]);
#pragma unroll
            for (int o = 0; o < NOUT; ++o) acc[o] = fmaf(W[o * NINP + B * U + u], x, acc[o]);
        }
        if constexpr (B + 1 < K) accumulate<NOUT, U, B + 1>(W, own, acc);
    }

    // Hidden layer 2 may take its input vector through LDS instead of by broadcasts: every lane
    // writes its U elements to the sample's slot (H1 floats), then reads the whole vector back
    // four elements at a time. The K lanes sit in one wavefront, whose LDS accesses are carried
    // out in issue order, so only the compiler has to be kept from moving them. Used for K >= 8,
    // whose broadcasts are LDS swizzles or DPP row broadcasts (K = 4 broadcasts by quad
    // permutes, cheaper than the exchange).
    static constexpr bool LDS_X = K >= 8 && H2 > 0 && U1 % 2 == 0 && H1 % 4 == 0;
    static constexpr int ACT = LDS_X ? H1 : 0;      // floats of one sample's slot

    // acc[o] += sum_j W[o][j] x[j] as in accumulate, x exchanged through the slot act.
    template <int NOUT, int U>
    __device__ __forceinline__ static void accumulate_lds(const float *W, const float (&own)[U],
                                                          float (&acc)[NOUT], float *act, int q)
    {
        constexpr int NINP = U * K;
        static_assert(U % 2 == 0 && NINP % 4 == 0, "whole float2 writes and float4 reads");
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // last step's reads first
        __builtin_amdgcn_wave_barrier();
        if constexpr (U % 4 == 0) {
#pragma unroll
            for (int c = 0; c < U / 4; ++c)
                *reinterpret_cast<float4 *>(act + q * U + 4 * c) =
                    make_float4(own[4 * c], own[4 * c + 1], own[4 * c + 2], own[4 * c + 3]);
        } else {
            *reinterpret_cast<float2 *>(act + q * U) = make_float2(own[0], own[1]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int c = 0; c < NINP / 4; ++c) {
            const float4 x4 = *reinterpret_cast<const float4 *>(act + 4 * c);
            const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int o = 0; o < NOUT; ++o)
                    acc[o] = fmaf(W[o * NINP + 4 * c + u], xs[u], acc[o]);
        }
    }

    // Pairwise tree over n consecutive chunk sums (n a power of two).
    template <int N>
    __device__ __forceinline__ static float tree(const float *v)
    {
        if constexpr (N == 1) return v[0];
        else return tree<N / 2>(v) + tree<N / 2>(v + N / 2);
    }

    // The upper tree levels across lanes: level l adds the sums of the lane groups whose chunk
    // sets differ in bit l (exchange patterns: lane ^ 1, lane ^ 2 within a quad, mirrored quads
    // of a half-row, mirrored half-rows of a row).
    template <int LEVEL>
    __device__ __forceinline__ static float cross(float v)
    {
        if constexpr (LEVEL == 0) return v + dpp_f<0xB1>(v);
        else if constexpr (LEVEL == 1) return v + dpp_f<0x4E>(v);
        else if constexpr (LEVEL == 2) return v + dpp_f<0x141>(v);
        else return v + dpp_f<0x140>(v);
    }

    template <int L0, int L1>
    __device__ __forceinline__ static float cross_levels(float v)
    {
        if constexpr (L0 < L1) return cross_levels<L0 + 1, L1>(cross<L0>(v));
        else return v;
    }

    static constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

    // Output sums of the chunked layout: the chunks of this lane from its inputs `own`.
    __device__ __forceinline__ void outputs(const float (&own)[UL], int q, float &o0,
                                            float &o1) const
    {
        float x[LW];
        if constexpr (UL >= 4) {
#pragma unroll
            for (int e = 0; e < LW; ++e) x[e] = own[e];
        } else {                    // K = 16: the chunk's other two inputs come from lane ^ 1
            const float p0 = dpp_f<0xB1>(own[0]), p1 = dpp_f<0xB1>(own[1]);
            const bool odd = q & 1;
            x[0] = odd ? p0 : own[0];
            x[1] = odd ? p1 : own[1];
            x[2] = odd ? own[0] : p0;
            x[3] = odd ? own[1] : p1;
        }
        float c[2][NCH];
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int k = 0; k < NCH; ++k) {
                float t = wo[o][4 * k] * x[4 * k];
                t = fmaf(wo[o][4 * k + 1], x[4 * k + 1], t);
                t = fmaf(wo[o][4 * k + 2], x[4 * k + 2], t);
                c[o][k] = fmaf(wo[o][4 * k + 3], x[4 * k + 3], t);
            }
        constexpr int L0 = ilog2(LPC), L1 = ilog2(K);
        o0 = cross_levels<L0, L1>(tree<NCH>(c[0])) + bo[0];
        o1 = cross_levels<L0, L1>(tree<NCH>(c[1])) + bo[1];
    }

    // XLDS: hidden layer 2 takes its input through the LDS slot act (LDS_X layouts only).
    template <bool XLDS = false>
    __device__ __forceinline__ void forward(const float (&s)[NIN], float &a0, float &a1,
                                            int q, float *act = nullptr) const
    {
        float h1o[U1];
#pragma unroll
        for (int u = 0; u < U1; ++u) {
            float acc = b1[u];
#pragma unroll
            for (int i = 0; i < NIN; ++i) acc = fmaf(w1[u * NIN + i], s[i], acc);
            h1o[u] = tanh_f32(acc);
        }
        float h2o[U2];
        if constexpr (H2) {
#pragma unroll
            for (int o = 0; o < U2; ++o) h2o[o] = b2[o];
            if constexpr (XLDS && LDS_X) accumulate_lds<U2, U1>(w2, h1o, h2o, act, q);
            else accumulate<U2, U1>(w2, h1o, h2o);
#pragma unroll
            for (int o = 0; o < U2; ++o) h2o[o] = tanh_f32(h2o[o]);
        }
        const float(&hl)[UL] = *reinterpret_cast<const float(*)[UL]>(H2 ? h2o : h1o);
        float o0, o1;
        if constexpr (CHUNKED) {
            outputs(hl, q, o0, o1);
        } else {
            o0 = bo[0];
            o1 = bo[1];
#pragma unroll
            for (int j = 0; j < HL; ++j) {
                o0 = fmaf(wo[0][j], hl[j], o0);
                o1 = fmaf(wo[1][j], hl[j], o1);
            }
        }
        a0 = tanh_f32(o0);
        a1 = tanh_f32(o1);
    }
};

// ---------------------------------------------------------------------------------------------
// The vehicle pose at one step in the form the obstacle pass consumes.
// ---------------------------------------------------------------------------------------------
struct Pose {
    float x, y;
    float cxi, sxi, oxi;      // xi' = (c dx + s dy - oc) / hl  = cxi dx + sxi dy + oxi
    float ceta, nseta;        // eta' = (c dy - s dx) / hw     = ceta dy + nseta dx

    // Eq. (2) for one extrapolated point, folded into the running minima of the normalised
    // margin max(|xi'|, |eta'|) (< 1 exactly when the point is strictly inside) and of the
    // squared distance to the reference point. Translate first, then rotate: dx, dy are exact
    // for points near the vehicle, which keeps the test accurate near the faces.
    // CENTRED: the rectangle is centred on the reference point (oxi = 0), so the inner
    // fmaf(sxi, dy, 0) is the plain product sxi * dy (up to the sign of a zero, which |xi'|
    // drops): same margins, and a 32-bit-encoded multiply instead of a three-operand FMA.
    template <bool CENTRED = false>
    __device__ __forceinline__ void point(float px, float py, float &mg, float &d2) const
    {
        const float dx = px - x, dy = py - y;
        const float xi = fmaf(cxi, dx, CENTRED ? sxi * dy : fmaf(sxi, dy, oxi));
        const float et = fmaf(ceta, dy, nseta * dx);   // nseta = -seta: a plain multiply
        mg = fmaxf(fabsf(xi), fabsf(et));
        d2 = fmaf(dx, dx, dy * dy);
    }

    template <bool CENTRED = false>
    __device__ __forceinline__ void pair(v4f p, float &mm, float &md) const
    {
        float m0, d0, m1, d1;
        point<CENTRED>(p.x, p.y, m0, d0);
        point<CENTRED>(p.z, p.w, m1, d1);
        mm = fminf(fminf(mm, m0), m1);   // one v_min3 per pair
        md = fminf(fminf(md, d0), d1);
    }
};

// Goal tolerances of Table II at state (x, y, phi, v) with c = cos phi, s = sin phi: the goal's
// offset in the vehicle frame within (eps_xi, eps_eta), heading error within eps_phi and speed
// error within eps_v.
__device__ __forceinline__ int within_tolerance(float eps_xi, float eps_eta, float eps_phi,
                                                float eps_v, const float (&goal)[4], float x,
                                                float y, float phi, float v, float c, float s)
{
    const float gx = goal[0] - x, gy = goal[1] - y;
    const float xi_g = fmaf(c, gx, s * gy);
    const float eta_g = fmaf(c, gy, -(s * gx));
    const float dphi = wrap_pi(goal[2] - phi);
    return fabsf(xi_g) <= eps_xi && fabsf(eta_g) <= eps_eta && fabsf(dphi) <= eps_phi &&
           fabsf(goal[3] - v) <= eps_v;
}

// Control map and one explicit Euler step of the kinematic model (Sect. II-F, eq. (5)) with the
// applied controls (a0, a1); c, s are the cosine and sine of the current heading.
// cos(phi + beta)/cos(beta) = cos(phi) - sin(phi) tan(beta) and likewise for sin, with
// tan(beta) = l_r tan(delta) / L, so no atan or second sincos is needed.
// The model step in two parts, with td = tan(delta_max a0) computed by the caller (model_step)
// or ahead of time: heading and speed (they do not depend on the position) and the position
// (from the old heading's c, s and the old speed).
template <bool SELECT_WRAP = false>
__device__ __forceinline__ void heading_speed_step(const DevModel &m, float a1, float td,
                                                   float &phi, float &v)
{
    const float u = fmaf(a1 + 1.0f, m.u_half_range, m.u_min);
    const float ds = m.dt * v;
    float nphi = fmaf(ds * td, m.inv_L, phi);
    nphi = SELECT_WRAP ? wrap_pi_select(nphi) : wrap_pi(nphi);
    phi = nphi;
    v = fminf(fmaxf(fmaf(m.dt, u, v), m.v_min), m.v_max);
}

__device__ __forceinline__ void position_step(const DevModel &m, float td, float c, float s,
                                              float v, float &x, float &y)
{
    const float tb = m.lr_over_L * td;
    const float ds = m.dt * v;
    const float nx = fmaf(ds, fmaf(-s, tb, c), x);
    const float ny = fmaf(ds, fmaf(c, tb, s), y);
    x = nx;
    y = ny;
}

__device__ __forceinline__ void model_step_td(const DevModel &m, float a1, float td, float c,
                                              float s, float &x, float &y, float &phi, float &v)
{
    position_step(m, td, c, s, v, x, y);
    heading_speed_step(m, a1, td, phi, v);
}

__device__ __forceinline__ void model_step(const DevModel &m, float a0, float a1, float c,
                                           float s, float &x, float &y, float &phi, float &v)
{
    model_step_td(m, a1, tanf(m.delta_max * a0), c, s, x, y, phi, v);
}

// ---------------------------------------------------------------------------------------------
// One sample's closed-loop state.
// ---------------------------------------------------------------------------------------------
template <class NetT, int K>
struct SampleSim {
    Controller<NetT, K> ctl;
    float x, y, phi, v;       // z_h
    float ap0, ap1;           // a_{h-1}
    float effort;             // sum of |a|^2 so far
    float min_margin;         // min over steps and points of the normalised margin
    int first;                // first step with a point inside, -1 if none
    float c, s;               // cos / sin of phi at the current step

    __device__ __forceinline__ void init(const float (&z0)[4], const float (&a_prev)[2])
    {
        x = z0[0];
        y = z0[1];
        phi = z0[2];
        v = z0[3];
        ap0 = a_prev[0];
        ap1 = a_prev[1];
        effort = 0.0f;
        min_margin = INFINITY;
        first = -1;
    }

    // Heading of step h and the pose constants of its obstacle pass.
    __device__ __forceinline__ Pose begin_step(const DevModel &m)
    {
        float sv, cv;
        sincosf(phi, &sv, &cv);
        s = sv;
        c = cv;
        Pose p;
        p.x = x;
        p.y = y;
        p.cxi = c * m.ihl;
        p.sxi = s * m.ihl;
        p.oxi = -m.oc * m.ihl;
        p.ceta = c * m.ihw;
        p.nseta = -(s * m.ihw);
        return p;
    }

    // Collision bookkeeping of step h from the step's minima over all points.
    __device__ __forceinline__ void record_collision(int h, float mm)
    {
        if (mm < 1.0f && first < 0) first = h;
        min_margin = fminf(min_margin, mm);
    }

    // Features s_h of eq. (3) and its variants.
    __device__ __forceinline__ void features(const DevModel &m, const float (&goal)[4], float md,
                                             float (&f)[NetT::NIN]) const
    {
        const float gx = goal[0] - x, gy = goal[1] - y;
        const float xi_g = fmaf(c, gx, s * gy);
        const float eta_g = fmaf(c, gy, -(s * gx));
        const float dphi = wrap_pi(goal[2] - phi);
        if constexpr (NetT::FEAT == 0) {
            f[0] = xi_g * m.inv_nxi;
            f[1] = eta_g * m.inv_neta;
            f[2] = dphi * m.inv_nphi;
            f[3] = (goal[3] - v) * m.inv_nv;
            f[4] = ap0;
        } else {
            const float dn = fminf(sqrtf(md), m.d_cap);
            f[0] = xi_g * m.inv_nxi;
            f[1] = eta_g * m.inv_neta;
            f[2] = dphi * m.inv_nphi;
            f[3] = v * m.inv_nv;
            f[4] = dn * m.inv_dcap;
            f[5] = ap0;
            if constexpr (NetT::FEAT == 2) {
                f[6] = (goal[3] - v) * m.inv_nv;
                f[7] = ap1;
            }
        }
    }

    // Controller, rate limit, then the control map and the model step (model_step).
    template <bool XLDS = false>
    __device__ __forceinline__ void advance(const DevModel &m, const float (&goal)[4], float md,
                                            float &a0, float &a1, int q, float *act = nullptr)
    {
        float f[NetT::NIN];
        features(m, goal, md, f);
        ctl.template forward<XLDS>(f, a0, a1, q, act);
        if (m.rate > 0.0f) a0 = fminf(fmaxf(a0, ap0 - m.rate), ap0 + m.rate);
        model_step(m, a0, a1, c, s, x, y, phi, v);
        effort = effort + fmaf(a0, a0, a1 * a1);
        ap0 = a0;
        ap1 = a1;
    }

    __device__ __forceinline__ float cost(const DevModel &m, const float (&goal)[4]) const
    {
        const float gx = x - goal[0], gy = y - goal[1];
        float J = sqrtf(fmaf(gx, gx, gy * gy)) + m.effort_scale * effort;
        if (m.w_phi > 0.0f) {
            const float dphi = wrap_pi(goal[2] - phi);
            J += m.w_phi * fabsf(dphi);
        }
        if (m.w_v > 0.0f) J += m.w_v * fabsf(goal[3] - v);
        if (first >= 0 || J != J) J = INFINITY;
        return J;
    }

    // Tolerance test of Table II at the current state.
    __device__ __forceinline__ int goal_reached(const DevModel &m, const float (&goal)[4]) const
    {
        return within_tolerance(m.eps_xi, m.eps_eta, m.eps_phi, m.eps_v, goal, x, y, phi, v, c, s);
    }
};

}  // namespace nnp
