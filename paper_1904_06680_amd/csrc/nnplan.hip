// nnplan: kernels and C-ABI of the MI355X rollout planner (declarations in include/nnplan.h).
//
// One planning call (Step 5 of Alg. 1, Sect. II-E) is four launches on the caller's stream:
//   1. order_kernel        a spatial order of the obstacle points (grid cells in Z-order) and a
//                          bound on how far any point moves between two steps.
//   2. extrapolate_kernel  obstacle points at every step h = 0..T under constant velocity
//                          (Sect. II-E items (ii)-(iv)) into a [T+1][P64/2] table of point pairs
//                          in that order, with the bounding box of every group of consecutive
//                          pairs; it also resets the argmin key.
//   3. rollout_kernel      every sample rolled over the horizon: Philox parameters in
//                          registers, per step a pass over the points (eq. (2) and the nearest
//                          distance) from LDS buffers filled by asynchronous copies, skipping the
//                          groups that cannot change any minimum of the wavefront's samples,
//                          features (eq. (3)), MLP (eq. (4)), model (Sect. II-F) and the cost; a
//                          u64 (cost bits, index) atomicMin selects the best sample, lowest index
//                          on ties. When the handle's record limit allows, every sample's applied
//                          controls are also stored (step-major, coalesced).
//   4. gather_kernel       re-integrates the winner's states from its recorded controls and
//      / replay_kernel     regenerates theta*; or, without records, one workgroup re-simulates
//                          the winner with the same device functions (points split over 256
//                          lanes). Both give the same bits.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/nnplan.h"
#include "philox.hpp"
#include "rollout.hpp"

using namespace nnp;

namespace {

constexpr int BLOCK = 256;
constexpr int POINT_PAD = 64;   // points per step padded to a multiple of this (pairs per
                                // subset then come in whole groups of four for K <= 8)
constexpr int TILE_PAIRS = 2048;  // point pairs per LDS buffer (two buffers: 64 KiB); 1536 for
                                  // K = 16, so that three workgroups share a CU, 1024 for K <= 2
constexpr int BUFFER_RSRC_FLAGS = 0x00020000;   // buffer descriptor word 3: 32-bit data format
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
constexpr int CHUNK = 64;         // pairs moved by one wavefront-wide asynchronous copy
// Point groups: every GP consecutive pairs of a step's table (GP = 16 or 32, the launch shape's
// group size; a multiple of it is never split by a tile) share a bounding box, and a
// wavefront skips a group at a step when the box lies farther than the cull radius from every
// one of its samples (see group_mask). Up to SORT_MAX points are first put in spatial order
// (order_kernel) so that the groups are compact; larger sets keep the caller's order.
constexpr int MAX_GROUP_PAIRS = 32;
constexpr int SORT_MAX = 1 << 20;
constexpr int ORDER_BLOCK = 1024;
constexpr int ORDER_GRID = 64;    // cells per axis of the spatial order

struct RolloutArgs {
    DevModel m;
    float z0[4], goal[4], a_prev[2];
    int N, T, P2;                    // P2 = padded points / 2 (float4 pairs per step)
    const float4 *ext;               // [T+1][P2] extrapolated point pairs
    PhiloxKey key;
    uint32_t inst;
    const float *theta;              // explicit [N][n_theta] or null
    const float *warm_theta;         // replaces sample 0 when not null
    unsigned long long *best_key;    // plan mode
    float *cost;                     // rollout mode outputs (each may be null)
    int32_t *collided, *first;
    float *min_margin, *traj, *controls;
    const float4 *obst;              // raw points [P][4] (batched extrapolation)
    int P;
    const float *mu, *log_sigma;     // Gaussian proposal for samples [0, n_prop)
    int n_prop;
    float2 *rec_ctrl;                // record mode: applied controls [T][N] of every sample
                                     // (step-major: coalesced stores)
    const float4 *bb;                // [T+1][P2 / gp] group boxes (xmin, ymin, xmax, ymax)
    uint32_t *perm;                  // [P] spatial order of the points, or null (caller's order)
    float *disp;                     // [1] bound on a point's move between two steps (order_kernel)
    unsigned long long *stats;       // [2] tested / all point groups per wavefront-tile, or null
    float cull_r2;                   // squared cull radius; +INFINITY tests every group
    float coll_r2;                   // squared collision radius (the rectangle's corner distance)
    float step_scale;                // bound on |z_{h+1} - z_h| (x, y) per unit of |v_h|
    int gp;                          // pairs per point group of the handle's launch shape
};

// Culling constants of a model (cull_consts): squared cull and collision radii, and the bound on
// the sample's move per step per unit of speed.
struct CullConsts {
    float cull_r2, coll_r2, step_scale;
};

struct ReplayOut {
    float *theta, *controls, *controls_phys, *traj, *cost;
    int32_t *best_index, *status, *goal_reached;
};

enum { MODE_PLAN = 0, MODE_OUT = 1 };

// ---------------------------------------------------------------------------------------------
// 1. Constant-velocity extrapolation table; padding repeats the last point (min-neutral).
// ---------------------------------------------------------------------------------------------
static_assert((POINT_PAD / 2) % MAX_GROUP_PAIRS == 0, "a step's pairs form whole groups");

// Entry (h, j) of the table (pair j of step h, entries numbered h * P2 + j) and the boxes of the
// point groups of gp pairs: P2 is a multiple of gp, so the pairs of one group sit in one aligned
// run of gp lanes, which reduce their coordinates (exact minima and maxima); the group's first
// lane writes the box. NaN coordinates are left out of a box, as the obstacle pass leaves them
// out of its minima. The caller runs whole groups of lanes.
__device__ __forceinline__ void table_entry(const float4 *__restrict__ pts,
                                            const uint32_t *__restrict__ perm, int P, int P2,
                                            int gp, float dt, long long gid,
                                            float4 *__restrict__ ext, float4 *__restrict__ bb)
{
    const int h = (int)(gid / P2);
    const int j = (int)(gid % P2);
    const float t = (float)h * dt;
    int i0 = min(2 * j, P - 1), i1 = min(2 * j + 1, P - 1);
    if (perm) {
        i0 = (int)perm[i0];
        i1 = (int)perm[i1];
    }
    const float4 a = pts[i0];
    const float4 b = pts[i1];
    const float4 e = make_float4(fmaf(t, a.z, a.x), fmaf(t, a.w, a.y), fmaf(t, b.z, b.x),
                                 fmaf(t, b.w, b.y));
    ext[gid] = e;
    float lx = fminf(e.x, e.z), ly = fminf(e.y, e.w), hx = fmaxf(e.x, e.z), hy = fmaxf(e.y, e.w);
#pragma unroll
    for (int off = MAX_GROUP_PAIRS / 2; off >= 1; off >>= 1) {
        if (off >= gp) continue;
        lx = fminf(lx, __shfl_xor(lx, off, 64));
        ly = fminf(ly, __shfl_xor(ly, off, 64));
        hx = fmaxf(hx, __shfl_xor(hx, off, 64));
        hy = fmaxf(hy, __shfl_xor(hy, off, 64));
    }
    if (j % gp == 0) bb[(size_t)h * (P2 / gp) + j / gp] = make_float4(lx, ly, hx, hy);
}

__global__ __launch_bounds__(BLOCK) void extrapolate_kernel(const float4 *__restrict__ pts,
                                                            const uint32_t *__restrict__ perm,
                                                            int P, int P2, int gp, int T,
                                                            float dt, float4 *__restrict__ ext,
                                                            float4 *__restrict__ bb,
                                                            unsigned long long *best_key)
{
    const long long n = (long long)(T + 1) * P2;
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid == 0 && best_key) *best_key = ~0ull;
    // n and the block size are multiples of gp: lanes leave in whole groups
    if (gid >= n || P == 0) return;
    table_entry(pts, perm, P, P2, gp, dt, gid, ext, bb);
}

// The same table for every problem of a batch: blockIdx.y is the problem, the x blocks stride
// over its entries. Also resets the problems' argmin keys.
__global__ __launch_bounds__(BLOCK) void extrapolate_batch_kernel(const RolloutArgs *probs)
{
    const RolloutArgs &a = probs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.best_key = ~0ull;
    if (a.P == 0) return;
    const long long n = (long long)(a.T + 1) * a.P2;
    float4 *ext = const_cast<float4 *>(a.ext);
    float4 *bb = const_cast<float4 *>(a.bb);
    for (long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x; gid < n;
         gid += (long long)gridDim.x * BLOCK)
        table_entry(a.obst, a.perm, a.P, a.P2, a.gp, a.m.dt, gid, ext, bb);
}

// Spread the low 16 bits of v over the even bit positions (one half of a Z-order key).
__device__ __forceinline__ uint32_t spread_bits(uint32_t v)
{
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Spatial order of P <= SORT_MAX points, by one workgroup of ORDER_BLOCK threads: each point's
// position at the middle of the horizon (tmid), on a 64 x 64 grid over the bounding box of
// those positions, falls into a cell, and the cells are laid out in Z-order (Morton code of the
// cell's coordinates). A counting sort gives that order: per-cell counts with LDS atomics, an
// exclusive scan, and a scatter in which every point takes the next free slot of its cell (so
// the points of one cell come in the order the atomics happen to run). perm[i] is the index of
// the i-th point. No result depends on the order (the obstacle pass takes exact minima); it keeps
// the points of a group close together, so that their box is small.
//
// It also writes *disp, a bound on how far any point of the table moves between two consecutive
// steps: |p_h - p_{h-1}| <= |v| (t_h - t_{h-1}) plus the rounding of the two table entries, with
// t_h = fl(h dt) (at most one ulp of T dt off, a relative 5e-4 of dt for T <= 4096) and entries
// no larger than M = max(|x| + T dt |vx|, |y| + T dt |vy|) (half an ulp each, per axis).
// Non-finite inputs give +INFINITY.
__device__ void order_points(const float4 *__restrict__ pts, int P, float tmid, float span,
                             float dt, uint32_t *__restrict__ perm, float *__restrict__ disp,
                             uint32_t *cnt, float (&red)[6][ORDER_BLOCK / 64])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY, v2 = 0.0f, pm = 0.0f;
    bool bad = false;
    for (int i = tid; i < P; i += ORDER_BLOCK) {
        const float4 p = pts[i];
        const float x = fmaf(tmid, p.z, p.x), y = fmaf(tmid, p.w, p.y);
        lx = fminf(lx, x);
        ly = fminf(ly, y);
        hx = fmaxf(hx, x);
        hy = fmaxf(hy, y);
        const float s2 = fmaf(p.z, p.z, p.w * p.w);
        const float m = fmaxf(fmaf(span, fabsf(p.z), fabsf(p.x)), fmaf(span, fabsf(p.w), fabsf(p.y)));
        bad = bad || !(s2 < INFINITY) || !(m < INFINITY);
        v2 = fmaxf(v2, s2);
        pm = fmaxf(pm, m);
    }
    if (bad) v2 = INFINITY;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lx = fminf(lx, __shfl_xor(lx, off, 64));
        ly = fminf(ly, __shfl_xor(ly, off, 64));
        hx = fmaxf(hx, __shfl_xor(hx, off, 64));
        hy = fmaxf(hy, __shfl_xor(hy, off, 64));
        v2 = fmaxf(v2, __shfl_xor(v2, off, 64));
        pm = fmaxf(pm, __shfl_xor(pm, off, 64));
    }
    if (lane == 0) {
        red[0][wave] = lx;
        red[1][wave] = ly;
        red[2][wave] = hx;
        red[3][wave] = hy;
        red[4][wave] = v2;
        red[5][wave] = pm;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < ORDER_BLOCK / 64; ++w) {
        lx = fminf(lx, red[0][w]);
        ly = fminf(ly, red[1][w]);
        hx = fmaxf(hx, red[2][w]);
        hy = fmaxf(hy, red[3][w]);
        v2 = fmaxf(v2, red[4][w]);
        pm = fmaxf(pm, red[5][w]);
    }
    if (tid == 0) {
        const float d = fmaf(sqrtf(v2) * dt, 1.001f, pm * 0x1p-21f);
        *disp = d < INFINITY ? d : INFINITY;
    }
    // grid scales (0 when the extent is empty or not finite: every point then has cell 0)
    const float sx = hx > lx ? (float)ORDER_GRID / (hx - lx) : 0.0f;
    const float sy = hy > ly ? (float)ORDER_GRID / (hy - ly) : 0.0f;
    for (int c = tid; c < ORDER_GRID * ORDER_GRID / 4; c += ORDER_BLOCK)
        reinterpret_cast<uint4 *>(cnt)[c] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    // cell code of point i: Z-order of its grid cell (fmaxf(NaN, 0) = 0: non-finite positions
    // fall into cell 0)
    auto cell_of = [&](int i) -> uint32_t {
        const float4 p = pts[i];
        const float x = fmaf(tmid, p.z, p.x), y = fmaf(tmid, p.w, p.y);
        const uint32_t cx = (uint32_t)fminf(fmaxf((x - lx) * sx, 0.0f), ORDER_GRID - 1.0f);
        const uint32_t cy = (uint32_t)fminf(fmaxf((y - ly) * sy, 0.0f), ORDER_GRID - 1.0f);
        return spread_bits(cx) | (spread_bits(cy) << 1);
    };
    for (int i = tid; i < P; i += ORDER_BLOCK) atomicAdd(&cnt[cell_of(i)], 1u);
    __syncthreads();
    if (wave == 0) {   // exclusive scan: 64 consecutive cells per lane, then across the lanes
        constexpr int PER4 = ORDER_GRID * ORDER_GRID / 64 / 4;
        uint4 *cnt4 = reinterpret_cast<uint4 *>(cnt) + lane * PER4;
        uint32_t run = 0;
#pragma unroll 4
        for (int k = 0; k < PER4; ++k) {
            const uint4 v = cnt4[k];
            run += v.x + v.y + v.z + v.w;
        }
        uint32_t incl = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        uint32_t base = incl - run;
#pragma unroll 4
        for (int k = 0; k < PER4; ++k) {
            const uint4 v = cnt4[k];
            uint4 o;
            o.x = base;
            o.y = o.x + v.x;
            o.z = o.y + v.y;
            o.w = o.z + v.z;
            base = o.w + v.w;
            cnt4[k] = o;
        }
    }
    __syncthreads();
    // scatter: each point takes the next free slot of its cell
    for (int i = tid; i < P; i += ORDER_BLOCK) perm[atomicAdd(&cnt[cell_of(i)], 1u)] = (uint32_t)i;
}

// The order and the displacement bound of one problem; a problem with more than SORT_MAX points
// keeps the caller's order and has no bound (+INFINITY: its culling uses the radius alone).
__device__ __forceinline__ void order_problem(const RolloutArgs &a, uint32_t *cnt,
                                              float (&red)[6][ORDER_BLOCK / 64])
{
    if (!a.perm) {
        if (threadIdx.x == 0) *a.disp = INFINITY;
        return;
    }
    const float span = (float)a.T * a.m.dt;
    order_points(a.obst, a.P, 0.5f * span, span, a.m.dt, a.perm, a.disp, cnt, red);
}

__global__ __launch_bounds__(ORDER_BLOCK) void order_kernel(const RolloutArgs a)
{
    __shared__ __align__(16) uint32_t cnt[ORDER_GRID * ORDER_GRID];
    __shared__ float red[6][ORDER_BLOCK / 64];
    order_problem(a, cnt, red);
}

// One workgroup per problem of a batch.
__global__ __launch_bounds__(ORDER_BLOCK) void order_batch_kernel(const RolloutArgs *probs)
{
    __shared__ __align__(16) uint32_t cnt[ORDER_GRID * ORDER_GRID];
    __shared__ float red[6][ORDER_BLOCK / 64];
    const RolloutArgs &a = probs[blockIdx.x];
    if (a.P > 0) order_problem(a, cnt, red);
}

template <class NetT>
__device__ __forceinline__ ThetaSource make_source(const RolloutArgs &a, int sample)
{
    ThetaSource src;
    src.key = a.key;
    src.inst = a.inst;
    src.sample = (uint32_t)sample;
    src.explicit_theta = nullptr;
    src.mu = nullptr;
    src.log_sigma = nullptr;
    src.n_theta = NetT::NTHETA;
    if (a.theta) {
        src.explicit_theta = a.theta + (size_t)sample * NetT::NTHETA;
    } else if (a.warm_theta && sample == 0) {
        src.explicit_theta = a.warm_theta;
    } else if (sample < a.n_prop) {
        src.mu = a.mu;                 // proposal draws: stream 1, own sample index
        src.log_sigma = a.log_sigma;
    } else {
        src.sample = (uint32_t)(sample - a.n_prop);   // uniform draws: stream 0 from index 0
    }
    return src;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ float wave_min_f(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

// Wavefront-wide mask of the groups of a tile segment that some sample of this wavefront needs:
// bit g for the group whose box is boxes[g] (g < ng <= 64). A sample needs a group unless the
// squared distance from its reference point (x, y) to the box exceeds r2; the K lanes of a
// sample test K groups at a time, and the wavefront's ballot is folded over its 64 / K samples.
// The box distance is a lower bound of the distance to every point of the group (up to a few
// rounding errors, which the host's margin in r2 covers), so a skipped group holds no point the
// obstacle pass could count: no minimum changes.
template <int K>
__device__ __forceinline__ uint64_t group_mask(const v4f *boxes, int ng, float x, float y,
                                               float r2, int q)
{
    static_assert(64 % K == 0 && K <= 16, "whole samples per wavefront");
    constexpr int R = 64 / K;      // rounds for a full segment; a partial one stops early
    constexpr int RB = 8;          // rounds whose boxes are held in registers at once
    uint64_t need = 0;
    // One round: the K lanes of every sample test boxes r K .. r K + K - 1.
    auto round = [&](const v4f b, int r) {
        const float ex = fmaxf(fmaxf(b.x - x, x - b.z), 0.0f);
        const float ey = fmaxf(fmaxf(b.y - y, y - b.w), 0.0f);
        const float d2 = fmaf(ex, ex, ey * ey);
        uint64_t m = __ballot(!(d2 > r2));       // NaN counts as near
#pragma unroll
        for (int sh = 32; sh >= K; sh >>= 1) m |= m >> sh;
        need |= (m & ((1ull << K) - 1)) << (r * K);
    };
    // The boxes of up to RB rounds are read first (in bounds), so the reads overlap; the empty asm
    // at the end uses them on every path, which keeps the compiler from moving a read past an
    // early exit. With fewer lanes per sample (more rounds) they are read RB rounds at a time,
    // which keeps the box registers at 4 RB.
    if constexpr (R <= RB) {
        v4f bx[R];
#pragma unroll
        for (int r = 0; r < R; ++r) bx[r] = boxes[r * K + q];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r * K >= ng) break;
            round(bx[r], r);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) asm volatile("" ::"v"(bx[r].x));
    } else {
        for (int r0 = 0; r0 < R && r0 * K < ng; r0 += RB) {
            v4f bx[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) bx[r] = boxes[(r0 + r) * K + q];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if ((r0 + r) * K >= ng) break;
                round(bx[r], r0 + r);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) asm volatile("" ::"v"(bx[r].x));
        }
    }
    return ng >= 64 ? need : need & ((1ull << ng) - 1);
}

// The obstacle pass of one lane over the groups of a tile segment marked in `need`, against one
// pose. The K = STRIDE lanes of a sample split the points: chunk c of the segment is the lane's
// pairs p[(c G + g) STRIDE], g < G, so one wavefront instruction reads K consecutive pairs (K x 16
// bytes on distinct banks), each broadcast to the 64 / K samples of the wavefront; a group is
// CPG chunks. The chunks of the marked groups are visited in order with two register groups of
// G pairs that alternate: one is read while the other is tested, so the LDS latency hides behind
// the arithmetic even at one wavefront per SIMD (G = 4 at one or two wavefronts per SIMD, 2 at
// three, where registers are short). The empty asm statements consume a group (forcing its wait
// there), and the scheduling barriers keep the compiler from sinking the reads next to their
// uses. The walk over the mask is wavefront-uniform (scalar) control: with one chunk per group,
// a find-first-set and a bit clear per chunk. In the general walk the last step reads the
// current chunk again instead of a next one (in bounds, unused).
template <int G, int GP, bool CENTRED, int STRIDE>
__device__ __forceinline__ void point_pass_groups(const Pose &pose, const v4f *p, uint64_t need,
                                                  float &mm, float &md)
{
    constexpr int CPG = GP / (STRIDE * G);
    static_assert(CPG >= 1 && CPG * STRIDE * G == GP, "whole chunks per group");
    if (!need) return;
    if constexpr (CPG == 1) {
        // one chunk per group: the walk is a find-first-set and a bit clear per chunk
        int j = __builtin_ctzll(need);
        need &= ~(1ull << j);
        v4f a[G], b[G];
#pragma unroll
        for (int g = 0; g < G; ++g) a[g] = p[(j * G + g) * STRIDE];
        for (;;) {
            if constexpr (G == 4) asm volatile("" ::"v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]));
            else asm volatile("" ::"v"(a[0]), "v"(a[1]));
            if (!need) {
#pragma unroll
                for (int g = 0; g < G; ++g) pose.pair<CENTRED>(a[g], mm, md);
                return;
            }
            j = __builtin_ctzll(need);
            need &= ~(1ull << j);
#pragma unroll
            for (int g = 0; g < G; ++g) b[g] = p[(j * G + g) * STRIDE];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < G; ++g) pose.pair<CENTRED>(a[g], mm, md);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (G == 4) asm volatile("" ::"v"(b[0]), "v"(b[1]), "v"(b[2]), "v"(b[3]));
            else asm volatile("" ::"v"(b[0]), "v"(b[1]));
            if (!need) {
#pragma unroll
                for (int g = 0; g < G; ++g) pose.pair<CENTRED>(b[g], mm, md);
                return;
            }
            j = __builtin_ctzll(need);
            need &= ~(1ull << j);
#pragma unroll
            for (int g = 0; g < G; ++g) a[g] = p[(j * G + g) * STRIDE];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < G; ++g) pose.pair<CENTRED>(b[g], mm, md);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    int j = __builtin_ctzll(need);
    need &= need - 1;
    int ca = j * CPG, end = ca + CPG, cb;
    v4f a[G], b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) a[g] = p[(ca * G + g) * STRIDE];
    for (;;) {
        if constexpr (G == 4) asm volatile("" ::"v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]));
        else asm volatile("" ::"v"(a[0]), "v"(a[1]));
        bool more = true;
        cb = ca + 1;
        if (cb == end) {
            if (need) {
                j = __builtin_ctzll(need);
                need &= need - 1;
                cb = j * CPG;
                end = cb + CPG;
            } else {
                more = false;
                cb = ca;
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) b[g] = p[(cb * G + g) * STRIDE];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < G; ++g) pose.pair<CENTRED>(a[g], mm, md);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (G == 4) asm volatile("" ::"v"(b[0]), "v"(b[1]), "v"(b[2]), "v"(b[3]));
        else asm volatile("" ::"v"(b[0]), "v"(b[1]));
        if (!more) break;
        ca = cb + 1;
        if (ca == end) {
            if (need) {
                j = __builtin_ctzll(need);
                need &= need - 1;
                ca = j * CPG;
                end = ca + CPG;
            } else {
                more = false;
                ca = cb;
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) a[g] = p[(ca * G + g) * STRIDE];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < G; ++g) pose.pair<CENTRED>(b[g], mm, md);
        __builtin_amdgcn_sched_barrier(0);
        if (!more) {
            if constexpr (G == 4) asm volatile("" ::"v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]));
            else asm volatile("" ::"v"(a[0]), "v"(a[1]));
            break;
        }
    }
}

// Asynchronous copy of `cnt` 16-byte entries (point pairs or group boxes) from global memory
// into an LDS buffer, in chunks of 64: each wavefront instruction moves one chunk, lane l entry l
// of it, with no register staging. The source is a buffer resource of exactly `cnt` entries (in
// scalar registers), so the lanes of a last partial chunk read zeros, never memory past the
// table, and the lane's byte offset is the only vector register the copies hold. Chunk c is
// moved by wavefront (first + c) mod WAVES (`wave` is wavefront-uniform). Completion is awaited
// with vmcnt before the barrier that publishes the buffer.
template <int WAVES>
__device__ __forceinline__ void copy_entries(const v4f *src, v4f *dst, int cnt, int first,
                                             int wave)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<v4f *>(src), 0, cnt * 16, BUFFER_RSRC_FLAGS);
    const unsigned vo = (threadIdx.x & 63) * 16u;
    for (int c = (wave - first + WAVES) % WAVES; c * CHUNK < cnt; c += WAVES)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            r, (__attribute__((address_space(3))) void *)(dst + c * CHUNK), 16, vo,
            c * CHUNK * 16, 0, 0);
}

__device__ __forceinline__ void wait_copies()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), other counters untouched
}

// ---------------------------------------------------------------------------------------------
// 2. The rollout of every sample.
//
// A workgroup of RB threads (the launch shape's) holds S = RB / K samples; a sample occupies K
// adjacent lanes of one wavefront, which split its weights for the controller and its points for
// the obstacle pass: lane q of a sample tests pairs q, q + K, q + 2K, ... of every tile against
// the sample's own pose (every lane holds the sample's state), and the K partial minima meet
// through DPP (exact mins: the result does not depend on K). Each step's extrapolated points
// stream into one of two LDS buffers (at most TP pairs at a time) while the other one
// is being tested; one barrier per tile publishes a buffer and frees the other. For K >= 8 the
// workgroup's LDS also holds one slot per sample through which the controller's second hidden
// layer receives its inputs.
// ---------------------------------------------------------------------------------------------
constexpr int rollout_block(int K) { return 256; }
// One or two lanes per sample serve the small networks, whose registers allow more wavefronts
// than two 64 KiB buffers per workgroup would: they take 1024-pair tiles (four workgroups per CU).
constexpr int tile_pairs(int K) { return K >= 16 ? 1536 : K <= 2 ? 1024 : TILE_PAIRS; }
#ifndef NNP_K8_GROUP_PAIRS
#define NNP_K8_GROUP_PAIRS 16
#endif
constexpr int group_pairs(int K) { return K == 8 ? NNP_K8_GROUP_PAIRS : MAX_GROUP_PAIRS; }

// Launch shape of the rollout kernels: K lanes per sample, RB threads per workgroup, TP point
// pairs per LDS buffer, GP pairs per point group (the defaults above per K; the batch autotuner
// chooses among the compiled shapes). G pairs per lane form one register group of the obstacle
// pass: four, or two where a group has fewer pairs per lane or registers are short. Every shape
// computes the same bits: minima are exact and the controller's sums do not depend on K.
template <int K_, int RB_ = rollout_block(K_), int TP_ = tile_pairs(K_), int GP_ = group_pairs(K_)>
struct Shape {
    static constexpr int K = K_, RB = RB_, TP = TP_, GP = GP_;
    static constexpr int G = GP / K >= 4 ? 4 : 2;
    static constexpr int WPE = K_ >= 16 ? 3 : 1;     // wavefronts per SIMD the build aims for
    static_assert(RB % 64 == 0 && RB % K == 0 && TP % CHUNK == 0, "whole wavefronts and chunks");
    static_assert(GP <= MAX_GROUP_PAIRS && GP % (K * G) == 0 && TP % GP == 0,
                  "whole register groups per point group, whole groups per tile");
};

// LDS of one rollout workgroup.
template <class NetT, class SH>
struct RolloutShared {
    static constexpr int TP = SH::TP;
    // Hidden-layer slots, one per sample, ACT floats each at a stride padded by four floats so
    // that the float4 reads of the slots in one wavefront start on different banks.
    static constexpr int ACT = Controller<NetT, SH::K>::ACT;
    static constexpr int ACT_STRIDE = ACT ? ACT + 4 : 0;
    v4f pbuf[2][TP];                 // point pairs of the current / next tile
    // their groups' boxes (whole copy chunks: a copy moves CHUNK entries)
    static constexpr int BOXES = (TP / SH::GP + CHUNK - 1) / CHUNK * CHUNK;
    v4f bbuf[2][BOXES];
    float act[ACT ? SH::RB / SH::K * ACT_STRIDE : 4];
};

// The rollout of samples [tile * S, tile * S + S) of one problem by one workgroup.
// CENTRED: the model's rectangle is centred on the reference point (oc = 0); see Pose::point.
template <class NetT, class SH, int MODE, bool CENTRED>
__device__ __forceinline__ void rollout_tile(const RolloutArgs &a, int tile,
                                             RolloutShared<NetT, SH> &sh)
{
    constexpr int K = SH::K;
    constexpr int RB = SH::RB;
    constexpr int S = RB / K;
    constexpr int WAVES = RB / 64;
    constexpr int TP = SH::TP;
    static_assert(ThetaSource::STAGE * RB <= 8 * TP, "weight staging fits the buffers");
    auto &pbuf = sh.pbuf;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = (tid & 63) % K;
    const int slot = tid / K;
    const int sample = tile * S + slot;
    const bool active = sample < a.N;
    const int si = active ? sample : a.N - 1;

    SampleSim<NetT, K> sim;
    sim.ctl.load(make_source<NetT>(a, si), q, reinterpret_cast<float *>(&pbuf[0][0]), tid, RB);
    sim.init(a.z0, a.a_prev);
    __syncthreads();

    const int P2 = a.P2;
    const int ntile = (P2 + TP - 1) / TP;                      // 0 when there are no points
    const v4f *ext = reinterpret_cast<const v4f *>(a.ext);
    constexpr int GP = SH::GP;
    const int NG = P2 / GP;                                    // groups per step
    constexpr int TG = TP / GP;                                // groups per full tile
    const v4f *bbs = reinterpret_cast<const v4f *>(a.bb);
    const bool cull = a.cull_r2 < INFINITY;
    auto copy_tile = [&](int h, int t, int buf) {
        const int n = min(TP, P2 - t * TP);
        copy_entries<WAVES>(ext + (size_t)h * P2 + (size_t)t * TP, pbuf[buf], n, 0, wave);
        if (cull)   // the boxes by the last wavefronts: the point chunks start at the first
            copy_entries<WAVES>(bbs + (size_t)h * NG + (size_t)t * TG, sh.bbuf[buf],
                                n / GP, WAVES - 1, wave);
    };
    if (ntile > 0) copy_tile(0, 0, 0);

    // Plan-mode records (when a.rec_ctrl is set) through a buffer resource: base and range in
    // scalar registers, a 32-bit lane offset, the step's offset as a scalar (the host keeps the
    // records below 2^31 bytes). Only the applied controls are recorded: the winner's states
    // follow from z0 and them by the model step alone (gather_kernel), bit for bit.
    const bool rec_on = MODE == MODE_PLAN && a.rec_ctrl != nullptr;
    const __amdgpu_buffer_rsrc_t rec_c = __builtin_amdgcn_make_buffer_rsrc(
        a.rec_ctrl, 0, rec_on ? a.N * a.T * 8 : 0, BUFFER_RSRC_FLAGS);
    // Step h's record: a_{h-1} (the controls the model applied last, still held for the
    // features). Issued right after the step's first wait for the copies, so the store retires
    // under the point pass instead of delaying the next wait (stores count in vmcnt).
    auto record = [&](int h) {
        if (rec_on && active && q == 0 && h > 0)
            __builtin_amdgcn_raw_buffer_store_b64(
                u32x2{__float_as_uint(sim.ap0), __float_as_uint(sim.ap1)}, rec_c, sample * 8,
                (h - 1) * a.N * 8, 0);
    };

    // Culling threshold of a step (per sample): the cull radius, lowered by a bound on the
    // step's nearest squared distance. The point p that was nearest at the previous step (or any
    // point at that distance) is now at most sqrt(md) + |dz| + disp away, where |dz| <= |v|
    // step_scale (plus half an ulp of x and y) is the sample's move and disp the points' move.
    // A group whose box is farther than that bound holds no point nearer than p, and p's own
    // group is never skipped, so the minimum over the tested points is the minimum over all;
    // the collision radius is kept as a floor, so no point that could be inside is skipped.
    // The factor 1.00001 covers the rounding of the bound, of the box distance and of the
    // points' squared distances (a few float ulps each).
    const float disp = cull ? *a.disp : INFINITY;
    float bnd = INFINITY;
    // work counter of the wavefront (wavefront-uniform), added to a.stats once at the end
    unsigned long long n_tested = 0, n_groups = 0;

    int it = 0;
    for (int h = 0; h <= a.T; ++h) {
        const Pose pose = sim.begin_step(a.m);
        const float thr = bnd < a.cull_r2 ? fmaxf(a.coll_r2, bnd) : a.cull_r2;
        float mm = INFINITY, md = INFINITY;
        for (int t = 0; t < ntile; ++t, ++it) {
            wait_copies();
            __syncthreads();            // buffer it & 1 ready; everyone is done with the other
            // the next tile in sequence streams into the other buffer: tile t + 1 of this step,
            // else the first tile of the next step
            if (t + 1 < ntile) copy_tile(h, t + 1, (it + 1) & 1);
            else if (h < a.T) copy_tile(h + 1, 0, (it + 1) & 1);
            if constexpr (MODE == MODE_PLAN)
                if (t == 0) record(h);
            // the tile's groups in segments of at most 64 (one mask word each)
            const int ngt = min(TP, P2 - t * TP) / GP;
            for (int g0 = 0; g0 < ngt; g0 += 64) {
                const int ng = min(64, ngt - g0);
                const uint64_t need =
                    cull ? group_mask<K>(sh.bbuf[it & 1] + g0, ng, pose.x, pose.y, thr, q)
                         : (ng >= 64 ? ~0ull : (1ull << ng) - 1);
                n_tested += (unsigned long long)__builtin_popcountll(need);
                n_groups += (unsigned long long)ng;
                point_pass_groups<SH::G, GP, CENTRED, K>(pose, pbuf[it & 1] + g0 * GP + q,
                                                         need, mm, md);
            }
        }
        if constexpr (MODE == MODE_PLAN)
            if (ntile == 0) record(h);
        mm = group_min<K>(mm);
        md = group_min<K>(md);
        if (cull) {
            const float reach = sqrtf(md) + fmaf(fabsf(sim.v), a.step_scale, disp) +
                                (fabsf(sim.x) + fabsf(sim.y)) * 0x1p-22f;
            bnd = reach * reach * 1.00001f;    // +INFINITY or NaN: the radius alone next step
        }
        sim.record_collision(h, mm);
        if constexpr (MODE == MODE_OUT) {
            if (a.traj && active && q == 0) {
                float *o = a.traj + ((size_t)sample * (a.T + 1) + h) * 4;
                *reinterpret_cast<float4 *>(o) = make_float4(sim.x, sim.y, sim.phi, sim.v);
            }
        }
        if (h < a.T) {
            float a0, a1;
            constexpr int ACT_STRIDE = RolloutShared<NetT, SH>::ACT_STRIDE;
            sim.template advance<(ACT_STRIDE > 0)>(a.m, a.goal, md, a0, a1, q,
                                                   sh.act + slot * ACT_STRIDE);
            if constexpr (MODE == MODE_OUT) {
                if (a.controls && active && q == 0) {
                    float *o = a.controls + ((size_t)sample * a.T + h) * 2;
                    *reinterpret_cast<float2 *>(o) = make_float2(a0, a1);
                }
            }
        }
    }

    if (a.stats && (tid & 63) == 0) {
        atomicAdd(a.stats, n_tested);
        atomicAdd(a.stats + 1, n_groups);
    }
    const float J = sim.cost(a.m, a.goal);
    if constexpr (MODE == MODE_PLAN) {
        unsigned long long key = ~0ull;
        if (active && q == 0)
            key = ((unsigned long long)__float_as_uint(J) << 32) | (unsigned int)sample;
        key = wave_min_u64(key);
        if ((tid & 63) == 0 && key != ~0ull) atomicMin(a.best_key, key);
    } else {
        if (active && q == 0) {
            if (a.cost) a.cost[sample] = J;
            if (a.collided) a.collided[sample] = sim.first >= 0;
            if (a.first) a.first[sample] = sim.first;
            if (a.min_margin) a.min_margin[sample] = sim.min_margin;
        }
    }
}


template <class NetT, class SH, int MODE, bool CENTRED>
__global__ __launch_bounds__(SH::RB)
__attribute__((amdgpu_waves_per_eu(SH::WPE))) void rollout_kernel(const RolloutArgs a)
{
    __shared__ RolloutShared<NetT, SH> sh;
    rollout_tile<NetT, SH, MODE, CENTRED>(a, blockIdx.x, sh);
}

// Many problems of uneven size in one launch: one workgroup per work item (problem, tile of S
// samples). The host writes the items longest problems first and the dispatcher starts
// workgroups in grid order, so short problems fill the tail. The item index comes from
// blockIdx, so the problem descriptor is read with scalar loads, like a kernel argument.
template <class NetT, class SH, bool CENTRED>
__global__ __launch_bounds__(SH::RB)
__attribute__((amdgpu_waves_per_eu(SH::WPE))) void rollout_batch_kernel(
    const RolloutArgs *__restrict__ probs, const int2 *__restrict__ items)
{
    __shared__ RolloutShared<NetT, SH> sh;
    const int2 item = items[blockIdx.x];
    rollout_tile<NetT, SH, MODE_PLAN, CENTRED>(probs[item.x], item.y, sh);
}

// ---------------------------------------------------------------------------------------------
// 3. Winner replay: every lane simulates the best sample; points are split over the workgroup
//    and reduced exactly (min), so the replay reproduces the rollout bit for bit.
// ---------------------------------------------------------------------------------------------
template <class NetT, int K>
__device__ __forceinline__ void replay_body(const RolloutArgs &a, const ReplayOut &o,
                                            float (&red)[2][BLOCK / 64], float *stage)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane % K;
    const unsigned long long key = *a.best_key;
    int best = (int)(unsigned int)(key & 0xffffffffull);
    if (key == ~0ull || best >= a.N) best = 0;
    const float key_cost = __uint_as_float((unsigned int)(key >> 32));

    const ThetaSource src = make_source<NetT>(a, best);
    SampleSim<NetT, K> sim;
    sim.ctl.load(src, q, stage, tid, BLOCK);
    sim.init(a.z0, a.a_prev);
    for (int h = 0; h <= a.T; ++h) {
        const Pose pose = sim.begin_step(a.m);
        float mm = INFINITY, md = INFINITY;
        const v4f *pts = reinterpret_cast<const v4f *>(a.ext) + (size_t)h * a.P2;
        for (int pi = tid; pi < a.P2; pi += BLOCK) pose.pair(pts[pi], mm, md);
        mm = wave_min_f(mm);
        md = wave_min_f(md);
        if (lane == 0) {
            red[0][wave] = mm;
            red[1][wave] = md;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            mm = fminf(mm, red[0][w]);
            md = fminf(md, red[1][w]);
        }
        __syncthreads();
        sim.record_collision(h, mm);
        if (tid == 0 && o.traj)
            *reinterpret_cast<float4 *>(o.traj + 4 * (size_t)h) =
                make_float4(sim.x, sim.y, sim.phi, sim.v);
        if (h < a.T) {
            float a0, a1;
            sim.advance(a.m, a.goal, md, a0, a1, q);
            if (tid == 0) {
                if (o.controls) {
                    o.controls[2 * h] = a0;
                    o.controls[2 * h + 1] = a1;
                }
                if (o.controls_phys) {
                    o.controls_phys[2 * h] = a.m.delta_max * a0;
                    o.controls_phys[2 * h + 1] = fmaf(a1 + 1.0f, a.m.u_half_range, a.m.u_min);
                }
            }
        }
    }
    if (tid == 0) {
        if (o.cost) o.cost[0] = sim.cost(a.m, a.goal);
        if (o.best_index) o.best_index[0] = best;
        if (o.status) o.status[0] = isinf(key_cost) ? NNP_INFEASIBLE : NNP_OK;
        if (o.goal_reached) {
            sim.begin_step(a.m);
            o.goal_reached[0] = sim.goal_reached(a.m, a.goal);
        }
    }
    if (o.theta)
        for (int k = tid; k < NetT::NTHETA; k += BLOCK) o.theta[k] = src.one(k);
}

template <class NetT, int K>
__global__ __launch_bounds__(BLOCK) void replay_kernel(const RolloutArgs a, const ReplayOut o)
{
    __shared__ float red[2][BLOCK / 64];
    __shared__ float stage[ThetaSource::STAGE * BLOCK];
    replay_body<NetT, K>(a, o, red, stage);
}

template <class NetT, int K>
__global__ __launch_bounds__(BLOCK) void replay_batch_kernel(const RolloutArgs *probs,
                                                             const ReplayOut *outs)
{
    __shared__ float red[2][BLOCK / 64];
    __shared__ float stage[ThetaSource::STAGE * BLOCK];
    replay_body<NetT, K>(probs[blockIdx.x], outs[blockIdx.x], red, stage);
}

// The winner's outputs from the records the rollout wrote (the same values the replay computes:
// the records are the rollout's own states and controls, the cost is the argmin key's), by one
// workgroup.
template <class NetT>
__device__ __forceinline__ void gather_body(const RolloutArgs &a, const ReplayOut &o)
{
    const int tid = threadIdx.x;
    const unsigned long long key = *a.best_key;
    int best = (int)(unsigned int)(key & 0xffffffffull);
    if (key == ~0ull || best >= a.N) best = 0;
    const float key_cost = __uint_as_float((unsigned int)(key >> 32));
    // The winner's states from z0 and its recorded controls by the model step's own functions
    // (same inputs, same operations, hence the same bits as in the rollout), reordered so that
    // little stays sequential: the steering tangents and, once the heading and speed chain is
    // known, every step's sincos are computed in parallel; the position chain comes last, and the
    // trajectory is written out by the whole workgroup. Staged in LDS (T <= NNP_MAX_T).
    __shared__ float2 ctl[NNP_MAX_T];
    __shared__ float tds[NNP_MAX_T];
    __shared__ float phis[NNP_MAX_T + 1], vs[NNP_MAX_T + 1], cs[NNP_MAX_T + 1], sn[NNP_MAX_T + 1];
    __shared__ float2 xys[NNP_MAX_T + 1];
    const int T = a.T;
    for (int h = tid; h < T; h += BLOCK) {
        const float2 c = a.rec_ctrl[(size_t)h * a.N + best];
        ctl[h] = c;
        tds[h] = tanf(a.m.delta_max * c.x);
        if (o.controls) {
            o.controls[2 * h] = c.x;
            o.controls[2 * h + 1] = c.y;
        }
        if (o.controls_phys) {
            o.controls_phys[2 * h] = a.m.delta_max * c.x;
            o.controls_phys[2 * h + 1] = fmaf(c.y + 1.0f, a.m.u_half_range, a.m.u_min);
        }
    }
    __syncthreads();
    // The two chains run in one lane, CH steps at a time: a full chunk's inputs are read from LDS
    // together before its steps, so its dependent steps wait for LDS once; the last steps (fewer
    // than CH) go one by one.
    constexpr int CH = 8;
    const int TF = T / CH * CH;
    if (tid == 0) {
        float phi = a.z0[2], v = a.z0[3];
        phis[0] = phi;
        vs[0] = v;
        for (int h0 = 0; h0 < TF; h0 += CH) {
            float cy[CH], td[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                cy[k] = ctl[h0 + k].y;
                td[k] = tds[h0 + k];
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                heading_speed_step<true>(a.m, cy[k], td[k], phi, v);
                phis[h0 + k + 1] = phi;
                vs[h0 + k + 1] = v;
            }
        }
        for (int h = TF; h < T; ++h) {
            heading_speed_step<true>(a.m, ctl[h].y, tds[h], phi, v);
            phis[h + 1] = phi;
            vs[h + 1] = v;
        }
    }
    __syncthreads();
    for (int h = tid; h <= T; h += BLOCK) {
        float sv, cv;
        sincosf(phis[h], &sv, &cv);
        sn[h] = sv;
        cs[h] = cv;
    }
    __syncthreads();
    if (tid == 0) {
        float x = a.z0[0], y = a.z0[1];
        for (int h0 = 0; h0 < TF; h0 += CH) {
            float td[CH], c[CH], sv[CH], vv[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                td[k] = tds[h0 + k];
                c[k] = cs[h0 + k];
                sv[k] = sn[h0 + k];
                vv[k] = vs[h0 + k];
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                xys[h0 + k] = make_float2(x, y);
                position_step(a.m, td[k], c[k], sv[k], vv[k], x, y);
            }
        }
        for (int h = TF; h < T; ++h) {
            xys[h] = make_float2(x, y);
            position_step(a.m, tds[h], cs[h], sn[h], vs[h], x, y);
        }
        xys[T] = make_float2(x, y);
        if (o.goal_reached)
            o.goal_reached[0] = within_tolerance(a.m.eps_xi, a.m.eps_eta, a.m.eps_phi, a.m.eps_v,
                                                 a.goal, x, y, phis[T], vs[T], cs[T], sn[T]);
        if (o.cost) o.cost[0] = key_cost;
        if (o.best_index) o.best_index[0] = best;
        if (o.status) o.status[0] = isinf(key_cost) ? NNP_INFEASIBLE : NNP_OK;
    }
    if (o.theta) {
        const ThetaSource src = make_source<NetT>(a, best);
        for (int k = tid; k < NetT::NTHETA; k += BLOCK) o.theta[k] = src.one(k);
    }
    __syncthreads();
    if (o.traj)
        for (int h = tid; h <= T; h += BLOCK)
            reinterpret_cast<float4 *>(o.traj)[h] = make_float4(xys[h].x, xys[h].y, phis[h], vs[h]);
}

template <class NetT>
__global__ __launch_bounds__(BLOCK) void gather_kernel(const RolloutArgs a, const ReplayOut o)
{
    gather_body<NetT>(a, o);
}

// One workgroup per problem of a batch whose records fit.
template <class NetT>
__global__ __launch_bounds__(BLOCK) void gather_batch_kernel(const RolloutArgs *probs,
                                                             const ReplayOut *outs)
{
    gather_body<NetT>(probs[blockIdx.x], outs[blockIdx.x]);
}

__global__ __launch_bounds__(BLOCK) void theta_kernel(PhiloxKey key, uint32_t inst, uint32_t i0,
                                                      uint32_t N, uint32_t nt,
                                                      const float *__restrict__ mu,
                                                      const float *__restrict__ log_sigma,
                                                      float *__restrict__ out)
{
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= (long long)N * nt) return;
    const uint32_t i = (uint32_t)(gid / nt), k = (uint32_t)(gid % nt);
    ThetaSource src;
    src.explicit_theta = nullptr;
    src.mu = mu;
    src.log_sigma = log_sigma;
    src.n_theta = (int)nt;
    src.key = key;
    src.inst = inst;
    src.sample = i0 + i;
    out[gid] = src.one((int)k);
}

// ---------------------------------------------------------------------------------------------
// Dispatch table over the compiled network shapes and lane layouts.
// ---------------------------------------------------------------------------------------------
struct Variant {
    int widths[NNP_MAX_LAYERS + 1];
    int n_layers, feature_set, K, block, tile, gp, ntheta;
    void (*launch_rollout)(const RolloutArgs &, int mode, dim3 grid, hipStream_t);
    void (*launch_replay)(const RolloutArgs &, const ReplayOut &, hipStream_t);
    void (*launch_rollout_batch)(const RolloutArgs *, const int2 *, int n_items, bool centred,
                                 hipStream_t);
    void (*launch_replay_batch)(const RolloutArgs *, const ReplayOut *, int count, hipStream_t);
    void (*launch_gather)(const RolloutArgs &, const ReplayOut &, hipStream_t);
    void (*launch_gather_batch)(const RolloutArgs *, const ReplayOut *, int count, hipStream_t);
};

template <class NetT, class SH>
void launch_rollout_t(const RolloutArgs &a, int mode, dim3 grid, hipStream_t s)
{
    const dim3 block(SH::RB);
    const bool centred = a.m.oc == 0.0f;
    if (mode == MODE_PLAN && centred)
        hipLaunchKernelGGL((rollout_kernel<NetT, SH, MODE_PLAN, true>), grid, block, 0, s, a);
    else if (mode == MODE_PLAN)
        hipLaunchKernelGGL((rollout_kernel<NetT, SH, MODE_PLAN, false>), grid, block, 0, s, a);
    else if (centred)
        hipLaunchKernelGGL((rollout_kernel<NetT, SH, MODE_OUT, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((rollout_kernel<NetT, SH, MODE_OUT, false>), grid, block, 0, s, a);
}

template <class NetT, int K>
void launch_replay_t(const RolloutArgs &a, const ReplayOut &o, hipStream_t s)
{
    hipLaunchKernelGGL((replay_kernel<NetT, K>), dim3(1), dim3(BLOCK), 0, s, a, o);
}

template <class NetT, class SH>
void launch_rollout_batch_t(const RolloutArgs *probs, const int2 *items, int n_items,
                            bool centred, hipStream_t s)
{
    if (centred)
        hipLaunchKernelGGL((rollout_batch_kernel<NetT, SH, true>), dim3(n_items), dim3(SH::RB),
                           0, s, probs, items);
    else
        hipLaunchKernelGGL((rollout_batch_kernel<NetT, SH, false>), dim3(n_items), dim3(SH::RB),
                           0, s, probs, items);
}

template <class NetT, int K>
void launch_replay_batch_t(const RolloutArgs *probs, const ReplayOut *outs, int count,
                           hipStream_t s)
{
    hipLaunchKernelGGL((replay_batch_kernel<NetT, K>), dim3(count), dim3(BLOCK), 0, s, probs,
                       outs);
}

template <class NetT>
void launch_gather_t(const RolloutArgs &a, const ReplayOut &o, hipStream_t s)
{
    hipLaunchKernelGGL((gather_kernel<NetT>), dim3(1), dim3(BLOCK), 0, s, a, o);
}

template <class NetT>
void launch_gather_batch_t(const RolloutArgs *probs, const ReplayOut *outs, int count,
                           hipStream_t s)
{
    hipLaunchKernelGGL((gather_batch_kernel<NetT>), dim3(count), dim3(BLOCK), 0, s, probs, outs);
}

#define NNP_SHAPED(NIN, H1, H2, FEAT, SH)                                                         \
    {{NIN, H1, (H2) ? (H2) : 2, (H2) ? 2 : 0}, (H2) ? 3 : 2, FEAT, SH::K, SH::RB, SH::TP, SH::GP,  \
     Net<NIN, H1, H2, FEAT>::NTHETA, launch_rollout_t<Net<NIN, H1, H2, FEAT>, SH>,                 \
     launch_replay_t<Net<NIN, H1, H2, FEAT>, SH::K>,                                               \
     launch_rollout_batch_t<Net<NIN, H1, H2, FEAT>, SH>,                                           \
     launch_replay_batch_t<Net<NIN, H1, H2, FEAT>, SH::K>,                                         \
     launch_gather_t<Net<NIN, H1, H2, FEAT>>, launch_gather_batch_t<Net<NIN, H1, H2, FEAT>>}
#define NNP_VARIANT(NIN, H1, H2, FEAT, K) NNP_SHAPED(NIN, H1, H2, FEAT, Shape<K>)

using ShapeWideTile = Shape<8, 512, 4096>;      // one LDS buffer holds an 8192-point step
using ShapeFullBlock = Shape<8, 512, 2048>;     // one 512-thread workgroup per CU

// The first listed shape of a network is its default.
const Variant kVariants[] = {
    NNP_VARIANT(8, 32, 32, NNP_FEAT_EIGHT, 8),   // 8-32-32-2, 1410 parameters (default: two
    NNP_VARIANT(8, 32, 32, NNP_FEAT_EIGHT, 4),   // 256-thread workgroups per CU, 8 lanes/sample)
    NNP_VARIANT(8, 32, 32, NNP_FEAT_EIGHT, 16),
    NNP_SHAPED(8, 32, 32, NNP_FEAT_EIGHT, ShapeWideTile),
    NNP_SHAPED(8, 32, 32, NNP_FEAT_EIGHT, ShapeFullBlock),
    NNP_VARIANT(6, 16, 0, NNP_FEAT_SIX, 1),      // 6-16-2, 146 parameters
    NNP_VARIANT(6, 16, 0, NNP_FEAT_SIX, 2),
    NNP_VARIANT(6, 16, 0, NNP_FEAT_SIX, 4),
    NNP_VARIANT(5, 2, 0, NNP_FEAT_PAPER, 1),     // NN-[5,2,2]
    NNP_VARIANT(5, 10, 0, NNP_FEAT_PAPER, 1),    // NN-[5,10,2]
    NNP_VARIANT(5, 10, 10, NNP_FEAT_PAPER, 1),   // NN-[5,10,10,2]
};

const Variant *find_variant(const nnp_model *m, int K, int block, int tile)
{
    for (const Variant &v : kVariants) {
        if (v.n_layers != m->n_layers || v.feature_set != m->feature_set) continue;
        bool same = true;
        for (int l = 0; l <= m->n_layers; ++l) same = same && v.widths[l] == m->widths[l];
        if (!same) continue;
        if ((K == 0 || K == v.K) && (block == 0 || block == v.block) &&
            (tile == 0 || tile == v.tile))
            return &v;   // the first listed shape that matches the request
    }
    return nullptr;
}

thread_local std::string g_create_error;

// Allocation-free planning (nnp_plan_noalloc): the argmin key (first 256 bytes) and the
// extrapolation table live in one file-scope device array. Each GPU holds its own copy at its own
// address, resolved once per device with hipGetSymbolAddress while that device is current; host
// code uses only that address (the array's name is a host-side stand-in, not a device pointer).
constexpr size_t NOALLOC_KEY_BYTES = 256;
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

}  // namespace

static __device__ __align__(256) unsigned char scratch[NNP_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of the current device's copy of `scratch` (the caller has made `device`
// current).
hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

bool finite_f(float v) { return isfinite(v); }

}  // namespace

struct nnp_handle {
    nnp_model model;
    DevModel dm;
    const Variant *var;
    int device;
    unsigned long long *d_key = nullptr;
    float4 *d_ext = nullptr;           // extrapolation table, group boxes, spatial order
    size_t ext_bytes = 0;
    CullConsts cull;                   // culling constants of the model (cull_consts)
    unsigned long long *d_stats = nullptr;   // culling work counter (nnp_set_cull_stats)
    bool stats = false;
    // per-sample records of nnp_plan (states and controls of every sample)
    void *d_rec = nullptr;
    size_t rec_bytes = 0;
    uint64_t rec_limit = 1ull << 32;
    uint64_t ws_limit = UINT64_MAX;    // cap on the grown device workspace (all buffers above)
    // batched planning: tables, keys, descriptors (device and pinned host)
    void *d_bext = nullptr, *d_bkeys = nullptr, *d_bmeta = nullptr, *h_bmeta = nullptr;
    size_t bext_bytes = 0, bkeys_bytes = 0, bmeta_bytes = 0, hmeta_bytes = 0;
    hipEvent_t meta_copied = nullptr;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double acc_ms = 0.0;
    int64_t launches = 0;
    void *scratch = nullptr;           // this device's copy of the file-scope scratch array
    std::string err;
};

namespace {

int fail(nnp_handle *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

// Fixed messages: copied into the handle's error string (capacity reserved by nnp_create, so
// validation allocates no host memory).
int fail(nnp_handle *h, int code, const char *msg)
{
    if (h) h->err.assign(msg);
    else g_create_error = msg;
    return code;
}

int hip_fail(nnp_handle *h, hipError_t e, const char *what)
{
    return fail(h, NNP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Error paths of the allocation-free entry point: the message is copied into the handle's error
// string, whose capacity nnp_create reserves, so that no host memory is allocated either.
int fail_fixed(nnp_handle *h, int code, const char *msg, const char *detail = nullptr)
{
    h->err.assign(msg);
    if (detail) {
        h->err.append(": ");
        h->err.append(detail);
    }
    return code;
}

int check_model(const nnp_model *m, std::string &why)
{
    const float pos[] = {m->dt, m->front + m->rear, m->half_width, m->lf + m->lr, m->delta_max,
                         m->norm_xi, m->norm_eta, m->norm_phi, m->norm_v, m->d_cap};
    for (float f : pos)
        if (!(f > 0.0f) || !finite_f(f)) {
            why = "model constants dt, front+rear, half_width, lf+lr, delta_max, norms and d_cap "
                  "must be finite and positive";
            return NNP_EINVAL;
        }
    const float fin[] = {m->lf, m->lr, m->front, m->rear, m->delta_rate_max, m->u_min, m->u_max,
                         m->effort_weight, m->eps_xi, m->eps_eta, m->eps_phi, m->eps_v,
                         m->goal_heading_weight, m->goal_speed_weight};
    for (float f : fin)
        if (!finite_f(f)) {
            why = "model constants must be finite";
            return NNP_EINVAL;
        }
    if (m->lr < 0.0f || m->front + m->rear <= 0.0f || m->delta_rate_max < 0.0f ||
        m->goal_heading_weight < 0.0f || m->goal_speed_weight < 0.0f ||
        !(m->u_max >= m->u_min) || isnan(m->v_min) || isnan(m->v_max) || !(m->v_max >= m->v_min)) {
        why = "inconsistent model bounds (lr >= 0, rate >= 0, u_min <= u_max, v_min <= v_max)";
        return NNP_EINVAL;
    }
    if (m->n_layers < 2 || m->n_layers > NNP_MAX_LAYERS || m->widths[m->n_layers] != 2) {
        why = "the MLP needs 2..3 weight layers and 2 outputs";
        return NNP_EINVAL;
    }
    const int nin = m->feature_set == NNP_FEAT_PAPER ? 5 : m->feature_set == NNP_FEAT_SIX ? 6
                                                   : m->feature_set == NNP_FEAT_EIGHT ? 8 : -1;
    if (nin < 0 || m->widths[0] != nin) {
        why = "feature_set does not match widths[0]";
        return NNP_EINVAL;
    }
    const int K = m->lanes_per_sample;
    if (K != 0 && K != 1 && K != 2 && K != 4 && K != 8 && K != 16) {
        why = "lanes_per_sample must be 0, 1, 2, 4, 8 or 16";
        return NNP_EINVAL;
    }
    if (m->all_points != 0 && m->all_points != 1) {
        why = "all_points must be 0 or 1";
        return NNP_EINVAL;
    }
    if (m->block_threads < 0 || m->tile_pairs < 0) {
        why = "block_threads and tile_pairs must be 0 (default) or a compiled shape's value";
        return NNP_EINVAL;
    }
    if (!find_variant(m, K, m->block_threads, m->tile_pairs)) {
        why = "no compiled kernel for this network shape, lane layout and launch shape";
        return NNP_EUNSUPPORTED;
    }
    return NNP_OK;
}

// Culling constants of the obstacle pass (all +INFINITY with all_points: every point tested).
// A point can change a sample's minima at a step only if it lies within R of the reference
// point: a margin below 1 means inside the rectangle, hence within its corner distance rc, and
// the distance features are constant (d_cap) beyond d_cap. Relative margins of 1e-3 on rc and
// 1e-5 on the squares cover the rounding of the box distance, of the point test and of the
// pose's sine and cosine (a few float ulps each). step_scale bounds the sample's move in one
// step per unit of speed: the model moves the reference point by dt |v| sqrt(1 + tan(beta)^2)
// with tan(beta) = l_r tan(delta) / L and |delta| <= delta_max.
float round_up_f(double v)
{
    const float f = (float)v;
    return (double)f >= v ? f : nextafterf(f, INFINITY);
}

CullConsts cull_consts(const nnp_model *m)
{
    CullConsts c = {INFINITY, INFINITY, INFINITY};
    if (m->all_points) return c;
    const double ext = std::max(fabs((double)m->front), fabs((double)m->rear));
    const double hw = m->half_width;
    const double rc = sqrt(ext * ext + hw * hw) * (1.0 + 1e-3);
    const double R = m->feature_set != NNP_FEAT_PAPER ? std::max(rc, (double)m->d_cap) : rc;
    c.coll_r2 = round_up_f(rc * rc * (1.0 + 1e-5));
    c.cull_r2 = round_up_f(R * R * (1.0 + 1e-5));
    const double dmax = m->delta_max;
    if (dmax < 0.5 * M_PI - 1e-3) {
        const double tb = (double)m->lr / ((double)m->lf + m->lr) * tan(dmax) * (1.0 + 1e-6);
        c.step_scale = round_up_f(m->dt * sqrt(1.0 + tb * tb) * (1.0 + 1e-5));
    }
    return c;
}

DevModel derive(const nnp_model *m)
{
    DevModel d;
    const float L = m->lf + m->lr;
    const float hl = 0.5f * (m->front + m->rear);
    d.dt = m->dt;
    d.lr_over_L = m->lr / L;
    d.inv_L = 1.0f / L;
    d.ihl = 1.0f / hl;
    d.ihw = 1.0f / m->half_width;
    d.oc = 0.5f * (m->front - m->rear);
    d.delta_max = m->delta_max;
    d.rate = m->delta_rate_max > 0.0f ? m->delta_rate_max * m->dt / m->delta_max : 0.0f;
    d.u_min = m->u_min;
    d.u_half_range = 0.5f * (m->u_max - m->u_min);
    d.v_min = m->v_min;
    d.v_max = m->v_max;
    d.inv_nxi = 1.0f / m->norm_xi;
    d.inv_neta = 1.0f / m->norm_eta;
    d.inv_nphi = 1.0f / m->norm_phi;
    d.inv_nv = 1.0f / m->norm_v;
    d.d_cap = m->d_cap;
    d.inv_dcap = 1.0f / m->d_cap;
    d.effort_scale = m->effort_weight * m->dt;
    d.w_phi = m->goal_heading_weight;
    d.w_v = m->goal_speed_weight;
    d.eps_xi = m->eps_xi;
    d.eps_eta = m->eps_eta;
    d.eps_phi = m->eps_phi;
    d.eps_v = m->eps_v;
    return d;
}

int check_problem(nnp_handle *h, const nnp_problem *p)
{
    if (!p) return fail(h, NNP_EINVAL, "null problem");
    if (p->N < 1) return fail(h, NNP_EINVAL, "N must be >= 1");
    if (p->T < 1 || p->T > NNP_MAX_T) return fail(h, NNP_EINVAL, "T must be in [1, NNP_MAX_T]");
    if (p->P < 0 || p->P > NNP_MAX_P) return fail(h, NNP_EINVAL, "P must be in [0, NNP_MAX_P]");
    if (p->P > 0 && !p->obst) return fail(h, NNP_EINVAL, "obst is null with P > 0");
    if ((long long)p->N * h->var->K >= (1ll << 31))
        return fail(h, NNP_EINVAL, "N too large for one launch");
    for (int i = 0; i < 4; ++i)
        if (!finite_f(p->z0[i]) || !finite_f(p->goal[i]))
            return fail(h, NNP_EINVAL, "z0 and goal must be finite");
    if (fabsf(p->z0[2]) > PI_F || fabsf(p->goal[2]) > PI_F)
        return fail(h, NNP_EINVAL, "headings must lie in [-pi, pi]");
    if (p->a_prev)
        for (int i = 0; i < 2; ++i)
            if (!(fabsf(p->a_prev[i]) <= 1.0f))
                return fail(h, NNP_EINVAL, "a_prev must be finite and in [-1, 1]");
    if (p->n_prop < 0 || p->n_prop > p->N) return fail(h, NNP_EINVAL, "n_prop must be in [0, N]");
    if (p->n_prop > 0 && (!p->prop_mu || !p->prop_log_sigma))
        return fail(h, NNP_EINVAL, "prop_mu / prop_log_sigma are null with n_prop > 0");
    if (p->own_goal_weights != 0 && p->own_goal_weights != 1)
        return fail(h, NNP_EINVAL, "own_goal_weights must be 0 or 1");
    if (p->own_goal_weights && !(p->goal_heading_weight >= 0.0f && finite_f(p->goal_heading_weight) &&
                                 p->goal_speed_weight >= 0.0f && finite_f(p->goal_speed_weight)))
        return fail(h, NNP_EINVAL, "a problem's goal weights must be finite and >= 0");
    return NNP_OK;
}

// Launch arguments of one problem (validated), without its extrapolation table.
int fill_args(nnp_handle *h, const nnp_problem *p, RolloutArgs &a)
{
    int rc = check_problem(h, p);
    if (rc) return rc;
    memset(&a, 0, sizeof a);
    a.m = h->dm;
    if (p->own_goal_weights) {
        a.m.w_phi = p->goal_heading_weight;
        a.m.w_v = p->goal_speed_weight;
    }
    for (int i = 0; i < 4; ++i) {
        a.z0[i] = p->z0[i];
        a.goal[i] = p->goal[i];
    }
    if (p->a_prev) {
        a.a_prev[0] = p->a_prev[0];
        a.a_prev[1] = p->a_prev[1];
    } else {
        a.a_prev[0] = 0.0f;
        a.a_prev[1] = -1.0f - 2.0f * h->model.u_min / (h->model.u_max - h->model.u_min);
        if (!(h->model.u_max > h->model.u_min)) a.a_prev[1] = 0.0f;
    }
    const int P16 = p->P > 0 ? (p->P + POINT_PAD - 1) / POINT_PAD * POINT_PAD : 0;
    a.N = p->N;
    a.T = p->T;
    a.P2 = P16 / 2;
    a.key.k0 = (uint32_t)(p->seed & 0xffffffffull);
    a.key.k1 = (uint32_t)(p->seed >> 32);
    a.inst = p->inst;
    a.warm_theta = p->warm_theta;
    a.obst = reinterpret_cast<const float4 *>(p->obst);
    a.P = p->P;
    a.n_prop = p->n_prop;
    a.mu = p->n_prop > 0 ? p->prop_mu : nullptr;
    a.log_sigma = p->n_prop > 0 ? p->prop_log_sigma : nullptr;
    a.cull_r2 = h->cull.cull_r2;
    a.coll_r2 = h->cull.coll_r2;
    a.step_scale = h->cull.step_scale;
    a.stats = h->stats ? h->d_stats : nullptr;
    a.gp = h->var->gp;
    return NNP_OK;
}

// Device tables of one problem, in float4 entries: the extrapolated pairs and the group boxes,
// each with the slack the LDS copies may read past its end, then the spatial order of the points
// (P <= SORT_MAX only).
struct TableLayout {
    size_t ext, bb, perm, disp;
};

TableLayout table_layout(const RolloutArgs &a)
{
    TableLayout l;
    l.ext = (size_t)(a.T + 1) * a.P2 + CHUNK;
    l.bb = (size_t)(a.T + 1) * (a.P2 / a.gp) + CHUNK;
    l.perm = (a.P > 0 && a.P <= SORT_MAX) ? ((size_t)a.P + 3) / 4 : 0;
    l.disp = 1;
    return l;
}

size_t table_entries(const RolloutArgs &a)
{
    const TableLayout l = table_layout(a);
    return l.ext + l.bb + l.perm + l.disp;
}

// Point a problem's table pointers into a region of table_entries(a) entries at `base`.
void place_tables(RolloutArgs &a, float4 *base)
{
    const TableLayout l = table_layout(a);
    a.ext = base;
    a.bb = base + l.ext;
    a.perm = l.perm ? reinterpret_cast<uint32_t *>(base + l.ext + l.bb) : nullptr;
    a.disp = reinterpret_cast<float *>(base + l.ext + l.bb + l.perm);
}

// The spatial order and the points' displacement bound, then the extrapolation table and its
// group boxes, of one problem whose tables are placed; also resets its argmin key.
hipError_t launch_tables(const RolloutArgs &a, hipStream_t s)
{
    if (a.P > 0) {
        hipLaunchKernelGGL(order_kernel, dim3(1), dim3(ORDER_BLOCK), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const long long n = (long long)(a.T + 1) * a.P2;
    const unsigned grid = (unsigned)(n > 0 ? (n + BLOCK - 1) / BLOCK : 1);
    hipLaunchKernelGGL(extrapolate_kernel, dim3(grid), dim3(BLOCK), 0, s, a.obst, a.perm, a.P,
                       a.P2, a.gp, a.T, a.m.dt, const_cast<float4 *>(a.ext),
                       const_cast<float4 *>(a.bb), a.best_key);
    return hipGetLastError();
}

// Device workspace held by the handle's grown buffers.
uint64_t workspace_bytes(const nnp_handle *h)
{
    return (uint64_t)h->ext_bytes + h->rec_bytes + h->bext_bytes + h->bkeys_bytes + h->bmeta_bytes;
}

// Grow a device buffer (contents are not kept). Synchronises the stream before freeing. Fails
// with NNP_ENOMEM, before any device work, when the handle's workspace would exceed its limit.
int grow(nnp_handle *h, void **buf, size_t *cap, size_t need, hipStream_t s, const char *what)
{
    if (need <= *cap) return NNP_OK;
    if (workspace_bytes(h) - *cap + need > h->ws_limit)
        return fail(h, NNP_ENOMEM, std::string("workspace limit exceeded by the ") + what);
    if (*buf) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    if (hipMalloc(buf, need) != hipSuccess) {
        *buf = nullptr;
        return fail(h, NNP_ENOMEM, std::string("hipMalloc failed: ") + what);
    }
    *cap = need;
    return NNP_OK;
}

// Build the launch arguments and the extrapolation table for one problem.
int prepare(nnp_handle *h, const nnp_problem *p, RolloutArgs &a, hipStream_t s)
{
    int rc = fill_args(h, p, a);
    if (rc) return rc;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    rc = grow(h, reinterpret_cast<void **>(&h->d_ext), &h->ext_bytes,
              table_entries(a) * sizeof(float4), s, "extrapolation table");
    if (rc) return rc;
    place_tables(a, h->d_ext);
    a.best_key = h->d_key;
    e = launch_tables(a, s);
    if (e != hipSuccess) return hip_fail(h, e, "extrapolate_kernel launch");
    return NNP_OK;
}

hipEvent_t pool_event(nnp_handle *h)
{
    if (!h->ev_pool.empty()) {
        hipEvent_t ev = h->ev_pool.back();
        h->ev_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
}

int launch_rollout(nnp_handle *h, const RolloutArgs &a, int mode, hipStream_t s)
{
    const long long lanes = (long long)a.N * h->var->K;
    const int rb = h->var->block;
    const dim3 grid((unsigned)((lanes + rb - 1) / rb));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->timing) {
        e0 = pool_event(h);
        e1 = pool_event(h);
        if (e0) hipEventRecord(e0, s);
    }
    h->var->launch_rollout(a, mode, grid, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "rollout_kernel launch");
    if (h->timing && e0 && e1) {
        hipEventRecord(e1, s);
        h->pending.emplace_back(e0, e1);
    }
    return NNP_OK;
}

}  // namespace

extern "C" {

const char *nnp_version(void) { return "nnplan 0.1 (gfx950)"; }

int nnp_create(nnp_handle **out, const nnp_model *m, int device)
{
    if (!out) return fail(nullptr, NNP_EINVAL, "null handle pointer");
    *out = nullptr;
    if (!m) return fail(nullptr, NNP_EINVAL, "null model");
    std::string why;
    const int rc = check_model(m, why);
    if (rc) return fail(nullptr, rc, why);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(nullptr, NNP_EINVAL, "no such device");
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    nnp_handle *h = new (std::nothrow) nnp_handle();
    if (!h) return fail(nullptr, NNP_ENOMEM, "host allocation failed");
    h->model = *m;
    h->dm = derive(m);
    h->cull = cull_consts(m);
    h->var = find_variant(m, m->lanes_per_sample, m->block_threads, m->tile_pairs);
    h->device = device;
    h->err.reserve(1024);
    e = scratch_address(device, &h->scratch);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(nullptr, e, "hipGetSymbolAddress of the scratch array");
    }
    e = hipMalloc(&h->d_key, sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete h;
        return fail(nullptr, NNP_ENOMEM, "hipMalloc of the argmin key failed");
    }
    *out = h;
    return NNP_OK;
}

void nnp_destroy(nnp_handle *h)
{
    if (!h) return;
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    for (auto &pr : h->pending) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    for (hipEvent_t ev : h->ev_pool) hipEventDestroy(ev);
    if (h->d_ext) hipFree(h->d_ext);
    if (h->d_rec) hipFree(h->d_rec);
    if (h->d_key) hipFree(h->d_key);
    if (h->d_stats) hipFree(h->d_stats);
    if (h->d_bext) hipFree(h->d_bext);
    if (h->d_bkeys) hipFree(h->d_bkeys);
    if (h->d_bmeta) hipFree(h->d_bmeta);
    if (h->h_bmeta) hipHostFree(h->h_bmeta);
    if (h->meta_copied) hipEventDestroy(h->meta_copied);
    delete h;
}

int nnp_n_theta(const nnp_handle *h) { return h ? h->var->ntheta : NNP_EINVAL; }

int nnp_set_record_limit(nnp_handle *h, uint64_t bytes)
{
    if (!h) return NNP_EINVAL;
    h->rec_limit = bytes;
    return NNP_OK;
}

int nnp_set_workspace_limit(nnp_handle *h, uint64_t bytes)
{
    if (!h) return NNP_EINVAL;
    h->ws_limit = bytes;
    return NNP_OK;
}

int nnp_plan(nnp_handle *h, const nnp_problem *p, nnp_result *r, void *hip_stream)
{
    if (!h) return NNP_EINVAL;
    if (!r) return fail(h, NNP_EINVAL, "null result");
    hipStream_t s = (hipStream_t)hip_stream;
    RolloutArgs a;
    int rc = prepare(h, p, a, s);
    if (rc) return rc;
    // records of every sample's states and controls when they fit the limit, so that the
    // winner's outputs are gathered instead of re-simulated
    const size_t rec_need = (size_t)p->N * (size_t)p->T * sizeof(float2);
    const bool record = rec_need <= h->rec_limit && rec_need < (1ull << 31) &&
                        workspace_bytes(h) - h->rec_bytes + std::max(rec_need, h->rec_bytes) <=
                            h->ws_limit;
    if (record) {
        rc = grow(h, &h->d_rec, &h->rec_bytes, rec_need, s, "sample records");
        if (rc) return rc;
        a.rec_ctrl = static_cast<float2 *>(h->d_rec);
    }
    rc = launch_rollout(h, a, MODE_PLAN, s);
    if (rc) return rc;
    ReplayOut o = {r->theta, r->controls, r->controls_phys, r->traj, r->cost, r->best_index,
                   r->status, r->goal_reached};
    if (record) h->var->launch_gather(a, o, s);
    else h->var->launch_replay(a, o, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, record ? "gather_kernel launch" : "replay_kernel launch");
    h->err.clear();
    return NNP_OK;
}

int nnp_plan_noalloc(nnp_handle *h, const nnp_problem *p, nnp_result *r, void *hip_stream)
{
    if (!h) return NNP_EINVAL;
    if (!r) return fail(h, NNP_EINVAL, "null result");
    RolloutArgs a;
    int rc = fill_args(h, p, a);
    if (rc) return rc;
    const size_t need = NOALLOC_KEY_BYTES + table_entries(a) * sizeof(float4);
    if (need > (size_t)NNP_NOALLOC_SCRATCH_BYTES) {
        char msg[256];
        snprintf(msg, sizeof msg,
                 "the extrapolation table of T = %d steps and P = %d points needs %zu bytes of "
                 "scratch, more than NNP_NOALLOC_SCRATCH_BYTES = %d; use nnp_plan",
                 p->T, p->P, need, (int)NNP_NOALLOC_SCRATCH_BYTES);
        return fail_fixed(h, NNP_EINVAL, msg);
    }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail_fixed(h, NNP_EDEVICE, "hipSetDevice", hipGetErrorString(e));
    if (!h->scratch) {
        e = scratch_address(h->device, &h->scratch);
        if (e != hipSuccess)
            return fail_fixed(h, NNP_EDEVICE, "hipGetSymbolAddress", hipGetErrorString(e));
    }
    hipStream_t s = (hipStream_t)hip_stream;
    char *base = static_cast<char *>(h->scratch);
    unsigned long long *key = reinterpret_cast<unsigned long long *>(base);
    float4 *ext = reinterpret_cast<float4 *>(base + NOALLOC_KEY_BYTES);
    a.best_key = key;
    place_tables(a, ext);
    // the tables and the key reset (every call starts the argmin from ~0)
    e = launch_tables(a, s);
    if (e != hipSuccess)
        return fail_fixed(h, NNP_EDEVICE, "extrapolate_kernel launch", hipGetErrorString(e));
    // the rollout without per-sample records, then the winner re-simulated
    const long long lanes = (long long)a.N * h->var->K;
    const int rb = h->var->block;
    h->var->launch_rollout(a, MODE_PLAN, dim3((unsigned)((lanes + rb - 1) / rb)), s);
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail_fixed(h, NNP_EDEVICE, "rollout_kernel launch", hipGetErrorString(e));
    ReplayOut o = {r->theta, r->controls, r->controls_phys, r->traj, r->cost, r->best_index,
                   r->status, r->goal_reached};
    h->var->launch_replay(a, o, s);
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail_fixed(h, NNP_EDEVICE, "replay_kernel launch", hipGetErrorString(e));
    h->err.clear();
    return NNP_OK;
}

int nnp_plan_batch(nnp_handle *h, const nnp_problem *probs, int count, nnp_result *results,
                   void *hip_stream)
{
    if (!h) return NNP_EINVAL;
    if (!probs || !results || count < 1) return fail(h, NNP_EINVAL, "empty batch");
    if (count > NNP_MAX_BATCH) return fail(h, NNP_EINVAL, "more than NNP_MAX_BATCH problems");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    std::vector<RolloutArgs> args((size_t)count);
    size_t entries = 0;
    for (int i = 0; i < count; ++i) {
        int rc = fill_args(h, &probs[i], args[i]);
        if (rc) return fail(h, rc, "problem " + std::to_string(i) + ": " + h->err);
        entries += table_entries(args[i]);
    }
    const int K = h->var->K;
    const int S = h->var->block / K;
    // Work items, longest problems first: (problem, tile of S samples).
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto work = [&](int i) { return (double)(args[i].T + 1) * (args[i].P2 + 64); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    std::vector<int2> items;
    for (int i : order)
        for (int t = 0; t * S < args[i].N; ++t) items.push_back(make_int2(i, t));
    const int n_items = (int)items.size();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamIsCapturing");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    const size_t meta = (size_t)count * (sizeof(RolloutArgs) + sizeof(ReplayOut)) +
                        (size_t)n_items * sizeof(int2);
    if (capturing && (entries * sizeof(float4) > h->bext_bytes || (size_t)count * 8 >
                      h->bkeys_bytes || meta > h->bmeta_bytes || meta > h->hmeta_bytes ||
                      !h->meta_copied))
        return fail(h, NNP_EINVAL, "the batch workspace must be sized by an uncaptured call "
                                   "with at least this batch before capture");
    // Device workspace.
    int rc = grow(h, &h->d_bext, &h->bext_bytes, entries * sizeof(float4), s, "batch tables");
    if (!rc) rc = grow(h, &h->d_bkeys, &h->bkeys_bytes, (size_t)count * 8, s, "batch keys");
    if (!rc) rc = grow(h, &h->d_bmeta, &h->bmeta_bytes, meta, s, "batch descriptors");
    if (rc) return rc;
    // Records of every problem's samples, one region after another, when all fit the limits as
    // in nnp_plan: the winners' outputs are then gathered instead of re-simulated (same bits).
    // Under stream capture only an allocation made before is used.
    size_t rec_need = 0;
    bool record = true;
    for (int i = 0; i < count && record; ++i) {
        const size_t one = (size_t)args[i].N * (size_t)args[i].T * sizeof(float2);
        record = one < (1ull << 31);
        rec_need += one;
    }
    record = record && rec_need <= h->rec_limit &&
             workspace_bytes(h) - h->rec_bytes + std::max(rec_need, h->rec_bytes) <= h->ws_limit &&
             (!capturing || rec_need <= h->rec_bytes);
    if (record) {
        rc = grow(h, &h->d_rec, &h->rec_bytes, rec_need, s, "sample records");
        if (rc) return rc;
        float2 *rec = static_cast<float2 *>(h->d_rec);
        for (int i = 0; i < count; ++i) {
            args[i].rec_ctrl = rec;
            rec += (size_t)args[i].N * (size_t)args[i].T;
        }
    }
    if (!h->meta_copied && hipEventCreateWithFlags(&h->meta_copied, hipEventDisableTiming) !=
                               hipSuccess)
        return fail(h, NNP_EDEVICE, "hipEventCreate failed");
    // The pinned staging buffer is reused: wait until the previous batch's copy has read it
    // (under stream capture nothing runs yet, and the caller orders its replays).
    if (!capturing) {
        e = hipEventSynchronize(h->meta_copied);
        if (e != hipSuccess) return hip_fail(h, e, "hipEventSynchronize");
    }
    if (meta > h->hmeta_bytes) {
        if (h->h_bmeta) hipHostFree(h->h_bmeta);
        h->h_bmeta = nullptr;
        h->hmeta_bytes = 0;
        if (hipHostMalloc(&h->h_bmeta, meta, hipHostMallocDefault) != hipSuccess)
            return fail(h, NNP_ENOMEM, "hipHostMalloc of the batch staging buffer failed");
        h->hmeta_bytes = meta;
    }
    char *dmeta = static_cast<char *>(h->d_bmeta);
    RolloutArgs *d_args = reinterpret_cast<RolloutArgs *>(dmeta);
    ReplayOut *d_outs = reinterpret_cast<ReplayOut *>(dmeta + (size_t)count * sizeof(RolloutArgs));
    int2 *d_items = reinterpret_cast<int2 *>(dmeta + (size_t)count *
                                                         (sizeof(RolloutArgs) + sizeof(ReplayOut)));
    char *hmeta = static_cast<char *>(h->h_bmeta);
    RolloutArgs *h_args = reinterpret_cast<RolloutArgs *>(hmeta);
    ReplayOut *h_outs = reinterpret_cast<ReplayOut *>(hmeta + (size_t)count * sizeof(RolloutArgs));
    int2 *h_items = reinterpret_cast<int2 *>(hmeta + (size_t)count *
                                                         (sizeof(RolloutArgs) + sizeof(ReplayOut)));
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        place_tables(args[i], static_cast<float4 *>(h->d_bext) + off);
        off += table_entries(args[i]);
        args[i].best_key = static_cast<unsigned long long *>(h->d_bkeys) + i;
        h_args[i] = args[i];
        const nnp_result &r = results[i];
        h_outs[i] = ReplayOut{r.theta, r.controls, r.controls_phys, r.traj, r.cost, r.best_index,
                              r.status, r.goal_reached};
    }
    memcpy(h_items, items.data(), items.size() * sizeof(int2));
    e = hipMemcpyAsync(dmeta, hmeta, meta, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync of the batch descriptors");
    if (!capturing) {
        e = hipEventRecord(h->meta_copied, s);
        if (e != hipSuccess) return hip_fail(h, e, "hipEventRecord");
    }
    hipLaunchKernelGGL(order_batch_kernel, dim3(count), dim3(ORDER_BLOCK), 0, s, d_args);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "order_batch_kernel launch");
    hipLaunchKernelGGL(extrapolate_batch_kernel, dim3(64, count), dim3(BLOCK), 0, s, d_args);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "extrapolate_batch_kernel launch");
    h->var->launch_rollout_batch(d_args, d_items, n_items, h->dm.oc == 0.0f, s);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "rollout_batch_kernel launch");
    if (record) h->var->launch_gather_batch(d_args, d_outs, count, s);
    else h->var->launch_replay_batch(d_args, d_outs, count, s);
    e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(h, e, record ? "gather_batch_kernel launch" : "replay_batch_kernel launch");
    h->err.clear();
    return NNP_OK;
}

int nnp_rollout(nnp_handle *h, const nnp_problem *p, const float *theta, nnp_rollout_out *o,
                void *hip_stream)
{
    if (!h) return NNP_EINVAL;
    if (!o) return fail(h, NNP_EINVAL, "null output");
    hipStream_t s = (hipStream_t)hip_stream;
    RolloutArgs a;
    int rc = prepare(h, p, a, s);
    if (rc) return rc;
    a.theta = theta;
    if (theta) a.warm_theta = nullptr;
    a.cost = o->cost;
    a.collided = o->collided;
    a.first = o->first_collision;
    a.min_margin = o->min_margin;
    if (o->min_margin) a.cull_r2 = INFINITY;   // the margin is a minimum over every point
    a.traj = o->traj;
    a.controls = o->controls;
    rc = launch_rollout(h, a, MODE_OUT, s);
    if (rc) return rc;
    h->err.clear();
    return NNP_OK;
}

int nnp_sample_theta(uint64_t seed, uint32_t inst, uint32_t i0, uint32_t N, uint32_t n_theta,
                     float *out, void *hip_stream)
{
    if (!out || N == 0 || n_theta == 0) return NNP_EINVAL;
    const long long n = (long long)N * n_theta;
    if (n >= (1ll << 40)) return NNP_EINVAL;
    PhiloxKey key = {(uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32)};
    hipLaunchKernelGGL(theta_kernel, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       (hipStream_t)hip_stream, key, inst, i0, N, n_theta, nullptr, nullptr, out);
    return hipGetLastError() == hipSuccess ? NNP_OK : NNP_EDEVICE;
}

int nnp_sample_gauss(uint64_t seed, uint32_t inst, uint32_t i0, uint32_t N, uint32_t n_theta,
                     const float *mu, const float *log_sigma, float *out, void *hip_stream)
{
    if (!out || !mu || !log_sigma || N == 0 || n_theta == 0) return NNP_EINVAL;
    const long long n = (long long)N * n_theta;
    if (n >= (1ll << 40)) return NNP_EINVAL;
    PhiloxKey key = {(uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32)};
    hipLaunchKernelGGL(theta_kernel, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       (hipStream_t)hip_stream, key, inst, i0, N, n_theta, mu, log_sigma, out);
    return hipGetLastError() == hipSuccess ? NNP_OK : NNP_EDEVICE;
}

const char *nnp_last_error(const nnp_handle *h)
{
    return h ? h->err.c_str() : g_create_error.c_str();
}

int nnp_set_timing(nnp_handle *h, int enable)
{
    if (!h) return NNP_EINVAL;
    h->timing = enable != 0;
    return NNP_OK;
}

int nnp_set_cull_stats(nnp_handle *h, int enable)
{
    if (!h) return NNP_EINVAL;
    if (enable) {
        hipError_t e = hipSetDevice(h->device);
        if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
        if (!h->d_stats && hipMalloc(&h->d_stats, 2 * sizeof(unsigned long long)) != hipSuccess) {
            h->d_stats = nullptr;
            return fail(h, NNP_ENOMEM, "hipMalloc of the culling counter failed");
        }
        e = hipMemset(h->d_stats, 0, 2 * sizeof(unsigned long long));
        if (e != hipSuccess) return hip_fail(h, e, "hipMemset");
    }
    h->stats = enable != 0;
    return NNP_OK;
}

int nnp_cull_stats(nnp_handle *h, uint64_t *tested, uint64_t *total, int reset)
{
    if (!h) return NNP_EINVAL;
    unsigned long long v[2] = {0, 0};
    if (h->d_stats) {
        hipError_t e = hipSetDevice(h->device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(v, h->d_stats, sizeof v, hipMemcpyDeviceToHost);
        if (e == hipSuccess && reset) e = hipMemset(h->d_stats, 0, sizeof v);
        if (e != hipSuccess) return hip_fail(h, e, "reading the culling counter");
    }
    if (tested) *tested = v[0];
    if (total) *total = v[1];
    return NNP_OK;
}

int nnp_kernel_time(nnp_handle *h, double *ms, int64_t *launches, int reset)
{
    if (!h) return NNP_EINVAL;
    for (auto &pr : h->pending) {
        hipError_t e = hipEventSynchronize(pr.second);
        if (e != hipSuccess) return hip_fail(h, e, "hipEventSynchronize");
        float t = 0.0f;
        e = hipEventElapsedTime(&t, pr.first, pr.second);
        if (e != hipSuccess) return hip_fail(h, e, "hipEventElapsedTime");
        h->acc_ms += t;
        h->launches += 1;
        h->ev_pool.push_back(pr.first);
        h->ev_pool.push_back(pr.second);
    }
    h->pending.clear();
    if (ms) *ms = h->acc_ms;
    if (launches) *launches = h->launches;
    if (reset) {
        h->acc_ms = 0.0;
        h->launches = 0;
    }
    return NNP_OK;
}

}  // extern "C"
