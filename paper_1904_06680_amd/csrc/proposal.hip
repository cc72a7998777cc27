// nnproposal: kernels and C-ABI of the learned Gaussian proposal (declarations and definitions
// in include/nnproposal.h). BF16 MFMA products with binary32 accumulation on gfx950.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/nnproposal.h"

namespace {

constexpr int ENC = NNP_PROP_ENC;
constexpr int ENC_PAD = 128;          // encoding padded with zero columns to a whole GEMM tile
constexpr int HID = NNP_PROP_HIDDEN;
constexpr int NEAR = NNP_PROP_NEAR;
constexpr int ROWS = 128;             // batch padding (GEMM tile rows)
constexpr int COL_CHUNKS_MAX = 128;   // most row chunks of the bias-gradient column sums
constexpr float PI_F = 3.14159265358979f;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// Round to the nearest bfloat16, ties to even (finite inputs; NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------------------------
// 1. BF16 MFMA matrix product: 128 x 128 tile per 256-thread workgroup, four wavefronts of
//    64 x 64 (2 x 2 v_mfma_f32_32x32x16_bf16 blocks), K in steps of 32 through double-buffered
//    LDS ([row][k] with a padded row of 40 bf16 so that 16-byte operand reads spread over banks).
// ---------------------------------------------------------------------------------------------
constexpr int TM = 128, TN = 128, TK = 32, LDK = 40;

struct GemmArgs {
    const uint16_t *A, *B;
    int lda, ldb, M, N, K;
    const float *bias, *mask;
    int ldm;
    float *C;
    int ldc;
    uint16_t *Cq;
    int ldcq;
    float *partial;     // split-K: per-slice sums [gridDim.z][M][N] instead of the epilogue
};

// Global -> registers for one K step: 512 chunks of 8 bf16 per operand tile, two per thread.
template <int LAYOUT>
__device__ __forceinline__ void load_tile(const uint16_t *__restrict__ X, int ld, int r0, int k0,
                                          int tid, uint4 (&reg)[2])
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = tid + 256 * i;
        if (LAYOUT == 0) {                      // X(r, k) = X[r * ld + k]: 128 rows x 4 chunks
            const int r = c >> 2, kc = (c & 3) * 8;
            reg[i] = *reinterpret_cast<const uint4 *>(X + (size_t)(r0 + r) * ld + k0 + kc);
        } else {                                // X(r, k) = X[k * ld + r]: 32 k-rows x 16 chunks
            const int kr = c >> 4, rc = (c & 15) * 8;
            reg[i] = *reinterpret_cast<const uint4 *>(X + (size_t)(k0 + kr) * ld + r0 + rc);
        }
    }
}

template <int LAYOUT>
__device__ __forceinline__ void store_tile(uint16_t (*S)[LDK], int tid, const uint4 (&reg)[2])
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = tid + 256 * i;
        if (LAYOUT == 0) {
            const int r = c >> 2, kc = (c & 3) * 8;
            *reinterpret_cast<uint4 *>(&S[r][kc]) = reg[i];
        } else {                                // transpose on the way into LDS
            const int kr = c >> 4, rc = (c & 15) * 8;
            const uint32_t w[4] = {reg[i].x, reg[i].y, reg[i].z, reg[i].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                S[rc + 2 * j][kr] = (uint16_t)(w[j] & 0xffffu);
                S[rc + 2 * j + 1][kr] = (uint16_t)(w[j] >> 16);
            }
        }
    }
}

template <int LA, int LB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[2][TM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][TN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    // K range of this slice (gridDim.z slices; one slice without split-K)
    const int nkt = g.K / TK;
    const int kt0 = (int)((long long)blockIdx.z * nkt / gridDim.z);
    const int kt1 = (int)((long long)(blockIdx.z + 1) * nkt / gridDim.z);

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    uint4 ra[2], rb[2];
    load_tile<LA>(g.A, g.lda, m0, kt0 * TK, tid, ra);
    load_tile<LB>(g.B, g.ldb, n0, kt0 * TK, tid, rb);
    store_tile<LA>(As[0], tid, ra);
    store_tile<LB>(Bs[0], tid, rb);
    __syncthreads();

    const int lr = lane & 31, lk = (lane >> 5) * 8;
    for (int kt = kt0; kt < kt1; ++kt) {
        const int buf = (kt - kt0) & 1;
        if (kt + 1 < kt1) {
            load_tile<LA>(g.A, g.lda, m0, (kt + 1) * TK, tid, ra);
            load_tile<LB>(g.B, g.ldb, n0, (kt + 1) * TK, tid, rb);
        }
#pragma unroll
        for (int kk = 0; kk < TK; kk += 16) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x8 *>(&As[buf][wm * 64 + i * 32 + lr][kk + lk]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][wn * 64 + j * 32 + lr][kk + lk]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0,
                                                                       0, 0);
        }
        if (kt + 1 < kt1) {
            store_tile<LA>(As[buf ^ 1], tid, ra);
            store_tile<LB>(Bs[buf ^ 1], tid, rb);
        }
        __syncthreads();
    }

    // Accumulator layout of the 32 x 32 block: lane l holds column l % 32 and rows
    // 8 (r / 4) + 4 (l / 32) + r % 4 for r = 0..15.
    if (g.partial) {
        float *P = g.partial + (size_t)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = n0 + wn * 64 + j * 32 + lr;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    P[(size_t)row * g.N + col] = acc[i][j][r];
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn * 64 + j * 32 + lr;
            const float bias = (EPI != 2 && g.bias) ? g.bias[col] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                float v = acc[i][j][r] + bias;
                if (EPI == 2) v = g.mask[(size_t)row * g.ldm + col] > 0.0f ? acc[i][j][r] : 0.0f;
                if (g.C) g.C[(size_t)row * g.ldc + col] = v;
                if (g.Cq) g.Cq[(size_t)row * g.ldcq + col] = to_bf16(EPI == 1 ? fmaxf(v, 0.0f) : v);
            }
        }
}

// Split-K finish: acc = sum over slices z = 0..S-1 in slice order (deterministic), then the
// same epilogue as gemm_kernel.
template <int EPI>
__global__ void splitk_reduce_kernel(const float *__restrict__ partial, int S, const GemmArgs g)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)g.M * g.N) return;
    const int row = (int)(i / g.N), col = (int)(i % g.N);
    float acc = 0.0f;
    for (int z = 0; z < S; ++z) acc += partial[(size_t)z * g.M * g.N + i];
    float v = acc + ((EPI != 2 && g.bias) ? g.bias[col] : 0.0f);
    if (EPI == 2) v = g.mask[(size_t)row * g.ldm + col] > 0.0f ? acc : 0.0f;
    if (g.C) g.C[(size_t)row * g.ldc + col] = v;
    if (g.Cq) g.Cq[(size_t)row * g.ldcq + col] = to_bf16(EPI == 1 ? fmaxf(v, 0.0f) : v);
}

int launch_gemm(int la, int lb, int epi, const GemmArgs &g, hipStream_t s, int splits = 1)
{
    const dim3 grid(g.N / TN, g.M / TM, splits), block(256);
#define NNP_GEMM_CASE(LA, LB, E)                                                          \
    if (la == LA && lb == LB && epi == E) {                                               \
        hipLaunchKernelGGL((gemm_kernel<LA, LB, E>), grid, block, 0, s, g);             \
        return hipGetLastError() == hipSuccess ? NNP_OK : NNP_EDEVICE;                    \
    }
    NNP_GEMM_CASE(0, 0, 0) NNP_GEMM_CASE(0, 0, 1) NNP_GEMM_CASE(0, 0, 2)
    NNP_GEMM_CASE(0, 1, 0) NNP_GEMM_CASE(0, 1, 1) NNP_GEMM_CASE(0, 1, 2)
    NNP_GEMM_CASE(1, 0, 0) NNP_GEMM_CASE(1, 0, 1) NNP_GEMM_CASE(1, 0, 2)
    NNP_GEMM_CASE(1, 1, 0) NNP_GEMM_CASE(1, 1, 1) NNP_GEMM_CASE(1, 1, 2)
#undef NNP_GEMM_CASE
    return NNP_EINVAL;
}

// ---------------------------------------------------------------------------------------------
// 2. Problem encoding: one workgroup per problem; the 16 nearest points are selected by 16
//    rounds of a workgroup-wide minimum over u64 keys (squared distance bits, index), each round
//    restricted to keys above the previous pick, so ties resolve to the lower index.
// ---------------------------------------------------------------------------------------------
struct EncProblem {
    float z0[4], goal[4], a_prev[2];
    int T, P;
    const float4 *obst;
};

struct EncNorms {
    float norm_xi, norm_eta, norm_phi, norm_v, d_cap;
};

__device__ __forceinline__ unsigned long long wave_min(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__global__ __launch_bounds__(256) void encode_kernel(const EncProblem *__restrict__ probs,
                                                     EncNorms nm, float *__restrict__ enc)
{
    const EncProblem &a = probs[blockIdx.x];
    __shared__ unsigned long long red[4];
    __shared__ int pick[NEAR];
    const int tid = threadIdx.x;
    const float x0 = a.z0[0], y0 = a.z0[1];
    unsigned long long last = 0;
    for (int r = 0; r < NEAR; ++r) {
        unsigned long long best = ~0ull;
        for (int j = tid; j < a.P; j += 256) {
            const float4 p = a.obst[j];
            const float dx = p.x - x0, dy = p.y - y0;
            const float d2 = fmaf(dx, dx, dy * dy);
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)j;
            if ((r == 0 || key > last) && key < best) best = key;
        }
        best = wave_min(best);
        if ((tid & 63) == 0) red[tid >> 6] = best;
        __syncthreads();
        unsigned long long b = red[0];
#pragma unroll
        for (int w = 1; w < 4; ++w) b = red[w] < b ? red[w] : b;
        if (tid == 0) pick[r] = b == ~0ull ? -1 : (int)(b & 0xffffffffull);
        last = b;
        __syncthreads();
    }
    float sn, cs;
    sincosf(a.z0[2], &sn, &cs);
    float *e = enc + (size_t)blockIdx.x * ENC;
    if (tid < 8) {
        float v;
        if (tid == 0) v = a.z0[3] / nm.norm_v;
        else if (tid == 1) v = a.a_prev[0];
        else if (tid == 2) v = a.a_prev[1];
        else if (tid == 3) v = (float)a.T / 100.0f;
        else if (tid == 4 || tid == 5) {
            const float dx = a.goal[0] - x0, dy = a.goal[1] - y0;
            v = tid == 4 ? (cs * dx + sn * dy) / nm.norm_xi : (cs * dy - sn * dx) / nm.norm_eta;
        } else if (tid == 6) {
            float d = a.goal[2] - a.z0[2];
            if (d >= PI_F) d -= 2.0f * PI_F;
            else if (d < -PI_F) d += 2.0f * PI_F;
            v = d / nm.norm_phi;
        } else {
            v = a.goal[3] / nm.norm_v;
        }
        e[tid] = v;
    } else if (tid < ENC) {
        const int j = (tid - 8) >> 2, c = (tid - 8) & 3;
        const int idx = pick[j];
        float v;
        if (idx < 0) {
            v = c == 0 ? 100.0f / nm.d_cap : 0.0f;
        } else {
            const float4 p = a.obst[idx];
            const float dx = p.x - x0, dy = p.y - y0;
            if (c == 0) v = (cs * dx + sn * dy) / nm.d_cap;
            else if (c == 1) v = (cs * dy - sn * dx) / nm.d_cap;
            else if (c == 2) v = (cs * p.z + sn * p.w) / nm.norm_v;
            else v = (cs * p.w - sn * p.z) / nm.norm_v;
        }
        e[tid] = v;
    }
}

// ---------------------------------------------------------------------------------------------
// 3. Element-wise kernels: input rounding, loss and its gradient, column sums, Adam, packing.
// ---------------------------------------------------------------------------------------------
// xq[Bp][128] = bf16(enc) with zero padding columns and rows.
__global__ void input_kernel(const float *__restrict__ enc, int B, int Bp, uint16_t *__restrict__ xq)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= Bp * ENC_PAD) return;
    const int b = i / ENC_PAD, k = i % ENC_PAD;
    xq[i] = (b < B && k < ENC) ? to_bf16(enc[(size_t)b * ENC + k]) : (uint16_t)0;
}

// One workgroup per padded row: dy = dL/dy (scaled by 1/B) in binary32 and bfloat16, zero in the
// padding; per-row loss partial sums.
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ y, int ldy,
                                                  const float *__restrict__ ts, int nt, int B,
                                                  float *__restrict__ dyf, uint16_t *__restrict__ dyq,
                                                  float *__restrict__ partial)
{
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ float red[4];
    float acc = 0.0f;
    const float invB = 1.0f / (float)B;
    for (int k = tid; k < ldy; k += 256) {
        float gm = 0.0f, gs = 0.0f;
        const bool live = b < B && k < nt;
        if (live) {
            const float mu = y[(size_t)b * ldy + k], s = y[(size_t)b * ldy + nt + k];
            const float r = ts[(size_t)b * nt + k] - mu;
            const float w = expf(-2.0f * s);
            const float rw = r * w;
            acc += 0.5f * r * rw + s;
            gm = -rw * invB;
            gs = (1.0f - r * rw) * invB;
        }
        if (k < nt) {
            dyf[(size_t)b * ldy + k] = gm;
            dyq[(size_t)b * ldy + k] = to_bf16(gm);
            dyf[(size_t)b * ldy + nt + k] = gs;
            dyq[(size_t)b * ldy + nt + k] = to_bf16(gs);
        } else if (k >= 2 * nt) {
            dyf[(size_t)b * ldy + k] = 0.0f;
            dyq[(size_t)b * ldy + k] = 0;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) partial[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Mean of the per-row partial losses: 256 strided binary64 sums, then a fixed-order tree.
__global__ __launch_bounds__(256) void loss_final_kernel(const float *__restrict__ partial, int B,
                                                         float *__restrict__ loss)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int b = tid; b < B; b += 256) s += partial[b];
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) *loss = (float)(red[0] / B);
}

// Column sums over rows b < B: chunk c = blockIdx.y of gridDim.y sums its rows in row order into
// part[c][n]; the final pass adds the chunks in order (deterministic).
__global__ void colsum_partial_kernel(const float *__restrict__ X, int ld, int B, int N,
                                      float *__restrict__ part)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const int c = blockIdx.y, C = gridDim.y;
    const int b0 = (int)((long long)c * B / C), b1 = (int)((long long)(c + 1) * B / C);
    float s = 0.0f;
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += X[(size_t)b * ld + n];
    part[(size_t)c * N + n] = s;
}

__global__ void colsum_final_kernel(const float *__restrict__ part, int chunks, int N,
                                    float *__restrict__ out)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * N + n];
    out[n] = s;
}

// Adam over the internal (padded) parameter layout (the bfloat16 copies are refreshed after).
__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int n, float lr, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    w[i] = wi;
}

__global__ void quantize_kernel(const float *__restrict__ w, int n, uint16_t *__restrict__ wq)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) wq[i] = to_bf16(w[i]);
}

// Copy between the external parameter vector and the internal padded layout (dir 0: in).
struct Layout {
    int ny, ny_pad;
    size_t oW1, ob1, oW2, ob2, oW3, ob3, total;   // internal offsets (floats)
    size_t eW1, eb1, eW2, eb2, eW3, eb3, etotal;  // external offsets
};

__global__ void pack_kernel(Layout L, const float *__restrict__ src, float *__restrict__ dst,
                            int dir)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= L.etotal) return;
    size_t o;
    if (i < L.eb1) o = L.oW1 + (i / ENC) * ENC_PAD + i % ENC;
    else if (i < L.eW2) o = L.ob1 + (i - L.eb1);
    else if (i < L.eb2) o = L.oW2 + (i - L.eW2);
    else if (i < L.eW3) o = L.ob2 + (i - L.eb2);
    else if (i < L.eb3) o = L.oW3 + (i - L.eW3);
    else o = L.ob3 + (i - L.eb3);
    if (dir == 0) dst[o] = src[i];
    else dst[i] = src[o];
}

__global__ void split_kernel(const float *__restrict__ y, int ldy, int B, int nt,
                             float *__restrict__ mu, float *__restrict__ ls)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)B * nt) return;
    const size_t b = i / nt, k = i % nt;
    if (mu) mu[i] = y[b * ldy + k];
    if (ls) ls[i] = y[b * ldy + nt + k];
}

inline unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// =============================================================================================
// Handle
// =============================================================================================
struct nnp_proposal {
    nnp_proposal_config cfg;
    int device = 0, Bmax = 0;                 // Bmax: max_batch padded to ROWS
    Layout L{};
    int step = 0;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grads = nullptr;
    uint16_t *wq = nullptr;                   // bf16 W1 | W2 | W3 (internal layouts)
    size_t qW1 = 0, qW2 = 0, qW3 = 0, nq = 0;
    // activations and back-propagation workspace
    uint16_t *xq = nullptr, *h1q = nullptr, *h2q = nullptr, *dyq = nullptr, *da2q = nullptr,
             *da1q = nullptr;
    float *a1 = nullptr, *a2 = nullptr, *y = nullptr, *dyf = nullptr, *da2 = nullptr,
          *da1 = nullptr, *partial = nullptr, *loss_tmp = nullptr;
    float *splitk = nullptr;                  // split-K slices of the weight gradients
    size_t splitk_floats = 0;
    float *colpart = nullptr;                 // column-sum partials [COL_CHUNKS_MAX][ny_pad]
    // encoding descriptors
    EncProblem *d_enc = nullptr, *h_enc = nullptr;
    int enc_cap = 0;
    hipEvent_t enc_copied = nullptr;
    std::vector<void *> allocs;
    std::string err;
};

namespace {

std::string g_create_error;

int pfail(nnp_proposal *q, int code, const std::string &msg)
{
    if (q) q->err = msg;
    else g_create_error = msg;
    return code;
}

template <class T>
int alloc(nnp_proposal *q, T **p, size_t count)
{
    void *ptr = nullptr;
    if (hipMalloc(&ptr, count * sizeof(T)) != hipSuccess) return NNP_ENOMEM;
    q->allocs.push_back(ptr);
    *p = static_cast<T *>(ptr);
    return NNP_OK;
}

// A product of the network. Shapes with fewer than 256 output tiles and a long K (the batch, or
// the 2 n_theta outputs) split K over enough slices to give the GPU about 512 workgroups; the
// slices are reduced in order and the epilogue runs on the sum.
int gemm(nnp_proposal *q, int la, int lb, int epi, int M, int N, int K, const uint16_t *A, int lda,
         const uint16_t *B, int ldb, const float *bias, const float *mask, int ldm, float *C,
         int ldc, uint16_t *Cq, int ldcq, hipStream_t s)
{
    GemmArgs g{A, B, lda, ldb, M, N, K, bias, mask, ldm, C, ldc, Cq, ldcq, nullptr};
    const int tiles = (M / TM) * (N / TN), nkt = K / TK;
    int S = 1;
    if (tiles < 256 && nkt >= 16) {
        S = std::min(std::min((1024 + tiles - 1) / tiles, nkt / 4), 32);
        while (S > 1 && (size_t)S * M * N > q->splitk_floats) --S;
    }
    if (S <= 1) {
        const int rc = launch_gemm(la, lb, epi, g, s);
        if (rc) return pfail(q, rc, "GEMM launch failed");
        return NNP_OK;
    }
    GemmArgs gs = g;
    gs.partial = q->splitk;
    int rc = launch_gemm(la, lb, 0, gs, s, S);
    if (rc) return pfail(q, rc, "GEMM launch failed");
    const dim3 grid(blocks((size_t)M * N)), block(256);
    if (epi == 0) hipLaunchKernelGGL(splitk_reduce_kernel<0>, grid, block, 0, s, q->splitk, S, g);
    else if (epi == 1) hipLaunchKernelGGL(splitk_reduce_kernel<1>, grid, block, 0, s, q->splitk, S, g);
    else hipLaunchKernelGGL(splitk_reduce_kernel<2>, grid, block, 0, s, q->splitk, S, g);
    return NNP_OK;
}

int gemm_splitk(nnp_proposal *q, int la, int lb, int M, int N, int K, const uint16_t *A, int lda,
                const uint16_t *B, int ldb, float *C, int ldc, hipStream_t s)
{
    return gemm(q, la, lb, 0, M, N, K, A, lda, B, ldb, nullptr, nullptr, 0, C, ldc, nullptr, 0, s);
}

// Column sums over the first B rows in two deterministic passes: C row chunks of at least 256
// rows (16 to COL_CHUNKS_MAX of them: more chunks fill the chip for large batches, but the second
// pass adds the C partials of a column in sequence), then the chunk partials in order.
void colsum(nnp_proposal *q, const float *X, int ld, int B, int N, float *out, hipStream_t s)
{
    const int nb = (int)blocks(N);
    const int C = std::max(1, std::min(std::max(16, B / 256), std::min(COL_CHUNKS_MAX, B)));
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(nb, C), dim3(256), 0, s, X, ld, B, N,
                       q->colpart);
    hipLaunchKernelGGL(colsum_final_kernel, dim3(nb), dim3(256), 0, s, q->colpart, C, N, out);
}

// Forward pass of B rows (padded to Bp) from enc into the workspace.
int forward_ws(nnp_proposal *q, const float *enc, int B, int Bp, hipStream_t s)
{
    const Layout &L = q->L;
    hipLaunchKernelGGL(input_kernel, dim3(blocks((size_t)Bp * ENC_PAD)), dim3(256), 0, s, enc, B,
                       Bp, q->xq);
    int rc = gemm(q, 0, 0, 1, Bp, HID, ENC_PAD, q->xq, ENC_PAD, q->wq + q->qW1, ENC_PAD,
                  q->params + L.ob1, nullptr, 0, q->a1, HID, q->h1q, HID, s);
    if (!rc) rc = gemm(q, 0, 0, 1, Bp, HID, HID, q->h1q, HID, q->wq + q->qW2, HID,
                       q->params + L.ob2, nullptr, 0, q->a2, HID, q->h2q, HID, s);
    if (!rc) rc = gemm(q, 0, 0, 0, Bp, L.ny_pad, HID, q->h2q, HID, q->wq + q->qW3, HID,
                       q->params + L.ob3, nullptr, 0, q->y, L.ny_pad, nullptr, 0, s);
    return rc;
}

// Loss and gradients into q->grads (internal layout); loss to `loss` if not null.
int backward_ws(nnp_proposal *q, const float *ts, int B, int Bp, float *loss, hipStream_t s)
{
    const Layout &L = q->L;
    const int nt = q->cfg.n_theta;
    hipLaunchKernelGGL(loss_kernel, dim3(Bp), dim3(256), 0, s, q->y, L.ny_pad, ts, nt, B, q->dyf,
                       q->dyq, q->partial);
    if (loss)
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, q->partial, B, loss);
    float *g = q->grads;
    // layer 3: dW3 = dy^T h2q, db3 = colsum(dy), dh2 = dy W3 -> da2 = dh2 * [a2 > 0]
    int rc = gemm_splitk(q, 1, 1, L.ny_pad, HID, Bp, q->dyq, L.ny_pad, q->h2q, HID, g + L.oW3,
                         HID, s);
    colsum(q, q->dyf, L.ny_pad, B, L.ny_pad, g + L.ob3, s);
    if (!rc) rc = gemm(q, 0, 1, 2, Bp, HID, L.ny_pad, q->dyq, L.ny_pad, q->wq + q->qW3, HID,
                       nullptr, q->a2, HID, q->da2, HID, q->da2q, HID, s);
    // layer 2
    if (!rc) rc = gemm_splitk(q, 1, 1, HID, HID, Bp, q->da2q, HID, q->h1q, HID, g + L.oW2, HID, s);
    colsum(q, q->da2, HID, B, HID, g + L.ob2, s);
    if (!rc) rc = gemm(q, 0, 1, 2, Bp, HID, HID, q->da2q, HID, q->wq + q->qW2, HID, nullptr,
                       q->a1, HID, q->da1, HID, q->da1q, HID, s);
    // layer 1
    if (!rc) rc = gemm_splitk(q, 1, 1, HID, ENC_PAD, Bp, q->da1q, HID, q->xq, ENC_PAD, g + L.oW1,
                              ENC_PAD, s);
    colsum(q, q->da1, HID, B, HID, g + L.ob1, s);
    if (!rc && hipGetLastError() != hipSuccess) rc = pfail(q, NNP_EDEVICE, "kernel launch failed");
    return rc;
}

// bfloat16 copies of the three weight matrices (W1 | W2 | W3, biases excluded).
void refresh_weights(nnp_proposal *q, hipStream_t s)
{
    const Layout &L = q->L;
    hipLaunchKernelGGL(quantize_kernel, dim3(blocks((size_t)HID * ENC_PAD)), dim3(256), 0, s,
                       q->params + L.oW1, HID * ENC_PAD, q->wq + q->qW1);
    hipLaunchKernelGGL(quantize_kernel, dim3(blocks((size_t)HID * HID)), dim3(256), 0, s,
                       q->params + L.oW2, HID * HID, q->wq + q->qW2);
    hipLaunchKernelGGL(quantize_kernel, dim3(blocks((size_t)L.ny_pad * HID)), dim3(256), 0, s,
                       q->params + L.oW3, L.ny_pad * HID, q->wq + q->qW3);
}

int check_batch(nnp_proposal *q, const float *enc, int B)
{
    if (!enc) return pfail(q, NNP_EINVAL, "null encodings");
    if (B < 1 || B > q->cfg.max_batch) return pfail(q, NNP_EINVAL, "B must be in [1, max_batch]");
    return NNP_OK;
}

}  // namespace

extern "C" {

int nnp_proposal_create(nnp_proposal **out, const nnp_proposal_config *c, int device)
{
    if (!out) return pfail(nullptr, NNP_EINVAL, "null handle pointer");
    *out = nullptr;
    if (!c) return pfail(nullptr, NNP_EINVAL, "null config");
    if (c->n_theta < 1 || c->n_theta > (1 << 20))
        return pfail(nullptr, NNP_EINVAL, "n_theta out of range");
    if (c->max_batch < 1 || c->max_batch > (1 << 20))
        return pfail(nullptr, NNP_EINVAL, "max_batch out of range");
    const float nv[5] = {c->norm_xi, c->norm_eta, c->norm_phi, c->norm_v, c->d_cap};
    for (float x : nv)
        if (!(x > 0.0f) || !isfinite(x)) return pfail(nullptr, NNP_EINVAL, "normalisers must be > 0");
    if (!isfinite(c->u_min) || !isfinite(c->u_max))
        return pfail(nullptr, NNP_EINVAL, "u_min / u_max must be finite");
    if (hipSetDevice(device) != hipSuccess) return pfail(nullptr, NNP_EDEVICE, "hipSetDevice failed");
    nnp_proposal *q = new nnp_proposal();
    q->cfg = *c;
    q->device = device;
    q->Bmax = (c->max_batch + ROWS - 1) / ROWS * ROWS;
    Layout &L = q->L;
    L.ny = 2 * c->n_theta;
    L.ny_pad = (L.ny + TN - 1) / TN * TN;
    L.oW1 = 0;
    L.ob1 = L.oW1 + (size_t)HID * ENC_PAD;
    L.oW2 = L.ob1 + HID;
    L.ob2 = L.oW2 + (size_t)HID * HID;
    L.oW3 = L.ob2 + HID;
    L.ob3 = L.oW3 + (size_t)L.ny_pad * HID;
    L.total = L.ob3 + L.ny_pad;
    L.eW1 = 0;
    L.eb1 = L.eW1 + (size_t)HID * ENC;
    L.eW2 = L.eb1 + HID;
    L.eb2 = L.eW2 + (size_t)HID * HID;
    L.eW3 = L.eb2 + HID;
    L.eb3 = L.eW3 + (size_t)L.ny * HID;
    L.etotal = L.eb3 + L.ny;
    q->qW1 = 0;
    q->qW2 = (size_t)HID * ENC_PAD;
    q->qW3 = q->qW2 + (size_t)HID * HID;
    q->nq = q->qW3 + (size_t)L.ny_pad * HID;
    const size_t Bp = (size_t)q->Bmax;
    int rc = alloc(q, &q->params, L.total);
    if (!rc) rc = alloc(q, &q->m, L.total);
    if (!rc) rc = alloc(q, &q->v, L.total);
    if (!rc) rc = alloc(q, &q->grads, L.total);
    if (!rc) rc = alloc(q, &q->wq, q->nq);
    if (!rc) rc = alloc(q, &q->xq, Bp * ENC_PAD);
    if (!rc) rc = alloc(q, &q->a1, Bp * HID);
    if (!rc) rc = alloc(q, &q->h1q, Bp * HID);
    if (!rc) rc = alloc(q, &q->a2, Bp * HID);
    if (!rc) rc = alloc(q, &q->h2q, Bp * HID);
    if (!rc) rc = alloc(q, &q->y, Bp * L.ny_pad);
    if (!rc) rc = alloc(q, &q->dyf, Bp * L.ny_pad);
    if (!rc) rc = alloc(q, &q->dyq, Bp * L.ny_pad);
    if (!rc) rc = alloc(q, &q->da2, Bp * HID);
    if (!rc) rc = alloc(q, &q->da2q, Bp * HID);
    if (!rc) rc = alloc(q, &q->da1, Bp * HID);
    if (!rc) rc = alloc(q, &q->da1q, Bp * HID);
    if (!rc) rc = alloc(q, &q->partial, Bp);
    if (!rc) rc = alloc(q, &q->loss_tmp, 1);
    q->splitk_floats = (size_t)32 * HID * HID;        // slices of the largest split products
    q->splitk_floats = std::max(q->splitk_floats, (size_t)16 * L.ny_pad * HID);
    if (!rc) rc = alloc(q, &q->splitk, q->splitk_floats);
    if (!rc) rc = alloc(q, &q->colpart, (size_t)COL_CHUNKS_MAX * L.ny_pad);
    if (rc) {
        nnp_proposal_destroy(q);
        return pfail(nullptr, NNP_ENOMEM, "device allocation failed");
    }
    bool ok = true;
    for (float *p : {q->params, q->m, q->v, q->grads})
        ok = ok && hipMemset(p, 0, L.total * sizeof(float)) == hipSuccess;
    ok = ok && hipMemset(q->wq, 0, q->nq * sizeof(uint16_t)) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&q->enc_copied, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        nnp_proposal_destroy(q);
        return pfail(nullptr, NNP_EDEVICE, "device initialisation failed");
    }
    *out = q;
    return NNP_OK;
}

void nnp_proposal_destroy(nnp_proposal *q)
{
    if (!q) return;
    hipSetDevice(q->device);
    hipDeviceSynchronize();
    for (void *p : q->allocs) hipFree(p);
    if (q->d_enc) hipFree(q->d_enc);
    if (q->h_enc) hipHostFree(q->h_enc);
    if (q->enc_copied) hipEventDestroy(q->enc_copied);
    delete q;
}

int nnp_proposal_n_params(const nnp_proposal *q) { return q ? (int)q->L.etotal : 0; }

int nnp_proposal_set_params(nnp_proposal *q, const float *params, void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    if (!params) return pfail(q, NNP_EINVAL, "null params");
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    const size_t bytes = q->L.total * sizeof(float);
    if (hipMemsetAsync(q->params, 0, bytes, s) != hipSuccess ||
        hipMemsetAsync(q->m, 0, bytes, s) != hipSuccess ||
        hipMemsetAsync(q->v, 0, bytes, s) != hipSuccess)
        return pfail(q, NNP_EDEVICE, "hipMemsetAsync failed");
    hipLaunchKernelGGL(pack_kernel, dim3(blocks(q->L.etotal)), dim3(256), 0, s, q->L, params,
                       q->params, 0);
    refresh_weights(q, s);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    q->step = 0;
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_get_params(nnp_proposal *q, float *params, void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    if (!params) return pfail(q, NNP_EINVAL, "null params");
    hipLaunchKernelGGL(pack_kernel, dim3(blocks(q->L.etotal)), dim3(256), 0,
                       (hipStream_t)hip_stream, q->L, q->params, params, 1);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_get_state(nnp_proposal *q, float *params, float *m, float *v, int64_t *step,
                           void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    if (!params || !step) return pfail(q, NNP_EINVAL, "null params or step");
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    const dim3 grid(blocks(q->L.etotal)), block(256);
    hipLaunchKernelGGL(pack_kernel, grid, block, 0, s, q->L, q->params, params, 1);
    if (m) hipLaunchKernelGGL(pack_kernel, grid, block, 0, s, q->L, q->m, m, 1);
    if (v) hipLaunchKernelGGL(pack_kernel, grid, block, 0, s, q->L, q->v, v, 1);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    *step = q->step;
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_set_state(nnp_proposal *q, const float *params, const float *m, const float *v,
                           int64_t step, void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    if (!params || !m || !v) return pfail(q, NNP_EINVAL, "null params, m or v");
    if (step < 0 || step > INT32_MAX) return pfail(q, NNP_EINVAL, "step out of range");
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    const size_t bytes = q->L.total * sizeof(float);
    if (hipMemsetAsync(q->params, 0, bytes, s) != hipSuccess ||
        hipMemsetAsync(q->m, 0, bytes, s) != hipSuccess ||
        hipMemsetAsync(q->v, 0, bytes, s) != hipSuccess)
        return pfail(q, NNP_EDEVICE, "hipMemsetAsync failed");
    const dim3 grid(blocks(q->L.etotal)), block(256);
    hipLaunchKernelGGL(pack_kernel, grid, block, 0, s, q->L, params, q->params, 0);
    hipLaunchKernelGGL(pack_kernel, grid, block, 0, s, q->L, m, q->m, 0);
    hipLaunchKernelGGL(pack_kernel, grid, block, 0, s, q->L, v, q->v, 0);
    refresh_weights(q, s);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    q->step = (int)step;
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_encode(nnp_proposal *q, const nnp_problem *probs, int count, float *enc,
                        void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    if (!probs || !enc) return pfail(q, NNP_EINVAL, "null argument");
    if (count < 1 || count > 65535) return pfail(q, NNP_EINVAL, "count must be in [1, 65535]");
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    std::vector<EncProblem> v((size_t)count);
    const float a_idle = q->cfg.u_max > q->cfg.u_min
                             ? -1.0f - 2.0f * q->cfg.u_min / (q->cfg.u_max - q->cfg.u_min)
                             : 0.0f;
    for (int i = 0; i < count; ++i) {
        const nnp_problem &p = probs[i];
        if (p.P < 0 || p.P > NNP_MAX_P || (p.P > 0 && !p.obst) || p.T < 1 || p.T > NNP_MAX_T)
            return pfail(q, NNP_EINVAL, "problem " + std::to_string(i) + ": bad P, obst or T");
        for (int k = 0; k < 4; ++k)
            if (!isfinite(p.z0[k]) || !isfinite(p.goal[k]))
                return pfail(q, NNP_EINVAL, "problem " + std::to_string(i) + ": non-finite state");
        EncProblem &e = v[(size_t)i];
        memcpy(e.z0, p.z0, sizeof e.z0);
        memcpy(e.goal, p.goal, sizeof e.goal);
        e.a_prev[0] = p.a_prev ? p.a_prev[0] : 0.0f;
        e.a_prev[1] = p.a_prev ? p.a_prev[1] : a_idle;
        e.T = p.T;
        e.P = p.P;
        e.obst = reinterpret_cast<const float4 *>(p.obst);
    }
    hipError_t err = hipEventSynchronize(q->enc_copied);   // staging buffer free again
    if (err != hipSuccess) return pfail(q, NNP_EDEVICE, "hipEventSynchronize failed");
    if (count > q->enc_cap) {
        if (q->h_enc) hipHostFree(q->h_enc);
        q->h_enc = nullptr;
        EncProblem *d = nullptr;
        if (hipHostMalloc(&q->h_enc, (size_t)count * sizeof(EncProblem), hipHostMallocDefault) !=
                hipSuccess ||
            hipMalloc(&d, (size_t)count * sizeof(EncProblem)) != hipSuccess) {
            q->enc_cap = 0;
            return pfail(q, NNP_ENOMEM, "encoding descriptor allocation failed");
        }
        if (q->d_enc) {
            hipStreamSynchronize(s);
            hipFree(q->d_enc);
        }
        q->d_enc = d;
        q->enc_cap = count;
    }
    memcpy(q->h_enc, v.data(), v.size() * sizeof(EncProblem));
    if (hipMemcpyAsync(q->d_enc, q->h_enc, v.size() * sizeof(EncProblem), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipEventRecord(q->enc_copied, s) != hipSuccess)
        return pfail(q, NNP_EDEVICE, "descriptor copy failed");
    const EncNorms nm{q->cfg.norm_xi, q->cfg.norm_eta, q->cfg.norm_phi, q->cfg.norm_v, q->cfg.d_cap};
    hipLaunchKernelGGL(encode_kernel, dim3(count), dim3(256), 0, s, q->d_enc, nm, enc);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "encode launch failed");
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_forward(nnp_proposal *q, const float *enc, int B, float *mu, float *log_sigma,
                         void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    int rc = check_batch(q, enc, B);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    const int Bp = (B + ROWS - 1) / ROWS * ROWS;
    rc = forward_ws(q, enc, B, Bp, s);
    if (rc) return rc;
    if (mu || log_sigma)
        hipLaunchKernelGGL(split_kernel, dim3(blocks((size_t)B * q->cfg.n_theta)), dim3(256), 0, s,
                           q->y, q->L.ny_pad, B, q->cfg.n_theta, mu, log_sigma);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_gradients(nnp_proposal *q, const float *enc, const float *theta_star, int B,
                           float *grads, float *loss, void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    int rc = check_batch(q, enc, B);
    if (rc) return rc;
    if (!theta_star) return pfail(q, NNP_EINVAL, "null theta_star");
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    const int Bp = (B + ROWS - 1) / ROWS * ROWS;
    rc = forward_ws(q, enc, B, Bp, s);
    if (!rc) rc = backward_ws(q, theta_star, B, Bp, loss, s);
    if (rc) return rc;
    if (grads)
        hipLaunchKernelGGL(pack_kernel, dim3(blocks(q->L.etotal)), dim3(256), 0, s, q->L, q->grads,
                           grads, 1);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    q->err.clear();
    return NNP_OK;
}

int nnp_proposal_train_step(nnp_proposal *q, const float *enc, const float *theta_star, int B,
                            float lr, float *loss, void *hip_stream)
{
    if (!q) return NNP_EINVAL;
    int rc = check_batch(q, enc, B);
    if (rc) return rc;
    if (!theta_star) return pfail(q, NNP_EINVAL, "null theta_star");
    if (!(lr > 0.0f) || !isfinite(lr)) return pfail(q, NNP_EINVAL, "lr must be positive");
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(q->device) != hipSuccess) return pfail(q, NNP_EDEVICE, "hipSetDevice failed");
    const int Bp = (B + ROWS - 1) / ROWS * ROWS;
    rc = forward_ws(q, enc, B, Bp, s);
    if (!rc) rc = backward_ws(q, theta_star, B, Bp, loss, s);
    if (rc) return rc;
    const int t = q->step + 1;
    const float c1 = (float)(1.0 / (1.0 - pow(0.9, t)));
    const float c2 = (float)(1.0 / (1.0 - pow(0.999, t)));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(q->L.total)), dim3(256), 0, s, q->params, q->m,
                       q->v, q->grads, (int)q->L.total, lr, c1, c2);
    refresh_weights(q, s);
    if (hipGetLastError() != hipSuccess) return pfail(q, NNP_EDEVICE, "kernel launch failed");
    q->step = t;
    q->err.clear();
    return NNP_OK;
}

int nnp_gemm_bf16(int a_layout, int b_layout, int M, int N, int K, const uint16_t *A, int lda,
                  const uint16_t *B, int ldb, int epilogue, const float *bias, const float *mask,
                  int ldm, float *C, int ldc, uint16_t *Cq, int ldcq, void *hip_stream)
{
    if (!A || !B || (!C && !Cq)) return NNP_EINVAL;
    if ((a_layout | b_layout) & ~1 || epilogue < 0 || epilogue > 2) return NNP_EINVAL;
    if (M <= 0 || N <= 0 || K <= 0 || M % TM || N % TN || K % TK) return NNP_EINVAL;
    if (M / TM > 65535) return NNP_EINVAL;
    if (lda % 8 || ldb % 8 || (C && ldc < N) || (Cq && ldcq < N)) return NNP_EINVAL;
    if (lda < (a_layout ? M : K) || ldb < (b_layout ? N : K)) return NNP_EINVAL;
    if (((uintptr_t)A | (uintptr_t)B) & 15) return NNP_EINVAL;
    if (epilogue == 2 && (!mask || ldm < N)) return NNP_EINVAL;
    GemmArgs g{A, B, lda, ldb, M, N, K, bias, mask, ldm, C, ldc, Cq, ldcq, nullptr};
    return launch_gemm(a_layout, b_layout, epilogue, g, (hipStream_t)hip_stream);
}

const char *nnp_proposal_last_error(const nnp_proposal *q)
{
    return q ? q->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
