// Learned cap corrector: a 6 -> 128 -> 128 -> 3 network with the tanh form of
// GELU that maps the inner-triangle vertices relative to the outer point (in
// the normalised frame of mlp_features) to the three basis-weighted integrals over the caps of
// the arc-subdivided ball (Sec. 4.2.2), in units of delta^2 times a fixed
// output scale.  Layer 1 (K = 6) runs on the FP32 vector unit; layers 2 and 3
// run on bf16 matrix cores (32x32x16 MFMA) with FP32 accumulation.  Training
// (forward, backward, Adam) uses the same kernels; labels come from the FP64
// arc subdivision on the GPU.
#include "nla_device.hpp"
#include <rocprim/device/device_select.hpp>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <vector>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int H = 128;
constexpr int LDW = 136;   // LDS row stride (bf16) of the 128-wide weight tiles: rows 16 bytes apart in bank space
enum { OW1 = 0, OB1 = 768, OW2 = 896, OB2 = 17280, OW3 = 17408, OB3 = 17792, NW = 17795 };

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// float -> bfloat16, round to nearest even: the hardware conversion
// (v_cvt_pk_bf16_f32, two values per instruction) under the default FP32 mode
// (round to nearest even, subnormals kept)
__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }
__device__ __forceinline__ float from_bf16(__bf16 b)
{
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, b) << 16);
}

// GELU, tanh form: g(z) = z/2 (1 + tanh(u)), u = sqrt(2/pi) (z + 0.044715 z^3),
// evaluated as z * sigmoid(2u) with the hardware exp2 and reciprocal; s = sigmoid(2u)
__device__ __forceinline__ float gelu_s(float z, float &s)
{
    const float u = 0.7978845608f * (z + 0.044715f * z * z * z);
    const float e = __builtin_amdgcn_exp2f(-2.8853900818f * u);
    s = __builtin_amdgcn_rcpf(1.f + e);
    return z * s;
}
// g'(z) = s + z s (1 - s) 2 u'(z)
__device__ __forceinline__ float gelu_d(float z, float s)
{
    const float du = 0.7978845608f * (1.f + 3.f * 0.044715f * z * z);
    return s + 2.f * z * s * (1.f - s) * du;
}

// SplitMix64 (Steele, Lea, Flood 2014), output number idx of the stream of seed
__device__ __forceinline__ double splitmix_u(uint64_t seed, uint64_t idx)
{
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}
inline uint64_t splitmix_host(uint64_t seed, uint64_t idx)
{
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// weights as the kernels read them
struct MlpW {
    const float *w;          // master FP32, flat layout (W1, b1, b2, b3 used directly)
    const __bf16 *w2, *w2t;  // W2 [out][in] and its transpose, bf16
    const __bf16 *w3p;       // W3 in the slot order of the layer-3 operand, rows 3..31 zero, bf16
    const float *w3e;        // W3 as the network uses it (bf16 values), [3][128]
};

// activations kept by a training forward pass (batch positions, padded to Bp)
struct TrainBuf {
    int64_t Bp;
    float *fpos;     // [Bp][6]
    float *gd1;      // [Bp][128] g'(z1)
    __bf16 *h1t;     // [128][Bp] bf16 h1 (transposed)
    float *gd2;      // [Bp][128] g'(z2)
    float *h2;       // [Bp][128] bf16-rounded h2
    float *dy;       // [Bp][3]
    float *sq;       // [Bp] squared error
    float *dz1;      // [Bp][128]
    float *dz2f;     // [Bp][128]
    __bf16 *dz2t;    // [128][Bp]
    float *part;     // [Bp/16][1412] chunk sums of the reduction
};

__global__ void k_mlp_refresh(const float *__restrict__ w, __bf16 *__restrict__ w2, __bf16 *__restrict__ w2t,
                              __bf16 *__restrict__ w3p, float *__restrict__ w3e)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < H * H) {
        const int o = i >> 7, c = i & 127;
        const __bf16 b = to_bf16(w[OW2 + i]);
        w2[i] = b;
        w2t[c * H + o] = b;
    } else if (i < H * H + 32 * H) {
        const int j = i - H * H, o = j >> 7, c = j & 127;
        const int kk = c >> 4, r = c & 15, hb = r >> 3, jj = r & 7;
        const int src = 16 * kk + 8 * (jj >> 2) + 4 * hb + (jj & 3);
        w3p[j] = to_bf16(o < 3 ? w[OW3 + o * H + src] : 0.f);
        if (o < 3) w3e[o * H + c] = from_bf16(to_bf16(w[OW3 + o * H + c]));
    }
}

__device__ __forceinline__ void load_tile_lds(__bf16 *dst, const __bf16 *__restrict__ src, int rows)
{
    // rows x 128 bf16, 16-byte chunks, into rows of stride LDW
    for (int c = threadIdx.x; c < rows * 16; c += blockDim.x) {
        const int r = c >> 4, k8 = (c & 15) * 8;
        *(uint4 *)&dst[r * LDW + k8] = *(const uint4 *)&src[r * H + k8];
    }
}

// Forward pass over tiles of 32 items, one wavefront per tile.
// MODE 0: inference, out[i][3] = network output.
// MODE 1: training step, item = permutation of the batch position; keeps the
//         activations and writes dy = gcoef (y - label/scale).
// MODE 2: gradient hook, dy = dout (identity order).
// Lane l handles item l%32 and the hidden half l/32; layer 1 produces the
// bf16 operand of layer 2 directly in the layout the MFMA expects.
template <int MODE>
__global__ __launch_bounds__(256, 3) void k_mlp_fwd(int64_t n, const float *__restrict__ feat,
                                                 const float *__restrict__ label, const float *__restrict__ dout,
                                                 MlpW W, float inv_scale, float gcoef, int64_t pa, int64_t pb,
                                                 int64_t base, int64_t n_total, float *__restrict__ out, TrainBuf T)
{
    __shared__ __attribute__((aligned(16))) __bf16 sW2[H * LDW];
    __shared__ __attribute__((aligned(16))) __bf16 sW3[32 * LDW];
    __shared__ float sW1[H * 6], sB1[H], sB2[H], sB3[4];
    load_tile_lds(sW2, W.w2, H);
    load_tile_lds(sW3, W.w3p, 32);
    for (int i = threadIdx.x; i < H * 6; i += blockDim.x) sW1[i] = W.w[OW1 + i];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        sB1[i] = W.w[OB1 + i];
        sB2[i] = W.w[OB2 + i];
    }
    if (threadIdx.x < 3) sB3[threadIdx.x] = W.w[OB3 + threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 31, hb = lane >> 5;
    const int64_t ntiles = (MODE == 0 ? n + 31 : T.Bp) / 32;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntiles; t += (int64_t)gridDim.x * 4) {
        // keeps the weight reads from LDS inside the loop (hoisted, they would not fit in registers)
        __asm__ volatile("" ::: "memory");
        const int64_t pos = t * 32 + m;
        const bool ok = pos < n;
        int64_t src = pos;
        if (MODE == 1 && ok) src = (pa * (base + pos) + pb) % n_total;
        float f[6];
#pragma unroll
        for (int c = 0; c < 6; c++) f[c] = ok ? feat[src * 6 + c] : 0.f;
        if (MODE != 0 && hb == 0)
#pragma unroll
            for (int c = 0; c < 6; c++) T.fpos[pos * 6 + c] = f[c];
        bf16x8 x1[8];
#pragma unroll
        for (int kk = 0; kk < 8; kk++) {
            float gd[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int h = 16 * kk + 8 * hb + j;
                float z = sB1[h];
#pragma unroll
                for (int c = 0; c < 6; c++) z += sW1[h * 6 + c] * f[c];
                float s;
                const float g = gelu_s(z, s);
                const __bf16 b = to_bf16(g);
                x1[kk][j] = b;
                if (MODE != 0) {
                    gd[j] = gelu_d(z, s);
                    T.h1t[(int64_t)h * T.Bp + pos] = b;
                }
            }
            if (MODE != 0) {
                float4 *d = (float4 *)&T.gd1[pos * H + 16 * kk + 8 * hb];
                d[0] = make_float4(gd[0], gd[1], gd[2], gd[3]);
                d[1] = make_float4(gd[4], gd[5], gd[6], gd[7]);
            }
        }
        // layer 2 one 32-row tile of hidden units at a time: MFMA, then bias + GELU;
        // acc[i] = z2[hidden 32 mt + 8 (i/4) + 4 hb + i%4][item m]
        bf16x8 x2[8];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            f32x16 acc;
#pragma unroll
            for (int i = 0; i < 16; i++) acc[i] = 0.f;
#pragma unroll
            for (int kk = 0; kk < 8; kk++) {
                const bf16x8 A = *(const bf16x8 *)&sW2[(32 * mt + m) * LDW + 16 * kk + 8 * hb];
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, x1[kk], acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int h = 32 * mt + 8 * (i >> 2) + 4 * hb + (i & 3);
                const float z = acc[i] + sB2[h];
                float s;
                const float g = gelu_s(z, s);
                const __bf16 b = to_bf16(g);
                x2[2 * mt + (i >> 3)][i & 7] = b;
                if (MODE != 0) {
                    T.gd2[pos * H + h] = gelu_d(z, s);
                    T.h2[pos * H + h] = from_bf16(b);
                }
            }
        }
        f32x16 a3;
#pragma unroll
        for (int i = 0; i < 16; i++) a3[i] = 0.f;
#pragma unroll
        for (int kk = 0; kk < 8; kk++) {
            const bf16x8 A = *(const bf16x8 *)&sW3[m * LDW + 16 * kk + 8 * hb];
            a3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, x2[kk], a3, 0, 0, 0);
        }
        // rows 0..2 of the output tile sit in a3[0..2] of lanes 0..31
        if (hb == 0) {
            float y[3] = {a3[0] + sB3[0], a3[1] + sB3[1], a3[2] + sB3[2]};
            if (MODE == 0) {
                if (ok)
#pragma unroll
                    for (int o = 0; o < 3; o++) out[pos * 3 + o] = y[o];
            } else if (MODE == 1) {
                float sq = 0.f;
#pragma unroll
                for (int o = 0; o < 3; o++) {
                    const float d = ok ? y[o] - label[src * 3 + o] * inv_scale : 0.f;
                    T.dy[pos * 3 + o] = gcoef * d;
                    sq += d * d;
                }
                T.sq[pos] = sq;
            } else {
#pragma unroll
                for (int o = 0; o < 3; o++) T.dy[pos * 3 + o] = ok ? dout[pos * 3 + o] : 0.f;
                T.sq[pos] = 0.f;
            }
        }
    }
}

// Backward through layers 3 and 2 per tile: dz2 = (W3^T dy) g'(z2) (vector
// unit, in the operand layout), dh1 = W2^T dz2 (MFMA), dz1 = dh1 g'(z1).
__global__ __launch_bounds__(256, 3) void k_mlp_bwd(MlpW W, TrainBuf T)
{
    __shared__ __attribute__((aligned(16))) __bf16 sW2T[H * LDW];
    __shared__ float sW3e[3 * H];
    load_tile_lds(sW2T, W.w2t, H);
    for (int i = threadIdx.x; i < 3 * H; i += blockDim.x) sW3e[i] = W.w3e[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 31, hb = lane >> 5;
    const int64_t ntiles = T.Bp / 32;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntiles; t += (int64_t)gridDim.x * 4) {
        __asm__ volatile("" ::: "memory");
        const int64_t pos = t * 32 + m;
        const float dy0 = T.dy[pos * 3], dy1 = T.dy[pos * 3 + 1], dy2 = T.dy[pos * 3 + 2];
        bf16x8 z2b[8];
#pragma unroll
        for (int kk = 0; kk < 8; kk++)
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int o = 16 * kk + 8 * hb + j;
                const float v = (sW3e[o] * dy0 + sW3e[H + o] * dy1 + sW3e[2 * H + o] * dy2) * T.gd2[pos * H + o];
                const __bf16 b = to_bf16(v);
                z2b[kk][j] = b;
                T.dz2f[pos * H + o] = v;
                T.dz2t[(int64_t)o * T.Bp + pos] = b;
            }
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            f32x16 acc;
#pragma unroll
            for (int i = 0; i < 16; i++) acc[i] = 0.f;
#pragma unroll
            for (int kk = 0; kk < 8; kk++) {
                const bf16x8 A = *(const bf16x8 *)&sW2T[(32 * mt + m) * LDW + 16 * kk + 8 * hb];
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, z2b[kk], acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int h = 32 * mt + 8 * (i >> 2) + 4 * hb + (i & 3);
                T.dz1[pos * H + h] = acc[i] * T.gd1[pos * H + h];
            }
        }
    }
}

// dW2[o][i] = sum_s dz2[s][o] h1[s][i]: one block per 32x32 output tile, the
// four waves split the batch and their partial tiles are added in wave order.
__global__ __launch_bounds__(256) void k_mlp_dw2(TrainBuf T, float *__restrict__ g)
{
    __shared__ float part[3][16][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 31, hb = lane >> 5;
    const int to = blockIdx.x >> 2, ti = blockIdx.x & 3;
    const int64_t q = T.Bp / 4, lo = q * wv, hi = lo + q;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; i++) acc[i] = 0.f;
    const __bf16 *ra = T.dz2t + (int64_t)(32 * to + m) * T.Bp + 8 * hb;
    const __bf16 *rb = T.h1t + (int64_t)(32 * ti + m) * T.Bp + 8 * hb;
    for (int64_t s0 = lo; s0 < hi; s0 += 16)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8 *)(ra + s0), *(const bf16x8 *)(rb + s0), acc, 0, 0, 0);
    if (wv > 0)
#pragma unroll
        for (int i = 0; i < 16; i++) part[wv - 1][i][lane] = acc[i];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int i = 0; i < 16; i++) {
            float v = acc[i];
            for (int w = 0; w < 3; w++) v += part[w][i][lane];
            const int o = 32 * to + 8 * (i >> 2) + 4 * hb + (i & 3), c = 32 * ti + m;
            g[OW2 + o * H + c] = v;
        }
    }
}

// the remaining gradients (dW1, b1, b2, dW3, b3) and the batch loss: each
// block sums a chunk of RCH batch positions for all 1412 values (threads over
// values, so reads of a position's row are coalesced), then the chunks are
// added in chunk order.  Short chunks give a 4096-sample batch 256 blocks, so
// the sums' load latency is spread over the whole chip.
constexpr int RCH = 16, NRED = 1412;

__device__ __forceinline__ float red_term(const TrainBuf &T, int r, int64_t p)
{
    if (r < 768) return T.dz1[p * H + r / 6] * T.fpos[p * 6 + r % 6];
    if (r < 896) return T.dz1[p * H + (r - 768)];
    if (r < 1024) return T.dz2f[p * H + (r - 896)];
    if (r < 1408) return T.dy[p * 3 + (r - 1024) / H] * T.h2[p * H + (r - 1024) % H];
    if (r < 1411) return T.dy[p * 3 + (r - 1408)];
    return T.sq[p];
}

// block (chunk x, value range y): one value per thread, so the chunk's values
// are summed by many waves at once
__global__ __launch_bounds__(256) void k_mlp_reduce_part(TrainBuf T, float *__restrict__ part)
{
    const int64_t p0 = (int64_t)blockIdx.x * RCH;
    const int r = blockIdx.y * blockDim.x + threadIdx.x;
    if (r >= NRED) return;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < RCH; i++) s += red_term(T, r, p0 + i);
    part[(int64_t)blockIdx.x * NRED + r] = s;
}

__global__ void k_mlp_reduce_final(int nchunk, const float *__restrict__ part, float *__restrict__ g,
                                   float *__restrict__ loss_out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= NRED) return;
    // four running sums over chunks c = 0, 1, 2, 3 mod 4, combined in a fixed
    // order; 32 chunks' loads are issued before their additions (each sum still
    // takes its chunks in increasing order)
    float s4[4] = {0.f, 0.f, 0.f, 0.f};
    int c = 0;
    for (; c + 32 <= nchunk; c += 32) {
        float v[32];
#pragma unroll
        for (int j = 0; j < 32; j++) v[j] = part[(int64_t)(c + j) * NRED + r];
#pragma unroll
        for (int j = 0; j < 32; j++) s4[j & 3] += v[j];
    }
    for (; c + 4 <= nchunk; c += 4) {
#pragma unroll
        for (int j = 0; j < 4; j++) s4[j] += part[(int64_t)(c + j) * NRED + r];
    }
    for (; c < nchunk; c++) s4[0] += part[(int64_t)c * NRED + r];
    const float s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    if (r < 768) g[OW1 + r] = s;
    else if (r < 896) g[OB1 + (r - 768)] = s;
    else if (r < 1024) g[OB2 + (r - 896)] = s;
    else if (r < 1408) g[OW3 + (r - 1024)] = s;
    else if (r < 1411) g[OB3 + (r - 1408)] = s;
    else if (loss_out) *loss_out = s;
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       float lr_t, float b1, float b2, float eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NW) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr_t * mi / (sqrtf(vi) + eps);
}

// root mean square of the labels (FP64, fixed order: strided thread sums, then a tree)
__global__ __launch_bounds__(1024) void k_label_rms(int64_t n3, const float *__restrict__ lab, double *__restrict__ out)
{
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n3; i += 1024) s += (double)lab[i] * lab[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0] / (double)(n3 > 0 ? n3 : 1));
}

// Training domain of n samples (MlpDomain): per block, the minimum and maximum
// of the squared vertex distances and squared edge lengths of the samples'
// triangles in units of delta, recovered from the float inputs f
// (v_a = R^-1 (f_a / 8 + (1, 0)), so |v_a|^2 = (f_a0 / 8 + 1)^2 + (f_a1 / 8)^2
// and |v_b - v_a|^2 = |f_b - f_a|^2 / 64) in FP64 with every operation rounded
// on its own; a second pass reduces the blocks.  Minima and maxima do not
// depend on the order.
constexpr int NDOM = 2;     // squared vertex distances, squared edge lengths
__global__ __launch_bounds__(256) void k_feat_domain(int64_t n, const float *__restrict__ feat, double *__restrict__ part)
{
#pragma clang fp contract(off)
    __shared__ double lo_s[NDOM][256], hi_s[NDOM][256];
    double lo[NDOM], hi[NDOM];
#pragma unroll
    for (int i = 0; i < NDOM; i++) {
        lo[i] = HUGE_VAL;
        hi[i] = -HUGE_VAL;
    }
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        double f[6];
#pragma unroll
        for (int i = 0; i < 6; i++) f[i] = (double)feat[6 * j + i];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int b = (a + 1) % 3;
            const double px = f[2 * a] * 0.125 + 1.0, py = f[2 * a + 1] * 0.125;
            const double r = px * px + py * py;
            const double dx = f[2 * b] - f[2 * a], dy = f[2 * b + 1] - f[2 * a + 1];
            const double e = (dx * dx + dy * dy) * (1.0 / 64.0);
            lo[0] = fmin(lo[0], r);
            hi[0] = fmax(hi[0], r);
            lo[1] = fmin(lo[1], e);
            hi[1] = fmax(hi[1], e);
        }
    }
#pragma unroll
    for (int i = 0; i < NDOM; i++) {
        lo_s[i][threadIdx.x] = lo[i];
        hi_s[i][threadIdx.x] = hi[i];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int i = 0; i < NDOM; i++) {
                lo_s[i][threadIdx.x] = fmin(lo_s[i][threadIdx.x], lo_s[i][threadIdx.x + w]);
                hi_s[i][threadIdx.x] = fmax(hi_s[i][threadIdx.x], hi_s[i][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < NDOM) {
        part[2 * NDOM * blockIdx.x + threadIdx.x] = lo_s[threadIdx.x][0];
        part[2 * NDOM * blockIdx.x + NDOM + threadIdx.x] = hi_s[threadIdx.x][0];
    }
}

// ------------------------------------------------------------- samples
struct LabelF {
    double *m;
    __device__ __forceinline__ void operator()(const double (&t)[3][5]) const
    {
        const double a = 0.5 * fabs((t[1][0] - t[0][0]) * (t[2][1] - t[0][1]) - (t[1][1] - t[0][1]) * (t[2][0] - t[0][0]));
#pragma unroll
        for (int b = 0; b < 3; b++) m[b] += a * ((t[0][2 + b] + t[1][2 + b]) + t[2][2 + b]) * (1.0 / 3.0);
    }
};

// One training candidate per thread from ten SplitMix64 uniforms (units of
// delta around x = 0): a right triangle of legs L from one of the four halves
// of a grid cell, centre at distance 1 + (2u1 - 1) sqrt(2) L in direction
// 2 pi u2, vertices jittered by jitter L (2u - 1), vertex order rotated by
// floor(3 u9).  Label = integrals of the basis over the cap triangles of the
// arc subdivision (the region with caps minus the inscribed polygon, both
// from the FP64 retriangulation).  Valid: at least one cap and every vertex
// at least band away from the circle.
template <bool POW2>
__global__ void k_cap_samples(int64_t n, uint64_t seed, int64_t first, double L, double jitter, double band,
                              int ncap, float *__restrict__ feat, float *__restrict__ lab, uint8_t *__restrict__ flag)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double u[10];
    for (int j = 0; j < 10; j++) u[j] = splitmix_u(seed, (uint64_t)(first + c) * 10 + j);
    const double shapes[4][6] = {{0, 0, 1, 0, 1, 1}, {0, 0, 1, 1, 0, 1}, {0, 0, 1, 0, 0, 1}, {1, 0, 1, 1, 0, 1}};
    int s = (int)(4.0 * u[0]);
    if (s > 3) s = 3;
    const double r = 1.0 + (2.0 * u[1] - 1.0) * sqrt(2.0) * L;
    const double ph = 2.0 * 3.14159265358979323846 * u[2];
    const double ox = r * cos(ph) - 0.5 * L, oy = r * sin(ph) - 0.5 * L;
    double V0[6], V[6];
    for (int a = 0; a < 3; a++) {
        V0[2 * a] = ox + L * shapes[s][2 * a] + jitter * L * (2.0 * u[3 + 2 * a] - 1.0);
        V0[2 * a + 1] = oy + L * shapes[s][2 * a + 1] + jitter * L * (2.0 * u[4 + 2 * a] - 1.0);
    }
    int rot = (int)(3.0 * u[9]);
    if (rot > 2) rot = 2;
    for (int a = 0; a < 3; a++) {
        const int b = (a + rot) % 3;
        V[2 * a] = V0[2 * b];
        V[2 * a + 1] = V0[2 * b + 1];
    }
    double mall[3] = {0, 0, 0}, mpoly[3] = {0, 0, 0};
    int ns = 0, ns0 = 0;
    LabelF fa{mall}, fp{mpoly};
    double cb[12];
    partial_item<POW2>(0.0, 0.0, V, 1.0, ncap, fa, ns, cb);
    partial_item<POW2>(0.0, 0.0, V, 1.0, 0, fp, ns0, cb);
    // every vertex at least band from the circle: |v|^2 >= (1 + band)^2 or |v|^2 <= (1 - band)^2
    const double hi = 1.0 + band, lo = band < 1.0 ? 1.0 - band : 0.0;
    bool far = true;
    for (int a = 0; a < 3; a++) {
        const double d2 = V[2 * a] * V[2 * a] + V[2 * a + 1] * V[2 * a + 1];
        far = far && (d2 >= hi * hi || d2 <= lo * lo);
    }
    const bool valid = (ns >> 16) > 0 && far;
    float fv[6];
    mlp_features(0.0, 0.0, V, 1.0, fv);
    for (int i = 0; i < 6; i++) feat[c * 6 + i] = fv[i];
    for (int b = 0; b < 3; b++) lab[c * 3 + b] = (float)(mall[b] - mpoly[b]);
    flag[c] = valid ? 1 : 0;
}

struct F6 { float v[6]; };
struct F3 { float v[3]; };

MlpDomain unbounded_domain() { return MlpDomain{-HUGE_VAL, HUGE_VAL, -HUGE_VAL, HUGE_VAL}; }

// {rlo, rhi, elo, ehi}: no NaN, lo <= hi
bool valid_domain(const double *d)
{
    for (int i = 0; i < 4; i++)
        if (std::isnan(d[i])) return false;
    return d[0] <= d[1] && d[2] <= d[3];
}

void domain_to(const MlpDomain &D, double *d)
{
    d[0] = D.rlo;
    d[1] = D.rhi;
    d[2] = D.elo;
    d[3] = D.ehi;
}

MlpDomain domain_from(const double *d) { return MlpDomain{d[0], d[1], d[2], d[3]}; }

} // namespace

// =====================================================================
struct nla_mlp {
    int device = 0;
    DeviceArena arena;
    float *w = nullptr, *g = nullptr, *am = nullptr, *av = nullptr, *w3e = nullptr;
    __bf16 *w2 = nullptr, *w2t = nullptr, *w3p = nullptr;
    double *rms = nullptr;
    float scale = 0.f;
    MlpDomain dom = unbounded_domain();
    int64_t step = 0;        // epochs trained (seeds the epoch orders)
    int64_t adam_t = 0;      // Adam steps taken
    // training scratch
    DeviceArena *scratch = nullptr;
    TrainBuf T{};
    float *lossb = nullptr;
    int64_t loss_cap = 0;
    ~nla_mlp() { delete scratch; }
};

static MlpW mlp_view(const nla_mlp *M) { return MlpW{M->w, M->w2, M->w2t, M->w3p, M->w3e}; }

static int mlp_refresh(nla_mlp *M, hipStream_t s)
{
    k_mlp_refresh<<<grid_for(H * H + 32 * H, 256), 256, 0, s>>>(M->w, M->w2, M->w2t, M->w3p, M->w3e);
    NLA_HIP(hipGetLastError());
    return NLA_OK;
}

static int mlp_scratch(nla_mlp *M, int64_t Bp, int64_t nloss)
{
    if (M->scratch && M->T.Bp >= Bp && M->loss_cap >= nloss) return NLA_OK;
    delete M->scratch;
    M->scratch = new (std::nothrow) DeviceArena();
    if (!M->scratch) { nla_set_error("host allocation failed"); return NLA_E_NOMEM; }
    DeviceArena &A = *M->scratch;
    TrainBuf &T = M->T;
    T.Bp = Bp;
    NLA_TRY(A.get(&T.fpos, 6 * Bp));
    NLA_TRY(A.get(&T.gd1, H * Bp));
    NLA_TRY(A.get(&T.h1t, H * Bp));
    NLA_TRY(A.get(&T.gd2, H * Bp));
    NLA_TRY(A.get(&T.h2, H * Bp));
    NLA_TRY(A.get(&T.dy, 3 * Bp));
    NLA_TRY(A.get(&T.sq, Bp));
    NLA_TRY(A.get(&T.dz1, H * Bp));
    NLA_TRY(A.get(&T.dz2f, H * Bp));
    NLA_TRY(A.get(&T.dz2t, H * Bp));
    NLA_TRY(A.get(&T.part, (Bp / RCH) * NRED));
    M->loss_cap = nloss > 1 ? nloss : 1;
    NLA_TRY(A.get(&M->lossb, M->loss_cap));
    return NLA_OK;
}

// Blocks for a forward pass over `tiles` 32-item tiles (four waves a block).
// Three blocks fit a CU (LDS); a grid of many rounds of resident blocks runs
// faster than a single round because block starts (the weight loads) stagger
// against other blocks' arithmetic: 4096 blocks (about 5 rounds on 256 CUs).
static int fwd_grid(int64_t tiles, int64_t cap = 2048)
{
    int64_t b = (tiles + 3) / 4;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

// one gradient evaluation on Bp (multiple of 64) batch positions
static int mlp_grad(nla_mlp *M, int mode, int64_t nB, const float *feat, const float *label, const float *dout,
                    float gcoef, int64_t pa, int64_t pb, int64_t base, int64_t n_total, float *loss_slot, hipStream_t s)
{
    const MlpW W = mlp_view(M);
    const int64_t tiles = M->T.Bp / 32;
    const float inv = M->scale > 0.f ? 1.f / M->scale : 1.f;
    if (mode == 1)
        k_mlp_fwd<1><<<fwd_grid(tiles), 256, 0, s>>>(nB, feat, label, dout, W, inv, gcoef, pa, pb, base, n_total, nullptr, M->T);
    else
        k_mlp_fwd<2><<<fwd_grid(tiles), 256, 0, s>>>(nB, feat, label, dout, W, inv, gcoef, pa, pb, base, n_total, nullptr, M->T);
    k_mlp_bwd<<<fwd_grid(tiles), 256, 0, s>>>(W, M->T);
    k_mlp_dw2<<<16, 256, 0, s>>>(M->T, M->g);
    const int nchunk = (int)(M->T.Bp / RCH);
    k_mlp_reduce_part<<<dim3(nchunk, (NRED + 255) / 256), 256, 0, s>>>(M->T, M->T.part);
    k_mlp_reduce_final<<<grid_for(NRED, 256), 256, 0, s>>>(nchunk, M->T.part, M->g, loss_slot);
    NLA_HIP(hipGetLastError());
    return NLA_OK;
}

int nla_mlp_infer_launch(const nla_mlp *M, const float *feat, int64_t n, float *out, hipStream_t s)
{
    if (n <= 0) return NLA_OK;
    TrainBuf none{};
    k_mlp_fwd<0><<<fwd_grid((n + 31) / 32, 4096), 256, 0, s>>>(n, feat, nullptr, nullptr, mlp_view(M), 1.f, 0.f, 1, 0,
                                                              0, n, out, none);
    NLA_HIP(hipGetLastError());
    return NLA_OK;
}

float nla_mlp_scale(const nla_mlp *M) { return M->scale; }
MlpDomain nla_mlp_domain_of(const nla_mlp *M) { return M->dom; }

extern "C" int nla_mlp_set_domain(nla_mlp *M, const double *dom)
{
    if (!M) { nla_set_error("null network"); return NLA_E_INVALID; }
    if (!dom) {
        M->dom = unbounded_domain();
        return NLA_OK;
    }
    if (!valid_domain(dom)) { nla_set_error("domain limits must satisfy lo <= hi and not be NaN"); return NLA_E_INVALID; }
    M->dom = domain_from(dom);
    return NLA_OK;
}

extern "C" int nla_mlp_get_domain(const nla_mlp *M, double *dom)
{
    if (!M || !dom) { nla_set_error("null argument"); return NLA_E_INVALID; }
    domain_to(M->dom, dom);
    return NLA_OK;
}

extern "C" int nla_mlp_create(uint64_t seed, nla_mlp **out)
{
    if (!out) { nla_set_error("out is null"); return NLA_E_INVALID; }
    *out = nullptr;
    nla_mlp *M = new (std::nothrow) nla_mlp();
    if (!M) { nla_set_error("host allocation failed"); return NLA_E_NOMEM; }
    int st = NLA_OK;
    do {
        if ((st = (hipGetDevice(&M->device) == hipSuccess ? NLA_OK : NLA_E_DEVICE)) != NLA_OK) break;
        if ((st = M->arena.get(&M->w, NW)) != NLA_OK) break;
        if ((st = M->arena.get(&M->g, NW)) != NLA_OK) break;
        if ((st = M->arena.get(&M->am, NW)) != NLA_OK) break;
        if ((st = M->arena.get(&M->av, NW)) != NLA_OK) break;
        if ((st = M->arena.get(&M->w3e, 3 * H)) != NLA_OK) break;
        if ((st = M->arena.get(&M->w2, H * H)) != NLA_OK) break;
        if ((st = M->arena.get(&M->w2t, H * H)) != NLA_OK) break;
        if ((st = M->arena.get(&M->w3p, 32 * H)) != NLA_OK) break;
        if ((st = M->arena.get(&M->rms, 1)) != NLA_OK) break;
        // uniform initial weights, bound sqrt(6/fan_in) (W3: sqrt(1/fan_in)), zero biases
        std::vector<float> w(NW, 0.f);
        auto fill = [&](int off, int rows, int fan_in, double gain) {
            const double bound = std::sqrt(gain / fan_in);
            for (int i = 0; i < rows * fan_in; i++) {
                const double u = (double)(splitmix_host(seed, (uint64_t)(off + i)) >> 11) * (1.0 / 9007199254740992.0);
                w[off + i] = (float)((2.0 * u - 1.0) * bound);
            }
        };
        fill(OW1, H, 6, 6.0);
        fill(OW2, H, H, 6.0);
        fill(OW3, 3, H, 1.0);
        if (hipMemcpy(M->w, w.data(), sizeof(float) * NW, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(M->am, 0, sizeof(float) * NW) != hipSuccess || hipMemset(M->av, 0, sizeof(float) * NW) != hipSuccess) {
            nla_set_error("device copy failed");
            st = NLA_E_DEVICE;
            break;
        }
        if ((st = mlp_refresh(M, nullptr)) != NLA_OK) break;
        if (hipDeviceSynchronize() != hipSuccess) { nla_set_error("device error"); st = NLA_E_DEVICE; }
    } while (0);
    if (st != NLA_OK) {
        delete M;
        return st;
    }
    *out = M;
    return NLA_OK;
}

extern "C" int nla_mlp_set_weights(nla_mlp *M, const float *w, float scale)
{
    if (!M || !w) { nla_set_error("null argument"); return NLA_E_INVALID; }
    if (!(scale > 0.f) || !std::isfinite(scale)) { nla_set_error("scale must be > 0"); return NLA_E_INVALID; }
    for (int i = 0; i < NW; i++)
        if (!std::isfinite(w[i])) { nla_set_error("weight %d is not finite", i); return NLA_E_INVALID; }
    NLA_HIP(hipMemcpy(M->w, w, sizeof(float) * NW, hipMemcpyHostToDevice));
    NLA_HIP(hipMemset(M->am, 0, sizeof(float) * NW));
    NLA_HIP(hipMemset(M->av, 0, sizeof(float) * NW));
    M->scale = scale;
    M->step = 0;
    M->adam_t = 0;
    M->dom = unbounded_domain();
    NLA_TRY(mlp_refresh(M, nullptr));
    NLA_HIP(hipDeviceSynchronize());
    return NLA_OK;
}

extern "C" int nla_mlp_get_weights(const nla_mlp *M, float *w, float *scale)
{
    if (!M || !w || !scale) { nla_set_error("null argument"); return NLA_E_INVALID; }
    NLA_HIP(hipDeviceSynchronize());
    NLA_HIP(hipMemcpy(w, M->w, sizeof(float) * NW, hipMemcpyDeviceToHost));
    *scale = M->scale;
    return NLA_OK;
}

extern "C" int nla_mlp_samples(int64_t n_cand, uint64_t seed, int64_t first, double L, double jitter, double band,
                               int32_t cap_edges, float *feat, float *label, int64_t *n_valid, void *stream)
{
    if (n_cand < 0 || !feat || !label || !n_valid) { nla_set_error("invalid sample arguments"); return NLA_E_INVALID; }
    if (!(L > 0.0 && L <= 0.5) || !(jitter >= 0.0 && jitter < 0.5) || !(band >= 0.0) || cap_edges < 2 ||
        cap_edges > NLA_MAX_CAP) {
        nla_set_error("need 0 < L <= 1/2, 0 <= jitter < 1/2, band >= 0, 2 <= cap_edges <= %d", NLA_MAX_CAP);
        return NLA_E_INVALID;
    }
    *n_valid = 0;
    if (n_cand == 0) return NLA_OK;
    hipStream_t s = (hipStream_t)stream;
    DeviceArena tmp;
    float *ft, *lt;
    uint8_t *fl;
    int64_t *cnt;
    NLA_TRY(tmp.get(&ft, 6 * n_cand));
    NLA_TRY(tmp.get(&lt, 3 * n_cand));
    NLA_TRY(tmp.get(&fl, n_cand));
    NLA_TRY(tmp.get(&cnt, 2));
    const bool pow2 = (cap_edges & (cap_edges - 1)) == 0;
    if (pow2)
        k_cap_samples<true><<<grid_for(n_cand, 128), 128, 0, s>>>(n_cand, seed, first, L, jitter, band, cap_edges, ft, lt, fl);
    else
        k_cap_samples<false><<<grid_for(n_cand, 128), 128, 0, s>>>(n_cand, seed, first, L, jitter, band, cap_edges, ft, lt, fl);
    NLA_HIP(hipGetLastError());
    size_t b6 = 0, b3 = 0;
    const F6 *i6 = (const F6 *)ft;
    const F3 *i3 = (const F3 *)lt;
    NLA_HIP(rocprim::select(nullptr, b6, i6, fl, (F6 *)feat, cnt, (size_t)n_cand, s));
    NLA_HIP(rocprim::select(nullptr, b3, i3, fl, (F3 *)label, cnt + 1, (size_t)n_cand, s));
    void *t;
    NLA_TRY(tmp.alloc(&t, b6 > b3 ? b6 : b3));
    NLA_HIP(rocprim::select(t, b6, i6, fl, (F6 *)feat, cnt, (size_t)n_cand, s));
    NLA_HIP(rocprim::select(t, b3, i3, fl, (F3 *)label, cnt + 1, (size_t)n_cand, s));
    int64_t c[2];
    NLA_HIP(hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    *n_valid = c[0];
    return NLA_OK;
}

extern "C" int nla_mlp_forward(const nla_mlp *M, const float *feat, int64_t n, float *out, void *stream)
{
    if (!M || n < 0 || (n > 0 && (!feat || !out))) { nla_set_error("invalid forward arguments"); return NLA_E_INVALID; }
    return nla_mlp_infer_launch(M, feat, n, out, (hipStream_t)stream);
}

extern "C" int nla_mlp_backward(nla_mlp *M, const float *feat, const float *dout, int64_t n, float *dw, void *stream)
{
    if (!M || n < 1 || !feat || !dout || !dw) { nla_set_error("invalid backward arguments"); return NLA_E_INVALID; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t Bp = (n + 63) / 64 * 64;
    NLA_TRY(mlp_scratch(M, Bp, 1));
    M->T.Bp = Bp;
    NLA_TRY(mlp_grad(M, 2, n, feat, nullptr, dout, 0.f, 1, 0, 0, n, nullptr, s));
    NLA_HIP(hipMemcpyAsync(dw, M->g, sizeof(float) * NW, hipMemcpyDeviceToDevice, s));
    return NLA_OK;
}

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

extern "C" int nla_mlp_train(nla_mlp *M, const float *feat, const float *label, int64_t n, int32_t epochs,
                             int32_t batch, float lr, uint64_t seed, float *loss_log, void *stream)
{
    if (!M || !feat || !label || epochs < 1 || batch < 64 || batch % 64 || n < batch || !(lr > 0.f) ||
        n >= ((int64_t)1 << 31)) {
        nla_set_error("need n >= batch, batch a multiple of 64, epochs >= 1, lr > 0, n < 2^31");
        return NLA_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t spe = n / batch, total = spe * (int64_t)epochs;
    NLA_TRY(mlp_scratch(M, batch, spe));
    M->T.Bp = batch;
    if (!(M->scale > 0.f)) {
        k_label_rms<<<1, 1024, 0, s>>>(3 * n, label, M->rms);
        double r = 0.0;
        NLA_HIP(hipMemcpyAsync(&r, M->rms, sizeof(double), hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        if (!(r > 0.0)) { nla_set_error("labels are all zero"); return NLA_E_INVALID; }
        M->scale = (float)r;
    }
    {
        // the training domain: the range of these samples (joined with the
        // earlier training calls' ranges)
        const int nb = (int)std::min<int64_t>(256, (n + 255) / 256);
        DeviceArena tmp;
        double *part;
        NLA_TRY(tmp.get(&part, 2 * (size_t)NDOM * nb));
        k_feat_domain<<<nb, 256, 0, s>>>(n, feat, part);
        NLA_HIP(hipGetLastError());
        std::vector<double> h(2 * (size_t)NDOM * nb);
        NLA_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        MlpDomain D = M->step > 0 ? M->dom : MlpDomain{HUGE_VAL, -HUGE_VAL, HUGE_VAL, -HUGE_VAL};
        for (int b = 0; b < nb; b++) {
            D.rlo = std::min(D.rlo, h[2 * NDOM * b + 0]);
            D.rhi = std::max(D.rhi, h[2 * NDOM * b + NDOM + 0]);
            D.elo = std::min(D.elo, h[2 * NDOM * b + 1]);
            D.ehi = std::max(D.ehi, h[2 * NDOM * b + NDOM + 1]);
        }
        M->dom = D;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gcoef = 2.f / (3.f * (float)batch);
    std::vector<float> lh((size_t)spe);
    int64_t t = 0;
    for (int e = 0; e < epochs; e++) {
        // epoch order: the affine permutation p -> (pa p + pb) mod n, gcd(pa, n) = 1
        int64_t pa = (int64_t)(splitmix_host(seed, 2 * (uint64_t)(M->step + e)) % (uint64_t)n) | 1;
        while (gcd64(pa, n) != 1) pa += 2;
        pa %= n;
        if (pa == 0) pa = 1;
        const int64_t pb = (int64_t)(splitmix_host(seed, 2 * (uint64_t)(M->step + e) + 1) % (uint64_t)n);
        for (int64_t st = 0; st < spe; st++, t++) {
            NLA_TRY(mlp_grad(M, 1, batch, feat, label, nullptr, gcoef, pa, pb, st * batch, n, M->lossb + st, s));
            const double sched = 0.5 * (1.0 + std::cos(3.14159265358979323846 * (double)t / (double)total));
            const int64_t k = ++M->adam_t;
            const double lr_t = lr * sched * std::sqrt(1.0 - std::pow((double)b2, (double)k)) /
                                (1.0 - std::pow((double)b1, (double)k));
            k_adam<<<grid_for(NW, 256), 256, 0, s>>>(M->w, M->g, M->am, M->av, (float)lr_t, b1, b2, eps);
            NLA_TRY(mlp_refresh(M, s));
        }
        NLA_HIP(hipMemcpyAsync(lh.data(), M->lossb, sizeof(float) * spe, hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        if (loss_log) {
            double a = 0.0;
            for (int64_t i = 0; i < spe; i++) a += lh[(size_t)i];
            loss_log[e] = (float)(a / (3.0 * (double)batch * (double)spe));
        }
    }
    M->step += epochs;
    return NLA_OK;
}

// checkpoint: magic, weights, scale, Adam moments and step, training domain
// (4 doubles; a version-1 file has none and loads with an unbounded domain)
extern "C" int nla_mlp_save(const nla_mlp *M, const char *path)
{
    if (!M || !path) { nla_set_error("null argument"); return NLA_E_INVALID; }
    std::vector<float> buf(3 * (size_t)NW);
    NLA_HIP(hipDeviceSynchronize());
    NLA_HIP(hipMemcpy(buf.data(), M->w, sizeof(float) * NW, hipMemcpyDeviceToHost));
    NLA_HIP(hipMemcpy(buf.data() + NW, M->am, sizeof(float) * NW, hipMemcpyDeviceToHost));
    NLA_HIP(hipMemcpy(buf.data() + 2 * NW, M->av, sizeof(float) * NW, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) { nla_set_error("cannot open %s", path); return NLA_E_INVALID; }
    const char magic[8] = {'N', 'L', 'A', 'M', 'L', 'P', '2', 0};
    const int32_t nw = NW;
    double dom[4];
    domain_to(M->dom, dom);
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&nw, 4, 1, f) == 1 && std::fwrite(&M->scale, 4, 1, f) == 1 &&
              std::fwrite(&M->step, 8, 1, f) == 1 && std::fwrite(&M->adam_t, 8, 1, f) == 1 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size() && std::fwrite(dom, 8, 4, f) == 4;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) { nla_set_error("write failed: %s", path); return NLA_E_INVALID; }
    return NLA_OK;
}

extern "C" int nla_mlp_load(const char *path, nla_mlp **out)
{
    if (!path || !out) { nla_set_error("null argument"); return NLA_E_INVALID; }
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) { nla_set_error("cannot open %s", path); return NLA_E_INVALID; }
    char magic[8];
    int32_t nw = 0;
    float scale = 0.f;
    int64_t step = 0, adam_t = 0;
    std::vector<float> buf(3 * (size_t)NW);
    double dom[4];
    bool ok = std::fread(magic, 1, 8, f) == 8 &&
              (std::memcmp(magic, "NLAMLP1", 8) == 0 || std::memcmp(magic, "NLAMLP2", 8) == 0) &&
              std::fread(&nw, 4, 1, f) == 1 && nw == NW && std::fread(&scale, 4, 1, f) == 1 &&
              std::fread(&step, 8, 1, f) == 1 && std::fread(&adam_t, 8, 1, f) == 1 &&
              std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    const bool v2 = ok && magic[6] == '2';
    if (v2) ok = std::fread(dom, 8, 4, f) == 4 && valid_domain(dom);
    std::fclose(f);
    if (!ok) { nla_set_error("%s is not a network checkpoint of this layout", path); return NLA_E_INVALID; }
    nla_mlp *M = nullptr;
    NLA_TRY(nla_mlp_create(0, &M));
    int st = nla_mlp_set_weights(M, buf.data(), scale > 0.f ? scale : 1.f);
    if (st == NLA_OK) {
        M->scale = scale;
        M->step = step;
        M->adam_t = adam_t;
        M->dom = v2 ? domain_from(dom) : unbounded_domain();
        if (hipMemcpy(M->am, buf.data() + NW, sizeof(float) * NW, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(M->av, buf.data() + 2 * NW, sizeof(float) * NW, hipMemcpyHostToDevice) != hipSuccess) {
            nla_set_error("device copy failed");
            st = NLA_E_DEVICE;
        }
    }
    if (st != NLA_OK) {
        delete M;
        return st;
    }
    *out = M;
    return NLA_OK;
}

extern "C" void nla_mlp_destroy(nla_mlp *M) { delete M; }
