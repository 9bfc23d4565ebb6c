// mgseg_net.hip -- learned warm start: a small convolutional encoder-decoder
// that maps (image, marker distance map, marker mask) to an initial level set
// phi0 = M tanh(o); the FAS V-cycle then finishes every solve.
//
// Architecture (depth D, base width C0, C_l = C0 2^l; every block is two
// 3x3 convolutions with ReLU, cb(x) = relu(conv_b(relu(conv_a(x))))):
//   encoder  e_l = cb(p_{l-1}), p_l = avgpool2(e_l)     (e_0 = cb(input))
//   decoder  d_l = cb([up2(d_{l+1}) | e_l])              (d_{D-1} = e_{D-1})
//   head     o = w . d_0 + b (1x1),  phi0 = M tanh(o)
//
// Storage: activations and their gradients in bf16, channels last (NHWC:
// pixel-major, the channels of a pixel contiguous; a batch is one run of
// pixels, image by image); convolution weights packed in bf16 as
// [OC][tap][IC] (and, for the data gradient, the tap-reversed transpose
// [IC][tap][OC]); FP32 master weights with Adam.  Every channel count is a
// multiple of 16 (the input's 3 channels are padded with zeros to 16).
//
// Convolutions are implicit GEMMs on the matrix cores (FP32 accumulation;
// k_conv on mfma_f32_16x16x32_bf16, a 16-channel remainder and k_wgrad on
// mfma_f32_16x16x16bf16_1k):
//   forward / data gradient (k_conv): M = output channels, N = pixels,
//     K = 9 taps x input channels.  A block computes 32 channels x an 8 x 32
//     pixel tile; per 32-channel chunk the tile's input halo (10 x 34
//     pixels) is staged in LDS and each wave keeps the weights of all 9
//     taps in registers.
//   weight gradient (k_wgrad): M = output channels, N = 9 taps x input
//     channels, K = pixels.  A block owns 32 x (9 x 16) weights and walks a
//     strided share of the pixel tiles, staging the output gradient and the
//     input halo transposed (pixels contiguous) in LDS; one partial sum per
//     block, added in a fixed order (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mgseg.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int CIN0 = 16;                       // input channels after padding
constexpr int TY = 8, TX = 32;                 // pixel tile of a block
constexpr int HY = TY + 2, HX = TX + 2;        // its halo
constexpr int HP = 40;                         // LDS elements per halo pixel in k_conv (32 used; 80 B keeps lanes apart)
constexpr int OCB = 32;                        // output channels per block
constexpr int GTS = TY * TX + 8;               // k_wgrad: LDS row of the transposed output gradient
constexpr int XRS = 36;                        // k_wgrad: LDS halo row (34 used)
constexpr int XTS = HY * XRS + 4;              // k_wgrad: LDS plane of one input channel

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float x)
{
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// --------------------------------------------------------------------------
// 3x3 convolution, zero padding, stride 1:
//   out[px, oc] = act( sum_{r, ic} W[oc, r, ic] in[px + off(r), ic] + bias[oc] ),  off(r) = (r/3 - 1, r%3 - 1)
// with act = ReLU (relu), then zeroed where mask[px, oc] <= 0 (mask set).
// Views: element (px, c) of a view is at ptr[px * ps + off + c].
struct ConvArgs {
    const uint16_t *in; int ips, ioff;
    const uint16_t *Wk;                  // packed [OC][9][IC]
    const float *bias;                   // [OC] or null
    uint16_t *out; int ops, ooff;
    float *out32;                        // optional dense FP32 copy [px][OC]
    const uint16_t *mask; int mps, moff; // optional
    int IC, OC, H, W, relu;
};

// One chunk of KC input channels (32: mfma_f32_16x16x32_bf16, 8 channels per
// lane and operand; 16: mfma_f32_16x16x16bf16_1k, 4 per lane).  Lane group
// g = lane / 16 brings the same channels c0 + V g .. c0 + V g + V - 1 to the
// weight operand (row l16 = output channel) and to the pixel operand (column
// l16 = pixel), so each product pairs one channel of both whatever order the
// instruction sums its K terms in.
template <int KC>
__device__ __forceinline__ void conv_chunk(const ConvArgs &A, uint16_t *halo, int c0, const uint16_t *w0,
                                           const uint16_t *w1, bool two, int ty0, int tx0, long long img, int wave,
                                           int l16, int g, f32x4 (&acc)[2][4])
{
    constexpr int V = KC / 4;
    typedef short vec __attribute__((ext_vector_type(V)));
    vec wa[2][9];
#pragma unroll
    for (int r = 0; r < 9; r++) {
        wa[0][r] = *(const vec *)(w0 + r * A.IC + c0 + V * g);
        wa[1][r] = two ? *(const vec *)(w1 + r * A.IC + c0 + V * g) : vec{};
    }
    __syncthreads();                                // the previous chunk's halo is no longer read
    constexpr int Q = KC / 8;                       // 16-byte pieces per halo pixel
    for (int u = threadIdx.x; u < HY * HX * Q; u += 256) {
        const int hp = u / Q, part = u - hp * Q;
        const int hy = hp / HX, hx = hp - hy * HX;
        const int y = ty0 + hy - 1, x = tx0 + hx - 1;
        uint4 v = {0u, 0u, 0u, 0u};
        if (y >= 0 && y < A.H && x >= 0 && x < A.W)
            v = *(const uint4 *)(A.in + (img + (long long)y * A.W + x) * A.ips + A.ioff + c0 + 8 * part);
        *(uint4 *)(halo + hp * HP + 8 * part) = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 9; r++) {
        const int dy = r / 3, dx = r % 3;
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const int yr = 2 * wave + (p >> 1), xo = 16 * (p & 1);
            const vec bv = *(const vec *)(halo + ((yr + dy) * HX + xo + l16 + dx) * HP + V * g);
            if constexpr (KC == 32) {
                typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
                const bf8 b = __builtin_bit_cast(bf8, bv);
                acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, wa[0][r]), b, acc[0][p], 0,
                                                                   0, 0);
                if (two)
                    acc[1][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, wa[1][r]), b,
                                                                       acc[1][p], 0, 0, 0);
            } else {
                acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[0][r], bv, acc[0][p], 0, 0, 0);
                if (two) acc[1][p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[1][r], bv, acc[1][p], 0, 0, 0);
            }
        }
    }
}

// At most 168 registers per lane (three waves per SIMD): the 9 taps' weights
// of two 16-channel tiles take 72 of them.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_conv(ConvArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t halo[HY * HX * HP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, g = lane >> 4, g4 = 4 * g;
    const int tilesx = (A.W + TX - 1) / TX;
    const int ty0 = (int)(blockIdx.x / tilesx) * TY, tx0 = (int)(blockIdx.x % tilesx) * TX;
    const int oc0 = blockIdx.y * OCB;
    const long long img = (long long)blockIdx.z * A.H * A.W;
    const bool two = oc0 + 16 < A.OC;               // second 16-channel tile present (uniform)
    f32x4 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int p = 0; p < 4; p++) acc[t][p] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const uint16_t *w0 = A.Wk + (long long)(oc0 + l16) * 9 * A.IC;
    const uint16_t *w1 = A.Wk + (long long)(oc0 + 16 + (two ? l16 : 0)) * 9 * A.IC;
    int c0 = 0;
    for (; c0 + 32 <= A.IC; c0 += 32) conv_chunk<32>(A, halo, c0, w0, w1, two, ty0, tx0, img, wave, l16, g, acc);
    if (c0 < A.IC) conv_chunk<16>(A, halo, c0, w0, w1, two, ty0, tx0, img, wave, l16, g, acc);
    // D[row = 4 (lane / 16) + i][col = lane % 16]: 4 consecutive channels of one pixel
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int y = ty0 + 2 * wave + (p >> 1), x = tx0 + 16 * (p & 1) + l16;
        if (y >= A.H || x >= A.W) continue;
        const long long px = img + (long long)y * A.W + x;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            if (t == 1 && !two) continue;
            const int oc = oc0 + 16 * t + g4;
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                v[i] = acc[t][p][i] + (A.bias ? A.bias[oc + i] : 0.0f);
                if (A.relu) v[i] = fmaxf(v[i], 0.0f);
            }
            if (A.mask) {
                const uint16_t *mk = A.mask + px * A.mps + A.moff + oc;
#pragma unroll
                for (int i = 0; i < 4; i++)
                    if (!(bf2f(mk[i]) > 0.0f)) v[i] = 0.0f;
            }
            bf16x4 o;
#pragma unroll
            for (int i = 0; i < 4; i++) o[i] = (short)f2bf(v[i]);
            *(bf16x4 *)(A.out + px * A.ops + A.ooff + oc) = o;
            if (A.out32) *(f32x4 *)(A.out32 + px * A.OC + oc) = f32x4{v[0], v[1], v[2], v[3]};
        }
    }
}

// --------------------------------------------------------------------------
// weight gradient: dW[oc, r, ic] = sum_px g[px, oc] x[px + off(r), ic],  db[oc] = sum_px g[px, oc].
// Block (p, oc block of 32, ic chunk of 16) adds up the pixel tiles p, p + P, ...
// and writes part[p][oc][r][ic] (IC = padded count) and, for ic chunk 0, partb[p][oc].
struct WgradArgs {
    const uint16_t *g; int gps, goff;    // output gradient (already ReLU-masked)
    const uint16_t *x; int xps, xoff;    // convolution input
    float *part, *partb;
    int IC, OC, H, W, B, P;
};

__device__ __forceinline__ uint32_t pack2(uint16_t a, uint16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs A)
{
    // gT [oc][tile pixel] and xT [ic][halo row][halo col]; at the end the same memory adds up the waves
    __shared__ __attribute__((aligned(16))) uint16_t lds[OCB * GTS + 16 * XTS];
    static_assert(3 * 9 * 256 * 2 <= OCB * GTS + 16 * XTS, "wave reduction does not fit");
    uint16_t *const gT = lds, *const xT = lds + OCB * GTS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, g4 = (lane >> 4) * 4;
    const int oc0 = blockIdx.y * OCB, c0 = blockIdx.z * 16;
    const bool two = oc0 + 16 < A.OC;
    const bool dobias = blockIdx.z == 0;
    const int tilesx = (A.W + TX - 1) / TX, tiles = tilesx * ((A.H + TY - 1) / TY);
    const int T = tiles * A.B;
    f32x4 acc[2][9];
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int r = 0; r < 9; r++) acc[t][r] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int tile = blockIdx.x; tile < T; tile += A.P) {
        const int b = tile / tiles, tt = tile % tiles;
        const int ty0 = (tt / tilesx) * TY, tx0 = (tt % tilesx) * TX;
        const long long img = (long long)b * A.H * A.W;
        __syncthreads();
        // g: pixel pairs x 8-channel groups, written transposed as (pixel, pixel + 1) pairs
        for (int u = threadIdx.x; u < (TY * TX / 2) * (OCB / 8); u += 256) {
            const int pp = u % (TY * TX / 2), cg = u / (TY * TX / 2);
            const int q = 2 * pp, yr = q / TX, xr = q % TX;
            const int y = ty0 + yr, x = tx0 + xr;
            uint4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
            const int oc = oc0 + 8 * cg;
            if (y < A.H && oc < A.OC) {
                const uint16_t *s = A.g + (img + (long long)y * A.W + x) * A.gps + A.goff + oc;
                if (x < A.W) v0 = *(const uint4 *)s;
                if (x + 1 < A.W) v1 = *(const uint4 *)(s + A.gps);
            }
            const uint16_t *a0 = (const uint16_t *)&v0, *a1 = (const uint16_t *)&v1;
#pragma unroll
            for (int j = 0; j < 8; j++) *(uint32_t *)(gT + (8 * cg + j) * GTS + q) = pack2(a0[j], a1[j]);
        }
        // x halo: column pairs x 8-channel halves
        for (int u = threadIdx.x; u < HY * (HX / 2) * 2; u += 256) {
            const int pp = u % (HY * (HX / 2)), half = u / (HY * (HX / 2));
            const int hy = pp / (HX / 2), hx = 2 * (pp % (HX / 2));
            const int y = ty0 + hy - 1, x = tx0 + hx - 1;
            uint4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
            if (y >= 0 && y < A.H) {
                const long long row = img + (long long)y * A.W;
                if (x >= 0 && x < A.W) v0 = *(const uint4 *)(A.x + (row + x) * A.xps + A.xoff + c0 + 8 * half);
                if (x + 1 < A.W) v1 = *(const uint4 *)(A.x + (row + x + 1) * A.xps + A.xoff + c0 + 8 * half);
            }
            const uint16_t *a0 = (const uint16_t *)&v0, *a1 = (const uint16_t *)&v1;
#pragma unroll
            for (int j = 0; j < 8; j++) *(uint32_t *)(xT + (8 * half + j) * XTS + hy * XRS + hx) = pack2(a0[j], a1[j]);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int yr = 2 * wave + (s >> 1), xo = 16 * (s & 1);
            const bf16x4 a0 = *(const bf16x4 *)(gT + l16 * GTS + yr * TX + xo + g4);
            const bf16x4 a1 = two ? *(const bf16x4 *)(gT + (16 + l16) * GTS + yr * TX + xo + g4) : bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int dy = 0; dy < 3; dy++) {
                const uint16_t *row = xT + l16 * XTS + (yr + dy) * XRS + xo + g4;
                const bf16x4 e0 = *(const bf16x4 *)row, e1 = *(const bf16x4 *)(row + 4);
                const bf16x4 b1 = bf16x4{e0[1], e0[2], e0[3], e1[0]};
                const bf16x4 b2 = bf16x4{e0[2], e0[3], e1[0], e1[1]};
                acc[0][3 * dy + 0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, e0, acc[0][3 * dy + 0], 0, 0, 0);
                acc[0][3 * dy + 1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc[0][3 * dy + 1], 0, 0, 0);
                acc[0][3 * dy + 2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b2, acc[0][3 * dy + 2], 0, 0, 0);
                if (two) {
                    acc[1][3 * dy + 0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, e0, acc[1][3 * dy + 0], 0, 0, 0);
                    acc[1][3 * dy + 1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc[1][3 * dy + 1], 0, 0, 0);
                    acc[1][3 * dy + 2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b2, acc[1][3 * dy + 2], 0, 0, 0);
                }
            }
        }
        if (dobias) {
            // thread (oc = tid / 8, part = tid % 8) adds 32 pixels of the tile
            const int oc = threadIdx.x >> 3, part = threadIdx.x & 7;
            float s = 0.0f;
            for (int q = 0; q < TY * TX / 8; q++) s += bf2f(gT[oc * GTS + part * (TY * TX / 8) + q]);
            bsum += s;
        }
    }
    // every wave holds the sums over its own rows of each tile: wave 0 adds waves 1, 2, 3 (in that order)
    // and writes the block's partial, D[row = oc][col = ic]
    float *red = (float *)lds;
    const long long K9 = 9LL * A.IC;
    float *pb = A.part + (long long)blockIdx.x * A.OC * K9;
#pragma unroll
    for (int t = 0; t < 2; t++) {
        if (t == 1 && !two) break;
        __syncthreads();
        if (wave > 0) {
#pragma unroll
            for (int r = 0; r < 9; r++)
#pragma unroll
                for (int i = 0; i < 4; i++) red[((wave - 1) * 9 + r) * 256 + i * 64 + lane] = acc[t][r][i];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int r = 0; r < 9; r++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    float v = acc[t][r][i];
                    for (int w = 0; w < 3; w++) v += red[(w * 9 + r) * 256 + i * 64 + lane];
                    pb[(long long)(oc0 + 16 * t + g4 + i) * K9 + r * A.IC + c0 + l16] = v;
                }
        }
    }
    if (dobias) {
        // the 8 threads of one channel are consecutive lanes
        bsum += __shfl_xor(bsum, 1);
        bsum += __shfl_xor(bsum, 2);
        bsum += __shfl_xor(bsum, 4);
        const int oc = oc0 + (threadIdx.x >> 3);
        if ((threadIdx.x & 7) == 0 && oc < A.OC) A.partb[(long long)blockIdx.x * A.OC + oc] = bsum;
    }
}

// dW (master layout [OC][ICr][3][3]) = sum over the P partials [OC][9][IC] of the real channels ic < ICr
__global__ void k_wgrad_reduce(const float *part, const float *partb, int P, int OC, int IC, int ICr, float *dW,
                               float *db)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long NW = (long long)OC * ICr * 9;
    const long long stride = (long long)OC * 9 * IC;
    if (t < NW) {
        const int oc = (int)(t / (ICr * 9)), rem = (int)(t % (ICr * 9)), ic = rem / 9, r = rem % 9;
        const float *s = part + ((long long)oc * 9 + r) * IC + ic;
        float acc = 0.0f;
        for (int p = 0; p < P; p++) acc += s[(long long)p * stride];
        dW[t] = acc;
    } else if (t < NW + OC) {
        const int oc = (int)(t - NW);
        float acc = 0.0f;
        for (int p = 0; p < P; p++) acc += partb[(long long)p * OC + oc];
        db[oc] = acc;
    }
}

// master [OC][ICr][3][3] -> packed [OC][9][IC] (zero for ic >= ICr) and, if Wt, the data-gradient
// weights [ICr][9][OC] with the taps reversed (Wt[ic, r, oc] = W[oc, ic, 8 - r])
__global__ void k_pack_weights(const float *w, int OC, int ICr, int IC, uint16_t *Wp, uint16_t *Wt)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (long long)OC * 9 * IC) {
        const int oc = (int)(t / (9 * IC)), rem = (int)(t % (9 * IC)), r = rem / IC, ic = rem % IC;
        Wp[t] = ic < ICr ? f2bf(w[((long long)oc * ICr + ic) * 9 + r]) : (uint16_t)0;
    }
    if (Wt && t < (long long)ICr * 9 * OC) {
        const int ic = (int)(t / (9 * OC)), rem = (int)(t % (9 * OC)), r = rem / OC, oc = rem % OC;
        Wt[t] = f2bf(w[((long long)oc * ICr + ic) * 9 + (8 - r)]);
    }
}

// --------------------------------------------------------------------------
// input features FP32 [B][3][H][W] -> bf16 [B*H*W][16] (channels 3..15 zero)
__global__ void k_pack_input(const float *x, long long HW, int B, uint16_t *y)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * HW) return;
    const long long b = t / HW, p = t % HW;
    bf16x4 v0 = {0, 0, 0, 0}, z = {0, 0, 0, 0};
    for (int c = 0; c < 3; c++) v0[c] = (short)f2bf(x[(b * 3 + c) * HW + p]);
    bf16x4 *d = (bf16x4 *)(y + t * CIN0);
    d[0] = v0; d[1] = z; d[2] = z; d[3] = z;
}

// 8 bf16 values in 16 bytes
struct bf8 {
    uint4 v;
    __device__ __forceinline__ float get(int i) const
    {
        const uint32_t w = i < 2 ? v.x : (i < 4 ? v.y : (i < 6 ? v.z : v.w));
        return bf2f((uint16_t)((i & 1) ? (w >> 16) : (w & 0xffffu)));
    }
};
__device__ __forceinline__ uint4 pack8(const float (&f)[8])
{
    uint4 o;
    o.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
    o.y = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
    o.z = (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
    o.w = (uint32_t)f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
    return o;
}
__device__ __forceinline__ bf8 ld8(const uint16_t *p) { return bf8{*(const uint4 *)p}; }

// The elementwise kernels below take 8 consecutive channels (16 bytes) per
// thread: channel counts, view strides and offsets are multiples of 8.

// 2x2 average pooling: out[(b, y, x), c] (dense, C per pixel) from the view (ps, off) at twice the size
__global__ void k_avgpool(const uint16_t *in, int ps, int off, int C, int h, int w, int B, uint16_t *out)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (t >= (long long)B * h * w * C8) return;
    const long long q = t / C8;
    const int c = (int)(t % C8) * 8;
    const long long b = q / ((long long)h * w);
    const int yy = (int)((q / w) % h), xx = (int)(q % w);
    const int W = 2 * w;
    const long long f = b * 4LL * h * w + (long long)(2 * yy) * W + 2 * xx;
    const uint16_t *s = in + off + c;
    const bf8 a = ld8(s + f * ps), bq = ld8(s + (f + 1) * ps), cq = ld8(s + (f + W) * ps), d = ld8(s + (f + W + 1) * ps);
    float o[8];
#pragma unroll
    for (int i = 0; i < 8; i++) o[i] = 0.25f * (a.get(i) + bq.get(i) + cq.get(i) + d.get(i));
    *(uint4 *)(out + q * C + c) = pack8(o);
}

// gradient of e (view g: the skip part of the concatenation's gradient) += 0.25 gpool of its coarse
// pixel, rounded, then zeroed where e <= 0
__global__ void k_avgpool_bwd(const uint16_t *gp, int C, int h, int w, int B, uint16_t *g, int gps, int goff,
                              const uint16_t *e, int eps, int eoff)
{
    const int H = 2 * h, W = 2 * w, C8 = C / 8;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * H * W * C8) return;
    const long long px = t / C8;
    const int c = (int)(t % C8) * 8;
    const long long b = px / ((long long)H * W);
    const int y = (int)((px / W) % H), x = (int)(px % W);
    const bf8 gc = ld8(gp + ((b * h + y / 2) * w + x / 2) * C + c);
    uint16_t *d = g + px * gps + goff + c;
    const bf8 gv = ld8(d), ev = ld8(e + px * eps + eoff + c);
    float o[8];
#pragma unroll
    for (int i = 0; i < 8; i++) o[i] = ev.get(i) > 0.0f ? gv.get(i) + 0.25f * gc.get(i) : 0.0f;
    *(uint4 *)d = pack8(o);
}

// nearest 2x up-sampling of the dense coarse d [(b, y, x)][C] into channels [0, C) of the view (ps, 0)
__global__ void k_upsample(const uint16_t *d, int C, int h, int w, int B, uint16_t *out, int ps)
{
    const int H = 2 * h, W = 2 * w, C8 = C / 8;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * H * W * C8) return;
    const long long px = t / C8;
    const int c = (int)(t % C8) * 8;
    const long long b = px / ((long long)H * W);
    const int y = (int)((px / W) % H), x = (int)(px % W);
    *(uint4 *)(out + px * ps + c) = *(const uint4 *)(d + ((b * h + y / 2) * w + x / 2) * C + c);
}

// adjoint of k_upsample (2x2 sums of channels [0, C) of the view), rounded, zeroed where y <= 0;
// writes the dense coarse gradient [(b, y, x)][C]
__global__ void k_upsample_bwd(const uint16_t *g, int ps, int C, int h, int w, int B, const uint16_t *y,
                               uint16_t *gd)
{
    const int C8 = C / 8;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * h * w * C8) return;
    const long long q = t / C8;
    const int c = (int)(t % C8) * 8;
    const long long b = q / ((long long)h * w);
    const int yy = (int)((q / w) % h), xx = (int)(q % w);
    const int W = 2 * w;
    const long long f = b * 4LL * h * w + (long long)(2 * yy) * W + 2 * xx;
    const uint16_t *s = g + c;
    const bf8 a = ld8(s + f * ps), bq = ld8(s + (f + 1) * ps), cq = ld8(s + (f + W) * ps), d = ld8(s + (f + W + 1) * ps);
    const bf8 yv = ld8(y + q * C + c);
    float o[8];
#pragma unroll
    for (int i = 0; i < 8; i++) o[i] = yv.get(i) > 0.0f ? a.get(i) + bq.get(i) + cq.get(i) + d.get(i) : 0.0f;
    *(uint4 *)(gd + q * C + c) = pack8(o);
}

// head: o = w . d0 + b, phi0 = M tanh(o) (FP32 from the FP32 copy of d0, [px][C]); keeps o for the loss
__global__ void k_head(const float *d0, int C, long long NP, const float *w, const float *b, float M, float *ob,
                       float *phi)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NP) return;
    const float4 *x = (const float4 *)(d0 + t * C);
    float o = b[0];
    for (int c = 0; c < C / 4; c++) {
        const float4 v = x[c];
        o = fmaf(w[4 * c], v.x, o);
        o = fmaf(w[4 * c + 1], v.y, o);
        o = fmaf(w[4 * c + 2], v.z, o);
        o = fmaf(w[4 * c + 3], v.w, o);
    }
    ob[t] = o;
    phi[t] = M * tanhf(o);
}

// Loss: binary cross-entropy of p = sigmoid(2 o) = (1 + tanh o) / 2 against the
// soft target q = (1 + tg) / 2, tg = clip(target / M, -1, 1), weighted by
// w = pw on the object (tg > 0) and 1 elsewhere, averaged over the N pixels:
//   loss = mean w (softplus(2 o) - 2 o q),   dloss/do = w (tanh o - tg) / N,
// whose minimum is at tanh o = tg and whose gradient does not vanish where the
// output saturates on the wrong side.  Per pixel: the loss term and dO to
// lossb / dob, and gd0 = w_head dO, zeroed where the stored d0 <= 0 (bf16, [px][C]).
__global__ void k_head_bwd(const float *ob, const float *target, float M, float pw, const uint16_t *d0b, int C,
                           long long N, const float *w, uint16_t *gd0, float *dob, float *lossb)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const float tg = fminf(fmaxf(target[t] / M, -1.0f), 1.0f);
    const float q = tg > 0.0f ? pw : 1.0f;
    const float x = 2.0f * ob[t];
    const float sp = fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
    lossb[t] = q * (sp - x * 0.5f * (1.0f + tg));
    const float dO = q * (tanhf(ob[t]) - tg) / (float)N;
    dob[t] = dO;
    for (int c = 0; c < C; c += 8) {
        const bf8 m = ld8(d0b + t * C + c);
        float o[8];
#pragma unroll
        for (int i = 0; i < 8; i++) o[i] = m.get(i) > 0.0f ? w[c + i] * dO : 0.0f;
        *(uint4 *)(gd0 + t * C + c) = pack8(o);
    }
}

// partial sums of the head gradient over chunks of HCH pixels: part[chunk][j], j = 0: loss,
// 1: db = sum dO, 2 + c: dw_c = sum dO d0[., c].  Thread (g, c) = (tid / C, tid % C) adds the
// pixels g, g + G, ... of the chunk (G = 256 / C groups, channel-coalesced reads), then the groups
// are added in a fixed order.
constexpr int HCH = 4096;
__global__ void __launch_bounds__(256) k_head_grad(const float *d0, const float *dob, const float *lossb, int C,
                                                   long long N, float *part)
{
    __shared__ float red[256], rl[256], rd[256];
    const int G = 256 / C, tid = threadIdx.x;
    const int g = tid / C, c = tid % C;
    const long long p0 = (long long)blockIdx.x * HCH, p1 = p0 + HCH < N ? p0 + HCH : N;
    float acc = 0.0f, al = 0.0f, ad = 0.0f;
    if (g < G) {
        for (long long px = p0 + g; px < p1; px += G) {
            const float d = dob[px];
            acc = fmaf(d, d0[px * C + c], acc);
            if (c == 0) { al += lossb[px]; ad += d; }
        }
    }
    red[tid] = acc; rl[tid] = al; rd[tid] = ad;
    __syncthreads();
    const int maxc = C + 2;
    if (tid < C) {
        float sw = 0.0f;
        for (int k = 0; k < G; k++) sw += red[k * C + tid];
        part[(long long)blockIdx.x * maxc + 2 + tid] = sw;
    }
    if (tid == 0) {
        float sl = 0.0f, sd = 0.0f;
        for (int k = 0; k < G; k++) { sl += rl[k * C]; sd += rd[k * C]; }
        part[(long long)blockIdx.x * maxc] = sl;
        part[(long long)blockIdx.x * maxc + 1] = sd;
    }
}

// column j of the partials (one block per column): loss / N, db, dw
__global__ void __launch_bounds__(256) k_head_reduce(const float *part, int nb, int maxc, float *loss, float *db,
                                                     float *dw, long long N)
{
    __shared__ float red[256];
    const int j = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(long long)b * maxc + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (j == 0) loss[0] = red[0] / (float)N;
        else if (j == 1) db[0] = red[0];
        else dw[j - 2] = red[0];
    }
}

// Adam on FP32 master weights
__global__ void k_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gg = g[t];
    m[t] = b1 * m[t] + (1.0f - b1) * gg;
    v[t] = b2 * v[t] + (1.0f - b2) * gg * gg;
    p[t] -= lr * (m[t] / c1) / (sqrtf(v[t] / c2) + eps);
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ==========================================================================
struct NetLayer {
    int IC, ICr, OC;                         // input channels as stored (padded), real input channels, outputs
    float *w32 = nullptr, *b32 = nullptr, *gw = nullptr, *gb = nullptr;
    float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;
    uint16_t *wp = nullptr, *wt = nullptr;   // packed forward weights, data-gradient weights (null: none needed)
};

// a bf16 NHWC view: element (px, c) at p[px * ps + off + c]
struct View {
    uint16_t *p; int ps, off;
};

struct mgseg_net {
    int base = 32, depth = 4;
    // enc[2l], enc[2l+1]: the two convolutions of encoder block l; dec[2l], dec[2l+1]: of decoder block l < depth-1
    std::vector<NetLayer> enc, dec;
    float *hw = nullptr, *hb = nullptr, *ghw = nullptr, *ghb = nullptr, *mhw = nullptr, *vhw = nullptr,
          *mhb = nullptr, *vhb = nullptr;
    // activations for the current (B, H, W), NHWC
    int B = 0, H = 0, W = 0;
    uint16_t *x0 = nullptr;                  // input [px][16]
    std::vector<uint16_t *> emid, dmid;      // first convolution's output of encoder / decoder block l [px][C_l]
    std::vector<uint16_t *> cat;             // cat[l]: [px][C_{l+1} + C_l] = [up(d_{l+1}) | e_l] (l < depth-1)
    std::vector<uint16_t *> pool;            // pool[l] = avgpool(e_l) at level l+1, [px][C_l]
    uint16_t *ebot = nullptr;                // e_{depth-1} [px][C_{depth-1}]
    std::vector<uint16_t *> dact;            // d_l [px][C_l] (l < depth-1)
    float *d0f = nullptr, *ob = nullptr, *phi = nullptr;   // FP32 d_0 [px][C_0], head output o, M tanh(o)
    // gradients (same shapes)
    std::vector<uint16_t *> gemid, gdmid, gcat, gpool, gdact;
    uint16_t *gebot = nullptr;
    float *part = nullptr, *partb = nullptr, *hpart = nullptr, *loss = nullptr;
    float *dob = nullptr, *lossb = nullptr;  // per-pixel dloss/do and loss terms
    std::vector<void *> act_allocs, par_allocs;
    int steps = 0;
    // k_conv launch timing (mgseg_net_profile): event pairs, algorithmic flops
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_flops = 0.0;
};

namespace {

constexpr long long PART_MAX = 16LL << 20;   // floats of weight-gradient partials

int chan(const mgseg_net *n, int l) { return n->base << l; }

template <typename T>
T *nalloc(std::vector<void *> &v, size_t count, bool &fail)
{
    void *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) { (void)hipGetLastError(); fail = true; return nullptr; }
    (void)hipMemset(p, 0, count * sizeof(T));
    v.push_back(p);
    return (T *)p;
}

void free_acts(mgseg_net *n)
{
    (void)hipDeviceSynchronize();
    for (void *p : n->act_allocs) (void)hipFree(p);
    n->act_allocs.clear();
    n->emid.clear(); n->dmid.clear(); n->cat.clear(); n->pool.clear(); n->dact.clear();
    n->gemid.clear(); n->gdmid.clear(); n->gcat.clear(); n->gpool.clear(); n->gdact.clear();
    n->B = n->H = n->W = 0;
}

// partial count of a weight gradient: at most 256, the pixel tile count, and PART_MAX floats in all
int wgrad_parts(const NetLayer &L, int B, int h, int w)
{
    const long long tiles = (long long)B * ((h + TY - 1) / TY) * ((w + TX - 1) / TX);
    const long long per = (long long)L.OC * 9 * L.IC;
    const long long P = std::min<long long>(256, std::max<long long>(1, PART_MAX / per));
    return (int)std::min(P, tiles);
}

bool ensure_acts(mgseg_net *n, int B, int H, int W)
{
    if (n->B == B && n->H == H && n->W == W) return true;
    free_acts(n);
    bool fail = false;
    auto &v = n->act_allocs;
    const int D = n->depth;
    n->x0 = nalloc<uint16_t>(v, (size_t)B * CIN0 * H * W, fail);
    for (int l = 0; l < D; l++) {
        const size_t np = (size_t)B * (H >> l) * (W >> l);
        const int ce = chan(n, l);
        n->emid.push_back(nalloc<uint16_t>(v, np * ce, fail));
        n->gemid.push_back(nalloc<uint16_t>(v, np * ce, fail));
        if (l == D - 1) break;
        const int cu = chan(n, l + 1);
        n->cat.push_back(nalloc<uint16_t>(v, np * (cu + ce), fail));
        n->gcat.push_back(nalloc<uint16_t>(v, np * (cu + ce), fail));
        n->pool.push_back(nalloc<uint16_t>(v, np / 4 * ce, fail));
        n->gpool.push_back(nalloc<uint16_t>(v, np / 4 * ce, fail));
        n->dmid.push_back(nalloc<uint16_t>(v, np * ce, fail));
        n->gdmid.push_back(nalloc<uint16_t>(v, np * ce, fail));
        n->dact.push_back(nalloc<uint16_t>(v, np * ce, fail));
        n->gdact.push_back(nalloc<uint16_t>(v, np * ce, fail));
    }
    const size_t npb = (size_t)B * (H >> (D - 1)) * (W >> (D - 1));
    n->ebot = nalloc<uint16_t>(v, npb * chan(n, D - 1), fail);
    n->gebot = nalloc<uint16_t>(v, npb * chan(n, D - 1), fail);
    n->d0f = nalloc<float>(v, (size_t)B * chan(n, 0) * H * W, fail);
    n->ob = nalloc<float>(v, (size_t)B * H * W, fail);
    n->phi = nalloc<float>(v, (size_t)B * H * W, fail);
    long long need = 0, needb = 0;
    for (int l = 0; l < D; l++) {
        const int h = H >> l, w = W >> l;
        auto acc_need = [&](const NetLayer &L) {
            const int P = wgrad_parts(L, B, h, w);
            need = std::max(need, (long long)P * L.OC * 9 * L.IC);
            needb = std::max(needb, (long long)P * L.OC);
        };
        acc_need(n->enc[2 * l]); acc_need(n->enc[2 * l + 1]);
        if (l < D - 1) { acc_need(n->dec[2 * l]); acc_need(n->dec[2 * l + 1]); }
    }
    n->part = nalloc<float>(v, (size_t)need, fail);
    n->partb = nalloc<float>(v, (size_t)needb, fail);
    n->hpart = nalloc<float>(v, (size_t)((B * (long long)H * W + HCH - 1) / HCH) * (chan(n, 0) + 2), fail);
    n->dob = nalloc<float>(v, (size_t)B * H * W, fail);
    n->lossb = nalloc<float>(v, (size_t)B * H * W, fail);
    n->loss = nalloc<float>(v, 4, fail);
    if (fail) { free_acts(n); return false; }
    n->B = B; n->H = H; n->W = W;
    return true;
}

// icr: the input channels that carry data (the stored count IC may include zero padding); used for the
// algorithmic flop count of a profiled launch
void conv(mgseg_net *n, hipStream_t s, View in, const uint16_t *Wk, const float *bias, int IC, int OC, View out, int H,
          int W, int B, int relu, float *out32 = nullptr, const uint16_t *mask = nullptr, int mps = 0, int moff = 0,
          int icr = 0)
{
    ConvArgs A;
    A.in = in.p; A.ips = in.ps; A.ioff = in.off; A.Wk = Wk; A.bias = bias;
    A.out = out.p; A.ops = out.ps; A.ooff = out.off; A.out32 = out32;
    A.mask = mask; A.mps = mps; A.moff = moff;
    A.IC = IC; A.OC = OC; A.H = H; A.W = W; A.relu = relu;
    const unsigned tiles = (unsigned)(((H + TY - 1) / TY) * ((W + TX - 1) / TX));
    dim3 g(tiles, (unsigned)((OC + OCB - 1) / OCB), (unsigned)B);
    hipEvent_t e[2] = {nullptr, nullptr};
    if (n->prof) {
        while (n->ev_pool.size() < n->ev_used + 2) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) { (void)hipGetLastError(); break; }
            n->ev_pool.push_back(ev);
        }
        if (n->ev_pool.size() >= n->ev_used + 2) {
            e[0] = n->ev_pool[n->ev_used]; e[1] = n->ev_pool[n->ev_used + 1];
            n->ev_used += 2;
            n->prof_flops += 2.0 * 9.0 * (icr ? icr : IC) * OC * (double)H * W * B;
            (void)hipEventRecord(e[0], s);
        }
    }
    hipLaunchKernelGGL(k_conv, g, dim3(256), 0, s, A);
    if (e[1]) (void)hipEventRecord(e[1], s);
}

void wgrad(mgseg_net *n, hipStream_t s, View g, View x, NetLayer &L, int H, int W, int B)
{
    WgradArgs A;
    A.g = g.p; A.gps = g.ps; A.goff = g.off; A.x = x.p; A.xps = x.ps; A.xoff = x.off;
    A.part = n->part; A.partb = n->partb;
    A.IC = L.IC; A.OC = L.OC; A.H = H; A.W = W; A.B = B;
    A.P = wgrad_parts(L, B, H, W);
    dim3 gr((unsigned)A.P, (unsigned)((L.OC + OCB - 1) / OCB), (unsigned)(L.IC / 16));
    hipLaunchKernelGGL(k_wgrad, gr, dim3(256), 0, s, A);
    const long long tot = (long long)L.OC * L.ICr * 9 + L.OC;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk(tot)), dim3(256), 0, s, n->part, n->partb, A.P, L.OC, L.IC, L.ICr,
                       L.gw, L.gb);
}

// forward of one block: mid = relu(conv_a(x)), y = relu(conv_b(mid))
void block_fwd(mgseg_net *n, hipStream_t s, NetLayer &a, NetLayer &b, View x, uint16_t *mid, View y, int h, int w,
               int B, float *y32 = nullptr)
{
    conv(n, s, x, a.wp, a.b32, a.IC, a.OC, View{mid, a.OC, 0}, h, w, B, 1, nullptr, nullptr, 0, 0, a.ICr);
    conv(n, s, View{mid, a.OC, 0}, b.wp, b.b32, b.IC, b.OC, y, h, w, B, 1, y32);
}

// backward of one block, gy = gradient of y already zeroed where y <= 0: weight gradients, and the
// gradient of x into gx when gx.p is set
void block_bwd(mgseg_net *n, hipStream_t s, NetLayer &a, NetLayer &b, View x, uint16_t *mid, uint16_t *gmid, View gy,
               View gx, int h, int w, int B)
{
    const View vm{mid, a.OC, 0}, vgm{gmid, a.OC, 0};
    wgrad(n, s, gy, vm, b, h, w, B);
    conv(n, s, gy, b.wt, nullptr, b.OC, b.IC, vgm, h, w, B, 0, nullptr, mid, a.OC, 0);
    wgrad(n, s, vgm, x, a, h, w, B);
    if (gx.p) conv(n, s, vgm, a.wt, nullptr, a.OC, a.ICr, gx, h, w, B, 0);
}

// SplitMix64 + Box-Muller: He-normal initial weights from the seed
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uni() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() { return std::sqrt(-2.0 * std::log(uni())) * std::cos(6.283185307179586 * uni()); }
};

void pack(hipStream_t s, NetLayer &L)
{
    const long long nt = std::max((long long)L.OC * 9 * L.IC, (long long)L.ICr * 9 * L.OC);
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(nt)), dim3(256), 0, s, L.w32, L.OC, L.ICr, L.IC, L.wp, L.wt);
}

bool make_layer(mgseg_net *n, NetLayer &L, int ICr, int IC, int OC, bool need_dgrad, Rng &rng)
{
    bool fail = false;
    auto &v = n->par_allocs;
    const size_t nw = (size_t)OC * ICr * 9;
    L.IC = IC; L.ICr = ICr; L.OC = OC;
    L.w32 = nalloc<float>(v, nw, fail); L.b32 = nalloc<float>(v, OC, fail);
    L.gw = nalloc<float>(v, nw, fail); L.gb = nalloc<float>(v, OC, fail);
    L.mw = nalloc<float>(v, nw, fail); L.vw = nalloc<float>(v, nw, fail);
    L.mb = nalloc<float>(v, OC, fail); L.vb = nalloc<float>(v, OC, fail);
    L.wp = nalloc<uint16_t>(v, (size_t)OC * 9 * IC, fail);
    L.wt = need_dgrad ? nalloc<uint16_t>(v, nw, fail) : nullptr;
    if (fail) return false;
    std::vector<float> w(nw);
    const double sd = std::sqrt(2.0 / (9.0 * ICr));
    for (auto &x : w) x = (float)(sd * rng.normal());
    (void)hipMemcpy(L.w32, w.data(), nw * sizeof(float), hipMemcpyHostToDevice);
    pack(0, L);
    return true;
}

// parameters in a fixed order: the convolutions enc[0..2D-1], then dec[0..2D-3], each w (OC*ICr*9) then b (OC);
// head w (C0), head b (1)
template <class F>
void for_params(mgseg_net *n, F f)
{
    for (auto *v : {&n->enc, &n->dec})
        for (auto &L : *v) {
            f(L.w32, L.gw, L.mw, L.vw, (long long)L.OC * L.ICr * 9);
            f(L.b32, L.gb, L.mb, L.vb, (long long)L.OC);
        }
    f(n->hw, n->ghw, n->mhw, n->vhw, (long long)chan(n, 0));
    f(n->hb, n->ghb, n->mhb, n->vhb, 1LL);
}

void pack_all(mgseg_net *n, hipStream_t s)
{
    for (auto *v : {&n->enc, &n->dec})
        for (auto &L : *v) pack(s, L);
}

}  // namespace

extern "C" {

void mgseg_net_destroy(mgseg_net *n)
{
    if (!n) return;
    free_acts(n);
    for (hipEvent_t e : n->ev_pool) (void)hipEventDestroy(e);
    for (void *p : n->par_allocs) (void)hipFree(p);
    delete n;
}

mgseg_status mgseg_net_create(int base_channels, int depth, uint64_t seed, mgseg_net **out)
{
    if (!out) return MGSEG_E_ARG;
    *out = nullptr;
    if (base_channels < 16 || base_channels > 256 || base_channels % 16 || depth < 2 || depth > 6) return MGSEG_E_ARG;
    if ((base_channels << (depth - 1)) > 512) return MGSEG_E_ARG;
    mgseg_net *n = new (std::nothrow) mgseg_net();
    if (!n) return MGSEG_E_NOMEM;
    n->base = base_channels; n->depth = depth;
    Rng rng{seed};
    n->enc.resize(2 * depth);
    n->dec.resize(2 * (depth - 1));
    bool ok = true;
    for (int l = 0; l < depth && ok; l++) {
        const int ic = l == 0 ? 3 : chan(n, l - 1);
        ok = make_layer(n, n->enc[2 * l], ic, l == 0 ? CIN0 : ic, chan(n, l), l > 0, rng);
        if (ok) ok = make_layer(n, n->enc[2 * l + 1], chan(n, l), chan(n, l), chan(n, l), true, rng);
    }
    for (int l = 0; l < depth - 1 && ok; l++) {
        const int ic = chan(n, l + 1) + chan(n, l);
        ok = make_layer(n, n->dec[2 * l], ic, ic, chan(n, l), true, rng);
        if (ok) ok = make_layer(n, n->dec[2 * l + 1], chan(n, l), chan(n, l), chan(n, l), true, rng);
    }
    bool fail = !ok;
    auto &v = n->par_allocs;
    const int C0 = chan(n, 0);
    n->hw = nalloc<float>(v, C0, fail); n->hb = nalloc<float>(v, 1, fail);
    n->ghw = nalloc<float>(v, C0, fail); n->ghb = nalloc<float>(v, 1, fail);
    n->mhw = nalloc<float>(v, C0, fail); n->vhw = nalloc<float>(v, C0, fail);
    n->mhb = nalloc<float>(v, 1, fail); n->vhb = nalloc<float>(v, 1, fail);
    if (fail) { mgseg_net_destroy(n); return MGSEG_E_NOMEM; }
    std::vector<float> hw(C0);
    for (auto &x : hw) x = (float)(std::sqrt(1.0 / C0) * rng.normal());
    (void)hipMemcpy(n->hw, hw.data(), C0 * sizeof(float), hipMemcpyHostToDevice);
    if (hipDeviceSynchronize() != hipSuccess) { mgseg_net_destroy(n); return MGSEG_E_HIP; }
    *out = n;
    return MGSEG_OK;
}

mgseg_status mgseg_net_forward(mgseg_net *n, const float *in_dev, int B, int H, int W, double M, float *phi0_dev,
                               void *stream)
{
    if (!n || !in_dev || B < 1 || H < 1 || W < 1 || !(M > 0.0)) return MGSEG_E_ARG;
    const int D = n->depth;
    if (H % (1 << (D - 1)) || W % (1 << (D - 1))) return MGSEG_E_SHAPE;
    if (!ensure_acts(n, B, H, W)) return MGSEG_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;
    const long long NP0 = (long long)B * H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(nblk(NP0)), dim3(256), 0, s, in_dev, (long long)H * W, B, n->x0);
    // encoder
    View cur{n->x0, CIN0, 0};
    for (int l = 0; l < D; l++) {
        const int h = H >> l, w = W >> l, ce = chan(n, l);
        const View e = l < D - 1 ? View{n->cat[l], chan(n, l + 1) + ce, chan(n, l + 1)} : View{n->ebot, ce, 0};
        block_fwd(n, s, n->enc[2 * l], n->enc[2 * l + 1], cur, n->emid[l], e, h, w, B);
        if (l < D - 1) {
            hipLaunchKernelGGL(k_avgpool, dim3(nblk((long long)B * (h / 2) * (w / 2) * (ce / 8))), dim3(256), 0, s, e.p,
                               e.ps, e.off, ce, h / 2, w / 2, B, n->pool[l]);
            cur = View{n->pool[l], ce, 0};
        }
    }
    // decoder
    const uint16_t *dn = n->ebot;
    for (int l = D - 2; l >= 0; l--) {
        const int h = H >> l, w = W >> l;
        const int cu = chan(n, l + 1), ce = chan(n, l);
        hipLaunchKernelGGL(k_upsample, dim3(nblk((long long)B * h * w * (cu / 8))), dim3(256), 0, s, dn, cu, h / 2, w / 2, B,
                           n->cat[l], cu + ce);
        block_fwd(n, s, n->dec[2 * l], n->dec[2 * l + 1], View{n->cat[l], cu + ce, 0}, n->dmid[l],
                  View{n->dact[l], ce, 0}, h, w, B, l == 0 ? n->d0f : nullptr);
        dn = n->dact[l];
    }
    hipLaunchKernelGGL(k_head, dim3(nblk(NP0)), dim3(256), 0, s, n->d0f, chan(n, 0), NP0, n->hw, n->hb, (float)M,
                       n->ob, phi0_dev ? phi0_dev : n->phi);
    if (hipGetLastError() != hipSuccess) return MGSEG_E_HIP;
    return MGSEG_OK;
}

mgseg_status mgseg_net_backward(mgseg_net *n, const float *target_dev, double M, double pos_weight, float *loss_host,
                                void *stream)
{
    if (!n || !target_dev || !(M > 0.0) || !(pos_weight > 0.0)) return MGSEG_E_ARG;
    if (n->B == 0) return MGSEG_E_STATE;
    hipStream_t s = (hipStream_t)stream;
    const int D = n->depth, B = n->B, H = n->H, W = n->W, C0 = chan(n, 0);
    const long long NP0 = (long long)B * H * W;
    const int maxc = C0 + 2;
    const unsigned nch = (unsigned)((NP0 + HCH - 1) / HCH);
    // head and loss; gradient of d_0 (masked) -> gdact[0]
    hipLaunchKernelGGL(k_head_bwd, dim3(nblk(NP0)), dim3(256), 0, s, n->ob, target_dev, (float)M, (float)pos_weight,
                       n->dact[0], C0, NP0, n->hw, n->gdact[0], n->dob, n->lossb);
    hipLaunchKernelGGL(k_head_grad, dim3(nch), dim3(256), 0, s, n->d0f, n->dob, n->lossb, C0, NP0, n->hpart);
    hipLaunchKernelGGL(k_head_reduce, dim3(maxc), dim3(256), 0, s, n->hpart, (int)nch, maxc, n->loss, n->ghb, n->ghw,
                       NP0);
    // decoder, level 0 first
    for (int l = 0; l <= D - 2; l++) {
        const int h = H >> l, w = W >> l;
        const int cu = chan(n, l + 1), ce = chan(n, l);
        block_bwd(n, s, n->dec[2 * l], n->dec[2 * l + 1], View{n->cat[l], cu + ce, 0}, n->dmid[l], n->gdmid[l],
                  View{n->gdact[l], ce, 0}, View{n->gcat[l], cu + ce, 0}, h, w, B);
        // up-sampled part of the input -> gradient of the level below's d (or of e_bottom), masked by it
        uint16_t *gdn = (l + 1 <= D - 2) ? n->gdact[l + 1] : n->gebot;
        const uint16_t *ydn = (l + 1 <= D - 2) ? n->dact[l + 1] : n->ebot;
        hipLaunchKernelGGL(k_upsample_bwd, dim3(nblk((long long)B * (h / 2) * (w / 2) * (cu / 8))), dim3(256), 0, s,
                           n->gcat[l], cu + ce, cu, h / 2, w / 2, B, ydn, gdn);
    }
    // encoder, bottom up
    for (int l = D - 1; l >= 0; l--) {
        const int h = H >> l, w = W >> l, ce = chan(n, l);
        View g;
        if (l == D - 1) {
            g = View{n->gebot, ce, 0};
        } else {
            const int cu = chan(n, l + 1);
            g = View{n->gcat[l], cu + ce, cu};
            // pooled path: g_e += avgpool^T(g_pool), then the ReLU mask of e
            hipLaunchKernelGGL(k_avgpool_bwd, dim3(nblk((long long)B * h * w * (ce / 8))), dim3(256), 0, s, n->gpool[l], ce,
                               h / 2, w / 2, B, g.p, g.ps, g.off, n->cat[l], cu + ce, cu);
        }
        const View x = l == 0 ? View{n->x0, CIN0, 0} : View{n->pool[l - 1], chan(n, l - 1), 0};
        const View gx = l > 0 ? View{n->gpool[l - 1], chan(n, l - 1), 0} : View{nullptr, 0, 0};
        block_bwd(n, s, n->enc[2 * l], n->enc[2 * l + 1], x, n->emid[l], n->gemid[l], g, gx, h, w, B);
    }
    if (hipGetLastError() != hipSuccess) return MGSEG_E_HIP;
    if (loss_host) {
        float lv = 0.0f;
        (void)hipMemcpyAsync(&lv, n->loss, sizeof(float), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess) return MGSEG_E_HIP;
        *loss_host = lv;
    }
    return MGSEG_OK;
}

mgseg_status mgseg_net_adam_step(mgseg_net *n, double lr, double b1, double b2, double eps, void *stream)
{
    if (!n || !(lr >= 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps > 0.0))
        return MGSEG_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    n->steps++;
    const float c1 = (float)(1.0 - std::pow(b1, n->steps)), c2 = (float)(1.0 - std::pow(b2, n->steps));
    for_params(n, [&](float *p, float *g, float *m, float *v, long long cnt) {
        hipLaunchKernelGGL(k_adam, dim3(nblk(cnt)), dim3(256), 0, s, p, g, m, v, cnt, (float)lr, (float)b1, (float)b2,
                           (float)eps, c1, c2);
    });
    pack_all(n, s);
    return hipGetLastError() == hipSuccess ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_param_count(mgseg_net *n, long long *count)
{
    if (!n || !count) return MGSEG_E_ARG;
    long long c = 0;
    for_params(n, [&](float *, float *, float *, float *, long long k) { c += k; });
    *count = c;
    return MGSEG_OK;
}

mgseg_status mgseg_net_get_params(mgseg_net *n, float *host, float *grad_host)
{
    if (!n || (!host && !grad_host)) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    long long off = 0;
    bool ok = true;
    for_params(n, [&](float *p, float *g, float *, float *, long long k) {
        if (host) ok &= hipMemcpy(host + off, p, k * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
        if (grad_host) ok &= hipMemcpy(grad_host + off, g, k * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
        off += k;
    });
    return ok ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_get_adam(mgseg_net *n, float *m_host, float *v_host, long long *steps)
{
    if (!n) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    long long off = 0;
    bool ok = true;
    for_params(n, [&](float *, float *, float *m, float *v, long long k) {
        if (m_host) ok &= hipMemcpy(m_host + off, m, k * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
        if (v_host) ok &= hipMemcpy(v_host + off, v, k * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
        off += k;
    });
    if (steps) *steps = n->steps;
    return ok ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_set_adam(mgseg_net *n, const float *m_host, const float *v_host, long long steps)
{
    if (!n || !m_host || !v_host || steps < 0 || steps > 0x7fffffffLL) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    long long off = 0;
    bool ok = true;
    for_params(n, [&](float *, float *, float *m, float *v, long long k) {
        ok &= hipMemcpy(m, m_host + off, k * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        ok &= hipMemcpy(v, v_host + off, k * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        off += k;
    });
    n->steps = (int)steps;
    return ok ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_set_params(mgseg_net *n, const float *host)
{
    if (!n || !host) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    long long off = 0;
    bool ok = true;
    for_params(n, [&](float *p, float *, float *m, float *v, long long k) {
        ok &= hipMemcpy(p, host + off, k * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        ok &= hipMemset(m, 0, k * sizeof(float)) == hipSuccess && hipMemset(v, 0, k * sizeof(float)) == hipSuccess;
        off += k;
    });
    pack_all(n, 0);
    n->steps = 0;
    return ok && hipDeviceSynchronize() == hipSuccess ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_profile(mgseg_net *n, int enable)
{
    if (!n) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    n->prof = enable != 0;
    n->ev_used = 0;
    n->prof_flops = 0.0;
    return MGSEG_OK;
}

mgseg_status mgseg_net_profile_read(mgseg_net *n, double *total_ms, int *launches, double *flops)
{
    if (!n) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    double ms = 0.0;
    for (size_t i = 0; i + 1 < n->ev_used; i += 2) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, n->ev_pool[i], n->ev_pool[i + 1]) != hipSuccess) return MGSEG_E_HIP;
        ms += t;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = (int)(n->ev_used / 2);
    if (flops) *flops = n->prof_flops;
    return MGSEG_OK;
}

}  // extern "C"
