// mgseg_net.hip -- learned warm start: a small convolutional encoder-decoder
// that maps (image, marker distance map, marker mask) to an initial level set
// phi0 = M tanh(o); the FAS V-cycle then finishes every solve.
//
// Architecture (depth D, base width C0, C_l = C0 2^l; every block is two
// 3x3 convolutions with ReLU, cb(x) = relu(conv_b(relu(conv_a(x))))):
//   encoder  e_l = cb(p_{l-1}), p_l = avgpool2(e_l)     (e_0 = cb(input))
//   decoder  d_l = cb([up2(d_{l+1}) | e_l])              (d_{D-1} = e_{D-1})
//   head     o = w . d_0 + b (1x1),  phi0 = M tanh(o)
// Storage: activations and convolution weights in bf16, accumulation in FP32
// (MFMA 16x16x16 bf16), FP32 master weights with Adam.  Tensors are NCHW.
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
// 3x3 convolution, zero padding, stride 1, as an implicit GEMM:
//   out[b, oc, p] = sum_{ic, r} Wk[oc, ic*9 + r] in[b, ic, p + off(r)] (+ bias[oc]), off(r) = (r/3-1, r%3-1)
// Block 256 = 4 waves; block tile 32 oc x 32 pixels (pixels of all images in
// one index, px = b*HW + p); each wave one 16 x 16 MFMA tile, K in steps of
// 16.  in / out: bf16 with channel stride HW and image strides ibs / obs.
struct ConvArgs {
    const uint16_t *in; long long ibs;
    const uint16_t *W; int K;            // Wk row-major [OC][K], K = IC*9
    const float *bias;                   // may be null
    uint16_t *out; long long obs;
    float *out32; long long o32bs;       // optional FP32 copy of the output (null: none)
    int IC, OC, H, Wd, B, relu;
};

__global__ void __launch_bounds__(256) k_conv3x3(ConvArgs A)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HW = A.H * A.Wd;
    const long long NP = (long long)A.B * HW;
    const int oc0 = blockIdx.y * 32 + (wave >> 1) * 16;
    const long long px0 = (long long)blockIdx.x * 32 + (wave & 1) * 16;
    // this lane's B-column pixel and A-row channel
    const long long pxb = px0 + (lane & 15);
    const bool pvalid = pxb < NP;
    const int bimg = pvalid ? (int)(pxb / HW) : 0;
    const int pp = pvalid ? (int)(pxb % HW) : 0;
    const int py = pp / A.Wd, pxx = pp % A.Wd;
    const uint16_t *inb = A.in + (long long)bimg * A.ibs;
    const int arow = oc0 + (lane & 15);
    const uint16_t *wrow = A.W + (long long)(arow < A.OC ? arow : 0) * A.K;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < A.K; k0 += 16) {
        bf16x4 a, bv;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int k = k0 + 4 * (lane >> 4) + i;
            uint16_t av = 0, bvv = 0;
            if (k < A.K) {
                if (arow < A.OC) av = wrow[k];
                if (pvalid) {
                    const int ic = k / 9, r = k - 9 * ic;
                    const int yy = py + r / 3 - 1, xx = pxx + r % 3 - 1;
                    if (yy >= 0 && yy < A.H && xx >= 0 && xx < A.Wd) bvv = inb[(long long)ic * HW + yy * A.Wd + xx];
                }
            }
            a[i] = (short)av;
            bv[i] = (short)bvv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc, 0, 0, 0);
    }
    // D[row = 4*(lane/16) + i][col = lane % 16]
    const long long px = px0 + (lane & 15);
    if (px >= NP) return;
    const int ob = (int)(px / HW), op = (int)(px % HW);
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int oc = oc0 + 4 * (lane >> 4) + i;
        if (oc >= A.OC) continue;
        float v = acc[i] + (A.bias ? A.bias[oc] : 0.0f);
        if (A.relu) v = fmaxf(v, 0.0f);
        A.out[(long long)ob * A.obs + (long long)oc * HW + op] = f2bf(v);
        if (A.out32) A.out32[(long long)ob * A.o32bs + (long long)oc * HW + op] = v;
    }
}

// weight gradient: dW[oc, ic*9 + r] = sum_{b, p} g[b, oc, p] x[b, ic, p + off(r)],
// dbias[oc] = sum g.  M = OC (16 per wave-tile), N = IC*9 (16), K = pixels;
// each block takes a chunk of CH pixels and writes its partial sums (FP32)
// to part[chunk][OC][K] / partb[chunk][OC]; k_wgrad_reduce adds the chunks in
// order (deterministic).  Block 256: 4 waves along N.
struct WgradArgs {
    const uint16_t *g; long long gbs;     // gradient of the conv output (relu-masked), bf16
    const uint16_t *x; long long xbs;     // conv input
    float *part, *partb;
    int IC, OC, H, Wd, B, chunk;
};

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs A)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HW = A.H * A.Wd, K = A.IC * 9;
    const long long NP = (long long)A.B * HW;
    const int oc0 = blockIdx.y * 16;
    const int n0 = blockIdx.z * 64 + wave * 16;
    const long long c0 = (long long)blockIdx.x * A.chunk;
    const int arow = oc0 + (lane & 15);            // A[m = oc][k = px]
    const int ncol = n0 + (lane & 15);             // B[k = px][n = ic*9 + r]
    const int ic = ncol / 9, r = ncol - 9 * (ncol / 9);
    const int dy = r / 3 - 1, dx = r % 3 - 1;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (long long k0 = c0; k0 < c0 + A.chunk && k0 < NP; k0 += 16) {
        bf16x4 a, bv;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const long long px = k0 + 4 * (lane >> 4) + i;
            uint16_t av = 0, bvv = 0;
            if (px < NP && px < c0 + A.chunk) {
                const int b = (int)(px / HW), p = (int)(px % HW);
                if (arow < A.OC) av = A.g[(long long)b * A.gbs + (long long)arow * HW + p];
                if (ncol < K) {
                    const int y = p / A.Wd + dy, xx = p % A.Wd + dx;
                    if (y >= 0 && y < A.H && xx >= 0 && xx < A.Wd)
                        bvv = A.x[(long long)b * A.xbs + (long long)ic * HW + y * A.Wd + xx];
                }
            }
            a[i] = (short)av;
            bv[i] = (short)bvv;
            if (wave == 0 && blockIdx.z == 0) bsum += bf2f(av);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc, 0, 0, 0);
    }
    const long long pbase = (long long)blockIdx.x * A.OC * K;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int oc = oc0 + 4 * (lane >> 4) + i;
        if (oc < A.OC && ncol < K) A.part[pbase + (long long)oc * K + ncol] = acc[i];
    }
    if (wave == 0 && blockIdx.z == 0) {
        // bias: lanes with the same row (lane % 16) hold the 4 pixel groups
        bsum += __shfl_xor(bsum, 16);
        bsum += __shfl_xor(bsum, 32);
        if (lane < 16 && arow < A.OC) A.partb[(long long)blockIdx.x * A.OC + arow] = bsum;
    }
}

__global__ void k_wgrad_reduce(const float *part, const float *partb, int nchunk, int OC, int K, float *dW, float *db)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long NW = (long long)OC * K;
    if (t < NW) {
        float s = 0.0f;
        for (int c = 0; c < nchunk; c++) s += part[(long long)c * NW + t];
        dW[t] = s;
    } else if (t < NW + OC) {
        const int oc = (int)(t - NW);
        float s = 0.0f;
        for (int c = 0; c < nchunk; c++) s += partb[(long long)c * OC + oc];
        db[oc] = s;
    }
}

// Wt[ic, oc*9 + r] = W[oc, ic*9 + 8 - r]: the data gradient is the convolution
// of the output gradient with the flipped, transposed kernel
__global__ void k_flip_weights(const uint16_t *W, int IC, int OC, uint16_t *Wt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= IC * OC * 9) return;
    const int ic = t / (OC * 9), rem = t % (OC * 9), oc = rem / 9, r = rem % 9;
    Wt[t] = W[(long long)oc * IC * 9 + ic * 9 + (8 - r)];
}

// g <- g * (y > 0) over C channels of B images (strides in elements)
__global__ void k_relu_mask(uint16_t *g, long long gbs, const uint16_t *y, long long ybs, int C, int HW, int B)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)C * HW;
    if (t >= per * B) return;
    const int b = (int)(t / per);
    const long long q = t % per;
    if (!(bf2f(y[(long long)b * ybs + q]) > 0.0f)) g[(long long)b * gbs + q] = 0;
}

// 2x2 average pooling and its adjoint (accumulating: g_in += 0.25 g_out)
__global__ void k_avgpool(const uint16_t *x, long long xbs, uint16_t *y, long long ybs, int C, int H, int W, int B)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int h = H / 2, w = W / 2;
    const long long per = (long long)C * h * w;
    if (t >= per * B) return;
    const int b = (int)(t / per);
    const long long q = t % per;
    const int c = (int)(q / (h * w)), yy = (int)(q % (h * w)) / w, xx = (int)(q % w);
    const uint16_t *s = x + (long long)b * xbs + (long long)c * H * W + (2 * yy) * W + 2 * xx;
    y[(long long)b * ybs + q] = f2bf(0.25f * (bf2f(s[0]) + bf2f(s[1]) + bf2f(s[W]) + bf2f(s[W + 1])));
}
__global__ void k_avgpool_bwd(const uint16_t *gy, long long gybs, uint16_t *gx, long long gxbs, int C, int H, int W,
                              int B)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)C * H * W;
    if (t >= per * B) return;
    const int b = (int)(t / per);
    const long long q = t % per;
    const int c = (int)(q / ((long long)H * W)), yy = (int)(q % ((long long)H * W)) / W, xx = (int)(q % W);
    const int h = H / 2, w = W / 2;
    const float g = bf2f(gy[(long long)b * gybs + (long long)c * h * w + (yy / 2) * w + xx / 2]);
    uint16_t *d = gx + (long long)b * gxbs + q;
    *d = f2bf(bf2f(*d) + 0.25f * g);
}

// nearest 2x upsampling into channels [0, C) of y, and its adjoint (2x2 sums)
__global__ void k_upsample(const uint16_t *x, long long xbs, uint16_t *y, long long ybs, int C, int h, int w, int B)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int H = 2 * h, W = 2 * w;
    const long long per = (long long)C * H * W;
    if (t >= per * B) return;
    const int b = (int)(t / per);
    const long long q = t % per;
    const int c = (int)(q / ((long long)H * W)), yy = (int)(q % ((long long)H * W)) / W, xx = (int)(q % W);
    y[(long long)b * ybs + q] = x[(long long)b * xbs + (long long)c * h * w + (yy / 2) * w + xx / 2];
}
__global__ void k_upsample_bwd(const uint16_t *gy, long long gybs, uint16_t *gx, long long gxbs, int C, int h, int w,
                               int B)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)C * h * w;
    if (t >= per * B) return;
    const int b = (int)(t / per);
    const long long q = t % per;
    const int c = (int)(q / ((long long)h * w)), yy = (int)(q % ((long long)h * w)) / w, xx = (int)(q % w);
    const int W = 2 * w;
    const uint16_t *s = gy + (long long)b * gybs + (long long)c * 4 * h * w + (2 * yy) * W + 2 * xx;
    gx[(long long)b * gxbs + q] = f2bf(bf2f(s[0]) + bf2f(s[1]) + bf2f(s[W]) + bf2f(s[W + 1]));
}

// input features (FP32 NCHW, 3 channels) to bf16
__global__ void k_to_bf16(const float *x, uint16_t *y, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = f2bf(x[t]);
}

// head: o = w . d0 + b, phi0 = M tanh(o) (FP32 from the FP32 copy of d0); keeps o for the loss
__global__ void k_head(const float *d0, int C, int HW, int B, const float *w, const float *b, float M, float *ob,
                       float *phi)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * HW) return;
    const int bi = (int)(t / HW), p = (int)(t % HW);
    const float *x = d0 + (long long)bi * C * HW + p;
    float o = b[0];
    for (int c = 0; c < C; c++) o = fmaf(w[c], x[(long long)c * HW], o);
    ob[t] = o;
    phi[t] = M * tanhf(o);
}

// Loss: binary cross-entropy of p = sigmoid(2 o) = (1 + tanh o) / 2 against the
// soft target q = (1 + tg) / 2, tg = clip(target / M, -1, 1), weighted by
// w = pw on the object (tg > 0) and 1 elsewhere, averaged over the N pixels:
//   loss = mean w (softplus(2 o) - 2 o q),   dloss/do = w (tanh o - tg) / N,
// whose minimum is at tanh o = tg and whose gradient does not vanish where the
// output saturates on the wrong side.  Head gradient partials per block;
// gd0 = w_head dO (bf16, then relu-masked by the caller).
__global__ void __launch_bounds__(256) k_head_bwd(const float *ob, const float *target, float M, float pw,
                                                  const float *d0, int C, int HW, int B, const float *w, uint16_t *gd0,
                                                  float *part, int maxc)
{
    __shared__ float red[256];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long N = (long long)B * HW;
    float loss = 0.0f, dO = 0.0f;
    int bi = 0, p = 0;
    if (t < N) {
        bi = (int)(t / HW); p = (int)(t % HW);
        const float tg = fminf(fmaxf(target[t] / M, -1.0f), 1.0f);
        const float q = tg > 0.0f ? pw : 1.0f;
        const float x = 2.0f * ob[t];
        const float sp = fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
        loss = q * (sp - x * 0.5f * (1.0f + tg));
        dO = q * (tanhf(ob[t]) - tg) / (float)N;
        for (int c = 0; c < C; c++) gd0[(long long)bi * C * HW + (long long)c * HW + p] = f2bf(w[c] * dO);
    }
    // partials: [0] loss, [1] db, [2 + c] dw_c
    for (int j = 0; j < C + 2 && j < maxc; j++) {
        float v = 0.0f;
        if (t < N) v = j == 0 ? loss : (j == 1 ? dO : dO * d0[(long long)bi * C * HW + (long long)(j - 2) * HW + p]);
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(long long)blockIdx.x * maxc + j] = red[0];
        __syncthreads();
    }
}

__global__ void k_head_reduce(const float *part, int nb, int maxc, int C, float *loss, float *db, float *dw, long long N)
{
    const int j = threadIdx.x;
    if (j >= C + 2) return;
    float s = 0.0f;
    for (int b = 0; b < nb; b++) s += part[(long long)b * maxc + j];
    if (j == 0) loss[0] = s / (float)N;
    else if (j == 1) db[0] = s;
    else dw[j - 2] = s;
}

// Adam on FP32 master weights; bf16 copies for the convolutions
__global__ void k_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t *pb)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gg = g[t];
    m[t] = b1 * m[t] + (1.0f - b1) * gg;
    v[t] = b2 * v[t] + (1.0f - b2) * gg * gg;
    p[t] -= lr * (m[t] / c1) / (sqrtf(v[t] / c2) + eps);
    if (pb) pb[t] = f2bf(p[t]);
}

__global__ void k_f32_to_bf16(const float *x, uint16_t *y, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = f2bf(x[t]);
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ==========================================================================
struct NetLayer {
    int IC, OC;
    float *w32 = nullptr, *b32 = nullptr, *gw = nullptr, *gb = nullptr;
    float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;
    uint16_t *wbf = nullptr, *wflip = nullptr;
};

struct mgseg_net {
    int base = 32, depth = 4;
    // enc[2l], enc[2l+1]: the two convolutions of encoder block l; dec[2l], dec[2l+1]: of decoder block l < depth-1
    std::vector<NetLayer> enc, dec;
    float *hw = nullptr, *hb = nullptr, *ghw = nullptr, *ghb = nullptr, *mhw = nullptr, *vhw = nullptr,
          *mhb = nullptr, *vhb = nullptr;
    // activations for the current (B, H, W)
    int B = 0, H = 0, W = 0;
    uint16_t *x0 = nullptr;                  // input, bf16
    std::vector<uint16_t *> emid, dmid;      // first convolution's output of encoder / decoder block l
    std::vector<uint16_t *> cat;             // cat[l]: [up(d_{l+1}) | e_l] at level l (l < depth-1)
    std::vector<uint16_t *> pool;            // pool[l] = avgpool(e_l), level l+1
    uint16_t *ebot = nullptr;                // e_{depth-1}
    std::vector<uint16_t *> dact;            // d_l (l < depth-1)
    float *d0f = nullptr, *ob = nullptr, *phi = nullptr;   // FP32 d_0, head output o, M tanh(o)
    // gradients
    std::vector<uint16_t *> gemid, gdmid, gcat, gpool, gdact;
    uint16_t *gebot = nullptr;
    float *part = nullptr, *partb = nullptr, *hpart = nullptr, *loss = nullptr;
    std::vector<void *> act_allocs, par_allocs;
    int steps = 0;
};

namespace {

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

bool ensure_acts(mgseg_net *n, int B, int H, int W)
{
    if (n->B == B && n->H == H && n->W == W) return true;
    free_acts(n);
    bool fail = false;
    auto &v = n->act_allocs;
    const int D = n->depth;
    n->x0 = nalloc<uint16_t>(v, (size_t)B * 3 * H * W, fail);
    for (int l = 0; l < D; l++) {
        const size_t hw = (size_t)(H >> l) * (W >> l);
        const int ce = chan(n, l);
        n->emid.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw, fail));
        n->gemid.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw, fail));
        if (l == D - 1) break;
        const int cu = chan(n, l + 1);
        n->cat.push_back(nalloc<uint16_t>(v, (size_t)B * (cu + ce) * hw, fail));
        n->gcat.push_back(nalloc<uint16_t>(v, (size_t)B * (cu + ce) * hw, fail));
        const size_t hw1 = (size_t)(H >> (l + 1)) * (W >> (l + 1));
        n->pool.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw1, fail));
        n->gpool.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw1, fail));
        n->dmid.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw, fail));
        n->gdmid.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw, fail));
        n->dact.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw, fail));
        n->gdact.push_back(nalloc<uint16_t>(v, (size_t)B * ce * hw, fail));
    }
    const size_t hwb = (size_t)(H >> (D - 1)) * (W >> (D - 1));
    n->ebot = nalloc<uint16_t>(v, (size_t)B * chan(n, D - 1) * hwb, fail);
    n->gebot = nalloc<uint16_t>(v, (size_t)B * chan(n, D - 1) * hwb, fail);
    n->d0f = nalloc<float>(v, (size_t)B * chan(n, 0) * H * W, fail);
    n->ob = nalloc<float>(v, (size_t)B * H * W, fail);
    n->phi = nalloc<float>(v, (size_t)B * H * W, fail);
    // weight-gradient partials: chunks of 4096 pixels, the largest convolution of any level
    long long need = 0, needb = 0;
    auto acc_need = [&](int IC, int OC, long long NP) {
        const long long ch = (NP + 4095) / 4096;
        need = std::max(need, ch * OC * IC * 9LL);
        needb = std::max(needb, ch * OC);
    };
    for (int l = 0; l < D; l++) {
        const long long NP = (long long)B * (H >> l) * (W >> l);
        acc_need(l == 0 ? 3 : chan(n, l - 1), chan(n, l), NP);
        acc_need(chan(n, l), chan(n, l), NP);
        if (l < D - 1) acc_need(chan(n, l + 1) + chan(n, l), chan(n, l), NP);
    }
    n->part = nalloc<float>(v, (size_t)need, fail);
    n->partb = nalloc<float>(v, (size_t)needb, fail);
    n->hpart = nalloc<float>(v, (size_t)nblk((long long)B * H * W) * (chan(n, 0) + 2), fail);
    n->loss = nalloc<float>(v, 4, fail);
    if (fail) { free_acts(n); return false; }
    n->B = B; n->H = H; n->W = W;
    return true;
}

void conv(hipStream_t s, const uint16_t *in, long long ibs, const uint16_t *W, const float *bias, int IC, int OC,
          uint16_t *out, long long obs, int H, int Wd, int B, int relu, float *out32 = nullptr, long long o32bs = 0)
{
    ConvArgs A;
    A.in = in; A.ibs = ibs; A.W = W; A.K = IC * 9; A.bias = bias; A.out = out; A.obs = obs;
    A.out32 = out32; A.o32bs = o32bs; A.IC = IC; A.OC = OC; A.H = H; A.Wd = Wd; A.B = B; A.relu = relu;
    const long long NP = (long long)B * H * Wd;
    dim3 g((unsigned)((NP + 31) / 32), (unsigned)((OC + 31) / 32));
    hipLaunchKernelGGL(k_conv3x3, g, dim3(256), 0, s, A);
}

void wgrad(mgseg_net *n, hipStream_t s, const uint16_t *g, long long gbs, const uint16_t *x, long long xbs, int IC,
           int OC, int H, int Wd, int B, float *dW, float *db)
{
    WgradArgs A;
    A.g = g; A.gbs = gbs; A.x = x; A.xbs = xbs; A.part = n->part; A.partb = n->partb;
    A.IC = IC; A.OC = OC; A.H = H; A.Wd = Wd; A.B = B; A.chunk = 4096;
    const long long NP = (long long)B * H * Wd;
    const int nch = (int)((NP + 4095) / 4096);
    const int K = IC * 9;
    dim3 gr((unsigned)nch, (unsigned)((OC + 15) / 16), (unsigned)((K + 63) / 64));
    hipLaunchKernelGGL(k_wgrad, gr, dim3(256), 0, s, A);
    const long long tot = (long long)OC * K + OC;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk(tot)), dim3(256), 0, s, n->part, n->partb, nch, OC, K, dW, db);
}

void dgrad(hipStream_t s, NetLayer &L, const uint16_t *g, long long gbs, uint16_t *gx, long long gxbs, int H, int Wd,
           int B)
{
    hipLaunchKernelGGL(k_flip_weights, dim3(nblk((long long)L.IC * L.OC * 9)), dim3(256), 0, s, L.wbf, L.IC, L.OC,
                       L.wflip);
    conv(s, g, gbs, L.wflip, nullptr, L.OC, L.IC, gx, gxbs, H, Wd, B, 0);
}

void relu_mask(hipStream_t s, uint16_t *g, long long gbs, const uint16_t *y, long long ybs, int C, long long hw, int B)
{
    hipLaunchKernelGGL(k_relu_mask, dim3(nblk((long long)B * C * hw)), dim3(256), 0, s, g, gbs, y, ybs, C, (int)hw, B);
}

// forward of one block: mid = relu(conv_a(x)), y = relu(conv_b(mid))
void block_fwd(hipStream_t s, NetLayer &a, NetLayer &b, const uint16_t *x, long long xbs, uint16_t *mid, uint16_t *y,
               long long ybs, int h, int w, int B, float *y32 = nullptr)
{
    const long long hw = (long long)h * w;
    conv(s, x, xbs, a.wbf, a.b32, a.IC, a.OC, mid, (long long)a.OC * hw, h, w, B, 1);
    conv(s, mid, (long long)a.OC * hw, b.wbf, b.b32, b.IC, b.OC, y, ybs, h, w, B, 1, y32, (long long)b.OC * hw);
}

// backward of one block: gy (gradient of y, overwritten) -> weight gradients and, when gx is set, the gradient of x
void block_bwd(mgseg_net *n, hipStream_t s, NetLayer &a, NetLayer &b, const uint16_t *x, long long xbs,
               const uint16_t *mid, uint16_t *gmid, const uint16_t *y, uint16_t *gy, long long ybs, uint16_t *gx, int h,
               int w, int B)
{
    const long long hw = (long long)h * w, mbs = (long long)a.OC * hw;
    relu_mask(s, gy, ybs, y, ybs, b.OC, hw, B);
    wgrad(n, s, gy, ybs, mid, mbs, b.IC, b.OC, h, w, B, b.gw, b.gb);
    dgrad(s, b, gy, ybs, gmid, mbs, h, w, B);
    relu_mask(s, gmid, mbs, mid, mbs, a.OC, hw, B);
    wgrad(n, s, gmid, mbs, x, xbs, a.IC, a.OC, h, w, B, a.gw, a.gb);
    if (gx) dgrad(s, a, gmid, mbs, gx, xbs, h, w, B);
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

bool make_layer(mgseg_net *n, NetLayer &L, int IC, int OC, Rng &rng)
{
    bool fail = false;
    auto &v = n->par_allocs;
    const size_t nw = (size_t)OC * IC * 9;
    L.IC = IC; L.OC = OC;
    L.w32 = nalloc<float>(v, nw, fail); L.b32 = nalloc<float>(v, OC, fail);
    L.gw = nalloc<float>(v, nw, fail); L.gb = nalloc<float>(v, OC, fail);
    L.mw = nalloc<float>(v, nw, fail); L.vw = nalloc<float>(v, nw, fail);
    L.mb = nalloc<float>(v, OC, fail); L.vb = nalloc<float>(v, OC, fail);
    L.wbf = nalloc<uint16_t>(v, nw, fail); L.wflip = nalloc<uint16_t>(v, nw, fail);
    if (fail) return false;
    std::vector<float> w(nw);
    const double sd = std::sqrt(2.0 / (9.0 * IC));
    for (auto &x : w) x = (float)(sd * rng.normal());
    (void)hipMemcpy(L.w32, w.data(), nw * sizeof(float), hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(nblk((long long)nw)), dim3(256), 0, 0, L.w32, L.wbf, (long long)nw);
    return true;
}

// parameters in a fixed order: the convolutions enc[0..2D-1], then dec[0..2D-3], each w (OC*IC*9) then b (OC);
// head w (C0), head b (1)
template <class F>
void for_params(mgseg_net *n, F f)
{
    for (auto *v : {&n->enc, &n->dec})
        for (auto &L : *v) {
            f(L.w32, L.gw, L.mw, L.vw, L.wbf, (long long)L.OC * L.IC * 9);
            f(L.b32, L.gb, L.mb, L.vb, (uint16_t *)nullptr, (long long)L.OC);
        }
    f(n->hw, n->ghw, n->mhw, n->vhw, (uint16_t *)nullptr, (long long)chan(n, 0));
    f(n->hb, n->ghb, n->mhb, n->vhb, (uint16_t *)nullptr, 1LL);
}

}  // namespace

extern "C" {

void mgseg_net_destroy(mgseg_net *n)
{
    if (!n) return;
    free_acts(n);
    for (void *p : n->par_allocs) (void)hipFree(p);
    delete n;
}

mgseg_status mgseg_net_create(int base_channels, int depth, uint64_t seed, mgseg_net **out)
{
    if (!out) return MGSEG_E_ARG;
    *out = nullptr;
    if (base_channels < 1 || base_channels > 256 || depth < 2 || depth > 6) return MGSEG_E_ARG;
    mgseg_net *n = new (std::nothrow) mgseg_net();
    if (!n) return MGSEG_E_NOMEM;
    n->base = base_channels; n->depth = depth;
    Rng rng{seed};
    n->enc.resize(2 * depth);
    n->dec.resize(2 * (depth - 1));
    bool ok = true;
    for (int l = 0; l < depth && ok; l++) {
        ok = make_layer(n, n->enc[2 * l], l == 0 ? 3 : chan(n, l - 1), chan(n, l), rng);
        if (ok) ok = make_layer(n, n->enc[2 * l + 1], chan(n, l), chan(n, l), rng);
    }
    for (int l = 0; l < depth - 1 && ok; l++) {
        ok = make_layer(n, n->dec[2 * l], chan(n, l + 1) + chan(n, l), chan(n, l), rng);
        if (ok) ok = make_layer(n, n->dec[2 * l + 1], chan(n, l), chan(n, l), rng);
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
    const long long HW0 = (long long)H * W;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk((long long)B * 3 * HW0)), dim3(256), 0, s, in_dev, n->x0,
                       (long long)B * 3 * HW0);
    // encoder
    const uint16_t *cur = n->x0;
    long long curbs = 3 * HW0;
    for (int l = 0; l < D; l++) {
        const int h = H >> l, w = W >> l, ce = chan(n, l);
        const long long hw = (long long)h * w;
        uint16_t *outp;
        long long obs;
        if (l < D - 1) {
            const int cu = chan(n, l + 1);
            outp = n->cat[l] + (long long)cu * hw;     // e_l in the skip slice of cat[l]
            obs = (long long)(cu + ce) * hw;
        } else {
            outp = n->ebot;
            obs = (long long)ce * hw;
        }
        block_fwd(s, n->enc[2 * l], n->enc[2 * l + 1], cur, curbs, n->emid[l], outp, obs, h, w, B);
        if (l < D - 1) {
            hipLaunchKernelGGL(k_avgpool, dim3(nblk((long long)B * ce * hw / 4)), dim3(256), 0, s, outp, obs,
                               n->pool[l], (long long)ce * hw / 4, ce, h, w, B);
            cur = n->pool[l];
            curbs = (long long)ce * hw / 4;
        }
    }
    // decoder
    const uint16_t *dn = n->ebot;
    long long dnbs = (long long)chan(n, D - 1) * (H >> (D - 1)) * (W >> (D - 1));
    for (int l = D - 2; l >= 0; l--) {
        const int h = H >> l, w = W >> l;
        const long long hw = (long long)h * w;
        const int cu = chan(n, l + 1), ce = chan(n, l);
        const long long cbs = (long long)(cu + ce) * hw;
        hipLaunchKernelGGL(k_upsample, dim3(nblk((long long)B * cu * hw)), dim3(256), 0, s, dn, dnbs, n->cat[l], cbs,
                           cu, h / 2, w / 2, B);
        block_fwd(s, n->dec[2 * l], n->dec[2 * l + 1], n->cat[l], cbs, n->dmid[l], n->dact[l], (long long)ce * hw, h,
                  w, B, l == 0 ? n->d0f : nullptr);
        dn = n->dact[l];
        dnbs = (long long)ce * hw;
    }
    hipLaunchKernelGGL(k_head, dim3(nblk((long long)B * HW0)), dim3(256), 0, s, n->d0f, chan(n, 0), (int)HW0, B, n->hw,
                       n->hb, (float)M, n->ob, phi0_dev ? phi0_dev : n->phi);
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
    const long long HW0 = (long long)H * W;
    const unsigned nb = nblk((long long)B * HW0);
    const int maxc = C0 + 2;
    // head and loss; gradient of d_0 -> gdact[0]
    hipLaunchKernelGGL(k_head_bwd, dim3(nb), dim3(256), 0, s, n->ob, target_dev, (float)M, (float)pos_weight, n->d0f,
                       C0, (int)HW0, B,
                       n->hw, n->gdact[0], n->hpart, maxc);
    hipLaunchKernelGGL(k_head_reduce, dim3(1), dim3(256), 0, s, n->hpart, (int)nb, maxc, C0, n->loss, n->ghb, n->ghw,
                       (long long)B * HW0);
    // decoder, level 0 first
    for (int l = 0; l <= D - 2; l++) {
        const int h = H >> l, w = W >> l;
        const long long hw = (long long)h * w;
        const int cu = chan(n, l + 1), ce = chan(n, l);
        const long long cbs = (long long)(cu + ce) * hw;
        block_bwd(n, s, n->dec[2 * l], n->dec[2 * l + 1], n->cat[l], cbs, n->dmid[l], n->gdmid[l], n->dact[l],
                  n->gdact[l], (long long)ce * hw, n->gcat[l], h, w, B);
        // up-sampled part of the input -> gradient of the level below's d (or of e_bottom)
        uint16_t *gdn = (l + 1 <= D - 2) ? n->gdact[l + 1] : n->gebot;
        hipLaunchKernelGGL(k_upsample_bwd, dim3(nblk((long long)B * cu * hw / 4)), dim3(256), 0, s, n->gcat[l], cbs,
                           gdn, (long long)cu * hw / 4, cu, h / 2, w / 2, B);
    }
    // encoder, bottom up
    for (int l = D - 1; l >= 0; l--) {
        const int h = H >> l, w = W >> l, ce = chan(n, l);
        const long long hw = (long long)h * w;
        uint16_t *g, *y;
        long long gbs;
        if (l == D - 1) {
            g = n->gebot; y = n->ebot; gbs = (long long)ce * hw;
        } else {
            const int cu = chan(n, l + 1);
            gbs = (long long)(cu + ce) * hw;
            g = n->gcat[l] + (long long)cu * hw; y = n->cat[l] + (long long)cu * hw;
            // pooled path: g_e += avgpool^T(g_pool)
            hipLaunchKernelGGL(k_avgpool_bwd, dim3(nblk((long long)B * ce * hw)), dim3(256), 0, s, n->gpool[l],
                               (long long)ce * hw / 4, g, gbs, ce, h, w, B);
        }
        const uint16_t *x = l == 0 ? n->x0 : n->pool[l - 1];
        const long long xbs = l == 0 ? 3 * hw : (long long)chan(n, l - 1) * hw;
        block_bwd(n, s, n->enc[2 * l], n->enc[2 * l + 1], x, xbs, n->emid[l], n->gemid[l], y, g, gbs,
                  l > 0 ? n->gpool[l - 1] : nullptr, h, w, B);
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
    for_params(n, [&](float *p, float *g, float *m, float *v, uint16_t *pb, long long cnt) {
        hipLaunchKernelGGL(k_adam, dim3(nblk(cnt)), dim3(256), 0, s, p, g, m, v, cnt, (float)lr, (float)b1, (float)b2,
                           (float)eps, c1, c2, pb);
    });
    return hipGetLastError() == hipSuccess ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_param_count(mgseg_net *n, long long *count)
{
    if (!n || !count) return MGSEG_E_ARG;
    long long c = 0;
    for_params(n, [&](float *, float *, float *, float *, uint16_t *, long long k) { c += k; });
    *count = c;
    return MGSEG_OK;
}

mgseg_status mgseg_net_get_params(mgseg_net *n, float *host, float *grad_host)
{
    if (!n || (!host && !grad_host)) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    long long off = 0;
    bool ok = true;
    for_params(n, [&](float *p, float *g, float *, float *, uint16_t *, long long k) {
        if (host) ok &= hipMemcpy(host + off, p, k * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
        if (grad_host) ok &= hipMemcpy(grad_host + off, g, k * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
        off += k;
    });
    return ok ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_net_set_params(mgseg_net *n, const float *host)
{
    if (!n || !host) return MGSEG_E_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return MGSEG_E_HIP;
    long long off = 0;
    bool ok = true;
    for_params(n, [&](float *p, float *, float *m, float *v, uint16_t *pb, long long k) {
        ok &= hipMemcpy(p, host + off, k * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        ok &= hipMemset(m, 0, k * sizeof(float)) == hipSuccess && hipMemset(v, 0, k * sizeof(float)) == hipSuccess;
        if (pb) hipLaunchKernelGGL(k_f32_to_bf16, dim3(nblk(k)), dim3(256), 0, 0, p, pb, k);
        off += k;
    });
    n->steps = 0;
    return ok && hipDeviceSynchronize() == hipSuccess ? MGSEG_OK : MGSEG_E_HIP;
}

}  // extern "C"
