// conv_bf16.hip — BF16 MFMA kernels of the warm-start network (gfx950).
//
// The warm start is not part of the paper: a small CNN predicts an initial
// image x0 and TV dual field p0, which only set u_0, d_0 (Theorem 1 allows any).
// Layers are 3x3 convolutions with dilation d (1 <= d <= 8), stride 1, zero
// padding, NHWC bf16 activations, FP32 accumulation on v_mfma_f32_16x16x32_bf16:
//
//   out[p][m] = bias[m] + sum_{tap, k} in[p + d off(tap)][k] * W[tap][m][k],
//   off(tap) = (tap / 3 - 1, tap % 3 - 1)
//
// as an implicit GEMM with M = output channels (16 per tile), N = 16 pixels
// of a row, K = taps x input channels packed 32 at a time (CIN = 32: one tap
// per K step; CIN = 16: two; CIN = 8: four). Operand layout of the MFMA (one
// wave): lane l supplies A[m = l % 16][k = 8 (l / 16) .. +7] and
// B[k = 8 (l / 16) .. +7][n = l % 16]; it receives D[m = 4 (l / 16) .. +3][n = l % 16].
// A lane's B operand is therefore 8 consecutive channels of one pixel (16 B of
// NHWC memory) and its result 4 consecutive channels of one pixel (8 B).
//
// dgrad is the same kernel applied to dY with weights flipped in space and
// transposed in channels (W'[8 - tap][k][m] = W[tap][m][k]); its epilogue
// multiplies by (x > 0), the derivative of the ReLU that produced the layer
// input x. wgrad reduces dW[tap][m][k] = sum_p dY[p][m] x[p + d off(tap)][k] over
// pixel chunks (split K) with LDS transposes, then a fixed-order second pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace admm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CW = 4;             // waves per block
constexpr int PIX_PER_WAVE = 64;  // 4 N tiles of 16 pixels along a row
constexpr int DIL_MAX = 8;        // largest dilation (the wgrad input tile's halo)

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

// Packed A-operand weights: wA[ks][m (MT*16)][32] bf16 (see host packer).
// x: [N][H][W][CIN], y: [N][H][W][MT*16], gate (optional): [N][H][W][MT*16].
template <int CIN, int MT>
__global__ __launch_bounds__(CW * 64) void k_conv3x3(const __bf16* __restrict__ x, const __bf16* __restrict__ wA,
                                                     const float* __restrict__ bias, const __bf16* __restrict__ gate,
                                                     __bf16* __restrict__ y, int N, int H, int W, int relu,
                                                     int dil) {
    constexpr int TPK = 32 / CIN;                 // taps per K step
    constexpr int KS = (9 + TPK - 1) / TPK;       // K steps
    constexpr int COUT = MT * 16;
    __shared__ bf16x8 wl[KS * MT * 16 * 4];       // A operands of every K step, per lane slot
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // stage weights: KS * MT * 16 rows of 32 bf16 = 4 bf16x8 each
    const bf16x8* wv = reinterpret_cast<const bf16x8*>(wA);
    for (int i = tid; i < KS * MT * 16 * 4; i += CW * 64) wl[i] = wv[i];
    __syncthreads();

    const int segs = (W + PIX_PER_WAVE - 1) / PIX_PER_WAVE;
    const long long job = (long long)blockIdx.x * CW + wave;    // one row segment per wave
    if (job >= (long long)N * H * segs) return;
    const int seg = (int)(job % segs);
    const long long nr = job / segs;
    const int r = (int)(nr % H), n = (int)(nr / H);
    const int c0 = seg * PIX_PER_WAVE;
    const int g = lane >> 4, col = lane & 15;

    f32x4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int s = 0; s < KS; ++s) {
        // which tap / channel group this lane feeds at K step s
        const int tap = s * TPK + g / (CIN / 8);
        const int ch0 = (g % (CIN / 8)) * 8;
        const int dy = (tap / 3 - 1) * dil, dx = (tap % 3 - 1) * dil;
        const int rr = r + dy;
        const bool rowok = tap < 9 && rr >= 0 && rr < H;
        bf16x8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = wl[((s * MT + mt) * 16 + col) * 4 + g];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int cc = c0 + t * 16 + col + dx;
            bf16x8 b = zero8();
            if (rowok && cc >= 0 && cc < W)
                b = *reinterpret_cast<const bf16x8*>(x + (((long long)n * H + rr) * W + cc) * CIN + ch0);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[mt][t], 0, 0, 0);
        }
    }
    // epilogue: lane holds channels m = mt*16 + 4g .. +3 of pixel c0 + 16t + col
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = c0 + t * 16 + col;
        if (c >= W) continue;
        const long long pix = ((long long)n * H + r) * W + c;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int m0 = mt * 16 + 4 * g;
            bf16x4 o;
            bf16x4 gt;
            if (gate) gt = *reinterpret_cast<const bf16x4*>(gate + pix * COUT + m0);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = acc[mt][t][j] + (bias ? bias[m0 + j] : 0.0f);
                if (relu) v = fmaxf(v, 0.0f);
                if (gate && !((float)gt[j] > 0.0f)) v = 0.0f;
                o[j] = (__bf16)v;
            }
            *reinterpret_cast<bf16x4*>(y + pix * COUT + m0) = o;
        }
    }
}

// wgrad partials: block b reduces dY^T x over `chunk` consecutive pixels of the
// flattened [N][H][W] range for every tap; out[b][tap][m][k] (FP32), dbias[b][m].
// Wave w owns taps w, w + 4, w + 8.
template <int CIN, int MT>
__global__ __launch_bounds__(CW * 64) void k_wgrad_part(const __bf16* __restrict__ x, const __bf16* __restrict__ dy,
                                                        float* __restrict__ part, float* __restrict__ dbpart, int N,
                                                        int H, int W, int chunk, int dil) {
    constexpr int COUT = MT * 16;
    constexpr int KT = CIN / 16 > 0 ? CIN / 16 : 1;      // k tiles of 16 channels (CIN 8 uses one, half empty)
    constexpr int PX = 32;                               // pixels per K step
    constexpr int PXW = PX + 2 * DIL_MAX;               // pixels of an input row with its halo
    // transposed tiles: dyT[m][px], xT[3 rows (r - d, r, r + d)][k][px], px = column - cb + d
    __shared__ __bf16 dyT[COUT][PX];
    __shared__ __bf16 xT[3][KT * 16][PXW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    const long long npx = (long long)N * H * W;
    const long long p0 = (long long)blockIdx.x * chunk;
    f32x4 acc[3][MT][KT];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) acc[q][mt][kt] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.0f;

    const long long pend = min(p0 + (long long)chunk, npx);
    for (long long pb = p0; pb < pend;) {
        // a K step never straddles a row or the chunk end; missing pixels are zero
        const long long nr = pb / W;
        const int cb = (int)(pb - nr * W);
        const int r = (int)(nr % H), n = (int)(nr / H);
        const int valid = (int)min((long long)min(PX, W - cb), pend - pb);
        __syncthreads();
        for (int i = tid; i < COUT * PX; i += CW * 64) {
            const int m = i / PX, px = i - (i / PX) * PX;
            const long long pp = pb + px;
            __bf16 v = (__bf16)0.0f;
            if (px < valid) v = dy[pp * COUT + m];
            dyT[m][px] = v;
        }
        for (int i = tid; i < 3 * KT * 16 * PXW; i += CW * 64) {
            const int row = i / (KT * 16 * PXW);
            const int rem = i - row * (KT * 16 * PXW);
            const int k = rem / PXW, px = rem - (rem / PXW) * PXW;
            const int rr = r + (row - 1) * dil, cc = cb + px - dil;
            __bf16 v = (__bf16)0.0f;
            if (k < CIN && rr >= 0 && rr < H && cc >= 0 && cc < W && px < valid + 2 * dil)
                v = x[(((long long)n * H + rr) * W + cc) * CIN + k];
            xT[row][k][px] = v;
        }
        __syncthreads();
        if (tid < COUT) {
            float s = 0.f;
            for (int px = 0; px < PX; ++px) s += (float)dyT[tid][px];
            dbacc += s;
        }
        // A operand: dY^T rows m, 8 consecutive pixels 8g..8g+7 (K = pixels)
        bf16x8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[mt][j] = dyT[mt * 16 + col][8 * g + j];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int tap = wave + 4 * q;
            if (tap >= 9) continue;
            const int dyo = tap / 3, dxo = (tap % 3) * dil;     // row index into xT, pixel shift 0, d, 2d
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = xT[dyo][kt * 16 + col][8 * g + j + dxo];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[q][mt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[q][mt][kt], 0, 0, 0);
            }
        }
        pb += valid;
    }
    // D[m = mt*16 + 4g + j][k = kt*16 + col]
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int tap = wave + 4 * q;
        if (tap >= 9) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m = mt * 16 + 4 * g + j, k = kt * 16 + col;
                    if (k < CIN)
                        part[(((long long)blockIdx.x * 9 + tap) * COUT + m) * CIN + k] = acc[q][mt][kt][j];
                }
    }
    if (tid < COUT) dbpart[(long long)blockIdx.x * COUT + tid] = dbacc;
}

// Fixed-order sum of the block partials: dw[i] = sum_b part[b][i], db likewise.
__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ dbpart, float* __restrict__ dw,
                               float* __restrict__ db, int nblk, int nw, int cout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part[(long long)b * nw + i];
        dw[i] = s;
    }
    if (i < cout) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += dbpart[(long long)b * cout + i];
        db[i] = s;
    }
}

// Pack FP32 master weights w[9][cout][cin] into the forward A layout
// wf[ks][MT*16][32] and the dgrad A layout wb[ks'][MT'*16][32] where the
// dgrad convolution has cin' = cout, cout' = cin, W'[8 - tap][k][m] = W[tap][m][k].
__global__ void k_pack_weights(const float* __restrict__ w, int cin, int cout, int cin_p, int cout_p,
                               __bf16* __restrict__ wf, __bf16* __restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // forward: cin_p in {8,16,32} channels per tap, rows cout_p
    const int tpk = 32 / cin_p, ks = (9 + tpk - 1) / tpk;
    const int nf = ks * cout_p * 32;
    if (i < nf) {
        const int s = i / (cout_p * 32), rem = i % (cout_p * 32), m = rem / 32, k = rem % 32;
        const int tap = s * tpk + k / cin_p, ci = k % cin_p;
        float v = 0.f;
        if (tap < 9 && m < cout && ci < cin) v = w[(tap * cout + m) * cin + ci];
        wf[i] = (__bf16)v;
    }
    // backward: input channels cout_p (dY), output rows cin_p' = max(16, cin padded)
    const int bin = cout_p, bout = cin_p < 16 ? 16 : cin_p;
    const int tpkb = 32 / bin, ksb = (9 + tpkb - 1) / tpkb;
    const int nb = ksb * bout * 32;
    if (wb && i < nb) {
        const int s = i / (bout * 32), rem = i % (bout * 32), m = rem / 32, k = rem % 32;
        const int tap = s * tpkb + k / bin, co = k % bin;
        float v = 0.f;
        if (tap < 9 && m < cin && co < cout) v = w[((8 - tap) * cout + co) * cin + m];
        wb[i] = (__bf16)v;
    }
}

// Adam (Kingma & Ba) on FP32 master parameters, bias-corrected at step t.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Network input, NHWC bf16 with 8 channels: [m y, m, e0, e1, e2, e3, 0, 0]
// (y zero-filled off the mask, the mask, and a 4-number kernel embedding).
__global__ void k_ws_input(const float* __restrict__ y, const uint8_t* __restrict__ mask,
                           const float* __restrict__ emb, int N, int H, int W, __bf16* __restrict__ x0) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n_px = (long long)N * H * W;
    if (i >= n_px) return;
    const int n = (int)(i / ((long long)H * W));
    const float m = mask[i] ? 1.0f : 0.0f;
    bf16x8 v;
    v[0] = (__bf16)(m * y[i]);
    v[1] = (__bf16)m;
    v[2] = (__bf16)emb[n * 4 + 0];
    v[3] = (__bf16)emb[n * 4 + 1];
    v[4] = (__bf16)emb[n * 4 + 2];
    v[5] = (__bf16)emb[n * 4 + 3];
    v[6] = (__bf16)0.0f;
    v[7] = (__bf16)0.0f;
    *reinterpret_cast<bf16x8*>(x0 + i * 8) = v;
}

// Loss L = (1/npx) sum [ (x0 - x*)^2 + alpha |p0 - p*|^2 ] with x0 = m y + out0,
// p0 = (out1, out2); writes dL/dout (16 channels, zero beyond 3) and per-block sums.
__global__ void k_ws_loss(const __bf16* __restrict__ out, const float* __restrict__ y, const uint8_t* __restrict__ mask,
                          const float* __restrict__ xt, const float* __restrict__ pt, int N, int H, int W, float alpha,
                          __bf16* __restrict__ dout, float* __restrict__ lpart) {
    __shared__ float red[256];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long hw = (long long)H * W, n_px = (long long)N * hw;
    float l = 0.f;
    if (i < n_px) {
        const long long n = i / hw, q = i - n * hw;
        const float m = mask[i] ? 1.0f : 0.0f;
        const float o0 = (float)out[i * 16 + 0], o1 = (float)out[i * 16 + 1], o2 = (float)out[i * 16 + 2];
        const float e0 = m * y[i] + o0 - xt[i];
        const float e1 = o1 - pt[(n * 2 + 0) * hw + q], e2 = o2 - pt[(n * 2 + 1) * hw + q];
        l = e0 * e0 + alpha * (e1 * e1 + e2 * e2);
        const float sc = 2.0f / (float)n_px;
        bf16x8 g0, g1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            g0[j] = (__bf16)0.0f;
            g1[j] = (__bf16)0.0f;
        }
        g0[0] = (__bf16)(sc * e0);
        g0[1] = (__bf16)(sc * alpha * e1);
        g0[2] = (__bf16)(sc * alpha * e2);
        *reinterpret_cast<bf16x8*>(dout + i * 16) = g0;
        *reinterpret_cast<bf16x8*>(dout + i * 16 + 8) = g1;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] / (float)n_px;
}

// Network output -> warm-start guess: x0 = m y + out0, p0 = (out1, out2).
__global__ void k_ws_output(const __bf16* __restrict__ out, const float* __restrict__ y,
                            const uint8_t* __restrict__ mask, int N, int H, int W, float* __restrict__ x0,
                            float* __restrict__ p0) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long hw = (long long)H * W, n_px = (long long)N * hw;
    if (i >= n_px) return;
    const long long n = i / hw, q = i - n * hw;
    x0[i] = (mask[i] ? y[i] : 0.0f) + (float)out[i * 16 + 0];
    p0[(n * 2 + 0) * hw + q] = (float)out[i * 16 + 1];
    p0[(n * 2 + 1) * hw + q] = (float)out[i * 16 + 2];
}

}  // namespace admm

using namespace admm;

#include "../../include/admm_warmstart.h"

extern "C" admm_status admm_conv3x3_bf16_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t cin,
                                             const uint16_t* wpacked, const float* bias, int32_t cout,
                                             int32_t relu, const uint16_t* gate, uint16_t* y, int32_t dilation,
                                             void* stream) {
    if (!x || !wpacked || !y || N < 1 || H < 1 || W < 1 || dilation < 1 || dilation > DIL_MAX) return ADMM_E_INVALID;
    if (!(cin == 8 || cin == 16 || cin == 32) || !(cout == 16 || cout == 32)) return ADMM_E_UNSUPPORTED;
    const long long jobs = (long long)N * H * ((W + PIX_PER_WAVE - 1) / PIX_PER_WAVE);
    const dim3 grid((unsigned)((jobs + CW - 1) / CW)), blk(CW * 64);
    hipStream_t s = (hipStream_t)stream;
    const __bf16* xb = (const __bf16*)x;
    const __bf16* wb = (const __bf16*)wpacked;
    const __bf16* gb = (const __bf16*)gate;
    __bf16* yb = (__bf16*)y;
#define CONV_CASE(CI, MTV) \
    if (cin == CI && cout == MTV * 16) hipLaunchKernelGGL((k_conv3x3<CI, MTV>), grid, blk, 0, s, xb, wb, bias, gb, yb, N, H, W, relu, dilation);
    CONV_CASE(8, 1) CONV_CASE(8, 2) CONV_CASE(16, 1) CONV_CASE(16, 2) CONV_CASE(32, 1) CONV_CASE(32, 2)
#undef CONV_CASE
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}

extern "C" size_t admm_conv3x3_bf16_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t cin, int32_t cout,
                                                    int32_t chunk) {
    const long long npx = (long long)N * H * W;
    const long long nblk = (npx + chunk - 1) / chunk;
    return (size_t)nblk * (9 * cout * cin + cout) * sizeof(float);
}

extern "C" admm_status admm_conv3x3_bf16_wgrad(const uint16_t* x, const uint16_t* dy, int32_t N, int32_t H, int32_t W,
                                               int32_t cin, int32_t cout, int32_t chunk, float* workspace,
                                               size_t ws_bytes, float* dw, float* db, int32_t dilation, void* stream) {
    if (!x || !dy || !dw || !db || !workspace || N < 1 || H < 1 || W < 1 || chunk < 32 || chunk % 32 ||
        dilation < 1 || dilation > DIL_MAX)
        return ADMM_E_INVALID;
    if (!(cin == 8 || cin == 16 || cin == 32) || !(cout == 16 || cout == 32)) return ADMM_E_UNSUPPORTED;
    if (ws_bytes < admm_conv3x3_bf16_wgrad_workspace(N, H, W, cin, cout, chunk)) return ADMM_E_INVALID;
    const long long npx = (long long)N * H * W;
    const int nblk = (int)((npx + chunk - 1) / chunk);
    hipStream_t s = (hipStream_t)stream;
    float* part = workspace;
    float* dbp = workspace + (size_t)nblk * 9 * cout * cin;
    const __bf16* xb = (const __bf16*)x;
    const __bf16* dyb = (const __bf16*)dy;
#define WG_CASE(CI, MTV) \
    if (cin == CI && cout == MTV * 16) hipLaunchKernelGGL((k_wgrad_part<CI, MTV>), dim3(nblk), dim3(CW * 64), 0, s, xb, dyb, part, dbp, N, H, W, chunk, dilation);
    WG_CASE(8, 1) WG_CASE(8, 2) WG_CASE(16, 1) WG_CASE(16, 2) WG_CASE(32, 1) WG_CASE(32, 2)
#undef WG_CASE
    const int nw = 9 * cout * cin;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((nw + 255) / 256), dim3(256), 0, s, part, dbp, dw, db, nblk, nw, cout);
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}

extern "C" admm_status admm_conv3x3_pack_weights(const float* w, int32_t cin, int32_t cout, uint16_t* wfwd,
                                                 uint16_t* wbwd, void* stream) {
    if (!w || !wfwd || cin < 1 || cin > 32 || cout < 1 || cout > 32) return ADMM_E_INVALID;
    const int cin_p = cin <= 8 ? 8 : (cin <= 16 ? 16 : 32);
    const int cout_p = cout <= 16 ? 16 : 32;
    const int n = 5 * 32 * 32 + 9 * 32 * 32;   // covers both layouts
    hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, w, cin, cout, cin_p,
                       cout_p, (__bf16*)wfwd, (__bf16*)wbwd);
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}

extern "C" admm_status admm_adam_step(float* p, const float* g, float* m, float* v, int32_t n, float lr, float beta1,
                                      float beta2, float eps, int32_t t, void* stream) {
    if (!p || !g || !m || !v || n < 0 || t < 1) return ADMM_E_INVALID;
    if (n == 0) return ADMM_OK;
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr, beta1,
                       beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}

extern "C" admm_status admm_ws_input(const float* y, const uint8_t* mask, const float* emb, int32_t N, int32_t H,
                                     int32_t W, uint16_t* x0, void* stream) {
    if (!y || !mask || !emb || !x0 || N < 1 || H < 1 || W < 1) return ADMM_E_INVALID;
    const long long n = (long long)N * H * W;
    hipLaunchKernelGGL(k_ws_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, y, mask, emb,
                       N, H, W, (__bf16*)x0);
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}

extern "C" admm_status admm_ws_loss(const uint16_t* out, const float* y, const uint8_t* mask, const float* xt,
                                    const float* pt, int32_t N, int32_t H, int32_t W, float alpha, uint16_t* dout,
                                    float* lpart, void* stream) {
    if (!out || !y || !mask || !xt || !pt || !dout || !lpart || N < 1 || H < 1 || W < 1) return ADMM_E_INVALID;
    const long long n = (long long)N * H * W;
    hipLaunchKernelGGL(k_ws_loss, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (const __bf16*)out, y, mask, xt, pt, N, H, W, alpha, (__bf16*)dout, lpart);
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}

extern "C" admm_status admm_ws_output(const uint16_t* out, const float* y, const uint8_t* mask, int32_t N, int32_t H,
                                      int32_t W, float* x0, float* p0, void* stream) {
    if (!out || !y || !mask || !x0 || !p0 || N < 1 || H < 1 || W < 1) return ADMM_E_INVALID;
    const long long n = (long long)N * H * W;
    hipLaunchKernelGGL(k_ws_output, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (const __bf16*)out, y, mask, N, H, W, x0, p0);
    return hipGetLastError() == hipSuccess ? ADMM_OK : ADMM_E_DEVICE;
}
