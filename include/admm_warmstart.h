/*
 * admm_warmstart.h — C ABI of the learned warm start (BF16 MFMA kernels, gfx950).
 *
 * Not part of the paper's method: a 6-layer 3x3 CNN predicts an initial image
 * x0 and a TV dual field p0 that set the ADMM state through admm_warmstart_map
 * (include/admm_deconv.h). By Theorem 1 of the paper any initial state
 * converges to a solution, so the network changes the iteration count, never
 * the minimiser.
 *
 * Conventions:
 *  - Activations are NHWC bf16 (stored as uint16_t) with C in {8, 16, 32}
 *    channels; all tensors are DEVICE memory and contiguous.
 *  - Weights of a layer are FP32 masters w[9][cout][cin] (tap = 3 ky + kx,
 *    cross-correlation: out[r][c] uses in[r + ky - 1][c + kx - 1]); the kernels
 *    consume packed bf16 copies made by admm_conv3x3_pack_weights.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = null stream) and is
 *    asynchronous; the caller synchronises.
 *  - Return ADMM_OK, ADMM_E_INVALID (null pointer, bad size) or
 *    ADMM_E_UNSUPPORTED (channel count), ADMM_E_DEVICE on a launch failure.
 */
#ifndef ADMM_WARMSTART_H
#define ADMM_WARMSTART_H

#include <stddef.h>
#include <stdint.h>

#include "admm_deconv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Pack w[9][cout][cin] (FP32, cin, cout <= 32) into the forward operand layout
 * wfwd (9 * 32 * 32 bf16 capacity) and, if wbwd is not NULL, the input-gradient
 * layout wbwd (same capacity: spatially flipped, channels transposed).          */
admm_status admm_conv3x3_pack_weights(const float* w, int32_t cin, int32_t cout, uint16_t* wfwd,
                                      uint16_t* wbwd, void* stream);

/* y = act(conv3x3_d(x, w) + bias), act = ReLU if relu != 0; if gate is not
 * NULL the result is zeroed wherever gate <= 0 (gate has cout channels).
 * conv3x3_d: taps at offsets dilation * (-1, 0, 1) in rows and columns, zero
 * padding; dilation in 1..8 (else ADMM_E_INVALID).
 * x: [N][H][W][cin], cin in {8,16,32}; y: [N][H][W][cout], cout in {16,32};
 * wpacked from admm_conv3x3_pack_weights (forward layout for a forward
 * convolution; the input-gradient layout, with cin/cout swapped and the same
 * dilation, computes dL/dx from dL/dy); bias: FP32 [cout] or NULL.            */
admm_status admm_conv3x3_bf16_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t cin,
                                  const uint16_t* wpacked, const float* bias, int32_t cout, int32_t relu,
                                  const uint16_t* gate, uint16_t* y, int32_t dilation, void* stream);

/* Workspace bytes for admm_conv3x3_bf16_wgrad with the given pixel chunk.     */
size_t admm_conv3x3_bf16_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t cin, int32_t cout,
                                         int32_t chunk);

/* dw[9][cout][cin] = sum_p dy[p][cout] x[p + dilation off(tap)][cin] and
 * db = sum_p dy (FP32 outputs, overwritten; dilation in 1..8). Split over pixel
 * chunks of `chunk` (multiple of 32) with a fixed-order second pass:
 * deterministic.                                                              */
admm_status admm_conv3x3_bf16_wgrad(const uint16_t* x, const uint16_t* dy, int32_t N, int32_t H, int32_t W,
                                    int32_t cin, int32_t cout, int32_t chunk, float* workspace, size_t ws_bytes,
                                    float* dw, float* db, int32_t dilation, void* stream);

/* One Adam step (Kingma & Ba) at step t >= 1 on n FP32 parameters.          */
admm_status admm_adam_step(float* p, const float* g, float* m, float* v, int32_t n, float lr, float beta1,
                           float beta2, float eps, int32_t t, void* stream);

/* Network input x0: [N][H][W][8] bf16 = [m y, m, e0, e1, e2, e3, 0, 0] from
 * y [N][H][W] FP32, mask [N][H][W] uint8 and a per-image kernel embedding
 * emb [N][4] FP32.                                                            */
admm_status admm_ws_input(const float* y, const uint8_t* mask, const float* emb, int32_t N, int32_t H,
                          int32_t W, uint16_t* x0, void* stream);

/* Training loss of the network output out [N][H][W][16] (channels 0..2 used):
 * x0 = m y + out0, p0 = (out1, out2); L = mean over pixels of
 * (x0 - xt)^2 + alpha |p0 - pt|^2 with xt [N][H][W], pt [N][2][H][W].
 * Writes dL/dout (bf16, 16 channels) and one partial sum of L per 256 pixels
 * to lpart (ceil(N H W / 256) floats; their sum is L).                         */
admm_status admm_ws_loss(const uint16_t* out, const float* y, const uint8_t* mask, const float* xt,
                         const float* pt, int32_t N, int32_t H, int32_t W, float alpha, uint16_t* dout,
                         float* lpart, void* stream);

/* Network output -> warm-start guess x0 [N][H][W] and p0 [N][2][H][W] (FP32). */
admm_status admm_ws_output(const uint16_t* out, const float* y, const uint8_t* mask, int32_t N, int32_t H,
                           int32_t W, float* x0, float* p0, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ADMM_WARMSTART_H */
