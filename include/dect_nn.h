/*
 * dect_nn.h -- C ABI of the BF16 MFMA network kernels (gfx950) used by the
 * learned warm start: a U-Net that maps an early ADM-TV iterate to a late
 * one, trained and run with these kernels.  Not part of the paper's method;
 * plain ADM-TV (dect_adm_tv) continues from the network's output and stays
 * the judge of its error.
 *
 * Conventions: activations NHWC [N][H][W][C] bfloat16 (stored as uint16 bit
 * patterns), FP32 accumulation on the matrix cores.  Convolution weights are
 * [taps][CoutP][Cin] bfloat16 with taps = ksize^2 in row-major (dy, dx)
 * order, CoutP = Cout rounded up to 16 (extra rows zero); biases FP32
 * [CoutP].  Cin must be a multiple of 8; Cin and Cout are at most 256.  All pointers are device memory owned by the caller; every call
 * is asynchronous on `stream` (a hipStream_t, NULL = null stream) and
 * returns a dect_status (dect_nn_last_error gives the message).
 */
#ifndef DECT_NN_H
#define DECT_NN_H

#include <stddef.h>
#include <stdint.h>

#include "dect.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv(x, w) + bias), 'same' zero padding, stride 1.  ksize 1 or 3;
 * relu 0/1; out_f32 1 writes FP32 output, else bfloat16.  bias may be NULL.
 * Also serves as the input-gradient convolution when given weights from
 * dect_nn_weight_flip. */
dect_status dect_nn_conv_fwd(const void *x, const void *w, const float *bias, void *y, int32_t N,
                             int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                             int32_t relu, int32_t out_f32, void *stream);

/* dect_nn_conv_fwd with a ReLU's backward fused into the output: y = 0
 * where mask <= 0 (mask [N][H][W][Cout] bfloat16, 16-byte aligned: the
 * output of the ReLU that fed the layer whose input gradient this is).
 * Bit for bit dect_nn_relu_bwd(dect_nn_conv_fwd(...), mask). */
dect_status dect_nn_conv_fwd_masked(const void *x, const void *w, const float *bias,
                                    const void *mask, void *y, int32_t N, int32_t H, int32_t W,
                                    int32_t Cin, int32_t Cout, int32_t ksize, int32_t relu,
                                    int32_t out_f32, void *stream);

/* Weights of the input-gradient convolution: wd[tap'][CinP][Cout] =
 * w[taps-1-tap'][co][ci] (CinP = Cin rounded up to 16, extra rows zero). */
dect_status dect_nn_weight_flip(const void *w, void *wd, int32_t Cin, int32_t Cout, int32_t ksize,
                                void *stream);

/* Weight and bias gradients of a convolution: dw [taps][CoutP][Cin] FP32 =
 * sum over pixels of dz (x) shifted x; db [CoutP] FP32 = sum of dz.  dz is
 * the gradient at the convolution output (after the activation's backward).
 * Partial sums per pixel chunk go to `workspace` (dect_nn_wgrad_workspace
 * bytes) and are summed in chunk order: results are deterministic. */
size_t dect_nn_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                               int32_t ksize);
dect_status dect_nn_conv_wgrad(const void *dz, const void *x, float *dw, float *db, int32_t N,
                               int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                               void *workspace, size_t ws_bytes, void *stream);

/* dz = dy where y > 0 else 0 (bfloat16, n elements). */
dect_status dect_nn_relu_bwd(const void *dy, const void *y, void *dz, size_t n, void *stream);

/* 2x2 max pool with stride 2 (H, W even).  Forward: x [N][H][W][C] -> y
 * [N][H/2][W/2][C] and idx (uint8, same size as y: winning sub-pixel).
 * Backward (backward = 1): x = dy (pooled size), y = dx (full size). */
dect_status dect_nn_pool(const void *x, void *y, void *idx, int32_t N, int32_t H, int32_t W,
                         int32_t C, int32_t backward, void *stream);

/* Depth-to-space: dst[n][2i+a][2j+b][c] = src[n][i][j][(2a+b)C + c]
 * (inverse = 1: the reverse map).  With a 1x1 convolution to 4C channels this
 * is a 2x2 stride-2 transposed convolution. */
dect_status dect_nn_shuffle(const void *src, void *dst, int32_t N, int32_t Hin, int32_t Win,
                            int32_t C, int32_t inverse, void *stream);

/* Channel concat z[p] = (a[p], b[p]) over P pixels; inverse = 1 splits z. */
dect_status dect_nn_concat(void *a, void *b, void *z, size_t P, int32_t C1, int32_t C2,
                           int32_t inverse, void *stream);

/* Depth-to-space of t followed by the channel concat with s, in one pass (the
 * decoder's upsampled input joined to its skip connection):
 * z[n][h][w] = (shuffle(t)[n][h][w], s[n][h][w]), t [N][Hin][Win][4 C1], s
 * [N][2 Hin][2 Win][C2], z [N][2 Hin][2 Win][C1 + C2] (bfloat16, device
 * memory owned by the caller).  inverse = 1 splits z into t (the inverse
 * shuffle of z's first C1 channels) and s.  Element for element the same as
 * dect_nn_shuffle then dect_nn_concat (or dect_nn_concat's split then the
 * inverse shuffle).  C1, C2 positive multiples of 8 and 16-byte aligned
 * pointers, else DECT_ERR_INVALID_ARG. */
dect_status dect_nn_shuffle_concat(void *t, void *s, void *z, int32_t N, int32_t Hin, int32_t Win,
                                   int32_t C1, int32_t C2, int32_t inverse, void *stream);

/* z = a + b (bfloat16, n elements, FP32 arithmetic). */
dect_status dect_nn_add(const void *a, const void *b, void *z, size_t n, void *stream);

/* z = bf16(a + b) where y > 0, else 0 (bfloat16, n elements): the gradient
 * of a sum that feeds a ReLU's backward, bit for bit dect_nn_relu_bwd(
 * dect_nn_add(a, b), y). */
dect_status dect_nn_add_relu_bwd(const void *a, const void *b, const void *y, void *z, size_t n,
                                 void *stream);

/* FP32 <-> bfloat16 (round to nearest even). */
dect_status dect_nn_convert(const void *src, void *dst, size_t n, int32_t to_bf16, void *stream);

/* Adam step on FP32 master weights w with moments m, v and gradient g;
 * w_bf16 (may be NULL) receives the rounded working copy.  step >= 1. */
dect_status dect_nn_adam(float *w, float *m, float *v, const float *g, void *w_bf16, size_t n,
                         double lr, double beta1, double beta2, double eps, int32_t step,
                         double weight_decay, void *stream);

/* Mean squared error of the first `used` of C channels of y [P][C] against
 * t [P][used]: per-block partial sums into partial (dect_nn_mse_partials
 * doubles; sum them in order) and, if dy != NULL, dy = d(mean)/dy. */
size_t dect_nn_mse_partials(size_t P, int32_t C);
dect_status dect_nn_mse(const float *y, const float *t, float *dy, double *partial, size_t P,
                        int32_t C, int32_t used, void *stream);

const char *dect_nn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DECT_NN_H */
