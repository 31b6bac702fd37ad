/*
 * das_learn.h -- C ABI of the learned-compounding kernels (gfx950).
 *
 * Not an operation of the paper: this project's growth direction that maps
 * delay-and-sum volumes beamformed from a few plane waves to an approximation
 * of the many-angle compound (the paper's Sec. 2.1 notes that compounding
 * multiplies the beamforming cost; Sec. 3.4 notes that beamformed output can
 * stay on the GPU for machine-learning inference).  The network is a 3D U-Net
 * trained with these kernels; the full delay-and-sum stays the reference.
 *
 * Conventions
 *   - Volumes are channels-last [D][H][W][C] (voxel-major, channel innermost).
 *     A tensor argument may be a channel slice of a wider buffer: row stride
 *     `*_stride` channels, first channel `*_coff`.
 *   - Activations and weights are bfloat16 (passed as void*); accumulation,
 *     biases, gradients of weights, optimiser state and losses are float32.
 *   - Convolutions are 3 x 3 x 3, stride 1, zero padding ("same"); weights are
 *     [Cout][27][Cin] with tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1).
 *   - All pointers are device memory unless stated; every call enqueues on
 *     `stream` (hipStream_t as void*) and allocates nothing.
 *   - Return 0 (DAS_OK) or a negative das_status from das.h; the message of
 *     the last failure on this thread is das_learn_last_error().
 */
#ifndef DAS_LEARN_H
#define DAS_LEARN_H

#include <stdint.h>

#include "das.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[v][out_coff + n] = act(sum_{tap,c} in[v + s*off(tap)][in_coff + c] * w[n][tap][c] + bias[n]) * m
 * on BF16 MFMA (16x16x32) with FP32 accumulation.  s = +1, or -1 with flip
 * (the input gradient of a convolution when w is the transposed weight from
 * das_transpose_weights).  act = ReLU when relu != 0.  m = (mask[v][mask_coff
 * + n] > 0) when mask is not NULL, else 1.  bias may be NULL.  out is float32
 * when out_f32 != 0, else bfloat16.  Cin a multiple of 8 (in_stride, in_coff
 * too; in and w 16-byte aligned), Cout a multiple of 16, at most 128. */
int das_conv3d(const void *in, int in_stride, int in_coff, const void *weight, const float *bias, void *out,
               int out_stride, int out_coff, int out_f32, const void *mask, int mask_stride, int mask_coff,
               int D, int H, int W, int cin, int cout, int flip, int relu, void *stream);

/* Weight and bias gradients of the (unflipped) convolution:
 *   dw[n][tap][c] = sum_v dy[v][n] * in[v + off(tap)][c],  db[n] = sum_v dy[v][n]
 * (float32 outputs, MFMA with FP32 accumulation) split over voxel chunks of
 * `chunk` voxels (a multiple of 32) whose partial sums are added in a fixed
 * order (parts r, r + 8, ... for r < 8, then the 8 sums in order: deterministic).  `work` holds das_conv3d_wgrad_work(...) floats.  Cin a
 * multiple of 8, Cout of 16; strides and channel offsets of in and dy multiples
 * of 8, both 16-byte aligned; fewer than 2^31 voxels. */
int das_conv3d_wgrad(const void *in, int in_stride, int in_coff, const void *dy, int dy_stride, int dy_coff,
                     float *dw, float *db, float *work, int64_t work_floats, int D, int H, int W, int cin,
                     int cout, int chunk, void *stream);

/* Floats of work space das_conv3d_wgrad needs (host call). */
int64_t das_conv3d_wgrad_work(int D, int H, int W, int cin, int cout, int chunk);

/* wt[ci][tap][co] = w[co][tap][ci] (bfloat16). */
int das_transpose_weights(const void *w, void *wt, int cin, int cout, void *stream);

/* 2x average pooling to a Do x Ho x Wo output (the input is 2Do x 2Ho x 2Wo),
 * and its gradient for a Di x Hi x Wi input (all even): each of the 8 inputs
 * receives 1/8 of its output's gradient, added to gin when accumulate.
 * DAS_ESHAPE for empty or odd sizes and channel slices outside their buffers. */
int das_avgpool2(const void *in, int in_stride, int in_coff, void *out, int out_stride, int out_coff,
                 int Do, int Ho, int Wo, int c, void *stream);
int das_avgpool2_bwd(const void *gout, int gout_stride, int gout_coff, void *gin, int gin_stride, int gin_coff,
                     int Di, int Hi, int Wi, int c, int accumulate, void *stream);

/* 2x nearest upsampling to a Do x Ho x Wo output (all even), and its gradient
 * for a Di x Hi x Wi input: the sum over the 8 outputs of each input, times
 * (mask > 0) when mask is not NULL.  DAS_ESHAPE as for pooling. */
int das_upsample2(const void *in, int in_stride, int in_coff, void *out, int out_stride, int out_coff,
                  int Do, int Ho, int Wo, int c, void *stream);
int das_upsample2_bwd(const void *gout, int gout_stride, int gout_coff, void *gin, int gin_stride, int gin_coff,
                      const void *mask, int mask_stride, int mask_coff, int Di, int Hi, int Wi, int c,
                      void *stream);

/* g = (a + b) * (mask > 0 when mask is not NULL), bfloat16 slices of V voxels x c channels. */
int das_add_mask(const void *a, int a_stride, int a_coff, const void *b, int b_stride, int b_coff,
                 const void *mask, int m_stride, int m_coff, void *g, int g_stride, int g_coff, int64_t V, int c,
                 void *stream);

/* Residual prediction pred = base + net[:, 0:2] (float32 [V][2]), squared
 * error against target [V][2]: loss_parts[b] = sum over block b (256 voxels)
 * of the squared errors (the mean is their sum / (2V)); grad (bfloat16
 * [V][grad_stride], may be NULL) = d(mean)/d(net) in channels 0, 1 and 0 in
 * the others; pred may be NULL. */
int das_mse_residual(const float *net, int net_stride, const float *base, const float *target, int64_t V,
                     void *grad, int grad_stride, float *pred, float *loss_parts, void *stream);

/* Adam step `step` (from 1) with bias correction on float32 master weights w
 * (moments m, v); also writes the bfloat16 copy w_bf16 when not NULL. */
int das_adam(float *w, float *m, float *v, const float *g, void *w_bf16, int64_t n, float lr, float beta1,
             float beta2, float eps, int step, void *stream);

/* y = bfloat16(x), round to nearest even. */
int das_f32_to_bf16(const float *x, void *y, int64_t n, void *stream);

/* Inputs of the network from n_in beamformed volumes y (complex64 [n_in][V],
 * one plane wave each): rms = sqrt(mean_v |sum_a y_a[v]|^2) (the RMS of the
 * few-angle compound); x[v][2a], x[v][2a+1] = bfloat16(Re, Im of y_a[v] / rms)
 * and x[v][c] = 0 for 2 n_in <= c < cin (x is bfloat16 [V][cin]); base (float32
 * [V][2], may be NULL) = gain * sum_a y_a[v] / rms.  scale (device, 2 floats)
 * receives {rms, 1 / rms} (1 / rms = 0 when rms = 0).  work holds
 * das_compound_work(V) floats.  Sum of squares in float32 per 256 voxels,
 * then float64. */
int das_compound_features(const void *y, int n_in, int64_t V, float gain, void *x, int cin, float *base, float *work,
                          float *scale, void *stream);

/* Floats of work space das_compound_features needs (host call). */
int64_t das_compound_work(int64_t V);

/* out = y * (restore ? rms : 1 / rms) for complex64 [V] volumes and the scale of
 * das_compound_features: normalises a target, or returns a prediction to the
 * beamformer's units.  out may equal y. */
int das_compound_rescale(const void *y, int64_t V, const float *scale, int restore, void *out, void *stream);

/* out[v] = (base[v] + net[v][0:2]) * rms (complex64 [V]): the learned compound
 * in the beamformer's units; scale from das_compound_features. */
int das_compound_output(const float *net, int net_stride, const float *base, int64_t V, const float *scale, void *out,
                        void *stream);

/* Thread-local message of the last failing call of this header ("" if none). */
const char *das_learn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DAS_LEARN_H */
