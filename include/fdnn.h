/*
 * fdnn.h -- C ABI of the learned coarse-grid correction network (part of
 * libfd.so; not in the paper: it corrects a 2x-coarser low-order propagation
 * of the acoustic equation of the appendix "Isotropic acoustic" toward the
 * fine high-order one).
 *
 * Network: conv3x3x3(3->16) - GELU - conv3x3x3(16->16) - GELU -
 * conv3x3x3(16->1), cross-correlation with zero "same" padding, GELU in the
 * erf form.  BF16 weights and activations, FP32 accumulation on MFMA
 * (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam moments.
 *
 * Conventions as fd.h (status codes, fd_last_error, caller-owned device
 * memory, asynchronous on `stream`, no allocation in any call).
 *
 * Layouts:
 *   params  FP32, nn_param_count() values: w1[16][3][27], b1[16],
 *           w2[16][16][27], b2[16], w3[1][16][27], b3[1]; the tap index is
 *           dz*9 + dy*3 + dx (the kernel's offset along z, y, x, each 0..2).
 *   packed  nn_packed_bytes() bytes: BF16 MFMA fragments of every layer
 *           (forward and data-gradient), rebuilt by nn_pack_weights.
 *   act8 / act16  channels-last BF16 (uint16 bit patterns) [nz][ny][nx][C],
 *           C = 8 or 16 (unused channels are zero).
 *   FP32 fields are addressed through an nn_view: element (z, y, x) at
 *           offset + z*pitch_z + y*pitch_y + x (a dense array, or a libfd
 *           padded field with its fd_layout).
 */
#ifndef FDNN_H
#define FDNN_H

#include <stdint.h>

#include "fd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t offset, pitch_y, pitch_z;
} nn_view;

int64_t nn_param_count(void);
int64_t nn_packed_bytes(void);

/* Bytes of the workspace nn_wgrad needs for a volume of nz*ny*nx points. */
int64_t nn_wgrad_workspace_bytes(int nz, int ny, int nx);

/* params (FP32) -> packed BF16 fragments (round to nearest even). */
int nn_pack_weights(const float *params_dev, void *packed_dev, void *stream);

/* Half-open index box [lo, hi) in (z, y, x) order; points inside it are
 * excluded (see nn_conv_out, nn_mse).  An empty box excludes nothing. */
typedef struct nn_box {
    int lo[3];
    int hi[3];
} nn_box;

/* x[p] = (a[p] * sa, b[p] * sa, c3, 0, 0, 0, 0, 0) as BF16, with
 * sa = 1 / scale_dev[0] if scale_dev is non-NULL (else 1), and
 * c3 = c[p] * a[p] * sa if c_times_a is non-zero (the third channel then
 * vanishes wherever a does), c3 = c[p] otherwise. */
int nn_pack_input(int nz, int ny, int nx, const float *a, nn_view va, const float *b,
                  nn_view vb, const float *c, nn_view vc, int c_times_a, const float *scale_dev,
                  void *x8_dev, void *stream);

/* scale_dev[0] = sqrt(mean(u^2)) + 1e-30 over the volume; flag_dev[0] (may
 * be NULL) is set to 1 if any value is not finite, left unchanged otherwise.
 * scale_dev must hold nn_rms_scratch_floats() floats, 8-byte aligned (the
 * rest is scratch for per-block partial sums, reduced in a fixed order). */
int nn_rms(int nz, int ny, int nx, const float *u, nn_view vu, float *scale_dev,
           unsigned *flag_dev, void *stream);
int64_t nn_rms_scratch_floats(void);

/* Forward layer 1 or 2: act16 = GELU(conv(x) + b); z16 (pre-activation,
 * may be NULL) is kept for training.  layer 1 reads act8, layer 2 act16. */
int nn_conv_gelu(int layer, int nz, int ny, int nx, const void *x_dev, const void *packed_dev,
                 const float *params_dev, void *z16_dev, void *a16_dev, void *stream);

/* Layer 1 straight from the three input fields: the same act16 (and z16)
 * as nn_pack_input(nz, ny, nx, a, va, b, vb, c, vc, c_times_a, scale_dev,
 * x8) followed by nn_conv_gelu(1, ..., x8, ...), bitwise (the staging forms
 * each point's packed input with nn_pack_input's arithmetic and rounding),
 * without writing the packed input: for inference, where nothing else reads
 * it.  Arguments as in those two calls; the fields are read in place.  Each
 * view's plane (pitch_z floats, at most 2^31 bytes) must hold ny rows of
 * pitch_y >= nx points, else FD_EINVAL. */
int nn_conv_gelu_fields(int nz, int ny, int nx, const float *a, nn_view va, const float *b,
                        nn_view vb, const float *c, nn_view vc, int c_times_a,
                        const float *scale_dev, const void *packed_dev, const float *params_dev,
                        void *z16_dev, void *a16_dev, void *stream);

/* Forward layer 3 (16 -> 1): y = conv(a16) + b3.  If y_dense_dev is
 * non-NULL it receives y (dense [nz][ny][nx]); if out_dev is non-NULL,
 * out[vout] = base[vbase] + gain * s * y with s = scale_dev[0] (or 1 if
 * NULL), except inside `skip` (may be NULL) where out[vout] = base[vbase].
 * out may alias base (same element for every point). */
int nn_conv_out(int nz, int ny, int nx, const void *a16_dev, const void *packed_dev,
                const float *params_dev, float *y_dense_dev, const float *base_dev,
                nn_view vbase, float *out_dev, nn_view vout, const float *scale_dev,
                float gain, const nn_box *skip, void *stream);

/* MSE over the volume against the target t / (gain * s) (s = scale_dev[0],
 * or 1 if scale_dev is NULL), with points inside `skip` (may be NULL)
 * contributing zero: with m[p] = 0 inside skip and 1 elsewhere and N the
 * number of points, loss_dev[0] += sum(m (y - t/(gain s))^2) / N (float
 * atomics) and gy8[p] = (2 m (y - t/(gain s)) / N, 0, ..., 0) as BF16.
 * gain must be positive. */
int nn_mse(int nz, int ny, int nx, const float *y_dev, const float *t_dev,
           const float *scale_dev, float gain, const nn_box *skip, void *gy8_dev,
           float *loss_dev, void *stream);

/* Data gradient through layer 3 (gin = gy8) or layer 2 (gin = gz16),
 * multiplied by GELU'(z) of the previous layer: gz_out16 = (W^T * gin) .
 * GELU'(z16_prev). */
int nn_dgrad_gelu(int layer, int nz, int ny, int nx, const void *gin_dev,
                  const void *packed_dev, const void *z16_prev_dev, void *gz_out16_dev,
                  void *stream);

/* Weight and bias gradient of layer 1, 2 or 3 into the layer's slice of
 * grads_dev (same layout as params): overwritten, or added to the slice's
 * current values if accumulate is non-zero (a mini-batch summed one sample
 * at a time).  x = act8 (layer 1) or act16, g = gz16 (layers 1, 2) or gy8
 * (layer 3).  Per-block partial sums in workspace, then an ordered reduction
 * (deterministic). */
int nn_wgrad(int layer, int nz, int ny, int nx, const void *x_dev, const void *g_dev,
             void *workspace_dev, float *grads_dev, int accumulate, void *stream);

/* nn_wgrad without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving or training loops, harnesses that forbid hipMalloc.  Same
 * kernels, arguments and results as nn_wgrad (bit-identical), but the
 * per-block partial sums live in a static device array of the library,
 * 512 partials x 6,928 floats = 14.2 MB per GPU, taken when the library's
 * device code is loaded and held until the process ends.  Runs on the
 * current device (its scratch address is looked up once per device on the
 * first call).  FD_EINVAL if a launch would need more partial sums than the
 * array holds, or for bad arguments; nothing is allocated, no memset is
 * issued (every partial that is read is written first in the same call).
 * Calls that overlap on one GPU (different streams) share the array and
 * race: serialise them. */
int nn_wgrad_noalloc(int layer, int nz, int ny, int nx, const void *x_dev, const void *g_dev,
                     float *grads_dev, int accumulate, void *stream);

/* Adam (t is the 1-based step) on every weight, and on the biases too if
 * train_bias is non-zero; otherwise biases and their moments are left as
 * they are (a bias-free network keeps N(0) = 0). */
int nn_adam(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int t,
            float lr, float beta1, float beta2, float eps, int train_bias, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FDNN_H */
