// Internal declarations of the batched multi-shot gradient (fd_batch.hip,
// k_batch.hip).
#pragma once

#include "fd_internal.h"
#include "../../include/fd_batch.h"

namespace fd {

// Field slots inside one shot's workspace (each a padded field of the shot).
enum : int {
    kFA = 0,       // forward state, buffer A
    kFB = 1,       // forward state, buffer B
    kLA = 2,       // adjoint state, buffer A
    kLB = 3,       // adjoint state, buffer B
    kVdt2 = 4,     // v^2 dt^2
    kGrad = 5,     // imaging accumulator (DOMAIN part used)
    kCkpt0 = 6     // 2 * nck checkpoints, then ckpt_every + 2 slots
};

// One shot as the kernels see it (device table, one entry per shot).
struct BatchShot {
    StepParams p;
    float *base;            // workspace: field f at base + f * stride
    int64_t stride;         // elements per padded field
    int ntx, nty, nzc;      // tiles of the batched step kernel
    int block0;             // first logical block of this shot
    int org[3];             // aperture origin in the full model (z, y, x)
    int ns, nr;
    const int32_t *sbase;
    const float *sfrac;
    const int32_t *rbase;
    const float *rfrac;
    const float *q;         // [nt][ns]
    const float *dobs;      // [nt][nr]
    float *d;               // [nt][nr]
};

// What a batched step does besides the update (workspace field slots):
// mode 0 nothing; mode 1 (recomputed forward step) writes the imaging factor
// D of its update to field fd; mode 2 (adjoint step) applies the imaging
// condition g -= lambda D to field fg, with lambda its input field and D
// read from field fd.
struct BatchEpi {
    int mode = 0;
    int fd = 0, fg = 0;
    float inv_dt2 = 0.0f, inv_2dt = 0.0f;
};

// batched z-marching step for stencil radius R (k_step_radius.hip)
template <int R>
int launch_batch_radius(const BatchShot *shots_dev, int nshots, int total_blocks,
                        const Tuning &t, int iu, int ium, int iup, const BatchEpi &e,
                        hipStream_t s);

// launchers (k_batch.hip)
int launch_batch_step(const BatchShot *shots_dev, int nshots, int total_blocks, int r,
                      const Tuning &t, int iu, int ium, int iup, hipStream_t s,
                      const BatchEpi &e = BatchEpi{});
// mode 0: inject sources q[n] into field f and sample receivers into d[n]
// mode 1: inject sources q[n] into field f only, and when fd >= 0 add the
//         injected amounts' share of the imaging factor (times
//         inv_dt2 + gamma inv_2dt) to field fd
// mode 2: inject residuals d[n] - dobs[n] at the receivers into field f
int launch_batch_sparse(const BatchShot *shots_dev, int nshots, int mode, int n, int f,
                        float hinv, hipStream_t s, int fd = -1, float inv_dt2 = 0.0f,
                        float inv_2dt = 0.0f);
int launch_batch_copy(const BatchShot *shots_dev, int nshots, int64_t max_stride, int fsrc,
                      int fdst, hipStream_t s);
int launch_batch_zero(const BatchShot *shots_dev, int nshots, int64_t max_stride, int f,
                      hipStream_t s);
int launch_batch_imaging(const BatchShot *shots_dev, int nshots, int64_t max_rows, int flam,
                         int fup, int fu, int fum, float inv_dt2, float inv_2dt, hipStream_t s);
// g -= lambda D with a stored imaging factor D (field fd)
int launch_batch_imaging_d(const BatchShot *shots_dev, int nshots, int64_t max_rows, int flam,
                           int fd, hipStream_t s);
int launch_batch_reduce(const BatchShot *shots_dev, int nshots, const int64_t full[3],
                        const float *vel_full, float *grad_v, hipStream_t s);
int launch_batch_vdt2(const BatchShot *shots_dev, int nshots, int64_t max_pts,
                      const int64_t full[3], const float *vel_full, float dt2,
                      unsigned *vmax_bits, hipStream_t s);

}  // namespace fd
