/*
 * fd_batch.h -- many acoustic shots with uneven apertures advanced together.
 *
 * A full-waveform-inversion gradient sums, over shots, the zero-lag imaging
 * condition of each shot's adjoint wavefield against its forward wavefield
 * (the FWI/RTM use of the propagators named in the paper's "Anisotropic
 * acoustic" section; the propagator itself is equation (acou) of appendix
 * "Isotropic acoustic").  Each shot runs on its own aperture: a sub-box of
 * the full model with its own damping layer and zero halo.
 *
 * All shots advance in lock-step: one work-list kernel launch per time step
 * covers every (shot, tile) pair, so uneven apertures share the GPU.  The
 * whole schedule of one gradient -- forward with checkpoints every
 * ckpt_every steps, per-segment recomputation, adjoint with the fused
 * imaging condition, the ordered sum into the full-model gradient and the
 * velocity chain rule -- is captured once into a hipGraph and replayed by a
 * single graph launch per call.
 *
 * Conventions are those of fd.h (status codes, fd_last_error, streams,
 * caller-owned inputs/outputs).  The batch owns its working memory: per
 * shot two forward and two adjoint fields, the coefficient field, 2 *
 * ceil(nt / ckpt_every) checkpoint fields, ckpt_every + 2 recomputation
 * slots and a gradient accumulator, all in the padded layout of fd.h.  It
 * is allocated by fd_batch_create; fd_batch_gradient allocates nothing after
 * its first call with a given set of pointers (which instantiates the graph).
 */
#ifndef FD_BATCH_H
#define FD_BATCH_H

#include "fd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fd_batch fd_batch;

/* common: spacing, space_order, nbl, dt, vmax, device (shape, physics and
 * boundary are ignored: acoustic, zero halo).  shapes[s] and origins[s] are
 * the (z, y, x) extent and origin of shot s's aperture inside the full model
 * of extent full_shape; every aperture must lie inside it.  FD_EUNSTABLE as
 * for fd_create_grid; FD_ENOMEM if the working memory does not fit. */
int fd_batch_create(const fd_grid_desc *common, int nshots, const int64_t *shapes,
                    const int64_t *origins, const int64_t *full_shape, int nt, int ckpt_every,
                    fd_batch **out);

void fd_batch_destroy(fd_batch *b);

/* Device bytes held by the batch. */
size_t fd_batch_device_bytes(const fd_batch *b);

/* Sources and receivers of shot s: host coordinates in metres from the
 * aperture's DOMAIN index 0 ([n][3]); prepared (FP64) and uploaded. */
int fd_batch_set_geometry(fd_batch *b, int shot, const double *src_m, int ns,
                          const double *rec_m, int nr);

/* Full-model velocity vel_full_dev (dense full_shape, m/s): each aperture's
 * v^2 dt^2 is extracted from it.  The pointer is kept for the chain rule of
 * fd_batch_gradient and must stay valid.  Synchronises `stream`;
 * FD_EUNSTABLE if max(v) > vmax. */
int fd_batch_set_model(fd_batch *b, const float *vel_full_dev, void *stream);

/* One gradient of J = 1/2 sum_s |d_s - dobs_s|^2 with respect to velocity
 * (forward with checkpoints; per segment the recomputation, whose steps
 * also store the imaging factor (u+ - 2u + u-)/dt^2 + gamma (u+ - u-)/(2 dt)
 * of each update -- for the last segment the forward steps store it, and
 * that segment is not recomputed -- and the adjoint steps, which apply the
 * imaging condition g -= lambda D to the adjoint field they read).
 *   q_dev[s]     [nt][ns_s] source signatures
 *   dobs_dev[s]  [nt][nr_s] observed traces
 *   d_dev[s]     [nt][nr_s] output: modelled traces
 *   grad_v_dev   full_shape dense output, overwritten: dJ/dv (zero outside
 *                every aperture); per point, the shots' contributions are
 *                added in shot order (deterministic)
 * The first call with a given set of pointers captures and instantiates the
 * schedule's graph; later calls with the same pointers replay it. */
int fd_batch_gradient(fd_batch *b, const float *const *q_dev, const float *const *dobs_dev,
                      float *const *d_dev, float *grad_v_dev, void *stream);

/* Apply a tile and flags (see fd_set_tile, 128-wide tiles included) to the
 * batched step kernel; invalidates the captured graph.  Every batched step
 * runs the buffer-addressed halo-ring body, so flags 1 (XCD remap), 4
 * (non-temporal hints) and 16 (128-wide tiles) matter and 2 and 8 do not.
 * The default is (8, 2, 32) with flags 12 (the tile the autotuner picks
 * for the 16-shot gradient). */
int fd_batch_set_tile(fd_batch *b, int by, int ry, int nzb, int flags);

/* Autotuner of the batched step (the paper's problem-setup section tunes
 * loop blocking per run): a timed search over tile shapes (by, ry), z
 * chunks of 16, 32 or 64 planes and flag sets (halo ring; with non-temporal
 * hints; 128-wide with hints; XCD remap with hints), each candidate
 * one launch of the batched step over every shot's aperture on the batch's
 * own forward fields (which the next gradient zeroes); the fastest is
 * applied with fd_batch_set_tile (so the next gradient captures its graph
 * with it).  With cache_path non-NULL the choice is first looked up in that
 * JSON file under "arch|batch|so|nshots|<hash of the aperture shapes>" and
 * stored on a miss.  out4 (may be NULL) receives (by, ry, nzb, flags);
 * ms_out (may be NULL) the best milliseconds per launch (0 on a cache hit).
 * Needs a loaded model; synchronises `stream`; allocates nothing.  The
 * first error of any candidate ends the search: its code is returned, the
 * batch keeps its tile and nothing is cached. */
int fd_batch_autotune(fd_batch *b, const char *cache_path, int *out4, double *ms_out,
                      void *stream);

/* The batched step's current tile (by, ry, nzb, flags) into out4. */
int fd_batch_get_tile(const fd_batch *b, int *out4);

#ifdef __cplusplus
}
#endif

#endif /* FD_BATCH_H */
