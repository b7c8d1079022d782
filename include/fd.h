/*
 * fd.h -- C ABI of libfd, an MI355X (gfx950) explicit finite-difference
 * wave-propagation library.
 *
 * One handle describes one rank's subdomain: a DOMAIN of (z, y, x) points
 * with a read-only HALO of width r = space_order/2 around it (paper,
 * "Access alignment" and "Data regions" paragraphs).  The library advances
 * the second-order-in-time wave equation of the appendix "Isotropic
 * acoustic" (equation (acou)), or the pseudo-acoustic TTI system of
 * appendix "Anisotropic acoustic (TTI)", with a damping layer, sparse source
 * injection and receiver interpolation, and the six-face halo pack/unpack of
 * the "basic" exchange pattern (table "Summary of communication/computation
 * patterns").
 *
 * Conventions (all entry points):
 *   - Every function returns an int status: FD_OK (0) or a negative FD_E*
 *     code; none aborts or throws.  fd_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Pointers suffixed _dev are device (HBM) pointers owned by the caller.
 *     The library never frees caller memory, and fd_forward / fd_adjoint /
 *     fd_pack_halo / fd_unpack_halo allocate nothing.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued asynchronously; execution errors surface at the caller's
 *     stream synchronisation.  Argument errors are reported synchronously.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Axis order is (z, y, x) with x unit-stride.  A 2-D grid (ndim = 2)
 *     lists its extents as (z, x) in shape[0], shape[1]; it has no y halo.
 */
#ifndef FD_H
#define FD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FD_OK = 0,
    FD_EINVAL = -1,     /* bad argument (shape, order, pointer, sparse point outside) */
    FD_ENOMEM = -2,     /* device allocation failed (handle creation / set_model only) */
    FD_EDEVICE = -3,    /* HIP runtime / launch error */
    FD_EUNSTABLE = -4,  /* time step violates the leapfrog stability limit */
    FD_ENOTSUP = -5     /* valid request this build does not implement */
};

/* Physics of a handle:
 *   FD_ACOUSTIC  equation (acou), second order in time, state {u, u-};
 *   FD_TTI       the pseudo-acoustic TTI system (appendix "Anisotropic
 *                acoustic (TTI)"), state {p, p-, r, r-};
 *   FD_ELASTIC   the isotropic elastic velocity-stress system (appendix
 *                "Isotropic elastic", equation (elas1)), first order in
 *                time on a staggered grid, state of nine components
 *                {vx, vy, vz, txx, tyy, tzz, txy, txz, tyz} updated in place.
 *                Storage index (z, y, x) holds vx at x+1/2, vy at y+1/2,
 *                vz at z+1/2, the normal stresses at the node, txy at
 *                (y+1/2, x+1/2), txz at (z+1/2, x+1/2), tyz at (z+1/2, y+1/2).
 *                3-D only; FD_BC_ZERO or FD_BC_LOOPBACK.
 *   FD_VISCO     the visco-elastic system with one relaxation mechanism
 *                (appendix "Visco-elastic", equations (model-equations)),
 *                the staggered grid of FD_ELASTIC plus six memory variables
 *                {rxx, ryy, rzz, rxy, rxz, ryz} at their stresses' positions:
 *                fifteen components in place.  The memory forcing carries
 *                the factors (tau_e / tau_s - 1), so tau_e = tau_s gives the
 *                elastic system; the memory variables advance by explicit
 *                Euler (first order in time, undamped), then the stresses
 *                take them at the new time level.  3-D only; FD_BC_ZERO or
 *                FD_BC_LOOPBACK. */
enum { FD_ACOUSTIC = 0, FD_TTI = 1, FD_ELASTIC = 2, FD_VISCO = 3 };

/* How the halo of the propagated field is refreshed before every step:
 *   FD_BC_ZERO      never written: stays as the caller allocated it (zero);
 *   FD_BC_LOOPBACK  the rank is its own neighbour on a periodic topology:
 *                   all faces are packed into device buffers and unpacked
 *                   into the opposite face's halo every step (3-D, nx a
 *                   multiple of 32: each x halo is written as part of a
 *                   whole 128-byte line, so the row padding beyond it, x in
 *                   [-32, -halo) and [n + halo, n + 32), also receives
 *                   periodic images; nothing reads the padding);
 *   FD_BC_EXTERNAL  left as the caller filled it (one step per call, with
 *                   fd_pack_halo / fd_unpack_halo around it). */
enum { FD_BC_ZERO = 0, FD_BC_LOOPBACK = 1, FD_BC_EXTERNAL = 2 };

typedef struct fd_grid fd_grid;   /* opaque, library-owned */

typedef struct {
    int ndim;               /* 2 or 3 */
    int64_t shape[3];       /* DOMAIN points, (z, y, x) or (z, x) */
    double spacing[3];      /* metres, same order as shape */
    int space_order;        /* even, 2..16 (TTI: 4..12) */
    int nbl;                /* damping-layer width in points, inside DOMAIN; 0 = none */
    int physics;            /* FD_ACOUSTIC, FD_TTI, FD_ELASTIC or FD_VISCO */
    int boundary;           /* FD_BC_* */
    double dt;              /* seconds */
    double vmax;            /* upper bound of the velocity model (m/s; FD_ELASTIC:
                               of the P velocity; FD_VISCO: of the unrelaxed P
                               velocity vp sqrt(tau_ep / tau_s)); sets the damping
                               strength and the stability check */
    double eps_max;         /* TTI: upper bound of epsilon (stability check); else 0 */
    int device;             /* HIP device ordinal */
} fd_grid_desc;

/* Field layout in HBM, identical for every padded field of a handle.
 * Element (z, y, x) of DOMAIN lives at offset + z*pitch_z + y*pitch_y + x;
 * halo points use z, y, x in [-halo, 0) and [n, n + halo).  DOMAIN rows start
 * 128-byte aligned (x is padded on the left and right). */
typedef struct {
    int64_t padded[3];      /* allocated extent (z, y, x) in elements */
    int64_t pitch_y;        /* elements between rows */
    int64_t pitch_z;        /* elements between planes */
    int64_t offset;         /* element offset of DOMAIN point (0, 0, 0) */
    int halo;               /* r = space_order / 2 */
    int64_t field_elems;    /* floats per padded field */
    size_t field_bytes;
} fd_layout;

/* A set of sparse (off-grid) points prepared by fd_sparse_prepare and copied
 * to the device by the caller: base[n][ndim] int32 lower node index and
 * frac[n][ndim] fractional offset in [0, 1], axis order as `shape`. */
typedef struct {
    int n;
    const int32_t *base_dev;
    const float *frac_dev;
} fd_sparse;

/* Validate `desc`, compute the layout and FP32 stencil weights, and allocate
 * the handle's own device memory (model coefficients and, for
 * FD_BC_LOOPBACK, six face buffers).  Returns FD_EUNSTABLE if
 * vmax*dt/h exceeds the leapfrog stability limit of the space order
 * (FD_ELASTIC, FD_VISCO: vmax dt sqrt(sum 1/h^2) sum_k |c_k| <= 1 with c_k
 * the staggered first-derivative weights). */
int fd_create_grid(const fd_grid_desc *desc, fd_grid **out);

void fd_destroy_grid(fd_grid *g);

int fd_field_layout(const fd_grid *g, fd_layout *out);

/* Select the 3-D step kernel's tile: blocks of 64 x by threads, each thread
 * computing ry consecutive rows (tile 64 x by*ry points), nzb planes per
 * block.  flags (0..31): bit 0 remaps blocks so each XCD sweeps a
 * contiguous tile range, bit 1 keeps two planes of loads in flight instead
 * of one, bit 2 puts the non-temporal hint on the streamed fields (u-,
 * v^2 dt^2 loads with bit 3, u+ stores), bit 3 issues each plane's x/y halo
 * loads together with the neighbouring tiles' loads of that plane (kept in
 * registers until used; bit 1 is then ignored), bit 4 makes the tile 128
 * columns wide with two columns per lane (with bit 3 behaviour; only for
 * (by, ry) = (8,2) (4,2) (4,4)).  by = 0 selects the
 * one-thread-per-point kernel.  FD_TTI grids: by = 0 selects the
 * one-thread-per-point passes; otherwise flags 0 gives the two z-marching
 * passes on 64 x 16 tiles with nzb planes per block (six vector
 * intermediates through memory), and flag 32 the whole step in one
 * z-marching kernel (by = 16 for 32-wide tiles, ry = 2 for two tile columns
 * per thread up to space order 6); flags 0..63.
 * FD_ELASTIC grids: by = 0 selects the
 * one-thread-per-point passes, (by, ry) = (4, 2), (8, 1) or (8, 2) the
 * z-marching passes on 64 x (by ry) tiles with nzb planes per block ((8, 2)
 * the default, with the deepest of 256 .. 8 planes giving 1024 blocks;
 * flags are ignored).  FD_VISCO grids
 * take the same tiles for their velocity pass; their stress-memory pass is
 * one thread per point.  Supported (by, ry): (4,1) (4,2) (4,4) (4,8)
 * (8,2) (8,4) (2,8).  Results do not depend on the tile or flags (same
 * arithmetic per point).  A 3-D grid starts with (8, 2, nzb, 28), nzb the
 * largest of 128, 64, 32 giving 512 blocks ((8, 2, 128, 28) at 512^3);
 * failing that, flags 12 and the first of (by, ry) = (8, 2), (4, 2), (4, 1)
 * whose launch reaches 1024 blocks with nzb = 64, 32, 16 or 8 (else
 * (4, 1, 8, 12)). */
int fd_set_tile(fd_grid *g, int by, int ry, int nzb, int flags);

/* Exchange mode of the halo update around each step (paper, section on
 * computation/communication patterns: the "basic" and "full" patterns).
 *   FD_XCHG_BASIC  the exchange finishes before the step kernel starts
 *                  (the default).
 *   FD_XCHG_FULL   the exchange runs on a second stream of this handle while
 *                  the step kernel computes the CORE, the points whose
 *                  stencil reads no HALO (every index in [r, n - r)); after
 *                  it completes, the REMAINDER (two z slabs of whole planes,
 *                  two y slabs, two x faces, all r deep) is computed.  The
 *                  caller's stream waits for the exchange before any later
 *                  work, so the call stays stream-ordered.
 * Results are bit-identical in both modes.  Full mode needs a 3-D acoustic
 * grid with FD_BC_LOOPBACK, every extent > 2 r, and a z-marching tile
 * (by > 0); FD_ENOTSUP otherwise, FD_EINVAL for an unknown mode.  The first
 * switch to full mode creates the second stream (default priority) and two
 * events; nothing on the device is allocated.  While full mode is on,
 * fd_set_tile rejects by = 0. */
enum { FD_XCHG_BASIC = 0, FD_XCHG_FULL = 1 };
int fd_set_exchange_mode(fd_grid *g, int mode);

/* Autotuner: pick the 3-D step kernel's tile for this handle by timed
 * search (each candidate (by, ry, nzb, xcd) launched a few times on scratch
 * fields of this handle's shape, fastest kept), then apply it.  With
 * cache_path non-NULL the choice is looked up first in that JSON file (an
 * object mapping "arch|so|nz|ny|nx" to [by, ry, nzb, xcd]) and appended on
 * a miss.  Writes the chosen tile to out4 (may be NULL) and the best
 * measured milliseconds per launch to ms_out (may be NULL; 0 on a cache
 * hit).  Allocates two scratch fields for the search (setup call);
 * synchronises `stream`.  2-D grids keep the one-thread-per-point kernel.
 * Errors: the first failing candidate (launch or event error) ends the
 * search and its code is returned; the handle then keeps its previous tile
 * and nothing is written to the cache. */
int fd_autotune(fd_grid *g, const char *cache_path, int *out4, double *ms_out, void *stream);

/* Multilinear weights of sparse points (paper, "Sparse data" paragraph:
 * injection and interpolation at points off the grid).  coords_m is host
 * [n][ndim] in metres from DOMAIN index 0.  base = floor(c/h) computed in
 * FP64, clamped to shape-2; frac = c/h - base rounded to FP32.  Writes host
 * arrays base_host[n][ndim], frac_host[n][ndim].  FD_EINVAL if any point lies
 * outside [0, (shape-1) h]. */
int fd_sparse_prepare(const fd_grid *g, const double *coords_m, int n,
                      int32_t *base_host, float *frac_host);

/* Load the model.  vel_dev is DOMAIN-shaped dense (nz, ny, nx) float32 in
 * m/s.  For FD_TTI, tti_dev = {epsilon, delta, theta, phi} DOMAIN-shaped
 * (theta: tilt from vertical, phi: azimuth, radians); NULL for acoustic.
 * For FD_ELASTIC, vel_dev is the P velocity and tti_dev = {vs, rho}: S
 * velocity (m/s) and density (kg/m^3) per node.  The library then builds
 * the medium at every component's position: buoyancy 1/rho averaged over
 * the two nodes along a velocity's staggered axis, mu = rho vs^2 averaged
 * over the four nodes of a shear stress's staggered plane, lambda = rho
 * (vp^2 - 2 vs^2) and mu at the node for the normal stresses (node values
 * beyond DOMAIN repeat the last one), each times dt.
 * Builds the handle's coefficient fields on the device, then synchronises
 * `stream` to check max(vel) <= vmax (FD_EUNSTABLE otherwise; FD_ELASTIC
 * also needs rho > 0 and 0 <= vs < vp sqrt(3)/2, i.e. mu >= 0 and
 * 3 lambda + 2 mu > 0).
 * For FD_VISCO, vel_dev is the relaxed P velocity (pi = rho vp^2) and
 * tti_dev = {vs, rho, tau_ep, tau_es, tau_s} (vs relaxed, mu = rho vs^2;
 * strain relaxation times for P and S and the stress relaxation time, in
 * seconds, per node).  The library builds b dt at the velocities as for
 * FD_ELASTIC; at nodes pi tau_ep/tau_s dt, mu tau_es/tau_s dt,
 * pi (tau_ep/tau_s - 1), mu (tau_es/tau_s - 1) and dt/tau_s; at each
 * shear-stress position the means over the four nodes of its plane of
 * mu tau_es/tau_s (times dt), mu (tau_es/tau_s - 1) and 1/tau_s (times dt).
 * Checks: unrelaxed vp sqrt(tau_ep/tau_s) <= vmax, rho > 0, 0 <= vs,
 * 4 vs^2 < 3 vp^2 relaxed and unrelaxed, tau_ep >= tau_s, tau_es >= tau_s
 * and tau_s >= dt (FD_EUNSTABLE otherwise). */
int fd_set_model(fd_grid *g, const float *vel_dev, const float *const *tti_dev, void *stream);

/* Forward modelling: nt leapfrog updates of equation (acou) (or the TTI
 * system), each followed by source injection and receiver sampling.
 *   state_dev  acoustic {u^n, u^(n-1)}, TTI {p^n, p^(n-1), r^n, r^(n-1)}:
 *              padded fields, in/out; on return they hold the states nt
 *              updates later in the same order.  FD_ELASTIC: the nine
 *              components in place (velocities at n - 1/2, stresses at n
 *              on entry); update k computes v^(k+1/2) from the stresses,
 *              then tau^(k+1) from the new velocities, with the halos of
 *              the six stresses, then of the three velocities, refreshed
 *              first for FD_BC_LOOPBACK.  Sources are explosive: q[k] w /
 *              h^3 times dt / (1 + gamma dt / 2) is added to txx, tyy and
 *              tzz at each node; receivers record txx + tyy + tzz.  No
 *              checkpoints (FD_ENOTSUP).  FD_VISCO: the fifteen components
 *              (memory variables at n like the stresses); the same update
 *              with the stress pass replaced by the stress-memory pass.
 *   src, q_dev ns sources and their signatures q[nt][ns]; update k uses q[k]
 *              to produce the state at k+1.  src may be NULL (no source).
 *   rec, d_dev nr receivers, traces d[nt][nr]: d[k] sampled after update k.
 *              rec may be NULL.
 *   ckpt_dev   NULL, or nstate * ceil(nt / ckpt_every) padded fields: before
 *              update k with k % ckpt_every == 0 the state is copied into
 *              ckpt_dev[(k / ckpt_every) * nstate + i] (nstate = 2 or 4).
 * Allocates nothing; enqueues on `stream`. */
int fd_forward(fd_grid *g, float *const *state_dev,
               const fd_sparse *src, const float *q_dev,
               const fd_sparse *rec, float *d_dev, int nt,
               float *const *ckpt_dev, int ckpt_every, void *stream);

/* One update of fd_forward in place, for callers that keep their own time
 * loop (acoustic only): um_up_dev holds u^(n-1) on entry and u^(n+1) on
 * return, u_dev holds u^n (for FD_BC_LOOPBACK its halo is refreshed first,
 * so it is written too).  Then src injects q_dev[ns] (this update's values;
 * src may be NULL) and rec samples u^(n+1) into d_dev[nr] (rec may be
 * NULL).  Bit-identical to the same update inside fd_forward; unlike
 * fd_forward with nt = 1 it moves no field between the two buffers, so the
 * caller alternates their roles.  Allocates nothing; enqueues on `stream`. */
int fd_step(fd_grid *g, float *u_dev, float *um_up_dev, const fd_sparse *src,
            const float *q_dev, const fd_sparse *rec, float *d_dev, void *stream);

/* fd_step with the receivers one level behind (paper, "Sparse data"
 * paragraph): the same update and injection, but rec samples u_dev (u^n, the
 * level this update reads, after its halo refresh) into d_dev, in the same
 * launch that injects src into the new level.  For callers that change each
 * new level before it is recorded (a correction applied after the update):
 * they sample it as the next update's input, and the last level with
 * fd_sample.  Same arguments, errors and allocation behaviour as fd_step. */
int fd_step_lagged(fd_grid *g, float *u_dev, float *um_up_dev, const fd_sparse *src,
                   const float *q_dev, const fd_sparse *rec, float *d_dev, void *stream);

/* Adjoint (exact transpose of fd_forward, acoustic): the same recurrence
 * run backwards in time, receivers injecting the residual resid[nt][nr]
 * (scaled by v^2 dt^2 / (1 + gamma dt/2), no cell-volume factor) and
 * sources sampling qadj[nt][ns] = h^-d sum w lambda_n.
 *   state_dev  {lambda_(n+1), lambda_(n+2)} padded work fields, zero on entry
 *              for the terminal condition; on return lambda_0, lambda_1.
 *   grad_m_dev NULL, or DOMAIN-shaped dense float32 accumulating (+=) the
 *              zero-lag imaging condition
 *                dJ/dm = - sum_n lambda_n [(1/dt^2 + gamma/2dt) u^(n+1)
 *                          - (2/dt^2) u^n + (1/dt^2 - gamma/2dt) u^(n-1)];
 *              then ckpt_dev / ckpt_every must be those of the forward run
 *              (with src, q_dev of that run) and slot_dev must hold
 *              ckpt_every + 2 padded work fields for the recomputation.
 * Allocates nothing; enqueues on `stream`. */
int fd_adjoint(fd_grid *g, float *const *state_dev,
               const fd_sparse *rec, const float *resid_dev,
               const fd_sparse *src, const float *q_dev, float *qadj_dev, int nt,
               float *const *ckpt_dev, int ckpt_every, float *const *slot_dev,
               float *grad_m_dev, void *stream);

/* Interpolate field_dev (a padded field of this handle) at the prepared
 * points `rec` into out_dev[rec->n] (multilinear, as fd_forward samples its
 * receivers).  Enqueues one kernel on `stream`; allocates nothing. */
int fd_sample(const fd_grid *g, const float *field_dev, const fd_sparse *rec, float *out_dev,
              void *stream);

/* grad_v = grad_m * (-2 / v^3) for the loaded model (both DOMAIN-shaped). */
int fd_gradient_to_velocity(const fd_grid *g, const float *grad_m_dev, float *grad_v_dev,
                            void *stream);

/* Halo faces.  face 0..5 = -z, +z, -y, +y, -x, +x.  The buffer of face f is
 * the r-deep slab of DOMAIN adjacent to that face over the full DOMAIN extent
 * of the other axes, in field axis order, row-major; fd_halo_face_elems gives
 * its length (0 for the y faces of a 2-D grid).  Returns < 0 on a bad face. */
int64_t fd_halo_face_elems(const fd_grid *g, int face);

/* Pack the OWNED slab of every face in face_mask (bit f = face f) of
 * field_dev into buf_dev[f].  One kernel launch for all selected faces. */
int fd_pack_halo(const fd_grid *g, const float *field_dev, unsigned face_mask,
                 float *const *buf_dev, void *stream);

/* Unpack buf_dev[f] (what the neighbour across face f sent: its packed face
 * f^1) into the HALO slab beyond face f, for every face in face_mask. */
int fd_unpack_halo(const fd_grid *g, float *field_dev, unsigned face_mask,
                   const float *const *buf_dev, void *stream);

/* Measurement hooks.  fd_profile_begin(g, n) arms HIP events around the
 * next n launches of the step kernel made by fd_forward / fd_adjoint (on the
 * stream they run on); fd_profile_end synchronises those events and returns
 * the summed kernel time in milliseconds and the number of launches timed,
 * then disarms.  In FD_XCHG_FULL mode one timed launch spans the CORE, the
 * overlapped exchange and the REMAINDER kernels; an FD_ELASTIC update
 * times two launches (the velocity pass and the stress pass).  Creates events (host-side
 * objects), allocates no device memory. */
int fd_profile_begin(fd_grid *g, int max_launches);
int fd_profile_end(fd_grid *g, double *total_ms, int *launches);

/* dst[0..n) = src[0..n) on the device (float4 streaming kernel when both
 * pointers are 16-byte aligned and n % 4 == 0).  Used for checkpoint copies
 * (a kernel, so graph captures stay free of copy nodes) and as the plain
 * copy of known size that calibrates HBM byte counters. */
int fd_copy_floats(float *dst_dev, const float *src_dev, int64_t n, void *stream);

/* Thread-local description of the calling thread's last error ("" if none). */
const char *fd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FD_H */
