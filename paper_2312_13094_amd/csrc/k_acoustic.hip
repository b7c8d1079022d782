// Acoustic leapfrog step kernels for gfx950.
//
// One update of the second-order-in-time acoustic wave equation (paper,
// appendix "Isotropic acoustic", equation (acou)) with a damping layer:
//
//   u+ = [2 u - (1 - a) u- + v^2 dt^2 * Lap_h u] / (1 + a),   a = gamma dt / 2,
//
// evaluated as u + [(1 - a)(u - u-) + v^2 dt^2 Lap_h u] / (1 + a), which rounds
// once at the magnitude of u per step instead of twice (FP32 error growth of
// the leapfrog over hundreds of steps is dominated by that rounding).
// where Lap_h is the centred star stencil of radius R on each active axis.
// u- is overwritten in place by u+ (every point reads only its own u-), so
// a step streams exactly four fields: u (read), u- (read), v^2 dt^2 (read),
// u+ (write) -- 16 bytes per point.  The stencil is memory-bound and never
// touches MFMA: it is not a contraction.
//
// k_acoustic_zmarch (3-D): a block owns a 64 x TY column tile and marches
// along z.  Each thread keeps the 2R+1 values of its column in registers (a
// z queue), so every u value enters the chip once per z chunk.  The current
// plane, plus an R-wide x/y halo, is staged in LDS (double buffered, one
// barrier per plane) for the x and y neighbours.  Loads for plane z+1 are
// issued before plane z is computed.  Blocks are remapped so that the eight
// XCDs each sweep a contiguous range of tiles, keeping the halo re-reads of
// neighbouring tiles inside one XCD's L2.
//
// k_acoustic_simple: one thread per point, neighbours straight from global
// memory; used for 2-D grids and as the reference GPU path.
#include "fd_internal.h"

namespace fd {

template <int R, bool TWO_D>
__global__ __launch_bounds__(256) void k_acoustic_simple(const float *__restrict__ u,
                                                         const float *um, float *up,
                                                         const float *__restrict__ vdt2,
                                                         const StepParams p, const int nxb,
                                                         const int nyb)
{
    int b = blockIdx.x;
    const int xb = b % nxb;
    b /= nxb;
    const int yb = b % nyb;
    const int z = b / nyb;
    const int x = xb * 64 + threadIdx.x;
    const int y = yb * 4 + threadIdx.y;
    if (x >= p.nx || y >= p.ny) return;
    const int64_t PY = p.pitch_y, PZ = p.pitch_z;
    const int64_t i = p.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
    const float c = u[i];
    float lz = 0.0f, ly = 0.0f, lx = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lz += p.cz[k] * (u[i + k * PZ] + u[i - k * PZ]);
        lx += p.cx[k] * (u[i + k] + u[i - k]);
        if (!TWO_D) ly += p.cy[k] * (u[i + k * PY] + u[i - k * PY]);
    }
    const float lap = p.c0 * c + lz + ly + lx;
    const float a = damp_a(p, z, y, x);
    // u+ = u + [(1-a)(u - u-) + v^2 dt^2 lap] / (1+a): algebraically the
    // leapfrog update, with one rounding at the field's magnitude per step
    up[i] = leapfrog_update(c, um[i], vdt2[i], lap, a);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int R>
static void simple_r(const fd_grid *g, const float *u, const float *um, float *up,
                     hipStream_t s)
{
    const StepParams &p = g->sp;
    const int nxb = (p.nx + 63) / 64, nyb = (p.ny + 3) / 4;
    const dim3 blk(64, 4);
    const unsigned nb = (unsigned)nxb * nyb * p.nz;
    if (g->ndim == 2)
        hipLaunchKernelGGL((k_acoustic_simple<R, true>), dim3(nb), blk, 0, s, u, um, up, g->vdt2,
                           p, nxb, nyb);
    else
        hipLaunchKernelGGL((k_acoustic_simple<R, false>), dim3(nb), blk, 0, s, u, um, up,
                           g->vdt2, p, nxb, nyb);
}

int launch_step_simple(const fd_grid *g, const float *u, const float *um, float *up,
                       hipStream_t s)
{
    switch (g->r) {
    case 1: simple_r<1>(g, u, um, up, s); break;
    case 2: simple_r<2>(g, u, um, up, s); break;
    case 3: simple_r<3>(g, u, um, up, s); break;
    case 4: simple_r<4>(g, u, um, up, s); break;
    case 5: simple_r<5>(g, u, um, up, s); break;
    case 6: simple_r<6>(g, u, um, up, s); break;
    case 7: simple_r<7>(g, u, um, up, s); break;
    case 8: simple_r<8>(g, u, um, up, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    return check_launch("acoustic step (simple)");
}

static int zmarch_box(const fd_grid *g, const StepParams &p, const Tuning &t, const float *u,
                      const float *um, float *up, hipStream_t s)
{
    switch (g->r) {
    case 1: return launch_zmarch_radius<1>(g, p, t, u, um, up, s);
    case 2: return launch_zmarch_radius<2>(g, p, t, u, um, up, s);
    case 3: return launch_zmarch_radius<3>(g, p, t, u, um, up, s);
    case 4: return launch_zmarch_radius<4>(g, p, t, u, um, up, s);
    case 5: return launch_zmarch_radius<5>(g, p, t, u, um, up, s);
    case 6: return launch_zmarch_radius<6>(g, p, t, u, um, up, s);
    case 7: return launch_zmarch_radius<7>(g, p, t, u, um, up, s);
    case 8: return launch_zmarch_radius<8>(g, p, t, u, um, up, s);
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
}

int launch_step(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s)
{
    if (g->ndim == 2 || g->tune.by == 0) return launch_step_simple(g, u, um, up, s);
    const int rc = zmarch_box(g, g->sp, g->tune, u, um, up, s);
    if (rc != FD_OK) return rc;
    return check_launch("acoustic step (z-march)");
}

// ---------------------------------------------------------------------------
// full exchange mode (paper, computation/communication patterns: the "full"
// pattern splits DOMAIN into a CORE, whose stencils read no HALO, and a
// REMAINDER, and overlaps the halo update with the CORE)
// ---------------------------------------------------------------------------

// The z-march over the DOMAIN sub-box [lo, hi) (z, y, x).  The launch origin
// moves to (lo_z, lo_y, x0) with x0 = lo_x rounded down to a multiple of 64,
// so tile rows stay on whole cache lines; columns x0 .. lo_x - 1 are read as
// the tile's rim but not written.  Damping edges move with the origin, so
// every point sees the damping of its DOMAIN position.
static int zmarch_subbox(const fd_grid *g, const int lo[3], const int hi[3], const Tuning &t,
                         const float *u, const float *um, float *up, hipStream_t s)
{
    StepParams p = g->sp;
    const int x0 = lo[2] / 64 * 64;
    const int shift[3] = {lo[0], lo[1], x0};
    p.offset += (int64_t)lo[0] * p.pitch_z + (int64_t)lo[1] * p.pitch_y + x0;
    p.nz = hi[0] - lo[0];
    p.ny = hi[1] - lo[1];
    p.nx = hi[2] - x0;
    p.xlo = lo[2] - x0;
    for (int a = 0; a < 3; ++a) {
        p.sl[a] -= shift[a];
        p.sh[a] -= shift[a];
    }
    return zmarch_box(g, p, t, u, um, up, s);
}

// The two x faces of the REMAINDER: R <= z < nz - R, R <= y < ny - R and
// x < R or x >= nx - R, one thread per point (2R consecutive threads per
// row, R on each side).  The stencil sums, damping and update are the
// z-march's, term for term, so both give the same bits.
template <int R>
__global__ __launch_bounds__(256) void k_acoustic_xfaces(const float *__restrict__ u,
                                                         const float *um, float *up,
                                                         const float *__restrict__ vdt2,
                                                         const StepParams p, const int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int c = (int)(t % (2 * R));
    const int64_t zy = t / (2 * R);
    const int ny2 = p.ny - 2 * R;
    const int y = R + (int)(zy % ny2);
    const int z = R + (int)(zy / ny2);
    const int x = c < R ? c : p.nx - 2 * R + c;
    const int64_t PY = p.pitch_y, PZ = p.pitch_z;
    const int64_t i = p.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
    const float uc = u[i];
    float lz = 0.0f, ly = 0.0f, lx = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lz += p.cz[k] * (u[i + k * PZ] + u[i - k * PZ]);
        ly += p.cy[k] * (u[i + k * PY] + u[i - k * PY]);
        lx += p.cx[k] * (u[i + k] + u[i - k]);
    }
    const float lap = p.c0 * uc + lz + ly + lx;
    const float az = p.nbl > 0 ? sponge_ax(p, 0, z, p.gz) : 0.0f;
    const float ax = p.nbl > 0 ? sponge_ax(p, 2, x, p.gx) : 0.0f;
    const float ay = p.nbl > 0 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
    const float a = p.half_dt * ((az + ax) + ay);
    up[i] = leapfrog_update(uc, um[i], vdt2[i], lap, a);
}

template <int R>
static void xfaces_r(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s)
{
    const StepParams &p = g->sp;
    const int64_t total = (int64_t)(p.nz - 2 * R) * (p.ny - 2 * R) * (2 * R);
    const unsigned nb = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL((k_acoustic_xfaces<R>), dim3(nb), dim3(256), 0, s, u, um, up, g->vdt2, p,
                       total);
}

static int launch_xfaces(const fd_grid *g, const float *u, const float *um, float *up,
                         hipStream_t s)
{
    switch (g->r) {
    case 1: xfaces_r<1>(g, u, um, up, s); break;
    case 2: xfaces_r<2>(g, u, um, up, s); break;
    case 3: xfaces_r<3>(g, u, um, up, s); break;
    case 4: xfaces_r<4>(g, u, um, up, s); break;
    case 5: xfaces_r<5>(g, u, um, up, s); break;
    case 6: xfaces_r<6>(g, u, um, up, s); break;
    case 7: xfaces_r<7>(g, u, um, up, s); break;
    case 8: xfaces_r<8>(g, u, um, up, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    return FD_OK;
}

int launch_step_full(fd_grid *g, float *u, const float *um, float *up, hipStream_t s)
{
    const int R = g->r, nz = g->n[0], ny = g->n[1], nx = g->n[2];
    if (g->ndim != 3 || g->tune.by == 0 || !g->xs || nz <= 2 * R || ny <= 2 * R || nx <= 2 * R)
        return set_error(FD_EINVAL, "full exchange mode: unsupported grid state");
    // fork: the exchange stream waits for all work queued so far on s
    if (hipEventRecord(g->xfork, s) != hipSuccess || hipStreamWaitEvent(g->xs, g->xfork, 0) != hipSuccess)
        return set_error(FD_EDEVICE, "full exchange mode: fork failed");
    int rc = launch_loopback(g, u, g->facebuf, g->xs);
    if (rc) return rc;
    if (hipEventRecord(g->xjoin, g->xs) != hipSuccess)
        return set_error(FD_EDEVICE, "full exchange mode: event record failed");
    // CORE: every index in [R, n - R), reading DOMAIN only
    const int clo[3] = {R, R, R}, chi[3] = {nz - R, ny - R, nx - R};
    if ((rc = zmarch_subbox(g, clo, chi, g->tune, u, um, up, s))) return rc;
    // join, then the REMAINDER, which reads the fresh HALO
    if (hipStreamWaitEvent(s, g->xjoin, 0) != hipSuccess)
        return set_error(FD_EDEVICE, "full exchange mode: join failed");
    // z slabs: R whole planes each, one z chunk per tile
    Tuning tz = g->tune;
    tz.nzb = R;
    const int zl0[3] = {0, 0, 0}, zh0[3] = {R, ny, nx};
    const int zl1[3] = {nz - R, 0, 0}, zh1[3] = {nz, ny, nx};
    if ((rc = zmarch_subbox(g, zl0, zh0, tz, u, um, up, s)) ||
        (rc = zmarch_subbox(g, zl1, zh1, tz, u, um, up, s)))
        return rc;
    // y slabs: R rows under the z slabs' span, on 64 x 4 tiles
    const Tuning ty{4, 1, 8, g->tune.flags & ~kTileWide};
    const int yl0[3] = {R, 0, 0}, yh0[3] = {nz - R, R, nx};
    const int yl1[3] = {R, ny - R, 0}, yh1[3] = {nz - R, ny, nx};
    if ((rc = zmarch_subbox(g, yl0, yh0, ty, u, um, up, s)) ||
        (rc = zmarch_subbox(g, yl1, yh1, ty, u, um, up, s)))
        return rc;
    // x faces: what is left
    if ((rc = launch_xfaces(g, u, um, up, s))) return rc;
    return check_launch("acoustic step (full exchange mode)");
}

}  // namespace fd
