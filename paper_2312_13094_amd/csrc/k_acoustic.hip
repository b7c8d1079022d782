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
    up[i] = c + ((1.0f - a) * (c - um[i]) + vdt2[i] * lap) / (1.0f + a);
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

int launch_step(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s)
{
    if (g->ndim == 2 || g->tune.by == 0) return launch_step_simple(g, u, um, up, s);
    int rc;
    switch (g->r) {
    case 1: rc = launch_zmarch_radius<1>(g, u, um, up, s); break;
    case 2: rc = launch_zmarch_radius<2>(g, u, um, up, s); break;
    case 3: rc = launch_zmarch_radius<3>(g, u, um, up, s); break;
    case 4: rc = launch_zmarch_radius<4>(g, u, um, up, s); break;
    case 5: rc = launch_zmarch_radius<5>(g, u, um, up, s); break;
    case 6: rc = launch_zmarch_radius<6>(g, u, um, up, s); break;
    case 7: rc = launch_zmarch_radius<7>(g, u, um, up, s); break;
    case 8: rc = launch_zmarch_radius<8>(g, u, um, up, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    if (rc != FD_OK) return rc;
    return check_launch("acoustic step (z-march)");
}

}  // namespace fd
