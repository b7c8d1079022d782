// Acoustic leapfrog step kernels for gfx950.
//
// One update of the second-order-in-time acoustic wave equation (paper,
// appendix "Isotropic acoustic", equation (acou)) with a damping layer:
//
//   u+ = [2 u - (1 - a) u- + v^2 dt^2 * Lap_h u] / (1 + a),   a = gamma dt / 2,
//
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
    up[i] = (2.0f * c - (1.0f - a) * um[i] + vdt2[i] * lap) / (1.0f + a);
}

template <int R, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_acoustic_zmarch(
    const float *__restrict__ u, const float *um, float *up, const float *__restrict__ vdt2,
    const StepParams p, const int ntx, const int nty, const int nzb, const int remap)
{
    constexpr int TX = 64, TY = BY * RY, LX = TX + 2 * R, LY = TY + 2 * R;
    constexpr int NT = 64 * BY;
    constexpr int NHY = 2 * R * TX;   // y-halo values per plane
    constexpr int NHX = 2 * R * TY;   // x-halo values per plane
    constexpr int HY = (NHY + NT - 1) / NT;
    constexpr int HX = (NHX + NT - 1) / NT;
    __shared__ float tile[2][LY * LX];

    int b = blockIdx.x;
    if (remap) {
        // the dispatcher deals block b to XCD b % 8: give XCD k the
        // contiguous logical range [k * nb/8, (k+1) * nb/8)
        const int per = gridDim.x >> 3;
        b = (b & 7) * per + (b >> 3);
    }
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;

    const int lane = threadIdx.x, wy = threadIdx.y;
    const int tid = wy * 64 + lane;
    const int x0 = tx * TX, y0 = ty * TY;
    const int x = x0 + lane;
    const int yb = y0 + wy * RY;
    const int z0 = zc * nzb;
    const int z1 = min(z0 + nzb, p.nz);
    const int64_t PY = p.pitch_y, PZ = p.pitch_z;
    const float *uo = u + p.offset;      // DOMAIN origin of u
    const float *umo = um + p.offset;
    const float *vo = vdt2 + p.offset;
    float *upo = up + p.offset;

    // which of this thread's rows are loadable (inside DOMAIN + halo) and
    // which are written (inside DOMAIN)
    const bool xl = x < p.nx + R;
    bool rl[RY], ro[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = xl && (yb + j) < p.ny + R;
        ro[j] = x < p.nx && (yb + j) < p.ny;
    }

    // halo descriptors, fixed over z: element offset within a plane, LDS slot
    int64_t hyo[HY], hxo[HX];
    int hys[HY], hxs[HX];
    bool hyk[HY], hxk[HX];
#pragma unroll
    for (int k = 0; k < HY; ++k) {
        const int e = tid + k * NT;
        const int row = e / TX, col = e % TX;
        const int yy = row < R ? y0 - R + row : y0 + TY + (row - R);
        const int ly = row < R ? row : TY + row;
        const int xx = x0 + col;
        hyk[k] = e < NHY && yy < p.ny + R && xx < p.nx + R;
        hyo[k] = (int64_t)yy * PY + xx;
        hys[k] = ly * LX + col + R;
    }
#pragma unroll
    for (int k = 0; k < HX; ++k) {
        const int e = tid + k * NT;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = y0 + row;
        const int xx = c < R ? x0 - R + c : x0 + TX + (c - R);
        const int lx = c < R ? c : TX + c;
        hxk[k] = e < NHX && yy < p.ny + R && xx < p.nx + R;
        hxo[k] = (int64_t)yy * PY + xx;
        hxs[k] = (row + R) * LX + lx;
    }

    // z queue: q[j][k] = u(z - R + k, yb + j, x)
    float q[RY][2 * R + 1];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int64_t col = (int64_t)(yb + j) * PY + x;
#pragma unroll
        for (int k = 0; k < 2 * R; ++k)
            q[j][k + 1] = rl[j] ? uo[(int64_t)(z0 - R + k) * PZ + col] : 0.0f;
    }

    // prefetch registers for the next plane
    float nf[RY], nm[RY], nv[RY], nhy[HY], nhx[HX];
    auto prefetch = [&](int z) {
        const int64_t pz = (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t col = (int64_t)(yb + j) * PY + x;
            nf[j] = rl[j] ? uo[pz + R * PZ + col] : 0.0f;
            nm[j] = ro[j] ? umo[pz + col] : 0.0f;
            nv[j] = ro[j] ? vo[pz + col] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < HY; ++k) nhy[k] = hyk[k] ? uo[pz + hyo[k]] : 0.0f;
#pragma unroll
        for (int k = 0; k < HX; ++k) nhx[k] = hxk[k] ? uo[pz + hxo[k]] : 0.0f;
    };
    if (z0 < z1) prefetch(z0);

    for (int z = z0; z < z1; ++z) {
        float cm[RY], cv[RY], chy[HY], chx[HX];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) q[j][k] = q[j][k + 1];
            q[j][2 * R] = nf[j];
            cm[j] = nm[j];
            cv[j] = nv[j];
        }
#pragma unroll
        for (int k = 0; k < HY; ++k) chy[k] = nhy[k];
#pragma unroll
        for (int k = 0; k < HX; ++k) chx[k] = nhx[k];
        if (z + 1 < z1) prefetch(z + 1);

        float *t = tile[z & 1];
#pragma unroll
        for (int j = 0; j < RY; ++j) t[(wy * RY + j + R) * LX + lane + R] = q[j][R];
#pragma unroll
        for (int k = 0; k < HY; ++k)
            if (tid + k * NT < NHY) t[hys[k]] = chy[k];
#pragma unroll
        for (int k = 0; k < HX; ++k)
            if (tid + k * NT < NHX) t[hxs[k]] = chx[k];
        __syncthreads();

        const float az = p.nbl > 0 ? sponge1(z, p.nz, p.nbl, p.inv_nbl, p.gz) : 0.0f;
        const float ax = p.nbl > 0 ? sponge1(x, p.nx, p.nbl, p.inv_nbl, p.gx) : 0.0f;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const float *c = t + (wy * RY + j + R) * LX + lane + R;
            float lz = 0.0f, ly = 0.0f, lx = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                lz += p.cz[k] * (q[j][R + k] + q[j][R - k]);
                ly += p.cy[k] * (c[k * LX] + c[-k * LX]);
                lx += p.cx[k] * (c[k] + c[-k]);
            }
            const float uc = q[j][R];
            const float lap = p.c0 * uc + lz + ly + lx;
            const int y = yb + j;
            // same summation order as damp_a(): (z + x) + y
            const float ay = p.nbl > 0 ? sponge1(y, p.ny, p.nbl, p.inv_nbl, p.gy) : 0.0f;
            const float a = p.half_dt * ((az + ax) + ay);
            if (ro[j])
                upo[(int64_t)z * PZ + (int64_t)y * PY + x] =
                    (2.0f * uc - (1.0f - a) * cm[j] + cv[j] * lap) / (1.0f + a);
        }
    }
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

template <int R, int BY, int RY>
static void zmarch(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s)
{
    const StepParams &p = g->sp;
    constexpr int TY = BY * RY;
    const int nzb = g->tune.nzb > 0 ? g->tune.nzb : 64;
    const int ntx = (p.nx + 63) / 64, nty = (p.ny + TY - 1) / TY, nzc = (p.nz + nzb - 1) / nzb;
    const unsigned nb = (unsigned)ntx * nty * nzc;
    const int remap = (g->tune.xcd && nb % 8 == 0) ? 1 : 0;
    hipLaunchKernelGGL((k_acoustic_zmarch<R, BY, RY>), dim3(nb), dim3(64, BY), 0, s, u, um, up,
                       g->vdt2, p, ntx, nty, nzb, remap);
}

template <int R>
static int zmarch_r(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s)
{
    const int by = g->tune.by, ry = g->tune.ry;
    if (by == 4 && ry == 4) zmarch<R, 4, 4>(g, u, um, up, s);
    else if (by == 4 && ry == 2) zmarch<R, 4, 2>(g, u, um, up, s);
    else if (by == 4 && ry == 8) zmarch<R, 4, 8>(g, u, um, up, s);
    else if (by == 8 && ry == 2) zmarch<R, 8, 2>(g, u, um, up, s);
    else if (by == 8 && ry == 4) zmarch<R, 8, 4>(g, u, um, up, s);
    else if (by == 2 && ry == 8) zmarch<R, 2, 8>(g, u, um, up, s);
    else if (by == 4 && ry == 1) zmarch<R, 4, 1>(g, u, um, up, s);
    else return set_error(FD_EINVAL, "unsupported tile shape");
    return FD_OK;
}

int launch_step(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s)
{
    if (g->ndim == 2 || g->tune.by == 0) return launch_step_simple(g, u, um, up, s);
    int rc;
    switch (g->r) {
    case 1: rc = zmarch_r<1>(g, u, um, up, s); break;
    case 2: rc = zmarch_r<2>(g, u, um, up, s); break;
    case 3: rc = zmarch_r<3>(g, u, um, up, s); break;
    case 4: rc = zmarch_r<4>(g, u, um, up, s); break;
    case 5: rc = zmarch_r<5>(g, u, um, up, s); break;
    case 6: rc = zmarch_r<6>(g, u, um, up, s); break;
    case 7: rc = zmarch_r<7>(g, u, um, up, s); break;
    case 8: rc = zmarch_r<8>(g, u, um, up, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    if (rc != FD_OK) return rc;
    return check_launch("acoustic step (z-march)");
}

}  // namespace fd
