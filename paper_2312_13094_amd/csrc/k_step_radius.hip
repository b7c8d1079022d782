// fd-build: one object per stencil radius (compiled with -DFD_RADIUS=1..8)
//
// Every variant of the z-marching 3-D step for one stencil radius: the
// single-grid kernel and the batched multi-shot kernel, over the supported
// tiles and flag combinations (see zmarch.h).  Compiling one radius per
// object keeps the build parallel.
#include <hip/hip_ext.h>

#include "batch_internal.h"
#include "zmarch.h"

#ifndef FD_RADIUS
#error "compile with -DFD_RADIUS=<stencil radius>"
#endif

namespace fd {

template <int R, int BY, int RY, int PF, bool NTS, bool RING, int CX = 1>
__global__ __launch_bounds__(64 * BY) void k_acoustic_zmarch(
    const float *__restrict__ u, const float *um, float *up, const float *__restrict__ vdt2,
    const StepParams p, const int ntx, const int nty, const int nzb, const int remap)
{
    __shared__ float lds[ZTile<R, BY, RY, CX>::LDS];
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

    if (RING) zmarch_buf_body<R, BY, RY, NTS, CX>(u, um, up, vdt2, p, tx, ty, zc, nzb, lds);
    else zmarch_body<R, BY, RY, PF, NTS>(u, um, up, vdt2, p, tx, ty, zc, nzb, lds);
}

template <int R, int BY, int RY, int PF, bool NTS, bool RING, int CX = 1>
static void zmarch_v(const fd_grid *g, const StepParams &p, const Tuning &t, const float *u,
                     const float *um, float *up, hipStream_t s)
{
    constexpr int TX = 64 * CX, TY = BY * RY;
    const int nzb = t.nzb > 0 ? t.nzb : 64;
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY, nzc = (p.nz + nzb - 1) / nzb;
    const unsigned nb = (unsigned)ntx * nty * nzc;
    const int remap = ((t.flags & kTileXcd) && nb % 8 == 0) ? 1 : 0;
    if (g->launch_ev[0])   // timed launch: the dispatch records the events
        hipExtLaunchKernelGGL((k_acoustic_zmarch<R, BY, RY, PF, NTS, RING, CX>), dim3(nb),
                              dim3(64, BY), 0, s, g->launch_ev[0], g->launch_ev[1], 0, u, um, up,
                              g->vdt2, p, ntx, nty, nzb, remap);
    else
        hipLaunchKernelGGL((k_acoustic_zmarch<R, BY, RY, PF, NTS, RING, CX>), dim3(nb),
                           dim3(64, BY), 0, s, u, um, up, g->vdt2, p, ntx, nty, nzb, remap);
}

// 128-wide tiles (two columns per lane): ring body, tiles (8,2) (4,2) (4,4)
// only ((8,4) would spill registers)
template <int R, int BY, int RY>
static bool zmarch_wide(const fd_grid *g, const StepParams &p, const Tuning &t, const float *u,
                        const float *um, float *up, hipStream_t s)
{
    if constexpr ((BY == 8 && RY == 2) || (BY == 4 && (RY == 2 || RY == 4))) {
        if (t.flags & kTileNts) zmarch_v<R, BY, RY, 1, true, true, 2>(g, p, t, u, um, up, s);
        else zmarch_v<R, BY, RY, 1, false, true, 2>(g, p, t, u, um, up, s);
        return true;
    }
    return false;
}

template <int R, int BY, int RY>
static bool zmarch(const fd_grid *g, const StepParams &p, const Tuning &t, const float *u,
                   const float *um, float *up, hipStream_t s)
{
    const int f = t.flags;
    const bool pf2 = f & kTilePf2, nts = f & kTileNts, ring = f & kTileRing;
    if (f & kTileWide) return zmarch_wide<R, BY, RY>(g, p, t, u, um, up, s);
    if (ring && nts) zmarch_v<R, BY, RY, 1, true, true>(g, p, t, u, um, up, s);
    else if (ring) zmarch_v<R, BY, RY, 1, false, true>(g, p, t, u, um, up, s);
    else if (pf2 && nts) zmarch_v<R, BY, RY, 2, true, false>(g, p, t, u, um, up, s);
    else if (pf2) zmarch_v<R, BY, RY, 2, false, false>(g, p, t, u, um, up, s);
    else if (nts) zmarch_v<R, BY, RY, 1, true, false>(g, p, t, u, um, up, s);
    else zmarch_v<R, BY, RY, 1, false, false>(g, p, t, u, um, up, s);
    return true;
}

template <int R>
int launch_zmarch_radius(const fd_grid *g, const StepParams &p, const Tuning &t, const float *u,
                         const float *um, float *up, hipStream_t s)
{
    const int by = t.by, ry = t.ry;
    bool ok = false;
    if (by == 4 && ry == 4) ok = zmarch<R, 4, 4>(g, p, t, u, um, up, s);
    else if (by == 4 && ry == 2) ok = zmarch<R, 4, 2>(g, p, t, u, um, up, s);
    else if (by == 4 && ry == 8) ok = zmarch<R, 4, 8>(g, p, t, u, um, up, s);
    else if (by == 8 && ry == 2) ok = zmarch<R, 8, 2>(g, p, t, u, um, up, s);
    else if (by == 8 && ry == 4) ok = zmarch<R, 8, 4>(g, p, t, u, um, up, s);
    else if (by == 2 && ry == 8) ok = zmarch<R, 2, 8>(g, p, t, u, um, up, s);
    else if (by == 4 && ry == 1) ok = zmarch<R, 4, 1>(g, p, t, u, um, up, s);
    if (!ok) return set_error(FD_EINVAL, "unsupported tile shape");
    return FD_OK;
}

// Batched step: every variant takes the buffer-addressed body (halo ring);
// EPI selects the gradient schedule's extra work (StepImaging in zmarch.h).
template <int R, int BY, int RY, bool NTS, int CX, int EPI>
__global__ __launch_bounds__(64 * BY) void k_batch_zmarch(const BatchShot *__restrict__ shots,
                                                          const int nshots, const int total,
                                                          const int iu, const int ium,
                                                          const int iup, const int nzb,
                                                          const int remap, const BatchEpi e)
{
    __shared__ float lds[ZTile<R, BY, RY, CX>::LDS];
    int b = blockIdx.x;
    if (remap) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
    if (b >= total) return;
    int s = 0;
    for (int k = 1; k < nshots; ++k)
        if (shots[k].block0 <= b) s = k;
    const BatchShot &S = shots[s];
    int lb = b - S.block0;
    const int tx = lb % S.ntx;
    lb /= S.ntx;
    const int ty = lb % S.nty;
    const int zc = lb / S.nty;
    float *base = S.base;
    const int64_t st = S.stride;
    const StepImaging img{base + e.fd * st, base + e.fg * st, e.inv_dt2, e.inv_2dt};
    zmarch_buf_body<R, BY, RY, NTS, CX, EPI, true>(base + iu * st, base + ium * st,
                                                   base + iup * st, base + kVdt2 * st, S.p, tx,
                                                   ty, zc, nzb, lds, img);
}

template <int R, int BY, int RY, bool NTS, int CX>
static void batch_step_v(const BatchShot *shots, int nshots, int total, const Tuning &t, int iu,
                         int ium, int iup, const BatchEpi &e, hipStream_t s)
{
    const int remap = (t.flags & kTileXcd) ? 1 : 0;
    const unsigned nb = remap ? (unsigned)((total + 7) / 8 * 8) : (unsigned)total;
    const dim3 g(nb), blk(64, BY);
    if (e.mode == 1)
        hipLaunchKernelGGL((k_batch_zmarch<R, BY, RY, NTS, CX, 1>), g, blk, 0, s, shots, nshots,
                           total, iu, ium, iup, t.nzb, remap, e);
    else if (e.mode == 2)
        hipLaunchKernelGGL((k_batch_zmarch<R, BY, RY, NTS, CX, 2>), g, blk, 0, s, shots, nshots,
                           total, iu, ium, iup, t.nzb, remap, e);
    else
        hipLaunchKernelGGL((k_batch_zmarch<R, BY, RY, NTS, CX, 0>), g, blk, 0, s, shots, nshots,
                           total, iu, ium, iup, t.nzb, remap, e);
}

template <int R, int BY, int RY>
static bool batch_step(const BatchShot *shots, int nshots, int total, const Tuning &t, int iu,
                       int ium, int iup, const BatchEpi &e, hipStream_t s)
{
    const bool nts = t.flags & kTileNts;
    if (t.flags & kTileWide) {
        // 128-wide tiles (fd_batch_set_tile admits only these shapes)
        if constexpr ((BY == 8 && RY == 2) || (BY == 4 && (RY == 2 || RY == 4))) {
            if (nts) batch_step_v<R, BY, RY, true, 2>(shots, nshots, total, t, iu, ium, iup, e, s);
            else batch_step_v<R, BY, RY, false, 2>(shots, nshots, total, t, iu, ium, iup, e, s);
            return true;
        }
        return false;
    }
    if (nts) batch_step_v<R, BY, RY, true, 1>(shots, nshots, total, t, iu, ium, iup, e, s);
    else batch_step_v<R, BY, RY, false, 1>(shots, nshots, total, t, iu, ium, iup, e, s);
    return true;
}

template <int R>
int launch_batch_radius(const BatchShot *shots, int nshots, int total, const Tuning &t, int iu,
                        int ium, int iup, const BatchEpi &e, hipStream_t s)
{
    bool ok = false;
    if (t.by == 4 && t.ry == 4) ok = batch_step<R, 4, 4>(shots, nshots, total, t, iu, ium, iup, e, s);
    else if (t.by == 4 && t.ry == 2) ok = batch_step<R, 4, 2>(shots, nshots, total, t, iu, ium, iup, e, s);
    else if (t.by == 4 && t.ry == 8) ok = batch_step<R, 4, 8>(shots, nshots, total, t, iu, ium, iup, e, s);
    else if (t.by == 8 && t.ry == 2) ok = batch_step<R, 8, 2>(shots, nshots, total, t, iu, ium, iup, e, s);
    else if (t.by == 8 && t.ry == 4) ok = batch_step<R, 8, 4>(shots, nshots, total, t, iu, ium, iup, e, s);
    else if (t.by == 2 && t.ry == 8) ok = batch_step<R, 2, 8>(shots, nshots, total, t, iu, ium, iup, e, s);
    else if (t.by == 4 && t.ry == 1) ok = batch_step<R, 4, 1>(shots, nshots, total, t, iu, ium, iup, e, s);
    if (!ok) return set_error(FD_EINVAL, "unsupported tile shape");
    return FD_OK;
}

template int launch_zmarch_radius<FD_RADIUS>(const fd_grid *, const StepParams &, const Tuning &,
                                             const float *, const float *, float *, hipStream_t);
template int launch_batch_radius<FD_RADIUS>(const BatchShot *, int, int, const Tuning &, int, int,
                                            int, const BatchEpi &, hipStream_t);

}  // namespace fd
