// z-marching kernels of the pseudo-acoustic TTI step (paper, appendix
// "Anisotropic acoustic (TTI)", equation (rot); the two-field system and the
// rotated operators are described in k_tti.hip).  Same two passes as there,
// with the stencil reads of each pass staged on chip the way the acoustic
// z-march does it (zmarch.h):
//
//   pass 1  p, r -> w = (I - a a^T) grad p,  s = a (a . grad r)
//           z derivatives from a register queue of 2R+1 planes per column,
//           x/y derivatives from an LDS plane with an R-wide ring;
//   pass 2  div w, div s and the coupled leapfrog update
//           d/dz of (w0, s0) from register queues, d/dy of (w1, s1) from an
//           LDS plane with a y ring, d/dx of (w2, s2) from one with an x ring.
//
// Every field enters the chip once per z chunk (plus 2R planes of queue
// warm-up); the intermediates are written once and read once.  A block is
// 64 x BY threads over a 64 x (BY*RY) column tile and nzb planes.
#include "fd_internal.h"

namespace fd {

namespace {

constexpr int kTtiBy = 8, kTtiRy = 2;

// Which halo element of a 64 x TY tile's R-wide ring a thread stages: y ring
// (rows above and below, 64 wide) or x ring (columns left and right, TY
// tall).  e indexes the ring elements; returns false past the ring.
template <int R, int TY>
__device__ __forceinline__ bool yring(int e, int y0, int x0, int &yy, int &xx, int &ly, int &lx)
{
    if (e >= 2 * R * 64) return false;
    const int row = e / 64, col = e % 64;
    yy = row < R ? y0 - R + row : y0 + TY + (row - R);
    ly = row < R ? row : TY + row;
    xx = x0 + col;
    lx = col;
    return true;
}

template <int R, int TY>
__device__ __forceinline__ bool xring(int e, int y0, int x0, int &yy, int &xx, int &ly, int &lx)
{
    if (e >= 2 * R * TY) return false;
    const int row = e / (2 * R), c = e % (2 * R);
    yy = y0 + row;
    ly = row;
    xx = c < R ? x0 - R + c : x0 + 64 + (c - R);
    lx = c < R ? c : 64 + c;
    return true;
}

}  // namespace

// Pass 1: rotated gradients.
template <int R>
__global__ __launch_bounds__(64 * kTtiBy) void k_tti_grad_zm(
    const float *__restrict__ p, const float *__restrict__ r, const float *__restrict__ th,
    const float *__restrict__ ph, float *__restrict__ w0, float *__restrict__ w1,
    float *__restrict__ w2, float *__restrict__ s0, float *__restrict__ s1,
    float *__restrict__ s2, const StepParams sp, const int ntx, const int nty, const int nzb)
{
    constexpr int BY = kTtiBy, RY = kTtiRy, TY = BY * RY, LX = 64 + 2 * R, LY = TY + 2 * R;
    constexpr int NT = 64 * BY;
    constexpr int HY = (2 * R * 64 + NT - 1) / NT, HX = (2 * R * TY + NT - 1) / NT;
    __shared__ float lp[2][LY * LX], lr[2][LY * LX];

    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int lane = threadIdx.x, wy = threadIdx.y, tid = wy * 64 + lane;
    const int x0 = tx * 64, y0 = ty * TY, x = x0 + lane, yb = y0 + wy * RY;
    const int z0 = zc * nzb, z1 = min(z0 + nzb, sp.nz);
    const int64_t PY = sp.pitch_y, PZ = sp.pitch_z;
    const int64_t o = sp.offset;

    bool rl[RY], ro[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = x < sp.nx + R && yb + j < sp.ny + R;
        ro[j] = x < sp.nx && yb + j < sp.ny;
    }
    // ring slots: plane offset, LDS slot, valid
    int64_t hyo[HY], hxo[HX];
    int hys[HY], hxs[HX];
    bool hyk[HY], hxk[HX];
#pragma unroll
    for (int k = 0; k < HY; ++k) {
        int yy, xx, ly, lx;
        hyk[k] = yring<R, TY>(tid + k * NT, y0, x0, yy, xx, ly, lx);
        hyk[k] = hyk[k] && yy < sp.ny + R && xx < sp.nx + R;
        hyo[k] = hyk[k] ? (int64_t)yy * PY + xx : 0;
        hys[k] = ly * LX + lx + R;
    }
#pragma unroll
    for (int k = 0; k < HX; ++k) {
        int yy, xx, ly, lx;
        hxk[k] = xring<R, TY>(tid + k * NT, y0, x0, yy, xx, ly, lx);
        hxk[k] = hxk[k] && yy < sp.ny + R && xx < sp.nx + R;
        hxo[k] = hxk[k] ? (int64_t)yy * PY + xx : 0;
        hxs[k] = (ly + R) * LX + lx;
    }

    // queues: q?[j][k] = field(z - R + k, yb + j, x)
    float qp[RY][2 * R + 1], qr[RY][2 * R + 1];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int64_t col = o + (int64_t)(yb + j) * PY + x;
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int64_t i = col + (int64_t)(z0 - R + k) * PZ;
            qp[j][k + 1] = rl[j] ? p[i] : 0.0f;
            qr[j][k + 1] = rl[j] ? r[i] : 0.0f;
        }
    }
    float fp[RY], fr[RY], ft[RY], ff[RY], hp[HY + HX], hr[HY + HX];
    auto prefetch = [&](const int z) {
        const int64_t pz = o + (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t i = pz + (int64_t)(yb + j) * PY + x;
            fp[j] = rl[j] ? p[i + R * PZ] : 0.0f;
            fr[j] = rl[j] ? r[i + R * PZ] : 0.0f;
            ft[j] = ro[j] ? __builtin_nontemporal_load(th + i) : 0.0f;
            ff[j] = ro[j] ? __builtin_nontemporal_load(ph + i) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < HY; ++k) {
            hp[k] = hyk[k] ? p[pz + hyo[k]] : 0.0f;
            hr[k] = hyk[k] ? r[pz + hyo[k]] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < HX; ++k) {
            hp[HY + k] = hxk[k] ? p[pz + hxo[k]] : 0.0f;
            hr[HY + k] = hxk[k] ? r[pz + hxo[k]] : 0.0f;
        }
    };
    if (z0 < z1) prefetch(z0);

    for (int z = z0; z < z1; ++z) {
        float ct[RY], cf[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                qp[j][k] = qp[j][k + 1];
                qr[j][k] = qr[j][k + 1];
            }
            qp[j][2 * R] = fp[j];
            qr[j][2 * R] = fr[j];
            ct[j] = ft[j];
            cf[j] = ff[j];
        }
        float *tp = lp[z & 1], *tr = lr[z & 1];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int l = (wy * RY + j + R) * LX + lane + R;
            tp[l] = qp[j][R];
            tr[l] = qr[j][R];
        }
#pragma unroll
        for (int k = 0; k < HY; ++k)
            if (tid + k * NT < 2 * R * 64) {
                tp[hys[k]] = hp[k];
                tr[hys[k]] = hr[k];
            }
#pragma unroll
        for (int k = 0; k < HX; ++k)
            if (tid + k * NT < 2 * R * TY) {
                tp[hxs[k]] = hp[HY + k];
                tr[hxs[k]] = hr[HY + k];
            }
        if (z + 1 < z1) prefetch(z + 1);
        __syncthreads();

#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int l = (wy * RY + j + R) * LX + lane + R;
            const float *cp = tp + l, *cr = tr + l;
            float gpz = 0.f, gpy = 0.f, gpx = 0.f, grz = 0.f, gry = 0.f, grx = 0.f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const float az = sp.dz[k - 1], ay = sp.dy[k - 1], ax = sp.dx[k - 1];
                gpz += az * (qp[j][R + k] - qp[j][R - k]);
                gpy += ay * (cp[k * LX] - cp[-k * LX]);
                gpx += ax * (cp[k] - cp[-k]);
                grz += az * (qr[j][R + k] - qr[j][R - k]);
                gry += ay * (cr[k * LX] - cr[-k * LX]);
                grx += ax * (cr[k] - cr[-k]);
            }
            float st, cs, sf, cf2;
            sincosf(ct[j], &st, &cs);
            sincosf(cf[j], &sf, &cf2);
            const float az = cs, ay = st * sf, ax = st * cf2;
            const float ap = az * gpz + ay * gpy + ax * gpx;
            const float ar = az * grz + ay * gry + ax * grx;
            if (ro[j]) {
                const int64_t i = o + (int64_t)z * PZ + (int64_t)(yb + j) * PY + x;
                __builtin_nontemporal_store(gpz - az * ap, w0 + i);
                __builtin_nontemporal_store(gpy - ay * ap, w1 + i);
                __builtin_nontemporal_store(gpx - ax * ap, w2 + i);
                __builtin_nontemporal_store(az * ar, s0 + i);
                __builtin_nontemporal_store(ay * ar, s1 + i);
                __builtin_nontemporal_store(ax * ar, s2 + i);
            }
        }
    }
}

// Pass 2: divergences and the coupled leapfrog update (pp may alias pm,
// rp may alias rm).
template <int R>
__global__ __launch_bounds__(64 * kTtiBy) void k_tti_div_zm(
    const float *__restrict__ p, const float *pm, float *pp, const float *__restrict__ r,
    const float *rm, float *rp, const float *__restrict__ w0, const float *__restrict__ w1,
    const float *__restrict__ w2, const float *__restrict__ s0, const float *__restrict__ s1,
    const float *__restrict__ s2, const float *__restrict__ c, const float *__restrict__ cpp,
    const float *__restrict__ cx, const StepParams sp, const int ntx, const int nty,
    const int nzb)
{
    constexpr int BY = kTtiBy, RY = kTtiRy, TY = BY * RY, LX = 64 + 2 * R, LY = TY + 2 * R;
    constexpr int NT = 64 * BY;
    constexpr int HY = (2 * R * 64 + NT - 1) / NT, HX = (2 * R * TY + NT - 1) / NT;
    // y-ringed planes of w1, s1 (LY x 64) and x-ringed planes of w2, s2 (TY x LX)
    __shared__ float lw1[2][LY * 64], ls1[2][LY * 64], lw2[2][TY * LX], ls2[2][TY * LX];

    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int lane = threadIdx.x, wy = threadIdx.y, tid = wy * 64 + lane;
    const int x0 = tx * 64, y0 = ty * TY, x = x0 + lane, yb = y0 + wy * RY;
    const int z0 = zc * nzb, z1 = min(z0 + nzb, sp.nz);
    const int64_t PY = sp.pitch_y, PZ = sp.pitch_z;
    const int64_t o = sp.offset;

    bool rl[RY], ro[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = x < sp.nx + R && yb + j < sp.ny + R;
        ro[j] = x < sp.nx && yb + j < sp.ny;
    }
    int64_t hyo[HY], hxo[HX];
    int hys[HY], hxs[HX];
    bool hyk[HY], hxk[HX];
#pragma unroll
    for (int k = 0; k < HY; ++k) {
        int yy, xx, ly, lx;
        hyk[k] = yring<R, TY>(tid + k * NT, y0, x0, yy, xx, ly, lx);
        hyk[k] = hyk[k] && yy < sp.ny + R && xx < sp.nx + R;
        hyo[k] = hyk[k] ? (int64_t)yy * PY + xx : 0;
        hys[k] = ly * 64 + lx;
    }
#pragma unroll
    for (int k = 0; k < HX; ++k) {
        int yy, xx, ly, lx;
        hxk[k] = xring<R, TY>(tid + k * NT, y0, x0, yy, xx, ly, lx);
        hxk[k] = hxk[k] && yy < sp.ny + R && xx < sp.nx + R;
        hxo[k] = hxk[k] ? (int64_t)yy * PY + xx : 0;
        hxs[k] = ly * LX + lx;
    }

    float qw[RY][2 * R + 1], qs[RY][2 * R + 1];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int64_t col = o + (int64_t)(yb + j) * PY + x;
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int64_t i = col + (int64_t)(z0 - R + k) * PZ;
            qw[j][k + 1] = rl[j] ? w0[i] : 0.0f;
            qs[j][k + 1] = rl[j] ? s0[i] : 0.0f;
        }
    }
    // prefetched plane: queue fronts, centre rows of w1 s1 w2 s2, rings,
    // and the point operands of the update
    float fw[RY], fs[RY], c1w[RY], c1s[RY], c2w[RY], c2s[RY];
    float fpc[RY], fpm[RY], frc[RY], frm[RY], fc[RY], fcp[RY], fcx[RY];
    float hw1[HY], hs1[HY], hw2[HX], hs2[HX];
    auto prefetch = [&](const int z) {
        const int64_t pz = o + (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t i = pz + (int64_t)(yb + j) * PY + x;
            fw[j] = rl[j] ? w0[i + R * PZ] : 0.0f;
            fs[j] = rl[j] ? s0[i + R * PZ] : 0.0f;
            c1w[j] = rl[j] ? w1[i] : 0.0f;
            c1s[j] = rl[j] ? s1[i] : 0.0f;
            c2w[j] = rl[j] ? w2[i] : 0.0f;
            c2s[j] = rl[j] ? s2[i] : 0.0f;
            fpc[j] = ro[j] ? __builtin_nontemporal_load(p + i) : 0.0f;
            fpm[j] = ro[j] ? __builtin_nontemporal_load(pm + i) : 0.0f;
            frc[j] = ro[j] ? __builtin_nontemporal_load(r + i) : 0.0f;
            frm[j] = ro[j] ? __builtin_nontemporal_load(rm + i) : 0.0f;
            fc[j] = ro[j] ? __builtin_nontemporal_load(c + i) : 0.0f;
            fcp[j] = ro[j] ? __builtin_nontemporal_load(cpp + i) : 0.0f;
            fcx[j] = ro[j] ? __builtin_nontemporal_load(cx + i) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < HY; ++k) {
            hw1[k] = hyk[k] ? w1[pz + hyo[k]] : 0.0f;
            hs1[k] = hyk[k] ? s1[pz + hyo[k]] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < HX; ++k) {
            hw2[k] = hxk[k] ? w2[pz + hxo[k]] : 0.0f;
            hs2[k] = hxk[k] ? s2[pz + hxo[k]] : 0.0f;
        }
    };
    if (z0 < z1) prefetch(z0);

    const float ax = sp.nbl > 0 ? sponge_ax(sp, 2, x, sp.gx) : 0.0f;
    for (int z = z0; z < z1; ++z) {
        float pc[RY], pmv[RY], rc[RY], rmv[RY], cc[RY], cp[RY], cxx[RY];
        float *t1w = lw1[z & 1], *t1s = ls1[z & 1], *t2w = lw2[z & 1], *t2s = ls2[z & 1];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                qw[j][k] = qw[j][k + 1];
                qs[j][k] = qs[j][k + 1];
            }
            qw[j][2 * R] = fw[j];
            qs[j][2 * R] = fs[j];
            const int ly = wy * RY + j;
            t1w[(ly + R) * 64 + lane] = c1w[j];
            t1s[(ly + R) * 64 + lane] = c1s[j];
            t2w[ly * LX + lane + R] = c2w[j];
            t2s[ly * LX + lane + R] = c2s[j];
            pc[j] = fpc[j];
            pmv[j] = fpm[j];
            rc[j] = frc[j];
            rmv[j] = frm[j];
            cc[j] = fc[j];
            cp[j] = fcp[j];
            cxx[j] = fcx[j];
        }
#pragma unroll
        for (int k = 0; k < HY; ++k)
            if (tid + k * NT < 2 * R * 64) {
                t1w[hys[k]] = hw1[k];
                t1s[hys[k]] = hs1[k];
            }
#pragma unroll
        for (int k = 0; k < HX; ++k)
            if (tid + k * NT < 2 * R * TY) {
                t2w[hxs[k]] = hw2[k];
                t2s[hxs[k]] = hs2[k];
            }
        if (z + 1 < z1) prefetch(z + 1);
        __syncthreads();

        const float az = sp.nbl > 0 ? sponge_ax(sp, 0, z, sp.gz) : 0.0f;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int ly = wy * RY + j;
            const float *a1w = t1w + (ly + R) * 64 + lane, *a1s = t1s + (ly + R) * 64 + lane;
            const float *a2w = t2w + ly * LX + lane + R, *a2s = t2s + ly * LX + lane + R;
            float h1 = 0.f, h2 = 0.f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const float dz = sp.dz[k - 1], dy = sp.dy[k - 1], dx = sp.dx[k - 1];
                h1 += dz * (qw[j][R + k] - qw[j][R - k]) + dy * (a1w[k * 64] - a1w[-k * 64]) +
                      dx * (a2w[k] - a2w[-k]);
                h2 += dz * (qs[j][R + k] - qs[j][R - k]) + dy * (a1s[k * 64] - a1s[-k * 64]) +
                      dx * (a2s[k] - a2s[-k]);
            }
            const int y = yb + j;
            // same summation order as damp_a(): (z + x) + y
            const float ayy = sp.nbl > 0 ? sponge_ax(sp, 1, y, sp.gy) : 0.0f;
            const float a = sp.half_dt * ((az + ax) + ayy);
            const float inv = 1.0f / (1.0f + a);
            const float pn = pc[j] + ((1.0f - a) * (pc[j] - pmv[j]) + cp[j] * h1 + cxx[j] * h2) * inv;
            const float rn = rc[j] + ((1.0f - a) * (rc[j] - rmv[j]) + cxx[j] * h1 + cc[j] * h2) * inv;
            if (ro[j]) {
                const int64_t i = o + (int64_t)z * PZ + (int64_t)y * PY + x;
                __builtin_nontemporal_store(pn, pp + i);
                __builtin_nontemporal_store(rn, rp + i);
            }
        }
    }
}

template <int R>
static void tti_zm_r(const fd_grid *g, const float *p, const float *pm, float *pp, const float *r,
                     const float *rm, float *rp, hipStream_t s)
{
    const StepParams &sp = g->sp;
    constexpr int TY = kTtiBy * kTtiRy;
    const int nzb = g->tune.nzb > 0 ? g->tune.nzb : 32;
    const int ntx = (sp.nx + 63) / 64, nty = (sp.ny + TY - 1) / TY, nzc = (sp.nz + nzb - 1) / nzb;
    const unsigned nb = (unsigned)ntx * nty * nzc;
    float *const *w = g->inter;
    hipLaunchKernelGGL((k_tti_grad_zm<R>), dim3(nb), dim3(64, kTtiBy), 0, s, p, r, g->tti[2],
                       g->tti[3], w[0], w[1], w[2], w[3], w[4], w[5], sp, ntx, nty, nzb);
    hipLaunchKernelGGL((k_tti_div_zm<R>), dim3(nb), dim3(64, kTtiBy), 0, s, p, pm, pp, r, rm, rp,
                       w[0], w[1], w[2], w[3], w[4], w[5], g->vdt2, g->tti[0], g->tti[1], sp, ntx,
                       nty, nzb);
}

int launch_tti_step_zm(const fd_grid *g, const float *p, const float *pm, float *pp,
                       const float *r, const float *rm, float *rp, hipStream_t s)
{
    switch (g->r) {
    case 2: tti_zm_r<2>(g, p, pm, pp, r, rm, rp, s); break;
    case 3: tti_zm_r<3>(g, p, pm, pp, r, rm, rp, s); break;
    case 4: tti_zm_r<4>(g, p, pm, pp, r, rm, rp, s); break;
    case 5: tti_zm_r<5>(g, p, pm, pp, r, rm, rp, s); break;
    case 6: tti_zm_r<6>(g, p, pm, pp, r, rm, rp, s); break;
    default: return set_error(FD_EINVAL, "TTI supports space orders 4..12");
    }
    return check_launch("TTI step (z-march)");
}

}  // namespace fd
