// One-kernel pseudo-acoustic TTI step (paper, appendix "Anisotropic acoustic
// (TTI)", equation (rot); the two-field system and the rotated operators are
// described in k_tti.hip):
//
//   p+ = p + [(1-a)(p - p-) + c_pp H_xy p + c_x H_z r] / (1 + a)
//   r+ = r + [(1-a)(r - r-) + c_x  H_xy p + c   H_z r] / (1 + a)
//   H_xy p = div w,  w = (I - a a^T) grad p;    H_z r = div s,  s = a (a . grad r)
//
// in one z-march that never writes w or s to memory.  A block of 512 threads
// owns a TX x TY column tile (TX = 64 or 32, TY = (512 / TX) CPT: CPT tile
// columns per thread) and a chunk of nzb output planes.  At march step t:
//
//   * each thread holds p and r of planes t-2R .. t in register queues for
//     its "cross" columns: its tile columns, and a share of the R-wide ring of
//     columns left/right of the tile (tile rows) and above/below it (tile
//     columns) that the divergence reads;
//   * p and r of plane zg = t - R go to an LDS plane over the cross region
//     plus a further 2R rim (loaded directly), for the x and y derivatives;
//   * every cross column forms grad p, grad r at zg and projects them on the
//     symmetry axis; x components go to LDS over the tile and x ring, y
//     components over the tile and y ring;
//   * each tile column adds the in-plane divergence of plane zg to its own
//     slot of a register ring of 2R+1 accumulators and scatters the z
//     components to the slots of the planes within R;
//   * plane zo = t - 2R is then complete, and the coupled update writes p+, r+.
//
// Intermediates are zero outside DOMAIN, as in the two-pass kernels, so the
// divergence stays the exact negative transpose of the gradient.  The axis
// a = (a_z, a_y, a_x) comes precomputed from the model stage (no sincos in
// the march).  Each block
// marches nzb + 4R planes (2R of queue warm-up, 2R of drain) for nzb outputs.
// Every access goes through per-plane buffer descriptors (zmarch.h): planes
// outside the padded field get an empty one, masked columns an offset past
// the plane, so loads return zero and stores drop without per-lane branches.
//
// It moves 48 B/pt against the two passes' 100, but it is bound by vector
// ALU work, not by HBM: every ring column repeats the six R-term
// derivatives, the projections and the queue shifts of a tile column, and at
// R = 6 the ring of a 64 x 8 tile holds 1.7 times as many columns as the
// tile.  At 384^3, so 12, it measured 2.07 ms per step against 1.22 ms for
// the two passes (about 800 vector instructions per thread and step), so
// the two passes stay the default and this kernel is selected by a tile flag.
#include "zmarch.h"

namespace fd {

namespace {

constexpr int kFusedNt = 512;

// descriptor of padded plane z, empty outside [-R, nz + R)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t fused_plane(const PlaneBuf &b, int z, int R,
                                                              int nz)
{
    const bool in = z >= -R && z < nz + R;
    return __builtin_amdgcn_make_buffer_rsrc((void *)(b.b0 + (int64_t)(in ? z : 0) * b.pz),
                                             (short)0, in ? b.nrec : 0, kBufWord3);
}

}  // namespace

template <int R, int CPT, int TX>
__global__ __launch_bounds__(kFusedNt) void k_tti_fused(
    const float *__restrict__ p, const float *pm, float *pp, const float *__restrict__ r,
    const float *rm, float *rp, const float *__restrict__ faz, const float *__restrict__ fay,
    const float *__restrict__ fax, const float *__restrict__ c, const float *__restrict__ cpp,
    const float *__restrict__ cx, const StepParams sp, const int ntx, const int nty,
    const int nzb)
{
    constexpr int NT = kFusedNt, TY = (NT / TX) * CPT;
    constexpr int RXN = TX + 4 * R, RYN = TY + 4 * R;  // p, r plane with its 2R rim
    constexpr int XN = TX + 2 * R, YN = TY + 2 * R;    // x and y component planes
    constexpr int NRING = 2 * R * TX + 2 * R * TY;
    constexpr int NRS = (NRING + NT - 1) / NT;         // ring slots per thread
    constexpr int NS = CPT + NRS;                      // cross slots per thread
    constexpr int NRIM = 2 * R * TX + 4 * R * R + 2 * R * TY;
    constexpr int NMS = (NRIM + NT - 1) / NT;          // rim slots per thread
    constexpr int Q = 2 * R + 1;
    __shared__ float lp[RYN * RXN], lr[RYN * RXN];
    __shared__ float xw[TY * XN], xs[TY * XN], yw[YN * TX], ys[YN * TX];

    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int tid = threadIdx.y * 64 + threadIdx.x;
    const int tcx = tid % TX, tcy = tid / TX;        // this thread's tile column
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = zc * nzb, z1 = min(z0 + nzb, sp.nz);
    const int NZ = sp.nz, NY = sp.ny, NX = sp.nx;
    const int PY = (int)sp.pitch_y;
    const PlaneBuf Bp = plane_buf(p, sp, R), Br = plane_buf(r, sp, R),
                   Bz = plane_buf(faz, sp, R), By = plane_buf(fay, sp, R),
                   Bx = plane_buf(fax, sp, R), Bpm = plane_buf(pm, sp, R),
                   Brm = plane_buf(rm, sp, R), Bc = plane_buf(c, sp, R),
                   Bcp = plane_buf(cpp, sp, R), Bcx = plane_buf(cx, sp, R),
                   Bpp = plane_buf(pp, sp, R), Brp = plane_buf(rp, sp, R);
    // in-plane byte offset of (y, x); outside the padded rows and columns it
    // lies past every plane descriptor
    auto boff = [&](const int y, const int x) -> uint32_t {
        if (y < -R || y >= NY + R || x < -R || x >= NX + R) return kBufOOB;
        return (uint32_t)(((y + R) * PY + (x + R)) * (int)sizeof(float));
    };
    auto lidx = [&](const int y, const int x) { return (y - y0 + 2 * R) * RXN + (x - x0 + 2 * R); };

    // cross slots: s < CPT the tile columns (y0 + tcy CPT + s, x0 + tcx);
    // then ring slots e = tid + (s - CPT) NT: y ring (2R rows of TX), x ring
    // (TY rows of 2R).  kind: 0 tile, 1 y ring, 2 x ring, -1 idle
    int cyy[NS], cxx[NS], kind[NS], cl[NS], dst[NS];
    uint32_t co[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int yy = 0, x = 0, k = -1;
        if (s < CPT) {
            yy = y0 + tcy * CPT + s;
            x = x0 + tcx;
            k = 0;
        } else {
            const int e = tid + (s - CPT) * NT;
            if (e < 2 * R * TX) {
                const int row = e / TX;
                yy = row < R ? y0 - R + row : y0 + TY + (row - R);
                x = x0 + e % TX;
                k = 1;
            } else if (e < NRING) {
                const int i = e - 2 * R * TX;
                const int row = i / (2 * R), cc = i % (2 * R);
                yy = y0 + row;
                x = cc < R ? x0 - R + cc : x0 + TX + (cc - R);
                k = 2;
            }
        }
        cyy[s] = yy;
        cxx[s] = x;
        kind[s] = k;
        co[s] = k >= 0 ? boff(yy, x) : kBufOOB;
        cl[s] = k >= 0 ? lidx(yy, x) : 0;
        // x-component slot (tile, x ring) or y-component slot (y ring)
        dst[s] = k == 1 ? (yy - y0 + R) * TX + (x - x0) : (yy - y0) * XN + (x - x0 + R);
    }
    // rim of the p, r plane: far rows above/below the y ring, the four
    // R x R corners, far columns beyond the x ring
    uint32_t mo[NMS];
    int ml[NMS];
#pragma unroll
    for (int s = 0; s < NMS; ++s) {
        const int e = tid + s * NT;
        int yy = 0, x = 0;
        bool ok = true;
        if (e < 2 * R * TX) {
            const int row = e / TX;
            yy = row < R ? y0 - 2 * R + row : y0 + TY + R + (row - R);
            x = x0 + e % TX;
        } else if (e < 2 * R * TX + 4 * R * R) {
            const int i = e - 2 * R * TX, q = i / (R * R), j = i % (R * R);
            yy = (q < 2 ? y0 - R : y0 + TY) + j / R;
            x = ((q & 1) == 0 ? x0 - R : x0 + TX) + j % R;
        } else if (e < NRIM) {
            const int i = e - 2 * R * TX - 4 * R * R;
            const int row = i / (2 * R), cc = i % (2 * R);
            yy = y0 + row;
            x = cc < R ? x0 - 2 * R + cc : x0 + TX + R + (cc - R);
        } else {
            ok = false;
        }
        mo[s] = ok ? boff(yy, x) : kBufOOB;
        ml[s] = ok ? lidx(yy, x) : -1;
    }
    // output offsets of the tile columns (DOMAIN only)
    uint32_t ot[CPT];
    float ayd[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const bool in = cyy[j] < NY && cxx[j] < NX;
        ot[j] = in ? boff(cyy[j], cxx[j]) : kBufOOB;
        ayd[j] = sp.nbl > 0 ? sponge_ax(sp, 1, cyy[j], sp.gy) : 0.0f;
    }
    const float axd = sp.nbl > 0 ? sponge_ax(sp, 2, x0 + tcx, sp.gx) : 0.0f;

    // queues: qp[s][k] = p(t - 2R + k) at cross column s
    float qp[NS][Q], qr[NS][Q];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
        const int z = z0 - 2 * R + k;
        const auto dp = fused_plane(Bp, z, R, NZ), dr = fused_plane(Br, z, R, NZ);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            qp[s][k + 1] = bload(dp, co[s]);
            qr[s][k + 1] = bload(dr, co[s]);
        }
    }
    // divergence accumulators of the tile columns: slot j is plane zg - R + j
    float aw[CPT][Q], as[CPT][Q];
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int k = 0; k < Q; ++k) aw[j][k] = as[j][k] = 0.0f;

    // prefetched operands of step t: queue fronts (plane t), the axis and
    // the rim (plane t - R), the update operands (plane t - 2R)
    float fp[NS], fr[NS], fz[NS], fy[NS], fx[NS], hp[NMS], hr[NMS];
    float upm[CPT], urm[CPT], uc[CPT], ucp[CPT], ucx[CPT];
    auto prefetch = [&](const int t) {
        const int zg = t - R, zo = t - 2 * R;
        const auto dp = fused_plane(Bp, t, R, NZ), dr = fused_plane(Br, t, R, NZ);
        const auto dz = fused_plane(Bz, zg, R, NZ), dy = fused_plane(By, zg, R, NZ),
                   dx = fused_plane(Bx, zg, R, NZ);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            fp[s] = bload(dp, co[s]);
            fr[s] = bload(dr, co[s]);
            fz[s] = bload(dz, co[s]);
            fy[s] = bload(dy, co[s]);
            fx[s] = bload(dx, co[s]);
        }
        const auto gp = fused_plane(Bp, zg, R, NZ), gr = fused_plane(Br, zg, R, NZ);
#pragma unroll
        for (int s = 0; s < NMS; ++s) {
            hp[s] = bload(gp, mo[s]);
            hr[s] = bload(gr, mo[s]);
        }
        const bool live = zo >= z0;
        const int zq = live ? zo : z0;
        const auto e0 = fused_plane(Bpm, zq, R, NZ), e1 = fused_plane(Brm, zq, R, NZ),
                   e2 = fused_plane(Bc, zq, R, NZ), e3 = fused_plane(Bcp, zq, R, NZ),
                   e4 = fused_plane(Bcx, zq, R, NZ);
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const uint32_t o = live ? ot[j] : kBufOOB;
            upm[j] = bload<2>(e0, o);
            urm[j] = bload<2>(e1, o);
            uc[j] = bload<2>(e2, o);
            ucp[j] = bload<2>(e3, o);
            ucx[j] = bload<2>(e4, o);
        }
    };
    const int tend = z1 + 2 * R;
    if (z0 < z1) prefetch(z0);

    for (int t = z0; t < tend; ++t) {
        const int zg = t - R, zo = t - 2 * R;
        float az[NS], ay[NS], ax[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                qp[s][k] = qp[s][k + 1];
                qr[s][k] = qr[s][k + 1];
            }
            qp[s][2 * R] = fp[s];
            qr[s][2 * R] = fr[s];
            az[s] = fz[s];
            ay[s] = fy[s];
            ax[s] = fx[s];
        }
        float rp_[NMS], rr_[NMS];
#pragma unroll
        for (int s = 0; s < NMS; ++s) {
            rp_[s] = hp[s];
            rr_[s] = hr[s];
        }
        float vpm[CPT], vrm[CPT], vc[CPT], vcp[CPT], vcx[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            vpm[j] = upm[j];
            vrm[j] = urm[j];
            vc[j] = uc[j];
            vcp[j] = ucp[j];
            vcx[j] = ucx[j];
        }
        if (t + 1 < tend) prefetch(t + 1);

        // p, r of plane zg: queue centres of the cross columns, and the rim
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (kind[s] >= 0) {
                lp[cl[s]] = qp[s][R];
                lr[cl[s]] = qr[s][R];
            }
#pragma unroll
        for (int s = 0; s < NMS; ++s)
            if (ml[s] >= 0) {
                lp[ml[s]] = rp_[s];
                lr[ml[s]] = rr_[s];
            }
        __syncthreads();

        // rotated gradients at the cross columns of plane zg
        const bool zin = zg >= 0 && zg < NZ;
        float wz[CPT], sz[CPT];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (kind[s] < 0) continue;
            const float *cp = lp + cl[s], *cr = lr + cl[s];
            float gpz = 0.f, gpy = 0.f, gpx = 0.f, grz = 0.f, gry = 0.f, grx = 0.f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const float dz = sp.dz[k - 1], dy = sp.dy[k - 1], dx = sp.dx[k - 1];
                gpz += dz * (qp[s][R + k] - qp[s][R - k]);
                gpy += dy * (cp[k * RXN] - cp[-k * RXN]);
                gpx += dx * (cp[k] - cp[-k]);
                grz += dz * (qr[s][R + k] - qr[s][R - k]);
                gry += dy * (cr[k * RXN] - cr[-k * RXN]);
                grx += dx * (cr[k] - cr[-k]);
            }
            const float ap = az[s] * gpz + ay[s] * gpy + ax[s] * gpx;
            const float ar = az[s] * grz + ay[s] * gry + ax[s] * grx;
            const bool in = zin && cyy[s] >= 0 && cyy[s] < NY && cxx[s] >= 0 && cxx[s] < NX;
            if (s < CPT) {
                xw[dst[s]] = in ? gpx - ax[s] * ap : 0.0f;
                xs[dst[s]] = in ? ax[s] * ar : 0.0f;
                const int l = (cyy[s] - y0 + R) * TX + tcx;
                yw[l] = in ? gpy - ay[s] * ap : 0.0f;
                ys[l] = in ? ay[s] * ar : 0.0f;
                wz[s] = in ? gpz - az[s] * ap : 0.0f;
                sz[s] = in ? az[s] * ar : 0.0f;
            } else if (kind[s] == 1) {
                yw[dst[s]] = in ? gpy - ay[s] * ap : 0.0f;
                ys[dst[s]] = in ? ay[s] * ar : 0.0f;
            } else {
                xw[dst[s]] = in ? gpx - ax[s] * ap : 0.0f;
                xs[dst[s]] = in ? ax[s] * ar : 0.0f;
            }
        }
        __syncthreads();

        const float azd = sp.nbl > 0 && zo >= 0 ? sponge_ax(sp, 0, zo, sp.gz) : 0.0f;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            // in-plane divergence of plane zg into its own slot; z components
            // scattered to the planes within R
            const int ly = cyy[j] - y0;
            const float *pxw = xw + ly * XN + tcx + R, *pxs = xs + ly * XN + tcx + R;
            const float *pyw = yw + (ly + R) * TX + tcx, *pys = ys + (ly + R) * TX + tcx;
            float hw = 0.0f, hs = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const float dy = sp.dy[k - 1], dx = sp.dx[k - 1];
                hw += dy * (pyw[k * TX] - pyw[-k * TX]) + dx * (pxw[k] - pxw[-k]);
                hs += dy * (pys[k * TX] - pys[-k * TX]) + dx * (pxs[k] - pxs[-k]);
            }
            aw[j][R] += hw;
            as[j][R] += hs;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const float dz = sp.dz[k - 1];
                aw[j][R - k] += dz * wz[j];
                as[j][R - k] += dz * sz[j];
                aw[j][R + k] -= dz * wz[j];
                as[j][R + k] -= dz * sz[j];
            }
            // plane zo is complete
            if (zo >= z0) {
                // same summation order as damp_a(): (z + x) + y
                const float a = sp.half_dt * ((azd + axd) + ayd[j]);
                const float inv = 1.0f / (1.0f + a);
                const float h1 = aw[j][0], h2 = as[j][0];
                const float pc = qp[j][0], rc = qr[j][0];
                const float pn = pc + ((1.0f - a) * (pc - vpm[j]) + vcp[j] * h1 + vcx[j] * h2) * inv;
                const float rn = rc + ((1.0f - a) * (rc - vrm[j]) + vcx[j] * h1 + vc[j] * h2) * inv;
                bstore<2>(pn, fused_plane(Bpp, zo, R, NZ), ot[j]);
                bstore<2>(rn, fused_plane(Brp, zo, R, NZ), ot[j]);
            }
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                aw[j][k] = aw[j][k + 1];
                as[j][k] = as[j][k + 1];
            }
            aw[j][2 * R] = as[j][2 * R] = 0.0f;
        }
    }
}

template <int R, int CPT, int TX>
static void tti_fused_r(const fd_grid *g, const float *p, const float *pm, float *pp,
                        const float *r, const float *rm, float *rp, int nzb, hipStream_t s)
{
    const StepParams &sp = g->sp;
    constexpr int TY = (kFusedNt / TX) * CPT;
    const int ntx = (sp.nx + TX - 1) / TX, nty = (sp.ny + TY - 1) / TY,
              nzc = (sp.nz + nzb - 1) / nzb;
    const unsigned nb = (unsigned)ntx * nty * nzc;
    hipLaunchKernelGGL((k_tti_fused<R, CPT, TX>), dim3(nb), dim3(64, kFusedNt / 64), 0, s, p, pm,
                       pp, r, rm, rp, g->tti[4], g->tti[5], g->tti[6], g->vdt2, g->tti[0],
                       g->tti[1], sp, ntx, nty, nzb);
}

template <int R, int TX>
static void tti_fused_c(const fd_grid *g, const float *p, const float *pm, float *pp,
                        const float *r, const float *rm, float *rp, int cpt, int nzb,
                        hipStream_t s)
{
    // two columns per thread only where the queues still fit in registers
    if constexpr (R <= 3) {
        if (cpt >= 2) {
            tti_fused_r<R, 2, TX>(g, p, pm, pp, r, rm, rp, nzb, s);
            return;
        }
    }
    tti_fused_r<R, 1, TX>(g, p, pm, pp, r, rm, rp, nzb, s);
}

template <int R>
static void tti_fused_x(const fd_grid *g, const float *p, const float *pm, float *pp,
                        const float *r, const float *rm, float *rp, int tx, int cpt, int nzb,
                        hipStream_t s)
{
    if (tx == 32) tti_fused_c<R, 32>(g, p, pm, pp, r, rm, rp, cpt, nzb, s);
    else tti_fused_c<R, 64>(g, p, pm, pp, r, rm, rp, cpt, nzb, s);
}

// tile: by = 16 selects 32-wide tiles (otherwise 64-wide), ry = 2 two tile
// columns per thread, nzb the z chunk
int launch_tti_step_fused(const fd_grid *g, const float *p, const float *pm, float *pp,
                          const float *r, const float *rm, float *rp, hipStream_t s)
{
    const int tx = g->tune.by == 16 ? 32 : 64;
    const int cpt = g->tune.ry >= 2 ? 2 : 1;
    const int nzb = g->tune.nzb > 0 ? g->tune.nzb : 64;
    switch (g->r) {
    case 2: tti_fused_x<2>(g, p, pm, pp, r, rm, rp, tx, cpt, nzb, s); break;
    case 3: tti_fused_x<3>(g, p, pm, pp, r, rm, rp, tx, cpt, nzb, s); break;
    case 4: tti_fused_x<4>(g, p, pm, pp, r, rm, rp, tx, cpt, nzb, s); break;
    case 5: tti_fused_x<5>(g, p, pm, pp, r, rm, rp, tx, cpt, nzb, s); break;
    case 6: tti_fused_x<6>(g, p, pm, pp, r, rm, rp, tx, cpt, nzb, s); break;
    default: return set_error(FD_EINVAL, "TTI supports space orders 4..12");
    }
    return check_launch("TTI step (one z-march)");
}

}  // namespace fd
