// The z-marching body of the 3-D acoustic step, shared by the single-grid
// kernel (k_acoustic.hip) and the batched multi-shot kernel (k_batch.hip).
//
// A block of 64 x BY threads owns a 64 x (BY*RY) column tile and marches
// along z over one chunk of nzb planes.  Each thread keeps the 2R+1 z values
// of its RY columns in registers (a queue shifted once per plane), so every
// u value enters the chip once per chunk; the current plane plus an R-wide
// x/y ring is staged in LDS, double buffered (one barrier per plane).  Loads
// for plane z+1 are issued before plane z is computed.
#pragma once

#include "fd_internal.h"

namespace fd {

template <int R, int BY, int RY, int CX = 1>
struct ZTile {
    static constexpr int TX = 64 * CX, TY = BY * RY, LX = TX + 2 * R, LY = TY + 2 * R;
    static constexpr int LDS = 2 * LY * LX;   // floats, double buffered
};

// One block's z-march over tile (tx, ty) and z chunk zc of the box that p
// describes (a whole DOMAIN, or a sub-box whose x columns below p.xlo are
// read but not written); u -> up with up possibly aliasing um (in place).  `lds` holds
// ZTile<R,BY,RY>::LDS floats.  PF planes of loads are kept in flight ahead of
// the plane being computed; NTS stores u+ with the non-temporal hint (it is
// not read again in this step).
template <int R, int BY, int RY, int PF, bool NTS>
__device__ __forceinline__ void zmarch_body(const float *__restrict__ u, const float *um,
                                            float *up, const float *__restrict__ vdt2,
                                            const StepParams &p, const int tx, const int ty,
                                            const int zc, const int nzb, float *lds)
{
    constexpr int TX = 64, TY = BY * RY, LX = TX + 2 * R, LY = TY + 2 * R;
    constexpr int NT = 64 * BY;
    constexpr int NHY = 2 * R * TX;   // y-halo values per plane
    constexpr int NHX = 2 * R * TY;   // x-halo values per plane
    constexpr int HY = (NHY + NT - 1) / NT;
    constexpr int HX = (NHX + NT - 1) / NT;
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

    // which of this thread's rows are loadable (inside the launch box plus
    // its R-wide rim) and which are written (inside the box, x >= p.xlo)
    const bool xl = x >= p.xlo - R && x < p.nx + R;
    const bool xw = x >= p.xlo && x < p.nx;
    bool rl[RY], ro[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = xl && (yb + j) < p.ny + R;
        ro[j] = xw && (yb + j) < p.ny;
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
        hyk[k] = e < NHY && yy < p.ny + R && xx >= p.xlo - R && xx < p.nx + R;
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
        hxk[k] = e < NHX && yy < p.ny + R && xx >= p.xlo - R && xx < p.nx + R;
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

    // PF slots of prefetched loads; slot d holds plane z with z - z0 == d mod PF
    float nf[PF][RY], nm[PF][RY], nv[PF][RY], nhy[PF][HY], nhx[PF][HX];
    auto prefetch = [&](const int z, const int d) {
        const int64_t pz = (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t col = (int64_t)(yb + j) * PY + x;
            nf[d][j] = rl[j] ? uo[pz + R * PZ + col] : 0.0f;
            nm[d][j] = ro[j] ? umo[pz + col] : 0.0f;
            nv[d][j] = ro[j] ? vo[pz + col] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < HY; ++k) nhy[d][k] = hyk[k] ? uo[pz + hyo[k]] : 0.0f;
#pragma unroll
        for (int k = 0; k < HX; ++k) nhx[d][k] = hxk[k] ? uo[pz + hxo[k]] : 0.0f;
    };
#pragma unroll
    for (int d = 0; d < PF; ++d)
        if (z0 + d < z1) prefetch(z0 + d, d);

    const float ax = p.nbl > 0 ? sponge_ax(p, 2, x, p.gx) : 0.0f;
    for (int zb = z0; zb < z1; zb += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            const int z = zb + d;
            if (z < z1) {
                float cm[RY], cv[RY], chy[HY], chx[HX];
#pragma unroll
                for (int j = 0; j < RY; ++j) {
#pragma unroll
                    for (int k = 0; k < 2 * R; ++k) q[j][k] = q[j][k + 1];
                    q[j][2 * R] = nf[d][j];
                    cm[j] = nm[d][j];
                    cv[j] = nv[d][j];
                }
#pragma unroll
                for (int k = 0; k < HY; ++k) chy[k] = nhy[d][k];
#pragma unroll
                for (int k = 0; k < HX; ++k) chx[k] = nhx[d][k];
                if (z + PF < z1) prefetch(z + PF, d);

                float *t = lds + (z & 1) * (LY * LX);
#pragma unroll
                for (int j = 0; j < RY; ++j) t[(wy * RY + j + R) * LX + lane + R] = q[j][R];
#pragma unroll
                for (int k = 0; k < HY; ++k)
                    if (tid + k * NT < NHY) t[hys[k]] = chy[k];
#pragma unroll
                for (int k = 0; k < HX; ++k)
                    if (tid + k * NT < NHX) t[hxs[k]] = chx[k];
                __syncthreads();

                const float az = p.nbl > 0 ? sponge_ax(p, 0, z, p.gz) : 0.0f;
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
                    const float ay = p.nbl > 0 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
                    const float a = p.half_dt * ((az + ax) + ay);
                    const float val = leapfrog_update(uc, cm[j], cv[j], lap, a);
                    if (ro[j]) {
                        float *dst = upo + (int64_t)z * PZ + (int64_t)y * PY + x;
                        if (NTS) __builtin_nontemporal_store(val, dst);
                        else *dst = val;
                    }
                }
            }
        }
    }
}

}  // namespace fd

namespace fd {

// ---------------------------------------------------------------------------
// Variant with the halo loads moved R planes earlier.  In the plain body a
// tile reads the x/y halo of plane z when it computes plane z, R iterations
// after its neighbours streamed plane z in as their queue front -- by then
// L2 has usually evicted it, so the halo costs HBM traffic.  Here the halo
// of plane z + R + 1 is issued in the same iteration as the neighbours'
// front loads of that plane and parked in a register ring of R + 1 planes
// until it is written to LDS; the streamed fields (u-, v^2 dt^2, u+) carry
// the non-temporal hint when NTS is set so they do not evict u from L2.
// With CX = 2 every lane owns two columns 64 apart (a 128-wide tile), which
// halves the share of x-halo cache lines per tile row.
//
// The march is addressed through buffer resources.
// Every access is a buffer load or store with a per-plane descriptor (base at
// the plane's row -R, column -R; as many bytes as the padded plane holds
// from there) and a 32-bit per-lane offset that stays fixed over the march.
// Lanes whose point is not loaded (or not written) carry an offset beyond the
// descriptor's range: the hardware returns 0 for such a load and drops such
// a store, so the hot loop has no per-lane branches and no 64-bit address
// arithmetic, and the compiler can count the memory operations in flight
// exactly between the waits.
// ---------------------------------------------------------------------------
constexpr uint32_t kBufOOB = 0xFFFFFFF0u;     // beyond every plane descriptor
constexpr int kBufWord3 = 0x00020000;         // gfx9 raw buffer: 32-bit data format

struct PlaneBuf {
    const char *b0;      // byte address of plane 0, row -R, column -R
    int64_t pz;          // bytes per plane
    int32_t nrec;        // bytes a plane descriptor covers
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t at(const int z) const
    {
        return __builtin_amdgcn_make_buffer_rsrc((void *)(b0 + (int64_t)z * pz), (short)0, nrec,
                                                 kBufWord3);
    }
};

__device__ __forceinline__ PlaneBuf plane_buf(const float *field, const StepParams &p, int R)
{
    PlaneBuf b;
    b.b0 = reinterpret_cast<const char *>(field + p.offset - (int64_t)R * p.pitch_y - R);
    b.pz = p.pitch_z * (int64_t)sizeof(float);
    b.nrec = (int32_t)(((int64_t)(p.ny + 2 * R) * p.pitch_y) * (int64_t)sizeof(float));
    return b;
}

// AUX is the cache policy: 0 default, 2 non-temporal
template <int AUX = 0>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}

template <int AUX = 0>
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, AUX);
}

// Extra per-point work of a batched gradient's steps (template EPI of
// zmarch_buf_body): EPI 1, a recomputed forward step also writes the
// imaging factor of its update, D = (u+ - 2u + u-)/dt^2 + gamma (u+ - u-)/(2 dt),
// to field d; EPI 2, an adjoint step also applies the imaging condition to
// its input field lambda with a stored D: g -= lambda D.
struct StepImaging {
    float *d;
    float *g;
    float inv_dt2, inv_2dt;
};

// LEND (whole zero-halo grids only, never a sub-box): the lanes past the last
// DOMAIN column of a row, up to the end of its 128-byte line, store 0 into
// every written field (zero halo, then row padding), so that the row's last
// line is stored whole rather than in part.
template <int R, int BY, int RY, bool NTS, int CX = 1, int EPI = 0, bool LEND = false>
__device__ __forceinline__ void zmarch_buf_body(const float *__restrict__ u, const float *um,
                                                float *up, const float *__restrict__ vdt2,
                                                const StepParams &p, const int tx, const int ty,
                                                const int zc, const int nzb, float *lds,
                                                const StepImaging img = StepImaging{})
{
    constexpr int TX = 64 * CX, TY = BY * RY, LX = TX + 2 * R, LY = TY + 2 * R;
    constexpr int NT = 64 * BY;
    constexpr int NHY = 2 * R * TX;
    constexpr int NHX = 2 * R * TY;
    constexpr int HY = (NHY + NT - 1) / NT;
    constexpr int HX = (NHX + NT - 1) / NT;
    constexpr int NR = R + 1;                 // halo ring depth (planes)
    constexpr int NTA = NTS ? 2 : 0;          // non-temporal cache policy
    const int lane = threadIdx.x, wy = threadIdx.y;
    const int tid = wy * 64 + lane;
    const int x0 = tx * TX, y0 = ty * TY;
    const int yb = y0 + wy * RY;
    const int z0 = zc * nzb;
    const int z1 = min(z0 + nzb, p.nz);
    const int PY = (int)p.pitch_y;
    const PlaneBuf Bu = plane_buf(u, p, R), Bm = plane_buf(um, p, R), Bv = plane_buf(vdt2, p, R),
                   Bp = plane_buf(up, p, R);
    const PlaneBuf Bd = plane_buf(EPI ? img.d : up, p, R), Bg = plane_buf(EPI == 2 ? img.g : up, p, R);
    // byte offset of in-plane point (y, x) from the plane descriptor's base
    auto boff = [&](const int y, const int x) -> uint32_t {
        return (uint32_t)(((y + R) * PY + (x + R)) * (int)sizeof(float));
    };

    int xs[CX];
    uint32_t ol[CX][RY], ow[CX][RY];          // load / store offsets (OOB if masked)
    bool zr[CX][RY];                          // LEND: a line-end lane, stores 0
#pragma unroll
    for (int c = 0; c < CX; ++c) {
        xs[c] = x0 + lane + 64 * c;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const bool rl = xs[c] >= p.xlo - R && xs[c] < p.nx + R && (yb + j) < p.ny + R;
            const bool ro = xs[c] >= p.xlo && xs[c] < p.nx && (yb + j) < p.ny;
            ol[c][j] = rl ? boff(yb + j, xs[c]) : kBufOOB;
            const bool le = LEND && !ro && xs[c] >= p.nx && xs[c] < ((p.nx + 31) & ~31) &&
                            (yb + j) < p.ny;
            zr[c][j] = le;
            ow[c][j] = ro || le ? boff(yb + j, xs[c]) : kBufOOB;
        }
    }
    uint32_t hyo[HY], hxo[HX];
    int hys[HY], hxs[HX];
#pragma unroll
    for (int k = 0; k < HY; ++k) {
        const int e = tid + k * NT;
        const int row = e / TX, col = e % TX;
        const int yy = row < R ? y0 - R + row : y0 + TY + (row - R);
        const int ly = row < R ? row : TY + row;
        const int xx = x0 + col;
        const bool ok = e < NHY && yy < p.ny + R && xx >= p.xlo - R && xx < p.nx + R;
        hyo[k] = ok ? boff(yy, xx) : kBufOOB;
        hys[k] = e < NHY ? ly * LX + col + R : -1;
    }
#pragma unroll
    for (int k = 0; k < HX; ++k) {
        const int e = tid + k * NT;
        const int row = e / (2 * R), c = e % (2 * R);
        const int yy = y0 + row;
        const int xx = c < R ? x0 - R + c : x0 + TX + (c - R);
        const int lx = c < R ? c : TX + c;
        const bool ok = e < NHX && yy < p.ny + R && xx >= p.xlo - R && xx < p.nx + R;
        hxo[k] = ok ? boff(yy, xx) : kBufOOB;
        hxs[k] = e < NHX ? (row + R) * LX + lx : -1;
    }

    // z queue of each column, NR - 1 slots longer than the 2R + 1 planes the
    // stencil reads, so that it shifts once per unrolled block of NR planes:
    // plane d of a block reads q[d .. d + 2R] (centre q[d + R]); its front
    // q[d + 2R] is loaded during plane d - 1 straight into its slot (into nf
    // for the block's first plane)
    constexpr int QL = 2 * R + NR;
    float q[CX][RY][QL];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
        const __amdgpu_buffer_rsrc_t r = Bu.at(z0 - R + k);
#pragma unroll
        for (int c = 0; c < CX; ++c)
#pragma unroll
            for (int j = 0; j < RY; ++j) q[c][j][k] = bload(r, ol[c][j]);
    }
    float hy[NR][HY], hx[NR][HX];
    auto load_halo = [&](const int z, const int d) {
        const __amdgpu_buffer_rsrc_t r = Bu.at(z);
#pragma unroll
        for (int k = 0; k < HY; ++k) hy[d][k] = bload(r, hyo[k]);
#pragma unroll
        for (int k = 0; k < HX; ++k) hx[d][k] = bload(r, hxo[k]);
    };
#pragma unroll
    for (int d = 0; d < NR; ++d)
        if (z0 + d < z1) load_halo(z0 + d, d);
    float nf[CX][RY], nm[CX][RY], nv[CX][RY], nd[CX][RY], ng[CX][RY];
    // the point operands of plane z (the queue front is loaded by the caller)
    auto prefetch = [&](const int z) {
        const __amdgpu_buffer_rsrc_t rm = Bm.at(z), rv = Bv.at(z);
#pragma unroll
        for (int c = 0; c < CX; ++c)
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                nm[c][j] = bload<NTA>(rm, ow[c][j]);
                nv[c][j] = bload<NTA>(rv, ow[c][j]);
            }
        if constexpr (EPI == 2) {
            const __amdgpu_buffer_rsrc_t rd = Bd.at(z), rg = Bg.at(z);
#pragma unroll
            for (int c = 0; c < CX; ++c)
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    nd[c][j] = bload<NTA>(rd, ow[c][j]);
                    ng[c][j] = bload<NTA>(rg, ow[c][j]);
                }
        }
    };
    if (z0 < z1) {
        const __amdgpu_buffer_rsrc_t rf = Bu.at(z0 + R);
#pragma unroll
        for (int c = 0; c < CX; ++c)
#pragma unroll
            for (int j = 0; j < RY; ++j) nf[c][j] = bload(rf, ol[c][j]);
        prefetch(z0);
    }

    float ax[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c)
        ax[c] = p.nbl > 0 ? sponge_ax(p, 2, xs[c], p.gx) : 0.0f;
    for (int zb = z0; zb < z1; zb += NR) {
#pragma unroll
        for (int d = 0; d < NR; ++d) {
            const int z = zb + d;
            if (z < z1) {
                float cm[CX][RY], cv[CX][RY], cd[CX][RY], cg[CX][RY];
#pragma unroll
                for (int c = 0; c < CX; ++c)
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        if (d == 0) q[c][j][2 * R] = nf[c][j];
                        cm[c][j] = nm[c][j];
                        cv[c][j] = nv[c][j];
                        if constexpr (EPI == 2) {
                            cd[c][j] = nd[c][j];
                            cg[c][j] = ng[c][j];
                        }
                    }
                if (z + 1 < z1) {
                    // front of plane z + 1: its queue slot, or nf across blocks
                    const __amdgpu_buffer_rsrc_t rf = Bu.at(z + 1 + R);
#pragma unroll
                    for (int c = 0; c < CX; ++c)
#pragma unroll
                        for (int j = 0; j < RY; ++j) {
                            if (d + 1 < NR) q[c][j][2 * R + d + 1] = bload(rf, ol[c][j]);
                            else nf[c][j] = bload(rf, ol[c][j]);
                        }
                    prefetch(z + 1);
                }
                float *t = lds + (z & 1) * (LY * LX);
#pragma unroll
                for (int c = 0; c < CX; ++c)
#pragma unroll
                    for (int j = 0; j < RY; ++j)
                        t[(wy * RY + j + R) * LX + lane + 64 * c + R] = q[c][j][d + R];
#pragma unroll
                for (int k = 0; k < HY; ++k)
                    if (NHY % NT == 0 || tid + k * NT < NHY) t[hys[k]] = hy[d][k];
#pragma unroll
                for (int k = 0; k < HX; ++k)
                    if (NHX % NT == 0 || tid + k * NT < NHX) t[hxs[k]] = hx[d][k];
                if (z + NR < z1) load_halo(z + NR, d);
                __syncthreads();

                const float az = p.nbl > 0 ? sponge_ax(p, 0, z, p.gz) : 0.0f;
                const __amdgpu_buffer_rsrc_t rp = Bp.at(z);
#pragma unroll
                for (int c = 0; c < CX; ++c)
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        const float *cc = t + (wy * RY + j + R) * LX + lane + 64 * c + R;
                        float lz = 0.0f, ly = 0.0f, lx = 0.0f;
#pragma unroll
                        for (int k = 1; k <= R; ++k) {
                            lz += p.cz[k] * (q[c][j][d + R + k] + q[c][j][d + R - k]);
                            ly += p.cy[k] * (cc[k * LX] + cc[-k * LX]);
                            lx += p.cx[k] * (cc[k] + cc[-k]);
                        }
                        const float uc = q[c][j][d + R];
                        const float lap = p.c0 * uc + lz + ly + lx;
                        const int y = yb + j;
                        const float ay = p.nbl > 0 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
                        const float gam = (az + ax[c]) + ay;
                        const float a = p.half_dt * gam;
                        const float un = leapfrog_update(uc, cm[c][j], cv[c][j], lap, a);
                        bstore<NTA>(LEND && zr[c][j] ? 0.0f : un, rp, ow[c][j]);
                        if constexpr (EPI == 1) {
                            const float um1 = cm[c][j];
                            const float dv = ((un - uc) - (uc - um1)) * img.inv_dt2 +
                                             gam * (un - um1) * img.inv_2dt;
                            bstore<NTA>(LEND && zr[c][j] ? 0.0f : dv, Bd.at(z), ow[c][j]);
                        }
                        if constexpr (EPI == 2) {
                            const float gv = cg[c][j] - uc * cd[c][j];
                            bstore<NTA>(LEND && zr[c][j] ? 0.0f : gv, Bg.at(z), ow[c][j]);
                        }
                    }
            }
        }
        // the next block's window starts NR planes further
#pragma unroll
        for (int c = 0; c < CX; ++c)
#pragma unroll
            for (int j = 0; j < RY; ++j)
#pragma unroll
                for (int k = 0; k < 2 * R; ++k) q[c][j][k] = q[c][j][k + NR];
    }
}

}  // namespace fd
