// Isotropic elastic velocity-stress kernels for gfx950 (paper, appendix
// "Isotropic elastic", equation (elas1)): v_t = b div(tau),
// tau_t = lambda tr(grad v) I + mu (grad v + grad v^T), b = 1/rho.
//
// Staggered grid (Virieux): storage index (z, y, x) holds vx at x+1/2,
// vy at y+1/2, vz at z+1/2, txx/tyy/tzz at the node, txy at (y+1/2, x+1/2),
// txz at (z+1/2, x+1/2), tyz at (z+1/2, y+1/2).  Two staggered first
// derivatives of order 2R, c_k / h per axis in StepParams.s{z,y,x}:
//   dp: sum_k c_k (f[i+k] - f[i-k+1])   node -> half point
//   dm: sum_k c_k (f[i+k-1] - f[i-k])   half point -> node
// One update is two in-place passes: velocities from the stresses, then
// stresses from the new velocities (each pass reads the other set only at
// neighbours and its own set only at the point it writes, so in place is
// safe).  Damping w+ = [(1 - a) w + dt rhs] / (1 + a) with the acoustic
// sponge a = gamma dt / 2 at the storage index.  The medium arrives
// premultiplied by dt at each component's position (k_el_model).
//
// Bytes per point and update: velocity pass reads 3 v, 6 tau, 3 b and
// writes 3 v (60 B); stress pass reads 6 tau, 3 v, 5 moduli and writes 6 tau
// (80 B).  Memory-bound, no contraction: no MFMA.
#include "fd_internal.h"

namespace fd {

namespace {

struct ElState {
    float *f[9];        // vx, vy, vz, txx, tyy, tzz, txy, txz, tyz
};

struct ElMedium {
    float *m[8];        // b dt at vx, vy, vz; lambda dt, mu dt; mu dt at txy, txz, tyz
};

enum { VX, VY, VZ, TXX, TYY, TZZ, TXY, TXZ, TYZ };
enum { M_BX, M_BY, M_BZ, M_LAM, M_MU, M_MXY, M_MXZ, M_MYZ };

template <int R>
__device__ __forceinline__ float dp(const float *__restrict__ f, const int64_t i, const int64_t s,
                                    const float *c)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) acc += c[k - 1] * (f[i + k * s] - f[i - (k - 1) * s]);
    return acc;
}

template <int R>
__device__ __forceinline__ float dm(const float *__restrict__ f, const int64_t i, const int64_t s,
                                    const float *c)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) acc += c[k - 1] * (f[i + (k - 1) * s] - f[i - k * s]);
    return acc;
}

__device__ __forceinline__ float damped(float w, float rhs, float a)
{
    return ((1.0f - a) * w + rhs) / (1.0f + a);
}

// ---------------------------------------------------------------------------
// medium
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_el_model(const float *__restrict__ vp,
                                                  const float *__restrict__ vs,
                                                  const float *__restrict__ rho, ElMedium med,
                                                  unsigned *flags, const StepParams p,
                                                  const float dt)
{
    const int64_t n = (int64_t)p.nz * p.ny * p.nx;
    const int64_t SY = p.nx, SZ = (int64_t)p.ny * p.nx;
    unsigned mx = 0u, bad = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % p.nx);
        const int64_t t = i / p.nx;
        const int y = (int)(t % p.ny);
        const int z = (int)(t / p.ny);
        // dense offsets of the next node along each axis (the last repeats)
        const int64_t ox = x + 1 < p.nx ? 1 : 0;
        const int64_t oy = y + 1 < p.ny ? SY : 0;
        const int64_t oz = z + 1 < p.nz ? SZ : 0;
        auto b = [&](int64_t j) { return 1.0f / rho[j]; };
        auto mu = [&](int64_t j) { return rho[j] * vs[j] * vs[j]; };
        const float a = vp[i], s = vs[i], r = rho[i];
        const float m0 = r * s * s;
        const int64_t j = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x;
        med.m[M_BX][j] = 0.5f * (b(i) + b(i + ox)) * dt;
        med.m[M_BY][j] = 0.5f * (b(i) + b(i + oy)) * dt;
        med.m[M_BZ][j] = 0.5f * (b(i) + b(i + oz)) * dt;
        med.m[M_LAM][j] = (r * a * a - 2.0f * m0) * dt;
        med.m[M_MU][j] = m0 * dt;
        med.m[M_MXY][j] = 0.25f * (m0 + mu(i + ox) + mu(i + oy) + mu(i + ox + oy)) * dt;
        med.m[M_MXZ][j] = 0.25f * (m0 + mu(i + ox) + mu(i + oz) + mu(i + ox + oz)) * dt;
        med.m[M_MYZ][j] = 0.25f * (m0 + mu(i + oy) + mu(i + oz) + mu(i + oy + oz)) * dt;
        // positive floats order like their bit patterns; flag <= 0 / NaN as +inf
        const unsigned bits = (a > 0.0f) ? __float_as_uint(a) : 0x7f800000u;
        mx = bits > mx ? bits : mx;
        if (!(r > 0.0f) || !(s >= 0.0f) || !(4.0f * s * s < 3.0f * a * a)) bad = 1u;
    }
    atomicMax(flags, mx);
    if (bad) atomicOr(flags + 1, 1u);
}

// ---------------------------------------------------------------------------
// one thread per point
// ---------------------------------------------------------------------------

template <int R>
__global__ __launch_bounds__(256) void k_el_velocity_pt(ElState st, const ElMedium med,
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
    const float a = damp_a(p, z, y, x);
    const float rx = dp<R>(st.f[TXX], i, 1, p.sx) + dm<R>(st.f[TXY], i, PY, p.sy) +
                     dm<R>(st.f[TXZ], i, PZ, p.sz);
    const float ry = dm<R>(st.f[TXY], i, 1, p.sx) + dp<R>(st.f[TYY], i, PY, p.sy) +
                     dm<R>(st.f[TYZ], i, PZ, p.sz);
    const float rz = dm<R>(st.f[TXZ], i, 1, p.sx) + dm<R>(st.f[TYZ], i, PY, p.sy) +
                     dp<R>(st.f[TZZ], i, PZ, p.sz);
    st.f[VX][i] = damped(st.f[VX][i], med.m[M_BX][i] * rx, a);
    st.f[VY][i] = damped(st.f[VY][i], med.m[M_BY][i] * ry, a);
    st.f[VZ][i] = damped(st.f[VZ][i], med.m[M_BZ][i] * rz, a);
}

template <int R>
__global__ __launch_bounds__(256) void k_el_stress_pt(ElState st, const ElMedium med,
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
    const float a = damp_a(p, z, y, x);
    const float *vx = st.f[VX], *vy = st.f[VY], *vz = st.f[VZ];
    const float exx = dm<R>(vx, i, 1, p.sx), eyy = dm<R>(vy, i, PY, p.sy),
                ezz = dm<R>(vz, i, PZ, p.sz);
    const float lt = med.m[M_LAM][i] * ((exx + eyy) + ezz);
    const float m2 = 2.0f * med.m[M_MU][i];
    st.f[TXX][i] = damped(st.f[TXX][i], lt + m2 * exx, a);
    st.f[TYY][i] = damped(st.f[TYY][i], lt + m2 * eyy, a);
    st.f[TZZ][i] = damped(st.f[TZZ][i], lt + m2 * ezz, a);
    st.f[TXY][i] = damped(st.f[TXY][i],
                          med.m[M_MXY][i] * (dp<R>(vx, i, PY, p.sy) + dp<R>(vy, i, 1, p.sx)), a);
    st.f[TXZ][i] = damped(st.f[TXZ][i],
                          med.m[M_MXZ][i] * (dp<R>(vx, i, PZ, p.sz) + dp<R>(vz, i, 1, p.sx)), a);
    st.f[TYZ][i] = damped(st.f[TYZ][i],
                          med.m[M_MYZ][i] * (dp<R>(vy, i, PZ, p.sz) + dp<R>(vz, i, PY, p.sy)), a);
}

// ---------------------------------------------------------------------------
// z-marching passes
//
// A block of 64 x BY threads owns a 64 x (BY*RY) column tile and marches
// along a chunk of nzb planes.  Fields differentiated along z travel in
// per-thread register queues of 2R+1 planes; fields differentiated along x
// or y are staged plane by plane in LDS with an R-wide rim (double
// buffered, one barrier per plane).  The next plane's loads are issued
// before the current plane is computed.  The point's own fields (the
// components it updates and its medium) are streamed with the non-temporal
// hint.  Sums, damping and updates are those of the one-thread-per-point
// kernels, term for term.
//
// velocity pass: queues txz, tyz, tzz; LDS txx (x rim), txy (x and y),
//                txz (x), tyy (y), tyz (y)
// stress pass:   queues vx, vy, vz; LDS vx, vy, vz (x and y rims)
// ---------------------------------------------------------------------------

template <int R, int BY, int RY>
struct ElZm {
    static constexpr int TX = 64, TY = BY * RY, LX = TX + 2 * R, LY = TY + 2 * R, PL = LY * LX;
    static constexpr int NT = 64 * BY;
    static constexpr int NHY = 2 * R * TX, NHX = 2 * R * TY;
    static constexpr int HY = (NHY + NT - 1) / NT, HX = (NHX + NT - 1) / NT;
};

// Offsets (within a plane, from the DOMAIN origin), LDS slots and in-range
// flags of this thread's share of a tile's y rim and x rim.
template <int R, int BY, int RY>
struct ElRim {
    using T = ElZm<R, BY, RY>;
    int64_t yo[T::HY], xo[T::HX];
    int ys[T::HY], xs[T::HX];
    bool yk[T::HY], xk[T::HX];

    __device__ __forceinline__ ElRim(const StepParams &p, const int x0, const int y0, const int tid)
    {
#pragma unroll
        for (int k = 0; k < T::HY; ++k) {
            const int e = tid + k * T::NT;
            const int row = e / T::TX, col = e % T::TX;
            const int yy = row < R ? y0 - R + row : y0 + T::TY + (row - R);
            const int ly = row < R ? row : T::TY + row;
            const int xx = x0 + col;
            yk[k] = e < T::NHY && yy < p.ny + R && xx < p.nx + R;
            yo[k] = (int64_t)yy * p.pitch_y + xx;
            ys[k] = ly * T::LX + col + R;
        }
#pragma unroll
        for (int k = 0; k < T::HX; ++k) {
            const int e = tid + k * T::NT;
            const int row = e / (2 * R), c = e % (2 * R);
            const int yy = y0 + row;
            const int xx = c < R ? x0 - R + c : x0 + T::TX + (c - R);
            const int lx = c < R ? c : T::TX + c;
            xk[k] = e < T::NHX && yy < p.ny + R && xx < p.nx + R;
            xo[k] = (int64_t)yy * p.pitch_y + xx;
            xs[k] = (row + R) * T::LX + lx;
        }
    }
};

template <bool NT_>
__device__ __forceinline__ float ld(const float *p)
{
    if constexpr (NT_) return __builtin_nontemporal_load(p);
    else return *p;
}

// staggered sums over LDS (stride 1 or LX) and over a z queue (centre R)
template <int R, int S>
__device__ __forceinline__ float dp_l(const float *c, const float *w)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) acc += w[k - 1] * (c[k * S] - c[-(k - 1) * S]);
    return acc;
}

template <int R, int S>
__device__ __forceinline__ float dm_l(const float *c, const float *w)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) acc += w[k - 1] * (c[(k - 1) * S] - c[-k * S]);
    return acc;
}

template <int R>
__device__ __forceinline__ float dp_q(const float *q, const float *w)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) acc += w[k - 1] * (q[R + k] - q[R - (k - 1)]);
    return acc;
}

template <int R>
__device__ __forceinline__ float dm_q(const float *q, const float *w)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) acc += w[k - 1] * (q[R + (k - 1)] - q[R - k]);
    return acc;
}

template <int R, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_el_velocity_zm(ElState st, const ElMedium med,
                                                            const StepParams p, const int ntx,
                                                            const int nty, const int nzb)
{
    using T = ElZm<R, BY, RY>;
    constexpr int Q = 2 * R + 1;
    __shared__ float lds[2][5][T::PL];   // txx, txy, txz, tyy, tyz
    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int lane = threadIdx.x, wy = threadIdx.y, tid = wy * 64 + lane;
    const int x0 = tx * T::TX, y0 = ty * T::TY, x = x0 + lane, yb = y0 + wy * RY;
    const int z0 = zc * nzb, z1 = min(z0 + nzb, p.nz);
    const int64_t PZ = p.pitch_z, PY = p.pitch_y;
    const float *fxx = st.f[TXX] + p.offset, *fxy = st.f[TXY] + p.offset,
                *fxz = st.f[TXZ] + p.offset, *fyy = st.f[TYY] + p.offset,
                *fyz = st.f[TYZ] + p.offset, *fzz = st.f[TZZ] + p.offset;
    float *vx = st.f[VX] + p.offset, *vy = st.f[VY] + p.offset, *vz = st.f[VZ] + p.offset;
    const float *bx = med.m[M_BX] + p.offset, *by = med.m[M_BY] + p.offset,
                *bz = med.m[M_BZ] + p.offset;
    bool rl[RY], ro[RY];
    int64_t col[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = x < p.nx + R && yb + j < p.ny + R;
        ro[j] = x < p.nx && yb + j < p.ny;
        col[j] = (int64_t)(yb + j) * PY + x;
    }
    const ElRim<R, BY, RY> rim(p, x0, y0, tid);

    float qxz[RY][Q], qyz[RY][Q], qzz[RY][Q];
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int64_t o = (int64_t)(z0 - R + k) * PZ + col[j];
            qxz[j][k + 1] = rl[j] ? fxz[o] : 0.0f;
            qyz[j][k + 1] = rl[j] ? fyz[o] : 0.0f;
            qzz[j][k + 1] = rl[j] ? fzz[o] : 0.0f;
        }
    // loads of one plane: queue fronts (z + R), LDS centres, rims, own fields
    float nfxz[RY], nfyz[RY], nfzz[RY], ncxx[RY], ncxy[RY], ncyy[RY];
    float nv[3][RY], nb[3][RY];
    float nyh[3][T::HY], nxh[3][T::HX];   // y rims of txy, tyy, tyz; x rims of txx, txy, txz
    auto prefetch = [&](const int z) {
        const int64_t pz = (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t o = pz + col[j];
            nfxz[j] = rl[j] ? fxz[o + R * PZ] : 0.0f;
            nfyz[j] = rl[j] ? fyz[o + R * PZ] : 0.0f;
            nfzz[j] = rl[j] ? fzz[o + R * PZ] : 0.0f;
            ncxx[j] = rl[j] ? fxx[o] : 0.0f;
            ncxy[j] = rl[j] ? fxy[o] : 0.0f;
            ncyy[j] = rl[j] ? fyy[o] : 0.0f;
            nv[0][j] = ro[j] ? ld<true>(vx + o) : 0.0f;
            nv[1][j] = ro[j] ? ld<true>(vy + o) : 0.0f;
            nv[2][j] = ro[j] ? ld<true>(vz + o) : 0.0f;
            nb[0][j] = ro[j] ? ld<true>(bx + o) : 0.0f;
            nb[1][j] = ro[j] ? ld<true>(by + o) : 0.0f;
            nb[2][j] = ro[j] ? ld<true>(bz + o) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < T::HY; ++k) {
            nyh[0][k] = rim.yk[k] ? fxy[pz + rim.yo[k]] : 0.0f;
            nyh[1][k] = rim.yk[k] ? fyy[pz + rim.yo[k]] : 0.0f;
            nyh[2][k] = rim.yk[k] ? fyz[pz + rim.yo[k]] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < T::HX; ++k) {
            nxh[0][k] = rim.xk[k] ? fxx[pz + rim.xo[k]] : 0.0f;
            nxh[1][k] = rim.xk[k] ? fxy[pz + rim.xo[k]] : 0.0f;
            nxh[2][k] = rim.xk[k] ? fxz[pz + rim.xo[k]] : 0.0f;
        }
    };
    if (z0 < z1) prefetch(z0);

    const float ax = p.nbl > 0 ? sponge_ax(p, 2, x, p.gx) : 0.0f;
    for (int z = z0; z < z1; ++z) {
        float cxx[RY], cxy[RY], cyy[RY], cv[3][RY], cb[3][RY], cyh[3][T::HY], cxh[3][T::HX];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                qxz[j][k] = qxz[j][k + 1];
                qyz[j][k] = qyz[j][k + 1];
                qzz[j][k] = qzz[j][k + 1];
            }
            qxz[j][2 * R] = nfxz[j];
            qyz[j][2 * R] = nfyz[j];
            qzz[j][2 * R] = nfzz[j];
            cxx[j] = ncxx[j];
            cxy[j] = ncxy[j];
            cyy[j] = ncyy[j];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cv[c][j] = nv[c][j];
                cb[c][j] = nb[c][j];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k) cyh[c][k] = nyh[c][k];
#pragma unroll
            for (int k = 0; k < T::HX; ++k) cxh[c][k] = nxh[c][k];
        }
        if (z + 1 < z1) prefetch(z + 1);

        float(*L)[T::PL] = lds[z & 1];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int c = (wy * RY + j + R) * T::LX + lane + R;
            L[0][c] = cxx[j];
            L[1][c] = cxy[j];
            L[2][c] = qxz[j][R];
            L[3][c] = cyy[j];
            L[4][c] = qyz[j][R];
        }
#pragma unroll
        for (int k = 0; k < T::HY; ++k)
            if (tid + k * T::NT < T::NHY) {
                L[1][rim.ys[k]] = cyh[0][k];
                L[3][rim.ys[k]] = cyh[1][k];
                L[4][rim.ys[k]] = cyh[2][k];
            }
#pragma unroll
        for (int k = 0; k < T::HX; ++k)
            if (tid + k * T::NT < T::NHX) {
                L[0][rim.xs[k]] = cxh[0][k];
                L[1][rim.xs[k]] = cxh[1][k];
                L[2][rim.xs[k]] = cxh[2][k];
            }
        __syncthreads();

        const float az = p.nbl > 0 ? sponge_ax(p, 0, z, p.gz) : 0.0f;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int c = (wy * RY + j + R) * T::LX + lane + R;
            constexpr int LXs = T::LX;
            const float rx = dp_l<R, 1>(&L[0][c], p.sx) + dm_l<R, LXs>(&L[1][c], p.sy) +
                             dm_q<R>(qxz[j], p.sz);
            const float ry = dm_l<R, 1>(&L[1][c], p.sx) + dp_l<R, LXs>(&L[3][c], p.sy) +
                             dm_q<R>(qyz[j], p.sz);
            const float rz = dm_l<R, 1>(&L[2][c], p.sx) + dm_l<R, LXs>(&L[4][c], p.sy) +
                             dp_q<R>(qzz[j], p.sz);
            const int y = yb + j;
            const float ay = p.nbl > 0 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
            const float a = p.half_dt * ((az + ax) + ay);
            if (ro[j]) {
                const int64_t o = (int64_t)z * PZ + col[j];
                __builtin_nontemporal_store(damped(cv[0][j], cb[0][j] * rx, a), vx + o);
                __builtin_nontemporal_store(damped(cv[1][j], cb[1][j] * ry, a), vy + o);
                __builtin_nontemporal_store(damped(cv[2][j], cb[2][j] * rz, a), vz + o);
            }
        }
    }
}

template <int R, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_el_stress_zm(ElState st, const ElMedium med,
                                                          const StepParams p, const int ntx,
                                                          const int nty, const int nzb)
{
    using T = ElZm<R, BY, RY>;
    constexpr int Q = 2 * R + 1;
    __shared__ float lds[2][3][T::PL];   // vx, vy, vz
    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int lane = threadIdx.x, wy = threadIdx.y, tid = wy * 64 + lane;
    const int x0 = tx * T::TX, y0 = ty * T::TY, x = x0 + lane, yb = y0 + wy * RY;
    const int z0 = zc * nzb, z1 = min(z0 + nzb, p.nz);
    const int64_t PZ = p.pitch_z, PY = p.pitch_y;
    const float *fv[3] = {st.f[VX] + p.offset, st.f[VY] + p.offset, st.f[VZ] + p.offset};
    float *ft[6];
    const float *fm[5];
#pragma unroll
    for (int c = 0; c < 6; ++c) ft[c] = st.f[TXX + c] + p.offset;
#pragma unroll
    for (int c = 0; c < 5; ++c) fm[c] = med.m[M_LAM + c] + p.offset;
    bool rl[RY], ro[RY];
    int64_t col[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = x < p.nx + R && yb + j < p.ny + R;
        ro[j] = x < p.nx && yb + j < p.ny;
        col[j] = (int64_t)(yb + j) * PY + x;
    }
    const ElRim<R, BY, RY> rim(p, x0, y0, tid);

    float q[3][RY][Q];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < RY; ++j)
#pragma unroll
            for (int k = 0; k < 2 * R; ++k)
                q[c][j][k + 1] = rl[j] ? fv[c][(int64_t)(z0 - R + k) * PZ + col[j]] : 0.0f;
    float nf[3][RY], nt[6][RY], nm[5][RY], nyh[3][T::HY], nxh[3][T::HX];
    auto prefetch = [&](const int z) {
        const int64_t pz = (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t o = pz + col[j];
#pragma unroll
            for (int c = 0; c < 3; ++c) nf[c][j] = rl[j] ? fv[c][o + R * PZ] : 0.0f;
#pragma unroll
            for (int c = 0; c < 6; ++c) nt[c][j] = ro[j] ? ld<true>(ft[c] + o) : 0.0f;
#pragma unroll
            for (int c = 0; c < 5; ++c) nm[c][j] = ro[j] ? ld<true>(fm[c] + o) : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k)
                nyh[c][k] = rim.yk[k] ? fv[c][pz + rim.yo[k]] : 0.0f;
#pragma unroll
            for (int k = 0; k < T::HX; ++k)
                nxh[c][k] = rim.xk[k] ? fv[c][pz + rim.xo[k]] : 0.0f;
        }
    };
    if (z0 < z1) prefetch(z0);

    const float ax = p.nbl > 0 ? sponge_ax(p, 2, x, p.gx) : 0.0f;
    for (int z = z0; z < z1; ++z) {
        float ct[6][RY], cm[5][RY], cyh[3][T::HY], cxh[3][T::HX];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int k = 0; k < 2 * R; ++k) q[c][j][k] = q[c][j][k + 1];
                q[c][j][2 * R] = nf[c][j];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) ct[c][j] = nt[c][j];
#pragma unroll
            for (int c = 0; c < 5; ++c) cm[c][j] = nm[c][j];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k) cyh[c][k] = nyh[c][k];
#pragma unroll
            for (int k = 0; k < T::HX; ++k) cxh[c][k] = nxh[c][k];
        }
        if (z + 1 < z1) prefetch(z + 1);

        float(*L)[T::PL] = lds[z & 1];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int c = (wy * RY + j + R) * T::LX + lane + R;
#pragma unroll
            for (int f = 0; f < 3; ++f) L[f][c] = q[f][j][R];
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k)
                if (tid + k * T::NT < T::NHY) L[f][rim.ys[k]] = cyh[f][k];
#pragma unroll
            for (int k = 0; k < T::HX; ++k)
                if (tid + k * T::NT < T::NHX) L[f][rim.xs[k]] = cxh[f][k];
        }
        __syncthreads();

        const float az = p.nbl > 0 ? sponge_ax(p, 0, z, p.gz) : 0.0f;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int c = (wy * RY + j + R) * T::LX + lane + R;
            constexpr int LXs = T::LX;
            const float exx = dm_l<R, 1>(&L[0][c], p.sx), eyy = dm_l<R, LXs>(&L[1][c], p.sy),
                        ezz = dm_q<R>(q[2][j], p.sz);
            const float lt = cm[0][j] * ((exx + eyy) + ezz);
            const float m2 = 2.0f * cm[1][j];
            const float sxy = cm[2][j] * (dp_l<R, LXs>(&L[0][c], p.sy) + dp_l<R, 1>(&L[1][c], p.sx));
            const float sxz = cm[3][j] * (dp_q<R>(q[0][j], p.sz) + dp_l<R, 1>(&L[2][c], p.sx));
            const float syz = cm[4][j] * (dp_q<R>(q[1][j], p.sz) + dp_l<R, LXs>(&L[2][c], p.sy));
            const int y = yb + j;
            const float ay = p.nbl > 0 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
            const float a = p.half_dt * ((az + ax) + ay);
            if (ro[j]) {
                const int64_t o = (int64_t)z * PZ + col[j];
                __builtin_nontemporal_store(damped(ct[0][j], lt + m2 * exx, a), ft[0] + o);
                __builtin_nontemporal_store(damped(ct[1][j], lt + m2 * eyy, a), ft[1] + o);
                __builtin_nontemporal_store(damped(ct[2][j], lt + m2 * ezz, a), ft[2] + o);
                __builtin_nontemporal_store(damped(ct[3][j], sxy, a), ft[3] + o);
                __builtin_nontemporal_store(damped(ct[4][j], sxz, a), ft[4] + o);
                __builtin_nontemporal_store(damped(ct[5][j], syz, a), ft[5] + o);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// visco-elastic stress-memory pass (one relaxation mechanism; paper,
// appendix "Visco-elastic", equations (model-equations)).  With strain rates
// e from the new velocities, tr = exx + eyy + ezz, dev = e_ii - tr:
//   r_ii+ = r_ii - KS (r_ii + PD tr + 2 MD dev)
//   s_ii+ = [(1 - a) s_ii + PU tr + 2 MU dev + dt r_ii+] / (1 + a)
//   r_ij+ = r_ij - KS_ij (r_ij + MD_ij (e_ij + e_ji))
//   s_ij+ = [(1 - a) s_ij + MU_ij (e_ij + e_ji) + dt r_ij+] / (1 + a)
// PU = pi tau_ep/tau_s dt, MU = mu tau_es/tau_s dt (unrelaxed moduli),
// PD = pi (tau_ep/tau_s - 1), MD = mu (tau_es/tau_s - 1) (memory forcing),
// KS = dt / tau_s; at shear positions the means over the four nodes of the
// staggered plane.  Bytes per point: read 6 s, 6 r, 3 v, 14 coefficients;
// write 6 s, 6 r (164 B).
// ---------------------------------------------------------------------------

struct ViState {
    float *f[15];       // vx, vy, vz, txx, tyy, tzz, txy, txz, tyz, rxx, ryy, rzz, rxy, rxz, ryz
};

struct ViMedium {
    float *m[17];
};

enum { V_BX, V_BY, V_BZ, V_PU, V_MU, V_PD, V_MD, V_KS,
       V_MUXY, V_MDXY, V_KSXY, V_MUXZ, V_MDXZ, V_KSXZ, V_MUYZ, V_MDYZ, V_KSYZ };
enum { RXX = 9, RYY, RZZ, RXY, RXZ, RYZ };

__global__ __launch_bounds__(256) void k_vi_model(const float *__restrict__ vp,
                                                  const float *__restrict__ vs,
                                                  const float *__restrict__ rho,
                                                  const float *__restrict__ tep,
                                                  const float *__restrict__ tes,
                                                  const float *__restrict__ ts, ViMedium med,
                                                  unsigned *flags, const StepParams p,
                                                  const float dt)
{
    const int64_t n = (int64_t)p.nz * p.ny * p.nx;
    const int64_t SY = p.nx, SZ = (int64_t)p.ny * p.nx;
    unsigned mx = 0u, bad = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % p.nx);
        const int64_t t = i / p.nx;
        const int y = (int)(t % p.ny);
        const int z = (int)(t / p.ny);
        const int64_t ox = x + 1 < p.nx ? 1 : 0;
        const int64_t oy = y + 1 < p.ny ? SY : 0;
        const int64_t oz = z + 1 < p.nz ? SZ : 0;
        auto b = [&](int64_t j) { return 1.0f / rho[j]; };
        auto muu = [&](int64_t j) { return rho[j] * vs[j] * vs[j] * (tes[j] / ts[j]); };
        auto mud = [&](int64_t j) { return rho[j] * vs[j] * vs[j] * (tes[j] / ts[j] - 1.0f); };
        auto ks = [&](int64_t j) { return 1.0f / ts[j]; };
        const float a = vp[i], s = vs[i], r = rho[i];
        const float pi = r * a * a, mu = r * s * s;
        const int64_t j = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x;
        med.m[V_BX][j] = 0.5f * (b(i) + b(i + ox)) * dt;
        med.m[V_BY][j] = 0.5f * (b(i) + b(i + oy)) * dt;
        med.m[V_BZ][j] = 0.5f * (b(i) + b(i + oz)) * dt;
        med.m[V_PU][j] = pi * (tep[i] / ts[i]) * dt;
        med.m[V_MU][j] = mu * (tes[i] / ts[i]) * dt;
        med.m[V_PD][j] = pi * (tep[i] / ts[i] - 1.0f);
        med.m[V_MD][j] = mu * (tes[i] / ts[i] - 1.0f);
        med.m[V_KS][j] = dt / ts[i];
        const int64_t pl[3][2] = {{oy, ox}, {oz, ox}, {oz, oy}};   // xy, xz, yz planes
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int64_t u = pl[q][0], v = pl[q][1];
            med.m[V_MUXY + 3 * q][j] = 0.25f * (muu(i) + muu(i + u) + muu(i + v) + muu(i + u + v)) * dt;
            med.m[V_MDXY + 3 * q][j] = 0.25f * (mud(i) + mud(i + u) + mud(i + v) + mud(i + u + v));
            med.m[V_KSXY + 3 * q][j] = 0.25f * (ks(i) + ks(i + u) + ks(i + v) + ks(i + u + v)) * dt;
        }
        // unrelaxed P velocity against vmax; positive floats order like
        // their bit patterns, <= 0 / NaN flagged as +inf
        const float vpu = a * sqrtf(tep[i] / ts[i]);
        const unsigned bits = (vpu > 0.0f) ? __float_as_uint(vpu) : 0x7f800000u;
        mx = bits > mx ? bits : mx;
        if (!(r > 0.0f) || !(s >= 0.0f) || !(ts[i] >= dt) || !(tep[i] >= ts[i]) ||
            !(tes[i] >= ts[i]) || !(4.0f * s * s < 3.0f * a * a) ||
            !(4.0f * s * s * tes[i] < 3.0f * a * a * tep[i]))
            bad = 1u;
    }
    atomicMax(flags, mx);
    if (bad) atomicOr(flags + 1, 1u);
}

template <int R>
__global__ __launch_bounds__(256) void k_vi_stress_pt(ViState st, const ViMedium med,
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
    const float a = damp_a(p, z, y, x);
    const float dt = 2.0f * p.half_dt;
    const float *vx = st.f[VX], *vy = st.f[VY], *vz = st.f[VZ];
    const float e[3] = {dm<R>(vx, i, 1, p.sx), dm<R>(vy, i, PY, p.sy), dm<R>(vz, i, PZ, p.sz)};
    const float tr = (e[0] + e[1]) + e[2];
    const float pu = med.m[V_PU][i], mu = med.m[V_MU][i], pd = med.m[V_PD][i],
                md = med.m[V_MD][i], ks = med.m[V_KS][i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float dev = e[c] - tr;
        const float r0 = st.f[RXX + c][i];
        const float r1 = r0 - ks * (r0 + pd * tr + 2.0f * md * dev);
        st.f[RXX + c][i] = r1;
        st.f[TXX + c][i] = damped(st.f[TXX + c][i], pu * tr + 2.0f * mu * dev + dt * r1, a);
    }
    const float sh[3] = {dp<R>(vx, i, PY, p.sy) + dp<R>(vy, i, 1, p.sx),
                         dp<R>(vx, i, PZ, p.sz) + dp<R>(vz, i, 1, p.sx),
                         dp<R>(vy, i, PZ, p.sz) + dp<R>(vz, i, PY, p.sy)};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float r0 = st.f[RXY + c][i];
        const float r1 = r0 - med.m[V_KSXY + 3 * c][i] * (r0 + med.m[V_MDXY + 3 * c][i] * sh[c]);
        st.f[RXY + c][i] = r1;
        st.f[TXY + c][i] = damped(st.f[TXY + c][i], med.m[V_MUXY + 3 * c][i] * sh[c] + dt * r1, a);
    }
}

// The stress-memory pass as a z-march: queues of vx, vy, vz; LDS planes of
// vx, vy, vz with both rims; the point's six stresses, six memory
// variables and fourteen coefficients streamed with the non-temporal hint.
template <int R, int BY, int RY>
__global__ __launch_bounds__(64 * BY) void k_vi_stress_zm(ViState st, const ViMedium med,
                                                          const StepParams p, const int ntx,
                                                          const int nty, const int nzb)
{
    using T = ElZm<R, BY, RY>;
    constexpr int Q = 2 * R + 1;
    constexpr int NC = 14;                // coefficients V_PU .. V_KSYZ
    __shared__ float lds[2][3][T::PL];    // vx, vy, vz
    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int lane = threadIdx.x, wy = threadIdx.y, tid = wy * 64 + lane;
    const int x0 = tx * T::TX, y0 = ty * T::TY, x = x0 + lane, yb = y0 + wy * RY;
    const int z0 = zc * nzb, z1 = min(z0 + nzb, p.nz);
    const int64_t PZ = p.pitch_z, PY = p.pitch_y;
    const float dt = 2.0f * p.half_dt;
    const float *fv[3] = {st.f[VX] + p.offset, st.f[VY] + p.offset, st.f[VZ] + p.offset};
    float *fs[12];                        // txx .. tyz, rxx .. ryz
    const float *fm[NC];
#pragma unroll
    for (int c = 0; c < 12; ++c) fs[c] = st.f[TXX + c] + p.offset;
#pragma unroll
    for (int c = 0; c < NC; ++c) fm[c] = med.m[V_PU + c] + p.offset;
    bool rl[RY], ro[RY];
    int64_t col[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        rl[j] = x < p.nx + R && yb + j < p.ny + R;
        ro[j] = x < p.nx && yb + j < p.ny;
        col[j] = (int64_t)(yb + j) * PY + x;
    }
    const ElRim<R, BY, RY> rim(p, x0, y0, tid);

    float q[3][RY][Q];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < RY; ++j)
#pragma unroll
            for (int k = 0; k < 2 * R; ++k)
                q[c][j][k + 1] = rl[j] ? fv[c][(int64_t)(z0 - R + k) * PZ + col[j]] : 0.0f;
    float nf[3][RY], ns[12][RY], nm[NC][RY], nyh[3][T::HY], nxh[3][T::HX];
    auto prefetch = [&](const int z) {
        const int64_t pz = (int64_t)z * PZ;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t o = pz + col[j];
#pragma unroll
            for (int c = 0; c < 3; ++c) nf[c][j] = rl[j] ? fv[c][o + R * PZ] : 0.0f;
#pragma unroll
            for (int c = 0; c < 12; ++c) ns[c][j] = ro[j] ? ld<true>(fs[c] + o) : 0.0f;
#pragma unroll
            for (int c = 0; c < NC; ++c) nm[c][j] = ro[j] ? ld<true>(fm[c] + o) : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k)
                nyh[c][k] = rim.yk[k] ? fv[c][pz + rim.yo[k]] : 0.0f;
#pragma unroll
            for (int k = 0; k < T::HX; ++k)
                nxh[c][k] = rim.xk[k] ? fv[c][pz + rim.xo[k]] : 0.0f;
        }
    };
    if (z0 < z1) prefetch(z0);

    const float ax = p.nbl > 0 ? sponge_ax(p, 2, x, p.gx) : 0.0f;
    for (int z = z0; z < z1; ++z) {
        float cs[12][RY], cm[NC][RY], cyh[3][T::HY], cxh[3][T::HX];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int k = 0; k < 2 * R; ++k) q[c][j][k] = q[c][j][k + 1];
                q[c][j][2 * R] = nf[c][j];
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) cs[c][j] = ns[c][j];
#pragma unroll
            for (int c = 0; c < NC; ++c) cm[c][j] = nm[c][j];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k) cyh[c][k] = nyh[c][k];
#pragma unroll
            for (int k = 0; k < T::HX; ++k) cxh[c][k] = nxh[c][k];
        }
        if (z + 1 < z1) prefetch(z + 1);

        float(*L)[T::PL] = lds[z & 1];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int c = (wy * RY + j + R) * T::LX + lane + R;
#pragma unroll
            for (int f = 0; f < 3; ++f) L[f][c] = q[f][j][R];
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
#pragma unroll
            for (int k = 0; k < T::HY; ++k)
                if (tid + k * T::NT < T::NHY) L[f][rim.ys[k]] = cyh[f][k];
#pragma unroll
            for (int k = 0; k < T::HX; ++k)
                if (tid + k * T::NT < T::NHX) L[f][rim.xs[k]] = cxh[f][k];
        }
        __syncthreads();

        const float az = p.nbl > 0 ? sponge_ax(p, 0, z, p.gz) : 0.0f;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int c = (wy * RY + j + R) * T::LX + lane + R;
            constexpr int LXs = T::LX;
            const float e[3] = {dm_l<R, 1>(&L[0][c], p.sx), dm_l<R, LXs>(&L[1][c], p.sy),
                                dm_q<R>(q[2][j], p.sz)};
            const float tr = (e[0] + e[1]) + e[2];
            const float sh[3] = {dp_l<R, LXs>(&L[0][c], p.sy) + dp_l<R, 1>(&L[1][c], p.sx),
                                 dp_q<R>(q[0][j], p.sz) + dp_l<R, 1>(&L[2][c], p.sx),
                                 dp_q<R>(q[1][j], p.sz) + dp_l<R, LXs>(&L[2][c], p.sy)};
            const int y = yb + j;
            const float ay = p.nbl > 0 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
            const float a = p.half_dt * ((az + ax) + ay);
            // coefficient slots relative to V_PU
            const float pu = cm[0][j], mu = cm[1][j], pd = cm[2][j], md = cm[3][j], ks = cm[4][j];
            float outs[12];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const float dev = e[f] - tr;
                const float r0 = cs[6 + f][j];
                const float r1 = r0 - ks * (r0 + pd * tr + 2.0f * md * dev);
                outs[6 + f] = r1;
                outs[f] = damped(cs[f][j], pu * tr + 2.0f * mu * dev + dt * r1, a);
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const float r0 = cs[9 + f][j];
                const float r1 = r0 - cm[7 + 3 * f][j] * (r0 + cm[6 + 3 * f][j] * sh[f]);
                outs[9 + f] = r1;
                outs[3 + f] = damped(cs[3 + f][j], cm[5 + 3 * f][j] * sh[f] + dt * r1, a);
            }
            if (ro[j]) {
                const int64_t o = (int64_t)z * PZ + col[j];
#pragma unroll
                for (int f = 0; f < 12; ++f) __builtin_nontemporal_store(outs[f], fs[f] + o);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// explosive source and stress-trace receivers
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_el_sparse(ElState st, const StepParams p,
                                                   const SparseArgs inj, const SparseArgs smp)
{
    const int64_t PY = p.pitch_y, PZ = p.pitch_z;
    for (int e = threadIdx.x; e < inj.n * 8; e += blockDim.x) {
        const int pt = e / 8, c = e % 8;
        int z, y, x;
        float w;
        corner(3, inj.base + pt * 3, inj.frac + pt * 3, c, z, y, x, w);
        const int64_t i = p.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
        const float add = inj.scale * w * inj.vals[pt] / (1.0f + damp_a(p, z, y, x));
        atomicAdd(st.f[TXX] + i, add);
        atomicAdd(st.f[TYY] + i, add);
        atomicAdd(st.f[TZZ] + i, add);
    }
    __threadfence();
    __syncthreads();
    for (int pt = threadIdx.x; pt < smp.n; pt += blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < 8; ++c) {
            int z, y, x;
            float w;
            corner(3, smp.base + pt * 3, smp.frac + pt * 3, c, z, y, x, w);
            const int64_t i = p.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
            s += w * ((st.f[TXX][i] + st.f[TYY][i]) + st.f[TZZ][i]);
        }
        smp.out[pt] = smp.scale * s;
    }
}

ElState state_of(float *const *f)
{
    ElState st;
    for (int k = 0; k < 9; ++k) st.f[k] = f[k];
    return st;
}

ElMedium medium_of(const fd_grid *g)
{
    ElMedium m;
    for (int k = 0; k < 8; ++k) m.m[k] = g->el[k];
    return m;
}

template <int R>
void el_pass_r(const fd_grid *g, float *const *f, const bool stress, hipStream_t s)
{
    const StepParams &p = g->sp;
    if (g->tune.by > 0) {
        // z-marching passes, both on the handle's tile: 64 x 16 (8 waves, 2
        // rows per thread; the default), 64 x 8 (4 waves x 2 rows, or 8 waves
        // x 1).  The stress pass runs fastest on the velocity pass's tile and
        // chunk order (it then finds the fresh velocities of the last chunks
        // in the memory-side cache): mixing tiles measured 3 % slower.
        const int nzb = g->tune.nzb > 0 ? g->tune.nzb : 64;
        const int by = g->tune.by, ry = g->tune.ry;
        const int ntx = (p.nx + 63) / 64, nty = (p.ny + by * ry - 1) / (by * ry);
        const unsigned nb = (unsigned)ntx * nty * ((p.nz + nzb - 1) / nzb);
        if (by == 8 && ry == 2) {
            if (stress)
                hipLaunchKernelGGL((k_el_stress_zm<R, 8, 2>), dim3(nb), dim3(64, 8), 0, s,
                                   state_of(f), medium_of(g), p, ntx, nty, nzb);
            else
                hipLaunchKernelGGL((k_el_velocity_zm<R, 8, 2>), dim3(nb), dim3(64, 8), 0, s,
                                   state_of(f), medium_of(g), p, ntx, nty, nzb);
        } else if (by == 8) {
            if (stress)
                hipLaunchKernelGGL((k_el_stress_zm<R, 8, 1>), dim3(nb), dim3(64, 8), 0, s,
                                   state_of(f), medium_of(g), p, ntx, nty, nzb);
            else
                hipLaunchKernelGGL((k_el_velocity_zm<R, 8, 1>), dim3(nb), dim3(64, 8), 0, s,
                                   state_of(f), medium_of(g), p, ntx, nty, nzb);
        } else if (stress) {
            hipLaunchKernelGGL((k_el_stress_zm<R, 4, 2>), dim3(nb), dim3(64, 4), 0, s,
                               state_of(f), medium_of(g), p, ntx, nty, nzb);
        } else {
            hipLaunchKernelGGL((k_el_velocity_zm<R, 4, 2>), dim3(nb), dim3(64, 4), 0, s,
                               state_of(f), medium_of(g), p, ntx, nty, nzb);
        }
        return;
    }
    const int nxb = (p.nx + 63) / 64, nyb = (p.ny + 3) / 4;
    const unsigned nb = (unsigned)nxb * nyb * p.nz;
    if (stress)
        hipLaunchKernelGGL((k_el_stress_pt<R>), dim3(nb), dim3(64, 4), 0, s, state_of(f),
                           medium_of(g), p, nxb, nyb);
    else
        hipLaunchKernelGGL((k_el_velocity_pt<R>), dim3(nb), dim3(64, 4), 0, s, state_of(f),
                           medium_of(g), p, nxb, nyb);
}

int el_pass(const fd_grid *g, float *const *f, const bool stress, hipStream_t s)
{
    switch (g->r) {
    case 1: el_pass_r<1>(g, f, stress, s); break;
    case 2: el_pass_r<2>(g, f, stress, s); break;
    case 3: el_pass_r<3>(g, f, stress, s); break;
    case 4: el_pass_r<4>(g, f, stress, s); break;
    case 5: el_pass_r<5>(g, f, stress, s); break;
    case 6: el_pass_r<6>(g, f, stress, s); break;
    case 7: el_pass_r<7>(g, f, stress, s); break;
    case 8: el_pass_r<8>(g, f, stress, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    return check_launch(stress ? "elastic stress pass" : "elastic velocity pass");
}

ViState vstate_of(float *const *f)
{
    ViState st;
    for (int k = 0; k < 15; ++k) st.f[k] = f[k];
    return st;
}

ViMedium vmedium_of(const fd_grid *g)
{
    ViMedium m;
    for (int k = 0; k < 17; ++k) m.m[k] = g->el[k];
    return m;
}

template <int R>
void vi_pass_r(const fd_grid *g, float *const *f, hipStream_t s)
{
    const StepParams &p = g->sp;
    if (g->tune.by > 0) {
        // z-marching stress-memory pass on 64 x 8 tiles (8 waves, one row
        // each: the 26 streamed values per point leave no room for two rows)
        constexpr int BY = 8, RY = 1, TY = BY * RY;
        const int nzb = g->tune.nzb > 0 ? g->tune.nzb : 64;
        const int ntx = (p.nx + 63) / 64, nty = (p.ny + TY - 1) / TY;
        const unsigned nb = (unsigned)ntx * nty * ((p.nz + nzb - 1) / nzb);
        hipLaunchKernelGGL((k_vi_stress_zm<R, BY, RY>), dim3(nb), dim3(64, BY), 0, s,
                           vstate_of(f), vmedium_of(g), p, ntx, nty, nzb);
        return;
    }
    const int nxb = (p.nx + 63) / 64, nyb = (p.ny + 3) / 4;
    const unsigned nb = (unsigned)nxb * nyb * p.nz;
    hipLaunchKernelGGL((k_vi_stress_pt<R>), dim3(nb), dim3(64, 4), 0, s, vstate_of(f),
                       vmedium_of(g), p, nxb, nyb);
}

}  // namespace

int launch_vi_model(const fd_grid *g, const float *vp, const float *const *aux, unsigned *flags,
                    hipStream_t s)
{
    const int64_t n = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_vi_model, dim3(nb), dim3(256), 0, s, vp, aux[0], aux[1], aux[2], aux[3],
                       aux[4], vmedium_of(g), flags, g->sp, (float)g->d.dt);
    return check_launch("visco-elastic medium");
}

int launch_vi_stress(const fd_grid *g, float *const *f, hipStream_t s)
{
    switch (g->r) {
    case 1: vi_pass_r<1>(g, f, s); break;
    case 2: vi_pass_r<2>(g, f, s); break;
    case 3: vi_pass_r<3>(g, f, s); break;
    case 4: vi_pass_r<4>(g, f, s); break;
    case 5: vi_pass_r<5>(g, f, s); break;
    case 6: vi_pass_r<6>(g, f, s); break;
    case 7: vi_pass_r<7>(g, f, s); break;
    case 8: vi_pass_r<8>(g, f, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    return check_launch("visco-elastic stress-memory pass");
}

int launch_el_model(const fd_grid *g, const float *vp, const float *vs, const float *rho,
                    unsigned *flags, hipStream_t s)
{
    const int64_t n = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_el_model, dim3(nb), dim3(256), 0, s, vp, vs, rho, medium_of(g), flags,
                       g->sp, (float)g->d.dt);
    return check_launch("elastic medium");
}

int launch_el_velocity(const fd_grid *g, float *const *f, hipStream_t s)
{
    return el_pass(g, f, false, s);
}

int launch_el_stress(const fd_grid *g, float *const *f, hipStream_t s)
{
    return el_pass(g, f, true, s);
}

int launch_el_sparse(const fd_grid *g, float *const *f, const SparseArgs &inj,
                     const SparseArgs &smp, hipStream_t s)
{
    if (inj.n == 0 && smp.n == 0) return FD_OK;
    hipLaunchKernelGGL(k_el_sparse, dim3(1), dim3(1024), 0, s, state_of(f), g->sp, inj, smp);
    return check_launch("elastic sparse inject/sample");
}

}  // namespace fd
