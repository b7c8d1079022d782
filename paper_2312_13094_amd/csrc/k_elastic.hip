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
enum { BX, BY, BZ, LAM, MU, MXY, MXZ, MYZ };

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
        med.m[BX][j] = 0.5f * (b(i) + b(i + ox)) * dt;
        med.m[BY][j] = 0.5f * (b(i) + b(i + oy)) * dt;
        med.m[BZ][j] = 0.5f * (b(i) + b(i + oz)) * dt;
        med.m[LAM][j] = (r * a * a - 2.0f * m0) * dt;
        med.m[MU][j] = m0 * dt;
        med.m[MXY][j] = 0.25f * (m0 + mu(i + ox) + mu(i + oy) + mu(i + ox + oy)) * dt;
        med.m[MXZ][j] = 0.25f * (m0 + mu(i + ox) + mu(i + oz) + mu(i + ox + oz)) * dt;
        med.m[MYZ][j] = 0.25f * (m0 + mu(i + oy) + mu(i + oz) + mu(i + oy + oz)) * dt;
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
    st.f[VX][i] = damped(st.f[VX][i], med.m[BX][i] * rx, a);
    st.f[VY][i] = damped(st.f[VY][i], med.m[BY][i] * ry, a);
    st.f[VZ][i] = damped(st.f[VZ][i], med.m[BZ][i] * rz, a);
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
    const float lt = med.m[LAM][i] * ((exx + eyy) + ezz);
    const float m2 = 2.0f * med.m[MU][i];
    st.f[TXX][i] = damped(st.f[TXX][i], lt + m2 * exx, a);
    st.f[TYY][i] = damped(st.f[TYY][i], lt + m2 * eyy, a);
    st.f[TZZ][i] = damped(st.f[TZZ][i], lt + m2 * ezz, a);
    st.f[TXY][i] = damped(st.f[TXY][i],
                          med.m[MXY][i] * (dp<R>(vx, i, PY, p.sy) + dp<R>(vy, i, 1, p.sx)), a);
    st.f[TXZ][i] = damped(st.f[TXZ][i],
                          med.m[MXZ][i] * (dp<R>(vx, i, PZ, p.sz) + dp<R>(vz, i, 1, p.sx)), a);
    st.f[TYZ][i] = damped(st.f[TYZ][i],
                          med.m[MYZ][i] * (dp<R>(vy, i, PZ, p.sz) + dp<R>(vz, i, PY, p.sy)), a);
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

}  // namespace

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
