// Model coefficients, the zero-lag imaging condition and the velocity chain
// rule.
//
// build_vdt2: v (DOMAIN-shaped, dense) -> v^2 dt^2 in the padded layout; the
// largest velocity (and any non-positive or NaN entry) is recorded so the
// host can check the stability bound.
//
// imaging: the derivative of the scheme's row n with respect to the squared
// slowness m (the leapfrog update written as
//   m (1/dt^2 + gamma/2dt) u+ - (2m/dt^2 + L) u + m (1/dt^2 - gamma/2dt) u- = f)
// paired with the adjoint field of that row:
//   g += -lambda_n * [ ((u+ - u) - (u - u-)) / dt^2 + gamma (u+ - u-) / (2 dt) ],
// the second difference taken before scaling to limit FP32 cancellation.
#include "fd_internal.h"

namespace fd {

__global__ __launch_bounds__(256) void k_build_vdt2(const float *__restrict__ vel, float *vdt2,
                                                    unsigned *vmax_bits, const StepParams p,
                                                    const float dt2)
{
    const int64_t n = (int64_t)p.nz * p.ny * p.nx;
    unsigned mx = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % p.nx);
        const int64_t t = i / p.nx;
        const int y = (int)(t % p.ny);
        const int z = (int)(t / p.ny);
        const float v = vel[i];
        vdt2[p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x] = v * v * dt2;
        // positive floats order like their bit patterns; flag <= 0 / NaN as +inf
        const unsigned bits = (v > 0.0f) ? __float_as_uint(v) : 0x7f800000u;
        mx = bits > mx ? bits : mx;
    }
    atomicMax(vmax_bits, mx);
}

int launch_build_vdt2(const fd_grid *g, const float *vel, float *vdt2, unsigned *vmax_bits,
                      hipStream_t s)
{
    const int64_t n = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    const float dt2 = (float)(g->d.dt * g->d.dt);
    hipLaunchKernelGGL(k_build_vdt2, dim3(nb), dim3(256), 0, s, vel, vdt2, vmax_bits, g->sp, dt2);
    return check_launch("build v^2 dt^2");
}

// One wave per (z, y) row of the DOMAIN, lanes along x (no per-point 64-bit
// division); every operand is streamed once, hence the non-temporal hints.
constexpr int kImgRows = 4;   // rows (waves) per block

__global__ __launch_bounds__(64 * kImgRows) void k_imaging(const float *__restrict__ lam,
                                                           const float *__restrict__ up,
                                                           const float *__restrict__ u0,
                                                           const float *__restrict__ um,
                                                           float *grad, const StepParams p,
                                                           const float inv_dt2,
                                                           const float inv_2dt)
{
    const int nrows = p.nz * p.ny;
    const bool damp = p.nbl > 0;
    for (int row = blockIdx.x * kImgRows + threadIdx.y; row < nrows;
         row += gridDim.x * kImgRows) {
        const int z = row / p.ny, y = row - z * p.ny;
        const float gzz = damp ? sponge_ax(p, 0, z, p.gz) : 0.0f;
        const float gyy = damp && p.ny > 1 ? sponge_ax(p, 1, y, p.gy) : 0.0f;
        const int64_t j0 = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y;
        float *gr = grad + (int64_t)row * p.nx;
        for (int x = threadIdx.x; x < p.nx; x += 64) {
            const int64_t j = j0 + x;
            const float gam = damp ? (gzz + sponge_ax(p, 2, x, p.gx)) + gyy : 0.0f;
            const float a = __builtin_nontemporal_load(up + j);
            const float b = __builtin_nontemporal_load(u0 + j);
            const float c = __builtin_nontemporal_load(um + j);
            const float l = __builtin_nontemporal_load(lam + j);
            const float dE = ((a - b) - (b - c)) * inv_dt2 + gam * (a - c) * inv_2dt;
            __builtin_nontemporal_store(__builtin_nontemporal_load(gr + x) - l * dE, gr + x);
        }
    }
}

int launch_imaging(const fd_grid *g, const float *lam, const float *up, const float *u0,
                   const float *um, float *grad, hipStream_t s)
{
    const int64_t rows = (int64_t)g->sp.nz * g->sp.ny;
    const int nb = (int)std::min<int64_t>((rows + kImgRows - 1) / kImgRows, 65535);
    const double dt = g->d.dt;
    hipLaunchKernelGGL(k_imaging, dim3(nb), dim3(64, kImgRows), 0, s, lam, up, u0, um, grad,
                       g->sp, (float)(1.0 / (dt * dt)), (float)(0.5 / dt));
    return check_launch("imaging condition");
}

__global__ __launch_bounds__(256) void k_grad_to_vel(const float *__restrict__ gm, float *gv,
                                                     const float *__restrict__ vdt2,
                                                     const StepParams p, const float dt)
{
    const int64_t n = (int64_t)p.nz * p.ny * p.nx;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % p.nx);
        const int64_t t = i / p.nx;
        const int y = (int)(t % p.ny);
        const int z = (int)(t / p.ny);
        const float v = sqrtf(vdt2[p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x]) / dt;
        gv[i] = gm[i] * (-2.0f / (v * v * v));
    }
}

int launch_grad_to_vel(const fd_grid *g, const float *gm, float *gv, hipStream_t s)
{
    const int64_t n = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_grad_to_vel, dim3(nb), dim3(256), 0, s, gm, gv, g->vdt2, g->sp,
                       (float)g->d.dt);
    return check_launch("gradient chain rule");
}

}  // namespace fd
