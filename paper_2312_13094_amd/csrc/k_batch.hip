// Batched multi-shot kernels: every launch covers all shots of a batch.
//
// k_batch_zmarch is a work list over (shot, tile): logical block b belongs
// to the shot whose block range contains it, and runs the same z-marching
// step body as the single-grid kernel on that shot's aperture.  Apertures
// of different sizes therefore share one launch per time step.  Field
// roles are passed as slot indices into each shot's workspace, so one
// captured graph node serves all shots.  The remaining kernels put the
// shot index on blockIdx.y.
#include "batch_internal.h"

namespace fd {

int launch_batch_step(const BatchShot *shots_dev, int nshots, int total_blocks, int r,
                      const Tuning &t, int iu, int ium, int iup, hipStream_t s, const BatchEpi &e)
{
    int rc;
    switch (r) {
    case 1: rc = launch_batch_radius<1>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 2: rc = launch_batch_radius<2>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 3: rc = launch_batch_radius<3>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 4: rc = launch_batch_radius<4>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 5: rc = launch_batch_radius<5>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 6: rc = launch_batch_radius<6>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 7: rc = launch_batch_radius<7>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    case 8: rc = launch_batch_radius<8>(shots_dev, nshots, total_blocks, t, iu, ium, iup, e, s); break;
    default: return set_error(FD_EINVAL, "unsupported stencil radius");
    }
    if (rc) return rc;
    return check_launch("batched step");
}

// One block per shot: injection (atomics), device fence + barrier, sampling.
// With fd >= 0 (modes 0 and 1) each injected amount also enters the imaging
// factor of the step it completes: D is linear in u+ with weight
// 1/dt^2 + gamma/(2 dt).
__global__ __launch_bounds__(256) void k_batch_sparse(const BatchShot *__restrict__ shots,
                                                      const int mode, const int n, const int f,
                                                      const float hinv, const int fd,
                                                      const float inv_dt2, const float inv_2dt)
{
    const BatchShot &S = shots[blockIdx.x];
    const StepParams &p = S.p;
    float *u = S.base + f * S.stride;
    const float *vdt2 = S.base + kVdt2 * S.stride;
    const int64_t PY = p.pitch_y, PZ = p.pitch_z;
    // injection set: sources (modes 0, 1) or receivers (mode 2)
    const bool rec_inj = mode == 2;
    const int ni = rec_inj ? S.nr : S.ns;
    const int32_t *ib = rec_inj ? S.rbase : S.sbase;
    const float *ifr = rec_inj ? S.rfrac : S.sfrac;
    const float scale = rec_inj ? 1.0f : hinv;
    for (int e = threadIdx.x; e < ni * 8; e += blockDim.x) {
        const int pt = e >> 3, c = e & 7;
        int z, y, x;
        float w;
        corner(3, ib + pt * 3, ifr + pt * 3, c, z, y, x, w);
        const float val = rec_inj ? S.d[(int64_t)n * S.nr + pt] - S.dobs[(int64_t)n * S.nr + pt]
                                  : S.q[(int64_t)n * S.ns + pt];
        const int64_t i = p.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
        const float a = damp_a(p, z, y, x);
        const float amt = scale * w * val * vdt2[i] / (1.0f + a);
        atomicAdd(u + i, amt);
        if (fd >= 0)
            atomicAdd(S.base + fd * S.stride + i, amt * (inv_dt2 + (a / p.half_dt) * inv_2dt));
    }
    if (mode != 0) return;
    __threadfence();
    __syncthreads();
    for (int pt = threadIdx.x; pt < S.nr; pt += blockDim.x) {
        float acc = 0.0f;
        for (int c = 0; c < 8; ++c) {
            int z, y, x;
            float w;
            corner(3, S.rbase + pt * 3, S.rfrac + pt * 3, c, z, y, x, w);
            acc += w * u[p.offset + (int64_t)z * PZ + (int64_t)y * PY + x];
        }
        S.d[(int64_t)n * S.nr + pt] = acc;
    }
}

int launch_batch_sparse(const BatchShot *shots_dev, int nshots, int mode, int n, int f,
                        float hinv, hipStream_t s, int fd, float inv_dt2, float inv_2dt)
{
    hipLaunchKernelGGL(k_batch_sparse, dim3(nshots), dim3(256), 0, s, shots_dev, mode, n, f, hinv,
                       mode != 2 ? fd : -1, inv_dt2, inv_2dt);
    return check_launch("batched sparse");
}

__global__ __launch_bounds__(256) void k_batch_copy(const BatchShot *__restrict__ shots,
                                                    const int fsrc, const int fdst)
{
    const BatchShot &S = shots[blockIdx.y];
    const float4 *a = reinterpret_cast<const float4 *>(S.base + fsrc * S.stride);
    float4 *b = reinterpret_cast<float4 *>(S.base + fdst * S.stride);
    const int64_t n4 = S.stride / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

int launch_batch_copy(const BatchShot *shots_dev, int nshots, int64_t max_stride, int fsrc,
                      int fdst, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((max_stride / 4 + 255) / 256, 2048);
    hipLaunchKernelGGL(k_batch_copy, dim3(nb, nshots), dim3(256), 0, s, shots_dev, fsrc, fdst);
    return check_launch("batched copy");
}

__global__ __launch_bounds__(256) void k_batch_zero(const BatchShot *__restrict__ shots,
                                                    const int f)
{
    const BatchShot &S = shots[blockIdx.y];
    float4 *a = reinterpret_cast<float4 *>(S.base + f * S.stride);
    const int64_t n4 = S.stride / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

int launch_batch_zero(const BatchShot *shots_dev, int nshots, int64_t max_stride, int f,
                      hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((max_stride / 4 + 255) / 256, 2048);
    hipLaunchKernelGGL(k_batch_zero, dim3(nb, nshots), dim3(256), 0, s, shots_dev, f);
    return check_launch("batched zero");
}

// g -= lambda * [((u+ - u) - (u - u-)) / dt^2 + gamma (u+ - u-) / (2 dt)]
// One wave per (z, y) row of a shot's DOMAIN, lanes along x: the row's
// sponge terms in z and y are taken once, and no per-point 64-bit division
// is needed to find a point's coordinates.  Every operand is streamed once
// per launch (the fields of all shots far exceed the caches), so the loads
// and the store carry non-temporal hints.
constexpr int kImgRows = 4;   // rows (waves) per block

__global__ __launch_bounds__(64 * kImgRows) void k_batch_imaging(
    const BatchShot *__restrict__ shots, const int flam, const int fup, const int fu,
    const int fum, const float inv_dt2, const float inv_2dt)
{
    const BatchShot &S = shots[blockIdx.y];
    const StepParams &p = S.p;
    const int nrows = p.nz * p.ny;
    const float *lam = S.base + flam * S.stride, *up = S.base + fup * S.stride;
    const float *u0 = S.base + fu * S.stride, *um = S.base + fum * S.stride;
    float *g = S.base + kGrad * S.stride;
    const bool damp = p.nbl > 0;
    for (int row = blockIdx.x * kImgRows + threadIdx.y; row < nrows;
         row += gridDim.x * kImgRows) {
        const int z = row / p.ny, y = row - z * p.ny;
        const float gzz = damp ? sponge_ax(p, 0, z, p.gz) : 0.0f;
        const float gyy = damp ? sponge_ax(p, 1, y, p.gy) : 0.0f;
        const int64_t j0 = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y;
        for (int x = threadIdx.x; x < p.nx; x += 64) {
            const int64_t j = j0 + x;
            const float gam = damp ? (gzz + sponge_ax(p, 2, x, p.gx)) + gyy : 0.0f;
            const float a = __builtin_nontemporal_load(up + j);
            const float b = __builtin_nontemporal_load(u0 + j);
            const float c = __builtin_nontemporal_load(um + j);
            const float l = __builtin_nontemporal_load(lam + j);
            const float gj = __builtin_nontemporal_load(g + j);
            __builtin_nontemporal_store(
                gj - l * (((a - b) - (b - c)) * inv_dt2 + gam * (a - c) * inv_2dt), g + j);
        }
    }
}

int launch_batch_imaging(const BatchShot *shots_dev, int nshots, int64_t max_rows, int flam,
                         int fup, int fu, int fum, float inv_dt2, float inv_2dt, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((max_rows + kImgRows - 1) / kImgRows, 65535);
    hipLaunchKernelGGL(k_batch_imaging, dim3(nb, nshots), dim3(64, kImgRows), 0, s, shots_dev,
                       flam, fup, fu, fum, inv_dt2, inv_2dt);
    return check_launch("batched imaging");
}

// g -= lambda D, D the imaging factor a recomputed step stored: the same
// row mapping as k_batch_imaging, three streamed operands instead of five.
__global__ __launch_bounds__(64 * kImgRows) void k_batch_imaging_d(
    const BatchShot *__restrict__ shots, const int flam, const int fd)
{
    const BatchShot &S = shots[blockIdx.y];
    const StepParams &p = S.p;
    const int nrows = p.nz * p.ny;
    const float *lam = S.base + flam * S.stride, *dd = S.base + fd * S.stride;
    float *g = S.base + kGrad * S.stride;
    for (int row = blockIdx.x * kImgRows + threadIdx.y; row < nrows;
         row += gridDim.x * kImgRows) {
        const int z = row / p.ny, y = row - z * p.ny;
        const int64_t j0 = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y;
        for (int x = threadIdx.x; x < p.nx; x += 64) {
            const int64_t j = j0 + x;
            const float l = __builtin_nontemporal_load(lam + j);
            const float d = __builtin_nontemporal_load(dd + j);
            const float gj = __builtin_nontemporal_load(g + j);
            __builtin_nontemporal_store(gj - l * d, g + j);
        }
    }
}

int launch_batch_imaging_d(const BatchShot *shots_dev, int nshots, int64_t max_rows, int flam,
                           int fd, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((max_rows + kImgRows - 1) / kImgRows, 65535);
    hipLaunchKernelGGL(k_batch_imaging_d, dim3(nb, nshots), dim3(64, kImgRows), 0, s, shots_dev,
                       flam, fd);
    return check_launch("batched imaging (stored factor)");
}

// Full-model gradient: for each point, add the shots covering it in shot
// order, then apply dJ/dv = dJ/dm * (-2 / v^3).
__global__ __launch_bounds__(256) void k_batch_reduce(const BatchShot *__restrict__ shots,
                                                      const int nshots, const int64_t fz,
                                                      const int64_t fy, const int64_t fx,
                                                      const float *__restrict__ vel,
                                                      float *__restrict__ gv)
{
    const int64_t n = fz * fy * fx;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % fx);
        const int64_t t = i / fx;
        const int y = (int)(t % fy);
        const int z = (int)(t / fy);
        float acc = 0.0f;
        for (int s = 0; s < nshots; ++s) {
            const BatchShot &S = shots[s];
            const int lz = z - S.org[0], ly = y - S.org[1], lx = x - S.org[2];
            if (lz >= 0 && lz < S.p.nz && ly >= 0 && ly < S.p.ny && lx >= 0 && lx < S.p.nx)
                acc += S.base[kGrad * S.stride + S.p.offset + (int64_t)lz * S.p.pitch_z +
                              (int64_t)ly * S.p.pitch_y + lx];
        }
        const float v = vel[i];
        gv[i] = acc * (-2.0f / (v * v * v));
    }
}

int launch_batch_reduce(const BatchShot *shots_dev, int nshots, const int64_t full[3],
                        const float *vel_full, float *grad_v, hipStream_t s)
{
    const int64_t n = full[0] * full[1] * full[2];
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_batch_reduce, dim3(nb), dim3(256), 0, s, shots_dev, nshots, full[0],
                       full[1], full[2], vel_full, grad_v);
    return check_launch("batched gradient reduction");
}

// v^2 dt^2 of each aperture, cut from the full model
__global__ __launch_bounds__(256) void k_batch_vdt2(const BatchShot *__restrict__ shots,
                                                    const int64_t fy, const int64_t fx,
                                                    const float *__restrict__ vel,
                                                    const float dt2, unsigned *vmax_bits)
{
    const BatchShot &S = shots[blockIdx.y];
    const StepParams &p = S.p;
    const int64_t n = (int64_t)p.nz * p.ny * p.nx;
    float *vd = S.base + kVdt2 * S.stride;
    unsigned mx = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % p.nx);
        const int64_t t = i / p.nx;
        const int y = (int)(t % p.ny);
        const int z = (int)(t / p.ny);
        const float v = vel[((int64_t)(z + S.org[0]) * fy + (y + S.org[1])) * fx + (x + S.org[2])];
        vd[p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x] = v * v * dt2;
        const unsigned bits = (v > 0.0f) ? __float_as_uint(v) : 0x7f800000u;
        mx = bits > mx ? bits : mx;
    }
    atomicMax(vmax_bits, mx);
}

int launch_batch_vdt2(const BatchShot *shots_dev, int nshots, int64_t max_pts,
                      const int64_t full[3], const float *vel_full, float dt2,
                      unsigned *vmax_bits, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((max_pts + 255) / 256, 2048);
    hipLaunchKernelGGL(k_batch_vdt2, dim3(nb, nshots), dim3(256), 0, s, shots_dev, full[1],
                       full[2], vel_full, dt2, vmax_bits);
    return check_launch("batched model");
}

}  // namespace fd
