// Sparse source injection and receiver interpolation (paper, "Sparse data"
// paragraph; equation (acou): the source delta(x_s) q(t) and the data
// d(t) = u(t, x_r)).
//
// Points are off the grid; each touches the 2^d nodes of its cell with
// multilinear weights.  Injection adds
//     scale * w * val * v^2 dt^2 / (1 + gamma dt/2)
// to every node (scale = h^-d for a physical source, 1 for the adjoint's
// receiver residuals) with float atomics, so points sharing nodes sum.
// Sampling then reads scale * sum_corners w * u.  Both run in one single-
// workgroup launch: the device-scope fence plus barrier between the phases
// makes the atomics visible to the sampling loads.
#include "fd_internal.h"

namespace fd {

__global__ __launch_bounds__(1024) void k_sparse(float *u, const float *__restrict__ vdt2,
                                                const StepParams p, const int ndim,
                                                const SparseArgs inj, const SparseArgs smp)
{
    const int nc = 1 << ndim;
    const int64_t PY = p.pitch_y, PZ = p.pitch_z;
    for (int e = threadIdx.x; e < inj.n * nc; e += blockDim.x) {
        const int pt = e / nc, c = e % nc;
        int z, y, x;
        float w;
        corner(ndim, inj.base + pt * ndim, inj.frac + pt * ndim, c, z, y, x, w);
        const int64_t i = p.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
        const float a = damp_a(p, z, y, x);
        atomicAdd(u + i, inj.scale * w * inj.vals[pt] * vdt2[i] / (1.0f + a));
    }
    __threadfence();
    __syncthreads();
    for (int pt = threadIdx.x; pt < smp.n; pt += blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < nc; ++c) {
            int z, y, x;
            float w;
            corner(ndim, smp.base + pt * ndim, smp.frac + pt * ndim, c, z, y, x, w);
            s += w * u[p.offset + (int64_t)z * PZ + (int64_t)y * PY + x];
        }
        smp.out[pt] = smp.scale * s;
    }
}

// Large point sets: injection over many blocks (one corner per thread,
// float atomics), then sampling over many blocks (one point per thread) in a
// second launch, which the stream orders after every injection.
__global__ __launch_bounds__(256) void k_inject(float *u, const float *__restrict__ vdt2,
                                               const StepParams p, const int ndim,
                                               const SparseArgs inj)
{
    const int nc = 1 << ndim;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= inj.n * nc) return;
    const int pt = e / nc, c = e % nc;
    int z, y, x;
    float w;
    corner(ndim, inj.base + pt * ndim, inj.frac + pt * ndim, c, z, y, x, w);
    const int64_t i = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x;
    const float a = damp_a(p, z, y, x);
    atomicAdd(u + i, inj.scale * w * inj.vals[pt] * vdt2[i] / (1.0f + a));
}

__global__ __launch_bounds__(256) void k_sample(const float *u, const StepParams p,
                                               const int ndim, const SparseArgs smp)
{
    const int pt = blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= smp.n) return;
    const int nc = 1 << ndim;
    float s = 0.0f;
    for (int c = 0; c < nc; ++c) {
        int z, y, x;
        float w;
        corner(ndim, smp.base + pt * ndim, smp.frac + pt * ndim, c, z, y, x, w);
        s += w * u[p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x];
    }
    smp.out[pt] = smp.scale * s;
}

// Injection into u_new and sampling of u_old in one launch: threads
// [0, inj.n * 2^d) take one injection corner each, the next smp.n threads one
// sample point each.  u_old is a finished field nobody writes here, so the
// halves need no ordering; small blocks spread the scattered loads over
// many compute units.
__global__ __launch_bounds__(64) void k_sparse_split(float *u_new, const float *u_old,
                                                    const float *__restrict__ vdt2,
                                                    const StepParams p, const int ndim,
                                                    const SparseArgs inj, const SparseArgs smp)
{
    const int nc = 1 << ndim;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int ni = inj.n * nc;
    if (e < ni) {
        const int pt = e / nc, c = e % nc;
        int z, y, x;
        float w;
        corner(ndim, inj.base + pt * ndim, inj.frac + pt * ndim, c, z, y, x, w);
        const int64_t i = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x;
        const float a = damp_a(p, z, y, x);
        atomicAdd(u_new + i, inj.scale * w * inj.vals[pt] * vdt2[i] / (1.0f + a));
        return;
    }
    const int pt = e - ni;
    if (pt >= smp.n) return;
    float acc = 0.0f;
    for (int c = 0; c < nc; ++c) {
        int z, y, x;
        float w;
        corner(ndim, smp.base + pt * ndim, smp.frac + pt * ndim, c, z, y, x, w);
        acc += w * u_old[p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x];
    }
    smp.out[pt] = smp.scale * acc;
}

int launch_sparse_split(const fd_grid *g, float *u_new, const SparseArgs &inj,
                        const float *u_old, const SparseArgs &smp, hipStream_t s)
{
    const int64_t work = (int64_t)inj.n * (1 << g->ndim) + smp.n;
    if (work == 0) return FD_OK;
    hipLaunchKernelGGL(k_sparse_split, dim3((unsigned)((work + 63) / 64)), dim3(64), 0, s, u_new,
                       u_old, g->vdt2, g->sp, g->ndim, inj, smp);
    return check_launch("sparse inject (new level) / sample (previous level)");
}

// point sets up to this many corners (injection) plus points (sampling) take
// the single-workgroup kernel; larger ones the two multi-block launches
constexpr int kSparseOneBlock = 4096;

int launch_sparse(const fd_grid *g, float *u, const SparseArgs &inj, const SparseArgs &smp,
                  hipStream_t s)
{
    if (inj.n == 0 && smp.n == 0) return FD_OK;
    const int nc = 1 << g->ndim;
    if ((int64_t)inj.n * nc + smp.n <= kSparseOneBlock) {
        // one block (injection before sampling needs a block-wide barrier);
        // 1024 threads so that up to 1024 receivers sample with their corner
        // loads in flight together
        hipLaunchKernelGGL(k_sparse, dim3(1), dim3(1024), 0, s, u, g->vdt2, g->sp, g->ndim, inj,
                           smp);
        return check_launch("sparse inject/sample");
    }
    if (inj.n > 0) {
        const int64_t work = (int64_t)inj.n * nc;
        hipLaunchKernelGGL(k_inject, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, u,
                           g->vdt2, g->sp, g->ndim, inj);
        const int rc = check_launch("sparse inject");
        if (rc) return rc;
    }
    if (smp.n > 0) {
        hipLaunchKernelGGL(k_sample, dim3((unsigned)((smp.n + 255) / 256)), dim3(256), 0, s, u,
                           g->sp, g->ndim, smp);
        return check_launch("sparse sample");
    }
    return FD_OK;
}

}  // namespace fd
