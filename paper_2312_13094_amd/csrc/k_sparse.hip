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

int launch_sparse(const fd_grid *g, float *u, const SparseArgs &inj, const SparseArgs &smp,
                  hipStream_t s)
{
    if (inj.n == 0 && smp.n == 0) return FD_OK;
    // one block (injection before sampling needs a block-wide barrier); 1024
    // threads so that up to 1024 receivers sample with their corner loads
    // in flight together
    hipLaunchKernelGGL(k_sparse, dim3(1), dim3(1024), 0, s, u, g->vdt2, g->sp, g->ndim, inj, smp);
    return check_launch("sparse inject/sample");
}

}  // namespace fd
