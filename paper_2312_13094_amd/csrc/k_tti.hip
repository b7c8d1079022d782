// Pseudo-acoustic TTI step (paper, appendix "Anisotropic acoustic (TTI)",
// equation (rot)), in the two-field form of the paper's references:
//
//   p+ = [2p - (1-a) p- + c_pp H_xy p + c_x H_z r] / (1+a)
//   r+ = [2r - (1-a) r- + c_x  H_xy p + c   H_z r] / (1+a)
//
// with c = v^2 dt^2, c_pp = c (1 + 2 eps), c_x = c sqrt(1 + 2 delta), the
// symmetry axis a = (sin t cos f, sin t sin f, cos t) from the tilt t and
// azimuth f, and
//
//   H_z  u = div( a (a . grad u) ),   H_xy u = div( (I - a a^T) grad u )
//
// built from centred first derivatives of order so.  Pass 1 forms the two
// rotated gradient vectors on DOMAIN (six fields whose halo stays zero, so
// the outer divergence is the exact negative transpose of the inner
// gradient); pass 2 takes their divergence and updates both fields in place.
#include "fd_internal.h"

namespace fd {

template <int R>
__global__ __launch_bounds__(256) void k_tti_pass1(const float *__restrict__ p,
                                                   const float *__restrict__ r,
                                                   const float *__restrict__ th,
                                                   const float *__restrict__ ph,
                                                   float *__restrict__ w0, float *__restrict__ w1,
                                                   float *__restrict__ w2, float *__restrict__ s0,
                                                   float *__restrict__ s1, float *__restrict__ s2,
                                                   const StepParams sp, const int nxb, const int nyb)
{
    int b = blockIdx.x;
    const int xb = b % nxb;
    b /= nxb;
    const int yb = b % nyb;
    const int z = b / nyb;
    const int x = xb * 64 + threadIdx.x;
    const int y = yb * 4 + threadIdx.y;
    if (x >= sp.nx || y >= sp.ny) return;
    const int64_t PY = sp.pitch_y, PZ = sp.pitch_z;
    const int64_t i = sp.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
    float gpz = 0.f, gpy = 0.f, gpx = 0.f, grz = 0.f, gry = 0.f, grx = 0.f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        const float az = sp.dz[k - 1], ay = sp.dy[k - 1], ax = sp.dx[k - 1];
        gpz += az * (p[i + k * PZ] - p[i - k * PZ]);
        gpy += ay * (p[i + k * PY] - p[i - k * PY]);
        gpx += ax * (p[i + k] - p[i - k]);
        grz += az * (r[i + k * PZ] - r[i - k * PZ]);
        gry += ay * (r[i + k * PY] - r[i - k * PY]);
        grx += ax * (r[i + k] - r[i - k]);
    }
    float st, ct, sf, cf;
    sincosf(th[i], &st, &ct);
    sincosf(ph[i], &sf, &cf);
    const float az = ct, ay = st * sf, ax = st * cf;
    const float ap = az * gpz + ay * gpy + ax * gpx;
    const float ar = az * grz + ay * gry + ax * grx;
    w0[i] = gpz - az * ap;
    w1[i] = gpy - ay * ap;
    w2[i] = gpx - ax * ap;
    s0[i] = az * ar;
    s1[i] = ay * ar;
    s2[i] = ax * ar;
}

template <int R>
__global__ __launch_bounds__(256) void k_tti_pass2(
    const float *__restrict__ p, const float *pm, float *pp, const float *__restrict__ r,
    const float *rm, float *rp, const float *__restrict__ w0, const float *__restrict__ w1,
    const float *__restrict__ w2, const float *__restrict__ s0, const float *__restrict__ s1,
    const float *__restrict__ s2, const float *__restrict__ c, const float *__restrict__ cpp,
    const float *__restrict__ cx, const StepParams sp, const int nxb, const int nyb)
{
    int b = blockIdx.x;
    const int xb = b % nxb;
    b /= nxb;
    const int yb = b % nyb;
    const int z = b / nyb;
    const int x = xb * 64 + threadIdx.x;
    const int y = yb * 4 + threadIdx.y;
    if (x >= sp.nx || y >= sp.ny) return;
    const int64_t PY = sp.pitch_y, PZ = sp.pitch_z;
    const int64_t i = sp.offset + (int64_t)z * PZ + (int64_t)y * PY + x;
    float h1 = 0.f, h2 = 0.f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        const float az = sp.dz[k - 1], ay = sp.dy[k - 1], ax = sp.dx[k - 1];
        h1 += az * (w0[i + k * PZ] - w0[i - k * PZ]) + ay * (w1[i + k * PY] - w1[i - k * PY]) +
              ax * (w2[i + k] - w2[i - k]);
        h2 += az * (s0[i + k * PZ] - s0[i - k * PZ]) + ay * (s1[i + k * PY] - s1[i - k * PY]) +
              ax * (s2[i + k] - s2[i - k]);
    }
    const float a = damp_a(sp, z, y, x);
    const float inv = 1.0f / (1.0f + a);
    const float cc = c[i], cp = cpp[i], cxx = cx[i];
    const float pc = p[i], rc = r[i];
    const float pn = pc + ((1.0f - a) * (pc - pm[i]) + cp * h1 + cxx * h2) * inv;
    const float rn = rc + ((1.0f - a) * (rc - rm[i]) + cxx * h1 + cc * h2) * inv;
    pp[i] = pn;
    rp[i] = rn;
}

__global__ __launch_bounds__(256) void k_tti_model(const float *__restrict__ vel,
                                                   const float *__restrict__ eps,
                                                   const float *__restrict__ delta,
                                                   const float *__restrict__ theta,
                                                   const float *__restrict__ phi, float *c,
                                                   float *cpp, float *cx, float *th, float *ph,
                                                   float *az, float *ay, float *ax,
                                                   unsigned *flags, const StepParams p,
                                                   const float dt2)
{
    const int64_t n = (int64_t)p.nz * p.ny * p.nx;
    unsigned vmx = 0u, emx = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % p.nx);
        const int64_t t = i / p.nx;
        const int y = (int)(t % p.ny);
        const int z = (int)(t / p.ny);
        const int64_t j = p.offset + (int64_t)z * p.pitch_z + (int64_t)y * p.pitch_y + x;
        const float v = vel[i], e = eps[i], d = delta[i];
        const float cv = v * v * dt2;
        c[j] = cv;
        cpp[j] = cv * (1.0f + 2.0f * e);
        cx[j] = cv * sqrtf(1.0f + 2.0f * d);
        th[j] = theta[i];
        ph[j] = phi[i];
        // the symmetry axis, for the one-kernel step
        float st, ct, sf, cf;
        sincosf(theta[i], &st, &ct);
        sincosf(phi[i], &sf, &cf);
        az[j] = ct;
        ay[j] = st * sf;
        ax[j] = st * cf;
        const unsigned vb = (v > 0.0f) ? __float_as_uint(v) : 0x7f800000u;
        // eps, delta must be > -1/2; flag otherwise (NaN included)
        const unsigned eb = (e >= 0.0f) ? __float_as_uint(e) : ((e > -0.5f) ? 0u : 0x7f800000u);
        const unsigned db = (d > -0.5f) ? 0u : 0x7f800000u;
        vmx = vb > vmx ? vb : vmx;
        emx = eb > emx ? eb : emx;
        emx = db > emx ? db : emx;
    }
    atomicMax(flags, vmx);
    atomicMax(flags + 1, emx);
}

int launch_tti_model(const fd_grid *g, const float *vel, const float *const *tti, unsigned *flags,
                     hipStream_t s)
{
    const int64_t n = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_tti_model, dim3(nb), dim3(256), 0, s, vel, tti[0], tti[1], tti[2],
                       tti[3], g->vdt2, g->tti[0], g->tti[1], g->tti[2], g->tti[3], g->tti[4],
                       g->tti[5], g->tti[6], flags, g->sp,
                       (float)(g->d.dt * g->d.dt));
    return check_launch("TTI model");
}

template <int R>
static void tti_r(const fd_grid *g, const float *p, const float *pm, float *pp, const float *r,
                  const float *rm, float *rp, hipStream_t s)
{
    const StepParams &sp = g->sp;
    const int nxb = (sp.nx + 63) / 64, nyb = (sp.ny + 3) / 4;
    const unsigned nb = (unsigned)nxb * nyb * sp.nz;
    float *const *w = g->inter;
    hipLaunchKernelGGL((k_tti_pass1<R>), dim3(nb), dim3(64, 4), 0, s, p, r, g->tti[2], g->tti[3],
                       w[0], w[1], w[2], w[3], w[4], w[5], sp, nxb, nyb);
    hipLaunchKernelGGL((k_tti_pass2<R>), dim3(nb), dim3(64, 4), 0, s, p, pm, pp, r, rm, rp, w[0],
                       w[1], w[2], w[3], w[4], w[5], g->vdt2, g->tti[0], g->tti[1], sp, nxb, nyb);
}

int launch_tti_step(const fd_grid *g, const float *p, const float *pm, float *pp, const float *r,
                    const float *rm, float *rp, hipStream_t s)
{
    if (g->ndim == 3 && g->tune.by > 0)
        return (g->tune.flags & kTileTti1) ? launch_tti_step_fused(g, p, pm, pp, r, rm, rp, s)
                                           : launch_tti_step_zm(g, p, pm, pp, r, rm, rp, s);
    switch (g->r) {
    case 2: tti_r<2>(g, p, pm, pp, r, rm, rp, s); break;
    case 3: tti_r<3>(g, p, pm, pp, r, rm, rp, s); break;
    case 4: tti_r<4>(g, p, pm, pp, r, rm, rp, s); break;
    case 5: tti_r<5>(g, p, pm, pp, r, rm, rp, s); break;
    case 6: tti_r<6>(g, p, pm, pp, r, rm, rp, s); break;
    default: return set_error(FD_EINVAL, "TTI supports space orders 4..12");
    }
    return check_launch("TTI step");
}

}  // namespace fd
