// Internal declarations shared by the libfd translation units (host side and
// kernel launchers).  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fd.h"

namespace fd {

constexpr int kMaxR = 8;          // space order 16
constexpr int kXOff = 32;         // DOMAIN x offset in a row: 128-byte aligned rows

// Per-launch constants of one leapfrog step; passed by value (kernarg
// segment, read through the scalar cache).
struct StepParams {
    int nz, ny, nx;               // DOMAIN extents (ny == 1 in 2-D)
    int nbl;                      // damping layer width (0 = none)
    int64_t pitch_y, pitch_z;     // elements
    int64_t offset;               // element offset of DOMAIN (0,0,0)
    float cz[kMaxR + 1];          // w_k / h_z^2, k = 0..r
    float cy[kMaxR + 1];          // w_k / h_y^2 (zero in 2-D)
    float cx[kMaxR + 1];          // w_k / h_x^2
    float c0;                     // cz[0] + cy[0] + cx[0]
    float dz[kMaxR], dy[kMaxR], dx[kMaxR];  // first-derivative a_k / h per axis (TTI)
    float sz[kMaxR], sy[kMaxR], sx[kMaxR];  // staggered first-derivative c_k / h (elastic)
    float gz, gy, gx;             // damping gamma_max per axis (1/s)
    float inv_nbl;                // 1 / nbl
    float half_dt;                // dt / 2
    // damping layer edges per axis (z, y, x) in the launch's own indices:
    // index i is in the layer below sl (depth sl - i) or above sh (depth
    // i - sh).  nbl and n - 1 - nbl for a whole grid; shifted by the origin
    // when a launch covers a sub-box of it.
    int sl[3], sh[3];
    // first x column written by a launch (0 for a whole grid; a sub-box
    // keeps its x origin on a multiple of 64 columns and masks below xlo)
    int xlo;
};

// Damping rate along one axis at DOMAIN index i: gamma_max * xi^2 with xi the
// depth into the layer, 0 at the inner edge, 1 at the outermost point.
__host__ __device__ inline float sponge1(int i, int n, int nbl, float inv_nbl, float gmax)
{
    float xi = 0.0f;
    if (i < nbl) xi = (float)(nbl - i) * inv_nbl;
    else if (i > n - 1 - nbl) xi = (float)(i - (n - 1 - nbl)) * inv_nbl;
    return gmax * xi * xi;
}

// The same damping rate along axis ax (0 z, 1 y, 2 x) at index i of a
// launch (whole grid or sub-box); same arithmetic as sponge1 for a whole grid.
__device__ inline float sponge_ax(const StepParams &p, int ax, int i, float gmax)
{
    float xi = 0.0f;
    if (i < p.sl[ax]) xi = (float)(p.sl[ax] - i) * p.inv_nbl;
    else if (i > p.sh[ax]) xi = (float)(i - p.sh[ax]) * p.inv_nbl;
    return gmax * xi * xi;
}

// a = (dt/2) * gamma(z, y, x)
__device__ inline float damp_a(const StepParams &p, int z, int y, int x)
{
    if (p.nbl <= 0) return 0.0f;
    float g = sponge_ax(p, 0, z, p.gz) + sponge_ax(p, 2, x, p.gx);
    if (p.ny > 1) g += sponge_ax(p, 1, y, p.gy);
    return p.half_dt * g;
}

// The damped leapfrog update (appendix "Isotropic acoustic"): given u, u-,
// v^2 dt^2, the Laplacian and a = gamma dt / 2, returns
// u + [(1 - a)(u - u-) + v^2 dt^2 lap] / (1 + a).  Every acoustic step kernel
// goes through this one expression, so they round identically.
__device__ __forceinline__ float leapfrog_update(float uc, float um, float vdt2, float lap,
                                                float a)
{
    return uc + ((1.0f - a) * (uc - um) + vdt2 * lap) / (1.0f + a);
}

// Node (z, y, x) and multilinear weight of corner c of a sparse point's
// cell; bit 2/1/0 of c selects the upper node along z/y/x (2-D: bits 1/0 for
// z/x).
__device__ inline void corner(const int ndim, const int32_t *base, const float *frac,
                              const int c, int &z, int &y, int &x, float &w)
{
    if (ndim == 3) {
        const int bz = (c >> 2) & 1, by = (c >> 1) & 1, bx = c & 1;
        z = base[0] + bz;
        y = base[1] + by;
        x = base[2] + bx;
        w = (bz ? frac[0] : 1.0f - frac[0]) * (by ? frac[1] : 1.0f - frac[1]) *
            (bx ? frac[2] : 1.0f - frac[2]);
    } else {
        const int bz = (c >> 1) & 1, bx = c & 1;
        z = base[0] + bz;
        y = 0;
        x = base[1] + bx;
        w = (bz ? frac[0] : 1.0f - frac[0]) * (bx ? frac[1] : 1.0f - frac[1]);
    }
}

// Tile choice for the z-marching 3-D kernel.
struct Tuning {
    int by;        // waves per block (block = 64 x by threads)
    int ry;        // rows per thread (tile height = by * ry)
    int nzb;       // planes per block (z chunk)
    int flags;     // bit 0: XCD-aware block remap; bit 1: prefetch two planes
                   // ahead; bit 2: non-temporal hints on the streamed fields;
                   // bit 3: halo loads issued with the neighbours' front loads;
                   // bit 4: 128-wide tiles, two columns per lane (implies bit 3);
                   // bit 5: TTI in one z-marching kernel instead of two passes
};
constexpr int kTileXcd = 1, kTilePf2 = 2, kTileNts = 4, kTileRing = 8, kTileWide = 16,
              kTileTti1 = 32;

// Default 3-D tile, with the halo ring and non-temporal hints.  Large grids
// take 128 x 16 tiles (8 waves of 2 rows, two columns per lane) with the
// deepest z chunk (128 down to 32 planes) that still gives 512 blocks;
// otherwise the first of 64 x 16 (8 x 2), 64 x 8 (4 x 2) and 64 x 4 (4 x 1)
// columns whose launch reaches 1024 blocks with chunks of 64 planes halved
// down to 8 (the smallest tile with 8-plane chunks if none does), so that
// small grids still fill 256 CUs.
inline Tuning default_tuning(const int n[3])
{
    const int64_t wide = (int64_t)((n[2] + 127) / 128) * ((n[1] + 15) / 16);
    for (int nzb = 128; nzb >= 32; nzb /= 2)
        if (wide * ((n[0] + nzb - 1) / nzb) >= 512)
            return Tuning{8, 2, nzb, kTileRing | kTileNts | kTileWide};
    const int shapes[3][2] = {{8, 2}, {4, 2}, {4, 1}};
    for (const auto &sh : shapes) {
        const int64_t tiles = (int64_t)((n[2] + 63) / 64) * ((n[1] + sh[0] * sh[1] - 1) / (sh[0] * sh[1]));
        for (int nzb = 64; nzb >= 8; nzb /= 2)
            if (tiles * ((n[0] + nzb - 1) / nzb) >= 1024)
                return Tuning{sh[0], sh[1], nzb, kTileRing | kTileNts};
    }
    return Tuning{4, 1, 8, kTileRing | kTileNts};
}

// TTI: the two z-marching passes with the acoustic default's z chunk
// (32 planes at 384^3); the one-kernel step (flag kTileTti1) measured slower.
inline Tuning tti_default_tuning(const int n[3])
{
    return Tuning{8, 2, default_tuning(n).nzb, 0};
}

// Elastic passes: z-marching 64 x 16 tiles, (by, ry) = (8, 2); the deepest
// z chunk of 256 .. 8 planes that still gives 1024 blocks.
inline Tuning el_default_tuning(const int n[3])
{
    const int64_t tiles = (int64_t)((n[2] + 63) / 64) * ((n[1] + 15) / 16);
    for (int nzb = 256; nzb > 8; nzb /= 2)
        if (tiles * ((n[0] + nzb - 1) / nzb) >= 1024) return Tuning{8, 2, nzb, 0};
    return Tuning{8, 2, 8, 0};
}

// One set of sparse points bound to a step.
struct SparseArgs {
    int n;
    const int32_t *base;   // [n][ndim]
    const float *frac;     // [n][ndim]
    const float *vals;     // injection: [n] values of this step; else NULL
    float *out;            // sampling: [n] outputs of this step; else NULL
    float scale;
};


}  // namespace fd

struct fd_grid {
    fd_grid_desc d;
    int ndim;
    int n[3];               // (nz, ny, nx); ny == 1 in 2-D
    double h[3];            // (hz, hy, hx); hy unused in 2-D
    int r;
    fd_layout L;
    fd::StepParams sp;
    fd::Tuning tune;
    float *vdt2 = nullptr;        // padded v^2 dt^2
    // padded c_pp = c (1 + 2 eps), c_x = c sqrt(1 + 2 delta), the tilt t and
    // azimuth f, and the symmetry axis (a_z, a_y, a_x) = (cos t, sin t sin f,
    // sin t cos f) of each point (read by the one-kernel step)
    float *tti[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // elastic medium times dt at each component's position (padded):
    // b dt at vx, vy, vz; lambda dt, mu dt at nodes; mu dt at txy, txz, tyz
    // visco-elastic: 17 fields (b dt at the velocities; at nodes the unrelaxed
    // moduli times dt, the memory forcing moduli and dt / tau_s; the same
    // three at each shear-stress position)
    float *el[17] = {};
    float *facebase = nullptr;    // the six loopback face buffers, back to back
    float *facebuf[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // into facebase
    float *inter[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // TTI pass-1 output
    unsigned *scratch_u32 = nullptr;  // small device scratch (model checks)
    bool model_loaded = false;
    std::vector<hipEvent_t> prof_ev;  // armed step-kernel timing events (pairs)
    int prof_used = 0;
    // set for one launch while profiling: the z-march step kernel is launched
    // with these as its start/stop events (recorded with the kernel's own
    // dispatch, so they time the kernel alone)
    mutable hipEvent_t launch_ev[2] = {nullptr, nullptr};
    int xmode = 0;                    // FD_XCHG_BASIC / FD_XCHG_FULL
    hipStream_t xs = nullptr;         // exchange stream of full mode
    hipEvent_t xfork = nullptr, xjoin = nullptr;
};

namespace fd {

// Makes the handle's device current for the duration of a call.
class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev_ >= 0) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = -1;
    bool ok_ = true;
};

// geometry shared by single grids and batched shots (fd_api.hip)
void make_geometry(const fd_grid_desc &d, int ndim, const int n[3], const double h[3], int r,
                   fd_layout &L, StepParams &p);
// stability check of a descriptor (FD_OK or FD_EUNSTABLE with the message set)
int check_stability(const fd_grid_desc &d, int ndim, const double h[3], int r);

// autotuner cache (fd_api.hip): the device's architecture name, and a flat
// JSON object mapping keys to [by, ry, nzb, flags]
std::string device_arch(int device);
bool tune_lookup(const char *path, const std::string &key, int t[4]);
void tune_store(const char *path, const std::string &key, const int t[4]);

// error helpers (fd_api.hip)
int set_error(int code, const std::string &msg);
int check_launch(const char *what);

// kernel launchers; each returns FD_OK or an error code
int launch_step(const fd_grid *g, const float *u, const float *um, float *up, hipStream_t s);
int launch_step_simple(const fd_grid *g, const float *u, const float *um, float *up,
                       hipStream_t s);
// step of full exchange mode: loopback exchange of u on g->xs overlapped
// with the CORE on s, then the REMAINDER on s (k_acoustic.hip)
int launch_step_full(fd_grid *g, float *u, const float *um, float *up, hipStream_t s);
// z-marching step for stencil radius R (k_step_radius.hip, one object per R)
template <int R>
int launch_zmarch_radius(const fd_grid *g, const StepParams &p, const Tuning &t, const float *u,
                         const float *um, float *up, hipStream_t s);
int launch_sparse(const fd_grid *g, float *u, const SparseArgs &inj, const SparseArgs &smp,
                  hipStream_t s);
// injection into u_new and sampling of u_old (a different, finished field)
// in one multi-block launch: the two halves are independent (k_sparse.hip)
int launch_sparse_split(const fd_grid *g, float *u_new, const SparseArgs &inj,
                        const float *u_old, const SparseArgs &smp, hipStream_t s);
int launch_pack(const fd_grid *g, const float *field, unsigned mask, float *const *buf,
                hipStream_t s);
int launch_unpack(const fd_grid *g, float *field, unsigned mask, const float *const *buf,
                  hipStream_t s);
int launch_loopback(const fd_grid *g, float *field, float *const *buf, hipStream_t s);
int launch_swap(float *a, float *b, int64_t n, hipStream_t s);
int launch_copy(float *dst, const float *src, int64_t n, hipStream_t s);
int launch_build_vdt2(const fd_grid *g, const float *vel, float *vdt2, unsigned *vmax_bits,
                      hipStream_t s);
int launch_imaging(const fd_grid *g, const float *lam, const float *up, const float *u0,
                   const float *um, float *grad, hipStream_t s);
int launch_grad_to_vel(const fd_grid *g, const float *gm, float *gv, hipStream_t s);
int launch_tti_model(const fd_grid *g, const float *vel, const float *const *tti, unsigned *flags,
                     hipStream_t s);
int launch_tti_step(const fd_grid *g, const float *p, const float *pm, float *pp, const float *r,
                    const float *rm, float *rp, hipStream_t s);
// isotropic elastic (k_elastic.hip): medium build with validity flags, the
// velocity and stress passes in place on the nine components {vx, vy, vz,
// txx, tyy, tzz, txy, txz, tyz}, and explosive-source / stress-trace sparse
int launch_el_model(const fd_grid *g, const float *vp, const float *vs, const float *rho,
                    unsigned *flags, hipStream_t s);
int launch_el_velocity(const fd_grid *g, float *const *f, hipStream_t s);
int launch_el_stress(const fd_grid *g, float *const *f, hipStream_t s);
int launch_el_sparse(const fd_grid *g, float *const *f, const SparseArgs &inj,
                     const SparseArgs &smp, hipStream_t s);
// visco-elastic (k_elastic.hip): medium build from vp and aux = {vs, rho,
// tau_ep, tau_es, tau_s}; the stress-memory pass on the fifteen components
// (the velocity pass is the elastic one)
int launch_vi_model(const fd_grid *g, const float *vp, const float *const *aux, unsigned *flags,
                    hipStream_t s);
int launch_vi_stress(const fd_grid *g, float *const *f, hipStream_t s);
// z-marching TTI steps for 3-D grids whose tile is not the one-thread-per-
// point kernel: two passes through memory (k_tti_zmarch.hip, the default) or
// one kernel (k_tti_fused.hip, tile flag kTileTti1)
int launch_tti_step_zm(const fd_grid *g, const float *p, const float *pm, float *pp,
                       const float *r, const float *rm, float *rp, hipStream_t s);
int launch_tti_step_fused(const fd_grid *g, const float *p, const float *pm, float *pp,
                          const float *r, const float *rm, float *rp, hipStream_t s);

}  // namespace fd
