// Host side of the batched multi-shot gradient: per-shot workspaces, the
// device shot table, and the capture of one gradient's whole schedule into
// a hipGraph (forward with checkpoints, per-segment recomputation, adjoint
// with the fused imaging condition, ordered reduction into the full model).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "batch_internal.h"

namespace {

struct ShotHost {
    int n[3] = {0, 0, 0};
    int org[3] = {0, 0, 0};
    fd_layout L{};
    fd::StepParams p{};
    float *ws = nullptr;
    int ns = 0, nr = 0;
    int32_t *sbase = nullptr, *rbase = nullptr;
    float *sfrac = nullptr, *rfrac = nullptr;
    int ntx = 0, nty = 0, nzc = 0, block0 = 0;
};

}  // namespace

struct fd_batch {
    fd_grid_desc d{};
    int nshots = 0, nt = 0, k = 1, nck = 0, nfields = 0, r = 0;
    double h[3] = {0, 0, 0};
    int64_t full[3] = {0, 0, 0};
    std::vector<ShotHost> sh;
    fd::BatchShot *table = nullptr;
    fd::Tuning tune{8, 2, 32, fd::kTileRing | fd::kTileNts};
    int total_blocks = 0;
    const float *vel_full = nullptr;
    unsigned *scratch = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> key;
    size_t bytes = 0;
    int64_t max_stride = 0, max_pts = 0, max_rows = 0;
    bool model_loaded = false;
};

namespace fd {
namespace {

void drop_graph(fd_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key.clear();
}

void layout_blocks(fd_batch *b)
{
    const int ty = b->tune.by * b->tune.ry;
    const int tx = (b->tune.flags & fd::kTileWide) ? 128 : 64;
    int acc = 0;
    for (ShotHost &s : b->sh) {
        s.ntx = (s.n[2] + tx - 1) / tx;
        s.nty = (s.n[1] + ty - 1) / ty;
        s.nzc = (s.n[0] + b->tune.nzb - 1) / b->tune.nzb;
        s.block0 = acc;
        acc += s.ntx * s.nty * s.nzc;
    }
    b->total_blocks = acc;
}

int upload_table(fd_batch *b, const float *const *q, const float *const *dobs, float *const *d)
{
    std::vector<BatchShot> t(b->nshots);
    for (int i = 0; i < b->nshots; ++i) {
        const ShotHost &s = b->sh[i];
        BatchShot &e = t[i];
        e.p = s.p;
        e.base = s.ws;
        e.stride = s.L.field_elems;
        e.ntx = s.ntx;
        e.nty = s.nty;
        e.nzc = s.nzc;
        e.block0 = s.block0;
        for (int a = 0; a < 3; ++a) e.org[a] = s.org[a];
        e.ns = s.ns;
        e.nr = s.nr;
        e.sbase = s.sbase;
        e.sfrac = s.sfrac;
        e.rbase = s.rbase;
        e.rfrac = s.rfrac;
        e.q = q ? q[i] : nullptr;
        e.dobs = dobs ? dobs[i] : nullptr;
        e.d = d ? d[i] : nullptr;
    }
    if (hipMemcpy(b->table, t.data(), sizeof(BatchShot) * t.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return set_error(FD_EDEVICE, "shot table upload failed");
    return FD_OK;
}

void free_batch(fd_batch *b)
{
    drop_graph(b);
    for (ShotHost &s : b->sh) {
        (void)hipFree(s.ws);
        (void)hipFree(s.sbase);
        (void)hipFree(s.sfrac);
        (void)hipFree(s.rbase);
        (void)hipFree(s.rfrac);
    }
    (void)hipFree(b->table);
    (void)hipFree(b->scratch);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

// the whole gradient schedule, enqueued on s (captured once into a graph)
int enqueue_schedule(fd_batch *b, float *grad_v, hipStream_t s)
{
    const BatchShot *T = b->table;
    const int ns = b->nshots;
    const int k = b->k;
    const float hinv = (float)(1.0 / (b->h[0] * b->h[1] * b->h[2]));
    const double dt = b->d.dt;
    const float inv_dt2 = (float)(1.0 / (dt * dt)), inv_2dt = (float)(0.5 / dt);
    const int slot0 = kCkpt0 + 2 * b->nck;
    int rc;
#define FD_TRY(x) \
    if ((rc = (x))) return rc
    for (int f : {(int)kFA, (int)kFB, (int)kLA, (int)kLB, (int)kGrad})
        FD_TRY(launch_batch_zero(T, ns, b->max_stride, f, s));
    // The forward run, with a checkpoint at the start of every segment but
    // the last: the last segment's steps store their imaging factors D_n
    // (as its recomputation would, in slot0 + 2 + (n - lo)), so that segment
    // is not recomputed.
    BatchEpi rec;
    rec.mode = 1;
    rec.inv_dt2 = inv_dt2;
    rec.inv_2dt = inv_2dt;
    const int lo_last = (b->nck - 1) * k;
    int cur = kFA, prev = kFB;
    for (int n = 0; n < b->nt; ++n) {
        if (n % k == 0 && n < lo_last) {
            FD_TRY(launch_batch_copy(T, ns, b->max_stride, cur, kCkpt0 + 2 * (n / k), s));
            FD_TRY(launch_batch_copy(T, ns, b->max_stride, prev, kCkpt0 + 2 * (n / k) + 1, s));
        }
        if (n >= lo_last) {
            rec.fd = slot0 + 2 + (n - lo_last);
            FD_TRY(launch_batch_step(T, ns, b->total_blocks, b->r, b->tune, cur, prev, prev, s, rec));
            FD_TRY(launch_batch_sparse(T, ns, 0, n, prev, hinv, s, rec.fd, inv_dt2, inv_2dt));
        } else {
            FD_TRY(launch_batch_step(T, ns, b->total_blocks, b->r, b->tune, cur, prev, prev, s));
            FD_TRY(launch_batch_sparse(T, ns, 0, n, prev, hinv, s));
        }
        std::swap(cur, prev);
    }
    // Per checkpoint segment [lo, hi), last segment first: recompute the
    // forward steps from the checkpoint in two rolling fields (slot0,
    // slot0 + 1), each step also storing the imaging factor D_n of its
    // update in slot0 + 2 + (n - lo) (the forward run stored the last
    // segment's); then the adjoint steps n = hi-1 .. lo.
    // The imaging condition g -= lambda_n D_n for n > lo rides on the
    // adjoint step that reads lambda_n (the next one, n - 1); lambda_lo is
    // imaged by its own pass before the next segment overwrites the D slots.
    int lam = kLA, lamo = kLB;
    BatchEpi img;
    img.mode = 2;
    img.fg = kGrad;
    img.inv_dt2 = inv_dt2;
    img.inv_2dt = inv_2dt;
    for (int j = b->nck - 1; j >= 0; --j) {
        const int lo = j * k, hi = std::min(b->nt, (j + 1) * k);
        int cu = slot0 + 1, cp = slot0;
        if (j < b->nck - 1) {
            FD_TRY(launch_batch_copy(T, ns, b->max_stride, kCkpt0 + 2 * j, cu, s));
            FD_TRY(launch_batch_copy(T, ns, b->max_stride, kCkpt0 + 2 * j + 1, cp, s));
        }
        for (int i = 0; i < hi - lo && j < b->nck - 1; ++i) {
            rec.fd = slot0 + 2 + i;
            FD_TRY(launch_batch_step(T, ns, b->total_blocks, b->r, b->tune, cu, cp, cp, s, rec));
            FD_TRY(launch_batch_sparse(T, ns, 1, lo + i, cp, hinv, s, rec.fd, inv_dt2, inv_2dt));
            std::swap(cu, cp);
        }
        for (int n = hi - 1; n >= lo; --n) {
            if (n + 1 < hi) {
                img.fd = slot0 + 2 + (n + 1 - lo);
                FD_TRY(launch_batch_step(T, ns, b->total_blocks, b->r, b->tune, lam, lamo, lamo,
                                         s, img));
            } else {
                FD_TRY(launch_batch_step(T, ns, b->total_blocks, b->r, b->tune, lam, lamo, lamo,
                                         s));
            }
            FD_TRY(launch_batch_sparse(T, ns, 2, n, lamo, hinv, s));
            std::swap(lam, lamo);
        }
        FD_TRY(launch_batch_imaging_d(T, ns, b->max_rows, lam, slot0 + 2, s));
    }
    FD_TRY(launch_batch_reduce(T, ns, b->full, b->vel_full, grad_v, s));
#undef FD_TRY
    return FD_OK;
}

}  // namespace
}  // namespace fd

using namespace fd;

extern "C" {

int fd_batch_create(const fd_grid_desc *common, int nshots, const int64_t *shapes,
                    const int64_t *origins, const int64_t *full_shape, int nt, int ckpt_every,
                    fd_batch **out)
{
    if (!common || !shapes || !origins || !full_shape || !out || nshots < 1 || nshots > 1024 ||
        nt < 1 || ckpt_every < 1)
        return set_error(FD_EINVAL, "fd_batch_create: bad argument");
    *out = nullptr;
    const fd_grid_desc &d = *common;
    if (d.space_order < 2 || d.space_order > 16 || d.space_order % 2)
        return set_error(FD_EINVAL, "space_order must be even, 2..16");
    if (!(d.dt > 0.0) || !(d.vmax > 0.0) || d.nbl < 0)
        return set_error(FD_EINVAL, "dt, vmax must be > 0 and nbl >= 0");
    double h[3];
    for (int a = 0; a < 3; ++a) {
        h[a] = d.spacing[a];
        if (!(h[a] > 0.0)) return set_error(FD_EINVAL, "spacing must be > 0");
        if (full_shape[a] < 1) return set_error(FD_EINVAL, "bad full shape");
    }
    const int r = d.space_order / 2;
    fd_grid_desc dd = d;
    dd.physics = FD_ACOUSTIC;
    dd.boundary = FD_BC_ZERO;
    dd.ndim = 3;
    if (check_stability(dd, 3, h, r)) return FD_EUNSTABLE;

    fd_batch *b = new fd_batch();
    b->d = dd;
    b->nshots = nshots;
    b->nt = nt;
    b->k = std::min(ckpt_every, nt);
    b->nck = (nt + b->k - 1) / b->k;
    b->nfields = kCkpt0 + 2 * b->nck + b->k + 2;
    b->r = r;
    for (int a = 0; a < 3; ++a) {
        b->h[a] = h[a];
        b->full[a] = full_shape[a];
    }
    b->sh.resize(nshots);
    for (int i = 0; i < nshots; ++i) {
        ShotHost &s = b->sh[i];
        for (int a = 0; a < 3; ++a) {
            const int64_t n = shapes[3 * i + a], o = origins[3 * i + a];
            if (n < std::max(2, r) || 2 * d.nbl > n || o < 0 || o + n > full_shape[a]) {
                delete b;
                return set_error(FD_EINVAL, "shot " + std::to_string(i) +
                                                ": aperture outside the model or too small");
            }
            s.n[a] = (int)n;
            s.org[a] = (int)o;
        }
        make_geometry(dd, 3, s.n, h, r, s.L, s.p);
        b->max_stride = std::max<int64_t>(b->max_stride, s.L.field_elems);
        b->max_pts = std::max<int64_t>(b->max_pts, (int64_t)s.n[0] * s.n[1] * s.n[2]);
        b->max_rows = std::max<int64_t>(b->max_rows, (int64_t)s.n[0] * s.n[1]);
    }
    layout_blocks(b);
    DeviceGuard dg(d.device);
    if (!dg.ok()) {
        delete b;
        return set_error(FD_EDEVICE, "cannot select device");
    }
    for (ShotHost &s : b->sh) {
        const size_t bytes = s.L.field_bytes * (size_t)b->nfields;
        if (hipMalloc(&s.ws, bytes) != hipSuccess) {
            free_batch(b);
            return set_error(FD_ENOMEM, "shot workspace allocation failed");
        }
        if (hipMemset(s.ws, 0, bytes) != hipSuccess) {
            free_batch(b);
            return set_error(FD_EDEVICE, "hipMemset failed");
        }
        b->bytes += bytes;
    }
    if (hipMalloc(&b->table, sizeof(BatchShot) * nshots) != hipSuccess ||
        hipMalloc(&b->scratch, 256) != hipSuccess || hipStreamCreate(&b->cap) != hipSuccess) {
        free_batch(b);
        return set_error(FD_ENOMEM, "batch allocation failed");
    }
    *out = b;
    return FD_OK;
}

void fd_batch_destroy(fd_batch *b)
{
    if (!b) return;
    DeviceGuard dg(b->d.device);
    free_batch(b);
}

size_t fd_batch_device_bytes(const fd_batch *b) { return b ? b->bytes : 0; }

int fd_batch_set_tile(fd_batch *b, int by, int ry, int nzb, int xcd)
{
    if (!b) return set_error(FD_EINVAL, "fd_batch_set_tile: null handle");
    const bool known = (by == 4 && (ry == 1 || ry == 2 || ry == 4 || ry == 8)) ||
                       (by == 8 && (ry == 2 || ry == 4)) || (by == 2 && ry == 8);
    const bool wide_ok = (by == 8 && ry == 2) || (by == 4 && (ry == 2 || ry == 4));
    if (!known || nzb < 1 || xcd < 0 || xcd > 31 || ((xcd & kTileWide) && !wide_ok))
        return set_error(FD_EINVAL, "unsupported tile shape");
    DeviceGuard dg(b->d.device);
    drop_graph(b);
    b->tune = Tuning{by, ry, nzb, xcd};
    layout_blocks(b);
    return FD_OK;
}

int fd_batch_autotune(fd_batch *b, const char *cache_path, int *out4, double *ms_out,
                      void *stream)
{
    if (!b) return set_error(FD_EINVAL, "fd_batch_autotune: null handle");
    if (!b->model_loaded) return set_error(FD_EINVAL, "fd_batch_autotune: load a model first");
    DeviceGuard dg(b->d.device);
    hipStream_t s = (hipStream_t)stream;
    // key: architecture, space order and the ordered list of aperture shapes
    // (FNV-1a over their extents)
    uint64_t hsh = 1469598103934665603ull;
    for (const ShotHost &sh : b->sh)
        for (int a = 0; a < 3; ++a) {
            hsh ^= (uint64_t)sh.n[a];
            hsh *= 1099511628211ull;
        }
    char hx[24];
    std::snprintf(hx, sizeof hx, "%016llx", (unsigned long long)hsh);
    const std::string key = device_arch(b->d.device) + "|batch|" +
                            std::to_string(b->d.space_order) + "|" + std::to_string(b->nshots) +
                            "|" + hx;
    int best[4] = {b->tune.by, b->tune.ry, b->tune.nzb, b->tune.flags};
    if (cache_path && tune_lookup(cache_path, key, best) &&
        fd_batch_set_tile(b, best[0], best[1], best[2], best[3]) == FD_OK) {
        if (out4) std::memcpy(out4, best, sizeof best);
        if (ms_out) *ms_out = 0.0;
        return FD_OK;
    }
    // timed search over tiles, z chunks and flag sets on the batch's own
    // forward fields (the gradient zeroes them before use); every candidate
    // is one launch of the batched step over all shots
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(FD_EDEVICE, "sync failed");
    drop_graph(b);
    const Tuning saved = b->tune;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = FD_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = set_error(FD_EDEVICE, "fd_batch_autotune: event creation failed");
    const int cand[7][2] = {{4, 1}, {4, 2}, {4, 4}, {4, 8}, {8, 2}, {8, 4}, {2, 8}};
    const int nzbs[3] = {16, 32, 64};
    // every batched variant takes the halo-ring body, so the flag sets differ
    // in the non-temporal hints, the 128-wide tile and the XCD remap
    const int flagsets[4] = {kTileRing, kTileRing | kTileNts, kTileWide | kTileRing | kTileNts,
                             kTileXcd | kTileRing | kTileNts};
    double best_ms = 1e30;
    auto time_one = [&](float *ms) -> int {
        layout_blocks(b);
        int r = upload_table(b, nullptr, nullptr, nullptr);
        if (r) return r;
        if ((r = launch_batch_step(b->table, b->nshots, b->total_blocks, b->r, b->tune, kFA, kFB,
                                   kFB, s)))
            return r;
        if (hipEventRecord(e0, s) != hipSuccess)
            return set_error(FD_EDEVICE, "fd_batch_autotune: hipEventRecord failed");
        for (int i = 0; i < 3; ++i)
            if ((r = launch_batch_step(b->table, b->nshots, b->total_blocks, b->r, b->tune,
                                       i % 2 ? kFB : kFA, i % 2 ? kFA : kFB, i % 2 ? kFA : kFB,
                                       s)))
                return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return set_error(FD_EDEVICE, "fd_batch_autotune: event timing failed");
        return FD_OK;
    };
    for (int ci = 0; ci < 7 && rc == FD_OK; ++ci)
        for (int zi = 0; zi < 3 && rc == FD_OK; ++zi)
            for (int fi = 0; fi < 4 && rc == FD_OK; ++fi) {
                const int *c = cand[ci];
                const int fl = flagsets[fi];
                const bool wide_ok = (c[0] == 8 && c[1] == 2) ||
                                     (c[0] == 4 && (c[1] == 2 || c[1] == 4));
                if ((fl & kTileWide) && !wide_ok) continue;
                b->tune = Tuning{c[0], c[1], nzbs[zi], fl};
                float ms = 0.0f;
                if ((rc = time_one(&ms))) break;
                if (ms / 3.0 < best_ms) {
                    best_ms = ms / 3.0;
                    best[0] = c[0];
                    best[1] = c[1];
                    best[2] = nzbs[zi];
                    best[3] = fl;
                }
            }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    b->tune = saved;
    layout_blocks(b);
    if (rc) return rc;   // nothing cached, the batch keeps its tile
    if ((rc = fd_batch_set_tile(b, best[0], best[1], best[2], best[3]))) return rc;
    if (cache_path) tune_store(cache_path, key, best);
    if (out4) std::memcpy(out4, best, sizeof best);
    if (ms_out) *ms_out = best_ms;
    return FD_OK;
}

int fd_batch_get_tile(const fd_batch *b, int *out4)
{
    if (!b || !out4) return set_error(FD_EINVAL, "fd_batch_get_tile: bad argument");
    out4[0] = b->tune.by;
    out4[1] = b->tune.ry;
    out4[2] = b->tune.nzb;
    out4[3] = b->tune.flags;
    return FD_OK;
}

int fd_batch_set_geometry(fd_batch *b, int shot, const double *src_m, int ns, const double *rec_m,
                          int nr)
{
    if (!b || shot < 0 || shot >= b->nshots || ns < 0 || nr < 0 || (ns && !src_m) ||
        (nr && !rec_m))
        return set_error(FD_EINVAL, "fd_batch_set_geometry: bad argument");
    ShotHost &s = b->sh[shot];
    auto prep = [&](const double *c, int n, std::vector<int32_t> &bs, std::vector<float> &fr) {
        bs.resize(3 * (size_t)n);
        fr.resize(3 * (size_t)n);
        for (int p = 0; p < n; ++p)
            for (int a = 0; a < 3; ++a) {
                const double x = c[3 * p + a] / b->h[a];
                if (!(x >= 0.0) || x > (double)(s.n[a] - 1)) return false;
                int64_t i = (int64_t)std::floor(x);
                if (i > s.n[a] - 2) i = s.n[a] - 2;
                bs[3 * p + a] = (int32_t)i;
                fr[3 * p + a] = (float)(x - (double)i);
            }
        return true;
    };
    std::vector<int32_t> sb, rb;
    std::vector<float> sf, rf;
    if (!prep(src_m, ns, sb, sf) || !prep(rec_m, nr, rb, rf))
        return set_error(FD_EINVAL, "shot " + std::to_string(shot) + ": sparse point outside aperture");
    DeviceGuard dg(b->d.device);
    drop_graph(b);
    for (void *p : {(void *)s.sbase, (void *)s.sfrac, (void *)s.rbase, (void *)s.rfrac})
        (void)hipFree(p);
    s.sbase = s.rbase = nullptr;
    s.sfrac = s.rfrac = nullptr;
    auto up = [](void **dst, const void *src, size_t bytes) {
        if (bytes == 0) return true;
        return hipMalloc(dst, bytes) == hipSuccess &&
               hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up((void **)&s.sbase, sb.data(), sb.size() * 4) ||
        !up((void **)&s.sfrac, sf.data(), sf.size() * 4) ||
        !up((void **)&s.rbase, rb.data(), rb.size() * 4) ||
        !up((void **)&s.rfrac, rf.data(), rf.size() * 4))
        return set_error(FD_ENOMEM, "geometry upload failed");
    s.ns = ns;
    s.nr = nr;
    return FD_OK;
}

int fd_batch_set_model(fd_batch *b, const float *vel_full_dev, void *stream)
{
    if (!b || !vel_full_dev) return set_error(FD_EINVAL, "fd_batch_set_model: bad argument");
    DeviceGuard dg(b->d.device);
    hipStream_t s = (hipStream_t)stream;
    drop_graph(b);
    int rc = upload_table(b, nullptr, nullptr, nullptr);
    if (rc) return rc;
    if (hipMemsetAsync(b->scratch, 0, sizeof(unsigned), s) != hipSuccess)
        return set_error(FD_EDEVICE, "hipMemsetAsync failed");
    if ((rc = launch_batch_vdt2(b->table, b->nshots, b->max_pts, b->full, vel_full_dev,
                                (float)(b->d.dt * b->d.dt), b->scratch, s)))
        return rc;
    unsigned bits = 0;
    if (hipMemcpyAsync(&bits, b->scratch, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(FD_EDEVICE, "model check failed");
    float vmax;
    std::memcpy(&vmax, &bits, sizeof(float));
    if (!(vmax <= (float)b->d.vmax * (1.0f + 1e-6f))) {
        b->model_loaded = false;
        return set_error(FD_EUNSTABLE, "velocity model exceeds vmax or is not positive");
    }
    b->vel_full = vel_full_dev;
    b->model_loaded = true;
    return FD_OK;
}

int fd_batch_gradient(fd_batch *b, const float *const *q_dev, const float *const *dobs_dev,
                      float *const *d_dev, float *grad_v_dev, void *stream)
{
    if (!b || !q_dev || !dobs_dev || !d_dev || !grad_v_dev)
        return set_error(FD_EINVAL, "fd_batch_gradient: bad argument");
    if (!b->model_loaded) return set_error(FD_EINVAL, "fd_batch_gradient: no model loaded");
    for (int i = 0; i < b->nshots; ++i) {
        const ShotHost &s = b->sh[i];
        if ((s.ns && !q_dev[i]) || (s.nr && (!dobs_dev[i] || !d_dev[i])))
            return set_error(FD_EINVAL, "fd_batch_gradient: null per-shot pointer");
    }
    DeviceGuard dg(b->d.device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<const void *> key;
    for (int i = 0; i < b->nshots; ++i) {
        key.push_back(q_dev[i]);
        key.push_back(dobs_dev[i]);
        key.push_back(d_dev[i]);
    }
    key.push_back(grad_v_dev);
    key.push_back(b->vel_full);
    if (!b->exec || key != b->key) {
        if (hipStreamSynchronize(s) != hipSuccess) return set_error(FD_EDEVICE, "sync failed");
        drop_graph(b);
        int rc = upload_table(b, q_dev, dobs_dev, d_dev);
        if (rc) return rc;
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return set_error(FD_EDEVICE, "graph capture failed to start");
        rc = enqueue_schedule(b, grad_v_dev, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess || !g) return set_error(FD_EDEVICE, "graph capture failed");
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            return set_error(FD_EDEVICE, "graph instantiation failed");
        }
        b->key = key;
    }
    if (hipGraphLaunch(b->exec, s) != hipSuccess) return set_error(FD_EDEVICE, "graph launch failed");
    return FD_OK;
}

}  // extern "C"
