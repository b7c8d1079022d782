// Halo face pack / unpack and state swap.
//
// The "basic" exchange pattern sends one message per face (table "Summary of
// communication/computation patterns": 6 messages in 3-D).  pack copies the
// r-deep OWNED slab next to each selected face into a contiguous device
// buffer; unpack copies a received buffer into the HALO slab beyond a face.
// All selected faces go in one launch (blockIdx.y = face).  Element k of a
// face buffer is slab point (k / (c1 c2), (k / c2) % c1, k % c2) in field axis
// order, so the z and y faces move whole 128-byte-aligned rows.
#include "fd_internal.h"

namespace fd {

struct FaceJob {
    float *buf[6];
    int cnt[6][3];        // slab extent (z, y, x)
    int start[6][3];      // DOMAIN coordinate of the slab origin
    int elems[6];
    int vec[6];           // 1: rows are whole float4 chunks on both sides
};

// One face per blockIdx.y; rows along x are copied as float4 chunks when the
// slab's x extent and origin are multiples of 4 (rows of a padded field are
// 128-byte aligned, buffers are dense), else element by element.
template <bool UNPACK>
__global__ __launch_bounds__(256) void k_faces(float *field, const FaceJob job,
                                               const int64_t offset, const int64_t PY,
                                               const int64_t PZ)
{
    const int f = blockIdx.y;
    const int n = job.elems[f];
    if (n == 0) return;
    const int c1 = job.cnt[f][1], c2 = job.cnt[f][2];
    const int sz = job.start[f][0], sy = job.start[f][1], sx = job.start[f][2];
    float *buf = job.buf[f];
    if (job.vec[f]) {
        const int q2 = c2 >> 2;                 // float4 chunks per row
        const int nq = n >> 2;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nq; e += gridDim.x * blockDim.x) {
            const int i2 = e % q2;
            const int t = e / q2;
            const int i1 = t % c1;
            const int i0 = t / c1;
            const int64_t idx =
                offset + (int64_t)(sz + i0) * PZ + (int64_t)(sy + i1) * PY + (sx + 4 * i2);
            float4 *fp = reinterpret_cast<float4 *>(field + idx);
            float4 *bp = reinterpret_cast<float4 *>(buf) + e;
            if (UNPACK) *fp = *bp;
            else *bp = *fp;
        }
        return;
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int i2 = e % c2;
        const int t = e / c2;
        const int i1 = t % c1;
        const int i0 = t / c1;
        const int64_t idx = offset + (int64_t)(sz + i0) * PZ + (int64_t)(sy + i1) * PY + (sx + i2);
        if (UNPACK) field[idx] = buf[e];
        else buf[e] = field[idx];
    }
}

// Loopback exchange in one pass: face f's OWNED slab is packed into buf[f]
// and, in the same pass, written into the HALO slab beyond face f^1 -- what
// unpack of the buffer received across face f^1 (buf[f] itself on a
// periodic self-neighbour) would write.  Owned slabs lie inside DOMAIN and
// halo slabs outside it, so no element is both read and written.
struct LoopJob {
    FaceJob own;          // owned slabs and their buffers
    int hstart[6][3];     // origin of the halo slab that face f's slab fills
    int nx;               // DOMAIN x extent
    int xline;            // 1: the x faces move whole 128-byte lines (below)
};

__global__ __launch_bounds__(256) void k_faces_loopback(float *field, const LoopJob job,
                                                        const int64_t offset, const int64_t PY,
                                                        const int64_t PZ)
{
    const int f = blockIdx.y;
    const int n = job.own.elems[f];
    if (n == 0) return;
    const int c1 = job.own.cnt[f][1], c2 = job.own.cnt[f][2];
    const int sz = job.own.start[f][0], sy = job.own.start[f][1], sx = job.own.start[f][2];
    const int hz = job.hstart[f][0], hy = job.hstart[f][1], hx = job.hstart[f][2];
    float *buf = job.own.buf[f];
    if (f >= 4 && job.xline) {
        // x faces with nx a multiple of 32 (rows start on a line boundary):
        // the line holding the halo beyond the opposite face is written
        // whole, as a copy of its periodic image (the first or last 32
        // DOMAIN columns), so the store covers a full line; the columns of
        // that line beyond the halo are row padding nothing reads.  The
        // owned slab (R columns at the start or the end of the image) also
        // goes to the face buffer.  8 float4 per row.
        const int R = c2;
        const int sx0 = f == 4 ? 0 : job.nx - 32, hx0 = f == 4 ? job.nx : -32;
        const int so = f == 4 ? 0 : 32 - R;
        const int rows = n / R;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * 8;
             e += gridDim.x * blockDim.x) {
            const int k = e & 7;
            const int t = e >> 3;
            const int i1 = t % c1;
            const int i0 = t / c1;
            const int64_t row = offset + (int64_t)(sz + i0) * PZ + (int64_t)(sy + i1) * PY;
            const float4 v = *reinterpret_cast<const float4 *>(field + row + sx0 + 4 * k);
            *reinterpret_cast<float4 *>(field + row + (int64_t)(hz - sz) * PZ +
                                        (int64_t)(hy - sy) * PY + hx0 + 4 * k) = v;
            if (4 * k >= so && 4 * k < so + R)
                reinterpret_cast<float4 *>(buf)[t * (R >> 2) + ((4 * k - so) >> 2)] = v;
        }
        return;
    }
    if (job.own.vec[f]) {
        const int q2 = c2 >> 2;
        const int nq = n >> 2;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nq; e += gridDim.x * blockDim.x) {
            const int i2 = e % q2;
            const int t = e / q2;
            const int i1 = t % c1;
            const int i0 = t / c1;
            const float4 v = *reinterpret_cast<const float4 *>(
                field + offset + (int64_t)(sz + i0) * PZ + (int64_t)(sy + i1) * PY + (sx + 4 * i2));
            reinterpret_cast<float4 *>(buf)[e] = v;
            *reinterpret_cast<float4 *>(field + offset + (int64_t)(hz + i0) * PZ +
                                        (int64_t)(hy + i1) * PY + (hx + 4 * i2)) = v;
        }
        return;
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int i2 = e % c2;
        const int t = e / c2;
        const int i1 = t % c1;
        const int i0 = t / c1;
        const float v = field[offset + (int64_t)(sz + i0) * PZ + (int64_t)(sy + i1) * PY + (sx + i2)];
        buf[e] = v;
        field[offset + (int64_t)(hz + i0) * PZ + (int64_t)(hy + i1) * PY + (hx + i2)] = v;
    }
}

static void face_job(const fd_grid *g, unsigned mask, bool halo_side, FaceJob &job, int &maxe)
{
    maxe = 0;
    for (int f = 0; f < 6; ++f) {
        const int axis = f / 2, plus = f & 1;
        const bool active = (mask >> f) & 1u && !(axis == 1 && g->ndim == 2);
        int cnt[3] = {g->n[0], g->n[1], g->n[2]}, st[3] = {0, 0, 0};
        cnt[axis] = g->r;
        if (!halo_side) st[axis] = plus ? g->n[axis] - g->r : 0;
        else st[axis] = plus ? g->n[axis] : -g->r;
        for (int a = 0; a < 3; ++a) {
            job.cnt[f][a] = cnt[a];
            job.start[f][a] = st[a];
        }
        job.elems[f] = active ? cnt[0] * cnt[1] * cnt[2] : 0;
        // DOMAIN x = 0 sits at a multiple of 4 floats in every row
        job.vec[f] = (cnt[2] % 4 == 0 && ((st[2] % 4) + 4) % 4 == 0) ? 1 : 0;
        const int work = job.vec[f] ? job.elems[f] / 4 : job.elems[f];
        if (work > maxe) maxe = work;
    }
}

int launch_pack(const fd_grid *g, const float *field, unsigned mask, float *const *buf,
                hipStream_t s)
{
    FaceJob job;
    int maxe;
    face_job(g, mask, false, job, maxe);
    for (int f = 0; f < 6; ++f) job.buf[f] = job.elems[f] ? buf[f] : nullptr;
    if (maxe == 0) return FD_OK;
    const int nbx = std::min((maxe + 255) / 256, 2048);
    hipLaunchKernelGGL(k_faces<false>, dim3(nbx, 6), dim3(256), 0, s, const_cast<float *>(field),
                       job, g->L.offset, g->L.pitch_y, g->L.pitch_z);
    return check_launch("halo pack");
}

int launch_unpack(const fd_grid *g, float *field, unsigned mask, const float *const *buf,
                  hipStream_t s)
{
    FaceJob job;
    int maxe;
    face_job(g, mask, true, job, maxe);
    for (int f = 0; f < 6; ++f) job.buf[f] = job.elems[f] ? const_cast<float *>(buf[f]) : nullptr;
    if (maxe == 0) return FD_OK;
    const int nbx = std::min((maxe + 255) / 256, 2048);
    hipLaunchKernelGGL(k_faces<true>, dim3(nbx, 6), dim3(256), 0, s, field, job, g->L.offset,
                       g->L.pitch_y, g->L.pitch_z);
    return check_launch("halo unpack");
}

int launch_loopback(const fd_grid *g, float *field, float *const *buf, hipStream_t s)
{
    LoopJob job;
    FaceJob halo;
    int maxe, maxh;
    face_job(g, 0x3fu, false, job.own, maxe);
    face_job(g, 0x3fu, true, halo, maxh);
    for (int f = 0; f < 6; ++f) {
        job.own.buf[f] = job.own.elems[f] ? buf[f] : nullptr;
        // face f's slab fills the halo beyond face f^1; both slabs have the
        // same extents, and the vector path needs both origins 4-aligned
        for (int a = 0; a < 3; ++a) job.hstart[f][a] = halo.start[f ^ 1][a];
        job.own.vec[f] = job.own.vec[f] && halo.vec[f ^ 1];
    }
    job.nx = g->n[2];
    // whole-line x faces: rows start on a line boundary (DOMAIN x = 0 at a
    // multiple of 32 floats), nx a multiple of 32 and the slab whole float4s
    job.xline = (g->ndim == 3 && g->n[2] % 32 == 0 && g->r % 4 == 0 && kXOff % 32 == 0 &&
                 g->L.pitch_y % 32 == 0 && job.own.elems[4] > 0)
                    ? 1
                    : 0;
    if (job.xline) maxe = std::max(maxe, job.own.elems[4] / g->r * 8);
    if (maxe == 0) return FD_OK;
    const int nbx = std::min((maxe + 255) / 256, 2048);
    hipLaunchKernelGGL(k_faces_loopback, dim3(nbx, 6), dim3(256), 0, s, field, job, g->L.offset,
                       g->L.pitch_y, g->L.pitch_z);
    return check_launch("halo loopback exchange");
}

__global__ __launch_bounds__(256) void k_swap(float4 *a, float4 *b, int64_t n4)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float4 t = a[i];
        a[i] = b[i];
        b[i] = t;
    }
}

// One 16-byte element per thread, non-temporal both ways: many short-lived
// blocks keep the most loads in flight (a grid-stride loop over a capped
// grid measured 4.7 TB/s on 2 GiB, this shape 6.6 TB/s).
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy4(v4f *dst, const v4f *src, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(256) void k_copy1(float *dst, const float *src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int launch_copy(float *dst, const float *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return FD_OK;
    if (n % 4 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(src) % 16 == 0) {
        const int64_t n4 = n / 4;
        const int64_t nb = (n4 + 255) / 256;
        if (nb > 0x7fffffff) return set_error(FD_EINVAL, "copy too large");
        hipLaunchKernelGGL(k_copy4, dim3((unsigned)nb), dim3(256), 0, s,
                           reinterpret_cast<v4f *>(dst), reinterpret_cast<const v4f *>(src), n4);
    } else {
        const int nb = (int)std::min<int64_t>((n + 255) / 256, 16384);
        hipLaunchKernelGGL(k_copy1, dim3(nb), dim3(256), 0, s, dst, src, n);
    }
    return check_launch("copy");
}

// n must be a multiple of 4 and both pointers 16-byte aligned (padded fields are)
int launch_swap(float *a, float *b, int64_t n, hipStream_t s)
{
    if (n % 4 || reinterpret_cast<uintptr_t>(a) % 16 || reinterpret_cast<uintptr_t>(b) % 16)
        return set_error(FD_EINVAL, "state fields must be 16-byte aligned");
    const int64_t n4 = n / 4;
    const int nb = (int)std::min<int64_t>((n4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_swap, dim3(nb), dim3(256), 0, s, reinterpret_cast<float4 *>(a),
                       reinterpret_cast<float4 *>(b), n4);
    return check_launch("state swap");
}

}  // namespace fd
