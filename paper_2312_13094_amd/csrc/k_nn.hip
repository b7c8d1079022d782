// Learned coarse-grid correction network on gfx950 MFMA.
//
// conv3x3x3(3->16) - GELU - conv3x3x3(16->16) - GELU - conv3x3x3(16->1), zero
// "same" padding, BF16 operands, FP32 accumulation.
//
// Forward and data-gradient convolutions are one implicit-GEMM kernel on
// v_mfma_f32_16x16x32_bf16 with the 16 output channels on M and 16
// consecutive x points on N; K runs over (tap, input channel) in steps of 32.
// Activations are channels-last BF16, so every lane feeds its B fragment
// with one 16-byte LDS read (8 channels of one neighbour point) from a
// 10 x 10 x 18-point halo tile, while the A fragments (weights) of all K
// steps stay in registers for the whole block.  Epilogues are fused: bias +
// GELU (keeping the pre-activation for training) or the GELU derivative of
// the data gradient.  The output layer (16 channels -> 1), whose single
// output channel would fill 1 of 16 rows of that tile, is a per-tap GEMM
// (points x taps, K = channels) followed by a gather of the 27 tap values of
// each point's neighbours (k_conv_out_mfma), with the residual update of the
// coarse wavefield fused.
//
// Weight gradients contract over points: M = output channels, N = input
// channels, K = 32 points along x; the tiles are staged channel-major in
// LDS, each wave owns a subset of the 27 taps, and per-block partial sums
// are reduced in a fixed order by a second kernel (deterministic).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fdnn.h"
#include "fd_internal.h"

namespace fd {
namespace nn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// parameter layout (floats)
constexpr int kW1 = 0, kB1 = 1296, kW2 = 1312, kB2 = 8224, kW3 = 8240, kB3 = 8672, kNP = 8673;
// packed fragment sets (each step is 64 lanes x 8 BF16 = 1 KiB)
constexpr int kF1 = 0, kF2 = 7, kF3 = 21, kD3 = 35, kD2 = 42, kSteps = 56;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even; NaN stays a (quiet) NaN.  Branch-free: the
    // epilogues convert many values per lane.
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t q = (u >> 16) | 0x40u;
    return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? q : r);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// two floats -> two BF16 (round to nearest even) in one word, first in the
// low half: one v_cvt_pk_bf16_f32 on gfx950
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2v));
}
__device__ __forceinline__ float lo_bf(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_bf(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// erf(a) for a >= 0 by Abramowitz & Stegun, Handbook of Mathematical
// Functions, formula 7.1.26 (absolute error <= 1.5e-7): with t = 1/(1 + p a),
// erf(a) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-a^2).  The
// caller passes e = exp(-a^2), which GELU's derivative reuses.  About a
// dozen VALU operations instead of a general-purpose erf, which dominated
// the convolution epilogues.
__device__ __forceinline__ float erf_as(float a, float e)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    return 1.0f - q * t * e;
}

// GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2
__device__ __forceinline__ float gelu(float x)
{
    const float a = fabsf(x) * 0.70710678118654752f;
    const float e = __expf(-a * a);
    const float r = erf_as(a, e);
    return 0.5f * x * (1.0f + copysignf(r, x));
}
// gelu() of four values, written stage by stage so that the four
// dependent chains interleave (each value's operations are those of gelu())
__device__ __forceinline__ void gelu4(const float x[4], float y[4])
{
    float a[4], e[4], t[4], q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = fabsf(x[i]) * 0.70710678118654752f;
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a[i], 1.0f));
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = __expf(-a[i] * a[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = fmaf(1.061405429f, t[i], -1.453152027f);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = fmaf(q[i], t[i], 1.421413741f);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = fmaf(q[i], t[i], -0.284496736f);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = fmaf(q[i], t[i], 0.254829592f);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = 1.0f - q[i] * t[i] * e[i];
        y[i] = 0.5f * x[i] * (1.0f + copysignf(r, x[i]));
    }
}

// GELU'(x) = Phi(x) + x phi(x), phi(x) = exp(-x^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_grad(float x)
{
    const float a = fabsf(x) * 0.70710678118654752f;
    const float e = __expf(-a * a);
    const float r = erf_as(a, e);
    return 0.5f * (1.0f + copysignf(r, x)) + x * e * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// weight packing: FP32 parameters -> BF16 A fragments
// ---------------------------------------------------------------------------
__device__ __forceinline__ int flip_tap(int t)
{
    const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
    return (2 - dz) * 9 + (2 - dy) * 3 + (2 - dx);
}

__global__ __launch_bounds__(256) void k_pack_weights(const float *__restrict__ P, uint16_t *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // element of kSteps*64*8
    if (e >= kSteps * 512) return;
    const int step = e / 512, lane = (e / 8) % 64, j = e % 8;
    const int m = lane & 15;
    int set, s, cin;
    if (step < kF2) { set = 0; s = step - kF1; cin = 8; }
    else if (step < kF3) { set = 1; s = step - kF2; cin = 16; }
    else if (step < kD3) { set = 2; s = step - kF3; cin = 16; }
    else if (step < kD2) { set = 3; s = step - kD3; cin = 8; }
    else { set = 4; s = step - kD2; cin = 16; }
    const int k = 32 * s + 8 * (lane >> 4) + j;
    const int tap = k / cin, c = k % cin;
    float w = 0.0f;
    if (tap < 27) {
        switch (set) {
        case 0:   // layer 1 forward: M = co (16), K = (tap, ci < 3)
            if (c < 3) w = P[kW1 + (m * 3 + c) * 27 + tap];
            break;
        case 1:   // layer 2 forward
            w = P[kW2 + (m * 16 + c) * 27 + tap];
            break;
        case 2:   // layer 3 forward: only output channel 0
            if (m == 0) w = P[kW3 + c * 27 + tap];
            break;
        case 3:   // through layer 3: M = ci of layer 3, K = (flipped tap, co < 1)
            if (c == 0) w = P[kW3 + m * 27 + flip_tap(tap)];
            break;
        default:  // through layer 2: M = ci, K = (flipped tap, co)
            w = P[kW2 + (c * 16 + m) * 27 + flip_tap(tap)];
            break;
        }
    }
    out[e] = f2bf(w);
}

// ---------------------------------------------------------------------------
// implicit-GEMM 3x3x3 convolution
// ---------------------------------------------------------------------------
enum Epi { EPI_GELU = 0, EPI_GELU_Z = 1, EPI_DGRAD = 3 };


struct ConvArgs {
    int nz, ny, nx;
    const uint16_t *in;       // channels-last [n][CIN]
    const uint16_t *frag;     // STEPS x 64 lanes x 8 BF16
    const float *bias;        // 16 (EPI_GELU*), 1 (output layer), NULL (EPI_DGRAD)
    uint16_t *a16;            // GELU output
    uint16_t *z16;            // pre-activation out (EPI_GELU_Z) / previous z in (EPI_DGRAD)
    float *ydense;            // output layer: dense y (may be NULL)
    const float *base;        // output layer: residual base (may be NULL with out NULL)
    nn_view vbase;
    float *out;
    nn_view vout;
    const float *scale;       // output layer: s = scale[0] (NULL = 1)
    float gain;               // output layer: out = base + gain * s * y
    nn_box skip;              // output layer: no correction inside (empty = none)
    int znb;                  // output planes per block (set by the launcher)
    // layer 1 staged straight from three fields (nn_conv_gelu_fields):
    // (fa sa, fb sa, fc3) as in k_pack_input, sa = 1 / fscale[0] (or 1)
    const float *fa, *fb, *fc;
    nn_view fva, fvb, fvc;
    int fct;                  // fc3 = fc fa sa (else fc)
    const float *fscale;
};

__device__ __forceinline__ bool in_box(const nn_box &b, int z, int y, int x)
{
    return z >= b.lo[0] && z < b.hi[0] && y >= b.lo[1] && y < b.hi[1] && x >= b.lo[2] &&
           x < b.hi[2];
}

// Epilogue of one MFMA row: bias, activation and stores (lane group g holds
// output channels 4g..4g+3 of its point).  The lane's 8 bytes of point p go
// through buffer descriptors of output plane z at byte offset
// off = 32 p_plane + 8 g (an offset past the plane for points outside the
// volume, whose loads return zero and whose stores are dropped), so the
// epilogue has no control flow.
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
constexpr uint32_t kNnOOB = 0xFFFFFFF0u;     // beyond every plane descriptor
constexpr int kNnWord3 = 0x00020000;         // gfx9 raw buffer: 32-bit data format

template <int EPI>
__device__ __forceinline__ void epilogue_buf(const floatx4 &acc, const __amdgpu_buffer_rsrc_t ra,
                                             const __amdgpu_buffer_rsrc_t rz, const uint32_t off,
                                             const float *bias4)
{
    if (EPI == EPI_DGRAD) {
        const v2u zp = __builtin_amdgcn_raw_buffer_load_b64(rz, off, 0, 0);
        const v2u o = {pack_bf16(acc[0] * gelu_grad(lo_bf(zp.x)), acc[1] * gelu_grad(hi_bf(zp.x))),
                       pack_bf16(acc[2] * gelu_grad(lo_bf(zp.y)), acc[3] * gelu_grad(hi_bf(zp.y)))};
        __builtin_amdgcn_raw_buffer_store_b64(o, ra, off, 0, 0);
    } else {
        const uint32_t z01 = pack_bf16(acc[0] + bias4[0], acc[1] + bias4[1]);
        const uint32_t z23 = pack_bf16(acc[2] + bias4[2], acc[3] + bias4[3]);
        // GELU of the stored (BF16) pre-activation, so training and its
        // backward see the same value
        const float xs[4] = {lo_bf(z01), hi_bf(z01), lo_bf(z23), hi_bf(z23)};
        float ys[4];
        gelu4(xs, ys);
        const v2u o = {pack_bf16(ys[0], ys[1]), pack_bf16(ys[2], ys[3])};
        __builtin_amdgcn_raw_buffer_store_b64(o, ra, off, 0, 0);
        if (EPI == EPI_GELU_Z) __builtin_amdgcn_raw_buffer_store_b64(v2u{z01, z23}, rz, off, 0, 0);
    }
}

// z-marching implicit-GEMM 3x3x3 convolution.  A block owns a 32 x 8 column
// tile and marches over znb output planes.  Input planes (tile plus a 1-point
// ring, channels-last BF16) live in a 4-slot LDS ring: planes z-1, z, z+1
// feed output plane z while plane z+2 is loaded into registers under the
// MFMAs and stored into the free slot afterwards (one barrier per plane).
// Every input plane is fetched once per column tile instead of with a full
// 3-D halo per block.  Per plane each wave computes 4 rows of 16 points (tile
// rows wave/2 + 2j, half wave%2), each row an STEPS-deep chain of
// v_mfma_f32_16x16x32_bf16 with A = the weights (registers, M = 16 output
// channels) and B = 8 consecutive K values of the row's 16 points (LDS).
// The LDS address of a lane's B fragment is fixed per K step up to the ring
// slot of its tap's z offset: it is precomputed once, the three slot bases
// are uniform per plane, and the four rows sit at constant offsets, so a
// fetch costs one address add per step instead of a per-read index
// computation (which had made the kernel bound by vector ALU work).
constexpr int ZX = 32, ZY = 8, ZHX = ZX + 2, ZHY = ZY + 2;

template <int CIN, int STEPS, int EPI, bool FIN = false>
__global__ __launch_bounds__(256) void k_conv(const ConvArgs a)
{
    static_assert(!FIN || CIN == 8, "fields input is layer 1's");
    constexpr int CH = CIN / 8;                 // 16-byte chunks per point
    // staged row pitch: with two chunks per point it is padded to 36 points
    // so that the bank swizzle (bit 2 of the point index) is the same in
    // every row a wave reads
    constexpr int ZHXS = CH == 2 ? 36 : ZHX;
    constexpr int PLANE = ZHY * ZHXS * CIN;     // BF16 per staged plane
    constexpr int PB = PLANE * 2;               // bytes per staged plane
    constexpr int NCH = ZHY * ZHX * CH;         // chunks per staged plane
    constexpr int NIT = (NCH + 255) / 256;
    constexpr int NR = 4;                       // rows per wave and plane
    constexpr int ROWB = 2 * ZHXS * CIN * 2;    // bytes between a wave's rows
    __shared__ __attribute__((aligned(16))) uint16_t ring[4 * PLANE];
    const int ntx = (a.nx + ZX - 1) / ZX, nty = (a.ny + ZY - 1) / ZY;
    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int x0 = tx * ZX, y0 = ty * ZY, z0 = zc * a.znb, z1 = min(z0 + a.znb, a.nz);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;

    // weights: all K steps resident in registers
    bf16x8 af[STEPS];
    const bf16x8 *fr = reinterpret_cast<const bf16x8 *>(a.frag);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) af[s] = fr[s * 64 + lane];

    // this lane's biases (output channels 4g..4g+3; channel 0 for layer 3)
    float bias4[4] = {0.f, 0.f, 0.f, 0.f};
    if (EPI != EPI_DGRAD)
#pragma unroll
        for (int j = 0; j < 4; ++j) bias4[j] = a.bias[4 * g + j];

    const float inv = FIN && a.fscale ? 1.0f / a.fscale[0] : 1.0f;
    // staging through buffer descriptors of input plane zz (empty outside
    // the volume): this thread's in-plane byte offsets are fixed over the
    // march, past the plane for points outside the volume, whose loads
    // return zero
    const int64_t plane = (int64_t)a.ny * a.nx;
    uint32_t soff[NIT], sfa[FIN ? NIT : 1], sfb[FIN ? NIT : 1], sfc[FIN ? NIT : 1];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int c = tid + it * 256;
        const int pt = c / CH, ch = c % CH;
        const int gx = x0 - 1 + pt % ZHX, gy = y0 - 1 + pt / ZHX;
        const bool in = c < NCH && gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny;
        soff[it] = in ? (uint32_t)((((int64_t)gy * a.nx + gx) * CH + ch) * 16) : kNnOOB;
        if constexpr (FIN) {
            sfa[it] = in ? (uint32_t)((gy * a.fva.pitch_y + gx) * 4) : kNnOOB;
            sfb[it] = in ? (uint32_t)((gy * a.fvb.pitch_y + gx) * 4) : kNnOOB;
            sfc[it] = in ? (uint32_t)((gy * a.fvc.pitch_y + gx) * 4) : kNnOOB;
        }
    }
    auto plane_rsrc = [&](const void *base, const int64_t elem_off, const int bytes,
                          const bool zin) {
        return __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const char *)base + (zin ? elem_off : 0)), (short)0, zin ? bytes : 0,
            kNnWord3);
    };
    uint4 stage[NIT];
    // plane zz of the tile + ring into registers (zero outside the volume);
    // from the three fields, the point's packed input is formed here with
    // k_pack_input's arithmetic
    auto load_plane = [&](const int zz) {
        const bool zin = zz >= 0 && zz < a.nz;
        if constexpr (FIN) {
            const auto ra = plane_rsrc(a.fa, (a.fva.offset + zz * a.fva.pitch_z) * 4,
                                       (int)(a.fva.pitch_z * 4), zin);
            const auto rb = plane_rsrc(a.fb, (a.fvb.offset + zz * a.fvb.pitch_z) * 4,
                                       (int)(a.fvb.pitch_z * 4), zin);
            const auto rc = plane_rsrc(a.fc, (a.fvc.offset + zz * a.fvc.pitch_z) * 4,
                                       (int)(a.fvc.pitch_z * 4), zin);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                // k_pack_input's products; the packed conversion rounds to
                // nearest even as f2bf does (they differ only in the bits of
                // a NaN); zeros outside the volume stay zeros
                const float va_ = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(ra, sfa[it], 0, 0)) * inv;
                const float vb_ = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rb, sfb[it], 0, 0)) * inv;
                const float cv = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rc, sfc[it], 0, 0));
                const float vc_ = a.fct ? cv * va_ : cv;
                stage[it] = make_uint4(pack_bf16(va_, vb_), pack_bf16(vc_, 0.0f), 0u, 0u);
            }
        } else {
            const auto rs = plane_rsrc(a.in, zz * plane * CIN * 2, (int)(plane * CIN * 2), zin);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                typedef unsigned int v4u __attribute__((ext_vector_type(4)));
                const v4u v = __builtin_amdgcn_raw_buffer_load_b128(rs, soff[it], 0, 0);
                stage[it] = make_uint4(v.x, v.y, v.z, v.w);
            }
        }
    };
    // with two chunks per point, the chunks of points whose (padded) index
    // has bit 2 set are stored swapped, so the 8 lanes served together by a
    // 128-bit LDS read (8 consecutive points, 32 bytes apart) hit distinct
    // banks
    auto store_plane = [&](const int zz) {
        uint4 *dst = reinterpret_cast<uint4 *>(ring + (zz & 3) * PLANE);
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int c = tid + it * 256;
            const int pt = c / CH, ch = c % CH;
            const int cc = ((pt / ZHX) * ZHXS + pt % ZHX) * CH + ch;
            if (c < NCH) dst[CH == 2 ? (cc ^ ((cc >> 3) & 1)) : cc] = stage[it];
        }
    };

    load_plane(z0 - 1);
    store_plane(z0 - 1);
    load_plane(z0);
    store_plane(z0);
    load_plane(z0 + 1);
    store_plane(z0 + 1);
    __syncthreads();

    // per-lane byte offset of the B fragment of every K step within a staged
    // plane (first row of this wave), and whether the lane's tap lies one z
    // offset above the step's first tap (steps whose taps straddle two
    // input planes)
    uint32_t boff[STEPS];
    bool zhi[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        const int kb = 32 * s + 8 * g;
        int tap = kb / CIN;
        tap = tap > 26 ? 26 : tap;              // padding steps: zero weights
        int t0 = (32 * s) / CIN;
        t0 = t0 > 26 ? 26 : t0;
        zhi[s] = tap / 9 != t0 / 9;
        const int pt = (wave / 2) * ZHXS + (wave % 2) * 16 + n + ((tap / 3) % 3) * ZHXS + tap % 3;
        const int c0 = kb % CIN;
        const int cs = CH == 2 ? (c0 ^ (((pt >> 2) & 1) << 3)) : c0;
        boff[s] = (uint32_t)((pt * CIN + cs) * 2);
    }
    const char *ringb = reinterpret_cast<const char *>(ring);
    // this lane's output bytes within a plane for its 4 rows (tile rows
    // wave/2 + 2j, half wave%2), past the plane outside the volume
    const uint32_t pbytes = (uint32_t)(plane * 32);
    uint32_t eoff[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int x = x0 + (wave % 2) * 16 + n, y = y0 + wave / 2 + 2 * j;
        eoff[j] = x < a.nx && y < a.ny ? (uint32_t)(((int64_t)y * a.nx + x) * 32 + 8 * g) : kNnOOB;
    }
    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;
        if (more) load_plane(z + 2);            // in flight under the MFMAs
        // byte bases of the slots holding input planes z - 1, z, z + 1
        const uint32_t sb0 = (uint32_t)(((z + 3) & 3) * PB), sb1 = (uint32_t)((z & 3) * PB),
                       sb2 = (uint32_t)(((z + 1) & 3) * PB);
        auto slot = [&](const int d) { return d == 0 ? sb0 : (d == 1 ? sb1 : sb2); };
        floatx4 acc[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
        // B fragments of step s+1 are read from LDS while the MFMAs of step s
        // run (two register sets)
        auto fetch = [&](const int s, bf16x8 *bv) {
            int d0 = (32 * s) / CIN;
            d0 = (d0 > 26 ? 26 : d0) / 9;
            const uint32_t base = d0 < 2 && zhi[s] ? slot(d0 + 1) : slot(d0);
            const char *p = ringb + base + boff[s];
#pragma unroll
            for (int j = 0; j < NR; ++j)
                bv[j] = *reinterpret_cast<const bf16x8 *>(p + j * ROWB);
        };
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.a16 + z * plane * 16), (short)0, (int)pbytes, kNnWord3);
        const __amdgpu_buffer_rsrc_t rz = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(EPI == EPI_GELU ? a.a16 : a.z16 + z * plane * 16), (short)0,
            EPI == EPI_GELU ? 0 : (int)pbytes, kNnWord3);
        bf16x8 bq[2][NR];
        fetch(0, bq[0]);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            if (s + 1 < STEPS) fetch(s + 1, bq[(s + 1) & 1]);
#pragma unroll
            for (int j = 0; j < NR; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s], bq[s & 1][j], acc[j], 0,
                                                                  0, 0);
        }
#pragma unroll
        for (int j = 0; j < NR; ++j) epilogue_buf<EPI>(acc[j], ra, rz, eoff[j], bias4);
        if (more) store_plane(z + 2);           // slot of plane z-2, read by nobody now
        __syncthreads();
    }
}

// The z chunk: each block marches znb + 2 input planes for znb outputs, and
// the blocks that fit on the device at once (the kernel's occupancy, one
// wave per SIMD per block) run in rounds; the chunk minimises rounds x
// (znb + 2).  Deep chunks on few blocks leave most of the device's block
// slots empty: the march is latency-bound per block (one barrier per plane).
static int pick_znb(int64_t tiles, int nz, int slots)
{
    int best = 16;
    int64_t best_cost = INT64_MAX;
    for (int znb = 1; znb <= 32; ++znb) {
        const int64_t nb = tiles * ((nz + znb - 1) / znb);
        const int64_t cost = ((nb + slots - 1) / slots) * (int64_t)(std::min(znb, nz) + 2);
        if (cost < best_cost || (cost == best_cost && znb > best)) {
            best_cost = cost;
            best = znb;
        }
    }
    return best;
}

// blocks of 256 threads of kernel k resident on the device at once
template <typename K>
static int device_slots(K k, int *slots)
{
    if (*slots > 0) return FD_OK;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
        return set_error(FD_EDEVICE, "nn conv: occupancy query failed");
    *slots = cus * per_cu;
    return FD_OK;
}

template <int CIN, int STEPS, int EPI, bool FIN = false>
static int conv(const ConvArgs &a0, hipStream_t s)
{
    // the epilogue addresses a plane's outputs with 32-bit byte offsets
    if ((int64_t)a0.ny * a0.nx * 32 > 0x7fffffff)
        return set_error(FD_EINVAL, "nn conv: an x-y plane holds at most 2^26 points");
    static int slots = 0;
    if (const int rc = device_slots(k_conv<CIN, STEPS, EPI, FIN>, &slots)) return rc;
    const int64_t tiles = (int64_t)((a0.nx + ZX - 1) / ZX) * ((a0.ny + ZY - 1) / ZY);
    ConvArgs a = a0;
    a.znb = pick_znb(tiles, a.nz, slots);
    const int64_t nb = tiles * ((a.nz + a.znb - 1) / a.znb);
    hipLaunchKernelGGL((k_conv<CIN, STEPS, EPI, FIN>), dim3((unsigned)nb), dim3(256), 0, s, a);
    return check_launch("nn conv");
}

// Layer 3 as a per-tap GEMM on the matrix cores plus a gather.  For every
// point q of a staged input plane (tile + 1-point ring) and every tap t,
// Y[q][t] = sum_c a[q][c] w[t][c] (v_mfma_f32_16x16x16_bf16 with M = 16
// points, N = 16 taps, K = the 16 channels; two MFMAs cover the 27 taps);
// each output point then adds the 9 in-plane neighbours' Y of the taps of
// every z offset into a ring of three accumulators (output planes zi + 1,
// zi, zi - 1), as in the vector version.  The matrix cores do the 432
// multiply-adds per point; the vector ALU 27 additions.  A block of 256
// threads owns a 32 x 8 column tile; Y rows are padded to 33 floats so that
// the gather's lanes hit distinct LDS banks.  (A single staging buffer, 52 KB
// of LDS and three blocks per CU instead of two, measured 5 % slower.)
constexpr int QX = 32, QY = 8, QHX = QX + 2, QHY = QY + 2, NQ = QHX * QHY;
constexpr int NQG = (NQ + 15) / 16, NQP = NQG * 16, QYS = 33;
typedef short short4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_conv_out_mfma(const ConvArgs a)
{
    __shared__ uint4 pl[2][NQP * 2];          // staged planes, 2 x 16 B per point
    __shared__ float yl[NQP * QYS];           // Y of the current input plane
    const int ntx = (a.nx + QX - 1) / QX, nty = (a.ny + QY - 1) / QY;
    int b = blockIdx.x;
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int zc = b / nty;
    const int x0 = tx * QX, y0 = ty * QY, z0 = zc * a.znb, z1 = min(z0 + a.znb, a.nz);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lx = tid % QX, ly = tid / QX;
    const int x = x0 + lx, y = y0 + ly;

    // B operand: taps (lane & 15) + 16 h, channels 4 (lane >> 4) .. + 3; the
    // BF16 weight of tap t, channel c is element k = 16 t + c of output
    // channel 0 in the packed layer-3 fragments
    short4v wb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = (lane & 15) + 16 * h;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * t + 4 * (lane >> 4) + j;
            wb[h][j] = t < 27 ? (short)a.frag[(k / 32) * 512 + ((k % 32) / 8) * 128 + (k % 8)]
                              : (short)0;
        }
    }
    const float bias = a.bias[0];
    const float gs = a.out ? a.gain * (a.scale ? a.scale[0] : 1.0f) : 0.0f;

    // zero the padding points of both staging buffers once
    for (int c = NQ * 2 + tid; c < NQP * 2; c += 256)
        pl[0][c] = pl[1][c] = make_uint4(0u, 0u, 0u, 0u);

    const uint4 *src = reinterpret_cast<const uint4 *>(a.in);
    constexpr int NIT = (NQ * 2 + 255) / 256;
    uint4 sa[NIT], sb[NIT];
    auto load = [&](uint4 *stg, const int zz) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int c = tid + it * 256;
            const int p = c >> 1;
            const int gx = x0 - 1 + p % QHX, gy = y0 - 1 + p / QHX;
            stg[it] = make_uint4(0u, 0u, 0u, 0u);
            if (c < NQ * 2 && zz >= 0 && zz < a.nz && gx >= 0 && gx < a.nx && gy >= 0 &&
                gy < a.ny)
                stg[it] = src[(((int64_t)zz * a.ny + gy) * a.nx + gx) * 2 + (c & 1)];
        }
    };
    auto store = [&](const uint4 *stg, const int buf) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int c = tid + it * 256;
            if (c < NQ * 2) pl[buf][c] = stg[it];
        }
    };

    float a_c = 0.0f, a_m = 0.0f;   // running sums of output planes zi and zi - 1
    auto plane = [&](const int zi, uint4 *stg) {
        const int cb = (zi - z0 + 1) & 1;
        const char *P = reinterpret_cast<const char *>(pl[cb]);
        // Y of every staged point: groups of 16 points dealt to the waves
        for (int g = wave; g < NQG; g += 4) {
            const int q = 16 * g + (lane & 15);
            const short4v av = *reinterpret_cast<const short4v *>(P + q * 32 + (lane >> 4) * 8);
            const floatx4 y0v = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, wb[0],
                                                                          floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            const floatx4 y1v = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, wb[1],
                                                                          floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int qo = 16 * g + 4 * (lane >> 4) + j;
                yl[qo * QYS + (lane & 15)] = y0v[j];
                yl[qo * QYS + 16 + (lane & 15)] = y1v[j];
            }
        }
        __syncthreads();
        // contributions to outputs zi + 1 (taps dz = -1), zi (dz = 0), zi - 1
        float sp = 0.0f, sc = 0.0f, sm = 0.0f;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const float *yq = yl + ((ly + dy) * QHX + lx + dx) * QYS + dy * 3 + dx;
                sp += yq[0];
                sc += yq[9];
                sm += yq[18];
            }
        const float yv = a_m + sm + bias;            // output plane zi - 1 is complete
        a_m = a_c + sc;
        a_c = sp;
        const int zo = zi - 1;
        if (zo >= z0 && x < a.nx && y < a.ny) {
            const int64_t p = ((int64_t)zo * a.ny + y) * a.nx + x;
            if (a.ydense) a.ydense[p] = yv;
            if (a.out) {
                const int64_t ib = a.vbase.offset + zo * a.vbase.pitch_z + y * a.vbase.pitch_y + x;
                const int64_t io = a.vout.offset + zo * a.vout.pitch_z + y * a.vout.pitch_y + x;
                a.out[io] = in_box(a.skip, zo, y, x) ? a.base[ib] : a.base[ib] + gs * yv;
            }
        }
        if (zi + 1 <= z1) store(stg, cb ^ 1);        // buffer of plane zi - 1, consumed
        __syncthreads();
        if (zi + 3 <= z1) load(stg, zi + 3);
    };

    load(sa, z0 - 1);
    store(sa, 0);
    __syncthreads();
    load(sa, z0);
    load(sb, z0 + 1);
    for (int zi = z0 - 1; zi <= z1; zi += 2) {
        plane(zi, sa);
        if (zi + 1 <= z1) plane(zi + 1, sb);
    }
}

static int conv_out_mfma(const ConvArgs &a0, hipStream_t s)
{
    static int slots = 0;
    if (const int rc = device_slots(k_conv_out_mfma, &slots)) return rc;
    const int64_t tiles = (int64_t)((a0.nx + QX - 1) / QX) * ((a0.ny + QY - 1) / QY);
    ConvArgs a = a0;
    a.znb = pick_znb(tiles, a.nz, slots);
    const int64_t nb = tiles * ((a.nz + a.znb - 1) / a.znb);
    hipLaunchKernelGGL(k_conv_out_mfma, dim3((unsigned)nb), dim3(256), 0, s, a);
    return check_launch("nn conv (output layer)");
}


// ---------------------------------------------------------------------------
// weight gradient
// ---------------------------------------------------------------------------
constexpr int TXW = 32, TYW = 4, TZW = 4;                    // points per tile
constexpr int HXW = TXW + 2, HYW = TYW + 2, HZW = TZW + 2;
constexpr int WG_PART = 27 * 256 + 16;                       // floats per block partial
constexpr int WG_BLOCKS = 512;                               // persistent blocks

template <int CIN, int GC>
__global__ __launch_bounds__(256) void k_wgrad(const int nz, const int ny, const int nx,
                                               const uint16_t *__restrict__ x,
                                               const uint16_t *__restrict__ gsrc,
                                               float *__restrict__ part)
{
    __shared__ __attribute__((aligned(16))) uint16_t gt[16][TZW * TYW * TXW];     // channel-major g
    __shared__ __attribute__((aligned(16))) uint16_t xt[16][HZW * HYW * HXW];     // channel-major x
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntx = (nx + TXW - 1) / TXW, nty = (ny + TYW - 1) / TYW, ntz = (nz + TZW - 1) / TZW;
    const int ntiles = ntx * nty * ntz;
    const int m = lane & 15, g = lane >> 4;
    // this wave's taps: wave, wave + 4, ... (7 or 6 taps)
    floatx4 acc[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.0f;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
        const int x0 = tx * TXW, y0 = ty * TYW, z0 = tz * TZW;
        __syncthreads();   // previous tile's reads done
        for (int e = tid; e < 16 * TZW * TYW * TXW; e += 256) {
            const int c = e / (TZW * TYW * TXW), pt = e % (TZW * TYW * TXW);
            const int px = pt % TXW, py = (pt / TXW) % TYW, pz = pt / (TXW * TYW);
            const int gx = x0 + px, gy = y0 + py, gz = z0 + pz;
            uint16_t v = 0;
            if (c < GC && gx < nx && gy < ny && gz < nz)
                v = gsrc[(((int64_t)gz * ny + gy) * nx + gx) * GC + c];
            gt[c][pt] = v;
        }
        for (int e = tid; e < 16 * HZW * HYW * HXW; e += 256) {
            const int c = e / (HZW * HYW * HXW), pt = e % (HZW * HYW * HXW);
            const int hx = pt % HXW, hy = (pt / HXW) % HYW, hz = pt / (HXW * HYW);
            const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
            uint16_t v = 0;
            if (c < CIN && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                v = x[(((int64_t)gz * ny + gy) * nx + gx) * CIN + c];
            xt[c][pt] = v;
        }
        __syncthreads();
        if (wave == 0 && lane < 16) {
            float sacc = 0.0f;
            for (int pt = 0; pt < TZW * TYW * TXW; ++pt) sacc += bf2f(gt[lane][pt]);
            dbacc += sacc;
        }
        for (int row = 0; row < TZW * TYW; ++row) {
            const int zl = row / TYW, yl = row % TYW;
            bf16x8 av;
            {
                const uint16_t *gp = &gt[m][row * TXW + 8 * g];
#pragma unroll
                for (int j = 0; j < 8; ++j) av[j] = __builtin_bit_cast(__bf16, gp[j]);
            }
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                const int tap = wave + 4 * i;
                if (tap < 27) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    const uint16_t *xp = &xt[m][((zl + dz) * HYW + (yl + dy)) * HXW + 8 * g + dx];
                    bf16x8 bv;
#pragma unroll
                    for (int j = 0; j < 8; ++j) bv[j] = __builtin_bit_cast(__bf16, xp[j]);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
                }
            }
        }
    }
    // C[co][ci]: lane holds co = 4 g + j, ci = m
    float *pb = part + (int64_t)blockIdx.x * WG_PART;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int tap = wave + 4 * i;
        if (tap < 27)
#pragma unroll
            for (int j = 0; j < 4; ++j) pb[tap * 256 + (4 * g + j) * 16 + m] = acc[i][j];
    }
    if (wave == 0 && lane < 16) pb[27 * 256 + lane] = dbacc;
}

// grads[layer slice] (+)= sum over blocks (in block order)
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part,
                                                      const int nparts, const int cin_real,
                                                      const int cout_real, float *wout,
                                                      float *bout, const int accumulate)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // co * cin_real * 27 + ci * 27 + tap
    const int nw = cout_real * cin_real * 27;
    if (e < nw) {
        const int tap = e % 27, ci = (e / 27) % cin_real, co = e / (27 * cin_real);
        float s = 0.0f;
        for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * WG_PART + tap * 256 + co * 16 + ci];
        wout[e] = accumulate ? wout[e] + s : s;
    } else if (e < nw + cout_real) {
        const int co = e - nw;
        float s = 0.0f;
        for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * WG_PART + 27 * 256 + co];
        bout[co] = accumulate ? bout[co] + s : s;
    }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_input(const int nz, const int ny, const int nx,
                                                    const float *a, const nn_view va,
                                                    const float *b, const nn_view vb,
                                                    const float *c, const nn_view vc,
                                                    const int c_times_a, const float *scale,
                                                    uint16_t *x8, const int seg)
{
    const float inv = scale ? 1.0f / scale[0] : 1.0f;
    // seg threads per x row, blockDim / seg rows per block iteration (no
    // 64-bit index division)
    const int rpi = blockDim.x / seg, sub = threadIdx.x / seg, xl = threadIdx.x % seg;
    for (int row = blockIdx.x * rpi + sub; row < nz * ny; row += gridDim.x * rpi)
    for (int x = xl; x < nx; x += seg) {
        const int y = row % ny, z = row / ny;
        const int64_t i = (int64_t)row * nx + x;
        const float va_ = a[va.offset + z * va.pitch_z + y * va.pitch_y + x] * inv;
        const float vb_ = b[vb.offset + z * vb.pitch_z + y * vb.pitch_y + x] * inv;
        const float cv = c[vc.offset + z * vc.pitch_z + y * vc.pitch_y + x];
        const float vc_ = c_times_a ? cv * va_ : cv;
        uint4 o;
        o.x = f2bf(va_) | ((uint32_t)f2bf(vb_) << 16);
        o.y = f2bf(vc_);
        o.z = 0u;
        o.w = 0u;
        reinterpret_cast<uint4 *>(x8)[i] = o;
    }
}

constexpr int kRmsBlocks = 1024;
static_assert(kRmsBlocks % 256 == 0, "k_rms_final splits the partials over 256 threads");

// stage 1: per-block sums of squares (double) and non-finite flags
// The fixed tree red[t] += red[t + w], w = 128 .. 1, over a 256-thread
// block's values: the same additions in the same order, the first two levels
// through LDS and the last six inside wave 0 by lane shuffles (no barriers).
// The sum is valid in thread 0.
__device__ __forceinline__ double tree_sum256(const double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < 128) red[threadIdx.x] += red[threadIdx.x + 128];
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < 64) {
        r = red[threadIdx.x] + red[threadIdx.x + 64];
#pragma unroll
        for (int w = 32; w > 0; w >>= 1) r += __shfl_down(r, w, 64);
    }
    return r;
}

__global__ __launch_bounds__(256) void k_rms_part(const int nz, const int ny, const int nx,
                                                  const float *u, const nn_view vu, double *part,
                                                  unsigned *flag, const int seg)
{
    __shared__ double red[256];
    double s = 0.0;
    bool bad = false;
    // x rows dealt to blocks in a fixed order; FP32 partial sums per row
    // segment, accumulated in FP64 per thread
    const int rpi = blockDim.x / seg, sub = threadIdx.x / seg, xl = threadIdx.x % seg;
    for (int row = blockIdx.x * rpi + sub; row < nz * ny; row += gridDim.x * rpi) {
        const int y = row % ny, z = row / ny;
        const float *r = u + vu.offset + z * vu.pitch_z + y * vu.pitch_y;
        float rs = 0.0f;
        for (int x = xl; x < nx; x += seg) {
            const float v = r[x];
            if (!isfinite(v)) bad = true;
            rs = fmaf(v, v, rs);
        }
        s += (double)rs;
    }
    const double t = tree_sum256(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    if (bad && flag) flag[0] = 1u;
}

// stage 2: ordered sum of the block sums -> sqrt(mean) (deterministic)
__global__ __launch_bounds__(256) void k_rms_final(const double *part, const int64_t n,
                                                   float *scale)
{
    // each thread sums kRmsBlocks / 256 consecutive partials, then a fixed
    // tree: the same order on every call
    __shared__ double red[256];
    double s = 0.0;
    constexpr int per = kRmsBlocks / 256;
#pragma unroll
    for (int b = 0; b < per; ++b) s += part[threadIdx.x * per + b];
    const double t = tree_sum256(s, red);
    if (threadIdx.x == 0) scale[0] = (float)sqrt(t / (double)n) + 1e-30f;
}

__global__ __launch_bounds__(256) void k_mse(const int nz, const int ny, const int nx,
                                             const float *__restrict__ y,
                                             const float *__restrict__ t,
                                             const float *__restrict__ scale, const float gain,
                                             const nn_box skip, uint16_t *gy8, float *loss,
                                             const int seg)
{
    __shared__ float red[256];
    float s = 0.0f;
    const int64_t n = (int64_t)nz * ny * nx;
    const float inv = 1.0f / (float)n;
    const float ts = 1.0f / (gain * (scale ? scale[0] : 1.0f));
    const int rpi = blockDim.x / seg, sub = threadIdx.x / seg, xl = threadIdx.x % seg;
    for (int row = blockIdx.x * rpi + sub; row < nz * ny; row += gridDim.x * rpi)
    for (int x = xl; x < nx; x += seg) {
        const int yy = row % ny, z = row / ny;
        const int64_t i = (int64_t)row * nx + x;
        const float d = in_box(skip, z, yy, x) ? 0.0f : y[i] - t[i] * ts;
        s += d * d;
        uint4 o = make_uint4(f2bf(2.0f * d * inv), 0u, 0u, 0u);
        reinterpret_cast<uint4 *>(gy8)[i] = o;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv);
}

__global__ __launch_bounds__(256) void k_adam(float *p, const float *__restrict__ g, float *m,
                                              float *v, const float c1, const float c2,
                                              const float lr, const float b1, const float b2,
                                              const float eps, const int train_bias)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNP) return;
    const bool bias = (i >= kB1 && i < kB1 + 16) || (i >= kB2 && i < kB2 + 16) || i == kB3;
    if (bias && !train_bias) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Scratch of nn_wgrad_noalloc: the per-block partial sums of the weight
// gradient, room for every persistent block (WG_BLOCKS x WG_PART floats,
// 14.2 MB).  One copy per GPU, in the code object's static device data, held
// until the process ends.  Host code never passes this name to a kernel: it
// is a host-side stand-in, the device address comes from
// hipGetSymbolAddress (wgrad_scratch below).
constexpr int64_t kWgScratchFloats = (int64_t)WG_BLOCKS * WG_PART;
static __device__ __align__(256) float scratch[kWgScratchFloats];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int wgrad_scratch(float **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(FD_EDEVICE, "nn_wgrad_noalloc: no usable current device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(FD_EDEVICE, std::string("nn_wgrad_noalloc: hipGetSymbolAddress "
                                                     "failed: ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return FD_OK;
}

}  // namespace nn
}  // namespace fd

using namespace fd;
using namespace fd::nn;

// Weight gradient of one layer: per-block partial sums in `part` (room for
// min(WG_BLOCKS, tiles) partials), then the ordered reduction.
static int wgrad_run(int layer, int nz, int ny, int nx, const void *x_dev, const void *g_dev,
                     float *part, float *grads_dev, int accumulate, hipStream_t s)
{
    const uint16_t *x = (const uint16_t *)x_dev, *g = (const uint16_t *)g_dev;
    const int ntiles = ((nx + TXW - 1) / TXW) * ((ny + TYW - 1) / TYW) * ((nz + TZW - 1) / TZW);
    const int nbk = std::min(WG_BLOCKS, ntiles);
    int cin_real, cout_real, woff, boff;
    if (layer == 1) {
        hipLaunchKernelGGL((k_wgrad<8, 16>), dim3(nbk), dim3(256), 0, s, nz, ny, nx, x, g, part);
        cin_real = 3; cout_real = 16; woff = kW1; boff = kB1;
    } else if (layer == 2) {
        hipLaunchKernelGGL((k_wgrad<16, 16>), dim3(nbk), dim3(256), 0, s, nz, ny, nx, x, g, part);
        cin_real = 16; cout_real = 16; woff = kW2; boff = kB2;
    } else {
        hipLaunchKernelGGL((k_wgrad<16, 8>), dim3(nbk), dim3(256), 0, s, nz, ny, nx, x, g, part);
        cin_real = 16; cout_real = 1; woff = kW3; boff = kB3;
    }
    int rc = check_launch("nn wgrad");
    if (rc) return rc;
    const int nout = cout_real * cin_real * 27 + cout_real;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 255) / 256), dim3(256), 0, s, part, nbk,
                       cin_real, cout_real, grads_dev + woff, grads_dev + boff, accumulate);
    return check_launch("nn wgrad reduce");
}

extern "C" {

int64_t nn_param_count(void) { return kNP; }
int64_t nn_packed_bytes(void) { return (int64_t)kSteps * 64 * 8 * 2; }

int64_t nn_wgrad_workspace_bytes(int nz, int ny, int nx)
{
    (void)nz;
    (void)ny;
    (void)nx;
    return (int64_t)WG_BLOCKS * WG_PART * (int64_t)sizeof(float);
}

int nn_pack_weights(const float *params_dev, void *packed_dev, void *stream)
{
    if (!params_dev || !packed_dev) return set_error(FD_EINVAL, "nn_pack_weights: null pointer");
    hipLaunchKernelGGL(k_pack_weights, dim3((kSteps * 512 + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, params_dev, (uint16_t *)packed_dev);
    return check_launch("nn pack weights");
}

static bool bad_shape(int nz, int ny, int nx) { return nz < 1 || ny < 1 || nx < 1; }

// threads per x row for the row-wise elementwise kernels (a power of two
// dividing 256, at least min(nx, 256))
static int row_seg(int nx)
{
    int s = 32;
    while (s < 256 && s < nx) s *= 2;
    return s;
}

static int row_blocks(int nz, int ny, int nx, int cap)
{
    const int64_t rows = (int64_t)nz * ny, rpi = 256 / row_seg(nx);
    return (int)std::min<int64_t>((rows + rpi - 1) / rpi, cap);
}

int nn_pack_input(int nz, int ny, int nx, const float *a, nn_view va, const float *b, nn_view vb,
                  const float *c, nn_view vc, int c_times_a, const float *scale_dev, void *x8_dev,
                  void *stream)
{
    if (bad_shape(nz, ny, nx) || !a || !b || !c || !x8_dev)
        return set_error(FD_EINVAL, "nn_pack_input: bad argument");
    hipLaunchKernelGGL(k_pack_input, dim3(row_blocks(nz, ny, nx, 8192)), dim3(256), 0,
                       (hipStream_t)stream, nz, ny, nx, a, va, b, vb, c, vc, c_times_a, scale_dev,
                       (uint16_t *)x8_dev, row_seg(nx));
    return check_launch("nn pack input");
}

int nn_rms(int nz, int ny, int nx, const float *u, nn_view vu, float *scale_dev,
           unsigned *flag_dev, void *stream)
{
    if (bad_shape(nz, ny, nx) || !u || !scale_dev) return set_error(FD_EINVAL, "nn_rms: bad argument");
    // scale_dev[0] is the result; the double-aligned block sums live from
    // scale_dev + 2 on (see fdnn.h: nn_rms_scratch_floats)
    double *part = reinterpret_cast<double *>(scale_dev + 2);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_rms_part, dim3(kRmsBlocks), dim3(256), 0, s, nz, ny, nx, u, vu, part,
                       flag_dev, row_seg(nx));
    hipLaunchKernelGGL(k_rms_final, dim3(1), dim3(256), 0, s, part, (int64_t)nz * ny * nx,
                       scale_dev);
    return check_launch("nn rms");
}

int64_t nn_rms_scratch_floats(void) { return 2 + 2 * kRmsBlocks; }

int nn_conv_gelu(int layer, int nz, int ny, int nx, const void *x_dev, const void *packed_dev,
                 const float *params_dev, void *z16_dev, void *a16_dev, void *stream)
{
    if (bad_shape(nz, ny, nx) || !x_dev || !packed_dev || !params_dev || !a16_dev ||
        (layer != 1 && layer != 2))
        return set_error(FD_EINVAL, "nn_conv_gelu: bad argument");
    ConvArgs a{};
    a.nz = nz;
    a.ny = ny;
    a.nx = nx;
    a.in = (const uint16_t *)x_dev;
    a.a16 = (uint16_t *)a16_dev;
    a.z16 = (uint16_t *)z16_dev;
    const uint16_t *pk = (const uint16_t *)packed_dev;
    hipStream_t s = (hipStream_t)stream;
    if (layer == 1) {
        a.frag = pk + kF1 * 512;
        a.bias = params_dev + kB1;
        return z16_dev ? conv<8, 7, EPI_GELU_Z>(a, s) : conv<8, 7, EPI_GELU>(a, s);
    }
    a.frag = pk + kF2 * 512;
    a.bias = params_dev + kB2;
    return z16_dev ? conv<16, 14, EPI_GELU_Z>(a, s) : conv<16, 14, EPI_GELU>(a, s);
}

int nn_conv_gelu_fields(int nz, int ny, int nx, const float *a, nn_view va, const float *b,
                        nn_view vb, const float *c, nn_view vc, int c_times_a,
                        const float *scale_dev, const void *packed_dev, const float *params_dev,
                        void *z16_dev, void *a16_dev, void *stream)
{
    if (bad_shape(nz, ny, nx) || !a || !b || !c || !packed_dev || !params_dev || !a16_dev)
        return set_error(FD_EINVAL, "nn_conv_gelu_fields: bad argument");
    // each field's plane is read with 32-bit byte offsets
    for (const nn_view *v : {&va, &vb, &vc})
        if (v->pitch_y < nx || v->pitch_z < (int64_t)ny * v->pitch_y || v->pitch_z * 4 > 0x7fffffff)
            return set_error(FD_EINVAL, "nn_conv_gelu_fields: a field view's plane does not hold "
                                        "ny rows of nx points, or exceeds 2^31 bytes");
    ConvArgs g{};
    g.nz = nz;
    g.ny = ny;
    g.nx = nx;
    g.fa = a;
    g.fb = b;
    g.fc = c;
    g.fva = va;
    g.fvb = vb;
    g.fvc = vc;
    g.fct = c_times_a ? 1 : 0;
    g.fscale = scale_dev;
    g.a16 = (uint16_t *)a16_dev;
    g.z16 = (uint16_t *)z16_dev;
    g.frag = (const uint16_t *)packed_dev + kF1 * 512;
    g.bias = params_dev + kB1;
    hipStream_t s = (hipStream_t)stream;
    return z16_dev ? conv<8, 7, EPI_GELU_Z, true>(g, s) : conv<8, 7, EPI_GELU, true>(g, s);
}

int nn_conv_out(int nz, int ny, int nx, const void *a16_dev, const void *packed_dev,
                const float *params_dev, float *y_dense_dev, const float *base_dev, nn_view vbase,
                float *out_dev, nn_view vout, const float *scale_dev, float gain,
                const nn_box *skip, void *stream)
{
    if (bad_shape(nz, ny, nx) || !a16_dev || !packed_dev || !params_dev ||
        (out_dev && !base_dev) || (!out_dev && !y_dense_dev) || !std::isfinite(gain))
        return set_error(FD_EINVAL, "nn_conv_out: bad argument");
    ConvArgs a{};
    a.nz = nz;
    a.ny = ny;
    a.nx = nx;
    a.in = (const uint16_t *)a16_dev;
    a.frag = (const uint16_t *)packed_dev + kF3 * 512;
    a.bias = params_dev + kB3;
    a.ydense = y_dense_dev;
    a.base = base_dev;
    a.vbase = vbase;
    a.out = out_dev;
    a.vout = vout;
    a.scale = scale_dev;
    a.gain = gain;
    a.skip = skip ? *skip : nn_box{{0, 0, 0}, {0, 0, 0}};
    return conv_out_mfma(a, (hipStream_t)stream);
}

int nn_mse(int nz, int ny, int nx, const float *y_dev, const float *t_dev,
           const float *scale_dev, float gain, const nn_box *skip, void *gy8_dev,
           float *loss_dev, void *stream)
{
    if (bad_shape(nz, ny, nx) || !y_dev || !t_dev || !gy8_dev || !loss_dev || !(gain > 0.0f) ||
        !std::isfinite(gain))
        return set_error(FD_EINVAL, "nn_mse: bad argument");
    const nn_box sk = skip ? *skip : nn_box{{0, 0, 0}, {0, 0, 0}};
    hipLaunchKernelGGL(k_mse, dim3(row_blocks(nz, ny, nx, 2048)), dim3(256), 0,
                       (hipStream_t)stream, nz, ny, nx, y_dev, t_dev, scale_dev, gain, sk,
                       (uint16_t *)gy8_dev, loss_dev, row_seg(nx));
    return check_launch("nn mse");
}

int nn_dgrad_gelu(int layer, int nz, int ny, int nx, const void *gin_dev, const void *packed_dev,
                  const void *z16_prev_dev, void *gz_out16_dev, void *stream)
{
    if (bad_shape(nz, ny, nx) || !gin_dev || !packed_dev || !z16_prev_dev || !gz_out16_dev ||
        (layer != 2 && layer != 3))
        return set_error(FD_EINVAL, "nn_dgrad_gelu: bad argument");
    ConvArgs a{};
    a.nz = nz;
    a.ny = ny;
    a.nx = nx;
    a.in = (const uint16_t *)gin_dev;
    a.z16 = (uint16_t *)z16_prev_dev;
    a.a16 = (uint16_t *)gz_out16_dev;
    const uint16_t *pk = (const uint16_t *)packed_dev;
    hipStream_t s = (hipStream_t)stream;
    if (layer == 3) {
        a.frag = pk + kD3 * 512;
        return conv<8, 7, EPI_DGRAD>(a, s);
    }
    a.frag = pk + kD2 * 512;
    return conv<16, 14, EPI_DGRAD>(a, s);
}

int nn_wgrad(int layer, int nz, int ny, int nx, const void *x_dev, const void *g_dev,
             void *workspace_dev, float *grads_dev, int accumulate, void *stream)
{
    if (bad_shape(nz, ny, nx) || !x_dev || !g_dev || !workspace_dev || !grads_dev ||
        layer < 1 || layer > 3)
        return set_error(FD_EINVAL, "nn_wgrad: bad argument");
    return wgrad_run(layer, nz, ny, nx, x_dev, g_dev, (float *)workspace_dev, grads_dev,
                     accumulate, (hipStream_t)stream);
}

int nn_wgrad_noalloc(int layer, int nz, int ny, int nx, const void *x_dev, const void *g_dev,
                     float *grads_dev, int accumulate, void *stream)
{
    if (bad_shape(nz, ny, nx) || !x_dev || !g_dev || !grads_dev || layer < 1 || layer > 3)
        return set_error(FD_EINVAL, "nn_wgrad_noalloc: bad argument");
    // tiles of the volume (the persistent launch takes min(WG_BLOCKS, tiles)
    // blocks, one partial sum each)
    const int64_t ntiles = (int64_t)((nx + TXW - 1) / TXW) * ((ny + TYW - 1) / TYW) *
                           ((nz + TZW - 1) / TZW);
    if (ntiles > INT32_MAX)
        return set_error(FD_EINVAL, "nn_wgrad_noalloc: volume has more tiles than a launch indexes");
    const int64_t need = std::min<int64_t>(WG_BLOCKS, ntiles) * WG_PART;
    if (need > kWgScratchFloats)
        return set_error(FD_EINVAL, "nn_wgrad_noalloc: " + std::to_string(need) +
                                        " partial-sum floats exceed the static scratch of " +
                                        std::to_string(kWgScratchFloats));
    float *part = nullptr;
    const int rc = wgrad_scratch(&part);
    if (rc) return rc;
    return wgrad_run(layer, nz, ny, nx, x_dev, g_dev, part, grads_dev, accumulate,
                     (hipStream_t)stream);
}

int nn_adam(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int t, float lr,
            float beta1, float beta2, float eps, int train_bias, void *stream)
{
    if (!params_dev || !grads_dev || !m_dev || !v_dev || t < 1)
        return set_error(FD_EINVAL, "nn_adam: bad argument");
    const float c1 = 1.0f - (float)std::pow((double)beta1, t);
    const float c2 = 1.0f - (float)std::pow((double)beta2, t);
    hipLaunchKernelGGL(k_adam, dim3((kNP + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params_dev, grads_dev, m_dev, v_dev, c1, c2, lr, beta1, beta2, eps,
                       train_bias);
    return check_launch("nn adam");
}

}  // extern "C"
