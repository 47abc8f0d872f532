// smc_device.hpp -- device building blocks of the SMC sweep for gfx950:
// Philox4x32-10 counter-based draws and their transforms, and deterministic
// (fixed-order) wavefront/workgroup reductions and scans.
//
// Tiling used by every per-particle kernel: a workgroup of TPB = 256 lanes
// (four wave64s) owns a tile of TILE = 1024 consecutive particles; lane t
// handles particles tile_base + k*256 + t for k = 0..3, so every load and
// store of a structure-of-arrays row is a fully coalesced 256-lane access.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "smc_math.hpp"

namespace smc {

constexpr int WAVE = 64;
constexpr int TPB = 256;
constexpr int ITEMS = 4;
constexpr int TILE = TPB * ITEMS;
constexpr int NWAVES = TPB / WAVE;

// Counter tags: counter = (particle, step, tag << 16 | call, problem).
enum : uint32_t {
    TAG_INIT = 1,
    TAG_PF_MOVE = 2,
    TAG_MH_MU = 3,
    TAG_MH_ETA = 4,
    TAG_MH_Z = 5,
    TAG_MH_ACCEPT = 6,
    TAG_RESAMPLE = 7
};

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr float kTwoPiF = 6.28318530717958647692f;

struct Key {
    uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed)
{
    return Key{(uint32_t)seed, (uint32_t)(seed >> 32)};
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies, the Weyl key schedule between rounds.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        Key key)
{
    // The key is wave-uniform (read from the first lane, which also holds
    // where the compiler cannot prove it, e.g. in a function that is not
    // inlined): advancing it round by round costs two scalar adds per round.
    // The empty asm keeps the compiler from precomputing the twenty round
    // keys once per kernel and holding them live across every call (which
    // exhausts the scalar registers of the larger kernels).
    uint32_t k0 = __builtin_amdgcn_readfirstlane(key.k0);
    uint32_t k1 = __builtin_amdgcn_readfirstlane(key.k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply per product (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input XOR in one instruction (gfx950 bitop3, truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 draw(Key key, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                                      uint32_t p)
{
    return philox(i, t, (tag << 16) | (j & 0xFFFFu), p, key);
}

// Uniform on (0,1]: (top 53 bits of (a:b) + 1) * 2^-53, assembled exactly.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    return fma((double)a, 0x1p-32, (double)((b >> 11) + 1u) * 0x1p-53);
}

// Uniform on (0,1] in single precision: ((w >> 8) + 1) * 2^-24.
__device__ __forceinline__ float u24(uint32_t w)
{
    return (float)((w >> 8) + 1u) * 0x1p-24f;
}

// Box-Muller: two standard normals from the four words of one call,
// r = sqrt(-2 log u1), angle 2 pi u2 (sin/cos of pi * (2 u2), exact argument).
__device__ __forceinline__ double2 normal2(uint4 w)
{
    const double u1 = u53(w.x, w.y);
    const double u2 = u53(w.z, w.w);
    const double r = sqrt_nonneg_d(-2.0 * log_pos_d(u1));
    double s, c;
    sincospi_d<true>(u2 + u2, &s, &c);  // argument in (0, 2]
    return make_double2(r * c, r * s);
}

// Single-precision Box-Muller: four normals from one call.
__device__ __forceinline__ float4 normal4f(uint4 w)
{
    float s0, c0, s1, c1;
    const float r0 = sqrtf(-2.0f * logf(u24(w.x)));
    const float a0 = u24(w.y);
    sincospif(a0 + a0, &s0, &c0);
    const float r1 = sqrtf(-2.0f * logf(u24(w.z)));
    const float a1 = u24(w.w);
    sincospif(a1 + a1, &s1, &c1);
    return make_float4(r0 * c0, r0 * s0, r1 * c1, r1 * s1);
}

// Gamma(shape, 1) from calls jbase, jbase+1, ...: exponential for shape 1,
// Marsaglia-Tsang with attempt k on calls jbase+1+2k (normal) and jbase+2+2k
// (uniform), boosted by u^(1/shape) (call jbase) for shape < 1.  *fail is set
// after 31 rejected attempts.
__device__ inline double gamma_draw(Key key, uint32_t i, uint32_t t, uint32_t tag,
                                    uint32_t jbase, uint32_t p, double shape, int *fail)
{
    if (shape == 1.0) {
        const uint4 w = draw(key, i, t, tag, jbase, p);
        return -log(u53(w.x, w.y));
    }
    const double a = shape < 1.0 ? shape + 1.0 : shape;
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double g = __builtin_nan("");
    for (int k = 0; k < 31; ++k) {
        const double z = normal2(draw(key, i, t, tag, jbase + 1 + 2 * k, p)).x;
        double v = 1.0 + c * z;
        if (v <= 0.0)
            continue;
        v = v * v * v;
        const uint4 w = draw(key, i, t, tag, jbase + 2 + 2 * k, p);
        const double u = u53(w.x, w.y);
        if (log(u) < 0.5 * z * z + d - d * v + d * log(v)) {
            g = d * v;
            break;
        }
    }
    if (g != g) {
        *fail = 1;
        return g;
    }
    if (shape < 1.0) {
        const uint4 w = draw(key, i, t, tag, jbase, p);
        g *= pow(u53(w.x, w.y), 1.0 / shape);
    }
    return g;
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Within a wave, DPP row shifts and row
// broadcasts (below) build the inclusive scan or the reduction in a fixed
// order, and the result is read back from the last lane; workgroup results
// combine the per-wave values in wave order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / WAVE; }

// Cross-lane moves through DPP (the VALU's data-parallel operand modes): a
// neighbour's value in a few cycles instead of a round trip through the LDS
// crossbar.  Lanes without a source (or in rows the row mask leaves out)
// receive `fill`.
namespace dpp {
enum : int {
    ROW_SHR1 = 0x111,
    ROW_SHR2 = 0x112,
    ROW_SHR4 = 0x114,
    ROW_SHR8 = 0x118,
    WAVE_SHR1 = 0x138,
    ROW_BCAST15 = 0x142,
    ROW_BCAST31 = 0x143
};

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int mov_i(int v, int fill)
{
    return __builtin_amdgcn_update_dpp(fill, v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double mov(double v, double fill)
{
    const long long b = __double_as_longlong(v), f = __double_as_longlong(fill);
    const int lo = mov_i<CTRL, ROW_MASK>((int)b, (int)f);
    const int hi = mov_i<CTRL, ROW_MASK>((int)(b >> 32), (int)(f >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double readlane(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Inclusive scan of op over the 64 lanes: shifts 1, 2, 4, 8 inside each row
// of 16 lanes, then the row totals carried across rows by the two
// broadcasts.  `id` is op's identity.
template <typename Op>
__device__ __forceinline__ double incl_scan(double v, double id, Op op)
{
    v = op(v, mov<ROW_SHR1>(v, id));
    v = op(v, mov<ROW_SHR2>(v, id));
    v = op(v, mov<ROW_SHR4>(v, id));
    v = op(v, mov<ROW_SHR8>(v, id));
    v = op(v, mov<ROW_BCAST15, 0xA>(v, id));
    v = op(v, mov<ROW_BCAST31, 0xC>(v, id));
    return v;
}

template <typename Op>
__device__ __forceinline__ int incl_scan_i(int v, int id, Op op)
{
    v = op(v, mov_i<ROW_SHR1>(v, id));
    v = op(v, mov_i<ROW_SHR2>(v, id));
    v = op(v, mov_i<ROW_SHR4>(v, id));
    v = op(v, mov_i<ROW_SHR8>(v, id));
    v = op(v, mov_i<ROW_BCAST15, 0xA>(v, id));
    v = op(v, mov_i<ROW_BCAST31, 0xC>(v, id));
    return v;
}
}  // namespace dpp

struct OpAdd {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMax {
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct OpMin {
    __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMaxI {
    __device__ int operator()(int a, int b) const { return a > b ? a : b; }
};

// Wave reductions (every lane receives the result: the last lane of the
// inclusive scan, read back as a wave-uniform value).
__device__ __forceinline__ double wave_sum(double v)
{
    return dpp::readlane(dpp::incl_scan(v, 0.0, OpAdd{}), WAVE - 1);
}

__device__ __forceinline__ double wave_max(double v)
{
    return dpp::readlane(dpp::incl_scan(v, -INFINITY, OpMax{}), WAVE - 1);
}

__device__ __forceinline__ double wave_min(double v)
{
    return dpp::readlane(dpp::incl_scan(v, INFINITY, OpMin{}), WAVE - 1);
}

__device__ __forceinline__ int wave_max_i(int v)
{
    return __builtin_amdgcn_readlane(dpp::incl_scan_i(v, INT_MIN, OpMaxI{}), WAVE - 1);
}

// Value of the previous lane (lane 0 receives `fill`).
__device__ __forceinline__ double lane_prev(double v, double fill)
{
    return dpp::mov<dpp::WAVE_SHR1>(v, fill);
}

// Block reductions over NW waves; `red` is __shared__ scratch of >= NW
// doubles.  All threads receive the result.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0)
        red[wave_id()] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
        s += red[w];
    return s;
}

template <int NW>
__device__ __forceinline__ double block_max(double v, double *red)
{
    v = wave_max(v);
    __syncthreads();
    if (lane_id() == 0)
        red[wave_id()] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
        s = fmax(s, red[w]);
    return s;
}

// Workgroup sums of R values at once: R independent wave reductions, then
// one barrier pair; `red` holds NW * R doubles.  Every lane receives the sums.
template <int NW, int R>
__device__ __forceinline__ void block_sum_n(double (&v)[R], double *red)
{
#pragma unroll
    for (int r = 0; r < R; ++r)
        v[r] = wave_sum(v[r]);
    __syncthreads();
    if (lane_id() == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            red[wave_id() * R + r] = v[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double a = red[r];
        for (int w = 1; w < NW; ++w)
            a += red[w * R + r];
        v[r] = a;
    }
}

// Inclusive prefix sum across one wave.
__device__ __forceinline__ double wave_incl_scan(double v)
{
    return dpp::incl_scan(v, 0.0, OpAdd{});
}

// Inclusive prefix sum across the workgroup; *total receives the sum.
template <int NW>
__device__ __forceinline__ double block_incl_scan(double v, double *red, double *total)
{
    v = wave_incl_scan(v);
    __syncthreads();
    if (lane_id() == WAVE - 1)
        red[wave_id()] = v;
    __syncthreads();
    double before = 0.0, all = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wave_id())
            before += red[w];
        all += red[w];
    }
    *total = all;
    return before + v;
}

// Exclusive prefix sum across the workgroup, defined as the inclusive value
// of the previous lane so that consecutive lanes agree exactly; *total
// receives the sum (sequential over the wave totals).
template <int NW>
__device__ __forceinline__ double block_excl_scan(double v, double *red, double *total)
{
    const double incl = wave_incl_scan(v);
    const double excl = lane_prev(incl, 0.0);
    __syncthreads();
    if (lane_id() == WAVE - 1)
        red[wave_id()] = incl;
    __syncthreads();
    double before = 0.0, all = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wave_id())
            before += red[w];
        all += red[w];
    }
    *total = all;
    return lane_id() == 0 ? before : before + excl;
}

// Inclusive prefix max across the workgroup (exact, order-free).
template <int NW>
__device__ __forceinline__ double block_incl_max_scan(double v, double *red)
{
    v = dpp::incl_scan(v, -INFINITY, OpMax{});
    __syncthreads();
    if (lane_id() == WAVE - 1)
        red[wave_id()] = v;
    __syncthreads();
    for (int w = 0; w < wave_id(); ++w)
        v = fmax(v, red[w]);
    return v;
}

// Per-tile weight summary written by every kernel that changes log-weights:
// m = max lw over the tile, s1 = sum exp(lw - m), s2 = sum exp(2 (lw - m)).
struct TilePartial {
    double m, s1, s2, pad;
};

// Reduces the ITEMS log-weights held by each lane of a TPB workgroup to a
// TilePartial (written by lane 0).  Out-of-range items must be -inf.
__device__ __forceinline__ void tile_partial(const double (&lw)[ITEMS], TilePartial *out,
                                             double *red)
{
    double m = lw[0];
#pragma unroll
    for (int k = 1; k < ITEMS; ++k)
        m = fmax(m, lw[k]);
    m = block_max<NWAVES>(m, red);
    double s1 = 0.0, s2 = 0.0;
    if (m > -INFINITY) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const double e = exp_nonpos_d(lw[k] - m);
            s1 += e;
            s2 += e * e;
        }
    }
    __shared__ double red2[2 * NWAVES];
    double v[2] = {s1, s2};
    block_sum_n<NWAVES, 2>(v, red2);
    if (threadIdx.x == 0) {
        out->m = m;
        out->s1 = v[0];
        out->s2 = v[1];
        out->pad = 0.0;
    }
}

}  // namespace smc
