// smc_pf.hip -- the almost-constant-velocity tracking filter of Section 5.1
// (Algorithm "pf") on gfx950: prior draws, the fused transition +
// incremental log-weight sweep, and the unfused reweight.
//
// State rows (x_pos, y_pos, x_vel, y_vel), structure of arrays, double or
// float.  Per particle-step the fused sweep moves 4 state elements in and
// out and the log-weight in and out: 80 B (double state) or 48 B (float
// state), plus 4 B of ancestor index after a resample.
//
// Every kernel body is a per-tile device function of a problem descriptor,
// launched either for one problem (blockIdx = tile) or for a batch of
// problems (blockIdx -> (problem, tile) through a map).
#include <math.h>

#include "smc_tiles.hpp"

namespace smc {

// Prior draws of one tile: x_0 ~ N(0, diag(init_sd^2)) and the weight of the
// first observation; tile partial of the log-weights.
template <typename T>
__device__ __forceinline__ void pf_init_tile(const Prob &P, T *__restrict__ x, int64_t tile)
{
    __shared__ double red[NWAVES];
    const int64_t n = P.n;
    double *__restrict__ lw = P.lw;
    const int64_t base = tile * TILE;
    const double yx = P.data[0], yy = P.data[1];
    const Key key = P.key;
    const uint32_t p = P.problem_id;
    double lwv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        lwv[k] = -INFINITY;
        if (i >= n)
            continue;
        T s0, s1, s2, s3;
        if constexpr (sizeof(T) == 8) {
            const double2 a = normal2(draw(key, (uint32_t)i, 0, TAG_INIT, 0, p));
            const double2 b = normal2(draw(key, (uint32_t)i, 0, TAG_INIT, 1, p));
            s0 = P.init_sd[0] * a.x;
            s1 = P.init_sd[1] * a.y;
            s2 = P.init_sd[2] * b.x;
            s3 = P.init_sd[3] * b.y;
        } else {
            const float4 z = normal4f(draw(key, (uint32_t)i, 0, TAG_INIT, 0, p));
            s0 = (float)P.init_sd[0] * z.x;
            s1 = (float)P.init_sd[1] * z.y;
            s2 = (float)P.init_sd[2] * z.z;
            s3 = (float)P.init_sd[3] * z.w;
        }
        x[i] = s0;
        x[n + i] = s1;
        x[2 * n + i] = s2;
        x[3 * n + i] = s3;
        const double l = P.obs((double)s0, yx, (double)s1, yy);
        lw[i] = l;
        lwv[k] = l;
    }
    tile_partial(lwv, P.partials + tile, red);
}

template <typename T>
__global__ __launch_bounds__(TPB) void pf_init_kernel(Prob P)
{
    pf_init_tile<T>(P, (T *)P.state[0], blockIdx.x);
}

hipError_t launch_pf_init(Ctx &c)
{
    const Prob P = make_prob(c);
    const dim3 grid((unsigned)c.ntiles);
    if (c.elem_bytes == 4)
        hipLaunchKernelGGL(pf_init_kernel<float>, grid, dim3(TPB), 0, c.stream, P);
    else
        hipLaunchKernelGGL(pf_init_kernel<double>, grid, dim3(TPB), 0, c.stream, P);
    return hipGetLastError();
}

template <typename T, bool FUSE, bool MON>
__global__ __launch_bounds__(TPB) void pf_move_kernel(Prob P, uint32_t t, int32_t obs_index,
                                                      int gather_check, int reset_check)
{
    pf_move_tile<T, FUSE, MON>(P, (const T *)P.state[0], (T *)P.state[1], blockIdx.x, t,
                               P.data + 2 * (int64_t)obs_index, gather_check != 0,
                               reset_check != 0);
}

template <typename T, bool FUSE, bool MON>
static void launch_move_t(Ctx &c, int32_t step, int32_t obs_index, bool gather_check,
                          bool reset_check)
{
    const Prob P = make_prob(c);
    hipEvent_t e0, e1;
    if (c.prof_take(&e0, &e1))
        hipExtLaunchKernelGGL((pf_move_kernel<T, FUSE, MON>), dim3((unsigned)c.ntiles), dim3(TPB),
                              0, c.stream, e0, e1, 0, P, (uint32_t)step, obs_index,
                              (int)gather_check, (int)reset_check);
    else
        hipLaunchKernelGGL((pf_move_kernel<T, FUSE, MON>), dim3((unsigned)c.ntiles), dim3(TPB),
                           0, c.stream, P, (uint32_t)step, obs_index, (int)gather_check,
                           (int)reset_check);
}

hipError_t launch_pf_move(Ctx &c, int32_t step, int32_t obs_index, bool fuse, bool gather_check,
                          bool reset_check, bool monitor)
{
    // the monitor needs the incoming weights, so it rides only on the fused sweep
    if (c.elem_bytes == 4) {
        if (fuse && monitor)
            launch_move_t<float, true, true>(c, step, obs_index, gather_check, reset_check);
        else if (fuse)
            launch_move_t<float, true, false>(c, step, obs_index, gather_check, reset_check);
        else
            launch_move_t<float, false, false>(c, step, obs_index, gather_check, false);
    } else {
        if (fuse && monitor)
            launch_move_t<double, true, true>(c, step, obs_index, gather_check, reset_check);
        else if (fuse)
            launch_move_t<double, true, false>(c, step, obs_index, gather_check, reset_check);
        else
            launch_move_t<double, false, false>(c, step, obs_index, gather_check, false);
    }
    c.cur ^= 1;
    return hipGetLastError();
}

// Unfused weighting at the current state (Eq. si with the observation
// density as the incremental weight).
template <typename T>
__global__ __launch_bounds__(TPB) void pf_reweight_kernel(Prob P, int reset_check,
                                                          int32_t obs_index)
{
    __shared__ double red[NWAVES];
    const T *__restrict__ x = (const T *)P.state[0];
    const int64_t n = P.n;
    double *__restrict__ lw = P.lw;
    const bool reset = reset_check && P.scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const double *y = P.data + 2 * (int64_t)obs_index;
    const double yx = y[0], yy = y[1];
    double lwv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        lwv[k] = -INFINITY;
        if (i >= n)
            continue;
        const double inc = P.obs((double)x[i], yx, (double)x[n + i], yy);
        const double l = (reset ? 0.0 : lw[i]) + inc;
        lw[i] = l;
        lwv[k] = l;
    }
    tile_partial(lwv, P.partials + blockIdx.x, red);
}

hipError_t launch_pf_reweight(Ctx &c, int32_t obs_index, bool reset_check)
{
    const Prob P = make_prob(c);
    const dim3 grid((unsigned)c.ntiles);
    if (c.elem_bytes == 4)
        hipLaunchKernelGGL(pf_reweight_kernel<float>, grid, dim3(TPB), 0, c.stream, P,
                           (int)reset_check, obs_index);
    else
        hipLaunchKernelGGL(pf_reweight_kernel<double>, grid, dim3(TPB), 0, c.stream, P,
                           (int)reset_check, obs_index);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched initialisation: blockIdx -> (problem, tile) through `map` (the
// steps of the batched form run in the persistent step kernel).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void pf_init_batch_kernel(const Prob *__restrict__ probs,
                                                            const int2 *__restrict__ map)
{
    const int2 pm = map[blockIdx.x];
    const Prob &P = probs[pm.x];
    if (P.elem_bytes == 4)
        pf_init_tile<float>(P, (float *)P.state[0], pm.y);
    else
        pf_init_tile<double>(P, (double *)P.state[0], pm.y);
}

hipError_t launch_pf_init_batch(const Prob *probs, const int2 *map, int64_t tiles, hipStream_t s)
{
    if (tiles == 0)
        return hipSuccess;
    hipLaunchKernelGGL(pf_init_batch_kernel, dim3((unsigned)tiles), dim3(TPB), 0, s, probs, map);
    return hipGetLastError();
}

}  // namespace smc
