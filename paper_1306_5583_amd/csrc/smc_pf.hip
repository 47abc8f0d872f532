// smc_pf.hip -- the almost-constant-velocity tracking filter of Section 5.1
// (Algorithm "pf") on gfx950: prior draws, the fused transition +
// incremental log-weight sweep, and the unfused reweight.
//
// State rows (x_pos, y_pos, x_vel, y_vel), structure of arrays, double or
// float.  Per particle-step the fused sweep moves 4 state elements in and
// out and the log-weight in and out: 80 B (double state) or 48 B (float
// state), plus 4 B of ancestor index after a resample.
#include <math.h>

#include "smc_internal.hpp"

namespace smc {

// Observation log-density of one coordinate: Student-t with nu degrees of
// freedom and scale s,  c - (nu+1)/2 log1p(((y-pos)/s)^2 / nu), or Gaussian
// c - ((y-pos)/s)^2 / 2 when gaussian != 0.
// The two coordinates are independent, so their Student-t terms combine
// into one logarithm: log1p(a) + log1p(b) = log((1 + a)(1 + b)).
struct ObsModel {
    double c, half_nu1, inv_nu, inv_s;
    int gaussian;
    __device__ __forceinline__ double operator()(double px, double yx, double py, double yy) const
    {
        const double rx = (yx - px) * inv_s;
        const double ry = (yy - py) * inv_s;
        if (gaussian)
            return (c + c) - 0.5 * (rx * rx + ry * ry);
        const double q = fma(rx * rx, inv_nu, 1.0) * fma(ry * ry, inv_nu, 1.0);
        return (c + c) - half_nu1 * log_d(q);
    }
};

struct Motion {
    double dt, sd_pos, sd_vel;
};

static ObsModel make_obs(const Ctx &c)
{
    ObsModel o;
    o.c = c.obs_const;
    o.half_nu1 = c.obs_half_nu1;
    o.inv_nu = isinf(c.cfg.obs_nu) ? 0.0 : 1.0 / c.cfg.obs_nu;
    o.inv_s = c.obs_inv_scale;
    o.gaussian = isinf(c.cfg.obs_nu) ? 1 : 0;
    return o;
}

template <typename T>
__global__ __launch_bounds__(TPB) void pf_init_kernel(T *__restrict__ x, double *__restrict__ lw,
                                                      int64_t n, Key key, uint32_t p,
                                                      double4 init_sd,
                                                      const double *__restrict__ y0, ObsModel obs,
                                                      TilePartial *__restrict__ part)
{
    __shared__ double red[NWAVES];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const double yx = y0[0], yy = y0[1];
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
            s0 = init_sd.x * a.x;
            s1 = init_sd.y * a.y;
            s2 = init_sd.z * b.x;
            s3 = init_sd.w * b.y;
        } else {
            const float4 z = normal4f(draw(key, (uint32_t)i, 0, TAG_INIT, 0, p));
            s0 = (float)init_sd.x * z.x;
            s1 = (float)init_sd.y * z.y;
            s2 = (float)init_sd.z * z.z;
            s3 = (float)init_sd.w * z.w;
        }
        x[i] = s0;
        x[n + i] = s1;
        x[2 * n + i] = s2;
        x[3 * n + i] = s3;
        const double l = obs((double)s0, yx, (double)s1, yy);
        lw[i] = l;
        lwv[k] = l;
    }
    tile_partial(lwv, part + blockIdx.x, red);
}

hipError_t launch_pf_init(Ctx &c)
{
    const Key key = make_key(c.cfg.seed);
    const double4 sd = make_double4(c.cfg.init_sd[0], c.cfg.init_sd[1], c.cfg.init_sd[2],
                                    c.cfg.init_sd[3]);
    const dim3 grid((unsigned)c.ntiles);
    if (c.elem_bytes == 4)
        hipLaunchKernelGGL(pf_init_kernel<float>, grid, dim3(TPB), 0, c.stream,
                           (float *)c.state_ptr(), c.buf.log_weight, c.n, key, c.cfg.problem_id,
                           sd, c.buf.data, make_obs(c), c.partials());
    else
        hipLaunchKernelGGL(pf_init_kernel<double>, grid, dim3(TPB), 0, c.stream,
                           (double *)c.state_ptr(), c.buf.log_weight, c.n, key, c.cfg.problem_id,
                           sd, c.buf.data, make_obs(c), c.partials());
    return hipGetLastError();
}

// One move of Algorithm "pf" for the particles of one tile, reading through
// the pending ancestors, writing the ping-pong partner; with FUSE the
// incremental log-weight of observation y is added (after a resample the
// previous weights count as zero) and the tile partial is produced.  With
// MON the tile also sums w_i and w_i x_i of the incoming population (the
// monitor of the previous step: w_i = 1 after a resample, else
// exp(lw_i - M)), column-major into mon[5][ntiles].
template <typename T, bool FUSE, bool MON>
__global__ __launch_bounds__(TPB) void pf_move_kernel(
    const T *__restrict__ xin, T *__restrict__ xout, double *__restrict__ lw,
    const int32_t *__restrict__ anc, const double *__restrict__ scalars, int gather_check,
    int reset_check, int64_t n, Key key, uint32_t t, uint32_t p, Motion mv,
    const double *__restrict__ y, ObsModel obs, TilePartial *__restrict__ part,
    double *__restrict__ mon, int64_t ntiles)
{
    __shared__ double red[NWAVES];
    const bool resampled = (gather_check | reset_check) ? scalars[SMC_S_RESAMPLED] != 0.0 : false;
    const bool gather = gather_check && resampled;
    const bool reset = reset_check && resampled;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    double yx = 0.0, yy = 0.0;
    if (FUSE) {
        yx = y[0];
        yy = y[1];
    }
    const double M = MON ? scalars[SMC_S_M] : 0.0;
    double ms[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double lwv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        lwv[k] = -INFINITY;
        if (i >= n)
            continue;
        const int64_t src = gather ? (int64_t)anc[i] : i;
        const T px = xin[src], py = xin[n + src], vx = xin[2 * n + src], vy = xin[3 * n + src];
        const double lw_in = (FUSE && !reset) || (MON && !reset) ? lw[i] : 0.0;
        if (MON) {
            const double w = reset ? 1.0 : (lw_in > -INFINITY ? exp(lw_in - M) : 0.0);
            if (w != 0.0) {
                ms[0] += w;
                ms[1] += w * (double)px;
                ms[2] += w * (double)py;
                ms[3] += w * (double)vx;
                ms[4] += w * (double)vy;
            }
        }
        T npx, npy, nvx, nvy;
        if constexpr (sizeof(T) == 8) {
            const double2 a = normal2(draw(key, (uint32_t)i, t, TAG_PF_MOVE, 0, p));
            const double2 b = normal2(draw(key, (uint32_t)i, t, TAG_PF_MOVE, 1, p));
            npx = (px + mv.dt * vx) + mv.sd_pos * a.x;
            npy = (py + mv.dt * vy) + mv.sd_pos * a.y;
            nvx = vx + mv.sd_vel * b.x;
            nvy = vy + mv.sd_vel * b.y;
        } else {
            const float4 z = normal4f(draw(key, (uint32_t)i, t, TAG_PF_MOVE, 0, p));
            const float dt = (float)mv.dt, sp = (float)mv.sd_pos, sv = (float)mv.sd_vel;
            npx = (px + dt * vx) + sp * z.x;
            npy = (py + dt * vy) + sp * z.y;
            nvx = vx + sv * z.z;
            nvy = vy + sv * z.w;
        }
        xout[i] = npx;
        xout[n + i] = npy;
        xout[2 * n + i] = nvx;
        xout[3 * n + i] = nvy;
        if (FUSE) {
            const double inc = obs((double)npx, yx, (double)npy, yy);
            const double l = lw_in + inc;
            lw[i] = l;
            lwv[k] = l;
        }
    }
    if (FUSE)
        tile_partial(lwv, part + blockIdx.x, red);
    if (MON) {
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const double v = block_sum<NWAVES>(ms[r], red);
            if (threadIdx.x == 0)
                mon[(int64_t)r * ntiles + blockIdx.x] = v;
        }
    }
}

template <typename T, bool FUSE, bool MON>
static void launch_move_t(Ctx &c, int32_t step, int32_t obs_index, bool gather_check,
                          bool reset_check)
{
    const Key key = make_key(c.cfg.seed);
    const Motion mv{c.cfg.dt, c.cfg.sd_pos, c.cfg.sd_vel};
    hipLaunchKernelGGL((pf_move_kernel<T, FUSE, MON>), dim3((unsigned)c.ntiles), dim3(TPB), 0,
                       c.stream, (const T *)c.state_ptr(), (T *)c.other_ptr(), c.buf.log_weight,
                       c.buf.ancestors, c.buf.scalars, (int)gather_check, (int)reset_check, c.n,
                       key, (uint32_t)step, c.cfg.problem_id, mv,
                       c.buf.data + 2 * (int64_t)obs_index, make_obs(c), c.partials(), c.mon(),
                       c.ntiles);
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
__global__ __launch_bounds__(TPB) void pf_reweight_kernel(const T *__restrict__ x,
                                                          double *__restrict__ lw,
                                                          const double *__restrict__ scalars,
                                                          int reset_check, int64_t n,
                                                          const double *__restrict__ y,
                                                          ObsModel obs,
                                                          TilePartial *__restrict__ part)
{
    __shared__ double red[NWAVES];
    const bool reset = reset_check && scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const double yx = y[0], yy = y[1];
    double lwv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        lwv[k] = -INFINITY;
        if (i >= n)
            continue;
        const double inc = obs((double)x[i], yx, (double)x[n + i], yy);
        const double l = (reset ? 0.0 : lw[i]) + inc;
        lw[i] = l;
        lwv[k] = l;
    }
    tile_partial(lwv, part + blockIdx.x, red);
}

hipError_t launch_pf_reweight(Ctx &c, int32_t obs_index, bool reset_check)
{
    const dim3 grid((unsigned)c.ntiles);
    const double *y = c.buf.data + 2 * (int64_t)obs_index;
    if (c.elem_bytes == 4)
        hipLaunchKernelGGL(pf_reweight_kernel<float>, grid, dim3(TPB), 0, c.stream,
                           (const float *)c.state_ptr(), c.buf.log_weight, c.buf.scalars,
                           (int)reset_check, c.n, y, make_obs(c), c.partials());
    else
        hipLaunchKernelGGL(pf_reweight_kernel<double>, grid, dim3(TPB), 0, c.stream,
                           (const double *)c.state_ptr(), c.buf.log_weight, c.buf.scalars,
                           (int)reset_check, c.n, y, make_obs(c), c.partials());
    return hipGetLastError();
}

}  // namespace smc
