// smc_gmm.hip -- host launchers of the Gaussian-mixture sampler (Section
// 5.2) and its kernels that do not depend on the number of components: the
// tempering reweight and the partials of equal weights.  The K-templated
// kernels (prior draws, likelihood, Metropolis blocks) are in
// smc_gmm_impl.hpp and instantiated in smc_gmm_k*.hip.
#include <math.h>

#include "smc_gmm_impl.hpp"
#include "smc_tiles.hpp"

namespace smc {

extern template struct GmmK<1>;
extern template struct GmmK<2>;
extern template struct GmmK<3>;
extern template struct GmmK<4>;
extern template struct GmmK<5>;
extern template struct GmmK<6>;
extern template struct GmmK<7>;
extern template struct GmmK<8>;
extern template struct GmmK<9>;
extern template struct GmmK<10>;
extern template struct GmmK<11>;
extern template struct GmmK<12>;
extern template struct GmmK<13>;
extern template struct GmmK<14>;
extern template struct GmmK<15>;
extern template struct GmmK<16>;

// Tile partials of all-zero log-weights: m = 0, s1 = s2 = particles in tile.
__global__ void const_partials_kernel(TilePartial *__restrict__ part, int64_t ntiles, int64_t n)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < ntiles) {
        const double len = (double)min((int64_t)TILE, n - b * TILE);
        part[b] = TilePartial{0.0, len, len, 0.0};
    }
}

__global__ void const_partials_batch_kernel(const Prob *__restrict__ probs,
                                            const int2 *__restrict__ map, int64_t tiles)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < tiles) {
        const int2 pm = map[g];
        const Prob &P = probs[pm.x];
        const double len = (double)min((int64_t)TILE, P.n - (int64_t)pm.y * TILE);
        P.partials[pm.y] = TilePartial{0.0, len, len, 0.0};
    }
}

__global__ __launch_bounds__(TPB) void gmm_reweight_kernel(Prob P, const double *__restrict__ llrow,
                                                           int reset_check, double dalpha)
{
    gmm_reweight_tile(P, llrow, blockIdx.x, reset_check, dalpha);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

// Waves per 64-particle tile: enough waves overall to fill the GPU, at most
// GMM_MAXW, and no more than the data can feed (>= 32 points per wave).
int gmm_waves(int64_t n, int64_t nd)
{
    const int64_t tiles = ceil_div(n, WAVE);
    int W = 1;
    while (W < GMM_MAXW && tiles * W < 8192 && nd >= (int64_t)(2 * W) * 32)
        W *= 2;
    return W;
}

#define SMC_K_SWITCH(K_, CALL)                                                                   \
    switch (K_) {                                                                                \
    case 1: return CALL(1);                                                                      \
    case 2: return CALL(2);                                                                      \
    case 3: return CALL(3);                                                                      \
    case 4: return CALL(4);                                                                      \
    case 5: return CALL(5);                                                                      \
    case 6: return CALL(6);                                                                      \
    case 7: return CALL(7);                                                                      \
    case 8: return CALL(8);                                                                      \
    case 9: return CALL(9);                                                                      \
    case 10: return CALL(10);                                                                    \
    case 11: return CALL(11);                                                                    \
    case 12: return CALL(12);                                                                    \
    case 13: return CALL(13);                                                                    \
    case 14: return CALL(14);                                                                    \
    case 15: return CALL(15);                                                                    \
    case 16: return CALL(16);                                                                    \
    default: return hipErrorInvalidValue;                                                        \
    }

hipError_t launch_gmm_init(Ctx &c)
{
    const int W = gmm_waves(c.n, c.cfg.n_data);
#define CALL_INIT(k) GmmK<k>::init(c, W)
    hipError_t e;
    {
        auto f = [&]() -> hipError_t { SMC_K_SWITCH(c.cfg.K, CALL_INIT) };
        e = f();
    }
#undef CALL_INIT
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(const_partials_kernel, dim3((unsigned)ceil_div(c.ntiles, 256)), dim3(256),
                       0, c.stream, c.partials(), c.ntiles, c.n);
    return hipGetLastError();
}

hipError_t launch_gmm_reweight(Ctx &c, double dalpha, bool reset_check)
{
    const int D = 3 * c.cfg.K - 1;
    const double *llrow = (const double *)c.state_ptr() + (int64_t)D * c.n;
    hipLaunchKernelGGL(gmm_reweight_kernel, dim3((unsigned)c.ntiles), dim3(TPB), 0, c.stream,
                       make_prob(c), llrow, (int)reset_check, dalpha);
    return hipGetLastError();
}

hipError_t launch_gmm_move(Ctx &c, int32_t step, const smc_move_args &a, bool gather_check)
{
    // every block of every sweep in one launch (gmm_step_kernel)
    const int W = gmm_waves(c.n, c.cfg.n_data);
    const int sweeps = a.sweeps > 0 ? a.sweeps : (c.cfg.sweeps > 0 ? c.cfg.sweeps : 1);
    const double scale[3] = {a.scale[0], a.scale[1], a.scale[2]};
#define CALL_STEP(k) GmmK<k>::step(c, W, step, sweeps, a.alpha, scale, gather_check)
    hipError_t e;
    {
        auto f = [&]() -> hipError_t { SMC_K_SWITCH(c.cfg.K, CALL_STEP) };
        e = f();
    }
#undef CALL_STEP
    if (e == hipSuccess && gather_check)
        c.cur ^= 1;
    return e;
}

hipError_t launch_gmm_loglik_grad(const double *mu, const double *eta, const double *z,
                                  int64_t n, int32_t K, const double *y, int64_t n_data,
                                  double *loglik, double *grad, hipStream_t stream)
{
#define CALL_LL(k) GmmK<k>::loglik(mu, eta, z, n, y, n_data, loglik, grad, stream)
    SMC_K_SWITCH(K, CALL_LL)
#undef CALL_LL
}

// ---------------------------------------------------------------------------
// Batched initialisation (one launch per K group; W waves per 64-particle tile)
// ---------------------------------------------------------------------------
hipError_t launch_gmm_init_batch(const Prob *probs, const int2 *map64, int64_t tiles64, int K,
                                 int W, bool mala, hipStream_t s)
{
    if (tiles64 == 0)
        return hipSuccess;
#define CALL_IB(k) GmmK<k>::init_batch(probs, map64, tiles64, W, mala, s)
    SMC_K_SWITCH(K, CALL_IB)
#undef CALL_IB
}

hipError_t launch_const_partials_batch(const Prob *probs, const int2 *map, int64_t tiles,
                                       hipStream_t s)
{
    if (tiles == 0)
        return hipSuccess;
    hipLaunchKernelGGL(const_partials_batch_kernel, dim3((unsigned)ceil_div(tiles, 256)),
                       dim3(256), 0, s, probs, map, tiles);
    return hipGetLastError();
}

}  // namespace smc
