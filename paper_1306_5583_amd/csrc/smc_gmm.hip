// smc_gmm.hip -- tempered Gaussian-mixture sampler kernels (Section 5.2).
#include "smc_internal.hpp"

namespace smc {

hipError_t launch_gmm_init(Ctx &) { return hipErrorNotSupported; }
hipError_t launch_gmm_reweight(Ctx &, double, bool) { return hipErrorNotSupported; }
hipError_t launch_gmm_move(Ctx &, int32_t, const smc_move_args &, bool) { return hipErrorNotSupported; }
hipError_t launch_gmm_loglik_grad(const double *, const double *, const double *, int64_t, int32_t,
                                  const double *, int64_t, double *, double *, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace smc
