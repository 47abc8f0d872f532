// smc_gmm_kc.hip -- instantiations of the K-templated mixture kernels for K = 9..12.
#include "smc_gmm_impl.hpp"

namespace smc {

template struct GmmK<9>;
template struct GmmK<10>;
template struct GmmK<11>;
template struct GmmK<12>;

}  // namespace smc
