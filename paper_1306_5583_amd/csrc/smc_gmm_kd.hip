// smc_gmm_kd.hip -- instantiations of the K-templated mixture kernels for K = 13..16.
#include "smc_gmm_impl.hpp"

namespace smc {

template struct GmmK<13>;
template struct GmmK<14>;
template struct GmmK<15>;
template struct GmmK<16>;

}  // namespace smc
