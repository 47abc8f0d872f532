// smc_gmm_ka.hip -- instantiations of the K-templated mixture kernels for K = 1..4.
#include "smc_gmm_impl.hpp"

namespace smc {

template struct GmmK<1>;
template struct GmmK<2>;
template struct GmmK<3>;
template struct GmmK<4>;

}  // namespace smc
