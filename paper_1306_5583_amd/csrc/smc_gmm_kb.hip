// smc_gmm_kb.hip -- instantiations of the K-templated mixture kernels for K = 5..8.
#include "smc_gmm_impl.hpp"

namespace smc {

template struct GmmK<5>;
template struct GmmK<6>;
template struct GmmK<7>;
template struct GmmK<8>;

}  // namespace smc
