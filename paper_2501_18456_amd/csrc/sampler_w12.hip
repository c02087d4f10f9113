// Heat-bath sweeps of the gather form for q > 16 and plans of at most
// kGMidWaves waves per workgroup (adabmDCA 2.0, Sec. 2.1): the gather kernel
// instantiated with a 768-thread bound, which leaves 168 registers per lane;
// under the 16-wave bound (128) the kernel spills two registers to scratch.
// Apart from the other instantiations so that they compile in parallel.
#include "gather_kernel.hpp"

namespace bmdca {

hipError_t launch_gather_heat_w12(int q, const GatherShape& gs, const GatherArgs& a) {
  if (gs.waves > kGMidWaves) return hipErrorInvalidValue;
  switch (q) {
#define BMDCA_GQ(n) \
  case n:           \
    return launch_gather_shape<n, false, kGMidWaves>(gs, a);
    BMDCA_GQ(17) BMDCA_GQ(18) BMDCA_GQ(19) BMDCA_GQ(20) BMDCA_GQ(21) BMDCA_GQ(22) BMDCA_GQ(23)
    BMDCA_GQ(24) BMDCA_GQ(25) BMDCA_GQ(26) BMDCA_GQ(27) BMDCA_GQ(28) BMDCA_GQ(29) BMDCA_GQ(30)
    BMDCA_GQ(31) BMDCA_GQ(32)
#undef BMDCA_GQ
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bmdca
