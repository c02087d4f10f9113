// Heat-bath sweeps of the gather form for q <= 16 and plans of at most
// kGSmallWaves waves per workgroup (adabmDCA 2.0, Sec. 2.1): the gather
// kernel instantiated with a 512-thread bound, which leaves 256 registers per
// lane, enough to read the tokens a chunk-step ahead with several site groups
// (the 16-wave instantiation spills there); apart from the 16-wave
// instantiation so that the two compile in parallel.
#include "gather_kernel.hpp"

namespace bmdca {

hipError_t launch_gather_heat_w8(int q, const GatherShape& gs, const GatherArgs& a) {
  if (gs.waves > kGSmallWaves) return hipErrorInvalidValue;
  switch (q) {
#define BMDCA_GQ(n) \
  case n:           \
    return launch_gather_shape<n, false, kGSmallWaves>(gs, a);
    BMDCA_GQ(2) BMDCA_GQ(3) BMDCA_GQ(4) BMDCA_GQ(5) BMDCA_GQ(6) BMDCA_GQ(7) BMDCA_GQ(8)
    BMDCA_GQ(9) BMDCA_GQ(10) BMDCA_GQ(11) BMDCA_GQ(12) BMDCA_GQ(13) BMDCA_GQ(14) BMDCA_GQ(15)
    BMDCA_GQ(16)
#undef BMDCA_GQ
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bmdca
