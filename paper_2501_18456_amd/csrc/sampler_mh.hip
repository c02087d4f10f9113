// Single-site Metropolis in the gather form (adabmDCA 2.0, Sec. 2.1, the
// Metropolis option of the sampler): the gather kernel with its Metropolis
// draw step, instantiated apart from the heat-bath draw so that the two
// compile in parallel.
#include "gather_kernel.hpp"

namespace bmdca {

hipError_t launch_gather_metropolis(const float* h, const float* Jt, int8_t* chains, int64_t N,
                                    int L, int q, int sweeps, uint64_t seed,
                                    uint64_t sweep_offset, float beta,
                                    unsigned long long* flips_out, int32_t* dev_err,
                                    hipStream_t s, const DevCtl& ctl) {
  return launch_gather_form<true>(h, Jt, chains, N, L, q, sweeps, seed, sweep_offset, beta,
                                  flips_out, dev_err, s, ctl);
}

}  // namespace bmdca
