// Matrix-core (MFMA) contraction for many-channel cubes.
#include "cg_internal.hpp"

namespace cg {

bool mfma_available() { return false; }

hipError_t launch_gather_mfma(const TileView&, const KernelParams&, int64_t, const uint32_t*,
                              const void*, int, int64_t, int64_t, int, const OutView&,
                              hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace cg
