// Matrix-core (MFMA) sketch kernels for gfx950.
#include "qsk_device.hpp"
#include "qsk_kernels.hpp"

namespace qsk {

hipError_t launch_sketch_mfma(const SketchArgs &s) {
  (void)s;
  return hipErrorNotSupported;
}

}  // namespace qsk
