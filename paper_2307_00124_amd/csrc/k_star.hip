// Dispatch of the star stencil kernels on the storage type of x (the kernels
// live in star_impl.hpp, instantiated by k_star_x8/x16/x32.hip).
#include "kernels.hpp"

namespace bfpk {

hipError_t launch_star_x8(const StarLaunch& L, hipStream_t s);
hipError_t launch_star_x16(const StarLaunch& L, hipStream_t s);
hipError_t launch_star_x32(const StarLaunch& L, hipStream_t s);

hipError_t launch_star(const StarLaunch& L, hipStream_t s) {
  switch (L.xbits) {
    case 8: return launch_star_x8(L, s);
    case 16: return launch_star_x16(L, s);
    case 32: return launch_star_x32(L, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace bfpk
