// Star stencil kernels for 32-bit x mantissas (one translation unit per
// x storage type keeps the instantiations of each file moderate).
#include "star_impl.hpp"

namespace bfpk {

hipError_t launch_star_x32(const StarLaunch& L, hipStream_t s) { return star_for_x<int32_t>(L, s); }

}  // namespace bfpk
