// Dispatch of the grid-transfer kernels on the dimension (the kernels live
// in transfer_impl.hpp, instantiated by k_transfer2d.hip / k_transfer3d.hip).
#include "kernels.hpp"

namespace bfpk {

hipError_t launch_transfer2d(const TransferLaunch& L, hipStream_t s);
hipError_t launch_transfer3d(const TransferLaunch& L, hipStream_t s);

hipError_t launch_transfer(const TransferLaunch& L, hipStream_t s) {
  return L.ndim == 2 ? launch_transfer2d(L, s) : launch_transfer3d(L, s);
}

}  // namespace bfpk
