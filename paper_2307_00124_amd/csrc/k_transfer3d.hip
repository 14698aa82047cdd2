// 3D grid-transfer kernels (one translation unit per dimension).
#include "transfer_impl.hpp"

namespace bfpk {

hipError_t launch_transfer3d(const TransferLaunch& L, hipStream_t s) { return transfer_nd<3>(L, s); }

}  // namespace bfpk
