// 2D grid-transfer kernels (one translation unit per dimension).
#include "transfer_impl.hpp"

namespace bfpk {

hipError_t launch_transfer2d(const TransferLaunch& L, hipStream_t s) { return transfer_nd<2>(L, s); }

}  // namespace bfpk
