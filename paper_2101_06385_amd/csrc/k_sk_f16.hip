// Persistent split squaring kernels for FP16 planes.
#include "k_square_sk.h"

namespace sp2 {
template hipError_t launch_sk_t<_Float16>(int tile, int variant, const SquareArgs& a, const StreamK& sk,
                                       hipStream_t s);
template hipError_t launch_dp_t<_Float16>(int tile, int variant, const SquareArgs& a, const SquareArgs* descs,
                                       const int* offs, int nprob, int blocks, hipStream_t s);
}  // namespace sp2
