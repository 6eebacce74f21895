// Persistent split squaring kernels on 256-wide tiles, BF16 planes.
#include "k_square_sk.h"

namespace sp2 {
template hipError_t launch_sk256_t<__bf16>(int variant, const SquareArgs& a, const StreamK& sk,
                                        hipStream_t s);
}  // namespace sp2
