// One-workgroup-per-tile split squaring kernels (single and grouped), BF16 planes.
#include "k_square_sk.h"

namespace sp2 {
template hipError_t launch_dp_t<__bf16>(int tile, int variant, const SquareArgs& a, const SquareArgs* descs,
                                     const int* map, int per, hipStream_t s);
}  // namespace sp2
