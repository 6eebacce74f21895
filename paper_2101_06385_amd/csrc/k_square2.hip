// Host side of the persistent split squaring schedule: variant table, schedule plan
// and dispatch to the kernel instantiations (k_sk_f16.hip, k_sk_bf16.hip).
#include "sp2_internal.h"

namespace sp2 {

template <typename T16>
hipError_t launch_sk256_t(int variant, const SquareArgs& a, const StreamK& sk, hipStream_t s);
template <typename T16>
hipError_t launch_sk128_t(int variant, const SquareArgs& a, const StreamK& sk, hipStream_t s);
extern template hipError_t launch_sk256_t<_Float16>(int, const SquareArgs&, const StreamK&, hipStream_t);
extern template hipError_t launch_sk256_t<__bf16>(int, const SquareArgs&, const StreamK&, hipStream_t);
extern template hipError_t launch_sk128_t<_Float16>(int, const SquareArgs&, const StreamK&, hipStream_t);
extern template hipError_t launch_sk128_t<__bf16>(int, const SquareArgs&, const StreamK&, hipStream_t);
template <typename T16>
hipError_t launch_sk_t(int tile, int variant, const SquareArgs& a, const StreamK& sk, hipStream_t s) {
    if (tile == 256) return launch_sk256_t<T16>(variant, a, sk, s);
    if (tile == 128) return launch_sk128_t<T16>(variant, a, sk, s);
    return hipErrorInvalidValue;
}
template <typename T16>
hipError_t launch_dp_t(int tile, int variant, const SquareArgs& a, const SquareArgs* descs, const int* map, int per,
                       hipStream_t s);
extern template hipError_t launch_dp_t<_Float16>(int, int, const SquareArgs&, const SquareArgs*, const int*, int,
                                                 hipStream_t);
extern template hipError_t launch_dp_t<__bf16>(int, int, const SquareArgs&, const SquareArgs*, const int*, int,
                                               hipStream_t);

// Variants of the persistent kernel per tile edge: (waves, slice width in halves, LDS
// stages, rolling fragment pipeline).
// Selected by index; the measured best is the automatic choice of the host driver.
namespace {
struct SkVariant {
    int waves, sk, stages, rolling;
};
// keep in step with the launch table in k_square_sk.h
constexpr SkVariant kV256[kSkVariants] = {{4, 16, 4, 0}, {8, 16, 4, 0}, {4, 32, 2, 0},
                                          {8, 32, 2, 0}, {4, 32, 2, 1}, {8, 32, 2, 1}};
constexpr SkVariant kV128[kSkVariants] = {{4, 32, 4, 0}, {4, 64, 2, 0}, {4, 16, 4, 0},
                                          {4, 32, 2, 0}, {4, 64, 2, 1}, {4, 32, 2, 1}};
const SkVariant* sk_variant(int tile, int variant) {
    if (variant < 0 || variant >= kSkVariants) return nullptr;
    if (tile == 256) return &kV256[variant];
    if (tile == 128) return &kV128[variant];
    return nullptr;
}
}  // namespace

// Persistent schedule for a split square on n_p: G = CUs x workgroups per CU (a multiple
// of 8, at most kMaxSkGrid), R whole rounds, and the leftover tiles cut into s = G / rem
// K-chunks.  With fewer tiles than workgroups the stream-K form splits all the K-slices of
// all tiles evenly over the workgroups (see StreamK).
bool square_sk_plan(int tile, int variant, int np, int cus, int* wg_per_cu, StreamK* sk, int* T, int* ntiles) {
    const SkVariant* V = sk_variant(tile, variant);
    if (!V) return false;
    *T = np / tile;
    *ntiles = ntiles_upper(*T);
    const int lds = V->stages * 4 * tile * V->sk * 2;
    int per_cu = (160 * 1024) / lds;
    if (tile == 256 || per_cu < 1) per_cu = 1;   // 256 tiles: the accumulators fill the register file
    if (per_cu > 2) per_cu = 2;
    int g = cus * per_cu;
    if (g > kSkGroupSlot) g = kSkGroupSlot;   // chunk partial slots stay below the group slots
    g -= g % 8;
    if (g < 8) return false;
    const int KS = np / V->sk;
    const int Q = V->sk >= 32 ? 1 : 2;   // tail chunks are cut on groups of Q slices
    sk->grid = g;
    sk->stream_k = 0;
    if (*ntiles < g) {
        // fewer tiles than workgroups: stream-K ranges of equal length over all tiles
        const long long ksq = KS / Q, U = (long long)*ntiles * ksq;
        const long long per = U / g;   // whole units of the shortest range
        if (per < 1 || 2 * g > kMaxSkGrid || *ntiles > kMaxSkGrid) return false;
        if ((ksq + per - 1) / per + 1 > kSkMaxContrib) return false;
        sk->rounds = 0;
        sk->tail_tiles = *ntiles;
        sk->chunks = 0;
        sk->stream_k = Q;
    } else {
        sk->rounds = *ntiles / g;
        sk->tail_tiles = *ntiles % g;
        sk->chunks = sk->tail_tiles ? g / sk->tail_tiles : 1;
        if (sk->chunks > KS / Q) sk->chunks = KS / Q;
    }
    *wg_per_cu = per_cu;
    return true;
}

size_t square_sk_partial_bytes(int tile, int np) {
    (void)np;
    return (size_t)kMaxSkGrid * tile * tile * sizeof(float);
}

hipError_t launch_square_sk(int precision, int tile, int variant, const SquareArgs& a, const StreamK& sk,
                            hipStream_t s) {
    if (precision == SP2_FP16X2) return launch_sk_t<_Float16>(tile, variant, a, sk, s);
    if (precision == SP2_BF16X2) return launch_sk_t<__bf16>(tile, variant, a, sk, s);
    return hipErrorInvalidValue;
}

}  // namespace sp2

namespace sp2 {
hipError_t launch_square_dp(int precision, int tile, int variant, const SquareArgs& a, hipStream_t s) {
    if (precision == SP2_FP16X2) return launch_dp_t<_Float16>(tile, variant, a, nullptr, nullptr, 0, s);
    if (precision == SP2_BF16X2) return launch_dp_t<__bf16>(tile, variant, a, nullptr, nullptr, 0, s);
    return hipErrorInvalidValue;
}
hipError_t launch_square_dp_g(int precision, int tile, int variant, const SquareArgs* descs, const int* map, int per,
                              hipStream_t s) {
    const SquareArgs unused{};
    if (precision == SP2_FP16X2) return launch_dp_t<_Float16>(tile, variant, unused, descs, map, per, s);
    if (precision == SP2_BF16X2) return launch_dp_t<__bf16>(tile, variant, unused, descs, map, per, s);
    return hipErrorInvalidValue;
}
}  // namespace sp2
