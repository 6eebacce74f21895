// Squaring layers of the SP2 recursion on gfx950 matrix cores.
//
// Every kernel here computes, for a symmetric X, one layer
//
//     Y = alpha * X^2 + beta * X + gamma * I
//
// which covers the SP2 activation and update of Alg. 1 (sigma = +1: (1, 0, 0) gives
// X^2; sigma = -1: (-1, 2, 0) gives 2X - X^2), both steps of Eq. Refinement, and the
// general second-order layer of Eq. general SP2.  Only output tiles (I, J) with I <= J
// are computed; each is written to (I, J) and mirrored to (J, I), so Y is exactly
// symmetric (the paper notes that only one half of a symmetric product is needed).
// Inside a diagonal tile only the elements with row <= col are kept and mirrored.
//
// k_square_split: Alg. 2 with the product of Eq. Square.  X is held as two
//   half-precision planes X0 = FP16[2^s X], X1 = FP16[2^s X - X0] (Eqs. Split1/Split2,
//   shifted by 2^s).  Because X is symmetric, rows of X are its columns, so both MFMA
//   operands are read as K-contiguous row panels: panel I gives A, panel J gives B.
//   Per K step the three products X0 X0 + X0 X1 + X1 X0 (= A + B + B^T of Alg. 2,
//   the X1 X1 term dropped) go into ONE FP32 accumulator with
//   v_mfma_f32_32x32x16_{f16,bf16}.  The epilogue scales by 2^-2s, applies the layer
//   coefficients, writes Y in FP32 and re-splits it into the planes of the next layer,
//   and reduces Tr Y and ||Y||_F^2 in FP64 (the traces that drive the next sigma).
// k_square_plain: the same layer with X in FP64 (v_mfma_f64_16x16x4_f64) or FP32
//   (v_mfma_f32_32x32x2_f32); used for the FP64/FP32 recursions and for the FP64
//   refinement layers.
//
// Staging: the K loop streams BK-deep slices of the row panels through LDS, double
// buffered; global loads of slice k+1 are in flight while slice k feeds the matrix
// cores.  LDS rows are XOR-swizzled (split kernel) or padded (plain kernel) so that
// the 64 lanes of a fragment read hit distinct banks.
#include "sp2_internal.h"

namespace sp2 {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T16>
struct HalfOps;
template <>
struct HalfOps<_Float16> {
    typedef f16x8 vec8;
    typedef f16x4 vec4;
    __device__ static inline f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct HalfOps<__bf16> {
    typedef bf16x8 vec8;
    typedef bf16x4 vec4;
    __device__ static inline f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block reduction of (tr, fr) in a fixed order; `scratch` holds >= 2 * waves doubles.
template <int NWAVES>
__device__ inline void tile_partials(double tr, double fr, double* scratch, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    tr = wave_sum(tr);
    fr = wave_sum(fr);
    if (lane == 0) {
        scratch[2 * wave] = tr;
        scratch[2 * wave + 1] = fr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NWAVES; ++w) {
            a += scratch[2 * w];
            b += scratch[2 * w + 1];
        }
        out[0] = a;
        out[1] = b;
    }
}

// ===================================================================================
// Split (dual half-precision) square.
// ===================================================================================
constexpr int kBK = 32;                 // halves per row per stage (64 bytes)
constexpr int kRowBytes = kBK * 2;

__device__ inline int swz(int r) { return (r >> 2) & 3; }

template <typename T16, int BT, int WM, int WN>
__device__ __forceinline__ void split_body(const SquareArgs& a, int t) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BT / WM, WTN = BT / WN;
    constexpr int MB = WTM / 32, NB = WTN / 32;
    constexpr int ARR = BT * kRowBytes;     // bytes of one array in one stage
    constexpr int STAGE = 4 * ARR;          // A0, A1, B0, B1
    constexpr int CPT = (4 * BT) / NT;      // 16-byte chunks per thread per array
    static_assert(CPT >= 1 && (4 * BT) % NT == 0, "tile / thread mismatch");
    static_assert(MB >= 1 && NB >= 1, "wave tile too small");
    typedef typename HalfOps<T16>::vec8 vec8;
    typedef typename HalfOps<T16>::vec4 vec4;

    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];

    int I, J;
    tile_of(t, a.T, 8, &I, &J);
    const int np = a.np;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    const T16* x0 = (const T16*)a.x0;
    const T16* x1 = (const T16*)a.x1;
    const size_t pld = (size_t)plane_ld(np);   // plane row stride
    const T16* src[4] = {x0 + (size_t)I * BT * pld, x1 + (size_t)I * BT * pld, x0 + (size_t)J * BT * pld,
                         x1 + (size_t)J * BT * pld};

    u32x4 stg[4][CPT];
    f32x16 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.f;

    const int KT = np / kBK;

    auto gload = [&](int k0) {
#pragma unroll
        for (int arr = 0; arr < 4; ++arr)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int q = tid + i * NT;
                const int r = q >> 2, c = q & 3;
                stg[arr][i] = *(const u32x4*)(src[arr] + (size_t)r * pld + k0 + c * 8);
            }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int arr = 0; arr < 4; ++arr)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int q = tid + i * NT;
                const int r = q >> 2, c = q & 3;
                *(u32x4*)(lds + buf * STAGE + arr * ARR + r * kRowBytes + ((c ^ swz(r)) << 4)) = stg[arr][i];
            }
    };

    gload(0);
    lstore(0);
    __syncthreads();

    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        // the last iteration reloads its own slice (in bounds, unused) so that the
        // staging registers are written unconditionally
        gload((kt + 1 < KT ? kt + 1 : kt) * kBK);
        __builtin_amdgcn_sched_barrier(0);   // keep the global loads ahead of the MFMA work
        const unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            vec8 a0[MB], a1[MB], b0[NB], b1[NB];
            const int c = kk * 2 + (lane >> 5);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int r = wm * WTM + m * 32 + (lane & 31);
                const int off = r * kRowBytes + ((c ^ swz(r)) << 4);
                a0[m] = *(const vec8*)(base + off);
                a1[m] = *(const vec8*)(base + ARR + off);
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int r = wn * WTN + n * 32 + (lane & 31);
                const int off = r * kRowBytes + ((c ^ swz(r)) << 4);
                b0[n] = *(const vec8*)(base + 2 * ARR + off);
                b1[n] = *(const vec8*)(base + 3 * ARR + off);
            }
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = HalfOps<T16>::mfma(a0[m], b0[n], acc[m][n]);
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = HalfOps<T16>::mfma(a0[m], b1[n], acc[m][n]);
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = HalfOps<T16>::mfma(a1[m], b0[n], acc[m][n]);
        }
        __builtin_amdgcn_sched_barrier(0);
        lstore(buf ^ 1);   // buf ^ 1 was last read before the previous barrier
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    const float alpha = a.coef[0], beta = a.coef[1], gamma = a.coef[2];
    const float osc = a.out_scale, isc = a.in_scale;
    float* so = (float*)a.s_out;
    const float* si = (const float*)a.s_in;
    T16* p0 = (T16*)a.p0_out;
    T16* p1 = (T16*)a.p1_out;
    const bool diag = (I == J);
    double tr = 0.0, fr = 0.0;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int col = J * BT + wn * WTN + n * 32 + (lane & 31);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int row0 = I * BT + wm * WTM + m * 32 + 8 * g + 4 * (lane >> 5);
                float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (beta != 0.f) s4 = *(const float4*)(si + (size_t)col * np + row0);  // = S[row0..+3][col]
                const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
                float v[4];
                T16 h0[4], h1[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float x = acc[m][n][4 * g + e] * osc;
                    float y = (beta != 0.f) ? fmaf(alpha, x, beta * sv[e]) : alpha * x;
                    if (row0 + e == col && col < a.n_real) y += gamma;
                    v[e] = y;
                    const float ys = y * isc;
                    h0[e] = (T16)ys;
                    h1[e] = (T16)(ys - (float)h0[e]);
                }
                if (!diag) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const size_t off = (size_t)(row0 + e) * np + col;
                        so[off] = v[e];
                        if (p0) {
                            const size_t poff = (size_t)(row0 + e) * pld + col;
                            p0[poff] = h0[e];
                            p1[poff] = h1[e];
                        }
                        fr += 2.0 * (double)v[e] * (double)v[e];
                    }
                    const size_t moff = (size_t)col * np + row0;
                    *(float4*)(so + moff) = make_float4(v[0], v[1], v[2], v[3]);
                    if (p0) {
                        vec4 q0 = {h0[0], h0[1], h0[2], h0[3]};
                        vec4 q1 = {h1[0], h1[1], h1[2], h1[3]};
                        const size_t pmoff = (size_t)col * pld + row0;
                        *(vec4*)(p0 + pmoff) = q0;
                        *(vec4*)(p1 + pmoff) = q1;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = row0 + e;
                        if (row > col) continue;
                        const size_t off = (size_t)row * np + col;
                        so[off] = v[e];
                        if (p0) {
                            const size_t poff = (size_t)row * pld + col;
                            p0[poff] = h0[e];
                            p1[poff] = h1[e];
                        }
                        if (row < col) {
                            const size_t moff = (size_t)col * np + row;
                            so[moff] = v[e];
                            if (p0) {
                                const size_t pmoff = (size_t)col * pld + row;
                                p0[pmoff] = h0[e];
                                p1[pmoff] = h1[e];
                            }
                            fr += 2.0 * (double)v[e] * (double)v[e];
                        } else {
                            tr += (double)v[e];
                            fr += (double)v[e] * (double)v[e];
                        }
                    }
                }
            }
        }
    }
    if (a.parts) {
        __syncthreads();   // LDS stages are free now
        tile_partials<NT / 64>(tr, fr, (double*)lds, a.parts + 2 * t);
    }
}

// ===================================================================================
// Plain (FP64 / FP32) square.
// ===================================================================================
template <typename E>
struct PlainOps;

// FP64: v_mfma_f64_16x16x4_f64.  Lane l holds A[l%16][l/16], B[l/16][l%16]; the
// result block element (4*e + l/16, l%16) is acc[e] (rows interleaved across the
// four 16-lane groups).
template <>
struct PlainOps<double> {
    typedef f64x4 accv;
    static constexpr int BLK = 16;       // output block edge
    static constexpr int KSTEP = 4;      // K per instruction
    static constexpr int ACCN = 4;       // accumulators per lane per block
    static constexpr int BK = 16;        // K per LDS stage (128 bytes per row)
    static constexpr int PAD = 1;        // elements of row padding
    __device__ static inline accv mfma(double a, double b, accv c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row / col of accumulator r of this lane inside a block
    __device__ static inline int arow(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static inline int acol(int lane) { return lane & 15; }
    __device__ static inline int frow(int lane) { return lane & 15; }
    __device__ static inline int fk(int lane) { return lane >> 4; }
};

// FP32: v_mfma_f32_32x32x2_f32.  Lane l holds A[l%32][l/32]; the result element
// (8*(r/4) + 4*(l/32) + r%4, l%32) is acc[r].
template <>
struct PlainOps<float> {
    typedef f32x16 accv;
    static constexpr int BLK = 32;
    static constexpr int KSTEP = 2;
    static constexpr int ACCN = 16;
    static constexpr int BK = 32;        // 128 bytes per row
    static constexpr int PAD = 1;
    __device__ static inline accv mfma(float a, float b, accv c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int arow(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    __device__ static inline int acol(int lane) { return lane & 31; }
    __device__ static inline int frow(int lane) { return lane & 31; }
    __device__ static inline int fk(int lane) { return lane >> 5; }
};

template <typename E, int BT, int WM, int WN>
__device__ __forceinline__ void plain_body(const SquareArgs& a, int t) {
    typedef PlainOps<E> Ops;
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BT / WM, WTN = BT / WN;
    constexpr int MB = WTM / Ops::BLK, NB = WTN / Ops::BLK;
    constexpr int BK = Ops::BK;
    constexpr int LROW = BK + Ops::PAD;                // elements per LDS row
    constexpr int ARR = BT * LROW;                     // elements per array per stage
    constexpr int EPC = 16 / (int)sizeof(E);           // elements per 16-byte chunk
    constexpr int CPR = BK / EPC;                      // chunks per row
    constexpr int CPT = (BT * CPR) / NT;               // chunks per thread per array
    static_assert(CPT >= 1 && (BT * CPR) % NT == 0, "tile / thread mismatch");
    static_assert(MB >= 1 && NB >= 1, "wave tile too small");

    __shared__ E lds[2 * 2 * ARR];
    __shared__ double red[2 * (NT / 64)];

    int I, J;
    tile_of(t, a.T, 8, &I, &J);
    const int np = a.np;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const E* x = (const E*)a.x0;
    const E* src[2] = {x + (size_t)I * BT * np, x + (size_t)J * BT * np};

    typedef typename Ops::accv accv;
    accv acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int r = 0; r < Ops::ACCN; ++r) acc[m][n][r] = (E)0;

    u32x4 stg[2][CPT];
    const int KT = np / BK;
    auto gload = [&](int k0) {
#pragma unroll
        for (int arr = 0; arr < 2; ++arr)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int q = tid + i * NT;
                const int r = q / CPR, c = q % CPR;
                stg[arr][i] = *(const u32x4*)(src[arr] + (size_t)r * np + k0 + c * EPC);
            }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int arr = 0; arr < 2; ++arr)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int q = tid + i * NT;
                const int r = q / CPR, c = q % CPR;
                E* dst = lds + (buf * 2 + arr) * ARR + r * LROW + c * EPC;
                const E* v = (const E*)&stg[arr][i];
#pragma unroll
                for (int e = 0; e < EPC; ++e) dst[e] = v[e];
            }
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < KT) gload((kt + 1) * BK);
        const E* A = lds + (buf * 2 + 0) * ARR;
        const E* B = lds + (buf * 2 + 1) * ARR;
#pragma unroll
        for (int ks = 0; ks < BK / Ops::KSTEP; ++ks) {
            const int k = ks * Ops::KSTEP + Ops::fk(lane);
            E av[MB], bv[NB];
#pragma unroll
            for (int m = 0; m < MB; ++m) av[m] = A[(wm * WTM + m * Ops::BLK + Ops::frow(lane)) * LROW + k];
#pragma unroll
            for (int n = 0; n < NB; ++n) bv[n] = B[(wn * WTN + n * Ops::BLK + Ops::frow(lane)) * LROW + k];
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = Ops::mfma(av[m], bv[n], acc[m][n]);
        }
        if (kt + 1 < KT) lstore(buf ^ 1);
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    const E alpha = a.coef64 ? (E)a.coef64[0] : (E)a.coef[0];
    const E beta = a.coef64 ? (E)a.coef64[1] : (E)a.coef[1];
    const E gamma = a.coef64 ? (E)a.coef64[2] : (E)a.coef[2];
    E* so = (E*)a.s_out;
    const E* si = (const E*)a.s_in;
    const int ldo = a.ld_out, nv = a.n_valid;
    const bool diag = (I == J);
    double tr = 0.0, fr = 0.0;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int col = J * BT + wn * WTN + n * Ops::BLK + Ops::acol(lane);
#pragma unroll
            for (int r = 0; r < Ops::ACCN; ++r) {
                const int row = I * BT + wm * WTM + m * Ops::BLK + Ops::arow(lane, r);
                if (diag && row > col) continue;
                const E xv = acc[m][n][r];
                E y = (beta != (E)0) ? alpha * xv + beta * si[(size_t)col * np + row] : alpha * xv;
                if (row == col && col < a.n_real) y += gamma;
                if (row < nv && col < nv) {
                    so[(size_t)row * ldo + col] = y;
                    if (row != col) so[(size_t)col * ldo + row] = y;
                }
                const double yd = (double)y;
                if (row == col) {
                    tr += yd;
                    fr += yd * yd;
                } else {
                    fr += 2.0 * yd * yd;
                }
            }
        }
    }
    if (a.parts) tile_partials<NT / 64>(tr, fr, red, a.parts + 2 * t);
}

// Single problem: hardware block -> XCD-grouped tile index.
template <typename T16, int BT, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_square_split(SquareArgs a) {
    if (a.skip && *a.skip) return;
    const int t = xcd_tile_index(blockIdx.x, a.per, a.ntiles);
    if (t < 0) return;
    split_body<T16, BT, WM, WN>(a, t);
}
template <typename E, int BT, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_square_plain(SquareArgs a) {
    if (a.skip && *a.skip) return;
    const int t = xcd_tile_index(blockIdx.x, a.per, a.ntiles);
    if (t < 0) return;
    plain_body<E, BT, WM, WN>(a, t);
}

// Many problems in one launch: block b belongs to the problem p with offs[p] <= b <
// offs[p + 1] and handles that problem's tile b - offs[p]; each problem brings its own
// arguments (buffers, coefficients, skip flag).
template <typename T16, int BT, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_square_split_g(const SquareArgs* __restrict__ descs,
                                                                 const int* __restrict__ offs, int nprob) {
    const int p = find_group(offs, nprob, blockIdx.x);
    const SquareArgs a = descs[p];
    if (a.skip && *a.skip) return;
    split_body<T16, BT, WM, WN>(a, blockIdx.x - offs[p]);
}
template <typename E, int BT, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_square_plain_g(const SquareArgs* __restrict__ descs,
                                                                 const int* __restrict__ offs, int nprob) {
    const int p = find_group(offs, nprob, blockIdx.x);
    const SquareArgs a = descs[p];
    if (a.skip && *a.skip) return;
    plain_body<E, BT, WM, WN>(a, blockIdx.x - offs[p]);
}

template <int BT>
int grid_of(int np, int* T, int* ntiles, int* per) {
    *T = np / BT;
    *ntiles = ntiles_upper(*T);
    *per = (*ntiles + 7) / 8;
    return 8 * *per;
}

}  // namespace

int square_split_grid(int tile, int np, int* T, int* ntiles, int* per) {
    if (tile == 256) return grid_of<256>(np, T, ntiles, per);
    if (tile == 128) return grid_of<128>(np, T, ntiles, per);
    return grid_of<64>(np, T, ntiles, per);
}
int square_plain_grid(int tile, int np, int* T, int* ntiles, int* per) {
    if (tile == 128) return grid_of<128>(np, T, ntiles, per);
    return grid_of<64>(np, T, ntiles, per);
}

hipError_t launch_square_split(int precision, int tile, const SquareArgs& a, hipStream_t s) {
    const int grid = 8 * a.per;
#define SP2_L(T16, BT, WM, WN) \
    hipLaunchKernelGGL((k_square_split<T16, BT, WM, WN>), dim3(grid), dim3(64 * WM * WN), 0, s, a)
    if (precision == SP2_FP16X2) {
        if (tile == 256) SP2_L(_Float16, 256, 2, 4);
        else if (tile == 128) SP2_L(_Float16, 128, 2, 2);
        else SP2_L(_Float16, 64, 2, 2);
    } else if (precision == SP2_BF16X2) {
        if (tile == 256) SP2_L(__bf16, 256, 2, 4);
        else if (tile == 128) SP2_L(__bf16, 128, 2, 2);
        else SP2_L(__bf16, 64, 2, 2);
    } else {
        return hipErrorInvalidValue;
    }
#undef SP2_L
    return hipGetLastError();
}

hipError_t launch_square_split_g(int precision, int tile, const SquareArgs* descs, const int* offs, int nprob,
                                 int blocks, hipStream_t s) {
#define SP2_L(T16, BT, WM, WN) \
    hipLaunchKernelGGL((k_square_split_g<T16, BT, WM, WN>), dim3(blocks), dim3(64 * WM * WN), 0, s, descs, offs, nprob)
    if (precision == SP2_FP16X2) {
        if (tile == 128) SP2_L(_Float16, 128, 2, 2);
        else SP2_L(_Float16, 64, 2, 2);
    } else if (precision == SP2_BF16X2) {
        if (tile == 128) SP2_L(__bf16, 128, 2, 2);
        else SP2_L(__bf16, 64, 2, 2);
    } else {
        return hipErrorInvalidValue;
    }
#undef SP2_L
    return hipGetLastError();
}

hipError_t launch_square_plain_g(int precision, int tile, const SquareArgs* descs, const int* offs, int nprob,
                                 int blocks, hipStream_t s) {
#define SP2_L(E, BT, WM, WN) \
    hipLaunchKernelGGL((k_square_plain_g<E, BT, WM, WN>), dim3(blocks), dim3(64 * WM * WN), 0, s, descs, offs, nprob)
    if (precision == SP2_FP64) {
        if (tile == 128) SP2_L(double, 128, 2, 2);
        else SP2_L(double, 64, 2, 2);
    } else if (precision == SP2_FP32) {
        if (tile == 128) SP2_L(float, 128, 2, 2);
        else SP2_L(float, 64, 2, 2);
    } else {
        return hipErrorInvalidValue;
    }
#undef SP2_L
    return hipGetLastError();
}

hipError_t launch_square_plain(int precision, int tile, const SquareArgs& a, hipStream_t s) {
    const int grid = 8 * a.per;
#define SP2_L(E, BT, WM, WN) \
    hipLaunchKernelGGL((k_square_plain<E, BT, WM, WN>), dim3(grid), dim3(64 * WM * WN), 0, s, a)
    if (precision == SP2_FP64) {
        if (tile == 128) SP2_L(double, 128, 2, 2);
        else SP2_L(double, 64, 2, 2);
    } else if (precision == SP2_FP32) {
        if (tile == 128) SP2_L(float, 128, 2, 2);
        else SP2_L(float, 64, 2, 2);
    } else {
        return hipErrorInvalidValue;
    }
#undef SP2_L
    return hipGetLastError();
}

}  // namespace sp2
