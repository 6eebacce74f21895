// Kernels of the differentiable generalized-SP2 network (Eq. general SP2 as matrix layers)
//
//     X_{k+1} = W_k X_k^2 + B_k X_k + c_k I,   k = 0 .. K-1
//
// The forward layers reuse the squaring kernels (alpha, beta, gamma) = (W_k, B_k, c_k).
// This file holds what the network adds:
//   k_pack_coef   : (W, B, c) device arrays -> per-layer coefficient triples
//   k_copy_pad    : n x n (leading dimension ld) <-> zero-padded n_p x n_p
//   k_adjoint     : one reverse layer.  With G = dL/dX_{k+1} (symmetric),
//                   M = G X_k + X_k G,  G_k = W_k M + B_k G,
//                   and the FP64 tile partials of  Tr G (= dL/dc_k),
//                   <G, X_k>_F (= dL/dB_k)  and  <M, X_k>_F / 2 = <G, X_k^2>_F (= dL/dW_k).
//                   FP32 operands on v_mfma_f32_32x32x2_f32: the adjoint can grow by up to
//                   a factor 2 per layer in the eigenbasis, which half-precision planes
//                   could not hold, and FP32 keeps the gradients accurate.
//   k_reduce3     : fixed-order sum of the adjoint partials into dW_k, dB_k, dc_k.
#include "sp2_internal.h"

namespace sp2 {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

__global__ void k_pack_coef(const float* __restrict__ w, const float* __restrict__ b, const float* __restrict__ c,
                            int K, float* __restrict__ out) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        out[3 * k + 0] = w[k];
        out[3 * k + 1] = b[k];
        out[3 * k + 2] = c[k];
    }
}

// to_pad = 1: dst (np x np, zero padding) <- src (n x n, ld);  0: dst (n x n, ld) <- src (np x np)
__global__ void k_copy_pad(const float* __restrict__ src, float* __restrict__ dst, int n, int ld, int np,
                           int to_pad) {
    const size_t total = to_pad ? (size_t)np * np : (size_t)n * n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        if (to_pad) {
            const int i = (int)(idx / np), j = (int)(idx % np);
            dst[idx] = (i < n && j < n) ? src[(size_t)i * ld + j] : 0.f;
        } else {
            const int i = (int)(idx / n), j = (int)(idx % n);
            dst[(size_t)i * ld + j] = src[(size_t)i * np + j];
        }
    }
}

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// FP32 adjoint layer.  Output tiles (I <= J) of the symmetric M = G X + X G: panel I of G
// against panel J of X plus panel I of X against panel J of G (rows of a symmetric matrix
// are its columns, so all four operands are K-contiguous row panels).
template <int BT, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_adjoint(AdjointArgs a) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BT / WM, WTN = BT / WN;
    constexpr int MB = WTM / 32, NB = WTN / 32;
    constexpr int BK = 32;                 // floats per row per stage
    constexpr int LROW = BK + 1;           // padded row (floats)
    constexpr int ARR = BT * LROW;
    constexpr int CPR = BK / 4;            // 16-byte chunks per row
    constexpr int CPT = BT * CPR / NT;     // chunks per thread per array
    static_assert(CPT >= 1 && (BT * CPR) % NT == 0, "tile / thread mismatch");

    __shared__ float lds[2 * 4 * ARR];
    __shared__ double red[3 * (NT / 64)];

    const int t = xcd_tile_index(blockIdx.x, a.per, a.ntiles);
    if (t < 0) return;
    int I, J;
    tile_of(t, a.T, 8, &I, &J);
    const int np = a.np;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    // stage arrays: 0 = G panel I, 1 = X panel I, 2 = X panel J, 3 = G panel J
    const float* src[4] = {a.g + (size_t)I * BT * np, a.x + (size_t)I * BT * np, a.x + (size_t)J * BT * np,
                           a.g + (size_t)J * BT * np};

    f32x16 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.f;

    f32x4 stg[4][CPT];
    auto gload = [&](int k0) {
#pragma unroll
        for (int arr = 0; arr < 4; ++arr)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int q = tid + i * NT;
                const int r = q / CPR, c = q % CPR;
                stg[arr][i] = *(const f32x4*)(src[arr] + (size_t)r * np + k0 + c * 4);
            }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int arr = 0; arr < 4; ++arr)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int q = tid + i * NT;
                const int r = q / CPR, c = q % CPR;
                float* dst = lds + (buf * 4 + arr) * ARR + r * LROW + c * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[e] = stg[arr][i][e];
            }
    };

    const int KT = np / BK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        gload((kt + 1 < KT ? kt + 1 : kt) * BK);
        const float* gI = lds + (buf * 4 + 0) * ARR;
        const float* xI = lds + (buf * 4 + 1) * ARR;
        const float* xJ = lds + (buf * 4 + 2) * ARR;
        const float* gJ = lds + (buf * 4 + 3) * ARR;
#pragma unroll
        for (int ks = 0; ks < BK / 2; ++ks) {
            const int k = 2 * ks + (lane >> 5);
            float ga[MB], xa[MB], xb[NB], gb[NB];
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int r = (wm * WTM + m * 32 + (lane & 31)) * LROW + k;
                ga[m] = gI[r];
                xa[m] = xI[r];
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int r = (wn * WTN + n * 32 + (lane & 31)) * LROW + k;
                xb[n] = xJ[r];
                gb[n] = gJ[r];
            }
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(ga[m], xb[n], acc[m][n], 0, 0, 0);
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[m], gb[n], acc[m][n], 0, 0, 0);
        }
        lstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue: G_k = W M + B G over row <= col, mirrored; FP64 partials
    const float wk = a.coef[0], bk = a.coef[1];
    const bool diag = (I == J);
    double p_tr = 0.0, p_gx = 0.0, p_mx = 0.0;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int col = J * BT + wn * WTN + n * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = I * BT + wm * WTM + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (diag && row > col) continue;
                const size_t off = (size_t)row * np + col;
                const float mv = acc[m][n][r];
                const float gv = a.g[off];
                const float xv = a.x[off];
                const float gn = fmaf(wk, mv, bk * gv);
                a.g_out[off] = gn;
                if (row != col) a.g_out[(size_t)col * np + row] = gn;
                const double wgt = (row == col) ? 1.0 : 2.0;
                if (row == col) p_tr += (double)gv;
                p_gx += wgt * (double)gv * (double)xv;
                p_mx += 0.5 * wgt * (double)mv * (double)xv;
            }
        }
    }
    p_tr = wsum(p_tr);
    p_gx = wsum(p_gx);
    p_mx = wsum(p_mx);
    if (lane == 0) {
        red[3 * wave + 0] = p_tr;
        red[3 * wave + 1] = p_gx;
        red[3 * wave + 2] = p_mx;
    }
    __syncthreads();
    if (tid == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            s0 += red[3 * w];
            s1 += red[3 * w + 1];
            s2 += red[3 * w + 2];
        }
        a.parts[3 * t + 0] = s0;
        a.parts[3 * t + 1] = s1;
        a.parts[3 * t + 2] = s2;
    }
}

// dc_k = sum of Tr G parts, dB_k = <G, X>, dW_k = <G, X^2>
__global__ __launch_bounds__(kThreads) void k_reduce3(const double* __restrict__ parts, int nparts,
                                                      float* __restrict__ dw, float* __restrict__ db,
                                                      float* __restrict__ dc, int k) {
    __shared__ double sh[3][kThreads];
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
        v0 += parts[3 * i];
        v1 += parts[3 * i + 1];
        v2 += parts[3 * i + 2];
    }
    sh[0][threadIdx.x] = v0;
    sh[1][threadIdx.x] = v1;
    sh[2][threadIdx.x] = v2;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dc[k] = (float)sh[0][0];
        db[k] = (float)sh[1][0];
        dw[k] = (float)sh[2][0];
    }
}

inline int grid_for(size_t total) {
    size_t g = (total + kThreads - 1) / kThreads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_pack_coef(const float* w, const float* b, const float* c, int K, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_coef, dim3(1), dim3(kThreads), 0, s, w, b, c, K, out);
    return hipGetLastError();
}

hipError_t launch_copy_pad(const float* src, float* dst, int n, int ld, int np, int to_pad, hipStream_t s) {
    const size_t total = to_pad ? (size_t)np * np : (size_t)n * n;
    hipLaunchKernelGGL(k_copy_pad, dim3(grid_for(total)), dim3(kThreads), 0, s, src, dst, n, ld, np, to_pad);
    return hipGetLastError();
}

int adjoint_grid(int tile, int np, int* T, int* ntiles, int* per) {
    *T = np / tile;
    *ntiles = ntiles_upper(*T);
    *per = (*ntiles + 7) / 8;
    return 8 * *per;
}

hipError_t launch_adjoint(int tile, const AdjointArgs& a, hipStream_t s) {
    const int grid = 8 * a.per;
    if (tile == 128)
        hipLaunchKernelGGL((k_adjoint<128, 2, 2>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint<64, 2, 2>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce3(const double* parts, int nparts, float* dw, float* db, float* dc, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce3, dim3(1), dim3(kThreads), 0, s, parts, nparts, dw, db, dc, k);
    return hipGetLastError();
}

}  // namespace sp2
