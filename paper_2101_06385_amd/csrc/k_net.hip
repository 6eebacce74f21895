// Kernels of the differentiable generalized-SP2 network (Eq. general SP2 as matrix layers)
//
//     X_{k+1} = W_k X_k^2 + B_k X_k + c_k I,   k = 0 .. K-1
//
// The forward layers reuse the squaring kernels (alpha, beta, gamma) = (W_k, B_k, c_k).
// This file holds what the network adds:
//   k_pack_coef   : (W, B, c) device arrays -> per-layer coefficient triples
//   k_copy_pad    : n x n (leading dimension ld) <-> zero-padded n_p x n_p
//   k_adjoint_dl  : one reverse layer.  With G = dL/dX_{k+1} (symmetric),
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

// dst (np x np, zero padding) <- (src + src^T)/2 for the n x n matrix src (leading dimension
// ld): the part of a loss gradient that acts on a symmetric layer output.  One 32 x 32 output
// tile per block; the mirrored input tile goes through LDS so that both reads are row
// segments.  a + b == b + a in IEEE arithmetic, so the result is exactly symmetric.
constexpr int kSymT = 32;
__global__ __launch_bounds__(kThreads) void k_sym_pad(const float* __restrict__ src, float* __restrict__ dst,
                                                      int n, int ld, int np) {
    __shared__ float tr[kSymT][kSymT + 1];
    const int bi = blockIdx.y * kSymT, bj = blockIdx.x * kSymT;
    const int c = threadIdx.x % kSymT, r0 = threadIdx.x / kSymT;   // 8 rows per pass
    for (int r = r0; r < kSymT; r += kThreads / kSymT) {
        const int i = bj + r, j = bi + c;   // mirrored tile: rows of bj, columns of bi
        tr[r][c] = (i < n && j < n) ? src[(size_t)i * ld + j] : 0.f;
    }
    __syncthreads();
    for (int r = r0; r < kSymT; r += kThreads / kSymT) {
        const int i = bi + r, j = bj + c;
        const float a = (i < n && j < n) ? src[(size_t)i * ld + j] : 0.f;
        dst[(size_t)i * np + j] = 0.5f * (a + tr[c][r]);
    }
}

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// FP32 adjoint layer on output tiles (I <= J) of the symmetric M = G X + X G (rows of a
// symmetric matrix are its columns, so all four operands are K-contiguous row panels).
// The four row panels (G_I, X_I,
// X_J, G_J) go from global memory into LDS with global_load_lds_dwordx4 in K-stages of 32
// floats (one 128-byte line per row; 1 KB blocks of 8 rows, 16-byte chunks XOR-swizzled by
// (row >> 1) & 7), two stages deep, issued from inline asm with explicit vmcnt accounting
// and spread among the MFMAs.  Each lane permutes its K order inside a unit of 8: MFMA s
// (0..3) takes, in its K lane j = lane / 32, the index 8 h + 4 j + s, for A and B alike, so
// one 16-byte LDS read feeds four v_mfma_f32_32x32x2f32.  4 waves of BT/2 x BT/2.
namespace dl {
constexpr int kBK = 32, kRow = 128, kRPB = 8;

__device__ inline int swz8(int r) { return (r >> 1) & 7; }
typedef __attribute__((address_space(3))) unsigned char lds_byte;
__device__ __forceinline__ unsigned lds_addr(const unsigned char* p) {
    return (unsigned)(uintptr_t)(const lds_byte*)p;
}
__device__ __forceinline__ void dma16(const void* g, unsigned lds_base) {
    asm volatile(
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %0, off"
        :
        : "v"(g), "s"(lds_base)
        : "memory", "m0");
}
// rounds n down to an available immediate (waiting for more is always safe)
__device__ __forceinline__ void wait_vm(int n) {
    if (n >= 48) asm volatile("s_waitcnt vmcnt(48)" ::: "memory");
    else if (n >= 32) asm volatile("s_waitcnt vmcnt(32)" ::: "memory");
    else if (n >= 24) asm volatile("s_waitcnt vmcnt(24)" ::: "memory");
    else if (n >= 16) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
    else if (n >= 8) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
}  // namespace dl

// BT = 128 (2 x 2 blocks of 32 x 32 per wave) or 64 (one block per wave).  Persistent
// schedule (as for the split squaring): sk.grid workgroups run whole rounds of tiles, then
// the leftover tiles are cut along K into sk.chunks chunks each; every chunk stores its FP32
// partial of M and the last of a tile's arrivals sums them in chunk order (deterministic)
// and runs the epilogue.
template <int BT, int kST>
__global__ __launch_bounds__(256) void k_adjoint_dl(AdjointArgs a, StreamK sk) {
    using namespace dl;
    constexpr int kBT = BT, kArr = kBT * kRow, kStage = 4 * kArr;
    constexpr int kBPR = kBT / kRPB, kLPW = 4 * kBPR / 4;   // direct loads per wave per stage
    constexpr int NB = BT / 64;                             // 32 x 32 blocks per wave and dimension
    constexpr int WT = BT / 2;                              // wave tile edge
    constexpr int NM = 4 * NB * NB * 2;                     // MFMAs per unit
    static_assert(NM % kLPW == 0, "loads spread evenly over the MFMAs");
    typedef float f32x4v __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) unsigned char lds[kST * kStage];
    __shared__ double red[3 * 4];
    __shared__ int s_flag;

    const int np = a.np;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int G = sk.grid;
    const int v = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);   // XCD-aware order
    const int nsl_all = np / kBK;
    const int items = sk.rounds + ((sk.tail_tiles > 0 && v < sk.tail_tiles * sk.chunks) ? 1 : 0);
    for (int item = 0; item < items; ++item) {
        int t, kb, ke, chunk = -1, tail_tile = 0;
        if (item < sk.rounds) {
            t = item * G + v;
            kb = 0;
            ke = nsl_all;
        } else {
            tail_tile = v / sk.chunks;
            chunk = v % sk.chunks;
            t = sk.rounds * G + tail_tile;
            kb = (int)(((long long)chunk * nsl_all) / sk.chunks);
            ke = (int)(((long long)(chunk + 1) * nsl_all) / sk.chunks);
        }
        const int nsl = ke - kb;
        int I, J;
        tile_of(t, a.T, 8, &I, &J);
        // stage arrays: 0 = G panel I, 1 = X panel I, 2 = X panel J, 3 = G panel J
        const float* src[4] = {a.g + (size_t)I * kBT * np, a.x + (size_t)I * kBT * np,
                               a.x + (size_t)J * kBT * np, a.g + (size_t)J * kBT * np};

        auto load_one = [&](int buf, int ks, int l) {
            const int j = wave * kLPW + l;
            const int arr = j / kBPR, qd = j % kBPR;
            const int row = qd * kRPB + (lane >> 3);
            const float* g = src[arr] + (size_t)row * np + ks * kBK + (((lane & 7) ^ swz8(row)) << 2);
            dma16(g, __builtin_amdgcn_readfirstlane(lds_addr(lds + buf * kStage + arr * kArr + qd * 1024)));
        };
        // fragments of unit h (K 8h .. 8h+7) in buffer buf: lane reads the 16-byte logical
        // chunk 2h + lane / 32 of row (block base + lane % 32) of each panel
        auto frags = [&](int buf, int h, f32x4v (&fg)[NB], f32x4v (&fx)[NB], f32x4v (&hx)[NB], f32x4v (&hg)[NB]) {
            const unsigned char* base = lds + buf * kStage;
            const int r32 = lane & 31;
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const int row = wm * WT + m * 32 + r32;
                const int off = row * kRow + ((((h << 1) + (lane >> 5)) ^ swz8(row)) << 4);
                fg[m] = *(const f32x4v*)(base + off);
                fx[m] = *(const f32x4v*)(base + kArr + off);
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int row = wn * WT + n * 32 + r32;
                const int off = row * kRow + ((((h << 1) + (lane >> 5)) ^ swz8(row)) << 4);
                hx[n] = *(const f32x4v*)(base + 2 * kArr + off);
                hg[n] = *(const f32x4v*)(base + 3 * kArr + off);
            }
        };
        // one accumulator per product (G_I X_J^T and X_I G_J^T): two independent MFMA chains
        f32x16 acc[2][NB][NB];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int m = 0; m < NB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[q][m][n][r] = 0.f;
        // the NM MFMAs of one unit, with the kLPW direct loads of stage ks into buffer buf
        // spread evenly among them when doit
        auto mma = [&](const f32x4v (&fg)[NB], const f32x4v (&fx)[NB], const f32x4v (&hx)[NB],
                       const f32x4v (&hg)[NB], int buf, int ks, bool doit) {
            constexpr int EVERY = NM / kLPW;
#pragma unroll
            for (int i = 0; i < NM; ++i) {
                const int s = i / (2 * NB * NB), pr = (i / (NB * NB)) & 1, m = (i / NB) % NB, n = i % NB;
                if (pr == 0)
                    acc[0][m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(fg[m][s], hx[n][s], acc[0][m][n], 0, 0, 0);
                else
                    acc[1][m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[m][s], hg[n][s], acc[1][m][n], 0, 0, 0);
                if (i % EVERY == EVERY - 1) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (doit) load_one(buf, ks, i / EVERY);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        };

        wait_vm(0);   // nothing of the previous item may still count against vmcnt
        const int pro = nsl < kST ? nsl : kST;
        for (int q = 0; q < pro; ++q)
            for (int l = 0; l < kLPW; ++l) load_one(q, kb + q, l);
        wait_vm((pro - 1) * kLPW);
        __syncthreads();
        f32x4v pg[NB], px[NB], phx[NB], phg[NB], qg[NB], qx[NB], qhx[NB], qhg[NB];
        frags(0, 0, pg, px, phx, phg);
        // Stages of 4 units, the units alternating between fragment sets P and Q.  After the
        // third unit of stage st: wait for stage st + 1 (later stages may stay in flight) and
        // the barrier (every wave has read stage st), then stage st + kST refills stage st's
        // buffer among the MFMAs of its fourth unit.
        for (int st = 0; st < nsl; ++st) {
            const int buf = st % kST;
            frags(buf, 1, qg, qx, qhx, qhg);
            mma(pg, px, phx, phg, 0, 0, false);
            frags(buf, 2, pg, px, phx, phg);
            mma(qg, qx, qhx, qhg, 0, 0, false);
            frags(buf, 3, qg, qx, qhx, qhg);
            mma(pg, px, phx, phg, 0, 0, false);
            if (st + 1 < nsl) {
                // stages issued so far: up to st + kST - 1; wait for st + 1 only
                const int last = (st + kST - 1 < nsl - 1) ? st + kST - 1 : nsl - 1;
                wait_vm((last - st - 1) * kLPW);
                __syncthreads();
                frags((st + 1) % kST, 0, pg, px, phx, phg);
                mma(qg, qx, qhx, qhg, buf, kb + st + kST, st + kST < nsl);
            } else {
                mma(qg, qx, qhx, qhg, 0, 0, false);
            }
        }
        __syncthreads();   // every fragment read done before the stages are reused
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[0][m][n] += acc[1][m][n];

        // ---------------------------------------------------------------- split tail
        bool finish = chunk < 0;
        if (!finish) {
            constexpr size_t TILE_F = (size_t)BT * BT;
            f32x4v* wp = (f32x4v*)(sk.partial + (size_t)v * TILE_F) + (size_t)wave * NB * NB * 4 * 64 + lane;
#pragma unroll
            for (int m = 0; m < NB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        f32x4v vv = {acc[0][m][n][4 * q], acc[0][m][n][4 * q + 1], acc[0][m][n][4 * q + 2],
                                     acc[0][m][n][4 * q + 3]};
                        st16_agent(wp, __builtin_bit_cast(u32x4_t, vv));
                        wp += 64;
                    }
            wait_stores();   // this partial is coherent before the arrival is counted
            __syncthreads();
            if (tid == 0) s_flag = atomicAdd(sk.counter + tail_tile, 1);
            __syncthreads();
            // each layer adds `chunks` arrivals per tail tile: the last one reduces
            finish = ((s_flag + 1) % sk.chunks) == 0;
            if (finish) {
                const f32x4v* rp = (const f32x4v*)(sk.partial + (size_t)tail_tile * sk.chunks * TILE_F) +
                                   (size_t)wave * NB * NB * 4 * 64 + lane;
                const size_t cstride = TILE_F / 4;
#pragma unroll
                for (int m = 0; m < NB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            f32x4v sum = __builtin_bit_cast(f32x4v, ld16_agent(rp));
                            for (int c = 1; c < sk.chunks; ++c)
                                sum += __builtin_bit_cast(f32x4v, ld16_agent(rp + c * cstride));
#pragma unroll
                            for (int e = 0; e < 4; ++e) acc[0][m][n][4 * q + e] = sum[e];
                            rp += 64;
                        }
            }
        }

        // ---------------------------------------------------------------- epilogue
        if (finish) {
            // G_k = W M + B G over row <= col, mirrored; FP64 partials
            const float wk = a.coef[0], bk = a.coef[1];
            const bool diag = (I == J);
            double p_tr = 0.0, p_gx = 0.0, p_mx = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) {
#pragma unroll
                for (int n = 0; n < NB; ++n) {
                    const int col = J * kBT + wn * WT + n * 32 + (lane & 31);
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = I * kBT + wm * WT + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        if (diag && row > col) continue;
                        const size_t off = (size_t)row * np + col;
                        const float mv = acc[0][m][n][r];
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
                for (int w = 0; w < 4; ++w) {
                    s0 += red[3 * w];
                    s1 += red[3 * w + 1];
                    s2 += red[3 * w + 2];
                }
                a.parts[3 * t + 0] = s0;
                a.parts[3 * t + 1] = s1;
                a.parts[3 * t + 2] = s2;
            }
        }
        __syncthreads();   // LDS and red are reused by the next item
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

hipError_t launch_sym_pad(const float* src, float* dst, int n, int ld, int np, hipStream_t s) {
    if (np % kSymT) return hipErrorInvalidValue;
    const dim3 grid(np / kSymT, np / kSymT);
    hipLaunchKernelGGL(k_sym_pad, grid, dim3(kThreads), 0, s, src, dst, n, ld, np);
    return hipGetLastError();
}

int adjoint_grid(int tile, int np, int* T, int* ntiles, int* per) {
    *T = np / tile;
    *ntiles = ntiles_upper(*T);
    *per = (*ntiles + 7) / 8;
    return 8 * *per;
}

// Adjoint variants: 0 = 64 tiles, 2 LDS stages (64 KB, two workgroups per CU); 1 = 64
// tiles, 4 stages (128 KB, one per CU); 2 = 128 tiles, 2 stages (128 KB, one per CU).
// Persistent schedule: G = CUs x workgroups per CU, whole rounds, then the leftover tiles in
// G / rem K-chunks (at most one chunk per K-stage; with fewer tiles than workgroups every
// tile is split).
int adjoint_tile(int variant) { return variant == 2 ? 128 : 64; }

void adjoint_plan(int variant, int np, int cus, StreamK* sk) {
    const int tile = adjoint_tile(variant);
    const int nt = ntiles_upper(np / tile);
    int g = cus * (variant == 0 ? 2 : 1);
    if (g > kMaxSkGrid) g = kMaxSkGrid;
    g -= g % 8;
    if (g < 8) g = 8;
    const int nsl = np / 32;
    sk->grid = g;
    sk->rounds = nt / g;
    sk->tail_tiles = nt % g;
    sk->chunks = sk->tail_tiles ? g / sk->tail_tiles : 1;
    if (sk->chunks > nsl) sk->chunks = nsl;
    if (sk->chunks < 1) sk->chunks = 1;
}

size_t adjoint_partial_bytes(int variant) {
    const int tile = adjoint_tile(variant);
    return (size_t)kMaxSkGrid * tile * tile * sizeof(float);
}

hipError_t launch_adjoint(int variant, const AdjointArgs& a, const StreamK& sk, hipStream_t s) {
    if (variant == 2)
        hipLaunchKernelGGL((k_adjoint_dl<128, 2>), dim3(sk.grid), dim3(256), 0, s, a, sk);
    else if (variant == 1)
        hipLaunchKernelGGL((k_adjoint_dl<64, 4>), dim3(sk.grid), dim3(256), 0, s, a, sk);
    else
        hipLaunchKernelGGL((k_adjoint_dl<64, 2>), dim3(sk.grid), dim3(256), 0, s, a, sk);
    return hipGetLastError();
}

hipError_t launch_reduce3(const double* parts, int nparts, float* dw, float* db, float* dc, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce3, dim3(1), dim3(kThreads), 0, s, parts, nparts, dw, db, dc, k);
    return hipGetLastError();
}

}  // namespace sp2
