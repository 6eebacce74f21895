// FP64 squaring layer Y = alpha X^2 + beta X + gamma I on v_mfma_f64_16x16x4f64 (gfx950),
// for the refinement layer (Eq. Refinement, computed in double precision) and the FP64
// mode.  Upper-triangle 128 x 128 output tiles, one workgroup per tile of 4 waves (2 x 2
// waves of 64 x 64, 4 x 4 blocks of 16 x 16 each) or 8 waves (2 x 4 waves of 64 x 32),
// mirrored on store.
//
//  * K-stages of 16 doubles: each row of a stage is one 128-byte line.  The two row
//    panels (I and J: X is symmetric, so both operands are K-contiguous rows) go straight
//    from global memory into LDS with global_load_lds_dwordx4 (16 bytes per lane, a
//    wavefront instruction fills a 1 KB block of 8 rows), ST stages deep, issued from
//    inline asm with explicit s_waitcnt accounting (the compiler would otherwise wait for
//    every load before each LDS read).
//  * Rows are XOR-swizzled in 16-byte chunks (chunk c of row r at c ^ ((r >> 1) & 7)), so
//    the 16 lanes of each ds_read_b128 pass hit distinct bank groups.
//  * The K order inside a stage is permuted per lane: MFMA s (0, 1) of unit h (0, 1) takes,
//    in its K lane j = lane / 16, the K index 8 h + 2 j + s.  A and B use the same map, so
//    every product term appears once; one 16-byte read then feeds two MFMAs.
#include "sp2_internal.h"

namespace sp2 {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kBT = 128;           // output tile edge
constexpr int kBK = 16;            // doubles per row per stage
constexpr int kRow = kBK * 8;      // 128 bytes
constexpr int kArr = kBT * kRow;   // bytes of one panel stage
constexpr int kStage = 2 * kArr;   // panels I and J
constexpr int kRPB = 1024 / kRow;  // rows per 1 KB direct-load block (8)
constexpr int kBPR = kBT / kRPB;   // blocks per panel stage (16)
constexpr int kMB = 4;                 // 16 x 16 blocks per wave along rows (64 rows)

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

#define SP2_VMCNT(n) asm volatile("s_waitcnt vmcnt(" #n ")" ::: "memory")
// waits until at most n (rounded down to an available immediate) vector-memory
// instructions of this wave are outstanding
__device__ __forceinline__ void wait_vm(int n) {
    if (n >= 24) SP2_VMCNT(24);
    else if (n >= 16) SP2_VMCNT(16);
    else if (n >= 8) SP2_VMCNT(8);
    else SP2_VMCNT(0);
}
#undef SP2_VMCNT

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// WN waves across the tile's columns (2: 4 waves of 64 x 64, 4: 8 waves of 64 x 32)
// One work item: tile t over K-stages [kb, ke).  chunk < 0: the whole tile, epilogue here;
// otherwise one K-chunk of tail tile `tail_tile`: the FP64 partial goes to slot v of
// sk.partial and the last arriving chunk sums the chunks in order and runs the epilogue.
template <int ST, int WN>
__device__ __forceinline__ void f64_body(const SquareArgs& a, int t, int kb, int ke, int chunk, int tail_tile,
                                         int v, const StreamK& sk, unsigned char* __restrict__ lds,
                                         double* __restrict__ red, int* __restrict__ s_flag) {
    static_assert(ST >= 2 && ST <= 4, "stages");
    constexpr int kNW = 2 * WN;
    constexpr int kLPW = 2 * kBPR / kNW;   // direct loads per wave per stage
    constexpr int kNB = kBT / (16 * WN);   // 16 x 16 blocks per wave along columns
    constexpr int WTN = kBT / WN;
    int I, J;
    tile_of(t, a.T, 8, &I, &J);
    const int np = a.np;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const double* x = (const double*)a.x0;
    const double* src[2] = {x + (size_t)I * kBT * np, x + (size_t)J * kBT * np};
    const int nsl = ke - kb;

    // direct load: lane L fills bytes [16 L, 16 L + 16) of block q: panel row q * 8 + L / 8,
    // physical chunk L % 8 = logical chunk (L % 8) ^ swz8(row)
    auto issue = [&](int buf, int ks) {
#pragma unroll
        for (int i = 0; i < kLPW; ++i) {
            const int j = wave * kLPW + i;
            const int arr = j / kBPR, qd = j % kBPR;
            const int row = qd * kRPB + (lane >> 3);
            const double* g = src[arr] + (size_t)row * np + ks * kBK + (((lane & 7) ^ swz8(row)) << 1);
            dma16(g, __builtin_amdgcn_readfirstlane(lds_addr(lds + buf * kStage + arr * kArr + qd * 1024)));
        }
    };
    // fragments of unit h (K 8h .. 8h+7) of the stage in buffer buf: lane reads the 16-byte
    // logical chunk 4h + lane / 16 of row (block base + lane % 16)
    auto frags = [&](int buf, int h, f64x2 (&fa)[kMB], f64x2 (&fb)[kNB]) {
        const int r16 = lane & 15;
        const unsigned char* base = lds + buf * kStage;
#pragma unroll
        for (int m = 0; m < kMB; ++m) {
            const int row = wm * 64 + m * 16 + r16;
            fa[m] = *(const f64x2*)(base + row * kRow + ((((h << 2) + (lane >> 4)) ^ swz8(row)) << 4));
        }
#pragma unroll
        for (int n = 0; n < kNB; ++n) {
            const int row = wn * WTN + n * 16 + r16;
            fb[n] = *(const f64x2*)(base + kArr + row * kRow + ((((h << 2) + (lane >> 4)) ^ swz8(row)) << 4));
        }
    };

    f64x4 acc[kMB][kNB];
#pragma unroll
    for (int m = 0; m < kMB; ++m)
#pragma unroll
        for (int n = 0; n < kNB; ++n) acc[m][n] = f64x4{0.0, 0.0, 0.0, 0.0};
    auto mma = [&](const f64x2 (&fa)[kMB], const f64x2 (&fb)[kNB]) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int m = 0; m < kMB; ++m)
#pragma unroll
                for (int n = 0; n < kNB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[m][s], fb[n][s], acc[m][n], 0, 0, 0);
    };

    // stage q is issued by advance(q - ST + 1); the prologue plays those of 0 .. ST - 1
    const int pro = nsl < ST ? nsl : ST;
    for (int q = 0; q < pro; ++q) issue(q, kb + q);
    wait_vm((pro - 1) * kLPW);
    __syncthreads();
    f64x2 pa[kMB], pb[kNB], qa[kMB], qb[kNB];
    frags(0, 0, pa, pb);
    // stage `next` readable: its loads landed (this wave's), every wave past the barrier
    auto arrive = [&](int next) {
        const int last = (next + ST - 2 < nsl - 1) ? next + ST - 2 : nsl - 1;
        wait_vm((last - next) * kLPW);
        __syncthreads();
    };
    // the MFMAs of one unit with the direct loads of stage ks (into buffer buf) spread
    // between them, so that their address arithmetic and issue overlap the matrix cores;
    // scheduling barriers keep the compiler from regrouping them
    auto mma_issue = [&](const f64x2 (&fa)[kMB], const f64x2 (&fb)[kNB], int buf, int ks, bool doit) {
        constexpr int NM = 2 * kMB * kNB;
        constexpr int EVERY = NM / kLPW;
        static_assert(EVERY >= 1 && NM % kLPW == 0, "interleave");
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            const int s = i / (kMB * kNB), m = (i / kNB) % kMB, n = i % kNB;
            acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[m][s], fb[n][s], acc[m][n], 0, 0, 0);
            if (i % EVERY == EVERY - 1) {
                __builtin_amdgcn_sched_barrier(0);
                if (doit) {
                    const int j = wave * kLPW + i / EVERY;
                    const int arr = j / kBPR, qd = j % kBPR;
                    const int row = qd * kRPB + (lane >> 3);
                    const double* g = src[arr] + (size_t)row * np + ks * kBK + (((lane & 7) ^ swz8(row)) << 1);
                    dma16(g, __builtin_amdgcn_readfirstlane(lds_addr(lds + buf * kStage + arr * kArr + qd * 1024)));
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    // units: two per stage (h = 0, 1); P holds h = 0 of a stage, Q h = 1.  Stage st + ST
    // refills the buffer of stage st once every wave has read it (after arrive(st + 1)).
    int st = 0;
    for (; st + 1 < nsl; ++st) {
        frags(st % ST, 1, qa, qb);
        mma(pa, pb);
        arrive(st + 1);
        frags((st + 1) % ST, 0, pa, pb);
        mma_issue(qa, qb, st % ST, kb + st + ST, st + ST < nsl);
    }
    frags(st % ST, 1, qa, qb);
    mma(pa, pb);
    mma(qa, qb);

    // ------------------------------------------------------------------- split tail
    if (chunk >= 0) {
        constexpr size_t TILE_D = (size_t)kBT * kBT;
        f64x4* wp = (f64x4*)(sk.fpartial + (size_t)v * TILE_D) + (size_t)wave * kMB * kNB * 64 + lane;
#pragma unroll
        for (int m = 0; m < kMB; ++m)
#pragma unroll
            for (int n = 0; n < kNB; ++n) {
                typedef double f64x2 __attribute__((ext_vector_type(2)));
                const f64x2 lo = {acc[m][n][0], acc[m][n][1]}, hi = {acc[m][n][2], acc[m][n][3]};
                st16_agent(wp, __builtin_bit_cast(u32x4_t, lo));
                st16_agent((char*)wp + 16, __builtin_bit_cast(u32x4_t, hi));
                wp += 64;
            }
        wait_stores();   // this partial is coherent before the arrival is counted
        __syncthreads();
        if (tid == 0) *s_flag = atomicAdd(sk.counter + tail_tile, 1);
        __syncthreads();
        // each executed layer adds `chunks` arrivals per tail tile: the last one reduces
        if (((*s_flag + 1) % sk.chunks) != 0) return;
        const f64x4* rp = (const f64x4*)(sk.fpartial + (size_t)tail_tile * sk.chunks * TILE_D) +
                          (size_t)wave * kMB * kNB * 64 + lane;
        const size_t cstride = TILE_D / 4;
        auto ld = [](const f64x4* q) -> f64x4 {
            typedef double f64x2 __attribute__((ext_vector_type(2)));
            const f64x2 lo = __builtin_bit_cast(f64x2, ld16_agent(q));
            const f64x2 hi = __builtin_bit_cast(f64x2, ld16_agent((const char*)q + 16));
            return f64x4{lo[0], lo[1], hi[0], hi[1]};
        };
#pragma unroll
        for (int m = 0; m < kMB; ++m)
#pragma unroll
            for (int n = 0; n < kNB; ++n) {
                f64x4 sum = ld(rp);
                for (int c = 1; c < sk.chunks; ++c) sum += ld(rp + c * cstride);
                acc[m][n] = sum;
                rp += 64;
            }
    }

    // ------------------------------------------------------------------- epilogue
    const double alpha = a.coef64 ? a.coef64[0] : (double)a.coef[0];
    const double beta = a.coef64 ? a.coef64[1] : (double)a.coef[1];
    const double gamma = a.coef64 ? a.coef64[2] : (double)a.coef[2];
    double* so = (double*)a.s_out;
    const double* si = (const double*)a.s_in;
    const int ldo = a.ld_out, nv = a.n_valid;
    const bool diag = (I == J);
    double tr = 0.0, fr = 0.0;
#pragma unroll
    for (int m = 0; m < kMB; ++m) {
#pragma unroll
        for (int n = 0; n < kNB; ++n) {
            const int col = J * kBT + wn * WTN + n * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = I * kBT + wm * 64 + m * 16 + 4 * r + (lane >> 4);
                if (diag && row > col) continue;
                const double xv = acc[m][n][r];
                double y = (beta != 0.0) ? alpha * xv + beta * si[(size_t)col * np + row] : alpha * xv;
                if (row == col && col < a.n_real) y += gamma;
                if (row < nv && col < nv) {
                    so[(size_t)row * ldo + col] = y;
                    if (row != col) so[(size_t)col * ldo + row] = y;
                }
                if (row == col) {
                    tr += y;
                    fr += y * y;
                } else {
                    fr += 2.0 * y * y;
                }
            }
        }
    }
    if (a.parts) {
        tr = wsum(tr);
        fr = wsum(fr);
        if (lane == 0) {
            red[2 * wave] = tr;
            red[2 * wave + 1] = fr;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < kNW; ++w) {
                s0 += red[2 * w];
                s1 += red[2 * w + 1];
            }
            a.parts[2 * t] = s0;
            a.parts[2 * t + 1] = s1;
        }
    }
}

template <int ST, int WN>
__global__ __launch_bounds__(128 * WN) void k_square_f64(SquareArgs a) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[ST * kStage];
    __shared__ double red[4 * WN];
    __shared__ int s_flag;
    if (a.skip && *a.skip) return;
    const int t = xcd_tile_index(blockIdx.x, a.per, a.ntiles);
    if (t < 0) return;
    StreamK none;
    none.grid = 0;
    none.rounds = 0;
    none.tail_tiles = 0;
    none.chunks = 1;
    none.partial = nullptr;
    none.counter = nullptr;
    none.fpartial = nullptr;
    f64_body<ST, WN>(a, t, 0, a.np / kBK, -1, 0, 0, none, lds, red, &s_flag);
}

// Persistent: sk.grid workgroups run whole rounds of tiles, then the leftover tiles cut into
// sk.chunks K-chunks each (the same schedule as the persistent split squaring).
template <int ST, int WN>
__global__ __launch_bounds__(128 * WN) void k_square_f64_sk(SquareArgs a, StreamK sk) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[ST * kStage];
    __shared__ double red[4 * WN];
    __shared__ int s_flag;
    if (a.skip && *a.skip) return;
    const int G = sk.grid;
    const int v = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);   // XCD-aware order
    const int nsl_all = a.np / kBK;
    const int items = sk.rounds + ((sk.tail_tiles > 0 && v < sk.tail_tiles * sk.chunks) ? 1 : 0);
    for (int item = 0; item < items; ++item) {
        if (item < sk.rounds) {
            f64_body<ST, WN>(a, item * G + v, 0, nsl_all, -1, 0, v, sk, lds, red, &s_flag);
        } else {
            const int tail_tile = v / sk.chunks, chunk = v % sk.chunks;
            const int kb = (int)(((long long)chunk * nsl_all) / sk.chunks);
            const int ke = (int)(((long long)(chunk + 1) * nsl_all) / sk.chunks);
            f64_body<ST, WN>(a, sk.rounds * G + tail_tile, kb, ke, chunk, tail_tile, v, sk, lds, red, &s_flag);
        }
        __syncthreads();   // LDS is reused by the next item
    }
}

// grouped: block b computes the tile that the tile map names for it (see kTileMapShift)
template <int ST, int WN>
__global__ __launch_bounds__(128 * WN) void k_square_f64_g(const SquareArgs* __restrict__ descs,
                                                          const int* __restrict__ map, int per) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[ST * kStage];
    __shared__ double red[4 * WN];
    const int e = map[(blockIdx.x & 7) * per + (blockIdx.x >> 3)];
    if (e < 0) return;
    const SquareArgs a = descs[e >> kTileMapShift];
    if (a.skip && *a.skip) return;
    __shared__ int s_flag;
    StreamK none;
    none.grid = 0;
    none.rounds = 0;
    none.tail_tiles = 0;
    none.chunks = 1;
    none.partial = nullptr;
    none.counter = nullptr;
    none.fpartial = nullptr;
    f64_body<ST, WN>(a, e & kTileMapMask, 0, a.np / kBK, -1, 0, 0, none, lds, red, &s_flag);
}

}  // namespace

// grouped FP64 layer on 128 tiles (8 waves, 4 stages) over a tile map
hipError_t launch_square_f64_g(const SquareArgs* descs, const int* map, int per, hipStream_t s) {
    hipLaunchKernelGGL((k_square_f64_g<4, 4>), dim3(8 * per), dim3(512), 0, s, descs, map, per);
    return hipGetLastError();
}

// Persistent FP64 schedule on 128 tiles: G = CUs (one 8-wave workgroup per CU), whole rounds,
// then the leftover tiles in G / rem K-chunks (at most one per K-stage).  False when there
// are fewer tiles than workgroups.
bool square_f64_sk_plan(int np, int cus, StreamK* sk) {
    const int nt = ntiles_upper(np / kBT);
    int g = cus;
    if (g > kMaxSkGrid) g = kMaxSkGrid;
    g -= g % 8;
    if (g < 8 || nt < g) return false;
    const int nsl = np / kBK;
    sk->grid = g;
    sk->rounds = nt / g;
    sk->tail_tiles = nt % g;
    sk->chunks = sk->tail_tiles ? g / sk->tail_tiles : 1;
    if (sk->chunks > nsl) sk->chunks = nsl;
    return true;
}

size_t square_f64_sk_partial_bytes() { return (size_t)kMaxSkGrid * kBT * kBT * sizeof(double); }

hipError_t launch_square_f64_sk(const SquareArgs& a, const StreamK& sk, hipStream_t s) {
    hipLaunchKernelGGL((k_square_f64_sk<4, 4>), dim3(sk.grid), dim3(512), 0, s, a, sk);
    return hipGetLastError();
}

// FP64 layer on 128 tiles (n_p a multiple of 128).  variant 0: 4 waves, 2 LDS stages;
// 1: 4 waves, 4 stages (128 KB); 2: 8 waves, 4 stages.
hipError_t launch_square_f64(int variant, const SquareArgs& a, hipStream_t s) {
    if (a.np % kBT) return hipErrorInvalidValue;
    const int grid = 8 * a.per;
    if (variant == 0) hipLaunchKernelGGL((k_square_f64<2, 2>), dim3(grid), dim3(256), 0, s, a);
    else if (variant == 1) hipLaunchKernelGGL((k_square_f64<4, 2>), dim3(grid), dim3(256), 0, s, a);
    else if (variant == 2) hipLaunchKernelGGL((k_square_f64<4, 4>), dim3(grid), dim3(512), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace sp2
