// Split (dual half-precision) squaring layer, persistent version (gfx950): kernel
// template and its per-variant launcher, instantiated once per half type by
// k_sk_f16.hip and k_sk_bf16.hip.
//
// Computes the same layer as k_square_split (Y = alpha X^2 + beta X + gamma I from the
// planes X0, X1 with the product X0 X0 + X0 X1 + X1 X0 of Eq. Square, over the
// upper-triangle tiles, mirrored) with G persistent workgroups:
//
//  * Whole rounds: tiles [0, R G) go round by round, workgroup v taking tile r G + v in
//    round r.  Every round starts at K = 0 on every CU, and the workgroups of one XCD
//    hold consecutive tiles of the strip order, so they stream the same panel slices at
//    the same time and share them in that XCD's L2.
//  * Split tail: the rem = ntiles - R G tiles left over are each cut into s = G / rem
//    K-chunks, one per workgroup, so the last round takes 1/s of a round instead of a
//    full one (528 tiles of 256^2 on 256 CUs: 2 rounds + 1/16 instead of 3).  Each chunk
//    stores its FP32 partial; the last of the s arrivals sums the s partials in chunk
//    order and runs the epilogue, so results are bit-reproducible.
//  * Staging: K-slices of the row panels go straight from global memory into LDS
//    (global_load_lds_dwordx4: each lane moves 16 bytes, one wavefront instruction fills
//    a 1 KB block of swizzled rows) through ST LDS stages, the loads running ST - 1
//    slices ahead of the matrix cores; no VGPRs hold staged data.
//  * Fragments are double buffered in registers: while the matrix cores work on one
//    16-wide K unit, the LDS reads of the next unit are in flight.
#pragma once

#include "sp2_internal.h"

#include <type_traits>

namespace sp2 {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T16>
struct H2;
template <>
struct H2<_Float16> {
    typedef f16x8 vec8;
    typedef f16x4 vec4;
    __device__ static inline f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct H2<__bf16> {
    typedef bf16x8 vec8;
    typedef bf16x4 vec4;
    __device__ static inline f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// LDS rows of a K-slice hold SK halves (2 SK bytes = CPR 16-byte chunks).  Row r stores
// logical chunk c at physical chunk c ^ swz(r).  gfx950 serves a ds_read_b128 16 lanes
// at a time from 64 banks (256 bytes); the 16 consecutive rows a lane group reads at one
// logical chunk then fall on 16 distinct groups of four banks:
//   CPR = 2: swz = (r >> 3) & 1,  CPR = 4: (r >> 2) & 3,  CPR = 8: (r >> 1) & 7.
template <int CPR>
__device__ inline int swz(int r) {
    return (r / (16 / CPR)) & (CPR - 1);
}

// Compile-time loop: f(integral_constant<int, i>) for i in [B, E).  Keeps every index
// into the accumulator array a constant, so the accumulators stay in registers.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// s_waitcnt needs an immediate: wait until at most n vector-memory instructions of this
// wavefront are outstanding, for the counts the pipeline below can ask for.
#define SP2_VMCNT(n) asm volatile("s_waitcnt vmcnt(" #n ")" ::: "memory")
// Rounds n down to an immediate it has (waiting for more than asked is always safe).
__device__ __forceinline__ void wait_vm(int n) {
    if (n >= 48) SP2_VMCNT(48);
    else if (n >= 40) SP2_VMCNT(40);
    else if (n >= 32) SP2_VMCNT(32);
    else if (n >= 28) SP2_VMCNT(28);
    else if (n >= 24) SP2_VMCNT(24);
    else if (n >= 20) SP2_VMCNT(20);
    else if (n >= 18) SP2_VMCNT(18);
    else if (n >= 16) SP2_VMCNT(16);
    else if (n >= 14) SP2_VMCNT(14);
    else if (n >= 12) SP2_VMCNT(12);
    else if (n >= 10) SP2_VMCNT(10);
    else if (n >= 8) SP2_VMCNT(8);
    else if (n >= 6) SP2_VMCNT(6);
    else if (n >= 4) SP2_VMCNT(4);
    else if (n >= 2) SP2_VMCNT(2);
    else SP2_VMCNT(0);
}
#undef SP2_VMCNT

// One 16-byte-per-lane direct load from global memory into LDS (global_load_lds_dwordx4:
// M0 holds the wave-uniform LDS base, lane L's 16 bytes land at base + 16 L).  Issued from
// inline asm so that the compiler does not treat it as an LDS store it must wait for
// before every later LDS read: completion is tracked explicitly with wait_vm() and a
// barrier before a slice is read.
typedef __attribute__((address_space(3))) unsigned char lds_byte;
__device__ __forceinline__ unsigned lds_addr(const unsigned char* p) {
    return (unsigned)(uintptr_t)(const lds_byte*)p;
}
// The same with a wave-uniform base address in SGPRs and a 32-bit per-lane byte offset:
// half the address data of the 64-bit form, and no per-load vector address arithmetic.
__device__ __forceinline__ void dma16s(unsigned voff, const void* sbase, unsigned lds_base) {
    asm volatile(
        "s_mov_b32 m0, %2\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %0, %1"
        :
        : "v"(voff), "s"(sbase), "s"(lds_base)
        : "memory", "m0");
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

// agent-coherent 16-byte store / load of FP32 partials (see st16_agent)
__device__ __forceinline__ void store_agent(f32x4* p, f32x4 v) { st16_agent(p, __builtin_bit_cast(u32x4_t, v)); }
__device__ __forceinline__ f32x4 load_agent(const f32x4* p) { return __builtin_bit_cast(f32x4, ld16_agent(p)); }

template <typename T16, int WM, int WN, int MB, int NB, int SK, int ST, int RP>
struct Cfg {
    static constexpr int NW = WM * WN;
    static constexpr int NT = 64 * NW;
    static constexpr int WTM = MB * 32, WTN = NB * 32;
    static constexpr int BT = WM * WTM;
    static_assert(BT == WN * WTN, "square tiles only");
    static_assert(SK == 16 || SK == 32 || SK == 64, "slice width");
    static constexpr int ROW = SK * 2;             // bytes per LDS row of a slice
    static constexpr int CPR = ROW / 16;           // 16-byte chunks per row
    static constexpr int RPB = 1024 / ROW;         // rows per 1 KB block (one wave-wide direct load)
    static constexpr int UPS = SK / 16;            // MFMA K steps (units) per slice
    static constexpr int ARR = BT * ROW;           // bytes of one panel slice in LDS
    static constexpr int STAGE = 4 * ARR;          // A0, A1, B0, B1
    static constexpr int LDS = ST * STAGE;
    static constexpr int BPR = BT / RPB;           // 1 KB blocks per panel slice
    static constexpr int LPW = 4 * BPR / NW;       // direct-load instructions per wave per slice
    static_assert((4 * BPR) % NW == 0, "slice blocks must split evenly over waves");
    static constexpr int LDS_ALL = LDS;
    static_assert(LDS_ALL <= 160 * 1024, "LDS budget");
    static_assert(LPW * (ST - 1) <= 48, "vmcnt range of wait_vm");
};

// The work of one workgroup.  ONE_TILE: exactly tile t0 over all of K (one workgroup per
// tile, used by the grouped launch that covers many problems); otherwise the persistent
// schedule of workgroup v: whole rounds, then at most one split-K tail chunk.
// (The LDS arrays are declared here, not passed in: a generic pointer to them cast back to
// an LDS address made the compiler emit an illegal instruction.)
template <typename T16, int WM, int WN, int MB, int NB, int SK, int ST, int RP, bool ONE_TILE>
__device__ __forceinline__ void sk_body(const SquareArgs& a, const StreamK& sk, int v, int t0) {
    typedef Cfg<T16, WM, WN, MB, NB, SK, ST, RP> C;
    __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS_ALL];
    __shared__ int s_flag;
    __shared__ int s_ticket;
    __shared__ int s_slot[kSkMaxContrib];
    typedef typename H2<T16>::vec8 vec8;
    typedef typename H2<T16>::vec4 vec4;
    constexpr int BT = C::BT;
    constexpr int LPW = C::LPW;
    constexpr int ROW = C::ROW;
    constexpr int UPS = C::UPS;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);   // the same, known to be wave-uniform
    const int wm = wave / WN, wn = wave % WN;
    const int np = a.np;
    const int KS = np / SK;    // K-slices per tile
    const int G = sk.grid;

    // lane L of a direct load fills LDS bytes [16 L, 16 L + 16) of 1 KB block q: panel
    // row q RPB + L / CPR, physical chunk L % CPR, i.e. logical chunk
    // (L % CPR) ^ swz(q RPB + L / CPR)
    const int lrow = lane / C::CPR;
    const int lpc = lane % C::CPR;
    // fragment reads: row base + lane % 32; unit u of a slice is logical chunks 2u, 2u + 1
    // (lanes 0-31 take the lower eight K values of the unit, lanes 32-63 the upper)
    const int rsub = lane & 31;

    const T16* x0 = (const T16*)a.x0;
    const T16* x1 = (const T16*)a.x1;
    const float alpha = a.coef[0], beta = a.coef[1], gamma = a.coef[2];

    // work items: whole rounds, then tail chunks taken from a queue until it is empty; or,
    // in the stream-K form, the tiles that this workgroup's range of units [u0, u1) touches
    const int SQ = ONE_TILE ? 0 : sk.stream_k;
    const int ksq = SQ ? KS / SQ : 1;
    const long long U = (long long)a.ntiles * ksq;
    const int u0 = SQ ? (int)((long long)v * U / G) : 0;
    const int u1 = SQ ? (int)((long long)(v + 1) * U / G) : 0;
    const int first_tile = u0 / ksq;
    int items;
    if (ONE_TILE) items = 1;
    else if (SQ) items = u1 > u0 ? (u1 - 1) / ksq - first_tile + 1 : 0;
    else items = sk.rounds + (sk.tail_tiles > 0 ? G : 0);   // the queue ends the tail items
    // Tail queue: one ticket per tail chunk plus one final (empty) ticket per workgroup, so
    // every executed launch draws exactly total + G tickets from a counter that is cleared
    // once per call; the ticket modulo total + G is the chunk.
    const int total = sk.tail_tiles * sk.chunks;
    for (int item = 0; item < items; ++item) {
        int t, kb, ke, chunk = -1, tail_tile = 0;
        int slot = v;                  // partial tile slot of this work item
        int contrib = sk.chunks;       // partials that make up the tile
        if (ONE_TILE) {
            t = t0;
            kb = 0;
            ke = KS;
        } else if (SQ) {
            t = first_tile + item;
            const int lo = t * ksq, hi = lo + ksq;
            const int a0 = u0 > lo ? u0 : lo, a1 = u1 < hi ? u1 : hi;
            kb = SQ * (a0 - lo);
            ke = SQ * (a1 - lo);
            if (a0 > lo || a1 < hi) {
                chunk = item == 0 ? 0 : 1;
                slot = 2 * v + chunk;
                tail_tile = t;
                // ranges v' with u0(v') < hi and u1(v') > lo (every range is non-empty)
                const int vf = (int)(((long long)(lo + 1) * G + U - 1) / U) - 1;
                const int vl = (int)(((long long)hi * G + U - 1) / U) - 1;
                contrib = vl - vf + 1;
            }
        } else if (item < sk.rounds) {
            t = item * G + v;
            kb = 0;
            ke = KS;
        } else {
            // Workgroups that finish their rounds early take the chunks, in tile-major
            // order; which workgroup computes a chunk does not change any result (the chunk
            // fixes the K range and the partial slot, and the partials are summed in chunk
            // order).
            if (tid == 0) s_ticket = atomicAdd(sk.counter + kSkQueueSlot, 1);
            __syncthreads();
            const int q = s_ticket % (total + G);
            if (q >= total) break;
            tail_tile = q / sk.chunks;
            chunk = q % sk.chunks;
            slot = q;
            t = sk.rounds * G + tail_tile;
            // chunk bounds on groups of Q slices, Q = 2 / UPS: every work item then runs an
            // even number of MFMA units
            constexpr int Q = UPS >= 2 ? 1 : 2;
            kb = Q * (int)(((long long)chunk * (KS / Q)) / sk.chunks);
            ke = Q * (int)(((long long)(chunk + 1) * (KS / Q)) / sk.chunks);
        }
        const int nsl = ke - kb;   // slices of this work item
        int I, J;
        tile_of(t, a.T, 8, &I, &J);
        const size_t pld = (size_t)plane_ld(np);   // plane row stride
        const T16* src[4] = {x0 + (size_t)I * BT * pld, x1 + (size_t)I * BT * pld, x0 + (size_t)J * BT * pld,
                             x1 + (size_t)J * BT * pld};

        // Direct load l of this wave's share of a slice: panel arr, 1 KB block qd; the
        // lane's byte offset in the panel slice does not depend on the slice.
        unsigned voff[LPW];
        static_for<0, LPW>([&](auto l) {
            const int j = wv * LPW + l;
            const int row = (j % C::BPR) * C::RPB + lrow;
            voff[l] = (unsigned)(row * pld * sizeof(T16)) + (unsigned)((lpc ^ swz<C::CPR>(row)) << 4);
        });
        // direct load l (0 <= l < LPW) of this wave's share of slice ks into buffer buf
        auto dma_one = [&](auto l, int buf, int ks) {
            const int j = wv * LPW + l;
            const int arr = j / C::BPR, qd = j % C::BPR;
            const unsigned char* base = (const unsigned char*)src[arr] + (size_t)ks * SK * sizeof(T16);
            dma16s(voff[l], base, lds_addr(lds + buf * C::STAGE + arr * C::ARR + qd * 1024));
        };
        auto issue = [&](int buf, int ks) { static_for<0, LPW>([&](auto l) { dma_one(l, buf, ks); }); };
        // fragments of unit u (0 <= u < UPS) of the slice in buffer buf
        auto frags = [&](int buf, int u, vec8 (&fa0)[MB], vec8 (&fa1)[MB], vec8 (&fb0)[NB], vec8 (&fb1)[NB]) {
            const int fchunk = ((2 * u + (lane >> 5)) ^ swz<C::CPR>(rsub)) << 4;
            const unsigned char* base = lds + buf * C::STAGE + rsub * ROW + fchunk;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int off = (wm * C::WTM + m * 32) * ROW;
                fa0[m] = *(const vec8*)(base + off);
                fa1[m] = *(const vec8*)(base + C::ARR + off);
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int off = (wn * C::WTN + n * 32) * ROW;
                fb0[n] = *(const vec8*)(base + 2 * C::ARR + off);
                fb1[n] = *(const vec8*)(base + 3 * C::ARR + off);
            }
        };

        f32x16 acc[MB][NB];
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.f;

        auto mma = [&](const vec8 (&fa0)[MB], const vec8 (&fa1)[MB], const vec8 (&fb0)[NB], const vec8 (&fb1)[NB]) {
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = H2<T16>::mfma(fa0[m], fb0[n], acc[m][n]);
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = H2<T16>::mfma(fa0[m], fb1[n], acc[m][n]);
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = H2<T16>::mfma(fa1[m], fb0[n], acc[m][n]);
        };

        // ---------------------------------------------------------------- main loop
        // slice kb + j lives in LDS buffer j % ST.  Prologue: the first ST slices in
        // flight and the first one landed.  Slice q >= ST is issued right after the barrier
        // that frees buffer q % ST.  To wait for slice t, a wave allows the direct loads it
        // issued after slice t to stay outstanding (they complete in order).
        wait_vm(0);   // nothing of the previous item may still count against vmcnt
        const int pro = nsl < ST ? nsl : ST;
        for (int q = 0; q < pro; ++q) issue(q, kb + q);
        wait_vm((pro - 1) * LPW);   // the first slice has landed
        __syncthreads();
        if constexpr (RP) {
            // Rolling fragment pipeline.  One set of fragment registers: each register takes
            // the next unit's fragment as soon as the last MFMA that reads it has been issued,
            // so the LDS reads of unit u + 1 overlap the MFMAs of unit u without a second
            // set.  Per unit the products go X0 X1 (B1 column-block major: B1[n] is free
            // after its MB products), X0 X0 (row-block major: A0[m] free after its NB
            // products), X1 X0 (A1[m] free likewise), then B0 is free.  Scheduling barriers
            // pin that order.  At the last unit of a slice the barrier sits after the X0 X1
            // products: the fragments of this slice are all in registers by then (an explicit
            // lgkmcnt(0) waits for the last of them).  The loads that refill its buffer go out
            // in two halves, one spread over the X0 X0 and X1 X0 products right after the
            // barrier, the other over the first unit of the next slice: issued in one burst by
            // every wave at once they queue up in the vector memory path and hold up the
            // waves' next MFMAs.
            static_assert(ST == 2 && UPS >= 2, "rolling pipeline: two LDS stages, two units per slice");
            constexpr int LH = LPW / 2;
            vec8 A0[MB], A1[MB], B0[NB], B1[NB];
            const int ra = wm * C::WTM, rb = wn * C::WTN;
            auto rd = [&](int buf, int u, int arr, int r0) -> vec8 {
                const int fchunk = ((2 * u + (lane >> 5)) ^ swz<C::CPR>(rsub)) << 4;
                return *(const vec8*)(lds + buf * C::STAGE + arr * C::ARR + (r0 + rsub) * ROW + fchunk);
            };
            static_for<0, MB>([&](auto m) {
                A0[m] = rd(0, 0, 0, ra + 32 * m);
                A1[m] = rd(0, 0, 1, ra + 32 * m);
            });
            static_for<0, NB>([&](auto n) {
                B0[n] = rd(0, 0, 2, rb + 32 * n);
                B1[n] = rd(0, 0, 3, rb + 32 * n);
            });
            // One unit on the fragments in registers.  NX: read the fragments of unit nu of
            // the slice in buffer nbuf meanwhile.  SE: that unit starts the next slice, so a
            // barrier comes first.  With dma, the direct loads [LB, LE) of slice dks go to
            // buffer dbuf, spread evenly over the MFMAs that follow the barrier (SE) or over
            // all of the unit's MFMAs.
            auto unit = [&](auto se_, auto nx_, auto lb_, auto le_, int nbuf, int nu, bool dma, int dbuf, int dks) {
                constexpr bool SE = decltype(se_)::value, NX = decltype(nx_)::value;
                constexpr int LB = decltype(lb_)::value, LE = decltype(le_)::value;
                constexpr int G = MB * NB;
                constexpr int NS = SE ? 2 * G : 3 * G;   // MFMA slots that loads may follow
                // the loads that go right after MFMA slot pos
                auto dma_at = [&](auto pos_) {
                    constexpr int pos = decltype(pos_)::value;
                    constexpr int l0 = LB + (pos * (LE - LB) + NS - 1) / NS;
                    constexpr int l1 = LB + ((pos + 1) * (LE - LB) + NS - 1) / NS;
                    if constexpr (l1 > l0) {
                        if (dma) {
                            static_for<l0, l1>([&](auto l) { dma_one(l, dbuf, dks); });
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                };
                static_for<0, NB>([&](auto n) {
                    static_for<0, MB>([&](auto m) {
                        acc[m][n] = H2<T16>::mfma(A0[m], B1[n], acc[m][n]);
                        __builtin_amdgcn_sched_barrier(0);
                        if constexpr (!SE) dma_at(std::integral_constant<int, n * MB + m>{});
                    });
                    if constexpr (NX && !SE) {
                        B1[n] = rd(nbuf, nu, 3, rb + 32 * n);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                });
                if constexpr (SE && NX) {
                    wait_vm(0);   // this wave's loads of the next slice (the only ones in flight)
                    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                    __builtin_amdgcn_sched_barrier(0);
                    static_for<0, NB>([&](auto n) { B1[n] = rd(nbuf, nu, 3, rb + 32 * n); });
                    __builtin_amdgcn_sched_barrier(0);
                }
                static_for<0, 2 * G>([&](auto i) {
                    constexpr int g3 = i >= G ? 1 : 0;
                    constexpr int m = (i % G) / NB, n = i % NB;
                    if constexpr (g3) acc[m][n] = H2<T16>::mfma(A1[m], B0[n], acc[m][n]);
                    else acc[m][n] = H2<T16>::mfma(A0[m], B0[n], acc[m][n]);
                    __builtin_amdgcn_sched_barrier(0);
                    dma_at(std::integral_constant<int, SE ? (int)i : G + (int)i>{});
                    if constexpr (NX && n == NB - 1) {
                        if constexpr (g3) A1[m] = rd(nbuf, nu, 1, ra + 32 * m);
                        else A0[m] = rd(nbuf, nu, 0, ra + 32 * m);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                });
                if constexpr (NX) {
                    static_for<0, NB>([&](auto n) { B0[n] = rd(nbuf, nu, 2, rb + 32 * n); });
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            using T_ = std::true_type;
            using F_ = std::false_type;
            using I0 = std::integral_constant<int, 0>;
            using IH = std::integral_constant<int, LH>;
            using IL = std::integral_constant<int, LPW>;
            // Slice sl: its first unit issues the second half of slice sl + 1 (the prologue
            // issued slices 0 and 1 whole); its last unit, after the barrier that frees
            // buffer sl & 1, the first half of slice sl + 2 into that buffer.
            int sl = 0;
            for (; sl + 1 < nsl; ++sl) {
                const int buf = sl & 1;
                unit(F_{}, T_{}, IH{}, IL{}, buf, 1, sl >= 1, buf ^ 1, kb + sl + 1);
                static_for<1, UPS - 1>([&](auto j) { unit(F_{}, T_{}, I0{}, I0{}, buf, j + 1, false, 0, 0); });
                unit(T_{}, T_{}, I0{}, IH{}, buf ^ 1, 0, sl + 2 < nsl, buf, kb + sl + 2);
            }
            static_for<0, UPS - 1>([&](auto j) { unit(F_{}, T_{}, I0{}, I0{}, sl & 1, j + 1, false, 0, 0); });
            unit(T_{}, F_{}, I0{}, I0{}, 0, 0, false, 0, 0);
        } else {
            // Two fragment sets (P, Q), double buffered per unit.
            auto arrive = [&](int next) {
                const int last = (next + ST - 2 < nsl - 1) ? next + ST - 2 : nsl - 1;   // last slice issued
                wait_vm((last - next) * LPW);
                __syncthreads();
            };
            vec8 pa0[MB], pa1[MB], pb0[NB], pb1[NB];   // fragments of even units
            vec8 qa0[MB], qa1[MB], qb0[NB], qb1[NB];   // fragments of odd units
            frags(0, 0, pa0, pa1, pb0, pb1);
            // The MFMAs of one unit with the direct loads that refill the buffer freed by
            // arrive(next) (slice next + ST - 1) spread between the X0 X0 and X0 X1 products, so
            // that their address arithmetic and issue overlap the matrix cores (scheduling
            // barriers keep the compiler from regrouping them), then `mid` (the fragment reads
            // of the next unit: by then the X0 fragments of this unit and its X1 column
            // fragments are dead, which keeps the register count down), then the X1 X0 products.
            auto mma_issue = [&](const vec8 (&fa0)[MB], const vec8 (&fa1)[MB], const vec8 (&fb0)[NB],
                                 const vec8 (&fb1)[NB], int next, auto&& mid) {
                constexpr int NM = 2 * MB * NB;
                const bool doit = next + ST - 1 < nsl;
                const int buf = (next - 1) % ST, ks = kb + next + ST - 1;
#pragma unroll
                for (int i = 0; i < NM; ++i) {
                    const int m = (i / NB) % MB, n = i % NB;
                    acc[m][n] = H2<T16>::mfma(fa0[m], i < MB * NB ? fb0[n] : fb1[n], acc[m][n]);
                    // the loads l with ceil(l NM / LPW) == i go right after MFMA i
                    const int l0 = (i * LPW + NM - 1) / NM, l1 = ((i + 1) * LPW + NM - 1) / NM;
                    if (l1 > l0) {
                        __builtin_amdgcn_sched_barrier(0);
                        if (doit) {
#pragma unroll
                            for (int l = l0; l < l1; ++l) dma_one(l, buf, ks);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                mid();
#pragma unroll
                for (int m = 0; m < MB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n) acc[m][n] = H2<T16>::mfma(fa1[m], fb0[n], acc[m][n]);
            };
            // Units run in pairs (P, Q); unit w is unit w % UPS of slice w / UPS.  Each step
            // reads the next unit's fragments while the matrix cores work on the current one.
            // The unit count is even; the last pair is peeled so that the loop body has no
            // branch and the LDS-read waits stay exact.
            const int nu = nsl * UPS;
            int w = 0;
            for (; w + 2 < nu; w += 2) {
                if constexpr (UPS == 1) {
                    arrive(w + 1);
                    mma_issue(pa0, pa1, pb0, pb1, w + 1, [&] { frags((w + 1) % ST, 0, qa0, qa1, qb0, qb1); });
                    arrive(w + 2);
                    mma_issue(qa0, qa1, qb0, qb1, w + 2, [&] { frags((w + 2) % ST, 0, pa0, pa1, pb0, pb1); });
                } else if constexpr (UPS == 2) {
                    frags((w / 2) % ST, 1, qa0, qa1, qb0, qb1);
                    mma(pa0, pa1, pb0, pb1);
                    arrive((w + 2) / 2);
                    mma_issue(qa0, qa1, qb0, qb1, (w + 2) / 2,
                              [&] { frags(((w + 2) / 2) % ST, 0, pa0, pa1, pb0, pb1); });
                } else {
                    frags((w / UPS) % ST, (w + 1) % UPS, qa0, qa1, qb0, qb1);
                    mma(pa0, pa1, pb0, pb1);
                    if ((w + 2) % UPS == 0) {
                        arrive((w + 2) / UPS);
                        mma_issue(qa0, qa1, qb0, qb1, (w + 2) / UPS,
                                  [&] { frags(((w + 2) / UPS) % ST, 0, pa0, pa1, pb0, pb1); });
                    } else {
                        frags(((w + 2) / UPS) % ST, (w + 2) % UPS, pa0, pa1, pb0, pb1);
                        mma(qa0, qa1, qb0, qb1);
                    }
                }
            }
            if constexpr (UPS == 1) {
                arrive(w + 1);
                frags((w + 1) % ST, 0, qa0, qa1, qb0, qb1);
            } else {
                frags((w / UPS) % ST, (w + 1) % UPS, qa0, qa1, qb0, qb1);
            }
            mma(pa0, pa1, pb0, pb1);
            mma(qa0, qa1, qb0, qb1);
        }
        __syncthreads();   // all fragment reads done before LDS is reused below

        // Per-lane index arithmetic below is recomputed from an opaque copy of the thread
        // index: otherwise it is loop-invariant across work items, gets hoisted above the
        // main loop and takes registers the pipeline needs.
        int otid = tid;
        asm volatile("" : "+v"(otid));
        const int olane = otid & 63, owave = otid >> 6;
        const int owm = owave / WN, own = owave % WN;

        // ---------------------------------------------------------------- split tail
        bool finish = chunk < 0;
        if (!finish) {
            constexpr size_t TILE_F = (size_t)BT * BT;
            constexpr size_t cstride = TILE_F / 4;   // f32x4 elements per partial tile
            // layout: per wave, per (m, n, quarter), 64 lanes x 4 floats
            f32x4* const wp0 = (f32x4*)(sk.partial + (size_t)owave * MB * NB * 16 * 64) + olane;
            auto store_partial = [&](size_t pslot) {
                f32x4* wp = wp0 + pslot * cstride;
                static_for<0, MB>([&](auto m) {
                    static_for<0, NB>([&](auto n) {
                        static_for<0, 4>([&](auto q4) {
                            f32x4 vv = {acc[m][n][4 * q4], acc[m][n][4 * q4 + 1], acc[m][n][4 * q4 + 2],
                                        acc[m][n][4 * q4 + 3]};
                            store_agent(wp, vv);
                            wp += 64;
                        });
                    });
                });
                wait_stores();   // this partial is coherent before the arrival is counted
                __syncthreads();
            };
            // acc = ((p_0 + p_1) + p_2) + ... over the partial slots slot_of(0 .. cnt - 1), one
            // partial at a time: the loads of a partial are independent and go out in batches
            // of RB row blocks (as many as the registers freed by the main loop hold)
            auto sum_partials = [&](int cnt, auto&& slot_of) {
                const f32x4* rp0 = wp0;
                constexpr int RB = MB * NB >= 16 ? 1 : (MB >= 2 ? 2 : 1);
                for (int c = 0; c < cnt; ++c) {
                    const f32x4* rp = rp0 + slot_of(c) * cstride;
                    static_for<0, MB / RB>([&](auto mb) {
                        f32x4 pv[RB][NB][4];
                        static_for<0, RB>([&](auto r) {
                            static_for<0, NB>([&](auto n) {
                                static_for<0, 4>([&](auto q4) {
                                    pv[r][n][q4] = load_agent(rp + (((mb * RB + r) * NB + n) * 4 + q4) * 64);
                                });
                            });
                        });
                        static_for<0, RB>([&](auto r) {
                            static_for<0, NB>([&](auto n) {
                                static_for<0, 4>([&](auto q4) {
                                    static_for<0, 4>([&](auto e) {
                                        const float d = acc[mb * RB + r][n][4 * q4 + e];
                                        acc[mb * RB + r][n][4 * q4 + e] = c == 0 ? pv[r][n][q4][(int)e]
                                                                                : d + pv[r][n][q4][(int)e];
                                    });
                                });
                            });
                        });
                        __builtin_amdgcn_sched_barrier(0);
                    });
                }
            };
            // Split tail with a multiple of 4 chunks per tile: two levels, so that no single
            // workgroup reads all the partials of a tile.  The last of each group of 4
            // consecutive chunks sums them (in chunk order) into a group partial; the last
            // group of the tile sums the group partials (in group order).  Counters: tile
            // arrivals at [0, tail_tiles), group arrivals from kSkGroupCounter; group partial
            // slots from kSkGroupSlot.
            const int gs = (!SQ && sk.chunks > 4 && sk.chunks % 4 == 0) ? 4 : contrib;
            const int ng = contrib / gs;                      // groups per tile (1: one level)
            const int grp = ng > 1 ? chunk / gs : 0;
            store_partial(slot);
            if (tid == 0) {
                int* cnt1 = ng > 1 ? sk.counter + kSkGroupCounter + tail_tile * ng + grp : sk.counter + tail_tile;
                s_flag = atomicAdd(cnt1, 1);
            }
            __syncthreads();
            // each executed layer adds gs arrivals per group (per tile with one level): the
            // last one reduces
            finish = ((s_flag + 1) % gs) == 0;
            if (finish) {
                // stream-K: the partial slots of the contributors in K order (at most
                // kSkMaxContrib by the plan); split tail: slots tail_tile * chunks + c
                if (SQ && tid < contrib) {
                    const int lo = t * ksq;
                    const int vf = (int)(((long long)(lo + 1) * G + U - 1) / U) - 1;
                    const int u = vf + tid;
                    const int ut0 = (int)((long long)u * U / G) / ksq;
                    s_slot[tid] = 2 * u + (ut0 == t ? 0 : 1);
                }
                __syncthreads();
                const size_t first = (size_t)tail_tile * sk.chunks + (size_t)grp * gs;
                sum_partials(gs, [&](int c) -> size_t { return SQ ? (size_t)s_slot[c] : first + c; });
                if (ng > 1) {
                    const size_t gslot0 = (size_t)kSkGroupSlot + (size_t)tail_tile * ng;
                    __syncthreads();   // every wave has read the chunk partials
                    store_partial(gslot0 + grp);
                    if (tid == 0) s_flag = atomicAdd(sk.counter + tail_tile, 1);
                    __syncthreads();
                    finish = ((s_flag + 1) % ng) == 0;
                    if (finish) {
                        sum_partials(ng, [&](int g) -> size_t { return gslot0 + g; });
                    }
                }
            }
        }

        // ---------------------------------------------------------------- epilogue
        if (finish) {
            float* so = (float*)a.s_out;
            const float* si = (const float*)a.s_in;
            T16* p0 = (T16*)a.p0_out;
            T16* p1 = (T16*)a.p1_out;
            const float osc = a.out_scale, isc = a.in_scale;
            const bool diag = (I == J);
            double tr = 0.0, fr = 0.0;
            // Off-diagonal tiles: each 32 x 32 block goes transposed through this wave's LDS
            // region (FP32 values, then both half planes) and is written to the mirror
            // position as whole row segments (128 bytes of FP32, 64 bytes per plane) instead
            // of one 16- or 8-byte piece per lane in 64 different rows.
            constexpr int TF = 36, TH = 40;    // padded row pitches (floats, halves): 16-byte aligned rows
            constexpr int WREG = 32 * TF * 4 + 2 * 32 * TH * 2;
            static_assert(C::NW * WREG <= C::LDS, "mirror staging fits in the pipeline stages");
            float* tf = (float*)(lds + owave * WREG);
            T16* th0 = (T16*)(lds + owave * WREG + 32 * TF * 4);
            T16* th1 = th0 + 32 * TH;
            static_for<0, MB>([&](auto m) {
                static_for<0, NB>([&](auto n) {
                    const int col = J * BT + own * C::WTN + n * 32 + (olane & 31);
                    static_for<0, 4>([&](auto g) {
                        const int row0 = I * BT + owm * C::WTM + m * 32 + 8 * g + 4 * (olane >> 5);
                        float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (beta != 0.f) s4 = *(const float4*)(si + (size_t)col * np + row0);
                        const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
                        float y4[4];
                        T16 h0[4], h1[4];
                        static_for<0, 4>([&](auto e) {
                            const float x = acc[m][n][4 * g + e] * osc;
                            float y = (beta != 0.f) ? fmaf(alpha, x, beta * sv[e]) : alpha * x;
                            if (row0 + e == col && col < a.n_real) y += gamma;
                            y4[e] = y;
                            const float ys = y * isc;
                            h0[e] = (T16)ys;
                            h1[e] = (T16)(ys - (float)h0[e]);
                        });
                        if (!diag) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const size_t off = (size_t)(row0 + e) * np + col;
                                so[off] = y4[e];
                                if (p0) {
                                    const size_t poff = (size_t)(row0 + e) * pld + col;
                                    p0[poff] = h0[e];
                                    p1[poff] = h1[e];
                                }
                                fr += 2.0 * (double)y4[e] * (double)y4[e];
                            }
                            // transposed into LDS: row (olane & 31) holds this block's column
                            const int lo = (olane & 31), ro = 8 * g + 4 * (olane >> 5);
                            *(float4*)(tf + lo * TF + ro) = make_float4(y4[0], y4[1], y4[2], y4[3]);
                            if (p0) {
                                vec4 q0 = {h0[0], h0[1], h0[2], h0[3]};
                                vec4 q1 = {h1[0], h1[1], h1[2], h1[3]};
                                *(vec4*)(th0 + lo * TH + ro) = q0;
                                *(vec4*)(th1 + lo * TH + ro) = q1;
                            }
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int row = row0 + e;
                                if (row > col) continue;
                                const size_t off = (size_t)row * np + col;
                                so[off] = y4[e];
                                if (p0) {
                                    const size_t poff = (size_t)row * pld + col;
                                    p0[poff] = h0[e];
                                    p1[poff] = h1[e];
                                }
                                if (row < col) {
                                    const size_t moff = (size_t)col * np + row;
                                    so[moff] = y4[e];
                                    if (p0) {
                                        const size_t pmoff = (size_t)col * pld + row;
                                        p0[pmoff] = h0[e];
                                        p1[pmoff] = h1[e];
                                    }
                                    fr += 2.0 * (double)y4[e] * (double)y4[e];
                                } else {
                                    tr += (double)y4[e];
                                    fr += (double)y4[e] * (double)y4[e];
                                }
                            }
                        }
                    });
                    if (!diag) {
                        // mirror rows: block columns J*BT + own*WTN + n*32 + c, entries at block rows
                        __syncthreads();
                        const size_t mrow0 = (size_t)(J * BT + own * C::WTN + n * 32);
                        const int mcol0 = I * BT + owm * C::WTM + m * 32;
                        static_for<0, 4>([&](auto k) {
                            const int c = 8 * k + (olane >> 3), q = olane & 7;
                            *(float4*)(so + (mrow0 + c) * np + mcol0 + 4 * q) = *(const float4*)(tf + c * TF + 4 * q);
                        });
                        if (p0) {
                            static_for<0, 2>([&](auto k) {
                                const int c = 16 * k + (olane >> 2), q = olane & 3;
                                const size_t goff = (mrow0 + c) * pld + mcol0 + 8 * q;
                                *(vec8*)(p0 + goff) = *(const vec8*)(th0 + c * TH + 8 * q);
                                *(vec8*)(p1 + goff) = *(const vec8*)(th1 + c * TH + 8 * q);
                            });
                        }
                        __syncthreads();
                    }
                });
            });
            if (a.parts) {
                tr = wsum(tr);
                fr = wsum(fr);
                double* scr = (double*)lds;   // the stages are free: every wave passed the last barrier
                __syncthreads();
                if (olane == 0) {
                    scr[2 * owave] = tr;
                    scr[2 * owave + 1] = fr;
                }
                __syncthreads();
                if (tid == 0) {
                    double s0 = 0.0, s1 = 0.0;
                    for (int w = 0; w < C::NW; ++w) {
                        s0 += scr[2 * w];
                        s1 += scr[2 * w + 1];
                    }
                    a.parts[2 * t] = s0;
                    a.parts[2 * t + 1] = s1;
                }
            }
        }
        __syncthreads();   // LDS is reused by the next item's prologue
    }
}

template <typename T16, int WM, int WN, int MB, int NB, int SK, int ST, int RP>
__global__ __launch_bounds__(64 * WM * WN) void k_square_sk(SquareArgs a, StreamK sk) {
    if (a.skip && *a.skip) return;
    // XCD-aware order: the workgroups of one XCD get consecutive virtual indices
    const int v = (blockIdx.x & 7) * (sk.grid >> 3) + (blockIdx.x >> 3);
    sk_body<T16, WM, WN, MB, NB, SK, ST, RP, false>(a, sk, v, 0);
}

// One workgroup per upper-triangle tile of one problem, XCD-aware tile order.
template <typename T16, int WM, int WN, int MB, int NB, int SK, int ST, int RP>
__global__ __launch_bounds__(64 * WM * WN) void k_square_dp(SquareArgs a) {
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
    sk_body<T16, WM, WN, MB, NB, SK, ST, RP, true>(a, none, 0, t);
}

// One workgroup per upper-triangle tile of many problems: block b computes the tile that
// the tile map names for it (see kTileMapShift), if any.
template <typename T16, int WM, int WN, int MB, int NB, int SK, int ST, int RP>
__global__ __launch_bounds__(64 * WM * WN) void k_square_dp_g(const SquareArgs* __restrict__ descs,
                                                             const int* __restrict__ map, int per) {
    const int e = map[(blockIdx.x & 7) * per + (blockIdx.x >> 3)];
    if (e < 0) return;
    const SquareArgs a = descs[e >> kTileMapShift];
    if (a.skip && *a.skip) return;
    StreamK none;
    none.grid = 0;
    none.rounds = 0;
    none.tail_tiles = 0;
    none.chunks = 1;
    none.partial = nullptr;
    none.counter = nullptr;
    none.fpartial = nullptr;
    sk_body<T16, WM, WN, MB, NB, SK, ST, RP, true>(a, none, 0, e & kTileMapMask);
}

}  // namespace

// Per-tile (one workgroup per tile) forms of the same pipeline.  Variants per tile edge,
// as (waves, K-slice halves, LDS stages, rolling fragment pipeline): 256: (8, 32, 2, 1),
// (4, 32, 2, 0); 128: (4, 32, 2, 1), (4, 64, 2, 0), (4, 16, 4, 0).  descs == nullptr: the
// single problem `a` (XCD-aware order, grid 8 a.per); otherwise the grouped launch over
// the tile map (grid 8 per).
template <typename T16>
hipError_t launch_dp_t(int tile, int variant, const SquareArgs& a, const SquareArgs* descs, const int* map,
                       int per, hipStream_t s) {
#define SP2_L(WM, WN, MB, NB, SK, ST, RP)                                                                   \
    do {                                                                                                   \
        if (descs)                                                                                         \
            hipLaunchKernelGGL((k_square_dp_g<T16, WM, WN, MB, NB, SK, ST, RP>), dim3(8 * per),           \
                               dim3(64 * WM * WN), 0, s, descs, map, per);                                 \
        else                                                                                               \
            hipLaunchKernelGGL((k_square_dp<T16, WM, WN, MB, NB, SK, ST, RP>), dim3(8 * a.per),           \
                               dim3(64 * WM * WN), 0, s, a);                                               \
    } while (0)
    if (tile == 256) {
        switch (variant) {
            case 0: SP2_L(2, 4, 4, 2, 32, 2, 1); break;
            case 1: SP2_L(2, 2, 4, 4, 32, 2, 0); break;
            default: return hipErrorInvalidValue;
        }
    } else if (tile == 128) {
        switch (variant) {
            case 0: SP2_L(2, 2, 2, 2, 32, 2, 1); break;
            case 1: SP2_L(2, 2, 2, 2, 64, 2, 0); break;
            case 2: SP2_L(2, 2, 2, 2, 16, 4, 0); break;
            case 3: SP2_L(2, 2, 2, 2, 64, 2, 1); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef SP2_L
    return hipGetLastError();
}

// Persistent launches per tile edge (instantiated in separate units so they compile in
// parallel).  Variant tables: keep in step with kV256 / kV128 in k_square2.hip.
#define SP2_L(WM, WN, MB, NB, SK, ST, RP)                                                            \
    hipLaunchKernelGGL((k_square_sk<T16, WM, WN, MB, NB, SK, ST, RP>), dim3(sk.grid), dim3(64 * WM * WN), 0, \
                       s, a, sk)
template <typename T16>
hipError_t launch_sk256_t(int variant, const SquareArgs& a, const StreamK& sk, hipStream_t s) {
    switch (variant) {
        case 0: SP2_L(2, 2, 4, 4, 16, 4, 0); break;
        case 1: SP2_L(2, 4, 4, 2, 16, 4, 0); break;
        case 2: SP2_L(2, 2, 4, 4, 32, 2, 0); break;
        case 3: SP2_L(2, 4, 4, 2, 32, 2, 0); break;
        case 4: SP2_L(2, 2, 4, 4, 32, 2, 1); break;
        case 5: SP2_L(2, 4, 4, 2, 32, 2, 1); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <typename T16>
hipError_t launch_sk128_t(int variant, const SquareArgs& a, const StreamK& sk, hipStream_t s) {
    switch (variant) {
        case 0: SP2_L(2, 2, 2, 2, 32, 4, 0); break;
        case 1: SP2_L(2, 2, 2, 2, 64, 2, 0); break;
        case 2: SP2_L(2, 2, 2, 2, 16, 4, 0); break;
        case 3: SP2_L(2, 2, 2, 2, 32, 2, 0); break;
        case 4: SP2_L(2, 2, 2, 2, 64, 2, 1); break;
        case 5: SP2_L(2, 2, 2, 2, 32, 2, 1); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef SP2_L

}  // namespace sp2
