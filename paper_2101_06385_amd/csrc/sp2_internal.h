// Internal declarations shared by the HIP kernels and the host driver of libsp2.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sp2.h"
#include "sp2_args.h"

namespace sp2 {

// Split-K partial tiles of the persistent kernels cross XCDs, whose L2 caches are not
// coherent with each other.  They are written with agent-coherent (write-through) stores
// and read with agent-scope atomic loads, so neither side needs a device-wide fence: such a
// fence writes back or invalidates the whole L2 of the XCD, which also holds the other
// workgroups' panels and output.  A writer waits for its stores (wait_stores) before its
// arrival is counted.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st16_agent(void* p, u32x4_t v) {
    asm volatile("global_store_dwordx4 %0, %1, off sc1" : : "v"(p), "v"(v) : "memory");
}
__device__ __forceinline__ u32x4_t ld16_agent(const void* p) {
    typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));
    const unsigned long long* q = (const unsigned long long*)p;
    const u64x2_t ab = {__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
    return __builtin_bit_cast(u32x4_t, ab);
}
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------------------------
// Per-call device state: lives at the start of the caller's workspace.
// Written by the control kernels; read by the layer kernels (skip flag, layer
// coefficients) and copied back to the host for sp2_info.
// ---------------------------------------------------------------------------------
struct DevState {
    int n, n_occ, n_padded, max_layers;
    int precision, tile, have_bounds, want_energy;
    int stopped;        // 1 once a stopping test held, a non-finite value appeared or the cap hit
    int converged;
    int layers;         // m
    int status;         // device-side sp2_status
    int skip;           // layer kernels of the current layer do nothing when set
    int first_sign;     // first composed step of the refinement
    int refine_src;     // ping-pong index of the state matrix that is refined
    int ran;            // squaring layers that ran (the last layer whose control let it run)
    float coef[3];      // (alpha, beta, gamma) of the current layer: Y = alpha X^2 + beta X + gamma I
    float rcoef[2][3];  // the two refinement layers
    float pad1;
    double eps, tol_tr, tol_id;
    double emin, emax;
    double asym;
    double trace_d, frob_d, energy;
    signed char sigma[SP2_MAX_LAYERS + 1];  // index n = layer n (sigma[0] = 0)
    double iderr[SP2_MAX_LAYERS + 1];
    double ns[SP2_MAX_LAYERS + 1];
    double nx[SP2_MAX_LAYERS + 1];
    // accelerated layers (Sec. Accelerated Deep-NN SP2)
    int accel;          // 1 when the caller's interval rescaled into 0 <= l < h <= 1
    int acc_layers;     // index of the last accelerated layer (0: none)
    int gap_violation;  // first layer whose interval consistency check failed (0: none)
    int pad2;
    double homo, lumo;  // caller's interval inside the gap (energies)
    double acc_l, acc_h;  // unoccupied eigenvalues of S_{n-1} in [0, acc_l], occupied in [acc_h, 1]
    double sigma_c[SP2_MAX_LAYERS + 1];
    double coef64[3];   // the current layer's (alpha, beta, gamma) unrounded, for the FP64 layer kernels
    double pad3;
};

// Upper-triangle tile enumeration shared by every kernel that works on (I <= J) tiles.
// The T x T tile grid is cut into column strips of width G; strips are enumerated left
// to right, and inside a strip the tiles go row by row.  Consecutive indices therefore
// form compact G-wide blocks of rows, so workgroups that run at the same time on one
// XCD share their row and column panels in that XCD's L2.
__host__ __device__ inline void tile_of(int t, int T, int G, int* pi, int* pj) {
    int s = 0, off = 0;
    for (;;) {
        int w = T - s * G < G ? T - s * G : G;
        int cnt = s * G * w + w * (w + 1) / 2;
        if (t < off + cnt) {
            int u = t - off;
            int sg = s * G;
            if (u < sg * w) {
                *pi = u / w;
                *pj = sg + u % w;
            } else {
                u -= sg * w;
                int i = 0;
                while (u >= w - i) { u -= w - i; ++i; }
                *pi = sg + i;
                *pj = sg + i + u;
            }
            return;
        }
        off += cnt;
        ++s;
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; this maps the
// hardware block index so that XCD x receives the contiguous tile range
// [x*per, (x+1)*per).  Returns -1 for the (at most 7) surplus blocks.
__device__ inline int xcd_tile_index(int b, int per, int ntiles) {
    int t = (b & 7) * per + (b >> 3);
    return t < ntiles ? t : -1;
}

inline int ntiles_upper(int T) { return T * (T + 1) / 2; }

// Group of a block in a launch that covers several problems: offs[0..n] are the first
// block of each problem (offs[0] = 0, offs[n] = total); returns p with offs[p] <= b < offs[p+1].
__device__ inline int find_group(const int* offs, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}



// Autotuner table (sp2_tune.hip): the fastest measured schedule per (device, kind,
// precision, key); kind single: key = n rounded up to 256; kind batched: key = hash of the
// sorted sizes.
constexpr int kTuneSingle = 0, kTuneBatched = 1;
unsigned long long tune_key_single(int n);
unsigned long long tune_key_batched(int batch, const int* n);
bool tune_lookup(int kind, int precision, unsigned long long key, int* tile, int* kernel);
void tune_store(int kind, int precision, unsigned long long key, int tile, int kernel, float ms);

// Arguments of the FP32 adjoint layer of the generalized-SP2 network.
struct AdjointArgs {
    const float* g;       // G = dL/dX_{k+1}, np x np, symmetric
    const float* x;       // X_k, np x np, symmetric
    float* g_out;         // G_k = W_k (G X_k + X_k G) + B_k G
    double* parts;        // 3 doubles per tile: Tr G, <G, X_k>, <G, X_k^2>
    const float* coef;    // (W_k, B_k, c_k)
    int np, T, ntiles, per;
};

hipError_t launch_pack_coef(const float* w, const float* b, const float* c, int K, float* out, hipStream_t s);
hipError_t launch_copy_pad(const float* src, float* dst, int n, int ld, int np, int to_pad, hipStream_t s);
// dst (np x np, zero padded) <- (src + src^T)/2 of the n x n src (ld); np a multiple of 32
hipError_t launch_sym_pad(const float* src, float* dst, int n, int ld, int np, hipStream_t s);
int adjoint_grid(int tile, int np, int* T, int* ntiles, int* per);
// adjoint variants 0..2 (k_net.hip): tile, schedule, split-K partial buffer, launch
int adjoint_tile(int variant);
void adjoint_plan(int variant, int np, int cus, StreamK* sk);
size_t adjoint_partial_bytes(int variant);
hipError_t launch_adjoint(int variant, const AdjointArgs& a, const StreamK& sk, hipStream_t s);
hipError_t launch_reduce3(const double* parts, int nparts, float* dw, float* db, float* dc, int k, hipStream_t s);

// One problem of a batched call (device copy; pointers into the batch workspace).  The
// batched path uses the FP32 state of the split and FP32 modes.
struct BatchProblem {
    const double* h;
    double* d;
    DevState* st;
    void* s[2];           // FP32 states, ping-pong
    void* pl[2][2];       // half-precision planes (split modes), ping-pong
    double* s64;          // refinement input (FP64)
    double* y;            // refinement intermediate (FP64)
    double* init_parts;   // 3 per input-layer tile
    double* main_parts;   // 2 per squaring tile
    double* gersh;        // 3 per Gershgorin block
    double* dstats;       // 3 per final-check block
    int ldh, ldd, n, np, n_occ, want_energy;
    int init_tiles, main_tiles, gersh_blocks, dstats_blocks;
    float in_scale, pad;
};

hipError_t launch_batch_gershgorin(const BatchProblem* pr, const int* offs, int nprob, int blocks, hipStream_t s);
hipError_t launch_batch_bounds(const BatchProblem* pr, int nprob, hipStream_t s);
hipError_t launch_batch_init(int precision, const BatchProblem* pr, const int* offs, int nprob, int blocks,
                             hipStream_t s);
hipError_t launch_batch_control(const BatchProblem* pr, int nprob, int layer, hipStream_t s);
hipError_t launch_batch_select(const BatchProblem* pr, int nprob, int per_problem, hipStream_t s);
hipError_t launch_batch_dstats(const BatchProblem* pr, const int* offs, int nprob, int blocks, hipStream_t s);
hipError_t launch_batch_finalize(const BatchProblem* pr, int nprob, hipStream_t s);
hipError_t launch_batch_states(const BatchProblem* pr, DevState* stage, int nprob, int to_regions, hipStream_t s);

// Host-side launchers (defined next to their kernels).
hipError_t launch_square_split(int precision, int tile, const SquareArgs& a, hipStream_t s);
hipError_t launch_square_plain(int precision, int tile, const SquareArgs& a, hipStream_t s);
// FP64 layer with direct-to-LDS staging, 128 tiles (k_square_f64.hip); variant 0 or 1
hipError_t launch_square_f64(int variant, const SquareArgs& a, hipStream_t s);
// grouped FP64 layer over a tile map (see kTileMapShift), grid 8 per
hipError_t launch_square_f64_g(const SquareArgs* descs, const int* map, int per, hipStream_t s);
// persistent FP64 layer (whole rounds + split-K tail), 128 tiles
bool square_f64_sk_plan(int np, int cus, StreamK* sk);
size_t square_f64_sk_partial_bytes();
hipError_t launch_square_f64_sk(const SquareArgs& a, const StreamK& sk, hipStream_t s);
hipError_t launch_square_split_g(int precision, int tile, const SquareArgs* descs, const int* offs, int nprob,
                                 int blocks, hipStream_t s);
hipError_t launch_square_plain_g(int precision, int tile, const SquareArgs* descs, const int* offs, int nprob,
                                 int blocks, hipStream_t s);
int square_split_grid(int tile, int np, int* T, int* ntiles, int* per);
int square_plain_grid(int tile, int np, int* T, int* ntiles, int* per);
// persistent split square: kSkVariants kernel variants per tile edge (128, 256)
bool square_sk_plan(int tile, int variant, int np, int cus, int* wg_per_cu, StreamK* sk, int* T, int* ntiles);
size_t square_sk_partial_bytes(int tile, int np);
hipError_t launch_square_sk(int precision, int tile, int variant, const SquareArgs& a, const StreamK& sk,
                            hipStream_t s);
// the same pipeline with one workgroup per tile (tiles 128, 256): one problem, or grouped
hipError_t launch_square_dp(int precision, int tile, int variant, const SquareArgs& a, hipStream_t s);
hipError_t launch_square_dp_g(int precision, int tile, int variant, const SquareArgs* descs, const int* map, int per,
                              hipStream_t s);
hipError_t launch_zero_ints(int* p, int count, hipStream_t s);

// preparation / control kernels (k_prep.hip)
hipError_t launch_state_init(DevState* st, const DevState& init, hipStream_t s);
hipError_t launch_gershgorin(const double* h, int ldh, int n, double* blk, int* nblk, hipStream_t s);
int gershgorin_blocks(int n);
hipError_t launch_bounds(DevState* st, const double* blk, int nblk, hipStream_t s);
hipError_t launch_init_np(const double* h, int ldh, DevState* st, int np, int precision, void* s_out,
                          void* p0, void* p1, int scale_log2, double* parts, hipStream_t s);
int init_tiles(int np);
hipError_t launch_control_stride(DevState* st, const double* parts, int nparts, int stride, int layer,
                                 int* host_flag, hipStream_t s);
hipError_t launch_select_f64(const DevState* st, const void* s0, const void* s1, int state_f64,
                             double* out, int ld_out, int n_valid, int np, hipStream_t s);
hipError_t launch_dstats(const double* d, int ldd, const double* h, int ldh, int n,
                         double* parts, int* nparts, hipStream_t s);
int dstats_blocks(int n);
hipError_t launch_finalize(DevState* st, const double* dparts, int ndparts, const double* init_parts,
                           int ninit, hipStream_t s);
hipError_t launch_fill(double* d, int ldd, int n, double diag, hipStream_t s);
hipError_t launch_split(const float* x, void* p0, void* p1, int np, int precision, int scale_log2,
                        hipStream_t s);
hipError_t launch_sum_parts(const double* parts, int nparts, double* out2, hipStream_t s);
hipError_t launch_set3(float* dst, float a, float b, float c, hipStream_t s);
// finite-temperature read-out: acc (FP64, n_p x n_p) = a X + diag I (first) or += a X
hipError_t launch_readout(int precision, double* acc, const void* x, int np, double a, double diag, int first,
                          hipStream_t s);
hipError_t launch_copy_out(const double* acc, int np, double* d, int ldd, int n, hipStream_t s);
hipError_t launch_store_coefs(float* dst, const double* vals, int count, hipStream_t s);   // rounded to FP32
hipError_t launch_store_coefs64(double* dst, const double* vals, int count, hipStream_t s);
hipError_t launch_sum3(const double* parts, int nparts, double* out3, hipStream_t s);
hipError_t launch_mark_trivial(DevState* st, hipStream_t s);

// The whole sp2_density path (sp2_api.hip); poll_flag = false never touches host memory
// beyond the final read-back of the state (no mapped flag).
int density_call(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                 const sp2_options* opt, sp2_info* info, void* dWork, size_t work_bytes, void* stream,
                 sp2_timing* timing, bool poll_flag);

}  // namespace sp2
