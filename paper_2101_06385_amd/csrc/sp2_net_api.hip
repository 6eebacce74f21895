// Host side of the differentiable generalized-SP2 network (Eq. general SP2 as matrix layers):
// forward with layer checkpoints, backward with per-segment recomputation and the FP32
// adjoint layer.  See include/sp2.h for the contract.
#include "sp2_internal.h"

#include <math.h>
#include <string.h>

using namespace sp2;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// adjoint variant for n <= 4096 (64 tiles): 0 = 2 LDS stages, two workgroups per CU;
// 1 = 4 stages, one per CU
constexpr int kAdjVariantSmall = 0;
// ckpt_every = 0 keeps every layer (no recomputation in the backward) while the K + 7
// padded matrices fit in this many bytes, a small share of the device memory; above it
// the checkpoints are sqrt(K) apart.
constexpr size_t kKeepAllBytes = size_t(8) << 30;

struct NetPlan {
    int n, np, K, c, nck, precision, tile_main, tile_adj, adj_variant, scale_log2;
    bool split;
    int T_main, nt_main, per_main, T_adj, nt_adj, per_adj;
    size_t off_coef, off_adj_parts, off_adj_partial, off_adj_counter, off_ckpt, off_seg, off_ping, off_planes, off_g,
        off_xout, total;
};

bool net_plan(int n, int K, int precision, int ckpt_every, NetPlan* p) {
    if (n <= 0 || n > 65536 || K <= 0 || K > 4096 || ckpt_every < 0) return false;
    if (precision != SP2_FP32 && precision != SP2_FP16X2 && precision != SP2_BF16X2) return false;
    p->n = n;
    p->K = K;
    p->precision = precision;
    p->split = precision != SP2_FP32;
    p->scale_log2 = precision == SP2_FP16X2 ? 12 : 0;
    p->tile_main = n <= 256 ? 64 : 128;
    // adjoint: 64 tiles until 128 tiles fill the GPU (136 tiles of 128 at n = 2048 left
    // half the CUs idle)
    p->adj_variant = n <= 4096 ? kAdjVariantSmall : 2;
    p->tile_adj = adjoint_tile(p->adj_variant);
    const int m = p->tile_main > p->tile_adj ? p->tile_main : p->tile_adj;
    p->np = round_up(n, m);
    if (p->split)
        square_split_grid(p->tile_main, p->np, &p->T_main, &p->nt_main, &p->per_main);
    else
        square_plain_grid(p->tile_main, p->np, &p->T_main, &p->nt_main, &p->per_main);
    adjoint_grid(p->tile_adj, p->np, &p->T_adj, &p->nt_adj, &p->per_adj);
    const size_t m2 = (size_t)p->np * p->np * sizeof(float);
    if (ckpt_every) p->c = ckpt_every;
    else p->c = (size_t)(K + 7) * m2 <= kKeepAllBytes ? 1 : (int)ceil(sqrt((double)K));
    if (p->c > K) p->c = K;
    p->nck = (K + p->c - 1) / p->c;
    size_t off = 0;
    p->off_coef = off;
    off = align_up(off + sizeof(float) * 3 * K);
    p->off_adj_parts = off;
    off = align_up(off + sizeof(double) * 3 * p->nt_adj);
    p->off_adj_partial = off;   // split-K partials of the adjoint's leftover tiles
    off = align_up(off + adjoint_partial_bytes(p->adj_variant));
    p->off_adj_counter = off;
    off = align_up(off + sizeof(int) * kMaxSkGrid);
    p->off_ckpt = off;
    off = align_up(off + m2 * p->nck);
    p->off_seg = off;
    off = align_up(off + m2 * p->c);
    p->off_ping = off;
    off = align_up(off + 2 * m2);
    p->off_planes = off;
    if (p->split) off = align_up(off + 4 * (size_t)p->np * plane_ld(p->np) * 2);
    p->off_g = off;
    off = align_up(off + 2 * m2);
    p->off_xout = off;
    off = align_up(off + m2);
    p->total = off;
    return true;
}

#define SP2_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return SP2_EDEVICE;   \
    } while (0)

struct NetBuffers {
    float* coef;
    double* adj_parts;
    float* ckpt;
    float* seg;
    float* ping[2];
    void* planes[2][2];
    float* g[2];
    float* xout;
    size_t m;   // elements per padded matrix
};

NetBuffers carve(const NetPlan& p, void* dWork) {
    char* ws = (char*)dWork;
    NetBuffers b;
    b.m = (size_t)p.np * p.np;
    b.coef = (float*)(ws + p.off_coef);
    b.adj_parts = (double*)(ws + p.off_adj_parts);
    b.ckpt = (float*)(ws + p.off_ckpt);
    b.seg = (float*)(ws + p.off_seg);
    b.ping[0] = (float*)(ws + p.off_ping);
    b.ping[1] = b.ping[0] + b.m;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            b.planes[i][j] =
                p.split ? (void*)(ws + p.off_planes + (size_t)(2 * i + j) * p.np * plane_ld(p.np) * 2) : nullptr;
    b.g[0] = (float*)(ws + p.off_g);
    b.g[1] = b.g[0] + b.m;
    b.xout = (float*)(ws + p.off_xout);
    return b;
}

// One forward layer X_out = W_k X_in^2 + B_k X_in + c_k I.  Planes of X_in are in
// planes[pin]; the layer writes the planes of X_out into planes[pin ^ 1].
hipError_t layer(const NetPlan& p, const NetBuffers& b, int k, const float* x_in, float* x_out, int pin,
                 hipStream_t s) {
    SquareArgs a;
    memset(&a, 0, sizeof(a));
    a.x0 = p.split ? b.planes[pin][0] : (const void*)x_in;
    a.x1 = p.split ? b.planes[pin][1] : nullptr;
    a.s_in = x_in;
    a.s_out = x_out;
    a.p0_out = p.split ? b.planes[pin ^ 1][0] : nullptr;
    a.p1_out = p.split ? b.planes[pin ^ 1][1] : nullptr;
    a.parts = nullptr;
    a.coef = b.coef + 3 * k;
    a.skip = nullptr;
    a.np = p.np;
    a.ld_out = p.np;
    a.n_valid = p.np;
    a.n_real = p.n;
    a.T = p.T_main;
    a.ntiles = p.nt_main;
    a.per = p.per_main;
    a.out_scale = ldexpf(1.f, -2 * p.scale_log2);
    a.in_scale = ldexpf(1.f, p.scale_log2);
    // one workgroup per 128 tile with 64-half K-slices (the single-problem choice)
    if (p.split && p.tile_main == 128) return launch_square_dp(p.precision, 128, 3, a, s);
    return p.split ? launch_square_split(p.precision, p.tile_main, a, s)
                   : launch_square_plain(p.precision, p.tile_main, a, s);
}

}  // namespace

extern "C" {

size_t sp2_net_workspace_size(int n, int K, int precision, int ckpt_every) {
    NetPlan p;
    if (!net_plan(n, K, precision, ckpt_every, &p)) return 0;
    return p.total;
}

int sp2_net_forward(const float* dX0, int ld0, int n, int K, const float* dW, const float* dB, const float* dC,
                    int precision, int ckpt_every, float* dXK, int ldk, void* dWork, size_t work_bytes,
                    void* stream) {
    NetPlan p;
    if (!net_plan(n, K, precision, ckpt_every, &p)) return SP2_EINVAL;
    if (!dX0 || !dW || !dB || !dC || !dXK || !dWork || ld0 < n || ldk < n) return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    if (work_bytes < p.total) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    NetBuffers b = carve(p, dWork);
    SP2_TRY(launch_pack_coef(dW, dB, dC, K, b.coef, s));
    SP2_TRY(launch_copy_pad(dX0, b.ckpt, n, ld0, p.np, 1, s));   // X_0 is checkpoint 0
    if (p.split) SP2_TRY(launch_split(b.ckpt, b.planes[0][0], b.planes[0][1], p.np, p.precision, p.scale_log2, s));
    const float* x_in = b.ckpt;
    for (int k = 0; k < K; ++k) {
        float* x_out;
        if (k + 1 == K) x_out = b.xout;
        else if ((k + 1) % p.c == 0) x_out = b.ckpt + (size_t)((k + 1) / p.c) * b.m;
        else x_out = b.ping[(k + 1) & 1];
        SP2_TRY(layer(p, b, k, x_in, x_out, k & 1, s));
        x_in = x_out;
    }
    SP2_TRY(launch_copy_pad(b.xout, dXK, n, ldk, p.np, 0, s));
    return SP2_OK;
}

int sp2_net_backward(const float* dGK, int ldg, int n, int K, const float* dW, const float* dB, const float* dC,
                     int precision, int ckpt_every, float* dG0, int ldg0, float* ddW, float* ddB, float* ddC,
                     void* dWork, size_t work_bytes, void* stream) {
    NetPlan p;
    if (!net_plan(n, K, precision, ckpt_every, &p)) return SP2_EINVAL;
    if (!dGK || !dW || !dB || !dC || !ddW || !ddB || !ddC || !dWork || ldg < n) return SP2_EINVAL;
    if (dG0 && ldg0 < n) return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    if (work_bytes < p.total) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    NetBuffers b = carve(p, dWork);
    // coefficients may have changed since the forward call only if the caller changed them;
    // the backward uses the ones passed here
    SP2_TRY(launch_pack_coef(dW, dB, dC, K, b.coef, s));
    int gc = 0;
    // X_K is symmetric, so only the symmetric part of G_K acts on it
    SP2_TRY(launch_sym_pad(dGK, b.g[gc], n, ldg, p.np, s));
    StreamK sk;
    memset(&sk, 0, sizeof(sk));
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return SP2_EDEVICE;
    adjoint_plan(p.adj_variant, p.np, cus, &sk);
    sk.partial = (float*)((char*)dWork + p.off_adj_partial);
    sk.counter = (int*)((char*)dWork + p.off_adj_counter);
    SP2_TRY(launch_zero_ints(sk.counter, kMaxSkGrid, s));   // arrivals count modulo chunks from here
    AdjointArgs aa;
    memset(&aa, 0, sizeof(aa));
    aa.parts = b.adj_parts;
    aa.np = p.np;
    aa.T = p.T_adj;
    aa.ntiles = p.nt_adj;
    aa.per = p.per_adj;
    for (int seg = p.nck - 1; seg >= 0; --seg) {
        const int s0 = seg * p.c;
        const int e = s0 + p.c < K ? s0 + p.c : K;
        const float* xs = b.ckpt + (size_t)seg * b.m;
        // recompute X_{s0+1} .. X_{e-1} into seg slots 1 .. e-1-s0 (bit-identical to the forward)
        if (e - 1 > s0) {
            if (p.split) SP2_TRY(launch_split(xs, b.planes[0][0], b.planes[0][1], p.np, p.precision, p.scale_log2, s));
            const float* x_in = xs;
            for (int k = s0; k < e - 1; ++k) {
                float* x_out = b.seg + (size_t)(k + 1 - s0) * b.m;
                SP2_TRY(layer(p, b, k, x_in, x_out, (k - s0) & 1, s));
                x_in = x_out;
            }
        }
        for (int k = e - 1; k >= s0; --k) {
            aa.g = b.g[gc];
            aa.x = (k == s0) ? xs : b.seg + (size_t)(k - s0) * b.m;
            aa.g_out = b.g[gc ^ 1];
            aa.coef = b.coef + 3 * k;
            SP2_TRY(launch_adjoint(p.adj_variant, aa, sk, s));
            SP2_TRY(launch_reduce3(b.adj_parts, p.nt_adj, ddW, ddB, ddC, k, s));
            gc ^= 1;
        }
    }
    if (dG0) SP2_TRY(launch_copy_pad(b.g[gc], dG0, n, ldg0, p.np, 0, s));
    return SP2_OK;
}

}  // extern "C"
