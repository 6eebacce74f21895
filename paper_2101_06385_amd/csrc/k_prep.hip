// Preparation, control and reduction kernels of libsp2 (gfx950).
//
//   k_state_init  : per-call device state
//   k_gershgorin  : FP64 Gershgorin row intervals, one wavefront per row
//   k_bounds      : min/max of the row intervals -> spectral bounds of Alg. 1
//   k_init        : input layer S_0 = W_0 H + B_0 of Alg. 1 (reversed rescale into [0,1]),
//                   symmetrized, stored in the state precision and split into planes
//   k_control     : one layer of Alg. 1's scalar logic: IdErr_n, sigma_n, stopping tests
//   k_select_f64  : widen the state matrix that is refined to FP64
//   k_dstats      : FP64 partial sums of Tr D, ||D||_F^2 and Tr[D H]
//   k_finalize    : final occupation / idempotency acceptance test
//
// All reductions use a fixed order (strided per-thread sums, then a fixed tree), so a
// given input reproduces bit-identical traces, histories and statuses.
#include "sp2_internal.h"

#include <math.h>

namespace sp2 {

namespace {

constexpr int kThreads = 256;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Fixed-order block sum of `count` doubles per thread (count <= 3), result in out[] of thread 0.
template <int C>
__device__ inline void block_sum(double (&v)[C], double* sh /* C * kThreads */) {
    const int t = threadIdx.x;
    for (int c = 0; c < C; ++c) sh[c * kThreads + t] = v[c];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < C; ++c) sh[c * kThreads + t] += sh[c * kThreads + t + w];
        __syncthreads();
    }
    for (int c = 0; c < C; ++c) v[c] = sh[c * kThreads];
}

struct StateParams {
    int n, n_occ, np, max_layers, precision, tile, have_bounds, want_energy, accel;
    double eps, tol_tr, tol_id, emin, emax, homo, lumo;
};

__global__ void k_state_init(DevState* st, StateParams p) {
    const int t = threadIdx.x;
    for (int i = t; i <= SP2_MAX_LAYERS; i += blockDim.x) {
        st->sigma[i] = 0;
        st->iderr[i] = 0.0;
        st->ns[i] = 0.0;
        st->nx[i] = 0.0;
        st->sigma_c[i] = 0.0;
    }
    if (t == 0) {
        st->n = p.n;
        st->n_occ = p.n_occ;
        st->n_padded = p.np;
        st->max_layers = p.max_layers;
        st->precision = p.precision;
        st->tile = p.tile;
        st->have_bounds = p.have_bounds;
        st->want_energy = p.want_energy;
        st->stopped = 0;
        st->converged = 0;
        st->layers = 0;
        st->status = SP2_OK;
        st->skip = 0;
        st->first_sign = 0;
        st->refine_src = 0;
        st->ran = 0;
        for (int i = 0; i < 3; ++i) {
            st->coef[i] = 0.f;
            st->coef64[i] = 0.0;
        }
        st->pad3 = 0.0;
        for (int i = 0; i < 6; ++i) st->rcoef[i / 3][i % 3] = 0.f;
        st->pad1 = 0.f;
        st->eps = p.eps;
        st->tol_tr = p.tol_tr;
        st->tol_id = p.tol_id;
        st->emin = p.emin;
        st->emax = p.emax;
        st->asym = 0.0;
        st->trace_d = 0.0;
        st->frob_d = 0.0;
        st->energy = 0.0;
        st->accel = p.accel;
        st->acc_layers = 0;
        st->gap_violation = 0;
        st->pad2 = 0;
        st->homo = p.homo;
        st->lumo = p.lumo;
        st->acc_l = 0.0;
        st->acc_h = 1.0;
    }
}

// One wavefront per row i: r_i = sum_{j != i} |H_ij| in FP64; the row interval
// [H_ii - r_i, H_ii + r_i] widened by (2n + 4) ulp-units for the summation error.
constexpr int kGershRowsPerBlock = kThreads / 64;

__device__ __forceinline__ void gershgorin_body(const double* __restrict__ h, int ldh, int n,
                                                         double* __restrict__ blk, int bid) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = bid * kGershRowsPerBlock + wave;
    __shared__ double sh[3][kGershRowsPerBlock];
    double lo = INFINITY, hi = -INFINITY, bad = 0.0;
    if (row < n) {
        const double* hr = h + (size_t)row * ldh;
        double s = 0.0;
        for (int j = lane; j < n; j += 64) s += fabs(hr[j]);
        s = wave_sum(s);
        const double d = hr[row];
        const double slack = (2.0 * n + 4.0) * 2.220446049250313e-16;
        const double r = (s - fabs(d)) * (1.0 + slack) + slack * fabs(d);
        lo = d - r;
        hi = d + r;
        if (!isfinite(s) || !isfinite(d)) bad = 1.0;
    }
    if (lane == 0) {
        sh[0][wave] = lo;
        sh[1][wave] = hi;
        sh[2][wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kGershRowsPerBlock; ++w) {
            lo = fmin(lo, sh[0][w]);
            hi = fmax(hi, sh[1][w]);
            bad = fmax(bad, sh[2][w]);
        }
        blk[3 * bid + 0] = lo;
        blk[3 * bid + 1] = hi;
        blk[3 * bid + 2] = bad;
    }
}

__device__ __forceinline__ void bounds_body(DevState* st, const double* __restrict__ blk, int nblk) {
    __shared__ double sh[3][kThreads];
    const int t = threadIdx.x;
    double lo = INFINITY, hi = -INFINITY, bad = 0.0;
    for (int i = t; i < nblk; i += kThreads) {
        lo = fmin(lo, blk[3 * i]);
        hi = fmax(hi, blk[3 * i + 1]);
        bad = fmax(bad, blk[3 * i + 2]);
    }
    sh[0][t] = lo;
    sh[1][t] = hi;
    sh[2][t] = bad;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] = fmin(sh[0][t], sh[0][t + w]);
            sh[1][t] = fmax(sh[1][t], sh[1][t + w]);
            sh[2][t] = fmax(sh[2][t], sh[2][t + w]);
        }
        __syncthreads();
    }
    if (t == 0) {
        lo = sh[0][0];
        hi = sh[1][0];
        if (sh[2][0] != 0.0 || !isfinite(lo) || !isfinite(hi)) {
            st->status = SP2_ENONFINITE;
            lo = 0.0;
            hi = 1.0;
        }
        st->emin = lo;
        st->emax = hi;
    }
}

// ---------------------------------------------------------------------------------
// Input layer.  64 x 64 tiles over the upper triangle of the padded matrix; each tile
// reads H(I,J) and H(J,I) so that the state is built from (H + H^T)/2 and is exactly
// symmetric.  Writes both the tile and its mirror; padding rows/cols are zero.
// parts: per tile [Tr part, ||.||_F^2 part, max |H_ij - H_ji|].
// ---------------------------------------------------------------------------------
constexpr int kInitTile = 64;

template <typename St, typename T16, bool kSplit>
__device__ __forceinline__ void init_body(const double* __restrict__ h, int ldh,
                                                   const DevState* __restrict__ st, St* __restrict__ s_out,
                                                   T16* __restrict__ p0, T16* __restrict__ p1, float in_scale,
                                                   double* __restrict__ parts, int bid) {
    __shared__ double a[kInitTile][kInitTile + 1];
    __shared__ double b[kInitTile][kInitTile + 1];
    __shared__ double red[3][kThreads];
    const int n = st->n, np = st->n_padded;
    const int T = np / kInitTile;
    int I, J;
    tile_of(bid, T, T, &I, &J);   // plain column-strip order
    const int t = threadIdx.x;
    const int r0 = I * kInitTile, c0 = J * kInitTile;
    for (int idx = t; idx < kInitTile * kInitTile; idx += kThreads) {
        const int r = idx / kInitTile, c = idx % kInitTile;
        const int gi = r0 + r, gj = c0 + c;
        a[r][c] = (gi < n && gj < n) ? h[(size_t)gi * ldh + gj] : 0.0;
        const int hi_ = c0 + r, hj = r0 + c;
        b[r][c] = (hi_ < n && hj < n) ? h[(size_t)hi_ * ldh + hj] : 0.0;
    }
    __syncthreads();
    const double emin = st->emin, emax = st->emax;
    double span = emax - emin;
    if (!(span > 0.0)) span = 1.0;   // degenerate spectrum: every eigenvalue maps to ~1
    const double w0 = -1.0 / span, b0 = emax / span;
    const bool diag = (I == J);
    double tr = 0.0, fr = 0.0, as = 0.0;
    // pass 1: the tile itself, row-major (coalesced); the value is kept in `a`
    for (int idx = t; idx < kInitTile * kInitTile; idx += kThreads) {
        const int r = idx / kInitTile, c = idx % kInitTile;
        const int gi = r0 + r, gj = c0 + c;
        const double x = a[r][c], y = b[c][r];
        const double hs = 0.5 * (x + y);
        as = fmax(as, fabs(x - y));
        double v = 0.0;
        if (gi < n && gj < n) v = w0 * hs + (gi == gj ? b0 : 0.0);
        const St vs = (St)v;
        s_out[(size_t)gi * np + gj] = vs;
        if (kSplit) {
            const float xs = (float)vs * in_scale;
            const T16 h0 = (T16)xs;
            const T16 h1 = (T16)(xs - (float)h0);
            p0[(size_t)gi * plane_ld(np) + gj] = h0;
            p1[(size_t)gi * plane_ld(np) + gj] = h1;
        }
        const double vd = (double)vs;
        if (gi == gj) tr += vd;
        fr += (diag ? 1.0 : 2.0) * vd * vd;
        a[r][c] = vd;
    }
    __syncthreads();
    // pass 2: the mirror tile (J, I), row-major over its rows (coalesced)
    if (!diag) {
        for (int idx = t; idx < kInitTile * kInitTile; idx += kThreads) {
            const int r = idx / kInitTile, c = idx % kInitTile;   // mirror element (c0 + r, r0 + c)
            const St vs = (St)a[c][r];
            const size_t off = (size_t)(c0 + r) * np + (r0 + c);
            s_out[off] = vs;
            if (kSplit) {
                const float xs = (float)vs * in_scale;
                const T16 h0 = (T16)xs;
                const T16 h1 = (T16)(xs - (float)h0);
                const size_t poff = (size_t)(c0 + r) * plane_ld(np) + (r0 + c);
                p0[poff] = h0;
                p1[poff] = h1;
            }
        }
    }
    double v2[2] = {tr, fr};
    block_sum<2>(v2, &red[0][0]);
    // max-reduction of the asymmetry (order independent)
    __syncthreads();
    red[2][t] = as;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[2][t] = fmax(red[2][t], red[2][t + w]);
        __syncthreads();
    }
    if (t == 0) {
        parts[3 * bid + 0] = v2[0];
        parts[3 * bid + 1] = v2[1];
        parts[3 * bid + 2] = red[2][0];
    }
}

// ---------------------------------------------------------------------------------
// Alg. 1 control for layer `layer` (n).  The partial sums describe S_{n-1}:
//   N_S = Tr S_{n-1}           (measured, FP64 sum of the stored diagonal)
//   N_X = Tr S_{n-1}^2 = ||S_{n-1}||_F^2   (S symmetric; FP64 sum of exact squares)
// so IdErr_n = Tr[S_{n-1} - S_{n-1}^2] is known before X_n is formed, and layer n's
// kernels receive sigma_n as coefficients (or a skip flag once a test has held).
// ---------------------------------------------------------------------------------
// Accelerated layers stop once both tracked bounds are this close to their fixed points.
constexpr double kAccSwitch = 0.01;

// One accelerated layer (Sec. Accelerated Deep-NN SP2) from the bounds l < h of the
// unoccupied / occupied eigenvalues of S_{n-1} in [0, 1].  The x^2 side applies
// ((x - v)/(1 - v))^2: the images of [0, l] and [h, 1] are [0, (l - v)^2/(1 - v)^2] and
// [(h - v)^2/(1 - v)^2, 1] for 0 <= v <= l/2, and their separation peaks at
// v = h + l - 1, hence v = clamp(h + l - 1, 0, l/2).  The 2x - x^2 side is its mirror image
// 1 - ((1 - w - x)/(1 - w))^2 with w = clamp(1 - h - l, 0, (1 - h)/2).  The wider
// separation wins (the x^2 side on a tie).  Writes Y = a X^2 + b X + c I, the real
// weight sigma_n = +-1/(1 - 2v) and the bounds after the layer.
__device__ inline void accelerated_choice(double l, double h, int* sgn, double* a, double* b, double* c,
                                          double* sigma, double* l1, double* h1) {
    const double v = fmin(fmax(h + l - 1.0, 0.0), 0.5 * l);
    const double dv = 1.0 - v;
    const double ld = (l - v) * (l - v) / (dv * dv), hd = (h - v) * (h - v) / (dv * dv);
    const double w = fmin(fmax(1.0 - h - l, 0.0), 0.5 * (1.0 - h));
    const double dw = 1.0 - w;
    const double lu = 1.0 - (dw - l) * (dw - l) / (dw * dw), hu = 1.0 - (dw - h) * (dw - h) / (dw * dw);
    if (hd - ld >= hu - lu) {
        *sgn = 1;
        *a = 1.0 / (dv * dv);
        *b = -2.0 * v / (dv * dv);
        *c = v * v / (dv * dv);
        *sigma = 1.0 / (1.0 - 2.0 * v);
        *l1 = ld;
        *h1 = hd;
    } else {
        *sgn = -1;
        *a = -1.0 / (dw * dw);
        *b = 2.0 / dw;
        *c = 0.0;
        *sigma = -1.0 / (1.0 - 2.0 * w);
        *l1 = lu;
        *h1 = hu;
    }
}

__device__ __forceinline__ void control_body(DevState* st, const double* __restrict__ parts,
                                                      int nparts, int stride, int layer,
                                                      volatile int* __restrict__ host_flag) {
    __shared__ double sh[2 * kThreads];
    if (st->stopped) {
        if (threadIdx.x == 0) {
            st->skip = 1;
            if (host_flag) *host_flag = 1;
        }
        return;
    }
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
        v[0] += parts[(size_t)stride * i];
        v[1] += parts[(size_t)stride * i + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x != 0) return;
    const int n = layer;
    const double n_s = v[0], n_x = v[1];
    const double e = n_s - n_x;
    const int sp = st->sigma[n - 1];
    st->ns[n] = n_s;
    st->nx[n] = n_x;
    st->iderr[n] = e;
    bool stop = false, conv = false;
    if (!isfinite(n_s) || !isfinite(n_x)) {
        st->status = SP2_ENONFINITE;
        stop = true;
    } else if (n > st->max_layers) {
        stop = true;   // S_{max_layers} is refined; status set by the final check
    } else {
        if (n == 1 && st->accel) {
            // rescaled bounds of S_0 = (emax I - H)/(emax - emin): the order is reversed
            const double span = st->emax - st->emin;
            const double l0 = (st->emax - st->lumo) / span, h0 = (st->emax - st->homo) / span;
            if (0.0 <= l0 && l0 < h0 && h0 <= 1.0) {
                st->acc_l = l0;
                st->acc_h = h0;
            } else {
                st->accel = 0;
            }
        }
        // Interval consistency: inside the gap, exactly n_occ eigenvalues start in [h, 1] and
        // every layer maps the tracked intervals onto the next ones, so Tr S_{n-1} lies within
        // (N - n_occ) l + n_occ (1 - h) of n_occ; a larger distance (beyond rounding) means the
        // interval was not inside the gap.
        if (st->accel && st->gap_violation == 0) {
            const double nn = (double)st->n, occ = (double)st->n_occ;
            const double noise = (st->precision == SP2_FP64 ? 1e-8 : 1e-3) * nn;
            if (fabs(n_s - occ) > (nn - occ) * st->acc_l + occ * (1.0 - st->acc_h) + noise) st->gap_violation = n;
        }
        int s;
        double ca, cb, cc, sc;
        if (st->accel && fmax(st->acc_l, 1.0 - st->acc_h) > kAccSwitch) {
            double l1, h1;
            accelerated_choice(st->acc_l, st->acc_h, &s, &ca, &cb, &cc, &sc, &l1, &h1);
            st->acc_l = l1;
            st->acc_h = h1;
            st->acc_layers = n;
        } else {
            const double occ = (double)st->n_occ;
            const double val = fabs(2.0 * n_s - n_x - occ) - fabs(n_x - occ) - sp * st->eps;
            s = val > 0.0 ? 1 : (val < 0.0 ? -1 : (sp != 0 ? -sp : 1));
            ca = s > 0 ? 1.0 : -1.0;
            cb = s > 0 ? 0.0 : 2.0;
            cc = 0.0;
            sc = (double)s;
            if (st->accel) {   // the tracked intervals follow the SP2 maps too
                const double l = st->acc_l, h = st->acc_h;
                st->acc_l = s > 0 ? l * l : 2.0 * l - l * l;
                st->acc_h = s > 0 ? h * h : 2.0 * h - h * h;
            }
        }
        st->sigma[n] = (signed char)s;
        st->sigma_c[n] = sc;
        // the alternation test bounds IdErr_n by the two layers before it; it is taken
        // only when both were layers of Alg. 1
        if (e <= 0.0) conv = true;
        else if (n > 2 && n >= st->acc_layers + 3 && st->sigma[n - 1] != st->sigma[n - 2] &&
                 e > 4.5 * st->iderr[n - 2] * st->iderr[n - 2])
            conv = true;
        if (!conv) {
            st->coef[0] = (float)ca;
            st->coef[1] = (float)cb;
            st->coef[2] = (float)cc;
            st->coef64[0] = ca;
            st->coef64[1] = cb;
            st->coef64[2] = cc;
            st->skip = 0;
            st->layers = n;
            st->ran = n;
            return;
        }
        stop = true;
    }
    // stopping: refine S_{n-1}
    st->stopped = 1;
    if (host_flag) *host_flag = 1;   // lets a host that polls stop enqueueing layers
    st->skip = 1;
    st->converged = conv ? 1 : 0;
    st->layers = (conv || !isfinite(n_s) || !isfinite(n_x)) ? n : n - 1;
    const int last = st->sigma[n - 1];
    const int fs = last != 0 ? -last : 1;
    st->first_sign = fs;
    st->refine_src = (n - 1) & 1;
    // first composed step, then the opposite one (Eq. Refinement)
    const float sq[3] = {1.f, 0.f, 0.f}, pr[3] = {-1.f, 2.f, 0.f};
    for (int i = 0; i < 3; ++i) {
        st->rcoef[0][i] = fs > 0 ? sq[i] : pr[i];
        st->rcoef[1][i] = fs > 0 ? pr[i] : sq[i];
    }
    (void)stop;
}

template <typename Src>
__device__ __forceinline__ void select_body(const DevState* __restrict__ st, const Src* __restrict__ s0,
                                                         const Src* __restrict__ s1, double* __restrict__ out,
                                                         int ld_out, int n_valid, int np, int bid, int nbid) {
    const Src* src = st->refine_src ? s1 : s0;
    const size_t total = (size_t)n_valid * n_valid;
    for (size_t idx = (size_t)bid * kThreads + threadIdx.x; idx < total;
         idx += (size_t)nbid * kThreads) {
        const int i = (int)(idx / n_valid), j = (int)(idx % n_valid);
        out[(size_t)i * ld_out + j] = (double)src[(size_t)i * np + j];
    }
}

// Rows per block of the final reductions.
constexpr int kStatRows = 4;

__device__ __forceinline__ void dstats_body(const double* __restrict__ d, int ldd,
                                                     const double* __restrict__ h, int ldh, int n,
                                                     double* __restrict__ parts, int bid) {
    __shared__ double sh[3 * kThreads];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double v[3] = {0.0, 0.0, 0.0};
    for (int rr = wave; rr < kStatRows; rr += kThreads / 64) {
        const int i = bid * kStatRows + rr;
        if (i >= n) break;
        const double* dr = d + (size_t)i * ldd;
        const double* hr = h ? h + (size_t)i * ldh : nullptr;
        for (int j = lane; j < n; j += 64) {
            const double x = dr[j];
            if (j == i) v[0] += x;
            v[1] += x * x;
            if (hr) v[2] += x * hr[j];
        }
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        parts[3 * bid + 0] = v[0];
        parts[3 * bid + 1] = v[1];
        parts[3 * bid + 2] = v[2];
    }
}

__device__ __forceinline__ void finalize_body(DevState* st, const double* __restrict__ dparts, int nd,
                                                       const double* __restrict__ iparts, int ni) {
    __shared__ double sh[3 * kThreads];
    __shared__ double mx[kThreads];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nd; i += kThreads) {
        v[0] += dparts[3 * i];
        v[1] += dparts[3 * i + 1];
        v[2] += dparts[3 * i + 2];
    }
    block_sum<3>(v, sh);
    double a = 0.0;
    for (int i = threadIdx.x; i < ni; i += kThreads) a = fmax(a, iparts[3 * i + 2]);
    mx[threadIdx.x] = a;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    st->trace_d = v[0];
    st->frob_d = v[1];
    st->energy = st->want_energy ? v[2] : 0.0;
    st->asym = mx[0];
    int status = st->status;
    const double scale = fmax(fmax(fabs(st->emin), fabs(st->emax)), 1.0);
    if (status == SP2_OK && !(mx[0] <= 1e-12 * scale)) status = SP2_EINVAL;
    if (status == SP2_OK) {
        const double idem = v[0] - v[1];
        if (!isfinite(v[0]) || !isfinite(v[1])) status = SP2_ENONFINITE;
        else if (st->gap_violation) status = SP2_ENOTIDEMP;   // the interval was not inside the gap
        else if (!st->converged) status = SP2_ENOCONV;
        else if (!(fabs(v[0] - st->n_occ) <= st->tol_tr) || !(fabs(idem) <= st->tol_id)) status = SP2_ENOTIDEMP;
    }
    st->status = status;
}

__global__ __launch_bounds__(kThreads) void k_fill(double* __restrict__ d, int ldd, int n, double diag) {
    const size_t total = (size_t)n * n;
    for (size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * kThreads) {
        const int i = (int)(idx / n), j = (int)(idx % n);
        d[(size_t)i * ldd + j] = (i == j) ? diag : 0.0;
    }
}

template <typename T16>
__global__ __launch_bounds__(kThreads) void k_split(const float* __restrict__ x, T16* __restrict__ p0,
                                                    T16* __restrict__ p1, int np, float in_scale) {
    // x: np x np (row stride np); planes: row stride plane_ld(np)
    const size_t total = (size_t)np * np, pld = (size_t)plane_ld(np);
    for (size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * kThreads) {
        const float xs = x[idx] * in_scale;
        const T16 h0 = (T16)xs;
        const size_t o = (idx / np) * pld + idx % np;
        p0[o] = h0;
        p1[o] = (T16)(xs - (float)h0);
    }
}

__global__ __launch_bounds__(kThreads) void k_sum_parts(const double* __restrict__ parts, int nparts,
                                                        double* __restrict__ out2) {
    __shared__ double sh[2 * kThreads];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
        v[0] += parts[2 * i];
        v[1] += parts[2 * i + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        out2[0] = v[0];
        out2[1] = v[1];
    }
}

__global__ void k_set3(float* dst, float a, float b, float c) {
    if (threadIdx.x == 0) {
        dst[0] = a;
        dst[1] = b;
        dst[2] = c;
    }
}

__global__ void k_zero_ints(int* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Finite-temperature read-out D = (1 - c_0) I + c_0 S_0 - sum_{k>=1} c_k X_k accumulated in
// FP64 over the padded matrix: first = 1 sets acc = a X + diag I, otherwise acc += a X.
// Two elements per thread and iteration (n_p is a multiple of 64).
template <typename St>
__global__ __launch_bounds__(kThreads) void k_readout(double* __restrict__ acc, const St* __restrict__ x, int np,
                                                      double a, double diag, int first) {
    const size_t total = (size_t)np * np / 2;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < total; q += (size_t)gridDim.x * kThreads) {
        const size_t idx = 2 * q;
        const int i = (int)(idx / np), j = (int)(idx % np);
        double v0 = a * (double)x[idx], v1 = a * (double)x[idx + 1];
        if (first) {
            if (i == j) v0 += diag;
            if (i == j + 1) v1 += diag;
            acc[idx] = v0;
            acc[idx + 1] = v1;
        } else {
            acc[idx] += v0;
            acc[idx + 1] += v1;
        }
    }
}

// n x n leading block of the padded accumulator into D (leading dimension ldd)
__global__ __launch_bounds__(kThreads) void k_copy_out(const double* __restrict__ acc, int np,
                                                       double* __restrict__ d, int ldd, int n) {
    const size_t total = (size_t)n * n;
    for (size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (size_t)gridDim.x * kThreads) {
        const int i = (int)(idx / n), j = (int)(idx % n);
        d[(size_t)i * ldd + j] = acc[(size_t)i * np + j];
    }
}

// Up to kMaxCoefs floats passed by value into device memory (kernel arguments are part of
// the launch, so this works inside a captured stream as well).
constexpr int kMaxCoefs = 3 * SP2_MAX_LAYERS;
template <typename T>
struct CoefBlock {
    T v[kMaxCoefs];
};
template <typename T>
__global__ void k_store_coefs(T* __restrict__ dst, CoefBlock<T> b, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = b.v[i];
}

// Fixed-order sum of per-block triples (Tr part, ||.||_F^2 part, Tr[DH] part).
__global__ __launch_bounds__(kThreads) void k_sum3(const double* __restrict__ parts, int nparts,
                                                   double* __restrict__ out3) {
    __shared__ double sh[3 * kThreads];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
        v[0] += parts[3 * i];
        v[1] += parts[3 * i + 1];
        v[2] += parts[3 * i + 2];
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        out3[0] = v[0];
        out3[1] = v[1];
        out3[2] = v[2];
    }
}

// Occupation 0 or n: no recursion is run; the state records a converged call of 0 layers.
__global__ void k_mark_trivial(DevState* st) {
    if (threadIdx.x == 0) {
        st->stopped = 1;
        st->converged = 1;
        st->layers = 0;
        st->skip = 1;
    }
}

__global__ __launch_bounds__(kThreads) void k_gershgorin(const double* __restrict__ h, int ldh, int n,
                                                         double* __restrict__ blk) {
    gershgorin_body(h, ldh, n, blk, blockIdx.x);
}
__global__ __launch_bounds__(kThreads) void k_bounds(DevState* st, const double* __restrict__ blk, int nblk) {
    bounds_body(st, blk, nblk);
}
__global__ __launch_bounds__(kThreads) void k_control(DevState* st, const double* __restrict__ parts, int nparts,
                                                      int stride, int layer, volatile int* __restrict__ host_flag) {
    control_body(st, parts, nparts, stride, layer, host_flag);
}
__global__ __launch_bounds__(kThreads) void k_finalize(DevState* st, const double* __restrict__ dparts, int nd,
                                                       const double* __restrict__ iparts, int ni) {
    finalize_body(st, dparts, nd, iparts, ni);
}
template <typename St, typename T16, bool kSplit>
__global__ __launch_bounds__(kThreads) void k_init(const double* __restrict__ h, int ldh,
                                                   const DevState* __restrict__ st, St* __restrict__ s_out,
                                                   T16* __restrict__ p0, T16* __restrict__ p1, float in_scale,
                                                   double* __restrict__ parts) {
    init_body<St, T16, kSplit>(h, ldh, st, s_out, p0, p1, in_scale, parts, blockIdx.x);
}
template <typename Src>
__global__ __launch_bounds__(kThreads) void k_select_f64(const DevState* __restrict__ st, const Src* __restrict__ s0,
                                                         const Src* __restrict__ s1, double* __restrict__ out,
                                                         int ld_out, int n_valid, int np) {
    select_body<Src>(st, s0, s1, out, ld_out, n_valid, np, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kThreads) void k_dstats(const double* __restrict__ d, int ldd,
                                                     const double* __restrict__ h, int ldh, int n,
                                                     double* __restrict__ parts) {
    dstats_body(d, ldd, h, ldh, n, parts, blockIdx.x);
}

// ---------------------------------------------------------------------------------
// Batched versions: one launch covers all problems; blocks are split between problems
// by the prefix offsets `offs`, single-block steps use one block per problem.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_gershgorin_g(const BatchProblem* __restrict__ pr,
                                                           const int* __restrict__ offs, int np_) {
    const int p = find_group(offs, np_, blockIdx.x);
    gershgorin_body(pr[p].h, pr[p].ldh, pr[p].n, pr[p].gersh, blockIdx.x - offs[p]);
}
__global__ __launch_bounds__(kThreads) void k_bounds_g(const BatchProblem* __restrict__ pr) {
    const BatchProblem& q = pr[blockIdx.x];
    if (q.st->have_bounds) return;
    bounds_body(q.st, q.gersh, q.gersh_blocks);
}
template <typename T16, bool kSplit>
__global__ __launch_bounds__(kThreads) void k_init_g(const BatchProblem* __restrict__ pr,
                                                     const int* __restrict__ offs, int np_) {
    const int p = find_group(offs, np_, blockIdx.x);
    const BatchProblem& q = pr[p];
    init_body<float, T16, kSplit>(q.h, q.ldh, q.st, (float*)q.s[0], (T16*)q.pl[0][0], (T16*)q.pl[0][1],
                                  q.in_scale, q.init_parts, blockIdx.x - offs[p]);
}
__global__ __launch_bounds__(kThreads) void k_control_g(const BatchProblem* __restrict__ pr, int layer) {
    const BatchProblem& q = pr[blockIdx.x];
    if (layer == 1) control_body(q.st, q.init_parts, q.init_tiles, 3, layer, nullptr);
    else control_body(q.st, q.main_parts, q.main_tiles, 2, layer, nullptr);
}
__global__ __launch_bounds__(kThreads) void k_select_g(const BatchProblem* __restrict__ pr, int per_problem) {
    const int p = blockIdx.x / per_problem;
    const BatchProblem& q = pr[p];
    select_body<float>(q.st, (const float*)q.s[0], (const float*)q.s[1], q.s64, q.np, q.np, q.np,
                       blockIdx.x - p * per_problem, per_problem);
}
__global__ __launch_bounds__(kThreads) void k_dstats_g(const BatchProblem* __restrict__ pr,
                                                       const int* __restrict__ offs, int np_) {
    const int p = find_group(offs, np_, blockIdx.x);
    const BatchProblem& q = pr[p];
    dstats_body(q.d, q.ldd, q.want_energy ? q.h : nullptr, q.ldh, q.n, q.dstats, blockIdx.x - offs[p]);
}
__global__ __launch_bounds__(kThreads) void k_finalize_g(const BatchProblem* __restrict__ pr) {
    const BatchProblem& q = pr[blockIdx.x];
    finalize_body(q.st, q.dstats, q.dstats_blocks, q.init_parts, q.init_tiles);
}

// Device state of problem blockIdx.x between its region and slot blockIdx.x of a
// contiguous staging array (to_regions: staging -> region), so that a batched call moves
// all the states with one host transfer each way.
static_assert(sizeof(DevState) % 4 == 0, "states move as 32-bit words");
__global__ __launch_bounds__(64) void k_state_copy_g(const BatchProblem* __restrict__ pr, DevState* stage,
                                                     int to_regions) {
    unsigned* r = (unsigned*)pr[blockIdx.x].st;
    unsigned* g = (unsigned*)(stage + blockIdx.x);
    for (int i = threadIdx.x; i < (int)(sizeof(DevState) / 4); i += 64) {
        if (to_regions) r[i] = g[i];
        else g[i] = r[i];
    }
}

inline int grid_for(size_t total) {
    size_t g = (total + kThreads - 1) / kThreads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

// ------------------------------------------------------------------------------ launchers
hipError_t launch_state_init(DevState* st, const DevState& in, hipStream_t s) {
    StateParams p;
    p.n = in.n;
    p.n_occ = in.n_occ;
    p.np = in.n_padded;
    p.max_layers = in.max_layers;
    p.precision = in.precision;
    p.tile = in.tile;
    p.have_bounds = in.have_bounds;
    p.want_energy = in.want_energy;
    p.eps = in.eps;
    p.tol_tr = in.tol_tr;
    p.tol_id = in.tol_id;
    p.emin = in.emin;
    p.emax = in.emax;
    p.accel = in.accel;
    p.homo = in.homo;
    p.lumo = in.lumo;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(kThreads), 0, s, st, p);
    return hipGetLastError();
}

int gershgorin_blocks(int n) { return (n + kGershRowsPerBlock - 1) / kGershRowsPerBlock; }

hipError_t launch_gershgorin(const double* h, int ldh, int n, double* blk, int* nblk, hipStream_t s) {
    *nblk = gershgorin_blocks(n);
    hipLaunchKernelGGL(k_gershgorin, dim3(*nblk), dim3(kThreads), 0, s, h, ldh, n, blk);
    return hipGetLastError();
}

hipError_t launch_bounds(DevState* st, const double* blk, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_bounds, dim3(1), dim3(kThreads), 0, s, st, blk, nblk);
    return hipGetLastError();
}

int init_tiles(int np) {
    const int T = np / kInitTile;
    return ntiles_upper(T);
}

hipError_t launch_init_np(const double* h, int ldh, DevState* st, int np, int precision, void* s_out, void* p0,
                          void* p1, int scale_log2, double* parts, hipStream_t s) {
    const int nt = init_tiles(np);
    const float in_scale = ldexpf(1.f, scale_log2);
    switch (precision) {
        case SP2_FP64:
            hipLaunchKernelGGL((k_init<double, _Float16, false>), dim3(nt), dim3(kThreads), 0, s, h, ldh, st,
                               (double*)s_out, (_Float16*)nullptr, (_Float16*)nullptr, 1.f, parts);
            break;
        case SP2_FP32:
            hipLaunchKernelGGL((k_init<float, _Float16, false>), dim3(nt), dim3(kThreads), 0, s, h, ldh, st,
                               (float*)s_out, (_Float16*)nullptr, (_Float16*)nullptr, 1.f, parts);
            break;
        case SP2_FP16X2:
            hipLaunchKernelGGL((k_init<float, _Float16, true>), dim3(nt), dim3(kThreads), 0, s, h, ldh, st,
                               (float*)s_out, (_Float16*)p0, (_Float16*)p1, in_scale, parts);
            break;
        case SP2_BF16X2:
            hipLaunchKernelGGL((k_init<float, __bf16, true>), dim3(nt), dim3(kThreads), 0, s, h, ldh, st,
                               (float*)s_out, (__bf16*)p0, (__bf16*)p1, in_scale, parts);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_control_stride(DevState* st, const double* parts, int nparts, int stride, int layer,
                                 int* host_flag, hipStream_t s) {
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kThreads), 0, s, st, parts, nparts, stride, layer,
                       (volatile int*)host_flag);
    return hipGetLastError();
}

hipError_t launch_select_f64(const DevState* st, const void* s0, const void* s1, int state_f64, double* out,
                             int ld_out, int n_valid, int np, hipStream_t s) {
    const int g = grid_for((size_t)n_valid * n_valid);
    if (state_f64)
        hipLaunchKernelGGL((k_select_f64<double>), dim3(g), dim3(kThreads), 0, s, st, (const double*)s0,
                           (const double*)s1, out, ld_out, n_valid, np);
    else
        hipLaunchKernelGGL((k_select_f64<float>), dim3(g), dim3(kThreads), 0, s, st, (const float*)s0,
                           (const float*)s1, out, ld_out, n_valid, np);
    return hipGetLastError();
}

int dstats_blocks(int n) { return (n + kStatRows - 1) / kStatRows; }

hipError_t launch_dstats(const double* d, int ldd, const double* h, int ldh, int n, double* parts, int* nparts,
                         hipStream_t s) {
    *nparts = dstats_blocks(n);
    hipLaunchKernelGGL(k_dstats, dim3(*nparts), dim3(kThreads), 0, s, d, ldd, h, ldh, n, parts);
    return hipGetLastError();
}

hipError_t launch_finalize(DevState* st, const double* dparts, int nd, const double* iparts, int ni,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, st, dparts, nd, iparts, ni);
    return hipGetLastError();
}

hipError_t launch_fill(double* d, int ldd, int n, double diag, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for((size_t)n * n)), dim3(kThreads), 0, s, d, ldd, n, diag);
    return hipGetLastError();
}

hipError_t launch_split(const float* x, void* p0, void* p1, int np, int precision, int scale_log2,
                        hipStream_t s) {
    const size_t total = (size_t)np * np;
    const float sc = ldexpf(1.f, scale_log2);
    if (precision == SP2_FP16X2)
        hipLaunchKernelGGL((k_split<_Float16>), dim3(grid_for(total)), dim3(kThreads), 0, s, x, (_Float16*)p0,
                           (_Float16*)p1, np, sc);
    else if (precision == SP2_BF16X2)
        hipLaunchKernelGGL((k_split<__bf16>), dim3(grid_for(total)), dim3(kThreads), 0, s, x, (__bf16*)p0,
                           (__bf16*)p1, np, sc);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sum_parts(const double* parts, int nparts, double* out2, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kThreads), 0, s, parts, nparts, out2);
    return hipGetLastError();
}

}  // namespace sp2

namespace sp2 {
hipError_t launch_set3(float* dst, float a, float b, float c, hipStream_t s) {
    hipLaunchKernelGGL(k_set3, dim3(1), dim3(64), 0, s, dst, a, b, c);
    return hipGetLastError();
}
hipError_t launch_readout(int precision, double* acc, const void* x, int np, double a, double diag, int first,
                          hipStream_t s) {
    const size_t pairs = (size_t)np * np / 2;
    size_t g = (pairs + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    if (precision == SP2_FP64)
        hipLaunchKernelGGL(k_readout<double>, dim3((unsigned)g), dim3(kThreads), 0, s, acc, (const double*)x, np, a,
                           diag, first);
    else
        hipLaunchKernelGGL(k_readout<float>, dim3((unsigned)g), dim3(kThreads), 0, s, acc, (const float*)x, np, a,
                           diag, first);
    return hipGetLastError();
}
hipError_t launch_copy_out(const double* acc, int np, double* d, int ldd, int n, hipStream_t s) {
    size_t g = ((size_t)n * n + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_copy_out, dim3((unsigned)g), dim3(kThreads), 0, s, acc, np, d, ldd, n);
    return hipGetLastError();
}
hipError_t launch_store_coefs(float* dst, const double* vals, int count, hipStream_t s) {
    if (count < 0 || count > kMaxCoefs) return hipErrorInvalidValue;
    CoefBlock<float> b;
    for (int i = 0; i < kMaxCoefs; ++i) b.v[i] = i < count ? (float)vals[i] : 0.f;
    hipLaunchKernelGGL(k_store_coefs<float>, dim3(1), dim3(128), 0, s, dst, b, count);
    return hipGetLastError();
}
hipError_t launch_store_coefs64(double* dst, const double* vals, int count, hipStream_t s) {
    if (count < 0 || count > kMaxCoefs) return hipErrorInvalidValue;
    CoefBlock<double> b;
    for (int i = 0; i < kMaxCoefs; ++i) b.v[i] = i < count ? vals[i] : 0.0;
    hipLaunchKernelGGL(k_store_coefs<double>, dim3(1), dim3(128), 0, s, dst, b, count);
    return hipGetLastError();
}
hipError_t launch_sum3(const double* parts, int nparts, double* out3, hipStream_t s) {
    hipLaunchKernelGGL(k_sum3, dim3(1), dim3(kThreads), 0, s, parts, nparts, out3);
    return hipGetLastError();
}
hipError_t launch_zero_ints(int* p, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_ints, dim3(4), dim3(256), 0, s, p, count);
    return hipGetLastError();
}
hipError_t launch_mark_trivial(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_mark_trivial, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}
}  // namespace sp2

namespace sp2 {
hipError_t launch_batch_gershgorin(const BatchProblem* pr, const int* offs, int nprob, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_gershgorin_g, dim3(blocks), dim3(kThreads), 0, s, pr, offs, nprob);
    return hipGetLastError();
}
hipError_t launch_batch_bounds(const BatchProblem* pr, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_bounds_g, dim3(nprob), dim3(kThreads), 0, s, pr);
    return hipGetLastError();
}
hipError_t launch_batch_init(int precision, const BatchProblem* pr, const int* offs, int nprob, int blocks,
                             hipStream_t s) {
    if (precision == SP2_FP16X2)
        hipLaunchKernelGGL((k_init_g<_Float16, true>), dim3(blocks), dim3(kThreads), 0, s, pr, offs, nprob);
    else if (precision == SP2_BF16X2)
        hipLaunchKernelGGL((k_init_g<__bf16, true>), dim3(blocks), dim3(kThreads), 0, s, pr, offs, nprob);
    else if (precision == SP2_FP32)
        hipLaunchKernelGGL((k_init_g<_Float16, false>), dim3(blocks), dim3(kThreads), 0, s, pr, offs, nprob);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
hipError_t launch_batch_control(const BatchProblem* pr, int nprob, int layer, hipStream_t s) {
    hipLaunchKernelGGL(k_control_g, dim3(nprob), dim3(kThreads), 0, s, pr, layer);
    return hipGetLastError();
}
hipError_t launch_batch_select(const BatchProblem* pr, int nprob, int per_problem, hipStream_t s) {
    hipLaunchKernelGGL(k_select_g, dim3(nprob * per_problem), dim3(kThreads), 0, s, pr, per_problem);
    return hipGetLastError();
}
hipError_t launch_batch_dstats(const BatchProblem* pr, const int* offs, int nprob, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_dstats_g, dim3(blocks), dim3(kThreads), 0, s, pr, offs, nprob);
    return hipGetLastError();
}
hipError_t launch_batch_finalize(const BatchProblem* pr, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_g, dim3(nprob), dim3(kThreads), 0, s, pr);
    return hipGetLastError();
}
hipError_t launch_batch_states(const BatchProblem* pr, DevState* stage, int nprob, int to_regions, hipStream_t s) {
    hipLaunchKernelGGL(k_state_copy_g, dim3(nprob), dim3(64), 0, s, pr, stage, to_regions);
    return hipGetLastError();
}
}  // namespace sp2
