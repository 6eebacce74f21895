// Host side of libsp2: argument checks, workspace layout and the launch sequence of
// Alg. 1.  Control stays on the device: every layer is a control kernel (IdErr_n,
// sigma_n, stopping tests) followed by a squaring kernel that reads its coefficients
// and a skip flag from the device state, so the host enqueues the whole recursion
// without reading anything back.
#include "sp2_internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

using namespace sp2;

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

struct Opts {
    int precision, max_layers, have_bounds, refine, scale_log2, want_energy, tile, kernel;
    int tile_ref;   // FP64 refinement tile, 0 = by size (set only by the batched path)
    int accelerate;
    double eps, emin, emax, homo, lumo;
};

bool read_opts(const sp2_options* o, Opts* r) {
    sp2_options d;
    sp2_default_options(&d);
    if (!o) o = &d;
    r->precision = o->precision;
    r->max_layers = o->max_layers == 0 ? 100 : o->max_layers;
    r->have_bounds = o->have_bounds;
    r->refine = o->refine;
    r->want_energy = o->want_energy;
    r->tile = o->tile;
    r->kernel = o->kernel;
    r->tile_ref = 0;
    r->eps = o->eps;
    r->emin = o->emin;
    r->emax = o->emax;
    r->accelerate = o->accelerate != 0;
    r->homo = o->homo;
    r->lumo = o->lumo;
    if (r->accelerate && !(isfinite(r->homo) && isfinite(r->lumo) && r->homo < r->lumo)) return false;
    if (r->precision < SP2_FP64 || r->precision > SP2_BF16X2) return false;
    const bool split = r->precision == SP2_FP16X2 || r->precision == SP2_BF16X2;
    r->scale_log2 = o->scale_log2 < 0 ? (r->precision == SP2_FP16X2 ? 12 : 0) : o->scale_log2;
    if (!split) r->scale_log2 = 0;
    if (r->scale_log2 > (r->precision == SP2_FP16X2 ? 14 : 60)) return false;
    if (r->max_layers < 1 || r->max_layers >= SP2_MAX_LAYERS) return false;
    if (r->tile != 0 && r->tile != 64 && r->tile != 128 && r->tile != 256) return false;
    if (r->tile == 256 && !split) return false;
    if (r->kernel < 0 || (r->kernel > 1 + kSkVariants && r->kernel != 8)) return false;
    if (r->precision == SP2_FP64 && r->kernel > 5) return false;
    if (!isfinite(r->eps)) return false;
    if (r->have_bounds && !(isfinite(r->emin) && isfinite(r->emax) && r->emax > r->emin)) return false;
    return true;
}

struct Plan {
    int n, np, precision, tile_main, tile_ref, scale_log2;
    bool split;
    int init_tiles, main_T, main_tiles, main_per, ref_T, ref_tiles, ref_per, gersh_blocks, dstats_blocks;
    int kernel;       // request: 0 = automatic, 1 = one workgroup per tile, 2.. = persistent variant - 2
    bool sk_capable;  // stream-K buffers are part of the workspace
    size_t off_init_parts, off_main_parts, off_gersh, off_dstats, off_s[2], off_p[2][2], off_s64, off_y;
    size_t off_sk_partial, off_sk_counter, off_f64_partial, off_f64_counter, total;
    bool f64_sk;      // persistent FP64 layer buffers reserved
};

// The persistent (whole rounds + split tail) schedule needs a tile of 128 or 256 in a
// split mode; kernel 1 asks for the one-workgroup-per-tile schedule.  The automatic choice
// (one layer, split included, MI355X): 128 tiles persistent from n_p = 3072 (n = 3072:
// 0.156 vs 0.167 ms per tile; 4096: 0.289-0.302 vs 0.339-0.347 ms), one workgroup per tile
// below; 256 tiles one workgroup per tile below n_p = 6144 (n = 5120: 0.486 vs 0.594 ms
// persistent) and persistent from there (6144: 0.807 vs 0.937 ms).
bool sk_wanted(bool split, int tile, int kernel, int np) {
    if (!split || tile < 128 || kernel == 1 || kernel == 8) return false;
    if (kernel != 0) return true;
    return tile == 128 ? np >= 3072 : np >= 6144;
}

// Persistent variant used when the caller leaves the choice open (index into the
// per-tile variant table of the kernel), the fastest measured on MI355X: for 256 tiles
// 8 waves with 32-half slices and the rolling fragment pipeline (one layer, split
// included, at n = 8192: 1.69 ms against 1.74 ms with two fragment sets; n = 16384: 10.49
// against 11.02 ms); for 128 tiles the 64-half slices with the rolling pipeline (n = 4096:
// 0.289 ms against 0.379 ms with two fragment sets).
int sk_auto_variant(int tile) { return tile == 256 ? 5 : 4; }

// Resolves the squaring schedule for this device; false = one workgroup per tile.
bool sk_resolve(const Plan& p, StreamK* sk, int* variant) {
    if (!p.sk_capable) return false;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    int per_cu = 0, T = 0, nt = 0;
    *variant = p.kernel >= 2 ? p.kernel - 2 : sk_auto_variant(p.tile_main);
    return square_sk_plan(p.tile_main, *variant, p.np, cus, &per_cu, sk, &T, &nt);
}

// Split layer with one workgroup per tile: the direct-to-LDS pipeline for 128/256 tiles
// (kernel option 0/1), the register-staged kernel for 64 tiles or kernel option 8.  On
// 128 tiles a single problem takes 64-half slices (one workgroup per CU; one layer at
// n = 2048: 0.079 against 0.089 ms with 32-half slices and two workgroups per CU, 6144:
// 0.88 against 0.97 ms); the grouped launches of the batched solve keep the 32-half
// slices, whose second workgroup per CU hides the prologue and epilogue of the short-K
// tiles there (114.9 against 116.7 ms per call on the 64-problem batch).
constexpr int kKernelLegacyTile = 8;
constexpr int kDpSingle128 = 3;
hipError_t launch_split_tile_layer(int precision, int tile, int kernel, const SquareArgs& a, hipStream_t s) {
    if ((tile == 128 || tile == 256) && kernel != kKernelLegacyTile)
        return launch_square_dp(precision, tile, tile == 128 ? kDpSingle128 : 0, a, s);
    return launch_square_split(precision, tile, a, s);
}

// FP64 layer on 128 tiles: kernel 0 (automatic) = the persistent schedule when `sk` holds a
// feasible plan, else the per-tile direct-load kernel (8 waves); 2 / 3 / 4 = per-tile
// variants 0 / 1 / 2; 5 = persistent (per-tile where infeasible); 1 or 64 tiles = the
// register-staged kernel.
constexpr int kF64AutoVariant = 2;
hipError_t launch_f64_layer(int tile, int kernel, const SquareArgs& a, const StreamK* sk, hipStream_t s) {
    if (tile == 128 && kernel != 1) {
        if ((kernel == 0 || kernel == 5) && sk && sk->grid > 0) return launch_square_f64_sk(a, *sk, s);
        return launch_square_f64(kernel >= 2 && kernel <= 4 ? kernel - 2 : kF64AutoVariant, a, s);
    }
    return launch_square_plain(SP2_FP64, tile, a, s);
}

// Persistent FP64 plan for this device, or grid = 0 when infeasible
StreamK f64_sk_resolve(int np, void* partial, int* counter) {
    StreamK sk;
    memset(&sk, 0, sizeof(sk));
    int dev = 0, cus = 0;
    if (!partial || !counter) return sk;
    if (hipGetDevice(&dev) != hipSuccess) return sk;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return sk;
    if (!square_f64_sk_plan(np, cus, &sk)) {
        memset(&sk, 0, sizeof(sk));
        return sk;
    }
    sk.fpartial = (double*)partial;
    sk.counter = counter;
    return sk;
}

// workspace for the persistent FP64 layer is reserved once there are enough 128 tiles
bool f64_sk_space(int np) { return ntiles_upper(np / 128) >= 64; }

int auto_tile_main(int n, bool split) {
    // split modes: 128 tiles from 2048 to 4608 (at 4096 the persistent 128-tile schedule
    // beats every 256-tile one: 0.289-0.302 against 0.307-0.338 ms per layer), 256 tiles
    // above; 64 tiles below 2048, where 128 tiles leave CUs idle (one layer at n = 1024:
    // 0.034 vs 0.049 ms, n = 1536: 0.048 vs 0.064 ms; equal at 2048)
    if (split) return n < 2048 ? 64 : (n <= 4608 ? 128 : 256);
    return n <= 512 ? 64 : 128;
}

void make_plan(int n, const Opts& o, Plan* p) {
    p->n = n;
    p->precision = o.precision;
    p->split = o.precision == SP2_FP16X2 || o.precision == SP2_BF16X2;
    p->scale_log2 = o.scale_log2;
    // automatic schedule: the autotuner's measurement for this size class if there is one
    int tile = o.tile, kernel = o.kernel;
    if (p->split && tile == 0 && kernel == 0) {
        int tt = 0, kk = 0;
        if (tune_lookup(kTuneSingle, o.precision, tune_key_single(n), &tt, &kk)) {
            tile = tt;
            kernel = kk;
        }
    }
    p->tile_main = tile ? tile : auto_tile_main(n, p->split);
    p->tile_ref = o.tile_ref ? o.tile_ref : (n <= 512 ? 64 : 128);
    const int m = p->tile_main > p->tile_ref ? p->tile_main : p->tile_ref;
    p->np = round_up(n, m);
    p->init_tiles = init_tiles(p->np);
    if (p->split)
        square_split_grid(p->tile_main, p->np, &p->main_T, &p->main_tiles, &p->main_per);
    else
        square_plain_grid(p->tile_main, p->np, &p->main_T, &p->main_tiles, &p->main_per);
    square_plain_grid(p->tile_ref, p->np, &p->ref_T, &p->ref_tiles, &p->ref_per);
    p->gersh_blocks = gershgorin_blocks(n);
    p->dstats_blocks = dstats_blocks(n);
    const size_t np2 = (size_t)p->np * p->np;
    const size_t es = o.precision == SP2_FP64 ? 8 : 4;
    size_t off = align_up(sizeof(DevState));
    p->off_init_parts = off;
    off = align_up(off + sizeof(double) * 3 * p->init_tiles);
    p->off_main_parts = off;
    off = align_up(off + sizeof(double) * 2 * p->main_tiles);
    p->off_gersh = off;
    off = align_up(off + sizeof(double) * 3 * p->gersh_blocks);
    p->off_dstats = off;
    off = align_up(off + sizeof(double) * 3 * p->dstats_blocks);
    for (int i = 0; i < 2; ++i) {
        p->off_s[i] = off;
        off = align_up(off + es * np2);
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            p->off_p[i][j] = off;
            if (p->split) off = align_up(off + 2 * (size_t)p->np * plane_ld(p->np));
        }
    p->off_s64 = off;
    off = align_up(off + (o.refine ? 8 * np2 : 0));
    p->off_y = off;
    off = align_up(off + (o.refine ? 8 * np2 : 0));
    p->kernel = kernel;
    p->sk_capable = sk_wanted(p->split, p->tile_main, kernel, p->np);
    p->off_sk_partial = off;
    if (p->sk_capable) off = align_up(off + square_sk_partial_bytes(p->tile_main, p->np));
    p->off_sk_counter = off;
    if (p->sk_capable) off = align_up(off + sizeof(int) * kSkCounterInts);
    // persistent FP64 layers (refinement on 128 tiles, FP64 mode on 128 tiles)
    p->f64_sk = ((o.refine && p->tile_ref == 128) || (o.precision == SP2_FP64 && p->tile_main == 128)) &&
                f64_sk_space(p->np);
    p->off_f64_partial = off;
    if (p->f64_sk) off = align_up(off + square_f64_sk_partial_bytes());
    p->off_f64_counter = off;
    if (p->f64_sk) off = align_up(off + sizeof(int) * kMaxSkGrid);
    p->total = off;
}

void fill_info(const DevState& st, const Plan* p, sp2_info* info) {
    memset(info, 0, sizeof(*info));
    info->status = st.status;
    info->layers = st.layers;
    info->converged = st.converged;
    info->first_sign = st.first_sign;
    info->n_padded = st.n_padded;
    info->tile = st.tile;
    info->emin = st.emin;
    info->emax = st.emax;
    info->trace = st.trace_d;
    info->idem = st.trace_d - st.frob_d;
    info->energy = st.energy;
    info->asym = st.asym;
    for (int k = 1; k <= SP2_MAX_LAYERS; ++k) {
        info->sigma[k - 1] = st.sigma[k];
        info->iderr[k - 1] = st.iderr[k];
        info->ns[k - 1] = st.ns[k];
        info->nx[k - 1] = st.nx[k];
        info->sigma_c[k - 1] = st.sigma_c[k];
    }
    info->accelerated = st.acc_layers;
    info->gap_violation = st.gap_violation;
    if (p) {
        StreamK sk;
        int variant = 0;
        info->kernel = sk_resolve(*p, &sk, &variant) ? 2 + variant : (p->kernel == 8 ? 8 : 1);
    }
}

#define SP2_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return SP2_EDEVICE;   \
    } while (0)

// Pinned, device-mapped ints that the control kernel sets when Alg. 1 stops.  They are
// allocated once per device and process (kFlagSlots slots of one 64-byte line each) and
// never freed.  A synchronous call owns one slot from before its first launch until its
// stream has drained, so no kernel of an earlier call can still write a slot that a later
// call has reset.  With every slot taken the call runs without a flag (all layers enqueued,
// as an asynchronous call does).
constexpr int kFlagSlots = 64, kFlagDevices = 64, kFlagStride = 16;   // 16 ints = 64 bytes
struct FlagPool {
    std::mutex mu;
    int* host[kFlagDevices] = {};
    int* dev[kFlagDevices] = {};
    unsigned long long used[kFlagDevices] = {};
};
FlagPool& flag_pool() {
    static FlagPool pool;
    return pool;
}

struct HostFlag {
    bool on = false, ok = true;
    int device = -1, slot = -1;
    volatile int* host = nullptr;
    int* dev = nullptr;
    hipStream_t stream = nullptr;
    HostFlag(bool enable, hipStream_t s) : stream(s) {
        if (!enable) return;
        if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kFlagDevices) return;
        FlagPool& fp = flag_pool();
        std::lock_guard<std::mutex> lock(fp.mu);
        if (!fp.host[device]) {
            int* h = nullptr;
            int* d = nullptr;
            if (hipHostMalloc((void**)&h, sizeof(int) * kFlagStride * kFlagSlots, hipHostMallocMapped) != hipSuccess) {
                ok = false;
                return;
            }
            if (hipHostGetDevicePointer((void**)&d, h, 0) != hipSuccess) {
                (void)hipHostFree(h);
                ok = false;
                return;
            }
            fp.host[device] = h;
            fp.dev[device] = d;
        }
        for (int i = 0; i < kFlagSlots; ++i)
            if (!((fp.used[device] >> i) & 1ull)) {
                slot = i;
                break;
            }
        if (slot < 0) return;
        fp.used[device] |= 1ull << slot;
        host = fp.host[device] + kFlagStride * slot;
        dev = fp.dev[device] + kFlagStride * slot;
        *host = 0;
        on = true;
    }
    ~HostFlag() {
        if (slot < 0) return;
        // a slot whose call's kernels may still be queued is never handed out again
        if (hipStreamSynchronize(stream) != hipSuccess) return;
        FlagPool& fp = flag_pool();
        std::lock_guard<std::mutex> lock(fp.mu);
        fp.used[device] &= ~(1ull << slot);
    }
};

struct ChunkEvents {
    bool ok = true;
    int count = 0;
    hipEvent_t ev[SP2_MAX_LAYERS + 2] = {};
    ChunkEvents(bool enable, int n) : count(enable ? n : 0) {
        for (int i = 0; i < count; ++i)
            ok = ok && hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
    }
    ~ChunkEvents() {
        for (int i = 0; i < count; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
};

// HIP events recorded between the kernels of one call (timed entry point only).
struct Events {
    bool on = false, ok = true;
    int layers = 0, launched = 0;
    hipEvent_t start = nullptr, prep = nullptr, loop_end = nullptr, end = nullptr;
    hipEvent_t ref[3] = {nullptr, nullptr, nullptr};
    hipEvent_t sq_b[SP2_MAX_LAYERS + 1] = {}, sq_e[SP2_MAX_LAYERS + 1] = {};
    Events(bool enable, int max_layers) : on(enable), layers(max_layers) {
        if (!on) return;
        hipEvent_t* all[] = {&start, &prep, &loop_end, &end, &ref[0], &ref[1], &ref[2]};
        for (hipEvent_t* e : all) ok = ok && hipEventCreate(e) == hipSuccess;
        for (int k = 1; k <= layers; ++k)
            ok = ok && hipEventCreate(&sq_b[k]) == hipSuccess && hipEventCreate(&sq_e[k]) == hipSuccess;
    }
    ~Events() {
        if (!on) return;
        hipEvent_t all[] = {start, prep, loop_end, end, ref[0], ref[1], ref[2]};
        for (hipEvent_t e : all)
            if (e) (void)hipEventDestroy(e);
        for (int k = 1; k <= layers; ++k) {
            if (sq_b[k]) (void)hipEventDestroy(sq_b[k]);
            if (sq_e[k]) (void)hipEventDestroy(sq_e[k]);
        }
    }
    hipError_t rec(hipEvent_t e, hipStream_t s) { return on ? hipEventRecord(e, s) : hipSuccess; }
    static double ms(hipEvent_t a, hipEvent_t b) {
        float t = 0.f;
        return hipEventElapsedTime(&t, a, b) == hipSuccess ? (double)t : -1.0;
    }
    hipError_t fill(sp2_timing* t, int ran, bool trivial) {
        hipError_t e = hipEventSynchronize(end);
        if (e != hipSuccess) return e;
        memset(t, 0, sizeof(*t));
        t->total_ms = ms(start, end);
        t->squarings = ran;
        if (trivial) return hipSuccess;
        t->prep_ms = ms(start, prep);
        t->loop_ms = ms(prep, loop_end);
        t->loop_active_ms = (ran > 0 && ran <= launched) ? ms(prep, sq_e[ran]) : 0.0;
        t->refine_ms = ms(loop_end, ref[2]);
        t->final_ms = ms(ref[2], end);
        for (int k = 1; k <= launched; ++k) t->square_ms[k - 1] = (float)ms(sq_b[k], sq_e[k]);
        t->refine_square_ms[0] = (float)ms(ref[0], ref[1]);
        t->refine_square_ms[1] = (float)ms(ref[1], ref[2]);
        return hipSuccess;
    }
};

}  // namespace

extern "C" {

void sp2_default_options(sp2_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->precision = SP2_FP16X2;
    opt->max_layers = 100;
    opt->eps = 0.0;
    opt->have_bounds = 0;
    opt->emin = 0.0;
    opt->emax = 0.0;
    opt->refine = 1;
    opt->scale_log2 = -1;
    opt->want_energy = 0;
    opt->tile = 0;
}

const char* sp2_strerror(int status) {
    switch (status) {
        case SP2_OK: return "success";
        case SP2_EINVAL: return "invalid argument or non-symmetric H";
        case SP2_ENONFINITE: return "non-finite value in H or in a layer";
        case SP2_ENOCONV: return "max_layers reached before the stopping test held";
        case SP2_ENOTIDEMP: return "result not idempotent or wrong occupation";
        case SP2_EDEVICE: return "HIP runtime error";
        case SP2_ENOMEM: return "workspace too small";
        default: return "unknown status";
    }
}

const char* sp2_version(void) { return "libsp2 0.1 (gfx950)"; }

size_t sp2_workspace_size(int n, const sp2_options* opt) {
    if (n <= 0) return 0;
    Opts o;
    if (!read_opts(opt, &o)) return 0;
    Plan p;
    make_plan(n, o, &p);
    return p.total;
}

static DevState initial_state(int n, int n_occ, double tol, const Opts& o, const Plan& p) {
    DevState init;
    memset(&init, 0, sizeof(init));
    init.n = n;
    init.n_occ = n_occ;
    init.n_padded = p.np;
    init.max_layers = o.max_layers;
    init.precision = o.precision;
    init.tile = p.tile_main;
    init.have_bounds = o.have_bounds;
    init.want_energy = o.want_energy;
    init.eps = o.eps;
    init.tol_tr = tol > 0 ? tol : 1e-6;
    init.tol_id = tol > 0 ? tol : 1e-6 * n;
    init.emin = o.have_bounds ? o.emin : 0.0;
    init.emax = o.have_bounds ? o.emax : 1.0;
    init.accel = o.accelerate;
    init.homo = o.homo;
    init.lumo = o.lumo;
    init.status = SP2_OK;
    return init;
}

// Occupation 0 or n: D = 0 or I is fixed by the occupation alone; the state (already
// initialised at the start of ws) records a converged call of 0 layers.
static hipError_t run_trivial(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, const Opts& o,
                       const Plan& p, char* ws, hipStream_t s) {
    DevState* st = (DevState*)ws;
    double* dstats = (double*)(ws + p.off_dstats);
    hipError_t e = launch_fill(dD, ldd, n, n_occ == n ? 1.0 : 0.0, s);
    int nd = 0;
    if (e == hipSuccess) e = launch_dstats(dD, ldd, o.want_energy ? dH : nullptr, ldh, n, dstats, &nd, s);
    if (e == hipSuccess) e = launch_mark_trivial(st, s);
    if (e == hipSuccess) e = launch_finalize(st, dstats, nd, (const double*)(ws + p.off_init_parts), 0, s);
    return e;
}

}  // extern "C"

// The whole path of sp2_density.  poll_flag: a synchronous call may poll a mapped host flag
// (allocated once per process) to stop enqueueing layers soon after Alg. 1 stops; without it
// every layer up to max_layers is enqueued (later ones return at once).
int sp2::density_call(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                      const sp2_options* opt, sp2_info* info, void* dWork, size_t work_bytes, void* stream,
                      sp2_timing* timing, bool poll_flag) {
    Opts o;
    if (!read_opts(opt, &o)) return SP2_EINVAL;
    if (n <= 0 || ldh < n || ldd < n || n_occ < 0 || n_occ > n || !dH || !dD || !dWork) return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    if (n > 65536) return SP2_EINVAL;
    Plan p;
    make_plan(n, o, &p);
    if (work_bytes < p.total) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dWork;
    DevState* st = (DevState*)ws;
    Events ev(timing != nullptr, o.max_layers);
    if (!ev.ok) return SP2_EDEVICE;
    SP2_TRY(ev.rec(ev.start, s));

    // declared before any launch and destroyed after the final synchronization
    HostFlag flag(poll_flag && (info != nullptr || timing != nullptr), s);
    if (!flag.ok) return SP2_EDEVICE;

    const DevState init = initial_state(n, n_occ, tol, o, p);
    SP2_TRY(launch_state_init(st, init, s));

    double* init_parts = (double*)(ws + p.off_init_parts);
    double* main_parts = (double*)(ws + p.off_main_parts);

    if (n_occ == 0 || n_occ == n) {
        SP2_TRY(run_trivial(dH, ldh, dD, ldd, n, n_occ, o, p, ws, s));
    } else {
        double* dstats = (double*)(ws + p.off_dstats);
        if (!o.have_bounds) {
            int nb = 0;
            double* gersh = (double*)(ws + p.off_gersh);
            SP2_TRY(launch_gershgorin(dH, ldh, n, gersh, &nb, s));
            SP2_TRY(launch_bounds(st, gersh, nb, s));
        }
        void* S[2] = {ws + p.off_s[0], ws + p.off_s[1]};
        void* P[2][2] = {{p.split ? ws + p.off_p[0][0] : nullptr, p.split ? ws + p.off_p[0][1] : nullptr},
                         {p.split ? ws + p.off_p[1][0] : nullptr, p.split ? ws + p.off_p[1][1] : nullptr}};
        SP2_TRY(launch_init_np(dH, ldh, st, p.np, o.precision, S[0], P[0][0], P[0][1], p.scale_log2, init_parts, s));
        SP2_TRY(ev.rec(ev.prep, s));

        StreamK sk;
        memset(&sk, 0, sizeof(sk));
        int sk_variant = 0;
        const bool use_sk = sk_resolve(p, &sk, &sk_variant);
        if (use_sk) {
            sk.partial = (float*)(ws + p.off_sk_partial);
            sk.counter = (int*)(ws + p.off_sk_counter);
            SP2_TRY(launch_zero_ints(sk.counter, kSkCounterInts, s));
        }
        StreamK f64sk;
        memset(&f64sk, 0, sizeof(f64sk));
        if (p.f64_sk) {
            f64sk = f64_sk_resolve(p.np, ws + p.off_f64_partial, (int*)(ws + p.off_f64_counter));
            if (f64sk.grid > 0) SP2_TRY(launch_zero_ints(f64sk.counter, kMaxSkGrid, s));
        }
        SquareArgs a;
        memset(&a, 0, sizeof(a));
        a.parts = main_parts;
        a.coef = st->coef;
        // FP64 layers take the unrounded coefficients (the accelerated layers' are not
        // representable in FP32)
        a.coef64 = o.precision == SP2_FP64 ? st->coef64 : nullptr;
        a.skip = &st->skip;
        a.np = p.np;
        a.ld_out = p.np;
        a.n_valid = p.np;
        a.n_real = n;
        a.T = p.main_T;
        a.ntiles = p.main_tiles;
        a.per = p.main_per;
        a.out_scale = ldexpf(1.f, -2 * p.scale_log2);
        a.in_scale = ldexpf(1.f, p.scale_log2);
        // Synchronous calls poll a mapped host flag that the control kernel sets when Alg. 1
        // stops, so that no layers are enqueued long after convergence: layers go out in
        // chunks, two chunks ahead of the one the host waits for.  Asynchronous calls
        // enqueue every layer up to max_layers (later ones return at once).
        const int chunk = n >= 4096 ? 2 : (n >= 1024 ? 4 : 8);
        ChunkEvents cev(flag.on, (o.max_layers + chunk) / chunk + 1);
        if (!cev.ok) return SP2_EDEVICE;
        int waited = 0;   // chunks whose completion the host has observed
        for (int layer = 1; layer <= o.max_layers + 1; ++layer) {
            if (flag.on && layer > 1 && (layer - 1) % chunk == 0) {
                const int c = (layer - 1) / chunk;          // chunk about to start
                SP2_TRY(hipEventRecord(cev.ev[c - 1], s));  // end of chunk c - 1
                if (c >= 2) {
                    SP2_TRY(hipEventSynchronize(cev.ev[c - 2]));
                    waited = c - 1;
                    if (*flag.host) break;
                }
            }
            if (layer == 1)
                SP2_TRY(launch_control_stride(st, init_parts, p.init_tiles, 3, layer, flag.dev, s));
            else
                SP2_TRY(launch_control_stride(st, main_parts, p.main_tiles, 2, layer, flag.dev, s));
            if (layer > o.max_layers) break;
            const int in = (layer - 1) & 1, out = layer & 1;
            a.x0 = p.split ? P[in][0] : S[in];
            a.x1 = p.split ? P[in][1] : nullptr;
            a.s_in = S[in];
            a.s_out = S[out];
            a.p0_out = P[out][0];
            a.p1_out = P[out][1];
            ev.launched = layer;
            SP2_TRY(ev.rec(ev.sq_b[layer], s));
            if (use_sk)
                SP2_TRY(launch_square_sk(o.precision, p.tile_main, sk_variant, a, sk, s));
            else if (p.split)
                SP2_TRY(launch_split_tile_layer(o.precision, p.tile_main, p.kernel, a, s));
            else if (o.precision == SP2_FP64)
                SP2_TRY(launch_f64_layer(p.tile_main, o.kernel, a, &f64sk, s));
            else
                SP2_TRY(launch_square_plain(o.precision, p.tile_main, a, s));
            SP2_TRY(ev.rec(ev.sq_e[layer], s));
        }
        (void)waited;
        SP2_TRY(ev.rec(ev.loop_end, s));
        if (o.refine) {
            double* s64 = (double*)(ws + p.off_s64);
            double* y = (double*)(ws + p.off_y);
            SP2_TRY(launch_select_f64(st, S[0], S[1], o.precision == SP2_FP64, s64, p.np, p.np, p.np, s));
            SP2_TRY(ev.rec(ev.ref[0], s));
            SquareArgs r;
            memset(&r, 0, sizeof(r));
            r.np = p.np;
            r.T = p.ref_T;
            r.ntiles = p.ref_tiles;
            r.per = p.ref_per;
            r.x0 = s64;
            r.s_in = s64;
            r.s_out = y;
            r.ld_out = p.np;
            r.n_valid = p.np;
            r.n_real = n;
            r.coef = st->rcoef[0];
            SP2_TRY(launch_f64_layer(p.tile_ref, o.precision == SP2_FP64 ? o.kernel : 0, r, &f64sk, s));
            SP2_TRY(ev.rec(ev.ref[1], s));
            r.x0 = y;
            r.s_in = y;
            r.s_out = dD;
            r.ld_out = ldd;
            r.n_valid = n;
            r.coef = st->rcoef[1];
            SP2_TRY(launch_f64_layer(p.tile_ref, o.precision == SP2_FP64 ? o.kernel : 0, r, &f64sk, s));
            SP2_TRY(ev.rec(ev.ref[2], s));
        } else {
            SP2_TRY(launch_select_f64(st, S[0], S[1], o.precision == SP2_FP64, dD, ldd, n, p.np, s));
            SP2_TRY(ev.rec(ev.ref[0], s));
            SP2_TRY(ev.rec(ev.ref[1], s));
            SP2_TRY(ev.rec(ev.ref[2], s));
        }
        int nd = 0;
        SP2_TRY(launch_dstats(dD, ldd, o.want_energy ? dH : nullptr, ldh, n, dstats, &nd, s));
        SP2_TRY(launch_finalize(st, dstats, nd, init_parts, p.init_tiles, s));
    }
    SP2_TRY(ev.rec(ev.end, s));
    if (!info && !timing) return SP2_OK;
    DevState host;
    SP2_TRY(hipStreamSynchronize(s));
    SP2_TRY(hipMemcpy(&host, st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (info) fill_info(host, &p, info);
    if (timing) {
        const bool trivial = (n_occ == 0 || n_occ == n);
        SP2_TRY(ev.fill(timing, trivial ? 0 : host.ran, trivial));
    }
    return host.status;
}

extern "C" {

int sp2_density(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                const sp2_options* opt, sp2_info* info, void* dWork, size_t work_bytes, void* stream) {
    return density_call(dH, ldh, dD, ldd, n, n_occ, tol, opt, info, dWork, work_bytes, stream, nullptr, true);
}

}  // extern "C"

// Scratch memory of sp2_density_static: one copy per device (module-scope device array,
// held while the library is loaded).  Host code never uses the array's name as an address:
// each device's copy is located once with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[SP2_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
struct ScratchTable {
    std::mutex mu;
    void* addr[kScratchDevices] = {};
};
ScratchTable& scratch_table() {
    static ScratchTable t;
    return t;
}
// Device address of the current device's scratch array (located on the first call on that
// device, with it current), or nullptr on a HIP error.
void* device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return nullptr;
    ScratchTable& t = scratch_table();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.addr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        t.addr[dev] = ptr;
    }
    return t.addr[dev];
}
}  // namespace

extern "C" {

int sp2_density_static(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                       const sp2_options* opt, sp2_info* info, void* stream) {
    Opts o;
    if (!read_opts(opt, &o) || n <= 0 || n > 65536) return SP2_EINVAL;
    if (ldh < n || ldd < n || n_occ < 0 || n_occ > n || !dH || !dD) return SP2_EINVAL;
    Plan p;
    make_plan(n, o, &p);
    if (p.total > (size_t)SP2_STATIC_SCRATCH_BYTES) return SP2_ENOMEM;
    void* ws = device_scratch();
    if (!ws) return SP2_EDEVICE;
    // no polled host flag (it is pinned memory allocated on first use) and no events
    return density_call(dH, ldh, dD, ldd, n, n_occ, tol, opt, info, ws, SP2_STATIC_SCRATCH_BYTES, stream, nullptr,
                        false);
}

int sp2_density_timed(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                      const sp2_options* opt, sp2_info* info, void* dWork, size_t work_bytes, void* stream,
                      sp2_timing* timing) {
    if (!timing) return SP2_EINVAL;
    return density_call(dH, ldh, dD, ldd, n, n_occ, tol, opt, info, dWork, work_bytes, stream, timing, true);
}



int sp2_query(const void* dWork, int n, const sp2_options* opt, sp2_info* info, void* stream) {
    Opts o;
    if (!dWork || !info || n <= 0 || !read_opts(opt, &o)) return SP2_EINVAL;
    Plan p;
    make_plan(n, o, &p);
    DevState host;
    SP2_TRY(hipStreamSynchronize((hipStream_t)stream));
    SP2_TRY(hipMemcpy(&host, dWork, sizeof(DevState), hipMemcpyDeviceToHost));
    fill_info(host, &p, info);
    return host.status;
}

// ----------------------------------------------------------------------------------
// Optimized finite-temperature expansion on matrices (Eq. general SP2 with its read-out)
// ----------------------------------------------------------------------------------
static bool fermi_plan(int n, const sp2_options* opt, Opts* o, Plan* p, size_t* off_coef, size_t* off_sum,
                       size_t* total) {
    if (n <= 0 || n > 65536 || !read_opts(opt, o)) return false;
    if (!o->have_bounds || o->accelerate) return false;
    o->refine = 1;   // the FP64 refinement buffer holds the read-out accumulator
    make_plan(n, *o, p);
    *off_coef = align_up(p->total);   // FP32 copy, then FP64 copy of the layer coefficients
    *off_sum = align_up(*off_coef + (sizeof(float) + sizeof(double)) * 3 * SP2_MAX_LAYERS);
    *total = align_up(*off_sum + sizeof(double) * 3);
    return true;
}

size_t sp2_fermi_workspace_size(int n, const sp2_options* opt) {
    Opts o;
    Plan p;
    size_t oc, os, total;
    return fermi_plan(n, opt, &o, &p, &oc, &os, &total) ? total : 0;
}

int sp2_fermi_apply(const double* dH, int ldh, double* dD, int ldd, int n, int layers, const double* theta,
                    const double* c, const sp2_options* opt, double* obs, void* dWork, size_t work_bytes,
                    void* stream) {
    Opts o;
    Plan p;
    size_t off_coef, off_sum, total;
    if (!fermi_plan(n, opt, &o, &p, &off_coef, &off_sum, &total)) return SP2_EINVAL;
    if (ldh < n || ldd < n || !dH || !dD || !dWork || !theta || !c) return SP2_EINVAL;
    if (layers < 1 || layers >= SP2_MAX_LAYERS || ((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    for (int k = 0; k < 3 * layers; ++k)
        if (!isfinite(theta[k])) return SP2_EINVAL;
    for (int k = 0; k <= layers; ++k)
        if (!isfinite(c[k])) return SP2_EINVAL;
    if (work_bytes < total) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dWork;
    DevState* st = (DevState*)ws;
    // S_0 = (emax I - H)/(emax - emin) is what the input layer builds; the model's input is
    // X_0 = I - S_0, so layer 0 is rewritten in S_0: t1 (1 - s)^2 + t2 (1 - s) + t3 =
    // t1 s^2 + (-2 t1 - t2) s + (t1 + t2 + t3), and the read-out starts from
    // I - c_0 X_0 = (1 - c_0) I + c_0 S_0.
    double coef[3 * SP2_MAX_LAYERS];
    for (int k = 0; k < layers; ++k) {
        const double t1 = theta[3 * k], t2 = theta[3 * k + 1], t3 = theta[3 * k + 2];
        coef[3 * k] = t1;
        coef[3 * k + 1] = k == 0 ? -2.0 * t1 - t2 : t2;
        coef[3 * k + 2] = k == 0 ? t1 + t2 + t3 : t3;
    }
    float* dcoef = (float*)(ws + off_coef);
    double* dcoef64 = (double*)(ws + off_coef + align_up(sizeof(float) * 3 * SP2_MAX_LAYERS));
    double* acc = (double*)(ws + p.off_s64);
    DevState init = initial_state(n, 0, 0.0, o, p);
    SP2_TRY(launch_state_init(st, init, s));
    SP2_TRY(launch_store_coefs(dcoef, coef, 3 * layers, s));
    SP2_TRY(launch_store_coefs64(dcoef64, coef, 3 * layers, s));
    void* S[2] = {ws + p.off_s[0], ws + p.off_s[1]};
    void* P[2][2] = {{p.split ? ws + p.off_p[0][0] : nullptr, p.split ? ws + p.off_p[0][1] : nullptr},
                     {p.split ? ws + p.off_p[1][0] : nullptr, p.split ? ws + p.off_p[1][1] : nullptr}};
    double* init_parts = (double*)(ws + p.off_init_parts);
    SP2_TRY(launch_init_np(dH, ldh, st, p.np, o.precision, S[0], P[0][0], P[0][1], p.scale_log2, init_parts, s));
    SP2_TRY(launch_readout(o.precision, acc, S[0], p.np, c[0], 1.0 - c[0], 1, s));
    StreamK sk;
    memset(&sk, 0, sizeof(sk));
    int sk_variant = 0;
    const bool use_sk = sk_resolve(p, &sk, &sk_variant);
    if (use_sk) {
        sk.partial = (float*)(ws + p.off_sk_partial);
        sk.counter = (int*)(ws + p.off_sk_counter);
        SP2_TRY(launch_zero_ints(sk.counter, kSkCounterInts, s));
    }
    StreamK f64sk;
    memset(&f64sk, 0, sizeof(f64sk));
    if (p.f64_sk) {
        f64sk = f64_sk_resolve(p.np, ws + p.off_f64_partial, (int*)(ws + p.off_f64_counter));
        if (f64sk.grid > 0) SP2_TRY(launch_zero_ints(f64sk.counter, kMaxSkGrid, s));
    }
    SquareArgs a;
    memset(&a, 0, sizeof(a));
    a.parts = nullptr;
    a.skip = nullptr;
    a.np = p.np;
    a.ld_out = p.np;
    a.n_valid = p.np;
    a.n_real = n;
    a.T = p.main_T;
    a.ntiles = p.main_tiles;
    a.per = p.main_per;
    a.out_scale = ldexpf(1.f, -2 * p.scale_log2);
    a.in_scale = ldexpf(1.f, p.scale_log2);
    for (int k = 0; k < layers; ++k) {
        const int in = k & 1, out = in ^ 1;
        a.coef = dcoef + 3 * k;
        a.coef64 = o.precision == SP2_FP64 ? dcoef64 + 3 * k : nullptr;
        a.x0 = p.split ? P[in][0] : S[in];
        a.x1 = p.split ? P[in][1] : nullptr;
        a.s_in = S[in];
        a.s_out = S[out];
        a.p0_out = P[out][0];
        a.p1_out = P[out][1];
        if (use_sk)
            SP2_TRY(launch_square_sk(o.precision, p.tile_main, sk_variant, a, sk, s));
        else if (p.split)
            SP2_TRY(launch_split_tile_layer(o.precision, p.tile_main, p.kernel, a, s));
        else if (o.precision == SP2_FP64)
            SP2_TRY(launch_f64_layer(p.tile_main, o.kernel, a, &f64sk, s));
        else
            SP2_TRY(launch_square_plain(o.precision, p.tile_main, a, s));
        SP2_TRY(launch_readout(o.precision, acc, S[out], p.np, -c[k + 1], 0.0, 0, s));
    }
    SP2_TRY(launch_copy_out(acc, p.np, dD, ldd, n, s));
    if (!obs) return SP2_OK;
    double* dstats = (double*)(ws + p.off_dstats);
    double* sums = (double*)(ws + off_sum);
    int nd = 0;
    SP2_TRY(launch_dstats(dD, ldd, dH, ldh, n, dstats, &nd, s));
    SP2_TRY(launch_sum3(dstats, nd, sums, s));
    SP2_TRY(hipMemcpyAsync(obs, sums, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    SP2_TRY(hipStreamSynchronize(s));
    return (isfinite(obs[0]) && isfinite(obs[1])) ? SP2_OK : SP2_ENONFINITE;
}

size_t sp2_spectral_bounds_workspace_size(int n) {
    if (n <= 0 || n > 65536) return 0;
    return align_up(sizeof(DevState)) + align_up(sizeof(double) * 3 * gershgorin_blocks(n));
}

int sp2_spectral_bounds(const double* dH, int ldh, int n, double* emin, double* emax, void* dWork,
                        size_t work_bytes, void* stream) {
    if (n <= 0 || n > 65536 || ldh < n || !dH || !emin || !emax || !dWork) return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    if (work_bytes < sp2_spectral_bounds_workspace_size(n)) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dWork;
    DevState* st = (DevState*)ws;
    double* gersh = (double*)(ws + align_up(sizeof(DevState)));
    DevState init;
    memset(&init, 0, sizeof(init));
    init.n = n;
    init.n_padded = n;
    init.status = SP2_OK;
    SP2_TRY(launch_state_init(st, init, s));
    int nb = 0;
    SP2_TRY(launch_gershgorin(dH, ldh, n, gersh, &nb, s));
    SP2_TRY(launch_bounds(st, gersh, nb, s));
    DevState host;
    SP2_TRY(hipStreamSynchronize(s));
    SP2_TRY(hipMemcpy(&host, st, sizeof(DevState), hipMemcpyDeviceToHost));
    *emin = host.emin;
    *emax = host.emax;
    return host.status;
}

size_t sp2_observable_workspace_size(int n) {
    if (n <= 0 || n > 65536) return 0;
    return align_up(sizeof(double) * 3 * dstats_blocks(n)) + align_up(sizeof(double) * 3);
}

int sp2_observable(const double* dD, int ldd, const double* dA, int lda, int n, double* out, void* dWork,
                   size_t work_bytes, void* stream) {
    if (n <= 0 || n > 65536 || ldd < n || lda < n || !dD || !dA || !out || !dWork) return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    if (work_bytes < sp2_observable_workspace_size(n)) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    double* parts = (double*)dWork;
    double* sums = (double*)((char*)dWork + align_up(sizeof(double) * 3 * dstats_blocks(n)));
    int nd = 0;
    SP2_TRY(launch_dstats(dD, ldd, dA, lda, n, parts, &nd, s));
    SP2_TRY(launch_sum3(parts, nd, sums, s));
    SP2_TRY(hipMemcpyAsync(out, sums, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    SP2_TRY(hipStreamSynchronize(s));
    return (isfinite(out[0]) && isfinite(out[1]) && isfinite(out[2])) ? SP2_OK : SP2_ENONFINITE;
}

int sp2_square_padded(int n, int precision, int tile) {
    if (n <= 0) return 0;
    const bool split = precision == SP2_FP16X2 || precision == SP2_BF16X2;
    const int t = tile ? tile : auto_tile_main(n, split);
    return round_up(n, t);
}

size_t sp2_square_workspace_size(int n, int precision, int tile, int kernel) {
    const int np = sp2_square_padded(n, precision, tile);
    if (np <= 0) return 0;
    const bool split = precision == SP2_FP16X2 || precision == SP2_BF16X2;
    const int t = tile ? tile : auto_tile_main(n, split);
    int T, nt, per;
    if (split) square_split_grid(t, np, &T, &nt, &per);
    else square_plain_grid(t, np, &T, &nt, &per);
    size_t off = kAlign;                               // coefficients
    off = align_up(off + sizeof(double) * 2 * nt);     // partials
    off = align_up(off + sizeof(double) * 2);          // sums
    if (split) off = align_up(off + 4 * (size_t)np * plane_ld(np));
    if (sk_wanted(split, t, kernel, np)) {
        off = align_up(off + square_sk_partial_bytes(t, np));
        off = align_up(off + sizeof(int) * kSkCounterInts);
    }
    if (precision == SP2_FP64 && t == 128 && (kernel == 0 || kernel == 5) && f64_sk_space(np)) {
        off = align_up(off + square_f64_sk_partial_bytes());
        off = align_up(off + sizeof(int) * kMaxSkGrid);
    }
    return off;
}

int sp2_square(const void* dX, void* dY, int n, int precision, int tile, int kernel, int scale_log2, float alpha,
               float beta, float gamma, double* trace_frob, void* dWork, size_t work_bytes, void* stream) {
    if (!dX || !dY || !dWork || n <= 0) return SP2_EINVAL;
    if (precision < SP2_FP64 || precision > SP2_BF16X2) return SP2_EINVAL;
    const bool split = precision == SP2_FP16X2 || precision == SP2_BF16X2;
    if (tile != 0 && tile != 64 && tile != 128 && !(tile == 256 && split)) return SP2_EINVAL;
    if (kernel < 0 || (kernel > 1 + kSkVariants && kernel != 8)) return SP2_EINVAL;
    if (precision == SP2_FP64 && kernel > 5) return SP2_EINVAL;
    if (scale_log2 < 0) scale_log2 = precision == SP2_FP16X2 ? 12 : 0;
    if (!split) scale_log2 = 0;
    if (scale_log2 > (precision == SP2_FP16X2 ? 14 : 60)) return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    const int t = tile ? tile : auto_tile_main(n, split);
    const int np = round_up(n, t);
    if (work_bytes < sp2_square_workspace_size(n, precision, tile, kernel)) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dWork;
    int T, nt, per;
    if (split) square_split_grid(t, np, &T, &nt, &per);
    else square_plain_grid(t, np, &T, &nt, &per);
    float* coef = (float*)ws;
    double* parts = (double*)(ws + kAlign);
    size_t off = align_up(kAlign + sizeof(double) * 2 * nt);
    double* sums = (double*)(ws + off);
    off = align_up(off + sizeof(double) * 2);
    SP2_TRY(launch_set3(coef, alpha, beta, gamma, s));
    SquareArgs a;
    memset(&a, 0, sizeof(a));
    a.s_in = dX;
    a.s_out = dY;
    a.parts = parts;
    a.coef = coef;
    a.np = np;
    a.ld_out = np;
    a.n_valid = np;
    a.n_real = n;
    a.T = T;
    a.ntiles = nt;
    a.per = per;
    a.out_scale = ldexpf(1.f, -2 * scale_log2);
    a.in_scale = ldexpf(1.f, scale_log2);
    if (split) {
        void* p0 = ws + off;
        void* p1 = ws + off + 2 * (size_t)np * plane_ld(np);
        off = align_up(off + 4 * (size_t)np * plane_ld(np));
        SP2_TRY(launch_split((const float*)dX, p0, p1, np, precision, scale_log2, s));
        a.x0 = p0;
        a.x1 = p1;
        Plan pl;
        memset(&pl, 0, sizeof(pl));
        pl.np = np;
        pl.tile_main = t;
        pl.kernel = kernel;
        pl.sk_capable = sk_wanted(true, t, kernel, np);
        StreamK sk;
        memset(&sk, 0, sizeof(sk));
        int variant = 0;
        if (sk_resolve(pl, &sk, &variant)) {
            sk.partial = (float*)(ws + off);
            off = align_up(off + square_sk_partial_bytes(t, np));
            sk.counter = (int*)(ws + off);
            SP2_TRY(launch_zero_ints(sk.counter, kSkCounterInts, s));
            SP2_TRY(launch_square_sk(precision, t, variant, a, sk, s));
        } else {
            SP2_TRY(launch_split_tile_layer(precision, t, kernel, a, s));
        }
    } else if (precision == SP2_FP64) {
        a.x0 = dX;
        StreamK f64sk;
        memset(&f64sk, 0, sizeof(f64sk));
        if (t == 128 && (kernel == 0 || kernel == 5) && f64_sk_space(np)) {
            void* part = ws + off;
            off = align_up(off + square_f64_sk_partial_bytes());
            f64sk = f64_sk_resolve(np, part, (int*)(ws + off));
            if (f64sk.grid > 0) SP2_TRY(launch_zero_ints(f64sk.counter, kMaxSkGrid, s));
        }
        SP2_TRY(launch_f64_layer(t, kernel, a, &f64sk, s));
    } else {
        a.x0 = dX;
        SP2_TRY(launch_square_plain(precision, t, a, s));
    }
    if (trace_frob) {
        SP2_TRY(launch_sum_parts(parts, nt, sums, s));
        SP2_TRY(hipStreamSynchronize(s));
        SP2_TRY(hipMemcpy(trace_frob, sums, 2 * sizeof(double), hipMemcpyDeviceToHost));
    }
    return SP2_OK;
}

// =====================================================================================
// Batched solve: many independent Hamiltonians of different sizes.  Every step of the
// single-problem sequence becomes one launch covering all problems (grouped kernels: the
// blocks of a launch are split between problems by prefix offsets), and the whole
// sequence is captured once into a hipGraph that is launched as one unit.
// =====================================================================================
namespace {

struct BatchLayout {
    int batch, tile, ref_tile;
    std::vector<int> nontrivial;        // indices of problems that run the recursion
    std::vector<Plan> plans;
    std::vector<size_t> region;         // byte offset of each problem's region
    size_t off_probs, off_sq, off_offs, off_map, off_stage, total;
    int n_offs;                         // stride of the offset arrays (batch + 1)
    size_t map_ints;                    // capacity of the tile map of the 128-tile grouped launches
};

// Tile map of the grouped 128-tile launches (squaring and FP64 refinement): every tile of
// the problems `order` lists.  Each problem's tiles are cut into kMapParts contiguous runs
// of the strip order, each run on one XCD (so that the tiles of a run share its L2);
// problems go largest first, and each run to the XCD with the least work so far (a run's
// work ~ its tiles x n_p).  Four runs per problem: the 64-problem batch (N = 256..3008)
// takes 107.3 ms per call, against 111.7 ms with whole problems per XCD (the last layers,
// with few problems left, then kept only some XCDs busy), 109.2 ms with 2 runs and
// 109.0 ms with 8 (each XCD's L2 then holds panels of every problem).
constexpr int kMapParts = 4;
int build_tile_map(const std::vector<Plan>& plans, const std::vector<int>& problems, std::vector<int>* map) {
    std::vector<int> order(problems.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return plans[problems[x]].np > plans[problems[y]].np;
    });
    std::vector<int> bins[8];
    double load[8] = {};
    for (int k : order) {
        const Plan& p = plans[problems[k]];
        const int nt = p.main_tiles;
        const int parts = nt < kMapParts ? nt : kMapParts;
        bool used[8] = {};
        for (int r = 0; r < parts; ++r) {
            const int t0 = (int)((long long)nt * r / parts), t1 = (int)((long long)nt * (r + 1) / parts);
            int x = -1;
            for (int j = 0; j < 8; ++j)
                if (!used[j] && (x < 0 || load[j] < load[x])) x = j;
            used[x] = true;
            for (int t = t0; t < t1; ++t) bins[x].push_back((k << kTileMapShift) | t);
            load[x] += (double)(t1 - t0) * p.np;
        }
    }
    size_t per = 0;
    for (auto& b : bins) per = b.size() > per ? b.size() : per;
    map->assign(8 * per, -1);
    for (int x = 0; x < 8; ++x)
        for (size_t j = 0; j < bins[x].size(); ++j) (*map)[x * per + j] = bins[x][j];
    return (int)per;
}

// problems of one batched call: the tile map encodes the problem in the bits above kTileMapShift
constexpr int kMaxBatch = 1 << (31 - kTileMapShift);

bool batch_layout(int batch, const int* n, const int* n_occ, const Opts& o, BatchLayout* L) {
    L->batch = batch;
    int nmax = 0;
    for (int i = 0; i < batch; ++i) nmax = n[i] > nmax ? n[i] : nmax;
    int tuned = 0, tuned_kernel = 0;
    if (o.tile == 0 && tune_lookup(kTuneBatched, o.precision, tune_key_batched(batch, n), &tuned, &tuned_kernel))
        L->tile = tuned;
    else
        L->tile = o.tile ? o.tile : (nmax < 1024 ? 64 : 128);
    if (L->tile == 256) L->tile = 128;
    L->plans.resize(batch);
    L->region.resize(batch);
    L->nontrivial.clear();
    for (int i = 0; i < batch; ++i) {
        Opts oi = o;
        oi.tile = L->tile;
        oi.tile_ref = L->tile;   // one refinement tile for every problem of the grouped launch
        oi.kernel = 1;           // one workgroup per tile: grouped launches
        make_plan(n[i], oi, &L->plans[i]);
        if (n_occ && n_occ[i] > 0 && n_occ[i] < n[i]) L->nontrivial.push_back(i);
    }
    // descriptor areas are sized for every problem, so the size does not depend on n_occ
    L->n_offs = batch + 1;
    size_t off = 0;
    L->off_probs = off;
    off = align_up(off + sizeof(BatchProblem) * batch);
    L->off_sq = off;
    off = align_up(off + sizeof(SquareArgs) * 4 * batch);   // even layer, odd layer, refine 1, refine 2
    L->off_offs = off;
    off = align_up(off + sizeof(int) * 5 * L->n_offs);      // gersh, init, main, ref, dstats
    L->map_ints = 0;
    if (L->tile == 128)
        for (int i = 0; i < batch; ++i) L->map_ints += 8 * (size_t)L->plans[i].main_tiles;
    L->off_map = off;
    off = align_up(off + sizeof(int) * L->map_ints);
    L->off_stage = off;   // the device states of the problems, staged for one transfer
    off = align_up(off + sizeof(DevState) * batch);
    // then one single-problem region per problem; its DevState sits at the region's start
    for (int i = 0; i < batch; ++i) {
        L->region[i] = off;
        off = align_up(off + L->plans[i].total);
    }
    L->total = off;
    return true;
}

bool batch_opts(const sp2_options* opt, Opts* o) {
    if (!read_opts(opt, o)) return false;
    if (o->precision == SP2_FP64) return false;   // the batched path keeps FP32 state
    if (o->have_bounds) return false;             // per-problem Gershgorin bounds only
    if (o->accelerate) return false;              // HOMO/LUMO values are per problem
    o->refine = 1;                                // the batched sequence always refines
    return true;
}

}  // namespace

size_t sp2_batched_workspace_size(int batch, const int* n, const sp2_options* opt) {
    if (batch <= 0 || batch > kMaxBatch || !n) return 0;
    Opts o;
    if (!batch_opts(opt, &o)) return 0;
    for (int i = 0; i < batch; ++i)
        if (n[i] <= 0 || n[i] > 65536) return 0;
    BatchLayout L;
    batch_layout(batch, n, nullptr, o, &L);
    return L.total;
}

}  // extern "C"

namespace {

// Instantiated graphs of batched calls, keyed by everything the captured launches depend
// on (device, workspace address, layout and launch sizes); the most recent kGraphCache.
// Kept until the process ends.
constexpr size_t kGraphCache = 16;
struct GraphEntry {
    std::vector<long long> key;
    hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;   // least recently used first
hipGraphExec_t graph_cache_find(const std::vector<long long>& key) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size(); ++i)
        if (g_graphs[i].key == key) {
            GraphEntry e = g_graphs[i];
            g_graphs.erase(g_graphs.begin() + i);
            g_graphs.push_back(e);
            return e.exec;
        }
    return nullptr;
}
void graph_cache_add(const std::vector<long long>& key, hipGraphExec_t exec) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    if (g_graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back({key, exec});
}
// One non-blocking stream per device for the batched sequence, created on first use.
hipStream_t batch_stream() {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    for (auto& p : streams)
        if (p.first == dev) return p.second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams.push_back({dev, s});
    return s;
}

}  // namespace

// Layers in the first part of a batched sequence (see run_batched).
constexpr int kBatchLayersA = 48;

// The batched driver; homo/lumo (host, one per problem, or null) select accelerated layers.
static int run_batched(int batch, const double* const* dH, const int* ldh, double* const* dD, const int* ldd,
                       const int* n, const int* n_occ, const double* homo, const double* lumo, double tol,
                       const sp2_options* opt, sp2_info* infos, int use_graph, void* dWork, size_t work_bytes,
                       void* stream) {
    Opts o;
    if (batch <= 0 || batch > kMaxBatch || !dH || !ldh || !dD || !ldd || !n || !n_occ || !dWork ||
        !batch_opts(opt, &o))
        return SP2_EINVAL;
    if (((uintptr_t)dWork) % kAlign) return SP2_EINVAL;
    if ((homo == nullptr) != (lumo == nullptr)) return SP2_EINVAL;
    for (int i = 0; i < batch; ++i) {
        if (!dH[i] || !dD[i] || n[i] <= 0 || n[i] > 65536 || ldh[i] < n[i] || ldd[i] < n[i] || n_occ[i] < 0 ||
            n_occ[i] > n[i])
            return SP2_EINVAL;
        if (homo && !(isfinite(homo[i]) && isfinite(lumo[i]) && homo[i] < lumo[i])) return SP2_EINVAL;
    }
    BatchLayout L;
    batch_layout(batch, n, n_occ, o, &L);
    if (work_bytes < L.total) return SP2_ENOMEM;
    char* ws = (char*)dWork;
    hipStream_t user = (hipStream_t)stream;
    // problems with an empty or full occupation: D = 0 or I, on the caller's stream
    for (int i = 0; i < batch; ++i) {
        if (n_occ[i] > 0 && n_occ[i] < n[i]) continue;
        char* r = ws + L.region[i];
        SP2_TRY(launch_state_init((DevState*)r, initial_state(n[i], n_occ[i], tol, o, L.plans[i]), user));
        SP2_TRY(run_trivial(dH[i], ldh[i], dD[i], ldd[i], n[i], n_occ[i], o, L.plans[i], r, user));
    }
    const int nt = (int)L.nontrivial.size();
    if (nt > 0) {
        // ---------------------------------------------------------------- descriptors
        std::vector<BatchProblem> probs(nt);
        std::vector<SquareArgs> sq(4 * nt);
        std::vector<int> offs(5 * L.n_offs, 0);
        std::vector<DevState> states(nt);
        int* o_g = offs.data();
        int* o_i = o_g + L.n_offs;
        int* o_m = o_i + L.n_offs;
        int* o_r = o_m + L.n_offs;
        int* o_d = o_r + L.n_offs;
        BatchProblem* d_probs = (BatchProblem*)(ws + L.off_probs);
        for (int k = 0; k < nt; ++k) {
            const int i = L.nontrivial[k];
            const Plan& p = L.plans[i];
            char* r = ws + L.region[i];
            BatchProblem& q = probs[k];
            memset(&q, 0, sizeof(q));
            q.h = dH[i];
            q.d = dD[i];
            q.st = (DevState*)r;
            for (int j = 0; j < 2; ++j) {
                q.s[j] = r + p.off_s[j];
                for (int l = 0; l < 2; ++l) q.pl[j][l] = p.split ? (void*)(r + p.off_p[j][l]) : nullptr;
            }
            q.s64 = (double*)(r + p.off_s64);
            q.y = (double*)(r + p.off_y);
            q.init_parts = (double*)(r + p.off_init_parts);
            q.main_parts = (double*)(r + p.off_main_parts);
            q.gersh = (double*)(r + p.off_gersh);
            q.dstats = (double*)(r + p.off_dstats);
            q.ldh = ldh[i];
            q.ldd = ldd[i];
            q.n = n[i];
            q.np = p.np;
            q.n_occ = n_occ[i];
            q.want_energy = o.want_energy;
            q.init_tiles = p.init_tiles;
            q.main_tiles = p.main_tiles;
            q.gersh_blocks = p.gersh_blocks;
            q.dstats_blocks = p.dstats_blocks;
            q.in_scale = ldexpf(1.f, p.scale_log2);
            o_g[k + 1] = o_g[k] + p.gersh_blocks;
            o_i[k + 1] = o_i[k] + p.init_tiles;
            o_m[k + 1] = o_m[k] + p.main_tiles;
            o_r[k + 1] = o_r[k] + p.ref_tiles;
            o_d[k + 1] = o_d[k] + p.dstats_blocks;
            // squaring layers (even: S[0] -> S[1], odd: S[1] -> S[0]) and the two refinement layers
            for (int par = 0; par < 2; ++par) {
                SquareArgs& a = sq[par * nt + k];
                memset(&a, 0, sizeof(a));
                const int in = par, out = par ^ 1;   // layer n reads S[(n-1)&1]: odd n -> par 0
                a.x0 = p.split ? q.pl[in][0] : q.s[in];
                a.x1 = p.split ? q.pl[in][1] : nullptr;
                a.s_in = q.s[in];
                a.s_out = q.s[out];
                a.p0_out = q.pl[out][0];
                a.p1_out = q.pl[out][1];
                a.parts = q.main_parts;
                a.coef = ((DevState*)r)->coef;
                a.skip = &((DevState*)r)->skip;
                a.np = p.np;
                a.ld_out = p.np;
                a.n_valid = p.np;
                a.n_real = n[i];
                a.T = p.main_T;
                a.ntiles = p.main_tiles;
                a.per = p.main_per;
                a.out_scale = ldexpf(1.f, -2 * p.scale_log2);
                a.in_scale = ldexpf(1.f, p.scale_log2);
            }
            for (int step = 0; step < 2; ++step) {
                SquareArgs& a = sq[(2 + step) * nt + k];
                memset(&a, 0, sizeof(a));
                a.x0 = step == 0 ? (const void*)q.s64 : (const void*)q.y;
                a.s_in = a.x0;
                a.s_out = step == 0 ? (void*)q.y : (void*)q.d;
                a.ld_out = step == 0 ? p.np : ldd[i];
                a.n_valid = step == 0 ? p.np : n[i];
                a.n_real = n[i];
                a.coef = ((DevState*)r)->rcoef[step];
                a.np = p.np;
                a.T = p.ref_T;
                a.ntiles = p.ref_tiles;
                a.per = p.ref_per;
            }
            states[k] = initial_state(n[i], n_occ[i], tol, o, p);
            if (homo) {
                states[k].accel = 1;
                states[k].homo = homo[i];
                states[k].lumo = lumo[i];
            }
        }
        // uploads (synchronous, before anything of this call is enqueued)
        SP2_TRY(hipStreamSynchronize(user));
        SP2_TRY(hipMemcpy(d_probs, probs.data(), sizeof(BatchProblem) * nt, hipMemcpyHostToDevice));
        SP2_TRY(hipMemcpy(ws + L.off_sq, sq.data(), sizeof(SquareArgs) * 4 * nt, hipMemcpyHostToDevice));
        int map_per = 0;
        if (L.tile == 128) {
            std::vector<int> map;
            map_per = build_tile_map(L.plans, L.nontrivial, &map);
            if (map.size() > L.map_ints) return SP2_EINVAL;
            SP2_TRY(hipMemcpy(ws + L.off_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
        }
        const int* d_map = (const int*)(ws + L.off_map);
        SP2_TRY(hipMemcpy(ws + L.off_offs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice));
        DevState* d_stage = (DevState*)(ws + L.off_stage);
        SP2_TRY(hipMemcpy(d_stage, states.data(), sizeof(DevState) * nt, hipMemcpyHostToDevice));
        const SquareArgs* d_sq = (const SquareArgs*)(ws + L.off_sq);
        const int* d_offs = (const int*)(ws + L.off_offs);
        const int* d_og = d_offs;
        const int* d_oi = d_og + L.n_offs;
        const int* d_om = d_oi + L.n_offs;
        const int* d_or = d_om + L.n_offs;
        const int* d_od = d_or + L.n_offs;

        // ---------------------------------------------------------------- the sequence
        hipStream_t cs = batch_stream();
        if (!cs) return SP2_EDEVICE;
        // The sequence runs in three parts: A = set-up and layers 1 .. la, B = layers
        // la + 1 .. max_layers (and the final check), C = refinement and statistics.  B is
        // skipped when every problem has stopped within A (the host reads the states
        // between A and B), so the launches of layers after the last problem stopped are
        // not made at all; la covers the layer counts of typical batches.
        const int la = o.max_layers < kBatchLayersA ? o.max_layers : kBatchLayersA;
        auto layers = [&](hipStream_t s, int l0, int l1) -> int {
            for (int layer = l0; layer <= l1; ++layer) {
                SP2_TRY(launch_batch_control(d_probs, nt, layer, s));
                if (layer > o.max_layers) break;
                const SquareArgs* a = d_sq + ((layer - 1) & 1) * nt;
                if (o.precision == SP2_FP32)
                    SP2_TRY(launch_square_plain_g(SP2_FP32, L.tile, a, d_om, nt, o_m[nt], s));
                else
                    SP2_TRY(L.tile == 128 ? launch_square_dp_g(o.precision, 128, 0, a, d_map, map_per, s)
                                          : launch_square_split_g(o.precision, L.tile, a, d_om, nt, o_m[nt], s));
            }
            return SP2_OK;
        };
        auto part = [&](hipStream_t s, int which) -> int {
            if (which == 0) {
                SP2_TRY(launch_batch_states(d_probs, d_stage, nt, 1, s));
                SP2_TRY(launch_batch_gershgorin(d_probs, d_og, nt, o_g[nt], s));
                SP2_TRY(launch_batch_bounds(d_probs, nt, s));
                SP2_TRY(launch_batch_init(o.precision, d_probs, d_oi, nt, o_i[nt], s));
                SP2_TRY(layers(s, 1, la < o.max_layers ? la : o.max_layers + 1));
                SP2_TRY(launch_batch_states(d_probs, d_stage, nt, 0, s));   // for the check after A
            } else if (which == 1) {
                SP2_TRY(layers(s, la + 1, o.max_layers + 1));
            } else {
                SP2_TRY(launch_batch_select(d_probs, nt, 64, s));
                for (int step = 2; step <= 3; ++step)
                    SP2_TRY(L.tile == 128
                                ? launch_square_f64_g(d_sq + step * nt, d_map, map_per, s)
                                : launch_square_plain_g(SP2_FP64, L.tile, d_sq + step * nt, d_or, nt, o_r[nt], s));
                SP2_TRY(launch_batch_dstats(d_probs, d_od, nt, o_d[nt], s));
                SP2_TRY(launch_batch_finalize(d_probs, nt, s));
                SP2_TRY(launch_batch_states(d_probs, d_stage, nt, 0, s));
            }
            return SP2_OK;
        };
        int dev = 0;
        SP2_TRY(hipGetDevice(&dev));
        // The graphs depend only on the addresses and launch sizes below (the problems'
        // matrices, coefficients and states are read from the descriptors uploaded above),
        // so a call with the same layout in the same workspace reuses them.
        auto run_part = [&](int which) -> int {
            if (!use_graph) return part(cs, which);
            const std::vector<long long> key = {which, dev, (long long)(uintptr_t)ws, (long long)L.total, L.batch,
                                                nt, L.tile, o.precision, o.max_layers, la, map_per, o_g[nt],
                                                o_i[nt], o_m[nt], o_r[nt], o_d[nt], (long long)L.off_probs,
                                                (long long)L.off_sq, (long long)L.off_offs, (long long)L.off_map,
                                                (long long)L.off_stage};
            hipGraphExec_t exec = graph_cache_find(key);
            if (!exec) {
                int prc = SP2_OK;
                hipGraph_t graph = nullptr;
                if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return SP2_EDEVICE;
                prc = part(cs, which);
                const hipError_t e = hipStreamEndCapture(cs, &graph);
                if (prc == SP2_OK && e != hipSuccess) prc = SP2_EDEVICE;
                if (prc == SP2_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                    exec = nullptr;
                    prc = SP2_EDEVICE;
                }
                if (graph) (void)hipGraphDestroy(graph);
                if (prc != SP2_OK) return prc;
                graph_cache_add(key, exec);
            }
            return hipGraphLaunch(exec, cs) == hipSuccess ? SP2_OK : SP2_EDEVICE;
        };
        int rc = run_part(0);
        if (rc == SP2_OK && la < o.max_layers) {
            std::vector<DevState> mid(nt);
            if (hipStreamSynchronize(cs) != hipSuccess ||
                hipMemcpy(mid.data(), d_stage, sizeof(DevState) * nt, hipMemcpyDeviceToHost) != hipSuccess)
                rc = SP2_EDEVICE;
            bool all_stopped = true;
            for (int k = 0; k < nt && rc == SP2_OK; ++k) all_stopped = all_stopped && mid[k].stopped;
            if (rc == SP2_OK && !all_stopped) rc = run_part(1);
        }
        if (rc == SP2_OK) rc = run_part(2);
        if (hipStreamSynchronize(cs) != hipSuccess && rc == SP2_OK) rc = SP2_EDEVICE;
        if (rc != SP2_OK) return rc;
    }
    SP2_TRY(hipStreamSynchronize(user));
    std::vector<DevState> done(nt);
    if (nt > 0)
        SP2_TRY(hipMemcpy(done.data(), ws + L.off_stage, sizeof(DevState) * nt, hipMemcpyDeviceToHost));
    int worst = SP2_OK;
    for (int i = 0, k = 0; i < batch; ++i) {
        DevState host;
        if (k < nt && L.nontrivial[k] == i) host = done[k++];
        else SP2_TRY(hipMemcpy(&host, ws + L.region[i], sizeof(DevState), hipMemcpyDeviceToHost));
        if (infos) fill_info(host, &L.plans[i], &infos[i]);
        if (host.status != SP2_OK && worst == SP2_OK) worst = host.status;
    }
    return worst;
}

extern "C" {

int sp2_density_batched(int batch, const double* const* dH, const int* ldh, double* const* dD, const int* ldd,
                        const int* n, const int* n_occ, double tol, const sp2_options* opt, sp2_info* infos,
                        int use_graph, void* dWork, size_t work_bytes, void* stream) {
    return run_batched(batch, dH, ldh, dD, ldd, n, n_occ, nullptr, nullptr, tol, opt, infos, use_graph, dWork,
                       work_bytes, stream);
}

int sp2_density_batched_gap(int batch, const double* const* dH, const int* ldh, double* const* dD, const int* ldd,
                            const int* n, const int* n_occ, const double* homo, const double* lumo, double tol,
                            const sp2_options* opt, sp2_info* infos, int use_graph, void* dWork, size_t work_bytes,
                            void* stream) {
    if (!homo || !lumo) return SP2_EINVAL;
    return run_batched(batch, dH, ldh, dD, ldd, n, n_occ, homo, lumo, tol, opt, infos, use_graph, dWork, work_bytes,
                       stream);
}

}  // extern "C"
