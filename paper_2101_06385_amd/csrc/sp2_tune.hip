// Autotuner: measures the squaring schedules on the device and records the fastest in a
// process-wide table that automatic options (tile = 0, kernel = 0) consult.
//
//  * sp2_autotune(n, precision): one split-precision layer Y = X^2 of an n x n symmetric
//    synthetic matrix (entries from a counter hash, zero padding), timed with HIP events for
//    every schedule that can run at this size: tiles 64 (small n), 128, 256 with one
//    workgroup per tile, and the persistent variants that have at least one tile per
//    workgroup.  Key: (device, precision, n rounded up to 256).
//  * sp2_autotune_batched: the batched solve itself on the caller's problems, once per
//    grouped-kernel tile (64, 128).  Key: (device, precision, the multiset of sizes).
//
// The table is guarded by a mutex; entries are only ever replaced by a later measurement.
#include "sp2_internal.h"

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace sp2 {
namespace {

struct TuneEntry {
    int tile, kernel;
    float ms;
};
typedef std::tuple<int, int, int, unsigned long long> TuneKey;   // device, kind, precision, key

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry>& table() {
    static std::map<TuneKey, TuneEntry> t;
    return t;
}

int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    return dev;
}

// X[i][j] = X[j][i] in (-1, 1) / sqrt(n) for i, j < n (a 32-bit mix of min(i,j), max(i,j)),
// zero in the padding
__global__ void k_tune_fill(float* x, int n, int np, float scale) {
    const size_t total = (size_t)np * np;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / np), j = (int)(idx % np);
        float v = 0.f;
        if (i < n && j < n) {
            unsigned h = (unsigned)(i < j ? i : j) * 0x9E3779B1u ^ (unsigned)(i < j ? j : i) * 0x85EBCA77u;
            h ^= h >> 15;
            h *= 0x2C1B3C6Du;
            h ^= h >> 12;
            h *= 0x297A2D39u;
            h ^= h >> 15;
            v = ((float)(h >> 8) * (1.f / 8388608.f) - 1.f) * scale;
        }
        x[idx] = v;
    }
}

struct Candidate {
    int tile, kernel;
};

// schedules that can run at size n on this device (a persistent variant only where it
// has a tile per workgroup: otherwise the library would run the per-tile kernel anyway)
std::vector<Candidate> candidates(int n) {
    std::vector<Candidate> c;
    int dev = current_device(), cus = 256;
    if (dev >= 0) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (n <= 2048) c.push_back({64, 1});
    for (int tile : {128, 256}) {
        if (tile == 256 && n <= 256) continue;
        c.push_back({tile, 1});
        const int np = (n + tile - 1) / tile * tile;
        for (int v = 0; v < kSkVariants; ++v) {
            int per_cu, T, nt;
            StreamK sk;
            if (square_sk_plan(tile, v, np, cus, &per_cu, &sk, &T, &nt)) c.push_back({tile, 2 + v});
        }
    }
    return c;
}

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

unsigned long long tune_key_single(int n) { return (unsigned long long)((n + 255) / 256 * 256); }

unsigned long long tune_key_batched(int batch, const int* n) {
    std::vector<int> v(n, n + batch);
    std::sort(v.begin(), v.end());
    unsigned long long h = 1469598103934665603ull;   // FNV-1a over the sorted sizes
    for (int x : v) {
        h ^= (unsigned long long)(unsigned)x;
        h *= 1099511628211ull;
    }
    return h;
}

bool tune_lookup(int kind, int precision, unsigned long long key, int* tile, int* kernel) {
    const int dev = current_device();
    if (dev < 0) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = table().find(TuneKey(dev, kind, precision, key));
    if (it == table().end()) return false;
    *tile = it->second.tile;
    *kernel = it->second.kernel;
    return true;
}

void tune_store(int kind, int precision, unsigned long long key, int tile, int kernel, float ms) {
    const int dev = current_device();
    if (dev < 0) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    table()[TuneKey(dev, kind, precision, key)] = TuneEntry{tile, kernel, ms};
}

}  // namespace sp2

using namespace sp2;

extern "C" {

size_t sp2_autotune_workspace_size(int n, int precision) {
    if (n <= 0 || n > 65536 || (precision != SP2_FP16X2 && precision != SP2_BF16X2)) return 0;
    const size_t np = (size_t)(n + 255) / 256 * 256;
    size_t ws = 0;
    for (const Candidate& c : candidates(n)) ws = std::max(ws, sp2_square_workspace_size(n, precision, c.tile, c.kernel));
    return 2 * align256(4 * np * np) + ws;
}

int sp2_autotune(int n, int precision, int reps, int* tile, int* kernel, float* ms, void* dWork, size_t work_bytes,
                 void* stream) {
    if (n <= 0 || n > 65536 || (precision != SP2_FP16X2 && precision != SP2_BF16X2) || reps < 1 || reps > 1000 ||
        !dWork)
        return SP2_EINVAL;
    if (((uintptr_t)dWork) % 256) return SP2_EINVAL;
    const size_t need = sp2_autotune_workspace_size(n, precision);
    if (work_bytes < need) return SP2_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const size_t npmax = (size_t)(n + 255) / 256 * 256;
    char* ws = (char*)dWork;
    float* x = (float*)ws;
    float* y = (float*)(ws + align256(4 * npmax * npmax));
    char* sq_ws = ws + 2 * align256(4 * npmax * npmax);
    const size_t sq_bytes = work_bytes - 2 * align256(4 * npmax * npmax);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SP2_EDEVICE;
    }
    int st = SP2_OK;
    Candidate best{0, 0};
    float best_ms = 0.f;
    for (const Candidate& c : candidates(n)) {
        const int np = sp2_square_padded(n, precision, c.tile);
        const size_t total = (size_t)np * np;
        size_t g = (total + 255) / 256;
        if (g > 8192) g = 8192;
        hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)g), dim3(256), 0, s, x, n, np, 1.f / sqrtf((float)n));
        if (hipGetLastError() != hipSuccess) {
            st = SP2_EDEVICE;
            break;
        }
        st = sp2_square(x, y, n, precision, c.tile, c.kernel, -1, 1.f, 0.f, 0.f, nullptr, sq_ws, sq_bytes, stream);
        if (st != SP2_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) {
            st = SP2_EDEVICE;
            break;
        }
        for (int r = 0; r < reps && st == SP2_OK; ++r)
            st = sp2_square(x, y, n, precision, c.tile, c.kernel, -1, 1.f, 0.f, 0.f, nullptr, sq_ws, sq_bytes, stream);
        if (st != SP2_OK) break;
        float t = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            st = SP2_EDEVICE;
            break;
        }
        t /= (float)reps;
        if (best.tile == 0 || t < best_ms) {
            best = c;
            best_ms = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SP2_OK) return st;
    if (best.tile == 0) return SP2_EINVAL;
    tune_store(kTuneSingle, precision, tune_key_single(n), best.tile, best.kernel, best_ms);
    if (tile) *tile = best.tile;
    if (kernel) *kernel = best.kernel;
    if (ms) *ms = best_ms;
    return SP2_OK;
}

size_t sp2_autotune_batched_workspace_size(int batch, const int* n, const sp2_options* opt) {
    sp2_options o;
    if (opt) o = *opt;
    else sp2_default_options(&o);
    size_t w = 0;
    for (int tile : {64, 128}) {
        o.tile = tile;
        const size_t b = sp2_batched_workspace_size(batch, n, &o);
        if (b == 0) return 0;
        w = std::max(w, b);
    }
    return w;
}

int sp2_autotune_batched(int batch, const double* const* dH, const int* ldh, double* const* dD, const int* ldd,
                         const int* n, const int* n_occ, const sp2_options* opt, int* tile, float* ms, void* dWork,
                         size_t work_bytes, void* stream) {
    if (batch <= 0 || !n) return SP2_EINVAL;
    const size_t need = sp2_autotune_batched_workspace_size(batch, n, opt);
    if (need == 0) return SP2_EINVAL;
    if (work_bytes < need) return SP2_ENOMEM;
    sp2_options o;
    if (opt) o = *opt;
    else sp2_default_options(&o);
    int best_tile = 0;
    float best_ms = 0.f;
    for (int t : {64, 128}) {
        o.tile = t;
        float elapsed = 0.f;
        for (int rep = 0; rep < 2; ++rep) {   // the first run also builds the graph's code paths
            const auto t0 = std::chrono::steady_clock::now();
            const int st = sp2_density_batched(batch, dH, ldh, dD, ldd, n, n_occ, 0.0, &o, nullptr, 1, dWork,
                                               work_bytes, stream);
            const auto t1 = std::chrono::steady_clock::now();
            if (st != SP2_OK && st != SP2_ENOCONV && st != SP2_ENOTIDEMP) return st;
            elapsed = std::chrono::duration<float, std::milli>(t1 - t0).count();
        }
        if (best_tile == 0 || elapsed < best_ms) {
            best_tile = t;
            best_ms = elapsed;
        }
    }
    tune_store(kTuneBatched, o.precision, tune_key_batched(batch, n), best_tile, 1, best_ms);
    if (tile) *tile = best_tile;
    if (ms) *ms = best_ms;
    return SP2_OK;
}

void sp2_autotune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    table().clear();
}

}  // extern "C"
