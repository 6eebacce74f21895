// Arguments of the squaring kernels and of their persistent schedule (the parts of the
// interface the kernel code depends on).
#pragma once

namespace sp2 {

// ---------------------------------------------------------------------------------
// Arguments of the squaring kernels: Y = alpha X^2 + beta X + gamma I, written to
// both triangles (exactly symmetric), optionally split into half-precision planes, with
// FP64 partial sums of Tr Y and ||Y||_F^2 per output tile.
// ---------------------------------------------------------------------------------
struct SquareArgs {
    const void* x0;       // split modes: high plane of X (np x np, row stride plane_ld(np)); plain: X itself
    const void* x1;       // split modes: low plane of X
    const void* s_in;     // X in the state precision (beta term), ld = np
    void* s_out;          // Y in the state precision, ld = ld_out
    void* p0_out;         // split modes: planes of Y (row stride plane_ld(np)), or null
    void* p1_out;
    double* parts;        // 2 doubles per tile, or null
    const float* coef;    // (alpha, beta, gamma)
    const double* coef64; // FP64 layer kernels: (alpha, beta, gamma) in FP64 when non-null
    const int* skip;      // null, or a flag that makes every workgroup return at once
    int np;               // padded edge (multiple of the tile)
    int ld_out;           // leading dimension of s_out
    int n_valid;          // rows/cols >= n_valid of s_out are not written
    int n_real;           // logical edge: the gamma I term stops here so the padding stays zero
    int T;                // tiles per edge
    int ntiles;           // T (T + 1) / 2
    int per;              // ceil(ntiles / 8)
    float out_scale;      // split modes: 2^-2s applied to the accumulated products
    float in_scale;       // split modes: 2^s applied before splitting Y
};

// Schedule of the persistent split-square kernel: G workgroups run `rounds` whole rounds
// of tiles, then the `tail_tiles` leftover tiles are each cut into `chunks` K-chunks.
// `partial` holds one FP32 tile accumulator per tail chunk, `counter` one arrival count
// per tail tile (zeroed at the start of every call; each executed layer adds `chunks`).
constexpr int kMaxSkGrid = 1024;
// The int array `counter` of the persistent split square: arrivals per split tile at
// [0, kMaxSkGrid), then the ticket counter of the tail-chunk queue at kSkQueueSlot.
constexpr int kSkQueueSlot = kMaxSkGrid;
constexpr int kSkCounterInts = kMaxSkGrid + 64;
// Two-level split tail: group arrival counters at [kSkGroupCounter, kMaxSkGrid) of
// `counter`, group partial tiles from slot kSkGroupSlot of `partial` (chunk partials use
// slots below it: at most one per workgroup).
constexpr int kSkGroupCounter = kMaxSkGrid / 2;
constexpr int kSkGroupSlot = kMaxSkGrid / 2;

// Tile maps of the grouped (many-problem) launches: entry (problem << kTileMapShift) |
// tile, or -1 for no work.  Block b reads entry (b mod 8) * per + b / 8, so the blocks that
// the hardware sends to one XCD (b mod 8 fixed) walk that XCD's part of the map.
constexpr int kTileMapShift = 18;
constexpr int kTileMapMask = (1 << kTileMapShift) - 1;

// Row stride (elements) of the half-precision planes of an np x np matrix.  With a row
// pitch of a power of two kilobytes, the rows of one K-slice of a panel fall on the same
// L2 channel; one extra 128-byte line per row spreads them.  One squaring layer at
// n = 16384 measured 14.5 ms with pitch np and 12.0 ms with this one (no change at 8192).
__host__ __device__ inline int plane_ld(int np) { return np + 64; }
constexpr int kSkVariants = 6;
// Stream-K form (split squaring, stream_k = Q > 0): the ntiles x (KS / Q) units of Q
// K-slices, tile-major, are cut into G contiguous ranges, one per workgroup; a tile that
// several ranges share is finished by the last of its contributors, which sums their FP32
// partials in K order.  Workgroup v keeps its partials in slots 2v (first tile of its
// range) and 2v + 1 (last tile); `counter` then counts arrivals per tile.
struct StreamK {
    int grid = 0, rounds = 0, tail_tiles = 0, chunks = 0;
    float* partial = nullptr;     // FP32 partial tiles (split squaring, adjoint)
    int* counter = nullptr;       // arrivals per tail tile, counted modulo chunks
    double* fpartial = nullptr;   // FP64 partial tiles (FP64 layer)
    int stream_k = 0;             // slices per stream-K unit; 0: whole rounds + split tail
    int pad = 0;
};
constexpr int kSkMaxContrib = 16;   // most stream-K ranges that may share one tile

}  // namespace sp2
