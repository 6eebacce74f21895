/*
 * sp2.h -- C ABI of libsp2: SP2 density matrices on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the zero-temperature density matrix D = theta(mu I - H)
 * (Eq. 3) of a dense symmetric Hamiltonian H by the Deep-NN formulation of the
 * second-order spectral projection recursion (Alg. 1): a rescale of H into [0,1]
 * with reversed order, a chain of matrix squarings S <- S^2 or 2S - S^2 chosen by
 * trace, the parameter-free stopping test of Alg. 1, and the enhanced-precision
 * refinement layer of Eq. Refinement.  The squarings can run in FP64, FP32 or in
 * the dual half-precision form of Alg. 2 (Eqs. Split1, Split2, Square) with FP32
 * accumulation; traces, bounds and the final checks are always FP64.
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major with a leading dimension (ld >= n, in elements).  For a
 *     symmetric matrix row- and column-major coincide.
 *   - Every matrix and workspace pointer is a DEVICE pointer owned by the caller.
 *     The library never allocates or frees device memory and keeps no state between
 *     calls; all per-call state lives in the caller's workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *     work is enqueued on it.  A call with `info == NULL` returns after enqueueing,
 *     without synchronizing; device-side outcomes can be read later with sp2_query.
 *     A call with `info != NULL` synchronizes the stream and fills *info.
 *   - Errors: argument errors are detected on the host before anything is enqueued
 *     and return SP2_EINVAL.  HIP errors return SP2_EDEVICE.  Numerical outcomes
 *     (non-finite values, no convergence, result not idempotent) are detected on the
 *     device and returned when the call synchronizes; D is written in every one of
 *     these numerical cases.
 */
#ifndef SP2_H
#define SP2_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SP2_OK = 0,
    SP2_EINVAL = -1,      /* bad argument, or H not symmetric (checked on the device) */
    SP2_ENONFINITE = -2,  /* NaN/Inf in H or in a layer */
    SP2_ENOCONV = -3,     /* max_layers reached before a stopping test of Alg. 1 held */
    SP2_ENOTIDEMP = -4,   /* |Tr D - n_occ| or |Tr[D - D^2]| above tolerance */
    SP2_EDEVICE = -5,     /* a HIP call failed */
    SP2_ENOMEM = -6       /* workspace smaller than sp2_workspace_size() */
} sp2_status;

/* Arithmetic of the squaring layers (the activation f(X) = X^2 of Alg. 1). */
typedef enum {
    SP2_FP64 = 0,    /* FP64 matrix cores, FP64 state */
    SP2_FP32 = 1,    /* FP32 matrix cores, FP32 state */
    SP2_FP16X2 = 2,  /* Alg. 2: X = X0 + X1 in two FP16 planes, 3 products, FP32 accumulate */
    SP2_BF16X2 = 3   /* the same with BF16 planes */
} sp2_precision;

#define SP2_MAX_LAYERS 128   /* capacity of the per-layer history; max_layers <= 127 */

typedef struct {
    int precision;     /* sp2_precision; default SP2_FP16X2 */
    int max_layers;    /* 1..127; default 100 */
    double eps;        /* the small constant epsilon of Alg. 1 (alternation bias); default 0 */
    int have_bounds;   /* nonzero: use [emin, emax] below as the spectral bounds of Alg. 1
                          (they must enclose the spectrum); zero: Gershgorin bounds computed
                          on the device in FP64 and widened outward by the rounding bound */
    double emin, emax;
    int refine;        /* nonzero (default): final layer f_final of Eq. Refinement in FP64;
                          zero: D = S_{m-1} widened to FP64 */
    int scale_log2;    /* split modes: both half-precision planes hold 2^s X (an exact shift
                          that keeps the low plane out of the FP16 subnormal range; the
                          products are scaled back by 2^-2s).  -1 (default) selects 12 for
                          FP16X2 and 0 for BF16X2; 0 is the paper's split exactly. */
    int want_energy;   /* nonzero: info->energy = Tr[D H] (the observable of Alg. 1) */
    int tile;          /* output tile edge of the squaring kernels: 0 = automatic, or 64/128/256 */
    int kernel;        /* split-mode squaring schedule: 0 = automatic, 1 = one workgroup per
                          tile (direct-to-LDS pipeline for tiles 128/256), 8 = one workgroup
                          per tile with register staging (every tile), 2..7 = persistent schedule (whole rounds of tiles, then the
                          leftover tiles split along K), kernel variant 0..5 for the tile,
                          as (waves, K-slice halves, LDS stages, rolling fragment pipeline:
                          one set of fragment registers refilled as the MFMAs free them):
                            256: (4,16,4,0) (8,16,4,0) (4,32,2,0) (8,32,2,0) (4,32,2,1) (8,32,2,1)
                            128: (4,32,4,0) (4,64,2,0) (4,16,4,0) (4,32,2,0) (4,64,2,1) (4,32,2,1)
                          Only split modes with tiles of 128/256 use these.  FP64 mode:
                          0 = automatic, 1 = register-staged kernel, 2 / 3 / 4 = direct-to-LDS
                          kernel (128 tiles) with (4 waves, 2 stages) / (4, 4) / (8, 4),
                          one workgroup per tile, 5 = the (8, 4) kernel on the persistent
                          schedule (whole rounds + split-K tail; per-tile where there are
                          fewer tiles than CUs).  The automatic choice (5, else 4) also
                          serves the FP64 refinement layer of every mode; 6, 7 are invalid. */
    int accelerate;    /* nonzero: accelerated Deep-NN SP2 (Sec. Accelerated Deep-NN SP2).  With
                          the occupied eigenvalues of S_{n-1} known to lie in [h, 1] and the
                          unoccupied ones in [0, l] (from homo, lumo below and the spectral
                          bounds), each layer uses a real weight sigma_n = +-1/(1 - 2v) with
                          the shift-and-rescale that maps its projection back onto [0, 1]:
                          S_n = ((S - vI)/(1 - v))^2 or I - (((1 - v)I - S)/(1 - v))^2, v and
                          the branch chosen for the widest rescaled HOMO-LUMO separation
                          without crossing.  Once max(l, 1 - h) <= 0.01 the layers of Alg. 1
                          continue; its alternation stopping test is taken only across two
                          such layers.  If homo/lumo do not rescale into 0 <= l < h <= 1 no
                          layer is accelerated (sp2_info.accelerated = 0).  Every layer
                          checks the interval against Tr S (sp2_info.gap_violation).
                          Single-problem calls (sp2_density_batched_gap for batches). */
    double homo, lumo; /* with accelerate: every occupied eigenvalue of H is <= homo and every
                          unoccupied one >= lumo, homo < lumo (an interval inside the
                          HOMO-LUMO gap, e.g. from a previous call).  An interval that is not
                          inside the gap can end on the projector onto the wrong states (with
                          the right trace); the per-layer consistency check reports that as
                          SP2_ENOTIDEMP with sp2_info.gap_violation > 0. */
} sp2_options;

typedef struct {
    int status;            /* sp2_status of the device-side checks */
    int layers;            /* m: the layer at which Alg. 1 stopped (S_{m-1} is refined) */
    int converged;         /* 1 if a stopping test of Alg. 1 held */
    int first_sign;        /* sign of the first of the two composed refinement steps */
    int n_padded;          /* internal matrix edge (n rounded up to the tile) */
    int tile;              /* output tile edge used */
    int kernel;            /* squaring schedule used: 1 = one workgroup per tile (also every
                              FP32/FP64 run), 8 = the register-staged per-tile kernel,
                              2 + v = persistent schedule, variant v */
    int accelerated;       /* number of accelerated layers (they are layers 1..accelerated) */
    int gap_violation;     /* accelerated runs: first layer n where |Tr S_{n-1} - n_occ| exceeded
                              (n - n_occ) l + n_occ (1 - h) (the tracked interval bounds) by more
                              than rounding, i.e. [homo, lumo] was not inside the gap; 0 if never.
                              A violation makes the status SP2_ENOTIDEMP. */
    int reserved;
    double emin, emax;     /* spectral bounds used */
    double trace;          /* Tr D */
    double idem;           /* Tr D - ||D||_F^2  (= Tr[D - D^2] for symmetric D) */
    double energy;         /* Tr[D H] if requested, else 0 */
    double asym;           /* max |H_ij - H_ji| */
    signed char sigma[SP2_MAX_LAYERS];  /* sigma_n, n = 1..layers at index n-1 */
    double iderr[SP2_MAX_LAYERS];       /* IdErr_n = Tr[S_{n-1} - S_{n-1}^2] */
    double ns[SP2_MAX_LAYERS];          /* N_S entering layer n: Tr S_{n-1} */
    double nx[SP2_MAX_LAYERS];          /* N_X of layer n: Tr X_n = ||S_{n-1}||_F^2 */
    double sigma_c[SP2_MAX_LAYERS];     /* real weight sigma_n of layer n: sigma_n itself on
                                           layers of Alg. 1, +-1/(1 - 2v) on accelerated ones */
} sp2_info;

/* Fill *opt with the defaults listed above. */
void sp2_default_options(sp2_options* opt);

/* Short description of a status code (static storage). */
const char* sp2_strerror(int status);

/* Library version string (static storage). */
const char* sp2_version(void);

/*
 * Workspace bytes needed by sp2_density for an n x n problem with these options
 * (opt may be NULL for defaults).  Returns 0 for n <= 0.
 */
size_t sp2_workspace_size(int n, const sp2_options* opt);

/*
 * sp2_density -- D = theta(mu I - H) with Tr D = n_occ, by Alg. 1.
 *
 *   dH     device, n x n FP64, leading dimension ldh >= n, symmetric; read only.
 *          Non-symmetric input (max|H_ij - H_ji| > 1e-12 * max(|emin|,|emax|,1)) is
 *          reported as SP2_EINVAL by the device check; the layers use (H + H^T)/2.
 *   dD     device, n x n FP64 output, leading dimension ldd >= n; exactly symmetric.
 *   n      matrix edge, >= 1.
 *   n_occ  number of occupied states, 0 <= n_occ <= n.  0 and n return D = 0 and
 *          D = I without running the recursion.
 *   tol    acceptance threshold: D is accepted when |Tr D - n_occ| <= tol and
 *          |Tr[D - D^2]| <= tol; tol <= 0 selects 1e-6 and 1e-6 * n.  The stopping
 *          rule of the recursion itself is Alg. 1's parameter-free test.
 *   opt    options (NULL = defaults).
 *   info   host pointer or NULL; see the stream conventions above.
 *   dWork  device workspace of work_bytes >= sp2_workspace_size(n, opt) bytes,
 *          256-byte aligned.  Its contents after the call describe the run (sp2_query).
 *   stream hipStream_t or NULL.
 */
int sp2_density(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                const sp2_options* opt, sp2_info* info, void* dWork, size_t work_bytes,
                void* stream);

/*
 * sp2_density_static -- sp2_density for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the workspace taken from a scratch array that the library
 * holds in device memory (SP2_STATIC_SCRATCH_BYTES per device, reserved while the library
 * is loaded).  The call allocates nothing: no hipMalloc/hipFree, no pinned host memory, no
 * events.  Problems whose sp2_workspace_size(n, opt) exceeds SP2_STATIC_SCRATCH_BYTES
 * return SP2_ENOMEM before any work (every n <= 1024 fits, in every precision).
 * Every call on one device uses that device's single scratch array: calls that overlap
 * on one device (other streams, other host threads) race and must be serialized by the
 * caller.  Each call clears the parts of the scratch it relies on, so a call's results do
 * not depend on earlier calls.  Arguments, stream and info semantics as sp2_density (with
 * info != NULL the call synchronizes `stream` and copies its state record to *info).
 */
#define SP2_STATIC_SCRATCH_BYTES (40u << 20)
int sp2_density_static(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                       const sp2_options* opt, sp2_info* info, void* stream);

/* Phase and per-layer durations of one sp2_density call, from HIP events on `stream`. */
typedef struct {
    double total_ms;       /* first kernel of the call .. last kernel */
    double prep_ms;        /* state init, spectral bounds, input layer */
    double loop_ms;        /* every layer launched (max_layers control + squaring pairs) */
    double loop_active_ms; /* start of the loop .. end of the last squaring that ran (S_{m-1}) */
    double refine_ms;      /* widening to FP64 and the two refinement layers */
    double final_ms;       /* final reductions and acceptance test */
    int squarings;         /* squaring layers that ran: m - 1 on convergence */
    int pad;
    float square_ms[SP2_MAX_LAYERS];   /* squaring kernel of layer n at index n - 1 */
    float refine_square_ms[2];         /* the two FP64 refinement layers */
} sp2_timing;

/*
 * sp2_density_timed -- sp2_density with HIP events recorded between the kernels it
 * enqueues (same kernels, same results); synchronizes and fills *timing (host).  For
 * benchmarks: event creation makes it slower to call than sp2_density.
 */
int sp2_density_timed(const double* dH, int ldh, double* dD, int ldd, int n, int n_occ, double tol,
                      const sp2_options* opt, sp2_info* info, void* dWork, size_t work_bytes,
                      void* stream, sp2_timing* timing);

/*
 * sp2_query -- synchronize `stream` and read the outcome of the last sp2_density call
 * that used this workspace (with the same n and options) into *info.  Returns the
 * device-side status.
 */
int sp2_query(const void* dWork, int n, const sp2_options* opt, sp2_info* info, void* stream);

/*
 * sp2_square -- one activation layer of Alg. 1 as a standalone operation (for tests
 * and benchmarks): Y = alpha X^2 + beta X + gamma I for a symmetric n x n matrix X
 * given in the state precision of `precision` (FP64 for SP2_FP64, FP32 otherwise;
 * leading dimension ld = n_padded from sp2_square_padded), written to dY with the same
 * layout.  For the split modes the planes of X are formed internally (Eq. Split2) and
 * the square uses Eq. Square.  The output is exactly symmetric.  dWork must hold
 * sp2_square_workspace_size(n, precision, tile, kernel) bytes.  Also returns, if trace_frob is
 * non-NULL (host, 2 doubles), Tr Y and ||Y||_F^2 in FP64 (synchronizes).
 */
int sp2_square_padded(int n, int precision, int tile);
size_t sp2_square_workspace_size(int n, int precision, int tile, int kernel);
int sp2_square(const void* dX, void* dY, int n, int precision, int tile, int kernel, int scale_log2,
               float alpha, float beta, float gamma, double* trace_frob, void* dWork,
               size_t work_bytes, void* stream);

/*
 * sp2_density_batched -- sp2_density for `batch` (1..8192) independent Hamiltonians of (possibly)
 * different sizes in one go: the batching of many small matrix products that the paper
 * (Sec. "Mixed Precision Fermi-operator expansion on tensor cores", its closing remark on
 * small N) expects to carry the SP2 recursion's rate to small matrices.  All arrays are HOST arrays of length `batch`; dH[i], dD[i]
 * are device pointers as in sp2_density.  Options apply to every problem (precision
 * SP2_FP16X2, SP2_BF16X2 or SP2_FP32; caller bounds are not accepted: each problem gets
 * its own Gershgorin bounds).  Every step of the recursion is one launch covering the
 * tiles of all problems (each problem keeps its own sigma history and stopping layer);
 * with use_graph != 0 the whole launch sequence is captured into a hipGraph and
 * launched once.  The call waits for `stream`, works on a private stream, synchronizes,
 * and fills infos[i] (host, may be NULL).  Returns SP2_OK or the first non-OK device
 * status; argument errors return before any work.  dWork: sp2_batched_workspace_size().
 */
size_t sp2_batched_workspace_size(int batch, const int* n, const sp2_options* opt);
int sp2_density_batched(int batch, const double* const* dH, const int* ldh, double* const* dD,
                        const int* ldd, const int* n, const int* n_occ, double tol,
                        const sp2_options* opt, sp2_info* infos, int use_graph, void* dWork,
                        size_t work_bytes, void* stream);

/*
 * sp2_density_batched_gap -- sp2_density_batched (the batching of Sec. "Mixed Precision
 * Fermi-operator expansion on tensor cores") with accelerated layers (Sec. Accelerated
 * Deep-NN SP2) for every problem: homo[i] < lumo[i] (host arrays, finite) is an interval
 * inside the HOMO-LUMO gap of H_i, as opt->homo/lumo of sp2_density with accelerate set;
 * opt->accelerate itself must be 0.  Each problem's result is the one sp2_density gives
 * with those options.  Same workspace as sp2_density_batched.
 */
int sp2_density_batched_gap(int batch, const double* const* dH, const int* ldh, double* const* dD,
                            const int* ldd, const int* n, const int* n_occ, const double* homo,
                            const double* lumo, double tol, const sp2_options* opt, sp2_info* infos,
                            int use_graph, void* dWork, size_t work_bytes, void* stream);

/*
 * Autotuner.  The automatic choices of sp2_density (tile = 0 and kernel = 0) and of
 * sp2_density_batched (tile = 0) come from a built-in rule unless the autotuner has
 * measured this case on the current device in this process; then its fastest choice is
 * used.  Tune before sizing workspaces: the workspace depends on the schedule.
 *
 * sp2_autotune -- for an n x n split-precision problem (SP2_FP16X2 or SP2_BF16X2): times
 *   one squaring layer of a synthetic symmetric matrix (reps launches after a warm-up,
 *   HIP events on `stream`) for every schedule that can run at this size (tiles 64/128/256,
 *   one workgroup per tile or a persistent variant, as the kernel option numbers them),
 *   records the fastest for sizes that round up to the same multiple of 256, and returns
 *   it in *tile, *kernel, *ms (host pointers, each may be NULL).  Synchronizes `stream`.
 *   dWork: sp2_autotune_workspace_size(n, precision) bytes, 256-byte aligned; its contents
 *   are overwritten.  Errors: SP2_EINVAL (bad n, precision, reps outside 1..1000, NULL or
 *   misaligned dWork), SP2_ENOMEM, SP2_EDEVICE; argument errors return before any work.
 * sp2_autotune_batched -- runs sp2_density_batched on these problems (same arguments; D is
 *   written) once per grouped-kernel tile (64, 128), twice each, timed on the host, and
 *   records the faster tile for this multiset of sizes.  dWork:
 *   sp2_autotune_batched_workspace_size() bytes.
 * sp2_autotune_reset -- forgets every measurement (built-in rules again).
 * The table is process-wide and guarded by a mutex.
 */
size_t sp2_autotune_workspace_size(int n, int precision);
int sp2_autotune(int n, int precision, int reps, int* tile, int* kernel, float* ms, void* dWork,
                 size_t work_bytes, void* stream);
size_t sp2_autotune_batched_workspace_size(int batch, const int* n, const sp2_options* opt);
int sp2_autotune_batched(int batch, const double* const* dH, const int* ldh, double* const* dD,
                         const int* ldd, const int* n, const int* n_occ, const sp2_options* opt,
                         int* tile, float* ms, void* dWork, size_t work_bytes, void* stream);
void sp2_autotune_reset(void);

/*
 * Differentiable generalized-SP2 network (Eq. general SP2 applied to matrices):
 *
 *     X_{k+1} = W_k X_k^2 + B_k X_k + c_k I,     k = 0 .. K-1
 *
 * with K trainable scalar triples (W_k, B_k, c_k) = (theta_{k,1}, theta_{k,2}, theta_{k,3}).
 * The SP2 branches are (1, 0, 0) for X^2 and (-1, 2, 0) for 2X - X^2.  X_0 must be
 * symmetric (e.g. the input layer S_0 of Alg. 1); every X_k then is.
 *
 *   precision   SP2_FP16X2 or SP2_BF16X2 (layers as in Alg. 2 with FP32 state) or SP2_FP32.
 *               The FP16X2 planes hold 2^12 X_k, so |X_k| entries must stay below 16.
 *   ckpt_every  c >= 1: X_k is kept for k = 0, c, 2c, ... and the backward recomputes the
 *               layers in between (memory: ceil(K/c) + c + 6 padded matrices); 0 selects
 *               c = 1 (every layer kept, nothing recomputed) while K + 7 padded FP32
 *               matrices take at most 8 GiB, else c = ceil(sqrt(K)).
 *   dW, dB, dC  device FP32 arrays of K coefficients.
 *
 * sp2_net_forward writes X_K (n x n FP32, leading dimension ldk) and keeps the checkpoints
 * in dWork.  sp2_net_backward takes G_K = dL/dX_K (FP32, any n x n matrix: X_K is symmetric,
 * so the library uses the symmetric part (G_K + G_K^T)/2, the gradient with respect to
 * symmetric perturbations) and the SAME dWork,
 * n, K, precision and ckpt_every as the preceding forward call, and writes
 * dL/dW_k = <G_{k+1}, X_k^2>_F, dL/dB_k = <G_{k+1}, X_k>_F, dL/dc_k = Tr G_{k+1} into
 * ddW, ddB, ddC (device FP32, K each) and, if dG0 != NULL, G_0 = dL/dX_0, where
 * G_k = W_k (G_{k+1} X_k + X_k G_{k+1}) + B_k G_{k+1}.  The adjoint layers run with FP32
 * operands on the matrix cores; reductions are FP64.  Both calls enqueue on `stream` and
 * return without synchronizing; errors are argument errors (SP2_EINVAL, SP2_ENOMEM) or
 * SP2_EDEVICE.
 */
size_t sp2_net_workspace_size(int n, int K, int precision, int ckpt_every);
int sp2_net_forward(const float* dX0, int ld0, int n, int K, const float* dW, const float* dB,
                    const float* dC, int precision, int ckpt_every, float* dXK, int ldk,
                    void* dWork, size_t work_bytes, void* stream);
int sp2_net_backward(const float* dGK, int ldg, int n, int K, const float* dW, const float* dB,
                     const float* dC, int precision, int ckpt_every, float* dG0, int ldg0,
                     float* ddW, float* ddB, float* ddC, void* dWork, size_t work_bytes,
                     void* stream);

/*
 * sp2_observable -- FP64 reductions of a density matrix D and an observable A (Alg. 1's
 * output Tr[D A]; with A = H the energy): out[0] = Tr D, out[1] = ||D||_F^2 and
 * out[2] = sum_ij D_ij A_ij, which is Tr[D A] for symmetric D and A.  dD, dA: device FP64
 * n x n (leading dimensions ldd, lda >= n); out: host, 3 doubles.  Fixed reduction order
 * (bit-reproducible).  dWork: sp2_observable_workspace_size(n) bytes, 256-byte aligned.
 * Synchronizes `stream`.  SP2_EINVAL, SP2_ENOMEM, SP2_EDEVICE, or SP2_ENONFINITE for a
 * non-finite sum.
 */
size_t sp2_observable_workspace_size(int n);
int sp2_observable(const double* dD, int ldd, const double* dA, int lda, int n, double* out, void* dWork,
                   size_t work_bytes, void* stream);

/*
 * sp2_estimate_gap -- HOMO/LUMO estimates from the history of a converged call (host
 * only; `info` as filled by sp2_density or sp2_density_batched for an n x n problem in
 * `precision`), for the accelerated layers of a later call on a similar H (opt->homo/lumo).
 * Near convergence IdErr is dominated by the LUMO image a and the HOMO deviation c; an
 * ordinary layer maps (a, c) to (a^2, 2c - c^2) or (2a - a^2, c^2), so two consecutive IdErr
 * values fix them, and the earlier layer maps (sigma_c, including accelerated ones) are
 * inverted exactly.  Every pair of layers with IdErr <= 0.25 and the next IdErr above the
 * rounding floor (1e-12 n in FP64, 1e-6 n otherwise) contributes; the highest HOMO and the
 * lowest LUMO estimate are kept and the interval is narrowed by 10 % of its width.
 * Estimates, not bounds: the accelerated call checks them (sp2_info.gap_violation).
 * Returns SP2_OK, or SP2_EINVAL when the history holds no usable pair (for example an
 * accelerated run whose last ordinary layers are at the rounding floor).
 */
int sp2_estimate_gap(const sp2_info* info, int n, int precision, double* homo, double* lumo);

/*
 * Optimized finite-temperature expansion (Sec. "Optimized SP2 Finite Temperature
 * Fermi-Operator Expansion"): L layers of Eq. general SP2 on the rescaled spectrum
 * x in [0, 1] of H,
 *     x_0 = x,  x_k = theta[3(k-1)] x_{k-1}^2 + theta[3(k-1)+1] x_{k-1} + theta[3(k-1)+2],
 * read out as F~(x) = 1 - sum_{i=0}^{L} c[i] x_i, fitted to the Fermi function
 * F = 1/(exp((e - mu)/kT) + 1) of Eq. fermi.
 *
 * sp2_fermi_fit (host only) fits theta (3 L doubles) and c (L + 1 doubles, host) by
 * Levenberg-Marquardt to F on `grid` equally spaced points of [0, 1] with trapezoid
 * weights, where x = (e - emin)/(emax - emin): mu and kT are in energy units and [emin,
 * emax] are the spectral bounds that sp2_fermi_apply will use.  Marquardt damping
 * (lambda from 1e-3, /10 on an accepted step, x10 otherwise), at most max_iter steps.
 * The start is the truncated SP2 expansion (x^2 or 2x - x^2 per layer, whichever keeps the
 * image of the rescaled mu closest to 1/2; read-out 1 - x_L).  *loss (may be NULL)
 * receives the weighted sum of squares.  1 <= layers <= 127, 3 <= grid <= 1e6,
 * kT > 0, emax > emin, or SP2_EINVAL.
 *
 * sp2_fermi_apply evaluates the fitted network on the matrix: X_0 = (H - emin I)/(emax -
 * emin) with opt->emin/emax (opt->have_bounds must be set: they are the bounds used in the
 * fit), X_{k+1} = theta_k,1 X_k^2 + theta_k,2 X_k + theta_k,3 I in opt->precision (the layer
 * kernels of sp2_density; split modes with FP32 state), and D = I - sum_i c_i X_i
 * accumulated in FP64, written n x n FP64 (leading dimension ldd, symmetric).  theta and c
 * are host arrays; dH, dD device.  Enqueued on `stream`; if obs (host, 3 doubles) is
 * non-NULL the call synchronizes and writes Tr D, ||D||_F^2 and Tr[D H] there.  dWork
 * (256-byte aligned) holds sp2_fermi_workspace_size(n, opt) bytes.  Errors: SP2_EINVAL
 * (arguments, non-finite coefficients, no bounds, accelerate set), SP2_ENOMEM,
 * SP2_EDEVICE, SP2_ENONFINITE (non-finite observables).
 *
 * sp2_spectral_bounds computes the FP64 Gershgorin bounds of Alg. 1's default (row
 * intervals widened outward by the summation error bound) on the device and returns them
 * to the host (synchronizes); workspace sp2_spectral_bounds_workspace_size(n) bytes.
 */
int sp2_fermi_fit(int layers, double mu, double kT, double emin, double emax, int grid, int max_iter,
                  double* theta, double* c, double* loss);
size_t sp2_fermi_workspace_size(int n, const sp2_options* opt);
int sp2_fermi_apply(const double* dH, int ldh, double* dD, int ldd, int n, int layers, const double* theta,
                    const double* c, const sp2_options* opt, double* obs, void* dWork, size_t work_bytes,
                    void* stream);
size_t sp2_spectral_bounds_workspace_size(int n);
int sp2_spectral_bounds(const double* dH, int ldh, int n, double* emin, double* emax, void* dWork,
                        size_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SP2_H */
