/*
 * dmp.h -- density-matrix purification with Ozaki-scheme products on AMD
 * Instinct MI355X (gfx950).  Plain C ABI: device pointers, sizes, status codes.
 *
 * Method (arXiv:2407.13299):
 *   - Ozaki scheme (Sec. 2.4): a product A B is computed by scaling every row
 *     of A and every column of B by a power of two, splitting the scaled
 *     values into S fixed-point slices that are exact in the low-precision
 *     format, multiplying the slice pairs (i + j <= S + 1, S(S+1)/2 products)
 *     without rounding error on the matrix cores, and summing the results in
 *     FP64.  Slices here are signed 8-bit digits: the first carries 6
 *     fractional bits, every further one 8 bits, rounded to nearest, so S
 *     slices hold 8S - 2 bits of every row (column) relative to its largest
 *     entry.  The slice products run on INT8 MFMA with exact INT32
 *     accumulation (DMP_OZ_INT8) or FP16 MFMA with FP32 accumulation flushed
 *     into INT32 before it can round (DMP_OZ_FP16).
 *   - Density-matrix purification (Sec. 2.3; canonical, trace-conserving
 *     form of Palser and Manolopoulos cited in Sec. 1): from
 *     P0 = lam (mu I - H) + (nocc/n) I the iteration
 *        c  = tr(P^2 - P^3) / tr(P - P^2)   (clamped to [0, 1])
 *        P <- ((1 + c) P^2 - P^3) / c                  if c >= 1/2
 *        P <- ((1 - 2c) P + (1 + c) P^2 - P^3) / (1 - c) otherwise
 *     converges to the projector onto the nocc lowest eigenvectors of H.
 *     Only the two products per iteration run in low precision; everything
 *     else is FP64 (Sec. 4).
 *   - Stopping (Sec. 3): |E_k - E_{k-1}| < tol with E = tr(P H); stagnation
 *     when E rose in each of the last two iterations by less than 1e-2 Ha;
 *     or max_iter.
 *
 * Conventions for every entry point
 *   - Matrices are row-major FP64 in DEVICE memory owned by the caller.
 *     H, P and W are n x n, symmetric, leading dimension n.  Outputs must not
 *     alias inputs.
 *   - ``stream`` is a hipStream_t (NULL = the default stream).  GEMM entry
 *     points are asynchronous on it; purification entry points block until
 *     the result is ready (they read the convergence state once per batch
 *     of iterations).
 *   - ``ws`` / ``ws_bytes``: caller-provided device workspace of at least the
 *     size returned by the matching *_workspace_bytes query; 256-byte
 *     alignment.  Its contents are scratch and need no initialisation.
 *   - Return value: a dmp_status.  Negative values are errors and leave the
 *     outputs unspecified; dmp_last_error() describes the last error of the
 *     calling thread.  DMP_NOT_CONVERGED is positive: P, E and info are
 *     still written.
 *   - Determinism: no floating-point atomics; identical inputs give
 *     bitwise-identical outputs on the same device.
 *   - Threads: the purification entry points (dmp_purify*, the batched and
 *     taped variants and dmp_purify_bwd) take one process-wide lock, so
 *     purifications from several host threads run one after another.  The
 *     GEMM entry points take no lock.  Calls that share a workspace must not
 *     overlap.
 *   - Purification runs with the same workspace, sizes, kind, slice count
 *     and method replay recorded launch sequences (hipGraphs, kept per
 *     device for the life of the process, at most 16): a repeated run is one
 *     graph launch of as many iterations as the previous such run needed,
 *     then one read of the device state.
 *   - Environment switches, for measurements only (results are the same,
 *     bit for bit, except for the tile height, which sets the order of the
 *     trace sums): DMP_TAIL_SPLIT=0 keeps every product tile whole,
 *     DMP_TILE_ROWS=64 or 128 forces the purification tile height,
 *     DMP_NO_GRAPH=1 launches the iterations eagerly.
 */
#ifndef DMP_H
#define DMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMP_OK = 0,
    DMP_NOT_CONVERGED = 1,   /* stagnated, hit max_iter or went non-finite */
    DMP_EINVAL = -1,         /* bad size, pointer, kind or slice count      */
    DMP_ENONFINITE = -2,     /* H holds a NaN or an infinity                */
    DMP_EHIP = -3,           /* a HIP or rocBLAS call failed                */
    DMP_ENOMEM = -4,         /* workspace missing or smaller than required  */
    DMP_EUNSUPPORTED = -5    /* no gfx950 device / combination not built    */
} dmp_status;

typedef enum {
    DMP_FP64_NATIVE = 0,     /* products by rocBLAS DGEMM (FP64 baseline)   */
    DMP_OZ_INT8 = 1,         /* Ozaki slices on INT8 MFMA, INT32 accumulate */
    DMP_OZ_FP16 = 2,         /* Ozaki slices on FP16 MFMA, FP32 accumulate  */
    DMP_MARKIDIS_FP16 = 3    /* Markidis split (Sec. 4.5): high and low FP16
                                parts after the same row / column power-of-two
                                scaling, 1..4 term products (``slices`` counts
                                the terms: A0B0, +A0B1, +A1B0, +A1B1) on FP16
                                MFMA with FP32 accumulation; not exact      */
} dmp_kind;

typedef enum {
    DMP_CANONICAL = 0,       /* canonical trace-conserving purification      */
    DMP_TRS4 = 1             /* trace-resetting fourth order (Sec. 3)        */
} dmp_method;

/* Flags of the *_ex purification entry points. */
enum {
    DMP_REFINE_MCWEENY = 1,  /* one FP64 step P <- 3P^2 - 2P^3 at the end    */
    DMP_NATIVE_TRIANGLE = 2  /* DMP_FP64_NATIVE: products by rocBLAS dsyrk /
                                dsyrkx on the upper triangle only (the saving
                                the Ozaki kinds make), ignored otherwise    */
};

enum {
    DMP_STOP_CONVERGED = 0,
    DMP_STOP_STAGNATED = 1,
    DMP_STOP_MAX_ITER = 2,
    DMP_STOP_NONFINITE = 3
};

/* Per-run report.  trace = tr P of the returned P; idem = tr(P - P^2)
 * (canonical) or ||P - P^2||_F^2 (TRS4) of the last iterate the products
 * were formed from. */
typedef struct {
    int iters;          /* purification updates performed                */
    int stop_reason;    /* DMP_STOP_*                                     */
    int slices;         /* S used (0 for DMP_FP64_NATIVE)                 */
    int kind;           /* dmp_kind used                                  */
    double E;           /* tr(P H) of the returned P (Ha)                 */
    double last_dE;     /* E_k - E_{k-1} at the last iteration            */
    double trace;       /* tr P                                           */
    double idem;        /* tr(P - P^2), computed before the last update   */
    double h_min, h_max;/* Gershgorin bounds of H                         */
    double mu, lambda;  /* canonical: tr(H)/n and the scale of the initial
                           guess; TRS4: h_max and 1 / (h_max - h_min)     */
    int method;         /* dmp_method used                                */
    int refined;        /* 1 if the McWeeny refinement step ran           */
    double E_unrefined; /* tr(P H) before refinement (= E if not refined) */
    int products;       /* n x n matrix products performed (canonical: 2 per
                           iteration; TRS4: 1 or 2; refinement: 2)        */
} dmp_info;

/* Text of the last error on the calling thread ("" if none). */
const char* dmp_last_error(void);
/* Library version string. */
const char* dmp_version(void);
/* Largest supported slice count for an Ozaki kind, term count for the
 * Markidis kind (4), 0 for native. */
int dmp_max_slices(dmp_kind kind);

/* ---------------------------------------------------------------------
 * Ozaki-scheme GEMM (Sec. 2.4):  C = op(A) op(B),  op(X) = X or X^T.
 *   op(A) is m x k, op(B) is k x n, C is m x n; all row-major with leading
 *   dimensions lda, ldb, ldc (>= the stored row length, >= 1).
 *   slices in [1, dmp_max_slices(kind)]; kind DMP_OZ_INT8 or DMP_OZ_FP16
 *   (DMP_FP64_NATIVE runs rocBLAS DGEMM, slices ignored).
 *   m, n, k >= 0 (k == 0 writes zeros; m or n == 0 does nothing).
 *   Result: for every (i, j) the FP64 sum of the slice products, within
 *   k 2^(e_i + f_j) (S + 3) 2^(2 - 8S) + (S + 2) 2^-53 (|A||B|)_ij of the
 *   exact product, where 2^(e_i - 1) <= max|row i of op(A)| < 2^e_i and f_j
 *   likewise for column j of op(B).  Asynchronous on ``stream``.
 *   The workspace size depends on the current device as well: when the
 *   output tiles do not fill whole rounds of its CUs, it includes a buffer
 *   for the last round's partial sums.  Query on the device that runs the
 *   product (DMP_TAIL_SPLIT=0 in the environment, at query and at run time,
 *   keeps every tile whole and the buffer out).
 * ------------------------------------------------------------------- */
size_t dmp_gemm_workspace_bytes(int m, int n, int k, int slices, dmp_kind kind);
int dmp_ozaki_gemm(char transA, char transB, int m, int n, int k,
                   const double* A, int lda, const double* B, int ldb,
                   double* C, int ldc, int slices, dmp_kind kind,
                   void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of dmp_ozaki_gemm, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, result and
 * asynchrony as dmp_ozaki_gemm with kind DMP_OZ_INT8, DMP_OZ_FP16 or
 * DMP_MARKIDIS_FP16 (DMP_FP64_NATIVE returns DMP_EINVAL), but no workspace:
 * the digit planes, exponents, maxima and tile list live in a 64 MiB array
 * that the library holds on every GPU it runs on until the process ends.
 * A product whose scratch exceeds it returns DMP_EINVAL with the size it
 * needs (it holds m = n = k = 2048 at S <= 7, about plane bytes
 * (m + n) k S plus a few arrays; FP16 planes take twice that).  All tiles
 * run whole (no split tail).  The call makes no allocation (no hipMalloc,
 * hipFree or allocating library routine).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (from several streams or
 * threads) race, so the caller orders them on one stream or serialises
 * them. */
int dmp_ozaki_gemm_noalloc(char transA, char transB, int m, int n, int k,
                           const double* A, int lda, const double* B, int ldb,
                           double* C, int ldc, int slices, dmp_kind kind,
                           void* stream);

/* Grouped GEMM: count independent products C_b = A_b B_b (no transposes,
 * row-major, leading dimensions equal to the row lengths), all with the
 * same slices and kind.  The row splits of all A_b and the slice GEMM of all
 * products are one grouped launch each; the column split of every B_b is a
 * launch of its own.  m, n, k and the pointer arrays are HOST arrays of
 * length count; the matrices are on the device.  Returns 0 from the
 * workspace query for a null array or a size below 1.  Synchronises the
 * stream once, after copying the per-product descriptors into the workspace
 * (so work queued on the stream before the call is waited for); the splits
 * and the product are then queued asynchronously, like dmp_ozaki_gemm. */
size_t dmp_gemm_batched_workspace_bytes(int count, const int* m, const int* n,
                                        const int* k, int slices, dmp_kind kind);
int dmp_ozaki_gemm_batched(int count, const int* m, const int* n, const int* k,
                           const double* const* A, const double* const* B,
                           double* const* C, int slices, dmp_kind kind,
                           void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Canonical purification of one symmetric H (n x n, device, row-major).
 *   nocc in [0, n] (nocc = 0 gives P = 0, nocc = n gives P = I, no
 *   iterations); tol > 0 (Ha); max_iter >= 1; slices per dmp_max_slices
 *   (ignored for DMP_FP64_NATIVE).
 *   Outputs: P (device, n x n, exactly symmetric), *E (host) = tr(P H),
 *   *info (host, may be NULL).
 *   H is read as symmetric (the initial guess and the energy use its upper
 *   triangle; the Gershgorin bounds use whole rows).  A non-finite entry in
 *   H returns DMP_ENONFINITE.  Blocks until done.
 * ------------------------------------------------------------------- */
size_t dmp_purify_workspace_bytes(int n, int slices, dmp_kind kind);
int dmp_purify(const double* H, int n, int nocc, double tol, int slices,
               dmp_kind kind, int max_iter, double* P, double* E,
               dmp_info* info, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Purification with a choice of method and an optional refinement step.
 *   method DMP_CANONICAL: as dmp_purify.
 *   method DMP_TRS4 (the purification the paper runs, Sec. 3):
 *     X0 = (h_max I - H) / (h_max - h_min) (Gershgorin bounds); per
 *     iteration X2 = X X, gamma = (nocc - tr F) / tr G with
 *     F = X2 (4X - 3 X2) and G = X2 (I - X)^2, and
 *       0 <= gamma <= 6:  X <- X2 T,  T = (4 - 2 gamma) X + (gamma - 3) X2 + gamma I
 *       gamma > 6:        X <- 2X - X2        (no second product)
 *       gamma < 0:        X <- X2             (no second product)
 *     (tr G = 0 is read as gamma = 0); the same stopping rule.
 *   flags & DMP_REFINE_MCWEENY: after the iteration stops (unless it went
 *     non-finite or ran no iteration) one McWeeny step P <- 3P^2 - 2P^3 runs
 *     with rocBLAS FP64 products (Sec. 4.1); *E and info->E are then the
 *     refined energy and info->E_unrefined the energy before it.
 *   flags & DMP_NATIVE_TRIANGLE (kind DMP_FP64_NATIVE only): X2 by rocBLAS
 *     dsyrk and the second product by dsyrkx, upper triangle only.
 *   Other arguments, the workspace (dmp_purify_workspace_bytes covers every
 *   method and flag) and the blocking behaviour are those of dmp_purify.
 * ------------------------------------------------------------------- */
int dmp_purify_ex(const double* H, int n, int nocc, double tol, int slices,
                  dmp_kind kind, int max_iter, int method, int flags,
                  double* P, double* E, dmp_info* info, void* ws,
                  size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Batched purification: count independent Hamiltonians of (possibly)
 * different sizes n[b] with nocc[b] occupied levels, sharing tol, kind and
 * max_iter.  slices <= 0 picks S per matrix from the tuned table (see
 * dmp_autotune_slices); matrices that need fewer slices than the batch's
 * largest count then run with that count (never less accurate) when they
 * carry under a quarter of the batch's n^3 work, so the batch stays one
 * group of launches.  info[b].slices reports the count used.  H and P are HOST arrays of device pointers; n,
 * nocc are host arrays; E (host, length count) and info (host, length
 * count, may be NULL) receive the per-matrix results.  Every phase of an
 * iteration runs as one grouped launch over all unfinished matrices, and
 * the per-iteration launch sequence is captured once in a hipGraph and
 * replayed.  Returns DMP_NOT_CONVERGED if any matrix did not converge.
 * ------------------------------------------------------------------- */
size_t dmp_purify_batched_workspace_bytes(int count, const int* n, int slices,
                                          dmp_kind kind);
int dmp_purify_batched(int count, const double* const* H, const int* n,
                       const int* nocc, double tol, int slices, dmp_kind kind,
                       int max_iter, double* const* P, double* E,
                       dmp_info* info, void* ws, size_t ws_bytes, void* stream);

/* dmp_purify_batched with a method and flags as in dmp_purify_ex (the
 * workspace query of dmp_purify_batched covers them). */
int dmp_purify_batched_ex(int count, const double* const* H, const int* n,
                          const int* nocc, double tol, int slices,
                          dmp_kind kind, int max_iter, int method, int flags,
                          double* const* P, double* E, dmp_info* info,
                          void* ws, size_t ws_bytes, void* stream);

/* Slice count the tuned table recommends for an n x n purification to reach
 * max|dP| <= target on the given kind: the smallest S whose modelled error
 * C n^a 2^(1 - 8S) is <= target, with C and a fitted to measured errors and
 * compiled in (the largest supported S if none qualifies). */
int dmp_autotune_slices(int n, double target, dmp_kind kind);

/* ---------------------------------------------------------------------
 * Adjoint of the purification (reverse mode).  dmp_purify_fwd_tape runs
 * dmp_purify and records, for every iteration, the branch, c and the
 * traces, plus a copy of H and the iterate P_k for every k that is a
 * multiple of ckpt_stride, in device memory owned by the tape (allocated
 * here, released by dmp_tape_free).  ckpt_stride = 1 also keeps X2_k = P_k^2
 * of every step, so that the backward pass recomputes nothing;
 * ckpt_stride <= 0 picks 1 when 2 max_iter n^2 doubles take at most a
 * quarter of the free device memory, else ceil(sqrt(max_iter)).  Only the
 * Ozaki kinds are supported.
 * dmp_purify_bwd takes Pbar = dL/dP (device, symmetric n x n; for
 * L = tr(P W) it is W) and writes Hbar = dL/dH (device, symmetric), the
 * derivative of the recorded iteration (fixed branch pattern) including the
 * dependence of every c_k on P_k and of the initial guess on tr H and the
 * Gershgorin bounds.  Iterates between checkpoints are recomputed with the
 * same products, so every ckpt_stride gives the same Hbar bit for bit.
 * Each backward step costs 3 products (M = Y P and M P in full, the
 * symmetric P M on its upper triangle), plus the recomputation of 2 unless
 * the tape holds every step (ckpt_stride 1).
 * ------------------------------------------------------------------- */
typedef struct dmp_tape dmp_tape;
int dmp_purify_fwd_tape(const double* H, int n, int nocc, double tol,
                        int slices, dmp_kind kind, int max_iter,
                        int ckpt_stride, double* P, double* E, dmp_info* info,
                        dmp_tape** tape, void* stream);
size_t dmp_purify_bwd_workspace_bytes(const dmp_tape* tape);
int dmp_purify_bwd(const dmp_tape* tape, const double* Pbar, double* Hbar,
                   void* ws, size_t ws_bytes, void* stream);
/* Number of iterations and branch of each (host array of length >= iters). */
int dmp_tape_info(const dmp_tape* tape, int* iters, int* branches);
/* Recorded c_k, tr(P_k - P_k^2) and tr(P_k^2 - P_k^3) of every iteration
 * (host arrays of length >= iters; any may be NULL). */
int dmp_tape_coefficients(const dmp_tape* tape, double* c, double* t1, double* t2);
void dmp_tape_free(dmp_tape* tape);

/* ---------------------------------------------------------------------
 * Kernel timing (instrumentation; process-wide state, not for concurrent
 * use from several host threads).  dmp_timing_enable(1) or (2): the
 * purification entry points record a HIP event pair on the caller's stream
 * around every slice-GEMM launch (and launch without graph capture), and
 * accumulate the durations once each batch of iterations has completed;
 * (2) also turns on the clock counters read by dmp_timing_clock (a few
 * instructions and two atomic adds per workgroup); 0 turns timing off.
 *   which = 0: the squaring GEMM (P P), 1: the update GEMM (X2 P).
 *   *total_ms: summed kernel time; *launches: number of launches timed;
 *   *ops: summed algorithmic integer (or FP16) operations of those
 *   launches, 2 * S(S+1)/2 * n * n(n+1)/2 per launch (the upper triangle of
 *   an n x n product; padding excluded).
 * ------------------------------------------------------------------- */
void dmp_timing_enable(int on);
void dmp_timing_reset(void);
int dmp_timing_read(int which, double* total_ms, long long* launches, double* ops);

/* Mean shader clock (GHz) inside the slice-GEMM launches of kind ``which``
 * timed in mode 2 since the last dmp_timing_reset: every workgroup adds its
 * span in shader-clock cycles (s_memtime) and in 100 MHz
 * real-time ticks (s_memrealtime) to two device counters, and the clock is
 * their ratio.  *ghz = 0 when nothing was timed.  Blocks for one small
 * device-to-host copy.  The device counters are allocated on the first
 * timed launch and kept until the process ends. */
int dmp_timing_clock(int which, double* ghz);

#ifdef __cplusplus
}
#endif
#endif /* DMP_H */
