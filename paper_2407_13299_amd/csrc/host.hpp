// Host-side helpers of libdmp (no device code).
#pragma once

#include <rocblas/rocblas.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.hpp"
#include "plan.hpp"

namespace dmp {

// Device copy of the tile order of a single tm x tn product, cached per
// device for the life of the process.
int cached_tiles(int tm, int tn, bool upper, const Tile** out, int TM = kTileM);

// rocBLAS handle of the current device (created once), bound to ``stream``.
int blas_handle(hipStream_t stream, rocblas_handle* out);

// C = A B for row-major n x n ... general: C (m x n) = op(A) op(B).
int native_dgemm(hipStream_t stream, bool ta, bool tb, int m, int n, int k, const double* A,
                 int lda, const double* B, int ldb, double* C, int ldc);

int launch_split(const SplitDesc& d, int S, dmp_kind kind, const DevState* st, hipStream_t s);
int launch_split_digits(const SplitDesc& d, int S, dmp_kind kind, const DevState* st,
                        hipStream_t stream);
int launch_split_grouped_rowmax(const SplitDesc* descs_dev, int count, int units,
                                const DevState* st, hipStream_t stream);
// coef.count > 0: the same launch also runs the coefficient step of the
// matrices (extra blocks ahead of the split's units).  combined: the
// descriptors hold combined operands (A2 set, every one of them); otherwise
// none may.
int launch_split_grouped_digits(const SplitDesc* descs_dev, int count, int units, int S,
                                dmp_kind kind, const DevState* st, hipStream_t stream,
                                const CoefArgs& coef = CoefArgs{}, bool combined = false);

struct GemmParams;
// 32-row blocks per slice-GEMM tile (2: 64-row tiles, 4: 128-row tiles) of
// the products of an n x n Ozaki purification (and of its adjoint); a
// function of (kind, S, n) only.  The general GEMM entry points keep 128-row
// tiles, which measured faster on dense random operands.
int tile_blocks_for(dmp_kind kind, int S, int n);

// rb: 32-row blocks per tile of the left operand (4, or 2 for the 64-row
// variant: Ozaki kinds, S <= kMaxSlices64)
int launch_ozgemm(int S, dmp_kind kind, const GemmParams& p, int ntiles, hipStream_t stream,
                  int rb = 4);
// Workgroups of the purification-mode slice GEMM (kind, S, rb) resident on
// the current device at once (CUs x workgroups per CU).
int gemm_slots(int S, dmp_kind kind, int rb, int* slots);
// gemm_slots cached per device (the query costs microseconds per call)
int resident_slots(int S, dmp_kind kind, int rb, int* slots);

// DMP_TAIL_SPLIT = 0 keeps every tile whole (for measurements).
bool tail_split_enabled();
// DMP_TILE_ROWS = 64 or 128 forces one tile height where both exist (for
// measurements): 2 or 4 row blocks, 0 when unset.
int forced_tile_rb();
// The tuned tile choice of an n x n purification's products, with the
// forced height applied.
TileChoice tile_choice_env(dmp_kind kind, int S, int n);

// Waits for the stream when it goes out of scope, so that host buffers
// declared before it outlive the asynchronous copies that read them, also
// on early error returns.
struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

int native_dsyrk_upper(hipStream_t stream, int n, const double* A, double* C);
int native_dsyrkx_upper(hipStream_t stream, int n, const double* A, const double* B, double* C);
int purify_many(int count, const double* const* H, const int* n, const int* nocc, double tol,
                const int* slices, dmp_kind kind, int max_iter, int method, int flags,
                double* const* P, double* E, dmp_info* info, void* ws, size_t ws_bytes,
                hipStream_t s, size_t* need_out);

// Small purification kernels (purify.hip), one block / matrix per entry of pd.
int launch_purify_init(const PurDesc* pd, DevState* st, int count, int max_n, double tol,
                       int max_iter, hipStream_t s);
int launch_finalize_coef(const PurDesc* pd, DevState* st, int count, hipStream_t s);
int launch_finalize_iter(const PurDesc* pd, DevState* st, int count, hipStream_t s);
int e0_blocks();

}  // namespace dmp
