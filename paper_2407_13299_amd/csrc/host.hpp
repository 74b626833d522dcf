// Host-side helpers of libdmp (no device code).
#pragma once

#include <rocblas/rocblas.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace dmp {

// Carves 256-byte-aligned regions out of a workspace; with base == nullptr it
// only measures.
class Carver {
public:
    explicit Carver(void* base) : base_(static_cast<uint8_t*>(base)) {}
    template <typename T>
    T* take(size_t count) {
        off_ = (off_ + 255) & ~size_t(255);
        T* p = base_ ? reinterpret_cast<T*>(base_ + off_) : nullptr;
        off_ += count * sizeof(T);
        return p;
    }
    size_t used() const { return (off_ + 255) & ~size_t(255); }

private:
    uint8_t* base_;
    size_t off_ = 0;
};

// Order of the TM x 64 output tiles of one matrix (TM = 128, or 64 for the
// 64-row variant): 512 x 512 super-tiles, row-major over super-tiles and
// within each; ``upper`` keeps the tiles that reach the upper triangle
// (column >= row somewhere in the tile).
void append_tiles(std::vector<Tile>& out, int tm, int tn, bool upper, uint32_t mat,
                  int TM = kTileM);
int tile_rows(int m, int TM = kTileM);
int tile_cols(int n);
int upper_tile_count(int n, int TM = kTileM);

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
// matrices (extra blocks ahead of the split's units)
int launch_split_grouped_digits(const SplitDesc* descs_dev, int count, int units, int S,
                                dmp_kind kind, const DevState* st, hipStream_t stream,
                                const CoefArgs& coef = CoefArgs{});
int split_units_rowmax(int R);
int split_units_digits(int R, int KC);

struct GemmParams;
// 32-row blocks per slice-GEMM tile (2: 64-row tiles, 4: 128-row tiles) of
// the products of an n x n Ozaki purification (and of its adjoint); a
// function of (kind, S, n) only.  The general GEMM entry points keep 128-row
// tiles, which measured faster on dense random operands.
int tile_blocks_for(dmp_kind kind, int S, int n);

// rb: 32-row blocks per tile of the left operand (4, or 2 for the 64-row
// variant: Ozaki kinds, S <= 7)
int launch_ozgemm(int S, dmp_kind kind, const GemmParams& p, int ntiles, hipStream_t stream,
                  int rb = 4);
// Workgroups of the purification-mode slice GEMM (kind, S, rb) resident on
// the current device at once (CUs x workgroups per CU).
int gemm_slots(int S, dmp_kind kind, int rb, int* slots);
// gemm_slots cached per device (the query costs microseconds per call)
int resident_slots(int S, dmp_kind kind, int rb, int* slots);

// Tail split of ``ntiles`` tiles of equal cost: tiles [0, nfull) whole, the
// rest in nsplit parts each (nsplit == 1: no split).
struct TailSplit {
    int nfull, nsplit;
};
// ``slots`` workgroups run at once, so the tiles run in full rounds and a
// last round of r = ntiles mod slots tiles that leaves the rest of the chip
// idle; when there is at least one full round, those r tiles are split into
// as many parts as fill it (at most
// kMaxSplit, at least kMinSplitChunks of the ``min_kc`` chunks each, at most
// ``max_pieces`` parts in all).
TailSplit plan_tail_split(int ntiles, int slots, int min_kc, int max_pieces);
// DMP_TAIL_SPLIT = 0 keeps every tile whole (for measurements).
bool tail_split_enabled();
// Parts of a tail split a group of ``ntiles`` tiles of height 32 rb may need
// (the size of its part buffer in pieces, 0 when no split can arise).
int tail_split_capacity(int ntiles, int min_kc, int rb);

int native_dsyrk_upper(hipStream_t stream, int n, const double* A, double* C);
int native_dsyrkx_upper(hipStream_t stream, int n, const double* A, const double* B, double* C);
int check_kind_slices(dmp_kind kind, int slices);
int validate_purify_args(const double* H, int n, int nocc, double tol, int max_iter,
                         const double* P);
int check_method_flags(int method, int flags);
int purify_many(int count, const double* const* H, const int* n, const int* nocc, double tol,
                const int* slices, dmp_kind kind, int max_iter, int method, int flags,
                double* const* P, double* E, dmp_info* info, void* ws, size_t ws_bytes,
                hipStream_t s, size_t* need_out);
int64_t chunks_of(int k, dmp_kind kind);

// Small purification kernels (purify.hip), one block / matrix per entry of pd.
int launch_purify_init(const PurDesc* pd, DevState* st, int count, int max_n, double tol,
                       int max_iter, hipStream_t s);
int launch_finalize_coef(const PurDesc* pd, DevState* st, int count, hipStream_t s);
int launch_finalize_iter(const PurDesc* pd, DevState* st, int count, hipStream_t s);
int e0_blocks();

}  // namespace dmp
