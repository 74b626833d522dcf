// Data layouts and descriptors of libdmp shared by host and device code.
// Pure C++17 (no HIP headers): the host-side planning code that includes it
// also builds with a plain host compiler, for the sanitizer tests.
#pragma once

#include <cstddef>
#include <cstdint>

#include "dmp.h"

namespace dmp {

#define DMP_CHECK(expr)                                                      \
    do {                                                                     \
        int st_ = (expr);                                                    \
        if (st_ < 0) return st_;                                             \
    } while (0)

// ---- error reporting (thread-local message) -------------------------------
void set_error(const char* fmt, ...);
void clear_error();
const char* error_text();

// ---- Ozaki split geometry -------------------------------------------------
// Digit planes are stored in "fragment blocks": 32 rows x CK reduction
// elements, 1 KiB each, laid out exactly as the 32x32 MFMA operand registers
// of one wavefront (lane l holds row l % 32 and 16 bytes of consecutive
// reduction index starting at (l / 32) * CK / 2).  For every (row block,
// chunk) the S planes are adjacent, so one chunk of one 32-row block is a
// single contiguous S KiB run.
//   INT8: CK = 32 (one v_mfma_i32_32x32x32_i8 per slice pair and chunk)
//   FP16: CK = 16 (one v_mfma_f32_32x32x16_f16 per slice pair and chunk)
constexpr int kFragRows = 32;
constexpr int kFragBytes = 1024;
constexpr int kTileM = 128;          // GEMM output tile rows (4 fragment rows)
constexpr int kTileN = 64;           // GEMM output tile columns (2 fragment rows)
constexpr int kGemmThreads = 512;    // 8 wavefronts, one 32 x 32 quadrant each
constexpr int kPad = 128;            // row padding of the digit planes
constexpr int kKPad = 64;            // reduction padding of the digit planes
constexpr int kMaxSlices = 12;
// Largest S with 64-row purification tiles (two workgroups per CU fit the
// registers without spills up to here).
constexpr int kMaxSlices64 = 8;
constexpr int kTopBits = 6;          // fractional bits of the first digit
constexpr int kDigitBits = 8;        // bits of every further digit
// Exponent recorded for a row (column) holding a NaN or an infinity; the
// products of such a row come out NaN.
constexpr int kNonFiniteExp = 1 << 20;

inline bool is_fp16_kind(dmp_kind kind) { return kind == DMP_OZ_FP16 || kind == DMP_MARKIDIS_FP16; }
inline int chunk_k(dmp_kind kind) { return is_fp16_kind(kind) ? 16 : 32; }
// Planes stored per operand: S digit planes for the Ozaki kinds, two (the
// high and low FP16 parts) for the Markidis kind, whose ``slices`` argument
// counts its terms.
inline int planes_of(int s, dmp_kind kind) { return kind == DMP_MARKIDIS_FP16 ? 2 : s; }
constexpr int kMaxTerms = 4;
constexpr int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Largest reduction length whose INT32 group sums cannot overflow:
// (g - 1) k 2^14 < 2^31 for every group g <= S + 1.
inline int64_t max_k_for_slices(int s) { return ((1ll << 31) - 1) / (int64_t(s) * 16384); }
// Reduction limit of a kind: the INT32 bound above for the Ozaki kinds; the
// Markidis kind accumulates in FP32 (inexact by design) and has none.
inline int64_t max_k_for(int s, dmp_kind kind) {
    return kind == DMP_MARKIDIS_FP16 ? (int64_t(1) << 30) : max_k_for_slices(s);
}

// Bytes of the digit planes of an R x K operand.
inline size_t plane_bytes(int64_t r, int64_t k, int s, dmp_kind kind) {
    return size_t(round_up(r, kPad)) * size_t(round_up(k, kKPad)) * size_t(planes_of(s, kind)) *
           (is_fp16_kind(kind) ? 2 : 1);
}

// One output tile of a (possibly grouped) GEMM: rows [128 I, 128 I + 128),
// columns [64 J, 64 J + 64) of matrix ``mat`` of a batch.
struct Tile {
    uint16_t I, J;
    uint32_t mat;
};

// Per-matrix descriptor of a grouped purification / GEMM, in device memory.
struct MatDesc {
    const uint8_t* pa;     // digit planes of the left operand (rows)
    const uint8_t* pb;     // digit planes of the right operand (columns)
    const int* ea;         // row exponents of the left operand
    const int* eb;         // column exponents of the right operand
    const double* P;       // current iterate
    const double* X2;      // square of the iterate
    const double* H;       // Hamiltonian
    double* out;           // output matrix
    uint64_t* colmax;      // nullable (EPI_STORE): atomicMax of the bit pattern
                           // of |out_ij| into colmax[j]; zeroed beforehand
    uint64_t* rowmax;      // nullable: atomicMax of the bit pattern of
                           // |out_ij| into rowmax[i] (and, in the mirrored
                           // modes, of |out_ji| into rowmax[j]), for the
                           // next split; zeroed beforehand by the caller
    int64_t a_rb_stride;   // bytes between 32-row blocks of pa
    int64_t b_rb_stride;   // bytes between 32-row blocks of pb
    int M, N, KC;          // rows, columns, reduction chunks
    int ldc;
    int state_index;       // index of the matrix's DevState
    int pad_;
};

// Device-side purification state of one matrix (host-readable copy).
struct DevState {
    double h_min, h_max, trace_h, mu, lambda, theta;
    double c, alpha, beta, gamma, t1, t2;
    double E, E_prev, dE, dE_prev, trace_p, tol;
    double ta, tb, tc;    // TRS4: T = ta X + tb X2 + tc I (right operand of X2 T)
    double E_unrefined;   // energy before the FP64 McWeeny refinement step
    int iters, done, stop_reason, branch;
    int method;           // DMP_CANONICAL or DMP_TRS4
    int refined;          // 1 once the McWeeny refinement step has run
    int products;         // matrix products performed so far
    int max_iter, nonfinite, n, nocc;
    int clamped;          // c_k clamped (or t1 == 0): no dependence of c on P
    int row_hmax;         // first row attaining h_max (Gershgorin)
    int row_hmin;         // first row attaining h_min
    int which;            // 0: lam = theta / (h_max - mu), 1: (1 - theta) / (mu - h_min)
};

// One operand to split (single launch: passed by value; grouped launch: an
// array in device memory, blocks mapped to matrices by the first-unit
// fields).
struct SplitDesc {
    const double* A;    // source matrix, row-major
    const double* A2;   // non-null: the operand is ta A + tb A2 + tc I with the
                        // coefficients of DevState state_index (trans == 0);
                        // skipped while that state's gamma is 0
    int64_t lda;
    int R, K;           // rows / reduction length of the operand
    int trans;          // 0: operand row r is A[r, :]; 1: operand row r is A[:, r]
    int KC;             // chunks along the reduction (padded K / CK)
    uint64_t* maxbits;  // [Rp] bit pattern of max |row|
    int* expo;          // [Rp] exponents
    uint8_t* planes;    // digit planes
    uint64_t* clear;    // nullable: rows [0, R padded) of this array are zeroed
                        // (the row maxima the next product accumulates)
    int ub_rowmax;      // first k_rowmax unit of this matrix (grouped)
    int ub_digits;      // first k_digits unit of this matrix (grouped)
    int state_index;    // -1: no state
    int sym;            // 1: A is symmetric and only its upper triangle (k >= r)
                        // holds it (trans == 0, A2 null): entry (r, k < r) is
                        // read as A[k, r]
};

// Per-matrix arguments of the small purification kernels.
struct PurDesc {
    const double* H;
    double* Pb[2];          // ping-pong iterates; Pb[0] is the caller's P
    double* X2;             // square (Ozaki) / X2 (native)
    double* X3;             // native only: X2 P (X2 T for TRS4)
    double* T;              // native TRS4: right operand T
    double* rows;           // [3 n]: Gershgorin low, high, diagonal per row
    int* rowbad;            // [n]: non-finite flag per row
    double* e0;             // [kE0Blocks] partial energies of P0
    double* partials;       // [(tile or block) count][kPartials]
    int n, nocc;
    int part_begin, part_end;   // partial range of this matrix
    int method;                 // DMP_CANONICAL or DMP_TRS4
    int pad_;
};

// Coefficient step run by extra blocks of a split launch (count > 0): block
// b < count computes the update weights of matrix b from the square's trace
// partials (method: DMP_CANONICAL or DMP_TRS4), the split's units follow.  The split of X2 reads only
// the done flags of the states these blocks write.
struct CoefArgs {
    const PurDesc* pd;
    DevState* st;
    int count;
    int method;
};

// Epilogue modes of the slice GEMM.
enum EpiMode : int {
    EPI_STORE = 0,     // C = A B (general, full tiles)
    EPI_SQUARE = 1,    // X2 = P P (upper tiles, mirrored) + traces for c
    EPI_UPDATE = 2,    // P' = a P + b X2 + g X2 P (upper, mirrored) + E, tr;
                       // g == 0 skips the products
    EPI_SQUARE_TRS4 = 3,  // X2 = X X (upper, mirrored) + tr F, tr G of TRS4
    EPI_STORE_SYM = 4, // C = A B known to be symmetric (square): upper tiles,
                       // C_ij stored and mirrored, no traces
};

constexpr int kPartials = 2;   // partial sums written per tile

// Arguments of one slice-GEMM launch.
struct GemmParams {
    const Tile* tiles;
    const MatDesc* descs;   // grouped launch (device); nullptr: use ``one``
    MatDesc one;
    double* partials;       // [tiles][kPartials] (purification modes)
    const DevState* states; // nullable; tiles of finished matrices exit
    int mode;
    // 0: give every XCD a contiguous slice of the tile list (L2 reuse of one
    // matrix's panels); 1: plain block order, for tile lists sorted from the
    // most to the least work (the hardware's round-robin over XCDs then
    // spreads every cost class evenly)
    int spread;
    // nullable (kernel timing): [0] += shader-clock cycles and [1] += 100 MHz
    // real-time ticks of every workgroup, from its start to its end
    unsigned long long* clk;
    // Reduction split of the last tiles (``fix`` null: no split).  Blocks [0, nfull) own tiles [0, nfull) whole.  Block nfull + u
    // owns part u % nsplit of tile nfull + u / nsplit: it reduces the chunks
    // [KC part / nsplit, KC (part + 1) / nsplit) and stores its INT32 group
    // sums at piece u of ``fix`` instead of running the epilogue.  The fixup
    // launch (one block per split tile) adds the parts of its tile (integer
    // sums: exact in any order) and runs the epilogue.
    int* fix;
    int nfull, nsplit;
    // purification modes: 1 stores only the upper triangle of the output
    // (no mirror; the next splits read it as symmetric, SplitDesc::sym)
    int upper_only;
};

// Tail split of a slice-GEMM launch: at most kMaxSplit parts per tile, at
// least kMinSplitChunks reduction chunks per part, at most kMaxPieces parts
// in all (the capacity of the part buffer).
constexpr int kMaxSplit = 8;
constexpr int kMinSplitChunks = 8;
constexpr int kMaxPieces = 512;
// INT32 group sums of one part: S accumulators of 16 values per lane of each
// wavefront.
inline size_t piece_ints(int S, int rb) { return size_t(2 * rb) * S * 16 * 64; }

}  // namespace dmp
