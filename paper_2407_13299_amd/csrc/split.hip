// Ozaki split (Sec. 2.4): power-of-two scaling per row (or column) and
// extraction of S signed 8-bit digits by round-to-nearest and shifts.
//
// For a row r with largest magnitude m_r, e_r is the frexp exponent
// (2^(e_r - 1) <= m_r < 2^e_r, 0 for a zero row) and every entry is scaled to
// x = a 2^(6 - e_r), |x| < 64.  Digit s is rint(x) (ties to even), the exact
// remainder x - rint(x) is shifted up by 8 bits for the next digit, and a
// final carry pass turns a digit of +128 into -128 plus one unit in the
// digit above, so digits 2..S are signed bytes and digit 1 lies in [-64, 65].
// Every step is exact in FP64; the value kept is a 2^-e_r rounded to the
// nearest multiple of 2^-(8S - 2).
//
// Output layout: see common.hpp (fragment blocks of 1 KiB, S planes of one
// (32-row block, chunk) adjacent).
#include "coef.hpp"
#include "common.hpp"
#include "plan.hpp"

#include <hip/hip_fp16.h>

namespace dmp {



template <bool ROWMAX>
__device__ inline const SplitDesc& pick(const SplitDesc* descs, int count,
                                        const SplitDesc& one, int unit, int* local) {
    if (descs == nullptr) {
        *local = unit;
        return one;
    }
    int lo = 0, hi = count - 1;
    while (lo < hi) {   // last matrix whose first unit <= unit
        int mid = (lo + hi + 1) >> 1;
        int b = ROWMAX ? descs[mid].ub_rowmax : descs[mid].ub_digits;
        if (b <= unit) lo = mid; else hi = mid - 1;
    }
    *local = unit - (ROWMAX ? descs[lo].ub_rowmax : descs[lo].ub_digits);
    return descs[lo];
}

__device__ inline bool finished(const DevState* st, int idx) {
    return st != nullptr && idx >= 0 && st[idx].done != 0;
}

// A combined operand (d.A2 set) is only needed when its product runs.
__device__ inline bool skipped(const SplitDesc& d, const DevState* st) {
    return finished(st, d.state_index) ||
           (d.A2 != nullptr && st[d.state_index].gamma == 0.0);
}

// Entry (r, k) of the combined operand ta A + tb A2 + tc I.  Written with
// explicit fused multiply-adds so that the row-max and the digit kernels
// compute the same value bit for bit.
__device__ inline double combine(double ta, double tb, double tc, double a, double a2, bool diag) {
    return __builtin_fma(ta, a, __builtin_fma(tb, a2, diag ? tc : 0.0));
}

__device__ inline double combined(const SplitDesc& d, const DevState& s, int r, int k) {
    const int64_t ij = int64_t(r) * d.lda + k;
    return combine(s.ta, s.tb, s.tc, d.A[ij], d.A2[ij], r == k);
}

// Magnitudes are compared as the bit patterns of |x|: for non-negative
// doubles the integer order is the numeric order, +inf sorts above every
// finite value and a NaN above +inf, so a non-finite entry is never lost.
__device__ inline uint64_t abs_bits(double x) {
    return static_cast<uint64_t>(__double_as_longlong(x)) & 0x7fffffffffffffffull;
}

__device__ inline uint64_t wave_max(uint64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t o = static_cast<uint64_t>(__shfl_xor(static_cast<long long>(v), off, 64));
        v = o > v ? o : v;
    }
    return v;
}

// Max |.| of every operand row (trans == 0): one wavefront per row, units are
// groups of 4 rows (one workgroup of 256 threads).
__global__ __launch_bounds__(256) void k_rowmax(const SplitDesc* descs, int count,
                                                SplitDesc one, const DevState* st) {
    int local;
    const SplitDesc& d = pick<true>(descs, count, one, blockIdx.x, &local);
    if (skipped(d, st)) return;
    const int lane = threadIdx.x & 63;
    const int r = local * 4 + (threadIdx.x >> 6);
    const int rp = int(round_up(d.R, kPad));
    if (r >= rp) return;
    uint64_t m = 0;
    if (r < d.R && d.A2 == nullptr) {
        const double* row = d.A + int64_t(r) * d.lda;
        for (int k = lane; k < d.K; k += 64) {
            const uint64_t b = abs_bits(row[k]);
            m = b > m ? b : m;
        }
    } else if (r < d.R) {
        const DevState& s = st[d.state_index];
        for (int k = lane; k < d.K; k += 64) {
            const uint64_t b = abs_bits(combined(d, s, r, k));
            m = b > m ? b : m;
        }
    }
    m = wave_max(m);
    if (lane == 0) d.maxbits[r] = m;
}

// Max |.| of every operand row when the operand row is a column of A
// (trans == 1).  Unit = (64 columns, 256 rows of A); partial maxima are
// combined with an integer atomicMax on the bit patterns (non-negative
// doubles order like their bits), so the result is order independent.
__global__ __launch_bounds__(256) void k_colmax(const SplitDesc* descs, int count,
                                                SplitDesc one, const DevState* st) {
    int local;
    const SplitDesc& d = pick<true>(descs, count, one, blockIdx.x, &local);
    if (finished(st, d.state_index)) return;
    const int cb = (d.R + 63) / 64;
    const int col = (local % cb) * 64 + (threadIdx.x & 63);
    const int k0 = (local / cb) * 256 + (threadIdx.x >> 6);
    __shared__ uint64_t red[4][64];
    uint64_t m = 0;
    if (col < d.R) {
        for (int k = k0, e = min(d.K, (local / cb) * 256 + 256); k < e; k += 4) {
            const uint64_t b = abs_bits(d.A[int64_t(k) * d.lda + col]);
            m = b > m ? b : m;
        }
    }
    red[threadIdx.x >> 6][threadIdx.x & 63] = m;
    __syncthreads();
    if (threadIdx.x < 64 && col < d.R) {
        uint64_t v = red[0][threadIdx.x];
        for (int w = 1; w < 4; ++w) v = red[w][threadIdx.x] > v ? red[w][threadIdx.x] : v;
        atomicMax(reinterpret_cast<unsigned long long*>(d.maxbits) + col,
                  static_cast<unsigned long long>(v));
    }
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int S>
__device__ inline void digits_of(double a, int e, int (&d)[S]) {
    // |x| < 64 for every finite entry; a row holding a non-finite value
    // (e == kNonFiniteExp) gets zero digits and NaN products.
    double x = e >= kNonFiniteExp ? 0.0 : ldexp(a, kTopBits - e);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        double q = rint(x);
        d[s] = int(q);
        x = (x - q) * 256.0;
    }
#pragma unroll
    for (int s = S - 1; s > 0; --s) {
        if (d[s] >= 128) {
            d[s] -= 256;
            d[s - 1] += 1;
        }
    }
}

// Nearest FP16 value of x (ties to even), computed exactly in FP64: 11
// significant bits for |x| >= 2^-14, a fixed quantum of 2^-24 below that (the
// FP16 subnormals).  Scaled entries have |x| < 1, so nothing overflows.
__device__ inline double nearest_fp16(double x) {
    int ex = 0;
    (void)frexp(x, &ex);
    const int q = ex - 11 > -24 ? ex - 11 : -24;
    return ldexp(rint(ldexp(x, -q)), q);
}

__device__ inline int exponent_of(uint64_t bits) {
    if (bits >= 0x7ff0000000000000ull) return kNonFiniteExp;
    int e = 0;
    (void)frexp(__longlong_as_double(static_cast<long long>(bits)), &e);
    return e;
}

// Digits: a workgroup of 4 wavefronts owns one 32-row block of the operand
// and 4 consecutive chunks of CK reduction elements (W = 4 CK); wave w turns
// chunk 4 q + w into its fragment block, where lane l owns operand row l % 32
// and NE = CK / 2 consecutive reduction elements (the MFMA operand layout).
// Operand rows that are matrix rows (trans == 0, also the combined operand)
// are first staged through LDS: the workgroup reads the 32 x W panel row by
// row, each wave 64 consecutive doubles per load, so the HBM reads are
// coalesced although every lane then needs a piece of its own row.  Columns
// (trans == 1) are read directly: there consecutive lanes own consecutive
// rows, which are adjacent in memory.
// HALVES (Markidis kind, S = 2, FP16): instead of digits, the high and low
// FP16 parts of x = a 2^-e (|x| < 1): X0 = FP16[x], X1 = FP16[x - X0].
// coef.count > 0: the first coef.count blocks of the grid run the coefficient
// step of the matrices instead (CoefArgs), beside the split's units.
template <int S, bool FP16, bool HALVES = false>
__global__ __launch_bounds__(256) void k_digits(const SplitDesc* descs, int count,
                                                SplitDesc one, const DevState* st, CoefArgs coef) {
    constexpr int CK = FP16 ? 16 : 32;
    constexpr int NE = CK / 2;
    constexpr int W = 4 * CK;
    constexpr int LDW = W + 2;   // row stride in doubles: rows start 4 banks apart
    constexpr int PER = kFragRows * W / 256;
    __shared__ double panel[kFragRows * LDW];
    if (int(blockIdx.x) < coef.count) {
        const int m = blockIdx.x;
        if (coef.method == DMP_TRS4)
            coef_trs4(coef.pd[m], coef.st[m], panel);
        else
            coef_canonical(coef.pd[m], coef.st[m], panel);
        return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int local;
    // a copy: held in scalar registers, so that the LDS stores below cannot
    // alias it and force its fields to be reloaded
    const SplitDesc d = pick<false>(descs, count, one, int(blockIdx.x) - coef.count, &local);
    if (skipped(d, st)) return;
    const int rb_count = int(round_up(d.R, kPad)) / kFragRows;
    const int kq_count = (d.KC + 3) / 4;
    if (local >= rb_count * kq_count) return;
    const int rb = local / kq_count, kq = local % kq_count;
    const int kc = kq * 4 + wave;
    const int r = rb * kFragRows + (lane & 31);
    const int k0 = kc * CK + (lane >> 5) * NE;
    const int e = exponent_of(d.maxbits[r]);
    if (kq == 0 && wave == 0 && lane < 32) {
        d.expo[r] = e;
        if (d.clear != nullptr) d.clear[r] = 0;
    }

    double v[NE];
    if (!d.trans) {
        // every wave takes part in the staging and the barrier
        // all loads are issued before the first LDS write, so PER of them
        // are in flight per lane
        const int kb = kq * W;
        double stage[PER];
        if (d.A2 != nullptr) {
            double stage2[PER];
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t, rr = q / W, cc = q % W;
                const int row = rb * kFragRows + rr, k = kb + cc;
                const bool in = row < d.R && k < d.K;
                stage[t] = in ? d.A[int64_t(row) * d.lda + k] : 0.0;
                stage2[t] = in ? d.A2[int64_t(row) * d.lda + k] : 0.0;
            }
            const DevState& s = st[d.state_index];
            const double ta = s.ta, tb = s.tb, tc = s.tc;
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t, rr = q / W, cc = q % W;
                const int row = rb * kFragRows + rr, k = kb + cc;
                stage[t] = (row < d.R && k < d.K)
                               ? combine(ta, tb, tc, stage[t], stage2[t], row == k)
                               : 0.0;
            }
        } else {
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t, rr = q / W, cc = q % W;
                const int row = rb * kFragRows + rr, k = kb + cc;
                stage[t] = (row < d.R && k < d.K) ? d.A[int64_t(row) * d.lda + k] : 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int q = threadIdx.x + 256 * t;
            panel[(q / W) * LDW + q % W] = stage[t];
        }
        __syncthreads();
        if (kc >= d.KC) return;
        const double* src = panel + (lane & 31) * LDW + wave * CK + (lane >> 5) * NE;
#pragma unroll
        for (int i = 0; i < NE; ++i) v[i] = src[i];
    } else {
        if (kc >= d.KC) return;
        if (r < d.R) {
#pragma unroll
            for (int i = 0; i < NE; ++i)
                v[i] = (k0 + i < d.K) ? d.A[int64_t(k0 + i) * d.lda + r] : 0.0;
        } else {
#pragma unroll
            for (int i = 0; i < NE; ++i) v[i] = 0.0;
        }
    }

    uint8_t* base = d.planes + (int64_t(rb) * d.KC + kc) * int64_t(S) * kFragBytes + lane * 16;
    if constexpr (HALVES) {
        static_assert(S == 2 && FP16, "the Markidis split stores two FP16 planes");
        uint32_t w[2][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint16_t hb[2][2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const double x = e >= kNonFiniteExp ? 0.0 : ldexp(v[2 * q + t], -e);
                const double hi = nearest_fp16(x);
                const double lo = nearest_fp16(x - hi);
                // both are FP16 values, so the conversions below are exact
                hb[0][t] = __half_as_ushort(__float2half_rn(float(hi)));
                hb[1][t] = __half_as_ushort(__float2half_rn(float(lo)));
            }
            w[0][q] = uint32_t(hb[0][0]) | (uint32_t(hb[0][1]) << 16);
            w[1][q] = uint32_t(hb[1][0]) | (uint32_t(hb[1][1]) << 16);
        }
        *reinterpret_cast<uint4*>(base) = make_uint4(w[0][0], w[0][1], w[0][2], w[0][3]);
        *reinterpret_cast<uint4*>(base + kFragBytes) = make_uint4(w[1][0], w[1][1], w[1][2], w[1][3]);
        return;
    }
    int dg[NE][S];
#pragma unroll
    for (int i = 0; i < NE; ++i) digits_of<S>(v[i], e, dg[i]);

#pragma unroll
    for (int s = 0; s < S; ++s) {
        uint4 out;
        if constexpr (!FP16) {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                w[q] = (uint32_t(uint8_t(dg[4 * q + 0][s]))) |
                       (uint32_t(uint8_t(dg[4 * q + 1][s])) << 8) |
                       (uint32_t(uint8_t(dg[4 * q + 2][s])) << 16) |
                       (uint32_t(uint8_t(dg[4 * q + 3][s])) << 24);
            out = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                __half lo = __int2half_rn(dg[2 * q][s]);
                __half hi = __int2half_rn(dg[2 * q + 1][s]);
                w[q] = uint32_t(__half_as_ushort(lo)) | (uint32_t(__half_as_ushort(hi)) << 16);
            }
            out = make_uint4(w[0], w[1], w[2], w[3]);
        }
        *reinterpret_cast<uint4*>(base + int64_t(s) * kFragBytes) = out;
    }
}

// ---------------------------------------------------------------------------
// Host launchers.

template <int S>
static void launch_digits_s(bool fp16, const SplitDesc* descs, int count, const SplitDesc& one,
                            const DevState* st, int units, const CoefArgs& coef,
                            hipStream_t stream) {
    if (fp16)
        k_digits<S, true><<<units + coef.count, 256, 0, stream>>>(descs, count, one, st, coef);
    else
        k_digits<S, false><<<units + coef.count, 256, 0, stream>>>(descs, count, one, st, coef);
}

using DigitsFn = void (*)(bool, const SplitDesc*, int, const SplitDesc&, const DevState*, int,
                          const CoefArgs&, hipStream_t);
static const DigitsFn kDigits[kMaxSlices + 1] = {
    nullptr,           launch_digits_s<1>,  launch_digits_s<2>,  launch_digits_s<3>,
    launch_digits_s<4>, launch_digits_s<5>,  launch_digits_s<6>,  launch_digits_s<7>,
    launch_digits_s<8>, launch_digits_s<9>,  launch_digits_s<10>, launch_digits_s<11>,
    launch_digits_s<12>};


// Split one operand.  ``d`` describes it; ``st`` (nullable) skips the work
// once the state's done flag is set.
int launch_split(const SplitDesc& d, int S, dmp_kind kind, const DevState* st,
                 hipStream_t stream) {
    const int rp = int(round_up(d.R, kPad));
    if (rp == 0) return DMP_OK;
    if (!d.trans) {
        k_rowmax<<<split_units_rowmax(d.R), 256, 0, stream>>>(nullptr, 0, d, st);
    } else {
        k_fill_u64<<<(rp + 255) / 256, 256, 0, stream>>>(d.maxbits, rp, 0ull);
        if (d.K > 0) k_colmax<<<split_units_colmax(d.R, d.K), 256, 0, stream>>>(nullptr, 0, d, st);
    }
    if (kind == DMP_MARKIDIS_FP16)
        k_digits<2, true, true><<<split_units_digits(d.R, d.KC), 256, 0, stream>>>(nullptr, 0, d, st,
                                                                                  CoefArgs{});
    else
        kDigits[S](kind == DMP_OZ_FP16, nullptr, 0, d, st, split_units_digits(d.R, d.KC),
                   CoefArgs{}, stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

// The digit kernel alone, for an operand whose maxima (d.maxbits: row maxima,
// or column maxima when d.trans) an earlier product's epilogue accumulated.
int launch_split_digits(const SplitDesc& d, int S, dmp_kind kind, const DevState* st,
                        hipStream_t stream) {
    if (round_up(d.R, kPad) == 0) return DMP_OK;
    if (kind == DMP_MARKIDIS_FP16)
        k_digits<2, true, true><<<split_units_digits(d.R, d.KC), 256, 0, stream>>>(nullptr, 0, d, st,
                                                                                  CoefArgs{});
    else
        kDigits[S](kind == DMP_OZ_FP16, nullptr, 0, d, st, split_units_digits(d.R, d.KC),
                   CoefArgs{}, stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

// Grouped split of count operands (row splits only); descs in device memory
// with ub_rowmax / ub_digits the first unit of every matrix in each kernel.
int launch_split_grouped_rowmax(const SplitDesc* descs_dev, int count, int units,
                                const DevState* st, hipStream_t stream) {
    if (units > 0) k_rowmax<<<units, 256, 0, stream>>>(descs_dev, count, SplitDesc{}, st);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

int launch_split_grouped_digits(const SplitDesc* descs_dev, int count, int units, int S,
                                dmp_kind kind, const DevState* st, hipStream_t stream,
                                const CoefArgs& coef) {
    if (units + coef.count <= 0) return DMP_OK;
    if (kind == DMP_MARKIDIS_FP16)
        k_digits<2, true, true><<<units + coef.count, 256, 0, stream>>>(descs_dev, count,
                                                                       SplitDesc{}, st, coef);
    else
        kDigits[S](kind == DMP_OZ_FP16, descs_dev, count, SplitDesc{}, st, units, coef, stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

}  // namespace dmp
