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
// nearest multiple of 2^-(8S - 2).  Up to S = 8 the kernel forms the same
// digits from that integer, X = rint(a 2^(8S - 2 - e_r)), and its bytes (see
// k_digits); the rounding steps above serve S >= 9.
//
// Output layout: see layout.hpp (fragment blocks of 1 KiB, S planes of one
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
// coalesced although every lane then needs a piece of its own row.  A
// symmetric source kept as its upper triangle (d.sym) is read the same way
// where the panel lies above the diagonal, as the transposed panel (32
// contiguous doubles of each of W rows) where it lies below, and entry by
// entry where it crosses the diagonal.  Columns (trans == 1) are read
// directly: there consecutive lanes own consecutive rows, which are adjacent
// in memory.
// HALVES (Markidis kind, S = 2, FP16): instead of digits, the high and low
// FP16 parts of x = a 2^-e (|x| < 1): X0 = FP16[x], X1 = FP16[x - X0].
// COMB: the operand is the combination ta A + tb A2 + tc I (d.A2 set; the
// TRS4 right operand); an instantiation of its own, so that the plain
// split keeps the registers of its second staging array free.
// coef.count > 0: the first coef.count blocks of the grid run the coefficient
// step of the matrices instead (CoefArgs), beside the split's units.
template <int S, bool FP16, bool HALVES = false, bool COMB = false>
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
        bool transposed = false;   // stage[t] holds entry (q % 32, q / 32)
        if constexpr (COMB) {
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
        } else if (d.sym && kb + W <= rb * kFragRows) {
            // symmetric source, panel entirely below the diagonal: entry
            // (row, k) is A[k, row], so thread q reads row k = kb + q / 32 at
            // column row = 32 rb + q % 32 (32 contiguous doubles per k)
            transposed = true;
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t, rr = q % kFragRows, cc = q / kFragRows;
                const int row = rb * kFragRows + rr, k = kb + cc;
                stage[t] = (row < d.R && k < d.K) ? d.A[int64_t(k) * d.lda + row] : 0.0;
            }
        } else if (d.sym && kb < rb * kFragRows + kFragRows - 1) {
            // symmetric source, panel across the diagonal: every entry from
            // its place in the upper triangle
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t, rr = q / W, cc = q % W;
                const int row = rb * kFragRows + rr, k = kb + cc;
                stage[t] = (row < d.R && k < d.K)
                               ? d.A[k >= row ? int64_t(row) * d.lda + k : int64_t(k) * d.lda + row]
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
        if (transposed) {
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t;
                panel[(q % kFragRows) * LDW + q / kFragRows] = stage[t];
            }
        } else {
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int q = threadIdx.x + 256 * t;
                panel[(q / W) * LDW + q % W] = stage[t];
            }
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
    // Each element's digits are packed as soon as they are formed (word q
    // of plane s holds digit s of elements 4 q .. 4 q + 3 for INT8, of 2 q,
    // 2 q + 1 for FP16), so only the packed words stay live, not all digits
    // of the lane's elements.
    uint32_t w[S][4];
    if constexpr (S <= 8) {
        // Digits from their integer definition: X = rint(a 2^(8S - 2 - e))
        // (ties to even; |X| <= 2^(8S - 2) <= 2^62) is the sum of d_s
        // 2^(8 (S - s)) with d_2 .. d_S in [-128, 127], the same digits the
        // rounding steps above give (their sum is rint of the same value, and
        // this balanced representation is unique).  Adding 128 in each of the
        // S - 1 low bytes makes byte S - s of X + bias equal to d_s + 128
        // (s >= 2) and the bytes above it d_1; the digit is that byte with
        // its top bit flipped (FP16: that signed byte as an FP16 value, exact).
        // Exact: the scaling is a power of two, the halves of X below are
        // exact in FP64.
        constexpr uint64_t kBias = S >= 2 ? 0x8080808080808080ull >> (8 * (9 - S)) : 0ull;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const double x = e >= kNonFiniteExp ? 0.0 : rint(ldexp(v[i], 8 * S - 2 - e));
            const double hi = floor(ldexp(x, -32));
            const uint32_t lo = uint32_t(__builtin_fma(hi, -4294967296.0, x));
            const uint64_t u = ((uint64_t(uint32_t(int32_t(hi))) << 32) | lo) + kBias;
#pragma unroll
            for (int p = 0; p < S; ++p) {
                const uint32_t byte = (uint32_t(u >> (8 * (S - 1 - p))) & 0xffu) ^ (p > 0 ? 0x80u : 0u);
                if constexpr (!FP16) {
                    const uint32_t part = byte << (8 * (i & 3));
                    w[p][i >> 2] = (i & 3) == 0 ? part : (w[p][i >> 2] | part);
                } else {
                    const int digit = int(int8_t(uint8_t(byte)));
                    const uint32_t part = uint32_t(__half_as_ushort(__int2half_rn(digit))) << (16 * (i & 1));
                    w[p][i >> 1] = (i & 1) == 0 ? part : (w[p][i >> 1] | part);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < S; ++p)
            *reinterpret_cast<uint4*>(base + int64_t(p) * kFragBytes) =
                make_uint4(w[p][0], w[p][1], w[p][2], w[p][3]);
        return;
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        int dd[S];
        digits_of<S>(v[i], e, dd);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            uint32_t part;
            int q;
            bool first;
            if constexpr (!FP16) {
                part = uint32_t(uint8_t(dd[s])) << (8 * (i & 3));
                q = i >> 2;
                first = (i & 3) == 0;
            } else {
                part = uint32_t(__half_as_ushort(__int2half_rn(dd[s]))) << (16 * (i & 1));
                q = i >> 1;
                first = (i & 1) == 0;
            }
            w[s][q] = first ? part : (w[s][q] | part);
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
        *reinterpret_cast<uint4*>(base + int64_t(s) * kFragBytes) =
            make_uint4(w[s][0], w[s][1], w[s][2], w[s][3]);
}

// ---------------------------------------------------------------------------
// Host launchers.

template <int S>
static void launch_digits_s(bool fp16, bool comb, const SplitDesc* descs, int count,
                            const SplitDesc& one, const DevState* st, int units,
                            const CoefArgs& coef, hipStream_t stream) {
    const unsigned grid = unsigned(units + coef.count);
    if (fp16 && comb)
        k_digits<S, true, false, true><<<grid, 256, 0, stream>>>(descs, count, one, st, coef);
    else if (fp16)
        k_digits<S, true><<<grid, 256, 0, stream>>>(descs, count, one, st, coef);
    else if (comb)
        k_digits<S, false, false, true><<<grid, 256, 0, stream>>>(descs, count, one, st, coef);
    else
        k_digits<S, false><<<grid, 256, 0, stream>>>(descs, count, one, st, coef);
}

// The Markidis kind's two FP16 parts (S = 2).
static void launch_halves(bool comb, const SplitDesc* descs, int count, const SplitDesc& one,
                          const DevState* st, int units, const CoefArgs& coef,
                          hipStream_t stream) {
    const unsigned grid = unsigned(units + coef.count);
    if (comb)
        k_digits<2, true, true, true><<<grid, 256, 0, stream>>>(descs, count, one, st, coef);
    else
        k_digits<2, true, true><<<grid, 256, 0, stream>>>(descs, count, one, st, coef);
}

using DigitsFn = void (*)(bool, bool, const SplitDesc*, int, const SplitDesc&, const DevState*,
                          int, const CoefArgs&, hipStream_t);
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
    const bool comb = d.A2 != nullptr;
    if (kind == DMP_MARKIDIS_FP16)
        launch_halves(comb, nullptr, 0, d, st, split_units_digits(d.R, d.KC), CoefArgs{}, stream);
    else
        kDigits[S](kind == DMP_OZ_FP16, comb, nullptr, 0, d, st, split_units_digits(d.R, d.KC),
                   CoefArgs{}, stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

// The digit kernel alone, for an operand whose maxima (d.maxbits: row maxima,
// or column maxima when d.trans) an earlier product's epilogue accumulated.
int launch_split_digits(const SplitDesc& d, int S, dmp_kind kind, const DevState* st,
                        hipStream_t stream) {
    if (round_up(d.R, kPad) == 0) return DMP_OK;
    const bool comb = d.A2 != nullptr;
    if (kind == DMP_MARKIDIS_FP16)
        launch_halves(comb, nullptr, 0, d, st, split_units_digits(d.R, d.KC), CoefArgs{}, stream);
    else
        kDigits[S](kind == DMP_OZ_FP16, comb, nullptr, 0, d, st, split_units_digits(d.R, d.KC),
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
                                const CoefArgs& coef, bool combined) {
    if (units + coef.count <= 0) return DMP_OK;
    if (kind == DMP_MARKIDIS_FP16)
        launch_halves(combined, descs_dev, count, SplitDesc{}, st, units, coef, stream);
    else
        kDigits[S](kind == DMP_OZ_FP16, combined, descs_dev, count, SplitDesc{}, st, units, coef,
                   stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

}  // namespace dmp
