// Device code shared by the purification kernels and the split kernel:
// fixed-order block sums and the per-iteration coefficients computed from the
// square's trace partials (the split of X2 runs them in extra blocks of its
// own launch).
#pragma once

#include "common.hpp"

namespace dmp {

__device__ inline double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order block sum of 256 values (one per thread).
__device__ inline double block_sum(double v, double* sh) {
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// Fixed-order sums of a matrix's partials, columns 0 and 1: thread t adds
// the tiles t, t + 256, ... in that order, then the block sum.  Eight tiles'
// loads are issued before they are added (the same additions, in the same
// order, as one load at a time, without a memory latency per tile).
__device__ inline void sum_partials(const PurDesc& d, double* sh, double* s0, double* s1) {
    static_assert(kPartials == 2, "two partial columns, loaded as one 16-byte pair");
    double v0 = 0.0, v1 = 0.0;
    int i = d.part_begin + int(threadIdx.x);
    for (; i + 7 * 256 < d.part_end; i += 8 * 256) {
        double2 t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            t[u] = *reinterpret_cast<const double2*>(d.partials + int64_t(i + u * 256) * kPartials);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v0 += t[u].x;
            v1 += t[u].y;
        }
    }
    for (; i < d.part_end; i += 256) {
        const double2 t = *reinterpret_cast<const double2*>(d.partials + int64_t(i) * kPartials);
        v0 += t.x;
        v1 += t.y;
    }
    *s0 = block_sum(v0, sh);
    *s1 = block_sum(v1, sh);
}

// Canonical purification (Sec. 2.3): c = tr(X2 - P^3) / tr(P - X2), clamped
// to [0, 1], the branch and the update weights.  One block of 256 threads.
__device__ inline void coef_canonical(const PurDesc& d, DevState& s, double* sh) {
    if (s.done) return;
    double t1, t2;
    sum_partials(d, sh, &t1, &t2);
    if (threadIdx.x == 0) {
        const double raw = t1 == 0.0 ? 0.5 : t2 / t1;
        const double c = fmin(fmax(raw, 0.0), 1.0);
        s.t1 = t1;
        s.t2 = t2;
        s.c = c;
        s.clamped = (t1 == 0.0 || raw != c) ? 1 : 0;
        if (c >= 0.5) {
            s.branch = 1;
            s.alpha = 0.0;
            s.beta = (1.0 + c) / c;
            s.gamma = -1.0 / c;
        } else {
            s.branch = 0;
            s.alpha = (1.0 - 2.0 * c) / (1.0 - c);
            s.beta = (1.0 + c) / (1.0 - c);
            s.gamma = -1.0 / (1.0 - c);
        }
    }
}

// TRS4 trace reset (Sec. 3): gamma = (nocc - tr F) / tr G (0 when tr G is
// exactly 0) and the branch; the update weights select X2 T, 2X - X2 or X2.
__device__ inline void coef_trs4(const PurDesc& d, DevState& s, double* sh) {
    if (s.done) return;
    double trf, trg;
    sum_partials(d, sh, &trf, &trg);
    if (threadIdx.x == 0) {
        const double g = trg == 0.0 ? 0.0 : (double(s.nocc) - trf) / trg;
        s.t1 = trg;
        s.t2 = trf;
        s.c = g;
        s.ta = 0.0;
        s.tb = 0.0;
        s.tc = 0.0;
        if (g > 6.0) {          // X <- 2X - X2
            s.branch = 2;
            s.alpha = 2.0;
            s.beta = -1.0;
            s.gamma = 0.0;
        } else if (g < 0.0) {   // X <- X2
            s.branch = 0;
            s.alpha = 0.0;
            s.beta = 1.0;
            s.gamma = 0.0;
        } else {                // X <- X2 T (also for a NaN gamma: it propagates)
            s.branch = 1;
            s.alpha = 0.0;
            s.beta = 0.0;
            s.gamma = 1.0;
            s.ta = 4.0 - 2.0 * g;
            s.tb = g - 3.0;
            s.tc = g;
        }
    }
}

}  // namespace dmp
