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

// Fixed-order sum of a matrix's partials, column q.
__device__ inline double sum_partials(const PurDesc& d, int q, double* sh) {
    double v = 0.0;
    for (int i = d.part_begin + threadIdx.x; i < d.part_end; i += 256)
        v += d.partials[int64_t(i) * kPartials + q];
    return block_sum(v, sh);
}

// Canonical purification (Sec. 2.3): c = tr(X2 - P^3) / tr(P - X2), clamped
// to [0, 1], the branch and the update weights.  One block of 256 threads.
__device__ inline void coef_canonical(const PurDesc& d, DevState& s, double* sh) {
    if (s.done) return;
    const double t1 = sum_partials(d, 0, sh);
    const double t2 = sum_partials(d, 1, sh);
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
    const double trf = sum_partials(d, 0, sh);
    const double trg = sum_partials(d, 1, sh);
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
