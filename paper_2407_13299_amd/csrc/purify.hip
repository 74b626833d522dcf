// Canonical density-matrix purification driven by Ozaki-scheme products
// (Sec. 2.3 and 2.4; canonical trace-conserving form cited in Sec. 1).
//
// Per iteration and per matrix (every phase is one launch over all matrices
// of a group; matrices that have stopped skip their blocks):
//   split(P)            row exponents + digit planes of P (serve as both
//                       operands: P is exactly symmetric)
//   gemm SQUARE         X2 = P P, partial traces
//   finalize_coef       t1 = tr(P - X2), t2 = tr(X2 - P^3), c, branch,
//                       (alpha, beta, gamma)
//   split(X2)
//   gemm UPDATE         P' = alpha P + beta X2 + gamma X2 P, partial tr(P'H)
//   finalize_iter       E, dE, stopping rule
// TRS4 (Sec. 3) runs the same phases: the square's epilogue gives tr F and
// tr G, finalize_trs4 picks gamma and the branch, and the second product is
// X2 T with T = (4 - 2 gamma) X + (gamma - 3) X2 + gamma I formed inside the
// split (or no product at all on the X2 and 2X - X2 branches).
// All reductions are fixed-order (no floating-point atomics), so runs are
// bitwise reproducible.  FP64 everywhere except the slice products (Sec. 4).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "coef.hpp"
#include "host.hpp"

namespace dmp {


// Kernel-timing instrumentation (see dmp_timing_*).
struct TimingState {
    bool on = false;
    bool clocks = false;   // also the per-workgroup clock counters
    double ms[2] = {0.0, 0.0};
    long long launches[2] = {0, 0};
    double ops[2] = {0.0, 0.0};
};
static TimingState g_timing;
// Clock counters of the timed launches (device memory, allocated on the
// first timed launch and kept until the process ends): per GEMM kind the
// summed shader-clock cycles and real-time ticks of its workgroups.
static unsigned long long* g_clk = nullptr;
static int g_clk_device = -1;

struct PendingTimer {
    hipEvent_t start, stop;
    int which;
    double ops;
};
constexpr double kStagnationWindow = 1e-2;


__device__ inline double block_min(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ inline double block_max(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

// Gershgorin discs per row: centre H_ii, radius sum_{j != i} |H_ij|; one
// wavefront per row, grid.y = matrix.
__global__ __launch_bounds__(256) void k_gershgorin(const PurDesc* pd) {
    const PurDesc& d = pd[blockIdx.y];
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= d.n) return;
    const double* row = d.H + int64_t(r) * d.n;
    double s = 0.0;
    int bad = 0;
    for (int j = lane; j < d.n; j += 64) {
        const double v = row[j];
        bad |= !isfinite(v);
        s += fabs(v);
    }
    s = wsum(s);
    for (int off = 32; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, 64);
    if (lane == 0) {
        const double dg = row[r];
        const double rad = s - fabs(dg);
        d.rows[r] = dg - rad;
        d.rows[d.n + r] = dg + rad;
        d.rows[2 * d.n + r] = dg;
        d.rowbad[r] = bad;
    }
}

// Bounds, trace and the canonical initial-guess scalars; one block per matrix.
__global__ __launch_bounds__(256) void k_finalize_init(const PurDesc* pd, DevState* states,
                                                       double tol, int max_iter) {
    __shared__ double sh[4];
    const PurDesc& d = pd[blockIdx.x];
    DevState& s = states[blockIdx.x];
    const int n = d.n;
    double lo = INFINITY, hi = -INFINITY, tr = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        lo = fmin(lo, d.rows[i]);
        hi = fmax(hi, d.rows[n + i]);
        tr += d.rows[2 * n + i];
        bad |= d.rowbad[i];
    }
    lo = block_min(lo, sh);
    hi = block_max(hi, sh);
    tr = block_sum(tr, sh);
    const double anybad = block_max(double(bad), sh);
    // first rows attaining the bounds (the subgradient rows of the adjoint)
    double ilo = 1e300, ihi = 1e300;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (d.rows[i] == lo) ilo = fmin(ilo, double(i));
        if (d.rows[n + i] == hi) ihi = fmin(ihi, double(i));
    }
    ilo = block_min(ilo, sh);
    ihi = block_min(ihi, sh);
    if (threadIdx.x == 0) {
        s = DevState{};
        s.n = n;
        s.nocc = d.nocc;
        s.tol = tol;
        s.max_iter = max_iter;
        s.h_min = lo;
        s.h_max = hi;
        s.row_hmin = ilo < 1e300 ? int(ilo) : 0;
        s.row_hmax = ihi < 1e300 ? int(ihi) : 0;
        s.trace_h = tr;
        s.method = d.method;
        s.mu = tr / n;
        s.theta = double(d.nocc) / n;
        double lam = 0.0;
        if (d.nocc > 0 && d.nocc < n && d.method == DMP_TRS4) {
            // X0 = (h_max I - H) / (h_max - h_min) = lam (mu I - H) + theta I
            if (hi - lo > 0.0) {
                lam = 1.0 / (hi - lo);
                s.mu = hi;
                s.theta = 0.0;
            }
        } else if (d.nocc > 0 && d.nocc < n) {
            const double a = (hi - s.mu) > 0.0 ? s.theta / (hi - s.mu) : 0.0;
            const double b = (s.mu - lo) > 0.0 ? (1.0 - s.theta) / (s.mu - lo) : 0.0;
            lam = fmin(a, b);
            s.which = a <= b ? 0 : 1;
        } else {
            s.done = 1;   // P = 0 or I exactly, no iterations
            s.stop_reason = DMP_STOP_CONVERGED;
        }
        s.lambda = lam;
        if (anybad != 0.0) {
            s.nonfinite = 1;
            s.done = 1;
            s.stop_reason = DMP_STOP_NONFINITE;
        }
    }
}

// Tile pair (I, J), I <= J, number pi of the T x T tile triangle numbered
// row by row (row I holds pairs [I T - I (I - 1) / 2, ...)).
__device__ inline int2 tile_pair(int pi, int T) {
    int I = int((2.0 * T + 1.0 - sqrt((2.0 * T + 1.0) * (2.0 * T + 1.0) - 8.0 * pi)) * 0.5);
    auto first = [&](int r) { return r * T - r * (r - 1) / 2; };
    if (I > 0 && first(I) > pi) --I;
    if (I + 1 < T && first(I + 1) <= pi) ++I;
    return make_int2(I, I + (pi - first(I)));
}

// P0 = lam (mu I - H) + theta I from the upper triangle of H (mirrored), and
// partial energies tr(P0 H); fixed grid of kE0Blocks blocks per matrix.
// Block x takes the 32 x 32 tile pairs (I, J), I <= J, numbered row by row,
// x, x + kE0Blocks, ...: it reads tile (I, J) of H with coalesced rows,
// writes P0's tile (I, J) and, transposed through LDS, tile (J, I), also
// with coalesced rows.  Its energy partial is the sum over the upper
// elements of (1 or 2) P0_ij H_ij, in a fixed order.
__global__ __launch_bounds__(256) void k_init_p0(const PurDesc* pd, const DevState* states) {
    __shared__ double sh[4];
    __shared__ double tileT[32][33];
    const PurDesc& d = pd[blockIdx.y];
    const DevState& s = states[blockIdx.y];
    // locals: the stores to P below could alias the descriptor and the state
    // as far as the compiler knows, and would force them to be reloaded
    const int n = d.n;
    const double* H = d.H;
    double* P = d.Pb[0];
    const double lam = s.lambda, mu = s.mu, theta = s.theta;
    const int T = (n + 31) / 32;
    const int npairs = T * (T + 1) / 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double e = 0.0;
    if (!s.nonfinite) {
        for (int pi = blockIdx.x; pi < npairs; pi += kE0Blocks) {
            const int2 ij = tile_pair(pi, T);
            const int I = ij.x, J = ij.y;
            for (int r = ty; r < 32; r += 8) {
                const int i = I * 32 + r, j = J * 32 + tx;
                double p = 0.0;
                if (i < n && j < n && !(I == J && j < i)) {
                    const int64_t ij = int64_t(i) * n + j;
                    const double h = H[ij];
                    p = lam * ((i == j ? mu : 0.0) - h) + (i == j ? theta : 0.0);
                    P[ij] = p;
                    e += (i == j ? 1.0 : 2.0) * p * h;
                }
                tileT[r][tx] = p;
            }
            __syncthreads();
            for (int r = ty; r < 32; r += 8) {
                // element (J 32 + r, I 32 + tx) = tile (I, J)[tx][r]
                const int i = J * 32 + r, j = I * 32 + tx;
                if (i < n && j < n && (I != J || j < i)) P[int64_t(i) * n + j] = tileT[tx][r];
            }
            __syncthreads();
        }
    }
    e = block_sum(e, sh);
    if (threadIdx.x == 0) d.e0[blockIdx.x] = e;
}

// The final iterate of a canonical Ozaki purification, which the products
// keep as its upper triangle, made full in place: tile (J, I) from tile
// (I, J), transposed through LDS, both with coalesced rows.  Grid
// (kE0Blocks, matrices); matrices that ran no iteration hold the full P0.
__global__ __launch_bounds__(256) void k_mirror_iterate(const PurDesc* pd, const DevState* states) {
    __shared__ double t[32][33];
    const PurDesc& d = pd[blockIdx.y];
    const DevState& s = states[blockIdx.y];
    if (s.iters == 0) return;
    const int n = d.n;
    double* X = d.Pb[s.iters & 1];
    const int T = (n + 31) / 32;
    const int npairs = T * (T + 1) / 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int pi = blockIdx.x; pi < npairs; pi += kE0Blocks) {
        const int2 ij = tile_pair(pi, T);
        const int I = ij.x, J = ij.y;
        for (int r = ty; r < 32; r += 8) {
            const int i = I * 32 + r, j = J * 32 + tx;
            t[r][tx] = (i < n && j < n) ? X[int64_t(i) * n + j] : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = J * 32 + r, j = I * 32 + tx;   // (i, j) = (j, i) of the upper part
            if (i < n && j < n && (I != J || j < i)) X[int64_t(i) * n + j] = t[tx][r];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_finalize_e0(const PurDesc* pd, DevState* states) {
    __shared__ double sh[4];
    const PurDesc& d = pd[blockIdx.x];
    DevState& s = states[blockIdx.x];
    double e = 0.0;
    for (int i = threadIdx.x; i < kE0Blocks; i += 256) e += d.e0[i];
    e = block_sum(e, sh);
    if (threadIdx.x == 0) {
        s.E = e;
        s.E_prev = e;
        s.trace_p = double(d.nocc);
    }
}

__global__ __launch_bounds__(256) void k_finalize_coef(const PurDesc* pd, DevState* states) {
    __shared__ double sh[4];
    coef_canonical(pd[blockIdx.x], states[blockIdx.x], sh);
}

__global__ __launch_bounds__(256) void k_finalize_trs4(const PurDesc* pd, DevState* states) {
    __shared__ double sh[4];
    coef_trs4(pd[blockIdx.x], states[blockIdx.x], sh);
}

// Energy of the new iterate and the stopping rule of Sec. 3.
__global__ __launch_bounds__(256) void k_finalize_iter(const PurDesc* pd, DevState* states) {
    __shared__ double sh[4];
    const PurDesc& d = pd[blockIdx.x];
    DevState& s = states[blockIdx.x];
    if (s.done) return;
    double e, tr;
    sum_partials(d, sh, &e, &tr);
    if (threadIdx.x == 0) {
        const double de = e - s.E;
        s.dE_prev = s.dE;
        s.dE = de;
        s.E_prev = s.E;
        s.E = e;
        s.trace_p = tr;
        s.iters += 1;
        s.products += s.gamma != 0.0 ? 2 : 1;
        int stop = -1;
        if (!isfinite(e)) stop = DMP_STOP_NONFINITE;
        else if (fabs(de) < s.tol) stop = DMP_STOP_CONVERGED;
        else if (s.iters >= 2 && de > 0.0 && s.dE_prev > 0.0 && fabs(de) < kStagnationWindow)
            stop = DMP_STOP_STAGNATED;
        else if (s.iters >= s.max_iter) stop = DMP_STOP_MAX_ITER;
        if (stop >= 0) {
            s.done = 1;
            s.stop_reason = stop;
        }
    }
}

// ---- native FP64 path: elementwise work around rocBLAS products -----------

// Partials of tr(P - X2) and sum_{i<=j} mult X2_ij (delta_ij - P_ij) over the
// upper triangle (mult 2 off the diagonal), fixed grid.
__global__ __launch_bounds__(256) void k_native_square(const PurDesc* pd, const DevState* states,
                                                       int nblocks) {
    __shared__ double sh[4];
    const PurDesc& d = pd[0];
    if (states[0].done) return;
    const int n = d.n;
    const double* P = d.Pb[states[0].iters & 1];
    const int64_t tot = int64_t(n) * n;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < tot;
         idx += int64_t(nblocks) * 256) {
        const int i = int(idx / n), j = int(idx % n);
        if (j < i) continue;
        const double x = d.X2[idx], p = P[idx];
        if (d.method == DMP_TRS4) {
            const double mult = i == j ? 1.0 : 2.0, r = p - x;
            s0 += mult * x * (4.0 * p - 3.0 * x);
            s1 += mult * r * r;
        } else if (i == j) {
            s0 += p - x;
            s1 += x * (1.0 - p);
        } else {
            s1 -= 2.0 * x * p;
        }
    }
    s0 = block_sum(s0, sh);
    s1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        d.partials[int64_t(blockIdx.x) * kPartials + 0] = s0;
        d.partials[int64_t(blockIdx.x) * kPartials + 1] = s1;
    }
}

// P' = alpha P + beta X2 + gamma X3 on 32 x 32 tile pairs I <= J, written to
// (I, J) and, transposed through LDS, to (J, I); partials of tr(P'H), tr P'.
__global__ __launch_bounds__(256) void k_native_update(const PurDesc* pd, const DevState* states,
                                                       const int2* pairs) {
    __shared__ double tileT[32][33];
    __shared__ double sh[4];
    const PurDesc& d = pd[0];
    const DevState& s = states[0];
    if (s.done) return;
    const int n = d.n;
    const double* P = d.Pb[s.iters & 1];
    double* Pn = d.Pb[(s.iters + 1) & 1];
    const int2 pr = pairs[blockIdx.x];
    const int I = pr.x, J = pr.y;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // locals: the stores to Pn could alias the descriptor and the state as
    // far as the compiler knows, and would force them to be reloaded
    const double alpha = s.alpha, beta = s.beta, gamma = s.gamma;
    const double *X2 = d.X2, *X3 = d.X3, *H = d.H;
    double se = 0.0, st = 0.0;
    for (int r = ty; r < 32; r += 8) {
        const int i = I * 32 + r, j = J * 32 + tx;
        double v = 0.0;
        if (i < n && j < n && !(I == J && j < i)) {
            const int64_t ij = int64_t(i) * n + j;
            // gamma == 0 (TRS4 without a second product): X3 is not read
            v = alpha * P[ij] + beta * X2[ij] + (gamma != 0.0 ? gamma * X3[ij] : 0.0);
            Pn[ij] = v;
            se += (i == j ? 1.0 : 2.0) * v * H[ij];
            if (i == j) st += v;
        }
        tileT[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        // element (J*32 + r, I*32 + tx) = tile(I,J)[tx][r]
        const int i = J * 32 + r, j = I * 32 + tx;
        if (i < n && j < n && (I != J ? true : j < i)) Pn[int64_t(i) * n + j] = tileT[tx][r];
    }
    se = block_sum(se, sh);
    st = block_sum(st, sh);
    if (threadIdx.x == 0) {
        d.partials[int64_t(blockIdx.x) * kPartials + 0] = se;
        d.partials[int64_t(blockIdx.x) * kPartials + 1] = st;
    }
}

// Copy the upper triangle of a row-major n x n matrix onto its lower one
// (32 x 32 tile pairs I <= J through LDS).
__global__ __launch_bounds__(256) void k_mirror_upper(double* X, int n, const int2* pairs) {
    __shared__ double t[32][33];
    const int2 pr = pairs[blockIdx.x];
    const int I = pr.x, J = pr.y;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = I * 32 + r, j = J * 32 + tx;
        t[r][tx] = (i < n && j < n) ? X[int64_t(i) * n + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = J * 32 + r, j = I * 32 + tx;   // element (i, j) = (j, i) of the upper part
        if (i < n && j < n && (I != J || j < i)) X[int64_t(i) * n + j] = t[tx][r];
    }
}

// Native TRS4: T = ta P + tb X2 + tc I (full matrix).
__global__ __launch_bounds__(256) void k_native_t(const PurDesc* pd, const DevState* states) {
    const PurDesc& d = pd[0];
    const DevState& s = states[0];
    if (s.done || s.gamma == 0.0) return;
    const int n = d.n;
    const double* P = d.Pb[s.iters & 1];
    // locals, as in k_native_update
    const double ta = s.ta, tb = s.tb, tc = s.tc;
    const double* X2 = d.X2;
    double* T = d.T;
    const int64_t tot = int64_t(n) * n;
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < tot;
         idx += int64_t(gridDim.x) * 256) {
        const bool diag = idx / n == idx % n;
        T[idx] = ta * P[idx] + tb * X2[idx] + (diag ? tc : 0.0);
    }
}

// McWeeny refinement (Sec. 4.1): P' = 3 X2 - 2 X3 with X2 = P P and X3 =
// X2 P from FP64 products, on 32 x 32 tile pairs I <= J, written over X3
// (each upper element is read by the thread that overwrites it; the mirrored
// lower half is never read) and mirrored through LDS; partials of tr(P'H)
// and tr P'.
__global__ __launch_bounds__(256) void k_mcweeny(const double* X2, double* X3P, const double* H,
                                                 int n, const int2* pairs, double* partials) {
    __shared__ double tileT[32][33];
    __shared__ double sh[4];
    const int2 pr = pairs[blockIdx.x];
    const int I = pr.x, J = pr.y;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double se = 0.0, st = 0.0;
    for (int r = ty; r < 32; r += 8) {
        const int i = I * 32 + r, j = J * 32 + tx;
        double v = 0.0;
        if (i < n && j < n && !(I == J && j < i)) {
            const int64_t ij = int64_t(i) * n + j;
            v = 3.0 * X2[ij] - 2.0 * X3P[ij];
            X3P[ij] = v;
            se += (i == j ? 1.0 : 2.0) * v * H[ij];
            if (i == j) st += v;
        }
        tileT[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = J * 32 + r, j = I * 32 + tx;
        if (i < n && j < n && (I != J ? true : j < i)) X3P[int64_t(i) * n + j] = tileT[tx][r];
    }
    se = block_sum(se, sh);
    st = block_sum(st, sh);
    if (threadIdx.x == 0) {
        partials[int64_t(blockIdx.x) * kPartials + 0] = se;
        partials[int64_t(blockIdx.x) * kPartials + 1] = st;
    }
}

__global__ __launch_bounds__(256) void k_finalize_refine(const double* partials, int count,
                                                         DevState* state) {
    __shared__ double sh[4];
    double e = 0.0, t = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) {
        e += partials[int64_t(i) * kPartials + 0];
        t += partials[int64_t(i) * kPartials + 1];
    }
    e = block_sum(e, sh);
    t = block_sum(t, sh);
    if (threadIdx.x == 0) {
        state->E_unrefined = state->E;
        state->dE = e - state->E;
        state->E = e;
        state->trace_p = t;
        state->refined = 1;
        state->products += 2;
    }
}

// ---------------------------------------------------------------------------
// Host wrappers of the small kernels (also used by the adjoint).

int launch_purify_init(const PurDesc* pd, DevState* st, int count, int max_n, double tol,
                       int max_iter, hipStream_t s) {
    k_gershgorin<<<dim3((max_n + 3) / 4, count), 256, 0, s>>>(pd);
    k_finalize_init<<<count, 256, 0, s>>>(pd, st, tol, max_iter);
    k_init_p0<<<dim3(kE0Blocks, count), 256, 0, s>>>(pd, st);
    k_finalize_e0<<<count, 256, 0, s>>>(pd, st);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

int launch_finalize_coef(const PurDesc* pd, DevState* st, int count, hipStream_t s) {
    k_finalize_coef<<<count, 256, 0, s>>>(pd, st);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

int launch_finalize_iter(const PurDesc* pd, DevState* st, int count, hipStream_t s) {
    k_finalize_iter<<<count, 256, 0, s>>>(pd, st);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

int e0_blocks() { return kE0Blocks; }

// ---------------------------------------------------------------------------
// Host driver.

namespace {

static_assert(sizeof(IPair) == sizeof(int2) && alignof(IPair) == alignof(int2),
              "tile pairs are passed to the kernels as int2");

const int2* as_int2(const IPair* p) { return reinterpret_cast<const int2*>(p); }

// Fill a carved group's descriptors on the host and copy them to the
// device; ``keep`` holds the host copies until the stream has passed the
// copies.
int upload_group(GroupPlan& g, const double* const* H, double* const* P, const int* n,
                 const int* nocc, hipStream_t s, std::vector<std::unique_ptr<GroupHost>>& keep) {
    int slots = 0;
    if (g.fix != nullptr && tail_split_enabled())
        DMP_CHECK(resident_slots(g.S, g.kind, g.rb, &slots));
    keep.push_back(std::make_unique<GroupHost>());
    GroupHost& h = *keep.back();
    build_group(g, H, P, n, nocc, slots, h);
    auto up = [&](void* dst, const void* src, size_t bytes) -> int {
        if (bytes == 0) return DMP_OK;
        DMP_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        return DMP_OK;
    };
    const size_t cnt = size_t(g.count);
    DMP_CHECK(up(g.pd, h.pd.data(), cnt * sizeof(PurDesc)));
    if (g.kind != DMP_FP64_NATIVE) {
        DMP_CHECK(up(g.splitP[0], h.sp0.data(), cnt * sizeof(SplitDesc)));
        DMP_CHECK(up(g.splitP[1], h.sp1.data(), cnt * sizeof(SplitDesc)));
        DMP_CHECK(up(g.splitX, h.sx.data(), cnt * sizeof(SplitDesc)));
        DMP_CHECK(up(g.splitT[0], h.st0.data(), cnt * sizeof(SplitDesc)));
        DMP_CHECK(up(g.splitT[1], h.st1.data(), cnt * sizeof(SplitDesc)));
        DMP_CHECK(up(g.sq[0], h.q0.data(), cnt * sizeof(MatDesc)));
        DMP_CHECK(up(g.sq[1], h.q1.data(), cnt * sizeof(MatDesc)));
        DMP_CHECK(up(g.up[0], h.u0.data(), cnt * sizeof(MatDesc)));
        DMP_CHECK(up(g.up[1], h.u1.data(), cnt * sizeof(MatDesc)));
        DMP_CHECK(up(g.tiles, h.tiles.data(), h.tiles.size() * sizeof(Tile)));
    }
    DMP_CHECK(up(g.pairs, h.pairs.data(), h.pairs.size() * sizeof(IPair)));
    return DMP_OK;
}

int launch_init(GroupPlan& g, double tol, int max_iter, hipStream_t s) {
    DMP_CHECK(launch_purify_init(g.pd, g.st, g.count, g.max_n, tol, max_iter, s));
    // row maxima of P0 (later iterates get theirs from the update's epilogue)
    if (g.kind != DMP_FP64_NATIVE)
        DMP_CHECK(launch_split_grouped_rowmax(g.splitP[0], g.count, g.units_rowmax, g.st, s));
    return DMP_OK;
}

double gemm_ops(const GroupPlan& g, const int* n) {
    double t = 0.0;
    for (int b = 0; b < g.count; ++b) {
        const double m = n[g.idx[b]];
        t += double(g.S) * (g.S + 1) * m * m * (m + 1) / 2.0;
    }
    return t;
}

int timed_gemm(GroupPlan& g, const GemmParams& p, int which, double ops, hipStream_t s,
               std::vector<PendingTimer>* timers) {
    PendingTimer t{};
    GemmParams q = p;
    if (timers) {
        if (g_timing.clocks) {
            int dev = 0;
            DMP_CHECK_HIP(hipGetDevice(&dev));
            if (g_clk == nullptr || g_clk_device != dev) {
                // instrumentation only: one small buffer for the process
                DMP_CHECK_HIP(hipMalloc(&g_clk, 4 * sizeof(unsigned long long)));
                DMP_CHECK_HIP(hipMemset(g_clk, 0, 4 * sizeof(unsigned long long)));
                g_clk_device = dev;
            }
            q.clk = g_clk + 2 * which;
        }
        DMP_CHECK_HIP(hipEventCreate(&t.start));
        DMP_CHECK_HIP(hipEventCreate(&t.stop));
        DMP_CHECK_HIP(hipEventRecord(t.start, s));
    }
    DMP_CHECK(launch_ozgemm(g.S, g.kind, q, g.ntiles, s, g.rb));
    if (timers) {
        DMP_CHECK_HIP(hipEventRecord(t.stop, s));
        t.which = which;
        t.ops = ops;
        timers->push_back(t);
    }
    return DMP_OK;
}

// One Ozaki iteration of the whole group with iterate parity ``par``.
int launch_oz_iteration(GroupPlan& g, int par, hipStream_t s,
                        std::vector<PendingTimer>* timers = nullptr, double ops = 0.0) {
    // the row maxima of P come from the previous update's epilogue
    DMP_CHECK(launch_split_grouped_digits(g.splitP[par], g.count, g.units_digits, g.S, g.kind, g.st, s));
    GemmParams p{};
    p.tiles = g.tiles;
    p.descs = g.sq[par];
    p.partials = g.partials;
    p.states = g.st;
    const bool trs4 = g.method == DMP_TRS4;
    p.mode = trs4 ? EPI_SQUARE_TRS4 : EPI_SQUARE;
    // canonical iterates and X2 stay upper triangles (their splits read them
    // as symmetric); TRS4's combined operand needs full rows
    p.upper_only = trs4 ? 0 : 1;
    p.spread = g.count > 1 ? 1 : 0;
    if (g.tail.nsplit > 1) {
        p.fix = g.fix;
        p.nfull = g.tail.nfull;
        p.nsplit = g.tail.nsplit;
    }
    DMP_CHECK(timed_gemm(g, p, 0, ops, s, timers));
    // the split of X2 (row maxima from the square's epilogue) and, in extra
    // blocks of the same launch, the coefficient step (it reads only the
    // done flags of the states that step writes)
    DMP_CHECK(launch_split_grouped_digits(g.splitX, g.count, g.units_digits, g.S, g.kind, g.st, s,
                                          CoefArgs{g.pd, g.st, g.count, g.method}));
    if (trs4) {
        DMP_CHECK(launch_split_grouped_rowmax(g.splitT[par], g.count, g.units_rowmax, g.st, s));
        DMP_CHECK(launch_split_grouped_digits(g.splitT[par], g.count, g.units_digits, g.S, g.kind,
                                              g.st, s, CoefArgs{}, true));
    }
    p.descs = g.up[par];
    p.mode = EPI_UPDATE;
    DMP_CHECK(timed_gemm(g, p, 1, ops, s, timers));
    k_finalize_iter<<<g.count, 256, 0, s>>>(g.pd, g.st);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

// Iterations per replay of the cached graph: even, so a replay ends with the
// iterate in the buffer it started from.
int iterations_per_sync(int max_n) {
    if (max_n >= 4096) return 2;
    if (max_n >= 1024) return 4;
    return 8;
}

bool graphs_enabled() {
    const char* e = std::getenv("DMP_NO_GRAPH");
    return !(e && e[0] == '1');
}

// A recorded sequence of m iterations of the groups, instantiated once and
// replayed by every later run with the same launch sequence (same
// workspace, sizes and plans; the matrices' pointers live in the uploaded
// descriptors, not in the launches).
struct CachedGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int last_iters = 0;    // iterations the previous run of this sequence took
};

constexpr size_t kGraphCacheCapacity = 16;

// Never destroyed: its graphs would otherwise be released by a static
// destructor after the HIP runtime may already have shut down.
KeyedCache<CachedGraph>& graph_cache() {
    static auto* cache = new KeyedCache<CachedGraph>(kGraphCacheCapacity);
    return *cache;
}

std::shared_ptr<CachedGraph> capture_iterations(std::vector<GroupPlan>& groups, int m) {
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    for (int it = 0; ok && it < m; ++it)
        for (auto& g : groups) ok = ok && launch_oz_iteration(g, it & 1, cap) == DMP_OK;
    hipGraph_t gr = nullptr;
    const bool ended = hipStreamEndCapture(cap, &gr) == hipSuccess;
    hipGraphExec_t exec = nullptr;
    if (!(ok && ended && gr && hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0) == hipSuccess)) {
        if (gr) (void)hipGraphDestroy(gr);
        exec = nullptr;
        gr = nullptr;
    }
    (void)hipStreamDestroy(cap);
    (void)hipGetLastError();
    clear_error();
    if (!exec) return nullptr;
    auto* v = new CachedGraph{gr, exec, 0};
    return std::shared_ptr<CachedGraph>(v, [](CachedGraph* c) {
        (void)hipGraphExecDestroy(c->exec);
        (void)hipGraphDestroy(c->graph);
        delete c;
    });
}

// Page-locked host memory for the state reads of the calling thread (grown
// as needed, kept until the process ends), so that a read is an
// asynchronous copy the host can wait for with an event.
DevState* pinned_states(size_t count) {
    static thread_local DevState* buf = nullptr;
    static thread_local size_t cap = 0;
    if (count > cap) {
        void* p = nullptr;
        if (hipHostMalloc(&p, count * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        buf = static_cast<DevState*>(p);   // the smaller old buffer is left to the process
        cap = count;
    }
    return buf;
}

// Instrumented run (kernel timing on): eager launches with HIP events around
// every product, the state read after each batch of m iterations.
int run_oz_timed(std::vector<GroupPlan>& groups, int max_iter, int m, hipStream_t s,
                 std::vector<DevState>& host_st, const int* n) {
    std::vector<PendingTimer> timers;
    const int rounds = (max_iter + m - 1) / m + 1;
    for (int r = 0; r < rounds; ++r) {
        for (int it = 0; it < m; ++it)
            for (auto& g : groups) DMP_CHECK(launch_oz_iteration(g, it & 1, s, &timers, gemm_ops(g, n)));
        size_t off = 0;
        for (auto& g : groups) {
            DMP_CHECK_HIP(hipMemcpyAsync(host_st.data() + off, g.st, g.count * sizeof(DevState),
                                         hipMemcpyDeviceToHost, s));
            off += g.count;
        }
        DMP_CHECK_HIP(hipStreamSynchronize(s));
        for (auto& t : timers) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
                g_timing.ms[t.which] += ms;
                g_timing.launches[t.which] += 1;
                g_timing.ops[t.which] += t.ops;
            }
            (void)hipEventDestroy(t.start);
            (void)hipEventDestroy(t.stop);
        }
        timers.clear();
        bool all = true;
        for (auto& h : host_st) all = all && h.done;
        if (all) break;
    }
    return DMP_OK;
}

// Run the Ozaki groups to completion.  Iterations run in replays of m at a
// time (one cached graph, or eager launches with DMP_NO_GRAPH=1); matrices
// that have stopped skip their work inside every launch.  Once a run of the
// same launch sequence has finished, later runs start with one launch of a
// second cached graph holding as many iterations as that run needed
// (rounded up to a multiple of m), and the host reads the device states
// once after it; a first run reads them after one replay.  A run that needs
// more continues with replays of m, one always queued ahead of the state read
// being checked, so the GPU does not wait for the host between replays.
int run_oz_groups(std::vector<GroupPlan>& groups, int max_iter, hipStream_t s,
                  std::vector<DevState>& host_st, const int* n) {
    int max_n = 0;
    for (auto& g : groups) max_n = std::max(max_n, g.max_n);
    const int m = iterations_per_sync(max_n);
    if (g_timing.on) return run_oz_timed(groups, max_iter, m, s, host_st, n);
    std::shared_ptr<CachedGraph> cg;
    if (graphs_enabled()) {
        int dev = 0;
        DMP_CHECK_HIP(hipGetDevice(&dev));
        // the measurement switch is read at capture: part of the key
        const int env = tail_split_enabled() ? 1 : 0;
        cg = graph_cache().get_or_create(launch_key(groups, m, dev, env),
                                         [&]() { return capture_iterations(groups, m); });
    }
    auto replay = [&]() -> int {
        if (cg) {
            DMP_CHECK_HIP(hipGraphLaunch(cg->exec, s));
            return DMP_OK;
        }
        for (int it = 0; it < m; ++it)
            for (auto& g : groups) DMP_CHECK(launch_oz_iteration(g, it & 1, s));
        return DMP_OK;
    };
    const size_t total = host_st.size();
    DevState* pin = pinned_states(2 * total);
    if (pin == nullptr) {
        set_error("page-locked host memory for the state reads unavailable");
        return DMP_EHIP;
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto& e : ev) DMP_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    struct EventGuard {
        hipEvent_t* e;
        ~EventGuard() {
            for (int i = 0; i < 2; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    auto read = [&](int slot) -> int {
        size_t off = 0;
        for (auto& g : groups) {
            DMP_CHECK_HIP(hipMemcpyAsync(pin + slot * total + off, g.st, g.count * sizeof(DevState),
                                         hipMemcpyDeviceToHost, s));
            off += g.count;
        }
        DMP_CHECK_HIP(hipEventRecord(ev[slot], s));
        return DMP_OK;
    };
    auto finished = [&](int slot) {
        for (size_t i = 0; i < total; ++i)
            if (!pin[slot * total + i].done) return false;
        return true;
    };
    const int max_replays = (max_iter + m - 1) / m + 1;
    const int first = cg && cg->last_iters > 0
                          ? std::min(max_replays, std::max(1, (cg->last_iters + m - 1) / m))
                          : 1;
    int launched = 0;
    // the predicted iterations as one graph (same parity at its end as after
    // ``first`` replays of m, since m is even)
    std::shared_ptr<CachedGraph> whole;
    if (cg && first > 1) {
        int dev = 0;
        DMP_CHECK_HIP(hipGetDevice(&dev));
        const int env = (tail_split_enabled() ? 1 : 0) | 2;
        whole = graph_cache().get_or_create(launch_key(groups, first * m, dev, env), [&]() {
            return capture_iterations(groups, first * m);
        });
    }
    if (whole) {
        DMP_CHECK_HIP(hipGraphLaunch(whole->exec, s));
        launched = first;
    }
    for (; launched < first; ++launched) DMP_CHECK(replay());
    DMP_CHECK(read(0));
    DMP_CHECK_HIP(hipEventSynchronize(ev[0]));
    int last = 0;                 // slot of the newest read checked
    bool done = finished(0);
    int pending = -1, slot = 1;   // read in flight, and the slot of the next one
    while (!done && launched < max_replays) {
        DMP_CHECK(replay());
        ++launched;
        DMP_CHECK(read(slot));
        if (pending >= 0) {
            DMP_CHECK_HIP(hipEventSynchronize(ev[pending]));
            last = pending;
            done = finished(pending);
        }
        pending = slot;
        slot ^= 1;
    }
    if (!done && pending >= 0) {  // the replay budget is spent: the newest read
        DMP_CHECK_HIP(hipEventSynchronize(ev[pending]));
        last = pending;
    }
    std::copy(pin + last * total, pin + last * total + total, host_st.begin());
    if (cg) {
        int it = 0;
        for (auto& h : host_st) it = std::max(it, h.iters);
        cg->last_iters = it;
    }
    return DMP_OK;
}

// Native FP64 purification of one matrix (group of one), host-checked
// every iteration.  ``tri``: every product by rocBLAS dsyrk / dsyrkx on the
// upper triangle only (the elementwise kernels read only that half; X2 is
// mirrored because it is a full operand of the second product).
int run_native(GroupPlan& g, int max_iter, hipStream_t s, DevState& host, bool tri) {
    const int n = g.max_n;
    const MatLayout& L = g.lay[0];
    PurDesc hd{};
    DMP_CHECK_HIP(hipMemcpyAsync(&hd, g.pd, sizeof(PurDesc), hipMemcpyDeviceToHost, s));
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    const int nb = native_blocks(n), np = native_pairs(n);
    const bool trs4 = g.method == DMP_TRS4;
    // host sources of the per-phase descriptor copies; the drain keeps them
    // alive until the stream has passed the copies, also on an error return
    PurDesc dsq = hd, dup = hd;
    dsq.part_begin = 0;
    dsq.part_end = nb;
    dup.part_begin = 0;
    dup.part_end = np;
    StreamDrain drain{s};
    for (int it = 0; it < max_iter; ++it) {
        DMP_CHECK_HIP(hipMemcpyAsync(&host, g.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        DMP_CHECK_HIP(hipStreamSynchronize(s));
        if (host.done) break;
        const double* P = host.iters & 1 ? L.Pw : hd.Pb[0];
        if (tri) {
            DMP_CHECK(native_dsyrk_upper(s, n, P, L.X2));
            k_mirror_upper<<<np, 256, 0, s>>>(L.X2, n, as_int2(g.pairs));
        } else {
            DMP_CHECK(native_dgemm(s, false, false, n, n, n, P, n, P, n, L.X2, n));
        }
        DMP_CHECK_HIP(hipMemcpyAsync(g.pd, &dsq, sizeof(PurDesc), hipMemcpyHostToDevice, s));
        k_native_square<<<nb, 256, 0, s>>>(g.pd, g.st, nb);
        if (trs4) {
            k_finalize_trs4<<<1, 256, 0, s>>>(g.pd, g.st);
            // the second product only runs on the X2 T branch
            DMP_CHECK_HIP(hipMemcpyAsync(&host, g.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
            DMP_CHECK_HIP(hipStreamSynchronize(s));
            if (host.gamma != 0.0) {
                k_native_t<<<2048, 256, 0, s>>>(g.pd, g.st);
                if (tri)
                    DMP_CHECK(native_dsyrkx_upper(s, n, L.X2, L.T, L.X3));
                else
                    DMP_CHECK(native_dgemm(s, false, false, n, n, n, L.X2, n, L.T, n, L.X3, n));
            }
        } else {
            k_finalize_coef<<<1, 256, 0, s>>>(g.pd, g.st);
            if (tri)
                DMP_CHECK(native_dsyrkx_upper(s, n, L.X2, P, L.X3));
            else
                DMP_CHECK(native_dgemm(s, false, false, n, n, n, L.X2, n, P, n, L.X3, n));
        }
        DMP_CHECK_HIP(hipMemcpyAsync(g.pd, &dup, sizeof(PurDesc), hipMemcpyHostToDevice, s));
        k_native_update<<<np, 256, 0, s>>>(g.pd, g.st, as_int2(g.pairs));
        k_finalize_iter<<<1, 256, 0, s>>>(g.pd, g.st);
        DMP_CHECK_HIP(hipGetLastError());
    }
    DMP_CHECK_HIP(hipMemcpyAsync(&host, g.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    return DMP_OK;
}

// One FP64 McWeeny step on matrix b's final iterate (Sec. 4.1): X2 = P P and
// X3 = X2 P by rocBLAS, P' = 3 X2 - 2 X3 written over X3, which is the other
// iterate buffer; the result then lives in Pb[(iters + 1) & 1].
int refine_mcweeny(GroupPlan& g, int b, const int* n, DevState& host, hipStream_t s) {
    const int m = n[g.idx[b]];
    PurDesc hd{};
    DMP_CHECK_HIP(hipMemcpyAsync(&hd, g.pd + b, sizeof(PurDesc), hipMemcpyDeviceToHost, s));
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    const double* P = hd.Pb[host.iters & 1];
    double* other = hd.Pb[(host.iters + 1) & 1];
    DMP_CHECK(native_dgemm(s, false, false, m, m, m, P, m, P, m, hd.X2, m));
    DMP_CHECK(native_dgemm(s, false, false, m, m, m, hd.X2, m, P, m, other, m));
    const int np = native_pairs(m);
    k_mcweeny<<<np, 256, 0, s>>>(hd.X2, other, hd.H, m, as_int2(g.pairs), g.partials);
    k_finalize_refine<<<1, 256, 0, s>>>(g.partials, np, g.st + b);
    DMP_CHECK_HIP(hipGetLastError());
    DMP_CHECK_HIP(hipMemcpyAsync(&host, g.st + b, sizeof(DevState), hipMemcpyDeviceToHost, s));
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    return DMP_OK;
}

void fill_info(const DevState& h, int S, dmp_kind kind, dmp_info* info) {
    if (!info) return;
    info->iters = h.iters;
    info->stop_reason = h.stop_reason;
    info->slices = kind == DMP_FP64_NATIVE ? 0 : S;
    info->kind = int(kind);
    info->E = h.E;
    info->last_dE = h.dE;
    info->trace = h.trace_p;
    info->idem = h.t1;
    info->h_min = h.h_min;
    info->h_max = h.h_max;
    info->mu = h.mu;
    info->lambda = h.lambda;
    info->method = h.method;
    info->refined = h.refined;
    info->E_unrefined = h.refined ? h.E_unrefined : h.E;
    info->products = h.products;
}

}  // namespace

// Purify count matrices that share the kind; used by both entry points.
int purify_many(int count, const double* const* H, const int* n, const int* nocc, double tol,
                const int* slices, dmp_kind kind, int max_iter, int method, int flags,
                double* const* P, double* E, dmp_info* info, void* ws, size_t ws_bytes,
                hipStream_t s, size_t* need_out) {
    // groups of equal slice count and tile choice (the choice follows from
    // each matrix's own n and S, so a matrix gets the same tiles, hence the
    // same fixed-order trace sums and bit-identical results, alone or in a
    // batch)
    std::vector<GroupPlan> groups;
    plan_groups(count, n, slices, kind, method, forced_tile_rb(), groups);
    Carver c(ws);
    for (auto& g : groups) carve_group(c, g, n);
    if (need_out) *need_out = c.used();
    if (ws == nullptr) return DMP_OK;
    if (ws_bytes < c.used()) {
        set_error("workspace of %zu bytes required", c.used());
        return DMP_ENOMEM;
    }
    DMP_CHECK(check_workspace_alignment(ws));
    // one purification at a time per process (see purify_mutex)
    std::lock_guard<std::mutex> serial(purify_mutex());
    std::vector<std::unique_ptr<GroupHost>> keep;
    StreamDrain drain{s};   // declared after ``keep``: the stream drains first
    for (auto& g : groups) {
        DMP_CHECK(upload_group(g, H, P, n, nocc, s, keep));
        DMP_CHECK(launch_init(g, tol, max_iter, s));
    }
    std::vector<DevState> host_st(count);
    {
        size_t off = 0;
        for (auto& g : groups) {
            DMP_CHECK_HIP(hipMemcpyAsync(host_st.data() + off, g.st, g.count * sizeof(DevState),
                                         hipMemcpyDeviceToHost, s));
            off += g.count;
        }
        DMP_CHECK_HIP(hipStreamSynchronize(s));
        keep.clear();
        for (auto& h : host_st)
            if (h.nonfinite) {
                set_error("H holds a non-finite entry");
                return DMP_ENONFINITE;
            }
    }
    if (kind == DMP_FP64_NATIVE) {
        size_t off = 0;
        for (auto& g : groups) {
            DMP_CHECK(run_native(g, max_iter, s, host_st[off], (flags & DMP_NATIVE_TRIANGLE) != 0));
            off += g.count;
        }
    } else {
        DMP_CHECK(run_oz_groups(groups, max_iter, s, host_st, n));
        for (auto& g : groups)
            if (g.method == DMP_CANONICAL) {
                k_mirror_iterate<<<dim3(kE0Blocks, g.count), 256, 0, s>>>(g.pd, g.st);
                DMP_CHECK_HIP(hipGetLastError());
            }
    }
    if (flags & DMP_REFINE_MCWEENY) {
        size_t off = 0;
        for (auto& g : groups) {
            for (int b = 0; b < g.count; ++b) {
                DevState& h = host_st[off + b];
                if (h.iters > 0 && h.stop_reason != DMP_STOP_NONFINITE)
                    DMP_CHECK(refine_mcweeny(g, b, n, h, s));
            }
            off += g.count;
        }
    }
    // results: final iterate lives in Pb[(iters + refined) & 1]
    int status = DMP_OK;
    size_t off = 0;
    for (auto& g : groups) {
        for (int b = 0; b < g.count; ++b) {
            const DevState& h = host_st[off + b];
            const int m = g.idx[b];
            if ((h.iters + h.refined) & 1)
                DMP_CHECK_HIP(hipMemcpyAsync(P[m], g.lay[b].Pw, size_t(n[m]) * n[m] * sizeof(double),
                                             hipMemcpyDeviceToDevice, s));
            if (E) E[m] = h.E;
            fill_info(h, g.S, kind, info ? info + m : nullptr);
            if (h.stop_reason != DMP_STOP_CONVERGED) status = DMP_NOT_CONVERGED;
        }
        off += g.count;
    }
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    return status;
}
}  // namespace dmp

using namespace dmp;

extern "C" {

void dmp_timing_enable(int on) {
    g_timing.on = on != 0;
    g_timing.clocks = on == 2;
}

void dmp_timing_reset(void) {
    const bool on = g_timing.on, clocks = g_timing.clocks;
    g_timing = TimingState{};
    g_timing.on = on;
    g_timing.clocks = clocks;
    if (g_clk != nullptr) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(g_clk_device);
        (void)hipMemset(g_clk, 0, 4 * sizeof(unsigned long long));
        (void)hipSetDevice(cur);
    }
}

int dmp_timing_clock(int which, double* ghz) {
    clear_error();
    if (which < 0 || which > 1 || ghz == nullptr) {
        set_error("which must be 0 or 1 and ghz non-null");
        return DMP_EINVAL;
    }
    *ghz = 0.0;
    if (g_clk == nullptr) return DMP_OK;
    unsigned long long c[2] = {0, 0};
    int cur = 0;
    DMP_CHECK_HIP(hipGetDevice(&cur));
    DMP_CHECK_HIP(hipSetDevice(g_clk_device));
    const hipError_t e = hipMemcpy(c, g_clk + 2 * which, sizeof(c), hipMemcpyDeviceToHost);
    DMP_CHECK_HIP(hipSetDevice(cur));
    DMP_CHECK_HIP(e);
    // the real-time counter runs at 100 MHz
    if (c[1] > 0) *ghz = double(c[0]) / (double(c[1]) * 10.0);
    return DMP_OK;
}

int dmp_timing_read(int which, double* total_ms, long long* launches, double* ops) {
    if (which < 0 || which > 1) return DMP_EINVAL;
    if (total_ms) *total_ms = g_timing.ms[which];
    if (launches) *launches = g_timing.launches[which];
    if (ops) *ops = g_timing.ops[which];
    return DMP_OK;
}

size_t dmp_purify_workspace_bytes(int n, int slices, dmp_kind kind) {
    if (n < 1) return 0;
    if (kind != DMP_FP64_NATIVE && (slices < 1 || slices > kMaxSlices)) return 0;
    if (kind == DMP_MARKIDIS_FP16 && slices > kMaxTerms) return 0;
    size_t need = 0;
    const double* h = nullptr;
    double* p = nullptr;
    int nocc = 0;
    purify_many(1, &h, &n, &nocc, 1.0, &slices, kind, 1, DMP_CANONICAL, 0, &p, nullptr, nullptr,
                nullptr, 0, nullptr, &need);
    return need;
}

int dmp_purify_ex(const double* H, int n, int nocc, double tol, int slices, dmp_kind kind,
                  int max_iter, int method, int flags, double* P, double* E, dmp_info* info,
                  void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    DMP_CHECK(check_method_flags(method, flags));
    DMP_CHECK(check_kind_slices(kind, slices));
    DMP_CHECK(validate_purify_args(H, n, nocc, tol, max_iter, P));
    if (kind != DMP_FP64_NATIVE && n > max_k_for(slices, kind)) {
        set_error("n = %d exceeds the exact INT32 range for %d slices", n, slices);
        return DMP_EINVAL;
    }
    if (ws == nullptr) {
        set_error("workspace of %zu bytes required", dmp_purify_workspace_bytes(n, slices, kind));
        return DMP_ENOMEM;
    }
    return purify_many(1, &H, &n, &nocc, tol, &slices, kind, max_iter, method, flags, &P, E, info,
                       ws, ws_bytes, static_cast<hipStream_t>(stream), nullptr);
}

int dmp_purify(const double* H, int n, int nocc, double tol, int slices, dmp_kind kind,
               int max_iter, double* P, double* E, dmp_info* info, void* ws, size_t ws_bytes,
               void* stream) {
    return dmp_purify_ex(H, n, nocc, tol, slices, kind, max_iter, DMP_CANONICAL, 0, P, E, info,
                         ws, ws_bytes, stream);
}

}  // extern "C"
