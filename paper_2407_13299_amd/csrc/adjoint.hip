// Reverse-mode derivative of the canonical purification (dL/dH for a scalar L
// of the converged density matrix; for L = tr(P W) the seed is W).
//
// Forward with tape: the same kernels as dmp_purify, one iteration at a time;
// for every iteration k the tape keeps c_k, its branch, t1 = tr(P - P^2),
// t2 = tr(P^2 - P^3) and whether c_k was clamped, and it keeps P_k for every
// k that is a multiple of the checkpoint stride.
//
// Backward, for k = K-1 .. 0 (segments of ``stride`` iterations are first
// recomputed from their checkpoint with the same deterministic products, so
// the recomputed iterates equal the forward ones bit for bit).  With Y the
// adjoint of P_{k+1} (symmetric), P = P_k, X2 = P_k^2 and the update
// P_{k+1} = a P + b P^2 + g P^3 on the recorded branch:
//   M = Y P,  MP = M P (= Y P^2),  PM = P M (= P Y P)        (3 Ozaki GEMMs)
//   cbar = a' <Y, P> + b' <Y, P^2> + g' <Y, P^3>,  <Y, P^3> = sum MP o P
//   Y <- a Y + b (M + M^T) + g (MP + MP^T + PM)
//        + cbar ((2P - 3X2) t1 - t2 (I - 2P)) / t1^2     (no cbar if clamped)
// and finally, for P0 = lam (mu I - H) + theta I with mu = tr H / n and lam
// from the Gershgorin bounds (the extremal row held fixed):
//   Hbar = sym(-lam Y + (lam tr Y / n) I + lambar dlam/dH),
//   lambar = mu tr Y - <Y, H>.
// This is the derivative of the recorded iteration (fixed branch pattern),
// the quantity the finite-difference and perturbation-theory checks compare.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "host.hpp"

namespace dmp {
namespace {

constexpr int kDotBlocks = 256;

// Single-matrix Ozaki context: device buffers for one split pair and the
// purification state of one matrix.
struct OzCtx {
    int n = 0, S = 0, KC = 0;
    dmp_kind kind = DMP_OZ_INT8;
    int64_t rb_stride = 0;
    const double* H = nullptr;
    uint8_t* pa = nullptr;
    uint8_t* pb = nullptr;
    int* ea = nullptr;
    int* eb = nullptr;
    uint64_t* ma = nullptr;
    uint64_t* mb = nullptr;
    uint64_t* mc = nullptr;     // column maxima of M = Y P (its column split)
    double* partials = nullptr;
    double* rows = nullptr;
    int* rowbad = nullptr;
    double* e0 = nullptr;
    double* dots = nullptr;     // [kDotBlocks][4]
    double* scal = nullptr;     // [8] device scalars
    PurDesc* pd = nullptr;
    DevState* st = nullptr;
    int rb = 4;                         // tile height, as dmp_purify uses for this
    const Tile* tiles_up = nullptr;     // n and S (upper tiles: purification
    int nt_up = 0;                      // products and the symmetric store)
    const Tile* tiles_full = nullptr;
    int nt_full = 0;
    int* fix = nullptr;                 // part buffer of the split tail of
    int fix_pieces = 0;                 // the purification products
    TailSplit tail{0, 1};
};

void carve_ctx(Carver& c, OzCtx& x, int n, int S, dmp_kind kind) {
    x.n = n;
    x.S = S;
    x.kind = kind;
    x.KC = int(chunks_of(n, kind));
    const TileChoice tc = tile_choice_env(kind, S, n);
    x.rb = tc.rb;
    x.rb_stride = int64_t(x.KC) * S * kFragBytes;
    x.pa = c.take<uint8_t>(plane_bytes(n, n, S, kind));
    x.pb = c.take<uint8_t>(plane_bytes(n, n, S, kind));
    x.ea = c.take<int>(round_up(n, kPad));
    x.eb = c.take<int>(round_up(n, kPad));
    x.ma = c.take<uint64_t>(round_up(n, kPad));
    x.mb = c.take<uint64_t>(round_up(n, kPad));
    x.mc = c.take<uint64_t>(round_up(n, kPad));
    x.partials = c.take<double>(size_t(std::max(upper_tile_count(n, 32 * x.rb), 1)) * kPartials);
    x.rows = c.take<double>(3 * size_t(n));
    x.rowbad = c.take<int>(n);
    x.e0 = c.take<double>(e0_blocks());
    x.dots = c.take<double>(kDotBlocks * 4);
    x.scal = c.take<double>(8);
    x.pd = c.take<PurDesc>(1);
    x.st = c.take<DevState>(1);
    x.fix_pieces = (kind == DMP_OZ_INT8 || kind == DMP_OZ_FP16) && tc.split_tail
                       ? tail_split_capacity(upper_tile_count(n, 32 * x.rb), x.KC, x.rb) : 0;
    x.fix = x.fix_pieces > 0 ? c.take<int>(size_t(x.fix_pieces) * piece_ints(S, x.rb)) : nullptr;
}

int bind_ctx(OzCtx& x, const double* H, int nocc, double* P0, hipStream_t s) {
    x.H = H;
    const int TM = 32 * x.rb;
    const int tm = tile_rows(x.n, TM), tn = tile_cols(x.n);
    DMP_CHECK(cached_tiles(tm, tn, true, &x.tiles_up, TM));
    DMP_CHECK(cached_tiles(tm, tn, false, &x.tiles_full, TM));
    x.nt_up = upper_tile_count(x.n, TM);
    x.nt_full = tm * tn;
    x.tail = TailSplit{x.nt_up, 1};
    if (x.fix != nullptr && tail_split_enabled()) {
        int slots = 0;
        DMP_CHECK(resident_slots(x.S, x.kind, x.rb, &slots));
        x.tail = plan_tail_split(x.nt_up, slots, x.KC, x.fix_pieces);
    }
    PurDesc d{};
    d.H = H;
    d.Pb[0] = P0;
    d.Pb[1] = P0;
    d.rows = x.rows;
    d.rowbad = x.rowbad;
    d.e0 = x.e0;
    d.partials = x.partials;
    d.n = x.n;
    d.nocc = nocc;
    d.part_begin = 0;
    d.part_end = x.nt_up;
    DMP_CHECK_HIP(hipMemcpyAsync(x.pd, &d, sizeof(d), hipMemcpyHostToDevice, s));
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    return DMP_OK;
}

SplitDesc split_of(const OzCtx& x, const double* A, bool trans, uint64_t* mb, int* ex,
                   uint8_t* planes, int state_index) {
    SplitDesc d{};
    d.A = A;
    d.lda = x.n;
    d.R = x.n;
    d.K = x.n;
    d.trans = trans ? 1 : 0;
    d.KC = x.KC;
    d.maxbits = mb;
    d.expo = ex;
    d.planes = planes;
    d.state_index = state_index;
    return d;
}

MatDesc gemm_desc(const OzCtx& x, const uint8_t* pa, const int* ea, const uint8_t* pb,
                  const int* eb, double* out) {
    MatDesc m{};
    m.pa = pa;
    m.pb = pb;
    m.ea = ea;
    m.eb = eb;
    m.out = out;
    m.a_rb_stride = x.rb_stride;
    m.b_rb_stride = x.rb_stride;
    m.M = x.n;
    m.N = x.n;
    m.KC = x.KC;
    m.ldc = x.n;
    m.state_index = 0;
    return m;
}

// One forward iteration P_in -> (X2_out, P_out) with the purification
// kernels; the coefficient is recomputed on the device from the traces.
// The row maxima of X2 and of P_out come from the products' epilogues (into
// x.mb and x.ma, each zeroed by the split before its product); p_maxima:
// x.ma already holds those of P_in (the previous iteration's update), so
// its split runs only the digit kernel.
int forward_iteration(const OzCtx& x, const double* P_in, double* X2_out, double* P_out,
                      bool finalize, bool p_maxima, hipStream_t s) {
    SplitDesc sp = split_of(x, P_in, false, x.ma, x.ea, x.pa, 0);
    sp.clear = x.mb;
    if (p_maxima)
        DMP_CHECK(launch_split_digits(sp, x.S, x.kind, x.st, s));
    else
        DMP_CHECK(launch_split(sp, x.S, x.kind, x.st, s));
    GemmParams p{};
    p.tiles = x.tiles_up;
    p.one = gemm_desc(x, x.pa, x.ea, x.pa, x.ea, X2_out);
    p.one.P = P_in;
    p.one.rowmax = x.mb;
    p.partials = x.partials;
    p.states = x.st;
    p.mode = EPI_SQUARE;
    if (x.tail.nsplit > 1) {   // the split tail of the purification products
        p.fix = x.fix;
        p.nfull = x.tail.nfull;
        p.nsplit = x.tail.nsplit;
    }
    DMP_CHECK(launch_ozgemm(x.S, x.kind, p, x.nt_up, s, x.rb));
    DMP_CHECK(launch_finalize_coef(x.pd, x.st, 1, s));
    SplitDesc sx = split_of(x, X2_out, false, x.mb, x.eb, x.pb, 0);
    sx.clear = x.ma;
    DMP_CHECK(launch_split_digits(sx, x.S, x.kind, x.st, s));
    p.one = gemm_desc(x, x.pb, x.eb, x.pa, x.ea, P_out);
    p.one.P = P_in;
    p.one.X2 = X2_out;
    p.one.H = x.H;
    p.one.rowmax = x.ma;
    p.mode = EPI_UPDATE;
    DMP_CHECK(launch_ozgemm(x.S, x.kind, p, x.nt_up, s, x.rb));
    if (finalize) DMP_CHECK(launch_finalize_iter(x.pd, x.st, 1, s));
    return DMP_OK;
}

// Coefficient data of one recorded step.
struct StepRecord {
    double c, t1, t2;
    int branch, clamped;
};

// Records the step the state has just finished (index iters - 1); once the
// run has stopped, every later launch rewrites that entry with the same
// values.
__global__ void k_record_step(const DevState* st, StepRecord* hist) {
    const DevState& s = *st;
    if (threadIdx.x == 0 && s.iters > 0)
        hist[s.iters - 1] = StepRecord{s.c, s.t1, s.t2, s.branch, s.clamped};
}

// C = A B for n x n operands already split: (pa, ea) rows of A, (pb, eb)
// columns of B.  rowmax / colmax (nullable, zeroed beforehand) receive the
// maxima of |C| per row / column for the splits of C.  ``sym``: C is known
// to be symmetric; only its upper tiles are computed and mirrored.
int gemm_store(const OzCtx& x, const uint8_t* pa, const int* ea, const uint8_t* pb,
               const int* eb, double* out, uint64_t* rowmax, uint64_t* colmax, bool sym,
               hipStream_t s) {
    GemmParams p{};
    p.tiles = sym ? x.tiles_up : x.tiles_full;
    p.one = gemm_desc(x, pa, ea, pb, eb, out);
    p.one.state_index = -1;
    p.one.rowmax = rowmax;
    p.one.colmax = colmax;
    p.mode = sym ? EPI_STORE_SYM : EPI_STORE;
    return launch_ozgemm(x.S, x.kind, p, sym ? x.nt_up : x.nt_full, s, x.rb);
}

__device__ inline double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double bsum(double v, double* sh) {
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// Y = (A + A^T) / 2 on 32 x 32 tile pairs (I <= J), through LDS.
__global__ __launch_bounds__(256) void k_sym(const double* A, double* Y, int n, const int2* pairs) {
    __shared__ double t[32][33];
    const int2 pr = pairs[blockIdx.x];
    const int I = pr.x, J = pr.y, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = J * 32 + r, j = I * 32 + tx;
        t[r][tx] = (i < n && j < n) ? A[int64_t(i) * n + j] : 0.0;   // tile (J, I)
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = I * 32 + r, j = J * 32 + tx;
        if (i < n && j < n) {
            const double v = 0.5 * (A[int64_t(i) * n + j] + t[tx][r]);
            Y[int64_t(i) * n + j] = v;
            Y[int64_t(j) * n + i] = v;
        }
    }
}

// Block partials of sum Y o P, sum Y o X2, sum MP o P (fixed grid).
__global__ __launch_bounds__(256) void k_adj_dots(const double* Y, const double* P,
                                                  const double* X2, const double* MP, int n,
                                                  double* out) {
    __shared__ double sh[4];
    const int64_t tot = int64_t(n) * n;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < tot; i += int64_t(kDotBlocks) * 256) {
        const double y = Y[i], p = P[i];
        a += y * p;
        b += y * X2[i];
        c += MP[i] * p;
    }
    a = bsum(a, sh);
    b = bsum(b, sh);
    c = bsum(c, sh);
    if (threadIdx.x == 0) {
        out[blockIdx.x * 4 + 0] = a;
        out[blockIdx.x * 4 + 1] = b;
        out[blockIdx.x * 4 + 2] = c;
    }
}

// cbar of one step from the dot partials and the recorded c, branch.
__global__ __launch_bounds__(256) void k_adj_cbar(const double* dots, double c, int branch,
                                                  int clamped, double* scal) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0, g = 0.0;
    for (int i = threadIdx.x; i < kDotBlocks; i += 256) {
        a += dots[i * 4 + 0];
        b += dots[i * 4 + 1];
        g += dots[i * 4 + 2];
    }
    a = bsum(a, sh);
    b = bsum(b, sh);
    g = bsum(g, sh);
    if (threadIdx.x == 0) {
        double cbar = 0.0;
        if (!clamped) {
            if (branch) {
                cbar = (-b + g) / (c * c);            // beta' = -1/c^2, gamma' = 1/c^2
            } else {
                const double q = (1.0 - c) * (1.0 - c);
                cbar = (-a + 2.0 * b - g) / q;        // alpha' = -1/q, beta' = 2/q, gamma' = -1/q
            }
        }
        scal[0] = cbar;
    }
}

// Y' = a Y + b (M + M^T) + g (MP + MP^T + PM) + cbar dc, on tile pairs
// (I <= J); symmetric, written to both tiles.  PM = P Y P is stored exactly
// symmetric (upper tiles mirrored), so it needs no transpose.
__global__ __launch_bounds__(256) void k_adj_combine(const double* Y, const double* M,
                                                     const double* MP, const double* PM,
                                                     const double* P, const double* X2,
                                                     double* Yn, int n, double a, double b,
                                                     double g, double t1, double t2,
                                                     const double* scal, const int2* pairs) {
    __shared__ double tM[32][33], tMP[32][33], tO[32][33];
    const int2 pr = pairs[blockIdx.x];
    const int I = pr.x, J = pr.y, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double cbar = scal[0];
    const double inv = (cbar != 0.0) ? 1.0 / (t1 * t1) : 0.0;
    for (int r = ty; r < 32; r += 8) {      // tile (J, I) of M and MP
        const int i = J * 32 + r, j = I * 32 + tx;
        const bool ok = i < n && j < n;
        const int64_t o = int64_t(i) * n + j;
        tM[r][tx] = ok ? M[o] : 0.0;
        tMP[r][tx] = ok ? MP[o] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = I * 32 + r, j = J * 32 + tx;
        double v = 0.0;
        if (i < n && j < n) {
            const int64_t o = int64_t(i) * n + j;
            const double p = P[o], x2 = X2[o];
            v = a * Y[o] + b * (M[o] + tM[tx][r]) + g * (MP[o] + tMP[tx][r] + PM[o]);
            if (cbar != 0.0) v += cbar * ((2.0 * p - 3.0 * x2) * t1 - t2 * ((i == j ? 1.0 : 0.0) - 2.0 * p)) * inv;
            Yn[o] = v;
        }
        tO[r][tx] = v;
    }
    __syncthreads();
    if (I != J) {
        for (int r = ty; r < 32; r += 8) {
            const int i = J * 32 + r, j = I * 32 + tx;
            if (i < n && j < n) Yn[int64_t(i) * n + j] = tO[tx][r];
        }
    }
}

// Partials of tr Y and <Y, H>.
__global__ __launch_bounds__(256) void k_adj_dots0(const double* Y, const double* H, int n,
                                                   double* out) {
    __shared__ double sh[4];
    const int64_t tot = int64_t(n) * n;
    double tr = 0.0, yh = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < tot; i += int64_t(kDotBlocks) * 256) {
        yh += Y[i] * H[i];
        if (i / n == i % n) tr += Y[i];
    }
    tr = bsum(tr, sh);
    yh = bsum(yh, sh);
    if (threadIdx.x == 0) {
        out[blockIdx.x * 4 + 0] = tr;
        out[blockIdx.x * 4 + 1] = yh;
    }
}

__global__ __launch_bounds__(256) void k_adj_scal0(const double* dots, double* scal) {
    __shared__ double sh[4];
    double tr = 0.0, yh = 0.0;
    for (int i = threadIdx.x; i < kDotBlocks; i += 256) {
        tr += dots[i * 4 + 0];
        yh += dots[i * 4 + 1];
    }
    tr = bsum(tr, sh);
    yh = bsum(yh, sh);
    if (threadIdx.x == 0) {
        scal[1] = tr;
        scal[2] = yh;
    }
}

// Hbar from the adjoint of P0 (see the header of this file).
__global__ __launch_bounds__(256) void k_adj_initial(const double* Y, const double* H, double* Hbar,
                                                     int n, double lam, double mu, double theta,
                                                     double h_min, double h_max, int which, int rmax,
                                                     int rmin, const double* scal) {
    const int64_t tot = int64_t(n) * n;
    const double trY = scal[1], yh = scal[2];
    const double lambar = mu * trY - yh;
    const int r = which == 0 ? rmax : rmin;
    const double sg = which == 0 ? 1.0 : -1.0;
    const double kap = which == 0 ? -theta / ((h_max - mu) * (h_max - mu))
                                  : -(1.0 - theta) / ((mu - h_min) * (mu - h_min));
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < tot;
         idx += int64_t(gridDim.x) * 256) {
        const int i = int(idx / n), j = int(idx % n);
        const double dij = i == j ? 1.0 : 0.0;
        auto gent = [&](int a, int b) -> double {
            if (a != r) return 0.0;
            if (b == r) return 1.0;
            const double h = H[int64_t(r) * n + b];
            return sg * (h > 0.0 ? 1.0 : (h < 0.0 ? -1.0 : 0.0));
        };
        const double gs = 0.5 * (gent(i, j) + gent(j, i));
        const double dl = which == 0 ? (gs - dij / n) : (dij / n - gs);
        double v = -lam * Y[idx] + dij * lam * trY / n;
        if (lam != 0.0) v += lambar * kap * dl;
        Hbar[idx] = v;
    }
}

std::vector<int2> tile_pairs32(int n) {
    std::vector<int2> v;
    const int t = (n + 31) / 32;
    for (int i = 0; i < t; ++i)
        for (int j = i; j < t; ++j) v.push_back(int2{i, j});
    return v;
}

}  // namespace
}  // namespace dmp

using namespace dmp;

struct dmp_tape {
    int n = 0, nocc = 0, S = 0, stride = 1, K = 0, device = 0;
    dmp_kind kind = DMP_OZ_INT8;
    const double* H = nullptr;
    DevState init{};
    std::vector<double> c, t1, t2;
    std::vector<int> branch, clamped;
    std::vector<double*> ckpt;   // device copies of P_0, P_stride, ...
    std::vector<double*> x2;     // stride 1: X2_0, X2_1, ... as well (no recomputation)
    std::vector<void*> owned;    // the device allocations holding them
    void* fwd_ws = nullptr;      // forward workspace (owned)
    double* H_copy = nullptr;    // tape-owned copy of H (the caller's may change)
};

extern "C" {

void dmp_tape_free(dmp_tape* t) {
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    for (void* p : t->owned) (void)hipFree(p);
    if (t->fwd_ws) (void)hipFree(t->fwd_ws);
    if (t->H_copy) (void)hipFree(t->H_copy);
    (void)hipSetDevice(cur);
    delete t;
}

int dmp_tape_info(const dmp_tape* t, int* iters, int* branches) {
    if (!t) {
        set_error("null tape");
        return DMP_EINVAL;
    }
    if (iters) *iters = t->K;
    if (branches)
        for (int k = 0; k < t->K; ++k) branches[k] = t->branch[k];
    return DMP_OK;
}

int dmp_tape_coefficients(const dmp_tape* t, double* c, double* t1, double* t2) {
    if (!t) {
        set_error("null tape");
        return DMP_EINVAL;
    }
    for (int k = 0; k < t->K; ++k) {
        if (c) c[k] = t->c[k];
        if (t1) t1[k] = t->t1[k];
        if (t2) t2[k] = t->t2[k];
    }
    return DMP_OK;
}

int dmp_purify_fwd_tape(const double* H, int n, int nocc, double tol, int slices, dmp_kind kind,
                        int max_iter, int ckpt_stride, double* P, double* E, dmp_info* info,
                        dmp_tape** tape, void* stream) {
    clear_error();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!tape) {
        set_error("tape pointer is null");
        return DMP_EINVAL;
    }
    *tape = nullptr;
    {
        const hipError_t pending = hipGetLastError();
        if (pending != hipSuccess) {
            set_error("a previous HIP call failed: %s", hipGetErrorString(pending));
            return DMP_EHIP;
        }
    }
    DMP_CHECK(check_kind_slices(kind, slices));
    if (kind != DMP_OZ_INT8 && kind != DMP_OZ_FP16) {
        set_error("the recorded adjoint is built for the Ozaki kinds");
        return DMP_EUNSUPPORTED;
    }
    DMP_CHECK(validate_purify_args(H, n, nocc, tol, max_iter, P));
    if (n > max_k_for_slices(slices)) {
        set_error("n = %d exceeds the exact INT32 range for %d slices", n, slices);
        return DMP_EINVAL;
    }
    // default: every iterate and its square when the worst case (max_iter
    // steps) takes at most a quarter of the free device memory (then the
    // backward recomputes nothing), else checkpoints every sqrt(max_iter)
    int stride = ckpt_stride;
    if (stride <= 0) {
        size_t free_b = 0, total_b = 0;
        const double full = 2.0 * double(max_iter) * double(n) * double(n) * sizeof(double);
        const bool fits = hipMemGetInfo(&free_b, &total_b) == hipSuccess && full <= 0.25 * double(free_b);
        (void)hipGetLastError();
        stride = fits ? 1 : std::max(1, int(std::ceil(std::sqrt(double(max_iter)))));
    }
    // one purification at a time per process (see purify_mutex)
    std::lock_guard<std::mutex> serial(purify_mutex());
    dmp_tape* t = new dmp_tape();
    t->n = n;
    t->nocc = nocc;
    t->S = slices;
    t->kind = kind;
    t->stride = stride;
    (void)hipGetDevice(&t->device);
    // the backward pass reads H again: keep a copy owned by the tape
    if (hipMalloc(&t->H_copy, size_t(n) * n * sizeof(double)) != hipSuccess ||
        hipMemcpyAsync(t->H_copy, H, size_t(n) * n * sizeof(double), hipMemcpyDefault, s) != hipSuccess) {
        set_error("copy of H into the tape failed");
        dmp_tape_free(t);
        return DMP_ENOMEM;
    }
    t->H = t->H_copy;

    // measure with exactly the takes used below (alignment padding included)
    Carver m(nullptr);
    OzCtx probe;
    carve_ctx(m, probe, n, slices, kind);
    m.take<double>(size_t(n) * n);   // X2
    m.take<double>(size_t(n) * n);   // second iterate
    const size_t need = m.used();
    if (hipMalloc(&t->fwd_ws, need) != hipSuccess) {
        set_error("hipMalloc of %zu bytes for the forward tape failed", need);
        dmp_tape_free(t);
        return DMP_ENOMEM;
    }
    Carver c(t->fwd_ws);
    OzCtx x;
    carve_ctx(c, x, n, slices, kind);
    double* X2 = c.take<double>(size_t(n) * n);
    double* Pw = c.take<double>(size_t(n) * n);
    int st = bind_ctx(x, t->H, nocc, P, s);
    if (st == DMP_OK) st = launch_purify_init(x.pd, x.st, 1, n, tol, max_iter, s);
    DevState h{};
    if (st == DMP_OK && (hipMemcpyAsync(&h, x.st, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess)) {
        set_error("state readback failed");
        st = DMP_EHIP;
    }
    if (st == DMP_OK && h.nonfinite) {
        set_error("H holds a non-finite entry");
        st = DMP_ENONFINITE;
    }
    if (st != DMP_OK) {
        dmp_tape_free(t);
        return st;
    }
    t->init = h;
    // n x n device slots owned by the tape, allocated in blocks that double
    // in size (8, 16, ... slots): a few allocations for a whole run
    const size_t nn = size_t(n) * n;
    std::vector<double*> pool;
    size_t grow = 8;
    auto slot = [&](double** out) -> int {
        if (pool.empty()) {
            void* blk = nullptr;
            if (hipMalloc(&blk, grow * nn * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipMalloc of %zu tape slots failed", grow);
                return DMP_ENOMEM;
            }
            t->owned.push_back(blk);
            for (size_t i = grow; i-- > 0;) pool.push_back(static_cast<double*>(blk) + i * nn);
            grow = std::min<size_t>(grow * 2, 64);
        }
        *out = pool.back();
        pool.pop_back();
        return DMP_OK;
    };
    auto checkpoint = [&](const double* src, std::vector<double*>& into) -> int {
        double* d = nullptr;
        DMP_CHECK(slot(&d));
        into.push_back(d);
        const hipError_t e = hipMemcpyAsync(d, src, nn * sizeof(double), hipMemcpyDefault, s);
        if (e != hipSuccess) {
            set_error("checkpoint copy failed: %s", hipGetErrorString(e));
            return DMP_EHIP;
        }
        return DMP_OK;
    };
    // the coefficient data of every step, recorded on the device and read
    // once at the end; the state is read after every kStepsPerRead steps only
    // (steps launched after the run stopped exit at once)
    StepRecord* hist = nullptr;
    if (hipMalloc(&hist, size_t(std::max(1, max_iter)) * sizeof(StepRecord)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of the step records failed");
        dmp_tape_free(t);
        return DMP_ENOMEM;
    }
    t->owned.push_back(hist);
    constexpr int kStepsPerRead = 4;
    double* cur = P;
    double* nxt = Pw;
    if (!h.done) st = checkpoint(P, t->ckpt);
    if (stride == 1 && !h.done) cur = t->ckpt[0];
    int launched = 0;
    bool done = h.done != 0;
    while (st == DMP_OK && !done && launched < max_iter) {
        for (int c = 0; st == DMP_OK && c < kStepsPerRead && launched < max_iter; ++c, ++launched) {
            // stride 1: X2_k and P_{k+1} are written straight into tape slots
            double* x2k = X2;
            if (stride == 1) {
                st = slot(&x2k);
                if (st == DMP_OK) st = slot(&nxt);
                if (st != DMP_OK) break;
                t->x2.push_back(x2k);
            }
            st = forward_iteration(x, cur, x2k, nxt, true, launched > 0, s);
            if (st != DMP_OK) break;
            k_record_step<<<1, 64, 0, s>>>(x.st, hist);
            if (hipGetLastError() != hipSuccess) {
                set_error("launch of the step record failed");
                st = DMP_EHIP;
                break;
            }
            if (stride == 1) {
                cur = nxt;
                t->ckpt.push_back(cur);
            } else {
                std::swap(cur, nxt);
                if ((launched + 1) % stride == 0) st = checkpoint(cur, t->ckpt);
            }
        }
        if (st != DMP_OK) break;
        if (hipMemcpyAsync(&h, x.st, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("state readback failed");
            st = DMP_EHIP;
            break;
        }
        done = h.done != 0;
    }
    const int K = st == DMP_OK ? h.iters : 0;
    std::vector<StepRecord> rec(size_t(std::max(K, 1)));
    if (st == DMP_OK && K > 0 &&
        (hipMemcpyAsync(rec.data(), hist, size_t(K) * sizeof(StepRecord), hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess)) {
        set_error("readback of the step records failed");
        st = DMP_EHIP;
    }
    if (st != DMP_OK) {
        dmp_tape_free(t);
        return st;
    }
    for (int k = 0; k < K; ++k) {
        t->c.push_back(rec[k].c);
        t->branch.push_back(rec[k].branch);
        t->t1.push_back(rec[k].t1);
        t->t2.push_back(rec[k].t2);
        t->clamped.push_back(rec[k].clamped);
    }
    t->K = K;
    // steps launched past the stop left their slots unwritten: P_K is slot K
    // (stride 1) or, ping-ponging from P, P for even K and Pw for odd K
    double* last = stride == 1 ? (K > 0 ? t->ckpt[K] : P) : (K % 2 == 0 ? P : Pw);
    if (stride == 1 && int(t->x2.size()) > K) t->x2.resize(K);
    if (last != P) {
        if (hipMemcpyAsync(P, last, size_t(n) * n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("copy of the result failed");
            dmp_tape_free(t);
            return DMP_EHIP;
        }
    }
    if (E) *E = h.E;
    if (info) {
        info->iters = h.iters;
        info->stop_reason = h.stop_reason;
        info->slices = slices;
        info->kind = int(kind);
        info->E = h.E;
        info->last_dE = h.dE;
        info->trace = h.trace_p;
        info->idem = h.t1;
        info->h_min = h.h_min;
        info->h_max = h.h_max;
        info->mu = h.mu;
        info->lambda = h.lambda;
    }
    *tape = t;
    return h.stop_reason == DMP_STOP_CONVERGED ? DMP_OK : DMP_NOT_CONVERGED;
}

static size_t carve_bwd(Carver& c, const dmp_tape* t, OzCtx* x, double** bufs, double** segP,
                        double** segX, int2** pairs) {
    const int n = t->n;
    const size_t nn = size_t(n) * n;
    OzCtx tmp;
    carve_ctx(c, x ? *x : tmp, n, t->S, t->kind);
    for (int i = 0; i < 5; ++i) {
        double* p = c.take<double>(nn);
        if (bufs) bufs[i] = p;
    }
    for (int i = 0; i <= t->stride; ++i) {
        double* p = c.take<double>(nn);
        if (segP) segP[i] = p;
    }
    for (int i = 0; i < t->stride; ++i) {
        double* p = c.take<double>(nn);
        if (segX) segX[i] = p;
    }
    const int t32 = (n + 31) / 32;
    int2* pr = c.take<int2>(size_t(t32) * (t32 + 1) / 2);
    if (pairs) *pairs = pr;
    return c.used();
}

size_t dmp_purify_bwd_workspace_bytes(const dmp_tape* t) {
    if (!t) return 0;
    Carver c(nullptr);
    return carve_bwd(c, t, nullptr, nullptr, nullptr, nullptr, nullptr);
}

int dmp_purify_bwd(const dmp_tape* t, const double* Pbar, double* Hbar, void* ws, size_t ws_bytes,
                   void* stream) {
    clear_error();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!t || !Pbar || !Hbar) {
        set_error("null argument");
        return DMP_EINVAL;
    }
    const size_t need = dmp_purify_bwd_workspace_bytes(t);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes required", need);
        return DMP_ENOMEM;
    }
    DMP_CHECK(check_workspace_alignment(ws));
    const int n = t->n;
    // one purification at a time per process (see purify_mutex)
    std::lock_guard<std::mutex> serial(purify_mutex());
    Carver c(ws);
    OzCtx x;
    double* b[5];
    std::vector<double*> segP(t->stride + 1), segX(t->stride);
    int2* pairs = nullptr;
    carve_bwd(c, t, &x, b, segP.data(), segX.data(), &pairs);
    DMP_CHECK(bind_ctx(x, t->H, t->nocc, segP[0], s));
    double *Y = b[0], *Yn = b[1], *M = b[2], *MP = b[3], *PM = b[4];
    std::vector<int2> hp = tile_pairs32(n);
    StreamDrain drain{s};   // ``hp`` outlives its copy, also on an error return
    DMP_CHECK_HIP(hipMemcpyAsync(pairs, hp.data(), hp.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    k_sym<<<unsigned(hp.size()), 256, 0, s>>>(Pbar, Y, n, pairs);
    DMP_CHECK_HIP(hipGetLastError());

    DevState fresh = t->init;
    fresh.done = 0;
    fresh.iters = 0;
    const int K = t->K;
    const int nseg = (K + t->stride - 1) / t->stride;
    // every step's P and X2 on the tape: nothing to recompute
    const bool stored = t->stride == 1 && int(t->x2.size()) == K && int(t->ckpt.size()) >= K;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int start = seg * t->stride, end = std::min(start + t->stride, K);
        if (!stored) {
            DMP_CHECK_HIP(hipMemcpyAsync(segP[0], t->ckpt[seg], size_t(n) * n * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
            DMP_CHECK_HIP(hipMemcpyAsync(x.st, &fresh, sizeof(fresh), hipMemcpyHostToDevice, s));
            for (int j = start; j < end; ++j)
                DMP_CHECK(forward_iteration(x, segP[j - start], segX[j - start], segP[j - start + 1],
                                            false, j > start, s));
        }
        for (int j = end - 1; j >= start; --j) {
            const double* P = stored ? t->ckpt[j] : segP[j - start];
            const double* X2 = stored ? t->x2[j] : segX[j - start];
            // M = Y P, MP = M P, PM = P M.  The row and column maxima of M
            // come from its product's epilogue (x.ma, x.mc: zeroed by the
            // digit kernels of the two splits before it, once their own
            // maxima are no longer read), so M's two splits run only their
            // digit kernels.  PM = P Y P is symmetric: upper tiles, mirrored.
            SplitDesc sy = split_of(x, Y, false, x.ma, x.ea, x.pa, -1);
            sy.clear = x.mc;
            DMP_CHECK(launch_split(sy, x.S, x.kind, nullptr, s));
            SplitDesc sp = split_of(x, P, false, x.mb, x.eb, x.pb, -1);
            sp.clear = x.ma;
            DMP_CHECK(launch_split(sp, x.S, x.kind, nullptr, s));
            DMP_CHECK(gemm_store(x, x.pa, x.ea, x.pb, x.eb, M, x.ma, x.mc, false, s));
            DMP_CHECK(launch_split_digits(split_of(x, M, false, x.ma, x.ea, x.pa, -1), x.S, x.kind,
                                          nullptr, s));
            DMP_CHECK(gemm_store(x, x.pa, x.ea, x.pb, x.eb, MP, nullptr, nullptr, false, s));
            DMP_CHECK(launch_split_digits(split_of(x, M, true, x.mc, x.ea, x.pa, -1), x.S, x.kind,
                                          nullptr, s));
            DMP_CHECK(gemm_store(x, x.pb, x.eb, x.pa, x.ea, PM, nullptr, nullptr, true, s));
            const double cc = t->c[j];
            const int br = t->branch[j];
            double a, bb, g;
            if (br) {
                a = 0.0;
                bb = (1.0 + cc) / cc;
                g = -1.0 / cc;
            } else {
                a = (1.0 - 2.0 * cc) / (1.0 - cc);
                bb = (1.0 + cc) / (1.0 - cc);
                g = -1.0 / (1.0 - cc);
            }
            k_adj_dots<<<kDotBlocks, 256, 0, s>>>(Y, P, X2, MP, n, x.dots);
            k_adj_cbar<<<1, 256, 0, s>>>(x.dots, cc, br, t->clamped[j], x.scal);
            k_adj_combine<<<unsigned(hp.size()), 256, 0, s>>>(Y, M, MP, PM, P, X2, Yn, n, a, bb, g,
                                                               t->t1[j], t->t2[j], x.scal, pairs);
            DMP_CHECK_HIP(hipGetLastError());
            std::swap(Y, Yn);
        }
    }
    const DevState& i0 = t->init;
    k_adj_dots0<<<kDotBlocks, 256, 0, s>>>(Y, t->H, n, x.dots);
    k_adj_scal0<<<1, 256, 0, s>>>(x.dots, x.scal);
    k_adj_initial<<<1024, 256, 0, s>>>(Y, t->H, Hbar, n, i0.lambda, i0.mu, i0.theta, i0.h_min, i0.h_max,
                                       i0.which, i0.row_hmax, i0.row_hmin, x.scal);
    DMP_CHECK_HIP(hipGetLastError());
    DMP_CHECK_HIP(hipStreamSynchronize(s));
    return DMP_OK;
}

}  // extern "C"
