// Allocation-free variant of the Ozaki-scheme GEMM (Sec. 2.4) for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid it).  Its scratch memory (the digit
// planes, exponents and maxima of both operands and the tile list) is one
// file-scope device array, held by every GPU the library runs on until the
// process ends; the tile list is written by a kernel, so nothing is staged
// from host memory either.  Every call on a GPU shares that GPU's array:
// calls that overlap on one GPU (several streams or threads) race.
#include <algorithm>
#include <mutex>

#include "host.hpp"

namespace dmp {

// 64 MiB: room for m = n = k = 2048 at up to 7 INT8 slices (56 MiB of digit
// planes), or for example 1024 x 4096 by 4096 x 1024 at S = 7.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

// Device address of ``scratch`` per device, looked up on the first call on
// that device (with that device current).  The array's name is a host-side
// stand-in in host code; only these addresses are passed to kernels.
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_address(void** out) {
    int dev = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the scratch table holds", dev, kMaxDevices);
        return DMP_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev] == nullptr) {
        void* p = nullptr;
        DMP_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) {
            set_error("hipGetSymbolAddress returned a null address for the scratch array");
            return DMP_EHIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DMP_OK;
}

// Tiles of a tm x tn grid of 128 x 64 output tiles in the order of
// append_tiles(..., upper = false): 512 x 512 super-tiles row-major, and
// row-major inside each.  Super-row si holds rows [GI si, GI si + ri) of
// all tn columns; its super-tile sj holds columns [GJ sj, GJ sj + cj).
__global__ void k_fill_tiles(Tile* out, int tm, int tn) {
    constexpr int GI = 512 / kTileM, GJ = 512 / kTileN;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tm * tn) return;
    const int si = t / (GI * tn);
    const int ri = min(GI, tm - si * GI);
    const int r = t - si * GI * tn;
    const int sj = r / (GJ * ri);
    const int cj = min(GJ, tn - sj * GJ);
    const int r2 = r - sj * GJ * ri;
    out[t] = Tile{uint16_t(si * GI + r2 / cj), uint16_t(sj * GJ + r2 % cj), 0u};
}

__global__ void k_zero_matrix(double* c, int m, int n, int ldc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < int64_t(m) * n) c[(i / n) * ldc + i % n] = 0.0;
}

struct NoAllocLayout {
    uint8_t* pa;
    uint8_t* pb;
    int* ea;
    int* eb;
    uint64_t* ma;
    uint64_t* mb;
    Tile* tiles;
};

NoAllocLayout carve_noalloc(Carver& c, int m, int n, int k, int s, dmp_kind kind) {
    NoAllocLayout g;
    g.pa = c.take<uint8_t>(plane_bytes(m, k, s, kind));
    g.pb = c.take<uint8_t>(plane_bytes(n, k, s, kind));
    g.ea = c.take<int>(round_up(m, kPad));
    g.eb = c.take<int>(round_up(n, kPad));
    g.ma = c.take<uint64_t>(round_up(m, kPad));
    g.mb = c.take<uint64_t>(round_up(n, kPad));
    g.tiles = c.take<Tile>(size_t(tile_rows(m)) * size_t(tile_cols(n)));
    return g;
}

bool trans_of(char t, bool* out) {
    if (t == 'N' || t == 'n') *out = false;
    else if (t == 'T' || t == 't') *out = true;
    else return false;
    return true;
}

}  // namespace

}  // namespace dmp

using namespace dmp;

extern "C" {

int dmp_ozaki_gemm_noalloc(char transA, char transB, int m, int n, int k, const double* A,
                           int lda, const double* B, int ldb, double* C, int ldc, int slices,
                           dmp_kind kind, void* stream) {
    clear_error();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kind != DMP_OZ_INT8 && kind != DMP_OZ_FP16 && kind != DMP_MARKIDIS_FP16) {
        set_error("the allocation-free GEMM runs the Ozaki and Markidis kinds only");
        return DMP_EINVAL;
    }
    DMP_CHECK(check_kind_slices(kind, slices));
    bool ta = false, tb = false;
    if (!trans_of(transA, &ta) || !trans_of(transB, &tb)) {
        set_error("trans must be 'N' or 'T'");
        return DMP_EINVAL;
    }
    if (m < 0 || n < 0 || k < 0) {
        set_error("negative size");
        return DMP_EINVAL;
    }
    const int a_cols = ta ? m : k, b_cols = tb ? k : n;
    if (lda < std::max(1, a_cols) || ldb < std::max(1, b_cols) || ldc < std::max(1, n)) {
        set_error("leading dimension too small");
        return DMP_EINVAL;
    }
    if (m == 0 || n == 0) return DMP_OK;
    if (C == nullptr || (k > 0 && (A == nullptr || B == nullptr))) {
        set_error("null matrix pointer");
        return DMP_EINVAL;
    }
    if (k == 0) {
        const int64_t tot = int64_t(m) * n;
        k_zero_matrix<<<unsigned((tot + 255) / 256), 256, 0, s>>>(C, m, n, ldc);
        DMP_CHECK_HIP(hipGetLastError());
        return DMP_OK;
    }
    if (k > max_k_for(slices, kind)) {
        set_error("k = %d exceeds the exact INT32 range for %d slices (max %lld)", k, slices,
                  (long long)max_k_for(slices, kind));
        return DMP_EINVAL;
    }
    if (m > 65535 * kTileN || n > 65535 * kTileN) {
        set_error("matrix too large");
        return DMP_EINVAL;
    }
    Carver measure(nullptr);
    carve_noalloc(measure, m, n, k, slices, kind);
    if (measure.used() > kNoAllocScratchBytes) {
        set_error("the product needs %zu bytes of scratch; the allocation-free GEMM holds %zu "
                  "(use dmp_ozaki_gemm with a workspace)", measure.used(), kNoAllocScratchBytes);
        return DMP_EINVAL;
    }
    void* base = nullptr;
    DMP_CHECK(scratch_address(&base));
    Carver c(base);
    const NoAllocLayout g = carve_noalloc(c, m, n, k, slices, kind);
    const int KC = int(chunks_of(k, kind));
    const int64_t rb_stride = int64_t(KC) * planes_of(slices, kind) * kFragBytes;

    SplitDesc da{};
    da.A = A;
    da.lda = lda;
    da.R = m;
    da.K = k;
    da.trans = ta ? 1 : 0;
    da.KC = KC;
    da.maxbits = g.ma;
    da.expo = g.ea;
    da.planes = g.pa;
    da.state_index = -1;
    SplitDesc db = da;
    db.A = B;
    db.lda = ldb;
    db.R = n;
    db.trans = tb ? 0 : 1;   // operand row j = column j of op(B)
    db.maxbits = g.mb;
    db.expo = g.eb;
    db.planes = g.pb;
    DMP_CHECK(launch_split(da, slices, kind, nullptr, s));
    DMP_CHECK(launch_split(db, slices, kind, nullptr, s));

    const int tm = tile_rows(m), tn = tile_cols(n);
    k_fill_tiles<<<unsigned((tm * tn + 255) / 256), 256, 0, s>>>(g.tiles, tm, tn);
    DMP_CHECK_HIP(hipGetLastError());
    GemmParams p{};
    p.tiles = g.tiles;
    p.descs = nullptr;
    p.one.pa = g.pa;
    p.one.pb = g.pb;
    p.one.ea = g.ea;
    p.one.eb = g.eb;
    p.one.out = C;
    p.one.a_rb_stride = rb_stride;
    p.one.b_rb_stride = rb_stride;
    p.one.M = m;
    p.one.N = n;
    p.one.KC = KC;
    p.one.ldc = ldc;
    p.one.state_index = -1;
    p.mode = EPI_STORE;
    // whole tiles only (a split tail would need its part buffer sized from
    // an occupancy query)
    return launch_ozgemm(slices, kind, p, tm * tn, s);
}

}  // extern "C"
