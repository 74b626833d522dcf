// Host-side helpers of libdmp: error text, tile orders, rocBLAS handles.
#include "host.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

namespace dmp {

static thread_local char g_error[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

static bool tile_in_upper(int i, int j, int TM) { return kTileN * j + kTileN - 1 >= TM * i; }

void append_tiles(std::vector<Tile>& out, int tm, int tn, bool upper, uint32_t mat, int TM) {
    // super-tiles of GI x GJ tiles = 512 x 512 elements
    const int GI = 512 / TM, GJ = 512 / kTileN;
    const int sm = (tm + GI - 1) / GI, sn = (tn + GJ - 1) / GJ;
    for (int si = 0; si < sm; ++si)
        for (int sj = 0; sj < sn; ++sj)
            for (int i = si * GI; i < std::min(tm, si * GI + GI); ++i)
                for (int j = sj * GJ; j < std::min(tn, sj * GJ + GJ); ++j) {
                    if (upper && !tile_in_upper(i, j, TM)) continue;
                    out.push_back(Tile{uint16_t(i), uint16_t(j), mat});
                }
}

int tile_rows(int m, int TM) { return int(round_up(m, TM) / TM); }
int tile_cols(int n) { return int(round_up(n, kTileN) / kTileN); }

int upper_tile_count(int n, int TM) {
    const int tm = tile_rows(n, TM), tn = tile_cols(n);
    int c = 0;
    for (int i = 0; i < tm; ++i)
        for (int j = 0; j < tn; ++j) c += tile_in_upper(i, j, TM) ? 1 : 0;
    return c;
}

int cached_tiles(int tm, int tn, bool upper, const Tile** out, int TM) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, bool, int>, Tile*> cache;
    int dev = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, tm, tn, upper, TM);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return DMP_OK;
    }
    std::vector<Tile> host;
    append_tiles(host, tm, tn, upper, 0, TM);
    Tile* devp = nullptr;
    DMP_CHECK_HIP(hipMalloc(&devp, std::max<size_t>(1, host.size()) * sizeof(Tile)));
    if (!host.empty())
        DMP_CHECK_HIP(hipMemcpy(devp, host.data(), host.size() * sizeof(Tile), hipMemcpyHostToDevice));
    cache[key] = devp;
    *out = devp;
    return DMP_OK;
}

// One rocBLAS handle per device and host thread: a handle carries its stream,
// so threads that share one would race between setting the stream and the
// call.  Handles live until the process ends.
int blas_handle(hipStream_t stream, rocblas_handle* out) {
    static thread_local std::map<int, rocblas_handle> handles;
    int dev = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    auto it = handles.find(dev);
    rocblas_handle h;
    if (it == handles.end()) {
        if (rocblas_create_handle(&h) != rocblas_status_success) {
            set_error("rocblas_create_handle failed");
            return DMP_EHIP;
        }
        handles[dev] = h;
    } else {
        h = it->second;
    }
    if (rocblas_set_stream(h, stream) != rocblas_status_success) {
        set_error("rocblas_set_stream failed");
        return DMP_EHIP;
    }
    *out = h;
    return DMP_OK;
}

// Row-major C = op(A) op(B) through column-major rocBLAS: the row-major
// matrices are the transposes of the column-major views, so compute
// C^T = op(B)^T op(A)^T.
int native_dgemm(hipStream_t stream, bool ta, bool tb, int m, int n, int k, const double* A,
                 int lda, const double* B, int ldb, double* C, int ldc) {
    rocblas_handle h;
    DMP_CHECK(blas_handle(stream, &h));
    const double one = 1.0, zero = 0.0;
    rocblas_status s = rocblas_dgemm(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                                     ta ? rocblas_operation_transpose : rocblas_operation_none, n,
                                     m, k, &one, B, ldb, A, lda, &zero, C, ldc);
    if (s != rocblas_status_success) {
        set_error("rocblas_dgemm failed (%d)", int(s));
        return DMP_EHIP;
    }
    return DMP_OK;
}

// Upper triangle (row-major) of symmetric products: rocBLAS is column-major,
// so the row-major upper triangle is its lower one.  C = A A (A symmetric).
int native_dsyrk_upper(hipStream_t stream, int n, const double* A, double* C) {
    rocblas_handle h;
    DMP_CHECK(blas_handle(stream, &h));
    const double one = 1.0, zero = 0.0;
    rocblas_status s = rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, n, n, &one, A,
                                     n, &zero, C, n);
    if (s != rocblas_status_success) {
        set_error("rocblas_dsyrk failed (%d)", int(s));
        return DMP_EHIP;
    }
    return DMP_OK;
}

// C = A B for symmetric A, B whose product is symmetric (they commute): the
// upper triangle by rocBLAS dsyrkx (A B^T = A B).
int native_dsyrkx_upper(hipStream_t stream, int n, const double* A, const double* B, double* C) {
    rocblas_handle h;
    DMP_CHECK(blas_handle(stream, &h));
    const double one = 1.0, zero = 0.0;
    rocblas_status s = rocblas_dsyrkx(h, rocblas_fill_lower, rocblas_operation_none, n, n, &one,
                                      A, n, B, n, &zero, C, n);
    if (s != rocblas_status_success) {
        set_error("rocblas_dsyrkx failed (%d)", int(s));
        return DMP_EHIP;
    }
    return DMP_OK;
}

int check_kind_slices(dmp_kind kind, int slices) {
    if (kind != DMP_OZ_INT8 && kind != DMP_OZ_FP16 && kind != DMP_FP64_NATIVE &&
        kind != DMP_MARKIDIS_FP16) {
        set_error("unknown kind %d", int(kind));
        return DMP_EINVAL;
    }
    if (kind == DMP_MARKIDIS_FP16 && (slices < 1 || slices > kMaxTerms)) {
        set_error("terms must lie in [1, %d], got %d", kMaxTerms, slices);
        return DMP_EINVAL;
    }
    if (kind != DMP_FP64_NATIVE && kind != DMP_MARKIDIS_FP16 && (slices < 1 || slices > kMaxSlices)) {
        set_error("slices must lie in [1, %d], got %d", kMaxSlices, slices);
        return DMP_EINVAL;
    }
    return DMP_OK;
}

int resident_slots(int S, dmp_kind kind, int rb, int* slots) {
    int dev = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    // a property of the device and the kernel: queried once, then cached
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    const auto key = std::make_tuple(dev, S, int(kind), rb);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *slots = it->second;
            return DMP_OK;
        }
    }
    DMP_CHECK(gemm_slots(S, kind, rb, slots));
    std::lock_guard<std::mutex> lock(mu);
    cache[key] = *slots;
    return DMP_OK;
}

static int split_parts_max(int min_kc) { return std::min(kMaxSplit, min_kc / kMinSplitChunks); }

TailSplit plan_tail_split(int ntiles, int slots, int min_kc, int max_pieces) {
    TailSplit t{ntiles, 1};
    // with no full round the fixup launch costs more than the parts save
    if (ntiles <= slots || slots <= 0) return t;
    const int r = ntiles % slots;
    if (r == 0) return t;
    const int parts = std::min({split_parts_max(min_kc), slots / r, max_pieces / r});
    if (parts < 2) return t;
    t.nfull = ntiles - r;
    t.nsplit = parts;
    return t;
}

int tail_split_capacity(int ntiles, int min_kc, int rb) {
    const int parts = split_parts_max(min_kc);
    if (parts < 2 || ntiles <= 0) return 0;
    // 128-row tiles: one workgroup per CU, so half the parts run at once
    const int cap = rb == 4 ? kMaxPieces / 2 : kMaxPieces;
    return int(std::min<int64_t>(cap, int64_t(ntiles) * parts));
}

int64_t chunks_of(int k, dmp_kind kind) { return round_up(k, kKPad) / chunk_k(kind); }

}  // namespace dmp

extern "C" {

const char* dmp_last_error(void) { return dmp::g_error; }

const char* dmp_version(void) { return "dmp 0.1 (gfx950)"; }

int dmp_max_slices(dmp_kind kind) {
    if (kind == DMP_MARKIDIS_FP16) return dmp::kMaxTerms;
    return (kind == DMP_OZ_INT8 || kind == DMP_OZ_FP16) ? dmp::kMaxSlices : 0;
}

}  // extern "C"
