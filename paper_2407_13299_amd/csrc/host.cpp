// Host-side helpers of libdmp that call HIP or rocBLAS: the device tile
// lists, rocBLAS handles and products, the occupancy cache.
#include "host.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <memory>

namespace dmp {

int cached_tiles(int tm, int tn, bool upper, const Tile** out, int TM) {
    // device copies live until the process ends (the cache has no limit)
    static KeyedCache<Tile> cache;
    int dev = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    int st = DMP_OK;
    auto v = cache.get_or_create({dev, tm, tn, upper ? 1 : 0, TM}, [&]() -> std::shared_ptr<Tile> {
        std::vector<Tile> host;
        append_tiles(host, tm, tn, upper, 0, TM);
        Tile* devp = nullptr;
        hipError_t e = hipMalloc(&devp, std::max<size_t>(1, host.size()) * sizeof(Tile));
        if (e == hipSuccess && !host.empty())
            e = hipMemcpy(devp, host.data(), host.size() * sizeof(Tile), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error("tile list upload failed: %s", hipGetErrorString(e));
            if (devp) (void)hipFree(devp);
            st = DMP_EHIP;
            return nullptr;
        }
        return std::shared_ptr<Tile>(devp, [](Tile*) {});   // kept for the process
    });
    if (!v) return st != DMP_OK ? st : DMP_EHIP;
    *out = v.get();
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

int resident_slots(int S, dmp_kind kind, int rb, int* slots) {
    int dev = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    // a property of the device and the kernel: queried once, then cached
    static KeyedCache<int> cache;
    int st = DMP_OK;
    auto v = cache.get_or_create({dev, S, int(kind), rb}, [&]() -> std::shared_ptr<int> {
        int q = 0;
        st = gemm_slots(S, kind, rb, &q);
        return st == DMP_OK ? std::make_shared<int>(q) : nullptr;
    });
    if (!v) return st != DMP_OK ? st : DMP_EHIP;
    *slots = *v;
    return DMP_OK;
}

bool tail_split_enabled() {
    const char* e = std::getenv("DMP_TAIL_SPLIT");
    return !(e && std::strcmp(e, "0") == 0);
}

int forced_tile_rb() {
    const char* e = std::getenv("DMP_TILE_ROWS");
    if (e && std::strcmp(e, "128") == 0) return 4;
    if (e && std::strcmp(e, "64") == 0) return 2;
    return 0;
}

TileChoice tile_choice_env(dmp_kind kind, int S, int n) {
    return tile_choice(kind, S, n, forced_tile_rb());
}

int tile_blocks_for(dmp_kind kind, int S, int n) { return tile_choice_env(kind, S, n).rb; }

}  // namespace dmp

extern "C" {

const char* dmp_last_error(void) { return dmp::error_text(); }

const char* dmp_version(void) { return "dmp 0.1 (gfx950)"; }

int dmp_max_slices(dmp_kind kind) {
    if (kind == DMP_MARKIDIS_FP16) return dmp::kMaxTerms;
    return (kind == DMP_OZ_INT8 || kind == DMP_OZ_FP16) ? dmp::kMaxSlices : 0;
}

}  // extern "C"
