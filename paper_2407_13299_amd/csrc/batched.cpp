// Batched purification entry point and the slice-count table.
#include <algorithm>
#include <cmath>
#include <vector>

#include "host.hpp"

using namespace dmp;

extern "C" {

int dmp_autotune_slices(int n, double target, dmp_kind kind) {
    return autotune_slices_model(n, target, kind);
}

}  // extern "C"


extern "C" {

size_t dmp_purify_batched_workspace_bytes(int count, const int* n, int slices, dmp_kind kind) {
    if (count < 1 || !n) return 0;
    for (int b = 0; b < count; ++b)
        if (n[b] < 1) return 0;
    std::vector<int> s;
    batch_slices(count, n, slices, kind, s);
    std::vector<const double*> h(count, nullptr);
    std::vector<double*> p(count, nullptr);
    std::vector<int> nocc(count, 0);
    size_t need = 0;
    purify_many(count, h.data(), n, nocc.data(), 1.0, s.data(), kind, 1, DMP_CANONICAL, 0, p.data(), nullptr,
                nullptr, nullptr, 0, nullptr, &need);
    return need;
}

int dmp_purify_batched_ex(int count, const double* const* H, const int* n, const int* nocc,
                          double tol, int slices, dmp_kind kind, int max_iter, int method,
                          int flags, double* const* P, double* E, dmp_info* info, void* ws,
                          size_t ws_bytes, void* stream) {
    clear_error();
    DMP_CHECK(check_method_flags(method, flags));
    if (count < 1 || !H || !n || !nocc || !P || !E) {
        set_error("bad batch arguments");
        return DMP_EINVAL;
    }
    for (int b = 0; b < count; ++b)
        DMP_CHECK(validate_purify_args(H[b], n[b], nocc[b], tol, max_iter, P[b]));
    std::vector<int> s;
    batch_slices(count, n, slices, kind, s);
    for (int b = 0; b < count; ++b) {
        if (kind != DMP_FP64_NATIVE) {
            DMP_CHECK(check_kind_slices(kind, s[b]));
            if (n[b] > max_k_for(s[b], kind)) {
                set_error("matrix %d: n = %d exceeds the exact INT32 range for %d slices", b, n[b], s[b]);
                return DMP_EINVAL;
            }
        }
    }
    if (ws == nullptr) {
        set_error("workspace required");
        return DMP_ENOMEM;
    }
    return purify_many(count, H, n, nocc, tol, s.data(), kind, max_iter, method, flags, P, E, info,
                       ws, ws_bytes, static_cast<hipStream_t>(stream), nullptr);
}

int dmp_purify_batched(int count, const double* const* H, const int* n, const int* nocc,
                       double tol, int slices, dmp_kind kind, int max_iter, double* const* P,
                       double* E, dmp_info* info, void* ws, size_t ws_bytes, void* stream) {
    return dmp_purify_batched_ex(count, H, n, nocc, tol, slices, kind, max_iter, DMP_CANONICAL, 0,
                                 P, E, info, ws, ws_bytes, stream);
}

}  // extern "C"
