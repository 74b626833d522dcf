// Batched purification entry point and the slice-count table.
#include <algorithm>
#include <cmath>
#include <vector>

#include "host.hpp"
#include "tuned_table.h"

using namespace dmp;

extern "C" {

int dmp_autotune_slices(int n, double target, dmp_kind kind) {
    if (kind == DMP_FP64_NATIVE) return 0;
    if (kind == DMP_MARKIDIS_FP16) return kMaxTerms;   // no term count reaches FP64 level
    if (n < 1 || !(target > 0.0)) return kMaxSlices;
    // error model max|dP| ~ C n^a 2^-(8S - 1), with (C, a) measured per kind
    const double c = kind == DMP_OZ_FP16 ? kTunedErrC[1] : kTunedErrC[0];
    const double a = kind == DMP_OZ_FP16 ? kTunedErrA[1] : kTunedErrA[0];
    for (int s = 1; s <= kMaxSlices; ++s) {
        const double err = c * std::pow(double(n), a) * std::ldexp(1.0, -(8 * s - 1));
        if (err <= target && n <= max_k_for_slices(s)) return s;
    }
    return kMaxSlices;
}

}  // extern "C"

namespace {

// Slice count per matrix of a batch.  slices > 0: that count for every
// matrix.  Otherwise the tuned table's count per matrix; matrices that need
// fewer slices than the batch maximum then run with the maximum (a larger S
// is always at least as accurate) when they carry under a quarter of the
// batch's n^3 work, so that the batch runs as one group of launches instead
// of one group per slice count.
void batch_slices(int count, const int* n, int slices, dmp_kind kind, std::vector<int>& s) {
    s.assign(count, 0);
    if (kind == DMP_FP64_NATIVE) return;
    int smax = 0;
    for (int b = 0; b < count; ++b) {
        s[b] = slices > 0 ? slices : dmp_autotune_slices(n[b], kTunedTarget, kind);
        smax = std::max(smax, s[b]);
    }
    if (slices > 0 || count < 2) return;
    double low = 0.0, all = 0.0;
    for (int b = 0; b < count; ++b) {
        const double w = double(n[b]) * n[b] * n[b];
        all += w;
        if (s[b] < smax) low += w;
    }
    if (low >= 0.25 * all) return;
    for (int b = 0; b < count; ++b)
        if (n[b] <= max_k_for(smax, kind)) s[b] = smax;
}

}  // namespace

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
