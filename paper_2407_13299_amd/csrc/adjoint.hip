// Adjoint of the purification sequence (placeholder until the reverse pass
// lands): every entry point reports DMP_EUNSUPPORTED.
#include "host.hpp"

using namespace dmp;

struct dmp_tape {
    int n;
};

extern "C" {

int dmp_purify_fwd_tape(const double*, int, int, double, int, dmp_kind, int, int, double*,
                        double*, dmp_info*, dmp_tape** tape, void*) {
    if (tape) *tape = nullptr;
    set_error("adjoint not built");
    return DMP_EUNSUPPORTED;
}

size_t dmp_purify_bwd_workspace_bytes(const dmp_tape*) { return 0; }

int dmp_purify_bwd(const dmp_tape*, const double*, double*, void*, size_t, void*) {
    set_error("adjoint not built");
    return DMP_EUNSUPPORTED;
}

int dmp_tape_info(const dmp_tape*, int* iters, int*) {
    if (iters) *iters = 0;
    return DMP_EUNSUPPORTED;
}

void dmp_tape_free(dmp_tape* t) { delete t; }

}  // extern "C"
