// Slice-count error model used by dmp_autotune_slices:
//   max|dP| ~ kTunedErrC[kind] * n^kTunedErrA[kind] * 2^-(8S - 1)
// (index 0: INT8, 1: FP16; both kinds give bit-identical products),
// and the default accuracy target of the batched entry point when it
// picks S itself.  Written by paper_2407_13299_amd/autotune.py from
// these measurements (spectrum-controlled H, half filled, gap 0.2 Ha,
// max |P_S - P_11|):
//   n =   128  S =  4  9.379e-07  stagnated
//   n =   128  S =  5  1.692e-09  stagnated
//   n =   128  S =  6  1.583e-11  converged
//   n =   128  S =  7  4.249e-14  converged
//   n =   128  S =  8  1.443e-15  converged
//   n =   256  S =  4  1.756e-06  stagnated
//   n =   256  S =  5  3.462e-09  stagnated
//   n =   256  S =  6  3.277e-11  converged
//   n =   256  S =  7  6.532e-14  converged
//   n =   256  S =  8  2.442e-15  converged
//   n =   512  S =  4  4.639e-06  stagnated
//   n =   512  S =  5  6.385e-09  stagnated
//   n =   512  S =  6  7.854e-11  stagnated
//   n =   512  S =  7  1.242e-13  converged
//   n =   512  S =  8  4.996e-15  converged
//   n =  1024  S =  4  1.407e-05  stagnated
//   n =  1024  S =  5  1.346e-08  stagnated
//   n =  1024  S =  6  1.887e-10  converged
//   n =  1024  S =  7  2.507e-13  converged
//   n =  1024  S =  8  1.321e-14  converged
//   n =  1536  S =  4  2.810e-05  max_iter
//   n =  1536  S =  5  1.789e-08  stagnated
//   n =  1536  S =  6  3.269e-10  stagnated
//   n =  1536  S =  7  3.986e-13  converged
//   n =  1536  S =  8  8.327e-15  converged
//   n =  2048  S =  4  3.866e-05  stagnated
//   n =  2048  S =  5  2.584e-08  stagnated
//   n =  2048  S =  6  4.666e-10  stagnated
//   n =  2048  S =  7  5.106e-13  converged
//   n =  2048  S =  8  1.110e-14  converged
//   n =  3072  S =  4  6.796e-05  stagnated
//   n =  3072  S =  5  3.428e-08  stagnated
//   n =  3072  S =  6  8.160e-10  converged
//   n =  3072  S =  7  7.632e-13  converged
//   n =  3072  S =  8  1.832e-14  converged
#pragma once
namespace dmp {
constexpr double kTunedErrC[2] = {26.1775, 26.1775};
constexpr double kTunedErrA[2] = {1.21846, 1.21846};
constexpr double kTunedTarget = 1e-10;
}  // namespace dmp
