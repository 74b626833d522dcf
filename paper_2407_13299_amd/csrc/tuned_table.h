// Slice-count error model used by dmp_autotune_slices:
//   max|dP| ~ kTunedErrC[kind] * n^kTunedErrA[kind] * 2^-(8S - 1)
// (index 0: INT8, 1: FP16), and the default accuracy target of the batched
// entry point when it picks S itself.
#pragma once
namespace dmp {
constexpr double kTunedErrC[2] = {40.0, 40.0};
constexpr double kTunedErrA[2] = {1.0, 1.0};
constexpr double kTunedTarget = 1e-10;
}  // namespace dmp
