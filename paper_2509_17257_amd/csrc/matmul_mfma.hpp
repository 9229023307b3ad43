// Matrix-core (MFMA) coupling kernel for the FP64 operator.
#pragma once

#include "device.hpp"

namespace h2x {

// Launches the matrix-core coupling stage when the operator's layout supports
// it; returns false (launching nothing) otherwise.
template <typename T, typename Acc>
bool launch_coupling_fast(const DevMat &, int64_t, const Acc *, Acc *, int64_t, hipStream_t) {
    return false;
}

}  // namespace h2x
