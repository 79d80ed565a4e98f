// Device-side types shared by the kernels and the runtime of the KKT library.
#pragma once

#include <cstdint>

#include "kkt_internal.h"

namespace kkt {

constexpr int kFlagNonfinite = 1;
constexpr int kFlagInternal = 2;    // a schedule invariant failed on the device
constexpr int kCountSlots = 1024;   // spread counter for replaced pivots

// Scalars written by the kernels and read back by the host.
struct DevStatus {
    double anorm_scaled;          // ||R A C||_inf of the last refactorization
    double anorm;                 // ||A||_inf of the last refactorization (same order)
    unsigned long long perturbed; // pivots replaced by the last refactorization
    int flags;                    // kFlagNonfinite
    int abort;                    // a persistent solve timed out waiting (sticky until refactor)
};

// Infinity norms of the last residual evaluation, read back by the host.
struct ResNorms {
    double rnorm, xnorm, bnorm;
};

}  // namespace kkt
