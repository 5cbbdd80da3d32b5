// LDS-staged (3+1)D conserved-functional reduction (norm3.hip); launch_norm3
// uses it where it applies (any row length for complex128, even ones for
// complex64) and the unstaged reduction otherwise.
#pragma once

#include "internal.h"

namespace dirac {

bool norm3_staged_supported(int nx, bool fp32);
template <typename R> hipError_t launch_norm3_staged(const ReduceArgs<R> &a, hipStream_t s);

}  // namespace dirac
