// LDS-staged (3+1)D conserved-functional reductions (norm3.hip), without and
// with gauge links; launch_norm3 and launch_norm_links use them where they apply
// (any row length for complex128, even ones for complex64) and the unstaged
// reductions otherwise.
#pragma once

#include "internal.h"

namespace dirac {

bool norm3_staged_supported(int nx, bool fp32);
template <typename R> hipError_t launch_norm3_staged(const ReduceArgs<R> &a, hipStream_t s);
// the same with gauge links (periodic lattices; the same row-length condition)
template <typename R> hipError_t launch_norm3_links_staged(const ReduceArgs<R> &a, const LinkPtrs &L, hipStream_t s);

}  // namespace dirac
