// Non-temporal store of one complex value: for results that no workgroup of
// the same launch reads again, so that they do not push the inputs' neighbour
// values out of L2.  The store is ordinary in every other respect.
#pragma once

#include <hip/hip_runtime.h>

namespace dirac {

typedef float nts2f __attribute__((ext_vector_type(2)));
typedef double nts2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(float2 *p, float2 v) { __builtin_nontemporal_store(nts2f{v.x, v.y}, (nts2f *)p); }
__device__ __forceinline__ void st_nt(double2 *p, double2 v) { __builtin_nontemporal_store(nts2d{v.x, v.y}, (nts2d *)p); }

}  // namespace dirac
