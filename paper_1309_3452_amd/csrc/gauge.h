// (2+1)D link step in one launch (gauge.hip), declared apart from the shared
// host declarations.
#pragma once

#include "internal.h"

namespace dirac {

// One step per launch with links, y-march over x strips, ping-pong in -> out.
template <typename R> hipError_t launch_fused2_links(const FusedArgs<R> &a, const LinkPtrs &L, bool site,
                                                     hipStream_t s);

}  // namespace dirac
