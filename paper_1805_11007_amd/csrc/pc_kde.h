// Agent-side form of the Gaussian kernel density deposit (Sect. 2.3).
#pragma once

#include <hip/hip_runtime.h>

#include "pc_internal.h"

namespace pc {

// sigma_l, upsilon_l of every node as in launch_kde, summed from the
// agents' side: each agent adds its kernel to the nodes of its ball, first
// in a per-work-group LDS table, then by device float atomics.  The order of
// the additions, and so the last bits of a sum, vary from run to run;
// launch_kde sums in a fixed order.
void launch_kde_scatter(const StepParams &p, const Buffers &b, int src, hipStream_t s);

}  // namespace pc
