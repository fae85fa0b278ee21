// Device-side plan builder (HIP kernels for the bounding cube, Morton sort,
// Ncrit tree, dual tree traversal, best directions and marks).  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace defmm {

// Fills hp from device coordinates X (nx x 3) and Y (ny x 3; ignored when
// prm.same_points), running on stream s; the operator tables are packed on
// the host at the end.  Returns false if a coordinate is not finite; throws
// std::runtime_error / std::bad_alloc on device errors.
bool build_device_plan(HostPlan& hp, const double* X, int64_t nx, const double* Y, int64_t ny,
                       const BuildParams& prm, hipStream_t s);

}  // namespace defmm
