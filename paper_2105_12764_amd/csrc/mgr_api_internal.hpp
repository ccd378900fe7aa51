// mgr_api_internal.hpp -- library-internal calls between the C ABI's
// translation units (not exported in include/mgr.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "../../include/mgr.h"

namespace mgr {

// Finds or builds the cached plan of a request (shape, coordinates, level
// count) on the current device, so that a later call with these arguments
// enqueues without building one.  Validates like mgr_decompose; the detail
// of an error is in mgr_last_error().
mgr_status prepare_plan(int ndim, const int64_t *shape, const double *const *coords, int nlevels);

// Destroys the recomposition helper streams registered for these caller
// streams on the current device (after waiting for their work), so that a
// caller that destroys its streams frees their registry entries.  The caller
// guarantees that no libmgr call on those streams is in progress.
void forget_helpers(const hipStream_t *callers, int n);

}  // namespace mgr
