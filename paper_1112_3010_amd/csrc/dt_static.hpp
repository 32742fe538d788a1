// Host-side hooks between the plan code and the library's fixed workspace
// array (k_static_ws.hip).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "dt.h"

namespace dt {
// Attach a workspace to a plan and build its tables (dt_plan_set_workspace).
dt_status plan_attach(dt_plan p, void* dev_ptr, size_t bytes, void* stream);
// Record that the plan's workspace is the fixed array of `dev`, held under `token`.
void plan_mark_static(dt_plan p, int dev, uint64_t token);
// Token of the plan whose tables the fixed array of `dev` holds (0: none).
uint64_t static_ws_owner(int dev);
// Give up the array of `dev` if `token` still holds it.
void static_ws_release(int dev, uint64_t token);
}  // namespace dt
