// Plan log: with the environment variable DT_LOG set to a nonzero value,
// plan creation, workspace attach (kernel norms, validity threshold) and
// dt_last_stats / dt_batch_stats print what the plan chose to stderr.
#pragma once

namespace dt {

// DT_LOG is read at each logging point (plan set-up and stats calls only).
bool log_enabled();
// One line on stderr, prefixed with "[dt] " (no-op when the log is off).
void logf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
// "S|grad|hess|..." for an output mask.
const char* mask_names(unsigned mask, char* buf, int cap);
// "fp32-scaled", "fp64", "fp64x2"
const char* precision_name(int precision);

}  // namespace dt
