// Plan log on stderr (environment variable DT_LOG), host only.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dt.h"
#include "dt_log.hpp"

namespace dt {

bool log_enabled() {
  const char* v = std::getenv("DT_LOG");
  return v && *v && std::strcmp(v, "0") != 0;
}

void logf(const char* fmt, ...) {
  if (!log_enabled()) return;
  char line[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(line, sizeof(line), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[dt] %s\n", line);
  std::fflush(stderr);
}

const char* mask_names(unsigned mask, char* buf, int cap) {
  static const struct { unsigned bit; const char* name; } names[] = {
      {DT_OUT_S, "S"}, {DT_OUT_GRAD, "grad"}, {DT_OUT_HESS, "hess"},
      {DT_OUT_SIGN, "sign"}, {DT_OUT_BACKWARD, "backward"}, {DT_OUT_CURV, "curv"}};
  if (cap < 1) return buf;
  buf[0] = 0;
  int used = 0;
  for (const auto& n : names) {
    if (!(mask & n.bit)) continue;
    const int w = std::snprintf(buf + used, (size_t)(cap - used), "%s%s", used ? "|" : "", n.name);
    if (w < 0 || used + w >= cap) break;
    used += w;
  }
  return buf;
}

const char* precision_name(int precision) {
  switch (precision) {
    case DT_FP32_SCALED: return "fp32-scaled";
    case DT_FP64: return "fp64";
    case DT_FP64X2: return "fp64x2";
    case DT_FP64X4: return "fp64x4";
    default: return "auto";
  }
}

}  // namespace dt
