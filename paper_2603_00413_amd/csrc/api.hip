// Error reporting of the C ABI (thread-local last-error message).
#include <stdarg.h>
#include <stdio.h>

#include "dt_internal.h"

namespace {
thread_local char g_err[512] = "";
}

void dt_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

extern "C" const char* dt_last_error(void) { return g_err; }

extern "C" const char* dt_status_string(dt_status s) {
  switch (s) {
    case DT_OK: return "ok";
    case DT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case DT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case DT_ERR_CAPACITY: return "ray queue capacity exceeded";
    case DT_ERR_HIP: return "HIP runtime error";
    case DT_ERR_UNSUPPORTED: return "unsupported";
    case DT_ERR_NOT_CONVERGED: return "not converged";
    default: return "unknown status";
  }
}
