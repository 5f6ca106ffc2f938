// Error reporting shared by every entry point.
#include <string>

#include "internal.h"

namespace bgk {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
int fail_static(int code, const char* msg) noexcept {
  try {
    g_last_error = msg;
  } catch (...) {
    g_last_error.clear();
  }
  return code;
}
const char* last_error_cstr() { return g_last_error.c_str(); }
}  // namespace bgk

extern "C" const char* bgk_last_error(void) { return bgk::last_error_cstr(); }
