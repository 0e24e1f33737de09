// Thread-local error message behind lv_last_error().
#include <cstdarg>
#include <cstdio>
#include <string>

#include "lv_error.h"

namespace lv {
namespace {
thread_local std::string g_err;
}

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

void clear_error() { g_err.clear(); }

}  // namespace lv

extern "C" const char *lv_last_error(void) { return lv::g_err.c_str(); }

extern "C" int lv_version(void) { return 10000; }
