// Error reporting shared by every translation unit (no HIP dependency).
#pragma once

#include <string>

#include "../../include/leanvec.h"

namespace lv {

void set_error(const char *fmt, ...);
void clear_error();

}  // namespace lv

#define LV_FAIL(code, ...)        \
  do {                            \
    ::lv::set_error(__VA_ARGS__); \
    return (code);                \
  } while (0)
