// Internal helpers shared by the translation units of libmlbm.so.
#pragma once

#include <cstdarg>
#include <cstdint>

namespace mlbm {

// Records a failure for mlbm_last_error() on the calling thread and returns
// the code.
int fail(int code, const char *fmt, ...);

// Clears the calling thread's error message.
void clear_error();

}  // namespace mlbm
