// Thread-local error reporting shared by every C-ABI entry point.
#pragma once
#include <cstdarg>
#include <cstdint>

namespace camelot {
// Records a formatted message for camelot_last_error() and returns `code`.
int32_t fail(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
}  // namespace camelot
