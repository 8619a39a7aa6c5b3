// errors.hpp -- thread-local error text behind fft_last_error().
#pragma once

#include <string>

#include "decomp.hpp"

namespace fftrw {

extern thread_local std::string g_last_error;

// Record `msg` as the calling thread's last error and return `code`.
int fail(int code, const std::string &msg);
int fail(const Status &s);

// Diagnostics on stderr, chosen by the environment variable FFTRW_LOG (read
// once): 0 or unset = none, 1 = errors and plans, 2 = also order searches,
// 3 = also every execution.  Lines start with "fftrw: ".
int log_level();
void log_line(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace fftrw
