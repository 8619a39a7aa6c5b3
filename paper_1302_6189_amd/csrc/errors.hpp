// errors.hpp -- thread-local error text behind fft_last_error().
#pragma once

#include <string>

#include "decomp.hpp"

namespace fftrw {

extern thread_local std::string g_last_error;

// Record `msg` as the calling thread's last error and return `code`.
int fail(int code, const std::string &msg);
int fail(const Status &s);

}  // namespace fftrw
