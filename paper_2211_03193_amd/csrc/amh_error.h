// amh_error.h -- the library's thread-local error message (read by amh_last_error).
#pragma once
#include "amh.h"

namespace amh {

// Record a printf-style message for amh_last_error() and return st.
amh_status sfail(amh_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace amh
