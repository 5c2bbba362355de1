// Error reporting shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

// Store a formatted thread-local message (nlse_last_error) and return code.
int nlse_fail(int code, const char* fmt, ...);
// NLSE_EDEVICE with the HIP error text.
int nlse_hip_fail(hipError_t e, const char* what);
