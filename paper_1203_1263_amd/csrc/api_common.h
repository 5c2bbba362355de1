// Error reporting shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

// Store a formatted thread-local message (nlse_last_error) and return code.
int nlse_fail(int code, const char* fmt, ...);
// NLSE_EDEVICE with the HIP error text.
int nlse_hip_fail(hipError_t e, const char* what);
// Autotuner cache ($NLSE_TUNE_CACHE, one "key|v1 .. vn ms" line per entry
// with n integers; the last entry of a key wins).  Lookup returns false
// without the variable or without an entry of n values.
bool nlse_cache_lookup(const std::string& key, int* t, int n);
void nlse_cache_store(const std::string& key, const int* t, int n, float ms);
