// Host-side helpers shared by the library's translation units: the
// thread-local error text behind hpc_last_error() and the HIP call check.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hpclust.h"

namespace hpc_host {

// Record an error message (printf format) and return `code`.
int fail(int code, const char* fmt, ...);

}  // namespace hpc_host

#define HPC_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return hpc_host::fail(HPC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)
