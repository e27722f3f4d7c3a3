// Host helpers shared by the single-simulation runtime and the serving pool (internal).
#pragma once

#include "kernels.hpp"
#include "vplbm.h"

namespace vplbm {

// Record a message for vplbm_last_error() on this thread and return `code`.
int fail(int code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::vplbm::fail(VPLBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// Host log on stderr when the environment variable VPLBM_LOG is 1 or more (read at each call).
void host_log(const char *fmt, ...);

int elem_bytes(int storage);
int check_config(const vplbm_config *c);
int check_bodies(const vplbm_body *b, int n);
NodeParams node_params(const vplbm_config &c);

}  // namespace vplbm
