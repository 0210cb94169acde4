// The library context (host memory only) and the error-reporting helpers
// shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include "dqo.h"

struct dqo_ctx {
    dqo_config cfg;
    mutable char err[512];
};

namespace dqo {

inline int fail(const dqo_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

inline int hip_fail(const dqo_ctx* c, hipError_t e, const char* where) {
    return fail(c, DQO_EHIP, "%s: %s", where, hipGetErrorString(e));
}

}  // namespace dqo
