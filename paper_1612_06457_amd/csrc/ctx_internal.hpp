// Library-internal access to a context, for host modules outside api.cpp.
#pragma once
#include <string>

#include "cvamx.h"

namespace cvamx {
// Store msg as the context's last error and return code.
int set_error(cvamx_ctx* ctx, int code, const std::string& msg);
// The context's device (-1: none) and its compute-unit count.
int ctx_device(const cvamx_ctx* ctx);
}  // namespace cvamx
