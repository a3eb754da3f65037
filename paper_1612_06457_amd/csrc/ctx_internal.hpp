// Library-internal access to a context, for host modules outside api.cpp.
#pragma once
#include <string>

#include "cvamx.h"

namespace cvamx {
// Store msg as the context's last error and return code.
int set_error(cvamx_ctx* ctx, int code, const std::string& msg);
// The context's device (-1: none).
int ctx_device(const cvamx_ctx* ctx);
// Per-context state of a host module (the page batches): a pointer the
// module owns, freed through fn by cvamx_destroy once the device is idle.
void** ctx_module_state(cvamx_ctx* ctx);
void ctx_set_module_free(cvamx_ctx* ctx, void (*fn)(void*));
}  // namespace cvamx
