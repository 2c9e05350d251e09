// Host-side helpers shared by the C-ABI translation units (no device code).
#pragma once

#include <string>

#include "../../include/rmg.h"

namespace rmg {

// Store `msg` as the context's last error and return `code`.
int set_error(rmg_ctx* c, int code, const std::string& msg);
// HIP device the context was created on.
int device_of(const rmg_ctx* c);

}  // namespace rmg
