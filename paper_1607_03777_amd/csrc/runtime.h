// Internal declarations shared by the host runtime files.
#pragma once

#include "sdg_common.h"

namespace sdg {
int ctx_device(const sdg_ctx* c);
}  // namespace sdg
