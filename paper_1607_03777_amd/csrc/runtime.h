// Internal declarations shared by the host runtime files.
#pragma once

#include "sdg_common.h"

namespace sdg {
int ctx_device(const sdg_ctx* c);
// Device memory through the context's block cache: ctx_alloc returns null
// on failure; ctx_release takes the same byte count, and no queued work may
// still use the block.
void* ctx_alloc(sdg_ctx* c, size_t bytes);
void ctx_release(sdg_ctx* c, void* p, size_t bytes);
// combined launches of the CG iterations of concurrent solves (the request
// server turns them on while it runs; off only when no solve is running)
int ctx_combine(sdg_ctx* c, int on);
void ctx_combine_stats(sdg_ctx* c, int64_t* launches, int64_t* combined, int* max_width);
}  // namespace sdg
