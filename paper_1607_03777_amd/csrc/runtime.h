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
void ctx_combine_stats(sdg_ctx* c, int64_t* launches, int64_t* combined, int* max_width, int64_t* graphs);
// Device bytes of a batched problem whose element blocks are nuniq distinct
// matrices (sdg_required_bytes_batch counts every block as distinct), and
// the number of distinct blocks that deduplication leaves for nbatch
// problems with viscosities eta (host, nel values each).
size_t required_bytes_blocks(const sdg_mesh* mesh, const sdg_options* opts, int stokes, int nbatch, int64_t nuniq);
int64_t unique_blocks(const sdg_mesh& m, const double* eta, int nbatch, bool dedup);
}  // namespace sdg
