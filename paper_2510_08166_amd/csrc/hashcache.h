// The paper's hash-map block cache (JPT_CACHE_HASH), internal entry points
// used by jpt_mark_blocks, jpt_resolve and jpt_cache_reset.
#pragma once
#include <hip/hip_runtime.h>

#include "jpt.h"

bool hash_cache_ok(const jpt_cache *c);
jpt_status hash_cache_reset(jpt_cache *cache, hipStream_t st);
jpt_status hash_mark_frame(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                           jpt_frame *frame, jpt_cache *cache, hipStream_t st);
jpt_status hash_resolve(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                        const jpt_cache *cache, hipStream_t st);
