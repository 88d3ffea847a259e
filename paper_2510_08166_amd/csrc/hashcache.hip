// The paper's Texture Block Cache, as the paper builds it (Method: Texture
// Block Cache, Mark, Update Cache, Resolve; Multiple Textures and Mip
// Mapping): a hash map from a 32-bit key -- 16 bits of block index inside
// the level, 13 bits of texture id, 3 bits of mip level -- to a slot of
// decoded texels.  Mark inserts every footprint block with atomicCAS (open
// addressing, linear probing); the thread that inserts a new key appends its
// bucket to the decode queue (insertion order), a key already present gets
// its visibility flag.  The queue becomes the decoder's work list and takes
// free slots.  Resolve finds every tap's slot by probing the map.  Update
// Cache evicts every block the frame does not read: after mark, before the
// new blocks take slots, the entries without the visibility flag free their
// slots (their keys stay, slotless, so that no probe chain breaks); the
// next frame starts from a map rebuilt from the kept entries (recorded per
// slot in `owner`).
//
// Limits of the key (those of the paper): at most 65,536 blocks per level
// (4096^2 texels), 8,191 textures, 8 levels per texture, 4:2:0 levels only
// (one MCU per block).  A pixel outside them raises JPT_ERR_PIXEL.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "hashcache.h"

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kVis = 0x80000000u;     // in a bucket's value: read this frame
constexpr uint32_t kSlotMask = 0x7FFFFFFFu;
constexpr int kThreads = 256;
constexpr int kTileW = 64, kTileH = 16;

__device__ __forceinline__ uint32_t bucket_of(uint32_t key, uint32_t mask) {
    return (key * 2654435761u) & mask;  // multiplicative hashing, table of mask + 1 buckets
}

// The key of block (bx, by) of footprint F of texture `tex` (level index
// F.level, the texture's first level `first`); kEmpty if it does not fit.
__device__ __forceinline__ uint32_t block_key(const LevelFoot &F, uint32_t tex, uint32_t first, uint32_t bx,
                                              uint32_t by) {
    const uint32_t lvl = F.level - first, idx = by * F.blk_cols + bx;
    const bool fits = lvl < 8u && tex < 8191u && idx < 65536u;
    return fits ? (idx << 16) | (tex << 3) | lvl : kEmpty;
}

// Slot of a key, or JPT_SLOT_NONE (probing stops at an empty bucket).
__device__ __forceinline__ uint32_t lookup(const uint32_t *__restrict__ hash, uint32_t mask, uint32_t key) {
    if (key == kEmpty) return JPT_SLOT_NONE;
    uint32_t h = bucket_of(key, mask);
    for (uint32_t p = 0; p <= mask; p++) {
        const uint32_t k = hash[2 * h];
        if (k == key) {
            const uint32_t v = hash[2 * h + 1] & kSlotMask;  // (all ones: queued without a slot)
            return v == kSlotMask ? JPT_SLOT_NONE : v;
        }
        if (k == kEmpty) return JPT_SLOT_NONE;
        h = (h + 1) & mask;
    }
    return JPT_SLOT_NONE;
}

// ------------------------------------------------------------ update cache
__global__ __launch_bounds__(kThreads) void k_hash_begin(uint32_t *__restrict__ meta, uint32_t *__restrict__ counters) {
    if (threadIdx.x < JPT_N_COUNTERS) counters[threadIdx.x] = threadIdx.x == JPT_CTR_ERROR_ITEM ? 0xFFFFFFFFu : 0u;
    if (threadIdx.x == 0) {
        meta[JPT_META_EVICTED] = 0;
        meta[JPT_META_QCOUNT] = 0;
        meta[JPT_META_VISIBLE] = 0;
    }
}

// Empty the map (its kept entries are in owner[]).
__global__ __launch_bounds__(kThreads) void k_hash_clear(uint32_t *__restrict__ hash, uint32_t n_buckets) {
    for (uint32_t h = blockIdx.x * kThreads + threadIdx.x; h < n_buckets; h += gridDim.x * kThreads) {
        hash[2 * h] = kEmpty;
        hash[2 * h + 1] = 0;
    }
}

// Update Cache, after mark: every entry this frame does not read gives its
// slot back to the free stack (before the new blocks take slots); its key
// stays in the map without a slot, so no probe chain breaks.
__global__ __launch_bounds__(kThreads) void k_hash_evict(uint32_t *__restrict__ hash, uint32_t n_buckets,
                                                         uint32_t *__restrict__ owner,
                                                         uint32_t *__restrict__ free_stack, uint32_t n_slots,
                                                         uint32_t *__restrict__ meta) {
    for (uint32_t h = blockIdx.x * kThreads + threadIdx.x; h < n_buckets; h += gridDim.x * kThreads) {
        const uint32_t key = hash[2 * h], val = hash[2 * h + 1];
        const uint32_t slot = val & kSlotMask;
        // (an entry queued without a slot is visible, so never evicted)
        if (key != kEmpty && !(val & kVis) && slot < n_slots) {
            owner[slot] = JPT_SLOT_NONE;
            free_stack[atomicAdd(meta + JPT_META_TOP, 1u)] = slot;
            atomicAdd(meta + JPT_META_EVICTED, 1u);
            hash[2 * h + 1] = kSlotMask;
        }
    }
}

// Put the kept entries back, not yet read this frame.
__global__ __launch_bounds__(kThreads) void k_hash_reinsert(uint32_t *__restrict__ hash, uint32_t mask,
                                                            const uint32_t *__restrict__ owner, uint32_t n_slots,
                                                            uint32_t *__restrict__ counters) {
    for (uint32_t s = blockIdx.x * kThreads + threadIdx.x; s < n_slots; s += gridDim.x * kThreads) {
        const uint32_t key = owner[s];
        if (key == JPT_SLOT_NONE) continue;
        uint32_t h = bucket_of(key, mask);
        bool done = false;
        for (uint32_t p = 0; p <= mask && !done; p++) {
            if (atomicCAS(hash + 2 * h, kEmpty, key) == kEmpty) {
                hash[2 * h + 1] = s;
                done = true;
            }
            h = (h + 1) & mask;
        }
        if (!done) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
    }
}

// ------------------------------------------------------------------- mark
// Insert a key; a new one appends its bucket to the queue.  A key counts
// as visible once per frame: the thread whose atomicOr sets its flag.
__device__ __forceinline__ void insert(uint32_t *__restrict__ hash, uint32_t mask, uint32_t key,
                                       uint32_t *__restrict__ queue, uint32_t max_items, uint32_t *__restrict__ meta,
                                       uint32_t *__restrict__ counters) {
    uint32_t h = bucket_of(key, mask);
    for (uint32_t p = 0; p <= mask; p++) {
        const uint32_t k = atomicCAS(hash + 2 * h, kEmpty, key);
        if (k == kEmpty) {
            // visible, no slot until the queue gives one; a thread that found
            // the key between the CAS and this may have set the flag first,
            // and only the one that sets it counts the block
            if (!(atomicOr(hash + 2 * h + 1, kVis | kSlotMask) & kVis)) atomicAdd(meta + JPT_META_VISIBLE, 1u);
            const uint32_t q = atomicAdd(meta + JPT_META_QCOUNT, 1u);
            if (q < max_items) queue[q] = h;
            return;
        }
        if (k == key) {
            if (!(atomicOr(hash + 2 * h + 1, kVis) & kVis)) atomicAdd(meta + JPT_META_VISIBLE, 1u);
            return;
        }
        h = (h + 1) & mask;
    }
    atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
}

// The keys of one pixel's footprint under filter kFilter (kEmpty for unused
// taps and levels of zero weight); `bad` for a pixel outside the key's limits.
template <uint32_t kFilter>
__device__ __forceinline__ int pixel_keys(const jpt_level_desc *__restrict__ levels,
                                          const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                          const jpt_gpixel &px, bool no_mip, uint32_t *keys, LevelFoot foot[2],
                                          int &nf, uint32_t &tw, bool &bad) {
    constexpr int kK = kFilter == JPT_FILTER_NEAREST ? 1 : (kFilter == JPT_FILTER_TRILINEAR ? 8 : 4);
#pragma unroll
    for (int k = 0; k < kK; k++) keys[k] = kEmpty;
    const int st = pixel_footprint(GlobalDesc{levels, texs}, n_tex, px, kFilter, foot, nf, tw, no_mip);
    bad = st == PIX_INVALID;
    if (st != PIX_VALID) return st;
    const uint32_t first = texs[px.tex].first_level;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (k >= nf || foot[k].lw == 0) continue;
        const LevelFoot &F = foot[k];
        bad |= levels[F.level].sampling != JPT_SAMPLING_420;
        if (kFilter == JPT_FILTER_NEAREST) {
            keys[0] = block_key(F, px.tex, first, F.x0 >> 4, F.y0 >> 4);
            bad |= keys[0] == kEmpty;
        } else {
            const uint32_t wx[2] = {256 - F.fx, F.fx}, wy[2] = {256 - F.fy, F.fy};
            const uint32_t xs[2] = {F.x0, F.x1}, ys[2] = {F.y0, F.y1};
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int a = 0; a < 2; a++) {
                    if (wx[a] * wy[b] == 0) continue;
                    const uint32_t key = block_key(F, px.tex, first, xs[a] >> 4, ys[b] >> 4);
                    bad |= key == kEmpty;
                    keys[4 * k + 2 * b + a] = key;
                }
        }
    }
    return st;
}

// A workgroup's LDS set of the distinct keys its pixel tile reads (open
// addressing, linear probing); false when the key finds no room.
constexpr int kTileSet = 1024, kTileProbes = 16;
__device__ __forceinline__ bool tile_set_insert(uint32_t *s_keys, uint32_t key) {
    uint32_t h = (key * 2654435761u) >> 22;  // 10 bits
#pragma unroll 1
    for (int p = 0; p < kTileProbes; p++) {
        const uint32_t old = atomicCAS(s_keys + h, kEmpty, key);
        if (old == kEmpty || old == key) return true;
        h = (h + 1) & (kTileSet - 1);
    }
    return false;
}
// The LDS set's entry of a key, or -1.
__device__ __forceinline__ int tile_set_find(const uint32_t *s_keys, uint32_t key) {
    uint32_t h = (key * 2654435761u) >> 22;
#pragma unroll 1
    for (int p = 0; p < kTileProbes; p++) {
        const uint32_t k = s_keys[h];
        if (k == key) return (int)h;
        if (k == kEmpty) return -1;
        h = (h + 1) & (kTileSet - 1);
    }
    return -1;
}

// Mark: the paper inserts every pixel's keys into the map with atomicCAS.
// Here a workgroup first gathers the distinct keys of its 64 x 16 pixel tile
// in LDS (the wave drops the keys its left neighbour, the previous pixel of
// the row, also holds), then inserts each once; the map, its flags and the
// queue's contents are the same, only the redundant global atomics go.  A
// key that finds no room in the LDS set goes to the map directly.
template <uint32_t kFilter>
__global__ __launch_bounds__(kThreads) void k_hash_mark(const jpt_level_desc *__restrict__ levels,
                                                        const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                        const jpt_gpixel *__restrict__ gbuf, uint32_t W, uint32_t H,
                                                        uint32_t pitch, bool no_mip, uint32_t *__restrict__ hash,
                                                        uint32_t mask, uint32_t *__restrict__ queue,
                                                        uint32_t max_items, uint32_t *__restrict__ meta,
                                                        uint32_t *__restrict__ counters) {
    constexpr int kK = kFilter == JPT_FILTER_NEAREST ? 1 : (kFilter == JPT_FILTER_TRILINEAR ? 8 : 4);
    __shared__ uint32_t s_keys[kTileSet];
    __shared__ uint32_t s_bad;
    for (int i = threadIdx.x; i < kTileSet; i += kThreads) s_keys[i] = kEmpty;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t x = blockIdx.x * kTileW + lane;
    const uint32_t y = blockIdx.y * kTileH + (threadIdx.x >> 6);
    bool any_bad = false;
    for (uint32_t yy = y; yy < min(H, blockIdx.y * kTileH + kTileH); yy += kThreads / 64) {
        const jpt_gpixel px = x < W ? gbuf[(size_t)yy * pitch + x] : jpt_gpixel{0.f, 0.f, JPT_TEX_BACKGROUND, 0.f};
        uint32_t keys[kK];
        LevelFoot foot[2];
        int nf;
        uint32_t tw;
        bool bad;
        pixel_keys<kFilter>(levels, texs, n_tex, px, no_mip, keys, foot, nf, tw, bad);
        if (bad) {
            any_bad = true;
#pragma unroll
            for (int k = 0; k < kK; k++) keys[k] = kEmpty;
        }
        uint32_t left[kK];
#pragma unroll
        for (int k = 0; k < kK; k++) {
            left[k] = __shfl_up(keys[k], 1, 64);
            if (lane == 0) left[k] = kEmpty;
        }
#pragma unroll
        for (int k = 0; k < kK; k++) {
            bool dup = keys[k] == kEmpty;
#pragma unroll
            for (int j = 0; j < kK; j++) dup |= left[j] == keys[k];
#pragma unroll
            for (int j = 0; j < k; j++) dup |= keys[j] == keys[k];
            if (!dup && !tile_set_insert(s_keys, keys[k]))
                insert(hash, mask, keys[k], queue, max_items, meta, counters);
        }
    }
    if (__ballot(any_bad) && lane == 0) atomicOr(&s_bad, 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kTileSet; i += kThreads)
        if (s_keys[i] != kEmpty) insert(hash, mask, s_keys[i], queue, max_items, meta, counters);
    if (threadIdx.x == 0 && s_bad) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_PIXEL);
}

// The queue (buckets in insertion order) becomes the work list: each new
// block takes a free slot, which goes into its bucket and owner[].
__global__ __launch_bounds__(kThreads) void k_hash_queue(const jpt_level_desc *__restrict__ levels,
                                                         const jpt_texture_desc *__restrict__ texs,
                                                         uint32_t *__restrict__ hash, uint32_t *__restrict__ work,
                                                         uint32_t max_items, uint32_t *__restrict__ slot_of,
                                                         uint32_t *__restrict__ owner,
                                                         const uint32_t *__restrict__ free_stack,
                                                         const uint32_t *__restrict__ meta,
                                                         uint32_t *__restrict__ counters) {
    const uint32_t n = min(meta[JPT_META_QCOUNT], max_items), top = meta[JPT_META_TOP];
    for (uint32_t q = blockIdx.x * kThreads + threadIdx.x; q < n; q += gridDim.x * kThreads) {
        const uint32_t h = work[q], key = hash[2 * h];
        const uint32_t tex = (key >> 3) & 8191u, lvl = key & 7u, idx = key >> 16;
        const uint32_t b = levels[texs[tex].first_level + lvl].blk_base + idx;
        work[q] = b << 2;
        uint32_t slot = JPT_SLOT_NONE;
        if (q < top) {
            slot = free_stack[top - 1 - q];
            owner[slot] = key;
        } else {
            atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
        }
        hash[2 * h + 1] = (slot & kSlotMask) | kVis;
        slot_of[b] = slot;
    }
}

__global__ void k_hash_finish(uint32_t *__restrict__ meta, uint32_t *__restrict__ counters, uint32_t max_items,
                              uint32_t n_slots) {
    if (threadIdx.x != 0) return;
    const uint32_t q = meta[JPT_META_QCOUNT], top = meta[JPT_META_TOP];
    if (q > max_items) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
    const uint32_t placed = min(min(q, max_items), top);
    meta[JPT_META_TOP] = top - placed;
    counters[JPT_CTR_ITEMS] = min(q, max_items);
    counters[JPT_CTR_NEW] = q;
    counters[JPT_CTR_VISIBLE] = meta[JPT_META_VISIBLE];
    counters[JPT_CTR_EVICTED] = meta[JPT_META_EVICTED];
    counters[JPT_CTR_RESIDENT] = n_slots - (top - placed);
}

// ---------------------------------------------------------------- resolve
// Resolve: the paper probes the map for every tap.  Here a workgroup probes
// it once per distinct key of its 64 x 16 pixel tile (gathered in LDS as in
// mark), and each tap then finds its key's slot in the LDS set (a tap whose
// key found no room there probes the map itself).
template <uint32_t kFilter>
__global__ __launch_bounds__(kThreads) void k_hash_resolve(const jpt_level_desc *__restrict__ levels,
                                                           const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                           const jpt_gpixel *__restrict__ gbuf, uint32_t W,
                                                           uint32_t H, uint32_t pitch, uint32_t *__restrict__ frame,
                                                           uint32_t frame_pitch, bool no_mip,
                                                           const uint32_t *__restrict__ hash, uint32_t mask,
                                                           const uint32_t *__restrict__ texels) {
    constexpr int kK = kFilter == JPT_FILTER_NEAREST ? 1 : (kFilter == JPT_FILTER_TRILINEAR ? 8 : 4);
    constexpr int kRows = kTileH / (kThreads / 64);
    __shared__ uint32_t s_keys[kTileSet];
    __shared__ uint32_t s_slot[kTileSet];
    for (int i = threadIdx.x; i < kTileSet; i += kThreads) s_keys[i] = kEmpty;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t x = blockIdx.x * kTileW + lane;
    const uint32_t y0 = blockIdx.y * kTileH + (threadIdx.x >> 6);
    jpt_gpixel px[kRows];
#pragma unroll
    for (int r = 0; r < kRows; r++) {
        const uint32_t y = y0 + r * (kThreads / 64);
        px[r] = x < W && y < H ? gbuf[(size_t)y * pitch + x] : jpt_gpixel{0.f, 0.f, JPT_TEX_BACKGROUND, 0.f};
    }
    // the tile's distinct keys
#pragma unroll
    for (int r = 0; r < kRows; r++) {
        uint32_t keys[kK];
        LevelFoot foot[2];
        int nf;
        uint32_t tw;
        bool bad;
        pixel_keys<kFilter>(levels, texs, n_tex, px[r], no_mip, keys, foot, nf, tw, bad);
        uint32_t left[kK];
#pragma unroll
        for (int k = 0; k < kK; k++) {
            left[k] = __shfl_up(keys[k], 1, 64);
            if (lane == 0) left[k] = kEmpty;
        }
#pragma unroll
        for (int k = 0; k < kK; k++) {
            bool dup = keys[k] == kEmpty;
#pragma unroll
            for (int j = 0; j < kK; j++) dup |= left[j] == keys[k];
            if (!dup) tile_set_insert(s_keys, keys[k]);
        }
    }
    __syncthreads();
    // one probe of the map per distinct key
    for (int i = threadIdx.x; i < kTileSet; i += kThreads) {
        const uint32_t key = s_keys[i];
        if (key != kEmpty) s_slot[i] = lookup(hash, mask, key);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRows; r++) {
        const uint32_t y = y0 + r * (kThreads / 64);
        if (x >= W || y >= H) continue;
        uint32_t keys[kK];
        LevelFoot foot[2];
        int nf;
        uint32_t tw;
        bool bad;
        const int st = pixel_keys<kFilter>(levels, texs, n_tex, px[r], no_mip, keys, foot, nf, tw, bad);
        uint32_t out;
        if (st == PIX_BACKGROUND) {
            out = 0;
        } else if (st == PIX_INVALID || bad) {
            out = JPT_TEXEL_INVALID;
        } else {
            uint32_t lvl[2][3] = {{0, 0, 0}, {0, 0, 0}};
            bool missing = false;
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const LevelFoot &F = foot[k];
                if (k >= nf || F.lw == 0) continue;  // a level of zero weight was not marked and is not read
                uint32_t acc[3] = {0, 0, 0};
                const uint32_t wx[2] = {256 - F.fx, F.fx}, wy[2] = {256 - F.fy, F.fy};
                const uint32_t xs[2] = {F.x0, F.x1}, ys[2] = {F.y0, F.y1};
                const int na = kFilter == JPT_FILTER_NEAREST ? 1 : 2;
#pragma unroll
                for (int b = 0; b < na; b++)
#pragma unroll
                    for (int a = 0; a < na; a++) {
                        const uint32_t w = kFilter == JPT_FILTER_NEAREST ? 65536u : wx[a] * wy[b];
                        if (w == 0) continue;
                        const uint32_t key = keys[kFilter == JPT_FILTER_NEAREST ? 0 : 4 * k + 2 * b + a];
                        // one lookup per tap (the paper's cost of linear filtering), in the tile's set
                        const int e = tile_set_find(s_keys, key);
                        const uint32_t slot = e >= 0 ? s_slot[e] : lookup(hash, mask, key);
                        if (slot == JPT_SLOT_NONE) {
                            missing = true;
                            continue;
                        }
                        const uint32_t v = texels[(size_t)slot * 256 + (ys[b] & 15) * 16 + (xs[a] & 15)];
#pragma unroll
                        for (int c = 0; c < 3; c++) acc[c] += ((v >> (8 * c)) & 255u) * w;
                    }
#pragma unroll
                for (int c = 0; c < 3; c++) lvl[k][c] = (acc[c] + 32768u) >> 16;
            }
            if (missing) {
                out = JPT_TEXEL_INVALID;
            } else {
                uint32_t a[3] = {lvl[0][0], lvl[0][1], lvl[0][2]};
                if (kFilter == JPT_FILTER_TRILINEAR && nf == 2) {
#pragma unroll
                    for (int c = 0; c < 3; c++) a[c] = (lvl[0][c] * (256 - tw) + lvl[1][c] * tw + 128) >> 8;
                }
                out = a[0] | (a[1] << 8) | (a[2] << 16) | 0xFF000000u;
            }
        }
        __builtin_nontemporal_store(out, frame + (size_t)y * frame_pitch + x);
    }
}

uint32_t grid_of(uint64_t n, uint32_t cap) {
    const uint64_t g = (n + kThreads - 1) / kThreads;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

bool hash_cache_ok(const jpt_cache *c) {
    return c->texels && c->slot_of && c->owner && c->free_stack && c->meta && c->hash && c->n_slots > 0 &&
           c->n_buckets >= 2 * c->n_slots && (c->n_buckets & (c->n_buckets - 1)) == 0 && c->n_slots < kSlotMask;
}

jpt_status hash_mark_frame(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                           jpt_frame *frame, jpt_cache *cache, hipStream_t st) {
    const uint32_t mask = cache->n_buckets - 1;
    hipLaunchKernelGGL(k_hash_begin, dim3(1), dim3(kThreads), 0, st, cache->meta, frame->counters);
    hipLaunchKernelGGL(k_hash_clear, dim3(grid_of(cache->n_buckets, 2048)), dim3(kThreads), 0, st, cache->hash,
                       cache->n_buckets);
    hipLaunchKernelGGL(k_hash_reinsert, dim3(grid_of(cache->n_slots, 2048)), dim3(kThreads), 0, st, cache->hash, mask,
                       cache->owner, cache->n_slots, frame->counters);
    HIP_CHECK_LAUNCH();
    const uint32_t mode = filter_mode(filter);
    const bool no_mip = filter_no_mip(filter);
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (!V.width || !V.height) continue;
        const dim3 grid((V.width + kTileW - 1) / kTileW, (V.height + kTileH - 1) / kTileH);
#define JPT_HASH_MARK(F)                                                                                          \
    hipLaunchKernelGGL(k_hash_mark<F>, grid, dim3(kThreads), 0, st, scene->levels, scene->textures,              \
                       scene->n_textures, V.gbuf, V.width, V.height, V.pitch, no_mip, cache->hash, mask,          \
                       frame->work, frame->max_items, cache->meta, frame->counters)
        if (mode == JPT_FILTER_NEAREST) JPT_HASH_MARK(JPT_FILTER_NEAREST);
        else if (mode == JPT_FILTER_BILINEAR) JPT_HASH_MARK(JPT_FILTER_BILINEAR);
        else if (mode == JPT_FILTER_BILINEAR_CLAMPED) JPT_HASH_MARK(JPT_FILTER_BILINEAR_CLAMPED);
        else JPT_HASH_MARK(JPT_FILTER_TRILINEAR);
#undef JPT_HASH_MARK
        HIP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_hash_evict, dim3(grid_of(cache->n_buckets, 2048)), dim3(kThreads), 0, st, cache->hash,
                       cache->n_buckets, cache->owner, cache->free_stack, cache->n_slots, cache->meta);
    hipLaunchKernelGGL(k_hash_queue, dim3(grid_of(frame->max_items, 1024)), dim3(kThreads), 0, st, scene->levels,
                       scene->textures, cache->hash, frame->work, frame->max_items, cache->slot_of, cache->owner,
                       cache->free_stack, cache->meta, frame->counters);
    hipLaunchKernelGGL(k_hash_finish, dim3(1), dim3(64), 0, st, cache->meta, frame->counters, frame->max_items,
                       cache->n_slots);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}

jpt_status hash_resolve(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                        const jpt_cache *cache, hipStream_t st) {
    const uint32_t mask = cache->n_buckets - 1;
    const uint32_t mode = filter_mode(filter);
    const bool no_mip = filter_no_mip(filter);
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (!V.width || !V.height) continue;
        const dim3 grid((V.width + kTileW - 1) / kTileW, (V.height + kTileH - 1) / kTileH);
#define JPT_HASH_RESOLVE(F)                                                                                       \
    hipLaunchKernelGGL(k_hash_resolve<F>, grid, dim3(kThreads), 0, st, scene->levels, scene->textures,           \
                       scene->n_textures, V.gbuf, V.width, V.height, V.pitch, V.frame, V.frame_pitch, no_mip,     \
                       cache->hash, mask, cache->texels)
        if (mode == JPT_FILTER_NEAREST) JPT_HASH_RESOLVE(JPT_FILTER_NEAREST);
        else if (mode == JPT_FILTER_BILINEAR) JPT_HASH_RESOLVE(JPT_FILTER_BILINEAR);
        else if (mode == JPT_FILTER_BILINEAR_CLAMPED) JPT_HASH_RESOLVE(JPT_FILTER_BILINEAR_CLAMPED);
        else JPT_HASH_RESOLVE(JPT_FILTER_TRILINEAR);
#undef JPT_HASH_RESOLVE
        HIP_CHECK_LAUNCH();
    }
    return JPT_OK;
}

namespace {
__global__ __launch_bounds__(kThreads) void k_hash_reset(uint32_t *__restrict__ hash, uint32_t n_buckets,
                                                         uint32_t *__restrict__ owner,
                                                         uint32_t *__restrict__ free_stack, uint32_t n_slots,
                                                         uint32_t *__restrict__ meta) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x, stride = gridDim.x * kThreads;
    for (uint32_t h = i; h < n_buckets; h += stride) { hash[2 * h] = kEmpty; hash[2 * h + 1] = 0; }
    for (uint32_t s = i; s < n_slots; s += stride) {
        owner[s] = JPT_SLOT_NONE;
        free_stack[s] = n_slots - 1 - s;
    }
    for (uint32_t k = i; k < JPT_CACHE_META_WORDS; k += stride) meta[k] = k == JPT_META_TOP ? n_slots : 0u;
}
}  // namespace

jpt_status hash_cache_reset(jpt_cache *cache, hipStream_t st) {
    const uint32_t n = cache->n_buckets > cache->n_slots ? cache->n_buckets : cache->n_slots;
    hipLaunchKernelGGL(k_hash_reset, dim3(grid_of(n, 4096)), dim3(kThreads), 0, st, cache->hash, cache->n_buckets,
                       cache->owner, cache->free_stack, cache->n_slots, cache->meta);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}
