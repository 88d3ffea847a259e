// Mark and compaction (paper: Method, "Mark"; the decoding queue of the
// overview figure; the visibility flags of "Texture Block Cache").
//
// Instead of an atomicCAS into a hash map per pixel, every pixel ORs one bit
// per footprint block into a dense bitmask (one bit per block id), with the
// wave first merging equal block ids so that one atomic is issued per
// distinct block.  A two-kernel scan over the bitmask then lists the new
// blocks in ascending id order (a deterministic order of the same set the
// paper queues) and assigns cache slots.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace {

constexpr int kMarkThreads = 256;  // 4 waves, each an 8x8 pixel tile -> 16x16 pixels per workgroup

__global__ __launch_bounds__(256) void k_clear(uint32_t *__restrict__ vis, uint32_t n_words,
                                               uint32_t *__restrict__ counters) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t w = i; w < n_words; w += gridDim.x * blockDim.x) vis[w] = 0;
    if (i < JPT_N_COUNTERS) counters[i] = (i == JPT_CTR_ERROR_ITEM) ? 0xFFFFFFFFu : 0u;
}

__global__ __launch_bounds__(kMarkThreads) void k_mark(const jpt_level_desc *__restrict__ levels,
                                                       const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                       const jpt_gpixel *__restrict__ gbuf, uint32_t W, uint32_t H,
                                                       uint32_t pitch, uint32_t filter, uint32_t *__restrict__ vis,
                                                       uint32_t *__restrict__ counters) {
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t x = blockIdx.x * 16 + (wv & 1) * 8 + (lane & 7);
    const uint32_t y = blockIdx.y * 16 + (wv >> 1) * 8 + (lane >> 3);
    uint32_t ids[8];
#pragma unroll
    for (int k = 0; k < 8; k++) ids[k] = 0xFFFFFFFFu;
    bool invalid = false;
    if (x < W && y < H) {
        const jpt_gpixel px = gbuf[(size_t)y * pitch + x];
        LevelFoot foot[2];
        int nf;
        uint32_t tw;
        int st = pixel_footprint(levels, texs, n_tex, px, filter, foot, nf, tw);
        if (st == PIX_INVALID) {
            invalid = true;
        } else if (st == PIX_VALID) {
#pragma unroll
            for (int k = 0; k < 2; k++) {
                if (k >= nf || foot[k].lw == 0) continue;
                const LevelFoot &F = foot[k];
                if (filter == JPT_FILTER_NEAREST) {
                    ids[4 * k] = block_of(F, F.x0, F.y0);
                } else {
                    const bool c0 = F.fx != 256, c1 = F.fx != 0, r0 = F.fy != 256, r1 = F.fy != 0;
                    if (c0 && r0) ids[4 * k + 0] = block_of(F, F.x0, F.y0);
                    if (c1 && r0) ids[4 * k + 1] = block_of(F, F.x1, F.y0);
                    if (c0 && r1) ids[4 * k + 2] = block_of(F, F.x0, F.y1);
                    if (c1 && r1) ids[4 * k + 3] = block_of(F, F.x1, F.y1);
                }
            }
        }
    }
    // One atomic per distinct block id of the wave: take the first pending id
    // of the first lane that has one, drop it everywhere, let that lane set it.
    while (true) {
        uint32_t cand = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 7; k >= 0; k--)
            if (ids[k] != 0xFFFFFFFFu) cand = ids[k];
        const uint64_t pending = __ballot(cand != 0xFFFFFFFFu);
        if (pending == 0) break;
        const int leader = __builtin_ctzll(pending);
        const uint32_t id = __builtin_amdgcn_readlane(cand, leader);
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (ids[k] == id) ids[k] = 0xFFFFFFFFu;
        if ((int)lane == leader) atomicOr(vis + (id >> 5), 1u << (id & 31));
    }
    const uint64_t bad = __ballot(invalid);
    if (bad && (int)lane == __builtin_ctzll(bad)) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_PIXEL);
}

// ---------------------------------------------------------- compaction
// Scan tile: 256 threads x 4 consecutive words.  Per word: the blocks to
// decode (visible and not resident) and their work items (1 per 4:2:0
// block, 4 per 4:4:4 block).  Packed sums: items in the low 32 bits, new
// blocks in the high 32 bits.

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, uint32_t lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

struct WordCounts {
    uint32_t newm[4];
    uint32_t sub[4];  // work items per block of that word's level
};

__device__ __forceinline__ uint64_t count_words(const uint32_t *__restrict__ vis, const uint32_t *__restrict__ resident,
                                                const uint32_t *__restrict__ word_level,
                                                const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                                uint32_t w0, WordCounts &wc, uint32_t &n_visible) {
    uint64_t sum = 0;
    n_visible = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t w = w0 + i;
        uint32_t v = 0, r = 0, sub = 1;
        if (w < n_words) {
            v = vis[w];
            r = resident ? resident[w] : 0u;
            if (v & ~r) sub = levels[word_level[w]].sampling == JPT_SAMPLING_444 ? 4u : 1u;
        }
        wc.newm[i] = v & ~r;
        wc.sub[i] = sub;
        uint32_t nb = __popc(v & ~r);
        n_visible += __popc(v);
        sum += ((uint64_t)nb << 32) | (uint64_t)(nb * sub);
    }
    return sum;
}

__global__ __launch_bounds__(256) void k_count(const uint32_t *__restrict__ vis, const uint32_t *__restrict__ resident,
                                               const uint32_t *__restrict__ word_level,
                                               const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                               uint64_t *__restrict__ tile_sums, uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_sum[4];
    __shared__ uint32_t s_vis[4];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WordCounts wc;
    uint32_t nv;
    uint64_t s = count_words(vis, resident, word_level, levels, n_words,
                             blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * 4, wc, nv);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        s += __shfl_xor(s, d, 64);
        nv += __shfl_xor(nv, d, 64);
    }
    if (lane == 0) { s_sum[wv] = s; s_vis[wv] = nv; }
    __syncthreads();
    if (threadIdx.x == 0) {
        tile_sums[blockIdx.x] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        uint32_t t = s_vis[0] + s_vis[1] + s_vis[2] + s_vis[3];
        if (t) atomicAdd(counters + JPT_CTR_VISIBLE, t);
    }
}

__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ vis, const uint32_t *__restrict__ resident,
                                              const uint32_t *__restrict__ word_level,
                                              const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                              const uint64_t *__restrict__ tile_sums, uint32_t n_tiles,
                                              uint32_t *__restrict__ work, uint32_t max_items,
                                              uint32_t *__restrict__ slot_of, uint32_t n_slots,
                                              uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_red[4];
    __shared__ uint64_t s_wave[4];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // prefix of all earlier tiles (a few hundred values at most)
    uint64_t pre = 0;
    for (uint32_t t = threadIdx.x; t < blockIdx.x; t += blockDim.x) pre += tile_sums[t];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pre += __shfl_xor(pre, d, 64);
    if (lane == 0) s_red[wv] = pre;
    WordCounts wc;
    uint32_t nv;
    uint64_t mine = count_words(vis, resident, word_level, levels, n_words,
                                blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * 4, wc, nv);
    uint64_t incl = wave_incl_scan(mine, lane);
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    uint64_t base = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    for (uint32_t k = 0; k < wv; k++) base += s_wave[k];
    base += incl - mine;
    uint32_t item = (uint32_t)base, blk = (uint32_t)(base >> 32);
    bool overflow = false;
    const uint32_t w0 = blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * 4;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t m = wc.newm[i];
        while (m) {
            const uint32_t bit = __builtin_ctz(m);
            m &= m - 1;
            const uint32_t b = (w0 + i) * 32 + bit;
            const uint32_t sub = wc.sub[i];
            bool fits = item + sub <= max_items;
            for (uint32_t q = 0; q < sub; q++)
                if (item + q < max_items) work[item + q] = (b << 2) | q;
            uint32_t slot = (blk < n_slots && fits) ? blk : JPT_SLOT_NONE;
            if (slot_of) slot_of[b] = slot;
            overflow |= !fits || (slot_of && blk >= n_slots);
            item += sub;
            blk += 1;
        }
    }
    if (overflow) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
    if (blockIdx.x == n_tiles - 1 && threadIdx.x == blockDim.x - 1) {
        // the last thread of the last tile ends with the totals
        counters[JPT_CTR_ITEMS] = item < max_items ? item : max_items;
        counters[JPT_CTR_NEW] = blk;
    }
}

}  // namespace

extern "C" jpt_status jpt_mark_blocks(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                      jpt_frame *frame, jpt_cache *cache, const jpt_tuning *tuning, void *stream) {
    (void)tuning;
    if (!scene || !frame || (n_views && !views)) return JPT_E_ARG;
    if (filter > JPT_FILTER_TRILINEAR) return JPT_E_ARG;
    if (!scene->levels || !scene->textures || !scene->word_level || scene->n_blocks == 0 ||
        (scene->n_blocks & 31) || scene->n_blocks > (1u << 29))
        return JPT_E_ARG;
    if (!frame->vis || !frame->work || !frame->counters || !frame->scan) return JPT_E_ARG;
    if (cache && cache->policy != JPT_CACHE_NONE) return JPT_E_ARG;  // LRU: not available in this build
    for (uint32_t v = 0; v < n_views; v++)
        if (!views[v].gbuf || views[v].pitch < views[v].width) return JPT_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t n_words = scene->n_blocks / 32;
    const uint32_t n_tiles = (n_words + JPT_SCAN_TILE_WORDS - 1) / JPT_SCAN_TILE_WORDS;
    uint32_t clear_groups = (n_words + 255) / 256;
    if (clear_groups > 1024) clear_groups = 1024;
    if (clear_groups == 0) clear_groups = 1;
    hipLaunchKernelGGL(k_clear, dim3(clear_groups), dim3(256), 0, st, frame->vis, n_words, frame->counters);
    HIP_CHECK_LAUNCH();
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (V.width == 0 || V.height == 0) continue;
        dim3 grid((V.width + 15) / 16, (V.height + 15) / 16);
        hipLaunchKernelGGL(k_mark, grid, dim3(kMarkThreads), 0, st, scene->levels, scene->textures,
                           scene->n_textures, V.gbuf, V.width, V.height, V.pitch, filter, frame->vis,
                           frame->counters);
        HIP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_count, dim3(n_tiles), dim3(256), 0, st, frame->vis, (const uint32_t *)nullptr,
                       scene->word_level, scene->levels, n_words, frame->scan, frame->counters);
    HIP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_emit, dim3(n_tiles), dim3(256), 0, st, frame->vis, (const uint32_t *)nullptr,
                       scene->word_level, scene->levels, n_words, frame->scan, n_tiles, frame->work,
                       frame->max_items, cache ? cache->slot_of : nullptr, cache ? cache->n_slots : 0u,
                       frame->counters);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}
