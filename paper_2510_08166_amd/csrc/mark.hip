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

constexpr int kMarkThreads = 256;  // 4 waves per workgroup

__global__ __launch_bounds__(256) void k_clear(uint32_t *__restrict__ vis, uint32_t n_words,
                                               uint32_t *__restrict__ counters) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t w = i; w < n_words; w += gridDim.x * blockDim.x) vis[w] = 0;
    if (i < JPT_N_COUNTERS) counters[i] = (i == JPT_CTR_ERROR_ITEM) ? 0xFFFFFFFFu : 0u;
}

// Pixel tile of one workgroup: 64 x 32 pixels; wave w handles rows
// w, w+4, ... so that each wave reads whole 1 KiB G-buffer row segments.
constexpr int kTileW = 64, kTileH = 32;
// LDS set of the bitmask words touched by the tile (open addressing).
constexpr int kSetSize = 1024, kSetProbes = 16;

__device__ __forceinline__ void set_insert(uint32_t *s_key, uint32_t *s_bits, uint32_t *__restrict__ vis,
                                           uint32_t id) {
    const uint32_t word = id >> 5, bit = 1u << (id & 31);
    uint32_t h = (word * 2654435761u) >> (32 - 10);
    for (int p = 0; p < kSetProbes; p++) {
        const uint32_t old = atomicCAS(s_key + h, 0xFFFFFFFFu, word);
        if (old == 0xFFFFFFFFu || old == word) {
            atomicOr(s_bits + h, bit);
            return;
        }
        h = (h + 1) & (kSetSize - 1);
    }
    atomicOr(vis + word, bit);  // set crowded: go straight to HBM
}

__global__ __launch_bounds__(kMarkThreads) void k_mark(const jpt_level_desc *__restrict__ levels,
                                                       const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                       const jpt_gpixel *__restrict__ gbuf, uint32_t W, uint32_t H,
                                                       uint32_t pitch, uint32_t filter, uint32_t *__restrict__ vis,
                                                       uint32_t *__restrict__ counters) {
    __shared__ uint32_t s_key[kSetSize], s_bits[kSetSize];
    __shared__ uint32_t s_bad;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kSetSize; i += kMarkThreads) {
        s_key[i] = 0xFFFFFFFFu;
        s_bits[i] = 0;
    }
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const uint32_t x = blockIdx.x * kTileW + lane;
    bool invalid = false;
    for (int row = (int)wv; row < kTileH; row += kMarkThreads / 64) {
        const uint32_t y = blockIdx.y * kTileH + row;
        if (y >= H) break;
        uint32_t ids[8];
#pragma unroll
        for (int k = 0; k < 8; k++) ids[k] = 0xFFFFFFFFu;
        if (x < W) {
            const jpt_gpixel px = gbuf[(size_t)y * pitch + x];
            LevelFoot foot[2];
            int nf;
            uint32_t tw;
            const int st = pixel_footprint(levels, texs, n_tex, px, filter, foot, nf, tw);
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
        // Distinct ids of the wave: take the first pending id of the first
        // lane that has one, drop it everywhere, let that lane record it.
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
            if ((int)lane == leader) set_insert(s_key, s_bits, vis, id);
        }
    }
    if (__ballot(invalid) && lane == 0) atomicOr(&s_bad, 1u);
    __syncthreads();
    // one HBM atomic per distinct bitmask word of the tile
    for (int i = threadIdx.x; i < kSetSize; i += kMarkThreads) {
        const uint32_t k = s_key[i];
        if (k != 0xFFFFFFFFu) atomicOr(vis + k, s_bits[i]);
    }
    if (threadIdx.x == 0 && s_bad) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_PIXEL);
}

// ---------------------------------------------------------- compaction
// Scan tile: 256 threads x kWpt consecutive bitmask words.  Per word: the
// blocks to decode (visible and not resident) and their work items (1 per
// 4:2:0 block, 4 per 4:4:4 block).  Packed sums: items in the low 32 bits,
// new blocks in the high 32 bits.
constexpr int kScanThreads = 256;
constexpr int kWpt = JPT_SCAN_TILE_WORDS / kScanThreads;
static_assert(kWpt * kScanThreads == JPT_SCAN_TILE_WORDS, "scan tile must be a multiple of the block size");

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, uint32_t lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

struct WordCounts {
    uint32_t newm[kWpt];
    uint32_t sub[kWpt];  // work items per block of that word's level
};

__device__ __forceinline__ uint64_t count_words(const uint32_t *__restrict__ vis, const uint32_t *__restrict__ resident,
                                                const uint32_t *__restrict__ word_level,
                                                const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                                uint32_t w0, WordCounts &wc, uint32_t &n_visible) {
    uint64_t sum = 0;
    n_visible = 0;
#pragma unroll
    for (int i = 0; i < kWpt; i++) {
        const uint32_t w = w0 + i;
        uint32_t v = 0, r = 0, sub = 1;
        if (w < n_words) {
            v = vis[w];
            r = resident ? resident[w] : 0u;
            if (v & ~r) sub = levels[word_level[w]].sampling == JPT_SAMPLING_444 ? 4u : 1u;
        }
        wc.newm[i] = v & ~r;
        wc.sub[i] = sub;
        const uint32_t nb = __popc(v & ~r);
        n_visible += __popc(v);
        sum += ((uint64_t)nb << 32) | (uint64_t)(nb * sub);
    }
    return sum;
}

__global__ __launch_bounds__(kScanThreads) void k_count(const uint32_t *__restrict__ vis,
                                                        const uint32_t *__restrict__ resident,
                                                        const uint32_t *__restrict__ word_level,
                                                        const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                                        uint64_t *__restrict__ tile_sums,
                                                        uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_sum[kScanThreads / 64];
    __shared__ uint32_t s_vis[kScanThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WordCounts wc;
    uint32_t nv;
    uint64_t s = count_words(vis, resident, word_level, levels, n_words,
                             blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt, wc, nv);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        s += __shfl_xor(s, d, 64);
        nv += __shfl_xor(nv, d, 64);
    }
    if (lane == 0) { s_sum[wv] = s; s_vis[wv] = nv; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        uint32_t tv = 0;
        for (int k = 0; k < kScanThreads / 64; k++) { t += s_sum[k]; tv += s_vis[k]; }
        tile_sums[blockIdx.x] = t;
        if (tv) atomicAdd(counters + JPT_CTR_VISIBLE, tv);
    }
}

__global__ __launch_bounds__(kScanThreads) void k_emit(const uint32_t *__restrict__ vis,
                                                       const uint32_t *__restrict__ resident,
                                                       const uint32_t *__restrict__ word_level,
                                                       const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                                       const uint64_t *__restrict__ tile_sums, uint32_t n_tiles,
                                                       uint32_t *__restrict__ work, uint32_t max_items,
                                                       uint32_t *__restrict__ slot_of, uint32_t n_slots,
                                                       uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_red[kScanThreads / 64];
    __shared__ uint64_t s_wave[kScanThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t w0 = blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt;
    // this tile's words and the sums of all earlier tiles, loads in flight together
    WordCounts wc;
    uint32_t nv;
    uint64_t mine = count_words(vis, resident, word_level, levels, n_words, w0, wc, nv);
    uint64_t pre = 0;
    for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kScanThreads) pre += tile_sums[t];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pre += __shfl_xor(pre, d, 64);
    if (lane == 0) s_red[wv] = pre;
    const uint64_t incl = wave_incl_scan(mine, lane);
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    uint64_t base = 0;
    for (int k = 0; k < kScanThreads / 64; k++) base += s_red[k];
    for (uint32_t k = 0; k < wv; k++) base += s_wave[k];
    base += incl - mine;
    uint32_t item = (uint32_t)base, blk = (uint32_t)(base >> 32);
    bool overflow = false;
#pragma unroll
    for (int i = 0; i < kWpt; i++) {
        uint32_t m = wc.newm[i];
        const uint32_t sub = wc.sub[i];
        while (m) {
            const uint32_t bit = __builtin_ctz(m);
            m &= m - 1;
            const uint32_t b = (w0 + i) * 32 + bit;
            const bool fits = item + sub <= max_items;
            for (uint32_t q = 0; q < sub; q++)
                if (item + q < max_items) work[item + q] = (b << 2) | q;
            if (slot_of) slot_of[b] = (blk < n_slots && fits) ? blk : JPT_SLOT_NONE;
            overflow |= !fits || (slot_of && blk >= n_slots);
            item += sub;
            blk += 1;
        }
    }
    if (overflow) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
    if (blockIdx.x == n_tiles - 1 && threadIdx.x == kScanThreads - 1) {
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
        dim3 grid((V.width + kTileW - 1) / kTileW, (V.height + kTileH - 1) / kTileH);
        hipLaunchKernelGGL(k_mark, grid, dim3(kMarkThreads), 0, st, scene->levels, scene->textures,
                           scene->n_textures, V.gbuf, V.width, V.height, V.pitch, filter, frame->vis,
                           frame->counters);
        HIP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_count, dim3(n_tiles), dim3(kScanThreads), 0, st, frame->vis, (const uint32_t *)nullptr,
                       scene->word_level, scene->levels, n_words, frame->scan, frame->counters);
    HIP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_emit, dim3(n_tiles), dim3(kScanThreads), 0, st, frame->vis, (const uint32_t *)nullptr,
                       scene->word_level, scene->levels, n_words, frame->scan, n_tiles, frame->work,
                       frame->max_items, cache ? cache->slot_of : nullptr, cache ? cache->n_slots : 0u,
                       frame->counters);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}
