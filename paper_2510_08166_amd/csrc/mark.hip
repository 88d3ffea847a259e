// Mark and compaction (paper: Method, "Mark"; the decoding queue of the
// overview figure; the visibility flags of "Texture Block Cache").
//
// Instead of an atomicCAS into a hash map per pixel, every pixel ORs one bit
// per footprint block into a dense bitmask (one bit per block id), with the
// wave first merging equal block ids so that one atomic is issued per
// distinct block.  The new blocks are then listed in ascending id order (a
// deterministic order of the same set the paper queues) with their cache
// slots: without a cache in one pass over the bitmask, from per-tile counts
// the mark kernel keeps as it sets bits; with the LRU cache by a two-kernel
// scan.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "dev_common.h"
#include "hashcache.h"

namespace {

// Workgroup sizes of the mark kernel: 4 waves (8 rows of a tile each) or 8
// waves (4 rows each); see launch_mark_desc.
constexpr int kMarkThreads = 256, kMarkThreadsWide = 512;

// (LRU frames) the bitmask, the counters, the eviction's tie mask, age
// histograms, evicted count and deep-selection flag
__global__ __launch_bounds__(256) void k_clear(uint32_t *__restrict__ vis, uint32_t *__restrict__ tie_mask,
                                               uint32_t n_words, uint32_t *__restrict__ counters,
                                               uint32_t *__restrict__ meta, uint32_t n_bins) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t w = i; w < n_words; w += gridDim.x * blockDim.x) {
        vis[w] = 0;
        tie_mask[w] = 0;
    }
    if (i < JPT_N_COUNTERS) counters[i] = (i == JPT_CTR_ERROR_ITEM) ? 0xFFFFFFFFu : 0u;
    for (uint32_t k = i; k < n_bins; k += gridDim.x * blockDim.x) meta[JPT_META_HIST + k] = 0;
    if (i == 0) {
        meta[JPT_META_EVICTED] = 0;
        meta[JPT_META_DEEP] = 0;
    }
}

// Pixel tile of one workgroup: 64 x 32 pixels; wave w handles rows
// w, w+4, ... so that each wave reads whole 1 KiB G-buffer row segments.
constexpr int kTileW = 64, kTileH = 32;
// LDS set of the bitmask words touched by the tile (open addressing).
constexpr int kSetSize = 1024, kSetProbes = 16;

// Per-tile counts of newly set bitmask bits (frame-local cache): tile t =
// words [256 t, 256 t + 256) in cnt[t], group g = 256 tiles spread over
// cnt2[kGrpSlots g, kGrpSlots g + kGrpSlots) (a slot per workgroup modulo
// kGrpSlots, so that the group's atomics do not all meet at one address); packed
// as new blocks in the high 32 bits and their work items in the low 32.
constexpr uint32_t kGrpSlots = 16;
struct TileCounts {
    uint64_t *cnt, *cnt2;
    const uint32_t *word_level;
    const jpt_level_desc *levels;
};

// vis[word] |= bits; with counts, the bits this call set are added to the
// word's tile (each bit goes from 0 to 1 once per frame).
__device__ __forceinline__ void or_bits(uint32_t *__restrict__ vis, uint32_t word, uint32_t bits, const TileCounts &tc) {
    if (!tc.cnt) {
        atomicOr(vis + word, bits);
        return;
    }
    const uint32_t old = atomicOr(vis + word, bits);
    const uint32_t sub = tc.levels[tc.word_level[word]].sampling == JPT_SAMPLING_444 ? 4u : 1u;
    const uint32_t nb = __popc(bits & ~old);
    if (nb) {
        const uint64_t packed = ((uint64_t)nb << 32) | (uint64_t)(nb * sub);
        atomicAdd((unsigned long long *)(tc.cnt + word / JPT_SCAN_TILE_WORDS), (unsigned long long)packed);
        atomicAdd((unsigned long long *)(tc.cnt2 + word / (JPT_SCAN_TILE_WORDS * 256u) * kGrpSlots +
                                         blockIdx.x % kGrpSlots),
                  (unsigned long long)packed);
    }
}

// One HBM atomic per distinct bitmask word of the tile's LDS set, all of a
// thread's in flight at once.  With counts, the bits they set are summed per
// scan tile in LDS (s_ctile / s_cval, a few entries: a pixel tile's blocks
// fall in a few scan tiles) and go out with one atomic per scan tile and
// group; a scan tile that finds no entry is counted in HBM directly.
constexpr int kCntSlots = 32;

__device__ __forceinline__ void add_count(uint64_t *__restrict__ cnt, uint64_t *__restrict__ cnt2, uint32_t tile,
                                          uint64_t packed) {
    atomicAdd((unsigned long long *)(cnt + tile), (unsigned long long)packed);
    atomicAdd((unsigned long long *)(cnt2 + tile / 256u * kGrpSlots + blockIdx.x % kGrpSlots),
              (unsigned long long)packed);
}

template <int kThreads>
__device__ __forceinline__ void flush_set(const uint32_t *s_key, const uint32_t *s_bits, uint32_t *s_ctile,
                                          unsigned long long *s_cval, uint32_t *__restrict__ vis,
                                          const TileCounts &tc) {
    constexpr int kPer = kSetSize / kThreads;
    uint32_t key[kPer], bits[kPer];
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        key[j] = s_key[threadIdx.x + j * kThreads];
        bits[j] = s_bits[threadIdx.x + j * kThreads];
    }
    if (!tc.cnt) {
#pragma unroll
        for (int j = 0; j < kPer; j++)
            if (key[j] != 0xFFFFFFFFu) atomicOr(vis + key[j], bits[j]);
        return;
    }
    uint32_t old[kPer], lv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; j++) old[j] = key[j] != 0xFFFFFFFFu ? atomicOr(vis + key[j], bits[j]) : bits[j];
#pragma unroll
    for (int j = 0; j < kPer; j++) lv[j] = key[j] != 0xFFFFFFFFu ? tc.word_level[key[j]] : 0u;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const uint32_t nb = __popc(bits[j] & ~old[j]);
        if (!nb) continue;
        const uint32_t sub = tc.levels[lv[j]].sampling == JPT_SAMPLING_444 ? 4u : 1u;
        const uint64_t packed = ((uint64_t)nb << 32) | (uint64_t)(nb * sub);
        const uint32_t tile = key[j] / JPT_SCAN_TILE_WORDS;
        uint32_t h = tile & (kCntSlots - 1);
        bool done = false;
        for (int p = 0; p < kCntSlots && !done; p++) {
            const uint32_t o = atomicCAS(s_ctile + h, 0xFFFFFFFFu, tile);
            if (o == 0xFFFFFFFFu || o == tile) {
                atomicAdd(s_cval + h, (unsigned long long)packed);
                done = true;
            }
            h = (h + 1) & (kCntSlots - 1);
        }
        if (!done) add_count(tc.cnt, tc.cnt2, tile, packed);
    }
    __syncthreads();
    if (threadIdx.x < kCntSlots && s_ctile[threadIdx.x] != 0xFFFFFFFFu)
        add_count(tc.cnt, tc.cnt2, s_ctile[threadIdx.x], s_cval[threadIdx.x]);
}

__device__ __forceinline__ void set_insert(uint32_t *s_key, uint32_t *s_bits, uint32_t *__restrict__ vis,
                                           uint32_t id, const TileCounts &tc) {
    const uint32_t word = id >> 5, bit = 1u << (id & 31);
    // slot of a word: its low bits (a tile touches runs of consecutive words,
    // which this spreads without collisions, at no 32-bit multiply)
    uint32_t h = word & (kSetSize - 1);
    for (int p = 0; p < kSetProbes; p++) {
        const uint32_t old = atomicCAS(s_key + h, 0xFFFFFFFFu, word);
        if (old == 0xFFFFFFFFu || old == word) {
            atomicOr(s_bits + h, bit);
            return;
        }
        h = (h + 1) & (kSetSize - 1);
    }
    or_bits(vis, word, bit, tc);  // set crowded: go straight to HBM
}

// One workgroup marks one 64 x 32 pixel tile per step and walks the tiles of
// every view in the launch's table with a stride of gridDim.x.  A wave takes
// rows wv, wv+4, ... of the tile, one row per step with the next row's
// G-buffer load in flight.  Each lane drops the block ids that its left
// neighbour (the previous pixel of the row) also touches, and inserts the
// rest into the tile's LDS set; the set is flushed to the bitmask with one
// HBM atomic per distinct word (and, with counts, one per tile level).
// The kernel asks the compiler for registers that let 8 waves share a SIMD
// (106 scalar registers allowed 7): 78 scalar registers, the rest spilled to
// vector lanes; for the 8-wave form that is 4 workgroups per compute unit
// instead of 3 (1080p: 14.3 against 16.5 us; 16 views with 4 waves: 208
// against 240 us).  The trilinear form holds two levels' footprints: it asks
// for 6 waves per SIMD (77 vector registers instead of 85, which allowed 5;
// the heavy 4K sequence: 78 against 87 us), since 7 or 8 would spill to memory.
template <uint32_t kFilter, int kDesc, int kThreads>
__global__ __launch_bounds__(kThreads, kFilter != JPT_FILTER_TRILINEAR ? 8 : 6) void k_mark(const jpt_level_desc *__restrict__ levels,
                                                       const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                       uint32_t n_lev, const ViewTable tab,
                                                       uint32_t *__restrict__ vis, const TileCounts tc,
                                                       uint32_t *__restrict__ err_word, bool no_mip) {
    constexpr int kRows = kTileH / (kThreads / 64);  // rows per wave
    constexpr int kIds = kFilter == JPT_FILTER_NEAREST ? 1 : (kFilter == JPT_FILTER_TRILINEAR ? 8 : 4);
    __shared__ uint32_t s_key[kSetSize], s_bits[kSetSize], s_ctile[kCntSlots];
    __shared__ unsigned long long s_cval[kCntSlots];
    __shared__ TexRec s_t[kDesc != DESC_HBM ? kLdsTexCap : 1];
    __shared__ LevRec s_l[kDesc == DESC_LDS ? kLdsLevCap : 1];
    __shared__ uint32_t s_bad;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_bad = 0;
    if constexpr (kDesc == DESC_LDS) load_desc_lds(levels, texs, n_tex, n_lev, s_t, s_l);
    if constexpr (kDesc == DESC_TEX_LDS) load_tex_lds(texs, n_tex, s_t);
    bool invalid = false;
    for (uint32_t slot = blockIdx.x; slot < tab.span; slot += gridDim.x) {
        uint32_t view, tx, ty;
        if (!tile_of(tab, slot, view, tx, ty)) continue;  // uniform over the workgroup
        const jpt_gpixel *__restrict__ gbuf = tab.v[view].gbuf;
        const uint32_t W = tab.v[view].width, H = tab.v[view].height, pitch = tab.v[view].pitch;
        const uint32_t x = tx * kTileW + lane, y0 = ty * kTileH + wv, xc = min(x, W - 1u);
        // loads from clamped in-bounds addresses (no branch), masked afterwards
        auto load_px = [&](uint32_t y) -> jpt_gpixel {
            const jpt_gpixel g = gbuf[(size_t)min(y, H - 1u) * pitch + xc];
            return (x < W && y < H) ? g : jpt_gpixel{0.f, 0.f, JPT_TEX_BACKGROUND, 0.f};
        };
        jpt_gpixel nxt = load_px(y0);
        for (int i = threadIdx.x; i < kSetSize; i += kThreads) {
            s_key[i] = 0xFFFFFFFFu;
            s_bits[i] = 0;
        }
        if (threadIdx.x < kCntSlots) {
            s_ctile[threadIdx.x] = 0xFFFFFFFFu;
            s_cval[threadIdx.x] = 0;
        }
        __syncthreads();
#pragma unroll 1
        for (int r = 0; r < kRows; r++) {
            const jpt_gpixel px = nxt;
            if (r + 1 < kRows) nxt = load_px(y0 + (r + 1) * (kThreads / 64));
            uint32_t ids[kIds];
#pragma unroll
            for (int k = 0; k < kIds; k++) ids[k] = 0xFFFFFFFFu;
            LevelFoot foot[2];
            int nf;
            uint32_t tw;
            int st;
            if constexpr (kDesc == DESC_LDS)
                st = pixel_footprint(LdsDesc{s_t, s_l}, n_tex, px, kFilter, foot, nf, tw, no_mip);
            else if constexpr (kDesc == DESC_TEX_LDS)
                st = pixel_footprint(MixDesc{s_t, levels}, n_tex, px, kFilter, foot, nf, tw, no_mip);
            else st = pixel_footprint(GlobalDesc{levels, texs}, n_tex, px, kFilter, foot, nf, tw, no_mip);
            if (st == PIX_INVALID) {
                invalid = true;
            } else if (st == PIX_VALID) {
#pragma unroll
                for (int k = 0; k < (kFilter == JPT_FILTER_TRILINEAR ? 2 : 1); k++) {
                    if (k >= nf || foot[k].lw == 0) continue;
                    const LevelFoot &F = foot[k];
                    if constexpr (kFilter == JPT_FILTER_NEAREST) {
                        ids[0] = block_of(F, F.x0, F.y0);
                    } else {
                        // the distinct blocks of the texels read with non-zero weight:
                        // column x1 counts only when x0 is unread or x1 lies in
                        // the next block column (likewise rows), so no two ids of
                        // a level are equal
                        const uint32_t bx0 = F.x0 >> 4, bx1 = F.x1 >> 4, by0 = F.y0 >> 4, by1 = F.y1 >> 4;
                        const bool c0 = F.fx != 256, c1 = F.fx != 0 && (!c0 || bx1 != bx0);
                        const bool r0 = F.fy != 256, r1 = F.fy != 0 && (!r0 || by1 != by0);
                        const uint32_t row0 = F.blk_base + __umul24(by0, F.blk_cols);
                        const uint32_t row1 = F.blk_base + __umul24(by1, F.blk_cols);
                        if (c0 && r0) ids[4 * k + 0] = row0 + bx0;
                        if (c1 && r0) ids[4 * k + 1] = row0 + bx1;
                        if (c0 && r1) ids[4 * k + 2] = row1 + bx0;
                        if (c1 && r1) ids[4 * k + 3] = row1 + bx1;
                    }
                }
            }
            // drop the ids the left neighbour (the previous pixel of the row)
            // also holds for the same level slot; ids of different levels
            // never coincide
            constexpr int kPerLevel = kFilter == JPT_FILTER_NEAREST ? 1 : 4;
            uint32_t left[kIds];
#pragma unroll
            for (int k = 0; k < kIds; k++) {
                left[k] = __shfl_up(ids[k], 1, 64);
                if (lane == 0) left[k] = 0xFFFFFFFFu;
            }
#pragma unroll
            for (int k = 0; k < kIds; k++) {
                const uint32_t id = ids[k];
                bool dup = id == 0xFFFFFFFFu;
                const int lv0 = (k / kPerLevel) * kPerLevel;
#pragma unroll
                for (int j = 0; j < kPerLevel; j++) dup |= left[lv0 + j] == id;
                if (!dup) set_insert(s_key, s_bits, vis, id, tc);
            }
        }
        __syncthreads();
        flush_set<kThreads>(s_key, s_bits, s_ctile, s_cval, vis, tc);
        __syncthreads();  // the set is reused by the next tile
    }
    if (__ballot(invalid) && lane == 0) atomicOr(&s_bad, 1u);
    __syncthreads();
    if (threadIdx.x == 0 && s_bad) atomicOr(err_word, JPT_ERR_PIXEL);
}

// Workgroups of the 8-wave mark the GPU holds at once (compute units x
// resident workgroups per unit), queried once per device.
template <uint32_t kFilter, int kDesc>
uint32_t wide_mark_capacity() {
    constexpr int kMaxDev = 64;
    static std::atomic<uint32_t> known[kMaxDev];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0u;
    uint32_t g = known[dev].load(std::memory_order_relaxed);
    if (g) return g;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mark<kFilter, kDesc, kMarkThreadsWide>,
                                                     kMarkThreadsWide, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
        cus <= 0)
        return 0u;
    g = (uint32_t)per_cu * (uint32_t)cus;
    known[dev].store(g, std::memory_order_relaxed);
    return g;
}

// A launch of at most two rounds of 8-wave workgroups takes 8 waves per
// tile: the tiles' rows are walked by twice the waves, each with half the
// serial chain of loads and set inserts (a 1080p frame, 1,020 tiles: 16.5
// against 18.0 us).  A longer launch, where the next round keeps the GPU
// full anyway, takes 4, whose tiles cost fewer barrier waits (16 views,
// 42,000 tiles: 235 against 265 us with 8).
template <uint32_t kFilter, int kDesc>
void launch_mark_desc(const jpt_scene *scene, const ViewTable &tab, uint32_t groups, jpt_frame *frame,
                      const TileCounts &tc, uint32_t *err_word, bool no_mip, hipStream_t st) {
    if (groups <= 2 * wide_mark_capacity<kFilter, kDesc>())
        hipLaunchKernelGGL((k_mark<kFilter, kDesc, kMarkThreadsWide>), dim3(groups), dim3(kMarkThreadsWide), 0, st,
                           scene->levels, scene->textures, scene->n_textures, scene->n_levels, tab, frame->vis, tc,
                           err_word, no_mip);
    else
        hipLaunchKernelGGL((k_mark<kFilter, kDesc, kMarkThreads>), dim3(groups), dim3(kMarkThreads), 0, st,
                           scene->levels, scene->textures, scene->n_textures, scene->n_levels, tab, frame->vis, tc,
                           err_word, no_mip);
}

template <uint32_t kFilter>
void launch_mark(const jpt_scene *scene, const ViewTable &tab, uint32_t groups, jpt_frame *frame,
                 const TileCounts &tc, uint32_t *err_word, bool no_mip, hipStream_t st) {
    switch (desc_mode(scene->n_textures, scene->n_levels)) {
    case DESC_LDS: launch_mark_desc<kFilter, DESC_LDS>(scene, tab, groups, frame, tc, err_word, no_mip, st); break;
    case DESC_TEX_LDS:
        launch_mark_desc<kFilter, DESC_TEX_LDS>(scene, tab, groups, frame, tc, err_word, no_mip, st);
        break;
    default: launch_mark_desc<kFilter, DESC_HBM>(scene, tab, groups, frame, tc, err_word, no_mip, st); break;
    }
}

// Frame number of an LRU frame: the caller's, or the cache's own counter.
__device__ __forceinline__ uint32_t lru_frame(uint32_t frame_no, const uint32_t *__restrict__ meta) {
    return frame_no != JPT_FRAME_AUTO ? frame_no : meta[JPT_META_FRAME];
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

// Exclusive prefix of this thread's packed sum within the whole scan: the
// sums of earlier tiles plus the earlier threads of this tile.
__device__ __forceinline__ uint64_t scan_base(const uint64_t *__restrict__ tile_sums, uint64_t mine) {
    __shared__ uint64_t s_red[kScanThreads / 64];
    __shared__ uint64_t s_wave[kScanThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
    return base + incl - mine;
}

// Sum of one value over the workgroup, written to tile_sums[blockIdx.x] and,
// with grp, added to the tile's group slot (kGrpSlots per 256 tiles).
__device__ __forceinline__ void tile_total(uint64_t s, uint64_t *__restrict__ tile_sums, uint32_t *vis_counter,
                                           uint32_t nv, uint64_t *__restrict__ grp = nullptr) {
    __shared__ uint64_t s_sum[kScanThreads / 64];
    __shared__ uint32_t s_vis[kScanThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
        if (vis_counter && tv) atomicAdd(vis_counter, tv);
        if (grp && t)
            atomicAdd((unsigned long long *)(grp + blockIdx.x / 256u * kGrpSlots + blockIdx.x % kGrpSlots),
                      (unsigned long long)t);
    }
}

// Work items (and blocks) of a scan tile that the counted compaction stages
// in LDS before storing them as whole rows.
constexpr uint32_t kEmitStage = 4096;

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
            const uint32_t lv = word_level[w];  // (loaded beside the bitmask word)
            v = vis[w];
            r = resident ? resident[w] : 0u;
            if (v & ~r) sub = levels[lv].sampling == JPT_SAMPLING_444 ? 4u : 1u;
        }
        wc.newm[i] = v & ~r;
        wc.sub[i] = sub;
        const uint32_t nb = __popc(v & ~r);
        n_visible += __popc(v);
        sum += ((uint64_t)nb << 32) | (uint64_t)(nb * sub);
    }
    return sum;
}

// Count the new blocks of each tile.  With a cache (LRU), visible resident
// blocks are touched here: last_used of their slot = frame_no.
__global__ __launch_bounds__(kScanThreads) void k_count(const uint32_t *__restrict__ vis,
                                                        const uint32_t *__restrict__ resident,
                                                        const uint32_t *__restrict__ word_level,
                                                        const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                                        uint64_t *__restrict__ tile_sums,
                                                        uint32_t *__restrict__ counters,
                                                        const uint32_t *__restrict__ slot_of,
                                                        uint32_t *__restrict__ last_used, uint32_t frame_no,
                                                        const uint32_t *__restrict__ meta, uint64_t *__restrict__ grp) {
    WordCounts wc;
    uint32_t nv;
    const uint32_t w0 = blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt;
    const uint64_t s = count_words(vis, resident, word_level, levels, n_words, w0, wc, nv);
    if (resident) {
        const uint32_t f = lru_frame(frame_no, meta);
#pragma unroll
        for (int i = 0; i < kWpt; i++) {
            if (w0 + i >= n_words) continue;
            uint32_t m = vis[w0 + i] & resident[w0 + i];
            while (m) {
                const uint32_t b = (w0 + i) * 32 + __builtin_ctz(m);
                m &= m - 1;
                last_used[slot_of[b]] = f;
            }
        }
    }
    tile_total(s, tile_sums, counters + JPT_CTR_VISIBLE, nv, grp);
}

// List the new blocks of an LRU frame: work items in ascending block id
// order and their cache slots, popped off the free stack.  The bitmask words
// are zeroed behind (the state the frame-local path expects).
__global__ __launch_bounds__(kScanThreads) void k_emit_lru(uint32_t *__restrict__ vis,
                                                       uint32_t *__restrict__ resident,
                                                       const uint32_t *__restrict__ word_level,
                                                       const jpt_level_desc *__restrict__ levels, uint32_t n_words,
                                                       const uint64_t *__restrict__ tile_sums, uint32_t n_tiles,
                                                       uint32_t *__restrict__ work, uint32_t max_items,
                                                       uint32_t *__restrict__ slot_of, uint32_t n_slots,
                                                       uint32_t *__restrict__ counters,
                                                       const uint32_t *__restrict__ free_stack,
                                                       const uint32_t *__restrict__ meta,
                                                       uint32_t *__restrict__ owner,
                                                       uint32_t *__restrict__ last_used, uint32_t frame_no) {
    const uint32_t w0 = blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt;
    WordCounts wc;
    uint32_t nv;
    const uint64_t mine = count_words(vis, resident, word_level, levels, n_words, w0, wc, nv);
#pragma unroll
    for (int i = 0; i < kWpt; i++)
        if (w0 + i < n_words) vis[w0 + i] = 0;  // (this thread read it above)
    const uint64_t base = scan_base(tile_sums, mine);
    const uint32_t top = meta[JPT_META_TOP];  // free slots after this frame's evictions
    const uint32_t f = lru_frame(frame_no, meta);
    uint32_t item = (uint32_t)base, blk = (uint32_t)(base >> 32);
    bool overflow = false;
#pragma unroll
    for (int i = 0; i < kWpt; i++) {
        uint32_t m = wc.newm[i];
        const uint32_t sub = wc.sub[i];
        uint32_t placed = 0;
        while (m) {
            const uint32_t bit = __builtin_ctz(m);
            m &= m - 1;
            const uint32_t b = (w0 + i) * 32 + bit;
            const bool fits = item + sub <= max_items;
            for (uint32_t q = 0; q < sub; q++)
                if (item + q < max_items) work[item + q] = (b << 2) | q;
            uint32_t slot = JPT_SLOT_NONE;
            if (blk < top && fits) {
                slot = free_stack[top - 1 - blk];
                owner[slot] = b;
                last_used[slot] = f;
                placed |= 1u << bit;
            }
            overflow |= !fits || blk >= top;
            slot_of[b] = slot;
            item += sub;
            blk += 1;
        }
        if (placed) resident[w0 + i] |= placed;  // this thread owns the word
    }
    if (overflow) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
    if (blockIdx.x == n_tiles - 1 && threadIdx.x == kScanThreads - 1) {
        // the last thread of the last tile ends with the totals
        counters[JPT_CTR_ITEMS] = item < max_items ? item : max_items;
        counters[JPT_CTR_NEW] = blk;
    }
}

// Compaction for a frame-local cache, one pass over the bitmask.  The mark
// kernel counted every tile's newly set bits, so a tile's offset is the sum
// of the counts before it (whole groups of 256 tiles from the slots of cnt2, then the
// tiles of its own group from cnt) and no workgroup waits for another.  Each
// workgroup lists its tile's work items and slots and zeroes its bitmask
// words for the next frame; the last one past reading the counts zeroes
// them and writes the frame's counters.  sync[0]: workgroups past reading;
// sync[1]: error flags raised by the mark kernel.
__global__ __launch_bounds__(kScanThreads) void k_emit_counted(uint32_t *__restrict__ vis,
                                                               const uint32_t *__restrict__ word_level,
                                                               const jpt_level_desc *__restrict__ levels,
                                                               uint32_t n_words, uint64_t *__restrict__ cnt,
                                                               uint64_t *__restrict__ cnt2, uint32_t *__restrict__ sync,
                                                               uint32_t n_tiles, uint32_t *__restrict__ work,
                                                               uint32_t max_items, uint32_t *__restrict__ slot_of,
                                                               uint32_t n_slots, uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_red[kScanThreads / 64], s_tot[kScanThreads / 64], s_wave[kScanThreads / 64];
    __shared__ uint32_t s_last;
    __shared__ uint32_t s_items[kEmitStage], s_blocks[kEmitStage];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tile = blockIdx.x;
    const uint32_t w0 = tile * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt;
    // offset of the tile (the groups before its group, the tiles before it
    // in its group) and the frame's total (all groups)
    const uint32_t grp = tile / 256u, t0 = grp * 256u, n_grp = (n_tiles + 255u) / 256u;
    uint64_t tot = 0, pre = t0 + threadIdx.x < tile ? cnt[t0 + threadIdx.x] : 0ull;
    for (uint32_t e = threadIdx.x; e < n_grp * kGrpSlots; e += kScanThreads) {
        const uint64_t g = cnt2[e];
        tot += g;
        if (e / kGrpSlots < grp) pre += g;
    }
    WordCounts wc;
    uint32_t nv;
    const uint64_t mine = count_words(vis, nullptr, word_level, levels, n_words, w0, wc, nv);
#pragma unroll
    for (int i = 0; i < kWpt; i++)
        if (w0 + i < n_words) vis[w0 + i] = 0;  // (this thread read it above)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        pre += __shfl_xor(pre, d, 64);
        tot += __shfl_xor(tot, d, 64);
    }
    const uint64_t incl = wave_incl_scan(mine, lane);
    if (lane == 0) { s_red[wv] = pre; s_tot[wv] = tot; }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    // every thread has consumed its count loads: tell the others
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(sync, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == n_tiles - 1;
    uint64_t base = incl - mine, all = 0;
    for (int k = 0; k < kScanThreads / 64; k++) {
        base += s_red[k] + (k < (int)wv ? s_wave[k] : 0ull);
        all += s_tot[k];
    }
    uint32_t item = (uint32_t)base, blk = (uint32_t)(base >> 32);
    // the tile's first item and block and its counts (uniform)
    uint64_t off = 0, tot_wg = 0;
    for (int k = 0; k < kScanThreads / 64; k++) {
        off += s_red[k];
        tot_wg += s_wave[k];
    }
    const uint32_t item0 = (uint32_t)off, blk0 = (uint32_t)(off >> 32);
    const uint32_t n_items_wg = (uint32_t)tot_wg, n_blocks_wg = (uint32_t)(tot_wg >> 32);
    if (n_items_wg <= kEmitStage && n_blocks_wg <= kEmitStage) {
        // each thread's items and blocks into LDS at their offsets in the
        // tile, then whole-workgroup stores (bit 31 of a block: its items do
        // not all fit the work list)
#pragma unroll
        for (int i = 0; i < kWpt; i++) {
            uint32_t m = wc.newm[i];
            const uint32_t sub = wc.sub[i];
            while (m) {
                const uint32_t bit = __builtin_ctz(m);
                m &= m - 1;
                const uint32_t b = (w0 + i) * 32 + bit;
                for (uint32_t q = 0; q < sub; q++) s_items[item - item0 + q] = (b << 2) | q;
                s_blocks[blk - blk0] = b | (item + sub <= max_items ? 0u : 0x80000000u);
                item += sub;
                blk += 1;
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n_items_wg; i += kScanThreads)
            if (item0 + i < max_items) work[item0 + i] = s_items[i];
        if (slot_of)
            for (uint32_t j = threadIdx.x; j < n_blocks_wg; j += kScanThreads) {
                const uint32_t e = s_blocks[j], s = blk0 + j;
                slot_of[e & 0x7FFFFFFFu] = s < n_slots && !(e >> 31) ? s : JPT_SLOT_NONE;
            }
    } else {
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
                if (slot_of) slot_of[b] = blk < n_slots && fits ? blk : JPT_SLOT_NONE;
                item += sub;
                blk += 1;
            }
        }
    }
    __syncthreads();
    if (!s_last) return;
    // the last workgroup: every other one has read its counts
    for (uint32_t t = threadIdx.x; t < n_tiles; t += kScanThreads) cnt[t] = 0;
    for (uint32_t e = threadIdx.x; e < n_grp * kGrpSlots; e += kScanThreads) cnt2[e] = 0;
    if (threadIdx.x == 0) {
        const uint32_t items = (uint32_t)all, blocks = (uint32_t)(all >> 32);
        const bool over = items > max_items || (slot_of && blocks > n_slots);
        for (uint32_t c = 0; c < JPT_N_COUNTERS; c++) counters[c] = 0;
        counters[JPT_CTR_ITEMS] = items < max_items ? items : max_items;
        counters[JPT_CTR_NEW] = blocks;
        counters[JPT_CTR_VISIBLE] = blocks;
        counters[JPT_CTR_ERROR] = sync[1] | (over ? JPT_ERR_CAPACITY : 0u);
        counters[JPT_CTR_ERROR_ITEM] = 0xFFFFFFFFu;
        sync[0] = 0;
        sync[1] = 0;
    }
}

// ------------------------------------------------------------ LRU update
// (paper: "Update Cache", with a slot capacity and least-recently-used
// eviction in place of evicting every block that was not visible.)  The
// candidates (resident, not visible) are ranked by age f - last_used, the
// oldest going first and equal ages by the smaller block id.  A histogram of
// ages capped at JPT_LRU_MAX_AGE finds the age where the evictions end; when
// that is the capped bin, three radix passes over the candidates' exact
// 32-bit ages (digits of 11, 11 and 10 bits) narrow it to one age.
constexpr int kAgeBins = JPT_LRU_MAX_AGE + 1;
constexpr uint32_t kCap = JPT_LRU_MAX_AGE;
constexpr int kDigitBins = 2048;

__device__ __forceinline__ bool bit_set(const uint32_t *__restrict__ mask, uint32_t b) {
    return (mask[b >> 5] >> (b & 31)) & 1u;
}

__device__ __forceinline__ uint32_t age_of(uint32_t frame_no, uint32_t last) { return frame_no - last; }
__device__ __forceinline__ uint32_t age_bin(uint32_t age) { return age < kCap ? age : kCap; }
__device__ __forceinline__ uint32_t digit0(uint32_t age) { return age >> 21; }
__device__ __forceinline__ uint32_t digit1(uint32_t age) { return (age >> 10) & 2047u; }
__device__ __forceinline__ uint32_t digit2(uint32_t age) { return age & 1023u; }

// Add an LDS histogram to one in HBM (non-zero bins only).
template <int kBins>
__device__ __forceinline__ void flush_hist(const uint32_t *s_h, uint32_t *__restrict__ g) {
    for (int k = threadIdx.x; k < kBins; k += 256)
        if (s_h[k]) atomicAdd(g + k, s_h[k]);
}

// The frame's plan (new blocks from the group sums of the count kernel;
// evictions needed = new blocks beyond the free slots), derived by every
// workgroup and published by the first, then the histogram of the
// candidates' capped ages and, for the candidates in the capped bin, of
// their first age digit.
__global__ __launch_bounds__(256) void k_lru_hist(const uint32_t *__restrict__ owner,
                                                  const uint32_t *__restrict__ last_used,
                                                  const uint32_t *__restrict__ vis, uint32_t n_slots,
                                                  uint32_t frame_no, uint32_t *__restrict__ meta,
                                                  const uint64_t *__restrict__ grp, uint32_t n_grp,
                                                  uint32_t evict_all) {
    __shared__ uint32_t s_h[kAgeBins];
    __shared__ uint32_t s_d[kDigitBins];
    __shared__ uint32_t s_need;
    if (threadIdx.x < 64) {
        uint64_t t = 0;
        for (uint32_t e = threadIdx.x; e < n_grp; e += 64) t += grp[e];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        if (threadIdx.x == 0) {
            const uint32_t n_new = (uint32_t)(t >> 32), top = meta[JPT_META_TOP];
            const uint32_t need = n_new > top ? n_new - top : 0u;
            s_need = need;
            if (blockIdx.x == 0) {
                meta[JPT_META_NEW] = n_new;
                meta[JPT_META_NEED] = need;
            }
        }
    }
    __syncthreads();
    if (s_need == 0 || evict_all) return;  // (evicting every candidate needs no ranking)
    const uint32_t f = lru_frame(frame_no, meta);
    for (int k = threadIdx.x; k < kAgeBins; k += 256) s_h[k] = 0;
    for (int k = threadIdx.x; k < kDigitBins; k += 256) s_d[k] = 0;
    __syncthreads();
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n_slots; s += gridDim.x * 256) {
        const uint32_t b = owner[s];
        if (b == JPT_SLOT_NONE || bit_set(vis, b)) continue;
        const uint32_t age = age_of(f, last_used[s]);
        atomicAdd(s_h + age_bin(age), 1u);
        if (age >= kCap) atomicAdd(s_d + digit0(age), 1u);
    }
    __syncthreads();
    flush_hist<kAgeBins>(s_h, meta + JPT_META_HIST);
    flush_hist<kDigitBins>(s_d, meta + JPT_META_DH0);
}

// Where `need` evictions end in a histogram taken oldest (highest bin)
// first: the bin of the last evicted candidates (higher bins go whole) and
// how many of that bin go; rest = 0xFFFFFFFF when the histogram holds fewer
// than `need` candidates (all of them go).  256 threads; every thread
// returns the same values.
template <int kBins>
__device__ __forceinline__ void select_bin(const uint32_t *__restrict__ hist, uint32_t need, uint32_t &bin,
                                           uint32_t &rest) {
    __shared__ uint32_t s_sum[256];
    __shared__ uint32_t s_res[2];
    constexpr int kPer = kBins / 256;
    static_assert(kPer * 256 == kBins, "bins must split over 256 threads");
    // thread t owns bins [kBins - kPer (t+1), kBins - kPer t): oldest first
    const int hi = kBins - kPer * (int)threadIdx.x;
    uint32_t mine = 0;
    for (int k = hi - kPer; k < hi; k++) mine += hist[k];
    s_sum[threadIdx.x] = mine;
    if (threadIdx.x == 0) {
        s_res[0] = 0;
        s_res[1] = 0xFFFFFFFFu;
    }
    __syncthreads();
    uint32_t before = 0;  // candidates in older bins
    for (uint32_t t = 0; t < threadIdx.x; t++) before += s_sum[t];
    if (before < need && before + mine >= need) {
        uint32_t c = before;
        for (int k = hi - 1; k >= hi - kPer; k--) {
            const uint32_t h = hist[k];
            if (c + h >= need) {
                s_res[0] = (uint32_t)k;
                s_res[1] = need - c;
                break;
            }
            c += h;
        }
    }
    __syncthreads();
    bin = s_res[0];
    rest = s_res[1];
}

__device__ __forceinline__ void evict(uint32_t s, uint32_t b, uint32_t *__restrict__ owner,
                                      uint32_t *__restrict__ slot_of, uint32_t *__restrict__ resident,
                                      uint32_t *__restrict__ free_stack, uint32_t *__restrict__ meta) {
    owner[s] = JPT_SLOT_NONE;
    slot_of[b] = JPT_SLOT_NONE;
    atomicAnd(resident + (b >> 5), ~(1u << (b & 31)));
    free_stack[atomicAdd(meta + JPT_META_TOP, 1u)] = s;
    atomicAdd(meta + JPT_META_EVICTED, 1u);
}

// Evict the candidates older than the threshold bin and mark that bin's in
// the tie mask; every workgroup derives the threshold itself, the first one
// publishes it for the tie kernels.  When the threshold is the capped bin,
// this is the first pass of the exact selection instead: the candidates of
// that bin whose first age digit is above the chosen one go, and the second
// digits of those at the chosen one are counted.
__global__ __launch_bounds__(256) void k_lru_evict(uint32_t *__restrict__ owner, const uint32_t *__restrict__ last_used,
                                                   const uint32_t *__restrict__ vis, uint32_t n_slots,
                                                   uint32_t frame_no, uint32_t *__restrict__ slot_of,
                                                   uint32_t *__restrict__ resident, uint32_t *__restrict__ free_stack,
                                                   uint32_t *__restrict__ tie_mask, uint32_t *__restrict__ meta,
                                                   uint32_t *__restrict__ counters, uint32_t evict_all) {
    __shared__ uint32_t s_d[kDigitBins];
    const uint32_t need = meta[JPT_META_NEED];
    if (evict_all) {
        // the paper's policy: every resident block this frame does not read goes
        if (blockIdx.x == 0 && threadIdx.x == 0) meta[JPT_META_TIES] = 0xFFFFFFFFu;
        for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n_slots; s += gridDim.x * 256) {
            const uint32_t b = owner[s];
            if (b != JPT_SLOT_NONE && !bit_set(vis, b)) evict(s, b, owner, slot_of, resident, free_stack, meta);
        }
        return;
    }
    if (need == 0) return;
    uint32_t abin, ties;
    select_bin<kAgeBins>(meta + JPT_META_HIST, need, abin, ties);
    const bool all = ties == 0xFFFFFFFFu;
    const bool deep = !all && abin == kCap;
    uint32_t d0 = 0, r0 = 0;
    if (deep) select_bin<kDigitBins>(meta + JPT_META_DH0, ties, d0, r0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        meta[JPT_META_ABIN] = abin;
        meta[JPT_META_TIES] = ties;
        meta[JPT_META_DEEP] = deep ? 1u : 0u;
        meta[JPT_META_D0] = d0;
        meta[JPT_META_R0] = r0;
        // fewer candidates than new blocks: all of them go, the rest find no slot
        if (all) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CAPACITY);
    }
    if (deep) {
        for (int k = threadIdx.x; k < kDigitBins; k += 256) s_d[k] = 0;
        __syncthreads();
    }
    const uint32_t f = lru_frame(frame_no, meta);
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n_slots; s += gridDim.x * 256) {
        const uint32_t b = owner[s];
        if (b == JPT_SLOT_NONE || bit_set(vis, b)) continue;
        const uint32_t age = age_of(f, last_used[s]);
        const uint32_t bin = age_bin(age);
        if (all || bin > abin) {
            evict(s, b, owner, slot_of, resident, free_stack, meta);
        } else if (bin == abin) {
            if (!deep) atomicOr(tie_mask + (b >> 5), 1u << (b & 31));
            else if (digit0(age) > d0) evict(s, b, owner, slot_of, resident, free_stack, meta);
            else if (digit0(age) == d0) atomicAdd(s_d + digit1(age), 1u);
        }
    }
    if (deep) {
        __syncthreads();
        flush_hist<kDigitBins>(s_d, meta + JPT_META_DH1);
    }
}

// Second pass of the exact selection: inside the chosen first digit, the
// candidates whose second digit is above the chosen one go, and the third
// digits of those at the chosen one are counted.
__global__ __launch_bounds__(256) void k_lru_deep1(uint32_t *__restrict__ owner,
                                                   const uint32_t *__restrict__ last_used,
                                                   const uint32_t *__restrict__ vis, uint32_t n_slots,
                                                   uint32_t frame_no, uint32_t *__restrict__ slot_of,
                                                   uint32_t *__restrict__ resident,
                                                   uint32_t *__restrict__ free_stack, uint32_t *__restrict__ meta) {
    __shared__ uint32_t s_d[1024];
    if (meta[JPT_META_DEEP] == 0) return;
    const uint32_t d0 = meta[JPT_META_D0];
    uint32_t d1, r1;
    select_bin<kDigitBins>(meta + JPT_META_DH1, meta[JPT_META_R0], d1, r1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        meta[JPT_META_D1] = d1;
        meta[JPT_META_R1] = r1;
    }
    for (int k = threadIdx.x; k < 1024; k += 256) s_d[k] = 0;
    __syncthreads();
    const uint32_t f = lru_frame(frame_no, meta);
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n_slots; s += gridDim.x * 256) {
        const uint32_t b = owner[s];
        if (b == JPT_SLOT_NONE || bit_set(vis, b)) continue;
        const uint32_t age = age_of(f, last_used[s]);
        if (age < kCap || digit0(age) != d0) continue;
        if (digit1(age) > d1) evict(s, b, owner, slot_of, resident, free_stack, meta);
        else if (digit1(age) == d1) atomicAdd(s_d + digit2(age), 1u);
    }
    __syncthreads();
    flush_hist<1024>(s_d, meta + JPT_META_DH2);
}

// Last pass: the candidates of the chosen first two digits whose third digit
// is above the chosen one go; those of exactly the chosen age are marked in
// the tie mask, of which the tie kernels evict the smallest ids.
__global__ __launch_bounds__(256) void k_lru_deep2(uint32_t *__restrict__ owner,
                                                   const uint32_t *__restrict__ last_used,
                                                   const uint32_t *__restrict__ vis, uint32_t n_slots,
                                                   uint32_t frame_no, uint32_t *__restrict__ slot_of,
                                                   uint32_t *__restrict__ resident,
                                                   uint32_t *__restrict__ free_stack,
                                                   uint32_t *__restrict__ tie_mask, uint32_t *__restrict__ meta) {
    if (meta[JPT_META_DEEP] == 0) return;
    const uint32_t d0 = meta[JPT_META_D0], d1 = meta[JPT_META_D1];
    uint32_t d2, r2;
    select_bin<1024>(meta + JPT_META_DH2, meta[JPT_META_R1], d2, r2);
    if (blockIdx.x == 0 && threadIdx.x == 0) meta[JPT_META_TIES] = r2;
    const uint32_t f = lru_frame(frame_no, meta);
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n_slots; s += gridDim.x * 256) {
        const uint32_t b = owner[s];
        if (b == JPT_SLOT_NONE || bit_set(vis, b)) continue;
        const uint32_t age = age_of(f, last_used[s]);
        if (age < kCap || digit0(age) != d0 || digit1(age) != d1) continue;
        if (digit2(age) > d2) evict(s, b, owner, slot_of, resident, free_stack, meta);
        else if (digit2(age) == d2) atomicOr(tie_mask + (b >> 5), 1u << (b & 31));
    }
}

// Count the marked blocks of the last bin per scan tile.
__global__ __launch_bounds__(kScanThreads) void k_tie_count(const uint32_t *__restrict__ tie_mask, uint32_t n_words,
                                                            uint64_t *__restrict__ tile_sums,
                                                            const uint32_t *__restrict__ meta) {
    const uint32_t w0 = blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt;
    uint64_t s = 0;
    if (meta[JPT_META_NEED] != 0)
#pragma unroll
        for (int i = 0; i < kWpt; i++)
            if (w0 + i < n_words) s += __popc(tie_mask[w0 + i]);
    tile_total(s, tile_sums, nullptr, 0);
}

// Evict the marked blocks with the smallest ids, as many as the plan says.
__global__ __launch_bounds__(kScanThreads) void k_tie_pick(const uint32_t *__restrict__ tie_mask, uint32_t n_words,
                                                           const uint64_t *__restrict__ tile_sums,
                                                           uint32_t *__restrict__ owner, uint32_t *__restrict__ slot_of,
                                                           uint32_t *__restrict__ resident,
                                                           uint32_t *__restrict__ free_stack,
                                                           uint32_t *__restrict__ meta) {
    const uint32_t need = meta[JPT_META_NEED];
    const uint32_t ties = meta[JPT_META_TIES];
    const uint32_t w0 = blockIdx.x * JPT_SCAN_TILE_WORDS + threadIdx.x * kWpt;
    uint32_t m[kWpt];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kWpt; i++) {
        m[i] = (need != 0 && w0 + i < n_words) ? tie_mask[w0 + i] : 0u;
        s += __popc(m[i]);
    }
    uint32_t rank = (uint32_t)scan_base(tile_sums, s);
    if (need == 0 || ties == 0xFFFFFFFFu) return;
#pragma unroll
    for (int i = 0; i < kWpt; i++) {
        while (m[i] && rank < ties) {
            const uint32_t b = (w0 + i) * 32 + __builtin_ctz(m[i]);
            m[i] &= m[i] - 1;
            evict(slot_of[b], b, owner, slot_of, resident, free_stack, meta);
            rank++;
        }
    }
}

// Pop the placed blocks off the free stack; report the update.
__global__ void k_lru_finish(uint32_t *__restrict__ meta, uint32_t *__restrict__ counters, uint32_t n_slots,
                             uint32_t frame_no, uint64_t *__restrict__ grp, uint32_t n_grp) {
    for (uint32_t e = threadIdx.x; e < n_grp; e += blockDim.x) grp[e] = 0;  // (zero again for the next frame)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    meta[JPT_META_FRAME] = lru_frame(frame_no, meta) + 1u;
    const uint32_t top = meta[JPT_META_TOP], n_new = meta[JPT_META_NEW];
    const uint32_t top2 = n_new < top ? top - n_new : 0u;
    meta[JPT_META_TOP] = top2;
    counters[JPT_CTR_EVICTED] = meta[JPT_META_EVICTED];
    counters[JPT_CTR_RESIDENT] = n_slots - top2;
}

__global__ __launch_bounds__(256) void k_cache_reset(uint32_t *__restrict__ slot_of, uint32_t n_blocks,
                                                     uint32_t *__restrict__ owner, uint32_t *__restrict__ last_used,
                                                     uint32_t *__restrict__ free_stack, uint32_t n_slots,
                                                     uint32_t *__restrict__ resident, uint32_t *__restrict__ tie_mask,
                                                     uint32_t n_words, uint32_t *__restrict__ meta) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    for (uint32_t b = i; b < n_blocks; b += stride) slot_of[b] = JPT_SLOT_NONE;
    for (uint32_t s = i; s < n_slots; s += stride) {
        owner[s] = JPT_SLOT_NONE;
        last_used[s] = 0;
        free_stack[s] = n_slots - 1 - s;  // pops hand out slots 0, 1, 2, ...
    }
    for (uint32_t w = i; w < n_words; w += stride) { resident[w] = 0; tie_mask[w] = 0; }
    for (uint32_t k = i; k < JPT_CACHE_META_WORDS; k += stride) meta[k] = k == JPT_META_TOP ? n_slots : 0u;
}

uint32_t grid_for(uint64_t n, uint32_t per_group, uint32_t cap) {
    uint64_t g = (n + per_group - 1) / per_group;
    if (g < 1) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

bool lru_ok(const jpt_cache *c) {
    // (the LRU and evict-invisible policies keep the same per-slot state)
    return c->texels && c->slot_of && c->owner && c->last_used && c->resident && c->free_stack && c->meta &&
           c->tie_mask && c->n_slots > 0;
}

}  // namespace

extern "C" jpt_status jpt_cache_reset(const jpt_scene *scene, jpt_cache *cache, void *stream) {
    if (scene && cache && cache->policy == JPT_CACHE_HASH)
        return hash_cache_ok(cache) ? hash_cache_reset(cache, (hipStream_t)stream) : JPT_E_ARG;
    if (!scene || !cache || (cache->policy != JPT_CACHE_LRU && cache->policy != JPT_CACHE_EVICT_INVISIBLE) ||
        !lru_ok(cache) || scene->n_blocks == 0 ||
        (scene->n_blocks & 31))
        return JPT_E_ARG;
    const uint32_t n_words = scene->n_blocks / 32;
    hipLaunchKernelGGL(k_cache_reset, dim3(grid_for(scene->n_blocks > cache->n_slots ? scene->n_blocks : cache->n_slots,
                                                    256, 4096)),
                       dim3(256), 0, (hipStream_t)stream, cache->slot_of, scene->n_blocks, cache->owner,
                       cache->last_used, cache->free_stack, cache->n_slots, cache->resident, cache->tie_mask, n_words,
                       cache->meta);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}

namespace {

// Argument checks shared by both mark entry points (all but the scan buffer).
jpt_status mark_args(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                     const jpt_frame *frame) {
    if (!scene || !frame || (n_views && !views)) return JPT_E_ARG;
    if (!filter_valid(filter)) return JPT_E_ARG;
    if (!scene->levels || !scene->textures || !scene->word_level || scene->n_blocks == 0 ||
        (scene->n_blocks & 31) || scene->n_blocks > (1u << 29))
        return JPT_E_ARG;
    if (!frame->vis || !frame->work || !frame->counters) return JPT_E_ARG;
    return JPT_OK;
}

jpt_status mark_frame(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                      jpt_frame *frame, uint64_t *scan, jpt_cache *cache, const jpt_tuning *tuning, void *stream);

}  // namespace

extern "C" jpt_status jpt_mark_blocks(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                      jpt_frame *frame, jpt_cache *cache, const jpt_tuning *tuning, void *stream) {
    const jpt_status s = mark_args(scene, views, n_views, filter, frame);
    if (s != JPT_OK) return s;
    if (!frame->scan) return JPT_E_ARG;
    return mark_frame(scene, views, n_views, filter, frame, frame->scan, cache, tuning, stream);
}

// ------------------------------------------------- no-allocation variant
// jpt_mark_blocks_static keeps the scan scratch in this array instead of
// frame->scan.  Each device holds its own copy at its own address, found
// once per device with hipGetSymbolAddress; host code uses only that
// address, never the array's name (which on the host is a stand-in, not a
// device address).  Calls that overlap on one device share it and race.
static __device__ __align__(256) uint64_t scratch[JPT_STATIC_SCAN_ENTRIES];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<uint64_t *> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's address of `scratch` (JPT_E_HIP if it cannot be had).
jpt_status static_scratch(uint64_t **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return JPT_E_HIP;
    uint64_t *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            void *addr = nullptr;
            if (hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)) != hipSuccess || !addr) return JPT_E_HIP;
            p = static_cast<uint64_t *>(addr);
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return JPT_OK;
}

// Zero n entries (a kernel, not a memset: safe inside a captured graph).
__global__ __launch_bounds__(256) void k_zero_scan(uint64_t *__restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

}  // namespace

extern "C" jpt_status jpt_mark_blocks_static(const jpt_scene *scene, const jpt_view *views, uint32_t n_views,
                                             uint32_t filter, jpt_frame *frame, jpt_cache *cache,
                                             const jpt_tuning *tuning, void *stream) {
    const jpt_status s = mark_args(scene, views, n_views, filter, frame);
    if (s != JPT_OK) return s;
    const uint32_t need = jpt_scan_entries(scene->n_blocks);
    if (need > JPT_STATIC_SCAN_ENTRIES) return JPT_E_CAPACITY;
    uint64_t *scan = nullptr;
    const jpt_status a = static_scratch(&scan);
    if (a != JPT_OK) return a;
    // the array keeps the last call's contents: the entries this scene uses
    // start at zero, as frame->scan does for jpt_mark_blocks
    hipLaunchKernelGGL(k_zero_scan, dim3(grid_for(need, 256, 256)), dim3(256), 0, (hipStream_t)stream, scan, need);
    HIP_CHECK_LAUNCH();
    return mark_frame(scene, views, n_views, filter, frame, scan, cache, tuning, stream);
}

namespace {

jpt_status mark_frame(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                      jpt_frame *frame, uint64_t *scan, jpt_cache *cache, const jpt_tuning *tuning, void *stream) {
    if (cache && cache->policy == JPT_CACHE_HASH) {
        if (!hash_cache_ok(cache)) return JPT_E_ARG;
        for (uint32_t v = 0; v < n_views; v++)
            if (!views[v].gbuf || views[v].pitch < views[v].width) return JPT_E_ARG;
        return hash_mark_frame(scene, views, n_views, filter, frame, cache, (hipStream_t)stream);
    }
    // both cache policies with resident state run the cache-update kernels
    const bool lru = cache && (cache->policy == JPT_CACHE_LRU || cache->policy == JPT_CACHE_EVICT_INVISIBLE);
    const uint32_t evict_all = cache && cache->policy == JPT_CACHE_EVICT_INVISIBLE ? 1u : 0u;
    if (cache && cache->policy > JPT_CACHE_EVICT_INVISIBLE) return JPT_E_ARG;
    if (lru && !lru_ok(cache)) return JPT_E_ARG;
    for (uint32_t v = 0; v < n_views; v++)
        if (!views[v].gbuf || views[v].pitch < views[v].width) return JPT_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t n_words = scene->n_blocks / 32;
    const uint32_t n_tiles = (n_words + JPT_SCAN_TILE_WORDS - 1) / JPT_SCAN_TILE_WORDS;
    // scan: [0, 2 n_tiles) the two scans of an LRU frame; then, for a
    // frame-local cache, the tile counts, the group counts (an LRU frame's
    // count kernel sums its tiles there) and two sync words
    uint64_t *scan2 = scan + n_tiles;  // second scan of the frame (LRU ties)
    TileCounts tc{nullptr, nullptr, scene->word_level, scene->levels};
    uint32_t *err_word = frame->counters + JPT_CTR_ERROR;
    uint32_t *sync = nullptr;
    if (!lru) {
        tc.cnt = scan + 2 * (size_t)n_tiles;
        tc.cnt2 = tc.cnt + n_tiles;
        sync = reinterpret_cast<uint32_t *>(tc.cnt2 + (n_tiles + 255) / 256 * kGrpSlots);
        err_word = sync + 1;
    }
    const uint32_t f = frame->frame_no;
    if (lru) {
        hipLaunchKernelGGL(k_clear, dim3(grid_for(n_words, 256, 1024)), dim3(256), 0, st, frame->vis,
                           cache->tie_mask, n_words, frame->counters, cache->meta,
                           (uint32_t)(JPT_CACHE_META_WORDS - JPT_META_HIST));
        HIP_CHECK_LAUNCH();
    }
    const bool xcd = tuning && (tuning->flags & JPT_TUNE_XCD_TILES);
    for (uint32_t v0 = 0; v0 < n_views; v0 += kMaxLaunchViews) {
        ViewTable tab;
        make_view_table(views, v0, n_views - v0 < kMaxLaunchViews ? n_views - v0 : kMaxLaunchViews, kTileW, kTileH,
                        xcd, tab);
        if (tab.total == 0) continue;
        uint32_t groups = tab.span;
        if (tuning && tuning->mark_groups && tuning->mark_groups < groups)
            groups = xcd ? (tuning->mark_groups + 7) / 8 * 8 : tuning->mark_groups;
        const uint32_t mode = filter_mode(filter);
        const bool no_mip = filter_no_mip(filter);
        if (mode == JPT_FILTER_NEAREST)
            launch_mark<JPT_FILTER_NEAREST>(scene, tab, groups, frame, tc, err_word, no_mip, st);
        else if (mode == JPT_FILTER_BILINEAR)
            launch_mark<JPT_FILTER_BILINEAR>(scene, tab, groups, frame, tc, err_word, no_mip, st);
        else if (mode == JPT_FILTER_BILINEAR_CLAMPED)
            launch_mark<JPT_FILTER_BILINEAR_CLAMPED>(scene, tab, groups, frame, tc, err_word, no_mip, st);
        else launch_mark<JPT_FILTER_TRILINEAR>(scene, tab, groups, frame, tc, err_word, no_mip, st);
        HIP_CHECK_LAUNCH();
    }
    if (!lru) {
        hipLaunchKernelGGL(k_emit_counted, dim3(n_tiles), dim3(kScanThreads), 0, st, frame->vis, scene->word_level,
                           scene->levels, n_words, tc.cnt, tc.cnt2, sync, n_tiles, frame->work, frame->max_items,
                           cache ? cache->slot_of : nullptr, cache ? cache->n_slots : 0u, frame->counters);
        HIP_CHECK_LAUNCH();
        return JPT_OK;
    }
    // group sums of the count kernel: the counted compaction's group slots,
    // unused by an LRU frame (zero between frames)
    uint64_t *grp = scan + 3 * (size_t)n_tiles;
    const uint32_t n_grp = (n_tiles + 255) / 256 * kGrpSlots;
    hipLaunchKernelGGL(k_count, dim3(n_tiles), dim3(kScanThreads), 0, st, frame->vis, cache->resident,
                       scene->word_level, scene->levels, n_words, scan, frame->counters, cache->slot_of,
                       cache->last_used, f, cache->meta, grp);
    HIP_CHECK_LAUNCH();
    const uint32_t sg = grid_for(cache->n_slots, 256, 2048);
    hipLaunchKernelGGL(k_lru_hist, dim3(sg), dim3(256), 0, st, cache->owner, cache->last_used, frame->vis,
                       cache->n_slots, f, cache->meta, grp, n_grp, evict_all);
    hipLaunchKernelGGL(k_lru_evict, dim3(sg), dim3(256), 0, st, cache->owner, cache->last_used, frame->vis,
                       cache->n_slots, f, cache->slot_of, cache->resident, cache->free_stack, cache->tie_mask,
                       cache->meta, frame->counters, evict_all);
    if (!evict_all) {  // (evicting every non-visible block ranks nothing: no exact-age passes, no ties)
        const uint32_t dg = grid_for(cache->n_slots, 256, 512);
        hipLaunchKernelGGL(k_lru_deep1, dim3(dg), dim3(256), 0, st, cache->owner, cache->last_used, frame->vis,
                           cache->n_slots, f, cache->slot_of, cache->resident, cache->free_stack, cache->meta);
        hipLaunchKernelGGL(k_lru_deep2, dim3(dg), dim3(256), 0, st, cache->owner, cache->last_used, frame->vis,
                           cache->n_slots, f, cache->slot_of, cache->resident, cache->free_stack, cache->tie_mask,
                           cache->meta);
        hipLaunchKernelGGL(k_tie_count, dim3(n_tiles), dim3(kScanThreads), 0, st, cache->tie_mask, n_words, scan2,
                           cache->meta);
        hipLaunchKernelGGL(k_tie_pick, dim3(n_tiles), dim3(kScanThreads), 0, st, cache->tie_mask, n_words, scan2,
                           cache->owner, cache->slot_of, cache->resident, cache->free_stack, cache->meta);
        HIP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_emit_lru, dim3(n_tiles), dim3(kScanThreads), 0, st, frame->vis, cache->resident,
                       scene->word_level, scene->levels, n_words, scan, n_tiles, frame->work,
                       frame->max_items, cache->slot_of, cache->n_slots, frame->counters, cache->free_stack,
                       cache->meta, cache->owner, cache->last_used, f);
    hipLaunchKernelGGL(k_lru_finish, dim3(1), dim3(64), 0, st, cache->meta, frame->counters, cache->n_slots, f, grp,
                       n_grp);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}

}  // namespace
