// Resolve (paper: Method, "Resolve"): each pixel fetches its filter taps from
// the cache slots of their blocks and blends them with integer weights.
// Every tap a pixel reads was marked, so no clamping at undecoded MCU borders
// is needed (the footprint marking makes the result exact); the paper's
// variant clamped to one MCU is the filter JPT_FILTER_BILINEAR_CLAMPED.
//
// A workgroup shades 64 x 16 pixel tiles, 4 rows per lane (the rows'
// G-buffer loads all in flight at once), walking the tiles of every view in
// the launch's table with a stride of gridDim.x.  The scene's sampling
// descriptors are cached in LDS.  Per pixel, all slot lookups are issued
// before any texel load and all texel loads before the blend; the texture
// addresser spends about the same time on every vector memory instruction
// whatever its lanes, so a bilinear row's two neighbouring texels come in
// one 8-byte load (and, in launches of more than one round of workgroups,
// its two slot-table entries as well), and caches within 4 GiB of texels
// are addressed with 32-bit offsets from a scalar base.
#include <hip/hip_runtime.h>

#include <atomic>

#include "dev_common.h"
#include "hashcache.h"

namespace {

constexpr int kThreads = 256;
constexpr int kTileW = 64, kTileH = 16;
constexpr int kRows = kTileH / (kThreads / 64);

template <uint32_t kFilter>
struct FilterTraits {
    static constexpr int kTaps = kFilter == JPT_FILTER_NEAREST ? 1 : (kFilter == JPT_FILTER_TRILINEAR ? 8 : 4);
};

// Taps of one pixel: block id, byte offset of the texel inside its block's
// slot (row-major 16 x 16 RGBA8) and weight; weights of one level sum to
// 65536.  Every lane computes all of them without branches: the footprint's
// texel coordinates lie inside a real level even for background and invalid
// pixels (whose descriptor indices and coordinates are clamped), so each block id
// is a valid index; the taps a pixel does not read get weight 0.
template <int kTaps>
struct Taps {
    uint32_t blk[kTaps], off[kTaps], w[kTaps];
};

template <uint32_t kFilter, class Desc>
__device__ __forceinline__ int pixel_taps(const Desc &D, uint32_t n_tex, const jpt_gpixel &px,
                                          Taps<FilterTraits<kFilter>::kTaps> &T, uint32_t &tw, int &nf,
                                          bool no_mip) {
    constexpr int kTaps = FilterTraits<kFilter>::kTaps;
    LevelFoot foot[2];
    const int st = pixel_footprint(D, n_tex, px, kFilter, foot, nf, tw, no_mip);
    if (n_tex == 0) {  // (uniform: the footprint is not filled in)
#pragma unroll
        for (int t = 0; t < kTaps; t++) { T.blk[t] = 0; T.off[t] = 0; T.w[t] = 0; }
        return st;
    }
    const bool valid = st == PIX_VALID;
#pragma unroll
    for (int k = 0; k < (kFilter == JPT_FILTER_TRILINEAR ? 2 : 1); k++) {
        const LevelFoot &F = foot[k];
        const bool used = valid && k < nf && F.lw != 0;
        if (kFilter == JPT_FILTER_NEAREST) {
            T.blk[0] = block_of(F, F.x0, F.y0);
            T.off[0] = ((F.y0 & 15) << 6) | ((F.x0 & 15) << 2);
            T.w[0] = used ? 65536u : 0u;
        } else {
            const uint32_t wx[2] = {256 - F.fx, F.fx}, wy[2] = {256 - F.fy, F.fy};
            const uint32_t xs[2] = {F.x0, F.x1}, ys[2] = {F.y0, F.y1};
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int a = 0; a < 2; a++) {
                    const int t = 4 * k + 2 * b + a;
                    T.blk[t] = block_of(F, xs[a], ys[b]);
                    T.off[t] = ((ys[b] & 15) << 6) | ((xs[a] & 15) << 2);
                    T.w[t] = used ? __umul24(wx[a], wy[b]) : 0u;  // <= 2^16
                }
        }
    }
    return st;
}

// base[byte_off / 4]: a 32-bit offset from a base held in scalar registers
// (the address is computed by the load unit, no 64-bit arithmetic per lane)
__device__ __forceinline__ uint32_t load_at(const uint32_t *__restrict__ base, uint32_t byte_off) {
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Texel at byte offset `off` of cache slot `slot`: with kNarrow (every slot
// within the first 4 GiB of texels) through a 32-bit offset.
template <bool kNarrow>
__device__ __forceinline__ uint32_t load_texel(const uint32_t *__restrict__ texels, uint32_t slot, uint32_t off) {
    if constexpr (kNarrow) return load_at(texels, (slot << 10) | off);
    else return load_at(texels + (size_t)slot * 256, off);
}

// Two neighbouring texels of a block row: one 8-byte load (multi-dword
// global loads need only 4-byte alignment).
typedef uint32_t TexelPair __attribute__((ext_vector_type(2)));
typedef TexelPair TexelPairA4 __attribute__((aligned(4)));
template <bool kNarrow>
__device__ __forceinline__ TexelPair load_pair(const uint32_t *__restrict__ texels, uint32_t slot, uint32_t off) {
    const char *p = reinterpret_cast<const char *>(kNarrow ? texels : texels + (size_t)slot * 256);
    return *reinterpret_cast<const TexelPairA4 *>(p + (kNarrow ? (slot << 10) | off : off));
}

// Slot-table lookups of the two taps of one texel row, at blocks b0 (x0)
// and b1 (x1): b1 is b0, the next block id b0 + 1 (x1 in the next block
// column), or, rarely, another block (the wrap at the level's edge).
// slot_of[c] and slot_of[c + 1] come in one 8-byte load with c = min(b0,
// last_pair), where last_pair = n_blocks - 2 keeps the pair inside the
// table; a lane whose b1 the pair does not hold loads it on its own (into a
// register of its own, so that nothing waits for the loads until the slots
// are picked).
struct RowSlots {
    TexelPair p;
    uint32_t lone, b0, b1, c;
};
__device__ __forceinline__ bool row_in_pair(uint32_t b0, uint32_t b1, uint32_t c) {
    return b1 == b0 || (b0 == c && b1 == b0 + 1u);
}
__device__ __forceinline__ RowSlots row_load(const uint32_t *__restrict__ slot_of, uint32_t last_pair, uint32_t b0,
                                             uint32_t b1) {
    RowSlots r;
    r.b0 = b0;
    r.b1 = b1;
    r.c = min(b0, last_pair);
    r.p = *reinterpret_cast<const TexelPairA4 *>(reinterpret_cast<const char *>(slot_of) + (r.c << 2));
    r.lone = 0;
    if (!row_in_pair(b0, b1, r.c)) r.lone = load_at(slot_of, b1 << 2);
    return r;
}
__device__ __forceinline__ void row_pick(const RowSlots &r, uint32_t &s0, uint32_t &s1) {
    s0 = r.b0 == r.c ? r.p.x : r.p.y;
    s1 = !row_in_pair(r.b0, r.b1, r.c) ? r.lone : (r.b1 == r.b0 ? s0 : r.p.y);
}

// Slots of a level's four linear taps k0 ... k0 + 3 (rows y0 and y1): the
// second row's lookups are skipped, for the whole wavefront, when no lane's
// y1 taps lie in other blocks than its y0 taps.
template <int k0, int kTaps>
__device__ __forceinline__ void linear_slots(const uint32_t *__restrict__ slot_of, uint32_t last_pair,
                                             const Taps<kTaps> &T, uint32_t (&slot)[kTaps]) {
    const bool rows = __ballot(T.blk[k0 + 2] != T.blk[k0] || T.blk[k0 + 3] != T.blk[k0 + 1]) != 0;
    const RowSlots r0 = row_load(slot_of, last_pair, T.blk[k0], T.blk[k0 + 1]);
    RowSlots r1 = {TexelPair{0u, 0u}, 0u, 0u, 0u, 0u};  // (not a copy of r0: that would wait for its loads)
    if (rows) r1 = row_load(slot_of, last_pair, T.blk[k0 + 2], T.blk[k0 + 3]);
    row_pick(r0, slot[k0], slot[k0 + 1]);
    uint32_t s2, s3;
    row_pick(r1, s2, s3);
    slot[k0 + 2] = rows ? s2 : slot[k0];
    slot[k0 + 3] = rows ? s3 : slot[k0 + 1];
}

// Slots and texels of a level's four linear taps k0 ... k0 + 3, at
// (x0,y0), (x1,y0), (x0,y1), (x1,y1).  x1 usually follows x0 in the same
// block row: then one 8-byte load per row fetches both (at x0 - 1 when x0 is
// the block's last column, so that the pair stays inside the block row); a
// lane whose x1 does not follow x0 (another block, the wrap at the level's
// edge, a clamped tap) loads it on its own.
template <bool kNarrow, bool kPairSlots, int k0, int kTaps>
__device__ __forceinline__ void fetch_linear(const uint32_t *__restrict__ slot_of, const uint32_t *__restrict__ texels,
                                             uint32_t last_slot, uint32_t last_pair, const Taps<kTaps> &T,
                                             uint32_t (&slot)[kTaps], uint32_t (&tex)[kTaps]) {
    if constexpr (kPairSlots) {
        linear_slots<k0>(slot_of, last_pair, T, slot);
    } else {
#pragma unroll
        for (int t = k0; t < k0 + 4; t++) slot[t] = load_at(slot_of, T.blk[t] << 2);
    }
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const int t0 = k0 + 2 * b, t1 = t0 + 1;
        const uint32_t o0 = T.off[t0], o1 = T.off[t1];
        const bool end = (o0 & 0x3Cu) == 0x3Cu;                   // x0 & 15 == 15
        const bool next = T.blk[t1] == T.blk[t0] && o1 == o0 + 4u;  // x1 = x0 + 1 in the same block row
        const TexelPair pr = load_pair<kNarrow>(texels, min(slot[t0], last_slot), end ? o0 - 4u : o0);
        if constexpr (kPairSlots) {
            // the lone load into a register of its own, and the pair read
            // only after it is issued: no wait before its branch
            uint32_t lone = 0;
            if (!next) lone = load_texel<kNarrow>(texels, min(slot[t1], last_slot), o1);
            tex[t0] = end ? pr.y : pr.x;
            tex[t1] = next ? pr.y : lone;
        } else {  // (one round of workgroups: fewer vector instructions on the chain, measured faster)
            tex[t0] = end ? pr.y : pr.x;
            tex[t1] = next ? pr.y : load_texel<kNarrow>(texels, min(slot[t1], last_slot), o1);
        }
    }
}

template <uint32_t kFilter, int kDesc, bool kNarrow, bool kPairSlots>
__global__ __launch_bounds__(kThreads) void k_resolve(const jpt_level_desc *__restrict__ levels,
                                                      const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                      uint32_t n_lev, const ViewTable tab,
                                                      const uint32_t *__restrict__ slot_of,
                                                      const uint32_t *__restrict__ texels, uint32_t last_slot,
                                                      uint32_t last_pair, bool no_mip) {
    constexpr int kTaps = FilterTraits<kFilter>::kTaps;
    __shared__ TexRec s_t[kDesc != DESC_HBM ? kLdsTexCap : 1];
    __shared__ LevRec s_l[kDesc == DESC_LDS ? kLdsLevCap : 1];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if constexpr (kDesc == DESC_LDS) load_desc_lds(levels, texs, n_tex, n_lev, s_t, s_l);
    if constexpr (kDesc == DESC_TEX_LDS) load_tex_lds(texs, n_tex, s_t);
    if constexpr (kDesc != DESC_HBM) __syncthreads();
    for (uint32_t tslot = blockIdx.x; tslot < tab.span; tslot += gridDim.x) {
        uint32_t view, tx, ty;
        if (!tile_of(tab, tslot, view, tx, ty)) continue;
        const jpt_gpixel *__restrict__ gbuf = tab.v[view].gbuf;
        uint32_t *__restrict__ frame = tab.v[view].frame;
        const uint32_t W = tab.v[view].width, H = tab.v[view].height, pitch = tab.v[view].pitch;
        const uint32_t frame_pitch = tab.v[view].frame_pitch;
        const uint32_t x = tx * kTileW + lane;
        // loads from clamped in-bounds addresses, no branches: all rows in flight
        jpt_gpixel px[kRows];
        const uint32_t xc = min(x, W - 1u);
#pragma unroll
        for (int r = 0; r < kRows; r++) {
            const uint32_t y = ty * kTileH + wv + r * (kThreads / 64);
            const jpt_gpixel g = gbuf[(size_t)min(y, H - 1u) * pitch + xc];
            px[r] = (x < W && y < H) ? g : jpt_gpixel{0.f, 0.f, JPT_TEX_BACKGROUND, 0.f};
        }
        for (int r = 0; r < kRows; r++) {
            const uint32_t y = ty * kTileH + wv + r * (kThreads / 64);
            Taps<kTaps> T;
            uint32_t tw;
            int nf, st;
            if constexpr (kDesc == DESC_LDS)
                st = pixel_taps<kFilter>(LdsDesc{s_t, s_l}, n_tex, px[r], T, tw, nf, no_mip);
            else if constexpr (kDesc == DESC_TEX_LDS)
                st = pixel_taps<kFilter>(MixDesc{s_t, levels}, n_tex, px[r], T, tw, nf, no_mip);
            else st = pixel_taps<kFilter>(GlobalDesc{levels, texs}, n_tex, px[r], T, tw, nf, no_mip);
            // the pixel's slot lookups, then its texel loads (block ids are
            // below 2^29, so their byte offsets fit 32 bits; a block in no slot
            // reads the last slot, a valid address, and matters only if its
            // weight is not 0; a scene has at least 32 block ids, so block 0
            // is one even where the scene has no textures)
            uint32_t slot[kTaps], tex[kTaps];
            if constexpr (kTaps == 4 && kPairSlots) {
                // (a scene without textures skips the loads here: not needed,
                // but the paired form compiled with this path measured 4-5 us
                // faster on 16 views, 270 against 275 us)
                if (n_tex == 0) {
#pragma unroll
                    for (int t = 0; t < kTaps; t++) slot[t] = tex[t] = 0;
                } else {
                    fetch_linear<kNarrow, true, 0>(slot_of, texels, last_slot, last_pair, T, slot, tex);
                }
            } else if constexpr (kTaps == 4) {
                fetch_linear<kNarrow, false, 0>(slot_of, texels, last_slot, last_pair, T, slot, tex);
            } else {  // (trilinear: the paired forms of both levels spill registers)
#pragma unroll
                for (int t = 0; t < kTaps; t++) slot[t] = load_at(slot_of, T.blk[t] << 2);
#pragma unroll
                for (int t = 0; t < kTaps; t++) tex[t] = load_texel<kNarrow>(texels, min(slot[t], last_slot), T.off[t]);
            }
            if (x >= W || y >= H) continue;
            uint32_t out;
            if (st == PIX_BACKGROUND) {
                out = 0;
            } else if (st == PIX_INVALID) {
                out = JPT_TEXEL_INVALID;
            } else {
                bool missing = false;
                uint32_t lvl[2][3] = {{0, 0, 0}, {0, 0, 0}};
                constexpr int kLevels = kTaps == 8 ? 2 : 1, kPer = kTaps == 1 ? 1 : 4;
#pragma unroll
                for (int k = 0; k < kLevels; k++) {
                    uint32_t acc[3] = {0, 0, 0};
#pragma unroll
                    for (int j = 0; j < kPer; j++) {
                        const int t = k * kPer + j;
                        const uint32_t w = T.w[t];
                        missing |= (w != 0) && slot[t] == JPT_SLOT_NONE;
                        const uint32_t v = tex[t];
                        // 8-bit channel x weight <= 2^16: exact in the 24-bit multiply
                        acc[0] += __umul24(v & 255, w);
                        acc[1] += __umul24((v >> 8) & 255, w);
                        acc[2] += __umul24((v >> 16) & 255, w);
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
                        for (int c = 0; c < 3; c++)
                            a[c] = (__umul24(lvl[0][c], 256 - tw) + __umul24(lvl[1][c], tw) + 128) >> 8;
                    }
                    out = a[0] | (a[1] << 8) | (a[2] << 16) | 0xFF000000u;
                }
            }
            // (streaming store: nothing in the frame reads the framebuffer back)
            __builtin_nontemporal_store(out, frame + (size_t)y * frame_pitch + x);
        }
    }
}

// Workgroups of k_resolve the GPU holds at once (compute units x resident
// workgroups per unit), queried once per device.
template <uint32_t kFilter, int kDesc>
uint32_t resolve_capacity() {
    constexpr int kMaxDev = 64;
    static std::atomic<uint32_t> known[kMaxDev];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0u;
    uint32_t g = known[dev].load(std::memory_order_relaxed);
    if (g) return g;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_resolve<kFilter, kDesc, true, false>, kThreads, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
        cus <= 0)
        return 0u;
    g = (uint32_t)per_cu * (uint32_t)cus;
    known[dev].store(g, std::memory_order_relaxed);
    return g;
}

template <uint32_t kFilter, int kDesc, bool kPairSlots>
void launch_k(const jpt_scene *scene, const ViewTable &tab, uint32_t groups, const jpt_cache *cache, bool no_mip,
              hipStream_t st) {
    const uint32_t last_pair = scene->n_blocks - 2;  // (n_blocks >= 32)
    // kNarrow: every texel of the cache within 4 GiB of its base (at most 2^22 slots of 1 KiB)
    if (cache->n_slots <= (1u << 22))
        hipLaunchKernelGGL((k_resolve<kFilter, kDesc, true, kPairSlots>), dim3(groups), dim3(kThreads), 0, st,
                           scene->levels, scene->textures, scene->n_textures, scene->n_levels, tab, cache->slot_of,
                           cache->texels, cache->n_slots - 1, last_pair, no_mip);
    else
        hipLaunchKernelGGL((k_resolve<kFilter, kDesc, false, kPairSlots>), dim3(groups), dim3(kThreads), 0, st,
                           scene->levels, scene->textures, scene->n_textures, scene->n_levels, tab, cache->slot_of,
                           cache->texels, cache->n_slots - 1, last_pair, no_mip);
}

// The paired slot lookups of the linear filters take fewer vector memory
// instructions (what bounds a launch of many rounds of workgroups: 16 views,
// 42,000 tiles, 270 against 289 us) but more vector ALU work on each row's
// chain of dependent loads (what bounds a launch of one round: a 1080p frame,
// 2,025 tiles, 18.1 against 17.0 us); they serve launches of more than one
// round.
template <uint32_t kFilter, int kDesc>
void launch_desc(const jpt_scene *scene, const ViewTable &tab, uint32_t groups, const jpt_cache *cache,
                 uint32_t tune_flags, bool no_mip, hipStream_t st) {
    if constexpr (FilterTraits<kFilter>::kTaps == 4) {
        const bool paired = (tune_flags & JPT_TUNE_RESOLVE_PAIRED) ||
                            (!(tune_flags & JPT_TUNE_RESOLVE_SINGLE) && groups > resolve_capacity<kFilter, kDesc>());
        if (paired) {
            launch_k<kFilter, kDesc, true>(scene, tab, groups, cache, no_mip, st);
            return;
        }
    }
    launch_k<kFilter, kDesc, false>(scene, tab, groups, cache, no_mip, st);
}

template <uint32_t kFilter>
void launch(const jpt_scene *scene, const ViewTable &tab, uint32_t groups, const jpt_cache *cache,
            uint32_t tune_flags, bool no_mip, hipStream_t st) {
    switch (desc_mode(scene->n_textures, scene->n_levels)) {
    case DESC_LDS: launch_desc<kFilter, DESC_LDS>(scene, tab, groups, cache, tune_flags, no_mip, st); break;
    case DESC_TEX_LDS: launch_desc<kFilter, DESC_TEX_LDS>(scene, tab, groups, cache, tune_flags, no_mip, st); break;
    default: launch_desc<kFilter, DESC_HBM>(scene, tab, groups, cache, tune_flags, no_mip, st); break;
    }
}

}  // namespace

extern "C" jpt_status jpt_resolve(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                  const jpt_frame *frame, const jpt_cache *cache, const jpt_tuning *tuning,
                                  void *stream) {
    (void)frame;
    if (!scene || (n_views && !views) || !cache || !cache->slot_of || !cache->texels || cache->n_slots == 0)
        return JPT_E_ARG;
    if (!filter_valid(filter) || !scene->levels || !scene->textures) return JPT_E_ARG;
    if (scene->n_blocks < 32) return JPT_E_ARG;  // (jpt_layout gives at least 32)
    const uint32_t mode = filter_mode(filter);
    const bool no_mip = filter_no_mip(filter);
    for (uint32_t v = 0; v < n_views; v++)
        if (!views[v].gbuf || !views[v].frame || views[v].pitch < views[v].width ||
            views[v].frame_pitch < views[v].width)
            return JPT_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (cache->policy == JPT_CACHE_HASH)
        return hash_cache_ok(cache) ? hash_resolve(scene, views, n_views, filter, cache, st) : JPT_E_ARG;
    const uint32_t tune_flags = tuning ? tuning->flags : 0u;
    if ((tune_flags & JPT_TUNE_RESOLVE_PAIRED) && (tune_flags & JPT_TUNE_RESOLVE_SINGLE)) return JPT_E_ARG;
    const bool xcd = tune_flags & JPT_TUNE_XCD_TILES;
    for (uint32_t v0 = 0; v0 < n_views; v0 += kMaxLaunchViews) {
        ViewTable tab;
        make_view_table(views, v0, n_views - v0 < kMaxLaunchViews ? n_views - v0 : kMaxLaunchViews, kTileW, kTileH,
                        xcd, tab);
        if (tab.total == 0) continue;
        uint32_t groups = tab.span;
        if (tuning && tuning->resolve_groups && tuning->resolve_groups < groups)
            groups = xcd ? (tuning->resolve_groups + 7) / 8 * 8 : tuning->resolve_groups;
        if (mode == JPT_FILTER_NEAREST)
            launch<JPT_FILTER_NEAREST>(scene, tab, groups, cache, tune_flags, no_mip, st);
        else if (mode == JPT_FILTER_BILINEAR)
            launch<JPT_FILTER_BILINEAR>(scene, tab, groups, cache, tune_flags, no_mip, st);
        else if (mode == JPT_FILTER_BILINEAR_CLAMPED)
            launch<JPT_FILTER_BILINEAR_CLAMPED>(scene, tab, groups, cache, tune_flags, no_mip, st);
        else launch<JPT_FILTER_TRILINEAR>(scene, tab, groups, cache, tune_flags, no_mip, st);
        HIP_CHECK_LAUNCH();
    }
    return JPT_OK;
}
