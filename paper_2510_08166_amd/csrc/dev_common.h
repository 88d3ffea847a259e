// Device helpers shared by the mark and resolve kernels: level selection and
// filter footprints of one G-buffer pixel, in the exact fp32 arithmetic that
// jpt.h specifies (every product and sum rounded separately).
#pragma once
#include <hip/hip_runtime.h>

#include "jpt.h"
#include "jpt_internal.h"

#define JPT_DEV __device__ __forceinline__
#define JPT_DEV_HOST_INLINE __host__ __device__ __forceinline__

// One level touched by a pixel: texel columns x0, x1 and rows y0, y1 with
// fractional weights fx, fy in [0,256] (linear filters) and the level's weight
// lw out of 256 (trilinear; 256 otherwise).  Taps of zero weight are skipped.
struct LevelFoot {
    uint32_t level;  // index into the scene's level array
    uint32_t blk_base, blk_cols;
    uint32_t x0, x1, y0, y1;
    uint32_t fx, fy;
    uint32_t lw;
};

enum { PIX_BACKGROUND = 0, PIX_VALID = 1, PIX_INVALID = -1 };

// Non-negative v mod n for sizes that are not powers of two: an out-of-line
// call, so that the common power-of-two case costs no division code.
static __device__ __noinline__ uint32_t wrap_general(int v, uint32_t n) {
    const int r = v % (int)n;
    return (uint32_t)(r < 0 ? r + (int)n : r);
}

JPT_DEV uint32_t wrap(int v, uint32_t n) {
    if (__builtin_expect((n & (n - 1)) == 0, 1)) return (uint32_t)v & (n - 1);  // two's complement mask
    return wrap_general(v, n);
}

// Texel coordinate along one axis.  Returns false for a non-finite value or
// |s| >= 2^30 (the outputs are then meaningless but harmless).
JPT_DEV bool axis(float u, uint32_t n, bool linear, uint32_t &x0, uint32_t &x1, uint32_t &f) {
    float prod = __fmul_rn(u, (float)n);
    float s = linear ? __fsub_rn(prod, 0.5f) : prod;
    const bool ok = fabsf(s) < 1073741824.0f;
    float fl = floorf(s);
    if (linear) {
        float fr = __fsub_rn(s, fl);
        float sc = __fmul_rn(fr, 256.0f);
        float t = __fadd_rn(sc, 0.5f);
        f = (uint32_t)(int)floorf(t);
    } else {
        f = 0;
    }
    x0 = wrap(ok ? (int)fl : 0, n);
    x1 = x0 + 1 == n ? 0u : x0 + 1;  // (x + 1) mod n
    return ok;
}

// Sampling view of the scene descriptors: texture -> (first level, level
// count); level -> (width, height, first block id, blocks per row).
struct TexRec { uint32_t first, n; };
struct LevRec { uint32_t w, h, blk_base, blk_cols; };

// Descriptors read from HBM.
struct GlobalDesc {
    const jpt_level_desc *__restrict__ levels;
    const jpt_texture_desc *__restrict__ texs;
    JPT_DEV TexRec tex(uint32_t t) const { return TexRec{texs[t].first_level, texs[t].n_levels}; }
    JPT_DEV LevRec lev(uint32_t l) const {
        const jpt_level_desc *d = levels + l;
        return LevRec{d->width, d->height, d->blk_base, d->blk_cols};
    }
};

// Descriptors copied into LDS by the workgroup (small scenes).
struct LdsDesc {
    const TexRec *t;
    const LevRec *l;
    JPT_DEV TexRec tex(uint32_t i) const { return t[i]; }
    JPT_DEV LevRec lev(uint32_t i) const { return l[i]; }
};

// Texture records in LDS, level records read from HBM (scenes with more
// levels than the LDS cache holds).
struct MixDesc {
    const TexRec *t;
    const jpt_level_desc *__restrict__ levels;
    JPT_DEV TexRec tex(uint32_t i) const { return t[i]; }
    JPT_DEV LevRec lev(uint32_t l) const {
        const jpt_level_desc *d = levels + l;
        return LevRec{d->width, d->height, d->blk_base, d->blk_cols};
    }
};

// LDS capacity of the descriptor cache of mark and resolve, and the modes:
// every record in HBM, texture records in LDS, or every record in LDS.
constexpr uint32_t kLdsTexCap = 512, kLdsLevCap = 1024;
enum { DESC_HBM = 0, DESC_TEX_LDS = 1, DESC_LDS = 2 };
inline int desc_mode(uint32_t n_tex, uint32_t n_lev) {
    return n_tex > kLdsTexCap ? DESC_HBM : (n_lev > kLdsLevCap ? DESC_TEX_LDS : DESC_LDS);
}

// Copy the texture records into LDS (all threads; the caller synchronises).
JPT_DEV void load_tex_lds(const jpt_texture_desc *__restrict__ texs, uint32_t n_tex, TexRec *s_t) {
    for (uint32_t i = threadIdx.x; i < n_tex; i += blockDim.x) s_t[i] = TexRec{texs[i].first_level, texs[i].n_levels};
}

// Copy the descriptors into LDS (all threads of the block take part; the
// caller synchronises).
JPT_DEV void load_desc_lds(const jpt_level_desc *__restrict__ levels, const jpt_texture_desc *__restrict__ texs,
                           uint32_t n_tex, uint32_t n_lev, TexRec *s_t, LevRec *s_l) {
    for (uint32_t i = threadIdx.x; i < n_tex; i += blockDim.x) s_t[i] = TexRec{texs[i].first_level, texs[i].n_levels};
    for (uint32_t i = threadIdx.x; i < n_lev; i += blockDim.x) {
        const jpt_level_desc *d = levels + i;
        s_l[i] = LevRec{d->width, d->height, d->blk_base, d->blk_cols};
    }
}

// Levels and footprints of a pixel (up to two levels).  Returns PIX_*.
// Filter modes and flags of the C ABI, split.
JPT_DEV_HOST_INLINE uint32_t filter_mode(uint32_t f) { return f & 0xFFu; }
JPT_DEV_HOST_INLINE bool filter_no_mip(uint32_t f) { return (f & JPT_FILTER_MIP_OFF) != 0; }
inline bool filter_valid(uint32_t f) { return filter_mode(f) <= JPT_FILTER_BILINEAR_CLAMPED && (f & ~0x1FFu) == 0; }

// Branch-free over the lanes of a wave: every lane computes with clamped
// descriptor indices and the checks only pick the status at the end.
// `filter` is a JPT_FILTER_* mode; with no_mip every pixel samples level 0
// (JPT_FILTER_MIP_OFF).  JPT_FILTER_BILINEAR_CLAMPED takes the bilinear
// taps and moves a tap that lies outside the 16x16 block of the texel under
// the sample point (the nearest filter's texel) onto that texel's column or
// row, so that every tap, and the footprint, is that one block.
template <class Desc>
JPT_DEV int pixel_footprint(const Desc &D, uint32_t n_tex, const jpt_gpixel &px, uint32_t filter, LevelFoot foot[2],
                            int &nfoot, uint32_t &tw, bool no_mip = false) {
    nfoot = 0;
    tw = 0;
    const bool bg = px.tex == JPT_TEX_BACKGROUND;
    if (n_tex == 0) return bg ? PIX_BACKGROUND : PIX_INVALID;  // (uniform)
    bool ok = px.tex < n_tex && isfinite(px.u) && isfinite(px.v) && isfinite(px.lod);
    const TexRec td = D.tex(px.tex < n_tex ? px.tex : 0u);
    const int L = no_mip && td.n > 0 ? 1 : (int)td.n;
    ok = ok && L > 0;
    int lv0, nl;
    uint32_t lw0, lw1 = 0;
    if (filter == JPT_FILTER_TRILINEAR) {
        const float lod = px.lod;
        const float fl = floorf(lod);
        const float fr = __fsub_rn(lod, fl);
        const float sc = __fmul_rn(fr, 256.0f);
        const float t = __fadd_rn(sc, 0.5f);
        const uint32_t twi = (uint32_t)(int)floorf(t);
        const bool lo = lod < 0.0f, hi = lod >= (float)(L - 1);
        const bool two = !lo && !hi;
        lv0 = lo ? 0 : (hi ? L - 1 : (int)fl);
        nl = two ? 2 : 1;
        tw = two ? twi : 0u;
        lw0 = two ? 256u - twi : 256u;
        lw1 = twi;
    } else {
        const float t = __fadd_rn(px.lod, 0.5f);
        lv0 = !(t >= 1.0f) ? 0 : (t >= (float)(L - 1) ? L - 1 : (int)floorf(t));
        nl = 1;
        lw0 = 256;
    }
    const bool linear = filter != JPT_FILTER_NEAREST;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (k == 1 && filter != JPT_FILTER_TRILINEAR) break;
        LevelFoot &F = foot[k];
        // (a second level exists only when lv0 + 1 <= L - 1)
        const uint32_t li = ok ? td.first + (uint32_t)(k == 0 ? lv0 : min(lv0 + 1, L - 1)) : 0u;
        const LevRec lr = D.lev(li);
        F.level = li;
        F.blk_base = lr.blk_base;
        F.blk_cols = lr.blk_cols;
        F.lw = k == 0 ? lw0 : lw1;
        const bool ax = axis(px.u, lr.w, linear, F.x0, F.x1, F.fx);
        const bool ay = axis(px.v, lr.h, linear, F.y0, F.y1, F.fy);
        if (filter == JPT_FILTER_BILINEAR_CLAMPED) {
            uint32_t xc, yc, d0, d1, f0;
            axis(px.u, lr.w, false, xc, d0, f0);
            axis(px.v, lr.h, false, yc, d1, f0);
            F.x0 = (F.x0 >> 4) == (xc >> 4) ? F.x0 : xc;
            F.x1 = (F.x1 >> 4) == (xc >> 4) ? F.x1 : xc;
            F.y0 = (F.y0 >> 4) == (yc >> 4) ? F.y0 : yc;
            F.y1 = (F.y1 >> 4) == (yc >> 4) ? F.y1 : yc;
        }
        if (k < nl) ok = ok && ax && ay;
    }
    if (bg) return PIX_BACKGROUND;
    if (!ok) {
        tw = 0;
        return PIX_INVALID;
    }
    nfoot = nl;
    return PIX_VALID;
}

// Block id of texel (x, y).  Levels are at most 65535 texels on a side, so
// both factors fit 24 bits and the full-rate 24-bit multiply is exact.
JPT_DEV uint32_t block_of(const LevelFoot &F, uint32_t x, uint32_t y) {
    return F.blk_base + __umul24(y >> 4, F.blk_cols) + (x >> 4);
}

// ------------------------------------------------------------ view tables
// One launch of mark or resolve covers the pixel tiles of up to
// kMaxLaunchViews views.  Tiles are numbered view by view, row-major inside
// a view.  With `xcd_chunk` set, launch slot s (workgroup s, or its k-th
// step in a strided loop with a stride that is a multiple of 8) serves tile
// (s % 8) * xcd_chunk + s / 8: the hardware deals workgroups to the 8 XCDs
// round-robin, so each XCD (and its L2) gets a contiguous run of tiles.
constexpr uint32_t kMaxLaunchViews = 16;

struct LaunchView {
    const jpt_gpixel *gbuf;
    uint32_t *frame;
    uint32_t width, height, pitch, frame_pitch;
    uint32_t tiles_x, tile_end;  // tiles per row; first tile of the next view
};

struct ViewTable {
    uint32_t n, total;  // views, tiles
    uint32_t span;      // launch slots: total, or 8 * xcd_chunk
    uint32_t xcd_chunk;
    LaunchView v[kMaxLaunchViews];
};

// Tile of launch slot `s`: view, tile column and row.  False for a padding
// slot.  The view search ends at the last view with tiles (tile_end = total).
JPT_DEV bool tile_of(const ViewTable &T, uint32_t s, uint32_t &view, uint32_t &tx, uint32_t &ty) {
    const uint32_t t = T.xcd_chunk ? (s & 7u) * T.xcd_chunk + (s >> 3) : s;
    if (t >= T.total) return false;
    uint32_t v = 0;
    while (t >= T.v[v].tile_end) v++;
    const uint32_t lt = t - (v ? T.v[v - 1].tile_end : 0u);
    ty = lt / T.v[v].tiles_x;
    tx = lt - ty * T.v[v].tiles_x;
    view = v;
    return true;
}

// Host side: fill a table with views [first, first + n) (n <= kMaxLaunchViews)
// for tiles of tw x th pixels; views without pixels get no tiles.
inline void make_view_table(const jpt_view *views, uint32_t first, uint32_t n, uint32_t tw, uint32_t th, bool xcd,
                            ViewTable &T) {
    T.n = n;
    uint32_t total = 0;
    for (uint32_t i = 0; i < kMaxLaunchViews; i++) {
        LaunchView &L = T.v[i];
        if (i < n) {
            const jpt_view &V = views[first + i];
            L.gbuf = V.gbuf; L.frame = V.frame;
            L.width = V.width; L.height = V.height; L.pitch = V.pitch; L.frame_pitch = V.frame_pitch;
            L.tiles_x = (V.width + tw - 1) / tw;
            total += (V.width && V.height) ? L.tiles_x * ((V.height + th - 1) / th) : 0u;
        } else {
            L = LaunchView{nullptr, nullptr, 0, 0, 0, 0, 1, 0};
        }
        L.tile_end = total;
    }
    T.total = total;
    T.xcd_chunk = xcd ? (total + 7) / 8 : 0u;
    T.span = xcd ? 8 * T.xcd_chunk : total;
}

#define HIP_CHECK_LAUNCH()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return JPT_E_HIP; \
    } while (0)
