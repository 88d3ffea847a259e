// The fixed-rate baseline (paper: Background, BC1): textures stored as BC1
// blocks are sampled directly by the resolve, with no mark, decode or cache
// pass, so its per-frame cost is the resolve alone.  Each tap fetches the
// 8-byte block of its texel, widens the two RGB565 endpoints, forms the one
// palette entry its 2-bit index selects and blends the taps with the same
// integer weights as jpt_resolve.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace {

constexpr int kBc1Threads = 256;
constexpr int kBc1TileW = 64, kBc1TileH = 4;

// Sampling view of a BC1 scene for pixel_footprint (block ids unused).
struct Bc1Desc {
    const jpt_bc1_level *__restrict__ levels;
    const jpt_texture_desc *__restrict__ texs;
    JPT_DEV TexRec tex(uint32_t t) const { return TexRec{texs[t].first_level, texs[t].n_levels}; }
    JPT_DEV LevRec lev(uint32_t l) const { return LevRec{levels[l].width, levels[l].height, 0u, 0u}; }
};

__device__ __forceinline__ uint32_t widen565(uint32_t c, int ch) {
    if (ch == 0) { const uint32_t r = (c >> 11) & 31u; return (r << 3) | (r >> 2); }
    if (ch == 1) { const uint32_t g = (c >> 5) & 63u; return (g << 2) | (g >> 4); }
    const uint32_t b = c & 31u;
    return (b << 3) | (b >> 2);
}

// Texel (x, y) of a BC1 level as packed RGB (R low byte).
__device__ __forceinline__ uint32_t bc1_texel(const jpt_bc1_level &L, uint32_t x, uint32_t y) {
    const uint2 b = *reinterpret_cast<const uint2 *>(L.blocks + ((size_t)(y >> 2) * L.blocks_per_row + (x >> 2)) * 8);
    const uint32_t c0 = b.x & 0xFFFFu, c1 = b.x >> 16;
    const uint32_t k = (b.y >> (2 * (4 * (y & 3) + (x & 3)))) & 3u;
    uint32_t out = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        const uint32_t e0 = widen565(c0, ch), e1 = widen565(c1, ch);
        uint32_t v;
        if (k == 0) v = e0;
        else if (k == 1) v = e1;
        else if (c0 > c1) v = k == 2 ? (2 * e0 + e1 + 1) / 3 : (e0 + 2 * e1 + 1) / 3;
        else v = k == 2 ? (e0 + e1 + 1) / 2 : 0u;
        out |= v << (8 * ch);
    }
    return out;
}

template <uint32_t kFilter>
__global__ __launch_bounds__(kBc1Threads) void k_bc1_resolve(const jpt_bc1_level *__restrict__ levels,
                                                             const jpt_texture_desc *__restrict__ texs,
                                                             uint32_t n_tex, const jpt_gpixel *__restrict__ gbuf,
                                                             uint32_t W, uint32_t H, uint32_t pitch,
                                                             uint32_t *__restrict__ frame, uint32_t frame_pitch,
                                                             bool no_mip) {
    const uint32_t x = blockIdx.x * kBc1TileW + (threadIdx.x & 63);
    const uint32_t y = blockIdx.y * kBc1TileH + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const jpt_gpixel px = gbuf[(size_t)y * pitch + x];
    LevelFoot foot[2];
    int nf;
    uint32_t tw;
    const Bc1Desc D{levels, texs};
    const int st = pixel_footprint(D, n_tex, px, kFilter, foot, nf, tw, no_mip);
    uint32_t out;
    if (st == PIX_BACKGROUND) {
        out = 0;
    } else if (st == PIX_INVALID) {
        out = JPT_TEXEL_INVALID;
    } else {
        uint32_t lvl[2][3] = {{0, 0, 0}, {0, 0, 0}};
        for (int k = 0; k < nf; k++) {
            const LevelFoot &F = foot[k];
            const jpt_bc1_level Lv = levels[F.level];
            uint32_t acc[3] = {0, 0, 0};
            const uint32_t wx[2] = {256 - F.fx, F.fx}, wy[2] = {256 - F.fy, F.fy};
            const uint32_t xs[2] = {F.x0, F.x1}, ys[2] = {F.y0, F.y1};
            if (kFilter == JPT_FILTER_NEAREST) {
                const uint32_t v = bc1_texel(Lv, F.x0, F.y0);
#pragma unroll
                for (int c = 0; c < 3; c++) acc[c] = ((v >> (8 * c)) & 255u) << 16;
            } else {
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int a = 0; a < 2; a++) {
                        const uint32_t w = wx[a] * wy[b];
                        if (w == 0) continue;
                        const uint32_t v = bc1_texel(Lv, xs[a], ys[b]);
#pragma unroll
                        for (int c = 0; c < 3; c++) acc[c] += ((v >> (8 * c)) & 255u) * w;
                    }
            }
#pragma unroll
            for (int c = 0; c < 3; c++) lvl[k][c] = (acc[c] + 32768u) >> 16;
        }
        uint32_t a[3] = {lvl[0][0], lvl[0][1], lvl[0][2]};
        if (kFilter == JPT_FILTER_TRILINEAR && nf == 2) {
#pragma unroll
            for (int c = 0; c < 3; c++) a[c] = (lvl[0][c] * (256 - tw) + lvl[1][c] * tw + 128) >> 8;
        }
        out = a[0] | (a[1] << 8) | (a[2] << 16) | 0xFF000000u;
    }
    __builtin_nontemporal_store(out, frame + (size_t)y * frame_pitch + x);
}

}  // namespace

extern "C" jpt_status jpt_bc1_resolve(const jpt_bc1_scene *scene, const jpt_view *views, uint32_t n_views,
                                      uint32_t filter, void *stream) {
    if (!scene || (n_views && !views) || !scene->levels || !scene->textures || !filter_valid(filter) ||
        filter_mode(filter) == JPT_FILTER_BILINEAR_CLAMPED)
        return JPT_E_ARG;
    for (uint32_t v = 0; v < n_views; v++)
        if (!views[v].gbuf || !views[v].frame || views[v].pitch < views[v].width ||
            views[v].frame_pitch < views[v].width)
            return JPT_E_ARG;
    const uint32_t mode = filter_mode(filter);
    const bool no_mip = filter_no_mip(filter);
    hipStream_t st = (hipStream_t)stream;
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (!V.width || !V.height) continue;
        const dim3 grid((V.width + kBc1TileW - 1) / kBc1TileW, (V.height + kBc1TileH - 1) / kBc1TileH);
        if (mode == JPT_FILTER_NEAREST)
            hipLaunchKernelGGL(k_bc1_resolve<JPT_FILTER_NEAREST>, grid, dim3(kBc1Threads), 0, st, scene->levels,
                               scene->textures, scene->n_textures, V.gbuf, V.width, V.height, V.pitch, V.frame,
                               V.frame_pitch, no_mip);
        else if (mode == JPT_FILTER_BILINEAR)
            hipLaunchKernelGGL(k_bc1_resolve<JPT_FILTER_BILINEAR>, grid, dim3(kBc1Threads), 0, st, scene->levels,
                               scene->textures, scene->n_textures, V.gbuf, V.width, V.height, V.pitch, V.frame,
                               V.frame_pitch, no_mip);
        else
            hipLaunchKernelGGL(k_bc1_resolve<JPT_FILTER_TRILINEAR>, grid, dim3(kBc1Threads), 0, st, scene->levels,
                               scene->textures, scene->n_textures, V.gbuf, V.width, V.height, V.pitch, V.frame,
                               V.frame_pitch, no_mip);
        HIP_CHECK_LAUNCH();
    }
    return JPT_OK;
}
