// Resolve (paper: Method, "Resolve"): each pixel fetches its filter taps from
// the cache slots of their blocks and blends them with integer weights.
// Every tap a pixel reads was marked, so no clamping at undecoded MCU borders
// is needed (the footprint marking makes the result exact).
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace {

__device__ __forceinline__ bool fetch(const uint32_t *__restrict__ slot_of, const uint32_t *__restrict__ texels,
                                      const LevelFoot &F, uint32_t x, uint32_t y, uint32_t &t) {
    const uint32_t slot = slot_of[block_of(F, x, y)];
    if (slot == JPT_SLOT_NONE) return false;
    t = texels[(size_t)slot * 256 + (y & 15) * 16 + (x & 15)];
    return true;
}

// Weighted sum of one level's taps, rounded: (sum texel * w + 32768) >> 16.
__device__ __forceinline__ bool level_sample(const uint32_t *__restrict__ slot_of, const uint32_t *__restrict__ texels,
                                             const LevelFoot &F, uint32_t filter, uint32_t rgb[3]) {
    if (filter == JPT_FILTER_NEAREST) {
        uint32_t t;
        if (!fetch(slot_of, texels, F, F.x0, F.y0, t)) return false;
        rgb[0] = t & 255; rgb[1] = (t >> 8) & 255; rgb[2] = (t >> 16) & 255;
        return true;
    }
    const uint32_t wx[2] = {256 - F.fx, F.fx}, wy[2] = {256 - F.fy, F.fy};
    const uint32_t xs[2] = {F.x0, F.x1}, ys[2] = {F.y0, F.y1};
    uint32_t acc[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int a = 0; a < 2; a++) {
            const uint32_t w = wx[a] * wy[b];
            if (w == 0) continue;
            uint32_t t;
            if (!fetch(slot_of, texels, F, xs[a], ys[b], t)) return false;
            acc[0] += (t & 255) * w;
            acc[1] += ((t >> 8) & 255) * w;
            acc[2] += ((t >> 16) & 255) * w;
        }
#pragma unroll
    for (int c = 0; c < 3; c++) rgb[c] = (acc[c] + 32768u) >> 16;
    return true;
}

__global__ __launch_bounds__(256) void k_resolve(const jpt_level_desc *__restrict__ levels,
                                                 const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                 const jpt_gpixel *__restrict__ gbuf, uint32_t W, uint32_t H,
                                                 uint32_t pitch, uint32_t filter, const uint32_t *__restrict__ slot_of,
                                                 const uint32_t *__restrict__ texels, uint32_t *__restrict__ frame,
                                                 uint32_t frame_pitch) {
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t x = blockIdx.x * 16 + (wv & 1) * 8 + (lane & 7);
    const uint32_t y = blockIdx.y * 16 + (wv >> 1) * 8 + (lane >> 3);
    if (x >= W || y >= H) return;
    const jpt_gpixel px = gbuf[(size_t)y * pitch + x];
    LevelFoot foot[2];
    int nf;
    uint32_t tw;
    const int st = pixel_footprint(levels, texs, n_tex, px, filter, foot, nf, tw);
    uint32_t out;
    if (st == PIX_BACKGROUND) {
        out = 0;
    } else if (st == PIX_INVALID) {
        out = JPT_TEXEL_INVALID;
    } else {
        uint32_t a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
        bool ok = true;
        if (foot[0].lw) ok = level_sample(slot_of, texels, foot[0], filter, a);
        if (ok && nf == 2 && foot[1].lw) ok = level_sample(slot_of, texels, foot[1], filter, b);
        if (!ok) {
            out = JPT_TEXEL_INVALID;
        } else {
            if (nf == 2) {
#pragma unroll
                for (int c = 0; c < 3; c++) a[c] = (a[c] * (256 - tw) + b[c] * tw + 128) >> 8;
            }
            out = a[0] | (a[1] << 8) | (a[2] << 16) | 0xFF000000u;
        }
    }
    frame[(size_t)y * frame_pitch + x] = out;
}

}  // namespace

extern "C" jpt_status jpt_resolve(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                  const jpt_frame *frame, const jpt_cache *cache, const jpt_tuning *tuning,
                                  void *stream) {
    (void)frame;
    (void)tuning;
    if (!scene || (n_views && !views) || !cache || !cache->slot_of || !cache->texels) return JPT_E_ARG;
    if (filter > JPT_FILTER_TRILINEAR || !scene->levels || !scene->textures) return JPT_E_ARG;
    for (uint32_t v = 0; v < n_views; v++)
        if (!views[v].gbuf || !views[v].frame || views[v].pitch < views[v].width ||
            views[v].frame_pitch < views[v].width)
            return JPT_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (V.width == 0 || V.height == 0) continue;
        dim3 grid((V.width + 15) / 16, (V.height + 15) / 16);
        hipLaunchKernelGGL(k_resolve, grid, dim3(256), 0, st, scene->levels, scene->textures, scene->n_textures,
                           V.gbuf, V.width, V.height, V.pitch, filter, cache->slot_of, cache->texels, V.frame,
                           V.frame_pitch);
        HIP_CHECK_LAUNCH();
    }
    return JPT_OK;
}
