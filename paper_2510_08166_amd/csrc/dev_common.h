// Device helpers shared by the mark and resolve kernels: level selection and
// filter footprints of one G-buffer pixel, in the exact fp32 arithmetic that
// jpt.h specifies (every product and sum rounded separately).
#pragma once
#include <hip/hip_runtime.h>

#include "jpt.h"
#include "jpt_internal.h"

#define JPT_DEV __device__ __forceinline__

// One level touched by a pixel: texel columns x0, x1 and rows y0, y1 with
// fractional weights fx, fy in [0,256] (linear filters) and the level's weight
// lw out of 256 (trilinear; 256 otherwise).  Taps of zero weight are skipped.
struct LevelFoot {
    uint32_t blk_base, blk_cols;
    uint32_t x0, x1, y0, y1;
    uint32_t fx, fy;
    uint32_t lw;
};

enum { PIX_BACKGROUND = 0, PIX_VALID = 1, PIX_INVALID = -1 };

JPT_DEV uint32_t wrap(int v, uint32_t n) {
    if ((n & (n - 1)) == 0) return (uint32_t)v & (n - 1);   // power of two: two's complement mask
    int r = v % (int)n;
    return (uint32_t)(r < 0 ? r + (int)n : r);
}

// Texel coordinate along one axis.  Returns false for a non-finite value or
// |s| >= 2^30.
JPT_DEV bool axis(float u, uint32_t n, bool linear, uint32_t &x0, uint32_t &x1, uint32_t &f) {
    float prod = __fmul_rn(u, (float)n);
    float s = linear ? __fsub_rn(prod, 0.5f) : prod;
    if (!(fabsf(s) < 1073741824.0f)) return false;
    float fl = floorf(s);
    if (linear) {
        float fr = __fsub_rn(s, fl);
        float sc = __fmul_rn(fr, 256.0f);
        float t = __fadd_rn(sc, 0.5f);
        f = (uint32_t)(int)floorf(t);
    } else {
        f = 0;
    }
    int xi = (int)fl;
    x0 = wrap(xi, n);
    x1 = wrap(xi + 1, n);
    return true;
}

// Levels and footprints of a pixel (up to two levels).  Returns PIX_*.
JPT_DEV int pixel_footprint(const jpt_level_desc *__restrict__ levels, const jpt_texture_desc *__restrict__ texs,
                            uint32_t n_tex, const jpt_gpixel &px, uint32_t filter, LevelFoot foot[2], int &nfoot,
                            uint32_t &tw) {
    nfoot = 0;
    tw = 0;
    if (px.tex == JPT_TEX_BACKGROUND) return PIX_BACKGROUND;
    if (px.tex >= n_tex) return PIX_INVALID;
    if (!isfinite(px.u) || !isfinite(px.v) || !isfinite(px.lod)) return PIX_INVALID;
    const jpt_texture_desc td = texs[px.tex];
    const int L = (int)td.n_levels;
    if (L <= 0) return PIX_INVALID;
    int lv[2];
    uint32_t lw[2];
    int nl;
    if (filter == JPT_FILTER_TRILINEAR) {
        float lod = px.lod;
        if (lod < 0.0f) {
            lv[0] = 0; nl = 1; lw[0] = 256;
        } else if (lod >= (float)(L - 1)) {
            lv[0] = L - 1; nl = 1; lw[0] = 256;
        } else {
            float fl = floorf(lod);
            float fr = __fsub_rn(lod, fl);
            float sc = __fmul_rn(fr, 256.0f);
            float t = __fadd_rn(sc, 0.5f);
            tw = (uint32_t)(int)floorf(t);
            lv[0] = (int)fl; lv[1] = lv[0] + 1; nl = 2;
            lw[0] = 256 - tw; lw[1] = tw;
        }
    } else {
        float t = __fadd_rn(px.lod, 0.5f);
        int l;
        if (!(t >= 1.0f)) l = 0;
        else if (t >= (float)(L - 1)) l = L - 1;
        else l = (int)floorf(t);
        lv[0] = l; nl = 1; lw[0] = 256;
    }
    const bool linear = filter != JPT_FILTER_NEAREST;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (k >= nl) break;
        LevelFoot &F = foot[k];
        const jpt_level_desc *ld = levels + td.first_level + lv[k];
        const uint32_t w = ld->width, h = ld->height;
        F.blk_base = ld->blk_base;
        F.blk_cols = ld->blk_cols;
        F.lw = lw[k];
        if (!axis(px.u, w, linear, F.x0, F.x1, F.fx) || !axis(px.v, h, linear, F.y0, F.y1, F.fy))
            return PIX_INVALID;
    }
    nfoot = nl;
    return PIX_VALID;
}

JPT_DEV uint32_t block_of(const LevelFoot &F, uint32_t x, uint32_t y) {
    return F.blk_base + (y >> 4) * F.blk_cols + (x >> 4);
}

#define HIP_CHECK_LAUNCH()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return JPT_E_HIP; \
    } while (0)
