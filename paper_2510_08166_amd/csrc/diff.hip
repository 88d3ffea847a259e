// Differentiable form of the decode + resolve path: the frame as a function
// of the dequantised DCT coefficients F of the visible blocks, with the
// rounding and clamping of the 8-bit path removed (texel = M (IDCT F + (128,0,0)),
// chroma replicated; frame = filter weights x texels, the quantised weights
// of the integer resolve taken as constants), and its hand-written adjoint.
//
//   jpt_dequantize   F = coef * Q, natural order (the leaf of the form)
//   jpt_fwd_float    F -> float texels -> float frame
//   jpt_backward     dL/dframe -> dL/dtexel (resolve adjoint, deterministic
//                    fixed-point atomics in a unit set by max |dL/dframe|)
//                    -> colour adjoint, 2x2 chroma sum -> transposed IDCT
//                    -> dL/dF
//
// The 8x8 transforms are separable fp32 products with the 1-D basis
// P[u][x] = C(u)/2 cos((2x+1) u pi / 16) held in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev_common.h"

namespace {

constexpr int kItemCoefs = JPT_ITEMS_DU * 64;
// dL/dtexel accumulates in 64-bit fixed point, so that the sum does not
// depend on the order of the atomics.  The unit is 2^-shift with shift
// chosen per call from m = max |dL/dframe|: every tap product g w (w <= 1)
// is below 2^kFixBits units, so a texel's sum stays exact for up to
// 2^(63 - kFixBits) taps, and each product is rounded to m 2^-(kFixBits+1)
// or better, whatever the scale of the loss.
constexpr int kFixBits = 36;

// The unit exponent for a largest |dL/dframe| whose fp32 bits are mbits
// (m < 2^e with e from the biased exponent; m = 0 gives the smallest e).
__device__ __forceinline__ int fix_shift(uint32_t mbits) {
    const int e = (int)((mbits >> 23) & 255u) - 126;
    return kFixBits - e;
}

struct ZigZagD {
    uint8_t nat[64];
};
constexpr ZigZagD make_zz() {
    ZigZagD z{};
    int i = 0;
    for (int d = 0; d < 15; d++) {
        const int lo = d < 8 ? 0 : d - 7, hi = d < 8 ? d : 7;
        if (d & 1)
            for (int r = lo; r <= hi; r++) z.nat[i++] = (uint8_t)(r * 8 + d - r);
        else
            for (int r = hi; r >= lo; r--) z.nat[i++] = (uint8_t)(r * 8 + d - r);
    }
    return z;
}
__constant__ ZigZagD kZZ = make_zz();

__device__ __forceinline__ float cos16(int k) {
    const float c[9] = {1.0f, 0.980785280403230f, 0.923879532511287f, 0.831469612302545f, 0.707106781186548f,
                        0.555570233019602f, 0.382683432365090f, 0.195090322016128f, 0.0f};
    k &= 31;
    if (k > 16) k = 32 - k;
    return k > 8 ? -c[16 - k] : c[k];
}
__device__ __forceinline__ float basis1d(int u, int x) { return u == 0 ? 0.5f * cos16(4) : 0.5f * cos16((2 * x + 1) * u); }

struct ItemGeom {
    uint32_t slot;   // cache slot of the item's block (JPT_SLOT_NONE: skip)
    uint32_t s444;   // 1 for a 4:4:4 MCU (one quadrant of the block)
    uint32_t q;      // quadrant of a 4:4:4 MCU
    uint32_t present;
};

__device__ __forceinline__ ItemGeom item_geom(const jpt_level_desc *__restrict__ levels,
                                              const uint32_t *__restrict__ word_level, const uint32_t *__restrict__ work,
                                              const uint32_t *__restrict__ slot_of, uint32_t it) {
    const uint32_t w = work[it];
    const uint32_t b = (w & 0x7FFFFFFFu) >> 2, q = w & 3u;
    const jpt_level_desc *L = levels + word_level[b >> 5];
    ItemGeom g{slot_of[b], L->sampling == JPT_SAMPLING_444 ? 1u : 0u, q, 1u};
    if (g.s444) {
        const uint32_t r = b - L->blk_base, by = r / L->blk_cols, bx = r - by * L->blk_cols;
        const uint32_t mx = 2 * bx + (q & 1), my = 2 * by + (q >> 1);
        g.present = mx < L->mcu_cols && my < L->n_mcu / L->mcu_cols;
    }
    if (w >> 31) g.present = 0;
    return g;
}

// ----------------------------------------------------------- dequantise
__global__ __launch_bounds__(256) void k_dequant(const jpt_level_desc *__restrict__ levels,
                                                 const uint32_t *__restrict__ word_level,
                                                 const uint16_t *__restrict__ quant, const uint32_t *__restrict__ work,
                                                 const uint32_t *__restrict__ counters,
                                                 const int16_t *__restrict__ coef, float *__restrict__ F,
                                                 uint32_t max_items) {
    const uint64_t n = (uint64_t)min(counters[JPT_CTR_ITEMS], max_items) * kItemCoefs;
    for (uint64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const uint32_t it = (uint32_t)(i / kItemCoefs), r = (uint32_t)(i - (uint64_t)it * kItemCoefs);
        const uint32_t du = r >> 6, k = r & 63;  // k: zigzag position
        const uint32_t b = (work[it] & 0x7FFFFFFFu) >> 2;
        const jpt_level_desc *L = levels + word_level[b >> 5];
        const bool s444 = L->sampling == JPT_SAMPLING_444;
        const int comp = s444 ? (int)du : (du < 4 ? 0 : 1);
        float v = 0.0f;
        if (!(s444 && du >= 3)) v = (float)coef[(size_t)it * kItemCoefs + du * 64 + k] *
                                    (float)quant[(size_t)L->quant * 128 + (comp ? 64 : 0) + k];
        F[(size_t)it * kItemCoefs + du * 64 + kZZ.nat[k]] = v;
    }
}

// ------------------------------------------------------- float texels
// One wave per work item: the item's data units through the separable
// IDCT in LDS, then colour without rounding or clamping.
__global__ __launch_bounds__(64) void k_fwd_texels(const jpt_level_desc *__restrict__ levels,
                                                   const uint32_t *__restrict__ word_level,
                                                   const uint32_t *__restrict__ work,
                                                   const uint32_t *__restrict__ counters,
                                                   const uint32_t *__restrict__ slot_of, const float *__restrict__ F,
                                                   float *__restrict__ texel_f, uint32_t max_items) {
    __shared__ float s_P[64];
    __shared__ float s_F[kItemCoefs];
    __shared__ float s_T[64];
    __shared__ float s_S[kItemCoefs];
    const uint32_t t = threadIdx.x, r = t >> 3, c = t & 7;
    const uint32_t n_items = min(counters[JPT_CTR_ITEMS], max_items);
    s_P[t] = basis1d((int)(t >> 3), (int)(t & 7));  // P[u][x], u = t/8, x = t%8
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ItemGeom g = item_geom(levels, word_level, work, slot_of, it);
        if (g.slot == JPT_SLOT_NONE || !g.present) continue;  // uniform over the wave
        for (int i = t; i < kItemCoefs; i += 64) s_F[i] = F[(size_t)it * kItemCoefs + i];
        __syncthreads();
        const int ndu = g.s444 ? 3 : 6;
        for (int d = 0; d < ndu; d++) {
            // rows: T[v][x] = sum_u F[v][u] P[u][x]  (thread = (v, x))
            float a = 0.0f;
#pragma unroll
            for (int u = 0; u < 8; u++) a += s_F[d * 64 + r * 8 + u] * s_P[u * 8 + c];
            s_T[t] = a;
            __syncthreads();
            // columns: S[y][x] = sum_v P[v][y] T[v][x]  (thread = (y, x))
            float s = 0.0f;
#pragma unroll
            for (int v = 0; v < 8; v++) s += s_P[v * 8 + r] * s_T[v * 8 + c];
            s_S[d * 64 + t] = s;
            __syncthreads();
        }
        float *dst = texel_f + (size_t)g.slot * 768;
        // thread t owns chroma sample (r, c) and, for 4:2:0, the 2x2 texel
        // square it covers; for 4:4:4, texel (r, c) of the MCU's quadrant
        const int nsub = g.s444 ? 1 : 4;
        for (int k = 0; k < nsub; k++) {
            uint32_t ty, tx;
            float Y, Cb, Cr;
            if (!g.s444) {
                ty = 2 * r + (k >> 1); tx = 2 * c + (k & 1);
                Y = s_S[((ty >> 3) * 2 + (tx >> 3)) * 64 + (ty & 7) * 8 + (tx & 7)] + 128.0f;
                Cb = s_S[4 * 64 + t];
                Cr = s_S[5 * 64 + t];
            } else {
                ty = 8 * (g.q >> 1) + r; tx = 8 * (g.q & 1) + c;
                Y = s_S[t] + 128.0f; Cb = s_S[64 + t]; Cr = s_S[128 + t];
            }
            float *o = dst + (ty * 16 + tx) * 3;
            o[0] = Y + 1.402f * Cr;
            o[1] = Y - 0.344136f * Cb - 0.714136f * Cr;
            o[2] = Y + 1.772f * Cb;
        }
        __syncthreads();
    }
}

// ------------------------------------------------- float resolve / adjoint
// Taps of a pixel with their float weights (tap weight x level weight / 2^24).
// Tap k of a pixel: slot (JPT_SLOT_NONE: block without a slot), texel
// offset and weight; tap 4j + (2b + a) is texel (x_a, y_b) of level j, and
// an unused tap has weight 0 (fixed positions keep the arrays in registers).
struct FTaps {
    uint32_t slot[8], off[8];
    float w[8];
};

template <class Desc>
__device__ __forceinline__ int float_taps(const Desc &D, uint32_t n_tex, const jpt_gpixel &px, uint32_t filter_flags,
                                          const uint32_t *__restrict__ slot_of, FTaps &T) {
#pragma unroll
    for (int k = 0; k < 8; k++) { T.slot[k] = 0; T.off[k] = 0; T.w[k] = 0.0f; }
    LevelFoot foot[2];
    int nf;
    uint32_t tw;
    const uint32_t filter = filter_mode(filter_flags);
    const int st = pixel_footprint(D, n_tex, px, filter, foot, nf, tw, filter_no_mip(filter_flags));
    if (st != PIX_VALID) return st;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (k >= nf || foot[k].lw == 0) continue;
        const LevelFoot &F = foot[k];
        if (filter == JPT_FILTER_NEAREST) {
            T.slot[4 * k] = slot_of[block_of(F, F.x0, F.y0)];
            T.off[4 * k] = (F.y0 & 15) * 16 + (F.x0 & 15);
            T.w[4 * k] = (float)(65536u * F.lw) * (1.0f / 16777216.0f);
            continue;
        }
        const uint32_t wx[2] = {256 - F.fx, F.fx}, wy[2] = {256 - F.fy, F.fy};
        const uint32_t xs[2] = {F.x0, F.x1}, ys[2] = {F.y0, F.y1};
#pragma unroll
        for (int b2 = 0; b2 < 2; b2++)
#pragma unroll
            for (int a = 0; a < 2; a++) {
                const int t = 4 * k + 2 * b2 + a;
                const uint32_t w = wx[a] * wy[b2];
                if (w == 0) continue;
                T.slot[t] = slot_of[block_of(F, xs[a], ys[b2])];
                T.off[t] = (ys[b2] & 15) * 16 + (xs[a] & 15);
                T.w[t] = (float)(w * F.lw) * (1.0f / 16777216.0f);  // w * lw <= 2^24: exact
            }
    }
    return PIX_VALID;
}

template <bool kLdsDesc>
__global__ __launch_bounds__(256) void k_fwd_resolve(const jpt_level_desc *__restrict__ levels,
                                                     const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                     uint32_t n_lev, const jpt_gpixel *__restrict__ gbuf, uint32_t W,
                                                     uint32_t H, uint32_t pitch, uint32_t filter,
                                                     const uint32_t *__restrict__ slot_of,
                                                     const float *__restrict__ texel_f, float *__restrict__ frame_f,
                                                     uint32_t *__restrict__ counters) {
    __shared__ TexRec s_t[kLdsDesc ? kLdsTexCap : 1];
    __shared__ LevRec s_l[kLdsDesc ? kLdsLevCap : 1];
    if constexpr (kLdsDesc) {
        load_desc_lds(levels, texs, n_tex, n_lev, s_t, s_l);
        __syncthreads();
    }
    const uint32_t x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const jpt_gpixel px = gbuf[(size_t)y * pitch + x];
    FTaps T;
    int st;
    if constexpr (kLdsDesc) st = float_taps(LdsDesc{s_t, s_l}, n_tex, px, filter, slot_of, T);
    else st = float_taps(GlobalDesc{levels, texs}, n_tex, px, filter, slot_of, T);
    float acc[3] = {0.0f, 0.0f, 0.0f};
    bool bad = st == PIX_INVALID;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        if (T.w[k] == 0.0f) continue;
        if (T.slot[k] == JPT_SLOT_NONE) { bad = true; continue; }
        const float *tx = texel_f + (size_t)T.slot[k] * 768 + T.off[k] * 3;
        acc[0] += T.w[k] * tx[0];
        acc[1] += T.w[k] * tx[1];
        acc[2] += T.w[k] * tx[2];
    }
    float *o = frame_f + ((size_t)y * W + x) * 3;
    o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2];
    if (bad) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_PIXEL);
}

// Backward of the resolve: every tap adds weight x dL/dpixel to its texel's
// adjoint.  A workgroup takes a 64 x 8 pixel tile and first sums the adds of
// the tile in an LDS table keyed by texel (neighbouring pixels share texels),
// then flushes each touched texel with one global atomic per channel.  All
// sums are 64-bit fixed point, so the result does not depend on the order.
// The tile and its 1,024-entry table are sized so that three workgroups fit
// a compute unit (48 KB of LDS each with the descriptors): the flushes'
// atomics need the waves in flight more than they need fewer tile borders
// (1080p: 0.198 ms against 0.237 for 64 x 16 tiles at two workgroups).
constexpr int kAccLog2 = 10, kAccSize = 1 << kAccLog2, kAccProbes = 8, kBwdRows = 2;

__device__ __forceinline__ void acc_add(uint32_t *s_key, unsigned long long *s_val,
                                        unsigned long long *__restrict__ dtexel, uint32_t addr, long long a0,
                                        long long a1, long long a2) {
    uint32_t h = addr & (kAccSize - 1);
    for (int p = 0; p < kAccProbes; p++) {
        const uint32_t old = atomicCAS(s_key + h, 0xFFFFFFFFu, addr);
        if (old == 0xFFFFFFFFu || old == addr) {
            atomicAdd(s_val + 3 * h + 0, (unsigned long long)a0);
            atomicAdd(s_val + 3 * h + 1, (unsigned long long)a1);
            atomicAdd(s_val + 3 * h + 2, (unsigned long long)a2);
            return;
        }
        h = (h + 1) & (kAccSize - 1);
    }
    unsigned long long *d = dtexel + (size_t)addr * 3;  // table crowded: straight to HBM
    atomicAdd(d + 0, (unsigned long long)a0);
    atomicAdd(d + 1, (unsigned long long)a1);
    atomicAdd(d + 2, (unsigned long long)a2);
}

template <bool kLdsDesc>
__global__ __launch_bounds__(256) void k_bwd_resolve(const jpt_level_desc *__restrict__ levels,
                                                     const jpt_texture_desc *__restrict__ texs, uint32_t n_tex,
                                                     uint32_t n_lev, const jpt_gpixel *__restrict__ gbuf, uint32_t W,
                                                     uint32_t H, uint32_t pitch, uint32_t filter,
                                                     const uint32_t *__restrict__ slot_of,
                                                     const float *__restrict__ dframe,
                                                     unsigned long long *__restrict__ dtexel,
                                                     const uint32_t *__restrict__ counters) {
    __shared__ TexRec s_t[kLdsDesc ? kLdsTexCap : 1];
    __shared__ LevRec s_l[kLdsDesc ? kLdsLevCap : 1];
    __shared__ uint32_t s_key[kAccSize];
    __shared__ unsigned long long s_val[3 * kAccSize];
    if constexpr (kLdsDesc) load_desc_lds(levels, texs, n_tex, n_lev, s_t, s_l);
    for (int i = threadIdx.x; i < kAccSize; i += 256) s_key[i] = 0xFFFFFFFFu;
    for (int i = threadIdx.x; i < 3 * kAccSize; i += 256) s_val[i] = 0ull;
    __syncthreads();
    const int shift = fix_shift(counters[JPT_CTR_GRAD_MAX]);
    const uint32_t x = blockIdx.x * 64 + (threadIdx.x & 63);
    for (int r = 0; r < kBwdRows; r++) {
        const uint32_t y = blockIdx.y * (4 * kBwdRows) + r * 4 + (threadIdx.x >> 6);
        if (x >= W || y >= H) continue;
        const jpt_gpixel px = gbuf[(size_t)y * pitch + x];
        FTaps T;
        int st;
        if constexpr (kLdsDesc) st = float_taps(LdsDesc{s_t, s_l}, n_tex, px, filter, slot_of, T);
        else st = float_taps(GlobalDesc{levels, texs}, n_tex, px, filter, slot_of, T);
        if (st != PIX_VALID) continue;
        const float *g = dframe + ((size_t)y * W + x) * 3;
        const float g0 = g[0], g1 = g[1], g2 = g[2];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (T.w[k] == 0.0f || T.slot[k] == JPT_SLOT_NONE) continue;
            acc_add(s_key, s_val, dtexel, T.slot[k] * 256u + T.off[k], __float2ll_rn(ldexpf(g0 * T.w[k], shift)),
                    __float2ll_rn(ldexpf(g1 * T.w[k], shift)), __float2ll_rn(ldexpf(g2 * T.w[k], shift)));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAccSize; i += 256) {
        const uint32_t a = s_key[i];
        if (a == 0xFFFFFFFFu) continue;
        unsigned long long *d = dtexel + (size_t)a * 3;
        atomicAdd(d + 0, s_val[3 * i + 0]);
        atomicAdd(d + 1, s_val[3 * i + 1]);
        atomicAdd(d + 2, s_val[3 * i + 2]);
    }
}

// One wave per work item: colour adjoint, chroma 2x2 sum, transposed IDCT.
__global__ __launch_bounds__(64) void k_bwd_texels(const jpt_level_desc *__restrict__ levels,
                                                   const uint32_t *__restrict__ word_level,
                                                   const uint32_t *__restrict__ work,
                                                   const uint32_t *__restrict__ counters,
                                                   const uint32_t *__restrict__ slot_of,
                                                   const unsigned long long *__restrict__ dtexel,
                                                   float *__restrict__ dF, uint32_t max_items) {
    const int shift = fix_shift(counters[JPT_CTR_GRAD_MAX]);
    __shared__ float s_P[64];
    __shared__ float s_dS[kItemCoefs];  // dL/d(sample) per data unit, pixel order
    __shared__ float s_R[64];
    const uint32_t t = threadIdx.x, r = t >> 3, c = t & 7;
    const uint32_t n_items = min(counters[JPT_CTR_ITEMS], max_items);
    s_P[t] = basis1d((int)(t >> 3), (int)(t & 7));
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ItemGeom g = item_geom(levels, word_level, work, slot_of, it);
        float *out = dF + (size_t)it * kItemCoefs;
        if (g.slot == JPT_SLOT_NONE || !g.present) {
            for (int i = t; i < kItemCoefs; i += 64) out[i] = 0.0f;
            continue;
        }
        const unsigned long long *src = dtexel + (size_t)g.slot * 768;
        const int nsub = g.s444 ? 1 : 4;
        float sCb = 0.0f, sCr = 0.0f;
        for (int k = 0; k < nsub; k++) {
            uint32_t ty, tx;
            if (!g.s444) { ty = 2 * r + (k >> 1); tx = 2 * c + (k & 1); }
            else { ty = 8 * (g.q >> 1) + r; tx = 8 * (g.q & 1) + c; }
            const unsigned long long *d = src + (ty * 16 + tx) * 3;
            const float dR = ldexpf((float)(long long)d[0], -shift), dG = ldexpf((float)(long long)d[1], -shift),
                        dB = ldexpf((float)(long long)d[2], -shift);
            // adjoint of R = Y + 1.402 Cr, G = Y - .344136 Cb - .714136 Cr, B = Y + 1.772 Cb
            const float dY = dR + dG + dB;
            sCb += -0.344136f * dG + 1.772f * dB;  // a chroma sample feeds its whole 2x2 square
            sCr += 1.402f * dR - 0.714136f * dG;
            if (!g.s444) s_dS[((ty >> 3) * 2 + (tx >> 3)) * 64 + (ty & 7) * 8 + (tx & 7)] = dY;
            else s_dS[t] = dY;
        }
        s_dS[(g.s444 ? 1 : 4) * 64 + t] = sCb;
        s_dS[(g.s444 ? 2 : 5) * 64 + t] = sCr;
        __syncthreads();
        const int ndu = g.s444 ? 3 : 6;
        for (int d = 0; d < ndu; d++) {
            // R[y][u] = sum_x dS[y][x] P[u][x]   (thread = (y, u))
            float a = 0.0f;
#pragma unroll
            for (int x = 0; x < 8; x++) a += s_dS[d * 64 + r * 8 + x] * s_P[c * 8 + x];
            s_R[t] = a;
            __syncthreads();
            // dF[v][u] = sum_y P[v][y] R[y][u]   (thread = (v, u))
            float s = 0.0f;
#pragma unroll
            for (int y = 0; y < 8; y++) s += s_P[r * 8 + y] * s_R[y * 8 + c];
            out[d * 64 + t] = s;
            __syncthreads();
        }
        for (int i = ndu * 64 + t; i < kItemCoefs; i += 64) out[i] = 0.0f;
    }
}

// The largest |dL/dframe| over all views (fp32 bits; non-negative floats
// order as their bits), max-reduced into counters[JPT_CTR_GRAD_MAX]; a
// non-finite entry raises JPT_ERR_GRAD.  Each thread keeps 8 loads in
// flight; the workgroup (16 waves) reduces in registers and LDS and makes
// one atomic (at most 256 workgroups: atomics on one address serialise).
constexpr int kAbsUnroll = 8;
constexpr uint32_t kAbsGroups = 256, kAbsThreads = 1024;
__global__ __launch_bounds__(kAbsThreads) void k_absmax(const float *__restrict__ g, uint64_t n,
                                                        uint32_t *__restrict__ counters) {
    constexpr int kWaves = kAbsThreads / 64;
    __shared__ uint32_t s_m[kWaves], s_bad[kWaves];
    uint32_t m = 0;
    bool bad = false;
    const uint64_t stride = (uint64_t)gridDim.x * kAbsThreads;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kAbsThreads + threadIdx.x; i0 < n; i0 += stride * kAbsUnroll) {
        float v[kAbsUnroll];
#pragma unroll
        for (int u = 0; u < kAbsUnroll; u++) {
            const uint64_t i = i0 + (uint64_t)u * stride;
            v[u] = i < n ? fabsf(g[i]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kAbsUnroll; u++) {
            bad |= !(v[u] <= 3.4028234664e38f);
            m = max(m, __float_as_uint(v[u]));
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    const bool wbad = __ballot(bad) != 0;
    if ((threadIdx.x & 63) == 0) {
        s_m[threadIdx.x >> 6] = m;
        s_bad[threadIdx.x >> 6] = wbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t bm = 0, bb = 0;
        for (int w = 0; w < kWaves; w++) {
            bm = max(bm, s_m[w]);
            bb |= s_bad[w];
        }
        if (bb) atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_GRAD);
        if (bm && !bb) atomicMax(counters + JPT_CTR_GRAD_MAX, bm);
    }
}

// Clear the texel adjoints of the listed items' slots (a block's 16 x 16 x 3
// entries once: by its 4:2:0 item, or by quadrant 0 of a 4:4:4 block), and
// the largest-gradient counter.
__global__ __launch_bounds__(256) void k_zero_items(const jpt_level_desc *__restrict__ levels,
                                                    const uint32_t *__restrict__ word_level,
                                                    const uint32_t *__restrict__ work,
                                                    uint32_t *__restrict__ counters,
                                                    const uint32_t *__restrict__ slot_of,
                                                    unsigned long long *__restrict__ dtexel, uint32_t max_items) {
    const uint32_t n_items = min(counters[JPT_CTR_ITEMS], max_items);
    if (blockIdx.x == 0 && threadIdx.x == 0) counters[JPT_CTR_GRAD_MAX] = 0;
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint32_t w = work[it];
        const uint32_t b = (w & 0x7FFFFFFFu) >> 2, q = w & 3u;
        if (q != 0) continue;
        const uint32_t slot = slot_of[b];
        if (slot == JPT_SLOT_NONE) continue;
        unsigned long long *d = dtexel + (size_t)slot * 768;
        for (uint32_t i = threadIdx.x; i < 768; i += 256) d[i] = 0ull;
    }
}

bool desc_fits(const jpt_scene *s) { return s->n_textures <= kLdsTexCap && s->n_levels <= kLdsLevCap; }

jpt_status check(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                 const jpt_frame *frame, const jpt_cache *cache) {
    if (!scene || !frame || !cache || (n_views && !views) || !filter_valid(filter)) return JPT_E_ARG;
    if (!scene->levels || !scene->textures || !scene->word_level || !frame->work || !frame->counters ||
        !cache->slot_of)
        return JPT_E_ARG;
    for (uint32_t v = 0; v < n_views; v++)
        if (!views[v].gbuf || views[v].pitch < views[v].width) return JPT_E_ARG;
    return JPT_OK;
}

}  // namespace

static uint32_t row_limit(const jpt_frame *frame, uint32_t n_rows) { return n_rows < frame->max_items ? n_rows : frame->max_items; }

extern "C" jpt_status jpt_dequantize(const jpt_scene *scene, const jpt_frame *frame, float *F, uint32_t n_rows,
                                     void *stream) {
    if (!scene || !frame || !F || !scene->levels || !scene->word_level || !scene->quant || !frame->work ||
        !frame->counters || !frame->coef)
        return JPT_E_ARG;
    hipLaunchKernelGGL(k_dequant, dim3(1024), dim3(256), 0, (hipStream_t)stream, scene->levels, scene->word_level,
                       scene->quant, frame->work, frame->counters, frame->coef, F, row_limit(frame, n_rows));
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}

extern "C" jpt_status jpt_fwd_float(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                    const jpt_frame *frame, const jpt_cache *cache, const float *F, uint32_t n_rows,
                                    float *texel_f, float *frame_f, void *stream) {
    jpt_status s = check(scene, views, n_views, filter, frame, cache);
    if (s) return s;
    if (!F || !texel_f || !frame_f) return JPT_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fwd_texels, dim3(4096), dim3(64), 0, st, scene->levels, scene->word_level, frame->work,
                       frame->counters, cache->slot_of, F, texel_f, row_limit(frame, n_rows));
    HIP_CHECK_LAUNCH();
    size_t off = 0;
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (!V.width || !V.height) continue;
        dim3 grid((V.width + 63) / 64, (V.height + 3) / 4);
        if (desc_fits(scene))
            hipLaunchKernelGGL(k_fwd_resolve<true>, grid, dim3(256), 0, st, scene->levels, scene->textures,
                               scene->n_textures, scene->n_levels, V.gbuf, V.width, V.height, V.pitch, filter,
                               cache->slot_of, texel_f, frame_f + off, frame->counters);
        else
            hipLaunchKernelGGL(k_fwd_resolve<false>, grid, dim3(256), 0, st, scene->levels, scene->textures,
                               scene->n_textures, scene->n_levels, V.gbuf, V.width, V.height, V.pitch, filter,
                               cache->slot_of, texel_f, frame_f + off, frame->counters);
        HIP_CHECK_LAUNCH();
        off += (size_t)V.width * V.height * 3;
    }
    return JPT_OK;
}

extern "C" jpt_status jpt_backward(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                   const jpt_frame *frame, const jpt_cache *cache, const float *dframe,
                                   int64_t *dtexel, float *dF, uint32_t n_rows, void *stream) {
    jpt_status s = check(scene, views, n_views, filter, frame, cache);
    if (s) return s;
    if (!dframe || !dtexel || !dF || cache->n_slots == 0 || cache->n_slots >= (1u << 24)) return JPT_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *dt = reinterpret_cast<unsigned long long *>(dtexel);
    hipLaunchKernelGGL(k_zero_items, dim3(2048), dim3(256), 0, st, scene->levels, scene->word_level, frame->work,
                       frame->counters, cache->slot_of, dt, row_limit(frame, n_rows));
    HIP_CHECK_LAUNCH();
    size_t total = 0;
    for (uint32_t v = 0; v < n_views; v++) total += (size_t)views[v].width * views[v].height * 3;
    if (total)
        hipLaunchKernelGGL(k_absmax, dim3((uint32_t)std::min<size_t>((total + 8191) / 8192, kAbsGroups)),
                           dim3(kAbsThreads), 0, st, dframe, (uint64_t)total, frame->counters);
    HIP_CHECK_LAUNCH();
    size_t off = 0;
    for (uint32_t v = 0; v < n_views; v++) {
        const jpt_view &V = views[v];
        if (!V.width || !V.height) continue;
        dim3 grid((V.width + 63) / 64, (V.height + 4 * kBwdRows - 1) / (4 * kBwdRows));
        if (desc_fits(scene))
            hipLaunchKernelGGL(k_bwd_resolve<true>, grid, dim3(256), 0, st, scene->levels, scene->textures,
                               scene->n_textures, scene->n_levels, V.gbuf, V.width, V.height, V.pitch, filter,
                               cache->slot_of, dframe + off, dt, frame->counters);
        else
            hipLaunchKernelGGL(k_bwd_resolve<false>, grid, dim3(256), 0, st, scene->levels, scene->textures,
                               scene->n_textures, scene->n_levels, V.gbuf, V.width, V.height, V.pitch, filter,
                               cache->slot_of, dframe + off, dt, frame->counters);
        HIP_CHECK_LAUNCH();
        off += (size_t)V.width * V.height * 3;
    }
    hipLaunchKernelGGL(k_bwd_texels, dim3(4096), dim3(64), 0, st, scene->levels, scene->word_level, frame->work,
                       frame->counters, cache->slot_of, dt, dF, row_limit(frame, n_rows));
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}
