// Decode (paper: Method, "Decode"; Implementation details, "Warp-Level
// Parallel Huffman Decoding").
//
// k_entropy: one lane per MCU.  The paper gives each MCU a 64-thread block
// that matches codes with a warp ballot; on wave64 hardware that leaves 63
// lanes idle per symbol, so here a lane walks its own MCU's symbol chain with
// a 10-bit lookup table in LDS (code, run, size and, when they fit, the
// appended value bits in one entry) and a canonical fallback for longer
// codes.  Coefficients go to a per-lane LDS tile (6 x 64 int16, zigzag
// order), which the wave then copies to HBM with coalesced 16-byte stores.
//
// k_idct_mfma: dequantise and inverse-DCT every 8x8 unit as one 64x64
// contraction X = K F (K = basis with its columns in zigzag order) on the
// matrix cores (v_mfma_f32_32x32x16_f16), 32 units per column tile.  K is
// split into fp16 hi + lo parts (lo scaled by 2^11) accumulated in fp32;
// F (integer, |F| <= 2048 for real encoders) is exact in fp16, and larger
// values take an exact hi/lo split of F as well.  Then +128, clamp,
// chroma replication and JFIF YCbCr -> RGB with one rounding, RGBA8 into
// the block's cache slot.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

constexpr int kItemCoefs = JPT_ITEMS_DU * 64;  // int16 per work item

__device__ __forceinline__ int sext12(uint32_t v) { return (int)(v << 20) >> 20; }
// branch-free select (c is 0 or 1)
__device__ __forceinline__ int bsel(uint32_t c, int a, int b) { return b ^ ((a ^ b) & -(int)c); }

// ------------------------------------------------------------- entropy
typedef const __attribute__((address_space(1))) uint32_t *gu32;

// Codes longer than the fast-table index: canonical decoding (the first
// length whose largest code is >= the prefix), returned in the fast-entry
// format without the value, or JPT_FE_BAD for no code / an invalid symbol.
__device__ __noinline__ uint32_t slow_entry(const uint32_t *tab, uint32_t tsel, uint32_t peek) {
    const uint32_t *sl = tab + JPT_SLOW_OFFSET + tsel * JPT_SLOW_WORDS;
    for (int c = JPT_FAST_BITS + 1; c <= 16; c++) {
        const uint32_t code = peek >> (32 - c);
        if ((int)code <= (int)sl[c]) {
            const uint32_t si = (code + sl[17 + c]) & 255u;
            const uint32_t sym = (sl[34 + (si >> 2)] >> ((si & 3) * 8)) & 0xFFu;
            uint32_t run, size;
            bool bad;
            if (tsel & 1) {
                run = sym >> 4; size = sym & 15;
                bad = size > 10 || (size == 0 && run != 0 && run != 15);
            } else {
                run = 0; size = sym;
                bad = size > 11;
            }
            return bad ? JPT_FE_BAD : ((uint32_t)c | (size << 6) | (run << 10));
        }
    }
    return JPT_FE_BAD;
}

// The table entry of the symbol that starts at the top of `peek` in table t
// (0 DC luma, 1 AC luma, 3 AC chroma): the 10-bit fast table, or the direct
// table of the long codes; entries that neither resolves come from the
// canonical fallback (never for tables whose long codes fit the direct
// table, so this stays off the common path).
__device__ __forceinline__ uint32_t fast_entry(const uint32_t *tab, uint32_t t, uint32_t thr, uint32_t peek) {
    const uint32_t p16 = peek >> 16;
    const uint32_t e1 = tab[t * JPT_FAST_SIZE + (peek >> (32 - JPT_FAST_BITS))];
    const uint32_t e2 = tab[JPT_LONG_OFFSET + t * JPT_LONG_SIZE + min(p16 - thr, (uint32_t)JPT_LONG_SIZE - 1u)];
    return p16 >= thr ? e2 : e1;
}

// Packed for the chain walk: bits 0-4 bits the symbol takes with its
// appended bits (0: no valid code), 5-8 run, 9-12 size, 16-31 the
// coefficient value (or DC difference).
__device__ __forceinline__ uint32_t pack_entry(uint32_t e, uint32_t peek) {
    const uint32_t len = e & 31u, size = (e >> 6) & 15u, run = (e >> 10) & 15u;
    const uint32_t fused = (e >> 5) & 1u;
    const uint32_t extra = (uint32_t)(((uint64_t)(peek << len) << size) >> 32);
    const uint32_t lim = (1u << size) >> 1;
    const int vn = (int)extra - (int)(extra < lim ? (1u << size) - 1u : 0u);
    const int value = bsel(fused, (int)e >> 16, vn);
    const uint32_t used = len + (fused ? 0u : size);
    const bool bad = len == 0 || (e & JPT_FE_BAD);
    return bad ? 0u : (used | (run << 5) | (size << 9) | ((uint32_t)value << 16));
}

// k_entropy: one wavefront per MCU.  Per step the wave covers the next 64
// bit positions of the MCU's stream: lane i decodes, from its own bit offset
// i, the symbol that would start there under each of the three tables the
// MCU can be in (DC luma, AC luma, AC chroma), all lookups in flight at
// once.  The scalar unit then walks the true symbol chain through these
// speculative decodes (readlane of the lane at the current offset), applies
// the decoder state (data unit, zigzag position, Y DC predictor) and hands
// each coefficient back to the lane that decoded it; those lanes write them
// to the MCU's LDS tile in one store.  About a dozen symbols per step
// instead of one.  The MCU's first 128 words sit in two VGPRs across the
// wave and reach the scalar unit by readlane.
constexpr int kEntWaves = 4;  // MCUs in flight per workgroup

// Orders the LDS accesses of one wavefront before and after this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool kLdsTables>
__global__ __launch_bounds__(64 * kEntWaves) void k_entropy(const jpt_level_desc *__restrict__ levels,
                                                            const uint32_t *__restrict__ word_level,
                                                            const uint32_t *__restrict__ tables,
                                                            uint32_t *__restrict__ work,
                                                            uint32_t *__restrict__ counters,
                                                            int16_t *__restrict__ coef) {
    __shared__ __attribute__((aligned(16))) uint32_t s_tab[kLdsTables ? JPT_TABLESET_WORDS : 4];
    __shared__ __attribute__((aligned(16))) int16_t s_coef[kEntWaves][kItemCoefs];
    // the wave index is uniform over the wave: say so, so that the MCU state
    // lives in scalar registers and the chain walk runs on the scalar unit
    const uint32_t lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t n_items = counters[JPT_CTR_ITEMS];
    if (blockIdx.x * (uint32_t)kEntWaves >= n_items) return;
    if constexpr (kLdsTables) {
        static_assert(JPT_TABLESET_WORDS % 4 == 0, "table set must split into uint4");
        const uint4 *src = reinterpret_cast<const uint4 *>(tables);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
#pragma unroll 7
        for (int i = threadIdx.x; i < JPT_TABLESET_WORDS / 4; i += 64 * kEntWaves) dst[i] = src[i];
        __syncthreads();
    }
    int16_t *cf = s_coef[wv];
    for (uint32_t item = blockIdx.x * kEntWaves + wv; item < n_items; item += gridDim.x * kEntWaves) {
        // ---- locate the MCU (all wave-uniform): level, record, bit span, absolute DCs
        const uint32_t w = work[item];
        const uint32_t b = (w & 0x7FFFFFFFu) >> 2, q = w & 3u;
        const jpt_level_desc *L = levels + word_level[b >> 5];
        const uint32_t blk_base = L->blk_base, blk_cols = L->blk_cols, mcu_cols = L->mcu_cols;
        const uint32_t n_mcu = L->n_mcu;
        const bool s444 = L->sampling == JPT_SAMPLING_444;
        const gu32 stream = (gu32)L->stream;
        const gu32 recs = (gu32)L->records;
        const uint32_t stream_bits = (uint32_t)L->stream_bits;
        const uint32_t *tab = kLdsTables ? s_tab : tables + (size_t)L->table_set * JPT_TABLESET_WORDS;
        const uint32_t r = b - blk_base, by = r / blk_cols, bx = r - by * blk_cols;
        uint32_t mcu;
        bool active = true;
        if (s444) {
            const uint32_t mx = 2 * bx + (q & 1), my = 2 * by + (q >> 1);
            active = mx < mcu_cols && my < n_mcu / mcu_cols;
            mcu = my * mcu_cols + mx;
        } else {
            mcu = by * mcu_cols + bx;
        }
        // zero the coefficient tile (48 lanes x 16 bytes)
        if (lane < kItemCoefs / 8) reinterpret_cast<int4 *>(cf)[lane] = make_int4(0, 0, 0, 0);
        wave_sync();
        bool ok = true;
        if (active) {
            const uint32_t g = mcu / 9, j = mcu - g * 9;
            const gu32 rec = recs + (size_t)g * 16;
            const bool last = mcu + 1 >= n_mcu;
            const uint32_t i1 = j ? 1 + ((j - 1) >> 1) : 0u;
            const uint32_t i2 = last ? 0u : (j < 8 ? 1 + (j >> 1) : 16u);
            const uint32_t bp = 160 + 36 * j;
            const uint32_t anchor = rec[0], w1 = rec[i1], w2 = rec[i2];
            const uint32_t d0 = rec[bp >> 5], d1 = rec[(bp >> 5) + 1];
            const uint32_t start = anchor + (j ? (w1 >> (((j - 1) & 1) * 16)) & 0xFFFFu : 0u);
            const uint32_t end = last ? stream_bits : (j < 8 ? anchor + ((w2 >> ((j & 1) * 16)) & 0xFFFFu) : w2);
            const uint64_t dv = ((((uint64_t)d1) << 32) | d0) >> (bp & 31);
            const int dc0 = sext12((uint32_t)dv & 0xFFFu);
            const int dc1 = sext12((uint32_t)(dv >> 12) & 0xFFFu);
            const int dc2 = sext12((uint32_t)(dv >> 24) & 0xFFFu);
            const uint32_t limit = (uint32_t)JPT_STREAM_WORDS(stream_bits);
            // the MCU's words: word wbase + i in lane i of mw0 (i < 64) / mw1 (64 + i)
            const uint32_t wbase = start >> 5;
            const uint32_t mw0 = stream[min(wbase + lane, limit - 1u)];
            const uint32_t mw1 = stream[min(wbase + 64u + lane, limit - 1u)];
            uint32_t thr[4];
#pragma unroll
            for (int t = 0; t < 4; t++) thr[t] = tab[JPT_SLOW_OFFSET + t * JPT_SLOW_WORDS + JPT_SLOW_T];
            wave_sync();  // the tile is zeroed before the DCs go in
            if (lane == 0) {
                cf[0] = (int16_t)dc0;
                cf[(s444 ? 1 : 4) * 64] = (int16_t)dc1;
                cf[(s444 ? 2 : 5) * 64] = (int16_t)dc2;
            }
            const int ndu = s444 ? 3 : 6;
            const int first_c = s444 ? 1 : 4;  // first chroma data unit
            uint32_t pos = start;
            int du = 0, k = 1, ypred = dc0;
            bool done = false, err = false;
            // every step consumes at least one symbol of >= 1 bit
            for (uint32_t step = 0; !done && !err; step++) {
                if (pos > end || step > (end - start) + 1u) { err = true; break; }
                // the 128 bits from word pos/32 on; lane i starts at bit (pos & 31) + i
                const uint32_t wi = (pos >> 5) - wbase;
                uint32_t W[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const uint32_t x = wi + i;
                    W[i] = x < 64u ? __builtin_amdgcn_readlane(mw0, x)
                                   : (x < 128u ? __builtin_amdgcn_readlane(mw1, x - 64u)
                                               : stream[min(wbase + x, limit - 1u)]);
                }
                const uint32_t bit = (pos & 31u) + lane;  // 0..94
                const uint32_t hi = bit < 32u ? W[0] : (bit < 64u ? W[1] : W[2]);
                const uint32_t lo = bit < 32u ? W[1] : (bit < 64u ? W[2] : W[3]);
                const uint32_t peek = (uint32_t)(((((uint64_t)hi) << 32) | lo) << (bit & 31u) >> 32);
                // one table per step: AC luma or AC chroma for the data unit in
                // progress; at the start of Y1..Y3 lane 0 looks up the DC
                // difference instead.  The step ends with the data unit.
                const uint32_t tac = du >= first_c ? 3u : 1u;
                const uint32_t tl = (lane == 0 && k == 0) ? 0u : tac;
                uint32_t e0 = fast_entry(tab, tl, tl == 0 ? thr[0] : thr[tac], peek);
                if ((e0 & 31u) == 0 && !(e0 & JPT_FE_BAD)) e0 = slow_entry(tab, tl, peek);
                const uint32_t p0 = pack_entry(e0, peek);
                // ---- the chain walk (scalar)
                uint32_t o = 0, wpos = 0xFFFFFFFFu;
                int wval = 0;
                if (k == 0) {  // DC difference of Y1..Y3 (lane 0)
                    const uint32_t e = __builtin_amdgcn_readlane(p0, 0);
                    ypred += (int)e >> 16;
                    if ((e & 31u) == 0 || (uint32_t)(ypred + 32768) > 65535u) { err = true; break; }
                    if (lane == 0) { wpos = (uint32_t)(du * 64); wval = ypred; }
                    o = e & 31u;
                    k = 1;
                }
                while (o < 64u) {
                    const uint32_t e = __builtin_amdgcn_readlane(p0, o);
                    const uint32_t used = e & 31u, run = (e >> 5) & 15u, size = (e >> 9) & 15u;
                    const int at = k + (int)run;
                    const int nk = size != 0 ? at + 1 : (run == 15 ? k + 16 : 64);  // ZRL / EOB
                    if (used == 0 || nk > 64) { err = true; break; }                 // (at <= 63 when nk <= 64)
                    if (size != 0 && lane == o) {  // the lane that decoded this coefficient stores it
                        wpos = (uint32_t)(du * 64 + at);
                        wval = (int)e >> 16;
                    }
                    o += used;
                    k = nk;
                    if (k == 64) break;
                }
                if (k == 64 && !err) {  // end of the data unit
                    du++;
                    done = du >= ndu;
                    k = du >= first_c ? 1 : 0;
                }
                if (wpos != 0xFFFFFFFFu) cf[wpos] = (int16_t)wval;
                pos += o;
            }
            ok = done && !err && pos == end;
        }
        // ---- publish
        if (!ok && lane == 0) {
            atomicOr(counters + JPT_CTR_ERROR, JPT_ERR_CORRUPT);
            atomicMin(counters + JPT_CTR_ERROR_ITEM, item);
            work[item] = w | 0x80000000u;
        }
        wave_sync();
        if (lane < kItemCoefs / 8)
            reinterpret_cast<int4 *>(coef + (size_t)item * kItemCoefs)[lane] = reinterpret_cast<const int4 *>(cf)[lane];
        wave_sync();  // the tile is read before the next MCU clears it
    }
}

// ---------------------------------------------------------------- IDCT
// zigzag scan position -> natural index (row = vertical frequency),
// generated by walking the anti-diagonals of the 8x8 block.
struct ZigZag {
    uint8_t nat[64];
};
constexpr ZigZag make_zigzag() {
    ZigZag z{};
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
__constant__ ZigZag kZigZag = make_zigzag();

// cos(k pi / 16) for k = 0..8, correctly rounded fp32
__device__ __forceinline__ float cos16(int k) {
    const float c[9] = {1.0f, 0.980785280403230f, 0.923879532511287f, 0.831469612302545f, 0.707106781186548f,
                        0.555570233019602f, 0.382683432365090f, 0.195090322016128f, 0.0f};
    k &= 31;
    if (k > 16) k = 32 - k;
    return k > 8 ? -c[16 - k] : c[k];
}
// half the 1-D basis: C(u)/2 cos((2x+1) u pi / 16), C(0) = 1/sqrt(2)
__device__ __forceinline__ float basis1d(int u, int x) { return u == 0 ? 0.5f * cos16(4) : 0.5f * cos16((2 * x + 1) * u); }

__device__ __forceinline__ uint32_t to_u8(float v) {
    float r = floorf(v + 0.5f);
    r = fminf(fmaxf(r, 0.0f), 255.0f);
    return (uint32_t)r;
}
__device__ __forceinline__ uint32_t ycc_to_rgba(float Y, float Cb, float Cr) {
    const float cb = Cb - 128.0f, cr = Cr - 128.0f;
    const uint32_t R = to_u8(Y + 1.402f * cr);
    const uint32_t G = to_u8(Y - 0.344136f * cb - 0.714136f * cr);
    const uint32_t B = to_u8(Y + 1.772f * cb);
    return R | (G << 8) | (B << 16) | 0xFF000000u;
}

constexpr int kIdctItems = 16;                       // items per workgroup iteration
constexpr int kIdctUnits = kIdctItems * JPT_ITEMS_DU;  // 96 = 3 column tiles of 32
constexpr int kIdctThreads = 256;                      // waves 0-2: one column tile each; all 4: colour

// per-item flags gathered once per tile
constexpr uint32_t kItem444 = 1u, kItemFailed = 2u, kItemPresent = 4u, kItemValid = 8u;

__global__ __launch_bounds__(kIdctThreads) void k_idct_mfma(const jpt_level_desc *__restrict__ levels,
                                                  const uint32_t *__restrict__ word_level,
                                                  const uint16_t *__restrict__ quant, const uint32_t *__restrict__ work,
                                                  const uint32_t *__restrict__ counters,
                                                  const int16_t *__restrict__ coef,
                                                  const uint32_t *__restrict__ slot_of,
                                                  uint32_t *__restrict__ texels) {
    __shared__ float s_samp[kIdctUnits * 64];
    __shared__ float s_P[64];
    __shared__ uint32_t s_slot[kIdctItems], s_quant[kIdctItems], s_flags[kIdctItems], s_q[kIdctItems];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t n_items = counters[JPT_CTR_ITEMS];
    if (blockIdx.x * (uint32_t)kIdctItems >= n_items) return;
    const uint32_t col = lane & 31, half = lane >> 5;

    // basis operands: A[m][s] holds K[32m + col][16s + 8 half + t], t = 0..7, built
    // from the 1-D table P[u][x] = C(u)/2 cos((2x+1) u pi / 16)
    if (threadIdx.x < 64) s_P[lane] = basis1d((int)(lane >> 3), (int)(lane & 7));
    __syncthreads();
    half8 Khi[2][4], Klo[2][4];
    if (wv < kIdctUnits / 32) {
#pragma unroll
        for (int m = 0; m < 2; m++)
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    const int i = 32 * m + (int)col;                     // pixel y*8+x
                    const int n = kZigZag.nat[16 * s + 8 * half + t];     // natural v*8+u
                    const float K = s_P[(n & 7) * 8 + (i & 7)] * s_P[(n >> 3) * 8 + (i >> 3)];
                    const _Float16 hi = (_Float16)K;
                    Khi[m][s][t] = hi;
                    Klo[m][s][t] = (_Float16)((K - (float)hi) * 2048.0f);
                }
    }

    for (uint32_t base = blockIdx.x * kIdctItems; base < n_items; base += gridDim.x * kIdctItems) {
        // ---- item metadata, one lane of the last wave per item
        if (wv == kIdctThreads / 64 - 1 && lane < (uint32_t)kIdctItems) {
            const uint32_t it = base + lane;
            uint32_t flags = 0, slot = JPT_SLOT_NONE, qi = 0, q = 0;
            if (it < n_items) {
                const uint32_t w = work[it];
                const uint32_t b = (w & 0x7FFFFFFFu) >> 2;
                q = w & 3u;
                const jpt_level_desc *L = levels + word_level[b >> 5];
                slot = slot_of[b];
                qi = L->quant;
                flags = kItemValid | ((w >> 31) ? kItemFailed : 0u);
                if (L->sampling == JPT_SAMPLING_444) {
                    flags |= kItem444;
                    const uint32_t r = b - L->blk_base, by = r / L->blk_cols, bx = r - by * L->blk_cols;
                    const uint32_t mx = 2 * bx + (q & 1), my = 2 * by + (q >> 1);
                    if (mx < L->mcu_cols && my < L->n_mcu / L->mcu_cols) flags |= kItemPresent;
                } else {
                    flags |= kItemPresent;
                }
            }
            s_slot[lane] = slot; s_quant[lane] = qi; s_flags[lane] = flags; s_q[lane] = q;
        }
        __syncthreads();
        if (wv < kIdctUnits / 32) {
            const uint32_t d = 32 * wv + col;
            const uint32_t li = d / JPT_ITEMS_DU, du = d % JPT_ITEMS_DU;
            const uint32_t flags = s_flags[li];
            int fv[4][8];
            bool wide = false;
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int t = 0; t < 8; t++) fv[s][t] = 0;
            const bool s444 = flags & kItem444;
            if ((flags & kItemValid) && !(s444 && du >= 3)) {
                const int comp = s444 ? (int)du : (du < 4 ? 0 : 1);
                const uint16_t *qt = quant + (size_t)s_quant[li] * 128 + (comp ? 64 : 0);
                const int16_t *cp = coef + (size_t)(base + li) * kItemCoefs + du * 64;
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    const int4 cv = *reinterpret_cast<const int4 *>(cp + 16 * s + 8 * half);
                    const uint4 qv = *reinterpret_cast<const uint4 *>(qt + 16 * s + 8 * half);
                    const int32_t cw[4] = {cv.x, cv.y, cv.z, cv.w};
                    const uint32_t qw[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
                    for (int p = 0; p < 4; p++) {
                        const int c0 = (int)(int16_t)(cw[p] & 0xFFFF), c1 = cw[p] >> 16;
                        const int q0 = (int)(qw[p] & 0xFFFFu), q1 = (int)(qw[p] >> 16);
                        fv[s][2 * p] = c0 * q0;
                        fv[s][2 * p + 1] = c1 * q1;
                    }
#pragma unroll
                    for (int t = 0; t < 8; t++) wide |= (fv[s][t] > 2048 || fv[s][t] < -2048);
                }
            }
            const bool any_wide = __ballot(wide) != 0;
            half8 Fh[4], Fl[4];
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    if (!any_wide) {
                        Fh[s][t] = (_Float16)(float)fv[s][t];
                        Fl[s][t] = (_Float16)0.0f;
                    } else {  // F = 128 * (F >> 7) + (F & 127), both parts exact in fp16
                        Fh[s][t] = (_Float16)(float)(fv[s][t] >> 7);
                        Fl[s][t] = (_Float16)(float)(fv[s][t] & 127);
                    }
                }
#pragma unroll
            for (int m = 0; m < 2; m++) {
                float16v ah = {}, al = {};
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    ah = __builtin_amdgcn_mfma_f32_32x32x16_f16(Khi[m][s], Fh[s], ah, 0, 0, 0);
                    al = __builtin_amdgcn_mfma_f32_32x32x16_f16(Klo[m][s], Fh[s], al, 0, 0, 0);
                }
                float16v X;
                if (!any_wide) {
                    X = ah + al * (1.0f / 2048.0f);
                } else {
                    float16v bh = {}, bl = {};
#pragma unroll
                    for (int s = 0; s < 4; s++) {
                        bh = __builtin_amdgcn_mfma_f32_32x32x16_f16(Khi[m][s], Fl[s], bh, 0, 0, 0);
                        bl = __builtin_amdgcn_mfma_f32_32x32x16_f16(Klo[m][s], Fl[s], bl, 0, 0, 0);
                    }
                    X = (ah + al * (1.0f / 2048.0f)) * 128.0f + (bh + bl * (1.0f / 2048.0f));
                }
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    const int row = 8 * (r >> 2) + 4 * (int)half + (r & 3);
                    const float v = fminf(fmaxf(X[r] + 128.0f, 0.0f), 255.0f);
                    s_samp[d * 64 + 32 * m + row] = v;
                }
            }
        }
        __syncthreads();
        // colour conversion and store, wave w takes items w, w+4, ... (1 KiB per 4:2:0 item)
        for (int li = (int)wv; li < kIdctItems; li += kIdctThreads / 64) {
            const uint32_t flags = s_flags[li], slot = s_slot[li];
            if (!(flags & kItemValid)) break;
            if (slot == JPT_SLOT_NONE || !(flags & kItemPresent)) continue;
            const bool failed = flags & kItemFailed;
            const float *sp = s_samp + li * JPT_ITEMS_DU * 64;
            uint32_t *dst = texels + (size_t)slot * 256;
            if (!(flags & kItem444)) {
                const uint32_t ty = lane >> 2, tx0 = (lane & 3) * 4;
                uint32_t o[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const uint32_t tx = tx0 + i;
                    const float Y = sp[((ty >> 3) * 2 + (tx >> 3)) * 64 + (ty & 7) * 8 + (tx & 7)];
                    const float Cb = sp[4 * 64 + (ty >> 1) * 8 + (tx >> 1)];
                    const float Cr = sp[5 * 64 + (ty >> 1) * 8 + (tx >> 1)];
                    o[i] = failed ? JPT_TEXEL_INVALID : ycc_to_rgba(Y, Cb, Cr);
                }
                *reinterpret_cast<uint4 *>(dst + ty * 16 + tx0) = make_uint4(o[0], o[1], o[2], o[3]);
            } else if (lane < 16) {
                const uint32_t q = s_q[li];
                const uint32_t ty = lane >> 1, tx0 = (lane & 1) * 4;
                uint32_t o[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const uint32_t p = ty * 8 + tx0 + i;
                    o[i] = failed ? JPT_TEXEL_INVALID : ycc_to_rgba(sp[p], sp[64 + p], sp[128 + p]);
                }
                *reinterpret_cast<uint4 *>(dst + (8 * (q >> 1) + ty) * 16 + 8 * (q & 1) + tx0) =
                    make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
        __syncthreads();
    }
}

// Separable fp32 IDCT on the vector ALUs, one wave per work item: a row pass
// T[v][x] = sum_u F[v][u] P[u][x] and a column pass S[y][x] = sum_v P[v][y]
// T[v][x], lane = (data unit, row); then the same sample clamp, colour
// conversion and store as k_idct_mfma.
__global__ __launch_bounds__(64) void k_idct_scalar(const jpt_level_desc *__restrict__ levels,
                                                    const uint32_t *__restrict__ word_level,
                                                    const uint16_t *__restrict__ quant,
                                                    const uint32_t *__restrict__ work,
                                                    const uint32_t *__restrict__ counters,
                                                    const int16_t *__restrict__ coef,
                                                    const uint32_t *__restrict__ slot_of,
                                                    uint32_t *__restrict__ texels) {
    __shared__ float s_P[64];
    __shared__ float s_F[kItemCoefs];
    __shared__ float s_T[kItemCoefs];
    const uint32_t lane = threadIdx.x;
    const uint32_t n_items = counters[JPT_CTR_ITEMS];
    s_P[lane] = basis1d((int)(lane >> 3), (int)(lane & 7));
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint32_t w = work[it];
        const uint32_t b = (w & 0x7FFFFFFFu) >> 2, q = w & 3u;
        const jpt_level_desc *L = levels + word_level[b >> 5];
        const uint32_t slot = slot_of[b];
        const bool s444 = L->sampling == JPT_SAMPLING_444;
        bool present = true;
        if (s444) {
            const uint32_t r = b - L->blk_base, by = r / L->blk_cols, bx = r - by * L->blk_cols;
            present = 2 * bx + (q & 1) < L->mcu_cols && 2 * by + (q >> 1) < L->n_mcu / L->mcu_cols;
        }
        if (slot == JPT_SLOT_NONE || !present) continue;  // uniform over the wave
        const bool failed = w >> 31;
        uint32_t *dst = texels + (size_t)slot * 256;
        if (failed) {
            if (!s444) {
                for (uint32_t i = lane; i < 256; i += 64) dst[i] = JPT_TEXEL_INVALID;
            } else {
                dst[(8 * (q >> 1) + (lane >> 3)) * 16 + 8 * (q & 1) + (lane & 7)] = JPT_TEXEL_INVALID;
            }
            continue;
        }
        const int ndu = s444 ? 3 : 6;
        const uint16_t *qt = quant + (size_t)L->quant * 128;
        for (int i = (int)lane; i < ndu * 64; i += 64) {
            const int du = i >> 6, k = i & 63;
            const int comp = s444 ? du : (du < 4 ? 0 : 1);
            s_F[du * 64 + kZigZag.nat[k]] =
                (float)((int)coef[(size_t)it * kItemCoefs + i] * (int)qt[(comp ? 64 : 0) + k]);
        }
        __syncthreads();
        const uint32_t du = lane >> 3, rr = lane & 7;
        if ((int)du < ndu) {
            float o[8];
#pragma unroll
            for (int x = 0; x < 8; x++) o[x] = 0.0f;
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const float f = s_F[du * 64 + rr * 8 + u];
#pragma unroll
                for (int x = 0; x < 8; x++) o[x] += f * s_P[u * 8 + x];
            }
#pragma unroll
            for (int x = 0; x < 8; x++) s_T[du * 64 + rr * 8 + x] = o[x];
        }
        __syncthreads();
        if ((int)du < ndu) {
            float o[8];
#pragma unroll
            for (int y = 0; y < 8; y++) o[y] = 0.0f;
#pragma unroll
            for (int v = 0; v < 8; v++) {
                const float t = s_T[du * 64 + v * 8 + rr];  // column rr
#pragma unroll
                for (int y = 0; y < 8; y++) o[y] += s_P[v * 8 + y] * t;
            }
#pragma unroll
            for (int y = 0; y < 8; y++) s_F[du * 64 + y * 8 + rr] = fminf(fmaxf(o[y] + 128.0f, 0.0f), 255.0f);
        }
        __syncthreads();
        if (!s444) {
            const uint32_t ty = lane >> 2, tx0 = (lane & 3) * 4;
            uint32_t o[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t tx = tx0 + i;
                o[i] = ycc_to_rgba(s_F[((ty >> 3) * 2 + (tx >> 3)) * 64 + (ty & 7) * 8 + (tx & 7)],
                                   s_F[4 * 64 + (ty >> 1) * 8 + (tx >> 1)], s_F[5 * 64 + (ty >> 1) * 8 + (tx >> 1)]);
            }
            *reinterpret_cast<uint4 *>(dst + ty * 16 + tx0) = make_uint4(o[0], o[1], o[2], o[3]);
        } else {
            dst[(8 * (q >> 1) + (lane >> 3)) * 16 + 8 * (q & 1) + (lane & 7)] =
                ycc_to_rgba(s_F[lane], s_F[64 + lane], s_F[128 + lane]);
        }
        __syncthreads();
    }
}

uint32_t default_groups(const jpt_tuning *t, bool idct) {
    uint32_t g = t ? (idct ? t->idct_groups : t->decode_groups) : 0u;
    return g ? g : (idct ? 2048u : 1024u);
}

jpt_status launch_entropy(const jpt_scene *scene, jpt_frame *frame, const jpt_tuning *tuning, hipStream_t st) {
    const uint32_t groups = default_groups(tuning, false);
    if (scene->n_tablesets == 1)
        hipLaunchKernelGGL(k_entropy<true>, dim3(groups), dim3(64 * kEntWaves), 0, st, scene->levels,
                           scene->word_level, scene->tables, frame->work, frame->counters, frame->coef);
    else
        hipLaunchKernelGGL(k_entropy<false>, dim3(groups), dim3(64 * kEntWaves), 0, st, scene->levels,
                           scene->word_level, scene->tables, frame->work, frame->counters, frame->coef);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}

jpt_status check_args(const jpt_scene *scene, const jpt_frame *frame) {
    if (!scene || !frame) return JPT_E_ARG;
    if (!scene->levels || !scene->word_level || !scene->tables || !scene->quant || scene->n_tablesets == 0)
        return JPT_E_ARG;
    if (!frame->work || !frame->counters || !frame->coef) return JPT_E_ARG;
    return JPT_OK;
}

}  // namespace

extern "C" jpt_status jpt_entropy_decode(const jpt_scene *scene, jpt_frame *frame, const jpt_tuning *tuning,
                                         void *stream) {
    jpt_status s = check_args(scene, frame);
    if (s) return s;
    return launch_entropy(scene, frame, tuning, (hipStream_t)stream);
}

extern "C" jpt_status jpt_idct_color(const jpt_scene *scene, jpt_frame *frame, jpt_cache *cache, uint32_t idct_mode,
                                     const jpt_tuning *tuning, void *stream) {
    jpt_status s = check_args(scene, frame);
    if (s) return s;
    if (!cache || !cache->texels || !cache->slot_of) return JPT_E_ARG;
    if (idct_mode == JPT_IDCT_MFMA_F16)
        hipLaunchKernelGGL(k_idct_mfma, dim3(default_groups(tuning, true)), dim3(kIdctThreads), 0,
                           (hipStream_t)stream,
                           scene->levels, scene->word_level, scene->quant, frame->work, frame->counters, frame->coef,
                           cache->slot_of, cache->texels);
    else if (idct_mode == JPT_IDCT_SCALAR_F32)
        hipLaunchKernelGGL(k_idct_scalar, dim3(4 * default_groups(tuning, true)), dim3(64), 0, (hipStream_t)stream,
                           scene->levels, scene->word_level, scene->quant, frame->work, frame->counters, frame->coef,
                           cache->slot_of, cache->texels);
    else
        return JPT_E_ARG;
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}

extern "C" jpt_status jpt_decode_blocks(const jpt_scene *scene, jpt_frame *frame, jpt_cache *cache,
                                        uint32_t idct_mode, const jpt_tuning *tuning, void *stream) {
    jpt_status s = check_args(scene, frame);
    if (s) return s;
    if (!cache || !cache->texels || !cache->slot_of) return JPT_E_ARG;
    if (idct_mode != JPT_IDCT_MFMA_F16 && idct_mode != JPT_IDCT_SCALAR_F32) return JPT_E_ARG;
    if ((s = launch_entropy(scene, frame, tuning, (hipStream_t)stream))) return s;
    return jpt_idct_color(scene, frame, cache, idct_mode, tuning, stream);
}
