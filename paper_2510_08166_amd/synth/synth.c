/*
 * Seeded synthetic inputs: procedural RGB8 textures, box-filtered mip levels
 * and a baseline (sequential, Huffman) JPEG encoder that turns them into the
 * compressed textures the decoder consumes.
 *
 * This module only produces inputs. It holds no step of the decode path
 * (no inverse DCT, no Huffman decoding, no YCbCr->RGB, no sampling); those
 * live separately in the GPU library and in the CPU checker.
 *
 * Encoder steps follow the baseline JPEG pipeline the paper summarises in its
 * JPEG background section (colour conversion, 4:2:0 subsampling, 8x8 DCT,
 * quantisation, differential DCs, run-length + Huffman coding):
 *   1. RGB8 -> YCbCr, JFIF full-range BT.601, fp64, round half up, clamp.
 *   2. 4:2:0: 2x2 box average of chroma, rounded half up.  4:4:4: none.
 *   3. Pad to whole MCUs by edge replication.
 *   4. Level shift by -128, forward DCT in fp64 (separable form of the
 *      definition F(u,v) = 1/4 C(u)C(v) sum f(x,y) cos((2x+1)u pi/16)
 *      cos((2y+1)v pi/16), C(0) = 1/sqrt 2).
 *   5. Quantise, round half away from zero; tables of ITU T.81 Annex K
 *      scaled by the IJG quality rule.
 *   6. Zigzag, DC differences per component, Annex K Huffman tables, byte
 *      stuffing, 1-bit padding of the last byte.
 *   7. Markers SOI APP0 DQT SOF0 DHT SOS <scan> EOI, one interleaved scan,
 *      no restart intervals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG */
/* splitmix64 (Steele, Lea, Flood 2014) used as a plain sequential stream. */
static uint64_t sm64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double sm_unit(uint64_t *s) { return (double)(sm64(s) >> 11) * (1.0 / 9007199254740992.0); }
static uint32_t sm_below(uint64_t *s, uint32_t n) { return n ? (uint32_t)(sm64(s) % n) : 0u; }

/* ------------------------------------------------------------- textures */
static double smooth(double t) { return t * t * (3.0 - 2.0 * t); }

/* Tileable value noise, 4 octaves (lattice spacing 64, 32, 16, 8 px,
 * amplitude halving per octave), uniform lattice values in [0,255] drawn per
 * channel, smoothstep interpolation; then 16-64 axis-aligned rectangles of
 * uniform random colour overlaid with hard edges (wrapping at the borders). */
int synth_texture(uint64_t seed, int w, int h, uint8_t *rgb) {
    if (w <= 0 || h <= 0 || !rgb) return -1;
    uint64_t s = seed ^ 0x5DEECE66Dull;
    const int spacing[4] = {64, 32, 16, 8};
    const double amp[4] = {1.0, 0.5, 0.25, 0.125};
    const double amp_sum = 1.875;
    double *acc = (double *)calloc((size_t)w * h * 3, sizeof(double));
    if (!acc) return -2;
    for (int o = 0; o < 4; o++) {
        int nx = w / spacing[o]; if (nx < 1) nx = 1;
        int ny = h / spacing[o]; if (ny < 1) ny = 1;
        double *lat = (double *)malloc((size_t)nx * ny * 3 * sizeof(double));
        if (!lat) { free(acc); return -2; }
        for (size_t i = 0; i < (size_t)nx * ny * 3; i++) lat[i] = 255.0 * sm_unit(&s);
        for (int y = 0; y < h; y++) {
            double fy = (y + 0.5) * ny / (double)h;
            int y0 = (int)floor(fy); double ty = smooth(fy - y0);
            y0 %= ny; int y1 = (y0 + 1) % ny;
            for (int x = 0; x < w; x++) {
                double fx = (x + 0.5) * nx / (double)w;
                int x0 = (int)floor(fx); double tx = smooth(fx - x0);
                x0 %= nx; int x1 = (x0 + 1) % nx;
                for (int c = 0; c < 3; c++) {
                    double a = lat[((size_t)y0 * nx + x0) * 3 + c], b = lat[((size_t)y0 * nx + x1) * 3 + c];
                    double d = lat[((size_t)y1 * nx + x0) * 3 + c], e = lat[((size_t)y1 * nx + x1) * 3 + c];
                    double top = a + (b - a) * tx, bot = d + (e - d) * tx;
                    acc[((size_t)y * w + x) * 3 + c] += amp[o] * (top + (bot - top) * ty);
                }
            }
        }
        free(lat);
    }
    for (size_t i = 0; i < (size_t)w * h * 3; i++) {
        double v = floor(acc[i] / amp_sum + 0.5);
        rgb[i] = (uint8_t)(v < 0 ? 0 : v > 255 ? 255 : v);
    }
    free(acc);
    int nrect = 16 + (int)sm_below(&s, 49);
    for (int r = 0; r < nrect; r++) {
        int x0 = (int)sm_below(&s, (uint32_t)w), y0 = (int)sm_below(&s, (uint32_t)h);
        int rw = 1 + w / 32 + (int)sm_below(&s, (uint32_t)(w / 4 + 1));
        int rh = 1 + h / 32 + (int)sm_below(&s, (uint32_t)(h / 4 + 1));
        uint8_t col[3];
        for (int c = 0; c < 3; c++) col[c] = (uint8_t)sm_below(&s, 256);
        for (int y = 0; y < rh && y < h; y++)
            for (int x = 0; x < rw && x < w; x++) {
                size_t p = ((size_t)((y0 + y) % h) * w + (size_t)((x0 + x) % w)) * 3;
                rgb[p] = col[0]; rgb[p + 1] = col[1]; rgb[p + 2] = col[2];
            }
    }
    return 0;
}

/* One mip step: 2x2 box filter, rounded half up; odd sizes clamp the
 * second tap to the last row/column. dst is max(1,w/2) x max(1,h/2). */
int synth_mip(const uint8_t *src, int w, int h, uint8_t *dst) {
    if (w <= 0 || h <= 0 || !src || !dst) return -1;
    int dw = w > 1 ? w / 2 : 1, dh = h > 1 ? h / 2 : 1;
    for (int y = 0; y < dh; y++) {
        int ya = 2 * y < h ? 2 * y : h - 1, yb = 2 * y + 1 < h ? 2 * y + 1 : h - 1;
        for (int x = 0; x < dw; x++) {
            int xa = 2 * x < w ? 2 * x : w - 1, xb = 2 * x + 1 < w ? 2 * x + 1 : w - 1;
            for (int c = 0; c < 3; c++) {
                int v = src[((size_t)ya * w + xa) * 3 + c] + src[((size_t)ya * w + xb) * 3 + c] +
                        src[((size_t)yb * w + xa) * 3 + c] + src[((size_t)yb * w + xb) * 3 + c];
                dst[((size_t)y * dw + x) * 3 + c] = (uint8_t)((v + 2) >> 2);
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------- Annex K tables */
static const uint8_t K1_LUMA[64] = {  /* natural order, row = vertical freq */
    16, 11, 10, 16, 24, 40, 51, 61,   12, 12, 14, 19, 26, 58, 60, 55,
    14, 13, 16, 24, 40, 57, 69, 56,   14, 17, 22, 29, 51, 87, 80, 62,
    18, 22, 37, 56, 68, 109, 103, 77, 24, 35, 55, 64, 81, 104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99};
static const uint8_t K2_CHROMA[64] = {
    17, 18, 24, 47, 99, 99, 99, 99,   18, 21, 26, 66, 99, 99, 99, 99,
    24, 26, 56, 99, 99, 99, 99, 99,   47, 66, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99,   99, 99, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99,   99, 99, 99, 99, 99, 99, 99, 99};

static const uint8_t DC_LUMA_BITS[16] = {0, 1, 5, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0};
static const uint8_t DC_CHROMA_BITS[16] = {0, 3, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0};
static const uint8_t DC_VALS[12] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
static const uint8_t AC_LUMA_BITS[16] = {0, 2, 1, 3, 3, 2, 4, 3, 5, 5, 4, 4, 0, 0, 1, 0x7d};
static const uint8_t AC_LUMA_VALS[162] = {
    0x01, 0x02, 0x03, 0x00, 0x04, 0x11, 0x05, 0x12, 0x21, 0x31, 0x41, 0x06, 0x13, 0x51, 0x61, 0x07,
    0x22, 0x71, 0x14, 0x32, 0x81, 0x91, 0xa1, 0x08, 0x23, 0x42, 0xb1, 0xc1, 0x15, 0x52, 0xd1, 0xf0,
    0x24, 0x33, 0x62, 0x72, 0x82, 0x09, 0x0a, 0x16, 0x17, 0x18, 0x19, 0x1a, 0x25, 0x26, 0x27, 0x28,
    0x29, 0x2a, 0x34, 0x35, 0x36, 0x37, 0x38, 0x39, 0x3a, 0x43, 0x44, 0x45, 0x46, 0x47, 0x48, 0x49,
    0x4a, 0x53, 0x54, 0x55, 0x56, 0x57, 0x58, 0x59, 0x5a, 0x63, 0x64, 0x65, 0x66, 0x67, 0x68, 0x69,
    0x6a, 0x73, 0x74, 0x75, 0x76, 0x77, 0x78, 0x79, 0x7a, 0x83, 0x84, 0x85, 0x86, 0x87, 0x88, 0x89,
    0x8a, 0x92, 0x93, 0x94, 0x95, 0x96, 0x97, 0x98, 0x99, 0x9a, 0xa2, 0xa3, 0xa4, 0xa5, 0xa6, 0xa7,
    0xa8, 0xa9, 0xaa, 0xb2, 0xb3, 0xb4, 0xb5, 0xb6, 0xb7, 0xb8, 0xb9, 0xba, 0xc2, 0xc3, 0xc4, 0xc5,
    0xc6, 0xc7, 0xc8, 0xc9, 0xca, 0xd2, 0xd3, 0xd4, 0xd5, 0xd6, 0xd7, 0xd8, 0xd9, 0xda, 0xe1, 0xe2,
    0xe3, 0xe4, 0xe5, 0xe6, 0xe7, 0xe8, 0xe9, 0xea, 0xf1, 0xf2, 0xf3, 0xf4, 0xf5, 0xf6, 0xf7, 0xf8,
    0xf9, 0xfa};
static const uint8_t AC_CHROMA_BITS[16] = {0, 2, 1, 2, 4, 4, 3, 4, 7, 5, 4, 4, 0, 1, 2, 0x77};
static const uint8_t AC_CHROMA_VALS[162] = {
    0x00, 0x01, 0x02, 0x03, 0x11, 0x04, 0x05, 0x21, 0x31, 0x06, 0x12, 0x41, 0x51, 0x07, 0x61, 0x71,
    0x13, 0x22, 0x32, 0x81, 0x08, 0x14, 0x42, 0x91, 0xa1, 0xb1, 0xc1, 0x09, 0x23, 0x33, 0x52, 0xf0,
    0x15, 0x62, 0x72, 0xd1, 0x0a, 0x16, 0x24, 0x34, 0xe1, 0x25, 0xf1, 0x17, 0x18, 0x19, 0x1a, 0x26,
    0x27, 0x28, 0x29, 0x2a, 0x35, 0x36, 0x37, 0x38, 0x39, 0x3a, 0x43, 0x44, 0x45, 0x46, 0x47, 0x48,
    0x49, 0x4a, 0x53, 0x54, 0x55, 0x56, 0x57, 0x58, 0x59, 0x5a, 0x63, 0x64, 0x65, 0x66, 0x67, 0x68,
    0x69, 0x6a, 0x73, 0x74, 0x75, 0x76, 0x77, 0x78, 0x79, 0x7a, 0x82, 0x83, 0x84, 0x85, 0x86, 0x87,
    0x88, 0x89, 0x8a, 0x92, 0x93, 0x94, 0x95, 0x96, 0x97, 0x98, 0x99, 0x9a, 0xa2, 0xa3, 0xa4, 0xa5,
    0xa6, 0xa7, 0xa8, 0xa9, 0xaa, 0xb2, 0xb3, 0xb4, 0xb5, 0xb6, 0xb7, 0xb8, 0xb9, 0xba, 0xc2, 0xc3,
    0xc4, 0xc5, 0xc6, 0xc7, 0xc8, 0xc9, 0xca, 0xd2, 0xd3, 0xd4, 0xd5, 0xd6, 0xd7, 0xd8, 0xd9, 0xda,
    0xe2, 0xe3, 0xe4, 0xe5, 0xe6, 0xe7, 0xe8, 0xe9, 0xea, 0xf2, 0xf3, 0xf4, 0xf5, 0xf6, 0xf7, 0xf8,
    0xf9, 0xfa};

/* IJG quality scaling of a base table, clamped to the baseline range [1,255]. */
static void scale_quant(const uint8_t *base, int quality, uint16_t *out) {
    if (quality < 1) quality = 1;
    if (quality > 100) quality = 100;
    long scale = quality < 50 ? 5000 / quality : 200 - 2 * quality;
    for (int i = 0; i < 64; i++) {
        long q = ((long)base[i] * scale + 50) / 100;
        if (q < 1) q = 1;
        if (q > 255) q = 255;
        out[i] = (uint16_t)q;
    }
}

int synth_quant_tables(int quality, uint16_t *luma, uint16_t *chroma) {
    scale_quant(K1_LUMA, quality, luma);
    scale_quant(K2_CHROMA, quality, chroma);
    return 0;
}

/* zigzag position -> natural index, generated by walking the anti-diagonals */
static void make_zigzag(int zz[64]) {
    int i = 0;
    for (int d = 0; d < 15; d++) {
        int lo = d < 8 ? 0 : d - 7, hi = d < 8 ? d : 7;
        if (d & 1)
            for (int r = lo; r <= hi; r++) zz[i++] = r * 8 + (d - r);      /* downwards */
        else
            for (int r = hi; r >= lo; r--) zz[i++] = r * 8 + (d - r);      /* upwards */
    }
}

/* ------------------------------------------------------- Huffman encode */
typedef struct { uint16_t code[256]; uint8_t len[256]; } ehuff;

/* Canonical code assignment (ITU T.81 Annex C): codes of each length are
 * consecutive, the code is doubled when moving to the next length. */
static void build_ehuff(const uint8_t bits[16], const uint8_t *vals, ehuff *t) {
    memset(t, 0, sizeof *t);
    int k = 0; uint32_t code = 0;
    for (int l = 1; l <= 16; l++) {
        for (int i = 0; i < bits[l - 1]; i++, k++) {
            t->code[vals[k]] = (uint16_t)code;
            t->len[vals[k]] = (uint8_t)l;
            code++;
        }
        code <<= 1;
    }
}

typedef struct {
    uint8_t *out; size_t cap, n; int overflow;
    uint32_t acc; int nacc;
} bitw;

static void put_byte(bitw *b, uint8_t v) {
    if (b->n < b->cap) b->out[b->n] = v; else b->overflow = 1;
    b->n++;
}
static void put_bits(bitw *b, uint32_t v, int n) {
    for (int i = n - 1; i >= 0; i--) {
        b->acc = (b->acc << 1) | ((v >> i) & 1u);
        if (++b->nacc == 8) {
            uint8_t byte = (uint8_t)b->acc;
            put_byte(b, byte);
            if (byte == 0xFF) put_byte(b, 0x00);      /* byte stuffing */
            b->acc = 0; b->nacc = 0;
        }
    }
}
static void flush_bits(bitw *b) { while (b->nacc) put_bits(b, 1, 1); }

static int bit_size(int v) { int a = v < 0 ? -v : v, s = 0; while (a) { s++; a >>= 1; } return s; }

static void emit_du(bitw *b, const int16_t *zzc, int *pred, const ehuff *dc, const ehuff *ac) {
    int diff = zzc[0] - *pred; *pred = zzc[0];
    int s = bit_size(diff);
    put_bits(b, dc->code[s], dc->len[s]);
    if (s) put_bits(b, (uint32_t)(diff < 0 ? diff - 1 : diff) & ((1u << s) - 1), s);
    int run = 0;
    for (int k = 1; k < 64; k++) {
        int v = zzc[k];
        if (v == 0) { run++; continue; }
        while (run > 15) { put_bits(b, ac->code[0xF0], ac->len[0xF0]); run -= 16; }
        int sz = bit_size(v), sym = (run << 4) | sz;
        put_bits(b, ac->code[sym], ac->len[sym]);
        put_bits(b, (uint32_t)(v < 0 ? v - 1 : v) & ((1u << sz) - 1), sz);
        run = 0;
    }
    if (run) put_bits(b, ac->code[0x00], ac->len[0x00]);
}

/* --------------------------------------------------------------- encoder */
#define SYN_PI 3.14159265358979323846
#define SYN_SQRT1_2 0.70710678118654752440

static void make_cos_table(double cosv[8][8]) {
    for (int u = 0; u < 8; u++)
        for (int x = 0; x < 8; x++) cosv[u][x] = cos((2 * x + 1) * u * SYN_PI / 16.0);
}

static void fdct8x8(const double cosv[8][8], const double in[64], double out[64]) {
    double tmp[64];
    for (int y = 0; y < 8; y++)                  /* rows: horizontal frequency u */
        for (int u = 0; u < 8; u++) {
            double s = 0; for (int x = 0; x < 8; x++) s += in[y * 8 + x] * cosv[u][x];
            tmp[y * 8 + u] = s;
        }
    for (int v = 0; v < 8; v++)
        for (int u = 0; u < 8; u++) {
            double s = 0; for (int y = 0; y < 8; y++) s += tmp[y * 8 + u] * cosv[v][y];
            double cu = u ? 1.0 : SYN_SQRT1_2, cv = v ? 1.0 : SYN_SQRT1_2;
            out[v * 8 + u] = 0.25 * cu * cv * s;
        }
}

static double rnd_away(double x) { return x < 0 ? -floor(-x + 0.5) : floor(x + 0.5); }

static void put16(bitw *b, int v) { put_byte(b, (uint8_t)(v >> 8)); put_byte(b, (uint8_t)v); }

static void put_dht(bitw *b, int cls_id, const uint8_t bits[16], const uint8_t *vals) {
    int n = 0; for (int i = 0; i < 16; i++) n += bits[i];
    put_byte(b, 0xFF); put_byte(b, 0xC4); put16(b, 2 + 1 + 16 + n);
    put_byte(b, (uint8_t)cls_id);
    for (int i = 0; i < 16; i++) put_byte(b, bits[i]);
    for (int i = 0; i < n; i++) put_byte(b, vals[i]);
}

/* Encode rgb (w x h x 3, row-major) as baseline JPEG.
 * sampling: 420 or 444.  On success returns 0 and *out_len bytes in out
 * (if out_len exceeds cap the call returns 1 and *out_len is the size needed).
 * coef (nullable): quantised coefficients, natural order, laid out
 * [mcu (raster)][du (scan order: Y.., Cb, Cr)][64]. */
int synth_encode(const uint8_t *rgb, int w, int h, int quality, int sampling,
                 uint8_t *out, size_t cap, size_t *out_len, int16_t *coef) {
    if (!rgb || w <= 0 || h <= 0 || w > 65535 || h > 65535 || !out_len) return -1;
    if (sampling != 420 && sampling != 444) return -1;
    const int ms = sampling == 420 ? 16 : 8;            /* MCU size in pixels */
    const int mcols = (w + ms - 1) / ms, mrows = (h + ms - 1) / ms;
    const int pw = mcols * ms, ph = mrows * ms;         /* padded luma size */
    const int cw = sampling == 420 ? pw / 2 : pw, ch = sampling == 420 ? ph / 2 : ph;
    uint8_t *Y = (uint8_t *)malloc((size_t)pw * ph), *Cb = (uint8_t *)malloc((size_t)pw * ph),
            *Cr = (uint8_t *)malloc((size_t)pw * ph);
    uint8_t *sCb = NULL, *sCr = NULL;
    if (!Y || !Cb || !Cr) { free(Y); free(Cb); free(Cr); return -2; }
    for (int y = 0; y < ph; y++) {
        int sy = y < h ? y : h - 1;
        for (int x = 0; x < pw; x++) {
            int sx = x < w ? x : w - 1;
            const uint8_t *p = rgb + ((size_t)sy * w + sx) * 3;
            double r = p[0], g = p[1], bl = p[2];
            double yy = 0.299 * r + 0.587 * g + 0.114 * bl;
            double cb = -0.168736 * r - 0.331264 * g + 0.5 * bl + 128.0;
            double cr = 0.5 * r - 0.418688 * g - 0.081312 * bl + 128.0;
            double v3[3] = {yy, cb, cr};
            uint8_t o3[3];
            for (int c = 0; c < 3; c++) {
                double t = floor(v3[c] + 0.5);
                o3[c] = (uint8_t)(t < 0 ? 0 : t > 255 ? 255 : t);
            }
            size_t i = (size_t)y * pw + x;
            Y[i] = o3[0]; Cb[i] = o3[1]; Cr[i] = o3[2];
        }
    }
    if (sampling == 420) {
        sCb = (uint8_t *)malloc((size_t)cw * ch); sCr = (uint8_t *)malloc((size_t)cw * ch);
        if (!sCb || !sCr) { free(Y); free(Cb); free(Cr); free(sCb); free(sCr); return -2; }
        for (int y = 0; y < ch; y++)
            for (int x = 0; x < cw; x++) {
                size_t a = (size_t)(2 * y) * pw + 2 * x, b2 = a + pw;
                sCb[(size_t)y * cw + x] = (uint8_t)((Cb[a] + Cb[a + 1] + Cb[b2] + Cb[b2 + 1] + 2) >> 2);
                sCr[(size_t)y * cw + x] = (uint8_t)((Cr[a] + Cr[a + 1] + Cr[b2] + Cr[b2 + 1] + 2) >> 2);
            }
    } else {
        sCb = Cb; sCr = Cr; Cb = NULL; Cr = NULL;
    }

    uint16_t ql[64], qc[64];
    synth_quant_tables(quality, ql, qc);
    int zz[64]; make_zigzag(zz);
    ehuff dcl, dcc, acl, acc;
    build_ehuff(DC_LUMA_BITS, DC_VALS, &dcl);
    build_ehuff(DC_CHROMA_BITS, DC_VALS, &dcc);
    build_ehuff(AC_LUMA_BITS, AC_LUMA_VALS, &acl);
    build_ehuff(AC_CHROMA_BITS, AC_CHROMA_VALS, &acc);

    bitw b = {out, cap, 0, 0, 0, 0};
    put_byte(&b, 0xFF); put_byte(&b, 0xD8);                               /* SOI */
    put_byte(&b, 0xFF); put_byte(&b, 0xE0); put16(&b, 16);                /* APP0 JFIF */
    put_byte(&b, 'J'); put_byte(&b, 'F'); put_byte(&b, 'I'); put_byte(&b, 'F'); put_byte(&b, 0);
    put_byte(&b, 1); put_byte(&b, 1); put_byte(&b, 0); put16(&b, 1); put16(&b, 1);
    put_byte(&b, 0); put_byte(&b, 0);
    for (int t = 0; t < 2; t++) {                                         /* DQT */
        const uint16_t *q = t ? qc : ql;
        put_byte(&b, 0xFF); put_byte(&b, 0xDB); put16(&b, 67); put_byte(&b, (uint8_t)t);
        for (int i = 0; i < 64; i++) put_byte(&b, (uint8_t)q[zz[i]]);
    }
    put_byte(&b, 0xFF); put_byte(&b, 0xC0); put16(&b, 17);               /* SOF0 */
    put_byte(&b, 8); put16(&b, h); put16(&b, w); put_byte(&b, 3);
    put_byte(&b, 1); put_byte(&b, sampling == 420 ? 0x22 : 0x11); put_byte(&b, 0);
    put_byte(&b, 2); put_byte(&b, 0x11); put_byte(&b, 1);
    put_byte(&b, 3); put_byte(&b, 0x11); put_byte(&b, 1);
    put_dht(&b, 0x00, DC_LUMA_BITS, DC_VALS);                              /* DHT */
    put_dht(&b, 0x10, AC_LUMA_BITS, AC_LUMA_VALS);
    put_dht(&b, 0x01, DC_CHROMA_BITS, DC_VALS);
    put_dht(&b, 0x11, AC_CHROMA_BITS, AC_CHROMA_VALS);
    put_byte(&b, 0xFF); put_byte(&b, 0xDA); put16(&b, 12); put_byte(&b, 3); /* SOS */
    put_byte(&b, 1); put_byte(&b, 0x00); put_byte(&b, 2); put_byte(&b, 0x11);
    put_byte(&b, 3); put_byte(&b, 0x11); put_byte(&b, 0); put_byte(&b, 63); put_byte(&b, 0);

    const int ndu = sampling == 420 ? 6 : 3;
    int pred[3] = {0, 0, 0};
    double cosv[8][8];
    make_cos_table(cosv);
    double blk[64], F[64];
    int16_t zzc[64];
    for (int my = 0; my < mrows; my++)
        for (int mx = 0; mx < mcols; mx++) {
            for (int d = 0; d < ndu; d++) {
                const uint8_t *plane; int stride, ox, oy, comp;
                if (sampling == 420 && d < 4) {
                    plane = Y; stride = pw; ox = mx * 16 + (d & 1) * 8; oy = my * 16 + (d >> 1) * 8; comp = 0;
                } else {
                    comp = sampling == 420 ? d - 3 : d;
                    plane = comp == 0 ? Y : comp == 1 ? sCb : sCr;
                    stride = comp == 0 ? pw : cw; ox = mx * 8; oy = my * 8;
                }
                for (int y = 0; y < 8; y++)
                    for (int x = 0; x < 8; x++)
                        blk[y * 8 + x] = (double)plane[(size_t)(oy + y) * stride + ox + x] - 128.0;
                fdct8x8(cosv, blk, F);
                const uint16_t *q = comp ? qc : ql;
                int16_t nat[64];
                for (int k = 0; k < 64; k++) nat[k] = (int16_t)rnd_away(F[k] / q[k]);
                for (int i = 0; i < 64; i++) zzc[i] = nat[zz[i]];
                if (coef) memcpy(coef + (((size_t)my * mcols + mx) * ndu + d) * 64, nat, sizeof nat);
                emit_du(&b, zzc, &pred[comp], comp ? &dcc : &dcl, comp ? &acc : &acl);
            }
        }
    flush_bits(&b);
    put_byte(&b, 0xFF); put_byte(&b, 0xD9);                               /* EOI */
    free(Y); free(Cb); free(Cr); free(sCb); free(sCr);
    *out_len = b.n;
    return b.overflow ? 1 : 0;
}

/* ------------------------------------------------------------ G-buffer */
/* One pixel of the deferred-shading G-buffer: texture coordinates (repeat
 * addressing, v = 0 is the top texel row), texture id (0xFFFFFFFF marks
 * background) and level of detail log2(texels per pixel). */
typedef struct { float u, v; uint32_t tex; float lod; } synth_gpixel;

/* Rasterise textured quads at pixel centres in the given order (painter's
 * order: later quads overwrite earlier ones).  Quad q maps the unit square
 * (s,t) to the screen by a homography whose inverse Ginv (row-major 3x3)
 * takes the homogeneous pixel centre (x+.5, y+.5, 1) back to (s,t).
 * uv = off + scale * (s,t).  The level of detail comes from the analytic
 * Jacobian of that inverse: lod = log2 max(|d(uw,vh)/dx|, |d(uw,vh)/dy|)
 * with (w,h) the texture's base size.  bbox = x0,y0,x1,y1 (half-open,
 * already clipped to the screen).  The caller fills background pixels. */
int synth_raster(int W, int H, int nq, const double *Ginv, const int *bbox,
                 const uint32_t *tex, const double *uvp, const double *texwh,
                 synth_gpixel *gbuf) {
    if (W <= 0 || H <= 0 || nq < 0 || !gbuf) return -1;
    for (int q = 0; q < nq; q++) {
        const double *G = Ginv + 9 * q;
        const double su = uvp[4 * q], sv = uvp[4 * q + 1], ou = uvp[4 * q + 2], ov = uvp[4 * q + 3];
        const double tw = texwh[2 * q], th = texwh[2 * q + 1];
        int x0 = bbox[4 * q], y0 = bbox[4 * q + 1], x1 = bbox[4 * q + 2], y1 = bbox[4 * q + 3];
        if (x0 < 0) x0 = 0; if (y0 < 0) y0 = 0; if (x1 > W) x1 = W; if (y1 > H) y1 = H;
        for (int y = y0; y < y1; y++)
            for (int x = x0; x < x1; x++) {
                double px = x + 0.5, py = y + 0.5;
                double q0 = G[0] * px + G[1] * py + G[2];
                double q1 = G[3] * px + G[4] * py + G[5];
                double q2 = G[6] * px + G[7] * py + G[8];
                if (!(q2 > 1e-12)) continue;
                double s = q0 / q2, t = q1 / q2;
                if (s < 0.0 || s > 1.0 || t < 0.0 || t > 1.0) continue;
                double dsdx = (G[0] - s * G[6]) / q2, dsdy = (G[1] - s * G[7]) / q2;
                double dtdx = (G[3] - t * G[6]) / q2, dtdy = (G[4] - t * G[7]) / q2;
                double ax = su * dsdx * tw, bx = sv * dtdx * th;
                double ay = su * dsdy * tw, by = sv * dtdy * th;
                double rx = ax * ax + bx * bx, ry = ay * ay + by * by;
                double rho2 = rx > ry ? rx : ry;
                synth_gpixel *o = gbuf + (size_t)y * W + x;
                o->u = (float)(ou + su * s);
                o->v = (float)(ov + sv * t);
                o->tex = tex[q];
                o->lod = rho2 > 0 ? (float)(0.5 * log2(rho2)) : -64.0f;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------ BC1 */
/* A simple BC1 encoder (input for the fixed-rate baseline): per 4x4 block,
 * edges replicated, the endpoints are the darkest and brightest texels by
 * luma (299 R + 587 G + 114 B), rounded to RGB565 and ordered so that
 * colour 0 > colour 1 (four-colour mode; equal endpoints give index 0
 * everywhere); each texel takes the nearest palette entry in RGB (the
 * first on ties).  out: 8 bytes per block, row-major. */
static uint32_t to565(const int *c) {
    return (uint32_t)(((c[0] * 31 + 127) / 255) << 11 | ((c[1] * 63 + 127) / 255) << 5 | ((c[2] * 31 + 127) / 255));
}
static void from565(uint32_t v, int *c) {
    int r = (v >> 11) & 31, g = (v >> 5) & 63, b = v & 31;
    c[0] = (r << 3) | (r >> 2); c[1] = (g << 2) | (g >> 4); c[2] = (b << 3) | (b >> 2);
}

int synth_bc1_encode(const uint8_t *rgb, int w, int h, uint8_t *out) {
    if (!rgb || !out || w <= 0 || h <= 0) return -1;
    const int bw = (w + 3) / 4, bh = (h + 3) / 4;
    for (int by = 0; by < bh; by++)
        for (int bx = 0; bx < bw; bx++) {
            int t[16][3];
            for (int j = 0; j < 4; j++)
                for (int i = 0; i < 4; i++) {
                    int x = 4 * bx + i, y = 4 * by + j;
                    if (x >= w) x = w - 1;
                    if (y >= h) y = h - 1;
                    for (int c = 0; c < 3; c++) t[4 * j + i][c] = rgb[((size_t)y * w + x) * 3 + c];
                }
            int lo = 0, hi = 0;
            long llo = 1L << 40, lhi = -1;
            for (int k = 0; k < 16; k++) {
                long l = 299L * t[k][0] + 587L * t[k][1] + 114L * t[k][2];
                if (l < llo) { llo = l; lo = k; }
                if (l > lhi) { lhi = l; hi = k; }
            }
            uint32_t c0 = to565(t[hi]), c1 = to565(t[lo]);
            if (c0 < c1) { uint32_t x = c0; c0 = c1; c1 = x; }
            int p[4][3];
            from565(c0, p[0]);
            from565(c1, p[1]);
            for (int c = 0; c < 3; c++) {
                p[2][c] = (2 * p[0][c] + p[1][c] + 1) / 3;
                p[3][c] = (p[0][c] + 2 * p[1][c] + 1) / 3;
            }
            uint32_t bits = 0;
            if (c0 != c1)
                for (int k = 0; k < 16; k++) {
                    int best = 0;
                    long bd = -1;
                    for (int e = 0; e < 4; e++) {
                        long d = 0;
                        for (int c = 0; c < 3; c++) d += (long)(t[k][c] - p[e][c]) * (t[k][c] - p[e][c]);
                        if (bd < 0 || d < bd) { bd = d; best = e; }
                    }
                    bits |= (uint32_t)best << (2 * k);
                }
            uint8_t *o = out + ((size_t)by * bw + bx) * 8;
            o[0] = c0 & 255; o[1] = c0 >> 8; o[2] = c1 & 255; o[3] = c1 >> 8;
            o[4] = bits & 255; o[5] = (bits >> 8) & 255; o[6] = (bits >> 16) & 255; o[7] = bits >> 24;
        }
    return 0;
}
