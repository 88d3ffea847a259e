/*
 * CPU oracle for the on-demand JPEG texture path -- TEST INFRASTRUCTURE.
 * See oracle.h for what each function computes and which passage it follows.
 * No blocking, fusion or reordering beyond the definitions it restates.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Zigzag scan position -> natural (row-major, row = vertical frequency)
 * coefficient index, as laid out in T.81 Figure A.6. */
static const int ZZ_TO_NAT[64] = {
    0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,
    12, 19, 26, 33, 40, 48, 41, 34, 27, 20, 13, 6,  7,  14, 21, 28,
    35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51,
    58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

/* ------------------------------------------------------------ Huffman -- */
/* Decoder tables of T.81 F.2.2.3, generated per Annex C. */
typedef struct {
    int present;
    uint8_t bits[17];      /* bits[l] = number of codes of length l */
    uint8_t val[256];
    int nval;
    int32_t maxcode[18];   /* -1 where no code of that length */
    int32_t mincode[17];
    int32_t valptr[17];
} huff_t;

static int huff_generate(huff_t *h) {
    /* C.1: HUFFSIZE; C.2: HUFFCODE; F.15: MAXCODE, MINCODE, VALPTR */
    int huffsize[257], huffcode[257];
    int k = 0;
    for (int l = 1; l <= 16; l++)
        for (int i = 0; i < h->bits[l]; i++) huffsize[k++] = l;
    huffsize[k] = 0;
    int lastk = k;
    if (lastk != h->nval) return ORC_E_CORRUPT;
    k = 0; int code = 0, si = huffsize[0];
    while (k < lastk) {
        while (huffsize[k] == si) { huffcode[k++] = code++; }
        if (k >= lastk) break;
        do { code <<= 1; si++; } while (huffsize[k] != si);
    }
    /* a code of length l must fit in l bits (else the table is over-full) */
    for (int i = 0; i < lastk; i++)
        if (huffcode[i] >= (1 << huffsize[i])) return ORC_E_CORRUPT;
    int j = 0;
    for (int l = 1; l <= 16; l++) {
        if (h->bits[l] == 0) { h->maxcode[l] = -1; h->mincode[l] = 0; h->valptr[l] = 0; continue; }
        h->valptr[l] = j;
        h->mincode[l] = huffcode[j];
        j += h->bits[l] - 1;
        h->maxcode[l] = huffcode[j];
        j++;
    }
    h->maxcode[17] = 0x7FFFFFFF;
    return ORC_OK;
}

/* ------------------------------------------------------------- parsing -- */
struct orc_jpeg {
    int w, h, sampling, mcu_cols, mcu_rows, n_mcu, n_du;
    int comp_id[3], comp_hv[3], comp_tq[3], comp_td[3], comp_ta[3];
    uint16_t qt[4][64];   /* natural order */
    int qt_present[4];
    huff_t dc[4], ac[4];
    uint8_t *ecs;         /* de-stuffed entropy-coded segment */
    uint64_t ecs_bits;
};

static int rd16(const uint8_t *p) { return (p[0] << 8) | p[1]; }

orc_jpeg *orc_open(const uint8_t *d, size_t len, int *err) {
    int e = ORC_E_CORRUPT;
    orc_jpeg *j = (orc_jpeg *)calloc(1, sizeof *j);
    if (!j) { if (err) *err = ORC_E_ARG; return NULL; }
    if (!d || len < 4 || d[0] != 0xFF || d[1] != 0xD8) goto fail;
    size_t p = 2;
    int have_sof = 0, have_sos = 0;
    while (p + 4 <= len && !have_sos) {
        if (d[p] != 0xFF) goto fail;
        int m = d[p + 1];
        if (m == 0xFF) { p++; continue; }                       /* fill byte */
        int L = rd16(d + p + 2);
        if (L < 2 || p + 2 + (size_t)L > len) goto fail;
        const uint8_t *s = d + p + 4; int n = L - 2;
        if (m == 0xDB) {                                        /* DQT */
            int o = 0;
            while (o < n) {
                int pq = s[o] >> 4, tq = s[o] & 15;
                if (pq != 0) { e = ORC_E_UNSUPPORTED; goto fail; }
                if (tq > 3 || o + 65 > n) goto fail;
                for (int i = 0; i < 64; i++) j->qt[tq][ZZ_TO_NAT[i]] = s[o + 1 + i];
                j->qt_present[tq] = 1;
                o += 65;
            }
        } else if (m == 0xC4) {                                 /* DHT */
            int o = 0;
            while (o < n) {
                if (o + 17 > n) goto fail;
                int tc = s[o] >> 4, th = s[o] & 15;
                if (tc > 1 || th > 3) goto fail;
                huff_t *h = tc ? &j->ac[th] : &j->dc[th];
                memset(h, 0, sizeof *h);
                int tot = 0;
                for (int l = 1; l <= 16; l++) { h->bits[l] = s[o + l]; tot += h->bits[l]; }
                if (tot > 256 || o + 17 + tot > n) goto fail;
                memcpy(h->val, s + o + 17, (size_t)tot);
                h->nval = tot;
                if (huff_generate(h) != ORC_OK) goto fail;
                h->present = 1;
                o += 17 + tot;
            }
        } else if (m == 0xC0) {                                 /* SOF0 */
            if (n < 6) goto fail;
            if (s[0] != 8) { e = ORC_E_UNSUPPORTED; goto fail; }
            j->h = rd16(s + 1); j->w = rd16(s + 3);
            if (s[5] != 3 || n < 6 + 9) { e = ORC_E_UNSUPPORTED; goto fail; }
            for (int c = 0; c < 3; c++) {
                j->comp_id[c] = s[6 + 3 * c]; j->comp_hv[c] = s[7 + 3 * c]; j->comp_tq[c] = s[8 + 3 * c];
                if (j->comp_tq[c] > 3) goto fail;
            }
            if (j->comp_hv[0] == 0x22 && j->comp_hv[1] == 0x11 && j->comp_hv[2] == 0x11) j->sampling = 420;
            else if (j->comp_hv[0] == 0x11 && j->comp_hv[1] == 0x11 && j->comp_hv[2] == 0x11) j->sampling = 444;
            else { e = ORC_E_UNSUPPORTED; goto fail; }
            if (j->w <= 0 || j->h <= 0) { e = ORC_E_UNSUPPORTED; goto fail; }
            have_sof = 1;
        } else if (m == 0xDD) {                                 /* DRI */
            if (n >= 2 && rd16(s) != 0) { e = ORC_E_UNSUPPORTED; goto fail; }
        } else if ((m >= 0xC1 && m <= 0xCF && m != 0xC4 && m != 0xC8 && m != 0xCC)) {
            e = ORC_E_UNSUPPORTED; goto fail;                   /* other SOF */
        } else if (m == 0xDA) {                                 /* SOS */
            if (!have_sof || n < 1 || s[0] != 3 || n < 1 + 6 + 3) { e = ORC_E_UNSUPPORTED; goto fail; }
            for (int c = 0; c < 3; c++) {
                if (s[1 + 2 * c] != j->comp_id[c]) { e = ORC_E_UNSUPPORTED; goto fail; }
                j->comp_td[c] = s[2 + 2 * c] >> 4; j->comp_ta[c] = s[2 + 2 * c] & 15;
                if (j->comp_td[c] > 3 || j->comp_ta[c] > 3) goto fail;
            }
            if (s[7] != 0 || s[8] != 63 || s[9] != 0) { e = ORC_E_UNSUPPORTED; goto fail; }
            have_sos = 1;
        } else if (m == 0xD9 || m == 0xD8) {
            goto fail;
        }
        p += 2 + (size_t)L;
    }
    if (!have_sos) goto fail;
    for (int c = 0; c < 3; c++) {
        if (!j->qt_present[j->comp_tq[c]] || !j->dc[j->comp_td[c]].present || !j->ac[j->comp_ta[c]].present)
            goto fail;
    }
    /* de-stuff the segment: drop the 0x00 after each 0xFF, stop at a marker */
    j->ecs = (uint8_t *)malloc(len - p + 1);
    if (!j->ecs) goto fail;
    size_t n = 0;
    while (p < len) {
        if (d[p] == 0xFF) {
            if (p + 1 < len && d[p + 1] == 0x00) { j->ecs[n++] = 0xFF; p += 2; continue; }
            break;
        }
        j->ecs[n++] = d[p++];
    }
    j->ecs_bits = (uint64_t)n * 8;
    int ms = j->sampling == 420 ? 16 : 8;
    j->mcu_cols = (j->w + ms - 1) / ms; j->mcu_rows = (j->h + ms - 1) / ms;
    j->n_mcu = j->mcu_cols * j->mcu_rows;
    j->n_du = j->sampling == 420 ? 6 : 3;
    if (err) *err = ORC_OK;
    return j;
fail:
    free(j->ecs); free(j);
    if (err) *err = e;
    return NULL;
}

void orc_close(orc_jpeg *j) { if (j) { free(j->ecs); free(j); } }

int orc_info(const orc_jpeg *j, int64_t info[10]) {
    if (!j || !info) return ORC_E_ARG;
    info[0] = j->w; info[1] = j->h; info[2] = j->sampling; info[3] = j->mcu_cols; info[4] = j->mcu_rows;
    info[5] = j->n_mcu; info[6] = j->n_du; info[7] = (int64_t)j->ecs_bits;
    info[8] = j->comp_tq[0]; info[9] = j->comp_tq[1];
    return ORC_OK;
}

int orc_quant(const orc_jpeg *j, uint16_t q[128]) {
    if (!j || !q) return ORC_E_ARG;
    memcpy(q, j->qt[j->comp_tq[0]], 64 * sizeof(uint16_t));
    memcpy(q + 64, j->qt[j->comp_tq[1]], 64 * sizeof(uint16_t));
    return ORC_OK;
}

/* ------------------------------------------------------- bit reading -- */
/* A bit source: either the de-stuffed byte segment (MSB first) or the
 * library's 32-bit word stream (MSB of word 0 first). */
typedef struct {
    const uint8_t *bytes; const uint32_t *words;
    uint64_t nbits, pos;
    int overrun;
} bits_t;

static int nextbit(bits_t *b) {
    if (b->pos >= b->nbits) { b->overrun = 1; b->pos++; return 0; }
    uint64_t p = b->pos++;
    if (b->bytes) return (b->bytes[p >> 3] >> (7 - (p & 7))) & 1;
    return (int)((b->words[p >> 5] >> (31 - (p & 31))) & 1u);
}

/* RECEIVE (F.2.2.4) */
static int receive(bits_t *b, int s) {
    int v = 0;
    for (int i = 0; i < s; i++) v = (v << 1) | nextbit(b);
    return v;
}

/* EXTEND (F.2.2.1) */
static int extend(int v, int t) { return (t && v < (1 << (t - 1))) ? v - (1 << t) + 1 : v; }

/* DECODE (F.2.2.3), bit-serial. Returns the symbol or -1 for an invalid code. */
static int decode_sym(bits_t *b, const huff_t *h) {
    int i = 1;
    int32_t code = nextbit(b);
    while (code > h->maxcode[i]) {
        if (++i > 16) return -1;
        code = (code << 1) | nextbit(b);
    }
    return h->val[h->valptr[i] + code - h->mincode[i]];
}

/* Decode the AC coefficients of one data unit (F.2.2.2) into zz[1..63]. */
static int decode_acs(bits_t *b, const huff_t *ac, int16_t zz[64]) {
    int k = 1;
    while (k < 64) {
        int rs = decode_sym(b, ac);
        if (rs < 0) return ORC_E_CORRUPT;
        int r = rs >> 4, s = rs & 15;
        if (s == 0) {
            if (r == 15) { k += 16; continue; }   /* ZRL: sixteen zeros */
            if (r != 0) return ORC_E_CORRUPT;      /* (r, 0) is defined only for r = 0 and 15 */
            break;                                 /* EOB */
        }
        if (s > 10) return ORC_E_CORRUPT;          /* baseline AC magnitudes take at most 10 bits (F.1.2.2) */
        k += r;
        if (k > 63) return ORC_E_CORRUPT;
        zz[k] = (int16_t)extend(receive(b, s), s);
        k++;
    }
    if (k > 64) return ORC_E_CORRUPT;
    return b->overrun ? ORC_E_CORRUPT : ORC_OK;
}

static int comp_of_du(const orc_jpeg *j, int d) {
    return j->sampling == 420 ? (d < 4 ? 0 : d - 3) : d;
}

/* One MCU in the original stream (the body of the F.2 MCU loop). */
static int decode_mcu(const orc_jpeg *j, bits_t *b, int32_t pred[3], int16_t *out, uint32_t *dc_bits) {
    if (dc_bits) *dc_bits = 0;
    for (int d = 0; d < j->n_du; d++) {
        int c = comp_of_du(j, d);
        int16_t zz[64];
        memset(zz, 0, sizeof zz);
        uint64_t p0 = b->pos;
        int t = decode_sym(b, &j->dc[j->comp_td[c]]);
        if (t < 0 || t > 11) return ORC_E_CORRUPT;
        int diff = extend(receive(b, t), t);
        pred[c] += diff;
        if (pred[c] < -32768 || pred[c] > 32767) return ORC_E_CORRUPT;
        zz[0] = (int16_t)pred[c];
        int first_of_comp = (c != 0) || (d == 0);
        if (dc_bits && first_of_comp) *dc_bits += (uint32_t)(b->pos - p0);
        int e = decode_acs(b, &j->ac[j->comp_ta[c]], zz);
        if (e) return e;
        for (int i = 0; i < 64; i++) out[d * 64 + ZZ_TO_NAT[i]] = zz[i];
    }
    return b->overrun ? ORC_E_CORRUPT : ORC_OK;
}

int orc_decode_seq(const orc_jpeg *j, int16_t *coef, uint64_t *mcu_bit, int32_t *pred_out, uint32_t *dc_bits) {
    if (!j || !coef) return ORC_E_ARG;
    bits_t b = {j->ecs, NULL, j->ecs_bits, 0, 0};
    int32_t pred[3] = {0, 0, 0};
    for (int m = 0; m < j->n_mcu; m++) {
        if (mcu_bit) mcu_bit[m] = b.pos;
        if (pred_out) { pred_out[3 * m] = pred[0]; pred_out[3 * m + 1] = pred[1]; pred_out[3 * m + 2] = pred[2]; }
        int e = decode_mcu(j, &b, pred, coef + (size_t)m * j->n_du * 64, dc_bits ? dc_bits + m : NULL);
        if (e) return e;
    }
    if (mcu_bit) mcu_bit[j->n_mcu] = b.pos;
    return ORC_OK;
}

int orc_decode_mcu_at(const orc_jpeg *j, uint64_t bitpos, const int32_t pred_in[3], int16_t *out,
                      uint64_t *end_bit) {
    if (!j || !out || !pred_in) return ORC_E_ARG;
    bits_t b = {j->ecs, NULL, j->ecs_bits, bitpos, 0};
    int32_t pred[3] = {pred_in[0], pred_in[1], pred_in[2]};
    int e = decode_mcu(j, &b, pred, out, NULL);
    if (end_bit) *end_bit = b.pos;
    return e;
}

/* -------------------------------------------- stripped-stream access -- */
/* Little-endian bit field of a 64-byte record. */
static uint32_t rec_bits(const uint8_t *rec, int bit, int n) {
    uint32_t v = 0;
    for (int i = 0; i < n; i++) {
        int p = bit + i;
        v |= (uint32_t)((rec[p >> 3] >> (p & 7)) & 1) << i;
    }
    return v;
}

int orc_decode_stripped_mcu(const orc_jpeg *j, const uint32_t *words, uint64_t n_words, uint64_t stream_bits,
                            const uint8_t *records, uint64_t n_records, uint32_t m, int16_t *out,
                            uint64_t *end_bit) {
    if (!j || !words || !records || !out || m >= (uint32_t)j->n_mcu) return ORC_E_ARG;
    uint64_t g = m / 9, r = m % 9;
    if (g >= n_records || stream_bits > n_words * 32) return ORC_E_ARG;
    const uint8_t *rec = records + g * 64;
    uint64_t start = rec_bits(rec, 0, 32);
    if (r) start += rec_bits(rec, 32 + 16 * (int)(r - 1), 16);
    int32_t dc[3];
    for (int c = 0; c < 3; c++) {
        int32_t v = (int32_t)rec_bits(rec, 160 + 12 * (int)(3 * r + c), 12);
        dc[c] = v >= 2048 ? v - 4096 : v;        /* 12-bit two's complement */
    }
    bits_t b = {NULL, words, stream_bits, start, 0};
    int32_t ypred = 0;
    for (int d = 0; d < j->n_du; d++) {
        int c = comp_of_du(j, d);
        int16_t zz[64];
        memset(zz, 0, sizeof zz);
        int absolute = (c != 0) || (d == 0);      /* first Y, Cb, Cr: stored in the record */
        if (absolute) {
            zz[0] = (int16_t)dc[c];
            if (c == 0) ypred = dc[0];
        } else {                                  /* Y1..Y3 of 4:2:0: difference to previous Y */
            int t = decode_sym(&b, &j->dc[j->comp_td[0]]);
            if (t < 0 || t > 11) return ORC_E_CORRUPT;
            ypred += extend(receive(&b, t), t);
            if (ypred < -32768 || ypred > 32767) return ORC_E_CORRUPT;
            zz[0] = (int16_t)ypred;
        }
        int e = decode_acs(&b, &j->ac[j->comp_ta[c]], zz);
        if (e) return e;
        for (int i = 0; i < 64; i++) out[d * 64 + ZZ_TO_NAT[i]] = zz[i];
    }
    if (end_bit) *end_bit = b.pos;
    return b.overrun ? ORC_E_CORRUPT : ORC_OK;
}

/* ------------------------------------- predictor-index random access -- */
/* The index reading with the segment untouched: the record's offsets point
 * into the original (de-stuffed) segment and its 12-bit fields hold the DC
 * predictors in force when each MCU starts; the MCU is then the plain F.2
 * MCU body started there with those predictors. */
int orc_decode_predicted_mcu(const orc_jpeg *j, const uint32_t *words, uint64_t n_words, uint64_t stream_bits,
                             const uint8_t *records, uint64_t n_records, uint32_t m, int16_t *out,
                             uint64_t *end_bit) {
    if (!j || !words || !records || !out || m >= (uint32_t)j->n_mcu) return ORC_E_ARG;
    uint64_t g = m / 9, r = m % 9;
    if (g >= n_records || stream_bits > n_words * 32) return ORC_E_ARG;
    const uint8_t *rec = records + g * 64;
    uint64_t start = rec_bits(rec, 0, 32);
    if (r) start += rec_bits(rec, 32 + 16 * (int)(r - 1), 16);
    int32_t pred[3];
    for (int c = 0; c < 3; c++) {
        int32_t v = (int32_t)rec_bits(rec, 160 + 12 * (int)(3 * r + c), 12);
        pred[c] = v >= 2048 ? v - 4096 : v;
    }
    bits_t b = {NULL, words, stream_bits, start, 0};
    int e = decode_mcu(j, &b, pred, out, NULL);
    if (end_bit) *end_bit = b.pos;
    return e;
}

/* --------------------------------------------------------------- IDCT -- */
#define ORC_PI 3.14159265358979323846

void orc_idct(const double F[64], double out[64]) {
    double cs[8][8];   /* cs[freq][pos] = cos((2 pos + 1) freq pi / 16) */
    for (int f = 0; f < 8; f++)
        for (int x = 0; x < 8; x++) cs[f][x] = cos((2 * x + 1) * f * ORC_PI / 16.0);
    for (int y = 0; y < 8; y++)
        for (int x = 0; x < 8; x++) {
            double s = 0.0;
            for (int v = 0; v < 8; v++)
                for (int u = 0; u < 8; u++) {
                    double f = F[v * 8 + u];
                    if (f == 0.0) continue;
                    double cu = u ? 1.0 : 1.0 / sqrt(2.0), cv = v ? 1.0 : 1.0 / sqrt(2.0);
                    s += cu * cv * f * cs[u][x] * cs[v][y];
                }
            out[y * 8 + x] = 0.25 * s;
        }
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : v > hi ? hi : v; }

/* Texels of one MCU (reading "single rounding"). tile = ms x ms texels. */
static void mcu_texels(const orc_jpeg *j, const int16_t *cm, uint8_t *rgb, double *f64) {
    const int ms = j->sampling == 420 ? 16 : 8;
    double samp[6][64];
    for (int d = 0; d < j->n_du; d++) {
        int c = comp_of_du(j, d);
        const uint16_t *q = j->qt[j->comp_tq[c]];
        double F[64];
        for (int k = 0; k < 64; k++) F[k] = (double)cm[d * 64 + k] * (double)q[k];
        orc_idct(F, samp[d]);
    }
    for (int ty = 0; ty < ms; ty++)
        for (int tx = 0; tx < ms; tx++) {
            double Y, Cb, Cr;
            if (j->sampling == 420) {
                int du = (ty / 8) * 2 + tx / 8;
                Y = samp[du][(ty % 8) * 8 + tx % 8];
                Cb = samp[4][(ty / 2) * 8 + tx / 2];
                Cr = samp[5][(ty / 2) * 8 + tx / 2];
            } else {
                Y = samp[0][ty * 8 + tx]; Cb = samp[1][ty * 8 + tx]; Cr = samp[2][ty * 8 + tx];
            }
            Y = clampd(Y + 128.0, 0.0, 255.0);
            Cb = clampd(Cb + 128.0, 0.0, 255.0) - 128.0;
            Cr = clampd(Cr + 128.0, 0.0, 255.0) - 128.0;
            double rgbv[3] = {Y + 1.402 * Cr, Y - 0.344136 * Cb - 0.714136 * Cr, Y + 1.772 * Cb};
            for (int c = 0; c < 3; c++) {
                size_t o = ((size_t)ty * ms + tx) * 3 + c;
                if (f64) f64[o] = rgbv[c];
                if (rgb) rgb[o] = (uint8_t)clampd(floor(rgbv[c] + 0.5), 0.0, 255.0);
            }
        }
}

/* Reduced-resolution texels of one MCU (the paper's Discussion: lower
 * resolutions from the DC and the first ACs instead of stored mip levels):
 * each data unit's N x N samples, N = 8 >> s, by the N-point inverse DCT of
 * its top-left N x N coefficients with the 8-point scaling,
 * r(x,y) = 1/4 sum_{u,v<N} C(u) C(v) F(v,u) cos((2x+1)u pi/2N) cos((2y+1)v pi/2N)
 * (N = 1: the block mean F00/8), then as mcu_texels: +128 and clamp, chroma
 * replicated over 2x2 luma samples (4:2:0), colour with a single rounding.
 * out_rgb: the (16 >> s) or (8 >> s) square tile, 3 bytes per texel. */
static void mcu_reduced(const orc_jpeg *j, const int16_t *cm, int s, uint8_t *rgb, double *f64) {
    const int N = 8 >> s, ms = (j->sampling == 420 ? 16 : 8) >> s;
    double samp[6][64];
    for (int d = 0; d < j->n_du; d++) {
        int c = comp_of_du(j, d);
        const uint16_t *q = j->qt[j->comp_tq[c]];
        for (int y = 0; y < N; y++)
            for (int x = 0; x < N; x++) {
                double acc = 0.0;
                for (int v = 0; v < N; v++)
                    for (int u = 0; u < N; u++) {
                        double F = (double)cm[d * 64 + v * 8 + u] * (double)q[v * 8 + u];
                        double cu = u ? 1.0 : 1.0 / sqrt(2.0), cv = v ? 1.0 : 1.0 / sqrt(2.0);
                        acc += cu * cv * F * cos((2 * x + 1) * u * ORC_PI / (2.0 * N)) *
                               cos((2 * y + 1) * v * ORC_PI / (2.0 * N));
                    }
                samp[d][y * N + x] = 0.25 * acc;
            }
    }
    for (int ty = 0; ty < ms; ty++)
        for (int tx = 0; tx < ms; tx++) {
            double Y, Cb, Cr;
            if (j->sampling == 420) {
                int du = (ty / N) * 2 + tx / N;
                Y = samp[du][(ty % N) * N + tx % N];
                Cb = samp[4][(ty / 2) * N + tx / 2];
                Cr = samp[5][(ty / 2) * N + tx / 2];
            } else {
                Y = samp[0][ty * N + tx]; Cb = samp[1][ty * N + tx]; Cr = samp[2][ty * N + tx];
            }
            Y = clampd(Y + 128.0, 0.0, 255.0);
            Cb = clampd(Cb + 128.0, 0.0, 255.0) - 128.0;
            Cr = clampd(Cr + 128.0, 0.0, 255.0) - 128.0;
            double rgbv[3] = {Y + 1.402 * Cr, Y - 0.344136 * Cb - 0.714136 * Cr, Y + 1.772 * Cb};
            for (int c = 0; c < 3; c++) {
                size_t o = ((size_t)ty * ms + tx) * 3 + c;
                if (f64) f64[o] = rgbv[c];
                if (rgb) rgb[o] = (uint8_t)clampd(floor(rgbv[c] + 0.5), 0.0, 255.0);
            }
        }
}

int orc_mcu_reduced(const orc_jpeg *j, const int16_t *coef_mcu, int scale_log2, uint8_t *out_rgb, double *out_f64) {
    if (!j || !coef_mcu || scale_log2 < 0 || scale_log2 > 3) return ORC_E_ARG;
    mcu_reduced(j, coef_mcu, scale_log2, out_rgb, out_f64);
    return ORC_OK;
}

int orc_mcu_pixels(const orc_jpeg *j, const int16_t *coef_mcu, uint8_t *out_rgb, double *out_f64) {
    if (!j || !coef_mcu) return ORC_E_ARG;
    mcu_texels(j, coef_mcu, out_rgb, out_f64);
    return ORC_OK;
}

int orc_pixels(const orc_jpeg *j, const int16_t *coef, uint8_t *rgb, double *rgb_f64) {
    if (!j || !coef) return ORC_E_ARG;
    const int ms = j->sampling == 420 ? 16 : 8;
    uint8_t tile[16 * 16 * 3];
    double tf[16 * 16 * 3];
    for (int my = 0; my < j->mcu_rows; my++)
        for (int mx = 0; mx < j->mcu_cols; mx++) {
            mcu_texels(j, coef + ((size_t)my * j->mcu_cols + mx) * j->n_du * 64, tile, rgb_f64 ? tf : NULL);
            for (int ty = 0; ty < ms; ty++)
                for (int tx = 0; tx < ms; tx++) {
                    int x = mx * ms + tx, y = my * ms + ty;
                    if (x >= j->w || y >= j->h) continue;
                    for (int c = 0; c < 3; c++) {
                        size_t o = ((size_t)y * j->w + x) * 3 + c, t = ((size_t)ty * ms + tx) * 3 + c;
                        if (rgb) rgb[o] = tile[t];
                        if (rgb_f64) rgb_f64[o] = tf[t];
                    }
                }
        }
    return ORC_OK;
}

/* ---------------------------------------------------- scene sampling -- */
uint64_t orc_scene_layout(int n_levels, const int32_t *lev_w, const int32_t *lev_h, uint32_t *blk_base) {
    uint64_t next = 0;
    for (int l = 0; l < n_levels; l++) {
        uint64_t bc = ((uint64_t)lev_w[l] + 15) / 16, br = ((uint64_t)lev_h[l] + 15) / 16;
        blk_base[l] = (uint32_t)next;
        next += bc * br;
        next = (next + 31) / 32 * 32;
    }
    return next;
}

/* One filter tap: a texel of one level and its integer weight. */
/* w: bilinear weight (the taps of one level sum to 65536); lw: weight of
 * the tap's level out of 256 (trilinear), 256 otherwise. */
typedef struct { int level; int64_t x, y; int64_t w; int64_t lw; } tap_t;

static int64_t mod_pos(int64_t a, int64_t n) { int64_t r = a % n; return r < 0 ? r + n : r; }

/* Texel coordinates along one axis, fp32 as the method defines them:
 * nearest: s = u*w, texel floor(s);  linear: s = u*w - 0.5, texels floor(s)
 * and floor(s)+1 with weights 256-f and f, f = floor(frac(s)*256 + 0.5).
 * Multiplication and subtraction are separate fp32 operations (no fused
 * multiply-add).  Returns 0 if the coordinate is not finite or |s| >= 2^30. */
static int axis(float u, int w, int linear, int64_t *x0, int64_t *x1, int *f) {
    volatile float prod = u * (float)w;       /* volatile: one rounding per op */
    float s = linear ? (float)(prod - 0.5f) : (float)prod;
    if (!isfinite(s) || fabsf(s) >= 1073741824.0f) return 0;
    float fl = floorf(s);
    if (linear) {
        volatile float fr = s - fl;
        volatile float sc = fr * 256.0f;
        float t = sc + 0.5f;
        *f = (int)floorf(t);
    } else {
        *f = 0;
    }
    *x0 = mod_pos((int64_t)fl, w);
    *x1 = mod_pos((int64_t)fl + 1, w);
    return 1;
}

/* All taps of a pixel with non-zero weight (paper: Resolve subsection;
 * mip levels as in "Multiple Textures and Mip Mapping").  Weights of the
 * bilinear taps sum to 65536 per level.  Returns the number of taps, or -1
 * for an invalid pixel.  For trilinear, *tw = weight of the second level
 * in [0,256] and level_of_tap distinguishes the two levels. */
static int pixel_taps(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                      const int32_t *lev_h, const orc_gpixel *px, int filter_flags, tap_t taps[8], int *lv0, int *lv1,
                      int *tw) {
    const int filter = filter_flags & ORC_FILTER_MASK;
    if (px->tex >= (uint32_t)n_tex) return -1;
    if (!isfinite(px->u) || !isfinite(px->v) || !isfinite(px->lod)) return -1;
    int L = tex_count[px->tex], first = tex_first[px->tex];
    if (L <= 0) return -1;
    /* without mip mapping every pixel samples level 0 */
    if (filter_flags & ORC_NO_MIP) L = 1;
    int lv[2]; int lw[2]; int nl;
    if (filter == ORC_TRILINEAR) {
        float lod = px->lod;
        if (lod < 0.0f) { lv[0] = 0; nl = 1; *tw = 0; }
        else if (lod >= (float)(L - 1)) { lv[0] = L - 1; nl = 1; *tw = 0; }
        else {
            float fl = floorf(lod);
            volatile float fr = lod - fl;
            volatile float sc = fr * 256.0f;
            float t = sc + 0.5f;
            int tt = (int)floorf(t);
            lv[0] = (int)fl; lv[1] = lv[0] + 1; nl = 2; *tw = tt;
        }
        if (nl == 1) { lw[0] = 256; }
        else { lw[0] = 256 - *tw; lw[1] = *tw; }
    } else {
        float t = px->lod + 0.5f;
        int l;
        if (!(t >= 1.0f)) l = 0;                          /* includes floor(t) <= 0 */
        else if (t >= (float)(L - 1)) l = L - 1;
        else l = (int)floorf(t);
        lv[0] = l; lw[0] = 256; nl = 1; *tw = 0;
    }
    *lv0 = first + lv[0]; *lv1 = nl == 2 ? first + lv[1] : first + lv[0];
    int n = 0;
    for (int k = 0; k < nl; k++) {
        if (lw[k] == 0) continue;
        int lev = first + lv[k];
        int w = lev_w[lev], h = lev_h[lev];
        int64_t x0, x1, y0, y1; int fx, fy;
        int lin = filter != ORC_NEAREST;
        if (!axis(px->u, w, lin, &x0, &x1, &fx) || !axis(px->v, h, lin, &y0, &y1, &fy)) return -1;
        if (filter == ORC_BILINEAR_CLAMPED) {
            /* the paper's single-MCU variant: a tap outside the block of the
             * texel under the sample point (the nearest filter's texel) reads
             * that texel's row or column instead */
            int64_t xc, yc, d0, d1; int f0;
            axis(px->u, w, 0, &xc, &d0, &f0);
            axis(px->v, h, 0, &yc, &d1, &f0);
            if (x0 / 16 != xc / 16) x0 = xc;
            if (x1 / 16 != xc / 16) x1 = xc;
            if (y0 / 16 != yc / 16) y0 = yc;
            if (y1 / 16 != yc / 16) y1 = yc;
        }
        if (!lin) {
            taps[n++] = (tap_t){lev, x0, y0, 65536, lw[k]};
        } else {
            int64_t wx[2] = {256 - fx, fx}, wy[2] = {256 - fy, fy};
            int64_t xs[2] = {x0, x1}, ys[2] = {y0, y1};
            for (int b = 0; b < 2; b++)
                for (int a = 0; a < 2; a++) {
                    int64_t wt = wx[a] * wy[b];
                    if (wt == 0) continue;
                    taps[n++] = (tap_t){lev, xs[a], ys[b], wt, lw[k]};
                }
        }
    }
    return n;
}

int64_t orc_mark(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                 const int32_t *lev_h, const uint32_t *blk_base, const orc_gpixel *g, int64_t n_px, int filter,
                 uint8_t *vis) {
    /* (filter: ORC_* mode, optionally with ORC_NO_MIP) */
    int64_t bad = 0;
    for (int64_t i = 0; i < n_px; i++) {
        if (g[i].tex == 0xFFFFFFFFu) continue;
        tap_t taps[8]; int l0, l1, tw;
        int n = pixel_taps(n_tex, tex_first, tex_count, lev_w, lev_h, &g[i], filter, taps, &l0, &l1, &tw);
        if (n < 0) { bad++; continue; }
        for (int k = 0; k < n; k++) {
            int64_t bc = (lev_w[taps[k].level] + 15) / 16;
            uint64_t b = blk_base[taps[k].level] + (uint64_t)(taps[k].y / 16) * (uint64_t)bc + (uint64_t)(taps[k].x / 16);
            vis[b] = 1;
        }
    }
    return bad;
}

int64_t orc_resolve(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                    const int32_t *lev_h, const uint8_t *const *level_rgb, const double *const *level_f64,
                    const orc_gpixel *g, int64_t n_px, int filter, uint32_t *frame, double *frame_f64) {
    int64_t bad = 0;
    for (int64_t i = 0; i < n_px; i++) {
        if (frame_f64) frame_f64[3 * i] = frame_f64[3 * i + 1] = frame_f64[3 * i + 2] = 0.0;
        if (g[i].tex == 0xFFFFFFFFu) { frame[i] = 0; continue; }
        tap_t taps[8]; int l0, l1, tw;
        int n = pixel_taps(n_tex, tex_first, tex_count, lev_w, lev_h, &g[i], filter, taps, &l0, &l1, &tw);
        if (n < 0) { frame[i] = 0xFFFF00FFu; bad++; continue; }
        int64_t acc[2][3] = {{0, 0, 0}, {0, 0, 0}};
        int missing = 0;
        for (int k = 0; k < n; k++) {
            const uint8_t *img = level_rgb[taps[k].level];
            if (!img) { missing = 1; break; }
            int side = ((filter & ORC_FILTER_MASK) == ORC_TRILINEAR && taps[k].level != l0) ? 1 : 0;
            const uint8_t *t = img + ((size_t)taps[k].y * lev_w[taps[k].level] + (size_t)taps[k].x) * 3;
            for (int c = 0; c < 3; c++) acc[side][c] += (int64_t)t[c] * taps[k].w;
            if (frame_f64) {
                const double *tf = level_f64 ? level_f64[taps[k].level] : NULL;
                for (int c = 0; c < 3; c++) {
                    double tv = tf ? tf[((size_t)taps[k].y * lev_w[taps[k].level] + (size_t)taps[k].x) * 3 + c]
                                   : (double)t[c];
                    frame_f64[3 * i + c] += tv * ((double)taps[k].w / 65536.0) * ((double)taps[k].lw / 256.0);
                }
            }
        }
        if (missing) { frame[i] = 0xFFFF00FFu; bad++; continue; }
        uint32_t rgb[3];
        for (int c = 0; c < 3; c++) {
            int64_t a = (acc[0][c] + 32768) >> 16;
            if ((filter & ORC_FILTER_MASK) == ORC_TRILINEAR && l1 != l0) {
                int64_t b = (acc[1][c] + 32768) >> 16;
                /* a level whose weight is zero contributed no taps (acc = 0) */
                a = (a * (256 - tw) + b * tw + 128) >> 8;
            }
            rgb[c] = (uint32_t)a;
        }
        frame[i] = rgb[0] | (rgb[1] << 8) | (rgb[2] << 16) | 0xFF000000u;
    }
    return bad;
}

int64_t orc_taps(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                 const int32_t *lev_h, const orc_gpixel *g, int64_t n_px, int filter, int32_t *level, int32_t *x,
                 int32_t *y, double *w) {
    int64_t bad = 0;
    for (int64_t i = 0; i < n_px; i++) {
        for (int k = 0; k < 8; k++) {
            level[8 * i + k] = -1; x[8 * i + k] = 0; y[8 * i + k] = 0; w[8 * i + k] = 0.0;
        }
        if (g[i].tex == 0xFFFFFFFFu) continue;
        tap_t taps[8]; int l0, l1, tw;
        int n = pixel_taps(n_tex, tex_first, tex_count, lev_w, lev_h, &g[i], filter, taps, &l0, &l1, &tw);
        if (n < 0) { bad++; continue; }
        for (int k = 0; k < n; k++) {
            level[8 * i + k] = taps[k].level;
            x[8 * i + k] = (int32_t)taps[k].x;
            y[8 * i + k] = (int32_t)taps[k].y;
            w[8 * i + k] = ((double)taps[k].w / 65536.0) * ((double)taps[k].lw / 256.0);
        }
    }
    return bad;
}
