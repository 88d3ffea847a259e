// Host side of libjpt: the offline per-level index (paper, Implementation
// details: "Indexing Table" and "Memory Overhead"), the GPU decode tables and
// the scene's block-id layout.  Plain C++17, no HIP calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "jpt.h"
#include "jpt_internal.h"

// The argument structs keep fixed sizes (bindings mirror them field by field).
static_assert(sizeof(jpt_level_desc) == 64 && sizeof(jpt_texture_desc) == 16, "descriptor layout");
static_assert(sizeof(jpt_scene) == 64 && sizeof(jpt_view) == 32 && sizeof(jpt_frame) == 48, "argument layout");
static_assert(sizeof(jpt_triangle) == 80 && sizeof(jpt_camera) == 64, "geometry layout");
static_assert(sizeof(jpt_cache) == 88 && sizeof(jpt_level_info) == 1464, "cache and level info layout");
static_assert(sizeof(jpt_bc1_level) == 24 && sizeof(jpt_bc1_scene) == 24, "BC1 layout");

namespace {

// --------------------------------------------------------------- parsing
struct HuffSpec {
    bool present = false;
    uint8_t bits[16] = {};
    uint8_t vals[256] = {};
    int n = 0;
};

struct Parsed {
    int w = 0, h = 0, sampling = 0;
    int comp_id[3] = {}, hv[3] = {}, tq[3] = {}, td[3] = {}, ta[3] = {};
    uint16_t qt_zz[4][64] = {};  // zigzag order as stored in DQT
    bool qt_present[4] = {};
    HuffSpec dc[4], ac[4];
    std::vector<uint8_t> ecs;    // de-stuffed scan bytes
};

inline int be16(const uint8_t *p) { return (p[0] << 8) | p[1]; }

jpt_status parse(const uint8_t *d, size_t len, Parsed &P) {
    if (!d || len < 4 || d[0] != 0xFF || d[1] != 0xD8) return JPT_E_CORRUPT;
    size_t p = 2;
    bool sof = false, sos = false;
    while (!sos) {
        if (p + 4 > len) return JPT_E_CORRUPT;
        if (d[p] != 0xFF) return JPT_E_CORRUPT;
        int m = d[p + 1];
        if (m == 0xFF) { p++; continue; }
        if (m == 0xD8 || m == 0xD9 || (m >= 0xD0 && m <= 0xD7) || m == 0x01) return JPT_E_CORRUPT;
        int L = be16(d + p + 2);
        if (L < 2 || p + 2 + (size_t)L > len) return JPT_E_CORRUPT;
        const uint8_t *s = d + p + 4;
        int n = L - 2;
        switch (m) {
        case 0xDB:
            for (int o = 0; o < n;) {
                int pq = s[o] >> 4, t = s[o] & 15;
                if (pq) return JPT_E_UNSUPPORTED;
                if (t > 3 || o + 65 > n) return JPT_E_CORRUPT;
                for (int i = 0; i < 64; i++) P.qt_zz[t][i] = s[o + 1 + i];
                P.qt_present[t] = true;
                o += 65;
            }
            break;
        case 0xC4:
            for (int o = 0; o < n;) {
                if (o + 17 > n) return JPT_E_CORRUPT;
                int tc = s[o] >> 4, th = s[o] & 15;
                if (tc > 1 || th > 3) return JPT_E_CORRUPT;
                HuffSpec &H = tc ? P.ac[th] : P.dc[th];
                H = HuffSpec();
                int tot = 0;
                for (int i = 0; i < 16; i++) { H.bits[i] = s[o + 1 + i]; tot += H.bits[i]; }
                if (tot > 256 || o + 17 + tot > n) return JPT_E_CORRUPT;
                std::memcpy(H.vals, s + o + 17, tot);
                H.n = tot;
                H.present = true;
                o += 17 + tot;
            }
            break;
        case 0xC0: {
            if (n < 6) return JPT_E_CORRUPT;
            if (s[0] != 8 || s[5] != 3) return JPT_E_UNSUPPORTED;
            if (n < 15) return JPT_E_CORRUPT;
            P.h = be16(s + 1);
            P.w = be16(s + 3);
            for (int c = 0; c < 3; c++) {
                P.comp_id[c] = s[6 + 3 * c];
                P.hv[c] = s[7 + 3 * c];
                P.tq[c] = s[8 + 3 * c];
                if (P.tq[c] > 3) return JPT_E_CORRUPT;
            }
            if (P.hv[1] != 0x11 || P.hv[2] != 0x11) return JPT_E_UNSUPPORTED;
            if (P.hv[0] == 0x22) P.sampling = 420;
            else if (P.hv[0] == 0x11) P.sampling = 444;
            else return JPT_E_UNSUPPORTED;
            if (P.w == 0 || P.h == 0) return JPT_E_UNSUPPORTED;
            sof = true;
            break;
        }
        case 0xDD:
            if (n >= 2 && be16(s) != 0) return JPT_E_UNSUPPORTED;
            break;
        case 0xDA: {
            if (!sof) return JPT_E_CORRUPT;
            if (n < 10 || s[0] != 3) return JPT_E_UNSUPPORTED;
            for (int c = 0; c < 3; c++) {
                if (s[1 + 2 * c] != P.comp_id[c]) return JPT_E_UNSUPPORTED;
                P.td[c] = s[2 + 2 * c] >> 4;
                P.ta[c] = s[2 + 2 * c] & 15;
                if (P.td[c] > 3 || P.ta[c] > 3) return JPT_E_CORRUPT;
            }
            if (s[7] != 0 || s[8] != 63 || s[9] != 0) return JPT_E_UNSUPPORTED;
            sos = true;
            break;
        }
        default:
            if (m >= 0xC1 && m <= 0xCF && m != 0xC4 && m != 0xC8 && m != 0xCC) return JPT_E_UNSUPPORTED;
            break;  // APPn, COM, DNL... skipped
        }
        p += 2 + (size_t)L;
    }
    for (int c = 0; c < 3; c++)
        if (!P.qt_present[P.tq[c]] || !P.dc[P.td[c]].present || !P.ac[P.ta[c]].present) return JPT_E_CORRUPT;
    if (P.tq[1] != P.tq[2] || P.td[1] != P.td[2] || P.ta[1] != P.ta[2]) return JPT_E_UNSUPPORTED;
    P.ecs.reserve(len - p + 8);
    while (p < len) {
        if (d[p] == 0xFF) {
            if (p + 1 < len && d[p + 1] == 0x00) { P.ecs.push_back(0xFF); p += 2; continue; }
            break;
        }
        P.ecs.push_back(d[p++]);
    }
    return JPT_OK;
}

// ------------------------------------------------------ canonical codes
// Codes of each length are consecutive integers; moving to the next length
// doubles the running code.  first[l] / count[l] / sym_base[l] describe the
// codes of length l (1..16) in symbol order.
struct Canon {
    int32_t first[17] = {}, count[17] = {}, sym_base[17] = {};
    uint8_t vals[256] = {};
    int n = 0;
};

jpt_status canon_build(const HuffSpec &H, Canon &C) {
    int32_t code = 0, k = 0;
    for (int l = 1; l <= 16; l++) {
        C.first[l] = code;
        C.count[l] = H.bits[l - 1];
        C.sym_base[l] = k;
        code += H.bits[l - 1];
        k += H.bits[l - 1];
        if (code > (1 << l)) return JPT_E_CORRUPT;  // over-full
        code <<= 1;
    }
    C.n = k;
    std::memcpy(C.vals, H.vals, 256);
    return JPT_OK;
}

// --------------------------------------------------------- host decoder
// MSB-first reader over the de-stuffed scan; reading past the end yields
// zero bits and is reported by overrun().
struct BitReader {
    const uint8_t *b;
    uint64_t nbits, pos = 0;
    BitReader(const uint8_t *bytes, uint64_t n) : b(bytes), nbits(n) {}
    uint32_t peek32() const {
        uint32_t v = 0;
        uint64_t byte = pos >> 3;
        int sh = (int)(pos & 7);
        uint64_t nbytes = nbits >> 3;
        uint64_t acc = 0;
        for (int i = 0; i < 5; i++) acc = (acc << 8) | (byte + i < nbytes ? b[byte + i] : 0);
        v = (uint32_t)(acc >> (8 - sh));
        return v;
    }
    bool overrun() const { return pos > nbits; }
};

// Decode one symbol: returns symbol or -1; *len = code length.
inline int decode_symbol(const Canon &C, uint32_t peek, int *len) {
    for (int l = 1; l <= 16; l++) {
        int32_t code = (int32_t)(peek >> (32 - l));
        int32_t off = code - C.first[l];
        if (off >= 0 && off < C.count[l]) { *len = l; return C.vals[C.sym_base[l] + off]; }
    }
    return -1;
}

inline int extend_bits(uint32_t v, int s) {
    return (s && v < (1u << (s - 1))) ? (int)v - (1 << s) + 1 : (int)v;
}

// Append bits [from, from+n) of src (MSB-first bytes) to the word stream.
struct WordWriter {
    std::vector<uint32_t> &w;
    uint64_t nbits = 0;
    explicit WordWriter(std::vector<uint32_t> &v) : w(v) {}
    void put(uint32_t v, int n) {  // n <= 32, v right-aligned
        if (!n) return;
        uint64_t word = nbits >> 5;
        int used = (int)(nbits & 31);
        if (word >= w.size()) w.push_back(0);
        uint64_t x = (uint64_t)v << (64 - n);  // left-aligned in 64 bits
        w[word] |= (uint32_t)(x >> (32 + used));
        if (used + n > 32) {
            if (word + 1 >= w.size()) w.push_back(0);
            w[word + 1] |= (uint32_t)(x >> used);
        }
        nbits += n;
    }
};

void copy_bits(WordWriter &out, const uint8_t *src, uint64_t src_nbits, uint64_t from, uint64_t n) {
    BitReader r(src, src_nbits);
    r.pos = from;
    while (n) {
        int take = n > 24 ? 24 : (int)n;
        uint32_t v = r.peek32() >> (32 - take);
        out.put(v, take);
        r.pos += take;
        n -= take;
    }
}

}  // namespace

// ======================================================================
extern "C" jpt_status jpt_build_index(const uint8_t *jpeg, size_t len, jpt_level_info *info, uint32_t *stream_out,
                                      size_t stream_cap_words, uint8_t *records_out, size_t records_cap_bytes) {
    return jpt_build_index_ex(jpeg, len, JPT_INDEX_SPLICED, info, stream_out, stream_cap_words, records_out,
                              records_cap_bytes);
}

extern "C" jpt_status jpt_build_index_ex(const uint8_t *jpeg, size_t len, uint32_t kind, jpt_level_info *info,
                                         uint32_t *stream_out, size_t stream_cap_words, uint8_t *records_out,
                                         size_t records_cap_bytes) {
    if (!jpeg || !info || kind > JPT_INDEX_PREDICTORS) return JPT_E_ARG;
    const bool spliced = kind == JPT_INDEX_SPLICED;
    Parsed P;
    jpt_status st = parse(jpeg, len, P);
    if (st != JPT_OK) return st;

    Canon dcC[2], acC[2];  // [0] luma, [1] chroma
    if ((st = canon_build(P.dc[P.td[0]], dcC[0])) || (st = canon_build(P.ac[P.ta[0]], acC[0])) ||
        (st = canon_build(P.dc[P.td[1]], dcC[1])) || (st = canon_build(P.ac[P.ta[1]], acC[1])))
        return st;

    jpt_level_info I;
    std::memset(&I, 0, sizeof I);
    I.width = P.w;
    I.height = P.h;
    I.sampling = P.sampling;
    const int ms = P.sampling == 420 ? 16 : 8;
    I.mcu_cols = (P.w + ms - 1) / ms;
    I.mcu_rows = (P.h + ms - 1) / ms;
    I.n_mcu = I.mcu_cols * I.mcu_rows;
    I.blk_cols = (P.w + 15) / 16;
    I.blk_rows = (P.h + 15) / 16;
    I.n_records = (I.n_mcu + 8) / 9;
    for (int i = 0; i < 64; i++) {
        I.quant[0][i] = P.qt_zz[P.tq[0]][i];
        I.quant[1][i] = P.qt_zz[P.tq[1]][i];
    }
    const HuffSpec *specs[4] = {&P.dc[P.td[0]], &P.ac[P.ta[0]], &P.dc[P.td[1]], &P.ac[P.ta[1]]};
    for (int t = 0; t < 4; t++) {
        std::memcpy(I.huff_bits[t], specs[t]->bits, 16);
        std::memcpy(I.huff_vals[t], specs[t]->vals, 256);
        I.huff_nvals[t] = (uint16_t)specs[t]->n;
    }

    // Walk the scan once.  For every MCU remember its start in the spliced
    // stream, its absolute first-Y / Cb / Cr DCs, and the bit ranges of the
    // DC codes that the splice removes.
    const int ndu = P.sampling == 420 ? 6 : 3;
    const uint64_t ecs_bits = (uint64_t)P.ecs.size() * 8;
    BitReader br(P.ecs.data(), ecs_bits);
    std::vector<uint32_t> words;
    words.reserve(P.ecs.size() / 4 + 16);
    WordWriter ww(words);
    std::vector<uint64_t> start(I.n_mcu + 1);
    std::vector<int32_t> dcs((size_t)I.n_mcu * 3);
    int32_t pred[3] = {0, 0, 0};
    uint64_t copied_from = 0;  // next original bit not yet copied
    uint64_t removed = 0;
    for (uint32_t m = 0; m < I.n_mcu; m++) {
        start[m] = ww.nbits + (br.pos - copied_from);
        if (!spliced)  // the predictors in force when the MCU starts
            for (int c = 0; c < 3; c++) dcs[(size_t)m * 3 + c] = pred[c];
        for (int d = 0; d < ndu; d++) {
            int c = P.sampling == 420 ? (d < 4 ? 0 : d - 3) : d;
            int tsel = c ? 1 : 0;
            bool absolute = (c != 0) || (d == 0);
            uint64_t dc_from = br.pos;
            int len;
            int s = decode_symbol(dcC[tsel], br.peek32(), &len);
            if (s < 0 || s > 11) return JPT_E_CORRUPT;
            br.pos += len;
            uint32_t raw = s ? (br.peek32() >> (32 - s)) : 0;
            br.pos += s;
            pred[c] += extend_bits(raw, s);
            if (pred[c] < -32768 || pred[c] > 32767) return JPT_E_CORRUPT;
            // every quantised DC of an 8-bit baseline image fits 12 bits; the
            // records store the absolute ones in 12 bits, and the decoders'
            // arithmetic assumes it of the differential ones too
            if (pred[c] < -2048 || pred[c] > 2047) return JPT_E_RANGE;
            if (absolute && spliced) {
                dcs[(size_t)m * 3 + c] = pred[c];
                // splice: copy the pending original bits, skip this DC code
                copy_bits(ww, P.ecs.data(), ecs_bits, copied_from, dc_from - copied_from);
                removed += br.pos - dc_from;
                copied_from = br.pos;
            }
            int k = 1;
            while (k < 64) {
                int rs = decode_symbol(acC[tsel], br.peek32(), &len);
                if (rs < 0) return JPT_E_CORRUPT;
                br.pos += len;
                int r = rs >> 4, sz = rs & 15;
                if (sz == 0) {
                    if (r == 15) { k += 16; continue; }
                    if (r != 0) return JPT_E_CORRUPT;
                    break;
                }
                if (sz > 10) return JPT_E_CORRUPT;
                k += r;
                if (k > 63) return JPT_E_CORRUPT;
                br.pos += sz;
                k++;
            }
            if (k > 64) return JPT_E_CORRUPT;  // a run of zeros (ZRL) past the last position
            if (br.overrun()) return JPT_E_CORRUPT;
        }
    }
    const uint64_t scan_end = br.pos;
    copy_bits(ww, P.ecs.data(), ecs_bits, copied_from, scan_end - copied_from);
    start[I.n_mcu] = ww.nbits;
    if (ww.nbits >= 0xFFFFFFFFull) return JPT_E_RANGE;
    I.stream_bits = ww.nbits;
    I.scan_bits = scan_end;
    I.removed_dc_bits = removed;
    I.stream_words = (uint32_t)JPT_STREAM_WORDS(ww.nbits);

    // offsets relative to each group anchor must fit 16 bits
    for (uint32_t g = 0; g < I.n_records; g++)
        for (uint32_t i = 1; i < 9 && 9 * g + i < I.n_mcu; i++)
            if (start[9 * g + i] - start[9 * g] > 0xFFFF) return JPT_E_RANGE;

    I.index_kind = (uint16_t)kind;
    I.index_bits_per_mcu = (32.0 + 16.0 * 8.0) / 9.0;
    I.dc_bits_per_mcu = 36.0;
    const double mcu_px = (double)ms * ms;
    I.overhead_bpp_bound = (I.index_bits_per_mcu + I.dc_bits_per_mcu) / mcu_px;
    I.overhead_bpp_effective =
        ((I.index_bits_per_mcu + I.dc_bits_per_mcu) * I.n_mcu - (double)removed) / (mcu_px * I.n_mcu);
    I.stored_bpp = ((double)I.n_records * JPT_RECORD_BYTES * 8 + (double)I.stream_bits) / ((double)P.w * P.h);
    *info = I;

    if (!stream_out && !records_out) return JPT_OK;
    if ((stream_out && stream_cap_words < I.stream_words) ||
        (records_out && records_cap_bytes < (size_t)I.n_records * JPT_RECORD_BYTES))
        return JPT_E_BUFSIZE;
    if (stream_out) {
        std::memset(stream_out, 0, (size_t)I.stream_words * 4);
        std::memcpy(stream_out, words.data(), std::min(words.size(), (size_t)I.stream_words) * 4);
    }
    if (records_out) {
        std::memset(records_out, 0, (size_t)I.n_records * JPT_RECORD_BYTES);
        for (uint32_t g = 0; g < I.n_records; g++) {
            uint8_t *rec = records_out + (size_t)g * JPT_RECORD_BYTES;
            uint32_t anchor = (uint32_t)start[9 * g];
            std::memcpy(rec, &anchor, 4);
            for (uint32_t i = 1; i < 9; i++) {
                uint16_t rel = 9 * g + i < I.n_mcu ? (uint16_t)(start[9 * g + i] - anchor) : 0;
                std::memcpy(rec + 4 + 2 * (i - 1), &rel, 2);
            }
            for (uint32_t j = 0; j < 9 && 9 * g + j < I.n_mcu; j++)
                for (int c = 0; c < 3; c++) {
                    uint32_t v = (uint32_t)dcs[(size_t)(9 * g + j) * 3 + c] & 0xFFFu;
                    int bit = 160 + 12 * (3 * (int)j + c);
                    for (int b = 0; b < 12; b++)
                        if (v >> b & 1u) rec[(bit + b) >> 3] |= (uint8_t)(1u << ((bit + b) & 7));
                }
        }
    }
    return JPT_OK;
}

// ----------------------------------------------------------- GPU tables
extern "C" jpt_status jpt_build_tables(const jpt_level_info *info, uint32_t *out, size_t cap_words, size_t *words) {
    if (!info) return JPT_E_ARG;
    if (words) *words = JPT_TABLESET_WORDS;
    if (!out) return JPT_OK;
    if (cap_words < JPT_TABLESET_WORDS) return JPT_E_BUFSIZE;
    std::memset(out, 0, JPT_TABLESET_WORDS * 4);
    for (int t = 0; t < 4; t++) {
        HuffSpec H;
        std::memcpy(H.bits, info->huff_bits[t], 16);
        std::memcpy(H.vals, info->huff_vals[t], 256);
        H.n = info->huff_nvals[t];
        int tot = 0;
        for (int i = 0; i < 16; i++) tot += H.bits[i];
        if (tot != H.n) return JPT_E_CORRUPT;
        Canon C;
        if (canon_build(H, C) != JPT_OK) return JPT_E_CORRUPT;
        const bool is_ac = (t & 1) != 0;
        uint32_t *fast = out + t * JPT_FAST_SIZE;
        uint32_t *slow = out + JPT_SLOW_OFFSET + t * JPT_SLOW_WORDS;
        // fast table: every FAST-bit prefix that starts with a code of length <= FAST
        for (int l = 1; l <= JPT_FAST_BITS; l++)
            for (int i = 0; i < C.count[l]; i++) {
                uint32_t code = (uint32_t)(C.first[l] + i);
                int sym = C.vals[C.sym_base[l] + i];
                int run = is_ac ? sym >> 4 : 0, size = is_ac ? sym & 15 : sym;
                bool bad = is_ac ? (size > 10 || (size == 0 && run != 0 && run != 15)) : size > 11;
                int rest = JPT_FAST_BITS - l;
                for (uint32_t tail = 0; tail < (1u << rest); tail++) {
                    uint32_t idx = (code << rest) | tail;
                    uint32_t e;
                    if (bad) {
                        e = JPT_FE_BAD;
                    } else if (size > 0 && l + size <= JPT_FAST_BITS) {
                        uint32_t raw = (tail >> (rest - size)) & ((1u << size) - 1);
                        int v = extend_bits(raw, size);
                        e = (uint32_t)(l + size) | JPT_FE_FUSED | ((uint32_t)size << 6) | ((uint32_t)run << 10) |
                            ((uint32_t)(uint16_t)(int16_t)v << 16);
                    } else {
                        e = (uint32_t)l | ((uint32_t)size << 6) | ((uint32_t)run << 10);
                    }
                    fast[idx] = e;
                }
            }
        // canonical data (codes longer than FAST bits): per length l, the
        // largest code (-1 if none) and the offset symbol index - code
        for (int l = 0; l <= 16; l++) {
            int32_t maxc = (l >= 1 && C.count[l]) ? C.first[l] + C.count[l] - 1 : -1;
            slow[l] = (uint32_t)maxc;
            slow[17 + l] = (uint32_t)(l >= 1 ? C.sym_base[l] - C.first[l] : 0);
        }
        uint8_t *vb = reinterpret_cast<uint8_t *>(slow + 34);
        for (int i = 0; i < 256; i++) vb[i] = C.vals[i];
        // long table: the codes of 11..16 bits occupy [T, 65536) of the
        // 16-bit prefix space, T = first code value after the 10-bit codes
        const uint32_t T = (uint32_t)(C.first[JPT_FAST_BITS] + C.count[JPT_FAST_BITS]) << (16 - JPT_FAST_BITS);
        slow[JPT_SLOW_T] = T;
        slow[JPT_SLOW_LONG_OK] = 0;
        if (T <= 65536u && 65536u - T <= (uint32_t)JPT_LONG_SIZE) {
            uint32_t *lt = out + JPT_LONG_OFFSET + t * JPT_LONG_SIZE;
            for (uint32_t i = 0; i < JPT_LONG_SIZE; i++) lt[i] = JPT_FE_BAD;  // prefixes of no code
            for (int l = JPT_FAST_BITS + 1; l <= 16; l++)
                for (int i = 0; i < C.count[l]; i++) {
                    const uint32_t code = (uint32_t)(C.first[l] + i);
                    const int sym = C.vals[C.sym_base[l] + i];
                    const int run = is_ac ? sym >> 4 : 0, size = is_ac ? sym & 15 : sym;
                    const bool bad = is_ac ? (size > 10 || (size == 0 && run != 0 && run != 15)) : size > 11;
                    const uint32_t e = bad ? JPT_FE_BAD : ((uint32_t)l | ((uint32_t)size << 6) | ((uint32_t)run << 10));
                    const int rest = 16 - l;
                    for (uint32_t tail = 0; tail < (1u << rest); tail++) {
                        const uint32_t p16 = (code << rest) | tail;
                        if (p16 >= T && p16 - T < (uint32_t)JPT_LONG_SIZE) lt[p16 - T] = e;
                    }
                }
            slow[JPT_SLOW_LONG_OK] = 1;
        }
    }
    return JPT_OK;
}

// --------------------------------------------------------------- layout
extern "C" jpt_status jpt_layout(const jpt_level_info *infos, uint32_t n_levels, uint32_t *blk_base,
                                 uint32_t *word_level, size_t word_level_cap, uint32_t *n_blocks) {
    if (!infos || !blk_base || !n_blocks) return JPT_E_ARG;
    uint64_t next = 0;
    for (uint32_t l = 0; l < n_levels; l++) {
        blk_base[l] = (uint32_t)next;
        next += (uint64_t)infos[l].blk_cols * infos[l].blk_rows;
        next = (next + 31) & ~uint64_t(31);
        if (next > (1ull << 29)) return JPT_E_CAPACITY;
    }
    *n_blocks = (uint32_t)next;
    if (!word_level) return JPT_OK;
    if (word_level_cap < next / 32) return JPT_E_BUFSIZE;
    for (uint32_t l = 0; l < n_levels; l++) {
        uint64_t end = l + 1 < n_levels ? blk_base[l + 1] : next;
        for (uint64_t w = blk_base[l] / 32; w < end / 32; w++) word_level[w] = l;
    }
    return JPT_OK;
}

extern "C" jpt_status jpt_make_level_desc(const jpt_level_info *info, uint64_t stream_dptr, uint64_t records_dptr,
                                          uint32_t blk_base, uint32_t table_set, uint32_t quant_index,
                                          jpt_level_desc *out) {
    if (!info || !out) return JPT_E_ARG;
    std::memset(out, 0, sizeof *out);
    out->stream = stream_dptr;
    out->records = records_dptr;
    out->stream_bits = (uint32_t)info->stream_bits;
    out->index_kind = info->index_kind;
    out->width = info->width;
    out->height = info->height;
    out->blk_cols = info->blk_cols;
    out->blk_rows = info->blk_rows;
    out->mcu_cols = info->mcu_cols;
    out->n_mcu = info->n_mcu;
    out->blk_base = blk_base;
    out->sampling = info->sampling;
    out->table_set = table_set;
    out->quant = quant_index;
    return JPT_OK;
}

extern "C" uint32_t jpt_scan_entries(uint32_t n_blocks) {
    // two scans of an LRU frame, or tile counts + group counts + sync words of a frame-local one
    const uint32_t words = (n_blocks + 31) / 32;
    const uint32_t tiles = (words + JPT_SCAN_TILE_WORDS - 1) / JPT_SCAN_TILE_WORDS;
    return 3 * tiles + (tiles + 255) / 256 * 16 + 1;  // 16 count slots per group of 256 tiles
}

extern "C" jpt_status jpt_query_sizes(const jpt_level_info *infos, uint32_t n_levels, const jpt_view *views,
                                      uint32_t n_views, uint32_t filter, jpt_sizes *out) {
    if (!infos || !out || (n_views && !views)) return JPT_E_ARG;
    const uint32_t mode = filter & 0xFFu;
    if (mode > JPT_FILTER_BILINEAR_CLAMPED || (filter & ~0x1FFu)) return JPT_E_ARG;
    const uint64_t taps = mode == JPT_FILTER_TRILINEAR ? 8 : (mode == JPT_FILTER_BILINEAR ? 4 : 1);
    uint64_t blocks = 0, items = 0, next = 0;
    bool any444 = false;
    for (uint32_t l = 0; l < n_levels; l++) {
        const uint64_t b = (uint64_t)infos[l].blk_cols * infos[l].blk_rows;
        const bool s444 = infos[l].sampling == JPT_SAMPLING_444;
        any444 |= s444;
        blocks += b;
        items += s444 ? 4 * b : b;
        next = (next + b + 31) & ~uint64_t(31);
        if (next > (1ull << 29)) return JPT_E_CAPACITY;
    }
    uint64_t px = 0;
    for (uint32_t v = 0; v < n_views; v++) px += (uint64_t)views[v].width * views[v].height;
    const uint64_t max_blocks = std::min(blocks, taps * px);
    const uint64_t max_items = std::min(items, taps * (any444 ? 4 : 1) * px);
    std::memset(out, 0, sizeof *out);
    out->n_blocks = (uint32_t)next;
    out->vis_words = (uint32_t)(next / 32);
    out->scan_entries = jpt_scan_entries((uint32_t)next);
    out->max_items = (uint32_t)max_items;  // (<= 4 x 2^29)
    out->coef_entries = max_items * JPT_ITEMS_DU * 64;
    out->max_blocks = (uint32_t)max_blocks;
    out->items_total = (uint32_t)items;
    out->texel_words = max_blocks * 256;
    out->pixels = px;
    return JPT_OK;
}

extern "C" uint32_t jpt_version(void) { return JPT_ABI_VERSION; }

extern "C" const char *jpt_status_string(jpt_status s) {
    switch (s) {
    case JPT_OK: return "ok";
    case JPT_E_ARG: return "bad argument";
    case JPT_E_UNSUPPORTED: return "unsupported JPEG";
    case JPT_E_CORRUPT: return "corrupt JPEG data";
    case JPT_E_RANGE: return "value out of index range";
    case JPT_E_BUFSIZE: return "buffer too small";
    case JPT_E_HIP: return "HIP runtime error";
    case JPT_E_CAPACITY: return "scene too large";
    default: return "unknown status";
    }
}
