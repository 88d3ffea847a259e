/*
 * CPU oracle for the on-demand JPEG texture path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library
 * never links, calls or includes it, and it shares no source with it.
 *
 * Plain, slow, obviously-correct C in fp64 wherever floating point appears
 * (except the texture-coordinate arithmetic, which the method defines in
 * fp32; see oracle_mark).  Each function names the passage it follows:
 *   - the paper's pipeline: mark / decode / resolve / update cache
 *     (Method section and its subsections), the MCU-id equation (Mark
 *     subsection), the indexing table and absolute-DC side data
 *     (Implementation details: Indexing Table, Memory Overhead);
 *   - the JPEG background section (4:2:0 MCUs of six 8x8 data units,
 *     differential DCs, run-length + Huffman coded ACs), written out with
 *     ITU-T T.81 Annex C (code generation) and Annex F.2 (sequential
 *     Huffman decoding procedures).
 */
#ifndef JPT_ORACLE_H
#define JPT_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (0 = ok). */
#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_UNSUPPORTED (-2)
#define ORC_E_CORRUPT (-3)

typedef struct orc_jpeg orc_jpeg;

/* Parse a baseline JPEG (SOF0, 8-bit, 3 components, 4:2:0 or 4:4:4, one
 * interleaved scan, no restart interval).  Returns NULL and *err on failure. */
orc_jpeg *orc_open(const uint8_t *data, size_t len, int *err);
void orc_close(orc_jpeg *j);

/* info[0..7] = width, height, sampling (420/444), mcu_cols, mcu_rows, n_mcu,
 * data units per MCU, bits in the de-stuffed entropy-coded segment.
 * info[8..9] = quant table id of Y, of Cb/Cr. */
int orc_info(const orc_jpeg *j, int64_t info[10]);

/* Quant tables, natural order: q[0..63] luma, q[64..127] chroma. */
int orc_quant(const orc_jpeg *j, uint16_t q[128]);

/* Sequential decode of the whole scan (T.81 F.2.2).  coef: [n_mcu][n_du][64]
 * quantised coefficients in natural order.  mcu_bit (nullable): n_mcu + 1
 * entries, start bit of each MCU in the de-stuffed segment, last = end of the
 * last MCU.  pred (nullable): [n_mcu][3] DC predictors (Y, Cb, Cr) in force
 * when each MCU starts.  dc_bits (nullable): [n_mcu] number of bits taken by
 * the DC codes (Huffman code + appended bits) of the first Y, the Cb and the
 * Cr data unit of each MCU (all three data units for 4:4:4). */
int orc_decode_seq(const orc_jpeg *j, int16_t *coef, uint64_t *mcu_bit, int32_t *pred, uint32_t *dc_bits);

/* Random access into the original segment: decode one MCU starting at bit
 * `bitpos` with DC predictors pred[3].  out: [n_du][64] natural order;
 * *end_bit = bit after the MCU. */
int orc_decode_mcu_at(const orc_jpeg *j, uint64_t bitpos, const int32_t pred[3], int16_t *out,
                      uint64_t *end_bit);

/* Random access into the GPU library's DC-stripped stream (format stated in
 * include/jpt.h: 32-bit words, MSB first; 64-byte records per 9 MCUs holding
 * one absolute 32-bit bit offset, eight 16-bit relative offsets and 27
 * 12-bit absolute DCs).  Decodes MCU `m` with its absolute DCs from the
 * record; Huffman tables and sampling come from `j`.  *end_bit = bit after
 * the MCU in the stripped stream. */
int orc_decode_stripped_mcu(const orc_jpeg *j, const uint32_t *words, uint64_t n_words, uint64_t stream_bits,
                            const uint8_t *records, uint64_t n_records, uint32_t m, int16_t *out,
                            uint64_t *end_bit);

/* The same for the library's predictor index (JPT_INDEX_PREDICTORS): the
 * stream is the original segment, the record fields hold the DC predictors
 * in force at each MCU; MCU `m` is decoded by the F.2 MCU body from its
 * recorded start with those predictors. */
int orc_decode_predicted_mcu(const orc_jpeg *j, const uint32_t *words, uint64_t n_words, uint64_t stream_bits,
                             const uint8_t *records, uint64_t n_records, uint32_t m, int16_t *out,
                             uint64_t *end_bit);

/* fp64 inverse DCT of one 8x8 block by its definition:
 * s(x,y) = 1/4 sum_u sum_v C(u) C(v) F(v,u) cos((2x+1)u pi/16) cos((2y+1)v pi/16),
 * F natural order (index v*8+u, v vertical frequency), out index y*8+x. */
void orc_idct(const double F[64], double out[64]);

/* Pixels of a whole level from quantised coefficients (reading "single
 * rounding"): F = coef * Q; s = IDCT(F); ycc = clamp(s + 128, 0, 255);
 * chroma replicated over 2x2 for 4:2:0; RGB = clamp(floor(M ycc' + .5)),
 * M the JFIF full-range BT.601 inverse.  rgb: height x width x 3 bytes.
 * rgb_f64 (nullable): the same before rounding and clamping (after the ycc
 * clamp). */
int orc_pixels(const orc_jpeg *j, const int16_t *coef, uint8_t *rgb, double *rgb_f64);

/* The same for one MCU: out_rgb is the MCU's (16x16 or 8x8) texel tile,
 * row-major, 3 bytes per texel, including texels beyond the image border. */
int orc_mcu_pixels(const orc_jpeg *j, const int16_t *coef_mcu, uint8_t *out_rgb, double *out_f64);

/* Reduced-resolution texels of one MCU, scale 1/2^scale_log2 (0..3): each
 * data unit's N x N samples (N = 8 >> scale_log2) by the N-point inverse
 * DCT of its top-left N x N coefficients with the 8-point scaling (N = 1:
 * the block mean), then +128, clamp, chroma replicated over 2x2 luma
 * samples, colour with a single rounding.  out_rgb: the ((16 or 8) >>
 * scale_log2) square tile, 3 bytes per texel; out_f64 (nullable) before
 * rounding.  scale_log2 = 0 gives orc_mcu_pixels. */
int orc_mcu_reduced(const orc_jpeg *j, const int16_t *coef_mcu, int scale_log2, uint8_t *out_rgb, double *out_f64);

/* ---------------------------------------------------------- scenes ---- */
/* A scene is a list of textures, each a chain of levels (level 0 first).
 * Levels are enumerated texture by texture, then level by level; level L
 * owns the global block ids [blk_base[L], blk_base[L] + blk_cols*blk_rows)
 * where blocks are 16x16 texels (block (bx,by) -> blk_base + by*blk_cols+bx,
 * blk_cols = ceil(w/16)) and each blk_base is the previous level's end
 * rounded up to a multiple of 32.  orc_scene_layout fills blk_base and
 * returns the total number of block ids. */
uint64_t orc_scene_layout(int n_levels, const int32_t *lev_w, const int32_t *lev_h, uint32_t *blk_base);

/* One G-buffer pixel: uv (repeat addressing), texture id (0xFFFFFFFF =
 * background), level of detail. */
typedef struct { float u, v; uint32_t tex; float lod; } orc_gpixel;

#define ORC_NEAREST 0
#define ORC_BILINEAR 1
#define ORC_TRILINEAR 2
/* Bilinear weights, but a tap outside the 16x16 block of the texel under
 * the sample point (the nearest filter's texel) takes that texel's column
 * (or row) instead: the paper's resolve clamped to a single MCU (Linear
 * Interpolation in the evaluation; Resolve).  The footprint, and so the
 * marked set, is then that one block: the paper's centre-only marking. */
#define ORC_BILINEAR_CLAMPED 3
#define ORC_FILTER_MASK 0xFF
/* OR'd into a filter: mip mapping off, every pixel samples level 0 (the
 * "no mip" rows of the paper's performance table). */
#define ORC_NO_MIP 0x100

/* Mark (paper, Mark subsection, generalised to a filter footprint): for
 * every non-background pixel, set vis[block] = 1 for every block holding a
 * texel that the filter reads with a non-zero weight.  tex_first[t] /
 * tex_count[t] give texture t's first level and number of levels.
 * Returns the number of invalid pixels (bad tex id, non-finite or too large
 * coordinates), which are skipped. */
int64_t orc_mark(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                 const int32_t *lev_h, const uint32_t *blk_base, const orc_gpixel *g, int64_t n_px,
                 int filter, uint8_t *vis);

/* Resolve (paper, Resolve subsection) from fully decoded levels:
 * level_rgb[L] points at level L's height x width x 3 texels (may be NULL
 * for a level no pixel reads).  frame: one u32 per pixel, R in the low byte,
 * A = 255; background -> 0; invalid pixel -> 0xFFFF00FF.  frame_f64
 * (nullable): 3 doubles per pixel, the same weighted sum with no rounding
 * anywhere (tap weight/65536 times level weight/256).
 * If level_f64 is non-NULL, texels are read from it (unrounded doubles,
 * 3 per texel) for frame_f64 instead of the rounded bytes. */
int64_t orc_resolve(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                    const int32_t *lev_h, const uint8_t *const *level_rgb, const double *const *level_f64,
                    const orc_gpixel *g, int64_t n_px, int filter, uint32_t *frame, double *frame_f64);

/* The taps of every pixel as the resolve uses them (at most 8 per pixel):
 * level, texel x, y and weight (tap weight / 65536 times level weight / 256;
 * unused taps have level -1 and weight 0).  Returns the number of invalid
 * pixels. */
int64_t orc_taps(int n_tex, const int32_t *tex_first, const int32_t *tex_count, const int32_t *lev_w,
                 const int32_t *lev_h, const orc_gpixel *g, int64_t n_px, int filter, int32_t *level, int32_t *x,
                 int32_t *y, double *w);

/* ------------------------------------------------------ geometry ---- */
/* A textured triangle (80 bytes) and a pinhole camera (64 bytes): the ray
 * of pixel (x, y) of a W x H view leaves eye along
 * fwd + sx right + sy up, sx = (2 (x + 0.5) / W - 1) tan_half_x,
 * sy = (1 - 2 (y + 0.5) / H) tan_half_y. */
typedef struct {
    float p0[3], p1[3], p2[3];
    float uv0[2], uv1[2], uv2[2];
    uint32_t tex;
    uint32_t reserved[4];
} orc_triangle;
typedef struct {
    float eye[3], fwd[3], right[3], up[3];
    float tan_half_x, tan_half_y;
    float reserved[2];
} orc_camera;

/* Geometry pass (geometry.c), fp64: each pixel takes the nearest triangle
 * (smallest t > 0; the lower index on equal t) whose closed area its centre
 * ray hits; uv = the hit's barycentric blend of the vertices' uv; lod =
 * log2 max(|(du, dv)_x|, |(du, dv)_y|) in texels of the texture's level 0
 * (tex_w/tex_h), the differences taken to the rays one pixel right and one
 * pixel down met with the same triangle's plane.  Pixels without a hit are
 * background.  tri_out (nullable): the hit triangle per pixel (-1 none). */
void orc_geometry(const orc_triangle *tris, int64_t n_tris, const orc_camera *cam, int W, int H,
                  const int32_t *tex_w, const int32_t *tex_h, int n_tex, orc_gpixel *g, int32_t *tri_out);

/* BC1 decoding by definition (bc1.c): blocks of a w x h image ->
 * h x w x 3 bytes.  See bc1.c for the block layout and palette. */
void orc_bc1_decode(const uint8_t *blocks, int w, int h, uint8_t *rgb);

/* CPU on-demand baseline (ondemand.c): one frame of the paper's method on
 * the host, on n_threads threads: mark (orc_mark over pixel ranges), list the
 * marked blocks, decode only their MCUs by random access into the original
 * segment (orc_decode_mcu_at from mcu_bit[L][m] with predictors
 * pred[L][3m..3m+2], as recorded by orc_decode_seq) into level_rgb[L]
 * (full-size level images; only the decoded blocks are written), then
 * orc_resolve over pixel ranges.  vis: n_blocks bytes of scratch; list:
 * n_blocks u32 of scratch.  times (nullable): seconds of mark, listing,
 * decode, resolve.  Returns the number of invalid pixels plus MCUs that
 * failed to decode, or -1 for bad arguments. */
int64_t orc_ondemand_frame(int n_tex, const int32_t *tex_first, const int32_t *tex_count, int n_levels,
                           const int32_t *lev_w, const int32_t *lev_h, const uint32_t *blk_base, uint64_t n_blocks,
                           const orc_jpeg *const *jpegs, const uint64_t *const *mcu_bit, const int32_t *const *pred,
                           uint8_t *const *level_rgb, const orc_gpixel *g, int64_t n_px, int filter,
                           uint32_t *frame, uint8_t *vis, uint32_t *list, int n_threads, double times[4],
                           uint64_t *n_decoded);

#ifdef __cplusplus
}
#endif
#endif
