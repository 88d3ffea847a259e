/*
 * jpt.h -- C ABI of libjpt: on-demand decoding of baseline-JPEG textures
 * during deferred shading, on AMD Instinct MI355X (gfx950).
 *
 * The method (Kristmann, Wimmer, Schuetz, "Variable-Rate Texture
 * Compression: Real-Time Rendering with JPEG", arXiv 2510.08166):
 *   - offline, per texture level: an indexing table of MCU offsets and the
 *     absolute DCs that break the DC prediction chain (Implementation
 *     details: "Indexing Table" and "Memory Overhead");
 *   - per frame, after the geometry pass wrote a G-buffer of (uv, texture
 *     id, mip level): Mark -> Decode -> Resolve -> Update Cache (Method
 *     section, pass list and subsections "Texture Block Cache", "Mark",
 *     "Decode", "Resolve", "Update Cache", "Multiple Textures and Mip
 *     Mapping").
 *
 * Conventions
 *   - Every function returns jpt_status (JPT_OK = 0, errors < 0).
 *   - The caller owns all memory.  Host outputs go into caller buffers;
 *     pass NULL outputs to query sizes where stated.  The library never
 *     allocates device memory.
 *   - Device calls enqueue work on the caller's HIP stream (`stream` is a
 *     hipStream_t passed as void*, NULL = the null stream).  They do not
 *     synchronise, allocate or read device data back, and their launch
 *     shapes depend only on host arguments, so they can be captured into a
 *     HIP graph.  Argument errors are returned before anything is enqueued.
 *     Errors found on the device (corrupt stream, capacity, bad pixel) set
 *     bits in counters[JPT_CTR_ERROR]; read it after the stream synchronises.
 *   - No global state; calls on disjoint buffers are thread-safe.
 *
 * Terms
 *   MCU    minimum coded unit: 16x16 texels (4:2:0, six 8x8 data units
 *          Y00 Y01 Y10 Y11 Cb Cr) or 8x8 texels (4:4:4, Y Cb Cr).
 *   block  16x16 texels of one (texture, level): one 4:2:0 MCU, or 2x2
 *          4:4:4 MCUs.  The unit of marking, caching and resolve.
 *   block id  dense global id: levels are numbered texture by texture, then
 *          level by level; level L owns [blk_base[L], blk_base[L] +
 *          blk_cols*blk_rows), block (bx,by) -> blk_base + by*blk_cols + bx,
 *          blk_cols = ceil(w/16); every blk_base is the previous level's end
 *          rounded up to a multiple of 32, so each 32-bit word of a block
 *          bitmask belongs to a single level.  (Generalises the paper's
 *          MCU id equation and 32-bit cache key of 16/13/3 bits, which
 *          cannot address 8192^2 textures or more than 8 levels.)
 *   work item  one MCU to decode, encoded (block id << 2) | q, q = quadrant
 *          (x + 2y) of a 4:4:4 MCU inside its block, 0 for 4:2:0.  Bit 31
 *          is set by the decoder on an item whose stream failed to decode.
 */
#ifndef JPT_H
#define JPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JPT_ABI_VERSION 1u

typedef int32_t jpt_status;
#define JPT_OK 0
#define JPT_E_ARG (-1)          /* bad argument (NULL, size, enum) */
#define JPT_E_UNSUPPORTED (-2)  /* valid JPEG outside the baseline subset handled here */
#define JPT_E_CORRUPT (-3)      /* malformed JPEG / entropy-coded data */
#define JPT_E_RANGE (-4)        /* a value does not fit the index format */
#define JPT_E_BUFSIZE (-5)      /* caller buffer too small */
#define JPT_E_HIP (-6)          /* a HIP runtime call failed */
#define JPT_E_CAPACITY (-7)     /* scene too large: 32-bit block ids, or the static scratch of
                                   jpt_mark_blocks_static */

#define JPT_SAMPLING_420 420u
#define JPT_SAMPLING_444 444u

#define JPT_FILTER_NEAREST 0u
#define JPT_FILTER_BILINEAR 1u
#define JPT_FILTER_TRILINEAR 2u
/* The paper's resolve clamped to a single MCU (Evaluation: Linear
 * Interpolation; Method: Resolve): bilinear weights, but a tap outside the
 * 16x16 block of the texel under the sample point (the nearest filter's
 * texel) reads that texel's column or row instead.  Its footprint is that
 * one block, so marking with it is the paper's centre-only marking. */
#define JPT_FILTER_BILINEAR_CLAMPED 3u
/* OR'd into any filter: mip mapping off, every pixel samples level 0 (the
 * paper's performance table without mip maps). */
#define JPT_FILTER_MIP_OFF 0x100u

#define JPT_CACHE_NONE 0u       /* each frame decodes every visible block; slot = rank */
#define JPT_CACHE_LRU 1u        /* frame-granular LRU with a slot capacity */
#define JPT_CACHE_EVICT_INVISIBLE 2u  /* the paper's Update Cache: after each frame every resident block the
                                         frame did not read is evicted (the LRU arrays, same reset) */
#define JPT_CACHE_HASH 3u       /* the paper's Texture Block Cache as it builds it: a hash map from a 32-bit
                                   key (16-bit block index, 13-bit texture, 3-bit level) to a slot, filled by
                                   atomicCAS in mark, probed per tap in resolve, every block a frame does not
                                   read evicted (see jpt_cache.hash) */

#define JPT_IDCT_MFMA_F16 0u    /* 64x64 basis on MFMA, split-fp16 operands, fp32 accumulate */
#define JPT_IDCT_SCALAR_F32 1u  /* separable fp32 row/column IDCT on the vector ALUs */
#define JPT_IDCT_FUSED_F32 2u   /* jpt_decode_blocks only: the entropy decoder's wavefront runs the
                                   JPT_IDCT_SCALAR_F32 arithmetic on its own MCU and stores the
                                   texels; frame->coef is not written */
#define JPT_IDCT_MFMA_BF16 3u   /* the JPT_IDCT_MFMA_F16 contraction with bf16 operands: the basis in
                                   three bf16 parts, coefficients in exact base-128 digits */

/* counters[] (u32) of a frame */
#define JPT_CTR_ITEMS 0         /* work items listed this frame (<= max_items) */
#define JPT_CTR_NEW 1           /* blocks to decode this frame */
#define JPT_CTR_VISIBLE 2       /* blocks read by this frame */
#define JPT_CTR_ERROR 3         /* JPT_ERR_* flags */
#define JPT_CTR_ERROR_ITEM 4    /* smallest failing work-item index (0xFFFFFFFF = none) */
#define JPT_CTR_EVICTED 5       /* blocks evicted this frame (LRU) */
#define JPT_CTR_RESIDENT 6      /* resident blocks after this frame (LRU) */
#define JPT_CTR_GRAD_MAX 7      /* jpt_backward: fp32 bits of the largest |dL/dframe| it scaled by */
#define JPT_N_COUNTERS 16u

#define JPT_ERR_CORRUPT 1u      /* invalid code, > 64 coefficients, or MCU span mismatch */
#define JPT_ERR_CAPACITY 2u     /* work list or cache slots exhausted */
#define JPT_ERR_PIXEL 4u        /* G-buffer pixel with bad texture id or coordinates */
#define JPT_ERR_INTERNAL 8u     /* reserved: a bounded device-side wait gave up (no kernel of this version waits) */
#define JPT_ERR_GRAD 16u        /* jpt_backward: a non-finite entry in dL/dframe */

#define JPT_SLOT_NONE 0xFFFFFFFFu
#define JPT_TEX_BACKGROUND 0xFFFFFFFFu
#define JPT_TEXEL_INVALID 0xFFFF00FFu   /* magenta, written for undecodable data */

#define JPT_ITEMS_DU 6u                 /* coefficient stride of a work item, in 8x8 units */
#define JPT_RECORD_BYTES 64u
#define JPT_MCUS_PER_RECORD 9u
#define JPT_STREAM_PAD_WORDS 4u

/* ------------------------------------------------------------------ *
 * Offline: per-level index (paper: "Indexing Table", "Memory Overhead")
 * ------------------------------------------------------------------ *
 * Spliced stream: the level's entropy-coded segment, de-stuffed, with the
 * DC codes (Huffman code + appended bits) of the first Y, the Cb and the Cr
 * data unit of every MCU removed (every data unit for 4:4:4).  Those DCs are
 * stored as absolute values in the records instead; the other Y DCs of a
 * 4:2:0 MCU stay coded as differences to the previous Y of the same MCU.
 * Stored as 32-bit words, bit 31 of word 0 is the first bit; followed by
 * at least JPT_STREAM_PAD_WORDS zero words, the total rounded up to a
 * multiple of 4 words (info.stream_words); the device address of a
 * level's stream must be 16-byte aligned.
 *
 * Records: one 64-byte record per 9 MCUs (raster order), little-endian:
 *   bytes 0..3    u32 bit offset of MCU 9g in the spliced stream
 *   bytes 4..19   u16 rel[8]: offset of MCU 9g+1+i minus that of MCU 9g
 *   bits 160..483 27 fields of 12 bits (bit b = bit b%8 of byte b/8):
 *                 field 3j+c = absolute quantised DC of component c
 *                 (0 Y, 1 Cb, 2 Cr) of MCU 9g+j, two's complement
 *   bytes 61..63  zero
 * MCU m spans [start(m), start(m+1)), the last one ends at stream_bits.
 * Index cost as the paper counts it: (32 + 16*8)/9 bits of offsets plus
 * 3*12 bits of DCs = 53.78 bits per MCU; the 64-byte record costs 56.9.   */
typedef struct jpt_level_info {
    uint32_t width, height;
    uint32_t sampling;            /* JPT_SAMPLING_420 / _444 */
    uint32_t mcu_cols, mcu_rows, n_mcu;
    uint32_t blk_cols, blk_rows;  /* ceil(width/16), ceil(height/16) */
    uint32_t n_records;           /* ceil(n_mcu / 9) */
    uint32_t stream_words;        /* words stream_out needs, padding included */
    uint64_t stream_bits;         /* bits of MCU data in the spliced stream */
    uint64_t scan_bits;           /* bits of MCU data in the original segment */
    uint64_t removed_dc_bits;     /* bits of DC codes removed by the splice */
    uint16_t quant[2][64];        /* zigzag order; [0] luma, [1] chroma */
    uint8_t huff_bits[4][16];     /* BITS (codes per length 1..16): DC luma, AC luma, DC chroma, AC chroma */
    uint8_t huff_vals[4][256];    /* HUFFVAL of each table */
    uint16_t huff_nvals[4];
    uint16_t index_kind;          /* JPT_INDEX_SPLICED / JPT_INDEX_PREDICTORS */
    uint16_t reserved0;
    double index_bits_per_mcu;    /* 160/9 */
    double dc_bits_per_mcu;       /* 36 */
    double overhead_bpp_bound;    /* (index + dc bits per MCU) / MCU texels */
    double overhead_bpp_effective;/* same minus the removed DC bits, over the level's MCU texels */
    double stored_bpp;            /* (records*64*8 + stream_bits) / (width*height) */
} jpt_level_info;

/* The two readings of the paper's index.  JPT_INDEX_SPLICED: the stream and
 * records described above (absolute DCs, DC codes spliced out).
 * JPT_INDEX_PREDICTORS: the level's entropy-coded segment untouched (only
 * de-stuffed), the records' offsets pointing into it and their 12-bit
 * fields holding the DC predictors (Y, Cb, Cr) in force when each MCU
 * starts; every data unit then decodes its DC difference as in T.81.  Any
 * baseline decoder can still read the stream; the overhead is the paper's
 * bound (53.78 bits per MCU) with nothing removed. */
#define JPT_INDEX_SPLICED 0u
#define JPT_INDEX_PREDICTORS 1u

/* Parse a baseline JPEG (SOF0, 8-bit, 3 components Y Cb Cr with Cb and Cr
 * sharing quant and Huffman tables, 4:2:0 or 4:4:4, one interleaved scan,
 * no restart interval) and build the spliced stream and records.
 *   jpeg/len       host bytes of the file (read only)
 *   info           host, filled on JPT_OK (and on JPT_E_BUFSIZE)
 *   stream_out     host, >= info->stream_words u32, or NULL to query
 *   records_out    host, >= info->n_records * 64 bytes, or NULL to query
 * Errors: JPT_E_ARG, JPT_E_UNSUPPORTED, JPT_E_CORRUPT (any MCU fails to
 * decode: an invalid code, a (run, size 0) symbol other than EOB and ZRL, an
 * AC size above 10, a run past coefficient 63), JPT_E_RANGE (a quantised DC
 * of any data unit outside [-2048, 2047], a relative offset above 65535
 * bits, stream above 2^32-1 bits), JPT_E_BUFSIZE. */
jpt_status jpt_build_index(const uint8_t *jpeg, size_t len, jpt_level_info *info, uint32_t *stream_out,
                           size_t stream_cap_words, uint8_t *records_out, size_t records_cap_bytes);

/* jpt_build_index with the index reading chosen by `kind`
 * (JPT_INDEX_SPLICED is jpt_build_index).  Errors: as jpt_build_index, and
 * JPT_E_ARG for an unknown kind. */
jpt_status jpt_build_index_ex(const uint8_t *jpeg, size_t len, uint32_t kind, jpt_level_info *info,
                              uint32_t *stream_out, size_t stream_cap_words, uint8_t *records_out,
                              size_t records_cap_bytes);

/* Decode tables for the GPU entropy decoder, built from info's Huffman
 * tables (the paper's per-code matching loop replaced by table lookup).
 * tables_out: host, JPT_TABLESET_WORDS u32 (or NULL to query *words).
 * Errors: JPT_E_ARG, JPT_E_CORRUPT (over-full code), JPT_E_BUFSIZE. */
#define JPT_TABLESET_WORDS 6656u
jpt_status jpt_build_tables(const jpt_level_info *info, uint32_t *tables_out, size_t cap_words, size_t *words);

/* Block-id layout of a scene (see "block id" above).  infos: n_levels
 * level infos in scene order.  blk_base: host, n_levels u32.  word_level:
 * host, one u32 per bitmask word (= *n_blocks / 32), the level owning that
 * word; NULL to query.  Errors: JPT_E_ARG, JPT_E_CAPACITY (more than 2^29
 * block ids), JPT_E_BUFSIZE. */
jpt_status jpt_layout(const jpt_level_info *infos, uint32_t n_levels, uint32_t *blk_base, uint32_t *word_level,
                      size_t word_level_cap, uint32_t *n_blocks);

/* ------------------------------------------------------------------ *
 * Device-side descriptors (arrays of these live in device memory)
 * ------------------------------------------------------------------ */
typedef struct jpt_level_desc {   /* 64 bytes */
    uint64_t stream;              /* device address of the level's stream (u32 words) */
    uint64_t records;             /* device address of the 64-byte records */
    uint32_t stream_bits;
    uint32_t index_kind;          /* JPT_INDEX_SPLICED / JPT_INDEX_PREDICTORS */
    uint32_t width, height;
    uint32_t blk_cols, blk_rows;
    uint32_t mcu_cols, n_mcu;
    uint32_t blk_base;
    uint32_t sampling;            /* 420 / 444 */
    uint32_t table_set;           /* index into jpt_scene.tables */
    uint32_t quant;               /* index into jpt_scene.quant */
} jpt_level_desc;

typedef struct jpt_texture_desc { /* 16 bytes */
    uint32_t first_level;         /* index of level 0 in the level array */
    uint32_t n_levels;
    uint32_t width, height;       /* of level 0 */
} jpt_texture_desc;

/* Fill a level descriptor from an index build (host helper). */
jpt_status jpt_make_level_desc(const jpt_level_info *info, uint64_t stream_dptr, uint64_t records_dptr,
                               uint32_t blk_base, uint32_t table_set, uint32_t quant_index, jpt_level_desc *out);

/* One G-buffer pixel (16 bytes): texture coordinates with repeat
 * addressing (v = 0 is the top texel row), texture id (JPT_TEX_BACKGROUND
 * for none) and level of detail log2(texels per pixel).  Texel
 * coordinates: nearest s = u*w, texel floor(s) mod w; linear
 * s = u*w - 0.5, texels floor(s), floor(s)+1 with weights 256-f, f,
 * f = floor(frac(s)*256 + 0.5); every product and sum a separate fp32
 * operation.  Level: nearest/linear clamp(floor(lod + 0.5), 0, n-1);
 * trilinear floor(lod) and the next level with weights 256-t, t,
 * t = floor(frac(lod)*256 + 0.5) (one level if lod < 0 or lod >= n-1).
 * Taps of zero weight are neither marked nor read.  A pixel with a bad
 * texture id, a non-finite field or |s| >= 2^30 is invalid. */
typedef struct jpt_gpixel { float u, v; uint32_t tex; float lod; } jpt_gpixel;

typedef struct jpt_scene {        /* host struct holding device pointers */
    const jpt_level_desc *levels;     /* n_levels */
    const jpt_texture_desc *textures; /* n_textures */
    const uint32_t *word_level;       /* n_blocks / 32 */
    const uint32_t *tables;           /* n_tablesets * JPT_TABLESET_WORDS */
    const uint16_t *quant;            /* n_quant * 128, zigzag, [luma 64][chroma 64] */
    uint32_t n_levels, n_textures, n_tablesets, n_quant;
    uint32_t n_blocks;                /* multiple of 32, <= 2^29 */
    uint32_t flags;                   /* JPT_SCENE_*: set JPT_SCENE_PREDICTOR_INDEX if any level uses
                                         JPT_INDEX_PREDICTORS (its MCUs fail to decode otherwise) */
} jpt_scene;
#define JPT_SCENE_PREDICTOR_INDEX 1u

typedef struct jpt_view {         /* host struct holding device pointers */
    const jpt_gpixel *gbuf;       /* height rows of pitch pixels */
    uint32_t *frame;              /* height rows of frame_pitch u32 (RGBA8, R low byte, A 255) */
    uint32_t width, height;
    uint32_t pitch, frame_pitch;
} jpt_view;

typedef struct jpt_frame {        /* per-frame device scratch, caller-allocated */
    uint32_t *vis;                /* n_blocks/32 words: blocks this frame reads; zero-filled by the
                                     caller before the first frame, every jpt_mark_blocks leaves it so */
    uint32_t *work;               /* max_items work items, ascending */
    uint32_t *counters;           /* JPT_N_COUNTERS */
    uint64_t *scan;               /* jpt_scan_entries(n_blocks) entries; zero-filled by the caller
                                     before the first frame, every jpt_mark_blocks leaves it so */
    int16_t *coef;                /* max_items * 6 * 64 quantised coefficients, zigzag order */
    uint32_t max_items;
    uint32_t frame_no;            /* LRU timestamp f of this frame, or JPT_FRAME_AUTO: the cache's own
                                     frame counter (0 after jpt_cache_reset, then one more after every
                                     frame), so that a captured graph can be replayed frame after frame */
} jpt_frame;

#define JPT_FRAME_AUTO 0xFFFFFFFFu

/* Decoded-block cache (paper: "Texture Block Cache", "Update Cache"),
 * caller-allocated.  JPT_CACHE_NONE needs texels and slot_of only; the
 * LRU policy also needs the other arrays and jpt_cache_reset before its
 * first frame.  LRU policy, per frame f with visible set V and resident
 * set R: visible resident blocks get last_used = f; the new blocks V - R
 * take free slots; if too few are free, the resident blocks outside V with
 * the smallest (last_used, block id) are evicted first.  Frame numbers must
 * not decrease from one frame to the next (ages f - last_used are taken
 * modulo 2^32).  The eviction ranks ages through a histogram of
 * JPT_LRU_MAX_AGE + 1 bins; when the evictions end among blocks at least
 * JPT_LRU_MAX_AGE frames old, three more passes select them by their exact
 * 32-bit age. */
#define JPT_LRU_MAX_AGE 1023u
#define JPT_CACHE_META_WORDS (16u + JPT_LRU_MAX_AGE + 1u + 2048u + 2048u + 1024u)
typedef struct jpt_cache {
    uint32_t *texels;             /* n_slots * 256 RGBA8 texels, slot-major, 16x16 row-major */
    uint32_t *slot_of;            /* n_blocks: slot of each block (valid while resident) */
    uint32_t *owner;              /* n_slots: block in each slot or JPT_SLOT_NONE (LRU) */
    uint32_t *last_used;          /* n_slots: frame_no of last use (LRU) */
    uint32_t *resident;           /* n_blocks/32 words: resident blocks (LRU) */
    uint32_t *free_stack;         /* n_slots: free slots, top of stack in meta (LRU) */
    uint32_t *meta;               /* JPT_CACHE_META_WORDS: stack top, eviction plan, age histograms (LRU) */
    uint32_t *tie_mask;           /* n_blocks/32 words: scratch of the eviction (LRU) */
    uint32_t n_slots;
    uint32_t policy;              /* JPT_CACHE_* */
    uint32_t *hash;               /* JPT_CACHE_HASH: 2 * n_buckets words, bucket i = (key, value) at
                                     [2i, 2i + 1]; value = slot | bit 31 when read this frame.  That policy
                                     also uses texels, slot_of (written for each frame's new blocks, for
                                     the decoder), owner (the key in each slot), free_stack and meta, and
                                     takes 4:2:0 levels of at most 65,536 blocks, 8,191 textures of at most
                                     8 levels (the key's fields); other pixels raise JPT_ERR_PIXEL.  The
                                     queue order of its work items is the order of insertion. */
    uint32_t n_buckets;           /* a power of two >= 2 n_slots */
    uint32_t reserved;
} jpt_cache;

/* Empty an LRU cache: every slot free, no block resident.  Device call on
 * `stream`.  Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_cache_reset(const jpt_scene *scene, jpt_cache *cache, void *stream);

typedef struct jpt_tuning {       /* launch knobs; NULL = defaults.  Results never depend on them. */
    uint32_t decode_groups;       /* workgroups of the entropy decoder (0 = as many as the device holds at once) */
    uint32_t idct_groups;         /* persistent workgroups of the IDCT kernel (0 = auto) */
    uint32_t mark_groups;         /* workgroups of the mark kernel (0 = one per pixel tile; else each
                                     walks the tiles of all views with that stride) */
    uint32_t resolve_groups;      /* the same for the resolve kernel */
    uint32_t flags;               /* JPT_TUNE_* */
    uint32_t wide_bits;           /* entropy decoder: MCUs of at least this many bits take steps of 128
                                     bit offsets instead of 64 (0 = auto) */
    uint32_t reserved[2];
} jpt_tuning;

/* jpt_tuning.flags: hand each of the GPU's 8 chiplets (XCDs, each with its
 * own L2) a contiguous run of pixel tiles in mark and resolve, instead of
 * interleaving neighbouring tiles over all of them. */
#define JPT_TUNE_XCD_TILES 1u
/* jpt_tuning.flags: how the bilinear resolves look up a pixel's slots.  By
 * default a launch of more than one round of workgroups (more pixel tiles
 * than the GPU holds at once) reads each texel row's two slot-table entries
 * in one 8-byte load, and a launch of one round reads the four entries one
 * by one; these flags force one form (both set: JPT_E_ARG). */
#define JPT_TUNE_RESOLVE_PAIRED 2u
#define JPT_TUNE_RESOLVE_SINGLE 4u

/* Buffer sizes for rendering a scene's views under `filter` (host query,
 * no device access): what jpt_frame and jpt_cache need so that no frame of
 * these views can overflow them.  A pixel reads at most T blocks (nearest
 * and the one-MCU clamp 1, bilinear 4, trilinear 8); a block is one work
 * item (4:2:0) or four (4:4:4); so a frame lists at most
 * min(items of the scene, T x 4:4:4-factor x pixels) work items and reads
 * at most min(blocks of the scene, T x pixels) blocks.
 *   infos   n_levels level infos in scene order (host), as for jpt_layout
 *   views   n_views views; only width and height are read (host)
 *   out     host, filled on JPT_OK
 * Errors: JPT_E_ARG (NULL, filter), JPT_E_CAPACITY (as jpt_layout). */
typedef struct jpt_sizes {
    uint32_t n_blocks;            /* block ids (jpt_layout) */
    uint32_t vis_words;           /* frame->vis, cache->resident, cache->tie_mask: u32 words */
    uint32_t scan_entries;        /* frame->scan: u64 entries (jpt_scan_entries) */
    uint32_t max_items;           /* frame->work and frame->max_items */
    uint64_t coef_entries;        /* frame->coef: max_items * 6 * 64 int16 */
    uint32_t max_blocks;          /* blocks one frame can read: the slots a JPT_CACHE_NONE cache needs */
    uint32_t items_total;         /* work items of the whole scene (every MCU) */
    uint64_t texel_words;         /* cache->texels for max_blocks slots (256 u32 each) */
    uint64_t pixels;              /* pixels of all views */
} jpt_sizes;
jpt_status jpt_query_sizes(const jpt_level_info *infos, uint32_t n_levels, const jpt_view *views, uint32_t n_views,
                           uint32_t filter, jpt_sizes *out);

/* Entries of jpt_frame.scan for a scene of n_blocks block ids: per-tile
 * and per-group counts of the block bitmask (an LRU frame also takes two
 * per-tile scans of it and sums its tiles into the group counts). */
uint32_t jpt_scan_entries(uint32_t n_blocks);

/* ------------------------------------------------------------------ *
 * Per frame
 * ------------------------------------------------------------------ */

/* Mark + compact (paper: Mark; decode queue of the overview figure; the
 * cache's visibility flags).  Marks in frame->vis every block a pixel of
 * any view reads with non-zero weight under `filter`, then lists the blocks
 * not yet resident as work items in ascending block-id order, assigns their
 * cache slots, sets frame->counters for the frame and zeroes frame->vis
 * again:
 *   JPT_CACHE_NONE: slot = rank of the block among this frame's new blocks
 *     (blocks beyond n_slots get JPT_SLOT_NONE and raise JPT_ERR_CAPACITY);
 *   JPT_CACHE_LRU: the policy stated at jpt_cache (frame_no is the frame
 *     index f; new blocks that find no slot get JPT_SLOT_NONE and raise
 *     JPT_ERR_CAPACITY).  counters[JPT_CTR_EVICTED] and
 *     [JPT_CTR_RESIDENT] report the update.
 * cache may be NULL only if nothing reads slots (block lists only).
 * Errors: JPT_E_ARG (NULL/short buffers, filter, view sizes), JPT_E_HIP. */
jpt_status jpt_mark_blocks(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                           jpt_frame *frame, jpt_cache *cache, const jpt_tuning *tuning, void *stream);

/* jpt_mark_blocks for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and results, but frame->scan is ignored and the scan
 * scratch is a device array inside the library, JPT_STATIC_SCAN_ENTRIES u64
 * entries (512 KiB) held by every device the library runs on until the
 * process ends.  The call allocates nothing; on its first call on a device
 * (the current device, which must own `stream`) it looks up that device's
 * copy of the array.  Each call first zeroes the jpt_scan_entries(n_blocks)
 * entries it uses (a kernel on `stream`, no memset), since the array keeps
 * the previous call's contents.  Calls that overlap on one device share the
 * array and race: serialise them (one stream, or events).
 * Errors: those of jpt_mark_blocks, JPT_E_CAPACITY (jpt_scan_entries(n_blocks)
 * > JPT_STATIC_SCAN_ENTRIES), JPT_E_HIP (the array's address). */
#define JPT_STATIC_SCAN_ENTRIES 65536u
jpt_status jpt_mark_blocks_static(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                                  jpt_frame *frame, jpt_cache *cache, const jpt_tuning *tuning, void *stream);

/* Decode (paper: Decode).  For every work item listed by the last
 * jpt_mark_blocks on this frame: entropy-decode the MCU through the index
 * into frame->coef (zigzag order, stride 6*64 per item), then dequantise,
 * inverse-DCT, convert YCbCr (JFIF, chroma replicated) to RGB with a
 * single rounding, and store RGBA8 texels into the block's cache slot.
 * A failed item gets bit 31 in frame->work, JPT_ERR_CORRUPT and
 * JPT_TEXEL_INVALID texels.  idct_mode: JPT_IDCT_*.
 * Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_decode_blocks(const jpt_scene *scene, jpt_frame *frame, jpt_cache *cache, uint32_t idct_mode,
                             const jpt_tuning *tuning, void *stream);

/* Reduced-resolution decode (paper: Discussion, lower resolutions from the
 * DC and the first ACs instead of stored mip levels).  For every work item
 * of the frame (as listed by jpt_mark_blocks, or written by the caller into
 * frame->work with counters[JPT_CTR_ITEMS]): entropy-decode its MCU, then
 * form its texels at scale 1/2^scale_log2 (1..3): each data unit's N x N
 * samples (N = 8 >> scale_log2) by the N-point inverse DCT of its top-left
 * N x N dequantised coefficients with the 8-point scaling (N = 1: the
 * block mean), +128 and clamp, chroma over 2x2 luma samples, colour with
 * one rounding.  texels_out: device memory, (16 >> scale_log2)^2 RGBA8
 * texels per work item, row-major (a 4:4:4 item fills the first
 * (8 >> scale_log2)^2); failed items get JPT_TEXEL_INVALID.  No cache slot
 * is used.  Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_decode_reduced(const jpt_scene *scene, jpt_frame *frame, uint32_t scale_log2, uint32_t *texels_out,
                              const jpt_tuning *tuning, void *stream);

/* Entropy decode only (the first half of jpt_decode_blocks): fills
 * frame->coef for the listed work items.  Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_entropy_decode(const jpt_scene *scene, jpt_frame *frame, const jpt_tuning *tuning, void *stream);

/* The second half of jpt_decode_blocks: dequantise, IDCT, colour-convert
 * and store the texels of the listed work items from frame->coef (filled by
 * jpt_entropy_decode).  Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_idct_color(const jpt_scene *scene, jpt_frame *frame, jpt_cache *cache, uint32_t idct_mode,
                          const jpt_tuning *tuning, void *stream);

/* Resolve (paper: Resolve): every pixel of every view reads its filter taps
 * from the cache slots of their blocks and writes the filtered RGBA8 value
 * (integer weights: bilinear (sum t*w + 32768) >> 16 per channel,
 * trilinear (a*(256-t) + b*t + 128) >> 8).  Background pixels get 0;
 * invalid pixels and taps in blocks without a slot get JPT_TEXEL_INVALID.
 * Errors: JPT_E_ARG (also a cache of 0 slots, or a scene of fewer than 32
 * block ids, which jpt_layout never makes), JPT_E_HIP. */
jpt_status jpt_resolve(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                       const jpt_frame *frame, const jpt_cache *cache, const jpt_tuning *tuning, void *stream);

/* ------------------------------------------------------------------ *
 * Geometry pass: the G-buffer the method starts from (paper: Method, the
 * pass before Mark, which writes texture coordinates, texture ids and mip
 * map levels), rendered on the GPU from textured triangles.
 * ------------------------------------------------------------------ */
typedef struct jpt_triangle {     /* 80 bytes */
    float p0[3], p1[3], p2[3];    /* vertices */
    float uv0[2], uv1[2], uv2[2]; /* texture coordinates of the vertices */
    uint32_t tex;                 /* texture id */
    uint32_t reserved[4];
} jpt_triangle;

typedef struct jpt_camera {       /* 64 bytes, passed by value to the kernel */
    float eye[3];                 /* ray origin */
    float fwd[3], right[3], up[3];/* pixel (x, y) of a W x H view looks along fwd + sx right + sy up, */
    float tan_half_x, tan_half_y; /* sx = (2 (x + 0.5) / W - 1) tan_half_x, sy = (1 - 2 (y + 0.5) / H) tan_half_y */
    float reserved[2];
} jpt_camera;

/* Every pixel of a width x height view takes the nearest triangle its centre
 * ray hits (smallest t > 0; on equal t the lower index) and writes
 * gbuf[y * pitch + x] = {u, v, tex, lod}: uv the hit's barycentric blend of
 * the vertices' uv, lod = log2 of the larger texel footprint, in texels of
 * the texture's level 0 (scene->textures), of the rays one pixel to the
 * right and one pixel down met with the hit triangle's plane.  Pixels with
 * no hit get tex = JPT_TEX_BACKGROUND.  fp32 arithmetic.  tris: device
 * memory, n_tris entries; cam: host struct; gbuf: device memory.
 * Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_geometry_pass(const jpt_scene *scene, const jpt_triangle *tris, uint32_t n_tris,
                             const jpt_camera *cam, uint32_t width, uint32_t height, uint32_t pitch,
                             jpt_gpixel *gbuf, void *stream);

/* ------------------------------------------------------------------ *
 * Fixed-rate baseline (paper: Background, BC1): textures stored as BC1
 * blocks, sampled directly by the resolve with no mark, decode or cache.
 * A level's blocks: 8 bytes per 4x4 texels, row-major, little-endian:
 * colour 0 and colour 1 (RGB565, u16), then 16 two-bit indices, texel
 * (i, j) of the block (column i, row j) at bits 2 (4 j + i).  Endpoints
 * widen to 8 bits by bit replication; palette {c0, c1, (2 c0 + c1 + 1) / 3,
 * (c0 + 2 c1 + 1) / 3} if colour 0 > colour 1, else {c0, c1,
 * (c0 + c1 + 1) / 2, black}, per channel in integers.
 * ------------------------------------------------------------------ */
typedef struct jpt_bc1_level {    /* 24 bytes */
    const uint8_t *blocks;        /* device memory, 8-byte aligned */
    uint32_t width, height;
    uint32_t blocks_per_row;      /* ceil(width / 4) */
    uint32_t reserved;
} jpt_bc1_level;

typedef struct jpt_bc1_scene {    /* host struct holding device pointers */
    const jpt_bc1_level *levels;  /* n_levels, texture by texture, level 0 first */
    const jpt_texture_desc *textures;
    uint32_t n_levels, n_textures;
} jpt_bc1_scene;

/* Every pixel of every view with the level selection, taps and integer
 * weights of jpt_resolve (JPT_FILTER_NEAREST / BILINEAR / TRILINEAR,
 * optionally JPT_FILTER_MIP_OFF) over the BC1 texels.
 * Errors: JPT_E_ARG (also JPT_FILTER_BILINEAR_CLAMPED), JPT_E_HIP. */
jpt_status jpt_bc1_resolve(const jpt_bc1_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                           void *stream);

/* ------------------------------------------------------------------ *
 * Batched form: one frame over all views (jpt_mark_blocks, then
 * jpt_decode_blocks, then jpt_resolve, each with the arguments given here)
 * captured into a HIP graph, so that a frame of any number of views is one
 * graph launch.  The argument structs are copied at capture; the device
 * buffers they point to must outlive the graph, and every replay reads the
 * G-buffers and rewrites the frames in place.  With JPT_CACHE_LRU use
 * frame->frame_no = JPT_FRAME_AUTO, or every replay reuses the captured
 * frame number.  `stream` must not be the null stream.  The handle is
 * host memory owned by the library until jpt_graph_destroy.
 * ------------------------------------------------------------------ */
typedef struct jpt_graph jpt_graph;

/* Errors: JPT_E_ARG (also: stream already capturing), the errors of the
 * captured calls, JPT_E_HIP. */
jpt_status jpt_graph_capture(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                             jpt_frame *frame, jpt_cache *cache, uint32_t idct_mode, const jpt_tuning *tuning,
                             void *stream, jpt_graph **out);
/* Enqueue one frame on `stream`.  Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_graph_launch(jpt_graph *graph, void *stream);
/* Free the graph (NULL is a no-op).  Errors: JPT_E_HIP. */
jpt_status jpt_graph_destroy(jpt_graph *graph);

/* ------------------------------------------------------------------ *
 * Differentiable form.  The frame as a function of the dequantised DCT
 * coefficients of this frame's work items (paper: Decode, whose stages are
 * dequantisation, the 8x8 IDCT and the colour transform, followed by the
 * filtered lookup of Resolve), with the rounding and clamping of the 8-bit
 * path removed:
 *   texel = M (IDCT(F) + (128, 0, 0)), chroma replicated over 2x2 (4:2:0),
 *   M the JFIF full-range inverse (R = Y + 1.402 Cr, G = Y - 0.344136 Cb
 *   - 0.714136 Cr, B = Y + 1.772 Cb);
 *   frame = sum over the filter taps of (tap weight / 65536) x (level
 *   weight / 256) x texel, with the integer weights of jpt_resolve held
 *   constant.
 * Requires every block the views read to be a work item of the last
 * jpt_mark_blocks (JPT_CACHE_NONE with n_slots >= the visible blocks).
 * F and dF: n_rows x 6 x 64 floats, natural order (index v*8+u, v the
 * vertical frequency), row i for work item i, one 64-entry unit per data
 * unit of the item (4:2:0: Y0..Y3, Cb, Cr; 4:4:4: Y, Cb, Cr, then three zero
 * units).  Only the first min(items listed, max_items, n_rows) rows are read
 * or written: n_rows should be counters[JPT_CTR_ITEMS] of the frame.
 * texel_f (and dtexel below): 16 x 16 x 3 entries per cache slot, for
 * every slot up to the largest one a listed item uses (with
 * JPT_CACHE_NONE: counters[JPT_CTR_NEW] slots).  frame_f / dframe: the
 * views' pixels in order, width x height x 3 floats each, packed.  All pointers
 * are device memory owned by the caller; calls are asynchronous on `stream`.
 * ------------------------------------------------------------------ */

/* F = coefficient x quantiser for the listed work items (from frame->coef).
 * Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_dequantize(const jpt_scene *scene, const jpt_frame *frame, float *F, uint32_t n_rows, void *stream);

/* Forward: F -> texel_f (the work items' texels) -> frame_f.  Invalid
 * pixels and taps in blocks without a slot raise JPT_ERR_PIXEL in
 * frame->counters; background pixels get 0.
 * Errors: JPT_E_ARG, JPT_E_HIP. */
jpt_status jpt_fwd_float(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                         const jpt_frame *frame, const jpt_cache *cache, const float *F, uint32_t n_rows,
                         float *texel_f, float *frame_f, void *stream);

/* Backward: dframe = dL/dframe_f -> dF = dL/dF.  dtexel is scratch of
 * 768 int64 per slot as texel_f: texel gradients in fixed point, summed
 * with integer atomics so that the result does not depend on their order.
 * The unit is 2^-s with s chosen per call from m = max |dframe| (kept in
 * counters[JPT_CTR_GRAD_MAX] as fp32 bits) so that every tap's product
 * stays below 2^36 units: sums are exact for up to 2^27 taps per texel and
 * each product is rounded to m 2^-37, at any scale of the loss.  Only the
 * listed items' slots are cleared and used.  A non-finite dframe entry
 * raises JPT_ERR_GRAD.  Errors: JPT_E_ARG (also n_slots >= 2^24),
 * JPT_E_HIP. */
jpt_status jpt_backward(const jpt_scene *scene, const jpt_view *views, uint32_t n_views, uint32_t filter,
                        const jpt_frame *frame, const jpt_cache *cache, const float *dframe, int64_t *dtexel,
                        float *dF, uint32_t n_rows, void *stream);

uint32_t jpt_version(void);
const char *jpt_status_string(jpt_status s);

#ifdef __cplusplus
}
#endif
#endif /* JPT_H */
