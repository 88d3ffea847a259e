// Internal constants of libjpt shared by its host and device code.
#pragma once
#include <stdint.h>

// GPU decode tables (one table set = JPT_TABLESET_WORDS u32), for table t
// (0 DC luma, 1 AC luma, 2 DC chroma, 3 AC chroma):
//   [t*1024, +1024)        fast table indexed by the next JPT_FAST_BITS bits;
//   [4096 + t*512, +512)   long table: canonical codes longer than
//                          JPT_FAST_BITS bits fill the top of the 16-bit code
//                          space, [T, 65536) with T = (first code value past
//                          the 10-bit codes) << 6; entry p16 - T for a 16-bit
//                          prefix p16 >= T (when 65536 - T <= 512);
//   [6144 + t*128, +128)   canonical data for the general case:
//                          [0..16] largest code of each length (-1 if none),
//                          [17..33] symbol index minus code per length,
//                          [34..97] the 256 symbol bytes, [98] T,
//                          [99] 1 if the long table covers [T, 65536).
// Entry: bits 0-4 bits consumed (0: not resolved by this table), bit 5
// value included (code and appended bits both fit the index), bits 6-9
// size (SSSS), bits 10-13 run (RRRR), bit 15 invalid symbol, bits 16-31
// value.
#define JPT_FAST_BITS 10
#define JPT_FAST_SIZE 1024
#define JPT_LONG_OFFSET 4096
#define JPT_LONG_SIZE 512
#define JPT_SLOW_OFFSET 6144
#define JPT_SLOW_WORDS 128
#define JPT_SLOW_T 98
#define JPT_SLOW_LONG_OK 99
#define JPT_FE_FUSED (1u << 5)
#define JPT_FE_BAD (1u << 15)

// Compaction: bitmask words per scan tile (256 threads, one word each).
#define JPT_SCAN_TILE_WORDS 256

// Words of a level's spliced stream as stored: the data, at least
// JPT_STREAM_PAD_WORDS zero words, rounded up to whole 16-byte vectors.
#define JPT_STREAM_WORDS(bits) (((((uint64_t)(bits) + 31) / 32 + JPT_STREAM_PAD_WORDS) + 3) & ~(uint64_t)3)

// LRU cache metadata (jpt_cache.meta): scalars, then the age histogram of
// the eviction candidates (ages capped at JPT_LRU_MAX_AGE), then the three
// digit histograms of the exact selection inside the capped bin (digit 0 =
// age >> 21, digit 1 = (age >> 10) & 2047, digit 2 = age & 1023).
#define JPT_META_TOP 0        // free slots on the stack
#define JPT_META_NEW 1        // blocks to place this frame
#define JPT_META_NEED 2       // evictions needed this frame
#define JPT_META_ABIN 3       // age bin of the last evicted blocks
#define JPT_META_TIES 4       // blocks of equal age to evict (smallest ids)
#define JPT_META_EVICTED 5    // evicted this frame
#define JPT_META_FRAME 6      // frame number of the next frame (JPT_FRAME_AUTO)
#define JPT_META_DEEP 7       // 1: the evictions end inside the capped bin
#define JPT_META_D0 8         // chosen digit 0, and evictions left below it
#define JPT_META_R0 9
#define JPT_META_D1 10        // chosen digit 1, and evictions left below it
#define JPT_META_R1 11
#define JPT_META_QCOUNT 12    // hash-map cache: blocks queued this frame
#define JPT_META_VISIBLE 13   // hash-map cache: blocks read this frame
#define JPT_META_HIST 16      // JPT_LRU_MAX_AGE + 1 bins
#define JPT_META_DH0 (JPT_META_HIST + JPT_LRU_MAX_AGE + 1)  // 2048 bins
#define JPT_META_DH1 (JPT_META_DH0 + 2048)                  // 2048 bins
#define JPT_META_DH2 (JPT_META_DH1 + 2048)                  // 1024 bins
