// Internal constants of libjpt shared by its host and device code.
#pragma once
#include <stdint.h>

// GPU decode tables (one table set = JPT_TABLESET_WORDS u32):
//   [t*1024, t*1024+1024)  fast table of table t (0 DC luma, 1 AC luma,
//                          2 DC chroma, 3 AC chroma), indexed by the next
//                          JPT_FAST_BITS stream bits;
//   [4096 + t*128, +128)   slow-path data of table t for longer codes:
//                          [0..16] largest code of each length (-1 if none),
//                          [17..33] symbol index minus code per length,
//                          [34..97] the 256 symbol bytes.
// Fast entry: bits 0-4 bits consumed (0: take the slow path), bit 5 value
// included (code and appended bits both fit the index), bits 6-9 size
// (SSSS), bits 10-13 run (RRRR), bit 15 invalid symbol, bits 16-31 value.
#define JPT_FAST_BITS 10
#define JPT_FAST_SIZE 1024
#define JPT_SLOW_OFFSET 4096
#define JPT_SLOW_WORDS 128
#define JPT_FE_FUSED (1u << 5)
#define JPT_FE_BAD (1u << 15)

// Compaction: bitmask words per scan tile (256 threads x 4 words).
#define JPT_SCAN_TILE_WORDS 1024
