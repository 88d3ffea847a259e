/*
 * BC1 (S3TC DXT1) decoding by definition -- TEST INFRASTRUCTURE.
 *
 * The fixed-rate baseline the paper compares against (Background: BC1):
 * every 4x4 texel block is 8 bytes, little-endian: colour 0 (RGB565, u16),
 * colour 1 (RGB565, u16), then 16 two-bit indices, texel (i, j) of the
 * block (column i, row j) at bits 2 (4 j + i).  Endpoints widen to 8 bits
 * by bit replication.  If colour 0 > colour 1 (as u16) the palette is
 * {c0, c1, (2 c0 + c1 + 1) / 3, (c0 + 2 c1 + 1) / 3}, else
 * {c0, c1, (c0 + c1 + 1) / 2, black}, per channel in integers.
 */
#include <stdint.h>
#include <string.h>

#include "oracle.h"

static void rgb565(uint32_t c, int out[3]) {
    int r = (c >> 11) & 31, g = (c >> 5) & 63, b = c & 31;
    out[0] = (r << 3) | (r >> 2);
    out[1] = (g << 2) | (g >> 4);
    out[2] = (b << 3) | (b >> 2);
}

void orc_bc1_decode(const uint8_t *blocks, int w, int h, uint8_t *rgb) {
    const int bw = (w + 3) / 4, bh = (h + 3) / 4;
    for (int by = 0; by < bh; by++)
        for (int bx = 0; bx < bw; bx++) {
            const uint8_t *b = blocks + ((size_t)by * bw + bx) * 8;
            uint32_t c0 = (uint32_t)b[0] | ((uint32_t)b[1] << 8), c1 = (uint32_t)b[2] | ((uint32_t)b[3] << 8);
            uint32_t idx = (uint32_t)b[4] | ((uint32_t)b[5] << 8) | ((uint32_t)b[6] << 16) | ((uint32_t)b[7] << 24);
            int p[4][3];
            rgb565(c0, p[0]);
            rgb565(c1, p[1]);
            for (int c = 0; c < 3; c++) {
                if (c0 > c1) {
                    p[2][c] = (2 * p[0][c] + p[1][c] + 1) / 3;
                    p[3][c] = (p[0][c] + 2 * p[1][c] + 1) / 3;
                } else {
                    p[2][c] = (p[0][c] + p[1][c] + 1) / 2;
                    p[3][c] = 0;
                }
            }
            for (int j = 0; j < 4; j++)
                for (int i = 0; i < 4; i++) {
                    int x = 4 * bx + i, y = 4 * by + j;
                    if (x >= w || y >= h) continue;
                    int k = (idx >> (2 * (4 * j + i))) & 3;
                    for (int c = 0; c < 3; c++) rgb[((size_t)y * w + x) * 3 + c] = (uint8_t)p[k][c];
                }
        }
}
