/*
 * Geometry pass of the CPU oracle -- TEST INFRASTRUCTURE.
 *
 * The pass before Mark in the paper's pipeline (Method: the geometry pass
 * renders a G-buffer of texture coordinates, texture ids and mip map
 * levels): every pixel of a pinhole camera takes the nearest triangle its
 * centre ray hits, in fp64, by plain ray-triangle intersection; uv is
 * interpolated with the hit's barycentric coordinates, and the level of
 * detail is log2 of the larger texel footprint of a one-pixel step along x
 * or y (the neighbouring rays met with the same triangle's plane).
 */
#include <math.h>
#include <stdint.h>

#include "oracle.h"

typedef struct { double x, y, z; } v3;

static v3 vsub(v3 a, v3 b) { return (v3){a.x - b.x, a.y - b.y, a.z - b.z}; }
static v3 vcross(v3 a, v3 b) { return (v3){a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vld(const float *p) { return (v3){p[0], p[1], p[2]}; }

/* Ray o + t d against the plane of triangle (p0, p1, p2): barycentric b1,
 * b2 and distance t by Cramer's rule (the Moller-Trumbore arrangement).
 * Returns 0 when the ray is parallel to the plane. */
static int plane_hit(v3 o, v3 d, v3 p0, v3 p1, v3 p2, double *t, double *b1, double *b2) {
    v3 e1 = vsub(p1, p0), e2 = vsub(p2, p0);
    v3 pv = vcross(d, e2);
    double det = vdot(e1, pv);
    if (det == 0.0) return 0;
    v3 tv = vsub(o, p0);
    v3 qv = vcross(tv, e1);
    *b1 = vdot(tv, pv) / det;
    *b2 = vdot(d, qv) / det;
    *t = vdot(e2, qv) / det;
    return 1;
}

static v3 ray_dir(const orc_camera *c, int W, int H, double px, double py) {
    double sx = (2.0 * px / W - 1.0) * c->tan_half_x;
    double sy = (1.0 - 2.0 * py / H) * c->tan_half_y;
    return (v3){c->fwd[0] + sx * c->right[0] + sy * c->up[0], c->fwd[1] + sx * c->right[1] + sy * c->up[1],
                c->fwd[2] + sx * c->right[2] + sy * c->up[2]};
}

void orc_geometry(const orc_triangle *tris, int64_t n_tris, const orc_camera *cam, int W, int H,
                  const int32_t *tex_w, const int32_t *tex_h, int n_tex, orc_gpixel *g, int32_t *tri_out) {
    v3 o = vld(cam->eye);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            v3 d = ray_dir(cam, W, H, x + 0.5, y + 0.5);
            double best = INFINITY;
            int64_t hit = -1;
            double hb1 = 0, hb2 = 0;
            for (int64_t i = 0; i < n_tris; i++) {
                double t, b1, b2;
                if (!plane_hit(o, d, vld(tris[i].p0), vld(tris[i].p1), vld(tris[i].p2), &t, &b1, &b2)) continue;
                if (b1 < 0.0 || b2 < 0.0 || b1 + b2 > 1.0 || !(t > 0.0)) continue;
                if (t < best) { best = t; hit = i; hb1 = b1; hb2 = b2; }
            }
            orc_gpixel *px = &g[(size_t)y * W + x];
            if (tri_out) tri_out[(size_t)y * W + x] = (int32_t)hit;
            if (hit < 0) {
                px->u = 0.0f; px->v = 0.0f; px->tex = 0xFFFFFFFFu; px->lod = 0.0f;
                continue;
            }
            const orc_triangle *T = &tris[hit];
            v3 p0 = vld(T->p0), p1 = vld(T->p1), p2 = vld(T->p2);
            double uv[3][2];
            /* uv at the centre ray and at the rays one pixel right and one down */
            const double dxs[3] = {0.0, 1.0, 0.0}, dys[3] = {0.0, 0.0, 1.0};
            for (int k = 0; k < 3; k++) {
                double t, b1 = hb1, b2 = hb2;
                if (k) {
                    v3 dk = ray_dir(cam, W, H, x + 0.5 + dxs[k], y + 0.5 + dys[k]);
                    if (!plane_hit(o, dk, p0, p1, p2, &t, &b1, &b2)) { b1 = hb1; b2 = hb2; }
                }
                double b0 = 1.0 - b1 - b2;
                uv[k][0] = b0 * T->uv0[0] + b1 * T->uv1[0] + b2 * T->uv2[0];
                uv[k][1] = b0 * T->uv0[1] + b1 * T->uv1[1] + b2 * T->uv2[1];
            }
            double w = 1.0, h = 1.0;
            if (T->tex < (uint32_t)n_tex) { w = tex_w[T->tex]; h = tex_h[T->tex]; }
            double ax = (uv[1][0] - uv[0][0]) * w, ay = (uv[1][1] - uv[0][1]) * h;
            double bx = (uv[2][0] - uv[0][0]) * w, by = (uv[2][1] - uv[0][1]) * h;
            double rho = fmax(sqrt(ax * ax + ay * ay), sqrt(bx * bx + by * by));
            px->u = (float)uv[0][0];
            px->v = (float)uv[0][1];
            px->tex = T->tex;
            px->lod = rho > 0.0 ? (float)log2(rho) : -64.0f;
        }
}
