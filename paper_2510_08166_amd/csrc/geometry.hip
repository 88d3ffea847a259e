// Geometry pass: the G-buffer the method starts from (paper: Method, the
// pass before Mark, which renders texture coordinates, texture ids and mip
// levels), produced on the GPU from textured triangles.
//
// Every pixel casts its centre ray from a pinhole camera and keeps the
// nearest triangle it hits (smallest t > 0, the lower index on equal t);
// uv is the hit's barycentric blend of the vertices' uv, and the level of
// detail is log2 of the larger texel footprint of a one-pixel step along x
// or y, the neighbouring rays met with the hit triangle's plane.  A
// workgroup shades a 64 x 4 pixel tile and walks the triangle list in
// chunks staged through LDS (one global load per triangle per workgroup).
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace {

constexpr int kGeoThreads = 256;
constexpr int kGeoTileW = 64, kGeoTileH = 4;
constexpr int kTriChunk = 256;

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// A triangle as the intersection test uses it: a vertex and two edges.
struct TriLds {
    V3 p0, e1, e2;
};

// Ray o + t d against the plane of (p0, e1, e2): barycentric b1, b2 and t
// (Cramer's rule, the Moller-Trumbore arrangement); false when parallel.
__device__ __forceinline__ bool plane_hit(V3 o, V3 d, const TriLds &T, float &t, float &b1, float &b2) {
    const V3 pv = cross(d, T.e2);
    const float det = dot(T.e1, pv);
    const float inv = 1.0f / det;
    const V3 tv = sub(o, T.p0);
    const V3 qv = cross(tv, T.e1);
    b1 = dot(tv, pv) * inv;
    b2 = dot(d, qv) * inv;
    t = dot(T.e2, qv) * inv;
    return det != 0.0f;
}

__device__ __forceinline__ V3 ray_dir(const jpt_camera &c, uint32_t W, uint32_t H, float px, float py) {
    const float sx = (2.0f * px / (float)W - 1.0f) * c.tan_half_x;
    const float sy = (1.0f - 2.0f * py / (float)H) * c.tan_half_y;
    return V3{c.fwd[0] + sx * c.right[0] + sy * c.up[0], c.fwd[1] + sx * c.right[1] + sy * c.up[1],
              c.fwd[2] + sx * c.right[2] + sy * c.up[2]};
}

__global__ __launch_bounds__(kGeoThreads) void k_geometry(const jpt_triangle *__restrict__ tris, uint32_t n_tris,
                                                          const jpt_camera cam, uint32_t W, uint32_t H,
                                                          uint32_t pitch, const jpt_texture_desc *__restrict__ texs,
                                                          uint32_t n_tex, jpt_gpixel *__restrict__ gbuf) {
    __shared__ TriLds s_tri[kTriChunk];
    const uint32_t x = blockIdx.x * kGeoTileW + (threadIdx.x & 63);
    const uint32_t y = blockIdx.y * kGeoTileH + (threadIdx.x >> 6);
    const V3 o{cam.eye[0], cam.eye[1], cam.eye[2]};
    const V3 d = ray_dir(cam, W, H, (float)x + 0.5f, (float)y + 0.5f);
    float best = INFINITY, hb1 = 0.0f, hb2 = 0.0f;
    uint32_t hit = 0xFFFFFFFFu;
    for (uint32_t base = 0; base < n_tris; base += kTriChunk) {
        __syncthreads();
        const uint32_t i = base + threadIdx.x;
        if (i < n_tris) {
            const jpt_triangle &T = tris[i];
            const V3 p0{T.p0[0], T.p0[1], T.p0[2]};
            s_tri[threadIdx.x] = TriLds{p0, sub(V3{T.p1[0], T.p1[1], T.p1[2]}, p0),
                                        sub(V3{T.p2[0], T.p2[1], T.p2[2]}, p0)};
        }
        __syncthreads();
        const uint32_t n = min((uint32_t)kTriChunk, n_tris - base);
        for (uint32_t k = 0; k < n; k++) {
            float t, b1, b2;
            const bool ok = plane_hit(o, d, s_tri[k], t, b1, b2);
            if (ok && b1 >= 0.0f && b2 >= 0.0f && b1 + b2 <= 1.0f && t > 0.0f && t < best) {
                best = t;
                hit = base + k;
                hb1 = b1;
                hb2 = b2;
            }
        }
    }
    if (x >= W || y >= H) return;
    jpt_gpixel out{0.0f, 0.0f, JPT_TEX_BACKGROUND, 0.0f};
    if (hit != 0xFFFFFFFFu) {
        const jpt_triangle &T = tris[hit];
        const V3 p0{T.p0[0], T.p0[1], T.p0[2]};
        const TriLds L{p0, sub(V3{T.p1[0], T.p1[1], T.p1[2]}, p0), sub(V3{T.p2[0], T.p2[1], T.p2[2]}, p0)};
        float u[3], v[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            float b1 = hb1, b2 = hb2, t;
            if (k) {
                const V3 dk = ray_dir(cam, W, H, (float)x + 0.5f + (k == 1 ? 1.0f : 0.0f),
                                      (float)y + 0.5f + (k == 2 ? 1.0f : 0.0f));
                if (!plane_hit(o, dk, L, t, b1, b2)) { b1 = hb1; b2 = hb2; }
            }
            const float b0 = 1.0f - b1 - b2;
            u[k] = b0 * T.uv0[0] + b1 * T.uv1[0] + b2 * T.uv2[0];
            v[k] = b0 * T.uv0[1] + b1 * T.uv1[1] + b2 * T.uv2[1];
        }
        float w = 1.0f, h = 1.0f;
        if (T.tex < n_tex) {
            w = (float)texs[T.tex].width;
            h = (float)texs[T.tex].height;
        }
        const float ax = (u[1] - u[0]) * w, ay = (v[1] - v[0]) * h;
        const float bx = (u[2] - u[0]) * w, by = (v[2] - v[0]) * h;
        const float rho = fmaxf(sqrtf(ax * ax + ay * ay), sqrtf(bx * bx + by * by));
        out = jpt_gpixel{u[0], v[0], T.tex, rho > 0.0f ? log2f(rho) : -64.0f};
    }
    gbuf[(size_t)y * pitch + x] = out;
}

}  // namespace

extern "C" jpt_status jpt_geometry_pass(const jpt_scene *scene, const jpt_triangle *tris, uint32_t n_tris,
                                        const jpt_camera *cam, uint32_t width, uint32_t height, uint32_t pitch,
                                        jpt_gpixel *gbuf, void *stream) {
    if (!scene || !cam || !gbuf || (n_tris && !tris) || pitch < width || !scene->textures) return JPT_E_ARG;
    if (width == 0 || height == 0) return JPT_OK;
    const dim3 grid((width + kGeoTileW - 1) / kGeoTileW, (height + kGeoTileH - 1) / kGeoTileH);
    hipLaunchKernelGGL(k_geometry, grid, dim3(kGeoThreads), 0, (hipStream_t)stream, tris, n_tris, *cam, width,
                       height, pitch, scene->textures, scene->n_textures, gbuf);
    HIP_CHECK_LAUNCH();
    return JPT_OK;
}
