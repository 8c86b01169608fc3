// Index signed-distance grid (gfx950): the SDF that the paper builds once from
// the template faces beside the BVH, storing only indices (Sec. 3.4,
// Initialization).  Grid nodes keep the ids of their k nearest template faces
// (found once with mg_knn_surface_query); every frame a node's signed distance
// is recomputed from those faces' current vertices - no search, one pass over
// the grid - and queries interpolate it trilinearly.
//
// Node (i, j, k) of an nx x ny x nz grid sits at lo + h (i, j, k); node index
// i + nx (j + ny k).  A node's value is the minimum point-to-triangle distance
// over its faces (ties to the lowest slot), signed by the winning face's normal
// (positive where the normal points, including the plane itself).
#include "mgu_internal.hpp"

namespace mgu {
namespace {

struct Grid {
    float lo_x, lo_y, lo_z, h;
    int32_t nx, ny, nz;
};

__device__ __forceinline__ f3 node_pos(const Grid &g, int64_t n) {
    const int64_t i = n % g.nx, j = (n / g.nx) % g.ny, k = n / (static_cast<int64_t>(g.nx) * g.ny);
    return f3{g.lo_x + g.h * static_cast<float>(i), g.lo_y + g.h * static_cast<float>(j),
              g.lo_z + g.h * static_cast<float>(k)};
}

__global__ __launch_bounds__(256) void grid_points_kernel(Grid g, int64_t n, float *__restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; v < n; v += stride)
        store3(out, n, v, node_pos(g, v));
}

__global__ __launch_bounds__(256) void sdf_update_kernel(const float *__restrict__ verts, int64_t nv,
                                                         const int32_t *__restrict__ faces, int64_t nf,
                                                         const int32_t *__restrict__ face_k, int k, Grid g,
                                                         int64_t n, float *__restrict__ sdf,
                                                         int32_t *__restrict__ face_out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; v < n; v += stride) {
        const f3 p = node_pos(g, v);
        float best = INFINITY;
        int32_t win = -1;
        float side = 1.0f;
        for (int s = 0; s < k; ++s) {
            const int32_t f = face_k[s * n + v];
            if (f < 0 || f >= nf) continue;       // ids outside the mesh are ignored
            const f3 A = load3(verts, nv, faces[f]);
            const f3 B = load3(verts, nv, faces[nf + f]);
            const f3 C = load3(verts, nv, faces[2 * nf + f]);
            float w1, w2;
            const float d2 = tri_closest(p, A, B, C, w1, w2);
            if (d2 < best) {
                best = d2;
                win = f;
                const f3 c = tri_point(A, B, C, w1, w2);
                side = fdot(p - c, tri_normal(A, B, C)) >= 0.0f ? 1.0f : -1.0f;
            }
        }
        sdf[v] = side * sqrtf(best);
        if (face_out) face_out[v] = win;
    }
}

// The values of sdf_update_kernel for a compile-time k: every face id and vertex of
// a node is loaded before any distance is computed (ids outside the mesh read face 0
// and do not count), so the gathers overlap instead of forming one chain per face,
// and the winner's sign is taken once, after the minimum.  Node coordinates use
// 32-bit index arithmetic (grids have fewer than 2^31 nodes).
template <int K>
__global__ __launch_bounds__(256) void sdf_update_k_kernel(const float *__restrict__ verts, int64_t nv,
                                                           const int32_t *__restrict__ faces, int64_t nf,
                                                           const int32_t *__restrict__ face_k, Grid g, int64_t n,
                                                           float *__restrict__ sdf, int32_t *__restrict__ face_out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    const uint32_t nx = static_cast<uint32_t>(g.nx), ny = static_cast<uint32_t>(g.ny);
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; v < n; v += stride) {
        const uint32_t u = static_cast<uint32_t>(v), i = u % nx, j = (u / nx) % ny, kk = u / (nx * ny);
        const f3 p = f3{g.lo_x + g.h * static_cast<float>(i), g.lo_y + g.h * static_cast<float>(j),
                        g.lo_z + g.h * static_cast<float>(kk)};
        int32_t fid[K];
        bool ok[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int32_t f = face_k[s * n + v];
            ok[s] = f >= 0 && f < nf;
            fid[s] = ok[s] ? f : 0;
        }
        f3 A[K], B[K], C[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            A[s] = load3(verts, nv, faces[fid[s]]);
            B[s] = load3(verts, nv, faces[nf + fid[s]]);
            C[s] = load3(verts, nv, faces[2 * nf + fid[s]]);
        }
        float best = INFINITY, bw1 = 0.0f, bw2 = 0.0f;
        int32_t win = -1;
        f3 bA = f3{0.0f, 0.0f, 0.0f}, bB = bA, bC = bA;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            float w1, w2;
            const float d2 = tri_closest(p, A[s], B[s], C[s], w1, w2);
            if (ok[s] && d2 < best) {             // ties keep the lowest slot
                best = d2; win = fid[s];
                bA = A[s]; bB = B[s]; bC = C[s]; bw1 = w1; bw2 = w2;
            }
        }
        float side = 1.0f;
        if (win >= 0) {
            const f3 c = tri_point(bA, bB, bC, bw1, bw2);
            side = fdot(p - c, tri_normal(bA, bB, bC)) >= 0.0f ? 1.0f : -1.0f;
        }
        sdf[v] = side * sqrtf(best);
        if (face_out) face_out[v] = win;
    }
}

__global__ __launch_bounds__(256) void sdf_sample_kernel(const float *__restrict__ sdf, Grid g,
                                                         const float *__restrict__ q, int64_t nq,
                                                         float *__restrict__ out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t >= nq) return;
    const f3 p = load3(q, nq, t);
    const float r = 1.0f / g.h;
    const float ux = (p.x - g.lo_x) * r, uy = (p.y - g.lo_y) * r, uz = (p.z - g.lo_z) * r;
    if (!(ux >= 0.0f && uy >= 0.0f && uz >= 0.0f && ux <= g.nx - 1 && uy <= g.ny - 1 && uz <= g.nz - 1)) {
        out[t] = INFINITY;
        return;
    }
    const int i = min(static_cast<int>(floorf(ux)), g.nx - 2);
    const int j = min(static_cast<int>(floorf(uy)), g.ny - 2);
    const int k = min(static_cast<int>(floorf(uz)), g.nz - 2);
    const float tx = ux - i, ty = uy - j, tz = uz - k;
    const int64_t sx = 1, sy = g.nx, sz = static_cast<int64_t>(g.nx) * g.ny;
    const int64_t b = i + sy * j + sz * k;
    const float c00 = (1.0f - tx) * sdf[b] + tx * sdf[b + sx];
    const float c10 = (1.0f - tx) * sdf[b + sy] + tx * sdf[b + sy + sx];
    const float c01 = (1.0f - tx) * sdf[b + sz] + tx * sdf[b + sz + sx];
    const float c11 = (1.0f - tx) * sdf[b + sz + sy] + tx * sdf[b + sz + sy + sx];
    const float c0 = (1.0f - ty) * c00 + ty * c10, c1 = (1.0f - ty) * c01 + ty * c11;
    out[t] = (1.0f - tz) * c0 + tz * c1;
}

inline bool bad_grid(float h, int32_t nx, int32_t ny, int32_t nz, int64_t &n) {
    if (!(h > 0.0f) || nx < 2 || ny < 2 || nz < 2) return true;
    n = static_cast<int64_t>(nx) * ny * nz;
    return n > INT32_MAX;
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_grid_points(float lo_x, float lo_y, float lo_z, float h, int32_t nx, int32_t ny, int32_t nz,
                                    float *points, void *stream) {
    int64_t n = 0;
    if (bad_grid(h, nx, ny, nz, n) || !points) return MG_ERR_INVALID_ARGUMENT;
    const Grid g{lo_x, lo_y, lo_z, h, nx, ny, nz};
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 4096));
    hipLaunchKernelGGL(grid_points_kernel, dim3(grid), dim3(256), 0, as_stream(stream), g, n, points);
    return launch_status();
}

extern "C" mg_status mg_sdf_update(const float *verts, int32_t n_verts, const int32_t *faces, int32_t n_faces,
                                   const int32_t *face_k, int32_t k, float lo_x, float lo_y, float lo_z, float h,
                                   int32_t nx, int32_t ny, int32_t nz, float *sdf, int32_t *face, void *stream) {
    int64_t n = 0;
    if (bad_grid(h, nx, ny, nz, n) || bad_count(n_verts) || bad_count(n_faces) || k < 1 || k > 64 || !face_k ||
        !sdf || (n_faces > 0 && (!verts || !faces)))
        return MG_ERR_INVALID_ARGUMENT;
    const Grid g{lo_x, lo_y, lo_z, h, nx, ny, nz};
    const int grid = static_cast<int>(std::min<int64_t>(blocks_for(n, 256), 8192));
    hipStream_t st = as_stream(stream);
    const int64_t nv = n_verts, nf = n_faces;
    if (n_faces > 0 && k == 1)
        hipLaunchKernelGGL(sdf_update_k_kernel<1>, dim3(grid), dim3(256), 0, st, verts, nv, faces, nf, face_k, g, n, sdf, face);
    else if (n_faces > 0 && k == 2)
        hipLaunchKernelGGL(sdf_update_k_kernel<2>, dim3(grid), dim3(256), 0, st, verts, nv, faces, nf, face_k, g, n, sdf, face);
    else if (n_faces > 0 && k == 4)
        hipLaunchKernelGGL(sdf_update_k_kernel<4>, dim3(grid), dim3(256), 0, st, verts, nv, faces, nf, face_k, g, n, sdf, face);
    else if (n_faces > 0 && k == 8)
        hipLaunchKernelGGL(sdf_update_k_kernel<8>, dim3(grid), dim3(256), 0, st, verts, nv, faces, nf, face_k, g, n, sdf, face);
    else
        hipLaunchKernelGGL(sdf_update_kernel, dim3(grid), dim3(256), 0, st, verts, nv, faces, nf, face_k, k, g, n,
                           sdf, face);
    return launch_status();
}

extern "C" mg_status mg_sdf_sample(const float *sdf, float lo_x, float lo_y, float lo_z, float h, int32_t nx,
                                   int32_t ny, int32_t nz, const float *queries, int32_t n_queries, float *out,
                                   void *stream) {
    int64_t n = 0;
    if (bad_grid(h, nx, ny, nz, n) || bad_count(n_queries) || !sdf) return MG_ERR_INVALID_ARGUMENT;
    if (n_queries == 0) return MG_OK;
    if (!queries || !out) return MG_ERR_INVALID_ARGUMENT;
    const Grid g{lo_x, lo_y, lo_z, h, nx, ny, nz};
    hipLaunchKernelGGL(sdf_sample_kernel, dim3(blocks_for(n_queries, 256)), dim3(256), 0, as_stream(stream), sdf,
                       g, queries, (int64_t)n_queries, out);
    return launch_status();
}
