// Sphere-mesh contact step from on-demand face normals (gfx950): collision
// response for spheres dropped on the reconstructed mesh (the falling-sphere
// simulation of Sec. 4.1 queries collisions every step and recomputes face
// normals on demand, Sec. 3.4 step 3).  One step of spheres of radius r:
//   mg_particles_integrate   v <- v + g dt, x <- x + v dt (semi-implicit Euler)
//   mg_closest_point_query   closest point c, face and unit face normal n at x
//   mg_contact_response      side = (x - c) . n; contact when side < 0 or
//                            |x - c| < r; contact normal nh = (x - c)/|x - c|
//                            when side >= 0 and |x - c| > 0, else n; then
//                            x <- c + r nh and, if v . nh < 0,
//                            v <- v - (1 + e)(v . nh) nh.
#include "mgu_internal.hpp"

namespace mgu {
namespace {

__global__ __launch_bounds__(256) void integrate_kernel(float *__restrict__ x, float *__restrict__ v, int64_t n,
                                                        f3 g, float dt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    f3 vi = load3(v, n, i) + dt * g;
    store3(v, n, i, vi);
    store3(x, n, i, load3(x, n, i) + dt * vi);
}

__global__ __launch_bounds__(256) void response_kernel(float *__restrict__ x, float *__restrict__ v, int64_t n,
                                                       const float *__restrict__ point,
                                                       const float *__restrict__ normal,
                                                       const int32_t *__restrict__ face, float radius, float e,
                                                       int32_t *__restrict__ contact) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const f3 p = load3(x, n, i), c = load3(point, n, i), nf = load3(normal, n, i);
    const f3 d = p - c;
    const float dist2 = dot(d, d);
    const float side = dot(d, nf);
    const bool has_face = face[i] >= 0 && dot(nf, nf) > 0.0f;
    const bool hit = has_face && (side < 0.0f || dist2 < radius * radius);
    if (contact) contact[i] = hit;
    if (!hit) return;
    const f3 nh = (side >= 0.0f && dist2 > 0.0f) ? (1.0f / sqrtf(dist2)) * d : nf;
    store3(x, n, i, c + radius * nh);
    f3 vi = load3(v, n, i);
    const float vn = dot(vi, nh);
    if (vn < 0.0f) store3(v, n, i, vi - ((1.0f + e) * vn) * nh);
}

}  // namespace
}  // namespace mgu

using namespace mgu;

extern "C" mg_status mg_particles_integrate(float *x, float *v, int32_t n, float gx, float gy, float gz, float dt,
                                            void *stream) {
    if (bad_count(n) || !(dt >= 0.0f)) return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    if (!x || !v) return MG_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(integrate_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, as_stream(stream), x, v,
                       (int64_t)n, f3{gx, gy, gz}, dt);
    return launch_status();
}

extern "C" mg_status mg_contact_response(float *x, float *v, int32_t n, const float *point, const float *normal,
                                         const int32_t *face, float radius, float restitution, int32_t *contact,
                                         void *stream) {
    if (bad_count(n) || !(radius >= 0.0f) || !(restitution >= 0.0f && restitution <= 1.0f))
        return MG_ERR_INVALID_ARGUMENT;
    if (n == 0) return MG_OK;
    if (!x || !v || !point || !normal || !face) return MG_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(response_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, as_stream(stream), x, v,
                       (int64_t)n, point, normal, face, radius, restitution, contact);
    return launch_status();
}
