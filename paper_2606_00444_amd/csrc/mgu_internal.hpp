// Internal helpers shared by the libmgu HIP translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mgu.h"

namespace mgu {

constexpr int kWave = 64;
constexpr int kMaxCount = 1 << 30;

// ---------------------------------------------------------------- host side
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool bad_count(int64_t n) { return n < 0 || n >= kMaxCount; }

inline int blocks_for(int64_t n, int threads) {
    return static_cast<int>((n + threads - 1) / threads);
}

// Maps the status of the last launch (or any HIP call) to mg_status.
inline mg_status launch_status() {
    return hipGetLastError() == hipSuccess ? MG_OK : MG_ERR_HIP;
}

// ---------------------------------------------------------------- device side
struct f3 {
    float x, y, z;
};

__device__ __forceinline__ f3 mk(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return f3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return f3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return f3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
    return f3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// a*b - c*d with both products rounded (not fused): exactly zero whenever the two
// products are the same, as the region determinants and the cross product of a
// triangle with two equal vertices are.
__device__ __forceinline__ float det2(float a, float b, float c, float d) {
#pragma clang fp contract(off)
    return a * b - c * d;
}
// Cross product of rounded products: exactly zero when a == b or either is zero,
// so a triangle with two equal vertices has no normal.
__device__ __forceinline__ f3 cross_rounded(f3 a, f3 b) {
    return f3{det2(a.y, b.z, a.z, b.y), det2(a.z, b.x, a.x, b.z), det2(a.x, b.y, a.y, b.x)};
}
__device__ __forceinline__ f3 fmin3(f3 a, f3 b) { return f3{fminf(a.x, b.x), fminf(a.y, b.y), fminf(a.z, b.z)}; }
__device__ __forceinline__ f3 fmax3(f3 a, f3 b) { return f3{fmaxf(a.x, b.x), fmaxf(a.y, b.y), fmaxf(a.z, b.z)}; }

// SoA [3][n] load of element i.
__device__ __forceinline__ f3 load3(const float *__restrict__ p, int64_t n, int64_t i) {
    return f3{p[i], p[n + i], p[2 * n + i]};
}
// Vertex i of [3][n] through an id stored in a BVH at build time, clamped into
// [0, n): a caller that passes fewer vertices than the build reads wrong values
// (and is told so by the BVH's status word) but never outside its array.
__device__ __forceinline__ f3 vload(const float *__restrict__ p, int64_t n, int64_t i) {
    i = static_cast<uint64_t>(i) < static_cast<uint64_t>(n) ? i : (i < 0 ? 0 : n - 1);
    return load3(p, n, i);
}
__device__ __forceinline__ void store3(float *__restrict__ p, int64_t n, int64_t i, f3 v) {
    p[i] = v.x;
    p[n + i] = v.y;
    p[2 * n + i] = v.z;
}

// Dot product with explicit fused multiply-adds.  The closest-point, normal and
// re-pose arithmetic below is written with contraction off and explicit fmaf
// (or separately rounded products), so its rounding is fixed by the source and
// not by the compiler's choice of where to fuse at each inlined call site: the
// brute-force kernel, every traversal variant and the batched kernel then give
// bitwise the same distances, points and normals for the same face.
__device__ __forceinline__ float fdot(f3 a, f3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The point (1 - w1 - w2) a + w1 b + w2 c.
__device__ __forceinline__ f3 tri_point(f3 a, f3 b, f3 c, float w1, float w2) {
#pragma clang fp contract(off)
    const float w0 = (1.0f - w1) - w2;
    return f3{fmaf(w2, c.x, fmaf(w1, b.x, w0 * a.x)), fmaf(w2, c.y, fmaf(w1, b.y, w0 * a.y)),
              fmaf(w2, c.z, fmaf(w1, b.z, w0 * a.z))};
}

__device__ __forceinline__ float seg_closest(f3 p, f3 a, f3 b, float &t) {
#pragma clang fp contract(off)
    const f3 ab = b - a;
    const float den = fdot(ab, ab);
    t = den > 0.0f ? fdot(p - a, ab) * rcp(den) : 0.0f;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    const f3 d = p - f3{fmaf(t, ab.x, a.x), fmaf(t, ab.y, a.y), fmaf(t, ab.z, a.z)};
    return fdot(d, d);
}

// Closest point on triangle abc to p by Voronoi regions (Ericson 2005,
// Sec. 5.1.5).  Returns squared distance; w1, w2 are the barycentric weights of
// b and c (weight of a = 1 - w1 - w2).  A triangle whose interior denominator
// is not positive (zero area in float32) falls back to the nearest of its edge
// segments, ties in the order ab, ac, bc.  Quotients use the hardware
// reciprocal (about 1 ulp); vertex regions return the vertex exactly.
// Triangles with two equal vertices (segments) are answered exactly: their region
// determinants va, vb, vc are exact zeros (det2), and edge AB takes d3 < 0
// strictly, which excludes d1 = d3 = 0 (a == b: the other tests of edge AB hold for
// every p) and nothing else that reaches it (d3 = 0 past vertex B means d4 > 0, so
// vc = d1 d4 > 0 unless d1 = 0).  Then a == b ends in vertex A, vertex C or edge AC,
// and b == c or a == c in vertex A, vertex B or edge AB.
__device__ __forceinline__ float tri_closest(f3 p, f3 a, f3 b, f3 c, float &w1, float &w2) {
#pragma clang fp contract(off)
    const f3 ab = b - a, ac = c - a, ap = p - a;
    const float d1 = fdot(ab, ap), d2 = fdot(ac, ap);
    if (d1 <= 0.0f && d2 <= 0.0f) {
        w1 = 0.0f; w2 = 0.0f;
    } else {
        const f3 bp = p - b;
        const float d3 = fdot(ab, bp), d4 = fdot(ac, bp);
        const float vc = det2(d1, d4, d3, d2);
        if (d3 >= 0.0f && d4 <= d3) {
            w1 = 1.0f; w2 = 0.0f;
        } else if (vc <= 0.0f && d1 >= 0.0f && d3 < 0.0f) {
            w1 = d1 * rcp(d1 - d3); w2 = 0.0f;
        } else {
            const f3 cp = p - c;
            const float d5 = fdot(ab, cp), d6 = fdot(ac, cp);
            const float vb = det2(d5, d2, d1, d6);
            const float va = det2(d3, d6, d5, d4);
            const float e43 = d4 - d3, e56 = d5 - d6;
            if (d6 >= 0.0f && d5 <= d6) {
                w1 = 0.0f; w2 = 1.0f;
            } else if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
                const float den = d2 - d6;
                w1 = 0.0f; w2 = den != 0.0f ? d2 * rcp(den) : 0.0f;
            } else if (va <= 0.0f && e43 >= 0.0f && e56 >= 0.0f) {
                const float den = e43 + e56;
                const float t = den != 0.0f ? e43 * rcp(den) : 0.0f;
                w1 = 1.0f - t; w2 = t;
            } else {
                const float den = (va + vb) + vc;
                if (den > 0.0f) {
                    const float r = rcp(den);
                    w1 = vb * r; w2 = vc * r;
                } else {
                    float t, best = seg_closest(p, a, b, t);
                    w1 = t; w2 = 0.0f;
                    float d = seg_closest(p, a, c, t);
                    if (d < best) { best = d; w1 = 0.0f; w2 = t; }
                    d = seg_closest(p, b, c, t);
                    if (d < best) { w1 = 1.0f - t; w2 = t; }
                }
            }
        }
    }
    const f3 d = p - tri_point(a, b, c, w1, w2);
    return fdot(d, d);
}

// Unit normal of triangle abc from its stored winding; zero when |ab| == 0 or
// |ab x ac| == 0 (degenerate; exact for repeated vertices, see cross_rounded).
__device__ __forceinline__ f3 tri_normal(f3 a, f3 b, f3 c) {
#pragma clang fp contract(off)
    const f3 e1 = b - a;
    const f3 n = cross_rounded(e1, c - a);
    const float l1 = fdot(e1, e1), ln = fdot(n, n);
    if (l1 == 0.0f || ln == 0.0f) return f3{0.0f, 0.0f, 0.0f};
    const float r = 1.0f / sqrtf(ln);
    return f3{r * n.x, r * n.y, r * n.z};
}

// Squared distance from p to an axis-aligned box.
__device__ __forceinline__ float box_dist2(f3 p, f3 lo, f3 hi) {
    float dx = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.0f);
    float dy = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.0f);
    float dz = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

// Order-preserving float <-> uint32 encoding (for atomic min/max of floats).
__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace mgu
