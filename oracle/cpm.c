/*
 * Brute-force closest point on a triangle mesh, float64, plain C.
 *
 * TEST INFRASTRUCTURE ONLY: part of the oracle; loaded by oracle/closest.py
 * through ctypes.  Shares no code with the HIP library.
 *
 * For every query p, every face is tested (NearestSurface read as the single
 * nearest face, Sec. 3.3 Eq. 2 of the paper); exact ties of the squared distance
 * keep the lowest face id.  Closest point on one triangle: Ericson, Real-Time
 * Collision Detection (2005), Sec. 5.1.5 (Voronoi regions).  A triangle of zero
 * area (ab x ac == 0 exactly: its vertices are collinear or repeated, so the
 * closed triangle is a segment or a point) is handled as the nearest of its edge
 * segments AB, AC, BC (ties in that order); the region tests assume a proper
 * triangle (with a == b they would accept edge AB for every query).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC cpm.c -o libmgu_oracle.so
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double x, y, z; } d3;

static d3 sub(d3 a, d3 b) { d3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

static double seg(d3 p, d3 a, d3 b, double *t_out)
{
    d3 ab = sub(b, a);
    double den = dot(ab, ab);
    double t = den > 0.0 ? dot(sub(p, a), ab) / den : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    d3 q = {a.x + t * ab.x, a.y + t * ab.y, a.z + t * ab.z};
    d3 d = sub(p, q);
    *t_out = t;
    return dot(d, d);
}

/* weights w[3] of the closest point of triangle abc to p; returns squared distance */
static double tri_closest(d3 p, d3 a, d3 b, d3 c, double w[3])
{
    d3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    d3 n = {ab.y * ac.z - ab.z * ac.y, ab.z * ac.x - ab.x * ac.z, ab.x * ac.y - ab.y * ac.x};
    if (dot(n, n) == 0.0) goto flat;
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { w[0] = 1; w[1] = 0; w[2] = 0; goto done; }
    d3 bp = sub(p, b);
    double d3_ = dot(ab, bp), d4 = dot(ac, bp);
    if (d3_ >= 0.0 && d4 <= d3_) { w[0] = 0; w[1] = 1; w[2] = 0; goto done; }
    double vc = d1 * d4 - d3_ * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3_ <= 0.0) {
        double v = d1 / (d1 - d3_);
        w[0] = 1 - v; w[1] = v; w[2] = 0; goto done;
    }
    d3 cp = sub(p, c);
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { w[0] = 0; w[1] = 0; w[2] = 1; goto done; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double t = d2 / (d2 - d6);
        w[0] = 1 - t; w[1] = 0; w[2] = t; goto done;
    }
    double va = d3_ * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3_) >= 0.0 && (d5 - d6) >= 0.0) {
        double t = (d4 - d3_) / ((d4 - d3_) + (d5 - d6));
        w[0] = 0; w[1] = 1 - t; w[2] = t; goto done;
    }
    {
        double den = va + vb + vc;
        if (den > 0.0) {
            double v = vb / den, u = vc / den;
            w[0] = 1 - v - u; w[1] = v; w[2] = u; goto done;
        }
    }
flat:
    {   /* zero area: nearest edge segment */
        double t, best = seg(p, a, b, &t);
        w[0] = 1 - t; w[1] = t; w[2] = 0;
        double d = seg(p, a, c, &t);
        if (d < best) { best = d; w[0] = 1 - t; w[1] = 0; w[2] = t; }
        d = seg(p, b, c, &t);
        if (d < best) { best = d; w[0] = 0; w[1] = 1 - t; w[2] = t; }
    }
done:;
    d3 q = {w[0] * a.x + w[1] * b.x + w[2] * c.x, w[0] * a.y + w[1] * b.y + w[2] * c.y,
            w[0] * a.z + w[1] * b.z + w[2] * c.z};
    d3 d = sub(p, q);
    return dot(d, d);
}

/*
 * verts: [3][nv] float64; faces: [3][nf] int64; queries: [3][nq] float64.
 * Outputs: face [nq] int64 (-1 if none within max_dist2), point [3][nq],
 * bary [2][nq] (w1, w2), dist2 [nq] (+inf if none).  Returns 0, or -1 on a bad
 * face index.
 */
int oracle_closest_point_mesh(const double *verts, int64_t nv, const int64_t *faces, int64_t nf,
                              const double *queries, int64_t nq, double max_dist2,
                              int64_t *face, double *point, double *bary, double *dist2)
{
    for (int64_t f = 0; f < 3 * nf; ++f)
        if (faces[f] < 0 || faces[f] >= nv) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < nq; ++q) {
        d3 p = {queries[q], queries[nq + q], queries[2 * nq + q]};
        double best = INFINITY, bw[3] = {0, 0, 0};
        int64_t bf = -1;
        for (int64_t f = 0; f < nf; ++f) {
            int64_t i0 = faces[f], i1 = faces[nf + f], i2 = faces[2 * nf + f];
            d3 a = {verts[i0], verts[nv + i0], verts[2 * nv + i0]};
            d3 b = {verts[i1], verts[nv + i1], verts[2 * nv + i1]};
            d3 c = {verts[i2], verts[nv + i2], verts[2 * nv + i2]};
            double w[3];
            double d = tri_closest(p, a, b, c, w);
            if (d < best) { best = d; bf = f; bw[0] = w[0]; bw[1] = w[1]; bw[2] = w[2]; }
        }
        if (bf >= 0 && best <= max_dist2) {
            int64_t i0 = faces[bf], i1 = faces[nf + bf], i2 = faces[2 * nf + bf];
            for (int k = 0; k < 3; ++k)
                point[k * nq + q] = bw[0] * verts[k * nv + i0] + bw[1] * verts[k * nv + i1] +
                                    bw[2] * verts[k * nv + i2];
            face[q] = bf;
            bary[q] = bw[1];
            bary[nq + q] = bw[2];
            dist2[q] = best;
        } else {
            face[q] = -1;
            for (int k = 0; k < 3; ++k) point[k * nq + q] = queries[k * nq + q];
            bary[q] = 0;
            bary[nq + q] = 0;
            dist2[q] = INFINITY;
        }
    }
    return 0;
}

/* Nearest point of dst [3][m] for each src [3][n], lowest index on exact ties. */
void oracle_nearest_points(const double *src, int64_t n, const double *dst, int64_t m,
                           int64_t *idx, double *dist2)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double px = src[i], py = src[n + i], pz = src[2 * n + i];
        double best = INFINITY;
        int64_t bi = -1;
        for (int64_t j = 0; j < m; ++j) {
            double dx = px - dst[j], dy = py - dst[m + j], dz = pz - dst[2 * m + j];
            double d = dx * dx + dy * dy + dz * dz;
            if (d < best) { best = d; bi = j; }
        }
        idx[i] = bi;
        dist2[i] = best;
    }
}

/* Thread count of the OpenMP loops above (for timing the checker on one core or
 * on all of them; the results do not depend on it).  n <= 0 is ignored. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
