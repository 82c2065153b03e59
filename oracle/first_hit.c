/*
 * first_hit.c -- FP64 brute-force first-hit query (TEST INFRASTRUCTURE ONLY).
 *
 * Part of the oracle: a plain, slow, obviously correct CPU reference used only
 * by the tests, the smoke check and the CPU-baseline leg of the benchmark.  The
 * product path never links or calls it, and it shares no code with the GPU
 * library.
 *
 * What it computes.  The paper obtains the range of each beam by reading the
 * depth of the first visible surface along that beam (Section II-A, depth
 * generation, and eq.3 which maps a beam to the pixel whose depth is read).
 * Stated without the raster detour, that is the first intersection of the beam
 * ray o + t d with the triangle soup: the smallest t in (t_min, t_max] over all
 * triangles the ray passes through, ties broken by the smaller triangle index.
 * Here every ray is tested against every triangle in double precision with the
 * Moller-Trumbore formulation (two-sided, edges inclusive: u >= 0, v >= 0,
 * u + v <= 1; a zero determinant is a miss).
 *
 * Besides the hit it reports, per ray, the quantities that decide whether a
 * 32-bit implementation can legitimately disagree with it:
 *   t_second  smallest t of any *other* triangle that is also hit (INF if none),
 *   edge_in   distance, in the plane of the hit triangle, from the hit point to
 *             the nearest edge of that triangle (>= 0; INF if no hit),
 *   near_t    smallest t over triangles that the ray misses by less than
 *             edge_abs + edge_rel * t (measured the same way, outside the
 *             triangle) -- a "near miss" that rounding could turn into a hit.
 * Vertices are given in double (oracle_first_hit_d) or float32
 * (oracle_first_hit, promoted exactly to double).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

int oracle_num_threads(void) { return omp_get_max_threads(); }

typedef struct { double v0[3], e1[3], e2[3]; double alt[3]; } tri64;

static inline void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* Returns 0 on success, -1 on allocation failure. */
int oracle_first_hit_d(int64_t n_rays, const double *orig, const double *dir,
                       int64_t n_tri, const double *vtx, const uint32_t *idx,
                       double t_min, double t_max, double edge_abs, double edge_rel,
                       int64_t *hit_tri, double *hit_t, double *t_second,
                       double *edge_in, double *near_t)
{
    tri64 *T = (tri64 *)malloc(sizeof(tri64) * (size_t)(n_tri > 0 ? n_tri : 1));
    if (!T) return -1;
    for (int64_t k = 0; k < n_tri; ++k) {
        double v[3][3];
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a)
                v[c][a] = vtx[3 * (size_t)idx[3 * k + c] + a];
        double e12[3], n[3];
        for (int a = 0; a < 3; ++a) {
            T[k].v0[a] = v[0][a];
            T[k].e1[a] = v[1][a] - v[0][a];
            T[k].e2[a] = v[2][a] - v[0][a];
            e12[a] = v[2][a] - v[1][a];
        }
        cross3(T[k].e1, T[k].e2, n);
        double twice_area = norm3(n);
        /* altitude onto the edge opposite vertex 0, 1, 2 */
        T[k].alt[0] = twice_area / norm3(e12);
        T[k].alt[1] = twice_area / norm3(T[k].e2);
        T[k].alt[2] = twice_area / norm3(T[k].e1);
    }

    /* Barycentric slack inside which near misses are examined: any point whose
       smallest barycentric coordinate is below -B is at least B * altitude
       outside the triangle. */
    const double B = 0.25;

#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t r = 0; r < n_rays; ++r) {
        const double *o = orig + 3 * r;
        const double *d = dir + 3 * r;
        int64_t k1 = -1;
        double t1 = INFINITY, t2 = INFINITY, e1 = INFINITY, nt = INFINITY;
        for (int64_t k = 0; k < n_tri; ++k) {
            const tri64 *tr = &T[k];
            double p[3], q[3], s[3];
            cross3(d, tr->e2, p);
            double det = dot3(tr->e1, p);
            if (det == 0.0) continue;
            double inv = 1.0 / det;
            s[0] = o[0] - tr->v0[0];
            s[1] = o[1] - tr->v0[1];
            s[2] = o[2] - tr->v0[2];
            double u = dot3(s, p) * inv;
            if (u < -B || u > 1.0 + 2.0 * B) continue;
            cross3(s, tr->e1, q);
            double v = dot3(d, q) * inv;
            if (v < -B || v > 1.0 + 2.0 * B) continue;
            double t = dot3(tr->e2, q) * inv;
            if (!(t > t_min && t <= t_max)) continue;
            double w = 1.0 - u - v;
            if (u >= 0.0 && v >= 0.0 && w >= 0.0) {
                if (t < t1 || (t == t1 && k < k1)) {
                    if (k1 >= 0) t2 = fmin(t2, t1);
                    t1 = t; k1 = k;
                    double ew = w * tr->alt[0], eu = u * tr->alt[1], ev = v * tr->alt[2];
                    e1 = fmin(ew, fmin(eu, ev));
                } else {
                    t2 = fmin(t2, t);
                }
            } else {
                double m = fmin(u, fmin(v, w));
                if (m < -B) continue;
                double ew = w * tr->alt[0], eu = u * tr->alt[1], ev = v * tr->alt[2];
                double e = fmin(ew, fmin(eu, ev));           /* < 0: outside */
                if (-e < edge_abs + edge_rel * t) nt = fmin(nt, t);
            }
        }
        hit_tri[r] = k1;
        hit_t[r] = t1;
        t_second[r] = t2;
        edge_in[r] = e1;
        near_t[r] = nt;
    }
    free(T);
    return 0;
}

/* The same query with float32 vertices (promoted exactly to double). */
int oracle_first_hit(int64_t n_rays, const double *orig, const double *dir,
                     int64_t n_tri, const float *vtx, const uint32_t *idx,
                     double t_min, double t_max, double edge_abs, double edge_rel,
                     int64_t *hit_tri, double *hit_t, double *t_second,
                     double *edge_in, double *near_t)
{
    int64_t nv = 0;
    for (int64_t k = 0; k < 3 * n_tri; ++k)
        if ((int64_t)idx[k] + 1 > nv) nv = (int64_t)idx[k] + 1;
    double *v = (double *)malloc(sizeof(double) * 3 * (size_t)(nv > 0 ? nv : 1));
    if (!v) return -1;
    for (int64_t k = 0; k < 3 * nv; ++k) v[k] = (double)vtx[k];
    int rc = oracle_first_hit_d(n_rays, orig, dir, n_tri, v, idx, t_min, t_max, edge_abs, edge_rel,
                                hit_tri, hit_t, t_second, edge_in, near_t);
    free(v);
    return rc;
}
