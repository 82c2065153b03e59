/*
 * walk_replay.c -- CPU replay of the BVH walk of one LiDAR scan over the tree
 * the GPU built (measurement infrastructure: it counts what the walk fetches).
 *
 * The roofline of the trace kernel needs, per beam, the number of 4-wide
 * nodes the walk fetches and the number of triangle records it tests.  This
 * file walks the tree copied from the device (lidar_debug_copy_bvh) with the
 * same FP32 decisions as the GPU's multi-lane walk, so that its counts depend
 * only on the tree and the beams, and can be checked against the GPU's own
 * counting kernel:
 *   - the ray: sensor-frame direction from FP64 cos/sin of the data-sheet
 *     angles, turned by the FP64 rotation of the (FP32) unit quaternion and
 *     rounded once to FP32; origin rounded once;
 *   - the box test: slab distances fma(b, 1/d, -o/d) in FP32, entry and exit
 *     clamped to [t_min, bound] by integer max/min of the bit patterns, the
 *     bound being 1.0000005 x the best hit distance so far (t_trace at first);
 *   - the order: children by their entry-distance bits with the two low bits
 *     replaced by the child slot, nearest first, depth first;
 *   - a leaf: every record tested by the watertight test (Woop, Benthin,
 *     Wald, JCGT 2013) in FP32, with an FP64 re-evaluation of the three edge
 *     functions when one rounds to zero, and the distance divided with one
 *     rounding; the best hit is the (t, original index) minimum.
 * Compiled with -ffp-contract=off (no fused operations but the explicit fmaf).
 * Layouts: node = four 32-byte slots {lo[3], ref, hi[3], pad}; ref bit 31
 * clear = node index, set = leaf (first record (ref >> 3) & 0x0FFFFFFF, count
 * (ref & 7) + 1), 0xFFFFFFFF = empty; record = 48 bytes
 * {v0[3], original index, v1[3], label, v2[3], material}.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define LEAF_BIT 0x80000000u
#define EMPTY_REF 0xFFFFFFFFu
#define NONE 0xFFFFFFFFu
#define MAX_STACK 256

typedef struct {
    float lo[3];
    uint32_t ref;
    float hi[3];
    uint32_t pad;
} slot_t;

typedef struct {
    float v0[3];
    uint32_t orig;
    float v1[3];
    uint32_t label;
    float v2[3];
    uint32_t mat;
} rec_t;

static uint32_t bits_of(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}
static float float_of(uint32_t u) {
    float f;
    memcpy(&f, &u, 4);
    return f;
}

typedef struct {
    float o[3], d[3];
    float inv[3], neg_o_inv[3];           /* 1/d (tiny components replaced), -o/d */
    int kx, ky, kz;
    float sx, sy, sz;                      /* shear of the watertight test */
} ray_t;

static float comp(const float v[3], int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

static void ray_setup(ray_t *r) {
    for (int a = 0; a < 3; ++a) {
        float da = r->d[a];
        if (fabsf(da) < 1e-20f) da = copysignf(1e-20f, da);
        r->inv[a] = 1.0f / da;
        r->neg_o_inv[a] = -r->o[a] * r->inv[a];
    }
    float ax = fabsf(r->d[0]), ay = fabsf(r->d[1]), az = fabsf(r->d[2]);
    int kz = (ax > ay) ? ((ax > az) ? 0 : 2) : ((ay > az) ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    float dkz = comp(r->d, kz);
    if (dkz < 0.0f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r->kx = kx;
    r->ky = ky;
    r->kz = kz;
    r->sx = comp(r->d, kx) / dkz;
    r->sy = comp(r->d, ky) / dkz;
    r->sz = 1.0f / dkz;
}

/* entry distance into a slot's box within [t_lo, bound], +inf if missed */
static float box_entry(const ray_t *r, const slot_t *c, float t_lo, float bound) {
    float x0 = fmaf(c->lo[0], r->inv[0], r->neg_o_inv[0]), x1 = fmaf(c->hi[0], r->inv[0], r->neg_o_inv[0]);
    float y0 = fmaf(c->lo[1], r->inv[1], r->neg_o_inv[1]), y1 = fmaf(c->hi[1], r->inv[1], r->neg_o_inv[1]);
    float z0 = fmaf(c->lo[2], r->inv[2], r->neg_o_inv[2]), z1 = fmaf(c->hi[2], r->inv[2], r->neg_o_inv[2]);
    float near = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fminf(z0, z1));
    float far = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fmaxf(z0, z1));
    int32_t tn = (int32_t)bits_of(near), tl = (int32_t)bits_of(t_lo);
    int32_t tf = (int32_t)bits_of(far), tb = (int32_t)bits_of(bound);
    tn = tn > tl ? tn : tl;
    tf = tf < tb ? tf : tb;
    return tn <= tf ? float_of((uint32_t)tn) : INFINITY;
}

/* watertight test; returns 1 and the distance if hit with t > t_lo */
static int tri_test(const ray_t *r, const rec_t *q, float t_lo, float *t_out) {
    float A0[3], B0[3], C0[3];
    for (int a = 0; a < 3; ++a) {
        A0[a] = q->v0[a] - r->o[a];
        B0[a] = q->v1[a] - r->o[a];
        C0[a] = q->v2[a] - r->o[a];
    }
    float akx = comp(A0, r->kx), aky = comp(A0, r->ky), akz = comp(A0, r->kz);
    float bkx = comp(B0, r->kx), bky = comp(B0, r->ky), bkz = comp(B0, r->kz);
    float ckx = comp(C0, r->kx), cky = comp(C0, r->ky), ckz = comp(C0, r->kz);
    float ax = fmaf(-r->sx, akz, akx), ay = fmaf(-r->sy, akz, aky);
    float bx = fmaf(-r->sx, bkz, bkx), by = fmaf(-r->sy, bkz, bky);
    float cx = fmaf(-r->sx, ckz, ckx), cy = fmaf(-r->sy, ckz, cky);
    float u = cx * by - cy * bx;
    float v = ax * cy - ay * cx;
    float w = bx * ay - by * ax;
    if (u == 0.0f || v == 0.0f || w == 0.0f) {
        u = (float)((double)cx * (double)by - (double)cy * (double)bx);
        v = (float)((double)ax * (double)cy - (double)ay * (double)cx);
        w = (float)((double)bx * (double)ay - (double)by * (double)ax);
    }
    int outside = (u < 0.0f || v < 0.0f || w < 0.0f) && (u > 0.0f || v > 0.0f || w > 0.0f);
    float det = u + v + w;
    float az_ = r->sz * akz, bz_ = r->sz * bkz, cz_ = r->sz * ckz;
    float tt = u * az_ + v * bz_ + w * cz_;
    float t = tt / det;
    *t_out = t;
    return !outside && det != 0.0f && t > t_lo;
}

/* One beam.  Returns 0, or -1 if the stack would overflow MAX_STACK. */
/* marks a fetched node or record (every writer stores 1) */
static void touch(uint8_t *flags, uint64_t k) {
    if (flags) {
#pragma omp atomic write
        flags[k] = 1;
    }
}

static int walk(const slot_t *nodes, const rec_t *recs, uint32_t root, const ray_t *r, float t_lo, float t_hi,
                uint32_t *n_nodes, uint32_t *n_tris, uint32_t *n_leaves, float *t_best, uint32_t *orig_best,
                uint8_t *node_touched, uint8_t *rec_touched, uint64_t *leaf_steps) {
    uint32_t stack[MAX_STACK];
    int sp = 0;
    float best_t = t_hi;
    uint32_t best_o = NONE;
    float bound = best_t * 1.0000005f;
    uint32_t nn = 0, nt = 0, nl = 0;
    uint32_t ref = root;
    for (;;) {
        if (leaf_steps && (ref & LEAF_BIT) && nn + nl < 128) leaf_steps[(nn + nl) >> 6] |= 1ull << ((nn + nl) & 63);
        if (ref & LEAF_BIT) {
            uint32_t first = (ref >> 3) & 0x0FFFFFFFu, cnt = (ref & 7u) + 1u;
            nt += cnt;
            ++nl;
            for (uint32_t k = 0; k < cnt; ++k) {
                const rec_t *q = recs + first + k;
                touch(rec_touched, first + k);
                float t;
                if (tri_test(r, q, t_lo, &t) && (t < best_t || (t == best_t && q->orig < best_o))) {
                    best_t = t;
                    best_o = q->orig;
                }
            }
            bound = best_t * 1.0000005f;
        } else {
            ++nn;
            touch(node_touched, ref);
            const slot_t *c = nodes + 4 * (size_t)ref;
            uint32_t key[4];
            for (uint32_t s = 0; s < 4; ++s) key[s] = (bits_of(box_entry(r, c + s, t_lo, bound)) & ~3u) | s;
            /* nearest first: sort the four keys (unique) ascending */
            uint32_t ord[4] = {0, 1, 2, 3};
            for (int a = 1; a < 4; ++a)
                for (int b = a; b > 0 && key[ord[b]] < key[ord[b - 1]]; --b) {
                    uint32_t t = ord[b];
                    ord[b] = ord[b - 1];
                    ord[b - 1] = t;
                }
            int hit = 0;
            for (int a = 0; a < 4; ++a) hit += key[a] < 0x7F800000u;
            if (hit > 0) {
                for (int a = hit - 1; a >= 1; --a) {
                    if (sp >= MAX_STACK) return -1;
                    stack[sp++] = c[ord[a]].ref;
                }
                ref = c[ord[0]].ref;
                continue;
            }
        }
        if (sp == 0) break;
        ref = stack[--sp];
    }
    *n_nodes = nn;
    *n_tris = nt;
    *n_leaves = nl;
    *t_best = best_t;
    *orig_best = best_o;
    return 0;
}

/*
 * Replays the walk for `n_beams` beams b (= j * n_az + i) of the scan:
 * elev_deg[n_ch] and the azimuth steps theta_i = az0 + i fov_h / n_az
 * (degrees), pose q = (w, x, y, z) (FP32, normalised in FP64) and p, traced
 * over (t_min, t_trace].  Writes per beam the node fetches, the triangle
 * records tested, the leaves visited, the best distance (t_trace if none) and the original index
 * of the best triangle (0xFFFFFFFF if none); node_touched / rec_touched (or
 * NULL) get 1 at every node and record the walks fetch; leaf_steps (or NULL,
 * two words per beam, zeroed by the caller) gets bit i set when step i of the
 * beam's walk is a leaf (steps beyond 128 are not marked).  Returns the number of beams
 * that could not be replayed (index beyond the scan, or a stack beyond 256
 * entries); their outputs are zero.
 */
int64_t walk_replay(const void *nodes, const void *recs, uint32_t root, const double *elev_deg, uint32_t n_ch,
                    uint32_t n_az, double az0_deg, double fov_h_deg, const float q[4], const float p[3],
                    float t_min, float t_trace, const uint32_t *beams, int64_t n_beams, uint32_t *node_visits,
                    uint32_t *tri_tests, uint32_t *leaf_visits, float *t_hit, uint32_t *tri_orig,
                    uint8_t *node_touched, uint8_t *rec_touched, uint64_t *leaf_steps) {
    const double deg = 3.14159265358979323846 / 180.0;
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n;
    x /= n;
    y /= n;
    z /= n;
    const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                         2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                         2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
    const float t_lo = t_min + 0.0f;
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
    for (int64_t k = 0; k < n_beams; ++k) {
        uint32_t b = beams[k], j = b / n_az, i = b % n_az;
        if (j >= n_ch) {
            node_visits[k] = tri_tests[k] = leaf_visits[k] = 0;
            t_hit[k] = 0.0f;
            tri_orig[k] = NONE;
            ++bad;
            continue;
        }
        double ae = elev_deg[j] * deg;
        double aa = (az0_deg + (double)i * (fov_h_deg / (double)n_az)) * deg;
        double cp = cos(ae), sp = sin(ae), ct = cos(aa), st = sin(aa);
        double s0 = cp * ct, s1 = cp * st, s2 = sp;
        ray_t r;
        r.d[0] = (float)(R[0] * s0 + R[1] * s1 + R[2] * s2);
        r.d[1] = (float)(R[3] * s0 + R[4] * s1 + R[5] * s2);
        r.d[2] = (float)(R[6] * s0 + R[7] * s1 + R[8] * s2);
        r.o[0] = p[0];
        r.o[1] = p[1];
        r.o[2] = p[2];
        ray_setup(&r);
        if (walk((const slot_t *)nodes, (const rec_t *)recs, root, &r, t_lo, t_trace, node_visits + k,
                 tri_tests + k, leaf_visits + k, t_hit + k, tri_orig + k, node_touched, rec_touched,
                 leaf_steps ? leaf_steps + 2 * k : NULL) != 0) {
            node_visits[k] = tri_tests[k] = leaf_visits[k] = 0;
            t_hit[k] = 0.0f;
            tri_orig[k] = NONE;
            ++bad;
        }
    }
    return bad;
}
