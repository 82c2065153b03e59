// lidar_device.hpp -- device-side building blocks of the LiDAR simulation path
// (gfx950, wave64).  Shared by the trace, batch and adjoint kernels.
//
// Data layouts in device memory
// -----------------------------
// BVH node (128 B, one per 4-wide node): four 32-byte child slots
//   { float lo[3]; uint32 ref; float hi[3]; uint32 pad; }
// so that one lane reads a whole node with 8 dwordx4 loads, or the four lanes
// of a quad each read their child slot with 2 dwordx4 loads (one 128 B line).
// child reference: bit 31 clear -> index of a 4-wide node;
//                  bit 31 set   -> leaf: first triangle record = (ref >> 3) & 0x0FFFFFFF,
//                                  count = (ref & 7) + 1;
//                  0xFFFFFFFF   -> empty slot (its box sits at 1e30, beyond any trace limit).
// Triangle record (48 B, leaf order = Morton order):
//   float4 a = (v0.xyz, original index bits), float4 b = (v1.xyz, label bits),
//   float4 c = (v2.xyz, material bits).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lidar {

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kEmptyRef = 0xFFFFFFFFu;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr float kBoxMullerBound = 6.6605f;   // |z| <= sqrt(64 ln 2) = 6.66043..

struct __align__(16) Child4 {
    float lo[3];
    uint32_t ref;
    float hi[3];
    uint32_t pad;
};

struct __align__(16) Node4 {
    Child4 c[4];
};
static_assert(sizeof(Node4) == 128, "node must be 128 bytes");

struct __align__(16) TriRec {
    float4 a, b, c;
};
static_assert(sizeof(TriRec) == 48, "triangle record must be 48 bytes");

__host__ __device__ inline uint32_t leaf_ref(uint32_t first, uint32_t count) {
    return kLeafBit | (first << 3) | (count - 1u);
}
__device__ inline uint32_t leaf_first(uint32_t ref) { return (ref >> 3) & 0x0FFFFFFFu; }
__device__ inline uint32_t leaf_count(uint32_t ref) { return (ref & 7u) + 1u; }

// ---------------------------------------------------------------------------
// Per-sensor parameters as seen by a kernel (one scan or one batch instance).
// Direction tables are FP64: cos/sin of the channel elevations and of the
// azimuth steps, computed on the device from the data-sheet angles.
// ---------------------------------------------------------------------------
// The parts of a partial sweep's column poses that are the same for every
// column of the tick (computed on the host): the head-angle window [a, b)
// (degrees), az0 and the azimuth step, the two end quaternions as given (qa,
// qb: the chord) and normalised with qb turned to the same hemisphere as qa
// (ua, ub), the arc w between them and 1 / sin(w), and the end positions.
struct SweepDev {
    double a, b, az0, step;
    double qa[4], qb[4], ua[4], ub[4];
    double w, inv_sin_w;
    float pa[3], pb[3];
    uint32_t chord;            // w < 1e-6: interpolate along the chord
    uint32_t pad_;
};

struct InstanceDev {
    const double *elev_cs;     // [2*n_ch]: cos phi_j, sin phi_j interleaved
    const double *az_cs;       // [2*n_az]: cos theta_i, sin theta_i interleaved
    uint32_t n_ch, n_az;
    uint32_t tiles_az;         // ceil(n_az / tile_az)
    uint32_t tiles_ch;         // ceil(n_ch / tile_ch)
    uint64_t ray_base;         // first padded ray index of this instance (batch)
    uint64_t out_base;         // output offset of beam 0
    float q[4];                // pose quaternion (w, x, y, z), unit
    float p[3];                // pose origin
    float wavelength_nm, d_max, r_l_max, t_min, sigma_i, t_trace;
    uint32_t noise_on;
    uint32_t seed_lo, seed_hi, scan, inst_id;
    // Columns traced by the launch.  A scan traces all n_az columns with one
    // pose.  A partial sweep (one engine tick) traces n_cols fired columns in
    // at most two runs: columns k < seg_n0 are azimuth seg_i0[0] + k of scan
    // `scan`, the rest azimuth seg_i0[1] + (k - seg_n0) of scan + 1; each
    // column takes the pose of its own firing time (sweep_pose).
    uint32_t sweep;            // 0 for a scan
    uint32_t n_cols;
    uint32_t seg_n0;
    uint32_t seg_i0[2];
    SweepDev sw;
};

// ---------------------------------------------------------------------------
// Dynamic scenes: meshes (own BVH over object-space triangles) placed in the
// world by actors, and a top-level BVH over the actors' world boxes whose
// leaf records carry the actor index in a.w.
// ---------------------------------------------------------------------------
struct ActorDev {
    double R[9];               // world <- object rotation, row-major
    double p[3];               // world position of the object origin
    uint32_t mesh;             // index into the mesh table
    uint32_t label;            // instance label of all its triangles
    uint32_t tri_base;         // index of its first triangle in the combined ordering
    uint32_t pad_;
};

struct MeshDev {
    const Node4 *nodes;
    const TriRec *tris;
    uint32_t max_steps;
    uint32_t n_tri;
};

struct ActorsDev {
    const Node4 *nodes;        // top-level BVH (root 0)
    const TriRec *recs;        // its leaf records: a.w = actor index
    const ActorDev *actors;
    const MeshDev *meshes;
    uint32_t max_steps;
    uint32_t n_actors;
};

struct MaterialsDev {
    const float *spectra;      // [nmat][nbins]
    const float *sigma;        // [nmat]
    const float *angle_exp;    // [nmat]
    uint32_t nmat, nbins;
    float lambda0, dlambda;
};

struct Overrides {
    const float *rho;          // [nmat] or null
    const float *angle_exp;    // [nmat] or null
    const float *pose_delta;   // [6] or null
    const float *spectra;      // [nmat][nbins] or null (replaces the material table)
};

// R_lambda(0) of material m: the override, else the spectral table at the
// wavelength, interpolated linearly between bins and clamped at the ends.
__device__ inline float reflectance0(const Overrides &ov, const MaterialsDev &M, float wavelength_nm, uint32_t m) {
    if (ov.rho) return ov.rho[m];
    float q = (wavelength_nm - M.lambda0) / M.dlambda;
    const float *T = (ov.spectra ? ov.spectra : M.spectra) + (size_t)m * M.nbins;
    if (q <= 0.0f) return T[0];
    if (q >= (float)(M.nbins - 1)) return T[M.nbins - 1];
    int i0 = (int)floorf(q);
    float f = q - (float)i0;
    return fmaf(f, T[i0 + 1], (1.0f - f) * T[i0]);
}

struct Outputs {
    float *x, *y, *z, *intensity;
    uint32_t *label;
    uint8_t *valid;
    float *range;
    uint32_t *tri;
    float *t_hit;
    uint16_t *material;
    float *normal;
    float *r_lambda;
    uint64_t plane;            // element stride between the normal's planes
};

// ---------------------------------------------------------------------------
// Pose: rotation matrix in FP64 from the unit quaternion, optionally
// left-multiplied by Exp(dw) (Rodrigues), origin p + dp.
// ---------------------------------------------------------------------------
struct Pose64 {
    double R[9];
    double p[3];
};

__device__ inline void quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ inline void so3_exp(const double w[3], double E[9]) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double a, b;  // E = I + a K + b K^2
    if (th < 1e-12) { a = 1.0; b = 0.5; }
    else { a = sin(th) / th; b = (1.0 - cos(th)) / th2; }
    double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double k2 = K[r * 3 + 0] * K[0 * 3 + c] + K[r * 3 + 1] * K[1 * 3 + c] + K[r * 3 + 2] * K[2 * 3 + c];
            E[r * 3 + c] = (r == c ? 1.0 : 0.0) + a * K[r * 3 + c] + b * k2;
        }
}

__device__ inline Pose64 make_pose(const InstanceDev &in, const float *pose_delta) {
    Pose64 P;
    const double q[4] = {in.q[0], in.q[1], in.q[2], in.q[3]};
    quat_to_rot(q, P.R);
    P.p[0] = in.p[0]; P.p[1] = in.p[1]; P.p[2] = in.p[2];
    if (pose_delta) {
        double w[3] = {pose_delta[3], pose_delta[4], pose_delta[5]};
        double E[9], R0[9];
        so3_exp(w, E);
        for (int i = 0; i < 9; ++i) R0[i] = P.R[i];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                P.R[r * 3 + c] = E[r * 3 + 0] * R0[0 * 3 + c] + E[r * 3 + 1] * R0[1 * 3 + c] + E[r * 3 + 2] * R0[2 * 3 + c];
        P.p[0] += pose_delta[0]; P.p[1] += pose_delta[1]; P.p[2] += pose_delta[2];
    }
    return P;
}

// Column k of a launch -> azimuth index, and the scan it belongs to.
__device__ inline uint32_t column_azimuth(const InstanceDev &in, uint32_t k, uint32_t &scan) {
    if (k < in.seg_n0) {
        scan = in.scan;
        return in.seg_i0[0] + k;
    }
    scan = in.scan + 1u;
    return in.seg_i0[1] + (k - in.seg_n0);
}

// Pose of column (scan s, azimuth i) of a partial sweep.  The column fires
// when the head reaches A = 360 s + az0 + i step, at the fraction
// tau = (A - a) / (b - a) of the tick.  The position moves linearly, the
// orientation along the great arc between the two quaternions (slerp,
// Shoemake 1985), or along the chord below an arc of 1e-6 rad, so that equal
// end poses give exactly the scan pose.
__device__ inline Pose64 sweep_pose(const SweepDev &S, uint32_t s, uint32_t i) {
    const double ang = 360.0 * (double)s + (S.az0 + (double)i * S.step);
    const double tau = (ang - S.a) / (S.b - S.a);
    double q[4];
    if (S.chord) {
        for (int e = 0; e < 4; ++e) q[e] = S.qa[e] + tau * (S.qb[e] - S.qa[e]);
    } else {
        const double ca = sin((1.0 - tau) * S.w) * S.inv_sin_w, cb = sin(tau * S.w) * S.inv_sin_w;
        for (int e = 0; e < 4; ++e) q[e] = ca * S.ua[e] + cb * S.ub[e];
    }
    Pose64 P;
    quat_to_rot(q, P.R);
    for (int e = 0; e < 3; ++e) P.p[e] = (double)S.pa[e] + tau * ((double)S.pb[e] - (double)S.pa[e]);
    return P;
}

// Pose of column k: the scan pose (with the calibration delta), or the
// per-column pose of a partial sweep.
__device__ inline Pose64 column_pose(const InstanceDev &in, const float *pose_delta, uint32_t k) {
    if (!in.sweep) return make_pose(in, pose_delta);
    uint32_t s;
    const uint32_t i = column_azimuth(in, k, s);
    return sweep_pose(in.sw, s, i);
}

// Beam (j, i) -> sensor-frame direction s (FP64 then rounded once) and world
// ray (origin rounded once, direction R s rounded once).
struct Ray {
    float ox, oy, oz;
    float dx, dy, dz;
    float sx, sy, sz;          // sensor-frame unit direction (for the output point)
};

__device__ inline Ray make_ray(const InstanceDev &in, const Pose64 &P, uint32_t j, uint32_t i) {
    double cp = in.elev_cs[2 * j], sp = in.elev_cs[2 * j + 1];
    double ct = in.az_cs[2 * i], st = in.az_cs[2 * i + 1];
    double s0 = cp * ct, s1 = cp * st, s2 = sp;
    Ray r;
    r.sx = (float)s0; r.sy = (float)s1; r.sz = (float)s2;
    r.dx = (float)(P.R[0] * s0 + P.R[1] * s1 + P.R[2] * s2);
    r.dy = (float)(P.R[3] * s0 + P.R[4] * s1 + P.R[5] * s2);
    r.dz = (float)(P.R[6] * s0 + P.R[7] * s1 + P.R[8] * s2);
    r.ox = (float)P.p[0]; r.oy = (float)P.p[1]; r.oz = (float)P.p[2];
    return r;
}

// The object-space ray of an actor: o' = R^T (o - p), d' = R^T d in FP64,
// rounded once.  R is a rotation, so the ray parameter t is the same in both
// spaces.
__device__ inline Ray object_ray(const ActorDev &A, const Ray &w) {
    const double ox = (double)w.ox - A.p[0], oy = (double)w.oy - A.p[1], oz = (double)w.oz - A.p[2];
    const double dx = w.dx, dy = w.dy, dz = w.dz;
    Ray r;
    r.ox = (float)(A.R[0] * ox + A.R[3] * oy + A.R[6] * oz);
    r.oy = (float)(A.R[1] * ox + A.R[4] * oy + A.R[7] * oz);
    r.oz = (float)(A.R[2] * ox + A.R[5] * oy + A.R[8] * oz);
    r.dx = (float)(A.R[0] * dx + A.R[3] * dy + A.R[6] * dz);
    r.dy = (float)(A.R[1] * dx + A.R[4] * dy + A.R[7] * dz);
    r.dz = (float)(A.R[2] * dx + A.R[5] * dy + A.R[8] * dz);
    r.sx = w.sx; r.sy = w.sy; r.sz = w.sz;
    return r;
}

// ---------------------------------------------------------------------------
// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), two-sided.
// The ray is sheared so that it becomes the +z axis; the three 2-D edge
// functions decide the hit, with an FP64 re-evaluation when one is exactly 0.
// ---------------------------------------------------------------------------
struct RayTri {
    float ox, oy, oz;
    int kx, ky, kz;
    float Sx, Sy, Sz;
};

__device__ inline float pick(float x, float y, float z, int k) {
    return k == 0 ? x : (k == 1 ? y : z);
}

// component K (0, 1, 2) if known at compile time, else component k
template <int K>
__device__ inline float pick_c(float x, float y, float z, int k) {
    if constexpr (K < 0) return pick(x, y, z, k);
    else return K == 0 ? x : (K == 1 ? y : z);
}

__device__ inline RayTri prep_tri_test(const Ray &r) {
    RayTri R;
    R.ox = r.ox; R.oy = r.oy; R.oz = r.oz;
    float ax = fabsf(r.dx), ay = fabsf(r.dy), az = fabsf(r.dz);
    int kz = (ax > ay) ? ((ax > az) ? 0 : 2) : ((ay > az) ? 1 : 2);
    int kx = kz + 1; if (kx == 3) kx = 0;
    int ky = kx + 1; if (ky == 3) ky = 0;
    float dkz = pick(r.dx, r.dy, r.dz, kz);
    if (dkz < 0.0f) { int t = kx; kx = ky; ky = t; }
    R.kx = kx; R.ky = ky; R.kz = kz;
    R.Sx = pick(r.dx, r.dy, r.dz, kx) / dkz;
    R.Sy = pick(r.dx, r.dy, r.dz, ky) / dkz;
    R.Sz = 1.0f / dkz;
    return R;
}

// Returns true and the distance t if the ray hits the triangle with
// t_lo < t; the caller compares t with its current best.  Apart from the rare
// FP64 recomputation of an edge function that rounds to zero, the test runs
// without branches (a wavefront tests its lanes' triangles together, so early
// exits would only add exec-mask work).
// KX, KY, KZ >= 0: the caller guarantees R.kx == KX etc. (a wavefront whose
// beams share the axis permutation), and the component selections are fixed.
template <int KX = -1, int KY = -1, int KZ = -1>
__device__ inline bool tri_hit(const RayTri &R, float4 a, float4 b, float4 c, float t_lo, float &t_out) {
    float Ax0 = a.x - R.ox, Ay0 = a.y - R.oy, Az0 = a.z - R.oz;
    float Bx0 = b.x - R.ox, By0 = b.y - R.oy, Bz0 = b.z - R.oz;
    float Cx0 = c.x - R.ox, Cy0 = c.y - R.oy, Cz0 = c.z - R.oz;
    float Akx = pick_c<KX>(Ax0, Ay0, Az0, R.kx), Aky = pick_c<KY>(Ax0, Ay0, Az0, R.ky);
    float Akz = pick_c<KZ>(Ax0, Ay0, Az0, R.kz);
    float Bkx = pick_c<KX>(Bx0, By0, Bz0, R.kx), Bky = pick_c<KY>(Bx0, By0, Bz0, R.ky);
    float Bkz = pick_c<KZ>(Bx0, By0, Bz0, R.kz);
    float Ckx = pick_c<KX>(Cx0, Cy0, Cz0, R.kx), Cky = pick_c<KY>(Cx0, Cy0, Cz0, R.ky);
    float Ckz = pick_c<KZ>(Cx0, Cy0, Cz0, R.kz);
    float Ax = fmaf(-R.Sx, Akz, Akx), Ay = fmaf(-R.Sy, Akz, Aky);
    float Bx = fmaf(-R.Sx, Bkz, Bkx), By = fmaf(-R.Sy, Bkz, Bky);
    float Cx = fmaf(-R.Sx, Ckz, Ckx), Cy = fmaf(-R.Sy, Ckz, Cky);
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    const bool outside = (U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f);
    const float det = U + V + W;
    const float Az = R.Sz * Akz, Bz = R.Sz * Bkz, Cz = R.Sz * Ckz;
    const float T = U * Az + V * Bz + W * Cz;
    const float t = __fdiv_rn(T, det);
    t_out = t;
    return !outside && det != 0.0f && t > t_lo;
}

// ---------------------------------------------------------------------------
// Ray / 4 boxes slab test.  Boxes are padded outward at build time by more
// than the triangle test's rounding error, so a triangle the test above
// accepts at t is never culled by a box whose computed entry exceeds t.
// ---------------------------------------------------------------------------
struct RayBox {
    float ix, iy, iz;          // 1/d (zero components replaced by +-1e-20)
    float nox, noy, noz;       // -o/d
};

__device__ inline RayBox prep_box_test(const Ray &r) {
    RayBox B;
    float dx = fabsf(r.dx) < 1e-20f ? copysignf(1e-20f, r.dx) : r.dx;
    float dy = fabsf(r.dy) < 1e-20f ? copysignf(1e-20f, r.dy) : r.dy;
    float dz = fabsf(r.dz) < 1e-20f ? copysignf(1e-20f, r.dz) : r.dz;
    B.ix = 1.0f / dx; B.iy = 1.0f / dy; B.iz = 1.0f / dz;
    B.nox = -r.ox * B.ix; B.noy = -r.oy * B.iy; B.noz = -r.oz * B.iz;
    return B;
}

// ---------------------------------------------------------------------------
// Buffer fetches of nodes and triangle records: a buffer resource (base in
// SGPRs) plus a 32-bit byte offset per lane, instead of a 64-bit address per
// lane.  Raw buffer, 32-bit data format; the range is not used for clamping
// (every offset the traversal forms is inside the array).
// ---------------------------------------------------------------------------
typedef int lidar_v4i __attribute__((ext_vector_type(4)));
typedef int lidar_v3i __attribute__((ext_vector_type(3)));

__device__ inline __amdgpu_buffer_rsrc_t raw_buffer(const void *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, 0x7FFFFFFF, 0x00020000);
}
__device__ inline float4 buf_load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const lidar_v4i v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z), __int_as_float(v.w));
}
__device__ inline float4 buf_load3(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const lidar_v3i v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)off, 0, 0);
    return make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z), 0.0f);
}

// ---------------------------------------------------------------------------
// Quad (4-lane) exchanges through DPP quad_perm
// ---------------------------------------------------------------------------
// value of lane (lane ^ 1) / (lane ^ 2) / (lane ^ 3) within the quad
__device__ inline uint32_t quad_xor1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
}
__device__ inline uint32_t quad_xor2(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
}
__device__ inline uint32_t quad_xor3(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x1B, 0xF, 0xF, true);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
// ---------------------------------------------------------------------------
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Standard normal from two words: u1 = (xa + 1) 2^-32, u2 = xb 2^-32,
// z = sqrt(-2 ln u1) cos(2 pi u2).  Evaluated with the hardware base-2
// logarithm and the hardware cosine, whose argument is in revolutions, so
// cos(2 pi u2) needs no range reduction; no branch, so a wavefront does not
// run two logarithms.  Near u1 = 1 the logarithm loses relative accuracy, but
// there z itself is near 0: the absolute error of z stays far below what a
// range noise of centimetres can show.
__device__ inline float box_muller(uint32_t xa, uint32_t xb) {
    const float u1 = (float)xa * 2.3283064365386963e-10f + 2.3283064365386963e-10f;   // in (0, 1]
    const float lnu = __builtin_amdgcn_logf(u1) * 0.69314718055994531f;
    const float u2 = (float)xb * 2.3283064365386963e-10f;
    return __builtin_sqrtf(-2.0f * lnu) * __builtin_amdgcn_cosf(u2);
}

}  // namespace lidar
