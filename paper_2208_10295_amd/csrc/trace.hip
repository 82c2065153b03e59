// trace.hip -- first-hit query and return model for every beam (gfx950).
//
// Three traversal shapes share one intersection test and one epilogue:
//   * lane-per-ray: one lane walks the 4-wide BVH for its beam and tests the
//     four child boxes itself;
//   * quad-per-ray: the four lanes of a DPP quad share a beam; lane s tests
//     child box s (one 128-byte node line per quad) or triangles s, s+4 of a
//     leaf, and the quad agrees on the traversal order through quad_perm
//     exchanges.  This gives 4x the wavefronts for the same beams, which a
//     single 131k-beam scan needs to hide the latency of dependent node
//     fetches;
//   * pair-per-ray: two lanes, two child boxes each (the batched form, which
//     has parallelism to spare, prefers its fewer instructions per beam).
// All return bit-identical hits.  The walks keep their stack in LDS without
// branches (push_level) and, where a wavefront's beams share the signs of
// their direction components, run a copy of the loop whose box test takes
// the near planes by sign (slab_t).
//
// Beams are grouped in 64-beam tiles of tile_ch channels x tile_az azimuth
// steps, numbered column-major (all channel rows of an azimuth column, then
// the next column).  With the XCD remap, blockIdx b runs logical block
// (b % 8) * (nb / 8) + b / 8, so the blocks that the hardware places on one
// XCD (b % 8 equal) cover one contiguous azimuth sector and share that XCD's
// L2.
//
// Return model, per beam (paper Sections II-A to II-D):
//   cos(theta) = |n . d| with n the hit triangle's unit normal (II-C),
//   R_lambda = R_lambda(0) cos^k(theta) (eq.4 for k = 1), R_lambda(0) the
//   material's spectral reflectance interpolated at the sensor wavelength,
//   d = t + sigma_m z (Gaussian range noise, II-A),
//   detected iff t_min < d <= d_max and R_L,max / d_max * d <= R_lambda (eq.5),
//   intensity = max(0, R_lambda + sigma_I z_I).
#include "lidar_device.hpp"
#include "lidar_kernels.hpp"

namespace lidar {

// Waves per SIMD to ask of the register allocator: `want`, or fewer when the
// block's LDS (160 KB per CU, four SIMDs) cannot hold that many blocks.  Asking
// for more than LDS allows would cap the VGPRs for occupancy never reached.
// Rounded up: 11 blocks of two waves put 6 waves on two SIMDs and 5 on two.
// Stack entries per beam beyond the capacity of a walk: its bottom entry and
// the scratch stores of the node steps (see push_level).
constexpr int kStackPad = 5;

constexpr int lds_waves(int want, int lds_bytes, int block) {
    int w = ((160 * 1024 / lds_bytes) * (block / 64) + 3) / 4;
    w = w < 1 ? 1 : w;
    return want < w ? want : w;
}

// ---------------------------------------------------------------------------
// FP64 direction tables from data-sheet angles (degrees)
// ---------------------------------------------------------------------------
__global__ void dir_tables_kernel(const double *__restrict__ elev_deg, uint32_t n_ch, double az0_deg,
                                  double fov_h_deg, uint32_t n_az, double *__restrict__ elev_cs,
                                  double *__restrict__ az_cs) {
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const double deg = 3.14159265358979323846 / 180.0;
    if (g < n_ch) {
        double a = elev_deg[g] * deg;
        elev_cs[2 * g] = cos(a);
        elev_cs[2 * g + 1] = sin(a);
    }
    if (g < n_az) {
        double a = (az0_deg + (double)g * (fov_h_deg / (double)n_az)) * deg;
        az_cs[2 * g] = cos(a);
        az_cs[2 * g + 1] = sin(a);
    }
}

void launch_dir_tables(const double *elev_deg, uint32_t n_ch, double az0_deg, double fov_h_deg,
                       uint32_t n_az, double *elev_cs, double *az_cs, hipStream_t s) {
    uint32_t n = n_ch > n_az ? n_ch : n_az;
    dir_tables_kernel<<<(n + 255) / 256, 256, 0, s>>>(elev_deg, n_ch, az0_deg, fov_h_deg, n_az, elev_cs, az_cs);
}

// ---------------------------------------------------------------------------
// common pieces
// ---------------------------------------------------------------------------
struct Hit {
    uint32_t slot;     // triangle record index, kNone if no hit
    uint32_t orig;     // original triangle index (actors: in the combined ordering)
    float t;
    uint32_t actor;    // kNone: static scene; else the actor whose mesh holds the record
};

struct Counts {
    uint32_t nodes, tris;
};

// (t, orig) < (bt, bo) lexicographically; non-short-circuit, so it compiles
// to compares and selects rather than branches
__device__ inline bool better(float t, uint32_t orig, float bt, uint32_t bo) {
    return (t < bt) | ((t == bt) & (orig < bo));
}

__device__ inline void csort(float &ka, uint32_t &va, float &kb, uint32_t &vb) {
    bool sw = kb < ka;
    float tk = sw ? kb : ka; kb = sw ? ka : kb; ka = tk;
    uint32_t tv = sw ? vb : va; vb = sw ? va : vb; va = tv;
}

// Entry distance of the ray into a child box, +inf if missed.  The clamps to
// [t_lo, tmax_lim] are integer max / min of the bit patterns: with t_lo >= +0
// and tmax_lim > 0 these order like the float values (a negative distance is
// a negative integer), and unlike float min / max they need no
// canonicalisation of the two loop-carried bounds on every step.
__device__ inline float slab(const RayBox &B, float4 lo, float4 hi, float t_lo, float tmax_lim) {
    float x0 = fmaf(lo.x, B.ix, B.nox), x1 = fmaf(hi.x, B.ix, B.nox);
    float y0 = fmaf(lo.y, B.iy, B.noy), y1 = fmaf(hi.y, B.iy, B.noy);
    float z0 = fmaf(lo.z, B.iz, B.noz), z1 = fmaf(hi.z, B.iz, B.noz);
    const float n3 = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fminf(z0, z1));
    const float f3 = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fmaxf(z0, z1));
    const int tn = max(__float_as_int(n3), __float_as_int(t_lo));
    const int tf = min(__float_as_int(f3), __float_as_int(tmax_lim));
    return tn <= tf ? __int_as_float(tn) : __builtin_inff();
}

// Walk modes.  A wavefront whose beams share the signs of their direction
// components (bits 0..2: component a of 1/d negative) and the dominant axis kz
// of the triangle test (bit 3: 0 = x, 1 = y) runs mode 0..15; a wavefront with
// kz = z (beams steeper than 45 degrees) or with mixed signs or axes runs
// kGeneralMode.
constexpr int kGeneralMode = 16;
constexpr int mode_kz(int m) { return m >> 3; }
constexpr bool mode_neg(int m, int axis) { return ((m >> axis) & 1) != 0; }
// the triangle test's axis permutation in mode m (as prep_tri_test: kx, ky
// follow kz cyclically and swap when the dominant component is negative)
constexpr int mode_kx(int m) { return mode_neg(m, mode_kz(m)) ? (mode_kz(m) + 2) % 3 : (mode_kz(m) + 1) % 3; }
constexpr int mode_ky(int m) { return mode_neg(m, mode_kz(m)) ? (mode_kz(m) + 1) % 3 : (mode_kz(m) + 2) % 3; }

// The box test in mode MODE.  The near plane of each slab is lo or hi by the
// sign alone, and since fma is monotonic in its first argument the near and
// far distances are the values the min / max above select: the keys are
// bit-identical, at 5 fewer instructions per box.
template <int MODE>
__device__ inline float slab_t(const RayBox &B, float4 lo, float4 hi, float t_lo, float tmax_lim) {
    if constexpr (MODE == kGeneralMode) {
        return slab(B, lo, hi, t_lo, tmax_lim);
    } else {
        const float nx = fmaf((MODE & 1) ? hi.x : lo.x, B.ix, B.nox), fx = fmaf((MODE & 1) ? lo.x : hi.x, B.ix, B.nox);
        const float ny = fmaf((MODE & 2) ? hi.y : lo.y, B.iy, B.noy), fy = fmaf((MODE & 2) ? lo.y : hi.y, B.iy, B.noy);
        const float nz = fmaf((MODE & 4) ? hi.z : lo.z, B.iz, B.noz), fz = fmaf((MODE & 4) ? lo.z : hi.z, B.iz, B.noz);
        const int tn = max(__float_as_int(fmaxf(fmaxf(nx, ny), nz)), __float_as_int(t_lo));
        const int tf = min(__float_as_int(fminf(fminf(fx, fy), fz)), __float_as_int(tmax_lim));
        return tn <= tf ? __int_as_float(tn) : __builtin_inff();
    }
}

// The mode of a wavefront's walk (wavefront-uniform).
__device__ inline int walk_mode(const RayBox &B, const RayTri &T) {
    int m = (int)((__float_as_uint(B.ix) >> 31) | ((__float_as_uint(B.iy) >> 31) << 1) |
                  ((__float_as_uint(B.iz) >> 31) << 2));
    m = T.kz < 2 ? m | (T.kz << 3) : kGeneralMode;
    const int m0 = __builtin_amdgcn_readfirstlane(m);
    return (__ballot(m != m0) == 0 && m0 != kGeneralMode) ? m0 : kGeneralMode;
}

// Orders the four children nearest first; returns whether any was hit.  The
// caller pushes c3, c2, c1 (those hit) and descends into c0.
__device__ inline void sort4(float &k0, uint32_t &c0, float &k1, uint32_t &c1, float &k2, uint32_t &c2, float &k3,
                             uint32_t &c3) {
    csort(k0, c0, k1, c1);
    csort(k2, c2, k3, c3);
    csort(k0, c0, k2, c2);
    csort(k1, c1, k3, c3);
    csort(k1, c1, k2, c2);
}

// Bound on the box exit distance: a hair above the current best hit so that
// a box whose computed entry equals the best distance is still opened (a tie
// with a smaller original index may be inside).
__device__ inline float box_limit(float best_t) { return best_t * 1.0000005f; }

// Traversal stack without branches.  A node step ranks the node's four
// children near to far (rank 0..3, a permutation) and finds h + 1 of them hit.
// The child of rank r is stored at entry sp + ((h - r) mod 4): ranks 1..h land
// in entries sp + h - 1 .. sp (nearest on top), the nearest child and the
// missed ones in entries sp + h .. sp + 3, above the new top, where they are
// never read.  The step leaves sp + h entries (h = -1 when every child was
// missed: the entry to pop next is then the top one).  A node that would push
// the stack past `lim` entries clamps it there (children are lost); `peak`
// records sp + h, and peak > lim after the walk marks the beam as overflowed.
// Stores reach entry lim + 3, hence kStackPad.
__device__ inline int push_level(int sp, int nh, int rank) { return sp + ((nh - rank) & 3); }

__device__ inline int push_clamp(int sp, int nh, int lim, int &peak) {
    const int top = sp + nh;
    peak = top > peak ? top : peak;
    return min(top, lim);
}

// ---------------------------------------------------------------------------
// lane-per-ray traversal
// ---------------------------------------------------------------------------
// max_steps bounds the loop: a correct traversal visits every node and leaf
// at most once, so exceeding it means a corrupt tree (flagged, never looped).
template <int STACK, int NSLOT, bool COUNT>
__device__ inline Hit traverse(const Node4 *__restrict__ nodes, const TriRec *__restrict__ tris, uint32_t root,
                               uint32_t max_steps, const Ray &ray, float t_lo, float t_hi,
                               uint32_t *__restrict__ stk, bool &overflow, Counts &cnt, int cap = STACK) {
    const __amdgpu_buffer_rsrc_t nbuf = raw_buffer(nodes), tbuf = raw_buffer(tris);
    const RayBox B = prep_box_test(ray);
    const RayTri T = prep_tri_test(ray);
    const float inf = __builtin_inff();
    Hit h{kNone, kNone, t_hi, kNone};
    float lim = box_limit(h.t);
    // Same stack discipline as the multi-lane walk below: entry 0 holds
    // kEmptyRef, the sorted children of rank 1..3 are stored without branches
    // at push_level, and the entry a pop returns is read ahead.
    uint32_t ref = root;
    stk[0] = kEmptyRef;
    int sp = 1, peak = 0;
    uint32_t steps = 0;
    for (; ref != kEmptyRef && steps <= max_steps; ++steps) {
        const uint32_t top = stk[(sp - 1) * NSLOT];
        uint32_t nxt = kEmptyRef;
        if (ref & kLeafBit) {
            uint32_t first = leaf_first(ref), n = leaf_count(ref);
            if (COUNT) cnt.tris += n;
            for (uint32_t k = 0; k < n; ++k) {
                const uint32_t off = (first + k) * (uint32_t)sizeof(TriRec);
                const float4 a = buf_load4(tbuf, off), b = buf_load3(tbuf, off + 16u), c = buf_load3(tbuf, off + 32u);
                float t;
                const uint32_t orig = __float_as_uint(a.w);
                const bool hit = tri_hit(T, a, b, c, t_lo, t);
                const bool take = hit && better(t, orig, h.t, h.orig);
                h.t = take ? t : h.t;
                h.orig = take ? orig : h.orig;
                h.slot = take ? first + k : h.slot;
            }
            lim = box_limit(h.t);
            --sp;
        } else {
            if (COUNT) cnt.nodes += 1;
            const uint32_t off = ref * (uint32_t)sizeof(Node4);
            const float4 a0 = buf_load4(nbuf, off), b0 = buf_load4(nbuf, off + 16u);
            const float4 a1 = buf_load4(nbuf, off + 32u), b1 = buf_load4(nbuf, off + 48u);
            const float4 a2 = buf_load4(nbuf, off + 64u), b2 = buf_load4(nbuf, off + 80u);
            const float4 a3 = buf_load4(nbuf, off + 96u), b3 = buf_load4(nbuf, off + 112u);
            float k0 = slab(B, a0, b0, t_lo, lim), k1 = slab(B, a1, b1, t_lo, lim);
            float k2 = slab(B, a2, b2, t_lo, lim), k3 = slab(B, a3, b3, t_lo, lim);
            uint32_t c0 = __float_as_uint(a0.w), c1 = __float_as_uint(a1.w), c2 = __float_as_uint(a2.w),
                     c3 = __float_as_uint(a3.w);
            sort4(k0, c0, k1, c1, k2, c2, k3, c3);
            const int nh = (int)(k0 != inf) + (int)(k1 != inf) + (int)(k2 != inf) + (int)(k3 != inf) - 1;
            stk[push_level(sp, nh, 1) * NSLOT] = c1;
            stk[push_level(sp, nh, 2) * NSLOT] = c2;
            stk[push_level(sp, nh, 3) * NSLOT] = c3;
            sp = push_clamp(sp, nh, cap + 1, peak);
            nxt = nh >= 0 ? c0 : kEmptyRef;
        }
        ref = nxt == kEmptyRef ? top : nxt;
    }
    if (steps > max_steps || peak > cap + 1) overflow = true;
    return h;
}

// ---------------------------------------------------------------------------
// multi-lane traversal: LANES (2 or 4) adjacent lanes of one DPP quad share a
// beam; lane s = lane % LANES tests child boxes s * 4 / LANES .. (one 32-byte
// slot each, so the lanes of a beam read one 128-byte node line together) and
// the triangles s, s + LANES, ... of a leaf.
//
// Quad (LANES = 4) node step: lane s holds the entry distance of child s.  The
// distance bits (positive floats and +inf order like unsigned integers), with
// the two low mantissa bits replaced by s, form a key unique within the quad;
// each lane counts the smaller keys of its three partners (quad_perm xor 1, 2,
// 3) to get its child's rank in near-to-far order.  The rank-0 child is
// descended into (its reference is OR-reduced over the quad), and the lane of
// the child of rank r >= 1 that was hit pushes its own reference to stack entry
// sp + h - r (h further children hit), so the nearest of them is popped first.
// Pair (LANES = 2): each lane tests two children and ranks its two keys the
// same way against the other three (pair_node_step).
//
// Leaves: each lane keeps the lexicographic (t, original index) minimum of the
// triangles it tested; after a leaf the lanes only agree on the smallest t (the
// culling bound), and the full minimum is reduced over the lanes once, at the
// end.  Culling uses the same bound as a per-leaf reduction would, so the same
// nodes are visited and the result is the same.
// ---------------------------------------------------------------------------
// Smallest t over the beam's lanes.  Distances are positive, so their bit
// patterns order like unsigned integers (no float canonicalisation needed).
template <int LANES>
__device__ inline float group_min_t(float t) {
    uint32_t u = __float_as_uint(t);
    u = min(u, quad_xor1(u));
    if (LANES == 4) u = min(u, quad_xor2(u));
    return __uint_as_float(u);
}

// One quad node step (see above): returns the nearest child hit by the beam,
// or kEmptyRef if it hits none, and pushes the further children hit; each
// lane stores its own child (push_level).
template <int NSLOT, int MODE = kGeneralMode>
__device__ inline uint32_t quad_node_step(__amdgpu_buffer_rsrc_t nodes, uint32_t ref, const RayBox &B, float t_lo,
                                          float lim, uint32_t s, uint32_t *__restrict__ stk, int &sp, int cap,
                                          int &peak) {
    const uint32_t off = ref * (uint32_t)sizeof(Node4) + s * 32u;   // child slot s of node ref
    const float4 a = buf_load4(nodes, off), b = buf_load4(nodes, off + 16u);
    const float key = slab_t<MODE>(B, a, b, t_lo, lim);
    const uint32_t cref = __float_as_uint(a.w);
    const uint32_t kk = (__float_as_uint(key) & ~3u) | s;
    // keys are below 2^31 (non-negative floats), so partner < kk is the sign of partner - kk
    const int rank = (int)(((quad_xor1(kk) - kk) >> 31) + ((quad_xor2(kk) - kk) >> 31) + ((quad_xor3(kk) - kk) >> 31));
    // children hit by the beam: the finite keys of its quad
    const uint64_t fin = __ballot(kk < 0x7F800000u);
    const int nh = __popc((uint32_t)(fin >> (threadIdx.x & 60u)) & 0xFu) - 1;
    // the rank-0 child, or kEmptyRef if even that one was missed
    uint32_t nxt = rank == 0 ? (kk < 0x7F800000u ? cref : kEmptyRef) : 0u;
    nxt |= quad_xor1(nxt);
    nxt |= quad_xor2(nxt);
    stk[push_level(sp, nh, rank) * NSLOT] = cref;
    sp = push_clamp(sp, nh, cap, peak);
    return nxt;
}

// One pair node step: lane s (0 or 1) of the beam's pair tests children 2s and
// 2s + 1 and ranks its two keys against the other three (its own other key
// and the partner's two, through one quad_perm swap each); otherwise as the
// quad step.
template <int NSLOT, int MODE = kGeneralMode>
__device__ inline uint32_t pair_node_step(__amdgpu_buffer_rsrc_t nodes, uint32_t ref, const RayBox &B, float t_lo,
                                          float lim, uint32_t s, uint32_t *__restrict__ stk, int &sp, int cap,
                                          int &peak) {
    const uint32_t off = ref * (uint32_t)sizeof(Node4) + s * 64u;   // child slots 2s, 2s + 1
    const float4 a0 = buf_load4(nodes, off), b0 = buf_load4(nodes, off + 16u);
    const float4 a1 = buf_load4(nodes, off + 32u), b1 = buf_load4(nodes, off + 48u);
    const uint32_t ca = __float_as_uint(a0.w), cb = __float_as_uint(a1.w);
    const uint32_t ka = (__float_as_uint(slab_t<MODE>(B, a0, b0, t_lo, lim)) & ~3u) | (2u * s);
    const uint32_t kb = (__float_as_uint(slab_t<MODE>(B, a1, b1, t_lo, lim)) & ~3u) | (2u * s + 1u);
    const uint32_t pa = quad_xor1(ka), pb = quad_xor1(kb);
    const int ra = (int)(((kb - ka) >> 31) + ((pa - ka) >> 31) + ((pb - ka) >> 31));   // as in the quad step
    const int rb = (int)(((ka - kb) >> 31) + ((pa - kb) >> 31) + ((pb - kb) >> 31));
    constexpr uint32_t kInfKey = 0x7F800000u;
    const int nh = (int)(ka < kInfKey) + (int)(kb < kInfKey) + (int)(pa < kInfKey) + (int)(pb < kInfKey) - 1;
    uint32_t nxt = (ra == 0 ? (ka < kInfKey ? ca : kEmptyRef) : 0u) | (rb == 0 ? (kb < kInfKey ? cb : kEmptyRef) : 0u);
    nxt |= quad_xor1(nxt);
    stk[push_level(sp, nh, ra) * NSLOT] = ca;
    stk[push_level(sp, nh, rb) * NSLOT] = cb;
    sp = push_clamp(sp, nh, cap, peak);
    return nxt;
}

template <int LANES, int STACK, int NSLOT, bool COUNT, int MODE>
__device__ inline Hit traverse_multi_mode(const Node4 *__restrict__ nodes, const TriRec *__restrict__ tris,
                                          uint32_t root, uint32_t max_steps, const Ray &ray, float t_lo, float t_hi,
                                          uint32_t *__restrict__ stk, uint32_t s, bool &overflow, Counts &cnt,
                                          int cap) {
    static_assert(LANES == 2 || LANES == 4, "2 or 4 lanes per beam");
    const __amdgpu_buffer_rsrc_t nbuf = raw_buffer(nodes), tbuf = raw_buffer(tris);
    const RayBox B = prep_box_test(ray);
    const RayTri T = prep_tri_test(ray);
    Hit h{kNone, kNone, t_hi, kNone};   // this lane's best
    float best_t = t_hi;                // the beam's best distance (minimum over its lanes)
    float lim = box_limit(best_t);      // its box-culling bound, updated after each leaf
    // Entry 0 holds kEmptyRef: popping it ends the walk, so the loop has one
    // exit, also taken when the step budget runs out.  The step count is the
    // wavefront's, so running out marks every beam of the wavefront as
    // overflowed.  Entries 1 .. cap hold pushed children, and the scratch
    // stores of the node steps reach entry cap + 4: the stack has
    // cap + kStackPad entries.
    uint32_t ref = root;
    stk[0] = kEmptyRef;
    int sp = 1, peak = 0;
    uint32_t steps = 0;
    for (; ref != kEmptyRef && steps <= max_steps; ++steps) {
        // the entry a pop would return, read before the node fetch so that
        // its latency is hidden (a step that pops has pushed nothing)
        const uint32_t top = stk[(sp - 1) * NSLOT];
        uint32_t nxt = kEmptyRef;
        if (ref & kLeafBit) {
            uint32_t first = leaf_first(ref), n = leaf_count(ref);
            if (COUNT) cnt.tris += n;
            for (uint32_t k = s; k < n; k += LANES) {
                const uint32_t off = (first + k) * (uint32_t)sizeof(TriRec);
                const float4 a = buf_load4(tbuf, off), b = buf_load3(tbuf, off + 16u), c = buf_load3(tbuf, off + 32u);
                float t;
                const uint32_t orig = __float_as_uint(a.w);
                bool hit;
                if constexpr (MODE == kGeneralMode) hit = tri_hit(T, a, b, c, t_lo, t);
                else hit = tri_hit<mode_kx(MODE), mode_ky(MODE), mode_kz(MODE)>(T, a, b, c, t_lo, t);
                const bool take = hit && better(t, orig, h.t, h.orig);
                h.t = take ? t : h.t;
                h.orig = take ? orig : h.orig;
                h.slot = take ? first + k : h.slot;
            }
            best_t = group_min_t<LANES>(h.t);
            lim = box_limit(best_t);
            --sp;
        } else {
            if (COUNT) cnt.nodes += 1;
            nxt = LANES == 4 ? quad_node_step<NSLOT, MODE>(nbuf, ref, B, t_lo, lim, s, stk, sp, cap + 1, peak)
                             : pair_node_step<NSLOT, MODE>(nbuf, ref, B, t_lo, lim, s, stk, sp, cap + 1, peak);
        }
        ref = nxt == kEmptyRef ? top : nxt;
    }
    if (steps > max_steps || peak > cap + 1) overflow = true;
    // lexicographic (t, original index) minimum over the beam's lanes
    {
        float ot = __uint_as_float(quad_xor1(__float_as_uint(h.t)));
        uint32_t oo = quad_xor1(h.orig), os = quad_xor1(h.slot);
        if (better(ot, oo, h.t, h.orig)) { h.t = ot; h.orig = oo; h.slot = os; }
        if (LANES == 4) {
            ot = __uint_as_float(quad_xor2(__float_as_uint(h.t)));
            oo = quad_xor2(h.orig);
            os = quad_xor2(h.slot);
            if (better(ot, oo, h.t, h.orig)) { h.t = ot; h.orig = oo; h.slot = os; }
        }
    }
    return h;
}

// The walk specialised for the wavefront's mode when SPECIALISE (one copy of
// the loop per mode: box test by direction signs, triangle test with a fixed
// axis permutation; chosen once per walk), else the general loop.
template <int LANES, int STACK, int NSLOT, bool COUNT, bool SPECIALISE = false>
__device__ inline Hit traverse_multi(const Node4 *__restrict__ nodes, const TriRec *__restrict__ tris,
                                     uint32_t root, uint32_t max_steps, const Ray &ray, float t_lo, float t_hi,
                                     uint32_t *__restrict__ stk, uint32_t s, bool &overflow, Counts &cnt,
                                     int cap = STACK) {
#define LIDAR_WALK(M) traverse_multi_mode<LANES, STACK, NSLOT, COUNT, M>(nodes, tris, root, max_steps, ray, t_lo, \
                                                                        t_hi, stk, s, overflow, cnt, cap)
    if constexpr (SPECIALISE) {
        switch (walk_mode(prep_box_test(ray), prep_tri_test(ray))) {
        case 0: return LIDAR_WALK(0);
        case 1: return LIDAR_WALK(1);
        case 2: return LIDAR_WALK(2);
        case 3: return LIDAR_WALK(3);
        case 4: return LIDAR_WALK(4);
        case 5: return LIDAR_WALK(5);
        case 6: return LIDAR_WALK(6);
        case 7: return LIDAR_WALK(7);
        case 8: return LIDAR_WALK(8);
        case 9: return LIDAR_WALK(9);
        case 10: return LIDAR_WALK(10);
        case 11: return LIDAR_WALK(11);
        case 12: return LIDAR_WALK(12);
        case 13: return LIDAR_WALK(13);
        case 14: return LIDAR_WALK(14);
        case 15: return LIDAR_WALK(15);
        default: break;
        }
    }
    return LIDAR_WALK(kGeneralMode);
#undef LIDAR_WALK
}

// ---------------------------------------------------------------------------
// Dynamic scenes: the top-level BVH over the actors.  Its nodes are tested
// like any 4-wide node (LANES lanes per beam); at a leaf, each actor's ray is
// taken to object space and the actor's mesh BVH is walked with the stack
// entries above the top-level ones, with the best distance so far as its
// limit.  Candidates are compared by (t, index in the combined ordering), the
// static scene's triangles first, so ties resolve as in one flat soup.
// ---------------------------------------------------------------------------
template <int LANES, int STACK, int NSLOT>
__device__ inline void traverse_actors(const ActorsDev &A, const Ray &ray, float t_lo, Hit &h,
                                       uint32_t *__restrict__ stk, uint32_t s, bool &overflow) {
    const RayBox B = prep_box_test(ray);
    const float inf = __builtin_inff();
    Counts cnt{0u, 0u};
    uint32_t ref = 0;
    int sp = 0, peak = 0;
    uint32_t steps = 0;
    while (true) {
        if (++steps > A.max_steps) { overflow = true; break; }
        if (ref & kLeafBit) {
            const uint32_t first = leaf_first(ref), n = leaf_count(ref);
            for (uint32_t k = 0; k < n; ++k) {
                const uint32_t a = __float_as_uint(A.recs[first + k].a.w);
                const ActorDev &act = A.actors[a];
                const Ray ro = object_ray(act, ray);
                const MeshDev m = A.meshes[act.mesh];
                Hit hb;
                if constexpr (LANES == 1)
                    hb = traverse<STACK, NSLOT, false>(m.nodes, m.tris, 0u, m.max_steps, ro, t_lo, h.t,
                                                       stk + sp * NSLOT, overflow, cnt, STACK - sp);
                else
                    hb = traverse_multi<LANES, STACK, NSLOT, false>(m.nodes, m.tris, 0u, m.max_steps, ro, t_lo, h.t,
                                                                    stk + sp * NSLOT, s, overflow, cnt, STACK - sp);
                if (hb.slot != kNone) {
                    const uint32_t g = act.tri_base + hb.orig;
                    if (better(hb.t, g, h.t, h.orig)) { h.t = hb.t; h.orig = g; h.slot = hb.slot; h.actor = a; }
                }
            }
            --sp;
        } else if constexpr (LANES == 4) {    // a miss leaves sp one lower (see quad_node_step)
            const uint32_t nxt =
                quad_node_step<NSLOT>(raw_buffer(A.nodes), ref, B, t_lo, box_limit(h.t), s, stk, sp, STACK, peak);
            if (nxt != kEmptyRef) {
                ref = nxt;
                continue;
            }
        } else if constexpr (LANES == 2) {
            const uint32_t nxt =
                pair_node_step<NSLOT>(raw_buffer(A.nodes), ref, B, t_lo, box_limit(h.t), s, stk, sp, STACK, peak);
            if (nxt != kEmptyRef) {
                ref = nxt;
                continue;
            }
        } else {
            const float lim = box_limit(h.t);
            const float4 *np = reinterpret_cast<const float4 *>(A.nodes + ref);
            float4 a0 = np[0], b0 = np[1], a1 = np[2], b1 = np[3], a2 = np[4], b2 = np[5], a3 = np[6], b3 = np[7];
            float k0 = slab(B, a0, b0, t_lo, lim), k1 = slab(B, a1, b1, t_lo, lim);
            float k2 = slab(B, a2, b2, t_lo, lim), k3 = slab(B, a3, b3, t_lo, lim);
            uint32_t c0 = __float_as_uint(a0.w), c1 = __float_as_uint(a1.w), c2 = __float_as_uint(a2.w),
                     c3 = __float_as_uint(a3.w);
            sort4(k0, c0, k1, c1, k2, c2, k3, c3);
            if (k0 != inf) {
                if (k3 != inf) { if (sp < STACK) { stk[sp * NSLOT] = c3; ++sp; } else overflow = true; }
                if (k2 != inf) { if (sp < STACK) { stk[sp * NSLOT] = c2; ++sp; } else overflow = true; }
                if (k1 != inf) { if (sp < STACK) { stk[sp * NSLOT] = c1; ++sp; } else overflow = true; }
                ref = c0;
                continue;
            }
            --sp;
        }
        if (sp < 0) break;
        ref = stk[sp * NSLOT];
    }
    if (peak > STACK) overflow = true;
}

// ---------------------------------------------------------------------------
// Hit attributes + return model + output write (fused epilogue)
// ---------------------------------------------------------------------------
// Attributes of a hit: unit world normal, noise-free eq.4 reflectance
// R_lambda = R_lambda(0) |n . d|^k, label, material and triangle index.  An
// actor's record is in object space: its label is the actor's, its index the
// combined one, and its normal is rotated to the world.
struct Shade {
    float nx, ny, nz, rl;
    uint32_t orig, label, mat;
};

__device__ inline Shade shade_hit(const MaterialsDev &M, const Overrides &ov, float wavelength_nm, const Ray &ray,
                                  const TriRec *__restrict__ r, const Hit &h, const ActorDev *act) {
    Shade S;
    float4 a = r->a, b = r->b, c = r->c;
    S.orig = act ? h.orig : __float_as_uint(a.w);
    S.label = act ? act->label : __float_as_uint(b.w);
    S.mat = __float_as_uint(c.w);
    float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    float cx = fmaf(e1y, e2z, -e1z * e2y);
    float cy = fmaf(e1z, e2x, -e1x * e2z);
    float cz = fmaf(e1x, e2y, -e1y * e2x);
    float len = __fsqrt_rn(fmaf(cx, cx, fmaf(cy, cy, cz * cz)));
    const float inv = 1.0f / len;
    S.nx = cx * inv; S.ny = cy * inv; S.nz = cz * inv;
    if (act) {
        const double X = S.nx, Y = S.ny, Z = S.nz;
        S.nx = (float)(act->R[0] * X + act->R[1] * Y + act->R[2] * Z);
        S.ny = (float)(act->R[3] * X + act->R[4] * Y + act->R[5] * Z);
        S.nz = (float)(act->R[6] * X + act->R[7] * Y + act->R[8] * Z);
    }
    float cd = fmaf(S.nx, ray.dx, fmaf(S.ny, ray.dy, S.nz * ray.dz));
    float cs = fabsf(cd);
    float r0 = reflectance0(ov, M, wavelength_nm, S.mat);
    float kx = ov.angle_exp ? ov.angle_exp[S.mat] : M.angle_exp[S.mat];
    S.rl = (kx == 1.0f) ? r0 * cs : r0 * exp2f(kx * log2f(cs));
    return S;
}

__device__ inline void shade_and_write(const InstanceDev &in, const MaterialsDev &M, const Overrides &ov,
                                       const Outputs &out, uint64_t o, uint32_t beam, uint32_t scan,
                                       const Ray &ray, const TriRec *__restrict__ tris, const Hit &h,
                                       const ActorDev *act = nullptr) {
    bool hit = h.slot != kNone;
    float nx = 0.f, ny = 0.f, nz = 0.f, rl = 0.f, dn = 0.f, inten = 0.f, tt = 0.f;
    uint32_t lab = kNone, orig = kNone;
    uint16_t mat16 = 0xFFFFu;
    bool det = false;
    if (hit) {
        const Shade sh = shade_hit(M, ov, in.wavelength_nm, ray, tris + h.slot, h, act);
        nx = sh.nx; ny = sh.ny; nz = sh.nz;
        rl = sh.rl;
        orig = sh.orig;
        const uint32_t label = sh.label, m = sh.mat;
        mat16 = (uint16_t)m;
        float zd = 0.0f, zi = 0.0f, sig = 0.0f, sig_i = 0.0f;
        if (in.noise_on) {
            uint4 x = philox4x32_10(make_uint4(beam, scan, in.inst_id, 0u), in.seed_lo, in.seed_hi);
            zd = box_muller(x.x, x.y);
            zi = box_muller(x.z, x.w);
            sig = M.sigma[m];
            sig_i = in.sigma_i;
        }
        tt = h.t;
        dn = fmaf(sig, zd, h.t);
        float rlim = (in.r_l_max / in.d_max) * dn;
        det = (dn > in.t_min) && (dn <= in.d_max) && (rlim <= rl);
        inten = fmaxf(0.0f, fmaf(sig_i, zi, rl));
        lab = det ? label : kNone;
    }
    if (out.valid) out.valid[o] = det ? 1 : 0;
    if (out.label) out.label[o] = lab;
    if (out.x) out.x[o] = det ? dn * ray.sx : 0.0f;
    if (out.y) out.y[o] = det ? dn * ray.sy : 0.0f;
    if (out.z) out.z[o] = det ? dn * ray.sz : 0.0f;
    if (out.intensity) out.intensity[o] = det ? inten : 0.0f;
    if (out.range) out.range[o] = det ? dn : 0.0f;
    if (out.tri) out.tri[o] = orig;
    if (out.t_hit) out.t_hit[o] = tt;
    if (out.material) out.material[o] = mat16;
    if (out.r_lambda) out.r_lambda[o] = rl;
    if (out.normal) {
        out.normal[o] = nx;
        out.normal[o + out.plane] = ny;
        out.normal[o + 2 * out.plane] = nz;
    }
}

// tile mapping: padded ray r of an instance -> (channel j, launch column k);
// tiles are numbered column-major (channel rows of one column first)
__device__ inline bool ray_coords(uint64_t r, const InstanceDev &in, int tile_az_log2, uint32_t &j, uint32_t &k) {
    uint32_t tile = (uint32_t)(r >> 6), lane = (uint32_t)(r & 63);
    uint32_t tcol = tile / in.tiles_ch, trow = tile - tcol * in.tiles_ch;
    uint32_t tile_ch = 64u >> tile_az_log2;
    j = trow * tile_ch + (lane >> tile_az_log2);
    k = (tcol << tile_az_log2) + (lane & ((1u << tile_az_log2) - 1u));
    return j < in.n_ch && k < in.n_cols;
}

// blockIdx -> logical block; see the file header for the XCD remap
__device__ inline uint32_t logical_block(int xcd_remap) {
    uint32_t b = blockIdx.x;
    if (!xcd_remap) return b;
    uint32_t full = gridDim.x & ~7u;
    if (b >= full) return b;
    return (b & 7u) * (full >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Kernel 1: one scan, lane per ray
// ---------------------------------------------------------------------------
// The pose of a scan is the same for every beam: thread 0 of the block builds
// it (make_pose, FP64) into LDS once, instead of every lane.  Must be reached
// by all threads of the block (it holds a barrier).
__device__ inline void block_pose(const InstanceDev &in, const Overrides &ov, double *lds) {
    if (threadIdx.x == 0) {
        const Pose64 P = make_pose(in, ov.pose_delta);
#pragma unroll
        for (int e = 0; e < 9; ++e) lds[e] = P.R[e];
#pragma unroll
        for (int e = 0; e < 3; ++e) lds[9 + e] = P.p[e];
    }
    __syncthreads();
}

template <bool SWEEP>
__device__ inline Ray beam_ray_lds(const InstanceDev &in, const double *lds, uint32_t j, uint32_t k, uint32_t &i,
                                   uint32_t &scan) {
    if (SWEEP) {
        i = column_azimuth(in, k, scan);
        return make_ray(in, column_pose(in, nullptr, k), j, i);
    }
    i = k;
    scan = in.scan;
    Pose64 P;
#pragma unroll
    for (int e = 0; e < 9; ++e) P.R[e] = lds[e];
#pragma unroll
    for (int e = 0; e < 3; ++e) P.p[e] = lds[9 + e];
    return make_ray(in, P, j, i);
}

template <int STACK, int BLOCK, bool COUNT, bool SWEEP, bool ACTORS>
__global__ __launch_bounds__(BLOCK) void trace_scan_kernel(SceneDev S, InstanceDev in, MaterialsDev M,
                                                           Overrides ov, Outputs out, int tile_az_log2,
                                                           uint64_t n_padded, int xcd_remap, uint32_t *err,
                                                           uint32_t *__restrict__ n_nodes,
                                                           uint32_t *__restrict__ n_tris, ActorsDev A) {
    __shared__ uint32_t stk[(STACK + kStackPad) * BLOCK];
    __shared__ double pose[12];
    if (!SWEEP) block_pose(in, ov, pose);
    uint64_t r = (uint64_t)logical_block(xcd_remap) * BLOCK + threadIdx.x;
    if (r >= n_padded) return;
    uint32_t j, k, i, scan;
    if (!ray_coords(r, in, tile_az_log2, j, k)) return;
    Ray ray = beam_ray_lds<SWEEP>(in, pose, j, k, i, scan);
    bool overflow = false;
    Counts c{0u, 0u};
    Hit h = traverse<STACK, BLOCK, COUNT>(S.nodes, S.tris, S.root, S.max_steps, ray, in.t_min, in.t_trace, stk + threadIdx.x,
                                          overflow, c, min(S.stack_cap, STACK));
    const ActorDev *act = nullptr;
    const TriRec *tris = S.tris;
    if constexpr (ACTORS) {
        traverse_actors<1, STACK, BLOCK>(A, ray, in.t_min, h, stk + threadIdx.x, 0u, overflow);
        if (h.actor != kNone) {
            act = A.actors + h.actor;
            tris = A.meshes[act->mesh].tris;
        }
    }
    if (overflow) atomicOr(err, 1u);
    uint32_t beam = j * in.n_az + i;
    if (COUNT) {
        n_nodes[beam] = c.nodes;
        n_tris[beam] = c.tris;
    }
    shade_and_write(in, M, ov, out, in.out_base + beam, beam, scan, ray, tris, h, act);
}

// ---------------------------------------------------------------------------
// Kernel 1m: one scan, LANES (2 or 4) lanes per ray (BLOCK / LANES rays)
// ---------------------------------------------------------------------------
// Without actors the kernel is held to 64 VGPRs (8 waves per SIMD: 65.6 vs
// 67.4 us on the 64 x 2048 scan, three spilled dwords outside the hot loop);
// the actor variant is held to 5 waves per SIMD (96 VGPRs, no spills; 117 vs
// 123 us unconstrained at 4 waves, 121 us at 6 with spills).
template <int STACK, int BLOCK, int LANES, bool COUNT, bool SWEEP, bool ACTORS>
__global__ __launch_bounds__(BLOCK, lds_waves(ACTORS ? 5 : 8, 4 * (STACK + kStackPad + 6) * (BLOCK / LANES) + 96, BLOCK))
void trace_scan_multi_kernel(SceneDev S, InstanceDev in, MaterialsDev M, Overrides ov, Outputs out,
                             int tile_az_log2, uint64_t n_padded, int xcd_remap, uint32_t *err,
                             uint32_t *__restrict__ n_nodes, uint32_t *__restrict__ n_tris, ActorsDev A) {
    constexpr int NR = BLOCK / LANES;
    static_assert(NR == 64, "one 64-beam tile per block; its epilogue runs in the first wavefront");
    static_assert(STACK + kStackPad > 6, "the epilogue's directions are handed over in stack entries 1..6");
    __shared__ uint32_t stk[(STACK + kStackPad) * NR];
    __shared__ double pose[12];
    // hits of the block's beams, handed from the walking lanes to the epilogue wavefront:
    // (j << 20 | launch column), record slot, triangle index, t bits, actor, beam active
    __shared__ uint32_t hand[6][NR];
    if (!SWEEP) block_pose(in, ov, pose);
    const uint32_t q = threadIdx.x / LANES, s = threadIdx.x % LANES;
    const uint64_t r = (uint64_t)logical_block(xcd_remap) * NR + q;
    uint32_t j = 0, k = 0;
    const bool active = r < n_padded && ray_coords(r, in, tile_az_log2, j, k);
    if (active) {
        uint32_t i, scan;
        const Ray ray = beam_ray_lds<SWEEP>(in, pose, j, k, i, scan);
        bool overflow = false;
        Counts c{0u, 0u};
        // the static walk, specialised for the wavefront's mode (not in the counting variant, which
        // keeps one copy of the loop)
        Hit h = traverse_multi<LANES, STACK, NR, COUNT, !COUNT>(
            S.nodes, S.tris, S.root, S.max_steps, ray, in.t_min, in.t_trace, stk + q, s, overflow, c,
            min(S.stack_cap, STACK));
        if constexpr (ACTORS) traverse_actors<LANES, STACK, NR>(A, ray, in.t_min, h, stk + q, s, overflow);
        if (overflow) atomicOr(err, 1u);
        if (SWEEP && s == 0) {
            // the beam's direction, world and sensor frame, for the epilogue: entries 1..6 of the beam's
            // stack, free once its walks are done
            stk[1 * NR + q] = __float_as_uint(ray.dx);
            stk[2 * NR + q] = __float_as_uint(ray.dy);
            stk[3 * NR + q] = __float_as_uint(ray.dz);
            stk[4 * NR + q] = __float_as_uint(ray.sx);
            stk[5 * NR + q] = __float_as_uint(ray.sy);
            stk[6 * NR + q] = __float_as_uint(ray.sz);
        }
        if (s == 0) {
            if (COUNT) {
                const uint32_t beam = j * in.n_az + i;
                n_nodes[beam] = c.nodes;
                n_tris[beam] = c.tris;
            }
            hand[0][q] = (j << 20) | k;
            hand[1][q] = h.slot;
            hand[2][q] = h.orig;
            hand[3][q] = __float_as_uint(h.t);
            hand[4][q] = h.actor;
        }
    }
    if (s == 0) hand[5][q] = active ? 1u : 0u;
    __syncthreads();
    // Epilogue: the block's 64 beams, one per lane of the first wavefront, instead
    // of one lane in LANES of every wavefront.
    if (threadIdx.x >= (unsigned)NR || !hand[5][threadIdx.x]) return;
    const uint32_t e = threadIdx.x;
    j = hand[0][e] >> 20;
    k = hand[0][e] & 0xFFFFFu;
    uint32_t i, scan;
    Ray ray;
    if (SWEEP) {
        i = column_azimuth(in, k, scan);
        ray.ox = ray.oy = ray.oz = 0.0f;   // shading uses the beam's directions only
        ray.dx = __uint_as_float(stk[1 * NR + e]);
        ray.dy = __uint_as_float(stk[2 * NR + e]);
        ray.dz = __uint_as_float(stk[3 * NR + e]);
        ray.sx = __uint_as_float(stk[4 * NR + e]);
        ray.sy = __uint_as_float(stk[5 * NR + e]);
        ray.sz = __uint_as_float(stk[6 * NR + e]);
    } else {
        ray = beam_ray_lds<false>(in, pose, j, k, i, scan);
    }
    const Hit h{hand[1][e], hand[2][e], __uint_as_float(hand[3][e]), hand[4][e]};
    const ActorDev *act = nullptr;
    const TriRec *tris = S.tris;
    if (ACTORS && h.actor != kNone) {
        act = A.actors + h.actor;
        tris = A.meshes[act->mesh].tris;
    }
    const uint32_t beam = j * in.n_az + i;
    shade_and_write(in, M, ov, out, in.out_base + beam, beam, scan, ray, tris, h, act);
}

// ---------------------------------------------------------------------------
// Kernel 1e: divergent beams.  Sub-ray k of beam (j, i) is the beam axis s
// turned by r_k towards cos(b_k) e_theta + sin(b_k) e_phi (unit azimuth and
// elevation tangents at s), in FP64 and rounded once after the rotation to the
// world: s_k = cos(r_k) s + sin(r_k) (cos(b_k) e_theta + sin(b_k) e_phi).
// Sub-ray 0 (r = 0) is exactly the beam of the single return.  The launch
// covers the beams once per sub-ray (slice k = padded ray / n_padded), and
// each sub-ray's first hit and noise-free R_lambda go to sub[beam][k].
// ---------------------------------------------------------------------------
__device__ inline Ray make_subray(const InstanceDev &in, const Pose64 &P, uint32_t j, uint32_t i, const double *pc) {
    const double cp = in.elev_cs[2 * j], sp = in.elev_cs[2 * j + 1];
    const double ct = in.az_cs[2 * i], st = in.az_cs[2 * i + 1];
    const double a0 = cp * ct, a1 = cp * st, a2 = sp;           // axis
    const double t0 = -st, t1 = ct, t2 = 0.0;                   // e_theta
    const double p0 = -sp * ct, p1 = -sp * st, p2 = cp;         // e_phi
    const double cr = pc[0], sr = pc[1], cb = pc[2], sb = pc[3];
    const double s0 = cr * a0 + sr * (cb * t0 + sb * p0);
    const double s1 = cr * a1 + sr * (cb * t1 + sb * p1);
    const double s2 = cr * a2 + sr * (cb * t2 + sb * p2);
    Ray r;
    r.sx = (float)a0; r.sy = (float)a1; r.sz = (float)a2;
    r.dx = (float)(P.R[0] * s0 + P.R[1] * s1 + P.R[2] * s2);
    r.dy = (float)(P.R[3] * s0 + P.R[4] * s1 + P.R[5] * s2);
    r.dz = (float)(P.R[6] * s0 + P.R[7] * s1 + P.R[8] * s2);
    r.ox = (float)P.p[0]; r.oy = (float)P.p[1]; r.oz = (float)P.p[2];
    return r;
}

template <int STACK, int BLOCK, int LANES, bool ACTORS>
__global__ __launch_bounds__(BLOCK) void trace_subrays_kernel(SceneDev S, InstanceDev in, MaterialsDev M,
                                                              SubrayPattern pat, SubHit *__restrict__ sub,
                                                              int tile_az_log2, uint64_t n_padded, int xcd_remap,
                                                              uint32_t *err, ActorsDev A) {
    constexpr int NR = BLOCK / LANES;
    __shared__ uint32_t stk[(STACK + kStackPad) * NR];
    __shared__ double pose[12];
    const Overrides ov{nullptr, nullptr, nullptr, nullptr};
    block_pose(in, ov, pose);
    const uint32_t q = threadIdx.x / LANES, s = threadIdx.x % LANES;
    const uint64_t r = (uint64_t)logical_block(xcd_remap) * NR + q;
    if (r >= n_padded * pat.n_sub) return;     // all lanes of the sub-ray
    const uint32_t k = (uint32_t)(r / n_padded);
    uint32_t j, i;
    if (!ray_coords(r - (uint64_t)k * n_padded, in, tile_az_log2, j, i)) return;
    Pose64 P;
#pragma unroll
    for (int e = 0; e < 9; ++e) P.R[e] = pose[e];
#pragma unroll
    for (int e = 0; e < 3; ++e) P.p[e] = pose[9 + e];
    const Ray ray = make_subray(in, P, j, i, pat.c[k]);
    bool overflow = false;
    Counts c{0u, 0u};
    Hit h;
    if constexpr (LANES == 1)
        h = traverse<STACK, NR, false>(S.nodes, S.tris, S.root, S.max_steps, ray, in.t_min, in.t_trace, stk + q,
                                       overflow, c, min(S.stack_cap, STACK));
    else
        h = traverse_multi<LANES, STACK, NR, false, !ACTORS>(S.nodes, S.tris, S.root, S.max_steps, ray, in.t_min,
                                                    in.t_trace, stk + q, s, overflow, c, min(S.stack_cap, STACK));
    const ActorDev *act = nullptr;
    const TriRec *tris = S.tris;
    if constexpr (ACTORS) {
        traverse_actors<LANES, STACK, NR>(A, ray, in.t_min, h, stk + q, s, overflow);
        if (h.actor != kNone) {
            act = A.actors + h.actor;
            tris = A.meshes[act->mesh].tris;
        }
    }
    if (overflow) atomicOr(err, 1u);
    if (s != 0) return;
    SubHit o{__builtin_inff(), kNone, 0.0f, kNone, 0xFFFFu, 0u};
    if (h.slot != kNone) {
        const Shade sh = shade_hit(M, ov, in.wavelength_nm, ray, tris + h.slot, h, act);
        o = SubHit{h.t, sh.orig, sh.rl, sh.label, sh.mat, 0u};
    }
    sub[(size_t)(j * in.n_az + i) * pat.n_sub + k] = o;
}

// ---------------------------------------------------------------------------
// Kernel 1f: echoes of one beam from its sub-ray hits.  The hits, ordered by
// (t, k) with a sorting network over KMAX registers, form
// echoes split where consecutive ranges differ by more than echo_sep.  Echo e:
// strength P = (1/K) sum R_k, range t_first + sum R_k (t_k - t_first) / sum R_k
// (plain mean if every R is 0), label/material/index of its strongest sub-ray
// (smallest k on ties), Philox counter (beam, scan, instance, e) for the range
// and intensity noise, then the eq.5 test with P in place of R_lambda.
// Outputs: plane e of every array holds echo e; unformed echoes read as
// misses.  With K = 1 the first echo is the single return, bit for bit.
// ---------------------------------------------------------------------------
template <int KMAX>
__global__ __launch_bounds__(128) void echo_kernel(InstanceDev in, MaterialsDev M, const SubHit *__restrict__ sub,
                                                   uint32_t K, uint32_t E, float sep, Outputs out) {
    const uint32_t nb = in.n_ch * in.n_az;
    const uint32_t beam = blockIdx.x * 128 + threadIdx.x;
    if (beam >= nb) return;
    float t[KMAX], rl[KMAX];
    uint32_t kk[KMAX], orig[KMAX], lab[KMAX], mat[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        kk[q] = (uint32_t)q;
        if ((uint32_t)q < K) {
            const SubHit h = sub[(size_t)beam * K + q];
            t[q] = h.t; rl[q] = h.rl; orig[q] = h.orig; lab[q] = h.label; mat[q] = h.mat;
        } else {
            t[q] = __builtin_inff(); rl[q] = 0.0f; orig[q] = kNone; lab[q] = kNone; mat[q] = 0xFFFFu;
        }
    }
    // compare-exchange of entries q < r by (t, k); (t, k) pairs are distinct, so any sorting network gives
    // the same order
    auto cx = [&](int q, int r) {
        const bool sw = t[r] < t[q] || (t[r] == t[q] && kk[r] < kk[q]);
#define LIDAR_CSWAP(A)                          \
        {                                       \
            auto lo_ = sw ? A[r] : A[q];        \
            auto hi_ = sw ? A[q] : A[r];        \
            A[q] = lo_;                         \
            A[r] = hi_;                         \
        }
        LIDAR_CSWAP(t) LIDAR_CSWAP(rl) LIDAR_CSWAP(kk) LIDAR_CSWAP(orig) LIDAR_CSWAP(lab) LIDAR_CSWAP(mat)
#undef LIDAR_CSWAP
    };
    if constexpr (KMAX == 4) {          // 5 comparators, depth 3
        cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2);
    } else if constexpr (KMAX == 8) {   // 19 comparators, depth 6 (checked by the 0-1 principle)
        cx(0, 2); cx(1, 3); cx(4, 6); cx(5, 7);
        cx(0, 4); cx(1, 5); cx(2, 6); cx(3, 7);
        cx(0, 1); cx(2, 3); cx(4, 5); cx(6, 7);
        cx(2, 4); cx(3, 5);
        cx(1, 4); cx(3, 6);
        cx(1, 2); cx(3, 4); cx(5, 6);
    } else {                            // odd-even transposition, KMAX rounds
#pragma unroll
        for (int round = 0; round < KMAX; ++round) {
#pragma unroll
            for (int q = round & 1; q + 1 < KMAX; q += 2) cx(q, q + 1);
        }
    }
    const uint32_t j = beam / in.n_az, i = beam - j * in.n_az;
    const double cp = in.elev_cs[2 * j], sp = in.elev_cs[2 * j + 1];
    const double ct = in.az_cs[2 * i], st = in.az_cs[2 * i + 1];
    const float sx = (float)(cp * ct), sy = (float)(cp * st), sz = (float)sp;
    const uint64_t plane = nb;
    // running group: first range, sums, strongest sub-ray
    uint32_t e = 0;
    int n_in = 0;
    float t0 = 0.0f, t_prev = 0.0f, sum_r = 0.0f, sum_rt = 0.0f, sum_dt = 0.0f, best_r = -1.0f;
    uint32_t best_k = kNone, best_orig = kNone, best_lab = kNone, best_mat = 0xFFFFu;
    auto emit = [&]() {
        if (e >= E) return;
        const float P = sum_r / (float)K;
        const float te = (sum_r > 0.0f) ? t0 + sum_rt / sum_r : t0 + sum_dt / (float)n_in;
        float zd = 0.0f, zi = 0.0f, sig = 0.0f, sig_i = 0.0f;
        if (in.noise_on) {
            const uint4 x = philox4x32_10(make_uint4(beam, in.scan, in.inst_id, e), in.seed_lo, in.seed_hi);
            zd = box_muller(x.x, x.y);
            zi = box_muller(x.z, x.w);
            sig = M.sigma[best_mat];
            sig_i = in.sigma_i;
        }
        const float dn = fmaf(sig, zd, te);
        const float rlim = (in.r_l_max / in.d_max) * dn;
        const bool det = (dn > in.t_min) && (dn <= in.d_max) && (rlim <= P);
        const float inten = fmaxf(0.0f, fmaf(sig_i, zi, P));
        const uint64_t o = in.out_base + (uint64_t)e * plane + beam;
        if (out.valid) out.valid[o] = det ? 1 : 0;
        if (out.label) out.label[o] = det ? best_lab : kNone;
        if (out.x) out.x[o] = det ? dn * sx : 0.0f;
        if (out.y) out.y[o] = det ? dn * sy : 0.0f;
        if (out.z) out.z[o] = det ? dn * sz : 0.0f;
        if (out.intensity) out.intensity[o] = det ? inten : 0.0f;
        if (out.range) out.range[o] = det ? dn : 0.0f;
        if (out.tri) out.tri[o] = best_orig;
        if (out.t_hit) out.t_hit[o] = te;
        if (out.material) out.material[o] = (uint16_t)best_mat;
        if (out.r_lambda) out.r_lambda[o] = P;
        ++e;
    };
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        if (t[q] != __builtin_inff()) {
            if (n_in > 0 && t[q] - t_prev > sep) {
                emit();
                n_in = 0;
            }
            if (n_in == 0) {
                t0 = t[q];
                sum_r = 0.0f; sum_rt = 0.0f; sum_dt = 0.0f; best_r = -1.0f; best_k = kNone;
            }
            sum_r += rl[q];
            sum_rt = fmaf(rl[q], t[q] - t0, sum_rt);
            sum_dt += t[q] - t0;
            if (rl[q] > best_r || (rl[q] == best_r && kk[q] < best_k)) {
                best_r = rl[q]; best_k = kk[q]; best_orig = orig[q]; best_lab = lab[q]; best_mat = mat[q];
            }
            t_prev = t[q];
            ++n_in;
        }
    }
    if (n_in > 0) emit();
    for (; e < E; ++e) {
        const uint64_t o = in.out_base + (uint64_t)e * plane + beam;
        if (out.valid) out.valid[o] = 0;
        if (out.label) out.label[o] = kNone;
        if (out.x) out.x[o] = 0.0f;
        if (out.y) out.y[o] = 0.0f;
        if (out.z) out.z[o] = 0.0f;
        if (out.intensity) out.intensity[o] = 0.0f;
        if (out.range) out.range[o] = 0.0f;
        if (out.tri) out.tri[o] = kNone;
        if (out.t_hit) out.t_hit[o] = 0.0f;
        if (out.material) out.material[o] = 0xFFFFu;
        if (out.r_lambda) out.r_lambda[o] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Kernel 2: one scan, every beam against every triangle (reference path).
// Triangle records are staged through LDS in chunks shared by the block.
// ---------------------------------------------------------------------------
template <int BLOCK, int CHUNK>
__global__ __launch_bounds__(BLOCK) void bruteforce_kernel(SceneDev S, InstanceDev in, MaterialsDev M,
                                                           Overrides ov, Outputs out, int tile_az_log2,
                                                           uint64_t n_padded) {
    __shared__ float4 lds[CHUNK * 3];
    uint64_t r = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    uint32_t j = 0, k = 0, scan = in.scan;
    bool active = r < n_padded && ray_coords(r, in, tile_az_log2, j, k);
    if (!active) j = k = 0;
    uint32_t i = column_azimuth(in, k, scan);
    Pose64 P = column_pose(in, ov.pose_delta, k);
    Ray ray = make_ray(in, P, j, i);
    RayTri T = prep_tri_test(ray);
    Hit h{kNone, kNone, in.t_trace, kNone};
    const float4 *src = reinterpret_cast<const float4 *>(S.tris);
    for (uint32_t base = 0; base < S.n_tri; base += CHUNK) {
        uint32_t cnt = min((uint32_t)CHUNK, S.n_tri - base);
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < cnt * 3; k += BLOCK) lds[k] = src[(size_t)base * 3 + k];
        __syncthreads();
        if (active) {
            for (uint32_t k = 0; k < cnt; ++k) {
                float4 a = lds[3 * k], b = lds[3 * k + 1], c = lds[3 * k + 2];
                float t;
                if (tri_hit(T, a, b, c, in.t_min, t)) {
                    uint32_t orig = __float_as_uint(a.w);
                    if (better(t, orig, h.t, h.orig)) { h.t = t; h.orig = orig; h.slot = base + k; }
                }
            }
        }
    }
    if (!active) return;
    uint32_t beam = j * in.n_az + i;
    shade_and_write(in, M, ov, out, in.out_base + beam, beam, scan, ray, S.tris, h);
}

// ---------------------------------------------------------------------------
// Kernel 3: batched persistent form.  Every wavefront pops packets of
// `packet` padded rays from a device counter until the queue is empty.  A
// packet is walked in groups of 64 padded rays; an instance's padded rays are
// a whole number of 64-ray tiles, so a group lies in one instance: the
// instance (binary search over the instances' first padded ray) and its pose
// are found once per group.  The group's rays are traversed 64 / LANES at a
// time; the hits go through LDS to an epilogue in which every lane of the
// wavefront shades and writes one beam.
// ---------------------------------------------------------------------------
__device__ inline Pose64 lds_pose(const double *q) {
    Pose64 P;
#pragma unroll
    for (int e = 0; e < 9; ++e) P.R[e] = q[e];
#pragma unroll
    for (int e = 0; e < 3; ++e) P.p[e] = q[9 + e];
    return P;
}

__device__ inline uint32_t find_instance(const InstanceDev *__restrict__ insts, uint32_t n_inst, uint64_t r) {
    uint32_t lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (insts[mid].ray_base <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// LDS exchange between the lanes of one wavefront (waves of a block run
// different numbers of packets, so no block barrier can be used here)
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int STACK, int BLOCK, int LANES>
__global__ __launch_bounds__(BLOCK, lds_waves(LANES == 4 ? 8 : LANES == 2 ? 6 : 1,
                                           4 * (STACK + kStackPad) * (BLOCK / LANES) + (BLOCK / 64) * (3 * 64 * 4 + 96), BLOCK))
void trace_batch_kernel(SceneDev S, const InstanceDev *__restrict__ insts, uint32_t n_inst, MaterialsDev M,
                        Outputs out, int tile_az_log2, uint64_t n_padded_total, uint32_t packet,
                        uint32_t *queue, uint32_t *err, uint32_t *__restrict__ redo, uint32_t *redo_count,
                        uint32_t redo_cap) {
    constexpr int NSLOT = BLOCK / LANES;
    constexpr uint32_t RAYS_PER_WAVE = 64u / LANES;
    __shared__ uint32_t stk[(STACK + kStackPad) * NSLOT];
    // per wavefront, per ray of the current 64-ray group: record slot, triangle index, t bits
    __shared__ uint32_t hand[BLOCK / 64][3][64];
    __shared__ double gpose[BLOCK / 64][12];    // per wavefront: the group's FP64 pose (R row-major, p)
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t slot = threadIdx.x / LANES;
    const uint32_t sub_lane = lane / LANES;
    const uint32_t s = threadIdx.x % LANES;
    const Overrides ov{nullptr, nullptr, nullptr, nullptr};
    const uint64_t n_packets = (n_padded_total + packet - 1) / packet;
    bool overflow = false;
    Counts cnt{0u, 0u};
    while (true) {
        uint32_t pk = 0;
        if (lane == 0) pk = atomicAdd(queue, 1u);
        pk = __shfl(pk, 0, 64);
        if ((uint64_t)pk >= n_packets) break;
        for (uint32_t g = 0; g < packet; g += 64u) {
            const uint64_t base = (uint64_t)pk * packet + g;      // uniform over the wave
            if (base >= n_padded_total) break;
            const uint32_t ii = __builtin_amdgcn_readfirstlane(find_instance(insts, n_inst, base));
            const InstanceDev &in = insts[ii];
            {
                const Pose64 P = make_pose(in, nullptr);
                if (lane == 0) {
#pragma unroll
                    for (int e = 0; e < 9; ++e) gpose[wave][e] = P.R[e];
#pragma unroll
                    for (int e = 0; e < 3; ++e) gpose[wave][9 + e] = P.p[e];
                }
            }
            wave_lds_sync();
            const uint64_t r0 = base - in.ray_base;
            for (uint32_t sub = 0; sub < 64u; sub += RAYS_PER_WAVE) {
                uint32_t j, k;
                Hit h{kNone, kNone, 0.0f, kNone};
                if (ray_coords(r0 + sub + sub_lane, in, tile_az_log2, j, k)) {
                    const Ray ray = make_ray(in, lds_pose(gpose[wave]), j, k);
                    bool ovf = false;
                    if constexpr (LANES == 1)
                        h = traverse<STACK, NSLOT, false>(S.nodes, S.tris, S.root, S.max_steps, ray, in.t_min,
                                                          in.t_trace, stk + slot, ovf, cnt,
                                                          min(S.stack_cap, STACK));
                    else
                        h = traverse_multi<LANES, STACK, NSLOT, false, true>(S.nodes, S.tris, S.root, S.max_steps, ray,
                                                                       in.t_min, in.t_trace, stk + slot, s, ovf,
                                                                       cnt, min(S.stack_cap, STACK));
                    // a walk that ran out of this pass's stack (the same for all lanes of its ray) is
                    // listed for the second pass, which traces it again with the whole stack
                    if (ovf) {
                        if (!redo) {
                            overflow = true;
                        } else if (s == 0) {
                            const uint32_t slot_r = atomicAdd(redo_count, 1u);
                            if (slot_r < redo_cap) redo[slot_r] = (uint32_t)(base + sub + sub_lane);
                            else overflow = true;
                        }
                    }
                }
                if (s == 0) {
                    hand[wave][0][sub + sub_lane] = h.slot;
                    hand[wave][1][sub + sub_lane] = h.orig;
                    hand[wave][2][sub + sub_lane] = __float_as_uint(h.t);
                }
            }
            wave_lds_sync();
            uint32_t j, k;
            if (ray_coords(r0 + lane, in, tile_az_log2, j, k)) {
                const Ray ray = make_ray(in, lds_pose(gpose[wave]), j, k);
                const Hit h{hand[wave][0][lane], hand[wave][1][lane], __uint_as_float(hand[wave][2][lane]), kNone};
                const uint32_t beam = j * in.n_az + k;
                shade_and_write(in, M, ov, out, in.out_base + beam, beam, in.scan, ray, S.tris, h);
            }
            wave_lds_sync();     // the hand-off slots are rewritten by the next group
        }
    }
    if (overflow) atomicOr(err, 1u);
}

__global__ void reset_queue_kernel(uint32_t *queue, uint32_t *redo_count) {
    *queue = 0u;
    if (redo_count) *redo_count = 0u;
}

// Second pass of a batch whose first pass ran with a short stack: every listed
// ray (its padded index) is traced again by one lane with the whole stack,
// shaded and written over the first pass's output.  The hit is the same as
// any walk's that kept all of its children (the lexicographic (t, index)
// minimum), so the batch's results do not depend on the first pass's stack.
template <int STACK>
__global__ __launch_bounds__(64) void batch_redo_kernel(SceneDev S, const InstanceDev *__restrict__ insts,
                                                        uint32_t n_inst, MaterialsDev M, Outputs out,
                                                        int tile_az_log2, const uint32_t *__restrict__ redo,
                                                        const uint32_t *__restrict__ redo_count, uint32_t redo_cap,
                                                        uint32_t *err) {
    __shared__ uint32_t stk[(STACK + kStackPad) * 64];
    const Overrides ov{nullptr, nullptr, nullptr, nullptr};
    const uint32_t n = min(*redo_count, redo_cap);
    bool overflow = false;
    Counts cnt{0u, 0u};
    for (uint32_t i = blockIdx.x * 64u + threadIdx.x; i < n; i += gridDim.x * 64u) {
        const uint64_t r = redo[i];
        const InstanceDev &in = insts[find_instance(insts, n_inst, r)];
        uint32_t j, k;
        if (!ray_coords(r - in.ray_base, in, tile_az_log2, j, k)) continue;
        const Ray ray = make_ray(in, make_pose(in, nullptr), j, k);
        const Hit h = traverse<STACK, 64, false>(S.nodes, S.tris, S.root, S.max_steps, ray, in.t_min, in.t_trace,
                                                 stk + threadIdx.x, overflow, cnt, min(S.stack_cap, STACK));
        const uint32_t beam = j * in.n_az + k;
        shade_and_write(in, M, ov, out, in.out_base + beam, beam, in.scan, ray, S.tris, h);
    }
    if (overflow) atomicOr(err, 1u);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int kBlock = 128;       // lane-per-ray block (2 waves, 128 rays)
constexpr int kPairBlock = 128;   // pair-per-ray block (2 waves, 64 rays)
constexpr int kQuadBlock = 256;   // quad-per-ray block (4 waves, 64 rays)

template <int STACK, bool COUNT, bool SWEEP, bool ACTORS>
static void launch_scan_t(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                          const Overrides &ov, const Outputs &out, uint64_t n_padded, uint32_t *err,
                          uint32_t *nn, uint32_t *nt, const ActorsDev &A, hipStream_t s) {
    if (t.lanes_per_ray == 4) {
        uint32_t blocks = (uint32_t)((n_padded * 4 + kQuadBlock - 1) / kQuadBlock);
        trace_scan_multi_kernel<STACK, kQuadBlock, 4, COUNT, SWEEP, ACTORS><<<blocks, kQuadBlock, 0, s>>>(
            S, in, M, ov, out, t.tile_az_log2, n_padded, t.xcd_remap, err, nn, nt, A);
    } else if (t.lanes_per_ray == 2) {
        uint32_t blocks = (uint32_t)((n_padded * 2 + kPairBlock - 1) / kPairBlock);
        trace_scan_multi_kernel<STACK, kPairBlock, 2, COUNT, SWEEP, ACTORS><<<blocks, kPairBlock, 0, s>>>(
            S, in, M, ov, out, t.tile_az_log2, n_padded, t.xcd_remap, err, nn, nt, A);
    } else {
        uint32_t blocks = (uint32_t)((n_padded + kBlock - 1) / kBlock);
        trace_scan_kernel<STACK, kBlock, COUNT, SWEEP, ACTORS><<<blocks, kBlock, 0, s>>>(
            S, in, M, ov, out, t.tile_az_log2, n_padded, t.xcd_remap, err, nn, nt, A);
    }
}

template <int STACK>
static void launch_scan_s(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                          const Overrides &ov, const Outputs &out, uint64_t n_padded, uint32_t *err,
                          uint32_t *nn, uint32_t *nt, const ActorsDev *A, hipStream_t s) {
    const bool sweep = in.sweep != 0;
    const ActorsDev none{};
    if (A) {   // dynamic scene (never counted)
        if (sweep) launch_scan_t<STACK, false, true, true>(t, S, in, M, ov, out, n_padded, err, nullptr, nullptr, *A, s);
        else launch_scan_t<STACK, false, false, true>(t, S, in, M, ov, out, n_padded, err, nullptr, nullptr, *A, s);
    } else if (sweep) {
        launch_scan_t<STACK, false, true, false>(t, S, in, M, ov, out, n_padded, err, nullptr, nullptr, none, s);
    } else if (nn) {
        launch_scan_t<STACK, true, false, false>(t, S, in, M, ov, out, n_padded, err, nn, nt, none, s);
    } else {
        launch_scan_t<STACK, false, false, false>(t, S, in, M, ov, out, n_padded, err, nullptr, nullptr, none, s);
    }
}

void launch_trace_scan(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                       const Overrides &ov, const Outputs &out, uint64_t n_padded, uint32_t *err, uint32_t *n_nodes,
                       uint32_t *n_tris, const ActorsDev *actors, hipStream_t s) {
    if (t.stack <= 32) launch_scan_s<32>(t, S, in, M, ov, out, n_padded, err, n_nodes, n_tris, actors, s);
    else if (t.stack <= 48) launch_scan_s<48>(t, S, in, M, ov, out, n_padded, err, n_nodes, n_tris, actors, s);
    else if (t.stack <= 64) launch_scan_s<64>(t, S, in, M, ov, out, n_padded, err, n_nodes, n_tris, actors, s);
    else launch_scan_s<96>(t, S, in, M, ov, out, n_padded, err, n_nodes, n_tris, actors, s);
}

template <int STACK, bool ACTORS>
static void launch_subrays_t(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                             const SubrayPattern &pat, SubHit *sub, uint64_t n_padded, uint32_t *err,
                             const ActorsDev &A, hipStream_t s) {
    const uint64_t rays = n_padded * pat.n_sub;
    if (t.lanes_per_ray == 4) {
        uint32_t blocks = (uint32_t)((rays * 4 + kQuadBlock - 1) / kQuadBlock);
        trace_subrays_kernel<STACK, kQuadBlock, 4, ACTORS><<<blocks, kQuadBlock, 0, s>>>(
            S, in, M, pat, sub, t.tile_az_log2, n_padded, t.xcd_remap, err, A);
    } else if (t.lanes_per_ray == 2) {
        uint32_t blocks = (uint32_t)((rays * 2 + kPairBlock - 1) / kPairBlock);
        trace_subrays_kernel<STACK, kPairBlock, 2, ACTORS><<<blocks, kPairBlock, 0, s>>>(
            S, in, M, pat, sub, t.tile_az_log2, n_padded, t.xcd_remap, err, A);
    } else {
        uint32_t blocks = (uint32_t)((rays + kBlock - 1) / kBlock);
        trace_subrays_kernel<STACK, kBlock, 1, ACTORS><<<blocks, kBlock, 0, s>>>(
            S, in, M, pat, sub, t.tile_az_log2, n_padded, t.xcd_remap, err, A);
    }
}

void launch_trace_subrays(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                          const SubrayPattern &pat, SubHit *sub, uint64_t n_padded, uint32_t *err,
                          const ActorsDev *actors, hipStream_t s) {
    const ActorsDev none{};
    if (actors) {
        if (t.stack <= 32) launch_subrays_t<32, true>(t, S, in, M, pat, sub, n_padded, err, *actors, s);
        else if (t.stack <= 48) launch_subrays_t<48, true>(t, S, in, M, pat, sub, n_padded, err, *actors, s);
        else if (t.stack <= 64) launch_subrays_t<64, true>(t, S, in, M, pat, sub, n_padded, err, *actors, s);
        else launch_subrays_t<96, true>(t, S, in, M, pat, sub, n_padded, err, *actors, s);
    } else {
        if (t.stack <= 32) launch_subrays_t<32, false>(t, S, in, M, pat, sub, n_padded, err, none, s);
        else if (t.stack <= 48) launch_subrays_t<48, false>(t, S, in, M, pat, sub, n_padded, err, none, s);
        else if (t.stack <= 64) launch_subrays_t<64, false>(t, S, in, M, pat, sub, n_padded, err, none, s);
        else launch_subrays_t<96, false>(t, S, in, M, pat, sub, n_padded, err, none, s);
    }
}

void launch_echoes(const InstanceDev &in, const MaterialsDev &M, const SubHit *sub, uint32_t n_sub,
                   uint32_t max_echoes, float echo_sep, const Outputs &out, hipStream_t s) {
    const uint32_t nb = in.n_ch * in.n_az;
    const uint32_t blocks = (nb + 127) / 128;
    if (n_sub <= 4) echo_kernel<4><<<blocks, 128, 0, s>>>(in, M, sub, n_sub, max_echoes, echo_sep, out);
    else if (n_sub <= 8) echo_kernel<8><<<blocks, 128, 0, s>>>(in, M, sub, n_sub, max_echoes, echo_sep, out);
    else echo_kernel<kMaxSub><<<blocks, 128, 0, s>>>(in, M, sub, n_sub, max_echoes, echo_sep, out);
}

void launch_bruteforce(const SceneDev &S, const InstanceDev &in, const MaterialsDev &M, const Overrides &ov,
                       const Outputs &out, int tile_az_log2, uint64_t n_padded, hipStream_t s) {
    constexpr int B = 256, C = 512;
    uint64_t blocks = (n_padded + B - 1) / B;
    bruteforce_kernel<B, C><<<(uint32_t)blocks, B, 0, s>>>(S, in, M, ov, out, tile_az_log2, n_padded);
}

template <int STACK, int LANES>
static void launch_batch_t(const SceneDev &S, const InstanceDev *insts, uint32_t n_inst, const MaterialsDev &M,
                           const Outputs &out, int tile_az_log2, uint64_t n_padded, uint32_t packet,
                           uint32_t *queue, uint32_t *err, const BatchRedo &R, uint32_t grid, hipStream_t s) {
    constexpr int B = LANES == 4 ? kQuadBlock : LANES == 2 ? kPairBlock : kBlock;
    trace_batch_kernel<STACK, B, LANES><<<grid, B, 0, s>>>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet,
                                                           queue, err, R.list, R.count, R.cap);
}

template <int STACK>
static void launch_batch_s(int lanes, const SceneDev &S, const InstanceDev *insts, uint32_t n_inst,
                           const MaterialsDev &M, const Outputs &out, int tile_az_log2, uint64_t n_padded,
                           uint32_t packet, uint32_t *queue, uint32_t *err, const BatchRedo &R, uint32_t grid,
                           hipStream_t s) {
    if (lanes == 4)
        launch_batch_t<STACK, 4>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet, queue, err, R, grid, s);
    else if (lanes == 2)
        launch_batch_t<STACK, 2>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet, queue, err, R, grid, s);
    else
        launch_batch_t<STACK, 1>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet, queue, err, R, grid, s);
}

template <int STACK>
static void launch_redo_s(const SceneDev &S, const InstanceDev *insts, uint32_t n_inst, const MaterialsDev &M,
                          const Outputs &out, int tile_az_log2, uint32_t *err, const BatchRedo &R, hipStream_t s) {
    batch_redo_kernel<STACK><<<kRedoBlocks, 64, 0, s>>>(S, insts, n_inst, M, out, tile_az_log2, R.list, R.count,
                                                         R.cap, err);
}

void launch_trace_batch(const TraceOpts &t, const SceneDev &S, const InstanceDev *insts, uint32_t n_inst,
                        const MaterialsDev &M, const Outputs &out, uint64_t n_padded, uint32_t packet,
                        uint32_t *queue, uint32_t *err, const BatchRedo &R, uint32_t grid, hipStream_t s) {
    reset_queue_kernel<<<1, 1, 0, s>>>(queue, R.count);
    // the first pass: a short stack (at most R.first_cap entries) when R.list is set, else the whole one
    SceneDev S1 = S;
    int st = t.stack;
    if (R.list) {
        st = R.first_stack;
        S1.stack_cap = min(S.stack_cap, R.first_cap);
    }
    if (st <= 32) launch_batch_s<32>(t.lanes_per_ray, S1, insts, n_inst, M, out, t.tile_az_log2, n_padded, packet, queue, err, R, grid, s);
    else if (st <= 48) launch_batch_s<48>(t.lanes_per_ray, S1, insts, n_inst, M, out, t.tile_az_log2, n_padded, packet, queue, err, R, grid, s);
    else if (st <= 64) launch_batch_s<64>(t.lanes_per_ray, S1, insts, n_inst, M, out, t.tile_az_log2, n_padded, packet, queue, err, R, grid, s);
    else launch_batch_s<96>(t.lanes_per_ray, S1, insts, n_inst, M, out, t.tile_az_log2, n_padded, packet, queue, err, R, grid, s);
    if (!R.list) return;
    if (t.stack <= 32) launch_redo_s<32>(S, insts, n_inst, M, out, t.tile_az_log2, err, R, s);
    else if (t.stack <= 48) launch_redo_s<48>(S, insts, n_inst, M, out, t.tile_az_log2, err, R, s);
    else if (t.stack <= 64) launch_redo_s<64>(S, insts, n_inst, M, out, t.tile_az_log2, err, R, s);
    else launch_redo_s<96>(S, insts, n_inst, M, out, t.tile_az_log2, err, R, s);
}

int batch_blocks_per_cu(const TraceOpts &t, int stack) {
    // LDS per block = stack entries x stack slots x 4 bytes; 160 KB per CU on gfx950.  Blocks beyond what
    // the registers let reside (pairs with a 32-entry stack: 12 of 14) start when the queue is empty and
    // leave at once.
    int st = stack <= 32 ? 32 : stack <= 48 ? 48 : stack <= 64 ? 64 : 96;
    int lanes = t.lanes_per_ray;
    int block = lanes == 4 ? kQuadBlock : lanes == 2 ? kPairBlock : kBlock;
    int slots = block / lanes;
    int waves = block / 64;
    int by_lds = (160 * 1024) / ((st + kStackPad) * slots * 4 + waves * (3 * 64 * 4 + 96));   // stacks, hand-off, poses
    int by_waves = 32 / waves;          // at most 8 waves per SIMD
    int b = by_lds < by_waves ? by_lds : by_waves;
    return b < 1 ? 1 : b;
}

}  // namespace lidar
