// dynamic.hip -- dynamic scenes on gfx950: meshes placed in the world by
// moving actors (Section II-B labels every object instance; an actor is one
// labelled instance of a mesh).
//
// * A mesh has its own 4-wide BVH over object-space triangles (built by the
//   scene builder).  A deformed mesh (same topology, new vertices) is refit:
//   its records are rewritten from the new vertices and every node's child
//   boxes are recomputed level by level, deepest level first.
// * The actors' world boxes (the mesh root box, its 8 corners transformed in
//   FP64, rounded outward) are the primitives of a top-level BVH, built by the
//   same builder from degenerate triangles (lo, hi, lo) whose bounding box is
//   exactly the actor box.  A per-frame update rewrites those records from the
//   new boxes and refits the tree; a rebuild (new actor set) builds it again.
//   Up to a few thousand actors the tree is instead rebuilt on every update by
//   one workgroup (Morton order, four entries per node), which costs less than
//   the refit and keeps the tree tight as the actors move.
// Refit reproduces the builder's boxes exactly for unchanged inputs: a leaf
// slot is the union of its records' vertices minus/plus the pad, an inner slot
// the union of its child node's (padded) slots, and the pad is 2^-20 of the
// larger of the largest coordinate and the tree's reach, as in the build.
#include "lidar_kernels.hpp"

namespace lidar {

namespace {

constexpr float kInf = __builtin_inff();

// word[0] = bits of max |x| over the values (non-negative floats order like their bits)
__global__ __launch_bounds__(256) void maxabs_kernel(const float *__restrict__ v, uint64_t n, uint32_t *word) {
    float m = 0.0f;
    for (uint64_t k = blockIdx.x * 256ull + threadIdx.x; k < n; k += (uint64_t)gridDim.x * 256ull)
        m = fmaxf(m, fabsf(v[k]));
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(word, __float_as_uint(m));
}

__global__ void zero_words_kernel(uint32_t *word) {
    word[0] = 0u;
    word[1] = 0u;
}

// word[1] = bits of the box pad 2^-20 max(max |x|, reach) + 1e-20 (the builder's formula)
__global__ void pad_kernel(uint32_t *word, float reach) {
    word[1] = __float_as_uint(fmaxf(__uint_as_float(word[0]), reach) * 9.5367431640625e-07f + 1e-20f);
}

__global__ __launch_bounds__(256) void mesh_records_kernel(TriRec *__restrict__ recs, uint32_t nt,
                                                           const uint32_t *__restrict__ idx,
                                                           const float *__restrict__ v) {
    uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= nt) return;
    TriRec r = recs[s];
    uint32_t k = __float_as_uint(r.a.w);
    uint32_t i0 = idx[3 * (size_t)k], i1 = idx[3 * (size_t)k + 1], i2 = idx[3 * (size_t)k + 2];
    r.a.x = v[3 * (size_t)i0]; r.a.y = v[3 * (size_t)i0 + 1]; r.a.z = v[3 * (size_t)i0 + 2];
    r.b.x = v[3 * (size_t)i1]; r.b.y = v[3 * (size_t)i1 + 1]; r.b.z = v[3 * (size_t)i1 + 2];
    r.c.x = v[3 * (size_t)i2]; r.c.y = v[3 * (size_t)i2 + 1]; r.c.z = v[3 * (size_t)i2 + 2];
    recs[s] = r;
}

__device__ inline float round_down(double x) {
    float f = (float)x;
    return ((double)f > x) ? nextafterf(f, -kInf) : f;
}
__device__ inline float round_up(double x) {
    float f = (float)x;
    return ((double)f < x) ? nextafterf(f, kInf) : f;
}

// the box of a mesh: the union of its root's slots
__device__ inline void mesh_root_box(const MeshDev *__restrict__ meshes, uint32_t mesh, float lo[3], float hi[3]) {
    const Node4 root = meshes[mesh].nodes[0];
    for (int e = 0; e < 3; ++e) {
        lo[e] = kInf;
        hi[e] = -kInf;
    }
    for (int k = 0; k < 4; ++k) {
        if (root.c[k].ref == kEmptyRef) continue;
        for (int e = 0; e < 3; ++e) {
            lo[e] = fminf(lo[e], root.c[k].lo[e]);
            hi[e] = fmaxf(hi[e], root.c[k].hi[e]);
        }
    }
}

// world box of an actor (anything with R and p) whose mesh box is (lo, hi):
// its 8 corners transformed in FP64, rounded outward
template <class Xf>
__device__ inline void actor_box_from(const Xf &A, const float lo[3], const float hi[3], float lo_w[3],
                                      float hi_w[3]) {
    double wl[3] = {1e300, 1e300, 1e300}, wh[3] = {-1e300, -1e300, -1e300};
    for (int c = 0; c < 8; ++c) {
        const double x = (c & 1) ? hi[0] : lo[0], y = (c & 2) ? hi[1] : lo[1], z = (c & 4) ? hi[2] : lo[2];
        for (int e = 0; e < 3; ++e) {
            const double w = A.R[3 * e] * x + A.R[3 * e + 1] * y + A.R[3 * e + 2] * z + A.p[e];
            wl[e] = fmin(wl[e], w);
            wh[e] = fmax(wh[e], w);
        }
    }
    for (int e = 0; e < 3; ++e) {
        lo_w[e] = round_down(wl[e]);
        hi_w[e] = round_up(wh[e]);
    }
}

__device__ inline void actor_box_of(const ActorDev &A, const MeshDev *__restrict__ meshes, float lo_w[3],
                                    float hi_w[3]) {
    float lo[3], hi[3];
    mesh_root_box(meshes, A.mesh, lo, hi);
    actor_box_from(A, lo, hi, lo_w, hi_w);
}

// world box of actor a into lohi; returns max |coordinate|
__device__ inline float actor_box(const ActorDev *__restrict__ actors, uint32_t a,
                                  const MeshDev *__restrict__ meshes, float *__restrict__ lohi) {
    float lo[3], hi[3], m = 0.0f;
    actor_box_of(actors[a], meshes, lo, hi);
    for (int e = 0; e < 3; ++e) {
        lohi[6 * (size_t)a + e] = lo[e];
        lohi[6 * (size_t)a + 3 + e] = hi[e];
        m = fmaxf(m, fmaxf(fabsf(lo[e]), fabsf(hi[e])));
    }
    return m;
}

// world box of each actor; also max |coordinate| of all boxes into word[0]
__global__ __launch_bounds__(256) void actor_boxes_kernel(const ActorDev *__restrict__ actors, uint32_t n,
                                                          const MeshDev *__restrict__ meshes, float *__restrict__ lohi,
                                                          uint32_t *word) {
    uint32_t a = blockIdx.x * 256 + threadIdx.x;
    float m = 0.0f;
    if (a < n) m = actor_box(actors, a, meshes, lohi);
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(word, __float_as_uint(m));
}

// builder input for the top-level BVH: vertices 2a = lo, 2a + 1 = hi, triangle (lo, hi, lo)
__global__ __launch_bounds__(256) void actor_prims_kernel(const float *__restrict__ lohi, uint32_t n,
                                                          float *__restrict__ vtx, uint32_t *__restrict__ idx,
                                                          uint16_t *__restrict__ mat) {
    uint32_t a = blockIdx.x * 256 + threadIdx.x;
    if (a >= n) return;
    for (int e = 0; e < 6; ++e) vtx[6 * (size_t)a + e] = lohi[6 * (size_t)a + e];
    idx[3 * (size_t)a] = 2 * a;
    idx[3 * (size_t)a + 1] = 2 * a + 1;
    idx[3 * (size_t)a + 2] = 2 * a;
    mat[a] = 0;
}

__global__ __launch_bounds__(256) void tlas_records_kernel(TriRec *__restrict__ recs, uint32_t n,
                                                           const float *__restrict__ lohi) {
    uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    TriRec r = recs[s];
    const uint32_t a = __float_as_uint(r.a.w);
    const float *b = lohi + 6 * (size_t)a;
    r.a.x = b[0]; r.a.y = b[1]; r.a.z = b[2];
    r.b.x = b[3]; r.b.y = b[4]; r.b.z = b[5];
    r.c.x = b[0]; r.c.y = b[1]; r.c.z = b[2];
    recs[s] = r;
}

// the child boxes of node n from its children (records or child nodes, already refit)
__device__ inline void refit_node(Node4 *__restrict__ nodes, const TriRec *__restrict__ recs, uint32_t n, float pad) {
    Node4 nd = nodes[n];
    for (int k = 0; k < 4; ++k) {
        const uint32_t ref = nd.c[k].ref;
        if (ref == kEmptyRef) continue;
        float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
        if (ref & kLeafBit) {
            const uint32_t f = leaf_first(ref), c = leaf_count(ref);
            for (uint32_t r = 0; r < c; ++r) {
                const TriRec t = recs[f + r];
                lo[0] = fminf(lo[0], fminf(t.a.x, fminf(t.b.x, t.c.x)));
                lo[1] = fminf(lo[1], fminf(t.a.y, fminf(t.b.y, t.c.y)));
                lo[2] = fminf(lo[2], fminf(t.a.z, fminf(t.b.z, t.c.z)));
                hi[0] = fmaxf(hi[0], fmaxf(t.a.x, fmaxf(t.b.x, t.c.x)));
                hi[1] = fmaxf(hi[1], fmaxf(t.a.y, fmaxf(t.b.y, t.c.y)));
                hi[2] = fmaxf(hi[2], fmaxf(t.a.z, fmaxf(t.b.z, t.c.z)));
            }
            for (int e = 0; e < 3; ++e) {
                lo[e] = lo[e] - pad;
                hi[e] = hi[e] + pad;
            }
        } else {
            const Node4 &ch = nodes[ref];
            for (int j = 0; j < 4; ++j) {
                if (ch.c[j].ref == kEmptyRef) continue;
                for (int e = 0; e < 3; ++e) {
                    lo[e] = fminf(lo[e], ch.c[j].lo[e]);
                    hi[e] = fmaxf(hi[e], ch.c[j].hi[e]);
                }
            }
        }
        for (int e = 0; e < 3; ++e) {
            nd.c[k].lo[e] = lo[e];
            nd.c[k].hi[e] = hi[e];
        }
    }
    nodes[n] = nd;
}

__global__ __launch_bounds__(256) void refit_level_kernel(Node4 *__restrict__ nodes, const TriRec *__restrict__ recs,
                                                          uint32_t first, uint32_t count,
                                                          const uint32_t *__restrict__ word) {
    const uint32_t n = blockIdx.x * 256 + threadIdx.x;
    if (n < count) refit_node(nodes, recs, first + n, __uint_as_float(word[1]));
}

// Small trees (a few thousand nodes) refit in one workgroup: the phases and the
// levels are separated by workgroup barriers instead of kernel launches, which
// would cost more than the work.  Same operations, same results.
constexpr uint32_t kSmallRefitThreads = 1024;
constexpr uint32_t kSmallRefitNodes = 4096;

struct Levels {
    uint32_t depth;
    uint32_t base[kMaxLevels + 1];
};

__device__ inline void refit_levels_block(Node4 *__restrict__ nodes, const TriRec *__restrict__ recs,
                                          const Levels &L, float pad) {
    for (int l = (int)L.depth - 1; l >= 0; --l) {
        for (uint32_t n = L.base[l] + threadIdx.x; n < L.base[l + 1]; n += kSmallRefitThreads)
            refit_node(nodes, recs, n, pad);
        __syncthreads();
    }
}

// Trees of up to kLdsRefitNodes nodes keep each node's box (the union of its
// child slots) in LDS.  Every thread owns nodes t and t + 1024: it first reads
// their child references and computes their leaf slots from the records (all
// nodes at once), then, level by level, deepest first, fills their inner slots
// from the children's boxes in LDS.  Only the leaf slots read global memory,
// so the refit costs a few memory round trips instead of two per level.  The
// slot boxes are the same unions as refit_node's.
constexpr uint32_t kLdsRefitNodes = 2 * kSmallRefitThreads;

__device__ inline void refit_levels_lds(Node4 *__restrict__ nodes, const TriRec *__restrict__ recs,
                                        const Levels &L, float pad, float (*box)[6]) {
    const uint32_t n_nodes = L.base[L.depth];
    uint32_t refs[2][4];
    for (int o = 0; o < 2; ++o) {
        const uint32_t n = threadIdx.x + o * kSmallRefitThreads;
        if (n >= n_nodes) continue;
        float u[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
        for (int k = 0; k < 4; ++k) {
            const uint32_t ref = nodes[n].c[k].ref;
            refs[o][k] = ref;
            if (ref == kEmptyRef || !(ref & kLeafBit)) continue;
            float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
            const uint32_t f = leaf_first(ref), c = leaf_count(ref);
            for (uint32_t r = 0; r < c; ++r) {
                const TriRec t = recs[f + r];
                lo[0] = fminf(lo[0], fminf(t.a.x, fminf(t.b.x, t.c.x)));
                lo[1] = fminf(lo[1], fminf(t.a.y, fminf(t.b.y, t.c.y)));
                lo[2] = fminf(lo[2], fminf(t.a.z, fminf(t.b.z, t.c.z)));
                hi[0] = fmaxf(hi[0], fmaxf(t.a.x, fmaxf(t.b.x, t.c.x)));
                hi[1] = fmaxf(hi[1], fmaxf(t.a.y, fmaxf(t.b.y, t.c.y)));
                hi[2] = fmaxf(hi[2], fmaxf(t.a.z, fmaxf(t.b.z, t.c.z)));
            }
            for (int e = 0; e < 3; ++e) {
                lo[e] = lo[e] - pad;
                hi[e] = hi[e] + pad;
                nodes[n].c[k].lo[e] = lo[e];
                nodes[n].c[k].hi[e] = hi[e];
                u[e] = fminf(u[e], lo[e]);
                u[3 + e] = fmaxf(u[3 + e], hi[e]);
            }
        }
        for (int e = 0; e < 6; ++e) box[n][e] = u[e];
    }
    __syncthreads();
    for (int l = (int)L.depth - 1; l >= 0; --l) {
        for (int o = 0; o < 2; ++o) {
            const uint32_t n = threadIdx.x + o * kSmallRefitThreads;
            if (n < L.base[l] || n >= L.base[l + 1]) continue;
            float u[6];
            for (int e = 0; e < 6; ++e) u[e] = box[n][e];
            for (int k = 0; k < 4; ++k) {
                const uint32_t ref = refs[o][k];
                if (ref == kEmptyRef || (ref & kLeafBit)) continue;
                for (int e = 0; e < 3; ++e) {
                    const float lo = box[ref][e], hi = box[ref][3 + e];
                    nodes[n].c[k].lo[e] = lo;
                    nodes[n].c[k].hi[e] = hi;
                    u[e] = fminf(u[e], lo);
                    u[3 + e] = fmaxf(u[3 + e], hi);
                }
            }
            for (int e = 0; e < 6; ++e) box[n][e] = u[e];
        }
        __syncthreads();
    }
}

// max |x| over a block's values into LDS, then the builder's pad formula
__device__ inline float block_pad(float m, uint32_t *lds_max, float reach) {
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(lds_max, __float_as_uint(m));
    __syncthreads();
    return fmaxf(__uint_as_float(*lds_max), reach) * 9.5367431640625e-07f + 1e-20f;
}

__global__ __launch_bounds__(kSmallRefitThreads) void refit_mesh_small_kernel(Node4 *__restrict__ nodes,
                                                                              TriRec *__restrict__ recs, Levels L,
                                                                              uint32_t nt,
                                                                              const uint32_t *__restrict__ idx,
                                                                              const float *__restrict__ v,
                                                                              uint64_t nv, float reach) {
    __shared__ uint32_t lds_max;
    __shared__ float box[kLdsRefitNodes][6];
    if (threadIdx.x == 0) lds_max = 0u;
    __syncthreads();
    float m = 0.0f;
    for (uint64_t k = threadIdx.x; k < 3 * nv; k += kSmallRefitThreads) m = fmaxf(m, fabsf(v[k]));
    const float pad = block_pad(m, &lds_max, reach);
    for (uint32_t s = threadIdx.x; s < nt; s += kSmallRefitThreads) {
        TriRec r = recs[s];
        const uint32_t k = __float_as_uint(r.a.w);
        const uint32_t i0 = idx[3 * (size_t)k], i1 = idx[3 * (size_t)k + 1], i2 = idx[3 * (size_t)k + 2];
        r.a.x = v[3 * (size_t)i0]; r.a.y = v[3 * (size_t)i0 + 1]; r.a.z = v[3 * (size_t)i0 + 2];
        r.b.x = v[3 * (size_t)i1]; r.b.y = v[3 * (size_t)i1 + 1]; r.b.z = v[3 * (size_t)i1 + 2];
        r.c.x = v[3 * (size_t)i2]; r.c.y = v[3 * (size_t)i2 + 1]; r.c.z = v[3 * (size_t)i2 + 2];
        recs[s] = r;
    }
    __syncthreads();
    if (L.base[L.depth] <= kLdsRefitNodes) refit_levels_lds(nodes, recs, L, pad, box);
    else refit_levels_block(nodes, recs, L, pad);
}

// per-frame update of a small top-level BVH: actor boxes, pad, leaf records, levels
__global__ __launch_bounds__(kSmallRefitThreads) void update_tlas_small_kernel(const ActorDev *__restrict__ actors,
                                                                               uint32_t n,
                                                                               const MeshDev *__restrict__ meshes,
                                                                               float *__restrict__ lohi,
                                                                               Node4 *__restrict__ nodes,
                                                                               TriRec *__restrict__ recs, Levels L,
                                                                               float reach) {
    __shared__ uint32_t lds_max;
    __shared__ float box[kLdsRefitNodes][6];
    if (threadIdx.x == 0) lds_max = 0u;
    __syncthreads();
    float m = 0.0f;
    for (uint32_t a = threadIdx.x; a < n; a += kSmallRefitThreads) m = fmaxf(m, actor_box(actors, a, meshes, lohi));
    const float pad = block_pad(m, &lds_max, reach);     // its barrier also publishes the boxes
    for (uint32_t s = threadIdx.x; s < n; s += kSmallRefitThreads) {
        TriRec r = recs[s];
        const float *b = lohi + 6 * (size_t)__float_as_uint(r.a.w);
        r.a.x = b[0]; r.a.y = b[1]; r.a.z = b[2];
        r.b.x = b[3]; r.b.y = b[4]; r.b.z = b[5];
        r.c.x = b[0]; r.c.y = b[1]; r.c.z = b[2];
        recs[s] = r;
    }
    __syncthreads();
    if (L.base[L.depth] <= kLdsRefitNodes) refit_levels_lds(nodes, recs, L, pad, box);
    else refit_levels_block(nodes, recs, L, pad);
}

// Small actor sets: the top-level tree is rebuilt in one workgroup on every
// update.  The actors are put in Morton order of their box centres within the
// static scene's cube (one scale for the three axes, so a street scene, flat
// against its extent, orders mostly by x and y), each record is one actor, and
// every node packs four consecutive entries of the level below, up to the
// root.  A rebuild stays as tight as a fresh build however far the actors
// move, where the refit of a tree built for the first frame loosens as they
// drift apart.  A leaf slot is the actor's box widened by the pad and an inner
// slot the union of its child's slots, as in the builder's tree, so the walk
// returns the same hits on either tree.
// The actors are read from `src` (a per-frame upload, which may be pinned host
// memory read over the bus) and copied to `actors`, where the scan reads them.
// Up to one actor per thread, each thread finds its actor's place in the order
// by counting the smaller keys and writes its record and leaf slot directly;
// larger sets sort the keys with a bitonic network.  With up to kRootCache
// meshes their root boxes are fetched into LDS while the actors are read, so
// the two fetches overlap instead of following each other.
constexpr uint32_t kPackedNodesMax = 1365;   // 1024 + 256 + 64 + 16 + 4 + 1 nodes for kPackedTlasMax actors
constexpr uint32_t kRootCache = 256;
static_assert(kPackedTlasMax == 4 * kSmallRefitThreads, "one bottom node per thread");

// bit b of v moved to bit 3 b
__device__ inline uint32_t spread3(uint32_t v) {
    uint32_t r = 0u;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

// an actor's transform and mesh, read as the seven 16-byte words of its ActorDev
static_assert(sizeof(ActorDev) == 112 && offsetof(ActorDev, p) == 72 && offsetof(ActorDev, mesh) == 96,
              "ActorDev layout");
struct ActorWords {
    float4 w[7];
    __device__ inline double dbl(int k) const {    // double k of the record (k < 12)
        const float4 &v = w[k >> 1];
        return (k & 1) ? __hiloint2double(__float_as_int(v.w), __float_as_int(v.z))
                       : __hiloint2double(__float_as_int(v.y), __float_as_int(v.x));
    }
    __device__ inline uint32_t mesh() const { return __float_as_uint(w[6].x); }
};
struct ActorXf {
    double R[9], p[3];
    uint32_t mesh;
};
// actor a of src: copied to dst (unless the same), its transform and mesh returned
__device__ inline ActorXf take_actor(const ActorDev *__restrict__ src, ActorDev *__restrict__ dst, uint32_t a) {
    ActorWords r;
    const float4 *q = reinterpret_cast<const float4 *>(src + a);
    for (int k = 0; k < 7; ++k) r.w[k] = q[k];
    if (src != dst) {
        float4 *d = reinterpret_cast<float4 *>(dst + a);
        for (int k = 0; k < 7; ++k) d[k] = r.w[k];
    }
    ActorXf X;
    for (int k = 0; k < 9; ++k) X.R[k] = r.dbl(k);
    for (int e = 0; e < 3; ++e) X.p[e] = r.dbl(9 + e);
    X.mesh = r.mesh();
    return X;
}

__device__ inline void empty_slot(Child4 &c) {
    for (int e = 0; e < 3; ++e) c.lo[e] = c.hi[e] = 1e30f;
    c.ref = kEmptyRef;
    c.pad = 0u;
}

__global__ __launch_bounds__(kSmallRefitThreads) void rebuild_tlas_small_kernel(const ActorDev *__restrict__ src,
                                                                                ActorDev *__restrict__ actors,
                                                                                uint32_t n,
                                                                                const MeshDev *__restrict__ meshes,
                                                                                uint32_t n_meshes,
                                                                                float *__restrict__ lohi,
                                                                                Node4 *__restrict__ nodes,
                                                                                TriRec *__restrict__ recs, Levels L,
                                                                                float reach) {
    __shared__ uint32_t lds_max;
    __shared__ float mbox[kRootCache][6];
    // the sort keys, then (once the records are written) the boxes of the nodes
    __shared__ union {
        uint64_t key[kPackedTlasMax];
        float box[kPackedNodesMax][6];
    } u;
    __shared__ float sbox[kSmallRefitThreads][6];   // leaf slots in Morton order (one actor per thread)
    const uint32_t t = threadIdx.x;
    if (t == 0) lds_max = 0u;
    const bool cached = n_meshes <= kRootCache;
    // the first actor of every thread is read before the mesh boxes are fetched
    const ActorXf X0 = take_actor(src, t < n ? actors : const_cast<ActorDev *>(src), t < n ? t : 0);
    if (cached && t < n_meshes) {
        float l[3], h[3];
        mesh_root_box(meshes, t, l, h);
        for (int e = 0; e < 3; ++e) {
            mbox[t][e] = l[e];
            mbox[t][3 + e] = h[e];
        }
    }
    __syncthreads();
    const float half = reach > 0.0f ? reach : 1.0f;
    const float scale = 1023.0f / (2.0f * half);
    float m = 0.0f, lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {0.0f, 0.0f, 0.0f};
    // actor a: copy for the scan, world box, its Morton key
    auto place = [&](const ActorXf &X, uint32_t a) {
        const uint32_t mesh = X.mesh;
        float ml[3], mh[3];
        if (cached) {
            for (int e = 0; e < 3; ++e) {
                ml[e] = mbox[mesh][e];
                mh[e] = mbox[mesh][3 + e];
            }
        } else {
            mesh_root_box(meshes, mesh, ml, mh);
        }
        actor_box_from(X, ml, mh, lo, hi);
        uint32_t code = 0u;
        for (int e = 0; e < 3; ++e) {
            lohi[6 * (size_t)a + e] = lo[e];
            lohi[6 * (size_t)a + 3 + e] = hi[e];
            m = fmaxf(m, fmaxf(fabsf(lo[e]), fabsf(hi[e])));
            const float q = (0.5f * (lo[e] + hi[e]) + half) * scale;
            const uint32_t qi = q > 0.0f ? (q < 1023.0f ? (uint32_t)q : 1023u) : 0u;
            code |= spread3(qi) << e;
        }
        u.key[a] = ((uint64_t)code << 32) | a;     // unique: the actor index breaks ties
    };
    if (n <= kSmallRefitThreads) {
        if (t < n) place(X0, t);
    } else {
        for (uint32_t a = t; a < n; a += kSmallRefitThreads) place(a == t ? X0 : take_actor(src, actors, a), a);
    }
    const uint32_t D = L.depth, bb = L.base[D - 1], nb = L.base[D] - bb;
    if (n <= kSmallRefitThreads) {
        const float pad = block_pad(m, &lds_max, reach);     // its barrier also publishes the keys
        if (t < n) {
            const uint64_t mine = u.key[t];
            uint32_t r = 0u;
            for (uint32_t j = 0; j < n; ++j) r += u.key[j] < mine ? 1u : 0u;
            TriRec rec;
            rec.a = make_float4(lo[0], lo[1], lo[2], __uint_as_float(t));
            rec.b = make_float4(hi[0], hi[1], hi[2], __uint_as_float(0u));
            rec.c = make_float4(lo[0], lo[1], lo[2], __uint_as_float(0u));
            recs[r] = rec;
            Child4 c;
            for (int e = 0; e < 3; ++e) {
                c.lo[e] = lo[e] - pad;
                c.hi[e] = hi[e] + pad;
                sbox[r][e] = c.lo[e];
                sbox[r][3 + e] = c.hi[e];
            }
            c.ref = leaf_ref(r, 1u);
            c.pad = 0u;
            nodes[bb + r / 4].c[r % 4] = c;
        }
        __syncthreads();      // every key read and every leaf slot in sbox
        if (t < nb) {
            float un[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
            for (uint32_t k = 0; k < 4; ++k) {
                const uint32_t s = 4 * t + k;
                if (s >= n) {
                    Child4 c;
                    empty_slot(c);
                    nodes[bb + t].c[k] = c;
                    continue;
                }
                for (int e = 0; e < 3; ++e) {
                    un[e] = fminf(un[e], sbox[s][e]);
                    un[3 + e] = fmaxf(un[3 + e], sbox[s][3 + e]);
                }
            }
            for (int e = 0; e < 6; ++e) u.box[bb + t][e] = un[e];
        }
    } else {
        uint32_t P = 2;
        while (P < n) P <<= 1;
        for (uint32_t a = n + t; a < P; a += kSmallRefitThreads) u.key[a] = ~0ull;
        const float pad = block_pad(m, &lds_max, reach);     // its barrier also publishes the keys and boxes
        // bitonic sort of the P keys
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = t; i < P; i += kSmallRefitThreads) {
                    const uint32_t l = i ^ j;
                    if (l > i) {
                        const uint64_t x = u.key[i], y = u.key[l];
                        if ((x > y) == ((i & k) == 0)) {
                            u.key[i] = y;
                            u.key[l] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // bottom level: node t holds records 4t .. 4t + 3, record s is the s-th actor in Morton order
        uint32_t act[4];
        for (int k = 0; k < 4; ++k) {
            const uint32_t s = 4 * t + k;
            act[k] = (t < nb && s < n) ? (uint32_t)u.key[s] : kNone;
        }
        __syncthreads();     // every key read: the LDS now holds node boxes
        if (t < nb) {
            Node4 nd;
            float un[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
            for (int k = 0; k < 4; ++k) {
                if (act[k] == kNone) {
                    empty_slot(nd.c[k]);
                    continue;
                }
                const uint32_t s = 4 * t + k;
                const float *b = lohi + 6 * (size_t)act[k];
                TriRec r;
                r.a = make_float4(b[0], b[1], b[2], __uint_as_float(act[k]));
                r.b = make_float4(b[3], b[4], b[5], __uint_as_float(0u));
                r.c = make_float4(b[0], b[1], b[2], __uint_as_float(0u));
                recs[s] = r;
                for (int e = 0; e < 3; ++e) {
                    nd.c[k].lo[e] = b[e] - pad;
                    nd.c[k].hi[e] = b[3 + e] + pad;
                    un[e] = fminf(un[e], nd.c[k].lo[e]);
                    un[3 + e] = fmaxf(un[3 + e], nd.c[k].hi[e]);
                }
                nd.c[k].ref = leaf_ref(s, 1u);
                nd.c[k].pad = 0u;
            }
            nodes[bb + t] = nd;
            for (int e = 0; e < 6; ++e) u.box[bb + t][e] = un[e];
        }
    }
    // the levels above, each node over four consecutive nodes of the level below
    for (int l = (int)D - 2; l >= 0; --l) {
        __syncthreads();
        const uint32_t b0 = L.base[l], cnt = L.base[l + 1] - b0, cb = L.base[l + 1], ccnt = L.base[l + 2] - cb;
        if (t < cnt) {
            Node4 nd;
            float un[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
            for (int k = 0; k < 4; ++k) {
                const uint32_t j = 4 * t + k;
                if (j >= ccnt) {
                    empty_slot(nd.c[k]);
                    continue;
                }
                for (int e = 0; e < 3; ++e) {
                    nd.c[k].lo[e] = u.box[cb + j][e];
                    nd.c[k].hi[e] = u.box[cb + j][3 + e];
                    un[e] = fminf(un[e], nd.c[k].lo[e]);
                    un[3 + e] = fmaxf(un[3 + e], nd.c[k].hi[e]);
                }
                nd.c[k].ref = cb + j;
                nd.c[k].pad = 0u;
            }
            nodes[b0 + t] = nd;
            for (int e = 0; e < 6; ++e) u.box[b0 + t][e] = un[e];
        }
    }
}

Levels levels_of(const BuildResult &br) {
    Levels L{};
    L.depth = br.depth;
    for (uint32_t l = 0; l <= br.depth && l <= (uint32_t)kMaxLevels; ++l) L.base[l] = br.level_base[l];
    return L;
}

inline uint32_t grid_of(uint64_t n) { return (uint32_t)((n + 255) / 256); }

// child boxes of every node, deepest level first
void refit_tree(Node4 *nodes, const TriRec *recs, const BuildResult &br, const uint32_t *word, hipStream_t s) {
    for (int L = (int)br.depth - 1; L >= 0; --L) {
        const uint32_t first = br.level_base[L], count = br.level_base[L + 1] - first;
        if (count) refit_level_kernel<<<grid_of(count), 256, 0, s>>>(nodes, recs, first, count, word);
    }
}

}  // namespace

bool refit_supported(const BuildResult &br) { return br.depth >= 1 && br.depth <= (uint32_t)kMaxLevels; }

void refit_mesh(Node4 *nodes, TriRec *recs, const BuildResult &br, uint32_t nt, const uint32_t *idx,
                const float *vertices, uint64_t nv, uint32_t *word, hipStream_t s) {
    if (br.n_nodes <= kSmallRefitNodes) {
        refit_mesh_small_kernel<<<1, kSmallRefitThreads, 0, s>>>(nodes, recs, levels_of(br), nt, idx, vertices, nv,
                                                                 br.reach);
        return;
    }
    zero_words_kernel<<<1, 1, 0, s>>>(word);
    uint32_t g = grid_of(3 * nv);
    maxabs_kernel<<<g < 1024 ? g : 1024, 256, 0, s>>>(vertices, 3 * nv, word);
    pad_kernel<<<1, 1, 0, s>>>(word, br.reach);
    mesh_records_kernel<<<grid_of(nt), 256, 0, s>>>(recs, nt, idx, vertices);
    refit_tree(nodes, recs, br, word, s);
}

void actor_boxes(const ActorDev *actors, uint32_t n, const MeshDev *meshes, float *lohi, uint32_t *word,
                 hipStream_t s) {
    zero_words_kernel<<<1, 1, 0, s>>>(word);
    actor_boxes_kernel<<<grid_of(n), 256, 0, s>>>(actors, n, meshes, lohi, word);
}

void actor_prims(const float *lohi, uint32_t n, float *vtx, uint32_t *idx, uint16_t *mat, hipStream_t s) {
    actor_prims_kernel<<<grid_of(n), 256, 0, s>>>(lohi, n, vtx, idx, mat);
}

void update_tlas(const ActorDev *actors, uint32_t n, const MeshDev *meshes, float *lohi, Node4 *nodes,
                 TriRec *recs, const BuildResult &br, uint32_t *word, hipStream_t s) {
    if (br.n_nodes <= kSmallRefitNodes && n <= 4 * kSmallRefitNodes) {
        update_tlas_small_kernel<<<1, kSmallRefitThreads, 0, s>>>(actors, n, meshes, lohi, nodes, recs, levels_of(br),
                                                                  br.reach);
        return;
    }
    actor_boxes(actors, n, meshes, lohi, word, s);
    refit_tlas(nodes, recs, br, n, lohi, word, s);
}

BuildResult packed_tlas_shape(uint32_t n, float reach) {
    BuildResult br{};
    uint32_t size[kMaxLevels], depth = 0;
    uint32_t c = n;
    do {                               // level sizes from the bottom: ceil(c / 4) nodes over c entries
        c = (c + 3) / 4;
        size[depth++] = c;
    } while (c > 1);
    br.root = 0;
    br.depth = depth;
    br.n_leaves = n;
    br.reach = reach;
    br.level_base[0] = 0;
    for (uint32_t l = 0; l < depth; ++l) br.level_base[l + 1] = br.level_base[l] + size[depth - 1 - l];
    br.n_nodes = br.level_base[depth];
    return br;
}

void rebuild_tlas(const ActorDev *src, ActorDev *actors, uint32_t n, const MeshDev *meshes, uint32_t n_meshes,
                  float *lohi, Node4 *nodes, TriRec *recs, const BuildResult &shape, hipStream_t s) {
    rebuild_tlas_small_kernel<<<1, kSmallRefitThreads, 0, s>>>(src, actors, n, meshes, n_meshes, lohi, nodes, recs,
                                                               levels_of(shape), shape.reach);
}

void refit_tlas(Node4 *nodes, TriRec *recs, const BuildResult &br, uint32_t n, const float *lohi, uint32_t *word,
                hipStream_t s) {
    pad_kernel<<<1, 1, 0, s>>>(word, br.reach);
    tlas_records_kernel<<<grid_of(n), 256, 0, s>>>(recs, n, lohi);
    refit_tree(nodes, recs, br, word, s);
}

}  // namespace lidar
