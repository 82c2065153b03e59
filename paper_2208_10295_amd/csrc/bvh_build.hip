// bvh_build.hip -- GPU construction of the 4-wide BVH (gfx950).
//
// 1. per triangle: index validation, centroid, scene bounds (block partials)
// 2. 63-bit Morton code of the centroid (21 bits per axis) -> stable LSD radix
//    sort of (code, triangle) pairs, 8 passes of 8 bits
// 3. triangle records written in sorted order (leaves are contiguous ranges)
// 4. binary tree, either
//    (a) PLOC (default; Meister and Bittner, "Parallel Locally-Ordered
//        Clustering for Bounding Volume Hierarchy Construction", TVCG 2018):
//        clusters in Morton order repeatedly find their nearest neighbour
//        (smallest merged surface area, its horizontal faces optionally
//        weighted below the vertical ones for rays near the horizontal; the
//        collapse's cost uses the same metric) within +-R positions (R = 32 by
//        default, at most 128); mutual nearest
//        pairs merge into a new node; the survivors are compacted in order.
//        Boxes are formed during the merges.  The leaves are then renumbered
//        depth-first so that every subtree covers a contiguous range of
//        triangle records; or
//    (b) LBVH: binary radix tree over the sorted codes (Karras, HPG 2012),
//        identical codes split by position, then a bottom-up bounding-box
//        refit where the second child to arrive at a node computes its box
// 5. (nothing: both trees have their boxes)
// 6. level-synchronous collapse to 4 children.  By default the shape comes
//    from a surface-area cost minimised over the binary tree (the dynamic
//    programme of Ylitie, Karras and Laine, "Efficient incoherent ray
//    traversal on GPUs through compressed wide BVHs", HPG 2017, for 4 slots):
//    bottom-up, every binary node n gets the least cost C(n, i) of covering its
//    subtree with at most i children of a 4-wide node, where a child is either
//    a leaf of <= leaf_width triangles (cost: leaf weight x area) or a 4-wide
//    node (node weight x area + the best split of its binary children over 4
//    slots); the walk fetches a node's 4 boxes, or a leaf's triangles, in one
//    step, hence one weight per step kind.  The collapse then follows the
//    recorded choices top-down.  The greedy alternative replaces, starting
//    from the node's two children, the child with the largest surface area
//    that holds more than leaf_width triangles by its two children until there
//    are 4; children with <= leaf_width triangles become leaves.  New nodes of
//    a level are numbered by an exclusive scan, so the layout is deterministic
//    and breadth-first.
// Child boxes are padded outward by 2^-20 of M = max(largest |vertex
// coordinate|, reach).  The FP32 slab distance fma(b, 1/d, -o/d) is off by at
// most 2^-24 (2|b_i| + 3|o_i|) along axis i, and the watertight test's distance
// by a few units of 2^-24 (|v| + |o|); with |b_i|, |o_i| <= M both stay below
// the pad 16 * 2^-24 M, so for every ray origin inside the cube
// |x|, |y|, |z| <= M the walk never culls a triangle the test accepts.
#include <utility>
#include <vector>

#include "lidar_kernels.hpp"

namespace lidar {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan of one value per thread over a 256-thread block
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *lds_w /*[4]*/, uint32_t &total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds_w[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    total = 0;
    for (int k = 0; k < 4; ++k) {
        uint32_t t = lds_w[k];
        if (k < w) off += t;
        total += t;
    }
    __syncthreads();
    return off + inc - v;
}
}  // namespace

// ---------------------------------------------------------------------------
// exclusive scan (3 phases)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t *__restrict__ in, uint32_t n,
                                                                   uint32_t *__restrict__ sums) {
    __shared__ uint32_t w4[4];
    uint32_t base = blockIdx.x * kScanTile;
    uint32_t v = 0;
    for (int k = 0; k < kScanItems; ++k) {
        uint32_t idx = base + k * kScanThreads + threadIdx.x;
        if (idx < n) v += in[idx];
    }
    uint32_t total;
    block_excl_scan(v, w4, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(uint32_t *sums, uint32_t nb) {
    __shared__ uint32_t w4[4];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanThreads) {
        uint32_t idx = base + threadIdx.x;
        uint32_t v = idx < nb ? sums[idx] : 0;
        uint32_t total;
        uint32_t ex = block_excl_scan(v, w4, total);
        if (idx < nb) sums[idx] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t *__restrict__ in, uint32_t *out,
                                                                  uint32_t n, const uint32_t *__restrict__ sums) {
    __shared__ uint32_t w4[4];
    // each thread owns kScanItems consecutive elements
    uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t t = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        t += v[k];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan(t, w4, total) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

size_t scan_tmp_bytes(uint32_t n) { return align_up(((size_t)n + kScanTile - 1) / kScanTile * 4 + 4, 256); }

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *tmp, hipStream_t s) {
    if (n == 0) return;
    uint32_t nb = (n + kScanTile - 1) / kScanTile;
    scan_reduce_kernel<<<nb, kScanThreads, 0, s>>>(in, n, tmp);
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(tmp, nb);
    scan_apply_kernel<<<nb, kScanThreads, 0, s>>>(in, out, n, tmp);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint64_t *__restrict__ keys, uint32_t n,
                                                                  int shift, uint32_t *__restrict__ ghist,
                                                                  uint32_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t base = blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        uint32_t idx = base + it * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    ghist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint32_t n, int shift, const uint32_t *__restrict__ offsets, uint32_t nblocks) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    base[tid] = offsets[tid * nblocks + blockIdx.x];
    wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < kSortItems; ++it) {
        uint32_t idx = blockIdx.x * kSortTile + it * kSortThreads + tid;
        bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0;
        uint32_t val = valid ? vin[idx] : 0;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (uint32_t k = 0; k < w; ++k) pos += wcnt[k][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
        __syncthreads();
    }
}

size_t radix_sort_tmp_bytes(uint32_t n) {
    uint32_t nb = (n + kSortTile - 1) / kSortTile;
    size_t h = (size_t)256 * nb;
    return align_up(h * 4, 256) * 2 + scan_tmp_bytes((uint32_t)h);
}

void radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint32_t n,
                    int key_bits, void *tmp, hipStream_t s) {
    if (n <= 1) return;
    uint32_t nb = (n + kSortTile - 1) / kSortTile;
    size_t h = (size_t)256 * nb;
    uint32_t *ghist = (uint32_t *)tmp;
    uint32_t *goff = (uint32_t *)((char *)tmp + align_up(h * 4, 256));
    uint32_t *stmp = (uint32_t *)((char *)goff + align_up(h * 4, 256));
    uint64_t *ka = keys, *kb = keys_alt;
    uint32_t *va = vals, *vb = vals_alt;
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        radix_hist_kernel<<<nb, kSortThreads, 0, s>>>(ka, n, shift, ghist, nb);
        scan_exclusive_u32(ghist, goff, (uint32_t)h, stmp, s);
        radix_scatter_kernel<<<nb, kSortThreads, 0, s>>>(ka, va, kb, vb, n, shift, goff, nb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        hipMemcpyAsync(keys, ka, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, va, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
    }
}

// ---------------------------------------------------------------------------
// build kernels
// ---------------------------------------------------------------------------
struct Bounds {
    float lo[3], hi[3];
    float maxabs;
    float pad_;
};

__global__ __launch_bounds__(256) void tri_prep_kernel(BuildInputs in, float *__restrict__ cent,
                                                       Bounds *__restrict__ partials, uint32_t *stat) {
    __shared__ float red[7][256];
    uint32_t k = blockIdx.x * 256 + threadIdx.x;
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    float mabs = 0.0f;
    if (k < in.nt) {
        uint32_t i0 = in.idx[3 * (size_t)k], i1 = in.idx[3 * (size_t)k + 1], i2 = in.idx[3 * (size_t)k + 2];
        if (i0 >= in.nv || i1 >= in.nv || i2 >= in.nv) {
            atomicOr(&stat[1], 1u);
            i0 = i1 = i2 = 0;
        }
        atomicMax(&stat[0], (uint32_t)in.mat[k]);
        float c[3];
        for (int a = 0; a < 3; ++a) {
            float x0 = in.vtx[3 * (size_t)i0 + a], x1 = in.vtx[3 * (size_t)i1 + a], x2 = in.vtx[3 * (size_t)i2 + a];
            c[a] = (x0 + x1 + x2) * (1.0f / 3.0f);
            mabs = fmaxf(mabs, fmaxf(fabsf(x0), fmaxf(fabsf(x1), fabsf(x2))));
            lo[a] = c[a];
            hi[a] = c[a];
            cent[3 * (size_t)k + a] = c[a];
        }
    }
    for (int a = 0; a < 3; ++a) { red[a][threadIdx.x] = lo[a]; red[3 + a][threadIdx.x] = hi[a]; }
    red[6][threadIdx.x] = mabs;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + st]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + st]);
            }
            red[6][threadIdx.x] = fmaxf(red[6][threadIdx.x], red[6][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Bounds b;
        for (int a = 0; a < 3; ++a) { b.lo[a] = red[a][0]; b.hi[a] = red[3 + a][0]; }
        b.maxabs = red[6][0];
        b.pad_ = 0.0f;
        partials[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(256) void bounds_reduce_kernel(Bounds *__restrict__ partials, uint32_t nb, float reach) {
    __shared__ float red[7][256];
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    float mabs = 0.0f;
    for (uint32_t k = threadIdx.x; k < nb; k += 256) {
        Bounds b = partials[k];
        for (int a = 0; a < 3; ++a) { lo[a] = fminf(lo[a], b.lo[a]); hi[a] = fmaxf(hi[a], b.hi[a]); }
        mabs = fmaxf(mabs, b.maxabs);
    }
    for (int a = 0; a < 3; ++a) { red[a][threadIdx.x] = lo[a]; red[3 + a][threadIdx.x] = hi[a]; }
    red[6][threadIdx.x] = mabs;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + st]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + st]);
            }
            red[6][threadIdx.x] = fmaxf(red[6][threadIdx.x], red[6][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Bounds b;
        for (int a = 0; a < 3; ++a) { b.lo[a] = red[a][0]; b.hi[a] = red[3 + a][0]; }
        b.maxabs = red[6][0];
        b.pad_ = fmaxf(b.maxabs, reach) * 9.5367431640625e-07f + 1e-20f;  // 2^-20 * max(max |coordinate|, reach)
        partials[0] = b;
    }
}

__device__ inline uint64_t spread21(uint32_t x) {
    uint64_t v = x & 0x1FFFFFu;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ __launch_bounds__(256) void morton_kernel(const float *__restrict__ cent, uint32_t nt,
                                                     const Bounds *__restrict__ bnd, uint64_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals) {
    uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nt) return;
    const Bounds b = bnd[0];
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float ext = b.hi[a] - b.lo[a];
        float f = ext > 0.0f ? (cent[3 * (size_t)k + a] - b.lo[a]) / ext : 0.0f;
        float s = f * 2097152.0f;
        s = fminf(fmaxf(s, 0.0f), 2097151.0f);
        q[a] = (uint32_t)s;
    }
    keys[k] = spread21(q[0]) | (spread21(q[1]) << 1) | (spread21(q[2]) << 2);
    vals[k] = k;
}

__global__ __launch_bounds__(256) void write_records_kernel(BuildInputs in, const uint32_t *__restrict__ order,
                                                            TriRec *__restrict__ recs, uint32_t *__restrict__ slot_of) {
    uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= in.nt) return;
    uint32_t k = order[s];
    uint32_t i0 = in.idx[3 * (size_t)k], i1 = in.idx[3 * (size_t)k + 1], i2 = in.idx[3 * (size_t)k + 2];
    if (i0 >= in.nv || i1 >= in.nv || i2 >= in.nv) i0 = i1 = i2 = 0;
    const float *v = in.vtx;
    TriRec r;
    r.a = make_float4(v[3 * (size_t)i0], v[3 * (size_t)i0 + 1], v[3 * (size_t)i0 + 2], __uint_as_float(k));
    r.b = make_float4(v[3 * (size_t)i1], v[3 * (size_t)i1 + 1], v[3 * (size_t)i1 + 2],
                      __uint_as_float(in.label ? in.label[k] : 0u));
    r.c = make_float4(v[3 * (size_t)i2], v[3 * (size_t)i2 + 1], v[3 * (size_t)i2 + 2], __uint_as_float((uint32_t)in.mat[k]));
    recs[s] = r;
    slot_of[k] = s;
}

__device__ inline int delta(const uint64_t *__restrict__ keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = keys[i], b = keys[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

struct BinTree {
    uint32_t *left, *right;    // child codes: kLeafBit | sorted index, or internal index
    uint32_t *first, *last;    // sorted range covered by internal node
    uint32_t *parent_int;      // [n-1]
    uint32_t *parent_leaf;     // [n]
    float *box;                // [n-1][6] lo xyz, hi xyz
    uint32_t *visit;           // [n-1]
};

__global__ __launch_bounds__(256) void karras_kernel(const uint64_t *__restrict__ keys, int n, BinTree T) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, n, i, i - d);
    int lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = delta(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + (d < 0 ? -1 : 0);
    int first = i < j ? i : j, last = i < j ? j : i;
    uint32_t lc = (first == gamma) ? (kLeafBit | (uint32_t)gamma) : (uint32_t)gamma;
    uint32_t rc = (last == gamma + 1) ? (kLeafBit | (uint32_t)(gamma + 1)) : (uint32_t)(gamma + 1);
    T.left[i] = lc;
    T.right[i] = rc;
    T.first[i] = (uint32_t)first;
    T.last[i] = (uint32_t)last;
    if (lc & kLeafBit) T.parent_leaf[gamma] = (uint32_t)i; else T.parent_int[gamma] = (uint32_t)i;
    if (rc & kLeafBit) T.parent_leaf[gamma + 1] = (uint32_t)i; else T.parent_int[gamma + 1] = (uint32_t)i;
}

__device__ inline void rec_box(const TriRec *__restrict__ recs, uint32_t s, float lo[3], float hi[3]) {
    TriRec r = recs[s];
    lo[0] = fminf(r.a.x, fminf(r.b.x, r.c.x)); hi[0] = fmaxf(r.a.x, fmaxf(r.b.x, r.c.x));
    lo[1] = fminf(r.a.y, fminf(r.b.y, r.c.y)); hi[1] = fmaxf(r.a.y, fmaxf(r.b.y, r.c.y));
    lo[2] = fminf(r.a.z, fminf(r.b.z, r.c.z)); hi[2] = fmaxf(r.a.z, fmaxf(r.b.z, r.c.z));
}

__device__ inline void child_box(const BinTree &T, const TriRec *__restrict__ recs, uint32_t code, float lo[3],
                                 float hi[3]) {
    if (code & kLeafBit) {
        rec_box(recs, code & ~kLeafBit, lo, hi);
    } else {
        const float *b = T.box + 6 * (size_t)code;
        for (int a = 0; a < 3; ++a) { lo[a] = b[a]; hi[a] = b[3 + a]; }
    }
}

__global__ __launch_bounds__(256) void refit_kernel(BinTree T, const TriRec *__restrict__ recs, int n) {
    int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    uint32_t p = T.parent_leaf[s];
    while (true) {
        __threadfence();
        uint32_t old = atomicAdd(&T.visit[p], 1u);
        if (old == 0) return;
        __threadfence();
        float l0[3], h0[3], l1[3], h1[3];
        child_box(T, recs, T.left[p], l0, h0);
        child_box(T, recs, T.right[p], l1, h1);
        float *b = T.box + 6 * (size_t)p;
        for (int a = 0; a < 3; ++a) {
            b[a] = fminf(l0[a], l1[a]);
            b[3 + a] = fmaxf(h0[a], h1[a]);
        }
        if (p == 0) return;
        p = T.parent_int[p];
    }
}

__device__ inline uint32_t code_count(const BinTree &T, uint32_t code) {
    return (code & kLeafBit) ? 1u : (T.last[code] - T.first[code] + 1u);
}
__device__ inline uint32_t code_first(const BinTree &T, uint32_t code) {
    return (code & kLeafBit) ? (code & ~kLeafBit) : T.first[code];
}

// One 4-wide node per frontier entry.  Writes boxes and leaf references;
// internal children are listed in `pending` (4 per entry, in slot order, with
// their slot in the top 2 bits... kept separately) and counted in `counts`.
__global__ __launch_bounds__(256) void collapse_kernel(BinTree T, const TriRec *__restrict__ recs,
                                                       const uint32_t *__restrict__ frontier, uint32_t n_front,
                                                       uint32_t node_base, uint32_t W, const Bounds *__restrict__ bnd,
                                                       Node4 *__restrict__ nodes, uint32_t *__restrict__ pending,
                                                       uint32_t *__restrict__ counts, uint32_t *stat) {
    uint32_t f = blockIdx.x * 256 + threadIdx.x;
    if (f >= n_front) return;
    const float pad = bnd[0].pad_;
    uint32_t b = frontier[f];
    uint32_t C[4];
    uint32_t nc = 2;
    C[0] = T.left[b];
    C[1] = T.right[b];
    while (nc < 4) {
        int best = -1;
        float best_area = -1.0f;
        for (uint32_t k = 0; k < nc; ++k) {
            uint32_t c = C[k];
            if ((c & kLeafBit) || code_count(T, c) <= W) continue;
            const float *bx = T.box + 6 * (size_t)c;
            float ex = bx[3] - bx[0], ey = bx[4] - bx[1], ez = bx[5] - bx[2];
            float area = ex * ey + ey * ez + ez * ex;
            if (area > best_area) { best_area = area; best = (int)k; }
        }
        if (best < 0) break;
        uint32_t c = C[best];
        C[best] = T.left[c];
        C[nc++] = T.right[c];
    }
    Node4 nd;
    uint32_t n_int = 0, n_leaf = 0;
    for (uint32_t k = 0; k < 4; ++k) {
        if (k < nc) {
            float lo[3], hi[3];
            child_box(T, recs, C[k], lo, hi);
            for (int a = 0; a < 3; ++a) {
                nd.c[k].lo[a] = lo[a] - pad;
                nd.c[k].hi[a] = hi[a] + pad;
            }
            uint32_t cnt = code_count(T, C[k]);
            if (cnt <= W) {
                nd.c[k].ref = leaf_ref(code_first(T, C[k]), cnt);
                ++n_leaf;
            } else {
                nd.c[k].ref = 0u;   // set by assign_kernel
                pending[4 * (size_t)f + n_int] = C[k] | ((uint32_t)k << 29);
                ++n_int;
            }
        } else {
            for (int a = 0; a < 3; ++a) nd.c[k].lo[a] = nd.c[k].hi[a] = 1e30f;
            nd.c[k].ref = kEmptyRef;
        }
        nd.c[k].pad = 0u;
    }
    nodes[node_base + f] = nd;
    counts[f] = n_int;
    atomicAdd(&stat[2], n_leaf);
}

__global__ __launch_bounds__(256) void assign_kernel(const uint32_t *__restrict__ pending,
                                                     const uint32_t *__restrict__ counts,
                                                     const uint32_t *__restrict__ offsets, uint32_t n_front,
                                                     uint32_t node_base, uint32_t next_base,
                                                     Node4 *__restrict__ nodes, uint32_t *__restrict__ next_frontier) {
    uint32_t f = blockIdx.x * 256 + threadIdx.x;
    if (f >= n_front) return;
    uint32_t cnt = counts[f], off = offsets[f];
    for (uint32_t q = 0; q < cnt; ++q) {
        uint32_t e = pending[4 * (size_t)f + q];
        uint32_t slot = e >> 29, code = e & 0x1FFFFFFFu;
        nodes[node_base + f].c[slot].ref = next_base + off + q;
        next_frontier[off + q] = code;
    }
}

__global__ void single_leaf_root_kernel(const TriRec *__restrict__ recs, uint32_t nt, const Bounds *__restrict__ bnd,
                                        Node4 *__restrict__ nodes, uint32_t *stat) {
    const float pad = bnd[0].pad_;
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    for (uint32_t s = 0; s < nt; ++s) {
        float l[3], h[3];
        rec_box(recs, s, l, h);
        for (int a = 0; a < 3; ++a) { lo[a] = fminf(lo[a], l[a]); hi[a] = fmaxf(hi[a], h[a]); }
    }
    Node4 nd;
    for (int k = 0; k < 4; ++k) {
        for (int a = 0; a < 3; ++a) nd.c[k].lo[a] = nd.c[k].hi[a] = 1e30f;
        nd.c[k].ref = kEmptyRef;
        nd.c[k].pad = 0;
    }
    for (int a = 0; a < 3; ++a) {
        nd.c[0].lo[a] = lo[a] - pad;
        nd.c[0].hi[a] = hi[a] + pad;
    }
    nd.c[0].ref = leaf_ref(0, nt);
    nodes[0] = nd;
    stat[2] = 1;
}

// ---------------------------------------------------------------------------
// PLOC
// ---------------------------------------------------------------------------
constexpr int kPlocRMax = 128;   // largest search radius in Morton order
constexpr int kPlocBlock = 256;

// Half the surface area of a box, its two horizontal faces weighted by wz (1: the plain surface area).
// A weight below 1 prices boxes for rays that are mostly horizontal, as a LiDAR's are.
__device__ inline float half_area(float lx, float ly, float lz, float hx, float hy, float hz, float wz) {
    float ex = hx - lx, ey = hy - ly, ez = hz - lz;
    return wz * (ex * ey) + ey * ez + ez * ex;
}

// node ids: leaves 0..n-1 (Morton positions), internal nodes n..2n-2 in creation order
__global__ __launch_bounds__(256) void ploc_init_kernel(const TriRec *__restrict__ recs, uint32_t n,
                                                        float *__restrict__ nbox, uint32_t *__restrict__ ncount,
                                                        uint32_t *__restrict__ C) {
    uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float lo[3], hi[3];
    rec_box(recs, s, lo, hi);
    float *b = nbox + 6 * (size_t)s;
    for (int a = 0; a < 3; ++a) { b[a] = lo[a]; b[3 + a] = hi[a]; }
    ncount[s] = 1;
    C[s] = s;
}

__global__ __launch_bounds__(kPlocBlock) void ploc_nn_kernel(const uint32_t *__restrict__ C, uint32_t m,
                                                             const float *__restrict__ nbox, uint32_t *__restrict__ nn,
                                                             int R, float wz) {
    __shared__ float sb[(kPlocBlock + 2 * kPlocRMax) * 6];
    const int base = (int)(blockIdx.x * kPlocBlock);
    const int lo_i = base - R;
    for (int k = threadIdx.x; k < kPlocBlock + 2 * R; k += kPlocBlock) {
        int idx = lo_i + k;
        if (idx >= 0 && idx < (int)m) {
            const float *b = nbox + 6 * (size_t)C[idx];
            for (int a = 0; a < 6; ++a) sb[k * 6 + a] = b[a];
        }
    }
    __syncthreads();
    const int i = base + (int)threadIdx.x;
    if (i >= (int)m) return;
    const int li = i - lo_i;
    const float lx = sb[li * 6 + 0], ly = sb[li * 6 + 1], lz = sb[li * 6 + 2];
    const float hx = sb[li * 6 + 3], hy = sb[li * 6 + 4], hz = sb[li * 6 + 5];
    float best = __builtin_inff();
    int bj = i == 0 ? 1 : i - 1;
    for (int d = -R; d <= R; ++d) {
        int j = i + d;
        if (d == 0 || j < 0 || j >= (int)m) continue;
        const float *o = sb + (li + d) * 6;
        float a = half_area(fminf(lx, o[0]), fminf(ly, o[1]), fminf(lz, o[2]), fmaxf(hx, o[3]), fmaxf(hy, o[4]),
                            fmaxf(hz, o[5]), wz);
        if (a < best) { best = a; bj = j; }    // ties keep the smaller j (ascending scan)
    }
    nn[i] = (uint32_t)bj;
}

__global__ __launch_bounds__(256) void ploc_flags_kernel(const uint32_t *__restrict__ nn, uint32_t m,
                                                         uint32_t *__restrict__ leader, uint32_t *__restrict__ keep) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    uint32_t j = nn[i];
    bool mutual = nn[j] == i;
    leader[i] = (mutual && i < j) ? 1u : 0u;
    keep[i] = (mutual && i > j) ? 0u : 1u;
}

__global__ __launch_bounds__(256) void ploc_merge_kernel(const uint32_t *__restrict__ C, const uint32_t *__restrict__ nn,
                                                         uint32_t m, const uint32_t *__restrict__ leader,
                                                         const uint32_t *__restrict__ loff,
                                                         const uint32_t *__restrict__ keep,
                                                         const uint32_t *__restrict__ koff, uint32_t next_id,
                                                         uint32_t n, float *__restrict__ nbox,
                                                         uint32_t *__restrict__ ncount, uint32_t *__restrict__ nleft,
                                                         uint32_t *__restrict__ nright, uint32_t *__restrict__ C_out) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m || !keep[i]) return;
    uint32_t c = C[i];
    if (leader[i]) {
        uint32_t a = C[i], b = C[nn[i]];
        uint32_t id = next_id + loff[i];
        const float *ba = nbox + 6 * (size_t)a, *bb = nbox + 6 * (size_t)b;
        float *bo = nbox + 6 * (size_t)id;
        for (int q = 0; q < 3; ++q) {
            bo[q] = fminf(ba[q], bb[q]);
            bo[3 + q] = fmaxf(ba[3 + q], bb[3 + q]);
        }
        ncount[id] = ncount[a] + ncount[b];
        nleft[id - n] = a;
        nright[id - n] = b;
        c = id;
    }
    C_out[koff[i]] = c;
}

__global__ void set_u32_kernel(uint32_t *p, uint32_t v) { *p = v; }

// top-down leaf offsets, one creation round at a time (parents before children)
__global__ __launch_bounds__(256) void ploc_first_kernel(uint32_t id0, uint32_t cnt, uint32_t n,
                                                         const uint32_t *__restrict__ nleft,
                                                         const uint32_t *__restrict__ nright,
                                                         const uint32_t *__restrict__ ncount,
                                                         uint32_t *__restrict__ first) {
    uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= cnt) return;
    uint32_t id = id0 + k;
    uint32_t l = nleft[id - n], r = nright[id - n];
    uint32_t f = first[id];
    first[l] = f;
    first[r] = f + ncount[l];
}

// records into depth-first order; slot_of follows
__global__ __launch_bounds__(256) void ploc_leaves_kernel(const TriRec *__restrict__ recs_m, uint32_t n,
                                                          const uint32_t *__restrict__ first,
                                                          TriRec *__restrict__ recs, uint32_t *__restrict__ slot_of) {
    uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    uint32_t pos = first[s];
    TriRec r = recs_m[s];
    recs[pos] = r;
    slot_of[__float_as_uint(r.a.w)] = pos;
}

// PLOC tree -> the binary-tree form the collapse reads (codes as in the LBVH path)
__global__ __launch_bounds__(256) void ploc_bintree_kernel(uint32_t n, const uint32_t *__restrict__ nleft,
                                                           const uint32_t *__restrict__ nright,
                                                           const uint32_t *__restrict__ ncount,
                                                           const uint32_t *__restrict__ first,
                                                           const float *__restrict__ nbox, BinTree T) {
    uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n - 1) return;
    uint32_t id = n + k;
    uint32_t l = nleft[k], r = nright[k];
    T.left[k] = l < n ? (kLeafBit | first[l]) : (l - n);
    T.right[k] = r < n ? (kLeafBit | first[r]) : (r - n);
    T.first[k] = first[id];
    T.last[k] = first[id] + ncount[id] - 1;
    const float *b = nbox + 6 * (size_t)id;
    for (int a = 0; a < 6; ++a) T.box[6 * (size_t)k + a] = b[a];
}

// ---------------------------------------------------------------------------
// Surface-area-cost collapse
// ---------------------------------------------------------------------------
// Per binary internal node k: cost[4k + i - 1] = C(k, i), i = 1..4, and a
// packed choice word:
//   bit 0        C(k, 1) is a leaf (else a 4-wide node)
//   bits 1+3(i-2)..  (i = 2..4, 3 bits) the number of children e <= i that
//                C(k, i) uses: 1 = k itself as one child, e >= 2 = k's two
//                binary children spread over e slots
//   bits 10+2(e-2).. (e = 2..4, 2 bits) how many of those e slots go to the
//                left child in the best spread
struct SahTables {
    float *cost;
    uint32_t *choice;
};

__device__ inline uint32_t sah_uses(uint32_t w, int i) { return i == 1 ? 1u : (w >> (1 + 3 * (i - 2))) & 7u; }
__device__ inline uint32_t sah_left(uint32_t w, int e) { return (w >> (10 + 2 * (e - 2))) & 3u; }

__device__ inline float box_half_area(const float lo[3], const float hi[3], float wz) {
    const float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    return wz * (ex * ey) + ey * ez + ez * ex;
}

// C(c, 1..4) of a child code: a single triangle is a leaf whatever the slots
__device__ inline void sah_child_costs(const BinTree &T, const TriRec *__restrict__ recs, const float *cost,
                                       uint32_t code, float leaf_w, float wz, float C[4]) {
    if (code & kLeafBit) {
        float lo[3], hi[3];
        rec_box(recs, code & ~kLeafBit, lo, hi);
        const float c = leaf_w * box_half_area(lo, hi, wz);
        for (int i = 0; i < 4; ++i) C[i] = c;
    } else {
        // written by another thread of this pass: read past the vector L1
        for (int i = 0; i < 4; ++i)
            C[i] = __hip_atomic_load(cost + 4 * (size_t)code + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// C(p, 1..4) and the choice word of binary node p from its children's costs
__device__ inline void sah_eval(const BinTree &T, const TriRec *__restrict__ recs, uint32_t p, uint32_t W,
                                float leaf_w, float wz, const SahTables &S) {
    float L[4], R[4];
    sah_child_costs(T, recs, S.cost, T.left[p], leaf_w, wz, L);
    sah_child_costs(T, recs, S.cost, T.right[p], leaf_w, wz, R);
    const float *b = T.box + 6 * (size_t)p;
    const float area = box_half_area(b, b + 3, wz);
    // best spread of the two children over e = 2..4 slots (smallest left share on ties)
    float spread[5];
    uint32_t w = 0;
    for (int e = 2; e <= 4; ++e) {
        int best_k = 1;
        float best = L[0] + R[e - 2];
        for (int k = 2; k < e; ++k) {
            const float c = L[k - 1] + R[e - k - 1];
            if (c < best) { best = c; best_k = k; }
        }
        spread[e] = best;
        w |= (uint32_t)best_k << (10 + 2 * (e - 2));
    }
    const uint32_t count = T.last[p] - T.first[p] + 1u;
    // a leaf is one walk step for up to 4 triangles (the lanes of a ray test them side by side)
    const float as_leaf = count <= W ? leaf_w * area * (float)((count + 3u) / 4u) : __builtin_inff();
    const float as_node = area + spread[4];
    float C[4];
    C[0] = fminf(as_leaf, as_node);
    if (as_leaf <= as_node) w |= 1u;
    uint32_t uses = 1;
    for (int i = 2; i <= 4; ++i) {
        if (spread[i] < C[i - 2]) { C[i - 1] = spread[i]; uses = (uint32_t)i; }
        else C[i - 1] = C[i - 2];
        w |= uses << (1 + 3 * (i - 2));
    }
    for (int i = 0; i < 4; ++i)
        __hip_atomic_store(S.cost + 4 * (size_t)p + i, C[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    S.choice[p] = w;
}

// Bottom-up over the binary tree, one thread per triangle climbing from its
// leaf; the second thread to reach a node evaluates it (both children done).
// For the LBVH, whose nodes carry no creation order.
__global__ __launch_bounds__(256) void sah_cost_kernel(BinTree T, const TriRec *__restrict__ recs, int n,
                                                       uint32_t root, uint32_t W, float leaf_w, float wz,
                                                       SahTables S) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    uint32_t p = T.parent_leaf[s];
    while (true) {
        __threadfence();
        if (atomicAdd(&T.visit[p], 1u) == 0) return;
        __threadfence();
        sah_eval(T, recs, p, W, leaf_w, wz, S);
        if (p == root) return;
        p = T.parent_int[p];
    }
}

// The nodes one clustering round created, [k0, k0 + cnt): their children come from earlier rounds, so
// running the rounds in creation order evaluates every node after its children, without atomics.
__global__ __launch_bounds__(256) void sah_round_kernel(BinTree T, const TriRec *__restrict__ recs, uint32_t k0,
                                                        uint32_t cnt, uint32_t W, float leaf_w, float wz,
                                                        SahTables S) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < cnt) sah_eval(T, recs, k0 + k, W, leaf_w, wz, S);
}

// One 4-wide node per frontier entry, shaped by the recorded choices: the
// node's binary children spread over 4 slots, each part expanded until it is
// one child.  Output as collapse_kernel.
__global__ __launch_bounds__(256) void collapse_sah_kernel(BinTree T, const TriRec *__restrict__ recs,
                                                           const uint32_t *__restrict__ frontier, uint32_t n_front,
                                                           uint32_t node_base, const uint32_t *__restrict__ choice,
                                                           const Bounds *__restrict__ bnd, Node4 *__restrict__ nodes,
                                                           uint32_t *__restrict__ pending,
                                                           uint32_t *__restrict__ counts, uint32_t *stat) {
    const uint32_t f = blockIdx.x * 256 + threadIdx.x;
    if (f >= n_front) return;
    const float pad = bnd[0].pad_;
    const uint32_t b = frontier[f];
    // work list of (code, slots); the slots of all entries plus the children found sum to 4
    uint32_t wc[4], wi[4];
    int nw = 0;
    const uint32_t k4 = sah_left(choice[b], 4);
    wc[nw] = T.right[b]; wi[nw++] = 4u - k4;
    wc[nw] = T.left[b]; wi[nw++] = k4;
    uint32_t C[4];
    uint32_t nc = 0;
    while (nw > 0) {
        --nw;
        const uint32_t c = wc[nw], i = wi[nw];
        const uint32_t e = (c & kLeafBit) ? 1u : sah_uses(choice[c], (int)i);
        const uint32_t k = e >= 2u ? sah_left(choice[c], (int)e) : 0u;
        // (the guards never fail for choices written by sah_cost_kernel: the slots still open
        // always cover the list, so it holds at most 4 entries)
        if (e >= 2u && e <= i && k >= 1u && k < e && nw <= 2) {
            wc[nw] = T.right[c]; wi[nw++] = e - k;
            wc[nw] = T.left[c]; wi[nw++] = k;
        } else if (nc < 4) {
            C[nc++] = c;
        }
    }
    Node4 nd;
    uint32_t n_int = 0, n_leaf = 0;
    for (uint32_t k = 0; k < 4; ++k) {
        if (k < nc) {
            float lo[3], hi[3];
            child_box(T, recs, C[k], lo, hi);
            for (int a = 0; a < 3; ++a) {
                nd.c[k].lo[a] = lo[a] - pad;
                nd.c[k].hi[a] = hi[a] + pad;
            }
            if ((C[k] & kLeafBit) || (choice[C[k]] & 1u)) {
                nd.c[k].ref = leaf_ref(code_first(T, C[k]), code_count(T, C[k]));
                ++n_leaf;
            } else {
                nd.c[k].ref = 0u;   // set by assign_kernel
                pending[4 * (size_t)f + n_int] = C[k] | ((uint32_t)k << 29);
                ++n_int;
            }
        } else {
            for (int a = 0; a < 3; ++a) nd.c[k].lo[a] = nd.c[k].hi[a] = 1e30f;
            nd.c[k].ref = kEmptyRef;
        }
        nd.c[k].pad = 0u;
    }
    nodes[node_base + f] = nd;
    counts[f] = n_int;
    atomicAdd(&stat[2], n_leaf);
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
namespace {
struct ScratchLayout {
    size_t cent, partials, keys, vals, keys2, vals2, sort_tmp, left, right, first, last, pint, pleaf, box,
        visit, front_a, front_b, pending, counts, offsets, scan_tmp, stat, recs_m, nbox, ncount, nleft, nright,
        nfirst, ca, cb, nn, leader, keep, loff, koff, sah_cost, sah_choice, total;
};

ScratchLayout scratch_layout(uint32_t nt) {
    ScratchLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
    size_t n = nt;
    size_t nb = (n + 255) / 256;
    L.cent = take(12 * n);
    L.partials = take(sizeof(Bounds) * (nb + 1));
    L.keys = take(8 * n);
    L.vals = take(4 * n);
    L.keys2 = take(8 * n);
    L.vals2 = take(4 * n);
    L.sort_tmp = take(radix_sort_tmp_bytes(nt));
    L.left = take(4 * n);
    L.right = take(4 * n);
    L.first = take(4 * n);
    L.last = take(4 * n);
    L.pint = take(4 * n);
    L.pleaf = take(4 * n);
    L.box = take(24 * n);
    L.visit = take(4 * n);
    L.front_a = take(4 * n);
    L.front_b = take(4 * n);
    L.pending = take(16 * n);
    L.counts = take(4 * n);
    L.offsets = take(4 * n);
    L.scan_tmp = take(scan_tmp_bytes(nt));
    L.stat = take(64);
    L.recs_m = take(sizeof(TriRec) * n);
    L.nbox = take(24 * 2 * n);
    L.ncount = take(4 * 2 * n);
    L.nleft = take(4 * n);
    L.nright = take(4 * n);
    L.nfirst = take(4 * 2 * n);
    L.ca = take(4 * n);
    L.cb = take(4 * n);
    L.nn = take(4 * n);
    L.leader = take(4 * n);
    L.keep = take(4 * n);
    L.loff = take(4 * n);
    L.koff = take(4 * n);
    L.sah_cost = take(16 * n);
    L.sah_choice = take(4 * n);
    L.total = o;
    return L;
}
}  // namespace

size_t build_scratch_bytes(uint32_t nt) { return scratch_layout(nt).total; }

size_t persistent_nodes_bytes(uint32_t nt) {
    size_t nodes = nt > 1 ? nt : 1;  // a 4-wide node per binary internal node at most
    return align_up(sizeof(Node4) * nodes, 256);
}
size_t persistent_recs_bytes(uint32_t nt) { return align_up(sizeof(TriRec) * (size_t)nt, 256); }

size_t build_persistent_bytes(uint32_t nt) {
    return persistent_nodes_bytes(nt) + persistent_recs_bytes(nt) + align_up(4 * (size_t)nt, 256);
}

#define HIP_TRY(x)                             \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

hipError_t build_bvh(const BuildInputs &in, void *persistent, void *scratch, BuildResult &res, hipStream_t s) {
    const uint32_t nt = in.nt;
    ScratchLayout L = scratch_layout(nt);
    char *sc = (char *)scratch;
    float *cent = (float *)(sc + L.cent);
    Bounds *partials = (Bounds *)(sc + L.partials);
    uint64_t *keys = (uint64_t *)(sc + L.keys);
    uint32_t *vals = (uint32_t *)(sc + L.vals);
    uint32_t *stat = (uint32_t *)(sc + L.stat);
    Node4 *nodes = (Node4 *)persistent;
    TriRec *recs = (TriRec *)((char *)persistent + persistent_nodes_bytes(nt));
    uint32_t *slot_of = (uint32_t *)((char *)recs + persistent_recs_bytes(nt));
    const uint32_t nb = (nt + 255) / 256;
    const float wz = in.up_weight > 0.0f ? in.up_weight : 1.0f;   // horizontal-face weight of the area metric

    const bool ploc = in.builder == 0 && nt > in.leaf_width;
    TriRec *recs_m = ploc ? (TriRec *)(sc + L.recs_m) : recs;   // Morton-order records
    HIP_TRY(hipMemsetAsync(stat, 0, 64, s));
    tri_prep_kernel<<<nb, 256, 0, s>>>(in, cent, partials, stat);
    bounds_reduce_kernel<<<1, 256, 0, s>>>(partials, nb, in.reach);
    morton_kernel<<<nb, 256, 0, s>>>(cent, nt, partials, keys, vals);
    radix_sort_u64(keys, vals, (uint64_t *)(sc + L.keys2), (uint32_t *)(sc + L.vals2), nt, 63, sc + L.sort_tmp, s);
    write_records_kernel<<<nb, 256, 0, s>>>(in, vals, recs_m, slot_of);
    HIP_TRY(hipGetLastError());

    uint32_t depth = 1, n_nodes = 1;
    if (nt <= in.leaf_width) {
        single_leaf_root_kernel<<<1, 1, 0, s>>>(recs, nt, partials, nodes, stat);
    } else {
        BinTree T;
        T.left = (uint32_t *)(sc + L.left);
        T.right = (uint32_t *)(sc + L.right);
        T.first = (uint32_t *)(sc + L.first);
        T.last = (uint32_t *)(sc + L.last);
        T.parent_int = (uint32_t *)(sc + L.pint);
        T.parent_leaf = (uint32_t *)(sc + L.pleaf);
        T.box = (float *)(sc + L.box);
        T.visit = (uint32_t *)(sc + L.visit);
        uint32_t *stmp = (uint32_t *)(sc + L.scan_tmp);
        uint32_t root_code = 0;
        std::vector<std::pair<uint32_t, uint32_t>> ploc_rounds;   // (first node id, count) per round
        if (ploc) {
            float *nbox = (float *)(sc + L.nbox);
            uint32_t *ncount = (uint32_t *)(sc + L.ncount), *nleft = (uint32_t *)(sc + L.nleft),
                     *nright = (uint32_t *)(sc + L.nright), *nfirst = (uint32_t *)(sc + L.nfirst);
            uint32_t *ca = (uint32_t *)(sc + L.ca), *cb = (uint32_t *)(sc + L.cb), *nn = (uint32_t *)(sc + L.nn);
            uint32_t *leader = (uint32_t *)(sc + L.leader), *keep = (uint32_t *)(sc + L.keep);
            uint32_t *loff = (uint32_t *)(sc + L.loff), *koff = (uint32_t *)(sc + L.koff);
            ploc_init_kernel<<<nb, 256, 0, s>>>(recs_m, nt, nbox, ncount, ca);
            std::vector<uint32_t> round_start, round_count;
            uint32_t m = nt, next_id = nt;
            while (m > 1) {
                if (round_start.size() > 100000) return hipErrorIllegalState;
                uint32_t g = (m + 255) / 256;
                ploc_nn_kernel<<<(m + kPlocBlock - 1) / kPlocBlock, kPlocBlock, 0, s>>>(ca, m, nbox, nn,
                                                                                         (int)in.ploc_radius, wz);
                ploc_flags_kernel<<<g, 256, 0, s>>>(nn, m, leader, keep);
                scan_exclusive_u32(leader, loff, m, stmp, s);
                scan_exclusive_u32(keep, koff, m, stmp, s);
                uint32_t h[4];
                HIP_TRY(hipMemcpyAsync(&h[0], leader + m - 1, 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipMemcpyAsync(&h[1], loff + m - 1, 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipMemcpyAsync(&h[2], keep + m - 1, 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipMemcpyAsync(&h[3], koff + m - 1, 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                uint32_t merges = h[0] + h[1], survivors = h[2] + h[3];
                if (merges == 0 || next_id + merges > 2 * nt - 1) return hipErrorIllegalState;
                ploc_merge_kernel<<<g, 256, 0, s>>>(ca, nn, m, leader, loff, keep, koff, next_id, nt, nbox, ncount,
                                                    nleft, nright, cb);
                HIP_TRY(hipGetLastError());
                round_start.push_back(next_id);
                round_count.push_back(merges);
                next_id += merges;
                m = survivors;
                uint32_t *t = ca; ca = cb; cb = t;
            }
            // depth-first leaf offsets: root first, then each creation round in reverse
            const uint32_t root = 2 * nt - 2;
            set_u32_kernel<<<1, 1, 0, s>>>(nfirst + root, 0u);
            for (size_t r = round_start.size(); r-- > 0;)
                ploc_first_kernel<<<(round_count[r] + 255) / 256, 256, 0, s>>>(round_start[r], round_count[r], nt, nleft,
                                                                               nright, ncount, nfirst);
            ploc_leaves_kernel<<<nb, 256, 0, s>>>(recs_m, nt, nfirst, recs, slot_of);
            ploc_bintree_kernel<<<nb, 256, 0, s>>>(nt, nleft, nright, ncount, nfirst, nbox, T);
            HIP_TRY(hipGetLastError());
            root_code = root - nt;
            for (size_t r = 0; r < round_start.size(); ++r) ploc_rounds.emplace_back(round_start[r], round_count[r]);
        } else {
            HIP_TRY(hipMemsetAsync(T.visit, 0, 4 * (size_t)nt, s));
            karras_kernel<<<nb, 256, 0, s>>>(keys, (int)nt, T);
            refit_kernel<<<nb, 256, 0, s>>>(T, recs, (int)nt);
        }
        const bool sah = in.collapse == 0;
        SahTables sah_t{(float *)(sc + L.sah_cost), (uint32_t *)(sc + L.sah_choice)};
        if (sah && ploc) {
            for (size_t r = 0; r < ploc_rounds.size(); ++r)
                sah_round_kernel<<<(ploc_rounds[r].second + 255) / 256, 256, 0, s>>>(
                    T, recs, ploc_rounds[r].first - nt, ploc_rounds[r].second, in.leaf_width, in.leaf_cost, wz, sah_t);
            HIP_TRY(hipGetLastError());
        } else if (sah) {
            HIP_TRY(hipMemsetAsync(T.visit, 0, 4 * (size_t)nt, s));
            sah_cost_kernel<<<nb, 256, 0, s>>>(T, recs, (int)nt, root_code, in.leaf_width, in.leaf_cost, wz, sah_t);
            HIP_TRY(hipGetLastError());
        }
        uint32_t *fa = (uint32_t *)(sc + L.front_a), *fb = (uint32_t *)(sc + L.front_b);
        uint32_t *pending = (uint32_t *)(sc + L.pending);
        uint32_t *counts = (uint32_t *)(sc + L.counts), *offsets = (uint32_t *)(sc + L.offsets);
        set_u32_kernel<<<1, 1, 0, s>>>(fa, root_code);   // frontier = [binary root]
        uint32_t n_front = 1, base = 0;
        depth = 0;
        n_nodes = 0;
        while (n_front > 0) {
            if (depth >= 1024 || n_nodes + n_front > (nt > 1 ? nt : 1)) return hipErrorIllegalState;
            if (depth <= (uint32_t)kMaxLevels) res.level_base[depth] = base;
            uint32_t g = (n_front + 255) / 256;
            if (sah)
                collapse_sah_kernel<<<g, 256, 0, s>>>(T, recs, fa, n_front, base, sah_t.choice, partials, nodes,
                                                      pending, counts, stat);
            else
                collapse_kernel<<<g, 256, 0, s>>>(T, recs, fa, n_front, base, in.leaf_width, partials, nodes,
                                                  pending, counts, stat);
            scan_exclusive_u32(counts, offsets, n_front, stmp, s);
            uint32_t last_cnt = 0, last_off = 0;
            HIP_TRY(hipMemcpyAsync(&last_cnt, counts + n_front - 1, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(&last_off, offsets + n_front - 1, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            uint32_t next = last_cnt + last_off;
            uint32_t next_base = base + n_front;
            assign_kernel<<<g, 256, 0, s>>>(pending, counts, offsets, n_front, base, next_base, nodes, fb);
            HIP_TRY(hipGetLastError());
            n_nodes += n_front;
            ++depth;
            base = next_base;
            n_front = next;
            uint32_t *t = fa; fa = fb; fb = t;
        }
    }
    uint32_t hstat[4] = {0, 0, 0, 0};
    Bounds hb;
    HIP_TRY(hipMemcpyAsync(hstat, stat, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hb, partials, sizeof(Bounds), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (nt <= in.leaf_width) res.level_base[0] = 0;
    if (depth <= (uint32_t)kMaxLevels) res.level_base[depth] = n_nodes;
    res.root = 0;
    res.n_nodes = n_nodes;
    res.n_leaves = hstat[2];
    res.depth = depth;
    res.max_material = hstat[0];
    res.bad_index = hstat[1];
    res.box_pad = hb.pad_;
    res.max_abs = hb.maxabs;
    res.reach = in.reach;
    return hipSuccess;
}

}  // namespace lidar
