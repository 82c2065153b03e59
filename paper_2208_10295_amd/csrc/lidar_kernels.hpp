// lidar_kernels.hpp -- host-visible launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lidar_device.hpp"

namespace lidar {

struct SceneDev {
    const Node4 *nodes;
    const TriRec *tris;
    uint32_t root;
    uint32_t n_tri;
    uint32_t max_steps;    // bound on traversal loop iterations (nodes + leaves)
    int32_t stack_cap;     // stack entries a walk of this tree may use (fewer than needed only to test overflow)
};

// --- scan / sort utilities (bvh_build.hip) ---
size_t scan_tmp_bytes(uint32_t n);
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *tmp, hipStream_t s);
size_t radix_sort_tmp_bytes(uint32_t n);
// Stable LSD sort of (key, value) pairs on bits [0, key_bits); result in keys/vals.
void radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint32_t n,
                    int key_bits, void *tmp, hipStream_t s);

// --- BVH build ---
struct BuildInputs {
    const float *vtx;          // device [nv][3]
    const uint32_t *idx;       // device [nt][3]
    const uint16_t *mat;       // device [nt]
    const uint32_t *label;     // device [nt], or null (label 0)
    uint64_t nv;
    uint32_t nt;
    uint32_t leaf_width;
    uint32_t builder;          // 0 = PLOC, 1 = LBVH (binary radix tree)
    uint32_t ploc_radius;      // PLOC search radius, 1..128
    uint32_t collapse;         // 0 = surface-area cost (default), 1 = greedy (largest child first)
    float leaf_cost;           // leaf step weight of the cost model, a node step weighing 1
    float up_weight;           // weight of a box's two horizontal faces in the area metric of the clustering
                               // and the collapse (0 or 1: the surface area; below 1: for rays near the
                               // horizontal)
    float reach;               // child boxes are padded by 2^-20 max(max |vertex coordinate|, reach):
                               // 0 for a scene, the object-space origin bound for a mesh, the static
                               // scene's largest coordinate for the actors' top-level tree
};

// Persistent layout: [nodes: Node4 x max(nt,1)] [records: TriRec x nt] [slot_of: u32 x nt]
size_t persistent_nodes_bytes(uint32_t nt);
size_t persistent_recs_bytes(uint32_t nt);

constexpr int kMaxLevels = 64;   // refit supports trees up to this depth

struct BuildResult {
    uint32_t root;
    uint32_t n_nodes;
    uint32_t n_leaves;
    uint32_t depth;
    uint32_t max_material;
    uint32_t bad_index;
    float box_pad;
    float max_abs;             // largest |vertex coordinate| of the input
    float reach;               // BuildInputs::reach of the build (refits pad the same way)
    uint32_t level_base[kMaxLevels + 1];   // nodes of level L: [level_base[L], level_base[L + 1])
};

size_t build_scratch_bytes(uint32_t nt);
size_t build_persistent_bytes(uint32_t nt);
// Runs the whole build on `s`; synchronises the stream (reads back sizes).
hipError_t build_bvh(const BuildInputs &in, void *persistent, void *scratch, BuildResult &res, hipStream_t s);

// --- trace (trace.hip) ---
struct TraceOpts {
    int stack;            // traversal stack entries (32, 64 or 96)
    int tile_az_log2;     // wavefront tile: 2^tile_az_log2 azimuth steps x 64 / that channels
    int lanes_per_ray;    // 1 (lane per ray) or 4 (quad per ray)
    int xcd_remap;        // 1: blocks of one XCD take one contiguous azimuth sector
};

void launch_dir_tables(const double *elev_deg, uint32_t n_ch, double az0_deg, double fov_h_deg,
                       uint32_t n_az, double *elev_cs, double *az_cs, hipStream_t s);

// n_nodes / n_tris: optional per-beam traversal counts (null = plain kernel);
// actors: the dynamic part of the scene, or null
void launch_trace_scan(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                       const Overrides &ov, const Outputs &out, uint64_t n_padded, uint32_t *err, uint32_t *n_nodes,
                       uint32_t *n_tris, const ActorsDev *actors, hipStream_t s);
void launch_bruteforce(const SceneDev &S, const InstanceDev &in, const MaterialsDev &M, const Overrides &ov,
                       const Outputs &out, int tile_az_log2, uint64_t n_padded, hipStream_t s);
// A batch's walks may first run with a short stack (more wavefronts fit on a CU): a ray whose walk
// needs more entries is listed, and a second pass traces the listed rays again with the whole stack.
struct BatchRedo {
    uint32_t *list;       // padded ray indices, room for `cap`; null: one pass with the whole stack
    uint32_t *count;      // rays listed by the last launch (one device word)
    uint32_t cap;
    int first_stack;      // stack entries the first pass is compiled for (32, 48, 64 or 96)
    int first_cap;        // entries its walks may use
};
constexpr uint32_t kRedoBlocks = 256;   // second pass: 64-lane blocks striding over the list
void launch_trace_batch(const TraceOpts &t, const SceneDev &S, const InstanceDev *insts, uint32_t n_inst,
                        const MaterialsDev &M, const Outputs &out, uint64_t n_padded, uint32_t packet,
                        uint32_t *queue, uint32_t *err, const BatchRedo &R, uint32_t grid, hipStream_t s);
// blocks of the batched kernel per CU for a first pass compiled for `stack` entries
int batch_blocks_per_cu(const TraceOpts &t, int stack);

// --- divergent beams and multi-echo returns (trace.hip) ---
constexpr int kMaxSub = 16;      // sub-rays per beam
constexpr int kMaxEchoes = 4;
struct SubrayPattern {
    double c[kMaxSub][4];        // cos r_k, sin r_k, cos b_k, sin b_k
    uint32_t n_sub;
};
struct SubHit {                  // first hit of one sub-ray (t = +inf: none)
    float t;
    uint32_t orig;
    float rl;                    // noise-free R_lambda (eq.4)
    uint32_t label;
    uint32_t mat;
    uint32_t pad_;
};
void launch_trace_subrays(const TraceOpts &t, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                          const SubrayPattern &pat, SubHit *sub, uint64_t n_padded, uint32_t *err,
                          const ActorsDev *actors, hipStream_t s);
void launch_echoes(const InstanceDev &in, const MaterialsDev &M, const SubHit *sub, uint32_t n_sub,
                   uint32_t max_echoes, float echo_sep, const Outputs &out, hipStream_t s);

// --- dynamic scenes (dynamic.hip) ---
// word: two device words of scratch (max |coordinate| bits, pad bits)
bool refit_supported(const BuildResult &br);
void refit_mesh(Node4 *nodes, TriRec *recs, const BuildResult &br, uint32_t nt, const uint32_t *idx,
                const float *vertices, uint64_t nv, uint32_t *word, hipStream_t s);
void actor_boxes(const ActorDev *actors, uint32_t n, const MeshDev *meshes, float *lohi, uint32_t *word,
                 hipStream_t s);
void actor_prims(const float *lohi, uint32_t n, float *vtx, uint32_t *idx, uint16_t *mat, hipStream_t s);
// actor boxes + top-level refit of a per-frame update (one workgroup for small trees)
void update_tlas(const ActorDev *actors, uint32_t n, const MeshDev *meshes, float *lohi, Node4 *nodes,
                 TriRec *recs, const BuildResult &br, uint32_t *word, hipStream_t s);
void refit_tlas(Node4 *nodes, TriRec *recs, const BuildResult &br, uint32_t n, const float *lohi, uint32_t *word,
                hipStream_t s);
// Top-level tree of at most kPackedTlasMax actors rebuilt in one workgroup:
// Morton order of the actor boxes, one actor per leaf, four entries per node.
// packed_tlas_shape gives its node levels (root 0, breadth-first) for n actors.
constexpr uint32_t kPackedTlasMax = 4096;
BuildResult packed_tlas_shape(uint32_t n, float reach);
// The actors are read from src (device or host-mapped memory) and copied to actors when the two differ.
void rebuild_tlas(const ActorDev *src, ActorDev *actors, uint32_t n, const MeshDev *meshes, uint32_t n_meshes,
                  float *lohi, Node4 *nodes, TriRec *recs, const BuildResult &shape, hipStream_t s);

// --- bandwidth probes (probe.hip) ---
void launch_probe_stream(const void *buf, uint64_t bytes, float *sink, hipStream_t s);
void launch_probe_gather(const void *table, uint32_t n_lines, uint32_t blocks, uint32_t steps, int chase,
                         float *sink, hipStream_t s);

// --- point-cloud compaction (compact.hip) ---
// counts: compact_blocks(n) device words of scratch; count: one device word
uint64_t compact_blocks(uint64_t n);
// the allocation-free variant's counts: a static device array per GPU (compact_static_max_beams() beams);
// compact_static_init (device current) looks its address up once per device
uint64_t compact_static_max_beams();
hipError_t compact_static_init(int device);
uint32_t *compact_static_counts(int device);
void launch_compact(const Outputs &dense, const Outputs &comp, uint32_t *beam_index, uint32_t *count, uint64_t n,
                    uint32_t *counts, hipStream_t s);

// --- adjoint (adjoint.hip) ---
constexpr int kAdjBlock = 256;
size_t adjoint_partial_bytes(uint32_t n_beams, uint32_t nmat);
void launch_adjoint(const SceneDev &S, const uint32_t *slot_of, const InstanceDev &in, const MaterialsDev &M,
                    const Overrides &ov,
                    const uint32_t *tri, const uint8_t *valid, const float *clamp_I, const float *gI, const float *gd,
                    double *partials,
                    float *d_rho, float *d_k, float *d_pose6, float *d_spectra, hipStream_t s);

}  // namespace lidar
