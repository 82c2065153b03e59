// lidar_api.cpp -- the C ABI (include/lidar.h): argument checks on the host,
// context state, and stream-ordered launches of the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lidar.h"
#include "lidar_kernels.hpp"

using namespace lidar;

namespace {

constexpr int kMaxStack = 96;
constexpr uint64_t kRedoMax = 1ull << 22;   // rays a batch's short-stack pass can list for the second pass
constexpr uint32_t kMaxAdjMaterials = 256;

thread_local std::string g_create_error;

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= n) return hipSuccess;
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = bytes;
        return e;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct SensorHost {
    lidar_sensor_desc d;
    std::vector<double> elev;
};

struct MeshHost {
    MeshDev dev;
    BuildResult br;
    Node4 *nodes;
    TriRec *recs;
    const uint32_t *idx;    // device copy of the indices (in the mesh workspace)
    uint64_t nv;
};

constexpr uint32_t kMaxMeshes = 4096;
constexpr uint32_t kMaxActors = 1u << 20;

}  // namespace

struct lidar_ctx {
    int device = 0;
    int n_cu = 256;
    std::string err;
    // scene
    bool has_scene = false;
    SceneDev S{};
    const uint32_t *slot_of = nullptr;
    BuildResult br{};
    int stack = 32;
    int stack_cap_opt = 0;   // LIDAR_OPT_STACK_CAP (0: the whole stack)
    std::vector<lidar_batch *> batches;   // live batches made on this context (detached by lidar_destroy)
    int batch_stack_opt = 0;   // LIDAR_OPT_BATCH_STACK (0: automatic, -1: off, n: first-pass cap n)
    uint32_t leaf_width = 4;
    float build_ms = 0.f;
    // materials
    bool has_mat = false;
    DevBuf mat_buf;
    MaterialsDev M{};
    std::vector<float> sigma_h;
    // sensor
    bool has_sensor = false;
    SensorHost sensor;
    DevBuf sensor_tables;   // elev_cs then az_cs
    DevBuf adj_partials;
    // pose
    float p[3] = {0, 0, 0};
    float q[4] = {1, 0, 0, 0};
    // device words: [0] error flags, [1] queue counter, [2..3] refit scratch, [4] rays of the last batch
    // launch traced again by its second pass
    DevBuf words;
    int tile_az_log2 = -1;    // -1: automatic (tile_log2())
    int lanes_per_ray = 4;
    int xcd_remap = 1;
    int actor_tree_opt = 0;   // LIDAR_OPT_ACTOR_TREE (0: packed rebuild up to kPackedTlasMax actors)
    // dynamic scene: meshes and the actors placing them
    std::vector<MeshHost> meshes;
    DevBuf mesh_table;        // MeshDev[kMaxMeshes]
    bool has_actors = false;
    bool tlas_stale = false;  // a mesh was refit after the actors' boxes were computed
    bool tlas_packed = false; // the top-level tree is rebuilt by every update (else refit)
    ActorsDev A{};
    BuildResult tlas_br{};
    TriRec *tlas_recs = nullptr;
    ActorDev *actors_dev = nullptr;
    float *actor_lohi = nullptr;
    std::vector<uint32_t> actor_mesh;
    std::vector<ActorDev> actor_host;
    // pinned, device-mapped upload buffers of lidar_actors_update: a ring of staging_slots slots of
    // staging_n actors in two halves.  An event is recorded after the work that reads the last slot of a
    // half, and the host waits for it before it writes the first slot of that half again: one event per
    // half a ring instead of one per update (each event on the stream costs the GPU a few microseconds).
    ActorDev *staging = nullptr;
    const ActorDev *staging_dev = nullptr;
    size_t staging_n = 0;
    uint32_t staging_slots = 0;
    uint64_t staging_next = 0;
    hipStream_t staging_stream = nullptr;   // the stream of the ring's last use (valid once staging_used)
    bool staging_used = false;
    hipEvent_t staging_ev[2] = {nullptr, nullptr};
    int actor_stack = 0;
    float actor_reach_need = 0.f;   // twice the largest coordinate of any placed mesh
    // generations: bumped when the scene (or its stack cap) or the materials change, so that a
    // batch's captured graph, which holds their device pointers by value, is captured again
    uint64_t scene_gen = 1, mat_gen = 1;

    int trace_stack() const { return has_actors && actor_stack > stack ? actor_stack : stack; }
    // automatic tile shape (measured on the 64 x 2048 scan): 2 azimuth steps x 32 channels for the
    // static scene, 8 x 8 with actors (their nested mesh walks diverge less), 16 x 4 for batches
    int tile_log2() const { return tile_az_log2 >= 0 ? tile_az_log2 : (has_actors ? 3 : 1); }
    int batch_tile_log2() const { return tile_az_log2 >= 0 ? tile_az_log2 : 4; }
    TraceOpts opts(int tile) const { return TraceOpts{trace_stack(), tile, lanes_per_ray, xcd_remap}; }
    uint32_t *refit_word() const { return (uint32_t *)words.p + 2; }

    lidar_status fail(lidar_status st, const std::string &msg) {
        err = msg;
        return st;
    }
    lidar_status hip_fail(hipError_t e, const char *what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LIDAR_ERR_HIP;
    }
};

struct lidar_batch {
    lidar_ctx *ctx = nullptr;   // null once the context is destroyed (then only lidar_batch_destroy applies)
    int device = 0;
    uint32_t n_inst = 0;
    std::vector<InstanceDev> h_insts;   // pointers into `tables`
    DevBuf d_insts;
    DevBuf tables;
    uint64_t n_rays = 0, n_padded = 0;
    uint32_t packet = 256;
    int tile_az_log2 = 3;      // tile shape fixed at creation (padded ray layout depends on it)
    TraceOpts graph_opts{-1, -1, -1, -1};
    uint64_t graph_scene_gen = 0, graph_mat_gen = 0;   // context generations the graph was captured at
    uint64_t inst_mat_gen = 0;                         // material generation of the instances' t_trace
    DevBuf redo;                                       // rays the first pass lists for the second
    uint32_t redo_cap = 0;
    int graph_first_stack = -1, graph_first_cap = -1;  // first-pass stack the graph was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Outputs bound{};
    bool has_graph = false;
    hipStream_t cap_stream = nullptr;
    void drop_graph() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        has_graph = false;
    }
};

namespace {

// collapse options of a scene or mesh build from the descriptor flags
constexpr float kDefaultLeafCost = 1.5f;   // a leaf step costs about 1.5 node steps of the walk
void set_collapse(BuildInputs &in, uint32_t flags) {
    in.collapse = (flags & LIDAR_SCENE_COLLAPSE_GREEDY) ? 1u : 0u;
    const uint32_t sixteenths = (flags >> 16) & 0xFFu;
    in.leaf_cost = sixteenths ? (float)sixteenths / 16.0f : kDefaultLeafCost;
}

bool finite3(const float *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

lidar_status check_sensor(lidar_ctx *ctx, const lidar_sensor_desc *d) {
    if (!d) return ctx->fail(LIDAR_ERR_INVALID_ARG, "sensor descriptor is null");
    if (d->n_ch < 1 || d->n_ch > 4096) return ctx->fail(LIDAR_ERR_INVALID_ARG, "n_ch must be in 1..4096");
    if (d->n_az < 1 || d->n_az > (1u << 20)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "n_az must be in 1..2^20");
    if ((uint64_t)d->n_ch * d->n_az >= (1ull << 31)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "too many beams");
    if (!d->elev_deg) return ctx->fail(LIDAR_ERR_INVALID_ARG, "elev_deg is null");
    for (uint32_t j = 0; j < d->n_ch; ++j)
        if (!std::isfinite(d->elev_deg[j]) || std::fabs(d->elev_deg[j]) > 90.0)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "elevations must be finite and within [-90, 90] deg");
    if (!std::isfinite(d->az0_deg) || !std::isfinite(d->fov_h_deg) || d->fov_h_deg <= 0.0 || d->fov_h_deg > 360.0)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "fov_h_deg must be in (0, 360]");
    if (!(d->d_max > 0.f) || !std::isfinite(d->d_max)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "d_max must be > 0");
    if (!(d->t_min >= 0.f) || !(d->t_min < d->d_max)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "need 0 <= t_min < d_max");
    if (!(d->r_l_max >= 0.f) || !std::isfinite(d->r_l_max)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "r_l_max must be >= 0");
    if (!(d->sigma_intensity >= 0.f) || !std::isfinite(d->sigma_intensity))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "sigma_intensity must be >= 0");
    if (!std::isfinite(d->wavelength_nm)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "wavelength must be finite");
    return LIDAR_OK;
}

bool wavelength_clamped(const lidar_ctx *ctx, float lam) {
    if (!ctx->has_mat) return false;
    float q = (lam - ctx->M.lambda0) / ctx->M.dlambda;
    return q < 0.0f || q > (float)(ctx->M.nbins - 1);
}

lidar_status check_quat(lidar_ctx *ctx, const float *p, const float *q) {
    if (!p || !q) return ctx->fail(LIDAR_ERR_INVALID_ARG, "pose pointer is null");
    if (!finite3(p) || !std::isfinite(q[0]) || !finite3(q + 1))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "pose has NaN/inf");
    double n = std::sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    if (std::fabs(n - 1.0) > 1e-4) return ctx->fail(LIDAR_ERR_INVALID_ARG, "quaternion is not unit (|q| - 1 > 1e-4)");
    return LIDAR_OK;
}

float trace_limit(const lidar_ctx *ctx, float d_max, bool noise_on) {
    if (!noise_on) return d_max;
    float smax = 0.f;
    for (float s : ctx->sigma_h) smax = std::max(smax, s);
    return d_max + kBoxMullerBound * smax;
}

float trace_limit(const lidar_ctx *ctx, const lidar_sensor_desc &d) { return trace_limit(ctx, d.d_max, d.noise_on != 0); }

// LIDAR_WARN_ORIGIN_OUTSIDE_SCENE if a scene is loaded and p lies outside its cube, else 0
lidar_status origin_warning(const lidar_ctx *ctx, const float *p) {
    if (!ctx->has_scene) return LIDAR_OK;
    return lidar_origin_check(ctx->br.max_abs, p) == LIDAR_WARN_ORIGIN_OUTSIDE_SCENE ? LIDAR_WARN_ORIGIN_OUTSIDE_SCENE
                                                                                       : LIDAR_OK;
}

// with actors: the object-space origin of a mesh walk is within the traceable range plus the mesh's
// extent of the mesh origin; warn when that can exceed the reach its boxes were padded for
lidar_status actor_reach_warning(const lidar_ctx *ctx, const lidar_sensor_desc &d) {
    if (!ctx->has_actors) return LIDAR_OK;
    return trace_limit(ctx, d) + ctx->actor_reach_need > LIDAR_MESH_REACH ? LIDAR_WARN_ORIGIN_OUTSIDE_SCENE : LIDAR_OK;
}

uint32_t tiles_az(int tile_az_log2, uint32_t n_az) {
    uint32_t ta = 1u << tile_az_log2;
    return (n_az + ta - 1) / ta;
}

uint64_t padded_rays(int tile_az_log2, uint32_t n_ch, uint32_t n_az) {
    uint32_t tc = 64u >> tile_az_log2;
    uint64_t rows = (n_ch + tc - 1) / tc;
    return rows * tiles_az(tile_az_log2, n_az) * 64ull;
}

InstanceDev make_instance(const lidar_ctx *ctx, int tile_az_log2, const lidar_sensor_desc &d, const double *elev_cs,
                          const double *az_cs, const float *p, const float *q, uint64_t seed, uint32_t scan,
                          uint32_t inst_id, uint64_t ray_base, uint64_t out_base) {
    InstanceDev in{};
    in.elev_cs = elev_cs;
    in.az_cs = az_cs;
    in.n_ch = d.n_ch;
    in.n_az = d.n_az;
    in.tiles_az = tiles_az(tile_az_log2, d.n_az);
    in.tiles_ch = (d.n_ch + (64u >> tile_az_log2) - 1) / (64u >> tile_az_log2);
    in.ray_base = ray_base;
    in.out_base = out_base;
    for (int k = 0; k < 4; ++k) in.q[k] = q[k];
    for (int k = 0; k < 3; ++k) in.p[k] = p[k];
    in.wavelength_nm = d.wavelength_nm;
    in.d_max = d.d_max;
    in.r_l_max = d.r_l_max;
    in.t_min = d.t_min + 0.0f;   // -0 becomes +0 (the box test compares bit patterns)
    in.sigma_i = d.sigma_intensity;
    in.t_trace = trace_limit(ctx, d);
    in.noise_on = d.noise_on ? 1u : 0u;
    in.seed_lo = (uint32_t)(seed & 0xFFFFFFFFu);
    in.seed_hi = (uint32_t)(seed >> 32);
    in.scan = scan;
    in.inst_id = inst_id;
    in.sweep = 0;
    in.sw = SweepDev{};
    in.n_cols = d.n_az;
    in.seg_n0 = d.n_az;
    in.seg_i0[0] = in.seg_i0[1] = 0;
    return in;
}

Outputs to_outputs(const lidar_outputs *o, uint64_t plane) {
    Outputs r{};
    r.x = o->x; r.y = o->y; r.z = o->z; r.intensity = o->intensity; r.label = o->label; r.valid = o->valid;
    r.range = o->range; r.tri = o->tri; r.t_hit = o->t_hit; r.material = o->material; r.normal = o->normal;
    r.r_lambda = o->r_lambda; r.plane = plane;
    return r;
}

bool same_outputs(const Outputs &a, const Outputs &b) { return std::memcmp(&a, &b, sizeof(Outputs)) == 0; }

lidar_status ready(lidar_ctx *ctx, bool need_sensor) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!ctx->has_scene) return ctx->fail(LIDAR_ERR_NOT_READY, "no scene loaded");
    if (!ctx->has_mat) return ctx->fail(LIDAR_ERR_NOT_READY, "no materials set");
    if (need_sensor && !ctx->has_sensor) return ctx->fail(LIDAR_ERR_NOT_READY, "no sensor set");
    if (ctx->br.max_material >= ctx->M.nmat)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "scene uses a material id >= nmat");
    if (ctx->has_actors) {
        if (ctx->tlas_stale)
            return ctx->fail(LIDAR_ERR_NOT_READY, "a mesh was refit: call lidar_actors_update before simulating");
        for (uint32_t m : ctx->actor_mesh)
            if (ctx->meshes[m].br.max_material >= ctx->M.nmat)
                return ctx->fail(LIDAR_ERR_INVALID_ARG, "a mesh uses a material id >= nmat");
    }
    return LIDAR_OK;
}

lidar_status no_actors(lidar_ctx *ctx, const char *what) {
    if (ctx->has_actors)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, std::string(what) + " covers the static scene only: clear the actors");
    return LIDAR_OK;
}

int stack_for_depth(uint32_t depth) {
    int need = 3 * (int)(depth > 0 ? depth - 1 : 0) + 1;
    if (need <= 32) return 32;
    if (need <= 48) return 48;
    if (need <= 64) return 64;
    if (need <= 96) return 96;
    return -1;
}

}  // namespace

extern "C" {

lidar_status lidar_create(int hip_device, lidar_ctx **out) {
    if (!out) return LIDAR_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        g_create_error = "no HIP device available";
        return LIDAR_ERR_HIP;
    }
    if (hip_device < 0 || hip_device >= n) {
        g_create_error = "device index out of range";
        return LIDAR_ERR_INVALID_ARG;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, hip_device);
    if (e != hipSuccess) {
        g_create_error = hipGetErrorString(e);
        return LIDAR_ERR_HIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("unsupported device ") + prop.gcnArchName + " (gfx950 required)";
        return LIDAR_ERR_UNSUPPORTED_DEVICE;
    }
    lidar_ctx *ctx = new (std::nothrow) lidar_ctx();
    if (!ctx) return LIDAR_ERR_OUT_OF_MEMORY;
    ctx->device = hip_device;
    ctx->n_cu = prop.multiProcessorCount;
    hipSetDevice(hip_device);
    if (ctx->words.ensure(256) != hipSuccess || hipMemset(ctx->words.p, 0, 256) != hipSuccess) {
        delete ctx;
        g_create_error = "device allocation failed";
        return LIDAR_ERR_OUT_OF_MEMORY;
    }
    if ((e = compact_static_init(hip_device)) != hipSuccess) {
        ctx->words.release();
        delete ctx;
        g_create_error = std::string("static scratch lookup failed: ") + hipGetErrorString(e);
        return LIDAR_ERR_HIP;
    }
    *out = ctx;
    return LIDAR_OK;
}

lidar_status lidar_destroy(lidar_ctx *ctx) {
    if (!ctx) return LIDAR_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    ctx->mat_buf.release();
    ctx->sensor_tables.release();
    ctx->adj_partials.release();
    ctx->mesh_table.release();
    if (ctx->staging) hipHostFree(ctx->staging);
    for (hipEvent_t ev : ctx->staging_ev)
        if (ev) hipEventDestroy(ev);
    ctx->words.release();
    for (lidar_batch *b : ctx->batches) b->ctx = nullptr;   // each is freed by its own lidar_batch_destroy
    delete ctx;
    return LIDAR_OK;
}

const char *lidar_last_error(const lidar_ctx *ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

lidar_status lidar_scene_bytes(const lidar_scene_desc *desc, uint64_t *persistent_bytes, uint64_t *scratch_bytes) {
    if (!desc || !persistent_bytes || !scratch_bytes) return LIDAR_ERR_INVALID_ARG;
    if (desc->n_triangles < 1 || desc->n_triangles > LIDAR_MAX_TRIANGLES || desc->n_vertices < 1 ||
        desc->n_vertices >= (1ull << 32))
        return LIDAR_ERR_INVALID_ARG;
    uint32_t nt = (uint32_t)desc->n_triangles;
    *persistent_bytes = build_persistent_bytes(nt);
    uint64_t sc = build_scratch_bytes(nt);
    if (!(desc->flags & LIDAR_SCENE_DEVICE_PTRS)) {
        auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
        sc += al(12 * desc->n_vertices) + al(12 * (uint64_t)nt) + al(2 * (uint64_t)nt) + al(4 * (uint64_t)nt);
    }
    *scratch_bytes = sc;
    return LIDAR_OK;
}

lidar_status lidar_scene_load(lidar_ctx *ctx, const lidar_scene_desc *desc, void *persistent,
                              uint64_t persistent_bytes, void *scratch, uint64_t scratch_bytes, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!desc) return ctx->fail(LIDAR_ERR_INVALID_ARG, "scene descriptor is null");
    if (!desc->vertices || !desc->indices || !desc->material || !desc->label)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "scene array pointer is null");
    uint32_t W = desc->leaf_width ? desc->leaf_width : 4u;
    if (W < 1 || W > 8) return ctx->fail(LIDAR_ERR_INVALID_ARG, "leaf_width must be in 1..8");
    uint64_t need_p = 0, need_s = 0;
    if (lidar_scene_bytes(desc, &need_p, &need_s) != LIDAR_OK)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "triangle count out of 1..LIDAR_MAX_TRIANGLES or vertex count out of range");
    if (!persistent || !scratch) return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspace pointer is null");
    if (((uintptr_t)persistent & 255) || ((uintptr_t)scratch & 255))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspaces must be 256-byte aligned");
    if (persistent_bytes < need_p || scratch_bytes < need_s)
        return ctx->fail(LIDAR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than lidar_scene_bytes()");
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    uint32_t nt = (uint32_t)desc->n_triangles;
    BuildInputs in{};
    in.nv = desc->n_vertices;
    in.nt = nt;
    in.leaf_width = W;
    in.builder = (desc->flags & LIDAR_SCENE_BUILD_LBVH) ? 1u : 0u;
    in.ploc_radius = (desc->flags >> 8) & 0xFFu;
    if (in.ploc_radius == 0) in.ploc_radius = 32;
    if (in.ploc_radius > 128) return ctx->fail(LIDAR_ERR_INVALID_ARG, "PLOC radius (flags bits 8-15) must be <= 128");
    set_collapse(in, desc->flags);
    {
        const uint32_t w128 = (desc->flags >> 24) & 0xFFu;   // horizontal-face weight of the area metric
        in.up_weight = w128 ? (float)w128 / 128.0f : 1.0f;
    }
    if (desc->flags & LIDAR_SCENE_DEVICE_PTRS) {
        in.vtx = desc->vertices;
        in.idx = desc->indices;
        in.mat = desc->material;
        in.label = desc->label;
    } else {
        auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
        char *base = (char *)scratch + build_scratch_bytes(nt);
        float *v = (float *)base;
        uint32_t *ix = (uint32_t *)(base + al(12 * in.nv));
        uint16_t *m = (uint16_t *)((char *)ix + al(12 * (uint64_t)nt));
        uint32_t *lb = (uint32_t *)((char *)m + al(2 * (uint64_t)nt));
        hipError_t e;
        if ((e = hipMemcpyAsync(v, desc->vertices, 12 * in.nv, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(ix, desc->indices, 12 * (uint64_t)nt, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(m, desc->material, 2 * (uint64_t)nt, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(lb, desc->label, 4 * (uint64_t)nt, hipMemcpyHostToDevice, s)) != hipSuccess)
            return ctx->hip_fail(e, "scene upload");
        in.vtx = v;
        in.idx = ix;
        in.mat = m;
        in.label = lb;
    }
    ctx->has_scene = false;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, s);
    BuildResult br{};
    hipError_t e = build_bvh(in, persistent, scratch, br, s);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return ctx->hip_fail(e, "BVH build");
    if (br.bad_index) return ctx->fail(LIDAR_ERR_INVALID_ARG, "a triangle index is >= n_vertices");
    if (br.n_nodes > LIDAR_MAX_NODES)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "the BVH has more than LIDAR_MAX_NODES nodes (2 GiB of nodes)");
    int stack = stack_for_depth(br.depth);
    if (stack < 0) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "BVH depth %u needs more than %d stack entries", br.depth, kMaxStack);
        return ctx->fail(LIDAR_ERR_STACK_OVERFLOW, buf);
    }
    ctx->br = br;
    ctx->stack = stack;
    ctx->leaf_width = W;
    ctx->build_ms = ms;
    ctx->S.nodes = (const Node4 *)persistent;
    ctx->S.tris = (const TriRec *)((const char *)persistent + persistent_nodes_bytes(nt));
    ctx->slot_of = (const uint32_t *)((const char *)ctx->S.tris + persistent_recs_bytes(nt));
    ctx->S.root = br.root;
    ctx->S.n_tri = nt;
    ctx->S.max_steps = br.n_nodes + br.n_leaves + 1;
    ctx->S.stack_cap = ctx->stack_cap_opt > 0 && ctx->stack_cap_opt < stack ? ctx->stack_cap_opt : stack;
    ctx->has_scene = true;
    ++ctx->scene_gen;
    return origin_warning(ctx, ctx->p);
}

lidar_status lidar_materials_set(lidar_ctx *ctx, const lidar_material_desc *d) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!d || !d->spectra || !d->sigma_range) return ctx->fail(LIDAR_ERR_INVALID_ARG, "material arrays are null");
    if (d->nmat < 1 || d->nmat > 65535 || d->nbins < 1 || d->nbins > 4096)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "nmat must be in 1..65535 and nbins in 1..4096");
    if (!(d->dlambda_nm > 0.f) || !std::isfinite(d->lambda0_nm))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "dlambda_nm must be > 0");
    size_t ns = (size_t)d->nmat * d->nbins;
    for (size_t k = 0; k < ns; ++k)
        if (!std::isfinite(d->spectra[k])) return ctx->fail(LIDAR_ERR_INVALID_ARG, "spectra contain NaN/inf");
    for (uint32_t k = 0; k < d->nmat; ++k) {
        if (!(d->sigma_range[k] >= 0.f) || !std::isfinite(d->sigma_range[k]))
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "sigma_range must be finite and >= 0");
        if (d->angle_exp && (!std::isfinite(d->angle_exp[k]) || d->angle_exp[k] < 0.f))
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "angle_exp must be finite and >= 0");
    }
    hipSetDevice(ctx->device);
    size_t bytes = ns * 4 + 2 * (size_t)d->nmat * 4;
    hipError_t e = ctx->mat_buf.ensure(bytes);
    if (e != hipSuccess) return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "material table allocation failed");
    float *base = (float *)ctx->mat_buf.p;
    std::vector<float> host(bytes / 4);
    std::memcpy(host.data(), d->spectra, ns * 4);
    std::memcpy(host.data() + ns, d->sigma_range, (size_t)d->nmat * 4);
    for (uint32_t k = 0; k < d->nmat; ++k) host[ns + d->nmat + k] = d->angle_exp ? d->angle_exp[k] : 1.0f;
    if ((e = hipMemcpy(base, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
        return ctx->hip_fail(e, "material upload");
    ctx->M.spectra = base;
    ctx->M.sigma = base + ns;
    ctx->M.angle_exp = base + ns + d->nmat;
    ctx->M.nmat = d->nmat;
    ctx->M.nbins = d->nbins;
    ctx->M.lambda0 = d->lambda0_nm;
    ctx->M.dlambda = d->dlambda_nm;
    ctx->sigma_h.assign(d->sigma_range, d->sigma_range + d->nmat);
    ctx->has_mat = true;
    ++ctx->mat_gen;
    if (ctx->has_sensor && d->nmat <= kMaxAdjMaterials) {
        size_t pb = adjoint_partial_bytes(ctx->sensor.d.n_ch * ctx->sensor.d.n_az, d->nmat);
        if (ctx->adj_partials.ensure(pb) != hipSuccess)
            return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "adjoint buffer allocation failed");
    }
    return LIDAR_OK;
}

lidar_status lidar_sensor_set(lidar_ctx *ctx, const lidar_sensor_desc *d) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    lidar_status st = check_sensor(ctx, d);
    if (st != LIDAR_OK) return st;
    hipSetDevice(ctx->device);
    size_t bytes = 16 * ((size_t)d->n_ch + d->n_az) + 8 * (size_t)d->n_ch;
    hipError_t e = ctx->sensor_tables.ensure(bytes);
    if (e != hipSuccess) return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "sensor table allocation failed");
    double *elev_cs = (double *)ctx->sensor_tables.p;
    double *az_cs = elev_cs + 2 * (size_t)d->n_ch;
    double *elev_deg = az_cs + 2 * (size_t)d->n_az;
    if ((e = hipMemcpy(elev_deg, d->elev_deg, 8 * (size_t)d->n_ch, hipMemcpyHostToDevice)) != hipSuccess)
        return ctx->hip_fail(e, "sensor upload");
    launch_dir_tables(elev_deg, d->n_ch, d->az0_deg, d->fov_h_deg, d->n_az, elev_cs, az_cs, 0);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return ctx->hip_fail(e, "direction tables");
    ctx->sensor.d = *d;
    ctx->sensor.elev.assign(d->elev_deg, d->elev_deg + d->n_ch);
    ctx->sensor.d.elev_deg = ctx->sensor.elev.data();
    ctx->has_sensor = true;
    if (ctx->has_mat && ctx->M.nmat <= kMaxAdjMaterials) {
        size_t pb = adjoint_partial_bytes(d->n_ch * d->n_az, ctx->M.nmat);
        if (ctx->adj_partials.ensure(pb) != hipSuccess)
            return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "adjoint buffer allocation failed");
    }
    return wavelength_clamped(ctx, d->wavelength_nm) ? LIDAR_WARN_WAVELENGTH_CLAMPED : LIDAR_OK;
}

lidar_status lidar_pose_set(lidar_ctx *ctx, const float p[3], const float q[4]) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    lidar_status st = check_quat(ctx, p, q);
    if (st != LIDAR_OK) return st;
    std::memcpy(ctx->p, p, 12);
    std::memcpy(ctx->q, q, 16);
    return origin_warning(ctx, p);
}

lidar_status lidar_origin_check(float max_abs_coord, const float p[3]) {
    if (!p || !finite3(p) || !std::isfinite(max_abs_coord)) return LIDAR_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k)
        if (!(std::fabs(p[k]) <= max_abs_coord)) return LIDAR_WARN_ORIGIN_OUTSIDE_SCENE;
    return LIDAR_OK;
}

static lidar_status simulate_common(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_params *params,
                                    const lidar_outputs *out, void *stream, bool brute, uint32_t *n_nodes = nullptr,
                                    uint32_t *n_tris = nullptr) {
    lidar_status st = ready(ctx, true);
    if (st != LIDAR_OK) return st;
    if (!out) return ctx->fail(LIDAR_ERR_INVALID_ARG, "outputs struct is null");
    if (brute && (st = no_actors(ctx, "the brute-force reference")) != LIDAR_OK) return st;
    if (n_nodes && (st = no_actors(ctx, "traversal counting")) != LIDAR_OK) return st;
    const lidar_sensor_desc &d = ctx->sensor.d;
    const double *elev_cs = (const double *)ctx->sensor_tables.p;
    const double *az_cs = elev_cs + 2 * (size_t)d.n_ch;
    InstanceDev in = make_instance(ctx, ctx->tile_log2(), d, elev_cs, az_cs, ctx->p, ctx->q, seed, scan, 0, 0, 0);
    Overrides ov{};
    if (params) {
        if (params->rho && params->spectra)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "params: give rho or spectra, not both");
        ov.rho = params->rho;
        ov.angle_exp = params->angle_exp;
        ov.pose_delta = params->pose_delta;
        ov.spectra = params->spectra;
    }
    uint64_t nb = (uint64_t)d.n_ch * d.n_az;
    Outputs o = to_outputs(out, nb);
    uint64_t np = padded_rays(ctx->tile_log2(), d.n_ch, d.n_az);
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (brute) launch_bruteforce(ctx->S, in, ctx->M, ov, o, ctx->tile_log2(), np, s);
    else launch_trace_scan(ctx->opts(ctx->tile_log2()), ctx->S, in, ctx->M, ov, o, np, (uint32_t *)ctx->words.p,
                           n_nodes, n_tris, ctx->has_actors ? &ctx->A : nullptr, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "trace launch");
    return (wavelength_clamped(ctx, d.wavelength_nm) && !(params && params->rho) ? LIDAR_WARN_WAVELENGTH_CLAMPED
                                                                                 : LIDAR_OK) |
           actor_reach_warning(ctx, d);
}

lidar_status lidar_simulate(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_outputs *out, void *stream) {
    return simulate_common(ctx, seed, scan, nullptr, out, stream, false);
}

lidar_status lidar_simulate_ex(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_params *params,
                               const lidar_outputs *out, void *stream) {
    return simulate_common(ctx, seed, scan, params, out, stream, false);
}

lidar_status lidar_simulate_bruteforce(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_outputs *out,
                                       void *stream) {
    return simulate_common(ctx, seed, scan, nullptr, out, stream, true);
}

lidar_status lidar_simulate_counts(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_outputs *out,
                                   uint32_t *node_visits, uint32_t *tri_tests, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!node_visits || !tri_tests) return ctx->fail(LIDAR_ERR_INVALID_ARG, "count arrays are null");
    return simulate_common(ctx, seed, scan, nullptr, out, stream, false, node_visits, tri_tests);
}

// ---------------------------------------------------------------------------
// point-cloud compaction
// ---------------------------------------------------------------------------
constexpr uint64_t kMaxCompactBeams = 1ull << 31;

lidar_status lidar_compact_bytes(uint64_t n_beams, uint64_t *workspace_bytes) {
    if (!workspace_bytes || n_beams > kMaxCompactBeams) return LIDAR_ERR_INVALID_ARG;
    *workspace_bytes = std::max<uint64_t>(256, (4 * compact_blocks(n_beams) + 255) / 256 * 256);
    return LIDAR_OK;
}

static lidar_status check_compact(lidar_ctx *ctx, const lidar_outputs *dense, uint64_t n_beams,
                                  const lidar_outputs *compact, const uint32_t *count) {
    if (!dense || !compact) return ctx->fail(LIDAR_ERR_INVALID_ARG, "outputs struct is null");
    if (!dense->valid && n_beams) return ctx->fail(LIDAR_ERR_INVALID_ARG, "dense outputs need the valid array");
    if (!count) return ctx->fail(LIDAR_ERR_INVALID_ARG, "count pointer is null");
    if (n_beams > kMaxCompactBeams) return ctx->fail(LIDAR_ERR_INVALID_ARG, "more than 2^31 beams");
    const void *pairs[][2] = {{compact->x, dense->x}, {compact->y, dense->y}, {compact->z, dense->z},
                              {compact->intensity, dense->intensity}, {compact->label, dense->label},
                              {compact->valid, dense->valid}, {compact->range, dense->range},
                              {compact->tri, dense->tri}, {compact->t_hit, dense->t_hit},
                              {compact->material, dense->material}, {compact->normal, dense->normal},
                              {compact->r_lambda, dense->r_lambda}};
    for (const auto &pr : pairs)
        if (pr[0] && !pr[1]) return ctx->fail(LIDAR_ERR_INVALID_ARG, "a compact field has no dense source");
    return LIDAR_OK;
}

lidar_status lidar_compact_points(lidar_ctx *ctx, const lidar_outputs *dense, uint64_t n_beams,
                                  const lidar_outputs *compact, uint32_t *beam_index, uint32_t *count,
                                  void *workspace, uint64_t workspace_bytes, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    lidar_status st = check_compact(ctx, dense, n_beams, compact, count);
    if (st != LIDAR_OK) return st;
    uint64_t need = 0;
    lidar_compact_bytes(n_beams, &need);
    if (!workspace || ((uintptr_t)workspace & 255)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < need) return ctx->fail(LIDAR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than lidar_compact_bytes()");
    hipSetDevice(ctx->device);
    launch_compact(to_outputs(dense, n_beams), to_outputs(compact, n_beams), beam_index, count, n_beams,
                   (uint32_t *)workspace, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "compaction launch");
    return LIDAR_OK;
}

lidar_status lidar_compact_points_noalloc(lidar_ctx *ctx, const lidar_outputs *dense, uint64_t n_beams,
                                          const lidar_outputs *compact, uint32_t *beam_index, uint32_t *count,
                                          void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    lidar_status st = check_compact(ctx, dense, n_beams, compact, count);
    if (st != LIDAR_OK) return st;
    if (n_beams > compact_static_max_beams())
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "n_beams above LIDAR_COMPACT_NOALLOC_MAX_BEAMS (the static scratch "
                                                "holds the counts of 2^25 beams): use lidar_compact_points");
    uint32_t *counts = compact_static_counts(ctx->device);   // the device address, never the array's name
    if (!counts) return ctx->fail(LIDAR_ERR_NOT_READY, "static scratch of this device not set up");
    hipSetDevice(ctx->device);
    launch_compact(to_outputs(dense, n_beams), to_outputs(compact, n_beams), beam_index, count, n_beams, counts,
                   (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "compaction launch");
    return LIDAR_OK;
}

// ---------------------------------------------------------------------------
// partial sweep per engine tick
// ---------------------------------------------------------------------------
// The parts of a tick's column poses shared by all its columns (see SweepDev):
// the end quaternions as given and normalised, qb turned to qa's hemisphere,
// and the arc between them.
static SweepDev sweep_dev(double a, double b, const lidar_sensor_desc &d, const lidar_sweep_desc *sw) {
    SweepDev S{};
    S.a = a;
    S.b = b;
    S.az0 = d.az0_deg;
    S.step = d.fov_h_deg / (double)d.n_az;
    double na = 0.0, nb = 0.0;
    for (int e = 0; e < 4; ++e) {
        S.qa[e] = sw->q_begin[e];
        S.qb[e] = sw->q_end[e];
        na += S.qa[e] * S.qa[e];
        nb += S.qb[e] * S.qb[e];
    }
    na = std::sqrt(na);
    nb = std::sqrt(nb);
    double dot = 0.0;
    for (int e = 0; e < 4; ++e) {
        S.ua[e] = S.qa[e] / na;
        S.ub[e] = S.qb[e] / nb;
        dot += S.ua[e] * S.ub[e];
    }
    if (dot < 0.0) {
        for (int e = 0; e < 4; ++e) {
            S.qb[e] = -S.qb[e];
            S.ub[e] = -S.ub[e];
        }
        dot = -dot;
    }
    S.w = std::acos(std::fmin(dot, 1.0));
    S.chord = S.w < 1e-6 ? 1u : 0u;
    S.inv_sin_w = S.chord ? 0.0 : 1.0 / std::sin(S.w);
    for (int e = 0; e < 3; ++e) {
        S.pa[e] = sw->p_begin[e];
        S.pb[e] = sw->p_end[e];
    }
    return S;
}

lidar_status lidar_simulate_sweep(lidar_ctx *ctx, const lidar_sweep_desc *sw, const lidar_outputs *out,
                                  lidar_sweep_info *info, void *stream) {
    lidar_status st = ready(ctx, true);
    if (st != LIDAR_OK) return st;
    if (!sw) return ctx->fail(LIDAR_ERR_INVALID_ARG, "sweep descriptor is null");
    if (!out) return ctx->fail(LIDAR_ERR_INVALID_ARG, "outputs struct is null");
    if ((st = check_quat(ctx, sw->p_begin, sw->q_begin)) != LIDAR_OK) return st;
    if ((st = check_quat(ctx, sw->p_end, sw->q_end)) != LIDAR_OK) return st;
    if (!std::isfinite(sw->head_deg) || !std::isfinite(sw->spin_hz) || !(sw->spin_hz > 0.0) ||
        !std::isfinite(sw->dt_s) || !(sw->dt_s >= 0.0))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "need finite head_deg, spin_hz > 0 and dt_s >= 0");
    const lidar_sensor_desc &d = ctx->sensor.d;
    const double a = sw->head_deg;
    const double b = a + 360.0 * sw->spin_hz * sw->dt_s;
    if (!(b - a <= 360.0)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "a tick may sweep at most 360 degrees");
    const double s_a = std::floor((a - d.az0_deg) / 360.0);
    if (s_a + 1.0 >= 4294967295.0) return ctx->fail(LIDAR_ERR_INVALID_ARG, "revolution index out of range");
    // fired columns: ceil(c_s(a)) <= i < ceil(c_s(b)), c_s(x) = ((x - az0) - 360 s) n_az / fov_h
    uint32_t run_scan[2] = {0, 0}, run_first[2] = {0, 0}, run_count[2] = {0, 0}, n_runs = 0;
    for (int r = 0; r < 2; ++r) {
        double sr = s_a + r;
        if (sr < 0.0) continue;
        double ca = ((a - d.az0_deg) - 360.0 * sr) * (double)d.n_az / d.fov_h_deg;
        double cb = ((b - d.az0_deg) - 360.0 * sr) * (double)d.n_az / d.fov_h_deg;
        double lo = std::max(0.0, std::ceil(ca));
        double hi = std::min((double)d.n_az, std::ceil(cb));
        if (hi > lo) {
            run_scan[n_runs] = (uint32_t)sr;
            run_first[n_runs] = (uint32_t)lo;
            run_count[n_runs] = (uint32_t)(hi - lo);
            ++n_runs;
        }
    }
    uint32_t n_cols = run_count[0] + run_count[1];
    if (n_runs == 2 && run_scan[1] != run_scan[0] + 1)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "internal: runs are not in consecutive revolutions");
    if (n_cols > d.n_az) return ctx->fail(LIDAR_ERR_INVALID_ARG, "internal: more columns than azimuth steps");
    if (info) {
        info->n_runs = n_runs;
        info->n_columns = n_cols;
        for (int r = 0; r < 2; ++r) {
            info->scan[r] = run_scan[r];
            info->first[r] = run_first[r];
            info->count[r] = run_count[r];
        }
    }
    lidar_status ok = (wavelength_clamped(ctx, d.wavelength_nm) ? LIDAR_WARN_WAVELENGTH_CLAMPED : LIDAR_OK) |
                      origin_warning(ctx, sw->p_begin) | origin_warning(ctx, sw->p_end) | actor_reach_warning(ctx, d);
    if (n_cols == 0) return ok;
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const double *elev_cs = (const double *)ctx->sensor_tables.p;
    const double *az_cs = elev_cs + 2 * (size_t)d.n_ch;
    InstanceDev in = make_instance(ctx, ctx->tile_log2(), d, elev_cs, az_cs, sw->p_begin, sw->q_begin, sw->seed,
                                   run_scan[0], 0, 0, 0);
    in.sweep = 1;
    in.sw = sweep_dev(a, b, d, sw);
    in.n_cols = n_cols;
    in.seg_n0 = run_count[0];
    in.seg_i0[0] = run_first[0];
    in.seg_i0[1] = run_first[1];
    in.tiles_az = tiles_az(ctx->tile_log2(), n_cols);
    uint64_t nb = (uint64_t)d.n_ch * d.n_az;
    Outputs o = to_outputs(out, nb);
    uint64_t np = padded_rays(ctx->tile_log2(), d.n_ch, n_cols);
    launch_trace_scan(ctx->opts(ctx->tile_log2()), ctx->S, in, ctx->M, Overrides{}, o, np,
                      (uint32_t *)ctx->words.p, nullptr, nullptr, ctx->has_actors ? &ctx->A : nullptr, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "sweep launch");
    return ok;
}

// ---------------------------------------------------------------------------
// divergent beams and multi-echo returns
// ---------------------------------------------------------------------------
static lidar_status check_echo(lidar_ctx *ctx, const lidar_echo_desc *d) {
    if (!d) return ctx->fail(LIDAR_ERR_INVALID_ARG, "echo descriptor is null");
    if (d->n_sub < 1 || d->n_sub > (uint32_t)kMaxSub) return ctx->fail(LIDAR_ERR_INVALID_ARG, "n_sub must be in 1..16");
    if (d->max_echoes < 1 || d->max_echoes > (uint32_t)kMaxEchoes)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "max_echoes must be in 1..4");
    if (!std::isfinite(d->divergence_rad) || !(d->divergence_rad >= 0.0f) || !(d->divergence_rad < 0.5f))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "divergence_rad must be in [0, 0.5)");
    if (!std::isfinite(d->echo_sep_m) || !(d->echo_sep_m > 0.0f))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "echo_sep_m must be > 0");
    return LIDAR_OK;
}

lidar_status lidar_echo_bytes(lidar_ctx *ctx, const lidar_echo_desc *echo, uint64_t *workspace_bytes) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!workspace_bytes) return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspace_bytes is null");
    if (!ctx->has_sensor) return ctx->fail(LIDAR_ERR_NOT_READY, "no sensor set");
    lidar_status st = check_echo(ctx, echo);
    if (st != LIDAR_OK) return st;
    *workspace_bytes = (uint64_t)ctx->sensor.d.n_ch * ctx->sensor.d.n_az * echo->n_sub * sizeof(SubHit);
    return LIDAR_OK;
}

lidar_status lidar_simulate_echoes(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_echo_desc *echo,
                                   void *workspace, uint64_t workspace_bytes, const lidar_outputs *out,
                                   void *stream) {
    lidar_status st = ready(ctx, true);
    if (st != LIDAR_OK) return st;
    if ((st = check_echo(ctx, echo)) != LIDAR_OK) return st;
    if (!out) return ctx->fail(LIDAR_ERR_INVALID_ARG, "outputs struct is null");
    if (out->normal) return ctx->fail(LIDAR_ERR_INVALID_ARG, "echo outputs have no normal (pass NULL)");
    uint64_t need = 0;
    lidar_echo_bytes(ctx, echo, &need);
    if (!workspace || ((uintptr_t)workspace & 255)) return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < need) return ctx->fail(LIDAR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than lidar_echo_bytes()");
    const lidar_sensor_desc &d = ctx->sensor.d;
    const double *elev_cs = (const double *)ctx->sensor_tables.p;
    const double *az_cs = elev_cs + 2 * (size_t)d.n_ch;
    InstanceDev in = make_instance(ctx, ctx->tile_log2(), d, elev_cs, az_cs, ctx->p, ctx->q, seed, scan, 0, 0, 0);
    SubrayPattern pat{};
    pat.n_sub = echo->n_sub;
    const double golden = 3.14159265358979323846 * (3.0 - std::sqrt(5.0));
    for (uint32_t k = 0; k < echo->n_sub; ++k) {
        const double r = echo->n_sub == 1 ? 0.0
                                          : (0.5 * (double)echo->divergence_rad) *
                                                std::sqrt((double)k / (double)(echo->n_sub - 1));
        const double b = (double)k * golden;
        pat.c[k][0] = std::cos(r);
        pat.c[k][1] = std::sin(r);
        pat.c[k][2] = std::cos(b);
        pat.c[k][3] = std::sin(b);
    }
    const uint64_t nb = (uint64_t)d.n_ch * d.n_az;
    Outputs o = to_outputs(out, nb);
    const uint64_t np = padded_rays(ctx->tile_log2(), d.n_ch, d.n_az);
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    SubHit *sub = (SubHit *)workspace;
    launch_trace_subrays(ctx->opts(ctx->tile_log2()), ctx->S, in, ctx->M, pat, sub, np, (uint32_t *)ctx->words.p,
                         ctx->has_actors ? &ctx->A : nullptr, s);
    launch_echoes(in, ctx->M, sub, echo->n_sub, echo->max_echoes, echo->echo_sep_m, o, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "echo launch");
    return wavelength_clamped(ctx, d.wavelength_nm) ? LIDAR_WARN_WAVELENGTH_CLAMPED : LIDAR_OK;
}

// ---------------------------------------------------------------------------
// dynamic scenes: meshes placed by actors
// ---------------------------------------------------------------------------
static uint64_t al256(uint64_t x) { return (x + 255) / 256 * 256; }

static void host_rotation(const float q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n = std::sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static int stack_for_need(int need) {
    if (need <= 32) return 32;
    if (need <= 48) return 48;
    if (need <= 64) return 64;
    if (need <= 96) return 96;
    return -1;
}

static int entries_for_depth(uint32_t depth) { return 3 * (int)(depth > 0 ? depth - 1 : 0) + 1; }

lidar_status lidar_mesh_bytes(const lidar_scene_desc *mesh, uint64_t *persistent_bytes, uint64_t *scratch_bytes) {
    if (!mesh || !persistent_bytes || !scratch_bytes) return LIDAR_ERR_INVALID_ARG;
    uint64_t p = 0, sc = 0;
    lidar_status st = lidar_scene_bytes(mesh, &p, &sc);
    if (st != LIDAR_OK) return st;
    *persistent_bytes = al256(p) + al256(12 * mesh->n_triangles);
    *scratch_bytes = sc;
    return LIDAR_OK;
}

lidar_status lidar_mesh_load(lidar_ctx *ctx, const lidar_scene_desc *desc, void *persistent,
                             uint64_t persistent_bytes, void *scratch, uint64_t scratch_bytes, void *stream,
                             uint32_t *mesh_id) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!desc || !mesh_id) return ctx->fail(LIDAR_ERR_INVALID_ARG, "mesh descriptor or mesh_id is null");
    if (!desc->vertices || !desc->indices || !desc->material)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "mesh array pointer is null");
    if (ctx->meshes.size() >= kMaxMeshes) return ctx->fail(LIDAR_ERR_INVALID_ARG, "too many meshes");
    uint32_t W = desc->leaf_width ? desc->leaf_width : 4u;
    if (W < 1 || W > 8) return ctx->fail(LIDAR_ERR_INVALID_ARG, "leaf_width must be in 1..8");
    uint64_t need_p = 0, need_s = 0;
    if (lidar_mesh_bytes(desc, &need_p, &need_s) != LIDAR_OK)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "triangle/vertex count out of range");
    if (!persistent || !scratch) return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspace pointer is null");
    if (((uintptr_t)persistent & 255) || ((uintptr_t)scratch & 255))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspaces must be 256-byte aligned");
    if (persistent_bytes < need_p || scratch_bytes < need_s)
        return ctx->fail(LIDAR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than lidar_mesh_bytes()");
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!ctx->mesh_table.p && (e = ctx->mesh_table.ensure(sizeof(MeshDev) * kMaxMeshes)) != hipSuccess)
        return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "mesh table allocation failed");
    const uint32_t nt = (uint32_t)desc->n_triangles;
    BuildInputs in{};
    in.nv = desc->n_vertices;
    in.nt = nt;
    in.leaf_width = W;
    in.builder = (desc->flags & LIDAR_SCENE_BUILD_LBVH) ? 1u : 0u;
    in.ploc_radius = (desc->flags >> 8) & 0xFFu;
    if (in.ploc_radius == 0) in.ploc_radius = 32;
    if (in.ploc_radius > 128) return ctx->fail(LIDAR_ERR_INVALID_ARG, "PLOC radius (flags bits 8-15) must be <= 128");
    set_collapse(in, desc->flags);
    if (desc->flags & LIDAR_SCENE_DEVICE_PTRS) {
        in.vtx = desc->vertices;
        in.idx = desc->indices;
        in.mat = desc->material;
    } else {
        char *base = (char *)scratch + build_scratch_bytes(nt);
        float *v = (float *)base;
        uint32_t *ix = (uint32_t *)(base + al256(12 * in.nv));
        uint16_t *m = (uint16_t *)((char *)ix + al256(12 * (uint64_t)nt));
        if ((e = hipMemcpyAsync(v, desc->vertices, 12 * in.nv, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(ix, desc->indices, 12 * (uint64_t)nt, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(m, desc->material, 2 * (uint64_t)nt, hipMemcpyHostToDevice, s)) != hipSuccess)
            return ctx->hip_fail(e, "mesh upload");
        in.vtx = v;
        in.idx = ix;
        in.mat = m;
    }
    in.label = nullptr;
    in.reach = LIDAR_MESH_REACH;
    uint32_t *idx_copy = (uint32_t *)((char *)persistent + al256(build_persistent_bytes(nt)));
    if ((e = hipMemcpyAsync(idx_copy, in.idx, 12 * (uint64_t)nt, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return ctx->hip_fail(e, "mesh index copy");
    BuildResult br{};
    if ((e = build_bvh(in, persistent, scratch, br, s)) != hipSuccess) return ctx->hip_fail(e, "mesh BVH build");
    if (br.bad_index) return ctx->fail(LIDAR_ERR_INVALID_ARG, "a triangle index is >= n_vertices");
    if (br.n_nodes > LIDAR_MAX_NODES)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "the mesh BVH has more than LIDAR_MAX_NODES nodes");
    if (!refit_supported(br) || stack_for_need(entries_for_depth(br.depth)) < 0)
        return ctx->fail(LIDAR_ERR_STACK_OVERFLOW, "mesh BVH too deep");
    MeshHost mh{};
    mh.nodes = (Node4 *)persistent;
    mh.recs = (TriRec *)((char *)persistent + persistent_nodes_bytes(nt));
    mh.dev.nodes = mh.nodes;
    mh.dev.tris = mh.recs;
    mh.dev.max_steps = br.n_nodes + br.n_leaves + 1;
    mh.dev.n_tri = nt;
    mh.br = br;
    mh.idx = idx_copy;
    mh.nv = desc->n_vertices;
    ctx->meshes.push_back(mh);
    const uint32_t id = (uint32_t)ctx->meshes.size() - 1;
    if ((e = hipMemcpy((MeshDev *)ctx->mesh_table.p + id, &mh.dev, sizeof(MeshDev), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return ctx->hip_fail(e, "mesh table upload");
    *mesh_id = id;
    return LIDAR_OK;
}

lidar_status lidar_mesh_refit(lidar_ctx *ctx, uint32_t mesh_id, const float *vertices, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (mesh_id >= ctx->meshes.size()) return ctx->fail(LIDAR_ERR_INVALID_ARG, "mesh id out of range");
    if (!vertices) return ctx->fail(LIDAR_ERR_INVALID_ARG, "vertices are null");
    hipSetDevice(ctx->device);
    MeshHost &m = ctx->meshes[mesh_id];
    refit_mesh(m.nodes, m.recs, m.br, m.dev.n_tri, m.idx, vertices, m.nv, ctx->refit_word(), (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "mesh refit");
    if (ctx->has_actors)
        for (uint32_t am : ctx->actor_mesh)
            if (am == mesh_id) ctx->tlas_stale = true;
    return LIDAR_OK;
}

lidar_status lidar_actors_bytes(uint32_t n_actors, uint64_t *persistent_bytes, uint64_t *scratch_bytes) {
    if (!persistent_bytes || !scratch_bytes || n_actors < 1 || n_actors > kMaxActors) return LIDAR_ERR_INVALID_ARG;
    const uint64_t n = n_actors;
    *persistent_bytes = al256(build_persistent_bytes(n_actors)) + al256(sizeof(ActorDev) * n) + al256(24 * n);
    *scratch_bytes = al256(build_scratch_bytes(n_actors)) + al256(24 * n) + al256(12 * n) + al256(2 * n);
    return LIDAR_OK;
}

static lidar_status actor_table(lidar_ctx *ctx, const lidar_actor *actors, uint32_t n, std::vector<ActorDev> &out) {
    out.resize(n);
    uint64_t base = ctx->S.n_tri;
    for (uint32_t k = 0; k < n; ++k) {
        const lidar_actor &a = actors[k];
        if (a.mesh >= ctx->meshes.size()) return ctx->fail(LIDAR_ERR_INVALID_ARG, "actor mesh id out of range");
        lidar_status st = check_quat(ctx, a.p, a.q_wxyz);
        if (st != LIDAR_OK) return st;
        ActorDev d{};
        host_rotation(a.q_wxyz, d.R);
        for (int e = 0; e < 3; ++e) d.p[e] = a.p[e];
        d.mesh = a.mesh;
        d.label = a.label;
        d.tri_base = (uint32_t)base;
        base += ctx->meshes[a.mesh].dev.n_tri;
        if (base >= 0xFFFFFFFFull) return ctx->fail(LIDAR_ERR_INVALID_ARG, "too many triangles in the scene");
        out[k] = d;
    }
    return LIDAR_OK;
}

lidar_status lidar_actors_set(lidar_ctx *ctx, const lidar_actor *actors, uint32_t n_actors, void *persistent,
                              uint64_t persistent_bytes, void *scratch, uint64_t scratch_bytes, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!ctx->has_scene) return ctx->fail(LIDAR_ERR_NOT_READY, "load the static scene before the actors");
    if (n_actors == 0) return lidar_actors_clear(ctx);
    if (!actors) return ctx->fail(LIDAR_ERR_INVALID_ARG, "actors are null");
    uint64_t need_p = 0, need_s = 0;
    if (lidar_actors_bytes(n_actors, &need_p, &need_s) != LIDAR_OK)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "actor count out of range");
    if (!persistent || !scratch) return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspace pointer is null");
    if (((uintptr_t)persistent & 255) || ((uintptr_t)scratch & 255))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "workspaces must be 256-byte aligned");
    if (persistent_bytes < need_p || scratch_bytes < need_s)
        return ctx->fail(LIDAR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than lidar_actors_bytes()");
    std::vector<ActorDev> h;
    lidar_status st = actor_table(ctx, actors, n_actors, h);
    if (st != LIDAR_OK) return st;
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const uint64_t n = n_actors;
    char *P = (char *)persistent, *Sc = (char *)scratch;
    ActorDev *ad = (ActorDev *)(P + al256(build_persistent_bytes(n_actors)));
    float *lohi = (float *)((char *)ad + al256(sizeof(ActorDev) * n));
    float *vtx = (float *)(Sc + al256(build_scratch_bytes(n_actors)));
    uint32_t *idx = (uint32_t *)((char *)vtx + al256(24 * n));
    uint16_t *mat = (uint16_t *)((char *)idx + al256(12 * n));
    ctx->has_actors = false;
    hipError_t e;
    if ((e = hipMemcpyAsync(ad, h.data(), sizeof(ActorDev) * n, hipMemcpyHostToDevice, s)) != hipSuccess)
        return ctx->hip_fail(e, "actor upload");
    const bool packed = ctx->actor_tree_opt == 0 && n_actors <= kPackedTlasMax;
    BuildResult br{};
    if (packed) {
        br = packed_tlas_shape(n_actors, ctx->br.max_abs);    // rays start in the static scene's cube
        rebuild_tlas(ad, ad, n_actors, (const MeshDev *)ctx->mesh_table.p, (uint32_t)ctx->meshes.size(), lohi,
                     (Node4 *)P, (TriRec *)(P + persistent_nodes_bytes(n_actors)), br, s);
        if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
            return ctx->hip_fail(e, "actor BVH build");
    } else {
        actor_boxes(ad, n_actors, (const MeshDev *)ctx->mesh_table.p, lohi, ctx->refit_word(), s);
        actor_prims(lohi, n_actors, vtx, idx, mat, s);
        BuildInputs in{};
        in.vtx = vtx;
        in.idx = idx;
        in.mat = mat;
        in.label = nullptr;
        in.nv = 2 * n;
        in.nt = n_actors;
        in.leaf_width = 4;
        in.builder = 0;
        in.ploc_radius = 32;
        set_collapse(in, 0u);
        in.reach = ctx->br.max_abs;     // rays start in the static scene's cube
        if ((e = build_bvh(in, persistent, scratch, br, s)) != hipSuccess) return ctx->hip_fail(e, "actor BVH build");
    }
    if (!refit_supported(br)) return ctx->fail(LIDAR_ERR_STACK_OVERFLOW, "actor BVH too deep");
    int mesh_need = 0;
    for (const ActorDev &d : h) mesh_need = std::max(mesh_need, entries_for_depth(ctx->meshes[d.mesh].br.depth));
    const int stack = stack_for_need(entries_for_depth(br.depth) + mesh_need);
    if (stack < 0) return ctx->fail(LIDAR_ERR_STACK_OVERFLOW, "actor and mesh BVHs too deep for the traversal stack");
    const uint32_t slots = n_actors <= kPackedTlasMax ? 8u : 2u;
    // the ring's events cover one stream: after updates on another stream (which may since have been
    // destroyed), wait for the device before the ring is reused or freed
    if (ctx->staging_used && ctx->staging_stream != s && (e = hipDeviceSynchronize()) != hipSuccess)
        return ctx->hip_fail(e, "staging wait");
    if (ctx->staging_n < n_actors || ctx->staging_slots != slots) {
        for (hipEvent_t ev : ctx->staging_ev)
            if (ev && (e = hipEventSynchronize(ev)) != hipSuccess) return ctx->hip_fail(e, "staging wait");
        if (ctx->staging) hipHostFree(ctx->staging);
        ctx->staging = nullptr;
        ctx->staging_dev = nullptr;
        ctx->staging_n = 0;
        ctx->staging_slots = 0;
        void *dev = nullptr;
        if ((e = hipHostMalloc((void **)&ctx->staging, slots * sizeof(ActorDev) * n,
                               hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
            return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "pinned staging allocation failed");
        if ((e = hipHostGetDevicePointer(&dev, ctx->staging, 0)) != hipSuccess) {
            hipHostFree(ctx->staging);
            ctx->staging = nullptr;
            return ctx->hip_fail(e, "staging mapping");
        }
        ctx->staging_dev = (const ActorDev *)dev;
        ctx->staging_n = n_actors;
        ctx->staging_slots = slots;
    }
    for (hipEvent_t &ev : ctx->staging_ev) {
        if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
            return ctx->hip_fail(e, "event");
        if ((e = hipEventRecord(ev, s)) != hipSuccess) return ctx->hip_fail(e, "event record");
    }
    ctx->staging_next = 0;
    ctx->staging_stream = s;
    ctx->staging_used = true;
    ctx->tlas_br = br;
    ctx->tlas_recs = (TriRec *)(P + persistent_nodes_bytes(n_actors));
    ctx->actors_dev = ad;
    ctx->actor_lohi = lohi;
    ctx->A.nodes = (const Node4 *)P;
    ctx->A.recs = ctx->tlas_recs;
    ctx->A.actors = ad;
    ctx->A.meshes = (const MeshDev *)ctx->mesh_table.p;
    ctx->A.max_steps = br.n_nodes + br.n_leaves + 1;
    ctx->A.n_actors = n_actors;
    ctx->actor_mesh.resize(n_actors);
    for (uint32_t k = 0; k < n_actors; ++k) ctx->actor_mesh[k] = actors[k].mesh;
    ctx->actor_stack = stack;
    ctx->actor_reach_need = 0.f;
    for (const ActorDev &d : h) ctx->actor_reach_need = std::max(ctx->actor_reach_need, 2.f * ctx->meshes[d.mesh].br.max_abs);
    ctx->tlas_stale = false;
    ctx->tlas_packed = packed;
    ctx->has_actors = true;
    return LIDAR_OK;
}

lidar_status lidar_actors_update(lidar_ctx *ctx, const lidar_actor *actors, uint32_t n_actors, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!ctx->has_actors) return ctx->fail(LIDAR_ERR_NOT_READY, "no actors set");
    if (!actors || n_actors != ctx->A.n_actors)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "update needs the actor count of lidar_actors_set");
    for (uint32_t k = 0; k < n_actors; ++k)
        if (actors[k].mesh != ctx->actor_mesh[k])
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "update keeps every actor's mesh (use lidar_actors_set)");
    lidar_status st = actor_table(ctx, actors, n_actors, ctx->actor_host);
    if (st != LIDAR_OK) return st;
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const uint32_t per_half = ctx->staging_slots / 2;
    const uint32_t slot = (uint32_t)(ctx->staging_next % ctx->staging_slots), half = slot / per_half;
    if (s != ctx->staging_stream) {
        // the events cover one stream's work: before switching, wait for the device (the previous
        // stream may since have been destroyed)
        if ((e = hipDeviceSynchronize()) != hipSuccess) return ctx->hip_fail(e, "staging wait");
        ctx->staging_stream = s;
    }
    if (slot % per_half == 0 && (e = hipEventSynchronize(ctx->staging_ev[half])) != hipSuccess)
        return ctx->hip_fail(e, "staging wait");
    ActorDev *host = ctx->staging + (size_t)slot * ctx->staging_n;
    std::memcpy(host, ctx->actor_host.data(), sizeof(ActorDev) * n_actors);
    if (ctx->tlas_packed) {
        // the rebuild reads the transforms from the mapped buffer itself: no copy on another engine
        rebuild_tlas(ctx->staging_dev + (size_t)slot * ctx->staging_n, ctx->actors_dev, n_actors,
                     (const MeshDev *)ctx->mesh_table.p, (uint32_t)ctx->meshes.size(), ctx->actor_lohi,
                     (Node4 *)ctx->A.nodes, ctx->tlas_recs, ctx->tlas_br, s);
    } else {
        if ((e = hipMemcpyAsync(ctx->actors_dev, host, sizeof(ActorDev) * n_actors, hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return ctx->hip_fail(e, "actor upload");
        update_tlas(ctx->actors_dev, n_actors, (const MeshDev *)ctx->mesh_table.p, ctx->actor_lohi,
                    (Node4 *)ctx->A.nodes, ctx->tlas_recs, ctx->tlas_br, ctx->refit_word(), s);
    }
    if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "actor update");
    if (slot % per_half == per_half - 1 && (e = hipEventRecord(ctx->staging_ev[half], s)) != hipSuccess)
        return ctx->hip_fail(e, "event record");
    ++ctx->staging_next;
    ctx->tlas_stale = false;
    return LIDAR_OK;
}

lidar_status lidar_actors_clear(lidar_ctx *ctx) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    ctx->has_actors = false;
    ctx->tlas_stale = false;
    ctx->tlas_packed = false;
    ctx->A = ActorsDev{};
    ctx->actor_mesh.clear();
    return LIDAR_OK;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
lidar_status lidar_batch_create(lidar_ctx *ctx, const lidar_instance *inst, uint32_t n_inst, uint32_t packet_rays,
                                lidar_batch **out) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!out) return ctx->fail(LIDAR_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!inst || n_inst == 0) return ctx->fail(LIDAR_ERR_INVALID_ARG, "no instances");
    if (packet_rays % 64 != 0 || packet_rays > 65536)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "packet_rays must be a multiple of 64 (<= 65536)");
    if (!ctx->has_mat) return ctx->fail(LIDAR_ERR_NOT_READY, "materials must be set before a batch");
    bool clamped = false, origin_out = false;
    size_t table_doubles = 0;
    for (uint32_t k = 0; k < n_inst; ++k) {
        lidar_status st = check_sensor(ctx, &inst[k].sensor);
        if (st != LIDAR_OK) return st;
        st = check_quat(ctx, inst[k].p, inst[k].q_wxyz);
        if (st != LIDAR_OK) return st;
        origin_out |= origin_warning(ctx, inst[k].p) != LIDAR_OK;
        table_doubles += 2 * ((size_t)inst[k].sensor.n_ch + inst[k].sensor.n_az) + inst[k].sensor.n_ch;
        clamped |= wavelength_clamped(ctx, inst[k].sensor.wavelength_nm);
    }
    lidar_batch *b = new (std::nothrow) lidar_batch();
    if (!b) return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "batch allocation failed");
    b->ctx = ctx;
    b->device = ctx->device;
    b->n_inst = n_inst;
    b->packet = packet_rays ? packet_rays : 256;
    b->tile_az_log2 = ctx->batch_tile_log2();
    hipSetDevice(ctx->device);
    if (b->tables.ensure(table_doubles * 8) != hipSuccess || b->d_insts.ensure(sizeof(InstanceDev) * n_inst) != hipSuccess) {
        delete b;
        return ctx->fail(LIDAR_ERR_OUT_OF_MEMORY, "batch table allocation failed");
    }
    double *t = (double *)b->tables.p;
    uint64_t ray_base = 0, out_base = 0;
    for (uint32_t k = 0; k < n_inst; ++k) {
        const lidar_sensor_desc &d = inst[k].sensor;
        double *elev_cs = t;
        double *az_cs = elev_cs + 2 * (size_t)d.n_ch;
        double *elev_deg = az_cs + 2 * (size_t)d.n_az;
        t = elev_deg + d.n_ch;
        hipMemcpy(elev_deg, d.elev_deg, 8 * (size_t)d.n_ch, hipMemcpyHostToDevice);
        launch_dir_tables(elev_deg, d.n_ch, d.az0_deg, d.fov_h_deg, d.n_az, elev_cs, az_cs, 0);
        b->h_insts.push_back(make_instance(ctx, b->tile_az_log2, d, elev_cs, az_cs, inst[k].p, inst[k].q_wxyz,
                                           inst[k].seed, inst[k].scan, k, ray_base, out_base));
        ray_base += padded_rays(b->tile_az_log2, d.n_ch, d.n_az);
        out_base += (uint64_t)d.n_ch * d.n_az;
    }
    b->n_padded = ray_base;
    b->n_rays = out_base;
    b->inst_mat_gen = ctx->mat_gen;
    // the list of the short-stack pass: padded ray indices as 32-bit words, up to 2^22 rays (16 MB); a batch
    // of 2^32 padded rays or more runs one pass with the whole stack
    if (b->n_padded < (1ull << 32)) {
        const uint32_t cap = (uint32_t)std::min<uint64_t>(b->n_padded, kRedoMax);
        if (b->redo.ensure(4 * (size_t)cap) == hipSuccess) b->redo_cap = cap;
    }
    hipError_t e = hipMemcpy(b->d_insts.p, b->h_insts.data(), sizeof(InstanceDev) * n_inst, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        b->tables.release();
        b->d_insts.release();
        b->redo.release();
        delete b;
        return ctx->hip_fail(e, "batch upload");
    }
    ctx->batches.push_back(b);
    *out = b;
    return (clamped ? LIDAR_WARN_WAVELENGTH_CLAMPED : LIDAR_OK) | (origin_out ? LIDAR_WARN_ORIGIN_OUTSIDE_SCENE : LIDAR_OK);
}

// The instances' traceable range depends on the material noise: after new materials it is derived
// again and the table re-uploaded (the stream is drained first: a replay may still read it).
static lidar_status refresh_batch(lidar_ctx *ctx, lidar_batch *b, hipStream_t s) {
    if (b->inst_mat_gen == ctx->mat_gen) return LIDAR_OK;
    for (InstanceDev &in : b->h_insts) in.t_trace = trace_limit(ctx, in.d_max, in.noise_on != 0);
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_insts.p, b->h_insts.data(), sizeof(InstanceDev) * b->n_inst, hipMemcpyHostToDevice);
    if (e != hipSuccess) return ctx->hip_fail(e, "batch instance refresh");
    b->inst_mat_gen = ctx->mat_gen;
    return LIDAR_OK;
}

lidar_status lidar_batch_rays(const lidar_batch *b, uint64_t *n) {
    if (!b || !n) return LIDAR_ERR_INVALID_ARG;
    *n = b->n_rays;
    return LIDAR_OK;
}

// The first pass of a batch (stack entries it is compiled for, entries its walks may use), or (0, 0) for
// one pass with the whole stack.  Automatic: 32 entries when the tree needs more and a ray has one or two
// lanes (their blocks are held to fewer wavefronts by the stack's LDS; quads are held by registers).
static void batch_first_pass(const lidar_ctx *ctx, const lidar_batch *b, int &first_stack, int &first_cap) {
    first_stack = first_cap = 0;
    const int full = ctx->trace_stack();
    const int opt = ctx->batch_stack_opt;
    if (!b->redo_cap || opt < 0) return;
    if (opt == 0) {
        if (full > 32 && ctx->lanes_per_ray != 4) first_stack = first_cap = 32;
        return;
    }
    if (opt >= full) return;
    first_stack = opt <= 32 ? 32 : opt <= 48 ? 48 : opt <= 64 ? 64 : 96;
    first_cap = opt;
}

lidar_status lidar_simulate_batch(lidar_ctx *ctx, lidar_batch *b, const lidar_outputs *out, void *stream) {
    lidar_status st = ready(ctx, false);
    if (st != LIDAR_OK) return st;
    if ((st = no_actors(ctx, "the batched form")) != LIDAR_OK) return st;
    if (!b || b->ctx != ctx || !out) return ctx->fail(LIDAR_ERR_INVALID_ARG, "bad batch or outputs");
    hipSetDevice(ctx->device);
    if ((st = refresh_batch(ctx, b, (hipStream_t)stream)) != LIDAR_OK) return st;
    Outputs o = to_outputs(out, b->n_rays);
    TraceOpts t = ctx->opts(b->tile_az_log2);
    int first_stack = 0, first_cap = 0;
    batch_first_pass(ctx, b, first_stack, first_cap);
    if (!b->has_graph || !same_outputs(o, b->bound) || std::memcmp(&t, &b->graph_opts, sizeof t) != 0 ||
        b->graph_scene_gen != ctx->scene_gen || b->graph_mat_gen != ctx->mat_gen ||
        b->graph_first_stack != first_stack || b->graph_first_cap != first_cap) {
        b->drop_graph();
        uint32_t grid = (uint32_t)(ctx->n_cu * batch_blocks_per_cu(t, first_stack ? first_stack : t.stack));
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return ctx->hip_fail(e, "graph capture begin");
        uint32_t *words = (uint32_t *)ctx->words.p;
        const BatchRedo R{first_stack ? (uint32_t *)b->redo.p : nullptr, words + 4, b->redo_cap, first_stack,
                          first_cap};
        launch_trace_batch(t, ctx->S, (const InstanceDev *)b->d_insts.p, b->n_inst, ctx->M, o, b->n_padded,
                           b->packet, words + 1, words, R, grid, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (e != hipSuccess) return ctx->hip_fail(e, "graph capture end");
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->drop_graph();
            return ctx->hip_fail(e, "graph instantiate");
        }
        b->bound = o;
        b->graph_opts = t;
        b->graph_first_stack = first_stack;
        b->graph_first_cap = first_cap;
        b->graph_scene_gen = ctx->scene_gen;
        b->graph_mat_gen = ctx->mat_gen;
        b->has_graph = true;
    }
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "graph launch");
    return LIDAR_OK;
}

lidar_status lidar_simulate_batch_sequential(lidar_ctx *ctx, lidar_batch *b, const lidar_outputs *out,
                                             void *stream) {
    lidar_status st = ready(ctx, false);
    if (st != LIDAR_OK) return st;
    if ((st = no_actors(ctx, "the batched form")) != LIDAR_OK) return st;
    if (!b || b->ctx != ctx || !out) return ctx->fail(LIDAR_ERR_INVALID_ARG, "bad batch or outputs");
    hipSetDevice(ctx->device);
    if ((st = refresh_batch(ctx, b, (hipStream_t)stream)) != LIDAR_OK) return st;
    Outputs o = to_outputs(out, b->n_rays);
    Overrides ov{};
    for (uint32_t k = 0; k < b->n_inst; ++k) {
        const InstanceDev &in = b->h_insts[k];
        uint64_t np = padded_rays(b->tile_az_log2, in.n_ch, in.n_az);
        launch_trace_scan(ctx->opts(b->tile_az_log2), ctx->S, in, ctx->M, ov, o, np, (uint32_t *)ctx->words.p,
                          nullptr, nullptr, nullptr, (hipStream_t)stream);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "sequential launches");
    return LIDAR_OK;
}

lidar_status lidar_batch_restarted(lidar_ctx *ctx, uint64_t *n_rays) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!n_rays) return ctx->fail(LIDAR_ERR_INVALID_ARG, "n_rays is null");
    hipSetDevice(ctx->device);
    hipError_t e = hipDeviceSynchronize();
    uint32_t w = 0;
    if (e == hipSuccess) e = hipMemcpy(&w, (const uint32_t *)ctx->words.p + 4, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "restart count");
    *n_rays = w;
    return LIDAR_OK;
}

lidar_status lidar_batch_destroy(lidar_batch *b) {
    if (!b) return LIDAR_OK;
    if (b->ctx) {
        std::vector<lidar_batch *> &v = b->ctx->batches;
        v.erase(std::remove(v.begin(), v.end(), b), v.end());
    }
    hipSetDevice(b->device);
    hipDeviceSynchronize();
    b->drop_graph();
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    b->tables.release();
    b->d_insts.release();
    b->redo.release();
    delete b;
    return LIDAR_OK;
}

lidar_status lidar_tune(lidar_ctx *ctx, const lidar_scene_desc *scene, void *persistent, uint64_t persistent_bytes,
                        void *scratch, uint64_t scratch_bytes, lidar_batch *b, const lidar_outputs *out,
                        const lidar_tune_desc *desc, lidar_tune_result *res, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!scene || !b || !out || !desc || !res) return ctx->fail(LIDAR_ERR_INVALID_ARG, "null argument");
    if (b->ctx != ctx) return ctx->fail(LIDAR_ERR_INVALID_ARG, "the batch belongs to another context");
    uint32_t cur_lanes = (uint32_t)ctx->lanes_per_ray;
    const uint32_t *lanes = desc->lanes_per_ray ? desc->lanes_per_ray : &cur_lanes;
    uint32_t n_lanes = desc->lanes_per_ray ? desc->n_lanes : 1;
    // candidate area weights as flags bits 24-31 (128ths, 0 for 1); none: the descriptor's own
    std::vector<uint32_t> ups;
    if (desc->n_packet > 64 || desc->n_leaf > 64 || n_lanes > 64 || (desc->up_weights && desc->n_up > 64))
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "need 1..64 candidate combinations");
    if (desc->up_weights) {
        for (uint32_t i = 0; i < desc->n_up; ++i) {
            const float w = desc->up_weights[i];
            const long w128 = std::isfinite(w) && w > 0.0f && w < 2.0f ? std::lround((double)w * 128.0) : 0;
            if (w128 < 1 || w128 > 255)
                return ctx->fail(LIDAR_ERR_INVALID_ARG, "area weights must be in [1/128, 255/128]");
            ups.push_back(w128 == 128 ? 0u : (uint32_t)w128);
        }
    } else {
        ups.push_back((scene->flags >> 24) & 0xFFu);
    }
    const uint32_t n_up = (uint32_t)ups.size();
    if (!desc->packet_rays || !desc->leaf_widths || desc->n_packet == 0 || desc->n_leaf == 0 || n_lanes == 0 ||
        n_up == 0 || (uint64_t)desc->n_packet * desc->n_leaf * n_lanes * n_up > 64)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "need 1..64 candidate combinations");
    for (uint32_t i = 0; i < desc->n_packet; ++i)
        if (desc->packet_rays[i] == 0 || desc->packet_rays[i] % 64 != 0 || desc->packet_rays[i] > 65536)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "packet sizes must be multiples of 64");
    for (uint32_t i = 0; i < desc->n_leaf; ++i)
        if (desc->leaf_widths[i] < 1 || desc->leaf_widths[i] > 8)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "leaf widths must be in 1..8");
    for (uint32_t i = 0; i < n_lanes; ++i)
        if (lanes[i] != 1 && lanes[i] != 2 && lanes[i] != 4)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "lanes per ray must be 1, 2 or 4");
    uint32_t reps = desc->reps ? desc->reps : 5;
    hipStream_t s = (hipStream_t)stream;
    std::memset(res, 0, sizeof *res);
    res->best_ms = 1e30f;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    lidar_scene_desc sd = *scene;
    lidar_status st = LIDAR_OK;
    uint32_t best_up = ups[0];
    for (uint32_t ui = 0; ui < n_up && st == LIDAR_OK; ++ui)
    for (uint32_t li = 0; li < desc->n_leaf && st == LIDAR_OK; ++li) {
        sd.leaf_width = desc->leaf_widths[li];
        sd.flags = (scene->flags & 0x00FFFFFFu) | (ups[ui] << 24);
        st = lidar_scene_load(ctx, &sd, persistent, persistent_bytes, scratch, scratch_bytes, stream);
        if (st > 0) st = LIDAR_OK;   // a warning (e.g. the pose's origin) does not stop the tuning
        for (uint32_t ni = 0; ni < n_lanes && st == LIDAR_OK; ++ni) {
            ctx->lanes_per_ray = (int)lanes[ni];
            for (uint32_t pi = 0; pi < desc->n_packet && st == LIDAR_OK; ++pi) {
                b->packet = desc->packet_rays[pi];
                b->drop_graph();
                std::vector<float> t;
                for (uint32_t r = 0; r < reps + 1 && st == LIDAR_OK; ++r) {
                    hipEventRecord(e0, s);
                    st = lidar_simulate_batch(ctx, b, out, stream);
                    hipEventRecord(e1, s);
                    hipEventSynchronize(e1);
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    if (r > 0) t.push_back(ms);   // the first run includes the graph capture
                }
                if (st != LIDAR_OK) break;
                std::sort(t.begin(), t.end());
                float med = t[t.size() / 2];
                res->ms[((ui * desc->n_leaf + li) * n_lanes + ni) * desc->n_packet + pi] = med;
                if (med < res->best_ms) {
                    res->best_ms = med;
                    res->best_packet_rays = desc->packet_rays[pi];
                    res->best_leaf_width = desc->leaf_widths[li];
                    res->best_lanes_per_ray = lanes[ni];
                    best_up = ups[ui];
                }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != LIDAR_OK) return st;
    sd.leaf_width = res->best_leaf_width;
    sd.flags = (scene->flags & 0x00FFFFFFu) | (best_up << 24);
    res->best_up_weight = best_up ? (float)best_up / 128.0f : 1.0f;
    st = lidar_scene_load(ctx, &sd, persistent, persistent_bytes, scratch, scratch_bytes, stream);
    if (st < 0) return st;
    ctx->lanes_per_ray = (int)res->best_lanes_per_ray;
    b->packet = res->best_packet_rays;
    b->drop_graph();
    return LIDAR_OK;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
static lidar_status backward_common(lidar_ctx *ctx, const lidar_params *params, const uint32_t *tri,
                                    const uint8_t *valid, const float *intensity, const float *dL_dI,
                                    const float *dL_drange, float *d_rho, float *d_k, float *d_pose6,
                                    float *d_spectra, void *stream) {
    lidar_status st = ready(ctx, true);
    if (st != LIDAR_OK) return st;
    if (!tri) return ctx->fail(LIDAR_ERR_NO_FORWARD_STATE, "backward needs the forward's triangle ids (tri)");
    if (!valid) return ctx->fail(LIDAR_ERR_NO_FORWARD_STATE, "backward needs the forward's valid mask");
    if (ctx->M.nmat > kMaxAdjMaterials) return ctx->fail(LIDAR_ERR_INVALID_ARG, "backward supports nmat <= 256");
    if (params && params->rho && params->spectra)
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "params: give rho or spectra, not both");
    if ((st = no_actors(ctx, "the adjoint")) != LIDAR_OK) return st;
    const lidar_sensor_desc &d = ctx->sensor.d;
    // the forward's intensity max(0, R_lambda + sigma_I z) is clamped where it reads 0
    const bool clamps = d.noise_on && d.sigma_intensity > 0.f;
    if (clamps && !intensity)
        return ctx->fail(LIDAR_ERR_NO_FORWARD_STATE,
                         "with intensity noise the backward needs the forward's intensity (clamped beams)");
    size_t pb = adjoint_partial_bytes(d.n_ch * d.n_az, ctx->M.nmat);
    if (ctx->adj_partials.n < pb) return ctx->fail(LIDAR_ERR_NOT_READY, "adjoint buffer not allocated");
    const double *elev_cs = (const double *)ctx->sensor_tables.p;
    const double *az_cs = elev_cs + 2 * (size_t)d.n_ch;
    InstanceDev in = make_instance(ctx, ctx->tile_log2(), d, elev_cs, az_cs, ctx->p, ctx->q, 0, 0, 0, 0, 0);
    Overrides ov{};
    if (params) {
        ov.rho = params->rho;
        ov.angle_exp = params->angle_exp;
        ov.pose_delta = params->pose_delta;
        ov.spectra = params->spectra;
    }
    hipSetDevice(ctx->device);
    launch_adjoint(ctx->S, ctx->slot_of, in, ctx->M, ov, tri, valid, clamps ? intensity : nullptr, dL_dI, dL_drange,
                   (double *)ctx->adj_partials.p, d_rho, d_k, d_pose6, d_spectra, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->hip_fail(e, "adjoint launch");
    return LIDAR_OK;
}

lidar_status lidar_backward(lidar_ctx *ctx, const lidar_params *params, const uint32_t *tri, const uint8_t *valid,
                            const float *intensity, const float *dL_dI, const float *dL_drange, float *d_rho,
                            float *d_k, float *d_pose6, void *stream) {
    return backward_common(ctx, params, tri, valid, intensity, dL_dI, dL_drange, d_rho, d_k, d_pose6, nullptr,
                           stream);
}

lidar_status lidar_backward_spectra(lidar_ctx *ctx, const lidar_params *params, const uint32_t *tri,
                                    const uint8_t *valid, const float *intensity, const float *dL_dI,
                                    const float *dL_drange, float *d_spectra, float *d_k, float *d_pose6,
                                    void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (params && params->rho) return ctx->fail(LIDAR_ERR_INVALID_ARG, "the spectral adjoint reads R_lambda(0) "
                                                                       "from the table: params->rho must be NULL");
    if (!d_spectra) return ctx->fail(LIDAR_ERR_INVALID_ARG, "d_spectra is null");
    return backward_common(ctx, params, tri, valid, intensity, dL_dI, dL_drange, nullptr, d_k, d_pose6, d_spectra,
                           stream);
}

// ---------------------------------------------------------------------------
// introspection
// ---------------------------------------------------------------------------
lidar_status lidar_get_stats(lidar_ctx *ctx, lidar_stats *o) {
    if (!ctx || !o) return LIDAR_ERR_INVALID_ARG;
    if (!ctx->has_scene) return ctx->fail(LIDAR_ERR_NOT_READY, "no scene loaded");
    std::memset(o, 0, sizeof *o);
    o->n_triangles = ctx->S.n_tri;
    o->n_nodes = ctx->br.n_nodes;
    o->n_leaves = ctx->br.n_leaves;
    o->depth = ctx->br.depth;
    o->leaf_width = ctx->leaf_width;
    o->stack_entries = (uint32_t)ctx->stack;
    o->root = ctx->S.root;
    o->node_bytes = (uint64_t)ctx->br.n_nodes * sizeof(Node4);
    o->tri_bytes = (uint64_t)ctx->S.n_tri * sizeof(TriRec);
    o->build_ms = ctx->build_ms;
    o->box_pad = ctx->br.box_pad;
    o->max_abs_coord = ctx->br.max_abs;
    return LIDAR_OK;
}

lidar_status lidar_sync_check(lidar_ctx *ctx, void *stream) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "stream synchronize");
    uint32_t w = 0;
    e = hipMemcpy(&w, ctx->words.p, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "error word read");
    if (w) {
        hipMemset(ctx->words.p, 0, 4);
        return ctx->fail(LIDAR_ERR_STACK_OVERFLOW, "a traversal overflowed its stack");
    }
    return LIDAR_OK;
}

lidar_status lidar_debug_copy_bvh(lidar_ctx *ctx, void *host_nodes, uint64_t node_bytes, void *host_tris,
                                  uint64_t tri_bytes) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    if (!ctx->has_scene) return ctx->fail(LIDAR_ERR_NOT_READY, "no scene loaded");
    uint64_t nb = (uint64_t)ctx->br.n_nodes * sizeof(Node4), tb = (uint64_t)ctx->S.n_tri * sizeof(TriRec);
    if (!host_nodes || !host_tris || node_bytes < nb || tri_bytes < tb)
        return ctx->fail(LIDAR_ERR_WORKSPACE_TOO_SMALL, "host buffers too small");
    hipSetDevice(ctx->device);
    hipError_t e = hipMemcpy(host_nodes, ctx->S.nodes, nb, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(host_tris, ctx->S.tris, tb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "BVH copy");
    return LIDAR_OK;
}

lidar_status lidar_set_option(lidar_ctx *ctx, uint32_t option, int32_t value) {
    if (!ctx) return LIDAR_ERR_INVALID_ARG;
    switch (option) {
    case LIDAR_OPT_TILE_AZ: {
        if (value == 0) {   // automatic
            ctx->tile_az_log2 = -1;
            return LIDAR_OK;
        }
        int lg = -1;
        for (int k = 0; k <= 6; ++k)
            if ((1 << k) == value) lg = k;
        if (lg < 0) return ctx->fail(LIDAR_ERR_INVALID_ARG, "tile_az must be 0 (automatic) or a power of two in 1..64");
        ctx->tile_az_log2 = lg;
        return LIDAR_OK;
    }
    case LIDAR_OPT_LANES_PER_RAY:
        if (value != 1 && value != 2 && value != 4)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "lanes per ray must be 1, 2 or 4");
        ctx->lanes_per_ray = value;
        return LIDAR_OK;
    case LIDAR_OPT_XCD_REMAP:
        if (value != 0 && value != 1) return ctx->fail(LIDAR_ERR_INVALID_ARG, "xcd remap must be 0 or 1");
        ctx->xcd_remap = value;
        return LIDAR_OK;
    case LIDAR_OPT_ACTOR_TREE:
        if (value != 0 && value != 1) return ctx->fail(LIDAR_ERR_INVALID_ARG, "actor tree must be 0 or 1");
        ctx->actor_tree_opt = value;
        return LIDAR_OK;
    case LIDAR_OPT_BATCH_STACK:
        if (value < -1 || value > kMaxStack)
            return ctx->fail(LIDAR_ERR_INVALID_ARG, "batch stack must be -1 (off), 0 (automatic) or 1..96");
        ctx->batch_stack_opt = value;
        return LIDAR_OK;
    case LIDAR_OPT_STACK_CAP:
        if (value < 0) return ctx->fail(LIDAR_ERR_INVALID_ARG, "stack cap must be >= 0");
        ctx->stack_cap_opt = value;
        if (ctx->has_scene) ctx->S.stack_cap = value > 0 && value < ctx->stack ? value : ctx->stack;
        ++ctx->scene_gen;
        return LIDAR_OK;
    default:
        return ctx->fail(LIDAR_ERR_INVALID_ARG, "unknown option");
    }
}

lidar_status lidar_probe_stream(const void *buf, uint64_t bytes, float *sink, void *stream) {
    if (!buf || !sink || bytes < 16 || ((uintptr_t)buf & 15u)) return LIDAR_ERR_INVALID_ARG;
    launch_probe_stream(buf, bytes, sink, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? LIDAR_OK : LIDAR_ERR_HIP;
}

lidar_status lidar_probe_gather(const void *table, uint64_t bytes, uint32_t blocks, uint32_t steps, int32_t chase,
                                float *sink, void *stream) {
    if (!table || !sink || bytes < 128 || bytes > (1ull << 31) || ((uintptr_t)table & 15u) || blocks == 0 ||
        blocks > (1u << 20) || steps == 0)
        return LIDAR_ERR_INVALID_ARG;
    launch_probe_gather(table, (uint32_t)(bytes / 128), blocks, steps, chase ? 1 : 0, sink, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? LIDAR_OK : LIDAR_ERR_HIP;
}

}  // extern "C"
