/*
 * lidar.h -- C ABI of the MI355X (gfx950) LiDAR simulation library.
 *
 * The library simulates a spinning multi-channel LiDAR in a triangle-mesh
 * scene, after Jansen, Huebel and Steckel, "Physical LiDAR Simulation in
 * Real-Time Engine" (arXiv:2208.10295).  For every beam it finds the first
 * surface along the beam (the paper's depth, Section II-A), the instance label
 * of that surface (Section II-B), the incidence angle from the surface normal
 * and the material's spectral reflectance at the sensor wavelength (Section
 * II-C, eq.4), adds Gaussian range noise (Section II-A) and applies the
 * linear reflectance-limit capability model with its maximum-range cutoff
 * (Section II-D, eq.5).  The result is a labelled point cloud (Fig.1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: 0 = success, < 0 = error (nothing was enqueued), > 0 = warning
 *   (the call succeeded; see each call): a bit set of LIDAR_WARN_* flags.  No
 *   C++ exception crosses the ABI.  lidar_last_error() returns a message for
 *   the last failing call.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Device work is enqueued on it and the call returns without
 *   waiting, unless the call says it synchronises.
 * - Memory: every output and every buffer named "device" is caller-owned
 *   device memory on the context's device (the Python binding uses PyTorch
 *   tensors).  The library allocates small context-owned device tables at
 *   set-up (lidar_sensor_set, lidar_materials_set, lidar_batch_create) and
 *   never allocates in lidar_simulate, lidar_simulate_batch or
 *   lidar_backward.
 * - Frames: right-handed, z up.  Azimuth 0 is the sensor's +x axis and grows
 *   counter-clockwise towards +y; elevation is positive upwards.  The beam of
 *   channel j and azimuth step i has sensor-frame direction
 *   s = (cos phi_j cos theta_i, cos phi_j sin theta_i, sin phi_j), the
 *   direction whose pinhole projection is eq.3 of the paper.
 * - Beam order: outputs of one scan are dense arrays in [n_ch][n_az] order,
 *   beam b = j * n_az + i.
 * - Threading: one context per host thread; contexts are independent.
 */
#ifndef LIDAR_H
#define LIDAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lidar_status;

#define LIDAR_OK                        0
#define LIDAR_ERR_INVALID_ARG          -1  /* null/misaligned pointer, bad size, NaN, non-unit quaternion */
#define LIDAR_ERR_NOT_READY            -2  /* no scene, sensor or materials set yet */
#define LIDAR_ERR_WORKSPACE_TOO_SMALL  -3  /* caller buffer smaller than the queried size */
#define LIDAR_ERR_HIP                  -4  /* a HIP runtime call failed (message has the HIP error) */
#define LIDAR_ERR_UNSUPPORTED_DEVICE   -5  /* device is not gfx950 */
#define LIDAR_ERR_STACK_OVERFLOW       -6  /* BVH deeper than the traversal stack; or a kernel overflowed it */
#define LIDAR_ERR_NO_FORWARD_STATE     -7  /* backward called without the forward's saved triangle ids */
#define LIDAR_ERR_OUT_OF_MEMORY        -8  /* a set-up allocation failed */
#define LIDAR_WARN_WAVELENGTH_CLAMPED   1  /* wavelength outside the spectral table: end bin used */
#define LIDAR_WARN_ORIGIN_OUTSIDE_SCENE 2  /* a ray origin lies outside the region the BVH's box padding
                                              covers (see lidar_origin_check): results are computed, but
                                              the walk may rarely miss a hit the brute force finds */

/* Size limits of a scene or mesh.  The walk addresses triangle records and
 * nodes with 32-bit byte offsets into buffers of at most 2^31 - 1 bytes:
 * records are 48 bytes, so at most LIDAR_MAX_TRIANGLES triangles
 * (lidar_scene_bytes and lidar_mesh_bytes refuse more), and nodes are 128
 * bytes, so a built tree may have at most LIDAR_MAX_NODES 4-wide nodes
 * (lidar_scene_load and lidar_mesh_load refuse a larger tree; only leaf
 * width 1 on scenes near the triangle limit comes close). */
#define LIDAR_MAX_TRIANGLES 44739242u   /* floor((2^31 - 1) / 48) */
#define LIDAR_MAX_NODES     16777216u   /* 2^24 */

/* Miss / drop encodings in the outputs. */
#define LIDAR_NO_LABEL     0xFFFFFFFFu
#define LIDAR_NO_TRIANGLE  0xFFFFFFFFu
#define LIDAR_NO_MATERIAL  0xFFFFu

typedef struct lidar_ctx lidar_ctx;
typedef struct lidar_batch lidar_batch;

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Creates a context on HIP device `hip_device`.  Fails with
 * LIDAR_ERR_UNSUPPORTED_DEVICE unless the device is gfx950. */
lidar_status lidar_create(int hip_device, lidar_ctx **out);

/* Frees the context and its context-owned device tables (synchronises the
 * device first).  Caller-owned buffers are untouched.  NULL is accepted.
 * Batches made on the context and not yet destroyed are detached: the only
 * call that still accepts them is lidar_batch_destroy. */
lidar_status lidar_destroy(lidar_ctx *ctx);

/* Message describing the last error on `ctx` (or of the last failing
 * lidar_create when ctx is NULL).  Owned by the library; valid until the next
 * call on the same context. */
const char *lidar_last_error(const lidar_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* Scene: triangle soup, per-triangle material and instance label, BVH       */
/* ------------------------------------------------------------------------ */

#define LIDAR_SCENE_DEVICE_PTRS 1u   /* the four arrays below are device pointers */
#define LIDAR_SCENE_BUILD_LBVH  2u   /* build the binary tree as an LBVH instead of by PLOC clustering */
#define LIDAR_SCENE_COLLAPSE_GREEDY 4u /* collapse to 4-wide nodes greedily (largest child first) instead
                                        of by the surface-area cost */
/* flags bits 8-15: PLOC search radius in Morton order, 1..128 (0 = 32)
 * flags bits 16-23: weight of a leaf step against a node step in the
 *   surface-area cost of the collapse, in sixteenths (0 = 24, i.e. 1.5)
 * flags bits 24-31: weight of a box's two horizontal (x-y) faces against its
 *   vertical ones in the area metric of the clustering and the collapse, in
 *   128ths (0 = 128, i.e. 1: the surface area).  Below 1 the tree is built for
 *   rays near the horizontal, as a LiDAR's mostly are: scans from many poses
 *   (trajectories, batches) run faster with 0.15 to 0.5; a single scan's time
 *   depends on how the top of the tree splits around its one origin.  Scenes
 *   only (meshes use the surface area).  Results never depend on the tree. */

typedef struct {
    uint64_t n_vertices;
    uint64_t n_triangles;      /* 1 .. LIDAR_MAX_TRIANGLES */
    const float *vertices;     /* [n_vertices][3] world coordinates, metres */
    const uint32_t *indices;   /* [n_triangles][3] vertex indices (< n_vertices) */
    const uint16_t *material;  /* [n_triangles] material id (< nmat of lidar_materials_set) */
    const uint32_t *label;     /* [n_triangles] instance label (the paper's per-object
                                  ground-truth id, Section II-B) */
    uint32_t leaf_width;       /* max triangles per BVH leaf, 1..8 (0 = 4) */
    uint32_t flags;            /* LIDAR_SCENE_DEVICE_PTRS (else host pointers) | LIDAR_SCENE_BUILD_LBVH */
} lidar_scene_desc;

/* Sizes of the two caller-owned device buffers that lidar_scene_load needs:
 * `persistent` holds the BVH and triangle records and must stay allocated
 * while the scene is used; `scratch` is only used during the load and may be
 * freed when it returns.  Both must be 256-byte aligned. */
lidar_status lidar_scene_bytes(const lidar_scene_desc *desc, uint64_t *persistent_bytes,
                               uint64_t *scratch_bytes);

/* Builds the BVH on the GPU into `persistent`, replacing any previous scene:
 * Morton codes and a radix sort, then a binary tree by PLOC clustering
 * (default) or as an LBVH, then a collapse to a 4-wide BVH with leaves of at
 * most leaf_width triangles, shaped by a surface-area cost (default) or
 * greedily.  Every build option gives the same simulation results (only the
 * speed differs).
 * Validates every triangle index on the device.  Synchronises `stream` (it
 * reads back the tree size and depth).  Errors: INVALID_ARG (bad sizes,
 * index out of range, more than LIDAR_MAX_NODES nodes), WORKSPACE_TOO_SMALL,
 * STACK_OVERFLOW (tree deeper than the traversal stack supports), HIP.
 * Warning: LIDAR_WARN_ORIGIN_OUTSIDE_SCENE if the current pose's origin lies
 * outside the new scene's cube (lidar_origin_check). */
lidar_status lidar_scene_load(lidar_ctx *ctx, const lidar_scene_desc *desc,
                              void *persistent, uint64_t persistent_bytes,
                              void *scratch, uint64_t scratch_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Materials (Section II-C)                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t nmat;             /* 1..65535 */
    uint32_t nbins;            /* spectral bins per material (61 for 400..1000 nm) */
    float lambda0_nm;          /* wavelength of bin 0 */
    float dlambda_nm;          /* bin spacing (> 0) */
    const float *spectra;      /* host [nmat][nbins] reflectance at normal incidence, fraction */
    const float *sigma_range;  /* host [nmat] Gaussian range-noise sigma, metres (>= 0) */
    const float *angle_exp;    /* host [nmat] exponent k of cos^k (NULL = all 1, eq.4) */
} lidar_material_desc;

/* Copies the material tables into context-owned device memory (allocates;
 * synchronous).  R_lambda(0) at a sensor wavelength is interpolated linearly
 * between bins on the GPU, clamped at the table ends. */
lidar_status lidar_materials_set(lidar_ctx *ctx, const lidar_material_desc *desc);

/* ------------------------------------------------------------------------ */
/* Sensor and pose (Sections II-A, II-C, II-D)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t n_ch;             /* channels (1..4096) */
    const double *elev_deg;    /* host [n_ch] channel elevations phi_j, degrees (data sheet) */
    uint32_t n_az;             /* azimuth steps (1..2^20) */
    double az0_deg;            /* theta_0 */
    double fov_h_deg;          /* horizontal FOV; theta_i = theta_0 + i * fov_h / n_az */
    float wavelength_nm;       /* sensor wavelength lambda */
    float d_max;               /* maximum range d_max, metres (> 0) */
    float r_l_max;             /* reflectance needed at d_max, fraction (eq.5) */
    float t_min;               /* minimum range, metres (>= 0) */
    float sigma_intensity;     /* additive intensity noise sigma (0 = none) */
    uint32_t noise_on;         /* 0: no range or intensity noise */
} lidar_sensor_desc;

/* Sets the sensor used by lidar_simulate.  Computes the FP64 direction
 * tables on the device (context-owned; synchronous).  Returns
 * LIDAR_WARN_WAVELENGTH_CLAMPED if the wavelength lies outside the material
 * table (materials must be set first for this check; otherwise it is made at
 * simulate time). */
lidar_status lidar_sensor_set(lidar_ctx *ctx, const lidar_sensor_desc *desc);

/* Sets the sensor pose used by lidar_simulate: origin p (world, metres) and
 * orientation quaternion q = (w, x, y, z), which must have unit norm to 1e-4
 * (it is renormalised).  World beam direction d = R(q) s.  Returns
 * LIDAR_WARN_ORIGIN_OUTSIDE_SCENE (the pose is still set) when a scene is
 * loaded and p lies outside its cube (lidar_origin_check). */
lidar_status lidar_pose_set(lidar_ctx *ctx, const float p[3], const float q_wxyz[4]);

/* The BVH's child boxes are padded outward by 2^-20 M, M the scene's largest
 * |vertex coordinate| (lidar_stats.max_abs_coord).  The FP32 slab test
 * fma(b, 1/d, -o/d) errs by at most 2^-24 (2|b_i| + 3|o_i|) along axis i and
 * the watertight triangle test by a few units of 2^-24 (|v| + |o|), both
 * below the pad when every |o_i| <= M: for ray origins in the cube
 * |x|, |y|, |z| <= M the BVH walk finds exactly the brute force's hits.  This
 * host-only check returns LIDAR_OK for an origin p in that cube (M =
 * max_abs_coord) and LIDAR_WARN_ORIGIN_OUTSIDE_SCENE otherwise, or
 * LIDAR_ERR_INVALID_ARG for a NULL or non-finite p.  lidar_pose_set,
 * lidar_scene_load, lidar_batch_create and lidar_simulate_sweep apply it to
 * their origins. */
lidar_status lidar_origin_check(float max_abs_coord, const float p[3]);

/* ------------------------------------------------------------------------ */
/* Simulation                                                                */
/* ------------------------------------------------------------------------ */

/* Per-beam outputs; every pointer is caller-owned device memory with one
 * element per beam (normal: 3 planes of n elements), or NULL to skip.
 * Detected points: xyz = d * s (sensor frame), intensity, label, valid = 1,
 * range = d (with noise).  Misses and dropped points: valid = 0,
 * label = LIDAR_NO_LABEL, zeros elsewhere.  The diagnostic outputs (tri,
 * t_hit, material, normal, r_lambda) describe the first hit within the
 * traceable range whether or not it is detected: tri = original triangle
 * index (LIDAR_NO_TRIANGLE if none), t_hit = noise-free distance,
 * material (LIDAR_NO_MATERIAL if none), unit geometric normal
 * normalize((v1 - v0) x (v2 - v0)), r_lambda = noise-free reflectance R_lambda
 * (eq.4, cos^k); zeros when there is no hit. */
typedef struct {
    float *x, *y, *z;
    float *intensity;
    uint32_t *label;
    uint8_t *valid;
    float *range;
    uint32_t *tri;
    float *t_hit;
    uint16_t *material;
    float *normal;             /* [3][n]: nx plane, ny plane, nz plane */
    float *r_lambda;
} lidar_outputs;

/* Optional parameter overrides for lidar_simulate_ex and lidar_backward; all
 * are caller-owned device pointers, NULL = not overridden. */
typedef struct {
    const float *rho;          /* [nmat] R_lambda(0) per material, used instead of the spectral table */
    const float *angle_exp;    /* [nmat] exponent k per material (cos^k) */
    const float *pose_delta;   /* [6] (dp, dw): p = p0 + dp, R = Exp(dw) R(q0) */
    const float *spectra;      /* [nmat][nbins] spectral table used instead of the one of
                                  lidar_materials_set (same lambda0, dlambda, nbins); not with rho */
} lidar_params;

/* One scan of the current sensor at the current pose.  Gaussian noise comes
 * from Philox4x32-10 (Salmon et al., SC'11) with key (seed low word, seed
 * high word) and counter (beam, scan, 0, 0), through Box-Muller
 * (z_range from words 0-1, z_intensity from words 2-3).  Asynchronous. */
lidar_status lidar_simulate(lidar_ctx *ctx, uint64_t seed, uint32_t scan,
                            const lidar_outputs *out, void *stream);

/* lidar_simulate with parameter overrides (`params` may be NULL). */
lidar_status lidar_simulate_ex(lidar_ctx *ctx, uint64_t seed, uint32_t scan,
                               const lidar_params *params, const lidar_outputs *out,
                               void *stream);

/* Reference path: the same scan with every beam tested against every
 * triangle (no BVH).  Outputs are bit-identical to lidar_simulate.  For
 * tests; O(beams x triangles). */
lidar_status lidar_simulate_bruteforce(lidar_ctx *ctx, uint64_t seed, uint32_t scan,
                                       const lidar_outputs *out, void *stream);

/* lidar_simulate that also writes, per beam, the number of 4-wide nodes the
 * traversal fetched and the number of triangle records it tested
 * (node_visits, tri_tests: caller-owned device [n_ch * n_az]).  Same results
 * as lidar_simulate; used to count the bytes a scan reads.  Asynchronous. */
lidar_status lidar_simulate_counts(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_outputs *out,
                                   uint32_t *node_visits, uint32_t *tri_tests, void *stream);

/* ------------------------------------------------------------------------ */
/* Point cloud: detected points only (Fig.1: the labelled point cloud)       */
/* ------------------------------------------------------------------------ */

/* Size of the caller-owned device workspace of lidar_compact_points for
 * n_beams dense elements (4 bytes per 256 beams, at least 256).  Errors:
 * INVALID_ARG (NULL pointer, n_beams > 2^31). */
lidar_status lidar_compact_bytes(uint64_t n_beams, uint64_t *workspace_bytes);

/* Order-preserving compaction of dense outputs: the elements b with
 * dense->valid[b] != 0 are copied, in increasing b, to elements 0, 1, ... of
 * every non-NULL array of `compact`; beam_index (device [n_beams], or NULL)
 * receives b, and *count (one device uint32) the number of detected points.
 * `dense` holds n_beams elements per array (the outputs of lidar_simulate,
 * lidar_simulate_batch, lidar_simulate_sweep, or of lidar_simulate_echoes with
 * n_beams = beams x echoes); it must have `valid`, and every array requested in
 * `compact` (normal: [3][n_beams] in both).  Every array of `compact` must
 * hold n_beams elements (the worst case); elements at and beyond *count are
 * left untouched.  Workspace: device, 256-byte aligned, at least
 * lidar_compact_bytes(n_beams).  Ballot and prefix sum per 256-beam block, no
 * atomics: the result is deterministic.  Asynchronous.  Errors: INVALID_ARG
 * (missing valid or source array, NULL count, misaligned workspace),
 * WORKSPACE_TOO_SMALL, HIP. */
lidar_status lidar_compact_points(lidar_ctx *ctx, const lidar_outputs *dense, uint64_t n_beams,
                                  const lidar_outputs *compact, uint32_t *beam_index, uint32_t *count,
                                  void *workspace, uint64_t workspace_bytes, void *stream);

/* lidar_compact_points for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments and results without the workspace: the per-block counts go to a
 * 512 KiB array of device memory that the library keeps on each GPU (set up
 * by the first lidar_create on that device, held until the process ends).
 * Allocates nothing (no hipMalloc, no allocating library call).  n_beams is
 * at most LIDAR_COMPACT_NOALLOC_MAX_BEAMS; nothing in the array has to start
 * at zero (every call writes each count before reading it).  All calls on one
 * GPU share the array: calls ordered on one stream are safe, calls that may
 * overlap on one GPU (other streams, other threads) race and give wrong
 * results.  Asynchronous.  Errors: as lidar_compact_points, and INVALID_ARG
 * for n_beams above the maximum. */
#define LIDAR_COMPACT_NOALLOC_MAX_BEAMS 33554432u   /* 2^25: 131,072 block counts */
lidar_status lidar_compact_points_noalloc(lidar_ctx *ctx, const lidar_outputs *dense, uint64_t n_beams,
                                          const lidar_outputs *compact, uint32_t *beam_index, uint32_t *count,
                                          void *stream);

/* ------------------------------------------------------------------------ */
/* Divergent beams and multi-echo returns (Section IV: named future work)    */
/* ------------------------------------------------------------------------ */

/* The paper's conclusion names beam divergence and multi-echo LiDAR as the
 * next physical effects; the model here is this library's reading.  A beam is
 * a cone of full angle divergence_rad sampled by n_sub equal-power sub-rays:
 * sub-ray 0 is the beam axis s, sub-ray k >= 1 is s turned by
 * r_k = (divergence_rad / 2) sqrt(k / (n_sub - 1)) towards
 * cos(b_k) e_theta + sin(b_k) e_phi with b_k = k pi (3 - sqrt 5) and e_theta,
 * e_phi the unit azimuth and elevation tangents at s (FP64, rounded once).
 * Each sub-ray takes its first hit and its noise-free R_lambda (eq.4).  Hits
 * ordered by (t, k) form echoes, a new echo starting where consecutive ranges
 * differ by more than echo_sep_m.  Echo e: strength
 * P = (1/n_sub) sum R_k, range t_first + sum R_k (t_k - t_first) / sum R_k
 * (plain mean if every R is 0), label, material and triangle of its strongest
 * sub-ray (smallest k on ties); range and intensity noise from Philox counter
 * (beam, scan, 0, e); detected iff t_min < d <= d_max and
 * (r_l_max / d_max) d <= P (eq.5 with P for R_lambda); intensity
 * max(0, P + sigma_I z).  With n_sub = 1 and divergence_rad = 0, echo 0 is
 * lidar_simulate's return bit for bit. */
typedef struct {
    uint32_t n_sub;            /* sub-rays per beam, 1..16 */
    uint32_t max_echoes;       /* echoes reported per beam, 1..4 (first ones in range order) */
    float divergence_rad;      /* full cone angle, >= 0 and < 0.5 */
    float echo_sep_m;          /* range resolution (> 0) */
} lidar_echo_desc;

/* Device workspace for lidar_simulate_echoes with the current sensor: 24 bytes
 * per sub-ray. */
lidar_status lidar_echo_bytes(lidar_ctx *ctx, const lidar_echo_desc *echo, uint64_t *workspace_bytes);

/* One scan with divergent beams.  Every output array (caller-owned device
 * memory) holds max_echoes planes of n_ch * n_az elements, echo e of beam b at
 * e * n_ch * n_az + b, laid out like lidar_simulate's; unformed or undetected
 * echoes read as misses.  Diagnostics per echo: tri / material of the
 * strongest sub-ray (LIDAR_NO_TRIANGLE / LIDAR_NO_MATERIAL if the echo was not
 * formed), t_hit = noise-free echo range, r_lambda = strength P; normal is
 * not produced (must be NULL).  Sees the actors of a dynamic scene.
 * Asynchronous; the workspace (>= lidar_echo_bytes, 256-byte aligned) is used
 * until the stream has passed the call. */
lidar_status lidar_simulate_echoes(lidar_ctx *ctx, uint64_t seed, uint32_t scan, const lidar_echo_desc *echo,
                                   void *workspace, uint64_t workspace_bytes, const lidar_outputs *out,
                                   void *stream);

/* ------------------------------------------------------------------------ */
/* Dynamic scenes: meshes placed by moving actors (Section II-B)             */
/* ------------------------------------------------------------------------ */

/* Section II-B gives every object instance its own label.  A dynamic scene
 * adds, to the static scene of lidar_scene_load, actors: each places a mesh
 * (object-space triangles with per-triangle materials) in the world with a
 * rigid transform x_world = R(q) x_object + p and gives all of the mesh's
 * triangles the actor's label.  Every mesh has its own BVH; a top-level BVH
 * over the actors' world boxes is built by lidar_actors_set and rebuilt or
 * refit by lidar_actors_update each frame.  The first hit is taken over the static
 * triangles and all placed meshes as one soup, ties broken by the index in
 * the combined ordering: static triangles 0 .. n_static - 1, then the
 * triangles of actor 0, actor 1, ... (outputs.tri reports that index).
 * lidar_simulate, lidar_simulate_ex and lidar_simulate_sweep see the actors;
 * the brute-force reference, traversal counting, the batched form and the
 * adjoint cover the static scene only and return LIDAR_ERR_INVALID_ARG while
 * actors are set.
 * A mesh is walked with the ray taken to object space, whose origin lies at
 * the sensor's distance from the actor.  Mesh boxes are therefore padded as
 * for a scene whose largest coordinate is at least LIDAR_MESH_REACH metres
 * (see lidar_origin_check), and the top-level tree as for the static scene's
 * cube.  lidar_simulate, lidar_simulate_ex and lidar_simulate_sweep return
 * LIDAR_WARN_ORIGIN_OUTSIDE_SCENE while actors are set if the traceable range
 * (d_max plus the largest noise excursion) plus twice a placed mesh's largest
 * coordinate exceeds LIDAR_MESH_REACH. */
#define LIDAR_MESH_REACH 1024.0f

/* Workspace sizes of a mesh (lidar_scene_desc with label ignored, may be NULL;
 * the workspaces hold the mesh BVH and a copy of the indices). */
lidar_status lidar_mesh_bytes(const lidar_scene_desc *mesh, uint64_t *persistent_bytes, uint64_t *scratch_bytes);

/* Builds a mesh's BVH into caller-owned workspaces (256-byte aligned; the
 * persistent one must stay allocated while the context uses the mesh, the
 * scratch one only during the call) and returns its id (0, 1, ... in load
 * order; at most 4096 meshes).  Synchronises `stream`. */
lidar_status lidar_mesh_load(lidar_ctx *ctx, const lidar_scene_desc *mesh, void *persistent,
                             uint64_t persistent_bytes, void *scratch, uint64_t scratch_bytes, void *stream,
                             uint32_t *mesh_id);

/* Deformed mesh: new object-space vertices (device [n_vertices][3], same
 * topology) replace the mesh's triangles and its BVH boxes are refit.  Call
 * lidar_actors_update afterwards (simulating before returns
 * LIDAR_ERR_NOT_READY).  Asynchronous; `vertices` must stay valid until the
 * stream reaches the call. */
lidar_status lidar_mesh_refit(lidar_ctx *ctx, uint32_t mesh_id, const float *vertices, void *stream);

typedef struct {
    uint32_t mesh;             /* mesh id from lidar_mesh_load */
    uint32_t label;            /* instance label of every triangle of the actor */
    float p[3];                /* object origin in the world, metres */
    float q_wxyz[4];           /* orientation, unit quaternion (1e-4) */
} lidar_actor;

/* Workspace sizes for n_actors actors (1 .. 2^20). */
lidar_status lidar_actors_bytes(uint32_t n_actors, uint64_t *persistent_bytes, uint64_t *scratch_bytes);

/* Sets the actors (host array) and builds the top-level BVH over their world
 * boxes into caller-owned workspaces (256-byte aligned; persistent kept while
 * the actors are in use, scratch only during the call).  n_actors = 0 clears
 * them.  Synchronises `stream`. */
lidar_status lidar_actors_set(lidar_ctx *ctx, const lidar_actor *actors, uint32_t n_actors, void *persistent,
                              uint64_t persistent_bytes, void *scratch, uint64_t scratch_bytes, void *stream);

/* Per-frame update: the same actors (count and meshes) at new poses.  Uploads
 * the transforms through a pinned buffer, recomputes the world boxes and
 * rebuilds the top-level BVH in one workgroup (up to 4,096 actors, see
 * LIDAR_OPT_ACTOR_TREE) or refits it (the builder's tree: call
 * lidar_actors_set again when the refit tree has degraded).  Asynchronous:
 * the transforms go through a pinned ring of eight slots (two for more than
 * 4,096 actors), and the call waits only when it reuses a slot the GPU may
 * still read; an update on another stream than the previous one first waits
 * for the device. */
lidar_status lidar_actors_update(lidar_ctx *ctx, const lidar_actor *actors, uint32_t n_actors, void *stream);

/* Removes the actors (the workspaces are the caller's). */
lidar_status lidar_actors_clear(lidar_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* Partial sweep per engine tick, rolling-shutter pose (Section II-A)        */
/* ------------------------------------------------------------------------ */

/* One engine tick of a spinning head.  Section II-A simulates per tick only
 * the part of the horizontal FOV that the head swept since the previous tick,
 * from the spin rate omega_l and the tick length dt.  The head angle is
 * unwrapped: revolution (scan) s >= 0 covers [360 s, 360 (s + 1)) + az0, and
 * column i of revolution s fires at head angle A = 360 s + az0 + i fov_h / n_az.
 * The tick covers the window [a, b) with a = head_deg and
 * b = a + 360 * spin_hz * dt_s (computed in FP64 in this order).  Column i of
 * revolution s is fired iff ceil(c_s(a)) <= i < ceil(c_s(b)), with
 * c_s(x) = ((x - az0) - 360 s) * n_az / fov_h in FP64, for
 * s in {floor((a - az0) / 360), that + 1}, s >= 0.  Consecutive ticks whose
 * windows share their ends fire every column exactly once.
 * Each fired column is traced with the pose at its firing fraction
 * tau = (A - a) / (b - a) of the tick: p = p_begin + tau (p_end - p_begin),
 * orientation on the great arc from q_begin to q_end (slerp, Shoemake 1985;
 * the shorter arc; the chord q_begin + tau (q_end - q_begin) below an arc of
 * 1e-6 rad).  Equal end poses reproduce lidar_simulate's pose exactly. */
typedef struct {
    double head_deg;           /* head angle at the tick start, degrees (unwrapped, finite) */
    double spin_hz;            /* omega_l, revolutions per second (> 0) */
    double dt_s;               /* tick length, seconds (>= 0; 360 * spin_hz * dt_s <= 360) */
    float p_begin[3];          /* pose at the tick start: origin (world, metres) */
    float q_begin[4];          /*   and unit quaternion (w, x, y, z) */
    float p_end[3];            /* pose at the tick end */
    float q_end[4];
    uint64_t seed;             /* Philox key, as in lidar_simulate */
} lidar_sweep_desc;

/* The columns a tick fired: up to two runs, the second one revolution after
 * the first (azimuth first[r] .. first[r] + count[r] - 1 of scan[r]). */
typedef struct {
    uint32_t n_runs;           /* 0, 1 or 2 */
    uint32_t n_columns;        /* count[0] + count[1] */
    uint32_t scan[2];
    uint32_t first[2];
    uint32_t count[2];
} lidar_sweep_info;

/* Simulates the columns fired in one tick with the current sensor.  Outputs
 * use the layout of lidar_simulate ([n_ch][n_az] range image, one element per
 * beam of the whole scan); only the beams of fired columns are written, the
 * others keep their contents, so successive ticks fill the range image.  The
 * Philox counter of beam (j, i) of revolution s is (j n_az + i, s, 0, 0):
 * the ticks of revolution s with one fixed pose give bit for bit
 * lidar_simulate(seed, scan = s) at that pose.  xyz are in the sensor frame
 * at each column's firing time.  `info` (host, may be NULL) receives the
 * fired columns.  Uses a context-owned pose table: sweeps on one context are
 * ordered on one stream.  Errors: LIDAR_ERR_INVALID_ARG for a window longer
 * than 360 degrees, non-finite values, non-unit quaternions (1e-4) or a
 * revolution index >= 2^32 - 1; nothing is launched when no column fires.
 * Warning: LIDAR_WARN_ORIGIN_OUTSIDE_SCENE if p_begin or p_end lies outside
 * the scene's cube (lidar_origin_check).  Asynchronous. */
lidar_status lidar_simulate_sweep(lidar_ctx *ctx, const lidar_sweep_desc *sweep, const lidar_outputs *out,
                                  lidar_sweep_info *info, void *stream);

/* Launch-shape options.  They change speed, never results.
 *   LIDAR_OPT_TILE_AZ: beams are traced in 64-beam tiles of `value` azimuth
 *     steps x 64 / value channels (power of two in 1..64), or 0 = automatic
 *     (default): 2 for the static scene, 8 while actors are set, 16 for a
 *     batch.  A batch keeps the tile shape that was current when it was
 *     created.
 *   LIDAR_OPT_LANES_PER_RAY: 1 = one lane walks the BVH for a beam; 2 = two
 *     lanes share a beam, two child boxes each; 4 = the four lanes of a quad
 *     share a beam, one child box each (default 4).
 *   LIDAR_OPT_XCD_REMAP: 1 = the thread blocks that run on one XCD take one
 *     contiguous azimuth sector (default 1); 0 = blocks in launch order.
 *   LIDAR_OPT_ACTOR_TREE: 0 = up to 4,096 actors, the top-level tree is
 *     rebuilt by lidar_actors_set and by every lidar_actors_update in one
 *     workgroup (Morton order of the actor boxes, one actor per leaf, four
 *     entries per node), so it stays tight as the actors move; more actors
 *     as for 1 (default 0).  1 = the scene builder's tree, built by
 *     lidar_actors_set and refit by lidar_actors_update.  Read by
 *     lidar_actors_set.
 *   LIDAR_OPT_BATCH_STACK: the batched form's walks first run with a short
 *     stack, so that more wavefronts fit on a CU, and a ray whose walk needs
 *     more entries is listed and traced again, after the batch's walks and
 *     in the same launch sequence, by one lane with the whole stack; its
 *     result is the same as with the whole stack from the start.  0 =
 *     automatic (default): 32 entries when the tree needs more and a ray
 *     has one or two lanes; n in 1..96 = at most n entries (to test the
 *     second pass); -1 = off (one pass with the whole stack).  Up to 2^22
 *     rays per launch can be listed; beyond that the walks keep what fits
 *     and lidar_sync_check reports LIDAR_ERR_STACK_OVERFLOW.
 * One option exists to test error handling and does change results:
 *   LIDAR_OPT_STACK_CAP: 0 = a walk of the static scene may use the whole
 *     traversal stack sized for the tree's depth (default); n > 0 = at most n
 *     entries.  A walk that needs more loses the children it cannot push,
 *     stays within its stack memory and ends normally, and the next
 *     lidar_sync_check returns LIDAR_ERR_STACK_OVERFLOW.  Kept across scene
 *     loads. */
#define LIDAR_OPT_TILE_AZ        1u
#define LIDAR_OPT_LANES_PER_RAY  2u
#define LIDAR_OPT_XCD_REMAP      3u
#define LIDAR_OPT_STACK_CAP      4u
#define LIDAR_OPT_ACTOR_TREE     5u
#define LIDAR_OPT_BATCH_STACK    6u
lidar_status lidar_set_option(lidar_ctx *ctx, uint32_t option, int32_t value);

/* ------------------------------------------------------------------------ */
/* Batched form: many sensors / poses in one persistent launch               */
/* ------------------------------------------------------------------------ */

typedef struct {
    lidar_sensor_desc sensor;  /* per-instance sensor (own tables, wavelength, range) */
    float p[3];                /* pose origin */
    float q_wxyz[4];           /* pose orientation (unit) */
    uint64_t seed;             /* Philox key */
    uint32_t scan;             /* Philox counter word 1 */
} lidar_instance;

/* Uploads n_inst instance descriptors and their direction tables
 * (allocates; synchronous).  The batch handle owns these tables and the
 * captured graph, so that lidar_simulate_batch allocates nothing and only
 * replays (instead of taking the instances on every call).  Instance k's beams are written at output
 * offset out_offset[k] = sum of n_ch * n_az of instances before k, in the
 * same [n_ch][n_az] order as a single scan; its Philox counter is
 * (beam, scan, k, 0).  `packet_rays` (multiple of 64, 0 = tuned/default)
 * is the number of rays a wavefront claims per queue pop.  Returns
 * LIDAR_WARN_WAVELENGTH_CLAMPED if any instance clamps and
 * LIDAR_WARN_ORIGIN_OUTSIDE_SCENE if a scene is loaded and an instance's
 * origin lies outside its cube. */
lidar_status lidar_batch_create(lidar_ctx *ctx, const lidar_instance *inst, uint32_t n_inst,
                                uint32_t packet_rays, lidar_batch **out);

/* Total rays of a batch (sum of n_ch * n_az). */
lidar_status lidar_batch_rays(const lidar_batch *batch, uint64_t *n_rays);

/* Runs every instance of the batch in one persistent kernel: wavefronts pop
 * ray packets from a device queue until it is empty.  The queue reset and
 * the kernel are captured once into a hipGraph per (stream-independent)
 * output binding and replayed on `stream`; a new scene, new materials or a
 * new stack cap since the capture make the next call capture again (and
 * re-derive each instance's traceable range from the material noise).
 * Outputs as in lidar_simulate,
 * indexed by out_offset[k] + beam.  Results are bit-identical to
 * lidar_simulate_batch_sequential, and instance k equals a plain scan of the
 * same sensor and pose whose Philox counter word 2 is k.  Asynchronous. */
lidar_status lidar_simulate_batch(lidar_ctx *ctx, lidar_batch *batch, const lidar_outputs *out,
                                  void *stream);

/* The same instances as n_inst separate plain launches on `stream`
 * (baseline for the batched form). */
lidar_status lidar_simulate_batch_sequential(lidar_ctx *ctx, lidar_batch *batch,
                                             const lidar_outputs *out, void *stream);

/* Number of rays that the last lidar_simulate_batch launch on this context
 * traced again with the whole stack (LIDAR_OPT_BATCH_STACK); waits for the
 * device.  Measurement and tests only. */
lidar_status lidar_batch_restarted(lidar_ctx *ctx, uint64_t *n_rays);

/* Frees the batch (synchronises its device first), before or after its
 * context.  NULL is accepted. */
lidar_status lidar_batch_destroy(lidar_batch *batch);

/* ------------------------------------------------------------------------ */
/* Autotuner                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint32_t *packet_rays;   /* host [n_packet] candidates (multiples of 64) */
    uint32_t n_packet;
    const uint32_t *leaf_widths;   /* host [n_leaf] candidates (1..8) */
    uint32_t n_leaf;
    const uint32_t *lanes_per_ray; /* host [n_lanes] candidates (1, 2 or 4); NULL = current only */
    uint32_t n_lanes;
    uint32_t reps;                 /* timed repetitions per candidate (median) */
    const float *up_weights;       /* host [n_up] candidate weights of the horizontal faces in the tree
                                      build's area metric (scene flags bits 24-31; 1/128 .. 255/128);
                                      NULL = the scene descriptor's own */
    uint32_t n_up;
} lidar_tune_desc;

typedef struct {
    uint32_t best_packet_rays;
    uint32_t best_leaf_width;
    uint32_t best_lanes_per_ray;
    float best_ms;
    float ms[64];                  /* [n_up][n_leaf][n_lanes][n_packet] medians, row-major (<= 64 entries) */
    float best_up_weight;
} lidar_tune_result;

/* Times lidar_simulate_batch for every (area weight, leaf width, lanes per
 * ray, packet size) candidate on the batch, rebuilding the BVH per area
 * weight and leaf width from `scene` into the given buffers, then leaves the
 * scene built with the best weight and leaf width, the context set to the
 * best lanes per ray and the batch to the best packet size.  Results never
 * depend on the choice.  Synchronous. */
lidar_status lidar_tune(lidar_ctx *ctx, const lidar_scene_desc *scene, void *persistent,
                        uint64_t persistent_bytes, void *scratch, uint64_t scratch_bytes,
                        lidar_batch *batch, const lidar_outputs *out, const lidar_tune_desc *desc,
                        lidar_tune_result *result, void *stream);

/* ------------------------------------------------------------------------ */
/* Adjoint (eq.4 intensity and range with the hit triangle held fixed)       */
/* ------------------------------------------------------------------------ */

/* Gradients of a scalar loss L with respect to the per-material reflectance
 * rho (R_lambda(0)), the per-material exponent k (I = rho |n.d|^k) and the
 * pose delta (dp, dw) of lidar_params, given dL/dI and dL/drange per beam of
 * the current sensor.  The forward state is the per-beam original triangle
 * id from the forward call (outputs.tri), the per-beam valid mask and the
 * forward's intensity output; beams with valid == 0 or
 * tri == LIDAR_NO_TRIANGLE contribute nothing.  With the triangle fixed,
 * range t = n.(v0 - p) / (n.d) (range noise is additive, so dL/drange flows
 * to t unchanged).  With intensity noise (noise_on and sigma_intensity > 0)
 * the forward's intensity is max(0, R_lambda + sigma_I z): where it is 0 the
 * clamp holds and the intensity terms of that beam are 0; `intensity` (device
 * [n], the forward's output) is then required (NO_FORWARD_STATE if NULL) and
 * is otherwise ignored (may be NULL).  Per-block partial sums
 * are reduced in a fixed order (deterministic); results are FP32 written to
 * d_rho[nmat], d_k[nmat], d_pose6[6] (device).  `params` must be the same as
 * in the forward call (without rho, R_lambda(0) is the spectral table at the
 * sensor wavelength).  Materials are limited to nmat <= 256.  Asynchronous.
 * Errors: NO_FORWARD_STATE if tri or valid is NULL, or intensity is NULL while
 * the sensor has intensity noise. */
lidar_status lidar_backward(lidar_ctx *ctx, const lidar_params *params, const uint32_t *tri,
                            const uint8_t *valid, const float *intensity, const float *dL_dI,
                            const float *dL_drange, float *d_rho, float *d_k, float *d_pose6, void *stream);

/* Full-spectrum adjoint: as lidar_backward, with R_lambda(0) read from the
 * spectral table (params->spectra, else the table of lidar_materials_set) at
 * the sensor wavelength.  Eq.4's R_lambda(0)_m = sum_b w_b T[m][b] with the
 * linear interpolation weights w of the wavelength (Section II-C: the
 * reflectance for the wavelength in use; clamped to the end bin outside the
 * table), so dL/dT[m][b] = w_b dL/dR_lambda(0)_m.  Writes d_spectra[nmat][nbins]
 * (device FP32; zero on bins the wavelength does not touch), d_k and d_pose6 as
 * lidar_backward (either may be NULL).  Gradients of scans at several
 * wavelengths add up to the multi-wavelength gradient.  Errors: INVALID_ARG if
 * params->rho is set or d_spectra is NULL; otherwise as lidar_backward.
 * Asynchronous. */
lidar_status lidar_backward_spectra(lidar_ctx *ctx, const lidar_params *params, const uint32_t *tri,
                                    const uint8_t *valid, const float *intensity, const float *dL_dI,
                                    const float *dL_drange, float *d_spectra, float *d_k, float *d_pose6,
                                    void *stream);

/* ------------------------------------------------------------------------ */
/* Introspection                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t n_triangles;
    uint64_t n_nodes;              /* 4-wide BVH nodes */
    uint64_t n_leaves;
    uint32_t depth;                /* levels of the 4-wide BVH */
    uint32_t leaf_width;
    uint32_t stack_entries;        /* traversal stack per ray */
    uint32_t root;                 /* root child reference */
    uint64_t node_bytes;           /* bytes of nodes in use */
    uint64_t tri_bytes;            /* bytes of triangle records */
    float build_ms;                /* last lidar_scene_load, GPU time */
    float box_pad;                 /* conservative bounding-box padding, metres */
    float max_abs_coord;           /* largest |vertex coordinate| M (lidar_origin_check) */
    uint32_t pad_;
} lidar_stats;

/* Facts of the current scene's BVH.  (Named lidar_get_stats because C gives a
 * function and the lidar_stats typedef one name space.) */
lidar_status lidar_get_stats(lidar_ctx *ctx, lidar_stats *out);

/* Synchronises `stream` and reads the device error word written by kernels
 * (e.g. traversal stack overflow).  Returns LIDAR_ERR_STACK_OVERFLOW if a
 * kernel flagged it since the last check (and clears it). */
lidar_status lidar_sync_check(lidar_ctx *ctx, void *stream);

/* Copies the BVH and triangle records to host memory for inspection:
 * nodes (n_nodes * 128 bytes) and triangle records (n_triangles * 48 bytes).
 * Synchronous.  For tests. */
lidar_status lidar_debug_copy_bvh(lidar_ctx *ctx, void *host_nodes, uint64_t node_bytes,
                                  void *host_tris, uint64_t tri_bytes);

/* ------------------------------------------------------------------------ */
/* Memory-roof probes (not part of the simulation)                          */
/* ------------------------------------------------------------------------ */

/* The trace kernels' traffic is reported as algorithmic bytes per second;
 * these probes measure the roofs to compare it with, on the caller's device
 * and stream.  Both are asynchronous single launches that read device memory
 * only (the caller times them, e.g. with events around repeated launches);
 * `sink` is one device float that is written only if the data sums to an
 * improbable value, so the loads stay and add no write traffic.
 *
 * lidar_probe_stream reads every 16-byte word of `buf` (device, 16-byte
 * aligned, `bytes` rounded down to a multiple of 16) once: the HBM read roof
 * when `bytes` is far larger than the caches.
 *
 * lidar_probe_gather runs `blocks` blocks of 256 threads; each quad of lanes
 * fetches `steps` 128-byte lines of `table` (device, 16-byte aligned, bytes in
 * [128, 2^31], rounded down to a multiple of 128), 32 bytes per lane, the way
 * a quad fetches a 4-wide BVH node.  Line indices are uniform over the table.
 * chase != 0: each index is a hash of the data of the quad's previous line
 * (a dependent chain per quad, like a BVH walk); chase == 0: a hash of a
 * counter (independent fetches).  Bytes fetched = blocks * 64 * steps * 128.
 *
 * Errors: INVALID_ARG (NULL pointers, misalignment, sizes out of range),
 * HIP (launch failure). */
lidar_status lidar_probe_stream(const void *buf, uint64_t bytes, float *sink, void *stream);
lidar_status lidar_probe_gather(const void *table, uint64_t bytes, uint32_t blocks, uint32_t steps,
                                int32_t chase, float *sink, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LIDAR_H */
