// trace.hip -- first-hit query and return model for every beam (gfx950).
//
// One lane traces one beam.  Wavefronts take 64-beam tiles of tile_ch
// channels x tile_az azimuth steps (tile_ch * tile_az = 64) so that the rays
// of a wave are close in angle and walk similar BVH paths.  The traversal
// stack lives in LDS, one column per lane ([depth][lane], conflict-free).  The
// hit's attributes and the return model are evaluated in the same kernel and
// the per-beam outputs are written once.
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
// BVH traversal: nearest hit with ties broken by the smaller original index.
// ---------------------------------------------------------------------------
struct Hit {
    uint32_t slot;     // triangle record index, kNone if no hit
    uint32_t orig;     // original triangle index
    float t;
};

__device__ inline void csort(float &ka, uint32_t &va, float &kb, uint32_t &vb) {
    bool sw = kb < ka;
    float tk = sw ? kb : ka; kb = sw ? ka : kb; ka = tk;
    uint32_t tv = sw ? vb : va; vb = sw ? va : vb; va = tv;
}

__device__ inline void test_leaf(const TriRec *__restrict__ tris, uint32_t ref, const RayTri &T,
                                 float t_lo, Hit &h) {
    uint32_t first = leaf_first(ref), cnt = leaf_count(ref);
    for (uint32_t k = 0; k < cnt; ++k) {
        const TriRec *r = tris + first + k;
        float4 a = r->a, b = r->b, c = r->c;
        float t;
        if (tri_hit(T, a, b, c, t_lo, t)) {
            uint32_t orig = __float_as_uint(a.w);
            if (t < h.t || (t == h.t && orig < h.orig)) {
                h.t = t; h.orig = orig; h.slot = first + k;
            }
        }
    }
}

template <int STACK, int BLOCK>
__device__ inline Hit traverse(const Node4 *__restrict__ nodes, const TriRec *__restrict__ tris,
                               uint32_t root, const Ray &ray, float t_lo, float t_hi,
                               uint32_t *__restrict__ stk, bool &overflow) {
    const RayBox B = prep_box_test(ray);
    const RayTri T = prep_tri_test(ray);
    Hit h{kNone, kNone, t_hi};
    uint32_t ref = root;
    int sp = 0;
    const float inf = __builtin_inff();
    while (true) {
        if (ref & kLeafBit) {
            test_leaf(tris, ref, T, t_lo, h);
        } else {
            const float4 *np = reinterpret_cast<const float4 *>(nodes + ref);
            float4 lx = np[0], hx = np[1], ly = np[2], hy = np[3], lz = np[4], hz = np[5];
            uint4 ch = reinterpret_cast<const uint4 *>(np)[6];
            float tmax_lim = h.t * 1.0000005f;
            float k0, k1, k2, k3;
#define LIDAR_SLAB(K, LX, HX, LY, HY, LZ, HZ)                                   \
            {                                                                   \
                float x0 = fmaf(LX, B.ix, B.nox), x1 = fmaf(HX, B.ix, B.nox);   \
                float y0 = fmaf(LY, B.iy, B.noy), y1 = fmaf(HY, B.iy, B.noy);   \
                float z0 = fmaf(LZ, B.iz, B.noz), z1 = fmaf(HZ, B.iz, B.noz);   \
                float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), t_lo)); \
                float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmax_lim)); \
                K = (tn <= tf) ? tn : inf;                                      \
            }
            LIDAR_SLAB(k0, lx.x, hx.x, ly.x, hy.x, lz.x, hz.x)
            LIDAR_SLAB(k1, lx.y, hx.y, ly.y, hy.y, lz.y, hz.y)
            LIDAR_SLAB(k2, lx.z, hx.z, ly.z, hy.z, lz.z, hz.z)
            LIDAR_SLAB(k3, lx.w, hx.w, ly.w, hy.w, lz.w, hz.w)
#undef LIDAR_SLAB
            uint32_t c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
            csort(k0, c0, k1, c1);
            csort(k2, c2, k3, c3);
            csort(k0, c0, k2, c2);
            csort(k1, c1, k3, c3);
            csort(k1, c1, k2, c2);
            if (k0 != inf) {
                if (k3 != inf) { if (sp < STACK) stk[(sp++) * BLOCK] = c3; else overflow = true; }
                if (k2 != inf) { if (sp < STACK) stk[(sp++) * BLOCK] = c2; else overflow = true; }
                if (k1 != inf) { if (sp < STACK) stk[(sp++) * BLOCK] = c1; else overflow = true; }
                ref = c0;
                continue;
            }
        }
        if (sp == 0) break;
        ref = stk[(--sp) * BLOCK];
    }
    return h;
}

// ---------------------------------------------------------------------------
// Hit attributes + return model + output write (fused epilogue)
// ---------------------------------------------------------------------------
__device__ inline void shade_and_write(const InstanceDev &in, const MaterialsDev &M, const Overrides &ov,
                                       const Outputs &out, uint64_t o, uint32_t beam, const Ray &ray,
                                       const TriRec *__restrict__ tris, const Hit &h) {
    bool hit = h.slot != kNone;
    float nx = 0.f, ny = 0.f, nz = 0.f, rl = 0.f, dn = 0.f, inten = 0.f, tt = 0.f;
    uint32_t lab = kNone, orig = kNone;
    uint16_t mat16 = 0xFFFFu;
    bool det = false;
    if (hit) {
        const TriRec *r = tris + h.slot;
        float4 a = r->a, b = r->b, c = r->c;
        orig = __float_as_uint(a.w);
        uint32_t label = __float_as_uint(b.w);
        uint32_t m = __float_as_uint(c.w);
        mat16 = (uint16_t)m;
        float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
        float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
        float cx = fmaf(e1y, e2z, -e1z * e2y);
        float cy = fmaf(e1z, e2x, -e1x * e2z);
        float cz = fmaf(e1x, e2y, -e1y * e2x);
        float len = __fsqrt_rn(fmaf(cx, cx, fmaf(cy, cy, cz * cz)));
        nx = cx / len; ny = cy / len; nz = cz / len;
        float cd = fmaf(nx, ray.dx, fmaf(ny, ray.dy, nz * ray.dz));
        float cs = fabsf(cd);
        // R_lambda(0): per-material override, else spectral table at lambda
        float r0;
        if (ov.rho) {
            r0 = ov.rho[m];
        } else {
            float q = (in.wavelength_nm - M.lambda0) / M.dlambda;
            const float *T = M.spectra + (size_t)m * M.nbins;
            if (q <= 0.0f) r0 = T[0];
            else if (q >= (float)(M.nbins - 1)) r0 = T[M.nbins - 1];
            else {
                int i0 = (int)floorf(q);
                float f = q - (float)i0;
                r0 = fmaf(f, T[i0 + 1], (1.0f - f) * T[i0]);
            }
        }
        float kx = ov.angle_exp ? ov.angle_exp[m] : M.angle_exp[m];
        rl = (kx == 1.0f) ? r0 * cs : r0 * exp2f(kx * log2f(cs));
        float zd = 0.0f, zi = 0.0f, sig = 0.0f, sig_i = 0.0f;
        if (in.noise_on) {
            uint4 x = philox4x32_10(make_uint4(beam, in.scan, in.inst_id, 0u), in.seed_lo, in.seed_hi);
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

// tile mapping: padded ray r of an instance -> (channel j, azimuth i)
__device__ inline bool ray_coords(uint64_t r, const InstanceDev &in, int tile_az_log2, uint32_t &j, uint32_t &i) {
    uint32_t tile = (uint32_t)(r >> 6), lane = (uint32_t)(r & 63);
    uint32_t trow = tile / in.tiles_az, tcol = tile - trow * in.tiles_az;
    uint32_t tile_ch = 64u >> tile_az_log2;
    j = trow * tile_ch + (lane >> tile_az_log2);
    i = (tcol << tile_az_log2) + (lane & ((1u << tile_az_log2) - 1u));
    return j < in.n_ch && i < in.n_az;
}

// ---------------------------------------------------------------------------
// Kernel 1: one scan, BVH traversal
// ---------------------------------------------------------------------------
template <int STACK, int BLOCK>
__global__ __launch_bounds__(BLOCK) void trace_scan_kernel(SceneDev S, InstanceDev in, MaterialsDev M,
                                                           Overrides ov, Outputs out, int tile_az_log2,
                                                           uint64_t n_padded, uint32_t *err) {
    __shared__ uint32_t stk[STACK * BLOCK];
    uint64_t r = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= n_padded) return;
    uint32_t j, i;
    if (!ray_coords(r, in, tile_az_log2, j, i)) return;
    Pose64 P = make_pose(in, ov.pose_delta);
    Ray ray = make_ray(in, P, j, i);
    bool overflow = false;
    Hit h = traverse<STACK, BLOCK>(S.nodes, S.tris, S.root, ray, in.t_min, in.t_trace, stk + threadIdx.x, overflow);
    if (overflow) atomicOr(err, 1u);
    uint32_t beam = j * in.n_az + i;
    shade_and_write(in, M, ov, out, in.out_base + beam, beam, ray, S.tris, h);
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
    uint32_t j = 0, i = 0;
    bool active = r < n_padded && ray_coords(r, in, tile_az_log2, j, i);
    Pose64 P = make_pose(in, ov.pose_delta);
    Ray ray = make_ray(in, P, active ? j : 0, active ? i : 0);
    RayTri T = prep_tri_test(ray);
    Hit h{kNone, kNone, in.t_trace};
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
                    if (t < h.t || (t == h.t && orig < h.orig)) { h.t = t; h.orig = orig; h.slot = base + k; }
                }
            }
        }
    }
    if (!active) return;
    uint32_t beam = j * in.n_az + i;
    shade_and_write(in, M, ov, out, in.out_base + beam, beam, ray, S.tris, h);
}

// ---------------------------------------------------------------------------
// Kernel 3: batched persistent form.  Every wavefront pops packets of
// `packet` padded rays from a device counter until the queue is empty; a
// packet may span instances, each lane finds its instance by binary search
// over the instances' first padded ray.
// ---------------------------------------------------------------------------
template <int STACK, int BLOCK>
__global__ __launch_bounds__(BLOCK) void trace_batch_kernel(SceneDev S, const InstanceDev *__restrict__ insts,
                                                            uint32_t n_inst, MaterialsDev M, Outputs out,
                                                            int tile_az_log2, uint64_t n_padded_total,
                                                            uint32_t packet, uint32_t *queue, uint32_t *err) {
    __shared__ uint32_t stk[STACK * BLOCK];
    const uint32_t lane = threadIdx.x & 63u;
    const Overrides ov{nullptr, nullptr, nullptr};
    const uint64_t n_packets = (n_padded_total + packet - 1) / packet;
    bool overflow = false;
    while (true) {
        uint32_t pk = 0;
        if (lane == 0) pk = atomicAdd(queue, 1u);
        pk = __shfl(pk, 0, 64);
        if ((uint64_t)pk >= n_packets) break;
        for (uint32_t sub = 0; sub < packet; sub += 64) {
            uint64_t r = (uint64_t)pk * packet + sub + lane;
            if (r >= n_padded_total) break;   // uniform: padded totals are multiples of 64
            // instance containing padded ray r
            uint32_t lo = 0, hi = n_inst;
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) >> 1;
                if (insts[mid].ray_base <= r) lo = mid; else hi = mid;
            }
            const InstanceDev &in = insts[lo];
            uint32_t j, i;
            if (!ray_coords(r - in.ray_base, in, tile_az_log2, j, i)) continue;
            Pose64 P = make_pose(in, nullptr);
            Ray ray = make_ray(in, P, j, i);
            Hit h = traverse<STACK, BLOCK>(S.nodes, S.tris, S.root, ray, in.t_min, in.t_trace, stk + threadIdx.x, overflow);
            uint32_t beam = j * in.n_az + i;
            shade_and_write(in, M, ov, out, in.out_base + beam, beam, ray, S.tris, h);
        }
    }
    if (overflow) atomicOr(err, 1u);
}

__global__ void reset_queue_kernel(uint32_t *queue) { *queue = 0u; }

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int kBlock = 128;

template <int STACK>
static void launch_scan_t(const SceneDev &S, const InstanceDev &in, const MaterialsDev &M, const Overrides &ov,
                          const Outputs &out, int tile_az_log2, uint64_t n_padded, uint32_t *err, hipStream_t s) {
    uint64_t blocks = (n_padded + kBlock - 1) / kBlock;
    trace_scan_kernel<STACK, kBlock><<<(uint32_t)blocks, kBlock, 0, s>>>(S, in, M, ov, out, tile_az_log2, n_padded, err);
}

void launch_trace_scan(int stack, const SceneDev &S, const InstanceDev &in, const MaterialsDev &M,
                       const Overrides &ov, const Outputs &out, int tile_az_log2, uint64_t n_padded,
                       uint32_t *err, hipStream_t s) {
    if (stack <= 32) launch_scan_t<32>(S, in, M, ov, out, tile_az_log2, n_padded, err, s);
    else if (stack <= 64) launch_scan_t<64>(S, in, M, ov, out, tile_az_log2, n_padded, err, s);
    else launch_scan_t<96>(S, in, M, ov, out, tile_az_log2, n_padded, err, s);
}

void launch_bruteforce(const SceneDev &S, const InstanceDev &in, const MaterialsDev &M, const Overrides &ov,
                       const Outputs &out, int tile_az_log2, uint64_t n_padded, hipStream_t s) {
    constexpr int B = 256, C = 512;
    uint64_t blocks = (n_padded + B - 1) / B;
    bruteforce_kernel<B, C><<<(uint32_t)blocks, B, 0, s>>>(S, in, M, ov, out, tile_az_log2, n_padded);
}

template <int STACK>
static void launch_batch_t(const SceneDev &S, const InstanceDev *insts, uint32_t n_inst, const MaterialsDev &M,
                           const Outputs &out, int tile_az_log2, uint64_t n_padded, uint32_t packet,
                           uint32_t *queue, uint32_t *err, uint32_t grid, hipStream_t s) {
    reset_queue_kernel<<<1, 1, 0, s>>>(queue);
    trace_batch_kernel<STACK, kBlock><<<grid, kBlock, 0, s>>>(S, insts, n_inst, M, out, tile_az_log2, n_padded,
                                                              packet, queue, err);
}

void launch_trace_batch(int stack, const SceneDev &S, const InstanceDev *insts, uint32_t n_inst,
                        const MaterialsDev &M, const Outputs &out, int tile_az_log2, uint64_t n_padded,
                        uint32_t packet, uint32_t *queue, uint32_t *err, uint32_t grid, hipStream_t s) {
    if (stack <= 32) launch_batch_t<32>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet, queue, err, grid, s);
    else if (stack <= 64) launch_batch_t<64>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet, queue, err, grid, s);
    else launch_batch_t<96>(S, insts, n_inst, M, out, tile_az_log2, n_padded, packet, queue, err, grid, s);
}

int batch_blocks_per_cu(int stack) {
    // LDS per block = stack * kBlock * 4 bytes; 160 KB per CU on gfx950
    int lds = (stack <= 32 ? 32 : stack <= 64 ? 64 : 96) * kBlock * 4;
    int by_lds = (160 * 1024) / lds;
    return by_lds < 8 ? by_lds : 8;
}

}  // namespace lidar
