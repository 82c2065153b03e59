// adjoint.hip -- gradients of an intensity/range loss with the hit triangle held
// fixed (gfx950).
//
// Per valid beam with hit triangle (v0, v1, v2), unit normal n, world beam
// direction d = R s and origin p:
//   c = n . d,  t = n . (v0 - p) / c,  I = rho_m |c|^k_m   (eq.4 with cos^k)
// Given g_I = dL/dI and g_t = dL/drange (g_I taken as 0 on beams whose
// forward intensity max(0, R_lambda + sigma_I z) was clamped at 0):
//   dL/drho_m += g_I |c|^k
//   dL/dk_m   += g_I rho |c|^k ln|c|
//   dL/dp     += -g_t n / c
//   dL/dw_left += gamma (d x n),  gamma = g_I rho k |c|^(k-1) sgn(c) - g_t t / c
// where w_left perturbs the rotation as R <- Exp(w) R.  The pose delta's
// rotation gradient is J_l(dw)^T dL/dw_left (left Jacobian of Exp at dw).
// Per-beam terms are FP32; every output is reduced in FP64 in a fixed order:
// inside a wavefront, the beams of each material present (grouped by ballot)
// are summed by a butterfly over the 64 lanes; the four wavefronts of a block
// are added in order; the blocks' partial sums are added by one block per
// output with a fixed stride pattern and tree.  Results are bit-reproducible.
#include "lidar_kernels.hpp"

namespace lidar {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kAdjBlock) void adjoint_kernel(SceneDev S, const uint32_t *__restrict__ slot_of,
                                                           InstanceDev in, MaterialsDev M, Overrides ov,
                                                           const uint32_t *__restrict__ tri,
                                                           const uint8_t *__restrict__ valid,
                                                           const float *__restrict__ clamp_I,
                                                           const float *__restrict__ gI_in,
                                                           const float *__restrict__ gd_in,
                                                           double *__restrict__ partials) {
    constexpr int NW = kAdjBlock / 64;
    __shared__ double acc[NW][2 * 256 + 6];
    const uint32_t nmat = M.nmat;
    const uint32_t n_out = 2 * nmat + 6;
    const uint32_t nb = in.n_ch * in.n_az;
    const uint32_t b = blockIdx.x * kAdjBlock + threadIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (uint32_t o = lane; o < n_out; o += 64) acc[w][o] = 0.0;

    float a_rho = 0.f, a_k = 0.f, a_p[3] = {0.f, 0.f, 0.f}, a_w[3] = {0.f, 0.f, 0.f};
    uint32_t m = kNone;
    if (b < nb && valid[b] && tri[b] != kNone) {
        uint32_t j = b / in.n_az, i = b - j * in.n_az;
        Pose64 P = make_pose(in, ov.pose_delta);
        Ray ray = make_ray(in, P, j, i);
        TriRec r = S.tris[slot_of[tri[b]]];
        m = __float_as_uint(r.c.w);
        float e1x = r.b.x - r.a.x, e1y = r.b.y - r.a.y, e1z = r.b.z - r.a.z;
        float e2x = r.c.x - r.a.x, e2y = r.c.y - r.a.y, e2z = r.c.z - r.a.z;
        float cx = fmaf(e1y, e2z, -e1z * e2y);
        float cy = fmaf(e1z, e2x, -e1x * e2z);
        float cz = fmaf(e1x, e2y, -e1y * e2x);
        float len = __fsqrt_rn(fmaf(cx, cx, fmaf(cy, cy, cz * cz)));
        float nx = cx / len, ny = cy / len, nz = cz / len;
        float c = fmaf(nx, ray.dx, fmaf(ny, ray.dy, nz * ray.dz));
        float qx = (float)((double)r.a.x - P.p[0]), qy = (float)((double)r.a.y - P.p[1]),
              qz = (float)((double)r.a.z - P.p[2]);
        float t = fmaf(nx, qx, fmaf(ny, qy, nz * qz)) / c;
        float ac = fabsf(c);
        float rho = reflectance0(ov, M, in.wavelength_nm, m);
        float k = ov.angle_exp ? ov.angle_exp[m] : M.angle_exp[m];
        float lnc = logf(ac);
        float ck = (k == 1.0f) ? ac : expf(k * lnc);              // |c|^k
        float ck1 = (k == 1.0f) ? 1.0f : expf((k - 1.0f) * lnc);  // |c|^(k-1)
        // the forward's intensity max(0, R_lambda + sigma_I z): 0 where the clamp holds, and
        // there I does not move with rho, k or the pose
        float gI = gI_in && !(clamp_I && clamp_I[b] == 0.0f) ? gI_in[b] : 0.0f;
        float gt = gd_in ? gd_in[b] : 0.0f;
        a_rho = gI * ck;
        a_k = gI * rho * ck * lnc;
        float ginv = -gt / c;
        a_p[0] = ginv * nx; a_p[1] = ginv * ny; a_p[2] = ginv * nz;
        float gamma = gI * rho * k * ck1 * copysignf(1.0f, c) - gt * t / c;
        // d x n
        a_w[0] = gamma * fmaf(ray.dy, nz, -ray.dz * ny);
        a_w[1] = gamma * fmaf(ray.dz, nx, -ray.dx * nz);
        a_w[2] = gamma * fmaf(ray.dx, ny, -ray.dy * nx);
    }
    __syncthreads();
    // per-material sums over the lanes of this wavefront, one material at a time
    uint64_t todo = __ballot(m != kNone);
    while (todo) {
        int leader = __ffsll((unsigned long long)todo) - 1;
        uint32_t mm = __shfl(m, leader, 64);
        bool mine = (m == mm);
        uint64_t grp = __ballot(mine);
        double vr = wave_sum(mine ? (double)a_rho : 0.0);
        double vk = wave_sum(mine ? (double)a_k : 0.0);
        if (lane == 0) {
            acc[w][mm] = vr;
            acc[w][nmat + mm] = vk;
        }
        todo &= ~grp;
    }
    for (int q = 0; q < 3; ++q) {
        double vp = wave_sum((double)a_p[q]);
        double vw = wave_sum((double)a_w[q]);
        if (lane == 0) {
            acc[w][2 * nmat + q] = vp;
            acc[w][2 * nmat + 3 + q] = vw;
        }
    }
    __syncthreads();
    for (uint32_t o = threadIdx.x; o < n_out; o += kAdjBlock) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += acc[q][o];
        partials[(size_t)blockIdx.x * n_out + o] = s;
    }
}

// one block per output: fixed-stride partial sums, then a fixed tree
__global__ __launch_bounds__(256) void adjoint_sum_kernel(const double *__restrict__ partials, uint32_t nblocks,
                                                          uint32_t n_out, double *__restrict__ tot) {
    __shared__ double red[256];
    const uint32_t o = blockIdx.x;
    double s = 0.0;
    for (uint32_t q = threadIdx.x; q < nblocks; q += 256) s += partials[(size_t)q * n_out + o];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[o] = red[0];
}

// Spectral form (d_spectra non-null): dL/dT[m][b] = w_b dL/dR_lambda(0)_m with
// the interpolation weights w of the wavelength, computed as in the forward.
__global__ __launch_bounds__(64) void adjoint_final_kernel(const double *__restrict__ tot, uint32_t nmat,
                                                           const float *__restrict__ pose_delta, float *d_rho,
                                                           float *d_k, float *d_pose6, float *d_spectra,
                                                           MaterialsDev M, float wavelength_nm) {
    for (uint32_t o = threadIdx.x; o < nmat; o += blockDim.x) {
        if (d_rho) d_rho[o] = (float)tot[o];
        if (d_k) d_k[o] = (float)tot[nmat + o];
    }
    if (d_spectra) {
        float q = (wavelength_nm - M.lambda0) / M.dlambda;
        int b0, b1;
        float w0, w1;
        if (q <= 0.0f) { b0 = b1 = 0; w0 = 1.0f; w1 = 0.0f; }
        else if (q >= (float)(M.nbins - 1)) { b0 = b1 = (int)M.nbins - 1; w0 = 1.0f; w1 = 0.0f; }
        else {
            b0 = (int)floorf(q);
            b1 = b0 + 1;
            w1 = q - (float)b0;
            w0 = 1.0f - w1;
        }
        const uint32_t n = nmat * M.nbins;
        for (uint32_t o = threadIdx.x; o < n; o += blockDim.x) {
            uint32_t m = o / M.nbins, b = o - m * M.nbins;
            double g = tot[m];
            double v = (b == (uint32_t)b0 ? (double)w0 * g : 0.0) + (b == (uint32_t)b1 && b1 != b0 ? (double)w1 * g : 0.0);
            d_spectra[o] = (float)v;
        }
    }
    if (threadIdx.x == 0 && d_pose6) {
        const double *g = tot + 2 * nmat;
        d_pose6[0] = (float)g[0]; d_pose6[1] = (float)g[1]; d_pose6[2] = (float)g[2];
        // rotation: J_l(dw)^T g_left
        double w0 = 0, w1 = 0, w2 = 0;
        if (pose_delta) { w0 = pose_delta[3]; w1 = pose_delta[4]; w2 = pose_delta[5]; }
        double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
        double A, B;   // J = I + A K + B K^2
        if (th < 1e-8) { A = 0.5; B = 1.0 / 6.0; }
        else { A = (1.0 - cos(th)) / th2; B = (th - sin(th)) / (th2 * th); }
        double K[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
        double J[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double k2 = K[r * 3] * K[c] + K[r * 3 + 1] * K[3 + c] + K[r * 3 + 2] * K[6 + c];
                J[r * 3 + c] = (r == c ? 1.0 : 0.0) + A * K[r * 3 + c] + B * k2;
            }
        const double *gl = g + 3;
        for (int c = 0; c < 3; ++c)
            d_pose6[3 + c] = (float)(J[0 * 3 + c] * gl[0] + J[1 * 3 + c] * gl[1] + J[2 * 3 + c] * gl[2]);
    }
}

size_t adjoint_partial_bytes(uint32_t n_beams, uint32_t nmat) {
    size_t nb = (n_beams + kAdjBlock - 1) / kAdjBlock;
    return (nb + 1) * (2 * (size_t)nmat + 6) * sizeof(double);
}

void launch_adjoint(const SceneDev &S, const uint32_t *slot_of, const InstanceDev &in, const MaterialsDev &M,
                    const Overrides &ov, const uint32_t *tri, const uint8_t *valid, const float *clamp_I,
                    const float *gI, const float *gd, double *partials, float *d_rho, float *d_k, float *d_pose6, float *d_spectra,
                    hipStream_t s) {
    uint32_t nb = in.n_ch * in.n_az;
    uint32_t blocks = (nb + kAdjBlock - 1) / kAdjBlock;
    uint32_t n_out = 2 * M.nmat + 6;
    double *tot = partials + (size_t)blocks * n_out;
    adjoint_kernel<<<blocks, kAdjBlock, 0, s>>>(S, slot_of, in, M, ov, tri, valid, clamp_I, gI, gd, partials);
    adjoint_sum_kernel<<<n_out, 256, 0, s>>>(partials, blocks, n_out, tot);
    adjoint_final_kernel<<<1, 64, 0, s>>>(tot, M.nmat, ov.pose_delta, d_rho, d_k, d_pose6, d_spectra, M,
                                          in.wavelength_nm);
}

}  // namespace lidar
