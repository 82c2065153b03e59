// probe.hip -- achievable-bandwidth probes (gfx950).  Not on the simulation
// path: they measure the memory roofs that the trace kernels' algorithmic
// bandwidth is compared with.
//
//   stream  every 16-byte word of a buffer read once (grid-stride float4
//           loads), nothing written: the HBM read roof for a buffer much
//           larger than the caches.
//   gather  128-byte lines fetched by the four lanes of a quad, 32 bytes each,
//           as a quad fetches a BVH node; line indices uniform over a working
//           set (for the trace kernels: the scene's nodes and records).  With
//           `chase`, each line index is a hash of the previous line's data, so
//           the fetches of a quad form a dependent chain like a walk's node
//           fetches; otherwise the indices come from a counter hash and every
//           fetch is independent.
// Both accumulate what they read and store it only if it equals an unlikely
// value, so the loads cannot be removed and no write traffic is added.
#include "lidar_device.hpp"
#include "lidar_kernels.hpp"

namespace lidar {

namespace {

constexpr int kProbeBlock = 256;

__device__ inline uint32_t mix32(uint32_t x) {   // a 32-bit finaliser (multiply-xorshift)
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(kProbeBlock) void stream_read_kernel(const float4 *__restrict__ buf, uint64_t n4,
                                                                  float *__restrict__ sink) {
    float acc = 0.0f;
    const uint64_t stride = (uint64_t)gridDim.x * kProbeBlock;
    for (uint64_t k = (uint64_t)blockIdx.x * kProbeBlock + threadIdx.x; k < n4; k += stride) {
        const float4 v = buf[k];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == 1.2345678e-30f) sink[0] = acc;
}

__global__ __launch_bounds__(kProbeBlock) void gather_kernel(const void *__restrict__ table, uint32_t n_lines,
                                                             uint32_t steps, int chase, float *__restrict__ sink) {
    const __amdgpu_buffer_rsrc_t rs = raw_buffer(table);
    const uint32_t quad = (blockIdx.x * kProbeBlock + threadIdx.x) >> 2, s = threadIdx.x & 3u;
    uint32_t h = mix32(quad * 0x9E3779B9u + 0x632BE5ABu);
    float acc = 0.0f;
    for (uint32_t i = 0; i < steps; ++i) {
        const uint32_t line = (uint32_t)(((uint64_t)h * n_lines) >> 32);   // uniform in [0, n_lines)
        const uint32_t off = line * 128u + s * 32u;
        const float4 a = buf_load4(rs, off), b = buf_load4(rs, off + 16u);
        acc += (a.x + a.y) + (b.z + b.w);
        if (chase) {
            // the quad's next line from the bits it just read (the same value in all four lanes) and the
            // quad's own index, so that two quads that meet on a line do not continue on one chain
            uint32_t d = __float_as_uint(a.x) ^ __float_as_uint(b.w);
            d ^= quad_xor1(d);
            d ^= quad_xor2(d);
            h = mix32(d ^ (quad * 0x9E3779B9u + i));
        } else {
            h = mix32(h + 0x9E3779B9u);
        }
    }
    if (acc == 1.2345678e-30f) sink[0] = acc;
}

}  // namespace

void launch_probe_stream(const void *buf, uint64_t bytes, float *sink, hipStream_t s) {
    const uint64_t n4 = bytes / 16;
    stream_read_kernel<<<256 * 16, kProbeBlock, 0, s>>>((const float4 *)buf, n4, sink);
}

void launch_probe_gather(const void *table, uint32_t n_lines, uint32_t blocks, uint32_t steps, int chase,
                         float *sink, hipStream_t s) {
    gather_kernel<<<blocks, kProbeBlock, 0, s>>>(table, n_lines, steps, chase, sink);
}

}  // namespace lidar
