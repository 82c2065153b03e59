// compact.hip -- order-preserving compaction of a point cloud (gfx950).
//
// The simulation writes dense per-beam arrays (one element per beam, misses
// and dropped returns included).  A consumer of the labelled point cloud
// (Fig.1 of the paper: points with depth, intensity and label) usually wants
// only the detected points.  Compaction copies the beams with valid != 0 to
// the front of the output arrays, in beam order, plus each point's beam index.
//
// Stream-ordered launches, no atomics (the result is deterministic):
//   1. per 256-beam block: the wavefront's detected beams as a 64-bit ballot,
//      their popcounts summed in LDS -> counts[block];
//   2. one 1024-thread block: exclusive prefix sum of counts, in chunks of
//      1024, and the total;
//   3. per 256-beam block: the beam's rank = the block's offset + the counts
//      of the block's earlier wavefronts + popcount(ballot & lanes below), then
//      every requested field is copied to that rank.
// Up to kFusedBlocks blocks (a scan of up to 524,288 beams) steps 2 and 3 are
// one launch: each block sums the counts before it itself (at most 8 loads per
// thread), which costs less than a launch of its own.
#include <mutex>

#include "lidar_device.hpp"
#include "lidar_kernels.hpp"

// Scratch of the allocation-free entry point: the per-block counts of up to
// kStaticCountWords blocks (2^25 beams), one copy per GPU, held by the library
// until the process ends.  Host code never uses this name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr uint32_t kStaticCountWords = 131072;   // 512 KiB
static __device__ __align__(256) uint32_t scratch[kStaticCountWords];

namespace lidar {

constexpr int kCompactBlock = 256;    // beams per block (4 wavefronts)
constexpr int kScanBlock = 1024;

__device__ inline uint64_t lanes_below() {
    const uint32_t lane = threadIdx.x & 63u;
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

__global__ __launch_bounds__(kCompactBlock) void compact_count_kernel(const uint8_t *__restrict__ valid, uint64_t n,
                                                                      uint32_t *__restrict__ counts) {
    __shared__ uint32_t wsum[kCompactBlock / 64];
    const uint64_t g = (uint64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const bool v = g < n && valid[g] != 0;
    const uint64_t m = __ballot(v);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kCompactBlock / 64; ++w) c += wsum[w];
        counts[blockIdx.x] = c;
    }
}

// Inclusive scan of one value per lane across the wavefront (shift-up steps).
__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__global__ __launch_bounds__(kScanBlock) void compact_scan_kernel(uint32_t *__restrict__ counts, uint32_t n_blocks,
                                                                  uint32_t *__restrict__ total) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    __shared__ uint32_t carry_s;
    if (threadIdx.x == 0) carry_s = 0u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint32_t base = 0; base < n_blocks; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < n_blocks ? counts[i] : 0u;
        const uint32_t inc = wave_inclusive_scan(x);
        if (lane == 63u) wsum[wave] = inc;
        __syncthreads();
        uint32_t before = carry_s;
        for (uint32_t w = 0; w < wave; ++w) before += wsum[w];
        if (i < n_blocks) counts[i] = before + inc - x;
        __syncthreads();     // every thread has read carry_s and wsum
        if (threadIdx.x == kScanBlock - 1) carry_s = before + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry_s;
}

constexpr uint32_t kFusedBlocks = 2048;

// FUSED: `offsets` holds the per-block counts of step 1; the block's offset is
// their sum over the blocks before it, and the last block writes the total.
template <bool FUSED>
__global__ __launch_bounds__(kCompactBlock) void compact_scatter_kernel(Outputs dense, Outputs comp,
                                                                        uint32_t *__restrict__ beam_index,
                                                                        const uint32_t *__restrict__ offsets,
                                                                        uint64_t n, uint32_t *__restrict__ total) {
    __shared__ uint32_t wsum[kCompactBlock / 64];
    __shared__ uint32_t wpre[kCompactBlock / 64];
    const uint64_t g = (uint64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const bool v = g < n && dense.valid[g] != 0;
    const uint64_t m = __ballot(v);
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) wsum[wave] = (uint32_t)__popcll(m);
    uint32_t base = 0;
    if constexpr (FUSED) {
        uint32_t part = 0;
        for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kCompactBlock) part += offsets[b];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
        if ((threadIdx.x & 63u) == 0) wpre[wave] = part;
    }
    __syncthreads();
    if constexpr (FUSED) {
#pragma unroll
        for (int w = 0; w < kCompactBlock / 64; ++w) base += wpre[w];
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
            uint32_t c = base;
#pragma unroll
            for (int w = 0; w < kCompactBlock / 64; ++w) c += wsum[w];
            *total = c;
        }
    } else {
        base = offsets[blockIdx.x];
    }
    if (!v) return;
    uint32_t pos = base;
    for (uint32_t w = 0; w < wave; ++w) pos += wsum[w];
    pos += (uint32_t)__popcll(m & lanes_below());
    if (comp.valid) comp.valid[pos] = dense.valid[g];
    if (comp.label) comp.label[pos] = dense.label[g];
    if (comp.x) comp.x[pos] = dense.x[g];
    if (comp.y) comp.y[pos] = dense.y[g];
    if (comp.z) comp.z[pos] = dense.z[g];
    if (comp.intensity) comp.intensity[pos] = dense.intensity[g];
    if (comp.range) comp.range[pos] = dense.range[g];
    if (comp.tri) comp.tri[pos] = dense.tri[g];
    if (comp.t_hit) comp.t_hit[pos] = dense.t_hit[g];
    if (comp.material) comp.material[pos] = dense.material[g];
    if (comp.r_lambda) comp.r_lambda[pos] = dense.r_lambda[g];
    if (comp.normal) {
        comp.normal[pos] = dense.normal[g];
        comp.normal[pos + comp.plane] = dense.normal[g + dense.plane];
        comp.normal[pos + 2 * comp.plane] = dense.normal[g + 2 * dense.plane];
    }
    if (beam_index) beam_index[pos] = (uint32_t)g;
}

uint64_t compact_blocks(uint64_t n) { return (n + kCompactBlock - 1) / kCompactBlock; }

uint64_t compact_static_max_beams() { return (uint64_t)kStaticCountWords * kCompactBlock; }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t compact_static_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    // the caller has made `device` current; each device holds its own copy of the array
    uint32_t *p = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
    return hipSuccess;
}

uint32_t *compact_static_counts(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

void launch_compact(const Outputs &dense, const Outputs &comp, uint32_t *beam_index, uint32_t *count, uint64_t n,
                    uint32_t *counts, hipStream_t s) {
    const uint64_t nb = compact_blocks(n);
    if (nb > 0) compact_count_kernel<<<(uint32_t)nb, kCompactBlock, 0, s>>>(dense.valid, n, counts);
    if (nb > 0 && nb <= kFusedBlocks) {
        compact_scatter_kernel<true><<<(uint32_t)nb, kCompactBlock, 0, s>>>(dense, comp, beam_index, counts, n, count);
        return;
    }
    compact_scan_kernel<<<1, kScanBlock, 0, s>>>(counts, (uint32_t)nb, count);
    if (nb > 0)
        compact_scatter_kernel<false><<<(uint32_t)nb, kCompactBlock, 0, s>>>(dense, comp, beam_index, counts, n,
                                                                            count);
}

}  // namespace lidar
