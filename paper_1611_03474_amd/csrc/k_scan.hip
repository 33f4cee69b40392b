// Device-wide exclusive prefix sum over int32 and small fill kernels (gfx950).
//
// Tiles of 2048 values per 256-thread workgroup: each thread owns 8
// consecutive values, threads are combined with a 64-wide wavefront scan
// (cross-lane shuffles) and the 4 wavefront totals through LDS.  Tile totals
// are scanned recursively.  The scan keeps input order, which is what makes
// every compaction in the library stable and its outputs reproducible.
#include "tms_internal.h"

namespace tms {

namespace {

constexpr int kBS = 256;
constexpr int kIPT = 8;
constexpr int kTile = kBS * kIPT;
constexpr int kWaves = kBS / 64;

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan of one tile held as 8 values per thread; returns the tile
// total; `vals` become exclusive prefixes inside the tile
__device__ __forceinline__ int block_scan(int vals[kIPT], int *sh_wave) {
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int run = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        int v = vals[k];
        vals[k] = run;
        run += v;
    }
    int incl = wave_incl_scan(run, lane);
    if (lane == 63) sh_wave[wave] = incl;
    __syncthreads();
    int wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        int t = sh_wave[w];
        if (w < wave) wbase += t;
        total += t;
    }
    int base = wbase + incl - run;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) vals[k] += base;
    return total;
}

__global__ void k_tile_sums(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ sums) {
    __shared__ int sh_wave[kWaves];
    int64_t base = (int64_t)blockIdx.x * kTile;
    int run = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        int64_t i = base + (int64_t)k * kBS + threadIdx.x;  // coalesced
        run += (i < n) ? in[i] : 0;
    }
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = wave_incl_scan(run, lane);
    if (lane == 63) sh_wave[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kWaves; ++w) t += sh_wave[w];
        sums[blockIdx.x] = t;
    }
}

// scan tiles; offs (may be null) holds the exclusive offset of each tile;
// the last tile writes the grand total
__global__ void k_tile_scan(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                            const int32_t *__restrict__ offs, int32_t *__restrict__ total) {
    __shared__ int sh[kTile];
    __shared__ int sh_wave[kWaves];
    int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        int idx = k * kBS + threadIdx.x;
        int64_t i = base + idx;
        sh[idx] = (i < n) ? in[i] : 0;
    }
    __syncthreads();
    int vals[kIPT];
#pragma unroll
    for (int k = 0; k < kIPT; ++k) vals[k] = sh[threadIdx.x * kIPT + k];
    int tot = block_scan(vals, sh_wave);
    int off = offs ? offs[blockIdx.x] : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kIPT; ++k) sh[threadIdx.x * kIPT + k] = vals[k] + off;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        int idx = k * kBS + threadIdx.x;
        int64_t i = base + idx;
        if (i < n) out[i] = sh[idx];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
    size_t b = 0;
    while (n > kTile) {
        int64_t nb = (n + kTile - 1) / kTile;
        b += 2 * sizeof(int32_t) * (size_t)nb + 256;
        n = nb;
    }
    return b + 256;
}

hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev, void *tmp,
                          hipStream_t s) {
    if (n <= 0) {
        // a fill kernel, not a memset: a captured pass holds no memset node
        if (total_dev) return launch_fill_u32(reinterpret_cast<uint32_t *>(total_dev), 0u, 1, s);
        return hipSuccess;
    }
    int64_t nb = (n + kTile - 1) / kTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kBS), 0, s, in, out, n, nullptr, total_dev);
        return hipGetLastError();
    }
    int32_t *sums = static_cast<int32_t *>(tmp);
    int32_t *offs = sums + nb;
    char *rest = reinterpret_cast<char *>(offs + nb);
    rest += (256 - (reinterpret_cast<uintptr_t>(rest) & 255)) & 255;
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nb), dim3(kBS), 0, s, in, n, sums);
    hipError_t e = exclusive_scan(sums, offs, nb, nullptr, rest, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nb), dim3(kBS), 0, s, in, out, n, offs, total_dev);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + kBS - 1) / kBS)), dim3(kBS), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + kBS - 1) / kBS)), dim3(kBS), 0, s, p, v, n);
    return hipGetLastError();
}

namespace {
__global__ void k_gather_i32(const int32_t *__restrict__ src, const int64_t *__restrict__ idx,
                             int n, int64_t *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = src[idx[i]];
}
}  // namespace

hipError_t launch_gather_i32(const int32_t *src, const int64_t *idx, int n, int64_t *out,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_i32, dim3((n + 255) / 256), dim3(256), 0, s, src, idx, n, out);
    return hipGetLastError();
}

}  // namespace tms
