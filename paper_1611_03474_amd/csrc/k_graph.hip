// Small kernels of the captured (host-synchronisation-free) pass: sizes that
// the eager pass reads back to the host stay on the device here.  gfx950.
#include "tms_device.h"

namespace tms {

namespace {

// ns[k] = clamp(*n - k S, 0, S): the entries of equal queue slices
__global__ void k_slice_counts(const int32_t *__restrict__ n, int64_t S, int nslices,
                               int32_t *__restrict__ ns) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nslices) return;
    const int64_t r = (int64_t)*n - (int64_t)k * S;
    ns[k] = (int32_t)(r < 0 ? 0 : (r > S ? S : r));
}

__global__ void k_acc_i64(int64_t *__restrict__ acc, const int32_t *__restrict__ v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *acc += (int64_t)*v;
}

// Regrouping plan of a batch's leaves (one thread; nseg = (K + 1) nconf is
// at most a few thousand): src[seg] is the first leaf of segment
// seg = level * nconf + conf in level order (-1: empty); dst[seg] its first
// slot in conformation order; leaf_off[b] the first leaf of conformation b.
__global__ void k_seg_plan(const int64_t *__restrict__ src, int nlev, int nconf,
                           const int64_t *__restrict__ L, int64_t lcap, int64_t *__restrict__ dst,
                           int64_t *__restrict__ leaf_off) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t nL = *L < lcap ? *L : lcap;  // leaves beyond the capacity were not written
    const int nseg = nlev * nconf;
    // counts into dst first: a present segment ends where the next one starts
    int64_t prev = -1;
    for (int seg = 0; seg < nseg; ++seg) {
        dst[seg] = 0;
        if (src[seg] < 0) continue;
        if (prev >= 0) dst[prev] = src[seg] - src[prev];
        prev = seg;
    }
    if (prev >= 0) dst[prev] = nL - src[prev];
    int64_t pos = 0;
    for (int b = 0; b < nconf; ++b) {
        leaf_off[b] = pos;
        for (int lev = 0; lev < nlev; ++lev) {
            const int seg = lev * nconf + b;
            const int64_t c = dst[seg];
            dst[seg] = pos;
            pos += c;
        }
    }
    leaf_off[nconf] = pos;
}

// after an overflow the next level sees an empty queue (its entries were
// not all written)
__global__ void k_stop_on_overflow(const unsigned *__restrict__ ovf, int32_t *__restrict__ n) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *ovf) *n = 0;
}

}  // namespace

hipError_t launch_stop_on_overflow(const unsigned *ovf, int32_t *n, hipStream_t s) {
    hipLaunchKernelGGL(k_stop_on_overflow, dim3(1), dim3(64), 0, s, ovf, n);
    return hipGetLastError();
}

hipError_t launch_slice_counts(const int32_t *n, int64_t S, int nslices, int32_t *ns,
                               hipStream_t s) {
    if (nslices <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_counts, dim3((nslices + 255) / 256), dim3(256), 0, s, n, S, nslices,
                       ns);
    return hipGetLastError();
}

hipError_t launch_acc_i64(int64_t *acc, const int32_t *v, hipStream_t s) {
    hipLaunchKernelGGL(k_acc_i64, dim3(1), dim3(64), 0, s, acc, v);
    return hipGetLastError();
}

hipError_t launch_seg_plan(const int64_t *src, int nlev, int nconf, const int64_t *L, int64_t lcap,
                           int64_t *dst, int64_t *leaf_off, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(64), 0, s, src, nlev, nconf, L, lcap, dst,
                       leaf_off);
    return hipGetLastError();
}

}  // namespace tms
