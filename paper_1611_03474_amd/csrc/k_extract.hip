// Edge intersection points of the trilinear surface g = c (eq. intersection)
// on SURFACE leaves.  gfx950.
//
// On a cube edge g is linear in the edge coordinate, so its root is
// t = (c - phi0) / (phi1 - phi0) from the lower end.  Edges shared by leaves of
// the same level are emitted once: each crossing edge is owned by one leaf
// (found in a per-level leaf-lattice bitmap), which sets its bit in a dense
// per-(conformation, level, axis) edge bitmap in key order; vertices are
// written at their bits' ranks, so the list comes out in edge-key order.
#include "tms_device.h"

namespace tms {

namespace {

constexpr int kBS = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

// Edge e of a leaf: axis = e / 4; the two other axes in ascending order take
// offsets (e & 1, (e >> 1) & 1).  Returns corner indices v0 (lower end) and v1.
__device__ __forceinline__ void edge_corners(int e, int &axis, int off[3], int &v0, int &v1) {
    axis = e >> 2;
    const int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
    const int lo = o1 < o2 ? o1 : o2, hi = o1 < o2 ? o2 : o1;
    off[0] = off[1] = off[2] = 0;
    off[lo] = e & 1;
    off[hi] = (e >> 1) & 1;
    v0 = off[0] + 2 * off[1] + 4 * off[2];
    v1 = v0 + (1 << axis);
}

__device__ __forceinline__ uint64_t edge_key(const tms_leaf &L, int axis, const int off[3], int K) {
    const int sh = K - L.level;
    const uint64_t X = (uint64_t)((L.ix + off[0]) << sh);
    const uint64_t Y = (uint64_t)((L.iy + off[1]) << sh);
    const uint64_t Z = (uint64_t)((L.iz + off[2]) << sh);
    return ((uint64_t)(uint32_t)L.conf << 53) | ((uint64_t)L.level << 50) |
           ((uint64_t)axis << 48) | (X << 32) | (Y << 16) | Z;
}

// ---- dense-bitmap edge de-duplication ------------------------------------
__device__ __forceinline__ int64_t edge_bit(const EdgeLat &el, const tms_leaf &L, int axis,
                                            const int off[3]) {
    const Lat &lat = el.l[L.level][axis];
    return (lat.base << 6) +
           (((int64_t)(L.ix + off[0]) * lat.n[1] + (L.iy + off[1])) * lat.n[2] + (L.iz + off[2]));
}

// Bit of cube (X, Y, Z) of level `lev` in the leaf-lattice bitmap; false
// outside the lattice.
__device__ __forceinline__ bool leaf_bit(const EdgeLat &el, int lev, int64_t X, int64_t Y,
                                         int64_t Z, int64_t &b) {
    const Lat &lat = el.leaf[lev];
    if (X < 0 || Y < 0 || Z < 0 || (X >> 2) >= lat.n[0] || (Y >> 2) >= lat.n[1] ||
        (Z >> 2) >= lat.n[2])
        return false;
    b = lat_bit(lat, X, Y, Z);
    return true;
}

// one bit per surface leaf in its level's leaf lattice; the wavefront merges
// the words of all its leaves (consecutive leaves share 4x4x4 blocks) and
// ORs each distinct word into the bitmap once
__global__ void k_leaf_mark(const tms_leaf *__restrict__ leaves, int64_t n,
                            const EdgeLat *__restrict__ et, unsigned long long *__restrict__ lbm,
                            const int64_t *__restrict__ nd) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    const int lane = threadIdx.x & 63;
    // every lane stays to the end: the merge reads all lanes' registers
    bool pend = false;
    int64_t w = 0;
    unsigned long long m = 0;
    if (q < n && !(nd && q >= *nd)) {
        const tms_leaf L = leaves[q];
        int64_t b;
        if (L.cls == TMS_CLS_SURFACE && leaf_bit(et[L.conf], L.level, L.ix, L.iy, L.iz, b)) {
            w = b >> 6;
            m = 1ull << (b & 63);
            pend = true;
        }
    }
    while (true) {
        const unsigned long long left = __ballot(pend);
        if (left == 0) break;
        const int leader = __ffsll(left) - 1;
        const int64_t W = __shfl(w, leader, 64);
        unsigned long long mine = 0;
        if (pend && w == W) {
            mine = m;
            pend = false;
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) mine |= __shfl_xor(mine, d, 64);
        if (lane == leader) atomicOr(lbm + W, mine);
    }
}

// One thread per surface leaf.  A crossing edge is shared by the leaves of
// its level around it (all of them surface leaves: they hold both of its end
// corners); the leaf in which the edge sits at the smallest offset pair
// (2 o1 + o2 over the two other axes, in edge order) that exists owns it.
// The owner ORs the edge's bit (merged per 64-bit word) and records the edge
// in own[q]; the leaves sharing an edge share its corner values, so the
// owner chosen does not change the vertex.
__global__ void k_edge_mark(const tms_leaf *__restrict__ leaves, int64_t n,
                            const EdgeLat *__restrict__ et, const uint64_t *__restrict__ lbm,
                            unsigned long long *__restrict__ bm, uint16_t *__restrict__ own,
                            const int64_t *__restrict__ nd) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (q >= n || (nd && q >= *nd)) return;
    const tms_leaf L = leaves[q];
    unsigned o = 0;
    if (L.cls == TMS_CLS_SURFACE) {
        const EdgeLat &el = et[L.conf];
        const int64_t P[3] = {L.ix, L.iy, L.iz};
        int64_t w[12];
        unsigned long long m[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            int axis, off[3], v0, v1;
            edge_corners(e, axis, off, v0, v1);
            m[e] = 0;
            w[e] = 0;
            if (!(((L.mask >> v0) ^ (L.mask >> v1)) & 1)) continue;
            // the other axes in ascending order and this leaf's offsets there
            const int b1 = axis == 0 ? 1 : 0, b2 = axis == 2 ? 1 : 2;
            const int o1 = off[b1], o2 = off[b2];
            bool mine = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int d1 = k >> 1, d2 = k & 1;  // offsets of the edge in that leaf
                if (2 * d1 + d2 >= 2 * o1 + o2) continue;
                int64_t C[3] = {P[0], P[1], P[2]};
                C[b1] += o1 - d1;
                C[b2] += o2 - d2;
                int64_t lb;
                if (leaf_bit(el, L.level, C[0], C[1], C[2], lb) && ((lbm[lb >> 6] >> (lb & 63)) & 1ull))
                    mine = false;
            }
            if (!mine) continue;
            const int64_t b = edge_bit(el, L, axis, off);
            w[e] = b >> 6;
            m[e] = 1ull << (b & 63);
            o |= 1u << e;
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            if (m[e] == 0) continue;
            unsigned long long bits = m[e];
#pragma unroll
            for (int u = e + 1; u < 12; ++u)
                if (m[u] != 0 && w[u] == w[e]) {
                    bits |= m[u];
                    m[u] = 0;
                }
            atomicOr(bm + w[e], bits);
        }
    }
    own[q] = (uint16_t)o;
}

// the vertices of the edges a leaf owns, each at its edge's rank (the list
// comes out in edge-key order).  One thread per leaf.
__global__ void k_edge_write(const Grid *__restrict__ gt, const tms_leaf *__restrict__ leaves,
                             const double *__restrict__ cphi, int64_t n,
                             const EdgeLat *__restrict__ et, const uint64_t *__restrict__ bm,
                             const int32_t *__restrict__ woff, const uint16_t *__restrict__ own,
                             tms_vertex *__restrict__ out, const int64_t *__restrict__ nd,
                             int64_t vcap, unsigned *__restrict__ ovf) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (q >= n || (nd && q >= *nd)) return;
    const unsigned o = own[q];
    if (!o) return;
    const tms_leaf L = leaves[q];
    const Grid &g = gt[L.conf];
    const EdgeLat &el = et[L.conf];
    const int sh = g.K - L.level;
    const double h = ldexp(g.h0, -(int)L.level);
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        if (!((o >> e) & 1)) continue;
        int axis, off[3], v0, v1;
        edge_corners(e, axis, off, v0, v1);
        const int64_t b = edge_bit(el, L, axis, off);
        const int64_t w = b >> 6;
        const int64_t r = (int64_t)woff[w] + __popcll(bm[w] & ((1ull << (b & 63)) - 1ull));
        if (ovf && r >= vcap) {  // capacity-sized buffer (capture path)
            atomicOr(ovf, 1u);
            continue;
        }
        const double f0 = cphi[8 * q + v0], f1 = cphi[8 * q + v1];
        double p[3] = {g.o[0] + (double)((L.ix + off[0]) << sh) * g.hmin,
                       g.o[1] + (double)((L.iy + off[1]) << sh) * g.hmin,
                       g.o[2] + (double)((L.iz + off[2]) << sh) * g.hmin};
        const double t = (g.c - f0) / (f1 - f0);
        p[axis] += t * h;
        tms_vertex V;
        V.edge_key = edge_key(L, axis, off, g.K);
        V.t = t;
        V.x = p[0];
        V.y = p[1];
        V.z = p[2];
        out[r] = V;
    }
}

}  // namespace

hipError_t launch_leaf_mark(const tms_leaf *leaves, int64_t n, const EdgeLat *et,
                            unsigned long long *lbm, hipStream_t s, const int64_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaf_mark, dim3(nblk(n)), dim3(kBS), 0, s, leaves, n, et, lbm, nd);
    return hipGetLastError();
}

hipError_t launch_edge_mark(const tms_leaf *leaves, int64_t n, const EdgeLat *et,
                            const uint64_t *lbm, unsigned long long *bm, uint16_t *own,
                            hipStream_t s, const int64_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_mark, dim3(nblk(n)), dim3(kBS), 0, s, leaves, n, et, lbm, bm, own,
                       nd);
    return hipGetLastError();
}

hipError_t launch_edge_write(const Grid *gt, const tms_leaf *leaves, const double *cphi, int64_t n,
                             const EdgeLat *et, const uint64_t *bm, const int32_t *woff,
                             const uint16_t *own, tms_vertex *out, hipStream_t s,
                             const int64_t *nd, int64_t vcap, unsigned *ovf) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_write, dim3(nblk(n)), dim3(kBS), 0, s, gt, leaves, cphi, n, et, bm,
                       woff, own, out, nd, vcap, ovf);
    return hipGetLastError();
}

}  // namespace tms
