// phi / grad phi at points (eq. Gaussian1) and the leaf-corner stage:
// unique finest-lattice corners, phi once per corner, 8-bit sign masks and
// classes against c (eq. linear1).  gfx950.
//
// Every phi value at a point is a pure function of the point: the atoms
// within R_c of it, summed in ascending atom order (cells row by row).  So
// corners shared by neighbouring leaves get bit-identical values and signs.
#include "tms_device.h"

namespace tms {

namespace {

constexpr int kBS = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

// FAST phi kernel: every term carries a relative error <= kFastExpErr, so
// |dphi| <= kFastExpErr phi.  guard[k] = 1 when the sign of phi - c is not
// certain (|phi - c| <= 2 kFastExpErr phi) or when |phi - c| <= band_rel * c;
// the caller recomputes those points with exact exponentials.
template <bool FAST, bool GRAD>
__global__ __launch_bounds__(kBS) void k_phi_points(const Grid *__restrict__ gt,
                                                    const int32_t *__restrict__ pconf,
                                                    const double *__restrict__ pts,
                                                    int64_t m, const int32_t *__restrict__ cs,
                                                    const double4 *__restrict__ xw,
                                                    double band_rel, double *__restrict__ phi,
                                                    double *__restrict__ grad,
                                                    uint8_t *__restrict__ guard,
                                                    const int32_t *__restrict__ nd) {
    int64_t k = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (k >= m || (nd && k >= (int64_t)*nd)) return;
    const Grid &g = gt[pconf ? pconf[k] : 0];
    const double p[3] = {pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]};
    double f, gr[3];
    phi_at<FAST, GRAD>(g, p, cs, xw, f, gr);
    phi[k] = f;
    if (GRAD) {
        grad[3 * k] = gr[0];
        grad[3 * k + 1] = gr[1];
        grad[3 * k + 2] = gr[2];
    }
    if (guard) {
        const double m_ = fabs(f - g.c);
        guard[k] = (m_ <= 2.0 * kFastExpErr * f + 1e-300 || m_ <= band_rel * g.c) ? 1 : 0;
    }
}

// ---- phi at the unique leaf corners, atoms staged per wavefront ------------
// The unique corners come in bitmap-rank order: 64 consecutive ones mostly lie
// in a few neighbouring 4x4x4 lattice blocks.  A wavefront splits its 64
// points into spatial groups (the first point left and every point left of
// its conformation within `reach` R_c of it along each axis; at most `gmax`
// groups, else every lane runs phi_at on its own).  For each group it loads,
// coalesced, the atoms of the cell rows around the group's bounding box, keeps
// those within R_c of the box and packs them, in atom order, into LDS; every
// lane of the group then sums its own point over the packed atoms with the
// same operations and the same distance test as phi_at.  phi_at takes exactly
// the atoms within R_c of its point (the packed set holds them all), in
// ascending atom order (cells are stored row by row), so each value is
// bit-identical to phi_at's: only the loads are shared.
constexpr int kCW = kBS / 64;   // wavefronts per workgroup
constexpr int kCCap = 256;      // packed atoms per wavefront before a sum

template <bool FAST>
__global__ __launch_bounds__(kBS) void k_phi_corners(
    const Grid *__restrict__ gt, const int32_t *__restrict__ pconf,
    const double *__restrict__ pts, int64_t m, const int32_t *__restrict__ cs,
    const double4 *__restrict__ xw, double band_rel, int gmax, double reach,
    double *__restrict__ phi, uint8_t *__restrict__ guard, const int32_t *__restrict__ nd) {
    __shared__ double4 s_at[kCW][kCCap + 4];
    __shared__ int s_rb[kCW][64];  // first atom of each row of a row group
    __shared__ int s_rp[kCW][64];  // exclusive prefix of the rows' atom counts
    const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    int64_t mm = m;
    if (nd) mm = min(mm, (int64_t)*nd);
    const int64_t k0 = blockIdx.x * (int64_t)kBS + (int64_t)(threadIdx.x - lane);
    if (k0 >= mm) return;  // uniform across the wavefront
    const int64_t k = k0 + lane;
    const bool valid = k < mm;
    const int64_t kk = valid ? k : k0;
    const int b = pconf ? pconf[kk] : 0;
    const double p0 = pts[3 * kk], p1 = pts[3 * kk + 1], p2 = pts[3 * kk + 2];

    // the group of the first point in `left` (every lane takes part: the
    // shuffles read the leader's registers)
    auto group_of = [&](unsigned long long left) -> unsigned long long {
        const int ld = __ffsll(left) - 1;
        const int lb = __shfl(b, ld, 64);
        const double r = reach * sqrt(gt[lb].rc2);
        const double lx = __shfl(p0, ld, 64), ly = __shfl(p1, ld, 64), lz = __shfl(p2, ld, 64);
        const bool mine = ((left >> lane) & 1ull) && b == lb && fabs(p0 - lx) <= r &&
                          fabs(p1 - ly) <= r && fabs(p2 - lz) <= r;
        // the leader always joins its own group, so every round takes a point
        return __ballot(mine) | (1ull << ld);
    };
    const unsigned long long all = __ballot(valid);
    unsigned long long left = all;
    for (int ng = 0; left != 0ull && ng <= gmax; ++ng) left &= ~group_of(left);

    double f = 0.0;
    if (left != 0ull) {  // more than gmax groups
        if (valid) {
            const double p[3] = {p0, p1, p2};
            double gr[3];
            phi_at<FAST, false>(gt[b], p, cs, xw, f, gr);
        }
    } else {
        double4 *at = s_at[wv];
        left = all;
        while (left != 0ull) {
            const unsigned long long gm = group_of(left);
            left &= ~gm;
            const bool ing = (gm >> lane) & 1ull;
            const int ld = __ffsll(gm) - 1;
            const int lb = __builtin_amdgcn_readfirstlane(__shfl(b, ld, 64));
            const Grid &g = gt[lb];
            const double rc2 = g.rc2, D = g.D;
            // the group's bounding box (lanes outside it take the leader's
            // point; the shuffles run on every lane)
            const double q0 = __shfl(p0, ld, 64), q1 = __shfl(p1, ld, 64),
                         q2 = __shfl(p2, ld, 64);
            double lo0 = ing ? p0 : q0, lo1 = ing ? p1 : q1, lo2 = ing ? p2 : q2;
            double hi0 = lo0, hi1 = lo1, hi2 = lo2;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                lo0 = fmin(lo0, __shfl_xor(lo0, d, 64));
                lo1 = fmin(lo1, __shfl_xor(lo1, d, 64));
                lo2 = fmin(lo2, __shfl_xor(lo2, d, 64));
                hi0 = fmax(hi0, __shfl_xor(hi0, d, 64));
                hi1 = fmax(hi1, __shfl_xor(hi1, d, 64));
                hi2 = fmax(hi2, __shfl_xor(hi2, d, 64));
            }
            // cells within the stencil of some point of the box (cell
            // indices clamped to +-1e8 before conversion; corners are lattice
            // points inside the grid)
            int c0[3], c1[3];
            {
                const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double fl = fmin(fmax(floor(over_cs(g, lo[a] - g.o[a])), -1.0e8), 1.0e8);
                    const double fh = fmin(fmax(floor(over_cs(g, hi[a] - g.o[a])), -1.0e8), 1.0e8);
                    c0[a] = max((int)fl - g.span, 0);
                    c1[a] = min((int)fh + g.span, g.nc[a] - 1);
                }
            }
            const int ny = c1[1] - c0[1] + 1;
            const int nrow = (ny > 0 && c1[2] >= c0[2] && c1[0] >= c0[0])
                                 ? (c1[2] - c0[2] + 1) * ny : 0;
            // atoms kept: within R_c of the box (a margin of 2^-40 relative
            // covers the rounding of either squared distance)
            const double keep2 = rc2 * (1.0 + 0x1p-40);
            int n = 0;  // packed atoms (uniform)
            // sum the packed atoms over the group's points: pad to a multiple
            // of four with atoms that no point takes, then four per step
            auto flush = [&]() {
                const int np = (n + 3) & ~3;
                if (lane < np - n) at[n + lane] = make_double4(1e300, 1e300, 1e300, 0.0);
                wave_lds_sync();
                if (ing) {
                    for (int j = 0; j < np; j += 4) {
                        double4 a[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) a[u] = at[j + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const double dx = p0 - a[u].x, dy = p1 - a[u].y, dz = p2 - a[u].z;
                            const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
                            if (!(d2 > rc2)) f = fma(a[u].w, expn<FAST>(-D * d2), f);
                        }
                    }
                }
                wave_lds_sync();
                n = 0;
            };
            for (int r0 = 0; r0 < nrow; r0 += 64) {
                // lane r: row r0 + r (z outer, y inner), its x range clipped
                // to the chord of the R_c neighbourhood of the box (enlarged
                // by 2^-16 relative: a row may keep a cell more than needed,
                // never one less)
                const int r = r0 + lane;
                int rb = 0, len = 0;
                if (r < nrow) {
                    const int cz = c0[2] + r / ny, cy = c0[1] + r % ny;
                    const double lz = g.o[2] + cz * g.cs, ly = g.o[1] + cy * g.cs;
                    const double ez = fmax(fmax(lz - hi2, lo2 - (lz + g.cs)), 0.0);
                    const double ey = fmax(fmax(ly - hi1, lo1 - (ly + g.cs)), 0.0);
                    const double ryz = (rc2 - ez * ez) - ey * ey;
                    if (ryz >= 0.0) {
                        const double hx = sqrt(ryz) * (1.0 + 0x1p-16);
                        const int x0 = max(c0[0], (int)floor(over_cs(g, lo0 - hx - g.o[0])));
                        const int x1 = min(c1[0], (int)floor(over_cs(g, hi0 + hx - g.o[0])));
                        if (x0 <= x1) {
                            const int row = (int)g.cell_base + (cz * g.nc[1] + cy) * g.nc[0];
                            rb = cs[row + x0];
                            len = cs[row + x1 + 1] - rb;
                        }
                    }
                }
                int inc = len;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int t = __shfl_up(inc, d, 64);
                    if (lane >= d) inc += t;
                }
                const int tot = __builtin_amdgcn_readfirstlane(__shfl(inc, 63, 64));
                const int nr = min(64, nrow - r0);
                s_rb[wv][lane] = rb;
                s_rp[wv][lane] = inc - len;
                wave_lds_sync();
                for (int t = 0; t < tot; t += 64) {
                    const int fi = t + lane;
                    bool keep = false;
                    double4 a = make_double4(0.0, 0.0, 0.0, 0.0);
                    if (fi < tot) {
                        // the row holding flattened atom fi: the last row whose
                        // prefix is <= fi
                        int lo = 0, hi = nr - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (s_rp[wv][mid] <= fi) lo = mid;
                            else hi = mid - 1;
                        }
                        a = xw[s_rb[wv][lo] + (fi - s_rp[wv][lo])];
                        const double ex = fmax(fmax(lo0 - a.x, a.x - hi0), 0.0);
                        const double ey = fmax(fmax(lo1 - a.y, a.y - hi1), 0.0);
                        const double ez = fmax(fmax(lo2 - a.z, a.z - hi2), 0.0);
                        keep = fma(ez, ez, fma(ey, ey, ex * ex)) <= keep2;
                    }
                    const unsigned long long bk = __ballot(keep);
                    if (keep) at[n + __popcll(bk & ((1ull << lane) - 1ull))] = a;
                    n += __popcll(bk);
                    if (n > kCCap - 64) flush();
                }
                wave_lds_sync();  // the row tables are rewritten next
            }
            flush();
        }
    }
    if (valid) {
        phi[k] = f;
        if (guard) {
            const double m_ = fabs(f - gt[b].c);
            guard[k] = (m_ <= 2.0 * kFastExpErr * f + 1e-300 || m_ <= band_rel * gt[b].c) ? 1 : 0;
        }
    }
}

// number of (point, atom) pairs within R_c over the points (the terms phi
// sums); one atomic add per wavefront
__global__ __launch_bounds__(kBS) void k_phi_pairs(const Grid *__restrict__ gt,
                                                   const double *__restrict__ pts, int64_t m,
                                                   const int32_t *__restrict__ cs,
                                                   const double4 *__restrict__ xw,
                                                   unsigned long long *__restrict__ count) {
    const int64_t k = blockIdx.x * (int64_t)kBS + threadIdx.x;
    unsigned long long c = 0;
    if (k < m) {
        const double p[3] = {pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]};
        double f, gr[3];
        phi_at<false, false, true>(gt[0], p, cs, xw, f, gr);
        c = (unsigned long long)f;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ __launch_bounds__(kBS) void k_phi_subset(const Grid *__restrict__ gt,
                                                    const int32_t *__restrict__ pconf,
                                                    const double *__restrict__ pts,
                                                    const int32_t *__restrict__ list, int64_t m,
                                                    const int32_t *__restrict__ cs,
                                                    const double4 *__restrict__ xw,
                                                    double *__restrict__ phi,
                                                    double *__restrict__ grad,
                                                    const int32_t *__restrict__ nd) {
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t >= m || (nd && t >= (int64_t)*nd)) return;
    const int64_t k = list[t];
    const Grid &g = gt[pconf ? pconf[k] : 0];
    const double p[3] = {pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]};
    double f, gr[3];
    phi_at<false>(g, p, cs, xw, f, gr);
    phi[k] = f;
    if (grad) {
        grad[3 * k] = gr[0];
        grad[3 * k + 1] = gr[1];
        grad[3 * k + 2] = gr[2];
    }
}

__device__ __forceinline__ void classify(tms_leaf &L, const double f[8], double c) {
    uint8_t m = 0;
#pragma unroll
    for (int v = 0; v < 8; ++v)
        if (f[v] >= c) m |= (uint8_t)(1u << v);
    L.mask = m;
    L.cls = (m == 0) ? TMS_CLS_OUTSIDE : (m == 0xFF ? TMS_CLS_INSIDE : TMS_CLS_SURFACE);
}

__global__ void k_uniform_leaves(Grid g, tms_leaf *__restrict__ leaves, int64_t n) {
    int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (q >= n) return;
    tms_leaf L;
    L.ix = (int32_t)(q % g.nr[0]);
    L.iy = (int32_t)((q / g.nr[0]) % g.nr[1]);
    L.iz = (int32_t)(q / ((int64_t)g.nr[0] * g.nr[1]));
    L.conf = 0;
    L.level = 0;
    L.reason = TMS_REASON_UNIFORM;
    L.mask = 0;
    L.cls = 0;
    leaves[q] = L;
}

__global__ void k_uniform_points(Grid g, double *__restrict__ pts, int64_t m) {
    int64_t k = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (k >= m) return;
    const int64_t px = g.nr[0] + 1, py = g.nr[1] + 1;
    const int64_t x = k % px, y = (k / px) % py, z = k / (px * py);
    pts[3 * k] = g.o[0] + (double)x * g.h0;
    pts[3 * k + 1] = g.o[1] + (double)y * g.h0;
    pts[3 * k + 2] = g.o[2] + (double)z * g.h0;
}

__global__ void k_uniform_gather(Grid g, const double *__restrict__ uphi, double c,
                                 tms_leaf *__restrict__ leaves, int64_t n,
                                 double *__restrict__ cphi) {
    int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (q >= n) return;
    tms_leaf L = leaves[q];
    const int64_t px = g.nr[0] + 1, py = g.nr[1] + 1;
    double f[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int64_t x = L.ix + (v & 1), y = L.iy + ((v >> 1) & 1), z = L.iz + ((v >> 2) & 1);
        f[v] = uphi[(z * py + y) * px + x];
    }
    classify(L, f, c);
    leaves[q] = L;
    if (cphi) {
#pragma unroll
        for (int v = 0; v < 8; ++v) cphi[8 * q + v] = f[v];
    }
}

__global__ void k_count_u8(const uint8_t *__restrict__ v, int64_t n, uint8_t value,
                           unsigned long long *__restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    unsigned long long c = (i < n && v[i] == value) ? 1ull : 0ull;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

__global__ void k_flags_u8(const uint8_t *__restrict__ gd, int64_t n,
                           const int32_t *__restrict__ nd, int32_t *__restrict__ f) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n) f[i] = ((!nd || i < (int64_t)*nd) && gd[i]) ? 1 : 0;
}

__global__ void k_list_emit2(const int32_t *__restrict__ f, const int32_t *__restrict__ off,
                             int64_t n, int32_t *__restrict__ list) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n && f[i]) list[off[i]] = (int32_t)i;
}

// Indices of the flagged points appended to `list`, one device-scope atomic
// per wavefront that holds any (the wave's lanes take consecutive slots in
// lane order).  The list order depends on the wavefronts' timing; every listed
// point is recomputed on its own, so results do not depend on it.
__global__ __launch_bounds__(kBS) void k_guard_append(const uint8_t *__restrict__ gd, int64_t n,
                                                      int32_t *__restrict__ list,
                                                      unsigned *__restrict__ cnt) {
    const int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    const bool f = i < n && gd[i];
    const unsigned long long b = __ballot(f);
    if (b == 0ull) return;  // uniform across the wavefront
    const int lane = (int)(threadIdx.x & 63);
    const int leader = __ffsll(b) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(cnt, (unsigned)__popcll(b));
    base = __shfl(base, leader, 64);
    if (f) list[base + (unsigned)__popcll(b & ((1ull << lane) - 1ull))] = (int32_t)i;
}

// number of SURFACE leaves: block partials, then one block
__global__ void k_count_surface(const tms_leaf *__restrict__ leaves, int64_t n,
                                const int64_t *__restrict__ nd,
                                unsigned long long *__restrict__ part) {
    __shared__ unsigned long long sh[kBS];
    unsigned long long c = 0;
    if (nd) n = min(n, *nd);
    for (int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBS)
        c += leaves[i].cls == TMS_CLS_SURFACE;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int st = kBS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const unsigned long long *__restrict__ part, int nb,
                            unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[kBS];
    unsigned long long t = 0;
    for (int b = threadIdx.x; b < nb; b += kBS) t += part[b];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int st = kBS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---- dense-bitmap corner de-duplication -----------------------------------
// Corner bitmaps are tiled: one 64-bit word per 4x4x4 block of lattice
// points (lat.n counts blocks per axis), blocks in raster order, so the
// unique corners come out in compact spatial groups and a wavefront of the
// phi kernel works on neighbouring points.
__device__ __forceinline__ void leaf_corner(const tms_leaf &L, int v, int K, int64_t &X, int64_t &Y,
                                            int64_t &Z) {
    const int sh = K - L.level;
    X = (int64_t)(L.ix + (v & 1)) << sh;
    Y = (int64_t)(L.iy + ((v >> 1) & 1)) << sh;
    Z = (int64_t)(L.iz + ((v >> 2) & 1)) << sh;
}

__global__ void k_popc(const uint64_t *__restrict__ bm, int64_t nw, int32_t *__restrict__ cnt) {
    const int64_t w = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (w < nw) cnt[w] = __popcll(bm[w]);
}

// one thread per leaf: its 8 corner bits, merged per 64-bit word (a
// finest-level leaf usually has all 8 in one 4x4x4 block); then the
// wavefront merges the words of all its leaves (consecutive leaves share
// blocks) and ORs each distinct word into the bitmap once
__global__ void k_corner_mark(const tms_leaf *__restrict__ leaves, int64_t n, int K,
                              const Grid *__restrict__ gt, unsigned long long *__restrict__ bm,
                              const int64_t *__restrict__ nd) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    const int lane = threadIdx.x & 63;
    // every lane stays to the end: the merge reads all lanes' registers
    const bool act = q < n && !(nd && q >= *nd);
    int64_t w[8];
    unsigned long long m[8];
    unsigned pend = 0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        w[v] = 0;
        m[v] = 0;
    }
    if (act) {
        const tms_leaf L = leaves[q];
        const Lat lat = gt[L.conf].clat;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            int64_t X, Y, Z;
            leaf_corner(L, v, K, X, Y, Z);
            const int64_t b = lat_bit(lat, X, Y, Z);
            w[v] = b >> 6;
            m[v] = 1ull << (b & 63);
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            if (m[v] == 0) continue;
#pragma unroll
            for (int u = v + 1; u < 8; ++u)
                if (m[u] != 0 && w[u] == w[v]) {
                    m[v] |= m[u];
                    m[u] = 0;
                }
            pend |= 1u << v;
        }
    }
    // one distinct word per round: the first lane with a word left names
    // it, every lane gives its bits of that word, one atomic OR
    while (true) {
        const unsigned long long left = __ballot(pend != 0);
        if (left == 0) break;
        const int leader = __ffsll(left) - 1;
        int64_t fw = 0;
#pragma unroll
        for (int v = 7; v >= 0; --v)
            if ((pend >> v) & 1) fw = w[v];
        const int64_t W = __shfl(fw, leader, 64);
        unsigned long long mine = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (((pend >> v) & 1) && w[v] == W) {
                mine |= m[v];
                pend &= ~(1u << v);
            }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) mine |= __shfl_xor(mine, d, 64);
        if (lane == leader) atomicOr(bm + W, mine);
    }
}

// Unique corner points from the bitmap alone, each at its bit's rank (points
// in rank order, each once).  A wavefront covers 64 consecutive words and
// walks its non-empty ones together: for each, lane j writes the point of
// bit j if it is set, so the points of a word go out as one contiguous run.
// Word w belongs to the last conformation whose block starts at or before
// it; inside a block, word ((bx n1 + by) n2 + bz) covers points
// (4 bx + i, 4 by + j, 4 bz + k) at bit 16 i + 4 j + k.
__global__ void k_corner_enum(const Grid *__restrict__ gt, int nconf,
                              const uint64_t *__restrict__ bm, const int32_t *__restrict__ woff,
                              int64_t nw, double *__restrict__ upts, int32_t *__restrict__ uconf,
                              int64_t ucap, unsigned *__restrict__ ovf) {
    const int64_t w = blockIdx.x * (int64_t)kBS + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint64_t m = w < nw ? bm[w] : 0ull;
    const int32_t wo = m ? woff[w] : 0;
    unsigned long long left = __ballot(m != 0ull);
    const int64_t w0 = w - lane;  // the wavefront's first word
    while (left) {
        const int j = __ffsll(left) - 1;
        left &= left - 1ull;
        const int64_t ww = w0 + j;
        const uint64_t mm = __shfl(m, j, 64);
        const int64_t base = __shfl(wo, j, 64);
        int lo = 0, hi = nconf - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (gt[mid].clat.base <= ww) lo = mid;
            else hi = mid - 1;
        }
        const Grid &g = gt[lo];
        // block coordinates in 32 bits (a conformation's bitmap holds fewer
        // than 2^31 words)
        const uint32_t lw = (uint32_t)(ww - g.clat.base);
        const uint32_t n2 = (uint32_t)g.clat.n[2], n1 = (uint32_t)g.clat.n[1];
        const uint32_t t = lw / n2, bz = lw - t * n2;
        const uint32_t bx = t / n1, by = t - bx * n1;
        if (!((mm >> lane) & 1ull)) continue;
        const int64_t u = base + __popcll(mm & ((1ull << lane) - 1ull));
        if (ovf && u >= ucap) {  // capacity-sized buffers (capture path)
            atomicOr(ovf, 1u);
            continue;
        }
        const int64_t X = 4 * (int64_t)bx + (lane >> 4), Y = 4 * (int64_t)by + ((lane >> 2) & 3),
                      Z = 4 * (int64_t)bz + (lane & 3);
        upts[3 * u] = g.o[0] + (double)X * g.hmin;
        upts[3 * u + 1] = g.o[1] + (double)Y * g.hmin;
        upts[3 * u + 2] = g.o[2] + (double)Z * g.hmin;
        uconf[u] = lo;
    }
}

__global__ void k_corner_gather_bm(const tms_leaf *__restrict__ lin, int64_t n, int K,
                                   const Grid *__restrict__ gt, const uint64_t *__restrict__ bm,
                                   const int32_t *__restrict__ woff, const double *__restrict__ uphi,
                                   double c, tms_leaf *__restrict__ lout,
                                   double *__restrict__ cphi, const int64_t *__restrict__ nd,
                                   int64_t ucap, unsigned *__restrict__ ovf) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (q >= n || (nd && q >= *nd)) return;
    tms_leaf L = lin[q];
    const Lat lat = gt[L.conf].clat;
    double f[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        int64_t X, Y, Z;
        leaf_corner(L, v, K, X, Y, Z);
        const int64_t u = bit_rank(bm, woff, lat_bit(lat, X, Y, Z));
        if (ovf && u >= ucap) {
            atomicOr(ovf, 1u);
            f[v] = 0.0;
        } else {
            f[v] = uphi[u];
        }
    }
    classify(L, f, c);
    lout[q] = L;
    if (cphi) {
#pragma unroll
        for (int v = 0; v < 8; ++v) cphi[8 * q + v] = f[v];
    }
}

}  // namespace

hipError_t launch_popc(const uint64_t *bm, int64_t nwords, int32_t *cnt, hipStream_t s) {
    if (nwords <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_popc, dim3(nblk(nwords)), dim3(kBS), 0, s, bm, nwords, cnt);
    return hipGetLastError();
}

hipError_t launch_corner_mark(const tms_leaf *leaves, int64_t n, int K, const Grid *gt,
                              unsigned long long *bm, hipStream_t s, const int64_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_corner_mark, dim3(nblk(n)), dim3(kBS), 0, s, leaves, n, K, gt, bm, nd);
    return hipGetLastError();
}

hipError_t launch_corner_enum(const Grid *gt, int nconf, const uint64_t *bm, const int32_t *woff,
                              int64_t nwords, double *upts, int32_t *uconf, hipStream_t s,
                              int64_t ucap, unsigned *ovf) {
    if (nwords <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_corner_enum, dim3(nblk(nwords)), dim3(kBS), 0, s, gt, nconf, bm, woff,
                       nwords, upts, uconf, ucap, ovf);
    return hipGetLastError();
}

hipError_t launch_corner_gather_bm(const tms_leaf *lin, int64_t n, int K, const Grid *gt,
                                   const uint64_t *bm, const int32_t *woff, const double *uphi,
                                   double c, tms_leaf *lout, double *cphi, hipStream_t s,
                                   const int64_t *nd, int64_t ucap, unsigned *ovf) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_corner_gather_bm, dim3(nblk(n)), dim3(kBS), 0, s, lin, n, K, gt, bm, woff,
                       uphi, c, lout, cphi, nd, ucap, ovf);
    return hipGetLastError();
}

hipError_t launch_phi_points(const Grid *gt, const int32_t *pconf, int precision, const double *pts,
                             int64_t m, const int32_t *cs, const double4 *xw, double band_rel,
                             double *phi, double *grad, uint8_t *guard, hipStream_t s,
                             const int32_t *nd) {
    if (m <= 0) return hipSuccess;
    // corner values need no gradient: a variant without it
    if (precision == TMS_PREC_FP32_GUARD) {
        if (grad)
            hipLaunchKernelGGL((k_phi_points<true, true>), dim3(nblk(m)), dim3(kBS), 0, s, gt, pconf,
                               pts, m, cs, xw, band_rel, phi, grad, guard, nd);
        else
            hipLaunchKernelGGL((k_phi_points<true, false>), dim3(nblk(m)), dim3(kBS), 0, s, gt,
                               pconf, pts, m, cs, xw, band_rel, phi, grad, guard, nd);
    } else {
        if (grad)
            hipLaunchKernelGGL((k_phi_points<false, true>), dim3(nblk(m)), dim3(kBS), 0, s, gt,
                               pconf, pts, m, cs, xw, 0.0, phi, grad, nullptr, nd);
        else
            hipLaunchKernelGGL((k_phi_points<false, false>), dim3(nblk(m)), dim3(kBS), 0, s, gt,
                               pconf, pts, m, cs, xw, 0.0, phi, grad, nullptr, nd);
    }
    return hipGetLastError();
}

hipError_t launch_phi_corners(const Grid *gt, const int32_t *pconf, int precision,
                              const double *pts, int64_t m, const int32_t *cs, const double4 *xw,
                              double band_rel, int groups, double reach, double *phi,
                              uint8_t *guard, hipStream_t s, const int32_t *nd) {
    if (m <= 0) return hipSuccess;
    if (groups <= 0)
        return launch_phi_points(gt, pconf, precision, pts, m, cs, xw, band_rel, phi, nullptr,
                                 guard, s, nd);
    if (precision == TMS_PREC_FP32_GUARD)
        hipLaunchKernelGGL(k_phi_corners<true>, dim3(nblk(m)), dim3(kBS), 0, s, gt, pconf, pts, m,
                           cs, xw, band_rel, groups, reach, phi, guard, nd);
    else
        hipLaunchKernelGGL(k_phi_corners<false>, dim3(nblk(m)), dim3(kBS), 0, s, gt, pconf, pts, m,
                           cs, xw, 0.0, groups, reach, phi, nullptr, nd);
    return hipGetLastError();
}

hipError_t launch_phi_points_subset(const Grid *gt, const int32_t *pconf, const double *pts,
                                    const int32_t *list, int64_t m, const int32_t *cs,
                                    const double4 *xw, double *phi, double *grad, hipStream_t s,
                                    const int32_t *nd) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_phi_subset, dim3(nblk(m)), dim3(kBS), 0, s, gt, pconf, pts, list, m, cs, xw,
                       phi, grad, nd);
    return hipGetLastError();
}

hipError_t launch_uniform_leaves(const Grid &g, tms_leaf *leaves, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uniform_leaves, dim3(nblk(n)), dim3(kBS), 0, s, g, leaves, n);
    return hipGetLastError();
}

hipError_t launch_uniform_points(const Grid &g, double *pts, int64_t m, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uniform_points, dim3(nblk(m)), dim3(kBS), 0, s, g, pts, m);
    return hipGetLastError();
}

hipError_t launch_uniform_gather(const Grid &g, const double *uphi, double c, tms_leaf *leaves,
                                 int64_t n, double *cphi, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uniform_gather, dim3(nblk(n)), dim3(kBS), 0, s, g, uphi, c, leaves, n, cphi);
    return hipGetLastError();
}

hipError_t launch_count_u8(const uint8_t *v, int64_t n, uint8_t value, unsigned long long *count,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_u8, dim3(nblk(n)), dim3(kBS), 0, s, v, n, value, count);
    return hipGetLastError();
}

hipError_t launch_guard_flags_u8(const uint8_t *gd, int64_t n, int32_t *flags, hipStream_t s,
                                 const int32_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flags_u8, dim3(nblk(n)), dim3(kBS), 0, s, gd, n, nd, flags);
    return hipGetLastError();
}

hipError_t launch_list_emit(const int32_t *flags, const int32_t *off, int64_t n, int32_t *list,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_list_emit2, dim3(nblk(n)), dim3(kBS), 0, s, flags, off, n, list);
    return hipGetLastError();
}

hipError_t launch_phi_pairs(const Grid *gt, const double *pts, int64_t m, const int32_t *cs,
                            const double4 *xw, unsigned long long *count, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_phi_pairs, dim3(nblk(m)), dim3(kBS), 0, s, gt, pts, m, cs, xw, count);
    return hipGetLastError();
}

hipError_t launch_guard_append(const uint8_t *gd, int64_t n, int32_t *list, unsigned *cnt,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_guard_append, dim3(nblk(n)), dim3(kBS), 0, s, gd, n, list, cnt);
    return hipGetLastError();
}

hipError_t launch_count_surface(const tms_leaf *leaves, int64_t n, unsigned long long *count,
                                unsigned long long *part, hipStream_t s, const int64_t *nd) {
    if (n <= 0) return hipSuccess;
    const int nb = (int)std::min<int64_t>(1024, (n + kBS - 1) / kBS);
    hipLaunchKernelGGL(k_count_surface, dim3(nb), dim3(kBS), 0, s, leaves, n, nd, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBS), 0, s, part, nb, count);
    return hipGetLastError();
}

}  // namespace tms
