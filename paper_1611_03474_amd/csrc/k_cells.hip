// Atom binning and per-root neighbourhood lists (gfx950).
//
// The sums of Section 2.2.1 (after eq. polynew) run only over atoms near a
// cube.  Atoms are counting-sorted into cells (edge: the smallest h0 * 2^m
// >= R_c / 4) aligned with the root grid; inside a cell they keep ascending
// input order, so every sum below visits atoms in one canonical order and
// results are reproducible bit for bit.  Each root cube then gets the list of
// atoms whose squared distance to the root box is <= R_c^2 -- a superset of
// the neighbourhood of every cube inside it.
//
// A batch of conformations shares these arrays: conformation b owns the
// cells [cell_base, ...) and roots [root_base, ...) of its geometry entry,
// and its atoms [atom_base, ...) of the concatenated input.
#include "tms_device.h"

namespace tms {

namespace {

constexpr int kBS = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Per conformation b (one workgroup each, atoms [off[b], off[b+1])):
// out[9b + 0..2] min xyz, [3..5] max xyz, [6] max r, [7] min r, [8] count of
// non-finite values.
// per (segment of kStatSeg atoms, conformation) partials: grid (S, nconf)
constexpr int64_t kStatSeg = 4096;

__global__ __launch_bounds__(kBS) void k_stats_conf(const double *__restrict__ xyzr,
                                                    const int64_t *__restrict__ off,
                                                    double *__restrict__ out) {
    const int b = blockIdx.y;
    const int64_t i0 = off[b] + (int64_t)blockIdx.x * kStatSeg,
                  i1 = min(off[b + 1], i0 + kStatSeg);
    double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
    double rmax = -1e308, rmin = 1e308, bad = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBS) {
        double v[4] = {xyzr[4 * i], xyzr[4 * i + 1], xyzr[4 * i + 2], xyzr[4 * i + 3]};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 4; ++a) ok = ok && isfinite(v[a]);
        if (!ok) {
            bad += 1.0;
            continue;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], v[a]);
            mx[a] = fmax(mx[a], v[a]);
        }
        rmax = fmax(rmax, v[3]);
        rmin = fmin(rmin, v[3]);
    }
    __shared__ double sh[9][kBS];
    for (int a = 0; a < 3; ++a) {
        sh[a][threadIdx.x] = mn[a];
        sh[3 + a][threadIdx.x] = mx[a];
    }
    sh[6][threadIdx.x] = rmax;
    sh[7][threadIdx.x] = rmin;
    sh[8][threadIdx.x] = bad;
    __syncthreads();
    for (int st = kBS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            int o = threadIdx.x + st;
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = fmin(sh[a][threadIdx.x], sh[a][o]);
                sh[3 + a][threadIdx.x] = fmax(sh[3 + a][threadIdx.x], sh[3 + a][o]);
            }
            sh[6][threadIdx.x] = fmax(sh[6][threadIdx.x], sh[6][o]);
            sh[7][threadIdx.x] = fmin(sh[7][threadIdx.x], sh[7][o]);
            sh[8][threadIdx.x] += sh[8][o];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9)
        out[9 * ((int64_t)b * gridDim.x + blockIdx.x) + threadIdx.x] = sh[threadIdx.x][0];
}

// per conformation: min / max / sum over its segments' partials (one
// wavefront; order-free: min, max, and sums of integer-valued counts)
__global__ void k_stats_final(const double *__restrict__ part, int S, double *__restrict__ out) {
    const int b = blockIdx.x, lane = threadIdx.x;
    double v[9] = {1e308, 1e308, 1e308, -1e308, -1e308, -1e308, -1e308, 1e308, 0.0};
    for (int k = lane; k < S; k += 64) {
        const double *p = part + 9 * ((int64_t)b * S + k);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], p[a]);
            v[3 + a] = fmax(v[3 + a], p[3 + a]);
        }
        v[6] = fmax(v[6], p[6]);
        v[7] = fmin(v[7], p[7]);
        v[8] += p[8];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], __shfl_xor(v[a], d, 64));
            v[3 + a] = fmax(v[3 + a], __shfl_xor(v[3 + a], d, 64));
        }
        v[6] = fmax(v[6], __shfl_xor(v[6], d, 64));
        v[7] = fmin(v[7], __shfl_xor(v[7], d, 64));
        v[8] += __shfl_xor(v[8], d, 64);
    }
    if (lane == 0)
#pragma unroll
        for (int a = 0; a < 9; ++a) out[9 * b + a] = v[a];
}

__device__ __forceinline__ int cell_of(const Grid &g, double x, int a) {
    return clampi((int)floor(over_cs(g, x - g.o[a])), 0, g.nc[a] - 1);
}

__global__ void k_bin(const Grid *__restrict__ gt, int nconf, const double *__restrict__ xyzr,
                      int64_t n, int32_t *__restrict__ key, int32_t *__restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    const Grid &g = gt[conf_of_atom(gt, nconf, i)];
    int cx = cell_of(g, xyzr[4 * i], 0), cy = cell_of(g, xyzr[4 * i + 1], 1),
        cz = cell_of(g, xyzr[4 * i + 2], 2);
    int k = (int)g.cell_base + (cz * g.nc[1] + cy) * g.nc[0] + cx;
    key[i] = k;
    atomicAdd(&cnt[k], 1);
}

__global__ void k_scatter(const Grid *__restrict__ gt, const double *__restrict__ xyzr, int64_t n,
                          const int32_t *__restrict__ key, int32_t *__restrict__ fill,
                          double *__restrict__ ax, double *__restrict__ ay, double *__restrict__ az,
                          double *__restrict__ aw, double *__restrict__ ar,
                          int32_t *__restrict__ aidx) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    int pos = atomicAdd(&fill[key[i]], 1);
    double r = xyzr[4 * i + 3];
    ax[pos] = xyzr[4 * i];
    ay[pos] = xyzr[4 * i + 1];
    az[pos] = xyzr[4 * i + 2];
    ar[pos] = r;
    aw[pos] = exp(gt[0].D * r * r);
    aidx[pos] = (int32_t)i;
}

// restore ascending input order inside each cell (insertion sort; cells hold
// a few tens of atoms)
__global__ void k_sort_cells(const int32_t *__restrict__ start, int64_t ncells, double *ax,
                             double *ay, double *az, double *aw, double *ar, int32_t *aidx) {
    int64_t c = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (c >= ncells) return;
    int b = start[c], e = start[c + 1];
    for (int i = b + 1; i < e; ++i) {
        int32_t ki = aidx[i];
        double x = ax[i], y = ay[i], z = az[i], w = aw[i], r = ar[i];
        int j = i - 1;
        while (j >= b && aidx[j] > ki) {
            aidx[j + 1] = aidx[j];
            ax[j + 1] = ax[j];
            ay[j + 1] = ay[j];
            az[j + 1] = az[j];
            aw[j + 1] = aw[j];
            ar[j + 1] = ar[j];
            --j;
        }
        aidx[j + 1] = ki;
        ax[j + 1] = x;
        ay[j + 1] = y;
        az[j + 1] = z;
        aw[j + 1] = w;
        ar[j + 1] = r;
    }
}

// Visit the atoms whose squared distance to the root box is <= R_c^2, in
// cell order.  EMIT=false counts, EMIT=true writes the sorted-atom indices.
// Each stencil row is clipped to the cells its atoms can reach: with ey, ez
// the row's y and z gaps to the box, an atom in it is within R_c only if its
// x gap is at most sqrt(R_c^2 - ey^2 - ez^2).  That chord is taken from
// R_c^2 enlarged by 2^-20 and the hardware reciprocal square root enlarged
// by 2^-20 (far above its error and the rounding of the gaps), so a row may
// keep a cell more than needed (whose atoms the test drops) but never one
// less: the list is the same set in the same order.
template <bool EMIT>
__global__ void k_root_lists(const Grid *__restrict__ gt, int nconf, const int32_t *__restrict__ cs,
                             const double4 *__restrict__ xw, int64_t nroots,
                             const int32_t *__restrict__ start, int32_t *__restrict__ out) {
    int64_t r = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (r >= nroots) return;
    const Grid &g = gt[conf_of_root(gt, nconf, r)];
    const int64_t rl = r - g.root_base;
    int rx = (int)(rl % g.nr[0]), ry = (int)((rl / g.nr[0]) % g.nr[1]),
        rz = (int)(rl / ((int64_t)g.nr[0] * g.nr[1]));
    double lo[3] = {g.o[0] + rx * g.h0, g.o[1] + ry * g.h0, g.o[2] + rz * g.h0};
    double hi[3] = {lo[0] + g.h0, lo[1] + g.h0, lo[2] + g.h0};
    const double rc2 = g.rc2, rc2m = rc2 * (1.0 + 0x1p-20);
    double R = sqrt(rc2);
    int c0[3], c1[3];
    for (int a = 0; a < 3; ++a) {
        c0[a] = clampi((int)floor(over_cs(g, lo[a] - R - g.o[a])), 0, g.nc[a] - 1);
        c1[a] = clampi((int)floor(over_cs(g, hi[a] + R - g.o[a])), 0, g.nc[a] - 1);
    }
    int cnt = 0;
    int w = EMIT ? start[r] : 0;
    for (int cz = c0[2]; cz <= c1[2]; ++cz) {
        const double lz = g.o[2] + cz * g.cs;
        const double ez = fmax(fmax(lz - hi[2], lo[2] - (lz + g.cs)), 0.0);
        for (int cy = c0[1]; cy <= c1[1]; ++cy) {
            const double ly = g.o[1] + cy * g.cs;
            const double ey = fmax(fmax(ly - hi[1], lo[1] - (ly + g.cs)), 0.0);
            const double ryz = (rc2m - ez * ez) - ey * ey;
            if (!(ryz >= 0.0)) continue;
            const double hx =
                ryz > 0.0 ? ryz * __builtin_amdgcn_rsq(ryz) * (1.0 + 0x1p-20) : 0.0;
            const int x0 = max(c0[0], (int)floor(over_cs(g, lo[0] - hx - g.o[0])));
            const int x1 = min(c1[0], (int)floor(over_cs(g, hi[0] + hx - g.o[0])));
            if (x0 > x1) continue;
            const int row = (int)g.cell_base + (cz * g.nc[1] + cy) * g.nc[0];
            const int b = cs[row + x0], e = cs[row + x1 + 1];
            for (int i = b; i < e; ++i) {
                const double4 a = xw[i];
                double dx = fmax(fmax(lo[0] - a.x, a.x - hi[0]), 0.0);
                double dy = fmax(fmax(lo[1] - a.y, a.y - hi[1]), 0.0);
                double dz = fmax(fmax(lo[2] - a.z, a.z - hi[2]), 0.0);
                if (dx * dx + dy * dy + dz * dz <= rc2) {
                    if (EMIT) out[w++] = i;
                    else ++cnt;
                }
            }
        }
    }
    if (!EMIT) out[r] = cnt;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

}  // namespace

size_t atom_stats_tmp_bytes(int nconf, int64_t max_atoms) {
    const int64_t S = std::max<int64_t>(1, (max_atoms + kStatSeg - 1) / kStatSeg);
    return sizeof(double) * 9 * (size_t)nconf * (size_t)S;
}

hipError_t launch_atom_stats(const double *xyzr, const int64_t *off, int nconf, int64_t max_atoms,
                             double *out, double *tmp, hipStream_t s) {
    const int64_t S = std::max<int64_t>(1, (max_atoms + kStatSeg - 1) / kStatSeg);
    hipLaunchKernelGGL(k_stats_conf, dim3((unsigned)S, (unsigned)nconf), dim3(kBS), 0, s, xyzr,
                       off, tmp);
    hipLaunchKernelGGL(k_stats_final, dim3((unsigned)nconf), dim3(64), 0, s, tmp, (int)S, out);
    return hipGetLastError();
}

hipError_t launch_bin_atoms(const Grid *gt, int nconf, const double *xyzr, int64_t n, int32_t *key,
                            int32_t *cnt, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin, dim3(nblk(n)), dim3(kBS), 0, s, gt, nconf, xyzr, n, key, cnt);
    return hipGetLastError();
}

hipError_t launch_scatter_atoms(const Grid *gt, const double *xyzr, int64_t n, const int32_t *key,
                                int32_t *fill, double *ax, double *ay, double *az, double *aw,
                                double *ar, int32_t *aidx, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(nblk(n)), dim3(kBS), 0, s, gt, xyzr, n, key, fill, ax, ay,
                       az, aw, ar, aidx);
    return hipGetLastError();
}

// (x, y, z, w) of each atom in one 32-byte record, in cell order: the point
// kernels read an atom with one pair of 16-byte loads
__global__ void k_pack_atoms(const double *__restrict__ ax, const double *__restrict__ ay,
                             const double *__restrict__ az, const double *__restrict__ aw, int64_t n,
                             double4 *__restrict__ xw) {
    const int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    xw[i] = make_double4(ax[i], ay[i], az[i], aw[i]);
}

hipError_t launch_pack_atoms(const double *ax, const double *ay, const double *az, const double *aw,
                             int64_t n, double4 *xw, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_atoms, dim3(nblk(n)), dim3(kBS), 0, s, ax, ay, az, aw, n, xw);
    return hipGetLastError();
}

hipError_t launch_sort_cells(const int32_t *cell_start, int64_t ncells, double *ax, double *ay,
                             double *az, double *aw, double *ar, int32_t *aidx, hipStream_t s) {
    hipLaunchKernelGGL(k_sort_cells, dim3(nblk(ncells)), dim3(kBS), 0, s, cell_start, ncells, ax, ay,
                       az, aw, ar, aidx);
    return hipGetLastError();
}

hipError_t launch_root_count(const Grid *gt, int nconf, const int32_t *cell_start,
                             const double4 *xw, int64_t nroots, int32_t *cnt, hipStream_t s) {
    if (nroots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_root_lists<false>, dim3(nblk(nroots)), dim3(kBS), 0, s, gt, nconf,
                       cell_start, xw, nroots, nullptr, cnt);
    return hipGetLastError();
}

hipError_t launch_root_fill(const Grid *gt, int nconf, const int32_t *cell_start,
                            const double4 *xw, int64_t nroots, const int32_t *start,
                            int32_t *atoms, hipStream_t s) {
    if (nroots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_root_lists<true>, dim3(nblk(nroots)), dim3(kBS), 0, s, gt, nconf,
                       cell_start, xw, nroots, start, atoms);
    return hipGetLastError();
}

}  // namespace tms
