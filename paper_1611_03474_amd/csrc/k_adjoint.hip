// Adjoint of the corner values and edge points of a pass with respect to the
// atom centres and radii.  gfx950.
//
// Differentiating eq. Gaussian1: a term exp(-D(|p - x_i|^2 - r_i^2)) moves by
// 2D (p - x_i) term under x_i and by 2D r_i term under r_i.  An edge point
// t = (c - phi0) / (phi1 - phi0) (eq. intersection) moves by (t - 1)/delta
// under phi0 and by -t/delta under phi1, delta = phi1 - phi0.  The discrete
// structure (leaves, masks, edges) is held fixed and the cut-off radius is a
// truncation level, not a model parameter, so it is held fixed as well.
//
// Two kernels:
//  * k_adjoint_fold: one thread per unique corner.  Its weight is the
//    caller's dL/dphi plus, for every crossing edge that ends at the corner
//    (found in the edge bitmaps of the extraction by the corner's lattice
//    coordinates: at most levels x 3 axes x 2 directions), dL/dt times the
//    derivative of t.  A gather in a fixed order: no atomics, deterministic.
//  * k_adjoint_atoms: one wavefront per atom (atoms in cell order).  The
//    corners sit in the dense corner bitmap in 4x4x4-block order, so the
//    corners of a column of blocks along z are one contiguous index range;
//    the wave walks the block columns within R_c of the atom and its lanes
//    stride each range, recomputing every (atom, corner) term instead of
//    storing per-pair values.  Wave reduction, one store per atom.
#include "tms_device.h"

namespace tms {

namespace {

constexpr int kBS = 256;
constexpr int kWavesPerBlock = kBS / 64;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

__global__ __launch_bounds__(kBS) void k_adjoint_fold(
    Grid g, Lat lat, const uint64_t *__restrict__ cbm, const int32_t *__restrict__ coff,
    const double *__restrict__ upts, const double *__restrict__ uphi, int64_t m,
    const double *__restrict__ dphi, EdgeLat el, const uint64_t *__restrict__ ebm,
    const int32_t *__restrict__ eoff, const double *__restrict__ dt, double *__restrict__ wbar,
    unsigned *__restrict__ bad) {
    const int64_t k = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (k >= m) return;
    double w = dphi ? dphi[k] : 0.0;
    if (dt) {
        // corners are lattice points: p = o + X hmin exactly
        int64_t X[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) X[a] = (int64_t)rint((upts[3 * k + a] - g.o[a]) / g.hmin);
        const double f = uphi[k];
        for (int lev = 0; lev <= g.K; ++lev) {
            const int sh = g.K - lev;
            const int64_t msk = (1ll << sh) - 1;
            if ((X[0] | X[1] | X[2]) & msk) continue;  // not a point of this level's lattice
            for (int axis = 0; axis < 3; ++axis) {
                const Lat &l = el.l[lev][axis];
                for (int dir = 0; dir < 2; ++dir) {
                    // dir 0: the corner is the lower end of the edge; 1: the upper end
                    int64_t E[3] = {X[0] >> sh, X[1] >> sh, X[2] >> sh};
                    E[axis] -= dir;
                    if (E[axis] < 0 || E[axis] + 1 >= l.n[axis]) continue;
                    const int64_t b = (l.base << 6) + (E[0] * l.n[1] + E[1]) * l.n[2] + E[2];
                    if (!bit_test(ebm, b)) continue;
                    const double d = dt[bit_rank(ebm, eoff, b)];
                    int64_t Y[3] = {X[0], X[1], X[2]};
                    Y[axis] += dir ? -(1ll << sh) : (1ll << sh);
                    const int64_t cb = lat_bit(lat, Y[0], Y[1], Y[2]);
                    if (!bit_test(cbm, cb)) {
                        // the edge's other end is not a kept corner: the
                        // extraction was not made from the kept leaves
                        atomicOr(bad, 1u);
                        continue;
                    }
                    const double fo = uphi[bit_rank(cbm, coff, cb)];
                    const double f0 = dir ? fo : f, f1 = dir ? f : fo;
                    const double delta = f1 - f0;
                    const double t = (g.c - f0) / delta;
                    w += dir ? d * (-t) / delta : d * (t - 1.0) / delta;
                }
            }
        }
    }
    wbar[k] = w;
}

template <bool FAST>
__global__ __launch_bounds__(kBS) void k_adjoint_atoms(
    Grid g, Lat lat, const uint64_t *__restrict__ cbm, const int32_t *__restrict__ coff,
    const double *__restrict__ upts, const double *__restrict__ wbar, int64_t n,
    const double *__restrict__ ax, const double *__restrict__ ay, const double *__restrict__ az,
    const double *__restrict__ aw, const double *__restrict__ ar,
    const int32_t *__restrict__ aidx, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x * (int64_t)kWavesPerBlock + (threadIdx.x >> 6);
    if (i >= n) return;  // uniform per wave
    const double x[3] = {ax[i], ay[i], az[i]};
    const double wi = aw[i], D = g.D, rc2 = g.rc2;
    const double T = 4.0 * g.hmin, R = sqrt(rc2);
    int64_t t0[3], t1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        t0[a] = max((int64_t)floor((x[a] - R - g.o[a]) / T), (int64_t)0);
        t1[a] = min((int64_t)floor((x[a] + R - g.o[a]) / T), lat.n[a] - 1);
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (t0[2] <= t1[2]) {
        for (int64_t tx = t0[0]; tx <= t1[0]; ++tx) {
            const double lx = g.o[0] + (double)tx * T;
            const double dx = fmax(fmax(lx - x[0], x[0] - (lx + T)), 0.0);
            for (int64_t ty = t0[1]; ty <= t1[1]; ++ty) {
                const double ly = g.o[1] + (double)ty * T;
                const double dy = fmax(fmax(ly - x[1], x[1] - (ly + T)), 0.0);
                if (dx * dx + dy * dy > rc2) continue;
                const int64_t w0 = lat.base + (tx * lat.n[1] + ty) * lat.n[2] + t0[2];
                const int64_t w1 = w0 + (t1[2] - t0[2]);
                const int64_t kb = coff[w0];
                const int64_t ke = (int64_t)coff[w1] + __popcll(cbm[w1]);
                for (int64_t k = kb + lane; k < ke; k += 64) {
                    const double wb = wbar[k];
                    const double px = upts[3 * k] - x[0], py = upts[3 * k + 1] - x[1],
                                 pz = upts[3 * k + 2] - x[2];
                    const double d2 = px * px + py * py + pz * pz;
                    if (d2 > rc2 || wb == 0.0) continue;
                    const double f = wb * wi * expn<FAST>(-D * d2);
                    acc[0] += f * px;
                    acc[1] += f * py;
                    acc[2] += f * pz;
                    acc[3] += f;
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) acc[a] += __shfl_xor(acc[a], d, 64);
    if (lane == 0) {
        const int64_t j = aidx[i];
        const double s = 2.0 * D;
        out[4 * j] = s * acc[0];
        out[4 * j + 1] = s * acc[1];
        out[4 * j + 2] = s * acc[2];
        out[4 * j + 3] = s * ar[i] * acc[3];
    }
}

}  // namespace

hipError_t launch_adjoint_fold(const Grid &g, const Lat &lat, const uint64_t *cbm,
                               const int32_t *coff, const double *upts, const double *uphi,
                               int64_t m, const double *dphi, const EdgeLat &el,
                               const uint64_t *ebm, const int32_t *eoff, const double *dt,
                               double *wbar, unsigned *bad, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_fold, dim3(nblk(m)), dim3(kBS), 0, s, g, lat, cbm, coff, upts,
                       uphi, m, dphi, el, ebm, eoff, dt, wbar, bad);
    return hipGetLastError();
}

hipError_t launch_adjoint_atoms(const Grid &g, int precision, const Lat &lat, const uint64_t *cbm,
                                const int32_t *coff, const double *upts, const double *wbar,
                                int64_t n, const double *ax, const double *ay, const double *az,
                                const double *aw, const double *ar, const int32_t *aidx,
                                double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock);
    if (precision == TMS_PREC_FP32_GUARD)
        hipLaunchKernelGGL(k_adjoint_atoms<true>, dim3(nb), dim3(kBS), 0, s, g, lat, cbm, coff,
                           upts, wbar, n, ax, ay, az, aw, ar, aidx, out);
    else
        hipLaunchKernelGGL(k_adjoint_atoms<false>, dim3(nb), dim3(kBS), 0, s, g, lat, cbm, coff,
                           upts, wbar, n, ax, ay, az, aw, ar, aidx, out);
    return hipGetLastError();
}

}  // namespace tms
