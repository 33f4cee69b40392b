// Adaptive partition and estimation kernels (Section 2.2, Steps 1-3) for
// gfx950.
//
//   roots      Q_0: root cubes with a non-empty neighbourhood, raster order
//   estimate   per cube: A = sum_i w_i a~x (x) a~y (x) a~z over the atoms within
//              R_c of the cube (eqs. polynew, tensor1, tensor2), plus the l1
//              scale S = sum_i w_i |a~x|_1 |a~y|_1 |a~z|_1 that sizes the
//              single-precision error band
//   decide     per cube: Step 3's stopping rule (2E <= tau, children only),
//              else Step 2's bound test L <= c <= U, then leaf / divide
//   compaction stable: leaves in queue order, children of a divided cube in
//              octant order at their parent's position
#include "tms_device.h"

namespace tms {

namespace {

constexpr int kBS = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

__global__ void k_roots_flags(const int32_t *__restrict__ rs, int64_t nroots, int32_t *__restrict__ f) {
    int64_t r = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (r < nroots) f[r] = (rs[r + 1] > rs[r]) ? 1 : 0;
}

__global__ void k_roots_emit(Grid g, const int32_t *__restrict__ f, const int32_t *__restrict__ off,
                             int64_t nroots, int4 *__restrict__ q) {
    int64_t r = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (r >= nroots || !f[r]) return;
    int rx = (int)(r % g.nr[0]), ry = (int)((r / g.nr[0]) % g.nr[1]),
        rz = (int)(r / ((int64_t)g.nr[0] * g.nr[1]));
    q[off[r]] = make_int4(rx, ry, rz, 0);
}

// wavefront sum of a 64-bit counter, one atomic per wavefront
__device__ __forceinline__ void wave_add(unsigned long long *ctr, unsigned long long v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(ctr, v);
}

// One thread per cube.  The thread walks its root's neighbourhood list (all
// threads of a wavefront usually share a root, so the list loads are
// uniform), keeps the atoms within R_c of its own cube, projects the three
// Gaussian factors and accumulates the 4x4x4 rank-one update in double
// precision.  With FAST exponentials it also accumulates the l1 error bound
// E of the tensor: a perturbation da of a factor moves w a (x) b (x) c by at
// most w (|da| |b| |c| + |a| |db| |c| + |a| |b| |dc|) in l1.
template <bool FAST, int QH>
__global__ __launch_bounds__(kBS) void k_estimate(
    Grid g, int level, GLRule<double> R, const int4 *__restrict__ q, int64_t n,
    const int32_t *__restrict__ subset, const int32_t *__restrict__ root_start,
    const int32_t *__restrict__ root_atoms, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ az, const double *__restrict__ aw,
    double *__restrict__ Aout, double *__restrict__ Eout, unsigned long long *__restrict__ pairs) {
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    unsigned long long np = 0;
    if (t < n) {
        int64_t qi = subset ? subset[t] : t;
        int4 c = q[qi];
        const double h = ldexp(g.h0, -level);
        const double lo[3] = {g.o[0] + c.x * h, g.o[1] + c.y * h, g.o[2] + c.z * h};
        const double hi[3] = {lo[0] + h, lo[1] + h, lo[2] + h};
        const double mid[3] = {lo[0] + 0.5 * h, lo[1] + 0.5 * h, lo[2] + 0.5 * h};
        const double s = 0.5 * h;
        const int64_t root =
            ((int64_t)(c.z >> level) * g.nr[1] + (c.y >> level)) * g.nr[0] + (c.x >> level);
        double A[64];
#pragma unroll
        for (int e = 0; e < 64; ++e) A[e] = 0.0;
        double EA = 0.0;
        const int b = root_start[root], e_ = root_start[root + 1];
        for (int p = b; p < e_; ++p) {
            const int i = root_atoms[p];
            const double x = ax[i], y = ay[i], z = az[i];
            const double dx = fmax(fmax(lo[0] - x, x - hi[0]), 0.0);
            const double dy = fmax(fmax(lo[1] - y, y - hi[1]), 0.0);
            const double dz = fmax(fmax(lo[2] - z, z - hi[2]), 0.0);
            if (dx * dx + dy * dy + dz * dz > g.rc2) continue;
            ++np;
            double px[4], py[4], pz[4], ex, ey, ez;
            project<FAST, QH>(R, g.D, s, mid[0] - x, px, ex);
            project<FAST, QH>(R, g.D, s, mid[1] - y, py, ey);
            project<FAST, QH>(R, g.D, s, mid[2] - z, pz, ez);
            const double w = aw[i];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double wx = w * px[j];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double wxy = wx * py[k];
#pragma unroll
                    for (int l = 0; l < 4; ++l) A[16 * j + 4 * k + l] += wxy * pz[l];
                }
            }
            if (FAST) {
                const double nx = fabs(px[0]) + fabs(px[1]) + fabs(px[2]) + fabs(px[3]);
                const double ny = fabs(py[0]) + fabs(py[1]) + fabs(py[2]) + fabs(py[3]);
                const double nz = fabs(pz[0]) + fabs(pz[1]) + fabs(pz[2]) + fabs(pz[3]);
                EA += w * ((ex * ny + nx * ey) * nz + nx * ny * ez);
            }
        }
        double *dst = Aout + 64 * qi;
#pragma unroll
        for (int e = 0; e < 64; ++e) dst[e] = A[e];
        Eout[qi] = EA;
    }
    if (pairs) wave_add(pairs, np);
}

// Safety factor on the first-order perturbation estimate band * amp of the
// bound (measured deviations of single-precision bounds stay below
// 0.25 band * amp; see the calibration notes in the design document).
constexpr double kKappa = 8.0;

// Per-cube decision in double precision.  For tensors built with FAST
// exponentials, decisions whose margin lies within the tensor's error band
// (amplified for the bound by the first-order factor amp) become DEC_GUARD
// and are redone with exact exponentials.
__global__ __launch_bounds__(kBS) void k_decide(Grid g, int level, int fast,
                                                const double *__restrict__ Ain,
                                                const double *__restrict__ Ein, int64_t n,
                                                const int32_t *__restrict__ subset,
                                                uint8_t *__restrict__ dec,
                                                unsigned long long *__restrict__ nbound) {
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    unsigned long long nb = 0;
    if (t < n) {
        const int64_t qi = subset ? subset[t] : t;
        double A[64];
        const double *src = Ain + 64 * qi;
#pragma unroll
        for (int e = 0; e < 64; ++e) A[e] = src[e];
        double E = 0.0, asum = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const double v = fabs(A[16 * j + 4 * k + l]);
                    asum += v;
                    if (j >= 2 || k >= 2 || l >= 2) E += v;
                }
        // l1 error band of A: the accumulated bound of the FAST exponentials
        // plus a floor for double-precision rounding; zero for exact
        // exponentials (no guard)
        const double band = fast ? Ein[qi] + 1e-13 * asum : 0.0;
        uint8_t d = 255;
        if (level >= 1) {
            // Step 3: higher-order mass under the user bound -> trilinear leaf
            if (band > 0.0 && fabs(2.0 * E - g.tau) <= 2.0 * band) d = DEC_GUARD;
            else if (2.0 * E <= g.tau) d = DEC_CONV;
        }
        if (d == 255) {
            bool keep;
            // any two sampled values of P on either side of c imply
            // L <= c <= U for every valid enclosure [L, U] of P
            double slo, shi;
            sample_range(A, slo, shi);
            const double tiny = 1e-12 * asum + band;
            if (slo <= g.c - tiny && shi >= g.c + tiny) {
                keep = true;
            } else {
                ++nb;
                BoundResult B = nested_bound(A, band);
                if (band > 0.0 && (B.jump || fabs(B.L - g.c) <= kKappa * band * B.amp ||
                                   fabs(B.U - g.c) <= kKappa * band * B.amp)) {
                    d = DEC_GUARD;
                }
                keep = (B.L <= g.c && g.c <= B.U);  // Step 2
            }
            if (d == 255) d = keep ? ((level == g.K) ? DEC_HMIN : DEC_REFINE) : DEC_DISCARD;
        }
        dec[qi] = d;
    }
    if (nbound) wave_add(nbound, nb);
}

__global__ void k_guard_flags(const uint8_t *__restrict__ dec, int64_t n, int32_t *__restrict__ f) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n) f[i] = dec[i] == DEC_GUARD;
}

__global__ void k_list_emit(const int32_t *__restrict__ f, const int32_t *__restrict__ off,
                            int64_t n, int32_t *__restrict__ list) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n && f[i]) list[off[i]] = (int32_t)i;
}

__global__ void k_level_counts(const uint8_t *__restrict__ dec, int64_t n, int32_t *__restrict__ lc,
                               int32_t *__restrict__ cc) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    const uint8_t d = dec[i];
    lc[i] = (d == DEC_CONV || d == DEC_HMIN) ? 1 : 0;
    cc[i] = (d == DEC_REFINE) ? 8 : 0;
}

__global__ void k_level_emit(const int4 *__restrict__ q, const uint8_t *__restrict__ dec, int64_t n,
                             int level, const int32_t *__restrict__ loff,
                             const int32_t *__restrict__ coff, tms_leaf *__restrict__ leaves,
                             int64_t leaf_base, int4 *__restrict__ qn) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    const uint8_t d = dec[i];
    const int4 c = q[i];
    if (d == DEC_CONV || d == DEC_HMIN) {
        tms_leaf L;
        L.ix = c.x;
        L.iy = c.y;
        L.iz = c.z;
        L.conf = c.w;
        L.level = (uint8_t)level;
        L.reason = (d == DEC_CONV) ? TMS_REASON_CONVERGED : TMS_REASON_HMIN;
        L.mask = 0;
        L.cls = 0;
        leaves[leaf_base + loff[i]] = L;
    } else if (d == DEC_REFINE) {
        int4 *o = qn + coff[i];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            o[k] = make_int4(2 * c.x + (k & 1), 2 * c.y + ((k >> 1) & 1), 2 * c.z + ((k >> 2) & 1), c.w);
    }
}

__global__ void k_level_histo(const uint8_t *__restrict__ dec, int64_t n,
                              unsigned long long *__restrict__ h) {
    __shared__ unsigned long long sh[5];
    if (threadIdx.x < 5) sh[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n && dec[i] < 5) atomicAdd(&sh[dec[i]], 1ull);
    __syncthreads();
    if (threadIdx.x < 5 && sh[threadIdx.x]) atomicAdd(&h[threadIdx.x], sh[threadIdx.x]);
}

__global__ __launch_bounds__(kBS) void k_bound_debug(const double *__restrict__ Ain,
                                                     const double *__restrict__ band, int64_t n,
                                                     double *__restrict__ out) {
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t >= n) return;
    double A[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) A[e] = Ain[64 * t + e];
    BoundResult B = nested_bound(A, band ? band[t] : 0.0);
    out[6 * t + 0] = B.L;
    out[6 * t + 1] = B.U;
    out[6 * t + 2] = B.rho;
    out[6 * t + 3] = (double)B.r;
    out[6 * t + 4] = B.jump ? 1.0 : 0.0;
    out[6 * t + 5] = B.amp;
}

__global__ void k_fast_exp_debug(const double *__restrict__ x, int64_t n, double *__restrict__ y) {
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t < n) y[t] = expn<true>(x[t]);
}

template <bool FAST, int QH>
hipError_t estimate_t(const Grid &g, int level, const int4 *q, int64_t n, const int32_t *subset,
                      const int32_t *rs, const int32_t *ra, const double *ax, const double *ay,
                      const double *az, const double *aw, double *A, double *E,
                      unsigned long long *pairs, hipStream_t s) {
    GLRule<double> R = gl_rule<double>(QH);
    hipLaunchKernelGGL((k_estimate<FAST, QH>), dim3(nblk(n)), dim3(kBS), 0, s, g, level, R, q, n,
                       subset, rs, ra, ax, ay, az, aw, A, E, pairs);
    return hipGetLastError();
}

template <bool FAST>
hipError_t estimate_dispatch(int qh, const Grid &g, int level, const int4 *q, int64_t n,
                             const int32_t *subset, const int32_t *rs, const int32_t *ra,
                             const double *ax, const double *ay, const double *az, const double *aw,
                             double *A, double *E, unsigned long long *pairs, hipStream_t s) {
    switch (qh) {
    case 4: return estimate_t<FAST, 4>(g, level, q, n, subset, rs, ra, ax, ay, az, aw, A, E, pairs, s);
    case 5: return estimate_t<FAST, 5>(g, level, q, n, subset, rs, ra, ax, ay, az, aw, A, E, pairs, s);
    case 6: return estimate_t<FAST, 6>(g, level, q, n, subset, rs, ra, ax, ay, az, aw, A, E, pairs, s);
    case 8: return estimate_t<FAST, 8>(g, level, q, n, subset, rs, ra, ax, ay, az, aw, A, E, pairs, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// Gauss-Legendre rules, computed once on the host by Newton's method on the
// Legendre recurrence, then folded into the even/odd coefficient form.
template <typename T>
GLRule<T> gl_rule(int half) {
    static bool ready[9] = {false};
    static GLRule<double> cache[9];
    if (!ready[half]) {
        const int n = 2 * half;
        GLRule<double> r{};
        for (int q = 0; q < half; ++q) {
            // q-th positive root of P_n (largest first): Tricomi's estimate
            long double th = 3.14159265358979323846L * (4.0L * (q + 1) - 1.0L) / (4.0L * n + 2.0L);
            long double x = (1.0L - (n - 1.0L) / (8.0L * n * n * n)) * cosl(th);
            long double dp = 1.0L;
            for (int it = 0; it < 50; ++it) {
                long double p0 = 1.0L, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (p0 - x * p1) / (1.0L - x * x);
                long double dx = p1 / dp;
                x -= dx;
                if (fabsl(dx) < 1e-19L) break;
            }
            long double p0 = 1.0L, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (p0 - x * p1) / (1.0L - x * x);
            long double wq = 2.0L / ((1.0L - x * x) * dp * dp);
            long double L2 = 1.5L * x * x - 0.5L, L3 = x * (2.5L * x * x - 1.5L);
            r.t[q] = (double)x;
            r.c0[q] = (double)(0.5L * wq);
            r.c1[q] = (double)(1.5L * wq * x);
            r.c2[q] = (double)(2.5L * wq * L2);
            r.c3[q] = (double)(3.5L * wq * L3);
            r.cs[q] = fabs(r.c0[q]) + fabs(r.c1[q]) + fabs(r.c2[q]) + fabs(r.c3[q]);
        }
        cache[half] = r;
        ready[half] = true;
    }
    GLRule<T> o{};
    for (int q = 0; q < 8; ++q) {
        o.t[q] = (T)cache[half].t[q];
        o.c0[q] = (T)cache[half].c0[q];
        o.c1[q] = (T)cache[half].c1[q];
        o.c2[q] = (T)cache[half].c2[q];
        o.c3[q] = (T)cache[half].c3[q];
        o.cs[q] = (T)cache[half].cs[q];
    }
    return o;
}
template GLRule<double> gl_rule<double>(int);

// beta = s sqrt(D): quadrature error of the projection below 2e-15
// (measured against 40-digit quadrature over |d| <= 7).  Both exponential
// policies use the same rule, so they differ only by exponential rounding.
int gl_half_nodes(double beta, bool fast) {
    (void)fast;
    if (beta <= 0.25) return 4;
    if (beta <= 0.5) return 5;
    if (beta <= 0.75) return 6;
    if (beta <= 1.25) return 8;
    return -1;
}

hipError_t launch_roots_flags(const int32_t *root_start, int64_t nroots, int32_t *flags,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_roots_flags, dim3(nblk(nroots)), dim3(kBS), 0, s, root_start, nroots, flags);
    return hipGetLastError();
}

hipError_t launch_roots_emit(const Grid &g, const int32_t *flags, const int32_t *off, int64_t nroots,
                             int4 *q, hipStream_t s) {
    hipLaunchKernelGGL(k_roots_emit, dim3(nblk(nroots)), dim3(kBS), 0, s, g, flags, off, nroots, q);
    return hipGetLastError();
}

hipError_t launch_estimate(const Grid &g, int level, int precision, const int4 *q, int64_t n,
                           const int32_t *subset, const int32_t *root_start,
                           const int32_t *root_atoms, const double *ax, const double *ay,
                           const double *az, const double *aw, double *A, double *S,
                           int64_t *pairs, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const double beta = 0.5 * ldexp(g.h0, -level) * sqrt(g.D);
    const bool fast = precision == TMS_PREC_FP32_GUARD;
    const int qh = gl_half_nodes(beta, fast);
    auto *pc = reinterpret_cast<unsigned long long *>(pairs);
    if (fast)
        return estimate_dispatch<true>(qh, g, level, q, n, subset, root_start, root_atoms, ax, ay,
                                       az, aw, A, S, pc, s);
    return estimate_dispatch<false>(qh, g, level, q, n, subset, root_start, root_atoms, ax, ay, az,
                                    aw, A, S, pc, s);
}

hipError_t launch_decide(const Grid &g, int level, int precision, const double *A, const double *S,
                         int64_t n, const int32_t *subset, uint8_t *dec, int32_t *nbound,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int fast = (precision == TMS_PREC_FP32_GUARD) ? 1 : 0;
    hipLaunchKernelGGL(k_decide, dim3(nblk(n)), dim3(kBS), 0, s, g, level, fast, A, S, n, subset,
                       dec, reinterpret_cast<unsigned long long *>(nbound));
    return hipGetLastError();
}

hipError_t launch_guard_list_flags(const uint8_t *dec, int64_t n, int32_t *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_guard_flags, dim3(nblk(n)), dim3(kBS), 0, s, dec, n, flags);
    return hipGetLastError();
}

hipError_t launch_guard_list_emit(const int32_t *flags, const int32_t *off, int64_t n, int32_t *list,
                                  hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_list_emit, dim3(nblk(n)), dim3(kBS), 0, s, flags, off, n, list);
    return hipGetLastError();
}

hipError_t launch_level_counts(const uint8_t *dec, int64_t n, int32_t *lc, int32_t *cc,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_counts, dim3(nblk(n)), dim3(kBS), 0, s, dec, n, lc, cc);
    return hipGetLastError();
}

hipError_t launch_level_emit(const int4 *q, const uint8_t *dec, int64_t n, int level,
                             const int32_t *loff, const int32_t *coff, tms_leaf *leaves,
                             int64_t leaf_base, int4 *qn, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_emit, dim3(nblk(n)), dim3(kBS), 0, s, q, dec, n, level, loff, coff,
                       leaves, leaf_base, qn);
    return hipGetLastError();
}

hipError_t launch_level_histo(const uint8_t *dec, int64_t n, unsigned long long *h, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_histo, dim3(nblk(n)), dim3(kBS), 0, s, dec, n, h);
    return hipGetLastError();
}

hipError_t launch_fast_exp_debug(const double *x, int64_t n, double *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fast_exp_debug, dim3(nblk(n)), dim3(kBS), 0, s, x, n, y);
    return hipGetLastError();
}

hipError_t launch_bound_debug(const double *A, const double *band, int64_t n, double *out,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bound_debug, dim3(nblk(n)), dim3(kBS), 0, s, A, band, n, out);
    return hipGetLastError();
}

}  // namespace tms
