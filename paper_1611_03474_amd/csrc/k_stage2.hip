// Stage-two points of the trilinear surface g = c on SURFACE leaves (Section
// 2.3): fold segments along each axis (eq. fold1) with their ends, the
// extreme points on the faces (eq. curve), and critical points (eq.
// critical).  One thread per leaf, double precision.  gfx950.
//
// On a leaf mapped to [-1,1]^3, g (eq. linear1) is
//   g = sum_e m_e prod_{i in e} x_i   over the subsets e of {x, y, z}
// (bit 0 x, bit 1 y, bit 2 z).  Along axis a, dg/da does not depend on x_a;
// where it vanishes, g does not depend on x_a either, so the fold set along a
// is a set of full segments parallel to a, over the points (u, v) of the two
// other axes that solve
//   dg/da(u, v) = 0  and  g(x_a = 0, u, v) = c,
// two bilinear equations.  Writing both as alpha(v) + beta(v) u and
// eliminating u leaves a quadratic in v.  The segment's ends are the extreme
// points on the faces x_a = -1 and +1.  A critical point of the pair (a, b)
// (third axis w) solves dg/da = dg/db = 0 and g = c; at fixed x_w the slice is
// k + P x_a + Q x_b + S x_a x_b, its stationary point is x_a = -Q/S,
// x_b = -P/S, where g = k - PQ/S; g = c there is a quadratic in x_w.
#include "tms_device.h"

namespace tms {

namespace {

constexpr int kBS = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

// Where a leaf's records go: the record slots of the leaf and the map from
// local coordinates u in [-1,1] to lo + (u + 1) h / 2.
struct S2Sink {
    tms_s2point *out;
    double lo[3], half;
    int32_t leaf;
    __device__ __forceinline__ void put(int k, double x, double y, double z, int kind, int axis,
                                        int root) const {
        tms_s2point r;
        r.leaf = leaf;
        r.kind = (uint8_t)kind;
        r.axis = (uint8_t)axis;
        r.root = (uint8_t)root;
        r.pad = 0;
        r.x = lo[0] + (x + 1.0) * half;
        r.y = lo[1] + (y + 1.0) * half;
        r.z = lo[2] + (z + 1.0) * half;
        out[k] = r;
    }
};

// Real roots of c0 + c1 t + c2 t^2, ascending; -1 when every coefficient is
// zero.
__device__ __forceinline__ int real_roots(double c0, double c1, double c2, double t[2]) {
    if (c2 == 0.0) {
        if (c1 == 0.0) return c0 == 0.0 ? -1 : 0;
        t[0] = -c0 / c1;
        return 1;
    }
    const double d = c1 * c1 - 4.0 * c2 * c0;
    if (d < 0.0) return 0;
    if (d == 0.0) {
        t[0] = -c1 / (2.0 * c2);
        return 1;
    }
    // the larger-magnitude root from the formula without cancellation, the
    // other from the product of the roots
    const double s = sqrt(d);
    const double big = (c1 >= 0.0) ? (-c1 - s) / (2.0 * c2) : (-c1 + s) / (2.0 * c2);
    const double small = (big != 0.0) ? c0 / (c2 * big) : big;
    t[0] = fmin(big, small);
    t[1] = fmax(big, small);
    return 2;
}

__device__ __forceinline__ bool in_unit(double x) { return x >= -1.0 && x <= 1.0; }

// whether p0 + p1 t and q0 + q1 t have a common real zero
__device__ __forceinline__ bool common_zero2(double p0, double p1, double q0, double q1) {
    if (p1 == 0.0 && q1 == 0.0) return p0 == 0.0 && q0 == 0.0;
    return p0 * q1 - p1 * q0 == 0.0;
}

// Every stage-two point of one leaf in local coordinates; returns the count
// (<= 12) and adds the number of degenerate (kind, axis) configurations to
// *ndeg.  EMIT = false only counts.
template <bool EMIT>
__device__ int leaf_points(const double f[8], double c, const S2Sink &sink, int *ndeg) {
    // monomial coefficients by a Walsh-Hadamard butterfly over the corner
    // index bits; index v's bit i set <-> factor x_i
    double m[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) m[v] = f[v];
#pragma unroll
    for (int b = 1; b < 8; b <<= 1) {
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (!(v & b)) {
                const double lo = m[v], hi = m[v | b];
                m[v] = lo + hi;
                m[v | b] = hi - lo;
            }
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) m[v] *= 0.125;
    const double m0 = m[0] - c;

    int n = 0;
    // fold segments along axis a; (u, v) the other axes, u the lower one
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int U = (a == 0) ? 2 : 1, V = (a == 2) ? 2 : 4;  // bits of u and v
        const int A = 1 << a;
        // dg/da = h0 + hu u + hv v + huv u v: exactly zero iff every edge
        // difference along a is (the butterfly subtracts equal operands)
        const double h0 = m[A], hu = m[A | U], hv = m[A | V], huv = m[A | U | V];
        if (h0 == 0.0 && hu == 0.0 && hv == 0.0 && huv == 0.0) {
            ++*ndeg;
            continue;
        }
        // g(x_a = 0) - c = g0 + gu u + gv v + guv u v
        const double g0 = m0, gu = m[U], gv = m[V], guv = m[U | V];
        // both as alpha(v) + beta(v) u; the resultant in u, a quadratic in v
        const double r0 = g0 * hu - gu * h0;
        const double r1 = g0 * huv + gv * hu - gu * hv - guv * h0;
        const double r2 = gv * huv - guv * hv;
        double t[2];
        const int nr = real_roots(r0, r1, r2, t);
        if (nr < 0) {
            // identically zero: if neither equation involves u they are
            // linear in v and either share a zero (a line along u) or have
            // no common solution; otherwise they share a factor (a curve)
            const bool free_u = gu == 0.0 && guv == 0.0 && hu == 0.0 && huv == 0.0;
            if (!free_u || common_zero2(g0, gv, h0, hv)) ++*ndeg;
            continue;
        }
        // a root where both equations vanish for every u: a line of solutions
        bool deg = false;
        for (int i = 0; i < nr; ++i) {
            const double v = t[i];
            if (gu + guv * v == 0.0 && hu + huv * v == 0.0 && g0 + gv * v == 0.0 &&
                h0 + hv * v == 0.0)
                deg = true;
        }
        if (deg) {
            ++*ndeg;
            continue;
        }
        double su[2], sv[2];
        int ns = 0;
        for (int i = 0; i < nr; ++i) {
            const double v = t[i];
            if (!in_unit(v)) continue;
            const double aG = g0 + gv * v, bG = gu + guv * v;
            const double aH = h0 + hv * v, bH = hu + huv * v;
            const double bmag = fmax(fabs(bG), fabs(bH));
            if (bmag == 0.0) continue;  // no u solves both
            const double u = (fabs(bG) >= fabs(bH)) ? -aG / bG : -aH / bH;
            if (!in_unit(u)) continue;
            su[ns] = u;
            sv[ns] = v;
            ++ns;
        }
        if (ns == 2 && su[1] < su[0]) {
            const double tu = su[0], tv = sv[0];
            su[0] = su[1];
            sv[0] = sv[1];
            su[1] = tu;
            sv[1] = tv;
        }
        for (int k = 0; k < ns; ++k) {
            if (EMIT) {
                // the end on the face x_a = -1
                double x[3];
                x[a] = -1.0;
                x[(a == 0) ? 1 : 0] = su[k];
                x[(a == 2) ? 1 : 2] = sv[k];
                sink.put(n, x[0], x[1], x[2], TMS_S2_FOLD, a, k);
            }
            ++n;
        }
    }
    // critical points of the pair of axes other than w
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        const int ia = (w == 0) ? 1 : 0, ib = (w == 2) ? 1 : 2;
        const int A = 1 << ia, B = 1 << ib, W = 1 << w;
        // k, P, Q, S of the slice at x_w, each linear in x_w
        const double k0 = m0, k1 = m[W];
        const double P0 = m[A], P1 = m[A | W];
        const double Q0 = m[B], Q1 = m[B | W];
        const double S0 = m[A | B], S1 = m[A | B | W];
        // (k - c) S - P Q as a polynomial in x_w
        const double w0 = k0 * S0 - P0 * Q0;
        const double w1 = (k0 * S1 - P0 * Q1) + (k1 * S0 - P1 * Q0);
        const double w2 = k1 * S1 - P1 * Q1;
        double t[2];
        const int nr = real_roots(w0, w1, w2, t);
        if (nr < 0) {
            // identically zero: with S not identically zero every slice's
            // stationary point is on the surface (a curve); with S = 0 a
            // solution needs P = Q = 0 and k = c at one x_w (a whole slice)
            bool deg = S0 != 0.0 || S1 != 0.0;
            if (!deg) {
                const double a3[3] = {P0, Q0, k0}, b3[3] = {P1, Q1, k1};
                bool rank1 = true, anyb = false, anya = false;
                for (int i = 0; i < 3; ++i) {
                    anyb |= b3[i] != 0.0;
                    anya |= a3[i] != 0.0;
                    for (int j = i + 1; j < 3; ++j)
                        if (a3[i] * b3[j] - a3[j] * b3[i] != 0.0) rank1 = false;
                }
                deg = rank1 && (anyb || !anya);
            }
            if (deg) ++*ndeg;
            continue;
        }
        bool deg = false;
        for (int i = 0; i < nr; ++i) {
            const double z = t[i];
            if (S0 + S1 * z == 0.0 && P0 + P1 * z == 0.0 && Q0 + Q1 * z == 0.0 &&
                k0 + k1 * z == 0.0)
                deg = true;  // a whole slice
        }
        if (deg) {
            ++*ndeg;
            continue;
        }
        double xs[2][3];
        int ns = 0;
        for (int i = 0; i < nr; ++i) {
            const double z = t[i];
            if (!in_unit(z)) continue;
            const double S = S0 + S1 * z, P = P0 + P1 * z, Q = Q0 + Q1 * z;
            if (S == 0.0) continue;  // no isolated stationary point on the slice
            const double xa = -Q / S, xb = -P / S;
            if (!in_unit(xa) || !in_unit(xb)) continue;
            xs[ns][ia] = xa;
            xs[ns][ib] = xb;
            xs[ns][w] = z;
            ++ns;
        }
        if (EMIT)
            for (int k = 0; k < ns; ++k)
                sink.put(n + k, xs[k][0], xs[k][1], xs[k][2], TMS_S2_CRITICAL, w, k);
        n += ns;
    }
    return n;
}

__device__ __forceinline__ bool load_leaf(const tms_leaf *__restrict__ leaves,
                                          const double *__restrict__ cphi, int64_t q,
                                          tms_leaf &L, double f[8]) {
    L = leaves[q];
    if (L.cls != TMS_CLS_SURFACE) return false;
    const double2 *c2 = reinterpret_cast<const double2 *>(cphi + 8 * q);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 v = c2[i];
        f[2 * i] = v.x;
        f[2 * i + 1] = v.y;
    }
    return true;
}

__global__ __launch_bounds__(kBS) void k_s2_count(const Grid *__restrict__ gt,
                                                  const tms_leaf *__restrict__ leaves,
                                                  const double *__restrict__ cphi, int64_t n,
                                                  int32_t *__restrict__ cnt,
                                                  unsigned long long *__restrict__ ndeg_total) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    int c = 0, nd = 0;
    if (q < n) {
        tms_leaf L;
        double f[8];
        if (load_leaf(leaves, cphi, q, L, f))
            c = leaf_points<false>(f, gt[L.conf].c, S2Sink{}, &nd);
        cnt[q] = c;
    }
    unsigned long long d = (unsigned long long)nd;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) d += __shfl_xor(d, s, 64);
    if ((threadIdx.x & 63) == 0 && d) atomicAdd(ndeg_total, d);
}

__global__ __launch_bounds__(kBS) void k_s2_emit(const Grid *__restrict__ gt,
                                                 const tms_leaf *__restrict__ leaves,
                                                 const double *__restrict__ cphi, int64_t n,
                                                 const int32_t *__restrict__ off,
                                                 tms_s2point *__restrict__ out, int64_t leaf0) {
    const int64_t q = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (q >= n) return;
    tms_leaf L;
    double f[8];
    if (!load_leaf(leaves, cphi, q, L, f)) return;
    const Grid &g = gt[L.conf];
    const double h = g.h0 / (double)(1 << L.level);
    S2Sink sink;
    sink.out = out + off[q];
    sink.lo[0] = g.o[0] + (double)L.ix * h;
    sink.lo[1] = g.o[1] + (double)L.iy * h;
    sink.lo[2] = g.o[2] + (double)L.iz * h;
    sink.half = 0.5 * h;
    sink.leaf = (int32_t)(leaf0 + q);
    int nd = 0;
    (void)leaf_points<true>(f, g.c, sink, &nd);
}

}  // namespace

hipError_t launch_s2_count(const Grid *gt, const tms_leaf *leaves, const double *cphi, int64_t n,
                           int32_t *cnt, unsigned long long *ndeg, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_s2_count, dim3(nblk(n)), dim3(kBS), 0, s, gt, leaves, cphi, n, cnt, ndeg);
    return hipGetLastError();
}

hipError_t launch_s2_emit(const Grid *gt, const tms_leaf *leaves, const double *cphi, int64_t n,
                          const int32_t *off, tms_s2point *out, int64_t leaf0, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_s2_emit, dim3(nblk(n)), dim3(kBS), 0, s, gt, leaves, cphi, n, off, out,
                       leaf0);
    return hipGetLastError();
}

}  // namespace tms
