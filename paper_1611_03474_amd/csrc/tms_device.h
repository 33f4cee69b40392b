// Device-side building blocks of the partition/estimation kernels (gfx950).
//
// Notation follows Section 2.2 of Liu, Chen & Lu (arXiv:1611.03474): a cube's
// polynomial is P(x,y,z) = sum_{jkl} A[j][k][l] L_j(x) L_k(y) L_l(z) in local
// coordinates [-1,1]^3 (eq. tensor1), A = sum_i w_i a~x (x) a~y (x) a~z with
// w_i = exp(D r_i^2) and a~ the endpoint-corrected degree-3 Legendre
// projections of the one-dimensional Gaussian factors (eqs. poly2_1, poly3,
// condition1, alpha).  Flat index of A: 16 j + 4 k + l.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tms_internal.h"

namespace tms {

// ---------------------------------------------------------------------------
// Exponentials.  On gfx950 a double-precision FMA issues at the same rate as
// an (unpacked) single-precision one, so the only place where single
// precision pays is the transcendental itself.  The FAST policy evaluates
// exp(x), x <= 0, as 2^n * 2^f with n = floor(x log2 e) and f = x log2 e - n
// split in double precision, 2^f from the hardware single-precision v_exp_f32
// (f in [0,1)), and the scaling by 2^n exact.  Its relative error is the
// exp2 rounding plus the rounding of f to single precision; kFastExpErr
// bounds it (checked on the device by the test-suite).  Everything around the
// exponential stays in double precision.
// ---------------------------------------------------------------------------
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kFastExpErr = 1.5e-7;  // 1 ulp of v_exp_f32 + rounding of f

template <bool FAST>
__device__ __forceinline__ double expn(double x) {
    if constexpr (FAST) {
        const double y = x * kLog2e;
        const double n = floor(y);
        const float f = (float)(y - n);
        const float e = __builtin_amdgcn_exp2f(f);
        return ldexp((double)e, (int)fmax(n, -1070.0));
    } else {
        return exp(x);
    }
}

// ---------------------------------------------------------------------------
// Endpoint-corrected degree-3 Legendre projection of f(t) = exp(-D (s t + d)^2)
// on t in [-1,1] (x = m + s t, d = m - x_i).  a[0..3] receive the corrected
// coefficients of eq. alpha.  QH is half the number of quadrature nodes.
// With FAST exponentials, *err receives an l1 bound on the error of a[]:
// every f value carries a relative error <= eps = kFastExpErr.  The
// endpoint correction cancels the errors of the raw a2, a3 exactly:
//   da~2 = (df(1) + df(-1))/2 - da0,   da~3 = (df(1) - df(-1))/2 - da1,
// and with c0, c1 >= 0 at the positive nodes and f > 0,
//   |da0| <= eps a0,  |da1| <= eps b1,  b1 = sum_q c1_q (f(t_q) + f(-t_q)),
// so sum_j |da~_j| <= eps (2 a0 + 2 b1 + f(1) + f(-1)).
//
// deg < 3 (Section 2.2.1 with n = deg): the series stops at L_deg (higher
// coefficients 0) and the endpoint corrections go on L_{n-1} and L_n, solved
// from eq. condition1 with L_j(+-1) = (+-1)^j: for odd n, e0 = (ep + em)/2
// on L_{n-1} and e1 = (ep - em)/2 on L_n; for even n the two swap.  The same
// cancellation leaves an error of at most eps (2 a0 + f(1) + f(-1)) (n = 2)
// or eps (f(1) + f(-1)) (n = 1), below the bound above.
// ---------------------------------------------------------------------------
template <bool FAST, int QH>
__device__ __forceinline__ void project(const GLRule<double> &R, double D, double s, double d,
                                        int deg, double a[4], double &err) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, sf = 0;
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const double up = s * R.t[q] + d, um = d - s * R.t[q];
        const double fp = expn<FAST>(-D * up * up);
        const double fm = expn<FAST>(-D * um * um);
        const double ev = fp + fm, od = fp - fm;
        a0 += R.c0[q] * ev;
        a2 += R.c2[q] * ev;
        a1 += R.c1[q] * od;
        a3 += R.c3[q] * od;
        if (FAST) sf += R.c1[q] * ev;
    }
    // eq. condition1: match f at t = +-1 by adding e0 L_{n-1} + e1 L_n
    const double f1 = expn<FAST>(-D * (s + d) * (s + d));
    const double fm1 = expn<FAST>(-D * (d - s) * (d - s));
    err = FAST ? kFastExpErr * (2.0 * (a0 + sf) + f1 + fm1) : 0.0;
    // the series stops at L_deg; the even-index correction goes on L2 (on L0
    // when deg = 1), the odd one on L_deg's odd neighbour (L3 when deg = 3,
    // else L1).  Selects, not branches: with deg = 3 the operations are those
    // of the degree-3 formula
    a2 = deg >= 2 ? a2 : 0.0;
    a3 = deg >= 3 ? a3 : 0.0;
    const double ep = f1 - (a0 + a1 + a2 + a3);
    const double em = fm1 - (a0 - a1 + a2 - a3);
    const double ee = 0.5 * (ep + em), eo = 0.5 * (ep - em);
    a[0] = deg == 1 ? a0 + ee : a0;
    a[1] = deg <= 2 ? a1 + eo : a1;
    a[2] = deg >= 2 ? a2 + ee : 0.0;
    a[3] = deg >= 3 ? a3 + eo : 0.0;
}

// ---------------------------------------------------------------------------
// Range of q0 L0 + q1 L1 + q2 L2 + q3 L3 on [-1,1]: extremes over the ends and
// the interior critical points (roots of the derivative
// (15/2) q3 t^2 + 3 q2 t + (q1 - 3/2 q3)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double leg3(const double q[4], double t) {
    double t2 = t * t;
    return q[0] + q[1] * t + q[2] * (1.5 * t2 - 0.5) + q[3] * t * (2.5 * t2 - 1.5);
}

__device__ __forceinline__ void leg3_range(const double q[4], double &lo, double &hi) {
    double vp = q[0] + q[1] + q[2] + q[3];
    double vm = q[0] - q[1] + q[2] - q[3];
    lo = fmin(vp, vm);
    hi = fmax(vp, vm);
    double qa = 7.5 * q[3], qb = 3.0 * q[2], qc = q[1] - 1.5 * q[3];
    double r0 = 2.0, r1 = 2.0;  // outside [-1,1] = absent
    if (qa != 0.0) {
        double disc = qb * qb - 4.0 * qa * qc;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double h = -0.5 * (qb + copysign(sq, qb));
            if (h != 0.0) {
                r0 = h / qa;
                r1 = qc / h;
            } else {
                r0 = 0.0;
            }
        }
    } else if (qb != 0.0) {
        r0 = -qc / qb;
    }
    if (r0 >= -1.0 && r0 <= 1.0) {
        double v = leg3(q, r0);
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    if (r1 >= -1.0 && r1 <= 1.0) {
        double v = leg3(q, r1);
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
}

__device__ __forceinline__ void imul(double a0, double a1, double b0, double b1, double &lo,
                                     double &hi) {
    double p0 = a0 * b0, p1 = a0 * b1, p2 = a1 * b0, p3 = a1 * b1;
    lo = fmin(fmin(p0, p1), fmin(p2, p3));
    hi = fmax(fmax(p0, p1), fmax(p2, p3));
}

// ---------------------------------------------------------------------------
// Symmetric 4x4 eigen-decomposition by Jacobi rotations in the parallel
// (round-robin) ordering: each sweep is three rounds of two rotations on
// disjoint index pairs, (0,1)+(2,3), (0,2)+(1,3), (0,3)+(1,2).  The two
// rotations of a round commute, so both parameter sets are taken from the
// matrix before the round -- two independent dependency chains per round.
// S is overwritten (diagonal = eigenvalues); V receives eigenvectors as
// columns; lam/vec are returned sorted by descending eigenvalue.
// ---------------------------------------------------------------------------
struct JRot {
    double c, s, t;
};

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimates (about
// single-precision accurate) refined by two Newton steps each, which reach
// double precision (each step squares the relative error).
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double q = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) q = fma(q, fma(-x, q, 1.0), q);
    return q;
}

// Rotation [[c, s], [-s, c]] on (p, q) that zeroes e in [[a, e], [e, b]]:
// t = tan(angle) is the root of smaller magnitude of t^2 + 2 theta t - 1 = 0,
// theta = (b - a) / (2 e), written as sign(d) 2 e / (|d| + sqrt(d^2 + 4 e^2))
// with d = b - a; then the new diagonal is a - t e, b + t e.  c and s are
// computed from t, so the rotation is orthogonal to rounding whatever the
// last bits of t; an off-diagonal whose rotation would need an r^2 below the
// normal range (negligible against the diagonal) gets t = 0 and is dropped.
__device__ __forceinline__ JRot jrot_params(double a, double b, double e) {
    const double d = b - a, r2 = d * d + 4.0 * e * e;
    const bool on = e != 0.0 && r2 >= 2.2250738585072014e-308;
    const double r = r2 * rsq_nr(on ? r2 : 1.0);
    double t = 2.0 * e * rcp_nr(on ? fabs(d) + r : 1.0);
    t = signbit(d) ? -t : t;
    t = on ? t : 0.0;
    JRot R;
    R.t = t;
    R.c = rsq_nr(fma(t, t, 1.0));
    R.s = t * R.c;
    return R;
}

__device__ __forceinline__ void jrot_apply(double S[4][4], double V[4][4], int p, int q,
                                           const JRot &R) {
    const double e = S[p][q];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k == p || k == q) continue;
        const double g = S[k][p], h = S[k][q];
        const double np = R.c * g - R.s * h, nq = R.s * g + R.c * h;
        S[k][p] = np;
        S[p][k] = np;
        S[k][q] = nq;
        S[q][k] = nq;
    }
    S[p][p] -= R.t * e;
    S[q][q] += R.t * e;
    S[p][q] = 0.0;
    S[q][p] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double g = V[k][p], h = V[k][q];
        V[k][p] = R.c * g - R.s * h;
        V[k][q] = R.s * g + R.c * h;
    }
}

__device__ __forceinline__ void jrot_round(double S[4][4], double V[4][4], int p1, int q1, int p2,
                                           int q2) {
    const JRot A = jrot_params(S[p1][p1], S[q1][q1], S[p1][q1]);
    const JRot B = jrot_params(S[p2][p2], S[q2][q2], S[p2][q2]);
    jrot_apply(S, V, p1, q1, A);
    jrot_apply(S, V, p2, q2, B);
}

__device__ __forceinline__ void eig4_sorted(double S[4][4], double lam[4], double V[4][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[0][3] * S[0][3] +
                     S[1][2] * S[1][2] + S[1][3] * S[1][3] + S[2][3] * S[2][3];
        double dg = S[0][0] * S[0][0] + S[1][1] * S[1][1] + S[2][2] * S[2][2] + S[3][3] * S[3][3];
        if (off <= 1e-34 * dg || off == 0.0) break;
        jrot_round(S, V, 0, 1, 2, 3);
        jrot_round(S, V, 0, 2, 1, 3);
        jrot_round(S, V, 0, 3, 1, 2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) lam[i] = S[i][i];
    // sorting network on (lam, V columns), descending
    auto cx = [&](int a, int b) {
        if (lam[b] > lam[a]) {
            double t = lam[a];
            lam[a] = lam[b];
            lam[b] = t;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double u = V[k][a];
                V[k][a] = V[k][b];
                V[k][b] = u;
            }
        }
    };
    cx(0, 1);
    cx(2, 3);
    cx(0, 2);
    cx(1, 3);
    cx(1, 2);
}

// smallest r with cum_r >= 0.99 total (eq. SVD3); 0 for an all-zero set.
// *m_lo/*m_hi receive |cum_r - target| and |target - cum_{r-1}| (absolute).
__device__ __forceinline__ int rank99(const double s[4], double &m_hi, double &m_lo) {
    double tot = (s[0] + s[1]) + (s[2] + s[3]);
    m_hi = 1e300;
    m_lo = 1e300;
    if (!(tot > 0.0)) return 0;
    double target = 0.99 * tot, cum = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double prev = cum;
        cum += s[i];
        if (cum >= target) {
            m_hi = cum - target;
            if (i > 0) m_lo = target - prev;
            return i + 1;
        }
    }
    return 4;
}

struct BoundResult {
    double L, U, rho;
    int r;
    double jump;  // largest move of L, U that a rank flip within the band could cause
    double amp;   // first-order amplification of an l1 perturbation of A into L, U
};

// gap of sorted value i to its neighbours that are part of the kept set
// boundary (i-1 if i > 0, i+1 always)
__device__ __forceinline__ double sgap(const double s[4], int i) {
    double g = (i + 1 < 4) ? s[i] - s[i + 1] : s[i];
    if (i > 0) g = fmin(g, s[i - 1] - s[i]);
    return g;
}

// Nested-SVD bound of Section 2.2.2 (eqs. matrix1, SVD1-SVD7, Sxyz,
// bound1-bound3) in double precision.  The 4 x 16 unfolding carries the
// x-degree on its rows and (k,l) as 4k+l on its columns.  The singular
// triplets come from the eigen-decomposition of the 4x4 Gram matrices
// (A1 A1^T, then V_i V_i^T), sigma = sqrt(lambda), right vectors by
// back-substitution.
//
// The residual R = A - A~ is formed in place: subtracting sigma_i u_i (x) V~_i
// does not change u_j^T A1 for j > i (the u are orthonormal), so the later
// right vectors come out the same, and rho = sum |R| is read off at the end.
// A is overwritten.
//
// With band > 0 (A known only up to an l1 perturbation of that size) it also
// reports a first-order amplification factor amp -- singular values move by
// at most band, singular vectors rotate by about band / gap (Wedin), and the
// interval bound moves by about sigma times that rotation, so
// |dL|, |dU| <~ band * amp -- and a cap on the move a 0.99 rank rule within
// its band could cause by flipping: with unit singular vectors every
// Legendre series range lies in [-2, 2] (|sum q_j L_j| <= |q|_1 <= 2), so
// adding or dropping inner term k of outer term i moves L and U by at most
// 16 sigma_i d_k, and an outer term i by at most 32 sigma_i.
// BAND = false: exact tensors (band is 0 and the perturbation terms are not
// formed).  The outer singular vectors and values, and each inner problem's
// eigenvectors, are parked in LDS (ws: this thread's 36 doubles at stride
// wstride) while the inner problems run, which keeps the register footprint
// within two waves per SIMD.
template <bool BAND = true>
__device__ inline BoundResult nested_bound(double *A, double band, double *ws, int wstride) {
    BoundResult R;
    R.jump = 0.0;
    R.amp = 1.0;
    double S[4][4], W[4][4], lam[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j) {
            double g = 0.0;
#pragma unroll
            for (int e = 0; e < 16; ++e) g += A[16 * i + e] * A[16 * j + e];
            S[i][j] = g;
            S[j][i] = g;
        }
    eig4_sorted(S, lam, W);
    double sig[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) sig[i] = sqrt(fmax(lam[i], 0.0));
    double mhi, mlo;
    int r = rank99(sig, mhi, mlo);
    R.r = r;
    if (BAND && band > 0.0) {
        // cum_r and the 0.99 target move by at most (r + 4) band <= 8 band
        if (mhi <= 8.0 * band && r < 4) R.jump += 32.0 * sig[r];
        if (mlo <= 8.0 * band && r > 0) R.jump += 32.0 * sig[r - 1];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) ws[(4 * a + b) * wstride] = W[a][b];
        ws[(16 + a) * wstride] = sig[a];
    }
    double Msum = 0.0, msum = 0.0;
    for (int i = 0; i < r; ++i) {
        double u[4] = {ws[i * wstride], ws[(4 + i) * wstride], ws[(8 + i) * wstride],
                       ws[(12 + i) * wstride]};
        const double sgi = ws[(16 + i) * wstride];
        double inv = 1.0 / sgi;
        double v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            v[e] = (u[0] * A[e] + u[1] * A[16 + e] + u[2] * A[32 + e] + u[3] * A[48 + e]) * inv;
        // V_i[k][l] = v[4k+l]; H = V_i V_i^T
        double H[4][4], Z[4][4], mu[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int k2 = k; k2 < 4; ++k2) {
                double g = v[4 * k] * v[4 * k2] + v[4 * k + 1] * v[4 * k2 + 1] +
                           v[4 * k + 2] * v[4 * k2 + 2] + v[4 * k + 3] * v[4 * k2 + 3];
                H[k][k2] = g;
                H[k2][k] = g;
            }
        eig4_sorted(H, mu, Z);
        // Z goes to the workspace too: the residual loop below reads one
        // column per rank, and holding all 16 would spill there
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) ws[(20 + 4 * a + b) * wstride] = Z[a][b];
        // v again, from A (unchanged so far) -- the same operations, hence the
        // same bits; the empty asm hides the equality from the optimiser so v
        // is not held in registers across the eigen-solve
        {
            double uu[4] = {u[0], u[1], u[2], u[3]}, iv = inv;
            __asm__ volatile("" : "+v"(uu[0]), "+v"(uu[1]), "+v"(uu[2]), "+v"(uu[3]), "+v"(iv));
#pragma unroll
            for (int e = 0; e < 16; ++e)
                v[e] = (uu[0] * A[e] + uu[1] * A[16 + e] + uu[2] * A[32 + e] + uu[3] * A[48 + e]) *
                       iv;
        }
        double d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = sqrt(fmax(mu[k], 0.0));
        double nhi, nlo;
        int ri = rank99(d, nhi, nlo);
        if (BAND && band > 0.0) {
            // outer rotation of (u_i, v_i) and the inner perturbation of V_i
            double sv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) sv[a] = ws[(16 + a) * wstride];
            const double go = sgap(sv, i);
            const double rot = (go > 0.0) ? band / go : 1e300;
            const double dv = band * inv + rot;  // |dV_i| (unit-norm matrix)
            double dg = 1e300;
            for (int k = 0; k < ri; ++k) dg = fmin(dg, sgap(d, k));
            const double irot = (dg > 0.0) ? dv / dg : 1e300;
            R.amp += sgi * (rot + irot) / band + 1.0;
            if (nhi <= 8.0 * dv && ri < 4) R.jump += 16.0 * sgi * d[ri];
            if (nlo <= 8.0 * dv && ri > 0) R.jump += 16.0 * sgi * d[ri - 1];
        }
        double ux0, ux1;
        leg3_range(u, ux0, ux1);
        double Myz = 0.0, myz = 0.0;
        for (int k = 0; k < ri; ++k) {
            double w[4] = {ws[(20 + k) * wstride], ws[(24 + k) * wstride], ws[(28 + k) * wstride],
                           ws[(32 + k) * wstride]};
            double iz = 1.0 / d[k];
            double z[4];
#pragma unroll
            for (int l = 0; l < 4; ++l)
                z[l] = (w[0] * v[l] + w[1] * v[4 + l] + w[2] * v[8 + l] + w[3] * v[12 + l]) * iz;
            // residual: A -= sigma_i u_i (x) d_k w_k (x) z_k  (eq. SVD7)
            double coef = sgi * d[k];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    double cjk = coef * u[j] * w[kk];
#pragma unroll
                    for (int l = 0; l < 4; ++l) A[16 * j + 4 * kk + l] -= cjk * z[l];
                }
            double w0, w1, z0, z1, p0, p1;
            leg3_range(w, w0, w1);
            leg3_range(z, z0, z1);
            imul(w0, w1, z0, z1, p0, p1);
            Myz += d[k] * p1;
            myz += d[k] * p0;
        }
        double q0, q1;
        imul(ux0, ux1, myz, Myz, q0, q1);
        Msum += sgi * q1;
        msum += sgi * q0;
    }
    double rho = 0.0;
#pragma unroll
    for (int e = 0; e < 64; ++e) rho += fabs(A[e]);
    R.rho = rho;
    R.L = msum - rho;
    R.U = Msum + rho;
    if (!(R.amp < 1e300)) R.amp = 1e300;
    return R;
}

// Values of P at the 8 corners of its cube and at the centre; returns the
// range of those samples (a sub-range of P's range on the cube).
__device__ __forceinline__ void sample_range(const double *A, double &lo, double &hi) {
    // contract z with L(+-1) = (1, +-1, 1, +-1)
    double Bp[16], Bm[16];
#pragma unroll
    for (int jk = 0; jk < 16; ++jk) {
        double e = A[4 * jk] + A[4 * jk + 2], o = A[4 * jk + 1] + A[4 * jk + 3];
        Bp[jk] = e + o;
        Bm[jk] = e - o;
    }
    lo = 1e300;
    hi = -1e300;
#pragma unroll
    for (int zz = 0; zz < 2; ++zz) {
        const double *B = zz ? Bp : Bm;
        double Cp[4], Cm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double e = B[4 * j] + B[4 * j + 2], o = B[4 * j + 1] + B[4 * j + 3];
            Cp[j] = e + o;
            Cm[j] = e - o;
        }
#pragma unroll
        for (int yy = 0; yy < 2; ++yy) {
            const double *Cq = yy ? Cp : Cm;
            double e = Cq[0] + Cq[2], o = Cq[1] + Cq[3];
            double v0 = e - o, v1 = e + o;
            lo = fmin(lo, fmin(v0, v1));
            hi = fmax(hi, fmax(v0, v1));
        }
    }
    // centre: L(0) = (1, 0, -1/2, 0)
    double ctr = 0.0;
#pragma unroll
    for (int j = 0; j < 4; j += 2)
#pragma unroll
        for (int k = 0; k < 4; k += 2)
#pragma unroll
            for (int l = 0; l < 4; l += 2) {
                double f = ((j == 2) ? -0.5 : 1.0) * ((k == 2) ? -0.5 : 1.0) * ((l == 2) ? -0.5 : 1.0);
                ctr += f * A[16 * j + 4 * k + l];
            }
    lo = fmin(lo, ctr);
    hi = fmax(hi, ctr);
}

// Lanes of one wavefront exchanging data through LDS: a wavefront's LDS
// accesses execute in order, so only the compiler must not move them across
// this point (no workgroup barrier, which would also wait for outstanding
// global-to-LDS copies).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// x / cs, as a multiplication when that is exact
__device__ __forceinline__ double over_cs(const Grid &g, double x) {
    return g.inv_cs != 0.0 ? x * g.inv_cs : x / g.cs;
}

// atoms whose records one step of the point loop loads together
constexpr int kPhiBatch = 2;

// ---------------------------------------------------------------------------
// phi and grad phi at one point (eq. Gaussian1).
// ---------------------------------------------------------------------------
// Sum over atoms within R_c of p, in canonical atom order (cell rows of the
// stencil, atoms in cell order); xw holds the atoms as (x, y, z, w).  COUNT:
// phi receives the number of terms instead (the sum's algorithmic work).
template <bool FAST, bool GRAD = true, bool COUNT = false>
__device__ __forceinline__ void phi_at(const Grid &g, const double p[3],
                                       const int32_t *__restrict__ cs,
                                       const double4 *__restrict__ xw, double &phi, double gr[3]) {
    const double D = g.D, m2D = -2.0 * g.D;
    phi = 0.0;
    gr[0] = gr[1] = gr[2] = 0.0;
    auto add = [&](double w, double dx, double dy, double dz, double d2) {
        if (COUNT) {
            phi += 1.0;
            return;
        }
        // explicit fused forms: every kernel that sums phi over atoms uses
        // these same operations, so their values agree bit for bit
        const double e = expn<FAST>(-D * d2);
        phi = fma(w, e, phi);
        if (GRAD) {
            const double f = m2D * (w * e);
            gr[0] += f * dx;
            gr[1] += f * dy;
            gr[2] += f * dz;
        }
    };
    int c0[3], c1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // points far outside the grid (or NaN) get an empty stencil
        const double fc = floor(over_cs(g, p[a] - g.o[a]));
        const int ci = (fc > -1.0e8 && fc < 1.0e8) ? (int)fc : -1000000;
        c0[a] = max(ci - g.span, 0);
        c1[a] = min(ci + g.span, g.nc[a] - 1);
    }
    // rows of the stencil along x, each clipped to the chord of the R_c
    // sphere (skipped cells hold only atoms beyond R_c); the chord's half
    // length comes from the hardware reciprocal square root, enlarged by
    // 2^-20 relative to cover its error, so a row may keep a cell more than
    // needed (whose atoms the distance test drops) but never one less
    auto row_range = [&](int cz, int cy, int &b, int &e) {
        b = 0;
        e = 0;
        const double lz = g.o[2] + cz * g.cs;
        const double ez = fmax(fmax(lz - p[2], p[2] - (lz + g.cs)), 0.0);
        const double ly = g.o[1] + cy * g.cs;
        const double ey = fmax(fmax(ly - p[1], p[1] - (ly + g.cs)), 0.0);
        const double ryz = (g.rc2 - ez * ez) - ey * ey;
        if (!(ryz >= 0.0)) return;
        const double hx = ryz > 0.0 ? ryz * __builtin_amdgcn_rsq(ryz) * (1.0 + 0x1p-20) : 0.0;
        const int x0 = max(c0[0], (int)floor(over_cs(g, p[0] - hx - g.o[0])));
        const int x1 = min(c1[0], (int)floor(over_cs(g, p[0] + hx - g.o[0])));
        if (x0 > x1) return;
        const int row = (int)g.cell_base + (cz * g.nc[1] + cy) * g.nc[0];
        b = cs[row + x0];
        e = cs[row + x1 + 1];
    };
    const int ny = c1[1] - c0[1] + 1;
    const int nrow = (ny > 0 && c1[2] >= c0[2]) ? (c1[2] - c0[2] + 1) * ny : 0;
    int cz = c0[2], cy = c0[1], b = 0, e = 0;
    if (nrow > 0) row_range(cz, cy, b, e);
    for (int r = 0; r < nrow; ++r) {
        const int rb = b, re = e;
        // the next row's cell range is requested before this row's atoms
        // are summed, so its loads overlap them
        if (++cy > c1[1]) {
            cy = c0[1];
            ++cz;
        }
        if (r + 1 < nrow) row_range(cz, cy, b, e);
        // kPhiBatch atoms per step, so that their loads are in flight
        // together; the terms are still added one atom at a time, in cell
        // order
        for (int i = rb; i < re; i += kPhiBatch) {
            double4 a[kPhiBatch];
#pragma unroll
            for (int k = 0; k < kPhiBatch; ++k) a[k] = xw[i + k < re ? i + k : i];
            // every record requested before any is used
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < kPhiBatch; ++k) {
                const double dx = p[0] - a[k].x, dy = p[1] - a[k].y, dz = p[2] - a[k].z;
                const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
                const bool in = i + k < re && !(d2 > g.rc2);
                // the weight selected here keeps its load beside the
                // coordinates'
                const double w = in ? a[k].w : 0.0;
                if (in) add(w, dx, dy, dz, d2);
            }
        }
    }
}

// Bit of finest-lattice point (X, Y, Z) in a dense corner bitmap: 4x4x4
// point blocks per 64-bit word, words X-major over blocks.
__device__ __forceinline__ int64_t lat_bit(const Lat &lat, int64_t X, int64_t Y, int64_t Z) {
    const int64_t w = ((X >> 2) * lat.n[1] + (Y >> 2)) * lat.n[2] + (Z >> 2);
    return ((lat.base + w) << 6) + ((X & 3) << 4) + ((Y & 3) << 2) + (Z & 3);
}

// Rank of set bit b among all set bits (woff: exclusive scan of word counts).
__device__ __forceinline__ int64_t bit_rank(const uint64_t *__restrict__ bm,
                                            const int32_t *__restrict__ woff, int64_t b) {
    const int64_t w = b >> 6;
    const uint64_t below = bm[w] & ((1ull << (b & 63)) - 1ull);
    return (int64_t)woff[w] + __popcll(below);
}

__device__ __forceinline__ bool bit_test(const uint64_t *__restrict__ bm, int64_t b) {
    return (bm[b >> 6] >> (b & 63)) & 1ull;
}

// Conformation owning position i of a batch-wide atom or root array: the
// last b whose base is <= i (bases ascend with b).
__device__ __forceinline__ int conf_of_atom(const Grid *__restrict__ gt, int nconf, int64_t i) {
    int lo = 0, hi = nconf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (gt[mid].atom_base <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int conf_of_root(const Grid *__restrict__ gt, int nconf, int64_t r) {
    int lo = 0, hi = nconf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (gt[mid].root_base <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace tms


