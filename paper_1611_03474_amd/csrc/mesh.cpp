// Host Stage 2 (Section 2.3): the trilinear surface g = c of every SURFACE
// leaf (eq. linear1) as triangles, and the manifold conditions of Section
// 3.2.  Host C++ over std::thread; the device results of the partition
// (leaves, corner values) and of the extraction (edge points) are copied in.
//
// Per leaf, the surface meets the cube's boundary in curves on its faces.  On
// a face g is bilinear, so g = c there is a hyperbola (or a pair of lines)
// whose branches join the face's edge points (eq. intersection) in pairs: two
// edge points on a face are joined directly; four (the corners alternate
// around the face) are paired by the value of g at the face's saddle point --
// at or above c the two corners at or above c are joined through the face and
// each corner below c is cut off, else the reverse.  Both leaves that share a
// face see the same four values and pair the same way, so neighbouring
// leaves' curves agree.  Each edge point lies on two faces of the cube, so
// the face segments link into closed loops on the cube's boundary, each
// enclosing one patch of the surface.
//
// A patch is triangulated by ear clipping (Section 2.3) in the plane normal
// to an axis along which it is single valued: the axis of the loop's largest
// projected area, else the next, as long as the loop projects to a simple
// polygon there, with no diagonal between two points of one cube face (that
// side would lie in the face, where the leaf across has its own triangles).
// A loop that cannot be clipped so along any axis is fanned from a point of
// its patch inside the cube and counted.  Triangles are oriented so that their normal
// points along -grad g (outward: phi >= c is inside).
//
// The checks: (a) every edge shared by exactly two triangles, traversed in
// opposite directions; (b) the neighbourhood of every vertex one single loop;
// (c) no two triangles without a shared vertex intersecting.  Vertices that
// fail (a) or (b) are the paper's non-manifold defects.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "tms_internal.h"

struct tms_mesh {
    std::vector<double> xyz;        // [nv][3]
    std::vector<int32_t> tri;       // [nt][3]
    std::vector<int32_t> tri_leaf;  // [nt] index of the leaf in the caller's list
    std::vector<int32_t> leaf_ijk;  // [n][3] of the caller's leaves (for the checks)
    std::vector<tms_leaf> added;    // cubes added across open faces
    std::vector<double> added_phi;  // [n_added][8] their corner values
    int level = 0;
    int64_t n_surface = 0, n_loops = 0, n_fallback = 0, open_faces = 0, n_face_points = 0;
};

namespace {

using tms::DevBuf;
using tms::Grid;

int32_t mfail(tms_ctx *ctx, int32_t code, const char *msg) {
    if (ctx) ctx->err = msg;
    return code;
}

// ---- cube topology ----------------------------------------------------------
// corner v = dx + 2 dy + 4 dz; edge e: axis = e / 4, the other two axes in
// ascending order take offsets (e & 1, (e >> 1) & 1) (the extraction's edge
// numbering).
struct EdgeInfo {
    int axis, off[3], v0, v1;
};

EdgeInfo edge_info(int e) {
    EdgeInfo E;
    E.axis = e >> 2;
    const int o1 = (E.axis + 1) % 3, o2 = (E.axis + 2) % 3;
    const int lo = std::min(o1, o2), hi = std::max(o1, o2);
    E.off[0] = E.off[1] = E.off[2] = 0;
    E.off[lo] = e & 1;
    E.off[hi] = (e >> 1) & 1;
    E.v0 = E.off[0] + 2 * E.off[1] + 4 * E.off[2];
    E.v1 = E.v0 + (1 << E.axis);
    return E;
}

// edge along axis b with offsets ob[] on the other axes
int edge_index(int b, const int off[3]) {
    const int o1 = (b + 1) % 3, o2 = (b + 2) % 3;
    const int lo = std::min(o1, o2), hi = std::max(o1, o2);
    return 4 * b + off[lo] + 2 * off[hi];
}

// Face (a, s): the plane u_a = s.  Its corners in cyclic order K0..K3 =
// (p, q) = (0,0), (1,0), (1,1), (0,1) with p, q the other two axes in
// ascending order, and its edges E_k between K_k and K_{k+1}.
struct FaceInfo {
    int corner[4];
    int edge[4];
};

FaceInfo face_info(int a, int s) {
    const int o1 = (a + 1) % 3, o2 = (a + 2) % 3;
    const int p = std::min(o1, o2), q = std::max(o1, o2);
    const int pq[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    FaceInfo F;
    for (int k = 0; k < 4; ++k) {
        int off[3];
        off[a] = s;
        off[p] = pq[k][0];
        off[q] = pq[k][1];
        F.corner[k] = off[0] + 2 * off[1] + 4 * off[2];
    }
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        // the axis along which K_k and K_k1 differ
        const int b = (pq[k][0] != pq[k1][0]) ? p : q;
        int off[3];
        off[a] = s;
        off[p] = std::min(pq[k][0], pq[k1][0]);
        off[q] = std::min(pq[k][1], pq[k1][1]);
        off[b] = 0;
        F.edge[k] = edge_index(b, off);
    }
    return F;
}

struct Topo {
    EdgeInfo E[12];
    FaceInfo F[6];  // face 2 a + s
    int edge_face[12][2];
    Topo() {
        for (int e = 0; e < 12; ++e) E[e] = edge_info(e);
        int cnt[12] = {0};
        for (int a = 0; a < 3; ++a)
            for (int s = 0; s < 2; ++s) {
                F[2 * a + s] = face_info(a, s);
                for (int k = 0; k < 4; ++k) {
                    const int e = F[2 * a + s].edge[k];
                    edge_face[e][cnt[e]++] = 2 * a + s;
                }
            }
    }
};

const Topo &topo() {
    static const Topo t;
    return t;
}

// ---- one leaf ---------------------------------------------------------------
// a loop visits each of the cube's 12 edges at most once; with up to 4
// points on each face it has at most 36 points
constexpr int kPolyMax = 48;
struct LeafOut {
    // corners: cube edge indices 0..11, 12 + k the k-th interior point, or
    // 64 + j the j-th face point (fpid[j] its mesh vertex id)
    std::vector<std::array<int, 3>> tri;
    std::vector<std::array<double, 3>> inner;  // interior points (local)
    std::vector<int64_t> fpid;
    std::vector<std::array<double, 3>> fpxyz;  // face points (local)
    int loops = 0, fallback = 0;
};

// face segments of a leaf: partner[e][j] = the edge joined to edge e on the
// j-th face containing e (-1: none)
void face_segments(const double f[8], double c, int partner[12][2]) {
    const Topo &T = topo();
    for (int e = 0; e < 12; ++e) partner[e][0] = partner[e][1] = -1;
    auto link = [&](int e1, int e2, int face) {
        const int j1 = T.edge_face[e1][0] == face ? 0 : 1;
        const int j2 = T.edge_face[e2][0] == face ? 0 : 1;
        partner[e1][j1] = e2;
        partner[e2][j2] = e1;
    };
    for (int fi = 0; fi < 6; ++fi) {
        const FaceInfo &F = T.F[fi];
        bool hi[4];
        for (int k = 0; k < 4; ++k) hi[k] = f[F.corner[k]] >= c;
        int cut[4], n = 0;
        for (int k = 0; k < 4; ++k)
            if (hi[k] != hi[(k + 1) & 3]) cut[n++] = k;
        if (n == 2) {
            link(F.edge[cut[0]], F.edge[cut[1]], fi);
        } else if (n == 4) {
            // corners alternate; bilinear h(p,q) on the face, saddle value
            // (h00 h11 - h10 h01) / (h00 + h11 - h10 - h01)
            const double h00 = f[F.corner[0]], h10 = f[F.corner[1]], h11 = f[F.corner[2]],
                         h01 = f[F.corner[3]];
            const double sad = (h00 * h11 - h10 * h01) / (h00 + h11 - h10 - h01);
            const bool join_high = sad >= c;
            // corner k is cut off by the segment joining its two edges
            // (E_{k-1}, E_k); cut the low corners when the high ones join
            for (int k = 0; k < 4; ++k)
                if (hi[k] != join_high) link(F.edge[(k + 3) & 3], F.edge[k], fi);
        }
    }
}

// An edge point closer than kTmin (of the edge) to a corner is moved to
// kTmin from it: a corner value equal to c (inside, phi >= c) would otherwise
// put the points of its three edges on the corner itself, and the polygon
// of the loop would repeat a point.  The move is at most kTmin h.
constexpr double kTmin = 1e-6;

double clamp_t(double t) { return std::min(std::max(t, kTmin), 1.0 - kTmin); }

// local position of the edge point of edge e
void edge_point(const double f[8], double c, int e, double P[3]) {
    const EdgeInfo &E = topo().E[e];
    const double t = clamp_t((c - f[E.v0]) / (f[E.v1] - f[E.v0]));
    for (int a = 0; a < 3; ++a) P[a] = (double)E.off[a];
    P[E.axis] = t;
}

// the trilinear interpolant at local point u
double g_at(const double f[8], const double u[3]) {
    double s = 0.0;
    for (int v = 0; v < 8; ++v) {
        double w = 1.0;
        for (int b = 0; b < 3; ++b) w *= ((v >> b) & 1) ? u[b] : 1.0 - u[b];
        s += w * f[v];
    }
    return s;
}

// gradient of the trilinear interpolant at local point u
void grad_g(const double f[8], const double u[3], double G[3]);

// a point of g = c near u: Newton steps along grad g, kept in the cube;
// false if the gradient vanishes or the steps do not converge
bool onto_surface(const double f[8], double c, double u[3]) {
    for (int it = 0; it < 50; ++it) {
        double G[3];
        grad_g(f, u, G);
        const double gg = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        const double r = g_at(f, u) - c;
        if (std::fabs(r) <= 1e-13 * (std::fabs(c) + 1.0)) return true;
        if (!(gg > 0.0)) return false;
        for (int a = 0; a < 3; ++a) u[a] = std::min(1.0, std::max(0.0, u[a] - r * G[a] / gg));
    }
    return false;
}

void grad_g(const double f[8], const double u[3], double G[3]) {
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int v = 0; v < 8; ++v) {
            double w = 1.0;
            for (int b = 0; b < 3; ++b) {
                if (b == a) continue;
                const int o = (v >> b) & 1;
                w *= o ? u[b] : 1.0 - u[b];
            }
            s += (((v >> a) & 1) ? 1.0 : -1.0) * w * f[v];
        }
        G[a] = s;
    }
}

double cross2(const double a[2], const double b[2], const double c[2]) {
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

// do segments ab and cd meet (including touching)?
bool seg_meet(const double a[2], const double b[2], const double c[2], const double d[2]) {
    const double d1 = cross2(a, b, c), d2 = cross2(a, b, d), d3 = cross2(c, d, a),
                 d4 = cross2(c, d, b);
    if (((d1 > 0 && d2 < 0) || (d1 < 0 && d2 > 0)) && ((d3 > 0 && d4 < 0) || (d3 < 0 && d4 > 0)))
        return true;
    auto on = [](const double p[2], const double q[2], const double r[2], double cr) {
        return cr == 0.0 && std::min(p[0], q[0]) <= r[0] && r[0] <= std::max(p[0], q[0]) &&
               std::min(p[1], q[1]) <= r[1] && r[1] <= std::max(p[1], q[1]);
    };
    return on(a, b, c, d1) || on(a, b, d, d2) || on(c, d, a, d3) || on(c, d, b, d4);
}

// Choices between candidates (ears, axes, the vertex spanning a fold) take
// a later candidate only if it is better by more than this, so that inputs
// equal up to rounding (a symmetric cube, corner values that differ in their
// last bits) give the same triangles.
constexpr double kTie = 1e-9;

// sine of a triangle's smallest angle (the angle at the vertex opposite its
// shortest side: twice the area over the two longer sides), 0 if degenerate
double shape(const double *p, const double *q, const double *r) {
    const double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    const double v[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
    const double w[3] = {r[0] - q[0], r[1] - q[1], r[2] - q[2]};
    const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double l[3] = {u[0] * u[0] + u[1] * u[1] + u[2] * u[2], v[0] * v[0] + v[1] * v[1] + v[2] * v[2],
                   w[0] * w[0] + w[1] * w[1] + w[2] * w[2]};
    std::sort(l, l + 3);
    const double d = std::sqrt(l[1] * l[2]);
    return d > 0.0 ? std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]) / d : 0.0;
}

// ear clipping of a simple polygon (counter-clockwise or clockwise) of m
// points; emits index triples with the polygon's winding.  fm[i]: the cube
// faces point i lies on (bit 2 a + s); no diagonal joins two points of one
// face -- such a side would lie in the face, where the leaf across puts its
// own triangles (a loop that crosses a face twice, through both branches of
// its hyperbola, would otherwise be capped in the face from both sides).
// Of the ears at each step the one whose triangle in space (X) is best
// shaped is cut.  Returns false if the polygon is not simple or has no ear
// left.
bool ear_clip(const double (*Q)[2], const double (*X)[3], int m, const unsigned *fm,
              std::array<int, 3> *out, int *nout) {
    *nout = 0;
    // simple: non-adjacent sides do not meet, no repeated point
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) {
            if (Q[i][0] == Q[j][0] && Q[i][1] == Q[j][1]) return false;
            if (j == i + 1 || (i == 0 && j == m - 1)) continue;
            if (seg_meet(Q[i], Q[(i + 1) % m], Q[j], Q[(j + 1) % m])) return false;
        }
    double area = 0.0;
    for (int i = 0; i < m; ++i) area += Q[i][0] * Q[(i + 1) % m][1] - Q[(i + 1) % m][0] * Q[i][1];
    if (area == 0.0) return false;
    const double sg = area > 0 ? 1.0 : -1.0;
    if (m > kPolyMax) return false;
    int idx[kPolyMax], k = m;
    for (int i = 0; i < m; ++i) idx[i] = i;
    while (k > 3) {
        // of the ears, the one whose triangle in space is best shaped
        int best = -1;
        double bq = -1.0;
        for (int i = 0; i < k; ++i) {
            const int ia = idx[(i + k - 1) % k], ib = idx[i], ic = idx[(i + 1) % k];
            if (fm[ia] & fm[ic]) continue;
            const double cr = cross2(Q[ia], Q[ib], Q[ic]) * sg;
            if (!(cr > 0.0)) continue;
            const double q = shape(X[ia], X[ib], X[ic]);
            if (!(q > bq + kTie)) continue;  // cannot replace the best ear so far
            bool inside = false;
            for (int j = 0; j < k && !inside; ++j) {
                const int ij = idx[j];
                if (ij == ia || ij == ib || ij == ic) continue;
                const double c1 = cross2(Q[ia], Q[ib], Q[ij]) * sg,
                             c2 = cross2(Q[ib], Q[ic], Q[ij]) * sg,
                             c3 = cross2(Q[ic], Q[ia], Q[ij]) * sg;
                if (c1 >= 0 && c2 >= 0 && c3 >= 0) inside = true;
            }
            if (inside) continue;
            bq = q;
            best = i;
        }
        if (best < 0) return false;
        out[(*nout)++] = {idx[(best + k - 1) % k], idx[best], idx[(best + 1) % k]};
        for (int j = best; j + 1 < k; ++j) idx[j] = idx[j + 1];
        --k;
    }
    out[(*nout)++] = {idx[0], idx[1], idx[2]};
    return true;
}

// ---- folds and face points (Section 2.3: eqs. curve, fold1) -----------------
// On a leaf's local cube [0,1]^3 the trilinear g = sum_S m_S prod_{i in S} x_i
// (S a set of axes; bit 0 x, bit 1 y, bit 2 z).  Along axis a, dg/da does
// not depend on x_a, and where it vanishes neither does g: the fold set along
// a (g = c, dg/da = 0) is a set of full segments parallel to a, over the
// points (u, v) of the two other axes (u the lower) where dg/da = 0 and
// g(x_a = 0) = c -- at most two -- and each ends at an extreme point (eq.
// curve) on the faces x_a = 0 and x_a = 1.  Folds on the cube's boundary (u
// or v within 1e-9 of 0 or 1) lie in a face curve and are left out.
struct Fold {
    double u, v;
};

constexpr double kFoldIn = 1e-9;
// face points closer than this (in face coordinates) are one point
constexpr double kFaceMerge = 1e-9;

void monomials01(const double f[8], double m[8]) {
    for (int v = 0; v < 8; ++v) m[v] = f[v];
    for (int b = 1; b < 8; b <<= 1)
        for (int v = 0; v < 8; ++v)
            if (v & b) m[v] -= m[v ^ b];
}

// real roots of r0 + r1 t + r2 t^2, ascending; -1 when every coefficient is 0
int quad_roots(double r0, double r1, double r2, double t[2]) {
    if (r2 == 0.0) {
        if (r1 == 0.0) return r0 == 0.0 ? -1 : 0;
        t[0] = -r0 / r1;
        return 1;
    }
    const double d = r1 * r1 - 4.0 * r2 * r0;
    if (d < 0.0) return 0;
    if (d == 0.0) {
        t[0] = -r1 / (2.0 * r2);
        return 1;
    }
    const double sq = std::sqrt(d);
    const double big = (r1 >= 0.0) ? (-r1 - sq) / (2.0 * r2) : (-r1 + sq) / (2.0 * r2);
    const double small = (big != 0.0) ? r0 / (r2 * big) : big;
    t[0] = std::min(big, small);
    t[1] = std::max(big, small);
    return 2;
}

int folds_along(const double m[8], double c, int a, Fold out[2]) {
    const int U = (a == 0) ? 2 : 1, V = (a == 2) ? 2 : 4, A = 1 << a;
    const double h0 = m[A], hu = m[A | U], hv = m[A | V], huv = m[A | U | V];
    if (h0 == 0.0 && hu == 0.0 && hv == 0.0 && huv == 0.0) return 0;  // g free of x_a
    const double g0 = m[0] - c, gu = m[U], gv = m[V], guv = m[U | V];
    // both equations as alpha(v) + beta(v) u; their resultant in u
    const double r0 = g0 * hu - gu * h0;
    const double r1 = g0 * huv + gv * hu - gu * hv - guv * h0;
    const double r2 = gv * huv - guv * hv;
    double t[2];
    const int nr = quad_roots(r0, r1, r2, t);
    if (nr <= 0) return 0;  // none, or infinitely many (a curve: not split)
    int n = 0;
    for (int i = 0; i < nr; ++i) {
        const double v = t[i];
        if (!(v > kFoldIn && v < 1.0 - kFoldIn)) continue;
        const double aG = g0 + gv * v, bG = gu + guv * v;
        const double aH = h0 + hv * v, bH = hu + huv * v;
        if (bG == 0.0 && bH == 0.0) continue;  // a line of solutions, or none
        const double u = (std::fabs(bG) >= std::fabs(bH)) ? -aG / bG : -aH / bH;
        if (!(u > kFoldIn && u < 1.0 - kFoldIn)) continue;
        out[n++] = {u, v};
    }
    if (n == 2 && out[1].u < out[0].u) std::swap(out[0], out[1]);
    return n;
}

// a point on a face of the leaf: face coordinates (u along the face's lower
// other axis, v along the higher) and its mesh vertex id
struct FacePt {
    double u, v;
    int64_t id;
};

// what the triangulation of a leaf knows besides its corner values: the
// points on each face (its own extreme points and the neighbour's, from
// both cubes sharing the face), and its own folds with the ids of their ends
struct LeafFolds {
    const FacePt *fp[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int nfp[6] = {0, 0, 0, 0, 0, 0};
    Fold fold[3][2];
    int64_t end_id[3][2][2];  // [axis][fold][side]
    int nfold[3] = {0, 0, 0};
};


// Corner codes of LeafOut triangles: 0..11 edge points, 12 + k the k-th
// interior point, 64 + j the j-th face point of the leaf (LeafOut::fpid).
constexpr int kCodeFace = 64;

// Ear clipping of one piece of a patch (loop indices pc, in loop order) in
// the plane normal to axis a.  A fold along a on the piece's boundary (two
// consecutive points of pc that are the two ends of one chord) projects to a
// single point W: the projected polygon takes W once, and after clipping the
// fan of triangles around W is lifted back, the triangles from W's neighbour
// after the fold up to the fan vertex u nearest the fold's middle along a on
// the fold's second end, the rest on its first end, with the triangle
// (first end, second end, u) spanning the fold.  Triangles keep the order of
// the loop.  False if the projection is not a simple polygon.
struct Piece {
    int v[kPolyMax];
    int n;
};

bool clip_piece(const double (*P)[3], const unsigned *fm, const int *pc, int pm,
                const int (*chord)[2], int nch, int a, std::array<int, 3> *tl, int *ntl) {
    const int b = (a + 1) % 3, cc = (a + 2) % 3;
    auto is_chord = [&](int x, int y) {
        for (int k = 0; k < nch; ++k)
            if ((chord[k][0] == x && chord[k][1] == y) || (chord[k][0] == y && chord[k][1] == x))
                return true;
        return false;
    };
    // rotate so that no fold pair wraps around the end of the list
    int r0 = 0;
    if (pm > 1 && is_chord(pc[pm - 1], pc[0])) r0 = pm - 1;
    int first[kPolyMax], second[kPolyMax], nk = 0;
    for (int t = 0; t < pm;) {
        const int x = pc[(r0 + t) % pm];
        if (t + 1 < pm && is_chord(x, pc[(r0 + t + 1) % pm])) {
            first[nk] = x;
            second[nk++] = pc[(r0 + t + 1) % pm];
            t += 2;
        } else {
            first[nk] = x;
            second[nk++] = -1;
            ++t;
        }
    }
    if (nk < 3) return false;
    double Q[kPolyMax][2], X[kPolyMax][3];
    unsigned qfm[kPolyMax];
    for (int i = 0; i < nk; ++i) {
        Q[i][0] = P[first[i]][b];
        Q[i][1] = P[first[i]][cc];
        for (int d = 0; d < 3; ++d)
            X[i][d] = second[i] < 0 ? P[first[i]][d] : 0.5 * (P[first[i]][d] + P[second[i]][d]);
        qfm[i] = fm[first[i]] | (second[i] >= 0 ? fm[second[i]] : 0u);
    }
    std::array<int, 3> rt[kPolyMax];
    int nrt = 0;
    if (!ear_clip(Q, X, nk, qfm, rt, &nrt)) return false;
    // per reduced triangle and corner: the loop index it stands for
    std::array<int, 3> out[kPolyMax];
    for (int k = 0; k < nrt; ++k)
        for (int z = 0; z < 3; ++z) out[k][(size_t)z] = first[rt[k][(size_t)z]];
    std::array<int, 3> bridge[kPolyMax];
    int nb = 0;
    for (int w = 0; w < nk; ++w) {
        if (second[w] < 0) continue;
        // the fan around w: triangles rotated to (w, x, y), chained from
        // x = the next vertex to y = the previous one
        const int nxt = (w + 1) % nk, prv = (w + nk - 1) % nk;
        int fan[kPolyMax], fu[kPolyMax + 1], nf = 0;
        int x = nxt;
        while (true) {
            int hit = -1, y = -1;
            for (int k = 0; k < nrt && hit < 0; ++k)
                for (int z = 0; z < 3; ++z)
                    if (rt[k][(size_t)z] == w && rt[k][(size_t)((z + 1) % 3)] == x) {
                        hit = k;
                        y = rt[k][(size_t)((z + 2) % 3)];
                    }
            if (hit < 0 || nf >= kPolyMax) return false;
            fu[nf] = x;
            fan[nf++] = hit;
            x = y;
            if (x == prv) break;
        }
        fu[nf] = prv;
        // the fan vertex where the triangles pass from the second end to
        // the first: nearest the fold's middle along a, not itself a fold
        const double mid = 0.5 * (P[first[w]][a] + P[second[w]][a]);
        int j = -1;
        double bd = 1e300;
        for (int t = 0; t <= nf; ++t) {
            if (second[fu[t]] >= 0) continue;
            const double d = std::fabs(P[first[fu[t]]][a] - mid);
            if (d < bd - kTie) {
                bd = d;
                j = t;
            }
        }
        if (j < 0) return false;
        for (int t = 0; t < nf; ++t)
            for (int z = 0; z < 3; ++z)
                if (rt[fan[t]][(size_t)z] == w) out[fan[t]][(size_t)z] = t < j ? second[w] : first[w];
        bridge[nb++] = {first[w], second[w], first[fu[j]]};
    }
    for (int k = 0; k < nrt; ++k) tl[(*ntl)++] = out[k];
    for (int k = 0; k < nb; ++k) tl[(*ntl)++] = bridge[k];
    return true;
}

void leaf_triangles(const double f[8], double c, const LeafFolds &lfo, LeafOut &L) {
    const Topo &T = topo();
    int partner[12][2];
    face_segments(f, c, partner);
    L.fpid.clear();
    L.fpxyz.clear();
    // the face points of each face on each of its branches (a face curve
    // has one or two branches, each joining two edge points, each monotone
    // in both face coordinates): a point goes to the branch whose bounding
    // box is nearest (contains it, barring rounding)
    struct Branch {
        int e1, e2;
        int pts[8];
        int np;
    };
    Branch br[6][2];
    int nbr[6] = {0, 0, 0, 0, 0, 0};
    double Pe[12][3];
    bool have[12] = {false};
    for (int e = 0; e < 12; ++e)
        if (partner[e][0] >= 0) {
            edge_point(f, c, e, Pe[e]);
            have[e] = true;
        }
    for (int fi = 0; fi < 6; ++fi) {
        for (int e = 0; e < 12; ++e)
            for (int j = 0; j < 2; ++j)
                if (partner[e][j] > e && T.edge_face[e][j] == fi && nbr[fi] < 2)
                    br[fi][nbr[fi]++] = {e, partner[e][j], {0}, 0};
        if (lfo.nfp[fi] == 0 || nbr[fi] == 0) continue;
        const int a = fi >> 1, p = (a == 0) ? 1 : 0, q = (a == 2) ? 1 : 2;
        for (int k = 0; k < lfo.nfp[fi]; ++k) {
            const FacePt &x = lfo.fp[fi][k];
            int best = 0;
            double bd = 1e300;
            for (int b = 0; b < nbr[fi]; ++b) {
                const double *P1 = Pe[br[fi][b].e1], *P2 = Pe[br[fi][b].e2];
                const double du = std::max({0.0, std::min(P1[p], P2[p]) - x.u, x.u - std::max(P1[p], P2[p])});
                const double dv = std::max({0.0, std::min(P1[q], P2[q]) - x.v, x.v - std::max(P1[q], P2[q])});
                const double d = du * du + dv * dv;
                if (d < bd) {
                    bd = d;
                    best = b;
                }
            }
            Branch &B = br[fi][best];
            if (B.np < 8) B.pts[B.np++] = k;
        }
    }
    bool used[12] = {false};
    for (int e0 = 0; e0 < 12; ++e0) {
        if (used[e0] || partner[e0][0] < 0) continue;
        // walk the loop through e0, with the face points of each branch crossed
        int code[kPolyMax], m = 0, ne = 0;
        int prev = -1, cur = e0;
        bool bad = false;
        while (true) {
            if (m >= kPolyMax) {
                bad = true;
                break;
            }
            code[m++] = cur;
            ++ne;
            used[cur] = true;
            const int j = (partner[cur][0] != prev) ? 0 : 1;
            const int nx = partner[cur][j], fi = T.edge_face[cur][j];
            if (nx < 0) break;
            // the branch (cur, nx) of face fi and its points, from cur to nx
            for (int b = 0; b < nbr[fi]; ++b) {
                const Branch &B = br[fi][b];
                if (!((B.e1 == cur && B.e2 == nx) || (B.e1 == nx && B.e2 == cur)) || B.np == 0)
                    continue;
                const int a = fi >> 1, p = (a == 0) ? 1 : 0, q = (a == 2) ? 1 : 2;
                const double d0 = Pe[nx][p] - Pe[cur][p], d1 = Pe[nx][q] - Pe[cur][q];
                int ord[8];
                double key[8];
                for (int k = 0; k < B.np; ++k) {
                    const FacePt &x = lfo.fp[fi][B.pts[k]];
                    ord[k] = B.pts[k];
                    key[k] = (x.u - Pe[cur][p]) * d0 + (x.v - Pe[cur][q]) * d1;
                }
                for (int k = 1; k < B.np; ++k)  // insertion sort along the branch
                    for (int l = k; l > 0 && key[l] < key[l - 1]; --l) {
                        std::swap(key[l], key[l - 1]);
                        std::swap(ord[l], ord[l - 1]);
                    }
                for (int k = 0; k < B.np && m < kPolyMax; ++k) {
                    const int64_t id = lfo.fp[fi][ord[k]].id;
                    int slot = -1;
                    for (int z = 0; z < (int)L.fpid.size(); ++z)
                        if (L.fpid[(size_t)z] == id) slot = z;
                    if (slot < 0) {
                        slot = (int)L.fpid.size();
                        L.fpid.push_back(id);
                        L.fpxyz.push_back({0.0, 0.0, 0.0});
                        double *X = L.fpxyz.back().data();
                        X[a] = (double)(fi & 1);
                        X[p] = lfo.fp[fi][ord[k]].u;
                        X[q] = lfo.fp[fi][ord[k]].v;
                    }
                    code[m++] = kCodeFace + slot;
                }
                break;
            }
            prev = cur;
            cur = nx;
            if (cur == e0 || ne > 12) break;
        }
        if (bad || cur != e0 || ne < 3) continue;  // not closed (cannot happen)
        ++L.loops;
        double P[kPolyMax + 1][3];  // the loop's points, then an interior point
        unsigned fm[kPolyMax];
        for (int i = 0; i < m; ++i) {
            if (code[i] < 12) {
                for (int a = 0; a < 3; ++a) P[i][a] = Pe[code[i]][a];
                fm[i] = (1u << T.edge_face[code[i]][0]) | (1u << T.edge_face[code[i]][1]);
            } else {
                const double *X = L.fpxyz[(size_t)(code[i] - kCodeFace)].data();
                for (int a = 0; a < 3; ++a) P[i][a] = X[a];
                unsigned mk = 0;
                for (int a = 0; a < 3; ++a)
                    if (X[a] == 0.0 || X[a] == 1.0) mk |= 1u << (2 * a + (X[a] == 1.0 ? 1 : 0));
                fm[i] = mk;
            }
        }
        // vector area of the loop and the outward direction -grad g decide
        // the projection order and the orientation
        double A[3] = {0, 0, 0}, ctr[3] = {0, 0, 0};
        for (int i = 0; i < m; ++i) {
            const double *pp = P[i], *qq = P[(i + 1) % m];
            A[0] += 0.5 * (pp[1] * qq[2] - pp[2] * qq[1]);
            A[1] += 0.5 * (pp[2] * qq[0] - pp[0] * qq[2]);
            A[2] += 0.5 * (pp[0] * qq[1] - pp[1] * qq[0]);
            for (int a = 0; a < 3; ++a) ctr[a] += pp[a] / m;
        }
        int order[3] = {0, 1, 2};
        for (int i = 1; i < 3; ++i)  // by |A| descending; near-equal keep axis order
            for (int j = i; j > 0 && std::fabs(A[order[j]]) > std::fabs(A[order[j - 1]]) + kTie; --j)
                std::swap(order[j], order[j - 1]);
        std::array<int, 3> tl[3 * kPolyMax];
        int ntl = 0;
        bool ok = false;
        for (int oi = 0; oi < 3 && !ok; ++oi) {
            // split the patch along its folds of this axis (each piece is a
            // single-valued graph over the other two axes), then clip every
            // piece in that projection
            const int a = order[oi], b = (a + 1) % 3, cc = (a + 2) % 3;
            int chord[2][2], nch = 0;
            for (int k = 0; k < lfo.nfold[a]; ++k) {
                int i0 = -1, i1 = -1;
                for (int i = 0; i < m; ++i)
                    if (code[i] >= kCodeFace) {
                        const int64_t id = L.fpid[(size_t)(code[i] - kCodeFace)];
                        if (id == lfo.end_id[a][k][0]) i0 = i;
                        if (id == lfo.end_id[a][k][1]) i1 = i;
                    }
                if (i0 >= 0 && i1 >= 0) {
                    chord[nch][0] = i0;
                    chord[nch][1] = i1;
                    ++nch;
                }
            }
            // pieces as index lists; a chord splits the piece holding both ends
            // (at most two folds per axis: at most three pieces, each no longer
            // than the loop)
            Piece pieces[3];
            int npc = 1;
            pieces[0].n = m;
            for (int i = 0; i < m; ++i) pieces[0].v[i] = i;
            bool split_ok = true;
            for (int k = 0; k < nch && split_ok; ++k) {
                bool done = false;
                for (int pi = 0; pi < npc && !done; ++pi) {
                    Piece &pc = pieces[pi];
                    int x0 = -1, x1 = -1;
                    for (int i = 0; i < pc.n; ++i) {
                        if (pc.v[i] == chord[k][0]) x0 = i;
                        if (pc.v[i] == chord[k][1]) x1 = i;
                    }
                    if (x0 < 0 || x1 < 0) continue;
                    if (x1 < x0) std::swap(x0, x1);
                    if (x1 - x0 < 2 || (x0 == 0 && x1 == pc.n - 1)) {
                        split_ok = false;  // the ends are neighbours: nothing to split
                        break;
                    }
                    Piece &p2 = pieces[npc++];
                    p2.n = 0;
                    for (int i = x1; i != x0; i = (i + 1) % pc.n) p2.v[p2.n++] = pc.v[i];
                    p2.v[p2.n++] = pc.v[x0];
                    for (int i = x0; i <= x1; ++i) pc.v[i - x0] = pc.v[i];
                    pc.n = x1 - x0 + 1;
                    done = true;
                }
            }
            if (!split_ok) continue;
            ntl = 0;
            ok = true;
            for (int pi = 0; pi < npc; ++pi) {
                if (!clip_piece(P, fm, pieces[pi].v, pieces[pi].n, chord, nch, a, tl, &ntl)) {
                    ok = false;
                    break;
                }
            }
        }
        int inner = -1;
        if (!ok) {
            // single valued along no axis even between folds: a fan from a
            // point of the patch inside the cube, the loop's centroid moved
            // onto g = c (else from the loop's first point)
            ntl = 0;
            double u[3] = {ctr[0], ctr[1], ctr[2]};
            if (onto_surface(f, c, u)) {
                inner = (int)L.inner.size();
                L.inner.push_back({u[0], u[1], u[2]});
                for (int a = 0; a < 3; ++a) P[m][a] = u[a];
                for (int i = 0; i < m; ++i) tl[ntl++] = {m, i, (i + 1) % m};
            } else {
                for (int i = 1; i + 1 < m; ++i) tl[ntl++] = {0, i, i + 1};
            }
            ++L.fallback;
        }
        // orientation: sum over the triangles of n . (-grad g) at their centroids
        double score = 0.0;
        for (int k = 0; k < ntl; ++k) {
            const auto &t = tl[k];
            const double *pp = P[t[0]], *qq = P[t[1]], *rr = P[t[2]];
            const double u1[3] = {qq[0] - pp[0], qq[1] - pp[1], qq[2] - pp[2]};
            const double u2[3] = {rr[0] - pp[0], rr[1] - pp[1], rr[2] - pp[2]};
            const double n[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                                 u1[0] * u2[1] - u1[1] * u2[0]};
            const double cen[3] = {(pp[0] + qq[0] + rr[0]) / 3, (pp[1] + qq[1] + rr[1]) / 3,
                                   (pp[2] + qq[2] + rr[2]) / 3};
            double G[3];
            grad_g(f, cen, G);
            score -= n[0] * G[0] + n[1] * G[1] + n[2] * G[2];
        }
        const bool flip = score < 0.0;
        auto id = [&](int k) { return k < m ? code[k] : 12 + inner; };
        for (int k = 0; k < ntl; ++k) {
            const auto &t = tl[k];
            if (flip) L.tri.push_back({id(t[0]), id(t[2]), id(t[1])});
            else L.tri.push_back({id(t[0]), id(t[1]), id(t[2])});
        }
    }
}

uint64_t edge_key(int conf, int level, int K, int32_t ix, int32_t iy, int32_t iz, int e) {
    const EdgeInfo &E = topo().E[e];
    const int sh = K - level;
    const uint64_t X = (uint64_t)((int64_t)(ix + E.off[0]) << sh);
    const uint64_t Y = (uint64_t)((int64_t)(iy + E.off[1]) << sh);
    const uint64_t Z = (uint64_t)((int64_t)(iz + E.off[2]) << sh);
    return ((uint64_t)(uint32_t)conf << 53) | ((uint64_t)level << 50) | ((uint64_t)E.axis << 48) |
           (X << 32) | (Y << 16) | Z;
}

template <typename F>
void parallel_for(int64_t n, F fn) {
    unsigned nt = std::max(1u, std::thread::hardware_concurrency());
    nt = (unsigned)std::min<int64_t>(nt, std::max<int64_t>(1, n / 1024));
    if (nt <= 1) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t b = n * t / nt, e = n * (t + 1) / nt;
        th.emplace_back([=, &fn] { fn(b, e, (int)t); });
    }
    for (auto &x : th) x.join();
}


// sorts v with cmp: chunks sorted on threads, then merged pairwise
template <typename T, typename C>
void parallel_sort(std::vector<T> &v, C cmp) {
    const int64_t n = (int64_t)v.size();
    unsigned nt = std::max(1u, std::thread::hardware_concurrency());
    nt = (unsigned)std::min<int64_t>(nt, std::max<int64_t>(1, n / 65536));
    if (nt <= 1) {
        std::sort(v.begin(), v.end(), cmp);
        return;
    }
    std::vector<int64_t> cut(nt + 1);
    for (unsigned t = 0; t <= nt; ++t) cut[t] = n * t / nt;
    {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t] { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1], cmp); });
        for (auto &x : th) x.join();
    }
    for (unsigned w = 1; w < nt; w *= 2) {
        std::vector<std::thread> th;
        for (unsigned t = 0; t + w < nt; t += 2 * w) {
            const int64_t b = cut[t], mid = cut[t + w], e = cut[std::min(t + 2 * w, nt)];
            th.emplace_back([&, b, mid, e] {
                std::inplace_merge(v.begin() + b, v.begin() + mid, v.begin() + e, cmp);
            });
        }
        for (auto &x : th) x.join();
    }
}
// ---- triangle-triangle intersection (Moller's interval overlap test) -------
void sub3(const double *a, const double *b, double *r) {
    r[0] = a[0] - b[0];
    r[1] = a[1] - b[1];
    r[2] = a[2] - b[2];
}
void crs3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// ---- exact orientation signs -------------------------------------------------
// Knuth's two-sum and the two-product by FMA are error-free; an expansion, a
// sum of nonoverlapping doubles kept smallest first (Shewchuk, "Adaptive
// precision floating-point arithmetic and fast robust geometric predicates",
// 1997), holds a sum or product of doubles exactly, and its sign is that of
// its last component.  A determinant is evaluated in doubles first; when its
// magnitude does not clear a generous bound on the rounding error (1e-14 of
// the sum of the magnitudes of its terms; the error is below 2e-15 of it),
// it is evaluated exactly.

inline void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bv = s - a;
    e = (a - (s - bv)) + (b - bv);
}

inline void two_prod(double a, double b, double &p, double &e) {
    p = a * b;
    e = std::fma(a, b, -p);
}

// h += b exactly (h nonoverlapping, smallest first, no zero components)
void grow(std::vector<double> &h, double b) {
    double q = b;
    size_t k = 0;
    for (size_t i = 0; i < h.size(); ++i) {
        double sum, err;
        two_sum(q, h[i], sum, err);
        if (err != 0.0) h[k++] = err;
        q = sum;
    }
    h.resize(k);
    if (q != 0.0) h.push_back(q);
}

int expansion_sign(const std::vector<double> &h) {
    return h.empty() ? 0 : (h.back() > 0.0 ? 1 : -1);
}

// h += sg x y z exactly (sg = +-1)
void add_prod3(std::vector<double> &h, double x, double y, double z, double sg) {
    if (x == 0.0 || y == 0.0 || z == 0.0) return;
    double p, e, p1, e1;
    two_prod(x, y, p, e);
    two_prod(p, z, p1, e1);
    grow(h, sg * p1);
    grow(h, sg * e1);
    if (e != 0.0) {
        two_prod(e, z, p1, e1);
        grow(h, sg * p1);
        grow(h, sg * e1);
    }
}

// sign of det[a - d; b - d; c - d] (positive when d lies below the plane of a,
// b, c seen with a, b, c counter-clockwise), exactly
int orient3d_exact(const double *a, const double *b, const double *c, const double *d) {
    double A[3][2], B[3][2], C[3][2];  // the differences, each as two doubles
    for (int i = 0; i < 3; ++i) {
        two_sum(a[i], -d[i], A[i][0], A[i][1]);
        two_sum(b[i], -d[i], B[i][0], B[i][1]);
        two_sum(c[i], -d[i], C[i][0], C[i][1]);
    }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}, {1, 0, 2}, {2, 0, 1}, {2, 1, 0}};
    static const double sgn[6] = {1.0, -1.0, 1.0, -1.0, 1.0, -1.0};
    std::vector<double> h;
    h.reserve(64);
    for (int t = 0; t < 6; ++t)
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v)
                for (int w = 0; w < 2; ++w)
                    add_prod3(h, A[perm[t][0]][u], B[perm[t][1]][v], C[perm[t][2]][w], sgn[t]);
    return expansion_sign(h);
}

int orient3d(const double *a, const double *b, const double *c, const double *d) {
    const double ax = a[0] - d[0], ay = a[1] - d[1], az = a[2] - d[2];
    const double bx = b[0] - d[0], by = b[1] - d[1], bz = b[2] - d[2];
    const double cx = c[0] - d[0], cy = c[1] - d[1], cz = c[2] - d[2];
    const double det = ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
    const double mag = std::fabs(ax) * (std::fabs(by * cz) + std::fabs(bz * cy)) +
                       std::fabs(ay) * (std::fabs(bz * cx) + std::fabs(bx * cz)) +
                       std::fabs(az) * (std::fabs(bx * cy) + std::fabs(by * cx));
    if (det > 1e-14 * mag) return 1;
    if (det < -1e-14 * mag) return -1;
    return orient3d_exact(a, b, c, d);
}

// sign of det[a - c; b - c] in the plane, exactly
int orient2d(const double *a, const double *b, const double *c) {
    const double det = (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0]);
    const double mag = std::fabs((a[0] - c[0]) * (b[1] - c[1])) + std::fabs((a[1] - c[1]) * (b[0] - c[0]));
    if (det > 1e-14 * mag) return 1;
    if (det < -1e-14 * mag) return -1;
    double A[2][2], B[2][2];
    for (int i = 0; i < 2; ++i) {
        two_sum(a[i], -c[i], A[i][0], A[i][1]);
        two_sum(b[i], -c[i], B[i][0], B[i][1]);
    }
    std::vector<double> h;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            add_prod3(h, A[0][u], B[1][v], 1.0, 1.0);
            add_prod3(h, A[1][u], B[0][v], 1.0, -1.0);
        }
    return expansion_sign(h);
}

// ---- triangle pairs for condition (c) ----------------------------------------
// Closed triangles and segments; every decision is an exact orientation sign.

// r on the closed segment pq, given that the three are collinear
bool on_segment2(const double *p, const double *q, const double *r) {
    return std::min(p[0], q[0]) <= r[0] && r[0] <= std::max(p[0], q[0]) &&
           std::min(p[1], q[1]) <= r[1] && r[1] <= std::max(p[1], q[1]);
}

bool segments_meet2(const double *p, const double *q, const double *r, const double *s) {
    const int o1 = orient2d(p, q, r), o2 = orient2d(p, q, s), o3 = orient2d(r, s, p),
              o4 = orient2d(r, s, q);
    if (o1 * o2 < 0 && o3 * o4 < 0) return true;
    return (o1 == 0 && on_segment2(p, q, r)) || (o2 == 0 && on_segment2(p, q, s)) ||
           (o3 == 0 && on_segment2(r, s, p)) || (o4 == 0 && on_segment2(r, s, q));
}

bool in_triangle2(const double *p, const double *a, const double *b, const double *c) {
    const int c1 = orient2d(a, b, p), c2 = orient2d(b, c, p), c3 = orient2d(c, a, p);
    return (c1 >= 0 && c2 >= 0 && c3 >= 0) || (c1 <= 0 && c2 <= 0 && c3 <= 0);
}

// does the closed segment pq meet the closed triangle abc?
bool segment_meets_triangle(const double *p, const double *q, const double *a, const double *b,
                            const double *c) {
    const int op = orient3d(a, b, c, p), oq = orient3d(a, b, c, q);
    if (op * oq > 0) return false;
    if (op == 0 && oq == 0) {
        // in the triangle's plane: in the coordinate plane where its normal
        // is largest (the projection keeps every orientation)
        double E1[3], E2[3], N[3];
        sub3(b, a, E1);
        sub3(c, a, E2);
        crs3(E1, E2, N);
        const int drop = (std::fabs(N[0]) >= std::fabs(N[1]) && std::fabs(N[0]) >= std::fabs(N[2]))
                             ? 0 : (std::fabs(N[1]) >= std::fabs(N[2]) ? 1 : 2);
        const int i0 = drop == 0 ? 1 : 0, i1 = drop == 2 ? 1 : 2;
        const double P[2] = {p[i0], p[i1]}, Q[2] = {q[i0], q[i1]}, A[2] = {a[i0], a[i1]},
                     B[2] = {b[i0], b[i1]}, C[2] = {c[i0], c[i1]};
        return in_triangle2(P, A, B, C) || in_triangle2(Q, A, B, C) ||
               segments_meet2(P, Q, A, B) || segments_meet2(P, Q, B, C) ||
               segments_meet2(P, Q, C, A);
    }
    // pq crosses the plane (or ends on it): the crossing is in the triangle
    // iff pq passes every directed edge on the same side
    const int s1 = orient3d(p, q, a, b), s2 = orient3d(p, q, b, c), s3 = orient3d(p, q, c, a);
    return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

// two closed triangles meet iff an edge of one meets the other
bool triangles_meet(const double *V0, const double *V1, const double *V2, const double *U0,
                    const double *U1, const double *U2) {
    const double *V[3] = {V0, V1, V2}, *U[3] = {U0, U1, U2};
    for (int k = 0; k < 3; ++k)
        if (segment_meets_triangle(V[k], V[(k + 1) % 3], U0, U1, U2) ||
            segment_meets_triangle(U[k], U[(k + 1) % 3], V0, V1, V2))
            return true;
    return false;
}

// A quick test in doubles that can only err towards "meet" (distances to the
// planes within 1e-9 of the coordinate scale count as on the plane, the
// intervals on the line of the planes' intersection get the same slack, and
// coplanar pairs pass); what it passes, triangles_meet decides.
bool may_meet(const double *V0, const double *V1, const double *V2, const double *U0,
              const double *U1, const double *U2) {
    double scale = 1.0;
    for (const double *P : {V0, V1, V2, U0, U1, U2})
        for (int i = 0; i < 3; ++i) scale = std::max(scale, std::fabs(P[i]));
    double E1[3], E2[3], N1[3], N2[3];
    sub3(V1, V0, E1);
    sub3(V2, V0, E2);
    crs3(E1, E2, N1);
    const double d1 = -dot3(N1, V0);
    double du0 = dot3(N1, U0) + d1, du1 = dot3(N1, U1) + d1, du2 = dot3(N1, U2) + d1;
    const double eps = 1e-9 * scale * std::sqrt(dot3(N1, N1));
    if (std::fabs(du0) <= eps) du0 = 0;
    if (std::fabs(du1) <= eps) du1 = 0;
    if (std::fabs(du2) <= eps) du2 = 0;
    if ((du0 > 0 && du1 > 0 && du2 > 0) || (du0 < 0 && du1 < 0 && du2 < 0)) return false;
    sub3(U1, U0, E1);
    sub3(U2, U0, E2);
    crs3(E1, E2, N2);
    const double d2 = -dot3(N2, U0);
    double dv0 = dot3(N2, V0) + d2, dv1 = dot3(N2, V1) + d2, dv2 = dot3(N2, V2) + d2;
    const double eps2 = 1e-9 * scale * std::sqrt(dot3(N2, N2));
    if (std::fabs(dv0) <= eps2) dv0 = 0;
    if (std::fabs(dv1) <= eps2) dv1 = 0;
    if (std::fabs(dv2) <= eps2) dv2 = 0;
    if ((dv0 > 0 && dv1 > 0 && dv2 > 0) || (dv0 < 0 && dv1 < 0 && dv2 < 0)) return false;
    if ((du0 == 0 && du1 == 0 && du2 == 0) || (dv0 == 0 && dv1 == 0 && dv2 == 0)) return true;
    double D[3];
    crs3(N1, N2, D);
    int ax = 0;
    if (std::fabs(D[1]) > std::fabs(D[ax])) ax = 1;
    if (std::fabs(D[2]) > std::fabs(D[ax])) ax = 2;
    // interval of a triangle on the line: the vertex alone on its side and
    // the two crossings of its edges to the others
    auto interval = [&](const double *P0, const double *P1, const double *P2, double d0, double dd1,
                        double dd2, double &lo, double &hi) {
        const double p0 = P0[ax], p1 = P1[ax], p2 = P2[ax];
        double a, b, c, da, db, dc;
        if (d0 * dd1 > 0) { a = p2; b = p0; c = p1; da = dd2; db = d0; dc = dd1; }
        else if (d0 * dd2 > 0) { a = p1; b = p0; c = p2; da = dd1; db = d0; dc = dd2; }
        else if (dd1 * dd2 > 0 || d0 != 0) { a = p0; b = p1; c = p2; da = d0; db = dd1; dc = dd2; }
        else if (dd1 != 0) { a = p1; b = p0; c = p2; da = dd1; db = d0; dc = dd2; }
        else { a = p2; b = p0; c = p1; da = dd2; db = d0; dc = dd1; }
        const double t1 = a + (b - a) * da / (da - db), t2 = a + (c - a) * da / (da - dc);
        lo = std::min(t1, t2);
        hi = std::max(t1, t2);
    };
    double a0, a1, b0, b1;
    interval(V0, V1, V2, dv0, dv1, dv2, a0, a1);
    interval(U0, U1, U2, du0, du1, du2, b0, b1);
    const double slack = 1e-9 * scale;
    return !(a1 < b0 - slack || b1 < a0 - slack);
}

// ---- building the mesh ------------------------------------------------------
// Vertex ids: the caller's edge points in key order (0 .. nv-1), then points
// appended later (interior points of fanned patches, edge points of added
// cubes).  Every SURFACE leaf ORs its position around each of its crossing
// edges into that edge point's ring bits: around an edge, the cube at offsets
// (u, v) along the edge's two other axes (ascending) is bit u + 2 v (the
// edge's index & 3 within that cube).  A crossing edge crosses every face
// that contains it, so a present cube whose ring neighbour across such a face
// is absent has an open face there; with no open face every ring is full.

using VidFn = std::function<int64_t(uint64_t)>;
using KeyFn = std::function<uint64_t(int64_t)>;

// Vertex ids by edge key: the caller's points in ascending key order (ids
// 0 .. nv-1), then points appended later (edge points of added cubes), found
// through a map.
struct VIndex {
    const std::vector<tms_vertex> *V = nullptr;
    std::unordered_map<uint64_t, int64_t> id;   // appended points: key -> id
    std::unordered_map<int64_t, uint64_t> key;  // and id -> key
    int64_t nv() const { return (int64_t)V->size(); }
    int64_t find(uint64_t k) const {
        auto it = std::lower_bound(V->begin(), V->end(), k,
                                   [](const tms_vertex &a, uint64_t kk) { return a.edge_key < kk; });
        if (it != V->end() && it->edge_key == k) return (int64_t)(it - V->begin());
        auto jt = id.find(k);
        return jt == id.end() ? -1 : jt->second;
    }
    uint64_t key_of(int64_t v) const { return v < nv() ? (*V)[(size_t)v].edge_key : key.at(v); }
    void add(uint64_t k, int64_t v) {
        id.emplace(k, v);
        key.emplace(v, k);
    }
};

// host copy only: a coarser SURFACE leaf meshed through its finest sub-cubes
constexpr uint8_t kClsSplit = 0xFE;

uint64_t cube_key(int64_t x, int64_t y, int64_t z) {
    return ((uint64_t)(x & 0x1FFFFF) << 42) | ((uint64_t)(y & 0x1FFFFF) << 21) |
           (uint64_t)(z & 0x1FFFFF);
}

// Face points (eq. curve): the ends of every SURFACE leaf's folds, on its two
// faces normal to the fold's axis.  Both leaves that share a face put the
// points of both into their loops (Section 2.3 joins a cube's points with
// those of its neighbours on the shared faces), so their face curves have
// the same vertices.  Sorted by face, then (u, v); ids follow the points so
// far, positions placed from an edge point of the leaf that made them.
struct FaceRec {
    uint64_t key;  // face: normal axis, lattice coordinates of its lower corner
    double u, v;
    int64_t id;
};

uint64_t face_key(int a, int64_t x, int64_t y, int64_t z) {
    return ((uint64_t)a << 62) | ((uint64_t)(x & 0xFFFFF) << 40) | ((uint64_t)(y & 0xFFFFF) << 20) |
           (uint64_t)(z & 0xFFFFF);
}

uint64_t leaf_face_key(const tms_leaf &lf, int fi) {
    const int a = fi >> 1;
    int64_t q[3] = {lf.ix, lf.iy, lf.iz};
    q[a] += fi & 1;
    return face_key(a, q[0], q[1], q[2]);
}

bool face_points(const std::vector<tms_leaf> &L, const std::vector<double> &cp,
                 const std::vector<int64_t> &idx, double c, int K, double h0, const VidFn &vid,
                 tms_mesh *M, std::vector<FaceRec> &FR) {
    const Topo &T = topo();
    const unsigned nth = std::max(1u, std::thread::hardware_concurrency());
    struct Rec {
        uint64_t key;
        double u, v, x[3];
    };
    std::vector<std::vector<Rec>> part(nth);
    std::atomic<int64_t> missing{0};
    parallel_for((int64_t)idx.size(), [&](int64_t b, int64_t e, int t) {
        for (int64_t s2 = b; s2 < e; ++s2) {
            const int64_t i = idx[(size_t)s2];
            const tms_leaf &lf = L[(size_t)i];
            const double *f = &cp[(size_t)i * 8];
            double m[8];
            monomials01(f, m);
            Fold fo[3][2];
            int nf[3], tot = 0;
            for (int a = 0; a < 3; ++a) tot += nf[a] = folds_along(m, c, a, fo[a]);
            if (!tot) continue;
            int e0 = -1;
            for (int ed = 0; ed < 12 && e0 < 0; ++ed)
                if ((f[T.E[ed].v0] >= c) != (f[T.E[ed].v1] >= c)) e0 = ed;
            const int64_t v0 = e0 < 0 ? -1 : vid(edge_key(lf.conf, lf.level, K, lf.ix, lf.iy, lf.iz, e0));
            if (v0 < 0) {
                ++missing;
                continue;
            }
            double P0[3];
            edge_point(f, c, e0, P0);
            const double h = std::ldexp(h0, -(int)lf.level);
            for (int a = 0; a < 3; ++a) {
                const int p = (a == 0) ? 1 : 0, q = (a == 2) ? 1 : 2;
                for (int k = 0; k < nf[a]; ++k)
                    for (int sd = 0; sd < 2; ++sd) {
                        Rec r;
                        r.key = leaf_face_key(lf, 2 * a + sd);
                        r.u = fo[a][k].u;
                        r.v = fo[a][k].v;
                        double loc[3];
                        loc[a] = (double)sd;
                        loc[p] = r.u;
                        loc[q] = r.v;
                        for (int d = 0; d < 3; ++d)
                            r.x[d] = M->xyz[3 * (size_t)v0 + d] + (loc[d] - P0[d]) * h;
                        part[(size_t)t].push_back(r);
                    }
            }
        }
    });
    if (missing.load()) return false;
    std::vector<Rec> all;
    for (auto &pp : part) all.insert(all.end(), pp.begin(), pp.end());
    std::sort(all.begin(), all.end(), [](const Rec &x, const Rec &y) {
        return x.key != y.key ? x.key < y.key : (x.u != y.u ? x.u < y.u : x.v < y.v);
    });
    FR.clear();
    for (const Rec &r : all) {
        // the same point made by both leaves of the face: their corner
        // orders differ, so the two solutions can differ in the last bits
        bool dup = false;
        for (size_t k = FR.size(); k-- > 0 && FR[k].key == r.key && r.u - FR[k].u <= kFaceMerge;)
            if (std::fabs(r.v - FR[k].v) <= kFaceMerge) dup = true;
        if (dup) continue;
        FR.push_back({r.key, r.u, r.v, (int64_t)(M->xyz.size() / 3)});
        M->xyz.insert(M->xyz.end(), r.x, r.x + 3);
    }
    return true;
}

// the face points of face fi of a leaf (a range of FR)
void face_range(const std::vector<FaceRec> &FR, uint64_t key, const FaceRec **b, int *n) {
    auto lo = std::lower_bound(FR.begin(), FR.end(), key,
                               [](const FaceRec &r, uint64_t k) { return r.key < k; });
    auto hi = lo;
    while (hi != FR.end() && hi->key == key) ++hi;
    *b = lo == hi ? nullptr : &*lo;
    *n = (int)(hi - lo);
}

// Ring bits of the leaves idx (their crossing edges); false if an edge point
// is missing.
bool ring_pass(const std::vector<tms_leaf> &L, const std::vector<double> &cp,
               const std::vector<int64_t> &idx, double c, int K, const VidFn &vid,
               std::vector<uint8_t> &em) {
    const Topo &T = topo();
    std::atomic<int64_t> missing{0};
    parallel_for((int64_t)idx.size(), [&](int64_t b, int64_t e, int) {
        for (int64_t s2 = b; s2 < e; ++s2) {
            const int64_t i = idx[(size_t)s2];
            const tms_leaf &lf = L[(size_t)i];
            const double *f = &cp[(size_t)i * 8];
            for (int ed = 0; ed < 12; ++ed) {
                if ((f[T.E[ed].v0] >= c) == (f[T.E[ed].v1] >= c)) continue;
                const int64_t id = vid(edge_key(lf.conf, lf.level, K, lf.ix, lf.iy, lf.iz, ed));
                if (id < 0) {
                    ++missing;
                    continue;
                }
                __atomic_fetch_or(&em[(size_t)id], (uint8_t)(1u << (ed & 3)), __ATOMIC_RELAXED);
            }
        }
    });
    return missing.load() == 0;
}

// Triangulates the leaves idx into M (triangles, then interior points
// appended in the order of idx), each with the face points of FR on its
// faces and its own folds.  Returns false if an edge point is missing.
bool triangulate(const std::vector<tms_leaf> &L, const std::vector<double> &cp,
                 const std::vector<int64_t> &idx, double c, int K, double h0, const VidFn &vid,
                 const std::vector<FaceRec> &FR, tms_mesh *M) {
    const Topo &T = topo();
    const int64_t ns = (int64_t)idx.size();
    const unsigned nth = std::max(1u, std::thread::hardware_concurrency());
    std::vector<std::vector<int32_t>> ptri(nth), pleaf(nth);
    std::vector<std::vector<double>> pxyz(nth);  // interior points of fanned loops
    std::vector<int64_t> loops(nth, 0), fb(nth, 0), missing(nth, 0);
    std::vector<int64_t> first(nth, -1);  // chunk starts, merged in order afterwards
    parallel_for(ns, [&](int64_t b, int64_t e, int t) {
        first[(size_t)t] = b;
        LeafOut out;
        std::vector<FacePt> fpbuf;
        for (int64_t s2 = b; s2 < e; ++s2) {
            const int64_t i = idx[(size_t)s2];
            const tms_leaf &lf = L[(size_t)i];
            const double *f = &cp[(size_t)i * 8];
            int64_t id[12];
            bool ok = true;
            for (int ed = 0; ed < 12; ++ed) {
                id[ed] = -1;
                if ((f[T.E[ed].v0] >= c) == (f[T.E[ed].v1] >= c)) continue;
                id[ed] = vid(edge_key(lf.conf, lf.level, K, lf.ix, lf.iy, lf.iz, ed));
                if (id[ed] < 0) ok = false;
            }
            if (!ok) {
                ++missing[(size_t)t];
                continue;
            }
            // the points on its faces and its own folds with their ends' ids
            LeafFolds lfo;
            fpbuf.clear();
            if (!FR.empty()) {
                int start[6];
                for (int fi = 0; fi < 6; ++fi) {
                    const FaceRec *r;
                    int n;
                    face_range(FR, leaf_face_key(lf, fi), &r, &n);
                    start[fi] = (int)fpbuf.size();
                    for (int k = 0; k < n; ++k) fpbuf.push_back({r[k].u, r[k].v, r[k].id});
                    lfo.nfp[fi] = n;
                }
                for (int fi = 0; fi < 6; ++fi) lfo.fp[fi] = fpbuf.data() + start[fi];
                double m[8];
                monomials01(f, m);
                for (int a = 0; a < 3; ++a) {
                    lfo.nfold[a] = folds_along(m, c, a, lfo.fold[a]);
                    for (int k = 0; k < lfo.nfold[a]; ++k)
                        for (int sd = 0; sd < 2; ++sd) {
                            lfo.end_id[a][k][sd] = -1;
                            const int fi = 2 * a + sd;
                            for (int z = 0; z < lfo.nfp[fi]; ++z)
                                if (std::fabs(lfo.fp[fi][z].u - lfo.fold[a][k].u) <= kFaceMerge &&
                                    std::fabs(lfo.fp[fi][z].v - lfo.fold[a][k].v) <= kFaceMerge)
                                    lfo.end_id[a][k][sd] = lfo.fp[fi][z].id;
                        }
                }
            }
            out.tri.clear();
            out.inner.clear();
            out.loops = out.fallback = 0;
            leaf_triangles(f, c, lfo, out);
            loops[(size_t)t] += out.loops;
            fb[(size_t)t] += out.fallback;
            // interior points: placed from an edge point of the leaf (its
            // global position minus its local one) -- numbered -1 - k in the
            // thread, renumbered after the merge
            std::vector<int32_t> inner_id(out.inner.size(), 0);
            if (!out.inner.empty()) {
                int e0 = -1;
                for (const auto &tr : out.tri)
                    for (int k = 0; k < 3 && e0 < 0; ++k)
                        if (tr[k] < 12) e0 = tr[k];
                if (e0 < 0) {
                    ++missing[(size_t)t];
                    continue;
                }
                double P0[3];
                edge_point(f, c, e0, P0);
                const double h = std::ldexp(h0, -(int)lf.level);
                for (size_t k = 0; k < out.inner.size(); ++k) {
                    inner_id[k] = -1 - (int32_t)(pxyz[(size_t)t].size() / 3);
                    for (int a = 0; a < 3; ++a)
                        pxyz[(size_t)t].push_back(M->xyz[3 * (size_t)id[e0] + a] +
                                                  (out.inner[k][a] - P0[a]) * h);
                }
            }
            for (const auto &tr : out.tri) {
                int32_t v[3];
                for (int k = 0; k < 3; ++k) {
                    const int cd = tr[k];
                    v[k] = cd < 12 ? (int32_t)id[cd]
                           : cd < kCodeFace ? inner_id[(size_t)(cd - 12)]
                                            : (int32_t)out.fpid[(size_t)(cd - kCodeFace)];
                }
                ptri[(size_t)t].insert(ptri[(size_t)t].end(), v, v + 3);
                pleaf[(size_t)t].push_back((int32_t)i);
            }
        }
    });
    std::vector<int> order;
    for (unsigned t = 0; t < nth; ++t)
        if (first[t] >= 0) order.push_back((int)t);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return first[a] < first[b]; });
    int64_t miss = 0;
    for (int t : order) {
        // interior points of this thread's leaves follow the points so far
        const int32_t base = (int32_t)(M->xyz.size() / 3);
        for (int32_t &v : ptri[(size_t)t])
            if (v < 0) v = base + (-1 - v);
        M->xyz.insert(M->xyz.end(), pxyz[(size_t)t].begin(), pxyz[(size_t)t].end());
        M->tri.insert(M->tri.end(), ptri[(size_t)t].begin(), ptri[(size_t)t].end());
        M->tri_leaf.insert(M->tri_leaf.end(), pleaf[(size_t)t].begin(), pleaf[(size_t)t].end());
        M->n_loops += loops[(size_t)t];
        M->n_fallback += fb[(size_t)t];
        miss += missing[(size_t)t];
    }
    return miss == 0;
}

// Open faces seen from the rings of the vertex ids `ids` (all ids when
// null): the number of distinct (cube, face) pairs, and the cubes across
// them (sorted, distinct) when `across` is given.
int64_t open_faces(const std::vector<uint8_t> &em, const std::vector<int64_t> *ids, int64_t nall,
                   const KeyFn &key_of, int K, std::vector<std::array<int32_t, 3>> *across) {
    const int64_t n = ids ? (int64_t)ids->size() : nall;
    const unsigned nth = std::max(1u, std::thread::hardware_concurrency());
    std::vector<std::vector<std::array<int32_t, 4>>> part(nth);  // cube, face
    parallel_for(n, [&](int64_t b, int64_t e, int t) {
        for (int64_t s = b; s < e; ++s) {
            const int64_t v = ids ? (*ids)[(size_t)s] : s;
            const unsigned m = em[(size_t)v];
            if (m == 0 || m == 0xF) continue;
            const uint64_t key = key_of(v);
            const int level = (int)((key >> 50) & 7), axis = (int)((key >> 48) & 3),
                      sh = K - level;
            const int32_t E[3] = {(int32_t)(((key >> 32) & 0xFFFF) >> sh),
                                  (int32_t)(((key >> 16) & 0xFFFF) >> sh),
                                  (int32_t)((key & 0xFFFF) >> sh)};
            const int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
            const int lo = std::min(o1, o2), hi = std::max(o1, o2);
            for (int p = 0; p < 4; ++p) {
                if (!((m >> p) & 1)) continue;
                const int u = p & 1, w = p >> 1;
                std::array<int32_t, 4> q = {E[0], E[1], E[2], 0};
                q[lo] -= u;
                q[hi] -= w;
                if (!((m >> (p ^ 1)) & 1)) {  // across the face normal to lo
                    q[3] = 2 * lo + u;
                    part[(size_t)t].push_back(q);
                }
                if (!((m >> (p ^ 2)) & 1)) {  // across the face normal to hi
                    q[3] = 2 * hi + w;
                    part[(size_t)t].push_back(q);
                }
            }
        }
    });
    std::vector<std::array<int32_t, 4>> all;
    for (auto &p : part) all.insert(all.end(), p.begin(), p.end());
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    if (across) {
        across->clear();
        for (const auto &q : all) {
            std::array<int32_t, 3> r = {q[0], q[1], q[2]};
            r[q[3] >> 1] += (q[3] & 1) ? 1 : -1;
            across->push_back(r);
        }
        std::sort(across->begin(), across->end());
        across->erase(std::unique(across->begin(), across->end()), across->end());
    }
    return (int64_t)all.size();
}

// the edge point of key `key` on a leaf's edge, moved off a corner as the
// caller's points are (t clamped to [kTmin, 1 - kTmin])
void place_vertex(uint64_t key, double t, double px, double py, double pz, double h0,
                  double out[3]) {
    out[0] = px;
    out[1] = py;
    out[2] = pz;
    const double tc = clamp_t(t);
    if (tc != t) {
        const int level = (int)((key >> 50) & 7), axis = (int)((key >> 48) & 3);
        out[axis] += (tc - t) * std::ldexp(h0, -level);
    }
}

// The mesh of host copies of the leaves, corner values and vertices, in two
// steps around the closing of open faces: prepare_mesh checks the inputs,
// places the points (the caller's, then X) and sets the ring bits of the
// SURFACE leaves; finish_mesh adds the face points of every SURFACE leaf
// and triangulates them all.  Each returns a message (empty: success).
std::string prepare_mesh(const std::vector<tms_leaf> &L, const std::vector<double> &cp,
                         const std::vector<tms_vertex> &V, const std::vector<tms_vertex> &X,
                         VIndex &VI, double c, int K, double h0, tms_mesh **out,
                         std::vector<uint8_t> &em) {
    *out = nullptr;
    const int64_t n = (int64_t)L.size(), nv = (int64_t)V.size();
    VI.V = &V;
    if (n >= (int64_t)0x7FFFFFFF || nv >= (int64_t)0x7FFFFFFF)
        return "too many leaves or vertices for 32-bit indices";
    std::atomic<bool> sorted{true};
    parallel_for(nv - 1, [&](int64_t b, int64_t e, int) {
        for (int64_t k = b; k < e; ++k)
            if (!(V[(size_t)k].edge_key < V[(size_t)k + 1].edge_key)) sorted = false;
    });
    if (!sorted) return "vertices must come in ascending edge-key order";
    auto *M = new tms_mesh();
    std::vector<int64_t> surf;
    for (int64_t i = 0; i < n; ++i)
        if (L[(size_t)i].cls == TMS_CLS_SURFACE) surf.push_back(i);
    M->n_surface = (int64_t)surf.size();
    M->level = surf.empty() ? K : L[(size_t)surf[0]].level;
    for (int64_t i : surf)
        if (L[(size_t)i].level != M->level || L[(size_t)i].level > K) {
            delete M;
            return "SURFACE leaves of different levels: faces between cubes of different sizes "
                   "(T-junctions) are not meshed";
        }
    M->leaf_ijk.resize((size_t)n * 3);
    M->xyz.resize((size_t)(nv + (int64_t)X.size()) * 3);
    parallel_for(n, [&](int64_t b, int64_t e, int) {
        for (int64_t i = b; i < e; ++i) {
            M->leaf_ijk[3 * i] = L[(size_t)i].ix;
            M->leaf_ijk[3 * i + 1] = L[(size_t)i].iy;
            M->leaf_ijk[3 * i + 2] = L[(size_t)i].iz;
        }
    });
    parallel_for(nv, [&](int64_t b, int64_t e, int) {
        for (int64_t k = b; k < e; ++k) {
            const tms_vertex &v = V[(size_t)k];
            place_vertex(v.edge_key, v.t, v.x, v.y, v.z, h0, &M->xyz[3 * (size_t)k]);
        }
    });
    // appended points (edge points of cubes that replace coarser leaves)
    for (size_t k = 0; k < X.size(); ++k) {
        const tms_vertex &v = X[k];
        place_vertex(v.edge_key, v.t, v.x, v.y, v.z, h0, &M->xyz[3 * ((size_t)nv + k)]);
        VI.add(v.edge_key, nv + (int64_t)k);
    }
    em.assign((size_t)(nv + (int64_t)X.size()), 0);
    if (!ring_pass(L, cp, surf, c, K, [&](uint64_t key) { return VI.find(key); }, em)) {
        delete M;
        return "a leaf's edge point is missing from the vertex list (vertices of other leaves?)";
    }
    M->open_faces = open_faces(em, nullptr, (int64_t)em.size(),
                               [&](int64_t v) { return VI.key_of(v); }, K, nullptr);
    *out = M;
    return std::string();
}

std::string finish_mesh(const std::vector<tms_leaf> &L, const std::vector<double> &cp,
                        const VIndex &VI, double c, int K, double h0, tms_mesh *M) {
    std::vector<int64_t> surf;
    for (int64_t i = 0; i < (int64_t)L.size(); ++i)
        if (L[(size_t)i].cls == TMS_CLS_SURFACE) surf.push_back(i);
    const VidFn vid = [&](uint64_t key) { return VI.find(key); };
    std::vector<FaceRec> FR;
    if (!face_points(L, cp, surf, c, K, h0, vid, M, FR) ||
        !triangulate(L, cp, surf, c, K, h0, vid, FR, M))
        return "a leaf's edge point is missing from the vertex list (vertices of other leaves?)";
    M->n_face_points = (int64_t)FR.size();
    return std::string();
}

// phi of the library (as tms_eval_phi, the precision of `cells`) of
// conformation conf at host points pts [m][3]; on failure *rc and a message
std::string eval_points(tms_ctx *ctx, const tms_cells *cells, int conf,
                        const std::vector<double> &pts, std::vector<double> &phi, DevBuf &dpts,
                        DevBuf &dphi, int32_t *rc) {
    const int64_t m = (int64_t)(pts.size() / 3);
    phi.assign((size_t)m, 0.0);
    if (m == 0) return std::string();
    if (dpts.ensure(sizeof(double) * pts.size()) != hipSuccess ||
        dphi.ensure(sizeof(double) * (size_t)m) != hipSuccess) {
        (void)hipGetLastError();
        *rc = TMS_E_OOM;
        return "device memory for the corner values of cubes added to the mesh";
    }
    if (hipMemcpyAsync(dpts.p, pts.data(), sizeof(double) * pts.size(), hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        *rc = TMS_E_DEVICE;
        return "copying the corners of cubes added to the mesh to the device";
    }
    const int32_t e = tms::eval_phi_conf(ctx, cells, conf, dpts.as<double>(), m, dphi.as<double>());
    if (e != TMS_OK) {
        *rc = e;
        return ctx->err;
    }
    if (hipMemcpyAsync(phi.data(), dphi.p, sizeof(double) * (size_t)m, hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        *rc = TMS_E_DEVICE;
        return "copying the corner values of cubes added to the mesh to the host";
    }
    return std::string();
}

// the edge point of a crossing edge e of the cube (ix, iy, iz) at `level`
// with corner values f, placed as the extraction places its points
tms_vertex new_vertex(const Grid &g, int conf, int level, int32_t ix, int32_t iy, int32_t iz,
                      int e, const double f[8]) {
    const EdgeInfo &E = topo().E[e];
    const int sh = g.K - level;
    const double h = std::ldexp(g.h0, -level);
    const double f0 = f[E.v0], f1 = f[E.v1];
    tms_vertex x;
    x.edge_key = edge_key(conf, level, g.K, ix, iy, iz, e);
    x.t = (g.c - f0) / (f1 - f0);
    const int64_t I[3] = {(int64_t)ix + E.off[0], (int64_t)iy + E.off[1], (int64_t)iz + E.off[2]};
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = g.o[a] + (double)(I[a] << sh) * g.hmin;
    p[E.axis] += x.t * h;
    x.x = p[0];
    x.y = p[1];
    x.z = p[2];
    return x;
}

// Coarser SURFACE leaves (device entry point).  With a loose tolerance a
// cube can meet the stopping rule (2E <= tau) above the finest level while
// its corner values straddle c; its faces would meet smaller cubes.  Each
// such leaf is meshed through the cubes of the finest level inside it whose
// corner values straddle c, added as SURFACE leaves (reason
// TMS_REASON_SPLIT): corner values from a SURFACE leaf of the finest level
// or from the coarse leaf itself wherever they have the same lattice point,
// else phi of the library; their edge points as the extraction places them
// (appended to X).  The coarse leaf is marked kClsSplit in the host copy;
// its own edge points stay in the vertex list, unused.
std::string split_coarse(tms_ctx *ctx, const tms_cells *cells, int conf, std::vector<tms_leaf> &L,
                         std::vector<double> &cp, const std::vector<tms_vertex> &V,
                         std::vector<tms_vertex> &X, int32_t *rc) {
    *rc = TMS_OK;
    const Grid &g = cells->gh[(size_t)conf];
    const int K = g.K;
    std::vector<int64_t> coarse;
    for (int64_t i = 0; i < (int64_t)L.size(); ++i)
        if (L[(size_t)i].cls == TMS_CLS_SURFACE && L[(size_t)i].level < K) coarse.push_back(i);
    if (coarse.empty()) return std::string();
    // lattice points of the finest level with a known value: the coarse
    // leaves' corners, and the corners of finest SURFACE leaves next to them
    std::unordered_map<uint64_t, double> val;
    std::unordered_set<uint64_t> halo;  // finest cubes within one cube of a coarse leaf
    for (int64_t i : coarse) {
        const tms_leaf &lf = L[(size_t)i];
        const int s = K - lf.level;
        const int64_t n = (int64_t)1 << s;
        const int64_t b[3] = {(int64_t)lf.ix << s, (int64_t)lf.iy << s, (int64_t)lf.iz << s};
        for (int v = 0; v < 8; ++v)
            val[cube_key(b[0] + (v & 1) * n, b[1] + ((v >> 1) & 1) * n, b[2] + ((v >> 2) & 1) * n)] =
                cp[(size_t)i * 8 + (size_t)v];
        for (int64_t z = -1; z <= n; ++z)
            for (int64_t y = -1; y <= n; ++y)
                for (int64_t x = -1; x <= n; ++x)
                    if (x < 0 || y < 0 || z < 0 || x == n || y == n || z == n)
                        halo.insert(cube_key(b[0] + x, b[1] + y, b[2] + z));
    }
    {
        const unsigned nth = std::max(1u, std::thread::hardware_concurrency());
        std::vector<std::vector<int64_t>> part(nth);
        parallel_for((int64_t)L.size(), [&](int64_t b, int64_t e, int t) {
            for (int64_t i = b; i < e; ++i) {
                const tms_leaf &lf = L[(size_t)i];
                if (lf.cls == TMS_CLS_SURFACE && lf.level == K &&
                    halo.count(cube_key(lf.ix, lf.iy, lf.iz)))
                    part[(size_t)t].push_back(i);
            }
        });
        for (auto &pp : part)
            for (int64_t i : pp) {
                const tms_leaf &lf = L[(size_t)i];
                for (int v = 0; v < 8; ++v)
                    val.emplace(cube_key(lf.ix + (v & 1), lf.iy + ((v >> 1) & 1), lf.iz + ((v >> 2) & 1)),
                                cp[(size_t)i * 8 + (size_t)v]);
            }
    }
    // every other lattice point inside the coarse leaves: phi
    std::vector<uint64_t> need;
    std::vector<double> pts;
    for (int64_t i : coarse) {
        const tms_leaf &lf = L[(size_t)i];
        const int s = K - lf.level;
        const int64_t n = (int64_t)1 << s;
        const int64_t b[3] = {(int64_t)lf.ix << s, (int64_t)lf.iy << s, (int64_t)lf.iz << s};
        for (int64_t z = 0; z <= n; ++z)
            for (int64_t y = 0; y <= n; ++y)
                for (int64_t x = 0; x <= n; ++x) {
                    const uint64_t k = cube_key(b[0] + x, b[1] + y, b[2] + z);
                    if (val.count(k)) continue;
                    val.emplace(k, 0.0);
                    need.push_back(k);
                    pts.push_back(g.o[0] + (double)(b[0] + x) * g.hmin);
                    pts.push_back(g.o[1] + (double)(b[1] + y) * g.hmin);
                    pts.push_back(g.o[2] + (double)(b[2] + z) * g.hmin);
                }
    }
    DevBuf dpts, dphi;
    std::vector<double> phi;
    const std::string why = eval_points(ctx, cells, conf, pts, phi, dpts, dphi, rc);
    if (*rc != TMS_OK) return why;
    for (size_t k = 0; k < need.size(); ++k) val[need[k]] = phi[k];
    // the straddling cubes of the finest level inside each coarse leaf
    const Topo &T = topo();
    std::unordered_set<uint64_t> seen;
    for (int64_t i : coarse) {
        const tms_leaf lc = L[(size_t)i];
        L[(size_t)i].cls = kClsSplit;
        const int s = K - lc.level;
        const int64_t n = (int64_t)1 << s;
        const int64_t b[3] = {(int64_t)lc.ix << s, (int64_t)lc.iy << s, (int64_t)lc.iz << s};
        for (int64_t z = 0; z < n; ++z)
            for (int64_t y = 0; y < n; ++y)
                for (int64_t x = 0; x < n; ++x) {
                    double f[8];
                    unsigned mask = 0;
                    for (int v = 0; v < 8; ++v) {
                        f[v] = val.at(cube_key(b[0] + x + (v & 1), b[1] + y + ((v >> 1) & 1),
                                               b[2] + z + ((v >> 2) & 1)));
                        if (f[v] >= g.c) mask |= 1u << v;
                    }
                    if (mask == 0 || mask == 0xFF) continue;
                    tms_leaf lf{};
                    lf.ix = (int32_t)(b[0] + x);
                    lf.iy = (int32_t)(b[1] + y);
                    lf.iz = (int32_t)(b[2] + z);
                    lf.conf = conf;
                    lf.level = (uint8_t)K;
                    lf.reason = TMS_REASON_SPLIT;
                    lf.mask = (uint8_t)mask;
                    lf.cls = TMS_CLS_SURFACE;
                    L.push_back(lf);
                    cp.insert(cp.end(), f, f + 8);
                    for (int e = 0; e < 12; ++e) {
                        if ((f[T.E[e].v0] >= g.c) == (f[T.E[e].v1] >= g.c)) continue;
                        const uint64_t key = edge_key(conf, K, K, lf.ix, lf.iy, lf.iz, e);
                        auto it = std::lower_bound(
                            V.begin(), V.end(), key,
                            [](const tms_vertex &a, uint64_t kk) { return a.edge_key < kk; });
                        if ((it != V.end() && it->edge_key == key) || !seen.insert(key).second)
                            continue;
                        X.push_back(new_vertex(g, conf, K, lf.ix, lf.iy, lf.iz, e, f));
                    }
                }
    }
    return std::string();
}

// Closing open faces (device entry point).  The partition keeps a cube when
// the bound of its polynomial reaches c; where the bound is not met on a
// coarse cube although phi at the finest lattice points inside it crosses c,
// the surface leaves a kept cube through a face with nothing across.  Each
// cube of the leaves' level across such a face is added as a SURFACE leaf,
// repeatedly (an added cube may itself have open faces), until none is left
// or `rounds` passes, and triangulated like the others.  Its corner values
// come from a SURFACE leaf that has the same lattice point as a corner
// wherever there is one (so both sides of a shared face pair its edge points
// alike), else from phi of the library (tms_eval_phi, the precision of
// `cells`); its new edge points are placed as the extraction places them and
// appended to the mesh's points.  Cubes outside the root grid are not added.
constexpr int kCloseRounds = 64;

std::string close_mesh(tms_ctx *ctx, const tms_cells *cells, int conf, std::vector<tms_leaf> &L,
                       std::vector<double> &cp, VIndex &VI, std::vector<uint8_t> &em,
                       tms_mesh *M, int32_t *rc) {
    *rc = TMS_OK;
    const Grid &g = cells->gh[(size_t)conf];
    const int level = M->level, sh = g.K - level;
    const Topo &T = topo();
    const VidFn vid = [&](uint64_t key) { return VI.find(key); };
    const KeyFn key_of = [&](int64_t v) { return VI.key_of(v); };
    std::vector<std::array<int32_t, 3>> q;
    open_faces(em, nullptr, (int64_t)em.size(), key_of, g.K, &q);
    DevBuf dpts, dphi;
    for (int r = 0; r < kCloseRounds; ++r) {
        q.erase(std::remove_if(q.begin(), q.end(),
                               [&](const std::array<int32_t, 3> &x) {
                                   for (int a = 0; a < 3; ++a)
                                       if (x[a] < 0 || (int64_t)x[a] >= ((int64_t)g.nr[a] << level))
                                           return true;
                                   return false;
                               }),
                q.end());
        if (q.empty()) break;
        // SURFACE leaves within one cube of the new cubes (their corners and
        // faces are the only ones the new cubes share)
        std::unordered_map<uint64_t, int64_t> at;
        {
            std::unordered_set<uint64_t> nb;
            for (const auto &x : q)
                for (int d = 0; d < 27; ++d)
                    nb.insert(cube_key(x[0] + d % 3 - 1, x[1] + (d / 3) % 3 - 1, x[2] + d / 9 - 1));
            const unsigned nth = std::max(1u, std::thread::hardware_concurrency());
            std::vector<std::vector<std::pair<uint64_t, int64_t>>> part(nth);
            parallel_for((int64_t)L.size(), [&](int64_t b, int64_t e, int t) {
                for (int64_t i = b; i < e; ++i) {
                    const tms_leaf &lf = L[(size_t)i];
                    if (lf.cls != TMS_CLS_SURFACE || lf.level != level) continue;
                    const uint64_t k = cube_key(lf.ix, lf.iy, lf.iz);
                    if (nb.count(k)) part[(size_t)t].push_back({k, i});
                }
            });
            for (auto &p : part)
                for (auto &kv : p) at.emplace(kv.first, kv.second);
        }
        q.erase(std::remove_if(q.begin(), q.end(),
                               [&](const std::array<int32_t, 3> &x) {
                                   return at.count(cube_key(x[0], x[1], x[2])) > 0;
                               }),
                q.end());
        if (q.empty()) break;
        // corner values: from a SURFACE leaf at the same lattice point, else phi
        const size_t nq = q.size();
        std::vector<double> f(nq * 8, 0.0);
        std::vector<int64_t> slot(nq * 8, -1);
        std::unordered_map<uint64_t, int64_t> need;
        std::vector<double> pts;
        for (size_t k = 0; k < nq; ++k)
            for (int v = 0; v < 8; ++v) {
                const int64_t P[3] = {q[k][0] + (v & 1), q[k][1] + ((v >> 1) & 1),
                                      q[k][2] + ((v >> 2) & 1)};
                bool found = false;
                for (int w = 0; w < 8 && !found; ++w) {
                    auto it = at.find(cube_key(P[0] - (w & 1), P[1] - ((w >> 1) & 1),
                                               P[2] - ((w >> 2) & 1)));
                    if (it == at.end()) continue;
                    f[k * 8 + v] = cp[(size_t)it->second * 8 + (size_t)w];
                    found = true;
                }
                if (found) continue;
                auto ins = need.emplace(cube_key(P[0], P[1], P[2]), (int64_t)(pts.size() / 3));
                if (ins.second)
                    for (int a = 0; a < 3; ++a)
                        pts.push_back(g.o[a] + (double)(P[a] << sh) * g.hmin);
                slot[k * 8 + v] = ins.first->second;
            }
        {
            std::vector<double> phi;
            const std::string why = eval_points(ctx, cells, conf, pts, phi, dpts, dphi, rc);
            if (*rc != TMS_OK) return why;
            for (size_t k = 0; k < nq * 8; ++k)
                if (slot[k] >= 0) f[k] = phi[(size_t)slot[k]];
        }
        // the new leaves, the edge points of their edges not yet in the mesh
        std::vector<int64_t> idx, touched;
        for (size_t k = 0; k < nq; ++k) {
            tms_leaf lf{};
            lf.ix = q[k][0];
            lf.iy = q[k][1];
            lf.iz = q[k][2];
            lf.conf = conf;
            lf.level = (uint8_t)level;
            lf.reason = TMS_REASON_CLOSED;
            unsigned mask = 0;
            for (int v = 0; v < 8; ++v)
                if (f[k * 8 + v] >= g.c) mask |= 1u << v;
            lf.mask = (uint8_t)mask;
            // a face of it crosses c, so it is a SURFACE cube
            lf.cls = mask == 0 ? TMS_CLS_OUTSIDE : mask == 0xFF ? TMS_CLS_INSIDE : TMS_CLS_SURFACE;
            idx.push_back((int64_t)L.size());
            L.push_back(lf);
            cp.insert(cp.end(), f.begin() + (ptrdiff_t)(k * 8), f.begin() + (ptrdiff_t)(k * 8 + 8));
            M->leaf_ijk.insert(M->leaf_ijk.end(), {lf.ix, lf.iy, lf.iz});
            for (int ed = 0; ed < 12; ++ed) {
                const EdgeInfo &E = T.E[ed];
                const double f0 = f[k * 8 + E.v0], f1 = f[k * 8 + E.v1];
                if ((f0 >= g.c) == (f1 >= g.c)) continue;
                const uint64_t key = edge_key(conf, level, g.K, lf.ix, lf.iy, lf.iz, ed);
                int64_t id = vid(key);
                if (id < 0) {
                    id = (int64_t)(M->xyz.size() / 3);
                    VI.add(key, id);
                    const tms_vertex nvx =
                        new_vertex(g, conf, level, lf.ix, lf.iy, lf.iz, ed, &f[k * 8]);
                    double x[3];
                    place_vertex(key, nvx.t, nvx.x, nvx.y, nvx.z, g.h0, x);
                    M->xyz.insert(M->xyz.end(), x, x + 3);
                    em.push_back(0);
                }
                touched.push_back(id);
            }
        }
        if (!ring_pass(L, cp, idx, g.c, g.K, vid, em)) {
            *rc = TMS_E_INVALID;
            return "an edge point of a cube added across an open face is missing";
        }
        std::sort(touched.begin(), touched.end());
        touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
        open_faces(em, &touched, 0, key_of, g.K, &q);
    }
    M->open_faces = open_faces(em, nullptr, (int64_t)em.size(), key_of, g.K, nullptr);
    return std::string();
}

void set_msg(char *msg, int64_t len, const std::string &s) {
    if (!msg || len <= 0) return;
    const size_t k = std::min<size_t>((size_t)len - 1, s.size());
    std::memcpy(msg, s.data(), k);
    msg[k] = 0;
}

}  // namespace

extern "C" {

int32_t tms_mesh_build(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves, int64_t n,
                       const double *corner_phi, const tms_vertex *verts, int64_t nv,
                       int32_t flags, tms_mesh **out) {
    if (!ctx) return TMS_E_INVALID;
    if (!out || !cells || n < 0 || nv < 0 || (n > 0 && (!leaves || !corner_phi)) ||
        (nv > 0 && !verts) || (flags & ~TMS_MESH_CLOSE))
        return mfail(ctx, TMS_E_INVALID, "invalid arguments to tms_mesh_build");
    *out = nullptr;
    if (std::find(ctx->cells.begin(), ctx->cells.end(), cells) == ctx->cells.end())
        return mfail(ctx, TMS_E_INVALID, "cells handle does not belong to this context");
    std::vector<tms_leaf> L((size_t)n);
    std::vector<double> cp((size_t)n * 8);
    std::vector<tms_vertex> V((size_t)nv);
    if (hipSetDevice(ctx->device) != hipSuccess ||
        (n > 0 && hipMemcpyAsync(L.data(), leaves, sizeof(tms_leaf) * n, hipMemcpyDeviceToHost,
                                 ctx->stream) != hipSuccess) ||
        (n > 0 && hipMemcpyAsync(cp.data(), corner_phi, sizeof(double) * 8 * n,
                                 hipMemcpyDeviceToHost, ctx->stream) != hipSuccess) ||
        (nv > 0 && hipMemcpyAsync(V.data(), verts, sizeof(tms_vertex) * nv, hipMemcpyDeviceToHost,
                                  ctx->stream) != hipSuccess) ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(ctx, TMS_E_DEVICE, "copying leaves, corner values or vertices to the host");
    }
    // one conformation: the cells' only one, or one of a batch's (its range
    // of the leaves and of the vertices)
    const int conf = n > 0 ? L[0].conf : 0;
    if (conf < 0 || conf >= cells->nconf)
        return mfail(ctx, TMS_E_INVALID, "leaves of a conformation the cells do not have");
    for (const tms_leaf &lf : L)
        if (lf.conf != conf)
            return mfail(ctx, TMS_E_INVALID, "leaves of several conformations: mesh one at a time");
    for (const tms_vertex &v : V)
        if ((int)(v.edge_key >> 53) != conf)
            return mfail(ctx, TMS_E_INVALID, "vertices of another conformation than the leaves");
    const Grid &g = cells->gh[(size_t)conf];
    // SURFACE leaves above the finest level are meshed through their finest
    // sub-cubes; then the mesh, then the cubes across open faces
    std::vector<tms_vertex> X;
    {
        int32_t rc = TMS_OK;
        const std::string w = split_coarse(ctx, cells, conf, L, cp, V, X, &rc);
        if (rc != TMS_OK) return mfail(ctx, rc, w.c_str());
    }
    std::vector<uint8_t> em;
    VIndex VI;
    const std::string why = prepare_mesh(L, cp, V, X, VI, g.c, g.K, g.h0, out, em);
    if (!why.empty()) return mfail(ctx, TMS_E_INVALID, why.c_str());
    if ((flags & TMS_MESH_CLOSE) && (*out)->open_faces > 0) {
        int32_t rc = TMS_OK;
        const std::string w = close_mesh(ctx, cells, conf, L, cp, VI, em, *out, &rc);
        if (rc != TMS_OK) {
            delete *out;
            *out = nullptr;
            return mfail(ctx, rc, w.c_str());
        }
    }
    const std::string w2 = finish_mesh(L, cp, VI, g.c, g.K, g.h0, *out);
    if (!w2.empty()) {
        delete *out;
        *out = nullptr;
        return mfail(ctx, TMS_E_INVALID, w2.c_str());
    }
    (*out)->added.assign(L.begin() + n, L.end());
    (*out)->added_phi.assign(cp.begin() + 8 * n, cp.end());
    return TMS_OK;
}

int32_t tms_mesh_build_host(const tms_leaf *leaves, int64_t n, const double *corner_phi,
                            const tms_vertex *verts, int64_t nv, double c, int32_t K, double h0,
                            tms_mesh **out, char *msg, int64_t msg_len) {
    set_msg(msg, msg_len, "");
    if (!out || n < 0 || nv < 0 || (n > 0 && (!leaves || !corner_phi)) || (nv > 0 && !verts) ||
        !(c > 0) || K < 0 || K >= TMS_MAX_LEVELS || !(h0 > 0)) {
        set_msg(msg, msg_len, "invalid arguments to tms_mesh_build_host");
        return TMS_E_INVALID;
    }
    std::vector<tms_leaf> L(leaves, leaves + n);
    std::vector<double> cp(corner_phi, corner_phi + 8 * n);
    std::vector<tms_vertex> V(verts, verts + nv);
    std::vector<uint8_t> em;
    VIndex VI;
    std::string why = prepare_mesh(L, cp, V, std::vector<tms_vertex>(), VI, c, K, h0, out, em);
    if (why.empty()) {
        why = finish_mesh(L, cp, VI, c, K, h0, *out);
        if (!why.empty()) {
            delete *out;
            *out = nullptr;
        }
    }
    if (!why.empty()) {
        set_msg(msg, msg_len, why);
        return TMS_E_INVALID;
    }
    return TMS_OK;
}

int32_t tms_mesh_info(const tms_mesh *m, int64_t *n_vertices, int64_t *n_triangles,
                      int64_t *n_loops, int64_t *n_fallback, int64_t *open_faces) {
    if (!m) return TMS_E_INVALID;
    if (n_vertices) *n_vertices = (int64_t)(m->xyz.size() / 3);
    if (n_triangles) *n_triangles = (int64_t)(m->tri.size() / 3);
    if (n_loops) *n_loops = m->n_loops;
    if (n_fallback) *n_fallback = m->n_fallback;
    if (open_faces) *open_faces = m->open_faces;
    return TMS_OK;
}

int32_t tms_mesh_get(const tms_mesh *m, double *xyz, int32_t *tri, int32_t *tri_leaf) {
    if (!m) return TMS_E_INVALID;
    if (xyz) std::memcpy(xyz, m->xyz.data(), sizeof(double) * m->xyz.size());
    if (tri) std::memcpy(tri, m->tri.data(), sizeof(int32_t) * m->tri.size());
    if (tri_leaf) std::memcpy(tri_leaf, m->tri_leaf.data(), sizeof(int32_t) * m->tri_leaf.size());
    return TMS_OK;
}

int32_t tms_mesh_added(const tms_mesh *m, tms_leaf *leaves, double *corner_phi, int64_t cap,
                       int64_t *n_out) {
    if (!m || cap < 0) return TMS_E_INVALID;
    const int64_t k = (int64_t)m->added.size();
    if (n_out) *n_out = k;
    if (!leaves && !corner_phi) return TMS_OK;
    if (cap < k) return TMS_E_CAPACITY;
    if (leaves) std::copy(m->added.begin(), m->added.end(), leaves);
    if (corner_phi) std::copy(m->added_phi.begin(), m->added_phi.end(), corner_phi);
    return TMS_OK;
}

int32_t tms_mesh_check(const tms_mesh *m, int32_t intersections, tms_mesh_report *r) {
    if (!m || !r) return TMS_E_INVALID;
    std::memset(r, 0, sizeof *r);
    const int64_t nv = (int64_t)(m->xyz.size() / 3), nt = (int64_t)(m->tri.size() / 3);
    const int32_t *T = m->tri.data();
    const double *X = m->xyz.data();
    r->n_vertices = nv;
    r->n_triangles = nt;
    r->n_loops = m->n_loops;
    r->n_fallback = m->n_fallback;
    r->open_faces = m->open_faces;
    r->added_cubes = (int64_t)m->added.size();
    // incident triangles of every vertex (CSR)
    std::vector<int64_t> off((size_t)nv + 1, 0);
    parallel_for(3 * nt, [&](int64_t b, int64_t e, int) {
        for (int64_t t = b; t < e; ++t) __atomic_fetch_add(&off[(size_t)T[t] + 1], 1, __ATOMIC_RELAXED);
    });
    for (int64_t v = 0; v < nv; ++v) off[(size_t)v + 1] += off[(size_t)v];
    std::vector<int32_t> inc((size_t)(3 * nt));
    {
        std::vector<int64_t> pos(off.begin(), off.end() - 1);
        parallel_for(nt, [&](int64_t b, int64_t e, int) {
            for (int64_t t = b; t < e; ++t)
                for (int k = 0; k < 3; ++k)
                    inc[(size_t)__atomic_fetch_add(&pos[(size_t)T[3 * t + k]], 1, __ATOMIC_RELAXED)] =
                        (int32_t)t;
        });
    }
    // per vertex: (a) the sides at it -- each neighbour joined through
    // exactly two triangles, once in each direction (sides counted at their
    // smaller end); (b) the sides opposite it in its triangles form a single
    // cycle
    const unsigned nth = std::max(1u, std::thread::hardware_concurrency());
    std::vector<std::array<int64_t, 5>> acc(nth, {0, 0, 0, 0, 0});
    parallel_for(nv, [&](int64_t b, int64_t e, int th) {
        std::array<int64_t, 5> &A = acc[(size_t)th];  // edges, boundary, >2, misoriented, bad v
        std::vector<std::pair<int32_t, int32_t>> nbr, link;
        for (int64_t v = b; v < e; ++v) {
            nbr.clear();
            link.clear();
            for (int64_t p = off[(size_t)v]; p < off[(size_t)v + 1]; ++p) {
                const int32_t t = inc[(size_t)p];
                int k = 0;
                while (k < 3 && T[3 * t + k] != v) ++k;
                const int32_t nx = T[3 * t + (k + 1) % 3], pv = T[3 * t + (k + 2) % 3];
                nbr.push_back({nx, 1});
                nbr.push_back({pv, -1});
                if (nx != v && pv != v) link.push_back({nx, pv});
            }
            std::sort(nbr.begin(), nbr.end());
            bool ok = !link.empty();
            for (size_t i = 0; i < nbr.size();) {
                size_t j = i;
                int sdir = 0;
                while (j < nbr.size() && nbr[j].first == nbr[i].first) sdir += nbr[j++].second;
                const size_t k = j - i;
                if (k != 2 || sdir != 0) ok = false;
                if (nbr[i].first > v) {
                    ++A[0];
                    if (k == 1) ++A[1];
                    else if (k > 2) ++A[2];
                    else if (sdir != 0) ++A[3];
                }
                i = j;
            }
            if (ok) {
                // every link vertex is in two link sides (each neighbour is in
                // two triangles); walk the cycle from the first side
                std::vector<char> seen(link.size(), 0);
                size_t cnt = 1;
                seen[0] = 1;
                int32_t cur = link[0].second;
                const int32_t start = link[0].first;
                while (cur != start && cnt <= link.size()) {
                    size_t nx = link.size();
                    for (size_t q = 0; q < link.size(); ++q)
                        if (!seen[q] && (link[q].first == cur || link[q].second == cur)) {
                            nx = q;
                            break;
                        }
                    if (nx == link.size()) break;
                    seen[nx] = 1;
                    ++cnt;
                    cur = link[nx].first == cur ? link[nx].second : link[nx].first;
                }
                ok = cur == start && cnt == link.size();
            }
            if (!ok && off[(size_t)v + 1] > off[(size_t)v]) ++A[4];
        }
    });
    int64_t nedges = 0;
    for (const auto &A : acc) {
        nedges += A[0];
        r->boundary_edges += A[1];
        r->nonmanifold_edges += A[2];
        r->misoriented_edges += A[3];
        r->nonmanifold_vertices += A[4];
    }
    // components (union-find over triangle sides) and Euler characteristic
    {
        std::vector<int32_t> par((size_t)nv);
        std::iota(par.begin(), par.end(), 0);
        std::function<int32_t(int32_t)> find = [&](int32_t x) {
            while (par[(size_t)x] != x) {
                par[(size_t)x] = par[(size_t)par[(size_t)x]];
                x = par[(size_t)x];
            }
            return x;
        };
        std::vector<char> usedv((size_t)nv, 0);
        for (int64_t t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) {
                usedv[(size_t)T[3 * t + k]] = 1;
                if (k == 2) break;  // two sides join all three corners
                const int32_t a = find(T[3 * t + k]), b = find(T[3 * t + k + 1]);
                if (a != b) par[(size_t)a] = b;
            }
        int64_t comps = 0, nvu = 0;
        for (int64_t v = 0; v < nv; ++v)
            if (usedv[(size_t)v]) {
                ++nvu;
                if (find((int32_t)v) == v) ++comps;
            }
        r->components = comps;
        r->euler = nvu - nedges + nt;
        r->unused_vertices = nv - nvu;
    }
    // area, enclosed volume (outward orientation gives a positive volume),
    // angles and degenerate triangles
    struct Acc {
        double area = 0.0, vol = 0.0, amin = 180.0;
        int64_t small = 0, zero = 0;
    };
    std::vector<Acc> av(nth);
    parallel_for(nt, [&](int64_t b, int64_t e, int th) {
        Acc a;
        for (int64_t t = b; t < e; ++t) {
            const double *P[3] = {X + 3 * T[3 * t], X + 3 * T[3 * t + 1], X + 3 * T[3 * t + 2]};
            double u[3], w[3], n[3];
            sub3(P[1], P[0], u);
            sub3(P[2], P[0], w);
            crs3(u, w, n);
            const double n2 = std::sqrt(dot3(n, n));
            a.area += 0.5 * n2;
            double qs[3];
            crs3(P[1], P[2], qs);
            a.vol += dot3(P[0], qs) / 6.0;
            // the angle at each corner: atan2(|x y|, x . y) of its two sides
            double tmin = 180.0, side2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double x[3], y[3], xy[3];
                sub3(P[(k + 1) % 3], P[k], x);
                sub3(P[(k + 2) % 3], P[k], y);
                crs3(x, y, xy);
                side2 = std::max(side2, dot3(x, x));
                tmin = std::min(tmin, std::atan2(std::sqrt(dot3(xy, xy)), dot3(x, y)) *
                                          (180.0 / 3.14159265358979323846));
            }
            a.amin = std::min(a.amin, tmin);
            if (tmin < 5.0) ++a.small;
            if (0.5 * n2 <= 1e-12 * side2) ++a.zero;
        }
        av[(size_t)th] = a;
    });
    double area = 0.0, vol = 0.0;
    r->min_angle = nt > 0 ? 180.0 : 0.0;
    for (const auto &x : av) {
        area += x.area;
        vol += x.vol;
        r->min_angle = std::min(r->min_angle, x.amin);
        r->small_angles += x.small;
        r->zero_area += x.zero;
    }
    r->area = area;
    r->volume = vol;
    r->density = area > 0 ? (double)nv / area : 0.0;
    // (c) intersecting pairs among triangles of the same or touching leaves:
    // the triangles of a leaf are contiguous (emitted leaf by leaf), so each
    // leaf is a run of triangles; runs sorted by the leaf's cube key, and
    // the neighbours of a leaf found by binary search
    if (intersections) {
        const int64_t nl = (int64_t)(m->leaf_ijk.size() / 3);
        struct Run {
            uint64_t key;
            int64_t b, e;
        };
        std::vector<Run> runs;
        for (int64_t t = 0; t < nt;) {
            int64_t e = t + 1;
            while (e < nt && m->tri_leaf[(size_t)e] == m->tri_leaf[(size_t)t]) ++e;
            const int32_t li = m->tri_leaf[(size_t)t];
            if (li >= 0 && li < nl) {
                const int32_t *c = &m->leaf_ijk[3 * (size_t)li];
                runs.push_back({cube_key(c[0], c[1], c[2]), t, e});
            }
            t = e;
        }
        parallel_sort(runs, [](const Run &x, const Run &y) {
            return x.key != y.key ? x.key < y.key : x.b < y.b;
        });
        auto first_run = [&](uint64_t k) {
            return std::lower_bound(runs.begin(), runs.end(), k,
                                    [](const Run &x, uint64_t kk) { return x.key < kk; }) -
                   runs.begin();
        };
        std::atomic<int64_t> hits{0};
        parallel_for((int64_t)runs.size(), [&](int64_t rb, int64_t re, int) {
            int64_t local = 0;
            for (int64_t ri = rb; ri < re; ++ri) {
                const Run &A = runs[(size_t)ri];
                const int64_t x = (int64_t)(A.key >> 42), y = (int64_t)((A.key >> 21) & 0x1FFFFF),
                              z = (int64_t)(A.key & 0x1FFFFF);
                for (int d = 0; d < 27; ++d) {
                    const uint64_t k1 = cube_key(x + d % 3 - 1, y + (d / 3) % 3 - 1, z + d / 9 - 1);
                    if (k1 < A.key) continue;  // each pair of leaves once
                    for (int64_t rj = first_run(k1);
                         rj < (int64_t)runs.size() && runs[(size_t)rj].key == k1; ++rj) {
                        const Run &B = runs[(size_t)rj];
                        if (k1 == A.key && rj < ri) continue;
                        for (int64_t s = A.b; s < A.e; ++s)
                            for (int64_t t = (rj == ri ? s + 1 : B.b); t < B.e; ++t) {
                                bool share = false;
                                for (int p = 0; p < 3; ++p)
                                    for (int q = 0; q < 3; ++q)
                                        if (T[3 * s + p] == T[3 * t + q]) share = true;
                                if (share) continue;
                                const double *V0 = X + 3 * T[3 * s], *V1 = X + 3 * T[3 * s + 1],
                                             *V2 = X + 3 * T[3 * s + 2], *U0 = X + 3 * T[3 * t],
                                             *U1 = X + 3 * T[3 * t + 1], *U2 = X + 3 * T[3 * t + 2];
                                if (may_meet(V0, V1, V2, U0, U1, U2) &&
                                    triangles_meet(V0, V1, V2, U0, U1, U2))
                                    ++local;
                            }
                    }
                }
            }
            hits.fetch_add(local);
        });
        r->intersecting_pairs = hits.load();
    } else {
        r->intersecting_pairs = -1;
    }
    return TMS_OK;
}

int32_t tms_mesh_write_off(const tms_mesh *m, const char *path) {
    if (!m || !path) return TMS_E_INVALID;
    FILE *fp = std::fopen(path, "w");
    if (!fp) return TMS_E_INVALID;
    const int64_t nv = (int64_t)(m->xyz.size() / 3), nt = (int64_t)(m->tri.size() / 3);
    std::fprintf(fp, "OFF\n%lld %lld 0\n", (long long)nv, (long long)nt);
    for (int64_t v = 0; v < nv; ++v)
        std::fprintf(fp, "%.17g %.17g %.17g\n", m->xyz[3 * v], m->xyz[3 * v + 1], m->xyz[3 * v + 2]);
    for (int64_t t = 0; t < nt; ++t)
        std::fprintf(fp, "3 %d %d %d\n", m->tri[3 * t], m->tri[3 * t + 1], m->tri[3 * t + 2]);
    const bool ok = std::fclose(fp) == 0;
    return ok ? TMS_OK : TMS_E_INVALID;
}

int32_t tms_mesh_free(tms_mesh *m) {
    delete m;
    return TMS_OK;
}

}  // extern "C"
