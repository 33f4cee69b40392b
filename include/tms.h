/*
 * tms.h -- C ABI of the MI355X (gfx950) implementation of the adaptive
 * partition-and-estimation stage of the Gaussian molecular surface method of
 * Liu, Chen & Lu, "Efficient and Qualified Mesh Generation for Gaussian
 * Molecular Surface Using Piecewise Trilinear Polynomial Approximation"
 * (arXiv:1611.03474).
 *
 * Problem statement (Section 1 and Section 2.1): atoms with centres x_i and
 * radii r_i define phi(x) = sum_i exp(-D(|x - x_i|^2 - r_i^2)) (eq. Gaussian1);
 * the surface is phi = c.  Stage one (Section 2.2) covers space with cubes of
 * several sizes in which phi is replaced by a trilinear interpolant whose error
 * is controlled by a user tolerance; its output is the list of cubes and the
 * points where the trilinear surface crosses the cube edges (eq. intersection).
 *
 * Conventions for every entry point
 *  - All functions return an int32 status: TMS_OK (0) or a negative TMS_E_*
 *    code.  No C++ exception crosses this boundary.  After an error,
 *    tms_last_error(ctx) returns a NUL-terminated message owned by ctx.
 *  - Pointers documented as "device" address HIP device memory of the
 *    context's device (for instance torch tensors on that device); pointers
 *    documented as "host" address host memory.  The library never keeps a
 *    pointer that the caller passes in.
 *  - Work is enqueued on the stream given to tms_create.  Calls return after
 *    their results are complete on that stream (each call synchronises the
 *    stream at least once, because output sizes are data dependent).
 *  - Coordinates are in the caller's length unit (angstrom in the paper).
 *  - A context is not thread-safe: one host thread at a time per context.
 */
#ifndef TMS_H
#define TMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define TMS_OK 0
#define TMS_E_INVALID (-1)  /* an argument or the input data is invalid       */
#define TMS_E_CAPACITY (-2) /* an output buffer is too small; see the call    */
#define TMS_E_DEVICE (-3)   /* a HIP runtime error (no device, launch, ...)   */
#define TMS_E_OOM (-4)      /* device memory allocation failed                */

/* ---- precision of the per-pair arithmetic -------------------------------- */
#define TMS_PREC_FP64 0       /* everything in double precision                 */
#define TMS_PREC_FP32_GUARD 1 /* the per-pair exponentials that are not shared  */
                              /* (phi at points and corners; 1-D projections    */
                              /* computed in place) from the single-precision   */
                              /* hardware exponential, relative error <= 1.5e-7; */
                              /* every sum and product stays double precision.  */
                              /* Any cube or point whose decision margin lies   */
                              /* within that error band is recomputed with      */
                              /* double-precision exponentials, so every        */
                              /* discrete result equals the double-precision one */

/* ---- partition mode ---------------------------------------------------- */
#define TMS_MODE_ADAPTIVE 0 /* Section 2.2 Steps 1-3: estimate, bound, divide   */
#define TMS_MODE_UNIFORM 1  /* plain method: every cube of the h0 grid is a leaf */

/* ---- tensors of the cubes below the roots (Section 2.2.3) ---------------- */
#define TMS_CHILD_PROJECT 0  /* projected from the atoms again on every child    */
                             /* (the default; Step 3 computes the expression of  */
                             /* P in each child)                                  */
#define TMS_CHILD_REEXPAND 1 /* the parent's polynomial written in the child's   */
                             /* Legendre basis (eq. childtensor): only the roots  */
                             /* loop over atoms.  The root-level approximation    */
                             /* error is carried down unchanged                   */

/* ---- leaf reasons and classes ------------------------------------------ */
#define TMS_REASON_UNIFORM 0   /* uniform mode                                   */
#define TMS_REASON_CONVERGED 1 /* higher-order mass 2E <= tau (Step 3)          */
#define TMS_REASON_HMIN 2      /* kept by the bound at the finest level          */
#define TMS_REASON_CLOSED 3    /* added by tms_mesh_build across an open face    */
#define TMS_REASON_SPLIT 4     /* finest cube of a coarser SURFACE leaf (mesh)   */
#define TMS_CLS_OUTSIDE 0      /* every corner value below c                     */
#define TMS_CLS_SURFACE 1      /* corner values on both sides of c               */
#define TMS_CLS_INSIDE 2       /* every corner value >= c                        */

#define TMS_MAX_LEVELS 8

typedef struct tms_ctx tms_ctx;
typedef struct tms_cells tms_cells;

/* Parameters of one surface (Section 1, Section 2.2).
 *  D       decay rate of the Gaussian kernel (> 0)
 *  c       isovalue (> 0)
 *  tau     bound on the higher-order coefficients that turns a child cube
 *          into a trilinear leaf: the cube is a leaf when 2E <= tau, E the
 *          l1 mass of the tensor entries of degree above one in some
 *          variable; 2E bounds |P - g| on the cube (> 0; adaptive mode)
 *  h0      edge of the initial coarse grid cubes (> 0)
 *  h_min   edge of the finest cubes; h0/h_min must be 2^K, 0 <= K < 8
 *  pad     margin added around the atom bounding box (>= 0)
 *  eps_cut every Gaussian term below eps_cut is dropped: the sums run over
 *          atoms within R_c, R_c^2 = max r_i^2 + ln(1/eps_cut)/D (0 < eps_cut < 1)
 *  precision TMS_PREC_*;  mode TMS_MODE_*
 *  degree  degree n of the 1-D Legendre series of each Gaussian factor
 *          (Section 2.2.1, eqs. poly2_1 to alpha): 1, 2 or 3 (0 means 3, the
 *          paper's choice); the endpoint corrections go on L_{n-1} and L_n
 *          and the tensor entries above n are zero
 *  child_tensor TMS_CHILD_* (adaptive mode)                                  */
typedef struct {
    double D, c, tau, h0, h_min, pad, eps_cut;
    int32_t precision;
    int32_t mode;
    int32_t degree;
    int32_t child_tensor;
} tms_params;

/* One leaf cube: the closed box origin + [i, i+1] * h0 / 2^level per axis.
 * mask bit v (v = dx + 2 dy + 4 dz, d* in {0,1} the corner offsets) is set
 * iff phi at that corner is >= c.  20 bytes, 4-byte aligned. */
typedef struct {
    int32_t ix, iy, iz;
    int32_t conf; /* conformation index (0 for a single structure) */
    uint8_t level, reason, mask, cls;
} tms_leaf;

/* One edge intersection point (eq. intersection).  edge_key packs
 * conf(11 bits) | level(3) | axis(2) | X(16) | Y(16) | Z(16), where X, Y, Z
 * are the finest-lattice coordinates (units of h_min) of the edge's lower
 * end; t in [0,1] is the position along the edge from that end; x, y, z the
 * point.  40 bytes. */
typedef struct {
    uint64_t edge_key;
    double t, x, y, z;
} tms_vertex;

/* Counters of one partition pass (host struct, filled on request). */
typedef struct {
    int64_t n_est[TMS_MAX_LEVELS];    /* cubes whose tensor was computed */
    int64_t n_disc[TMS_MAX_LEVELS];   /* cubes discarded by the bound    */
    int64_t n_refine[TMS_MAX_LEVELS]; /* cubes divided into 8 children   */
    int64_t n_conv[TMS_MAX_LEVELS];   /* converged leaves                */
    int64_t n_hmin[TMS_MAX_LEVELS];   /* leaves kept at the finest level */
    int64_t n_leaves, n_surface, n_corners;
    int64_t n_bound;        /* cubes that needed the full nested-SVD bound     */
    int64_t guard_cubes;    /* always 0: every partition level runs with       */
                            /* exact exponentials (kept for the layout)        */
    int64_t guard_points;   /* corner points recomputed with exact exponentials */
    int64_t n_pairs;        /* cube-atom pairs inside R_c (algorithmic work)   */
    int64_t n_pairs_lvl[TMS_MAX_LEVELS]; /* the same, per level           */
} tms_stats;

/* Create a context on HIP device `device`, enqueueing work on `stream`
 * (a hipStream_t; NULL means the device's null stream).  The stream is
 * borrowed: it must outlive the context.  *out receives the context.
 * Errors: TMS_E_INVALID (out NULL), TMS_E_DEVICE (no such device). */
int32_t tms_create(tms_ctx **out, int32_t device, void *stream);

/* Free a context and every buffer and cell structure it owns. */
int32_t tms_destroy(tms_ctx *ctx);

/* Message of the last failing call on ctx ("" if none); valid until the next
 * call on ctx.  With ctx == NULL: message of the last tms_create failure. */
const char *tms_last_error(const tms_ctx *ctx);

/* Host-only validation of a parameter set (no device needed).  Returns
 * TMS_OK or TMS_E_INVALID and writes a message into msg[0..msg_len). */
int32_t tms_check_params(const tms_params *p, char *msg, int64_t msg_len);

/* Host-only validation of an atom array xyzr (host, [n][4] double: x, y, z,
 * r) against p: finite values, r > 0, lattice size below 2^16 per axis. */
int32_t tms_check_atoms_host(const double *xyzr, int64_t n, const tms_params *p,
                             char *msg, int64_t msg_len);

/* Bin the atoms and build the neighbourhood lists (Section 2.2.1, after eq.
 * polynew: only atoms near a cube contribute).
 *  xyzr   device, [n][4] double (x, y, z, r), row-major; read, not kept.
 *  n      number of atoms (>= 0).
 *  p      parameters (copied).
 *  cells  in/out: if *cells is NULL a new structure is created; otherwise
 *         it is rebuilt in place and its device memory reused.  Owned by ctx;
 *         free with tms_free_cells or tms_destroy.
 * The initial grid (Section 2.2) has its origin at h0 * floor((min - pad)/h0)
 * per axis and ceil((max + pad - origin)/h0) cubes per axis.
 * Errors: TMS_E_INVALID (NaN/Inf, r <= 0, bad parameters, lattice too large),
 * TMS_E_OOM, TMS_E_DEVICE. */
int32_t tms_build_cells(tms_ctx *ctx, const double *xyzr, int64_t n, const tms_params *p,
                        tms_cells **cells);

/* Cells of a batch of conformations refined together (the same method and
 * parameters on every conformation, Section 2.2; each conformation keeps its
 * own root grid, cut-off radius and atom cells, exactly as if it were built
 * alone).  One tms_partition_estimate then refines every conformation in the
 * same launches: each level's work queue holds the cubes of all
 * conformations.
 *  xyzr     device [offsets[n_conf]][4] double: the conformations' atoms,
 *           concatenated; conformation b is atoms [offsets[b], offsets[b+1]).
 *           Caller-owned, copied.
 *  offsets  host [n_conf + 1] int64, offsets[0] = 0, non-decreasing.
 *  n_conf   1 .. 2048 (the conformation id takes 11 bits of an edge key).
 * Leaves carry their conformation in tms_leaf.conf and come out grouped by
 * conformation (each group in the single-conformation order); vertices are
 * in edge-key order, hence grouped by conformation too; tms_batch_counts
 * gives the group boundaries.  tms_eval_phi and tms_backward take
 * single-conformation cells only; the uniform grid takes one conformation.
 * Errors: as tms_build_cells, plus TMS_E_INVALID for bad offsets. */
int32_t tms_build_cells_batch(tms_ctx *ctx, const double *xyzr, const int64_t *offsets,
                              int32_t n_conf, const tms_params *p, tms_cells **cells);

/* Per-conformation boundaries of the kept results of `cells`: leaf_offsets
 * [n_conf + 1] of the last partition pass, vertex_offsets [n_conf + 1] of
 * the last extraction (host arrays; either may be NULL).
 * Errors: TMS_E_INVALID (no kept result of these cells). */
int32_t tms_batch_counts(tms_ctx *ctx, const tms_cells *cells, int64_t *leaf_offsets,
                         int64_t *vertex_offsets);

/* Grid of a cell structure (host outputs; any pointer may be NULL). */
int32_t tms_cells_info(const tms_cells *cells, double origin[3], int64_t dims[3], int32_t *K,
                       double *rc2, int64_t *n_atoms);

int32_t tms_free_cells(tms_ctx *ctx, tms_cells *cells);

/* phi and its gradient at m points (eq. Gaussian1), summed over the atoms
 * within R_c of each point.
 *  pts   device [m][3] double;  phi device [m] double;  grad device [m][3]
 *  double or NULL.  In TMS_PREC_FP32_GUARD each term's exponential comes
 *  from the single-precision hardware exponential (relative error <= 1.5e-7;
 *  the sums stay double precision) and every point with |phi - c| inside
 *  that error band is recomputed with double-precision exponentials, so the
 *  sign of phi - c is the double-precision one; *n_guard (host, may be NULL)
 *  receives the count.
 * Errors: TMS_E_INVALID, TMS_E_DEVICE. */
int32_t tms_eval_phi(tms_ctx *ctx, const tms_cells *cells, const double *pts, int64_t m,
                     double *phi, double *grad, int64_t *n_guard);

/* tms_eval_phi for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results as tms_eval_phi (bit for bit; n_guard equal),
 * but the FP32+guard path's per-point guard flags, guard list and count live
 * in a static device array of the library (about 20 MB per device, held until
 * the process ends) instead of context workspace.  This call allocates
 * nothing: no hipMalloc, no hipFree, no allocating library routine.
 *  m     0 .. 4194304 (2^22) points; larger m returns TMS_E_INVALID.
 *  other arguments as tms_eval_phi.
 * Every call on one device shares that array and keeps the last call's
 * contents (the count is cleared at the start of each call): calls that
 * overlap on one device -- from two contexts or two host threads -- race
 * and must be serialised by the caller.
 * Errors: TMS_E_INVALID, TMS_E_DEVICE (also when the context's device has no
 * such array: device index 64 or above). */
int32_t tms_eval_phi_noalloc(tms_ctx *ctx, const tms_cells *cells, const double *pts, int64_t m,
                             double *phi, double *grad, int64_t *n_guard);

/* The adaptive partition and estimation pass (Section 2.2, Steps 1-3), then
 * the classification of every leaf by the signs of phi - c at its corners
 * (the trilinear interpolant of eq. linear1 meets the closed cube iff the
 * corner values straddle c).
 *  leaves      device [cap] tms_leaf, or NULL to only count.
 *  cap         capacity of leaves (and of corner_phi rows).
 *  n_leaves    host out: number of leaves.
 *  corner_phi  device [cap][8] double (corner v = dx + 2dy + 4dz) or NULL.
 *  stats       host out or NULL.
 * Leaves are ordered by level, then by refinement order: the roots in raster
 * order (x fastest), and the 8 children of a divided cube in octant order
 * (bit 0 x, bit 1 y, bit 2 z) at the position of their parent.
 * When `leaves` holds the result (cap >= the count) the classified leaves,
 * and the corner values if corner_phi is given, are written straight into
 * the caller's buffers and ctx keeps no copy of them.  Otherwise (leaves
 * NULL, or cap too small) the result is kept in ctx until the next partition
 * call; a too-small cap returns TMS_E_CAPACITY with *n_leaves set to the
 * required count and nothing copied -- then call tms_get_leaves with a
 * larger buffer.
 * Corners are de-duplicated in a dense bitmap over the finest lattice; a
 * lattice whose bitmap would exceed 8 GiB (a box of about 1,000 h_min per
 * axis) is refused with TMS_E_INVALID.
 * Errors: TMS_E_CAPACITY, TMS_E_INVALID, TMS_E_OOM, TMS_E_DEVICE. */
int32_t tms_partition_estimate(tms_ctx *ctx, const tms_cells *cells, tms_leaf *leaves, int64_t cap,
                               int64_t *n_leaves, double *corner_phi, tms_stats *stats);

/* Copy the leaves (and corner values, if corner_phi is not NULL) of the last
 * partition pass, as kept in ctx; with leaves NULL only the count.
 * Errors: TMS_E_CAPACITY (*n_leaves = required), TMS_E_INVALID (also when
 * that pass wrote them into the caller's buffers and kept no copy). */
int32_t tms_get_leaves(tms_ctx *ctx, tms_leaf *leaves, double *corner_phi, int64_t cap,
                       int64_t *n_leaves);

/* Edge intersection points of the trilinear surface g = c (eq. intersection):
 * on every edge of a SURFACE leaf whose end signs differ, g is linear, and
 * the point is at t = (c - phi0)/(phi1 - phi0) from the lower end.  An edge
 * shared by leaves of the same level is emitted once.  Vertices come out in
 * ascending edge_key order.  Leaves that share an edge must carry the same
 * values at its ends (the corner values tms_partition_estimate produces do).
 *  leaves     device [n] tms_leaf (as produced by tms_partition_estimate).
 *  corner_phi device [n][8] double, or NULL to evaluate phi at the corners.
 *  out        device [cap] tms_vertex, or NULL to only count.
 *  n_out      host out: number of vertices.
 * When `out` holds the result (cap >= the count) the vertices are written
 * straight into it and ctx keeps no copy; otherwise the result is kept in
 * ctx until the next extract call (see tms_get_vertices).
 * Edges are de-duplicated in dense bitmaps over each level's lattice; a
 * lattice whose bitmaps would exceed 8 GiB (a box of about 1,000 h_min per
 * axis) is refused with TMS_E_INVALID.  Errors: TMS_E_CAPACITY (*n_out =
 * required), TMS_E_INVALID, TMS_E_OOM, TMS_E_DEVICE. */
int32_t tms_extract_cube_vertices(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves,
                                  int64_t n, const double *corner_phi, tms_vertex *out,
                                  int64_t cap, int64_t *n_out);

/* ---- stage-two points (Section 2.3) ----------------------------------------
 * On a SURFACE leaf mapped to [-1,1]^3 with the trilinear interpolant g of
 * eq. linear1:
 *  - fold segments along axis a (eq. fold1: g = c and dg/da = 0): g is linear
 *    in x_a, so wherever dg/da vanishes g does not depend on x_a and the fold
 *    set is a set of full segments parallel to a; each joins an extreme point
 *    on the face x_a = -1 to one on the face x_a = +1 (eq. curve: g = c,
 *    x_a = +-1, dg/da = 0), at most two per axis;
 *  - critical points (eq. critical: g = c, dg/da = 0, dg/db = 0, a != b), at
 *    most two per pair of axes.
 * Points on the boundary of the closed cube count.  A configuration with
 * infinitely many solutions (g constant along a; the two equations sharing a
 * factor) contributes no points and is counted as degenerate. */
#define TMS_S2_FOLD 0     /* fold segment along `axis`                       */
#define TMS_S2_CRITICAL 1 /* critical point of the two axes other than `axis` */

/* One stage-two record.  leaf: index into the leaf list given.  FOLD: (x, y,
 * z) is the segment's end on the face axis = lower (the extreme point there);
 * its other end, on the face axis = upper, is that point moved by the leaf's
 * edge along the axis.  CRITICAL: (x, y, z) is the point.  root numbers the
 * solutions of one (leaf, kind, axis) from 0 in ascending order of their
 * first free coordinate (FOLD: the lower of the two other axes; CRITICAL:
 * the coordinate along `axis`).  32 bytes. */
typedef struct {
    int32_t leaf;
    uint8_t kind, axis, root, pad;
    double x, y, z;
} tms_s2point;

/* Stage-two points of every SURFACE leaf of a leaf list (Section 2.3, eqs.
 * curve, fold1, critical), in double precision from the leaves' corner
 * values.  Records come out by leaf; inside a leaf the folds along x, y, z,
 * then the critical points of the pairs (y,z), (x,z), (x,y), each by root.
 *  leaves      device [n] tms_leaf (from tms_partition_estimate, or any
 *              leaves of the cells' lattice; conf indexes the batch).
 *  corner_phi  device [n][8] double, corner v = dx + 2dy + 4dz (required).
 *  out         device [cap] tms_s2point, or NULL to only count.
 *  n_out       host out: number of records.
 *  n_degenerate host out (or NULL): degenerate (leaf, kind, axis) cases.
 * Errors: TMS_E_CAPACITY (cap below the count; *n_out = required, nothing
 * written), TMS_E_INVALID, TMS_E_OOM, TMS_E_DEVICE. */
int32_t tms_stage2_points(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves, int64_t n,
                          const double *corner_phi, tms_s2point *out, int64_t cap,
                          int64_t *n_out, int64_t *n_degenerate);

/* Copy the vertices of the last extraction, as kept in ctx; with out NULL
 * only the count.  Errors: TMS_E_CAPACITY (*n_out = required),
 * TMS_E_INVALID (also when that extraction wrote them into the caller's
 * buffer and kept no copy). */
int32_t tms_get_vertices(tms_ctx *ctx, tms_vertex *out, int64_t cap, int64_t *n_out);

/* Unique leaf corners of the last pass (eq. linear1 evaluates phi once per
 * lattice corner shared by any number of leaves): their points and phi
 * values.  The pass is the last tms_partition_estimate, or the last
 * tms_extract_cube_vertices called with corner_phi NULL, whichever came
 * last.  Order: the corner-bitmap order of the adaptive pass (4x4x4 blocks
 * of the finest lattice, blocks x-major, points inside a block x-major), or
 * the raster order of the uniform grid.
 *  xyz  device [cap][3] double or NULL;  phi  device [cap] double or NULL.
 *  n_out host out: number of corners (both NULL: only count).
 * Errors: TMS_E_CAPACITY (*n_out = required), TMS_E_INVALID. */
int32_t tms_get_corners(tms_ctx *ctx, double *xyz, double *phi, int64_t cap, int64_t *n_out);

/* Adjoint of the kept corner values and edge points with respect to the
 * atoms (derivative of eq. Gaussian1 and of eq. intersection): for a loss L
 * given through dL/dphi at the kept corners and dL/dt at the kept edge
 * points, writes dL/d(x_i, y_i, z_i, r_i) for every atom.  Each edge point
 * t = (c - phi0)/(phi1 - phi0) passes dL/dt (t - 1)/(phi1 - phi0) to its
 * lower end and -dL/dt t/(phi1 - phi0) to its upper end; then
 *   dL/dx_i = sum_p wbar_p 2D (p - x_i) term_ip,
 *   dL/dr_i = sum_p wbar_p 2D r_i term_ip,
 * term_ip = exp(-D(|p - x_i|^2 - r_i^2)) over the pairs inside R_c.  The
 * leaves, masks and edge set are held fixed, and so is R_c (a truncation
 * level).  Each (atom, corner) term is recomputed, nothing per pair is
 * stored; terms use the precision of `cells` (TMS_PREC_FP32_GUARD: single
 * precision exponentials, relative error per term <= 1.5e-7, double sums).
 *  cells  the cells of the kept pass (the handle and its last build).
 *  dphi   device [m] double, dL/dphi in tms_get_corners order, or NULL (0);
 *         m must equal the kept corner count when dphi is given.
 *  dt     device [nv] double, dL/dt in the order of the last
 *         tms_extract_cube_vertices output, or NULL (0); nv must equal the
 *         kept vertex count.  That extraction must have been made from the
 *         kept leaves and corner values.
 *  dxyzr  device [n_atoms][4] double, written in the caller's atom order.
 * Errors: TMS_E_INVALID (no kept adaptive pass on these cells, count
 * mismatch, edge points that do not end on kept corners), TMS_E_DEVICE. */
int32_t tms_backward(tms_ctx *ctx, const tms_cells *cells, const double *dphi, int64_t m,
                     const double *dt, int64_t nv, double *dxyzr);

/* ---- captured pass ---------------------------------------------------------
 * The whole pass of tms_partition_estimate followed by
 * tms_extract_cube_vertices (roots, every level with its guard re-runs and
 * compaction, a batch's regrouping, corners, edge points) recorded once into
 * a HIP graph.  Every size stays on the device: launches are sized by
 * capacities (the counts of an eager pass of the same cells times `margin`)
 * and read their actual counts there, so a replay needs no host round trip
 * until its results are read.  Results are those of the eager pass, bit for
 * bit.
 *
 * tms_graph_capture: requires an eager tms_partition_estimate and
 * tms_extract_cube_vertices of `cells` (the last ones on ctx); margin in
 * [1, 64].  The context keeps one capture (private buffers); a new capture
 * replaces it.  The capture first frees the eager partition's workspace
 * (queues, staged tensors, projection table), which it duplicates; kept
 * results are untouched and the next eager pass allocates the workspace
 * again.  Errors: TMS_E_INVALID, TMS_E_OOM, TMS_E_DEVICE. */
int32_t tms_graph_capture(tms_ctx *ctx, const tms_cells *cells, double margin);

/* Capacities a capture of `cells` with this margin gives its results (the
 * eager pass's leaf and vertex counts times margin, plus 4096): the sizes
 * that buffers bound by tms_graph_capture_into must hold.  Same
 * preconditions and errors as tms_graph_capture; host arithmetic only. */
int32_t tms_graph_capacity(tms_ctx *ctx, const tms_cells *cells, double margin,
                           int64_t *leaf_cap, int64_t *vert_cap);

/* tms_graph_capture with the results written by the graph straight into
 * caller buffers, so that a replay into the same buffers copies nothing:
 *  leaves, corner_phi  device [leaf_cap] tms_leaf / [leaf_cap][8] double, or
 *                      NULL (that result stays in a private buffer);
 *  verts               device [vert_cap] tms_vertex, or NULL.
 * The buffers are borrowed: they must stay allocated while the capture is in
 * use (until the next capture or tms_destroy), and every replay overwrites
 * them.  A replay may still name other buffers; results are then copied
 * there from the bound ones.  Errors: TMS_E_CAPACITY when a bound buffer is
 * smaller than tms_graph_capacity's figure (nothing is captured and an
 * earlier capture stays); otherwise as tms_graph_capture. */
int32_t tms_graph_capture_into(tms_ctx *ctx, const tms_cells *cells, double margin,
                               tms_leaf *leaves, double *corner_phi, int64_t leaf_cap,
                               tms_vertex *verts, int64_t vert_cap);

/* Replay the captured pass on ctx's stream.  `cells` must be the captured
 * cells, or a rebuild of them with the same geometry and buffers.  Results
 * of a capture made with tms_graph_capture_into are written into the bound
 * buffers; naming those buffers here copies nothing, other buffers receive a
 * copy.
 *  leaves, corner_phi  device [leaf_cap] tms_leaf / [leaf_cap][8] double, or NULL;
 *  verts               device [vert_cap] tms_vertex, or NULL;
 *  n_leaves, n_verts   host out (or NULL);
 *  leaf_offsets, vertex_offsets  host [n_conf + 1] (or NULL): per-conformation
 *                      boundaries, as tms_batch_counts;
 *  stats               host out (or NULL).
 * Errors: TMS_E_CAPACITY when a count exceeded its captured capacity (capture
 * again with a larger margin) or an output buffer is too small (counts are
 * set); TMS_E_INVALID (no capture, other cells); TMS_E_DEVICE. */
int32_t tms_graph_launch(tms_ctx *ctx, const tms_cells *cells, tms_leaf *leaves,
                         double *corner_phi, int64_t leaf_cap, int64_t *n_leaves,
                         tms_vertex *verts, int64_t vert_cap, int64_t *n_verts,
                         int64_t *leaf_offsets, int64_t *vertex_offsets, tms_stats *stats);

/* ---- host Stage 2: the mesh (Section 2.3, manifold checks of Section 3.2) ---
 * The trilinear surface g = c (eq. linear1) of every SURFACE leaf as
 * triangles on the leaves' edge points (eq. intersection) and the extreme
 * points on their faces (eq. curve).  On each face of a leaf the curve g = c
 * is a hyperbola branch joining the face's edge points in pairs (two points:
 * joined; four: by the value of g at the face's saddle point, the same on
 * both leaves sharing the face).  The extreme points of both leaves beside a
 * face (where g = c and the derivative of g normal to the face vanishes; g
 * is trilinear, so each is an end of a straight fold segment, eq. fold1,
 * across a leaf) lie on its curve and are vertices of it in both leaves
 * (two within 1e-9 leaf edges of each other are one point; those within
 * 1e-9 leaf edges of the face's rim are left out).
 * The face segments link into closed loops on the cube's boundary.  Each
 * loop's patch is cut along the leaf's fold segments along one axis whose
 * two ends are on the loop (Section 2.3: pieces single-valued along that
 * axis) and every piece is triangulated by ear clipping in the plane normal
 * to that axis (the ear with the largest smallest angle first; candidates
 * within 1e-9 of each other keep their order, so rounding decides no
 * choice), the axes tried in order of the loop's projected area; no
 * triangle side joins two points of one cube face other than the face's
 * curve segments.  A loop that no axis admits is fanned from a point of the
 * patch inside the cube (counted).  Triangles point along -grad g (outward,
 * phi >= c inside).  Host code (threads); the inputs are copied from the
 * device.
 *
 * tms_mesh_build: leaves [n] and corner_phi [n][8] as tms_partition_estimate
 *   wrote them, verts [nv] as tms_extract_cube_vertices wrote them for those
 *   leaves (device pointers), of one conformation: the cells' only one, or
 *   one of a batch's (its ranges of the leaves and the vertices, from
 *   tms_batch_counts); leaves of several conformations are refused.
 *   The mesh's vertices are the nv edge points in that (key) order, then
 *   those of added cubes, the extreme points on leaf faces (by face, then
 *   face coordinates) and one interior point per fanned loop.  A SURFACE
 *   leaf above the finest level (a loose tau can stop a straddling cube
 *   early) is meshed through the cubes of the finest level inside it whose
 *   corner values straddle c, added as SURFACE leaves (reason
 *   TMS_REASON_SPLIT; corner values as for TMS_MESH_CLOSE below); its own
 *   edge points stay in the vertex list, unused.  *out receives a mesh owned
 *   by the caller (free it with tms_mesh_free).  An edge point within 1e-6 of its edge from a corner
 *   (a corner value equal to c puts three points on the corner) is moved to
 *   1e-6 of the edge from it, in the triangulation and in xyz.
 *   flags TMS_MESH_CLOSE: close open faces (below).  Where the bound of a
 *   coarse cube stayed clear of c although phi at the finest lattice points
 *   inside it crosses c, the surface leaves a SURFACE leaf through a face
 *   with nothing across; with the flag, every cube of the leaves' level
 *   across such a face (inside the root grid) is added as a SURFACE leaf
 *   (reason TMS_REASON_CLOSED), again for the added cubes' own open faces,
 *   up to 64 rounds.  An added cube takes the value of each corner from a
 *   SURFACE leaf with the same corner where one exists, else phi of the
 *   library at that point (as tms_eval_phi); its new edge points are placed
 *   as the extraction places them.
 *   Errors: TMS_E_INVALID (arguments, unknown flags, several levels, an edge
 *   point missing from verts), TMS_E_OOM, TMS_E_DEVICE.
 * tms_mesh_info: vertex and triangle counts, loops, fanned loops, and the
 *   faces of SURFACE leaves whose corner values cross c but that have no
 *   SURFACE leaf across (the surface is open there).
 * tms_mesh_get: host copies: xyz [nv][3], tri [nt][3] (vertex indices),
 *   tri_leaf [nt] (index of the triangle's leaf in the caller's list, n + k
 *   for the k-th added cube); any pointer may be NULL.
 * tms_mesh_added: host copies of the added cubes, split and closing ones
 *   (leaves [k], corner_phi [k][8]); *n_out = k; both NULL: only count;
 *   TMS_E_CAPACITY if cap < k.
 * tms_mesh_check: the three conditions of a manifold mesh (Section 3.2):
 *   (a) every edge shared by exactly two triangles (and traversed in opposite
 *   directions), (b) the neighbourhood of every vertex a single loop, (c) no
 *   pair of closed triangles that share no vertex and meet (tested among the
 *   triangles of the same or touching leaves, decided by exact orientation
 *   signs after a quick test in doubles; skipped, reported -1, when
 *   intersections = 0).  Non-manifold vertices are those failing (a) or (b).
 *   Also connected components, Euler characteristic V - E + F, area, enclosed
 *   volume, vertices per unit area, and the uniformness of the triangles
 *   (Section 1 lists sharp angles and zero-area elements among the defects
 *   of a mesh): the smallest angle, the triangles with an angle below 5
 *   degrees, and those whose area is at most 1e-12 of their longest side
 *   squared.
 * tms_mesh_write_off: the mesh as an OFF file. */
#define TMS_MESH_CLOSE 1
typedef struct tms_mesh tms_mesh;
typedef struct {
    int64_t n_vertices, n_triangles, n_loops, n_fallback, open_faces;
    int64_t added_cubes;          /* cubes added across open faces         */
    int64_t boundary_edges;       /* (a): sides in one triangle            */
    int64_t nonmanifold_edges;    /* (a): sides in more than two triangles */
    int64_t misoriented_edges;    /* (a): two triangles, same direction    */
    int64_t nonmanifold_vertices; /* vertices failing (a) or (b)           */
    int64_t intersecting_pairs;   /* (c), or -1 when not tested           */
    int64_t components, euler, unused_vertices;
    double area, volume, density; /* A^2, A^3, vertices per A^2           */
    double min_angle;             /* smallest triangle angle, degrees      */
    int64_t small_angles;         /* triangles with an angle below 5 deg   */
    int64_t zero_area;            /* triangles of area <= 1e-12 side^2     */
} tms_mesh_report;

int32_t tms_mesh_build(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves, int64_t n,
                       const double *corner_phi, const tms_vertex *verts, int64_t nv,
                       int32_t flags, tms_mesh **out);
/* The same from host arrays (leaves [n], corner_phi [n][8], verts [nv] in
 * ascending key order), with the isovalue c, the finest level K and the root
 * edge h0 of the cells they came from, without phi: no closing, and every
 * SURFACE leaf must have the same level (TMS_E_INVALID otherwise); errors as
 * above, with the message in msg. */
int32_t tms_mesh_build_host(const tms_leaf *leaves, int64_t n, const double *corner_phi,
                            const tms_vertex *verts, int64_t nv, double c, int32_t K, double h0,
                            tms_mesh **out, char *msg, int64_t msg_len);
int32_t tms_mesh_info(const tms_mesh *m, int64_t *n_vertices, int64_t *n_triangles,
                      int64_t *n_loops, int64_t *n_fallback, int64_t *open_faces);
int32_t tms_mesh_get(const tms_mesh *m, double *xyz, int32_t *tri, int32_t *tri_leaf);
int32_t tms_mesh_added(const tms_mesh *m, tms_leaf *leaves, double *corner_phi, int64_t cap,
                       int64_t *n_out);
int32_t tms_mesh_check(const tms_mesh *m, int32_t intersections, tms_mesh_report *report);
int32_t tms_mesh_write_off(const tms_mesh *m, const char *path);
int32_t tms_mesh_free(tms_mesh *m);

/* ---- tuning ---------------------------------------------------------------
 * Launch-shape knobs of the partition pass.  Results do not depend on them
 * (every cube's arithmetic is the same under any setting); only the time
 * does.  Defaults: slice_cubes 2^26, tiled_min_level 1, tile_atoms 8,
 * proj_table 1, tiled_persistent 0, tiled_half 0, corner_groups 2,
 * corner_reach 48.  A captured pass takes
 * them as they are at capture, except that its whole-wave tiled launches are
 * always one workgroup per chunk (sized from the eager pass's chunk count). */
typedef struct {
    int64_t slice_cubes;     /* largest queue slice per estimate + bound
                                launch (a level is cut into ceil(n / this)
                                equal slices); the staged tensors take
                                512 B per entry (>= 4096)                   */
    int32_t tiled_min_level; /* first level estimated one wavefront per chunk
                                of <= 64 cubes of one root (levels 0 and 1:
                                eight roots per wavefront, one 8-lane group
                                each, a level-0 root being one cube and a
                                level-1 root at most 8) (0..3; 4: none; the
                                levels before it and those above 3 use one
                                thread per cube)                             */
    int32_t tile_atoms;      /* atoms staged per LDS tile of that kernel:
                                8, 16 or 32                                  */
    int32_t proj_table;      /* 1: the tiled levels first tabulate every
                                atom's 1-D projections (Section 2.2.1) on
                                the intervals within R_c of it (48 B per
                                atom, axis and interval: about
                                3 * ceil(2 R_c / h) + 9 entries per atom at
                                spacing h) and gather from that table
                                (a level whose table does not fit in
                                device memory projects in place);
                                0: each chunk projects in place          */
    int32_t tiled_persistent; /* 1: the tiled estimate runs a fixed grid of
                                workgroups that draw chunks from per-XCD
                                counters (each XCD walks its chunks in
                                order); 0: one workgroup per chunk        */
    int32_t tiled_half;      /* 1: levels 2-3 in chunks of <= 32 cubes, two
                                per wavefront (half-wave groups, each with
                                its own atom stream); 2: level 2 so, level 3
                                whole-wave; 0: one chunk of <= 64 cubes per
                                wavefront                                   */
    int32_t corner_groups;   /* phi at the unique leaf corners: 0 one thread
                                per point; 1..8: a wavefront stages the
                                atoms near its 64 points in LDS once per
                                spatial group of them, for up to this many
                                groups (a wavefront needing more sums its
                                points one by one).  Values are
                                bit-identical under every setting          */
    int32_t corner_reach;    /* a group holds the points within
                                corner_reach / 16 R_c of its first point
                                along each axis (1..64)                     */
    int32_t reserved;        /* 0                                          */
} tms_tuning;

/* Set / read ctx's tuning.  Errors: TMS_E_INVALID (values out of range). */
int32_t tms_set_tuning(tms_ctx *ctx, const tms_tuning *t);
int32_t tms_get_tuning(tms_ctx *ctx, tms_tuning *t);

/* Autotuner: times tms_partition_estimate on `cells` (count only, device
 * results discarded) under candidate tunings -- atoms per tile, then the
 * projection table on or off, the tiled grid (persistent or one workgroup
 * per chunk), half-wave chunks (off, levels 2-3, level 2), the first tiled
 * level, then the slice size, each with the others at their best so far --
 * checks that every candidate gives the same leaf and cube counts, and
 * leaves the fastest set on ctx.
 *  best     host out (or NULL): the chosen tuning.
 *  best_ms  host out (or NULL): its wall time in ms.
 *  n_tried  host out (or NULL): passes timed.
 * Errors: those of tms_partition_estimate; TMS_E_DEVICE if two candidates
 * disagree. */
int32_t tms_autotune(tms_ctx *ctx, const tms_cells *cells, tms_tuning *best, double *best_ms,
                     int32_t *n_tried);

/* ---- device-time instrumentation ----------------------------------------
 * When enabled, the library brackets its kernel launches with HIP events on
 * the context's stream and accumulates the elapsed device time per phase
 * (TMS_T_* slots).  Off by default; costs two event records per launch. */
#define TMS_T_BUILD 0    /* binning and neighbourhood lists           */
#define TMS_T_ESTIMATE 1 /* tensor estimate, one thread per cube        */
#define TMS_T_DECIDE 2   /* decision / nested-SVD bound kernels        */
#define TMS_T_GUARD 3    /* double-precision recomputation of guards   */
#define TMS_T_COMPACT 4  /* scans, queue and leaf compaction           */
#define TMS_T_CORNER 5   /* corner de-duplication and gathering        */
#define TMS_T_PHI 6      /* phi kernels (corner values, tms_eval_phi)   */
#define TMS_T_EXTRACT 7  /* edge de-duplication and vertex emission    */
#define TMS_T_TILED 8    /* tensor estimate, one wave per chunk of
                            cubes of one root (tiled levels)           */
#define TMS_T_BACKWARD 9 /* adjoint kernels                             */
#define TMS_T_TABLE 10   /* per-level projection tables                */
#define TMS_T_GROUPED 11 /* tensor estimate, eight level-1 roots per
                            wavefront                                  */
#define TMS_T_STAGE2 12  /* stage-two points (tms_stage2_points)       */
#define TMS_T_SLOTS 13

typedef struct {
    double ms[TMS_T_SLOTS];       /* accumulated device milliseconds */
    int64_t launches[TMS_T_SLOTS];/* kernel launches timed           */
} tms_timing;

/* Enable (1) or disable (0) per-phase device timing on ctx. */
int32_t tms_set_timing(tms_ctx *ctx, int32_t enable);

/* Copy the accumulated timings into *out (host); reset them if reset != 0. */
int32_t tms_get_timing(tms_ctx *ctx, tms_timing *out, int32_t reset);

/* Debug: the coefficient tensor A (eqs. polynew, tensor1, tensor2) of given
 * cubes, computed by the same kernels as the partition pass.
 *  cubes  device [n][4] int32 (level, ix, iy, iz);  A device [n][64] double,
 *  A[16 j + 4 k + l], j/k/l the x/y/z Legendre degrees.
 *  S      device [n] double or NULL: the l1 scale sum_i w_i |a~x|_1 |a~y|_1
 *         |a~z|_1 that sizes the single-precision error band.
 *  precision TMS_PREC_* (FP32 results are widened to double). */
int32_t tms_debug_tensor(tms_ctx *ctx, const tms_cells *cells, const int32_t *cubes, int64_t n,
                         int32_t precision, double *A, double *S);

/* Debug: the nested-SVD bound (Section 2.2.2, eqs. SVD1-SVD7, Sxyz,
 * bound1-bound3) of given tensors.
 *  A     device [n][64] double;
 *  band  device [n] double or NULL (zeros): l1 perturbation size for the
 *        stability flag;
 *  out   device [n][6] double: L, U, rho (l1 mass of the residual tensor),
 *        r (outer rank kept by the 0.99 rule), jump (largest move of L and U
 *        that a 0.99 rank rule flipping within the perturbation band could
 *        cause; 0 if none can flip), amp (first-order factor by which an l1
 *        perturbation of A of size band can move L and U). */
int32_t tms_debug_bound(tms_ctx *ctx, const double *A, const double *band, int64_t n,
                        double *out);

/* Debug: the number of (point, atom) pairs within R_c that phi at m points
 * sums (the terms of eq. Gaussian1 kept by the cut-off), i.e. the
 * algorithmic work of tms_eval_phi and of the corner values on these points.
 *  pts device [m][3] double; *pairs host out.  Cells of one conformation.
 * Errors: TMS_E_INVALID, TMS_E_DEVICE. */
int32_t tms_debug_phi_pairs(tms_ctx *ctx, const tms_cells *cells, const double *pts, int64_t m,
                            int64_t *pairs);

/* Debug: the exponential used by TMS_PREC_FP32_GUARD, y[i] = exp(x[i]) for
 * x[i] <= 0, computed as 2^n 2^f with n, f split in double precision and 2^f
 * from the single-precision hardware exponential.  Its relative error is
 * bounded by 1.5e-7 (one unit in the last place of the single-precision
 * result plus the rounding of f); the guard band of the FP32+guard path
 * rests on that bound.  x, y device [n] double. */
int32_t tms_debug_fast_exp(tms_ctx *ctx, const double *x, int64_t n, double *y);

#ifdef __cplusplus
}
#endif
#endif /* TMS_H */
