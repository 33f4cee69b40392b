// Internal declarations shared by the host orchestration and the HIP kernels
// of the gfx950 partition/estimation library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tms.h"

namespace tms {

// Dense bitmaps over lattices of points, one bit per point, bit index
// (X * ny + Y) * nz + Z (X-major, which is also the order of the packed
// keys).  Sub-lattices start on 64-bit word boundaries.
struct Lat {
    int64_t n[3];   // points per axis
    int64_t base;   // first word
};
// Edge lattices: one per (level, axis), at the level's resolution, laid out
// level-major then axis, so the bit order is the edge-key order.
struct EdgeLat {
    Lat l[TMS_MAX_LEVELS][3];
    int64_t words;
    // leaf lattices: one bit per cube of each level, 4x4x4 blocks per word
    // (n = blocks per axis), bases in a bitmap of their own
    Lat leaf[TMS_MAX_LEVELS];
};

// ---------------------------------------------------------------------------
// Geometry of one conformation.  A batch keeps one per conformation in a
// device table (kernels index it by the conformation id carried by each
// cube, leaf and point); the method's parameters (h0, hmin, D, c, tau, K)
// are the same in every entry.
// ---------------------------------------------------------------------------
struct Grid {
    double o[3];     // origin of the root grid (multiple of h0)
    double h0;       // root cube edge
    double hmin;     // finest cube edge
    double D, c, tau;
    double rc2;      // squared cut-off radius (this conformation's largest radius)
    double cs;       // atom-cell edge (smallest h0 * 2^m >= R_c / 4)
    double inv_cs;   // 1 / cs when cs is a power of two (division by it is then
                     // exact scaling, so x * inv_cs == x / cs), else 0
    double inv_h0;   // 1 / h0 when h0 is a power of two, else 0 (likewise)
    int32_t nr[3];   // root cubes per axis
    int32_t nc[3];   // atom cells per axis
    int32_t K;       // finest level
    int32_t deg;     // degree n of the 1-D series (1..3; entries above n are 0)
    int32_t span;    // cell stencil half-width, ceil(R_c / cs)
    int64_t root_base;  // first root / cell / atom of this conformation in the
    int64_t cell_base;  // batch-wide root, cell and atom arrays
    int64_t atom_base;
    Lat clat;           // its block of the batch's corner bitmap
};

// Gauss-Legendre rule folded for the even/odd parts of a function on [-1,1]:
// with f+ = f(t_q) + f(-t_q), f- = f(t_q) - f(-t_q) for the positive nodes t_q,
//   a0 = sum c0 f+,  a1 = sum c1 f-,  a2 = sum c2 f+,  a3 = sum c3 f-
// gives the four Legendre projection coefficients (2j+1)/2 int f L_j.
// cs[q] = |c0| + |c1| + |c2| + |c3| at node q (error propagation).
template <typename T>
struct GLRule {
    T t[8], c0[8], c1[8], c2[8], c3[8], cs[8];
};

// Per-level table of the 1-D projections of Section 2.2.1 (eq. 1D-project):
// for every atom i, axis a and interval j of the level's lattice within R_c
// of the atom along that axis, the four Legendre coefficients of the atom's
// Gaussian factor on that interval, their exponential error bound and the
// squared distance from the atom to the interval, at
// t[6 * ((a * n + i) * ns + (j - first))], first = one interval below the
// one holding x_a - R_c (every kernel evaluates the same expression for it).  Projections farther than R_c are zero.  Built once
// per level; the tiled estimate gathers from it instead of recomputing each
// projection for every chunk that needs it.
struct ProjTab {
    const double *t = nullptr;   // null: projections are computed in place
    int64_t n = 0;               // atoms
    int ns = 0;                  // intervals per (axis, atom)
};

// Number of positive nodes (half the rule) used on a level whose cubes have
// half-width s: chosen from beta = s sqrt(D) so that the quadrature error of
// the projection stays below the arithmetic's own rounding.
int gl_half_nodes(double beta, bool fp32);
template <typename T>
GLRule<T> gl_rule(int half);

// Decision codes of the per-cube state machine.
enum : uint8_t {
    DEC_DISCARD = 0,
    DEC_REFINE = 1,
    DEC_CONV = 2,   // converged leaf
    DEC_HMIN = 3,   // kept at the finest level
    DEC_GUARD = 4,  // single-precision margin too small: redo in double
};

// ---------------------------------------------------------------------------
// Device buffer that only grows.
// ---------------------------------------------------------------------------
// Device buffer, grow-only; freed by release() or when its owner (a context,
// cells or graph state) is deleted, with the owner's device current.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), cap(o.cap) {
        o.p = nullptr;
        o.cap = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            cap = o.cap;
            o.p = nullptr;
            o.cap = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    hipError_t ensure(size_t bytes);
    void release();
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Pinned (page-locked) host buffer, grow-only: device-to-host copies of
// counts land here by DMA and are then copied out on the host.
struct PinBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes);
    void release();
    ~PinBuf() { release(); }
};

}  // namespace tms

// ---------------------------------------------------------------------------
// Public opaque types.
// ---------------------------------------------------------------------------
struct tms_cells {
    tms::Grid g{};               // geometry of conformation 0 (the only one unless batched)
    tms_params p{};
    int32_t nconf = 1;           // conformations in the batch
    std::vector<tms::Grid> gh;   // geometry per conformation (host copy of gtab)
    std::vector<int64_t> atom_off;  // [nconf + 1] atom offsets of the conformations
    int64_t corner_words = 0;    // words of the batch's corner bitmap
    int64_t n = 0;               // atoms
    int64_t nroots = 0;          // root cubes, all conformations
    int64_t ncells = 0;
    int64_t n_root_entries = 0;  // sum of root neighbourhood sizes
    int64_t n_nonempty = 0;      // roots with a non-empty neighbourhood
    double rmax = 0;
    uint64_t id = 0;             // changes with every build (kept results name it)
    // device memory, atoms sorted by cell (ascending original index inside a cell)
    tms::DevBuf ax, ay, az, aw, aidx, ar;   // double x3, w = exp(D r^2), int32 index, r
    tms::DevBuf axw;                        // double4 (x, y, z, w) per atom, cell order
    tms::DevBuf cell_start;                 // int32 [ncells + 1]
    tms::DevBuf root_start;                 // int32 [nroots + 1]
    tms::DevBuf root_atoms;                 // int32 [n_root_entries]
    tms::DevBuf tmp_key, tmp_cnt;           // scratch for binning
    tms::DevBuf gtab;                       // Grid [nconf] (device geometry table)
    tms::DevBuf aoff;                       // int64 [nconf + 1]
    void release();
};

// queue slices per level at most (estimate + bound launches)
constexpr int64_t kMaxSlices = 256;
// device buffers of a cells object that a captured pass reads
constexpr int kCellsBufs = 9;

// A pass recorded once into a HIP graph with every size kept on the device
// (capacity-sized launches), replayed without host round trips.
struct tms_graph_state {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    uint64_t cells_id = 0;          // cells build the graph was recorded for
    const void *cells_buf[kCellsBufs] = {};  // their device buffers (a rebuild must keep them)
    std::vector<tms::Grid> gh;      // and their geometry
    int64_t n_atoms = 0;            // and atom count and per-conformation offsets
    std::vector<int64_t> atom_off;  // (launch sizes and the projection table's rows)
    int nlev = 0, nconf = 1;
    int64_t qcap[TMS_MAX_LEVELS + 1] = {}, lcap = 0, ucap = 0, vcap = 0, ewords = 0, lwords = 0;
    int64_t nslices[TMS_MAX_LEVELS] = {}, slice[TMS_MAX_LEVELS] = {};
    int64_t ccap[TMS_MAX_LEVELS][kMaxSlices] = {};  // chunks per slice launch of a tiled level
    tms::DevBuf q[2], dec, abuf, ebuf, hidx, flags, scan_a, scan_b, idx, runs, chunks, chunks2,
        leaves, lsort, cphi, bmap, bmcnt, bmoff, uniq, uphi, uconf, uguard, ebmap, ebcnt,
        eboff, eown, lbmap, verts, etab, sz, ctr, stmp, seg, ptab;
    bool proj_table = false;        // recorded with projection tables
    bool leaves_in_lsort = false;   // a batch's regrouped leaves end in lsort
    // caller buffers the pass writes its results into (null: private ones)
    tms_leaf *out_leaves = nullptr;
    double *out_cphi = nullptr;
    tms_vertex *out_verts = nullptr;
    void release();
};

struct tms_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // device address of the library's static scratch array on this device
    // (tms_eval_phi_noalloc); resolved once per device by tms_create
    unsigned char *noalloc_scratch = nullptr;
    std::string err;
    std::vector<tms_cells *> cells;
    // last partition result
    tms::DevBuf leaves, corner_phi;
    int64_t n_leaves = 0;
    // last extract result
    tms::DevBuf verts;
    int64_t n_verts = 0;
    // unique corners of the last corner stage (uniq, uphi; ranks in the dense
    // corner bitmap bmap/bmoff when corner_dense) and the edge bitmaps of the
    // last extraction (ebmap/eboff when edge_dense); kept for the adjoint
    int64_t n_corners = 0;
    uint64_t corner_cells = 0, edge_cells = 0;  // tms_cells::id they belong to
    bool corner_dense = false, edge_dense = false;
    tms::EdgeLat edge_lat{};
    tms::DevBuf ebmap, ebcnt, eboff, eown, lbmap, wbar, uconf, etab, lsort, ctab;
    // batch bookkeeping of the last partition / extraction: per-conformation
    // leaf and vertex offsets ([nconf + 1] each)
    std::vector<int64_t> leaf_off, vert_off;
    // counters of the last partition (sizes the capture), and the capture
    tms_stats last_stats{};
    uint64_t last_stats_cells = 0;
    int64_t last_chunks[TMS_MAX_LEVELS] = {};  // whole-wave chunks per level of that pass (-1: none)
    // and their starts per kChunkBin queue positions (empty: not chunked so)
    std::vector<int32_t> last_chunk_bins[TMS_MAX_LEVELS];
    tms::DevBuf chist;
    tms_graph_state graph;
    // workspace (grow-only)
    tms::DevBuf q[2], qmeta, abuf, ebuf, dec, scan_a, scan_b, scan_c, flags, idx, uniq, uphi,
        uguard, ctmp, hidx, chunks, chunks2, runs, bmap, bmcnt, bmoff;
    // small device counters (u64 slots): [0,64) striped pair counts,
    // [72,77) decision histogram, 80 surface count, 96 adjoint consistency
    // flag, 100 scan total, 104 and 105 a level's leaf and child totals,
    // 112 stage-two degenerate count, 113 phi pair count;
    // [256, 256 + 5*1024) reduction partials;
    // [8192, 8192 + 512) hard-list lengths of the queue slices
    // tuning (results do not depend on it): queue entries per estimate
    // slice, first level estimated by the tiled kernel, atoms per LDS tile
    int64_t slice_cubes = (int64_t)1 << 26;
    int tiled_min_level = 1;
    int tile_atoms = 8;
    int tiled_half = 0;  // half-wave chunks of <= 32 cubes: 1 levels 2-3, 2 level 2
    int corner_groups = 2;  // spatial groups per wavefront of the corner phi kernel
    int corner_reach = 48;  // their reach, in R_c / 16
    int proj_table = 1;     // tiled levels gather 1-D projections from a table
    tms::DevBuf ptab;       // that table
    tms::DevBuf asave[2];   // re-expanded child tensors: every entry's tensor of
                            // the last two levels (by queue index)
    tms::DevBuf qpar;       // parent queue index of each group of 8 children
    tms::DevBuf tick;       // [8] chunk slot counters of the tiled estimate
    bool tiled_dyn = false; // eager tiled launches draw chunks from them
    tms::DevBuf counters;
    tms::PinBuf pin;       // pinned staging of device-to-host reads
    // whether the last partition's leaves and corner values, and the last
    // extraction's vertices, are kept in ctx (false: they went straight into
    // the caller's buffers)
    bool leaves_kept = true, cphi_kept = true, verts_kept = true;
    // per-phase device timing (HIP events on `stream`)
    bool timing = false;
    int tdepth = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double t_ms[TMS_T_SLOTS] = {0};
    int64_t t_launch[TMS_T_SLOTS] = {0};
};

namespace tms {
// Brackets the launches issued in its scope with events when timing is on.
struct TimedScope {
    tms_ctx *ctx;
    int slot;
    hipEvent_t e1 = nullptr;
    TimedScope(tms_ctx *c, int s);
    ~TimedScope();
};
void timing_flush(tms_ctx *ctx);
}  // namespace tms

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files).
// ---------------------------------------------------------------------------
namespace tms {

// k_cells.hip -- batch-wide arrays; gt: device table of nconf geometries
// per conformation {min xyz, max xyz, max r, min r, non-finite count};
// tmp: atom_stats_tmp_bytes of scratch
size_t atom_stats_tmp_bytes(int nconf, int64_t max_atoms);
hipError_t launch_atom_stats(const double *xyzr, const int64_t *off, int nconf, int64_t max_atoms,
                             double *out, double *tmp, hipStream_t s);
hipError_t launch_bin_atoms(const Grid *gt, int nconf, const double *xyzr, int64_t n, int32_t *key,
                            int32_t *cnt, hipStream_t s);
hipError_t launch_scatter_atoms(const Grid *gt, const double *xyzr, int64_t n, const int32_t *key,
                                int32_t *fill, double *ax, double *ay, double *az, double *aw,
                                double *ar, int32_t *aidx, hipStream_t s);
hipError_t launch_pack_atoms(const double *ax, const double *ay, const double *az, const double *aw,
                             int64_t n, double4 *xw, hipStream_t s);
hipError_t launch_sort_cells(const int32_t *cell_start, int64_t ncells, double *ax, double *ay,
                             double *az, double *aw, double *ar, int32_t *aidx, hipStream_t s);
hipError_t launch_root_count(const Grid *gt, int nconf, const int32_t *cell_start,
                             const double4 *xw, int64_t nroots, int32_t *cnt, hipStream_t s);
hipError_t launch_root_fill(const Grid *gt, int nconf, const int32_t *cell_start,
                            const double4 *xw, int64_t nroots, const int32_t *start,
                            int32_t *atoms, hipStream_t s);

// k_adjoint.hip
hipError_t launch_adjoint_fold(const Grid &g, const Lat &lat, const uint64_t *cbm,
                               const int32_t *coff, const double *upts, const double *uphi,
                               int64_t m, const double *dphi, const EdgeLat &el,
                               const uint64_t *ebm, const int32_t *eoff, const double *dt,
                               double *wbar, unsigned *bad, hipStream_t s);
hipError_t launch_adjoint_atoms(const Grid &g, int precision, const Lat &lat, const uint64_t *cbm,
                                const int32_t *coff, const double *upts, const double *wbar,
                                int64_t n, const double *ax, const double *ay, const double *az,
                                const double *aw, const double *ar, const int32_t *aidx,
                                double *out, hipStream_t s);

// k_stage2.hip -- per-leaf record counts (and the degenerate total, added
// to *ndeg), then the records at the scanned offsets
hipError_t launch_s2_count(const Grid *gt, const tms_leaf *leaves, const double *cphi, int64_t n,
                           int32_t *cnt, unsigned long long *ndeg, hipStream_t s);
hipError_t launch_s2_emit(const Grid *gt, const tms_leaf *leaves, const double *cphi, int64_t n,
                          const int32_t *off, tms_s2point *out, int64_t leaf0, hipStream_t s);

// k_graph.hip
hipError_t launch_slice_counts(const int32_t *n, int64_t S, int nslices, int32_t *ns,
                               hipStream_t s);
hipError_t launch_acc_i64(int64_t *acc, const int32_t *v, hipStream_t s);
hipError_t launch_seg_plan(const int64_t *src, int nlev, int nconf, const int64_t *L, int64_t lcap,
                           int64_t *dst, int64_t *leaf_off, hipStream_t s);
hipError_t launch_stop_on_overflow(const unsigned *ovf, int32_t *n, hipStream_t s);

// k_scan.hip -- exclusive scan of int32 values into int32 offsets; total
// written to *total_dev (device).  tmp must hold scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                          void *tmp, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// phi of conformation conf of cells at m device points (as tms_eval_phi;
// batch cells allowed); synchronizes the context's stream
int32_t eval_phi_conf(tms_ctx *ctx, const tms_cells *cells, int conf, const double *pts,
                      int64_t m, double *phi);
// out[i] = src[idx[i]]
hipError_t launch_gather_i32(const int32_t *src, const int64_t *idx, int n, int64_t *out,
                             hipStream_t s);

// k_partition.hip
hipError_t launch_roots_flags(const int32_t *root_start, int64_t nroots, int32_t *flags,
                              hipStream_t s);
hipError_t launch_roots_emit(const Grid *gt, int nconf, const int32_t *flags, const int32_t *off,
                             int64_t nroots, int4 *q, hipStream_t s);
// g: the batch's shared parameters (host copy); gt: device geometry table
hipError_t launch_estimate(const Grid &g, const Grid *gt, int level, int precision, const int4 *q,
                           int64_t n,
                           const int32_t *subset, const int32_t *root_start,
                           const int32_t *root_atoms, const double *ax, const double *ay,
                           const double *az, const double *aw, double *A, double *E,
                           int64_t *pairs, hipStream_t s);
// estimate + easy decisions; cubes needing the bound go to the hard list.
// chunks != nullptr selects the tiled kernel (levels 2..3); chunk positions
// index the subset list when one is given.
hipError_t launch_estimate_decide(const Grid &g, const Grid *gt, int level, int precision,
                                  const int4 *q, int64_t n,
                                  const int32_t *subset, const int2 *chunks, int64_t nchunks,
                                  const int32_t *root_start, const int32_t *root_atoms,
                                  const double *ax, const double *ay, const double *az,
                                  const double *aw, uint8_t *dec, double *hardA, double *hardE,
                                  int32_t *hardIdx, unsigned *hardCount, int64_t *pairs,
                                  int tile_atoms, hipStream_t s, const int32_t *ncount = nullptr,
                                  const ProjTab &pt = ProjTab{}, unsigned *tick = nullptr,
                                  bool half = false, unsigned *ovf = nullptr,
                                  double *allA = nullptr, int64_t hs = 0, int64_t as = 0);
// intervals per (axis, atom) of the projection table of a level
int proj_table_slots(const tms_cells *cells, int level);
// fill the projection table (t: [3 n ns][6] doubles)
hipError_t launch_proj_table(const Grid &g, const Grid *gt, int nconf, int level, int precision,
                             const double *ax, const double *ay, const double *az, int64_t n,
                             int ns, double *t, hipStream_t s);
// The hard list (hardA, hardE, hardIdx) has hs slots: hardA holds the
// tensors with entry pairs outermost, pair e of slot k at double2 e * hs + k.
hipError_t launch_bound(const Grid &g, int level, int precision, int64_t max_n, uint8_t *dec,
                        double *hardA, double *hardE, int32_t *hardIdx, unsigned *hardCount,
                        hipStream_t s, int64_t hs);
// Trailing device-count arguments (nd: count on the device, n then a
// capacity that sizes the launch) are for the capture path; null elsewhere.
hipError_t launch_run_flags(const Grid *gt, int level, const int4 *q, const int32_t *subset,
                            int64_t n, int32_t *f, hipStream_t s, const int32_t *nd = nullptr);
hipError_t launch_run_starts(const int32_t *f, const int32_t *off, int64_t n, int32_t *starts,
                             hipStream_t s);
// chunks of at most cmax (<= 64) consecutive entries of one run
hipError_t launch_run_chunk_counts(const int32_t *starts, int64_t nruns, int64_t n, int32_t *cnt,
                                   hipStream_t s, const int32_t *nrd = nullptr,
                                   const int32_t *nd = nullptr, int cmax = 64);
hipError_t launch_run_chunk_emit(const int32_t *starts, int64_t nruns, int64_t n,
                                 const int32_t *coff, int2 *chunks, hipStream_t s,
                                 const int32_t *nrd = nullptr, const int32_t *nd = nullptr,
                                 int cmax = 64);
// chunk starts of a slice (n chunks, ascending starts relative to the slice
// at level position off, len entries) added to hist[bin] for the bins of
// kChunkBin level positions the slice touches (hist zeroed per level)
constexpr int64_t kChunkBin = 65536;
hipError_t launch_chunk_bins(const int2 *chunks, int64_t n, int64_t off, int64_t len,
                             int32_t *hist, hipStream_t s);
// the n chunks (ncount: their device count, or null) reordered into out by
// the length of their root's atom list, longest first; bkt: [n] scratch,
// bcnt and boff: [chunks_by_length_scratch(n)] scratch each, tmp: scan
// scratch for that many entries
constexpr int kLenBuckets = 256;
int64_t chunks_by_length_scratch(int64_t n);
hipError_t launch_chunks_by_length(const Grid *gt, int level, const int4 *q, const int2 *chunks,
                                   int64_t n, const int32_t *ncount, const int32_t *root_start,
                                   int32_t *bkt, int32_t *bcnt, int32_t *boff, void *tmp,
                                   int2 *out, hipStream_t s);
hipError_t launch_level_counts(const uint8_t *dec, int64_t n, int32_t *leaf_cnt,
                               int32_t *child_cnt, hipStream_t s, const int32_t *nd = nullptr);
hipError_t launch_level_emit(const int4 *q, const uint8_t *dec, int64_t n, int level,
                             const int32_t *leaf_off, const int32_t *child_off, tms_leaf *leaves,
                             int64_t leaf_base, int4 *qnext, hipStream_t s,
                             const int32_t *nd = nullptr, const int64_t *leaf_base_dev = nullptr,
                             int64_t leaf_cap = 0, int64_t queue_cap = 0, unsigned *ovf = nullptr,
                             int32_t *qpar = nullptr);
// child tensors re-expanded from their parents' (eq. childtensor) for n
// entries of a level starting at off (q, dec, hard list as for the estimate);
// Apar: the previous level's tensors by queue index (aps entries, pair e of
// entry k at double2 e * aps + k), qpar[j]: the parent of entries
// 8 j .. 8 j + 7; allA: where this level's tensors go (as entries, the same
// layout; offset to the slice), or null
hipError_t launch_reexpand(const Grid &g, int level, const int4 *q, int64_t n, int64_t off,
                          const double *Apar, int64_t aps, const int32_t *qpar, uint8_t *dec,
                          double *hardA, double *hardE, int32_t *hardIdx, unsigned *hardCount,
                          double *allA, hipStream_t s, int64_t hs, int64_t as);
hipError_t launch_level_histo(const uint8_t *dec, int64_t n, unsigned long long *h5,
                              unsigned long long *part, hipStream_t s, const int32_t *nd = nullptr);
// regrouping of a batch's leaves by conformation (segments level * nconf + conf)
hipError_t launch_leaf_seg_heads(const tms_leaf *leaves, int64_t n, int nconf, int64_t *src,
                                 hipStream_t s, const int64_t *nd = nullptr);
hipError_t launch_leaf_seg_move(const tms_leaf *leaves, int64_t n, int nconf, const int64_t *src,
                                const int64_t *dst, tms_leaf *out, hipStream_t s,
                                const int64_t *nd = nullptr);
hipError_t launch_bound_debug(const double *A, const double *band, int64_t n, double *out,
                              hipStream_t s);
hipError_t launch_fast_exp_debug(const double *x, int64_t n, double *y, hipStream_t s);

// k_phi.hip
// pconf: conformation of every point (NULL: all in conformation 0)
// xw: the cells' packed atoms (x, y, z, w)
hipError_t launch_phi_points(const Grid *gt, const int32_t *pconf, int precision, const double *pts,
                             int64_t m, const int32_t *cell_start, const double4 *xw,
                             double band_rel, double *phi, double *grad, uint8_t *guard,
                             hipStream_t s, const int32_t *nd = nullptr);
// phi at unique corner points in bitmap-rank order (no gradient): up to
// `groups` (<= 8) spatial groups per wavefront sum over atoms staged in LDS (points
// within reach R_c of a group's first point per axis); 0: launch_phi_points.
// Values bit-identical to launch_phi_points'.
hipError_t launch_phi_corners(const Grid *gt, const int32_t *pconf, int precision,
                              const double *pts, int64_t m, const int32_t *cell_start,
                              const double4 *xw, double band_rel, int groups, double reach,
                              double *phi, uint8_t *guard, hipStream_t s,
                              const int32_t *nd = nullptr);
hipError_t launch_phi_points_subset(const Grid *gt, const int32_t *pconf, const double *pts,
                                    const int32_t *list, int64_t m, const int32_t *cell_start,
                                    const double4 *xw, double *phi, double *grad, hipStream_t s,
                                    const int32_t *nd = nullptr);
hipError_t launch_uniform_leaves(const Grid &g, tms_leaf *leaves, int64_t n, hipStream_t s);
hipError_t launch_uniform_points(const Grid &g, double *pts, int64_t m, hipStream_t s);
hipError_t launch_uniform_gather(const Grid &g, const double *uphi, double c, tms_leaf *leaves,
                                 int64_t n, double *corner_phi, hipStream_t s);
hipError_t launch_count_u8(const uint8_t *v, int64_t n, uint8_t value,
                           unsigned long long *count, hipStream_t s);
hipError_t launch_guard_flags_u8(const uint8_t *g, int64_t n, int32_t *flags, hipStream_t s,
                                 const int32_t *nd = nullptr);
hipError_t launch_list_emit(const int32_t *flags, const int32_t *off, int64_t n, int32_t *list,
                            hipStream_t s);
// *count += the (point, atom) pairs within R_c over m points (conformation 0)
hipError_t launch_phi_pairs(const Grid *gt, const double *pts, int64_t m, const int32_t *cs,
                            const double4 *xw, unsigned long long *count, hipStream_t s);
// indices i < n with gd[i] != 0 appended to list at slots taken from *cnt
// (which the caller zeroes); order arbitrary
hipError_t launch_guard_append(const uint8_t *gd, int64_t n, int32_t *list, unsigned *cnt,
                               hipStream_t s);
hipError_t launch_count_surface(const tms_leaf *leaves, int64_t n, unsigned long long *count,
                                unsigned long long *part, hipStream_t s,
                                const int64_t *nd = nullptr);

// bitmap helpers (k_phi.hip)
hipError_t launch_popc(const uint64_t *bm, int64_t nwords, int32_t *cnt, hipStream_t s);
// corner bitmap: conformation L.conf owns the words of gt[L.conf].clat
hipError_t launch_corner_mark(const tms_leaf *leaves, int64_t n, int K, const Grid *gt,
                              unsigned long long *bm, hipStream_t s, const int64_t *nd = nullptr);
// unique corner points and their conformations at their ranks, from the bitmap
hipError_t launch_corner_enum(const Grid *gt, int nconf, const uint64_t *bm, const int32_t *woff,
                              int64_t nwords, double *upts, int32_t *uconf, hipStream_t s,
                              int64_t ucap = 0, unsigned *ovf = nullptr);
hipError_t launch_corner_gather_bm(const tms_leaf *lin, int64_t n, int K, const Grid *gt,
                                   const uint64_t *bm, const int32_t *woff, const double *uphi,
                                   double c, tms_leaf *lout, double *cphi, hipStream_t s,
                                   const int64_t *nd = nullptr, int64_t ucap = 0,
                                   unsigned *ovf = nullptr);

// k_extract.hip
// et: device table of edge lattices, one per conformation
// lbm: the leaf-lattice bitmap (zeroed), one bit per surface leaf at its
// level's cube, so that each crossing edge has one owner among the leaves that
// share it; own: [n] edges the leaf owns (bit e for edge e), written by the
// mark and read by the write
hipError_t launch_leaf_mark(const tms_leaf *leaves, int64_t n, const EdgeLat *et,
                            unsigned long long *lbm, hipStream_t s, const int64_t *nd = nullptr);
hipError_t launch_edge_mark(const tms_leaf *leaves, int64_t n, const EdgeLat *et,
                            const uint64_t *lbm, unsigned long long *bm, uint16_t *own,
                            hipStream_t s, const int64_t *nd = nullptr);
hipError_t launch_edge_write(const Grid *gt, const tms_leaf *leaves, const double *cphi, int64_t n,
                             const EdgeLat *et, const uint64_t *bm, const int32_t *woff,
                             const uint16_t *own, tms_vertex *out, hipStream_t s,
                             const int64_t *nd = nullptr, int64_t vcap = 0,
                             unsigned *ovf = nullptr);

}  // namespace tms
