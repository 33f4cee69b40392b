// Host side of the C ABI declared in include/tms.h: argument validation, grid
// set-up, buffer management and the level-by-level orchestration of the
// partition/estimation kernels (Section 2.2 of Liu, Chen & Lu,
// arXiv:1611.03474) on one HIP stream.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tms_internal.h"

using namespace tms;

// ---------------------------------------------------------------------------
// Scratch of tms_eval_phi_noalloc, for callers that cannot allocate: a
// file-scope device array that every GPU the library runs on holds until the
// process ends.  Layout: a u32 guard count (first 256 bytes), the guard list
// (int32 [kNoAllocMaxPoints]), the per-point guard bytes (u8
// [kNoAllocMaxPoints]).  In host code `scratch` names a host-side stand-in,
// not device memory: its device address is taken once per device with
// hipGetSymbolAddress (tms_create) and only that address is used.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNoAllocMaxPoints = (int64_t)1 << 22;
constexpr size_t kNoAllocListOff = 256;
constexpr size_t kNoAllocFlagOff = kNoAllocListOff + sizeof(int32_t) * (size_t)kNoAllocMaxPoints;
constexpr size_t kNoAllocBytes = kNoAllocFlagOff + (size_t)kNoAllocMaxPoints;
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
unsigned char *g_noalloc_addr[kNoAllocDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace tms {

hipError_t DevBuf::ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    release();
    size_t nb = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
        p = nullptr;
        cap = 0;
        (void)hipGetLastError();
        return e;
    }
    cap = nb;
    return hipSuccess;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

hipError_t PinBuf::ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    release();
    const size_t nb = std::max<size_t>(bytes, 65536);
    hipError_t e = hipHostMalloc(&p, nb, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        cap = 0;
        (void)hipGetLastError();
        return e;
    }
    cap = nb;
    return hipSuccess;
}

void PinBuf::release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
}

static hipEvent_t ev_get(tms_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

TimedScope::TimedScope(tms_ctx *c, int s) : ctx(c), slot(s) {
    const bool outer = ctx->tdepth++ == 0;
    if (!ctx->timing || !outer) return;
    e1 = ev_get(ctx);
    if (e1) (void)hipEventRecord(e1, ctx->stream);
}

TimedScope::~TimedScope() {
    --ctx->tdepth;
    if (!ctx->timing || !e1) return;
    hipEvent_t e2 = ev_get(ctx);
    if (!e2) {
        ctx->ev_pool.push_back(e1);
        return;
    }
    (void)hipEventRecord(e2, ctx->stream);
    ctx->ev_pending.push_back({slot, {e1, e2}});
}

// resolve recorded event pairs (waits for them)
void timing_flush(tms_ctx *ctx) {
    for (auto &pe : ctx->ev_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(pe.second.second) == hipSuccess &&
            hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
            ctx->t_ms[pe.first] += ms;
            ctx->t_launch[pe.first] += 1;
        } else {
            (void)hipGetLastError();
        }
        ctx->ev_pool.push_back(pe.second.first);
        ctx->ev_pool.push_back(pe.second.second);
    }
    ctx->ev_pending.clear();
}

}  // namespace tms

void tms_graph_state::release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    exec = nullptr;
    graph = nullptr;
    cap_stream = nullptr;
    cells_id = 0;
    out_leaves = nullptr;
    out_cphi = nullptr;
    out_verts = nullptr;
    tms::DevBuf *b[] = {&q[0], &q[1], &dec, &abuf, &ebuf, &hidx, &flags, &scan_a, &scan_b, &idx,
                        &runs, &chunks, &chunks2, &leaves, &lsort, &cphi, &bmap, &bmcnt, &bmoff, &uniq,
                        &uphi, &uconf, &uguard, &ebmap, &ebcnt, &eboff, &eown, &lbmap, &verts, &etab, &sz, &ctr,
                        &stmp, &seg, &ptab};
    for (auto *x : b) x->release();
}

void tms_cells::release() {
    gtab.release();
    aoff.release();
    ax.release();
    axw.release();
    ay.release();
    az.release();
    aw.release();
    aidx.release();
    ar.release();
    cell_start.release();
    root_start.release();
    root_atoms.release();
    tmp_key.release();
    tmp_cnt.release();
}

namespace {

std::string g_create_err;

int32_t fail(tms_ctx *ctx, int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_err = buf;
    return code;
}

int32_t hip_fail(tms_ctx *ctx, hipError_t e, const char *what) {
    (void)hipGetLastError();
    return fail(ctx, e == hipErrorOutOfMemory ? TMS_E_OOM : TMS_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIPCK(expr)                                               \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr);    \
    } while (0)

void set_msg(char *msg, int64_t len, const std::string &s) {
    if (!msg || len <= 0) return;
    size_t n = std::min<size_t>((size_t)len - 1, s.size());
    memcpy(msg, s.data(), n);
    msg[n] = 0;
}

bool check_params(const tms_params *p, std::string &why, int *Kout) {
    if (!p) { why = "params is NULL"; return false; }
    auto pos = [](double v) { return std::isfinite(v) && v > 0; };
    if (!pos(p->D)) { why = "D must be finite and > 0"; return false; }
    if (!pos(p->c)) { why = "c must be finite and > 0"; return false; }
    if (!pos(p->h0)) { why = "h0 must be finite and > 0"; return false; }
    if (!pos(p->h_min)) { why = "h_min must be finite and > 0"; return false; }
    if (!(std::isfinite(p->pad) && p->pad >= 0)) { why = "pad must be finite and >= 0"; return false; }
    if (!(p->eps_cut > 0 && p->eps_cut < 1)) { why = "eps_cut must be in (0,1)"; return false; }
    if (p->precision != TMS_PREC_FP64 && p->precision != TMS_PREC_FP32_GUARD) {
        why = "precision must be TMS_PREC_FP64 or TMS_PREC_FP32_GUARD";
        return false;
    }
    if (p->mode != TMS_MODE_ADAPTIVE && p->mode != TMS_MODE_UNIFORM) {
        why = "mode must be TMS_MODE_ADAPTIVE or TMS_MODE_UNIFORM";
        return false;
    }
    if (p->degree < 0 || p->degree > 3) { why = "degree must be 1, 2 or 3 (0: 3)"; return false; }
    if (p->child_tensor != TMS_CHILD_PROJECT && p->child_tensor != TMS_CHILD_REEXPAND) {
        why = "child_tensor must be TMS_CHILD_PROJECT or TMS_CHILD_REEXPAND";
        return false;
    }
    int K = 0;
    if (p->mode == TMS_MODE_ADAPTIVE) {
        if (!pos(p->tau)) { why = "tau must be finite and > 0"; return false; }
        double r = p->h0 / p->h_min;
        bool ok = false;
        for (int k = 0; k < TMS_MAX_LEVELS; ++k)
            if (r == std::ldexp(1.0, k)) { K = k; ok = true; }
        if (!ok) { why = "h0 / h_min must be 2^K with 0 <= K < 8"; return false; }
        double beta = 0.5 * p->h0 * std::sqrt(p->D);
        if (gl_half_nodes(beta, p->precision == TMS_PREC_FP32_GUARD) < 0) {
            why = "h0 * sqrt(D) too large for the projection quadrature (need h0 sqrt(D) <= 2.5)";
            return false;
        }
    }
    if (Kout) *Kout = K;
    return true;
}

int64_t next_pow2(int64_t v) {
    int64_t p = 1024;
    while (p < v) p <<= 1;
    return p;
}

// grow a buffer keeping its first `used` bytes
hipError_t grow_keep(DevBuf &b, size_t need, size_t used, hipStream_t s) {
    if (need <= b.cap && b.p) return hipSuccess;
    void *np = nullptr;
    size_t nb = std::max<size_t>(need, b.cap + b.cap / 2);
    hipError_t e = hipMalloc(&np, nb);
    if (e != hipSuccess) return e;
    if (used && b.p) {
        e = hipMemcpyAsync(np, b.p, used, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
    }
    b.release();
    b.p = np;
    b.cap = nb;
    return hipSuccess;
}

// Device-to-host read on the context's stream, synchronous; through the
// context's pinned buffer (a DMA straight into page-locked memory returns
// sooner than one into pageable memory), else directly.
template <typename T>
hipError_t d2h(tms_ctx *ctx, T *dst, const void *src, size_t count) {
    const size_t bytes = sizeof(T) * count;
    if (bytes == 0) return hipSuccess;
    hipStream_t s = ctx->stream;
    if (ctx->pin.ensure(bytes) != hipSuccess) {
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }
    hipError_t e = hipMemcpyAsync(ctx->pin.p, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) memcpy(dst, ctx->pin.p, bytes);
    return e;
}

// Several device-to-host reads with one synchronization: each piece lands
// in the pinned buffer at its own 256-byte-aligned offset.
struct HostRead {
    void *dst;
    const void *src;
    size_t bytes;
};
hipError_t d2h_many(tms_ctx *ctx, const std::vector<HostRead> &rd) {
    size_t total = 0;
    for (const HostRead &r : rd) total += (r.bytes + 255) / 256 * 256;
    if (total == 0) return hipSuccess;
    hipStream_t s = ctx->stream;
    if (ctx->pin.ensure(total) != hipSuccess) {
        for (const HostRead &r : rd) {
            hipError_t e = hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
        }
        return hipStreamSynchronize(s);
    }
    char *base = static_cast<char *>(ctx->pin.p);
    size_t off = 0;
    for (const HostRead &r : rd) {
        if (r.bytes) {
            hipError_t e = hipMemcpyAsync(base + off, r.src, r.bytes, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
        }
        off += (r.bytes + 255) / 256 * 256;
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    off = 0;
    for (const HostRead &r : rd) {
        if (r.bytes) memcpy(r.dst, base + off, r.bytes);
        off += (r.bytes + 255) / 256 * 256;
    }
    return hipSuccess;
}

// scan `n` int32 values of `in` into `out` and return the total on the host
int32_t scan_total(tms_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int64_t *total) {
    HIPCK(ctx->scan_c.ensure(scan_tmp_bytes(n) + 512));
    int32_t *tot = reinterpret_cast<int32_t *>(ctx->counters.as<unsigned long long>() + 100);
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(exclusive_scan(in, out, n, tot, ctx->scan_c.p, ctx->stream));
    }
    int32_t h = 0;
    HIPCK(d2h(ctx, &h, tot, 1));
    *total = h;
    return TMS_OK;
}

// Corner values within this relative distance of c are always recomputed
// with exact exponentials.  An edge root t = (c - phi0)/(phi1 - phi0) from
// FAST values (relative error eps = kFastExpErr) is off by at most
// eps (phi0 + phi1) / |phi1 - phi0|; with every corner of |phi - c| <= b c
// exact, that is at most eps (1 + 1/b) <= 4.4e-6 for b = 0.035.
constexpr double kCornerBand = 0.035;

// Queue slices per level (estimate + bound, at most kMaxSlices); their
// hard-list lengths live in counter slots [kSliceCtr, kSliceCtr + kMaxSlices),
// the guard pass's after.
constexpr int64_t kSliceCtr = 8192;

std::atomic<uint64_t> g_cells_ids{0};

// Largest dense bitmap (bits) used for corner and edge de-duplication, 8 GiB
// (the finest lattice of a box about 1,000 h_min per axis); a pass on a larger
// lattice is refused.
constexpr double kMaxBitmapBits = 68719476736.0;

// phi at m points of `pts` (with the FAST-exponential guard); returns the
// number of points recomputed with exact exponentials.  corners: the points
// are unique leaf corners in bitmap-rank order (the staged corner kernel).
int32_t phi_with_guard(tms_ctx *ctx, const tms_cells *cells, const double *pts,
                       const int32_t *pconf, int64_t m, double *phi, double *grad,
                       int64_t *n_guard, double band_rel, bool corners) {
    const int prec = cells->p.precision;
    const Grid *gt = cells->gtab.as<Grid>();
    *n_guard = 0;
    if (m <= 0) return TMS_OK;
    uint8_t *gbuf = nullptr;
    if (prec == TMS_PREC_FP32_GUARD) {
        HIPCK(ctx->uguard.ensure((size_t)m));
        gbuf = ctx->uguard.as<uint8_t>();
    }
    {
        TimedScope ts_(ctx, TMS_T_PHI);
        if (corners && !grad)
            HIPCK(launch_phi_corners(gt, pconf, prec, pts, m, cells->cell_start.as<int32_t>(),
                                     cells->axw.as<double4>(), band_rel, ctx->corner_groups,
                                     ctx->corner_reach / 16.0, phi, gbuf, ctx->stream));
        else
            HIPCK(launch_phi_points(gt, pconf, prec, pts, m, cells->cell_start.as<int32_t>(),
                                    cells->axw.as<double4>(), band_rel, phi, grad, gbuf,
                                    ctx->stream));
    }
    if (prec == TMS_PREC_FP32_GUARD) {
        HIPCK(ctx->flags.ensure(sizeof(int32_t) * (size_t)m));
        HIPCK(ctx->scan_a.ensure(sizeof(int32_t) * (size_t)m));
        HIPCK(launch_guard_flags_u8(gbuf, m, ctx->flags.as<int32_t>(), ctx->stream));
        int64_t ng = 0;
        int32_t rc = scan_total(ctx, ctx->flags.as<int32_t>(), ctx->scan_a.as<int32_t>(), m, &ng);
        if (rc) return rc;
        if (ng > 0) {
            HIPCK(ctx->idx.ensure(sizeof(int32_t) * (size_t)ng));
            HIPCK(launch_list_emit(ctx->flags.as<int32_t>(), ctx->scan_a.as<int32_t>(), m,
                                   ctx->idx.as<int32_t>(), ctx->stream));
            TimedScope ts_(ctx, TMS_T_GUARD);
            HIPCK(launch_phi_points_subset(gt, pconf, pts, ctx->idx.as<int32_t>(), ng,
                                           cells->cell_start.as<int32_t>(),
                                           cells->axw.as<double4>(), phi, grad, ctx->stream));
        }
        *n_guard = ng;
    }
    return TMS_OK;
}

// unique corners of `leaves`, phi once per corner, masks and classes;
// writes leaves_out (may alias leaves) and cphi [n][8]
int32_t corner_stage(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves, int64_t n,
                     tms_leaf *leaves_out, double *cphi, int64_t *n_corners, int64_t *n_guard) {
    const Grid &g = cells->g;
    const Grid *gt = cells->gtab.as<Grid>();
    hipStream_t s = ctx->stream;
    *n_corners = 0;
    *n_guard = 0;
    ctx->n_corners = 0;
    ctx->corner_cells = cells->id;
    ctx->corner_dense = n <= 0;  // an empty pass has a (trivially) dense corner set
    if (n <= 0) return TMS_OK;
    {
        // dense bitmap over the finest lattice of every conformation (4x4x4
        // point blocks per word, one block of words per conformation) when
        // it fits the budget
        const int64_t nwords = cells->corner_words;
        const double bits = 64.0 * (double)nwords;
        if (bits <= kMaxBitmapBits && nwords < (int64_t)0x7FFFFFFF) {
            HIPCK(ctx->bmap.ensure(sizeof(uint64_t) * (size_t)nwords));
            HIPCK(ctx->bmcnt.ensure(sizeof(int32_t) * (size_t)nwords));
            HIPCK(ctx->bmoff.ensure(sizeof(int32_t) * (size_t)nwords));
            {
                TimedScope ts_(ctx, TMS_T_CORNER);
                HIPCK(launch_fill_u64(ctx->bmap.as<uint64_t>(), 0ull, nwords, s));
                HIPCK(launch_corner_mark(leaves, n, g.K, gt, ctx->bmap.as<unsigned long long>(),
                                         s));
                HIPCK(launch_popc(ctx->bmap.as<uint64_t>(), nwords, ctx->bmcnt.as<int32_t>(), s));
            }
            int64_t nu = 0;
            int32_t rc = scan_total(ctx, ctx->bmcnt.as<int32_t>(), ctx->bmoff.as<int32_t>(), nwords,
                                    &nu);
            if (rc) return rc;
            HIPCK(ctx->uniq.ensure(sizeof(double) * 3 * (size_t)std::max<int64_t>(nu, 1)));
            HIPCK(ctx->uphi.ensure(sizeof(double) * (size_t)std::max<int64_t>(nu, 1)));
            HIPCK(ctx->uconf.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nu, 1)));
            {
                TimedScope ts_(ctx, TMS_T_CORNER);
                HIPCK(launch_corner_enum(gt, cells->nconf, ctx->bmap.as<uint64_t>(),
                                         ctx->bmoff.as<int32_t>(), nwords, ctx->uniq.as<double>(),
                                         ctx->uconf.as<int32_t>(), s));
            }
            rc = phi_with_guard(ctx, cells, ctx->uniq.as<double>(), ctx->uconf.as<int32_t>(), nu,
                                ctx->uphi.as<double>(), nullptr, n_guard, kCornerBand, true);
            if (rc) return rc;
            {
                TimedScope ts_(ctx, TMS_T_CORNER);
                HIPCK(launch_corner_gather_bm(leaves, n, g.K, gt, ctx->bmap.as<uint64_t>(),
                                              ctx->bmoff.as<int32_t>(), ctx->uphi.as<double>(), g.c,
                                              leaves_out, cphi, s));
            }
            *n_corners = nu;
            ctx->n_corners = nu;
            ctx->corner_dense = true;
            return TMS_OK;
        }
    }
    return fail(ctx, TMS_E_INVALID,
                "the finest lattice needs %.4g bits of corner bitmap (limit %.4g): split the "
                "atoms into smaller boxes", 64.0 * (double)cells->corner_words, kMaxBitmapBits);
}

// Chunks of <= 64 consecutive entries of one root over q (or over the
// sorted subset list) for the tiled estimate kernel; uses flags/scan_a/
// scan_b/runs as scratch.
int32_t build_chunks(tms_ctx *ctx, const Grid *gt, int lev, const int4 *q, const int32_t *subset,
                     int64_t n, const int2 **chunks, int64_t *nchunks, int cmax) {
    hipStream_t s = ctx->stream;
    int64_t nruns = 0;
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(launch_run_flags(gt, lev, q, subset, n, ctx->flags.as<int32_t>(), s));
    }
    int32_t rc = scan_total(ctx, ctx->flags.as<int32_t>(), ctx->scan_a.as<int32_t>(), n, &nruns);
    if (rc) return rc;
    HIPCK(ctx->runs.ensure(4 * (size_t)std::max<int64_t>(nruns, 1)));
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(launch_run_starts(ctx->flags.as<int32_t>(), ctx->scan_a.as<int32_t>(), n,
                                ctx->runs.as<int32_t>(), s));
        HIPCK(launch_run_chunk_counts(ctx->runs.as<int32_t>(), nruns, n, ctx->flags.as<int32_t>(),
                                      s, nullptr, nullptr, cmax));
    }
    rc = scan_total(ctx, ctx->flags.as<int32_t>(), ctx->scan_b.as<int32_t>(), nruns, nchunks);
    if (rc) return rc;
    HIPCK(ctx->chunks.ensure(sizeof(int2) * (size_t)std::max<int64_t>(*nchunks, 1)));
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(launch_run_chunk_emit(ctx->runs.as<int32_t>(), nruns, n, ctx->scan_b.as<int32_t>(),
                                    ctx->chunks.as<int2>(), s, nullptr, nullptr, cmax));
    }
    *chunks = ctx->chunks.as<int2>();
    return TMS_OK;
}

// The chunks reordered by root-list length, longest first, for the grouped
// kernel (whose wavefronts take several consecutive chunks); uses flags,
// scan_a, scan_b and scan_c as scratch.
int32_t chunks_by_length(tms_ctx *ctx, const tms_cells *cells, int lev, const int4 *q,
                         const int2 **chunks, int64_t nchunks) {
    if (nchunks <= 0) return TMS_OK;
    hipStream_t s = ctx->stream;
    const size_t m = (size_t)chunks_by_length_scratch(nchunks);
    HIPCK(ctx->chunks2.ensure(sizeof(int2) * (size_t)nchunks));
    HIPCK(ctx->flags.ensure(4 * (size_t)nchunks));
    HIPCK(ctx->scan_a.ensure(4 * m));
    HIPCK(ctx->scan_b.ensure(4 * m));
    HIPCK(ctx->scan_c.ensure(scan_tmp_bytes((int64_t)m) + 512));
    TimedScope ts_(ctx, TMS_T_COMPACT);
    HIPCK(launch_chunks_by_length(cells->gtab.as<Grid>(), lev, q, *chunks, nchunks, nullptr,
                                  cells->root_start.as<int32_t>(), ctx->flags.as<int32_t>(),
                                  ctx->scan_a.as<int32_t>(), ctx->scan_b.as<int32_t>(),
                                  ctx->scan_c.p, ctx->chunks2.as<int2>(), s));
    *chunks = ctx->chunks2.as<int2>();
    return TMS_OK;
}

// A batch's leaves come out level by level with the conformations in order
// inside each level; regroup them conformation by conformation, each keeping
// the order of its own single-conformation pass (level, refinement order).
int32_t regroup_by_conf(tms_ctx *ctx, const tms_cells *cells, int64_t L) {
    hipStream_t s = ctx->stream;
    const int nconf = cells->nconf;
    const int nseg = (cells->g.K + 1) * nconf;
    ctx->leaf_off.assign((size_t)nconf + 1, 0);
    if (L == 0) return TMS_OK;
    HIPCK(ctx->ctab.ensure(sizeof(int64_t) * 2 * (size_t)nseg));
    int64_t *src = ctx->ctab.as<int64_t>(), *dst = src + nseg;
    HIPCK(ctx->lsort.ensure(sizeof(tms_leaf) * (size_t)L));
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(launch_fill_u64(reinterpret_cast<uint64_t *>(src), ~0ull, nseg, s));
        HIPCK(launch_leaf_seg_heads(ctx->leaves.as<tms_leaf>(), L, nconf, src, s));
    }
    std::vector<int64_t> hs((size_t)nseg), hd((size_t)nseg, 0), cnt((size_t)nseg, 0);
    HIPCK(d2h(ctx, hs.data(), src, (size_t)nseg));
    // segments ascend in the source order; a segment ends where the next
    // present one starts
    int64_t prev = -1;
    for (int seg = 0; seg < nseg; ++seg) {
        if (hs[(size_t)seg] < 0) continue;
        if (prev >= 0) cnt[(size_t)prev] = hs[(size_t)seg] - hs[(size_t)prev];
        prev = seg;
    }
    if (prev >= 0) cnt[(size_t)prev] = L - hs[(size_t)prev];
    int64_t pos = 0;
    for (int b = 0; b < nconf; ++b) {
        ctx->leaf_off[(size_t)b] = pos;
        for (int lev = 0; lev <= cells->g.K; ++lev) {
            const size_t seg = (size_t)lev * nconf + b;
            hd[seg] = pos;
            pos += cnt[seg];
        }
    }
    ctx->leaf_off[(size_t)nconf] = pos;
    if (pos != L) return fail(ctx, TMS_E_DEVICE, "leaf regrouping lost leaves");
    HIPCK(hipMemcpyAsync(dst, hd.data(), sizeof(int64_t) * (size_t)nseg, hipMemcpyHostToDevice, s));
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(launch_leaf_seg_move(ctx->leaves.as<tms_leaf>(), L, nconf, src, dst,
                                   ctx->lsort.as<tms_leaf>(), s));
    }
    HIPCK(hipStreamSynchronize(s));  // hd goes out of scope
    std::swap(ctx->leaves, ctx->lsort);
    return TMS_OK;
}

}  // namespace

namespace tms {

// phi of conformation `conf` of `cells` at m device points, the path of
// tms_eval_phi (with the FP32 guard of the cells' precision); the context's
// error is set on failure
int32_t eval_phi_conf(tms_ctx *ctx, const tms_cells *cells, int conf, const double *pts,
                      int64_t m, double *phi) {
    if (conf < 0 || conf >= cells->nconf)
        return fail(ctx, TMS_E_INVALID, "conformation %d out of range", conf);
    HIPCK(hipSetDevice(ctx->device));
    const int32_t *pconf = nullptr;
    DevBuf pc;
    if (cells->nconf > 1 && m > 0) {
        HIPCK(pc.ensure(sizeof(int32_t) * (size_t)m));
        HIPCK(launch_fill_u32(pc.as<uint32_t>(), (uint32_t)conf, m, ctx->stream));
        pconf = pc.as<int32_t>();
    }
    int64_t ng = 0;
    const int32_t rc = phi_with_guard(ctx, cells, pts, pconf, m, phi, nullptr, &ng, 0.0, false);
    if (rc) return rc;
    HIPCK(hipStreamSynchronize(ctx->stream));  // pc is released on return
    return TMS_OK;
}

}  // namespace tms

// ---------------------------------------------------------------------------
// public API
// ---------------------------------------------------------------------------
extern "C" {

int32_t tms_create(tms_ctx **out, int32_t device, void *stream) {
    if (!out) return fail(nullptr, TMS_E_INVALID, "out is NULL");
    *out = nullptr;
    int cnt = 0;
    hipError_t e = hipGetDeviceCount(&cnt);
    if (e != hipSuccess || cnt <= 0) {
        (void)hipGetLastError();
        return fail(nullptr, TMS_E_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= cnt)
        return fail(nullptr, TMS_E_DEVICE, "device %d out of range (%d devices)", device, cnt);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, TMS_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    unsigned char *scr = nullptr;
    if (device < kNoAllocDevices) {
        // the device address of this device's copy of `scratch`, once per device
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_addr[device]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(nullptr, TMS_E_DEVICE, "hipGetSymbolAddress(scratch): %s",
                            hipGetErrorString(e));
            g_noalloc_addr[device] = static_cast<unsigned char *>(p);
        }
        scr = g_noalloc_addr[device];
    }
    tms_ctx *ctx = new tms_ctx();
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->noalloc_scratch = scr;
    e = ctx->counters.ensure(1 << 20);
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, TMS_E_OOM, "counter allocation failed");
    }
    *out = ctx;
    return TMS_OK;
}

int32_t tms_destroy(tms_ctx *ctx) {
    if (!ctx) return TMS_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (tms_cells *c : ctx->cells) {
        c->release();
        delete c;
    }
    tms::DevBuf *bufs[] = {&ctx->leaves, &ctx->corner_phi, &ctx->verts, &ctx->q[0], &ctx->q[1],
                           &ctx->qmeta, &ctx->abuf, &ctx->ebuf, &ctx->dec, &ctx->scan_a,
                           &ctx->scan_b, &ctx->scan_c, &ctx->flags, &ctx->idx, &ctx->uniq,
                           &ctx->uphi, &ctx->uguard,
                           &ctx->ctmp, &ctx->counters, &ctx->hidx, &ctx->chunks,
                           &ctx->chunks2, &ctx->runs};
    for (auto *b : bufs) b->release();
    ctx->graph.release();
    timing_flush(ctx);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
    return TMS_OK;
}

const char *tms_last_error(const tms_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int32_t tms_check_params(const tms_params *p, char *msg, int64_t msg_len) {
    std::string why;
    if (!check_params(p, why, nullptr)) {
        set_msg(msg, msg_len, why);
        return TMS_E_INVALID;
    }
    set_msg(msg, msg_len, "");
    return TMS_OK;
}

int32_t tms_check_atoms_host(const double *xyzr, int64_t n, const tms_params *p, char *msg,
                             int64_t msg_len) {
    std::string why;
    int K = 0;
    if (!check_params(p, why, &K)) {
        set_msg(msg, msg_len, why);
        return TMS_E_INVALID;
    }
    if (n < 0 || (n > 0 && !xyzr)) {
        set_msg(msg, msg_len, "n < 0 or xyzr NULL");
        return TMS_E_INVALID;
    }
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 4; ++a)
            if (!std::isfinite(xyzr[4 * i + a])) {
                set_msg(msg, msg_len, "non-finite atom value");
                return TMS_E_INVALID;
            }
        if (!(xyzr[4 * i + 3] > 0)) {
            set_msg(msg, msg_len, "atom radius must be > 0");
            return TMS_E_INVALID;
        }
        for (int a = 0; a < 3; ++a) {
            double v = xyzr[4 * i + a];
            if (i == 0 || v < mn[a]) mn[a] = v;
            if (i == 0 || v > mx[a]) mx[a] = v;
        }
    }
    const double h0 = p->h0;
    if (p->mode == TMS_MODE_UNIFORM) K = 0;
    for (int a = 0; a < 3; ++a) {
        double o = h0 * std::floor((mn[a] - p->pad) / h0);
        double d = std::ceil((mx[a] + p->pad - o) / h0);
        if (d * std::ldexp(1.0, K) > 65535.0) {
            set_msg(msg, msg_len, "finest lattice exceeds 65535 points per axis");
            return TMS_E_INVALID;
        }
    }
    set_msg(msg, msg_len, "");
    return TMS_OK;
}

}  // extern "C"

namespace {

// Largest batch: the conformation id occupies 11 bits of the edge keys.
constexpr int kMaxConf = 2048;

// Cells of a batch of conformations (one conformation: off = {0, n}).
int32_t build_cells_impl(tms_ctx *ctx, const double *xyzr, const std::vector<int64_t> &off,
                         const tms_params *p, tms_cells **cells_io) {
    if (!cells_io) return fail(ctx, TMS_E_INVALID, "cells is NULL");
    std::string why;
    int K = 0;
    if (!check_params(p, why, &K)) return fail(ctx, TMS_E_INVALID, "%s", why.c_str());
    const int nconf = (int)off.size() - 1;
    if (nconf < 1 || nconf > kMaxConf)
        return fail(ctx, TMS_E_INVALID, "batch of %d conformations (1..%d)", nconf, kMaxConf);
    if (off[0] != 0) return fail(ctx, TMS_E_INVALID, "atom offsets must start at 0");
    for (int b = 0; b < nconf; ++b)
        if (off[b + 1] < off[b]) return fail(ctx, TMS_E_INVALID, "atom offsets must not decrease");
    const int64_t n = off[nconf];
    if (n > 0 && !xyzr) return fail(ctx, TMS_E_INVALID, "xyzr is NULL");
    if (n >= (int64_t)0x7FFFFFFF) return fail(ctx, TMS_E_INVALID, "too many atoms");
    if (p->mode == TMS_MODE_UNIFORM && nconf > 1)
        return fail(ctx, TMS_E_INVALID, "the uniform grid takes one conformation");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    TimedScope ts_build(ctx, TMS_T_BUILD);
    tms_cells *cells = *cells_io;
    if (cells && std::find(ctx->cells.begin(), ctx->cells.end(), cells) == ctx->cells.end())
        return fail(ctx, TMS_E_INVALID, "cells handle does not belong to this context");
    bool fresh = false;
    if (!cells) {
        cells = new tms_cells();
        fresh = true;
    }
    auto bail = [&](int32_t rc) {
        if (fresh) {
            cells->release();
            delete cells;
        }
        return rc;
    };
    cells->p = *p;
    cells->n = n;
    cells->id = ++g_cells_ids;
    cells->nconf = nconf;
    cells->atom_off = off;
    if (p->mode == TMS_MODE_UNIFORM) K = 0;

    // bounding box, radii, finiteness per conformation
    std::vector<double> st(9 * (size_t)nconf, 0.0);
    if (n > 0) {
        hipError_t e = cells->aoff.ensure(sizeof(int64_t) * (size_t)(nconf + 1));
        if (e == hipSuccess)
            e = hipMemcpyAsync(cells->aoff.p, off.data(), sizeof(int64_t) * (size_t)(nconf + 1),
                               hipMemcpyHostToDevice, s);
        int64_t max_atoms = 0;
        for (int b = 0; b < nconf; ++b) max_atoms = std::max(max_atoms, off[b + 1] - off[b]);
        const size_t tmpb = atom_stats_tmp_bytes(nconf, max_atoms);
        if (e == hipSuccess)
            e = ctx->ctmp.ensure(sizeof(double) * 9 * (size_t)nconf + 256 + tmpb);
        if (e == hipSuccess)
            e = launch_atom_stats(xyzr, cells->aoff.as<int64_t>(), nconf, max_atoms,
                                  ctx->ctmp.as<double>(),
                                  ctx->ctmp.as<double>() + 9 * (size_t)nconf + 32, s);
        if (e == hipSuccess) e = d2h(ctx, st.data(), ctx->ctmp.p, 9 * (size_t)nconf);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "atom stats"));
        for (int b = 0; b < nconf; ++b) {
            if (st[9 * b + 8] > 0)
                return bail(fail(ctx, TMS_E_INVALID, "atom array holds NaN or Inf (conformation %d)", b));
            if (off[b + 1] > off[b] && !(st[9 * b + 7] > 0))
                return bail(fail(ctx, TMS_E_INVALID, "atom radius must be > 0 (conformation %d)", b));
        }
    }
    cells->gh.assign((size_t)nconf, Grid{});
    int64_t root_base = 0, cell_base = 0, words = 0;
    cells->rmax = 0.0;
    for (int b = 0; b < nconf; ++b) {
        const bool has = off[b + 1] > off[b];
        const double *sb = st.data() + 9 * b;
        Grid g{};
        g.h0 = p->h0;
        g.hmin = (p->mode == TMS_MODE_UNIFORM) ? p->h0 : p->h_min;
        g.D = p->D;
        g.c = p->c;
        g.tau = p->tau;
        g.K = K;
        g.deg = p->degree > 0 ? p->degree : 3;
        const double rmax = has ? sb[6] : 0.0;
        cells->rmax = std::max(cells->rmax, rmax);
        g.rc2 = rmax * rmax + std::log(1.0 / p->eps_cut) / p->D;
        for (int a = 0; a < 3; ++a) {
            double mn = has ? sb[a] : 0.0, mx = has ? sb[3 + a] : 0.0;
            g.o[a] = p->h0 * std::floor((mn - p->pad) / p->h0);
            double d = std::ceil((mx + p->pad - g.o[a]) / p->h0);
            if (d < 1) d = 1;
            if (d * std::ldexp(1.0, K) > 65535.0)
                return bail(fail(ctx, TMS_E_INVALID, "finest lattice exceeds 65535 points per axis"));
            g.nr[a] = (int32_t)d;
        }
        // atom cells: the smallest edge h0 * 2^m >= R_c / 4, and a stencil
        // of +-span cells (span = ceil(R_c / edge)) around a point's cell;
        // point queries clip each row of the stencil to the R_c sphere
        const double Rc = std::sqrt(g.rc2);
        g.cs = p->h0;
        while (g.cs < 0.25 * Rc) g.cs *= 2.0;
        while (0.5 * g.cs >= 0.25 * Rc) g.cs *= 0.5;
        g.span = (int32_t)std::ceil(Rc / g.cs);
        {
            int ex = 0;
            g.inv_cs = (std::frexp(g.cs, &ex) == 0.5) ? 1.0 / g.cs : 0.0;
            g.inv_h0 = (std::frexp(g.h0, &ex) == 0.5) ? 1.0 / g.h0 : 0.0;
        }
        int64_t nc = 1, nrt = 1;
        for (int a = 0; a < 3; ++a) {
            g.nc[a] = (int32_t)std::max(1.0, std::ceil(g.nr[a] * p->h0 / g.cs));
            nc *= g.nc[a];
            nrt *= g.nr[a];
        }
        g.root_base = root_base;
        g.cell_base = cell_base;
        g.atom_base = off[b];
        // corner bitmap block: 4x4x4 finest-lattice points per word
        int64_t wb = 1;
        for (int a = 0; a < 3; ++a) {
            g.clat.n[a] = ((((int64_t)g.nr[a] << K) + 1) + 3) / 4;
            wb *= g.clat.n[a];
        }
        g.clat.base = words;
        words += wb;
        root_base += nrt;
        cell_base += nc;
        cells->gh[(size_t)b] = g;
    }
    if (cell_base >= (int64_t)0x7FFFFFFF || root_base >= (int64_t)0x7FFFFFFF)
        return bail(fail(ctx, TMS_E_INVALID, "batch grid too large"));
    cells->g = cells->gh[0];
    cells->ncells = cell_base;
    cells->nroots = root_base;
    cells->corner_words = words;
    const int64_t ncells = cell_base;

    auto ck = [&](hipError_t e, const char *what) -> int32_t {
        return e == hipSuccess ? TMS_OK : hip_fail(ctx, e, what);
    };
#define CK(expr)                                        \
    do {                                                \
        int32_t rc_ = ck((expr), #expr);                \
        if (rc_) return bail(rc_);                      \
    } while (0)
    CK(cells->gtab.ensure(sizeof(Grid) * (size_t)nconf));
    CK(hipMemcpyAsync(cells->gtab.p, cells->gh.data(), sizeof(Grid) * (size_t)nconf,
                      hipMemcpyHostToDevice, s));
    const Grid *gt = cells->gtab.as<Grid>();
    const size_t na = (size_t)std::max<int64_t>(n, 1);
    CK(cells->ax.ensure(8 * na));
    CK(cells->ay.ensure(8 * na));
    CK(cells->az.ensure(8 * na));
    CK(cells->aw.ensure(8 * na));
    CK(cells->axw.ensure(32 * na));
    CK(cells->ar.ensure(8 * na));
    CK(cells->aidx.ensure(4 * na));
    CK(cells->tmp_key.ensure(4 * na));
    CK(cells->cell_start.ensure(4 * (size_t)(ncells + 1)));
    CK(cells->tmp_cnt.ensure(4 * (size_t)(ncells + 1)));
    int32_t *cnt = cells->tmp_cnt.as<int32_t>();
    CK(launch_fill_u32(reinterpret_cast<uint32_t *>(cnt), 0u, ncells + 1, s));
    CK(launch_bin_atoms(gt, nconf, xyzr, n, cells->tmp_key.as<int32_t>(), cnt, s));
    {
        int64_t tot = 0;
        int32_t rc = scan_total(ctx, cnt, cells->cell_start.as<int32_t>(), ncells + 1, &tot);
        if (rc) return bail(rc);
    }
    // scatter positions start from the cell offsets
    CK(hipMemcpyAsync(cnt, cells->cell_start.p, 4 * (size_t)ncells, hipMemcpyDeviceToDevice, s));
    CK(launch_scatter_atoms(gt, xyzr, n, cells->tmp_key.as<int32_t>(), cnt, cells->ax.as<double>(),
                            cells->ay.as<double>(), cells->az.as<double>(), cells->aw.as<double>(),
                            cells->ar.as<double>(), cells->aidx.as<int32_t>(), s));
    CK(launch_sort_cells(cells->cell_start.as<int32_t>(), ncells, cells->ax.as<double>(),
                         cells->ay.as<double>(), cells->az.as<double>(), cells->aw.as<double>(),
                         cells->ar.as<double>(), cells->aidx.as<int32_t>(), s));
    CK(launch_pack_atoms(cells->ax.as<double>(), cells->ay.as<double>(), cells->az.as<double>(),
                         cells->aw.as<double>(), n, cells->axw.as<double4>(), s));
    cells->n_root_entries = 0;
    if (p->mode == TMS_MODE_ADAPTIVE) {
        const int64_t nr = cells->nroots;
        CK(cells->root_start.ensure(4 * (size_t)(nr + 1)));
        CK(ctx->flags.ensure(4 * (size_t)(nr + 1)));
        int32_t *rc_cnt = ctx->flags.as<int32_t>();
        CK(launch_fill_u32(reinterpret_cast<uint32_t *>(rc_cnt), 0u, nr + 1, s));
        CK(launch_root_count(gt, nconf, cells->cell_start.as<int32_t>(), cells->axw.as<double4>(),
                             nr, rc_cnt, s));
        int64_t tot = 0;
        int32_t rc = scan_total(ctx, rc_cnt, cells->root_start.as<int32_t>(), nr + 1, &tot);
        if (rc) return bail(rc);
        cells->n_root_entries = tot;
        // a quarter of room to spare: a rebuild from moved atoms (whose
        // lists may grow a little) keeps the buffer, and with it a capture
        if (4 * (size_t)std::max<int64_t>(tot, 1) > cells->root_atoms.cap)
            CK(cells->root_atoms.ensure(5 * (size_t)std::max<int64_t>(tot, 1) + 4096));
        CK(launch_root_fill(gt, nconf, cells->cell_start.as<int32_t>(), cells->axw.as<double4>(),
                            nr, cells->root_start.as<int32_t>(), cells->root_atoms.as<int32_t>(),
                            s));
    }
    CK(hipStreamSynchronize(s));
#undef CK
    if (fresh) ctx->cells.push_back(cells);
    *cells_io = cells;
    return TMS_OK;
}


// whether level lev of the tiled path runs in half-wave chunks
inline bool half_level(const tms_ctx *ctx, int lev) {
    return (ctx->tiled_half == 1 && lev >= 2) || (ctx->tiled_half == 2 && lev == 2);
}

// ---------------------------------------------------------------------------
// Captured pass: the whole partition (roots, every level, guard re-runs,
// compaction, batch regrouping), corner stage and edge extraction recorded
// once into a HIP graph.  Every size the eager pass reads back stays on the
// device; launches are sized by capacities planned from an eager pass of the
// same cells, and the kernels read their actual counts on the device.  A
// count beyond its capacity sets an overflow flag (nothing is written out of
// bounds) and the replay reports TMS_E_CAPACITY.
// ---------------------------------------------------------------------------

// device size slots (int32 unless noted)
constexpr int kSzNq = 0;        // [K + 2] queue entries per level
constexpr int kSzNl = 16;       // [K + 1] leaves per level
constexpr int kSzRuns = 32, kSzChunks = 33, kSzNu = 35, kSzNgp = 36, kSzNv = 37;
constexpr int kSzNg = 40;       // [K + 1] guarded cubes per level
constexpr int kSzSlices = 64;   // [kMaxSlices] entries of each slice
constexpr int kSzGSlices = 64 + (int)kMaxSlices;  // [kMaxSlices] guard-list slices
constexpr int kSz64 = 1024;     // int64 region: [0] leaves, [1] overflow, [8..) offsets
// counter slots (u64)
constexpr int kCtPairs = 0;     // [64 * lev, +64) pair counts of level lev
constexpr int kCtHisto = 1024;  // [8 lev, +5) decision histogram of level lev
constexpr int kCtHard = 2048;   // [2 kMaxSlices lev + k] hard-list lengths (guard after)
constexpr int kCtSurf = 6144;
constexpr int kCtPart = 8192;   // [5 * 1024] reduction partials
constexpr int kCtSlots = kCtPart + 5 * 1024;

void cells_buffers(const tms_cells *c, const void *p[kCellsBufs]) {
    p[0] = c->ax.p;
    p[1] = c->ay.p;
    p[2] = c->az.p;
    p[3] = c->aw.p;
    p[4] = c->cell_start.p;
    p[5] = c->root_start.p;
    p[6] = c->root_atoms.p;
    p[7] = c->gtab.p;
    p[8] = c->axw.p;
}

// Leaf lattices of every conformation (one bit per cube of each level, 4x4x4
// blocks per word) into et[b].leaf; returns the words of their bitmap.
int64_t leaf_lattices(std::vector<EdgeLat> &et, const tms_cells *cells) {
    int64_t words = 0;
    for (size_t b = 0; b < et.size(); ++b) {
        const Grid &gb = cells->gh[b];
        for (int lev = 0; lev < TMS_MAX_LEVELS; ++lev) {
            Lat &l = et[b].leaf[lev];
            if (lev > cells->g.K) {
                l = Lat{{0, 0, 0}, words};
                continue;
            }
            int64_t nw = 1;
            for (int k = 0; k < 3; ++k) {
                l.n[k] = (((int64_t)gb.nr[k] << lev) + 3) / 4;
                nw *= l.n[k];
            }
            l.base = words;
            words += nw;
        }
    }
    return words;
}

// Captured capacity for a count of the eager pass.
int64_t graph_grow(int64_t v, double margin) {
    return (int64_t)std::ceil((double)v * margin) + 4096;
}

// Capacities and private buffers of a capture of `cells`, from the eager
// pass kept in ctx (its counts times `margin`).
int32_t plan_graph(tms_ctx *ctx, const tms_cells *cells, double margin) {
    tms_graph_state &G = ctx->graph;
    const Grid &g = cells->g;
    const tms_stats &st = ctx->last_stats;
    auto grow = [&](int64_t v) { return graph_grow(v, margin); };
    G.nlev = g.K + 1;
    G.nconf = cells->nconf;
    G.qcap[0] = std::max<int64_t>(cells->nroots, 1);
    for (int l = 1; l <= g.K; ++l) G.qcap[l] = grow(st.n_est[l]);
    G.qcap[g.K + 1] = 0;
    G.lcap = grow(st.n_leaves);
    G.ucap = grow(st.n_corners);
    G.vcap = grow(ctx->n_verts);
    int64_t qmax = 1, smax = 1;
    for (int l = 0; l <= g.K; ++l) {
        const int64_t S0 = std::max<int64_t>(4096, ctx->slice_cubes);
        G.nslices[l] = (G.qcap[l] + S0 - 1) / S0;
        if (G.nslices[l] > kMaxSlices) return fail(ctx, TMS_E_INVALID, "capture: level too large for the slice size");
        G.slice[l] = (G.qcap[l] + G.nslices[l] - 1) / G.nslices[l];
        qmax = std::max(qmax, G.qcap[l]);
        smax = std::max(smax, G.slice[l]);
        // one workgroup per chunk for the tiled levels: a slice holds at most
        // as many chunks as cubes, and at most the level's (from the eager
        // pass, which counted them over its own slicing) plus one per cut
        for (int64_t k = 0; k < G.nslices[l]; ++k) {
            int64_t c = G.slice[l];
            const std::vector<int32_t> &bins = ctx->last_chunk_bins[l];
            if (ctx->last_chunks[l] >= 0 && !bins.empty()) {
                // chunks starting in the bins this slice overlaps, one more
                // for a run cut at its start (the replay refines the same
                // queue; the margin covers rebuilt cells)
                const int64_t a = k * G.slice[l], b = (k + 1) * G.slice[l];
                int64_t cnt = 1;
                for (int64_t j = a / kChunkBin; j < (int64_t)bins.size() && j * kChunkBin < b; ++j)
                    cnt += bins[(size_t)j];
                c = std::min(c, grow(cnt));
            } else if (ctx->last_chunks[l] >= 0) {
                c = std::min(c, grow(ctx->last_chunks[l]) + G.nslices[l]);
            }
            G.ccap[l][k] = c;
        }
    }
    // edge lattices, as the eager extraction lays them out
    std::vector<EdgeLat> et((size_t)G.nconf);
    std::vector<int64_t> fw((size_t)G.nconf);
    int64_t ewords = 0;
    double ebits = 0.0;
    for (int b = 0; b < G.nconf; ++b) {
        const Grid &gb = cells->gh[(size_t)b];
        fw[(size_t)b] = ewords;
        for (int lev = 0; lev <= g.K; ++lev)
            for (int a = 0; a < 3; ++a) {
                Lat &l = et[(size_t)b].l[lev][a];
                double bits = 1.0;
                for (int k = 0; k < 3; ++k) {
                    l.n[k] = ((int64_t)gb.nr[k] << lev) + 1;
                    bits *= (double)l.n[k];
                }
                l.base = ewords;
                ewords += (int64_t)((bits + 63.0) / 64.0);
                ebits += bits;
            }
        et[(size_t)b].words = ewords - fw[(size_t)b];
    }
    const int64_t cwords = cells->corner_words;
    G.ewords = ewords;
    G.lwords = leaf_lattices(et, cells);
    if (64.0 * (double)cwords > kMaxBitmapBits || ebits > kMaxBitmapBits ||
        64.0 * (double)G.lwords > kMaxBitmapBits || cwords >= (int64_t)0x7FFFFFFF ||
        ewords >= (int64_t)0x7FFFFFFF)
        return fail(ctx, TMS_E_INVALID, "capture needs the dense corner and edge bitmaps");
    // (+ kLenBuckets: the bucket counts of a chunk reordering round the
    // chunk count up to whole workgroups)
    const int64_t nmax = std::max({qmax, G.ucap, cells->nroots + 1, (int64_t)1}) + kLenBuckets;
    HIPCK(G.q[0].ensure(sizeof(int4) * (size_t)qmax));
    HIPCK(G.q[1].ensure(sizeof(int4) * (size_t)qmax));
    HIPCK(G.dec.ensure((size_t)qmax));
    HIPCK(G.abuf.ensure(sizeof(double) * 64 * (size_t)smax));
    HIPCK(G.ebuf.ensure(sizeof(double) * (size_t)smax));
    HIPCK(G.hidx.ensure(sizeof(int32_t) * (size_t)smax));
    HIPCK(G.flags.ensure(4 * (size_t)nmax));
    HIPCK(G.scan_a.ensure(4 * (size_t)nmax));
    HIPCK(G.scan_b.ensure(4 * (size_t)nmax));
    HIPCK(G.idx.ensure(4 * (size_t)nmax));
    HIPCK(G.runs.ensure(4 * (size_t)smax));
    HIPCK(G.chunks.ensure(sizeof(int2) * (size_t)smax));
    HIPCK(G.chunks2.ensure(sizeof(int2) * (size_t)smax));
    // a result bound to a caller buffer needs no private one
    const bool own_emit = !(G.out_leaves && G.nconf == 1);
    if (own_emit) HIPCK(G.leaves.ensure(sizeof(tms_leaf) * (size_t)G.lcap));
    if (G.nconf > 1 && !G.out_leaves) HIPCK(G.lsort.ensure(sizeof(tms_leaf) * (size_t)G.lcap));
    if (!G.out_cphi) HIPCK(G.cphi.ensure(sizeof(double) * 8 * (size_t)G.lcap));
    HIPCK(G.bmap.ensure(sizeof(uint64_t) * (size_t)cwords));
    HIPCK(G.bmcnt.ensure(4 * (size_t)cwords));
    HIPCK(G.bmoff.ensure(4 * (size_t)cwords));
    HIPCK(G.uniq.ensure(sizeof(double) * 3 * (size_t)G.ucap));
    HIPCK(G.uphi.ensure(sizeof(double) * (size_t)G.ucap));
    HIPCK(G.uconf.ensure(4 * (size_t)G.ucap));
    HIPCK(G.uguard.ensure((size_t)G.ucap));
    HIPCK(G.ebmap.ensure(sizeof(uint64_t) * (size_t)ewords));
    HIPCK(G.ebcnt.ensure(4 * (size_t)ewords));
    HIPCK(G.eown.ensure(sizeof(uint16_t) * (size_t)G.lcap));
    HIPCK(G.lbmap.ensure(sizeof(uint64_t) * (size_t)std::max<int64_t>(G.lwords, 1)));
    HIPCK(G.eboff.ensure(4 * (size_t)ewords));
    if (!G.out_verts) HIPCK(G.verts.ensure(sizeof(tms_vertex) * (size_t)G.vcap));
    HIPCK(G.etab.ensure(sizeof(EdgeLat) * (size_t)G.nconf + sizeof(int64_t) * (size_t)G.nconf));
    HIPCK(G.sz.ensure(sizeof(int32_t) * kSz64 + sizeof(int64_t) * (size_t)(16 + 2 * (G.nconf + 1))));
    HIPCK(G.ctr.ensure(sizeof(unsigned long long) * kCtSlots));
    HIPCK(G.stmp.ensure(scan_tmp_bytes(std::max(nmax, std::max(cwords, ewords))) + 512));
    HIPCK(G.seg.ensure(sizeof(int64_t) * 2 * (size_t)(G.nlev * G.nconf)));
    // projection tables (one buffer, refilled per level; the finest level
    // has the most intervals per atom)
    G.proj_table = false;
    if (ctx->proj_table && cells->n > 0) {
        // without room for the table the captured levels project in place
        const int ns = proj_table_slots(cells, g.K);
        G.proj_table =
            G.ptab.ensure(sizeof(double) * 6 * 3 * (size_t)cells->n * (size_t)ns) == hipSuccess;
    }
    hipStream_t s = ctx->stream;
    HIPCK(hipMemsetAsync(G.q[0].p, 0, G.q[0].cap, s));
    HIPCK(hipMemsetAsync(G.q[1].p, 0, G.q[1].cap, s));
    HIPCK(hipMemcpyAsync(G.etab.p, et.data(), sizeof(EdgeLat) * (size_t)G.nconf,
                         hipMemcpyHostToDevice, s));
    HIPCK(hipMemcpyAsync(G.etab.as<EdgeLat>() + G.nconf, fw.data(), sizeof(int64_t) * (size_t)G.nconf,
                         hipMemcpyHostToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    return TMS_OK;
}

// Enqueue the whole pass on stream s with device-side sizes only.
int32_t record_pass(tms_ctx *ctx, const tms_cells *cells, hipStream_t s) {
    tms_graph_state &G = ctx->graph;
    const Grid &g = cells->g;
    const Grid *gt = cells->gtab.as<Grid>();
    const int prec = cells->p.precision, nconf = cells->nconf, K = g.K;
    int32_t *sz = G.sz.as<int32_t>();
    int32_t *nq = sz + kSzNq, *nl = sz + kSzNl;
    int32_t *nruns = sz + kSzRuns, *nchunks = sz + kSzChunks;
    int32_t *nu = sz + kSzNu, *ngp = sz + kSzNgp, *nv = sz + kSzNv;
    int32_t *ns = sz + kSzSlices;
    // result arrays: the caller's where the capture bound them; the level
    // loop emits a single conformation's leaves in final order, a batch's
    // are regrouped into the final array afterwards
    tms_leaf *emit = (nconf == 1 && G.out_leaves) ? G.out_leaves : G.leaves.as<tms_leaf>();
    double *cphi_out = G.out_cphi ? G.out_cphi : G.cphi.as<double>();
    tms_vertex *vout = G.out_verts ? G.out_verts : G.verts.as<tms_vertex>();
    int64_t *s64 = reinterpret_cast<int64_t *>(sz + kSz64);
    int64_t *Ld = s64;
    unsigned *ovf = reinterpret_cast<unsigned *>(s64 + 1);
    int64_t *leaf_off = s64 + 16, *vert_off = leaf_off + (nconf + 1);
    unsigned long long *ctr = G.ctr.as<unsigned long long>();
    const int32_t *rs = cells->root_start.as<int32_t>(), *ra = cells->root_atoms.as<int32_t>();
    const double *ax = cells->ax.as<double>(), *ay = cells->ay.as<double>(),
                 *az = cells->az.as<double>(), *aw = cells->aw.as<double>();
    int32_t *flags = G.flags.as<int32_t>(), *sa = G.scan_a.as<int32_t>(),
            *sb = G.scan_b.as<int32_t>(), *idx = G.idx.as<int32_t>();
    void *tmp = G.stmp.p;
    uint8_t *dec = G.dec.as<uint8_t>();
    // sizes and counters start at zero (fill kernels: the graph holds no memset nodes)
    HIPCK(launch_fill_u32(reinterpret_cast<uint32_t *>(sz), 0u, (int64_t)(G.sz.cap / 4), s));
    HIPCK(launch_fill_u64(reinterpret_cast<uint64_t *>(ctr), 0ull, kCtSlots, s));
    // Q_0
    const int64_t nr = cells->nroots;
    HIPCK(launch_roots_flags(rs, nr, flags, s));
    HIPCK(exclusive_scan(flags, sa, nr, nq + 0, tmp, s));
    HIPCK(launch_roots_emit(gt, nconf, flags, sa, nr, G.q[0].as<int4>(), s));
    for (int lev = 0; lev <= K; ++lev) {
        const int cur = lev & 1;
        const int4 *q = G.q[cur].as<int4>();
        const int64_t QC = G.qcap[lev], S = G.slice[lev];
        const int nsl = (int)G.nslices[lev];
        const bool tiled = lev >= ctx->tiled_min_level && lev <= 3;
        const bool half = tiled && half_level(ctx, lev);
        const int cmax = half ? 32 : 64;
        ProjTab pt;
        const int lprec = TMS_PREC_FP64;  // as the eager pass: exact estimate and bound
        if (G.proj_table) {
            const int pns = proj_table_slots(cells, lev);
            HIPCK(launch_proj_table(g, gt, nconf, lev, lprec, ax, ay, az, cells->n, pns,
                                    G.ptab.as<double>(), s));
            pt = ProjTab{G.ptab.as<double>(), cells->n, pns};
        }
        HIPCK(launch_slice_counts(nq + lev, S, nsl, ns, s));
        for (int k = 0; k < nsl; ++k) {
            const int64_t off = (int64_t)k * S, cap = std::min(S, QC - off);
            unsigned *hard = reinterpret_cast<unsigned *>(ctr + kCtHard + 2 * kMaxSlices * lev + k);
            const int2 *chunks = nullptr;
            const int32_t *ncount = ns + k;
            if (tiled) {
                HIPCK(launch_run_flags(gt, lev, q + off, nullptr, cap, flags, s, ns + k));
                HIPCK(exclusive_scan(flags, sa, cap, nruns, tmp, s));
                HIPCK(launch_run_starts(flags, sa, cap, G.runs.as<int32_t>(), s));
                HIPCK(launch_run_chunk_counts(G.runs.as<int32_t>(), cap, cap, flags, s, nruns,
                                              ns + k, cmax));
                HIPCK(exclusive_scan(flags, sb, cap, nchunks, tmp, s));
                HIPCK(launch_run_chunk_emit(G.runs.as<int32_t>(), cap, cap, sb, G.chunks.as<int2>(),
                                            s, nruns, ns + k, cmax));
                chunks = G.chunks.as<int2>();
                ncount = nchunks;
                if (lev <= 1 || half) {
                    // grouped kernel: chunks by root-list length
                    HIPCK(launch_chunks_by_length(gt, lev, q + off, chunks, cap, ncount, rs, flags,
                                                  sa, idx, tmp, G.chunks2.as<int2>(), s));
                    chunks = G.chunks2.as<int2>();
                }
            }
            // levels 2-3 in whole-wave chunks: one workgroup per chunk up to
            // the planned capacity (the grouped kernels stride over theirs)
            const bool percap = tiled && !half && lev >= 2;
            HIPCK(launch_estimate_decide(g, gt, lev, lprec, q + off, cap, nullptr, chunks,
                                         percap ? std::min(cap, G.ccap[lev][k]) : cap, rs, ra,
                                         ax, ay, az, aw, dec + off, G.abuf.as<double>(),
                                         G.ebuf.as<double>(), G.hidx.as<int32_t>(), hard,
                                         reinterpret_cast<int64_t *>(ctr + kCtPairs + 64 * lev),
                                         ctx->tile_atoms, s, ncount, pt, nullptr, half,
                                         percap ? ovf : nullptr, nullptr, S));
            HIPCK(launch_bound(g, lev, lprec, cap, dec + off, G.abuf.as<double>(),
                               G.ebuf.as<double>(), G.hidx.as<int32_t>(), hard, s, S));
        }
        HIPCK(launch_level_histo(dec, QC, ctr + kCtHisto + 8 * lev, ctr + kCtPart, s, nq + lev));
        HIPCK(launch_level_counts(dec, QC, flags, idx, s, nq + lev));
        HIPCK(exclusive_scan(flags, sa, QC, nl + lev, tmp, s));
        HIPCK(exclusive_scan(idx, sb, QC, nq + lev + 1, tmp, s));
        HIPCK(launch_level_emit(q, dec, QC, lev, sa, sb, emit, 0,
                                G.q[cur ^ 1].as<int4>(), s, nq + lev, Ld, G.lcap, G.qcap[lev + 1],
                                ovf));
        HIPCK(launch_acc_i64(Ld, nl + lev, s));
        HIPCK(launch_stop_on_overflow(ovf, nq + lev + 1, s));
    }
    // regrouping by conformation (and the per-conformation leaf offsets)
    const int nseg = G.nlev * nconf;
    int64_t *seg_src = G.seg.as<int64_t>(), *seg_dst = seg_src + nseg;
    HIPCK(launch_fill_u64(reinterpret_cast<uint64_t *>(seg_src), ~0ull, nseg, s));
    HIPCK(launch_leaf_seg_heads(emit, G.lcap, nconf, seg_src, s, Ld));
    HIPCK(launch_seg_plan(seg_src, G.nlev, nconf, Ld, G.lcap, seg_dst, leaf_off, s));
    tms_leaf *lv = emit;
    G.leaves_in_lsort = false;
    if (nconf > 1) {
        lv = G.out_leaves ? G.out_leaves : G.lsort.as<tms_leaf>();
        HIPCK(launch_leaf_seg_move(emit, G.lcap, nconf, seg_src, seg_dst, lv, s, Ld));
        G.leaves_in_lsort = true;
    }
    // corners: dense bitmap, phi once per corner (exact recomputation near c
    // and inside the guard band), classes
    const int64_t cw = cells->corner_words;
    HIPCK(launch_fill_u64(G.bmap.as<uint64_t>(), 0ull, cw, s));
    HIPCK(launch_corner_mark(lv, G.lcap, K, gt, G.bmap.as<unsigned long long>(), s, Ld));
    HIPCK(launch_popc(G.bmap.as<uint64_t>(), cw, G.bmcnt.as<int32_t>(), s));
    HIPCK(exclusive_scan(G.bmcnt.as<int32_t>(), G.bmoff.as<int32_t>(), cw, nu, tmp, s));
    HIPCK(launch_corner_enum(gt, nconf, G.bmap.as<uint64_t>(), G.bmoff.as<int32_t>(), cw,
                             G.uniq.as<double>(), G.uconf.as<int32_t>(), s, G.ucap, ovf));
    const bool fast = prec == TMS_PREC_FP32_GUARD;
    HIPCK(launch_phi_corners(gt, G.uconf.as<int32_t>(), prec, G.uniq.as<double>(), G.ucap,
                             cells->cell_start.as<int32_t>(), cells->axw.as<double4>(), kCornerBand,
                             ctx->corner_groups, ctx->corner_reach / 16.0, G.uphi.as<double>(),
                             fast ? G.uguard.as<uint8_t>() : nullptr, s, nu));
    if (fast) {
        HIPCK(launch_guard_flags_u8(G.uguard.as<uint8_t>(), G.ucap, flags, s, nu));
        HIPCK(exclusive_scan(flags, sa, G.ucap, ngp, tmp, s));
        HIPCK(launch_list_emit(flags, sa, G.ucap, idx, s));
        HIPCK(launch_phi_points_subset(gt, G.uconf.as<int32_t>(), G.uniq.as<double>(), idx, G.ucap,
                                       cells->cell_start.as<int32_t>(), cells->axw.as<double4>(),
                                       G.uphi.as<double>(), nullptr, s, ngp));
    }
    HIPCK(launch_corner_gather_bm(lv, G.lcap, K, gt, G.bmap.as<uint64_t>(), G.bmoff.as<int32_t>(),
                                  G.uphi.as<double>(), g.c, lv, cphi_out, s, Ld, G.ucap,
                                  ovf));
    HIPCK(launch_count_surface(lv, G.lcap, ctr + kCtSurf, ctr + kCtPart, s, Ld));
    // edge points: bitmaps in key order, one rank per edge
    const EdgeLat *et = G.etab.as<EdgeLat>();
    const int64_t *fw = reinterpret_cast<const int64_t *>(et + nconf);
    const int64_t ew = G.ewords;
    HIPCK(launch_fill_u64(G.ebmap.as<uint64_t>(), 0ull, ew, s));
    HIPCK(launch_fill_u64(G.lbmap.as<uint64_t>(), 0ull, G.lwords, s));
    HIPCK(launch_leaf_mark(lv, G.lcap, et, G.lbmap.as<unsigned long long>(), s, Ld));
    HIPCK(launch_edge_mark(lv, G.lcap, et, G.lbmap.as<uint64_t>(),
                           G.ebmap.as<unsigned long long>(), G.eown.as<uint16_t>(), s, Ld));
    HIPCK(launch_popc(G.ebmap.as<uint64_t>(), ew, G.ebcnt.as<int32_t>(), s));
    HIPCK(exclusive_scan(G.ebcnt.as<int32_t>(), G.eboff.as<int32_t>(), ew, nv, tmp, s));
    HIPCK(launch_edge_write(gt, lv, cphi_out, G.lcap, et, G.ebmap.as<uint64_t>(),
                            G.eboff.as<int32_t>(), G.eown.as<uint16_t>(),
                            vout, s, Ld, G.vcap, ovf));
    HIPCK(launch_gather_i32(G.eboff.as<int32_t>(), fw, nconf, vert_off, s));
    return TMS_OK;
}

// the checks shared by a capture and its capacity query
int32_t capture_args(tms_ctx *ctx, const tms_cells *cells, double margin) {
    if (!cells || std::find(ctx->cells.begin(), ctx->cells.end(), cells) == ctx->cells.end())
        return fail(ctx, TMS_E_INVALID, "cells handle does not belong to this context");
    if (cells->p.mode != TMS_MODE_ADAPTIVE)
        return fail(ctx, TMS_E_INVALID, "capture takes cells built in adaptive mode");
    if (cells->p.child_tensor != TMS_CHILD_PROJECT)
        return fail(ctx, TMS_E_INVALID, "capture takes cells whose child tensors are projected");
    if (!(margin >= 1.0 && margin <= 64.0))
        return fail(ctx, TMS_E_INVALID, "margin must lie in [1, 64]");
    if (ctx->last_stats_cells != cells->id || ctx->edge_cells != cells->id)
        return fail(ctx, TMS_E_INVALID,
                    "capture is sized from an eager tms_partition_estimate and "
                    "tms_extract_cube_vertices of the same cells; run them first");
    return TMS_OK;
}
}  // namespace

extern "C" {

int32_t tms_build_cells(tms_ctx *ctx, const double *xyzr, int64_t n, const tms_params *p,
                        tms_cells **cells_io) {
    if (!ctx) return TMS_E_INVALID;
    if (n < 0 || (n > 0 && !xyzr)) return fail(ctx, TMS_E_INVALID, "n < 0 or xyzr NULL");
    return build_cells_impl(ctx, xyzr, std::vector<int64_t>{0, n}, p, cells_io);
}

int32_t tms_build_cells_batch(tms_ctx *ctx, const double *xyzr, const int64_t *offsets,
                              int32_t n_conf, const tms_params *p, tms_cells **cells_io) {
    if (!ctx) return TMS_E_INVALID;
    if (!offsets || n_conf < 1 || n_conf > kMaxConf)
        return fail(ctx, TMS_E_INVALID, "offsets NULL or n_conf outside 1..%d", kMaxConf);
    return build_cells_impl(ctx, xyzr, std::vector<int64_t>(offsets, offsets + n_conf + 1), p,
                            cells_io);
}

int32_t tms_cells_info(const tms_cells *cells, double origin[3], int64_t dims[3], int32_t *K,
                       double *rc2, int64_t *n_atoms) {
    if (!cells) return TMS_E_INVALID;
    for (int a = 0; a < 3; ++a) {
        if (origin) origin[a] = cells->g.o[a];
        if (dims) dims[a] = cells->g.nr[a];
    }
    if (K) *K = cells->g.K;
    if (rc2) *rc2 = cells->g.rc2;
    if (n_atoms) *n_atoms = cells->n;
    return TMS_OK;
}

int32_t tms_free_cells(tms_ctx *ctx, tms_cells *cells) {
    if (!ctx || !cells) return TMS_E_INVALID;
    auto it = std::find(ctx->cells.begin(), ctx->cells.end(), cells);
    if (it == ctx->cells.end()) return fail(ctx, TMS_E_INVALID, "unknown cells handle");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    cells->release();
    delete cells;
    ctx->cells.erase(it);
    return TMS_OK;
}

int32_t tms_eval_phi(tms_ctx *ctx, const tms_cells *cells, const double *pts, int64_t m,
                     double *phi, double *grad, int64_t *n_guard) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || m < 0 || (m > 0 && (!pts || !phi)))
        return fail(ctx, TMS_E_INVALID, "invalid arguments to tms_eval_phi");
    if (cells->nconf != 1)
        return fail(ctx, TMS_E_INVALID, "tms_eval_phi takes cells of one conformation");
    HIPCK(hipSetDevice(ctx->device));
    int64_t ng = 0;
    int32_t rc = phi_with_guard(ctx, cells, pts, nullptr, m, phi, grad, &ng, 0.0, false);
    if (rc) return rc;
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (n_guard) *n_guard = ng;
    return TMS_OK;
}

int32_t tms_eval_phi_noalloc(tms_ctx *ctx, const tms_cells *cells, const double *pts, int64_t m,
                             double *phi, double *grad, int64_t *n_guard) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || m < 0 || (m > 0 && (!pts || !phi)))
        return fail(ctx, TMS_E_INVALID, "invalid arguments to tms_eval_phi_noalloc");
    if (cells->nconf != 1)
        return fail(ctx, TMS_E_INVALID, "tms_eval_phi_noalloc takes cells of one conformation");
    if (m > kNoAllocMaxPoints)
        return fail(ctx, TMS_E_INVALID,
                    "tms_eval_phi_noalloc: %lld points exceed its maximum of %lld (use "
                    "tms_eval_phi, or split the points)", (long long)m,
                    (long long)kNoAllocMaxPoints);
    if (!ctx->noalloc_scratch)
        return fail(ctx, TMS_E_DEVICE, "no static scratch on device %d", ctx->device);
    HIPCK(hipSetDevice(ctx->device));
    if (n_guard) *n_guard = 0;
    if (m == 0) return TMS_OK;
    const int prec = cells->p.precision;
    const Grid *gt = cells->gtab.as<Grid>();
    hipStream_t s = ctx->stream;
    unsigned *cnt = reinterpret_cast<unsigned *>(ctx->noalloc_scratch);
    int32_t *list = reinterpret_cast<int32_t *>(ctx->noalloc_scratch + kNoAllocListOff);
    uint8_t *gflag = ctx->noalloc_scratch + kNoAllocFlagOff;
    if (prec != TMS_PREC_FP32_GUARD) {
        HIPCK(launch_phi_points(gt, nullptr, prec, pts, m, cells->cell_start.as<int32_t>(),
                                cells->axw.as<double4>(), 0.0, phi, grad, nullptr, s));
        HIPCK(hipStreamSynchronize(s));
        return TMS_OK;
    }
    // the count is cleared by a fill kernel (the array keeps the last call's
    // contents); every guard byte of [0, m) is written by the phi kernel
    HIPCK(launch_fill_u32(cnt, 0u, 1, s));
    HIPCK(launch_phi_points(gt, nullptr, prec, pts, m, cells->cell_start.as<int32_t>(),
                            cells->axw.as<double4>(), 0.0, phi, grad, gflag, s));
    HIPCK(launch_guard_append(gflag, m, list, cnt, s));
    HIPCK(launch_phi_points_subset(gt, nullptr, pts, list, m, cells->cell_start.as<int32_t>(),
                                   cells->axw.as<double4>(), phi, grad, s,
                                   reinterpret_cast<const int32_t *>(cnt)));
    unsigned ng = 0;
    HIPCK(hipMemcpyAsync(&ng, cnt, sizeof(ng), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (n_guard) *n_guard = (int64_t)ng;
    return TMS_OK;
}

int32_t tms_partition_estimate(tms_ctx *ctx, const tms_cells *cells, tms_leaf *leaves_out,
                               int64_t cap, int64_t *n_leaves, double *corner_phi_out,
                               tms_stats *stats) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || !n_leaves || cap < 0) return fail(ctx, TMS_E_INVALID, "invalid arguments");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const Grid &g = cells->g;  // shared parameters (every conformation has the same)
    const Grid *gt = cells->gtab.as<Grid>();
    const int nconf = cells->nconf;
    const int prec = cells->p.precision;
    tms_stats st;
    memset(&st, 0, sizeof st);
    unsigned long long *ctr = ctx->counters.as<unsigned long long>();
    int64_t L = 0;
    ctx->leaf_off.assign(1, 0);
    bool direct = false;      // leaves written into the caller's buffer
    tms_leaf *lres = nullptr;  // where the classified leaves are
    int64_t chunks_lvl[TMS_MAX_LEVELS];  // whole-wave chunks per level (-1: not chunked so)
    std::fill(chunks_lvl, chunks_lvl + TMS_MAX_LEVELS, (int64_t)-1);

    if (cells->p.mode == TMS_MODE_UNIFORM) {
        L = cells->nroots;
        if (L >= (int64_t)0x7FFFFFFF / 8) return fail(ctx, TMS_E_INVALID, "grid too large");
        HIPCK(ctx->leaves.ensure(sizeof(tms_leaf) * (size_t)L));
        HIPCK(ctx->corner_phi.ensure(sizeof(double) * 8 * (size_t)L));
        HIPCK(launch_uniform_leaves(g, ctx->leaves.as<tms_leaf>(), L, s));
        const int64_t m = (int64_t)(g.nr[0] + 1) * (g.nr[1] + 1) * (g.nr[2] + 1);
        HIPCK(ctx->uniq.ensure(sizeof(double) * 3 * (size_t)m));
        HIPCK(ctx->uphi.ensure(sizeof(double) * (size_t)m));
        HIPCK(launch_uniform_points(g, ctx->uniq.as<double>(), m, s));
        int64_t ng = 0;
        int32_t rc = phi_with_guard(ctx, cells, ctx->uniq.as<double>(), nullptr, m, ctx->uphi.as<double>(),
                                    nullptr, &ng, kCornerBand, false);
        if (rc) return rc;
        HIPCK(launch_uniform_gather(g, ctx->uphi.as<double>(), g.c, ctx->leaves.as<tms_leaf>(), L,
                                    ctx->corner_phi.as<double>(), s));
        st.n_corners = m;
        st.guard_points = ng;
        ctx->leaf_off = {0, L};
        ctx->n_corners = m;
        ctx->corner_cells = cells->id;
        ctx->corner_dense = false;
    } else {
        // Q_0: roots with a non-empty neighbourhood, conformation by
        // conformation, each in raster order
        const int64_t nr = cells->nroots;
        HIPCK(ctx->flags.ensure(4 * (size_t)nr));
        HIPCK(ctx->scan_a.ensure(4 * (size_t)nr));
        {
            TimedScope ts_(ctx, TMS_T_COMPACT);
            HIPCK(launch_roots_flags(cells->root_start.as<int32_t>(), nr, ctx->flags.as<int32_t>(), s));
        }
        int64_t nq = 0;
        int32_t rc = scan_total(ctx, ctx->flags.as<int32_t>(), ctx->scan_a.as<int32_t>(), nr, &nq);
        if (rc) return rc;
        int cur = 0;
        HIPCK(ctx->q[0].ensure(sizeof(int4) * (size_t)std::max<int64_t>(nq, 1)));
        {
            TimedScope ts_(ctx, TMS_T_COMPACT);
            HIPCK(launch_roots_emit(gt, nconf, ctx->flags.as<int32_t>(), ctx->scan_a.as<int32_t>(),
                                    nr, ctx->q[0].as<int4>(), s));
        }
        // re-expanded child tensors (eq. childtensor): every level below K
        // keeps its entries' tensors for its children, which take them from
        // there instead of projecting the atoms
        const bool reex = cells->p.child_tensor == TMS_CHILD_REEXPAND;
        int64_t nq_prev = 0;  // the previous level's entries (its saved tensors' stride)
        for (int lev = 0; lev <= g.K && nq > 0; ++lev) {
            if (nq >= (int64_t)0x7FFFFFFF) return fail(ctx, TMS_E_INVALID, "queue too large");
            st.n_est[lev] = nq;
            const bool reex_lev = reex && lev >= 1;
            double *allA = nullptr;
            if (reex && lev < g.K) {
                if (ctx->asave[lev & 1].ensure(sizeof(double) * 64 * (size_t)nq) != hipSuccess)
                    return fail(ctx, TMS_E_OOM, "re-expansion needs %.3g GB for the tensors of level %d",
                                64.0 * 8.0 * (double)nq * 1e-9, lev);
                allA = ctx->asave[lev & 1].as<double>();
            }
            // the tensors of the cubes that need the bound are staged in
            // slices of at most slice_cubes queue entries
            // (equal slices: ceil(nq / slice_cubes) of them)
            const int64_t S0 = std::max<int64_t>(1, ctx->slice_cubes);
            const int64_t nslices = (nq + S0 - 1) / S0;
            const int64_t S = (nq + nslices - 1) / nslices;
            const int64_t cap = std::min(nq, S);
            if (nslices > kMaxSlices) return fail(ctx, TMS_E_INVALID, "queue too large for the slice size");
            HIPCK(ctx->abuf.ensure(sizeof(double) * 64 * (size_t)cap));
            HIPCK(ctx->ebuf.ensure(sizeof(double) * (size_t)cap));
            HIPCK(ctx->hidx.ensure(sizeof(int32_t) * (size_t)cap));
            HIPCK(ctx->dec.ensure((size_t)nq));
            HIPCK(ctx->flags.ensure(4 * (size_t)nq));
            HIPCK(ctx->scan_a.ensure(4 * (size_t)nq));
            HIPCK(ctx->scan_b.ensure(4 * (size_t)nq));
            HIPCK(ctx->idx.ensure(4 * (size_t)nq));
            HIPCK(hipMemsetAsync(ctr, 0, 96 * sizeof(unsigned long long), s));
            HIPCK(hipMemsetAsync(ctr + kSliceCtr, 0, 2 * kMaxSlices * sizeof(unsigned long long), s));
            const int4 *q = ctx->q[cur].as<int4>();
            // deep levels: chunks of <= 64 consecutive cubes of one root
            const bool tiled = !reex_lev && lev >= ctx->tiled_min_level && lev <= 3;
            const bool half = tiled && half_level(ctx, lev);
            int64_t level_chunks = 0;
            ProjTab pt;
            // The estimate and the bound run with exact exponentials in both
            // precision modes: with the table the exponentials are shared by
            // every cube that reads an entry (no FP32 gain), and a bound
            // decision taken on a tensor with single-precision exponentials
            // could only be guarded by a perturbation estimate of the nested
            // SVD, not a certified one (near clustered singular values its
            // factors move arbitrarily), so classification would not be
            // guaranteed to equal the double-precision one.
            const int lprec = TMS_PREC_FP64;
            const int pns = proj_table_slots(cells, lev);
            // a table that does not fit in device memory leaves the level to
            // in-place projections
            if (!reex_lev && ctx->proj_table &&
                ctx->ptab.ensure(sizeof(double) * 6 * 3 * (size_t)cells->n * (size_t)pns) ==
                    hipSuccess) {
                const int ns = pns;
                const int64_t na = cells->n;
                {
                    TimedScope ts_(ctx, TMS_T_TABLE);
                    HIPCK(launch_proj_table(g, gt, nconf, lev, lprec, cells->ax.as<double>(),
                                            cells->ay.as<double>(), cells->az.as<double>(), na, ns,
                                            ctx->ptab.as<double>(), s));
                }
                pt = ProjTab{ctx->ptab.as<double>(), na, ns};
            }
            const int64_t nbins = (nq + kChunkBin - 1) / kChunkBin;
            if (tiled && !half) {
                HIPCK(ctx->chist.ensure(sizeof(int32_t) * (size_t)nbins));
                HIPCK(launch_fill_u32(ctx->chist.as<uint32_t>(), 0u, nbins, s));
            }
            for (int64_t k = 0; k < nslices; ++k) {
                const int64_t off = k * S, ns = std::min(S, nq - off);
                unsigned *hard = reinterpret_cast<unsigned *>(ctr + kSliceCtr + k);
                const int2 *chunks = nullptr;
                int64_t nchunks = 0;
                if (tiled) {
                    rc = build_chunks(ctx, gt, lev, q + off, nullptr, ns, &chunks, &nchunks,
                                      half ? 32 : 64);
                    if (rc) return rc;
                    level_chunks += nchunks;
                    if (!half) {  // where the chunks start (sizes a captured pass's launches)
                        TimedScope ts_(ctx, TMS_T_COMPACT);
                        HIPCK(launch_chunk_bins(chunks, nchunks, off, ns,
                                                ctx->chist.as<int32_t>(), s));
                    }
                    if (lev <= 1 || half) {
                        rc = chunks_by_length(ctx, cells, lev, q + off, &chunks, nchunks);
                        if (rc) return rc;
                    }
                }
                unsigned *tick = nullptr;
                if (tiled && ctx->tiled_dyn) {
                    HIPCK(ctx->tick.ensure(8 * sizeof(unsigned)));
                    tick = ctx->tick.as<unsigned>();
                    HIPCK(launch_fill_u32(ctx->tick.as<uint32_t>(), 0u, 8, s));
                }
                if (reex_lev) {  // Step 1 by re-expansion, and the easy decisions
                    TimedScope ts_(ctx, TMS_T_ESTIMATE);
                    HIPCK(launch_reexpand(g, lev, q + off, ns, off,
                                          ctx->asave[(lev - 1) & 1].as<double>(), nq_prev,
                                          ctx->qpar.as<int32_t>(), ctx->dec.as<uint8_t>() + off,
                                          ctx->abuf.as<double>(), ctx->ebuf.as<double>(),
                                          ctx->hidx.as<int32_t>(), hard,
                                          allA ? allA + 2 * off : nullptr, s, cap, nq));
                } else {  // Step 1 (tensor) and the decisions that need no bound
                    TimedScope ts_(ctx, !tiled ? TMS_T_ESTIMATE
                                               : (lev <= 1 ? TMS_T_GROUPED : TMS_T_TILED));
                    HIPCK(launch_estimate_decide(
                        g, gt, lev, lprec, q + off, ns, nullptr, chunks, nchunks,
                        cells->root_start.as<int32_t>(), cells->root_atoms.as<int32_t>(),
                        cells->ax.as<double>(), cells->ay.as<double>(), cells->az.as<double>(),
                        cells->aw.as<double>(), ctx->dec.as<uint8_t>() + off,
                        ctx->abuf.as<double>(), ctx->ebuf.as<double>(), ctx->hidx.as<int32_t>(),
                        hard, reinterpret_cast<int64_t *>(ctr + 0), ctx->tile_atoms, s, nullptr,
                        pt, half ? nullptr : tick, half, nullptr,
                        allA ? allA + 2 * off : nullptr, cap, nq));
                }
                {  // Step 2: nested-SVD bound on the cubes that need it
                    TimedScope ts_(ctx, TMS_T_DECIDE);
                    HIPCK(launch_bound(g, lev, lprec, ns, ctx->dec.as<uint8_t>() + off,
                                       ctx->abuf.as<double>(), ctx->ebuf.as<double>(),
                                       ctx->hidx.as<int32_t>(), hard, s, cap));
                }
            }
            chunks_lvl[lev] = tiled && !half ? level_chunks : -1;
            ctx->last_chunk_bins[lev].clear();
            if (tiled && !half) ctx->last_chunk_bins[lev].resize((size_t)nbins);
            int32_t *lcnt = ctx->flags.as<int32_t>(), *ccnt = ctx->idx.as<int32_t>();
            {
                TimedScope ts_(ctx, TMS_T_COMPACT);
                HIPCK(launch_level_histo(ctx->dec.as<uint8_t>(), nq, ctr + 72, ctr + 256, s));
                HIPCK(launch_level_counts(ctx->dec.as<uint8_t>(), nq, lcnt, ccnt, s));
            }
            // both scans' totals, the counters and the chunk bins in one read
            int32_t *tots = reinterpret_cast<int32_t *>(ctr + 104);
            HIPCK(ctx->scan_c.ensure(scan_tmp_bytes(nq) + 512));
            {
                TimedScope ts_(ctx, TMS_T_COMPACT);
                HIPCK(exclusive_scan(lcnt, ctx->scan_a.as<int32_t>(), nq, tots, ctx->scan_c.p, s));
                HIPCK(exclusive_scan(ccnt, ctx->scan_b.as<int32_t>(), nq, tots + 1, ctx->scan_c.p,
                                     s));
            }
            int32_t htot[2] = {0, 0};
            unsigned long long h[80];
            std::vector<unsigned long long> hs(2 * (size_t)kMaxSlices);
            std::vector<int32_t> &bins = ctx->last_chunk_bins[lev];
            HIPCK(d2h_many(ctx, {{htot, tots, sizeof htot},
                                 {h, ctr, sizeof h},
                                 {hs.data(), ctr + kSliceCtr, sizeof(unsigned long long) * hs.size()},
                                 {bins.data(), ctx->chist.p, sizeof(int32_t) * bins.size()}}));
            const int64_t nl = htot[0], nc = htot[1];
            for (int k = 0; k < 64; ++k) st.n_pairs_lvl[lev] += (int64_t)h[k];
            st.n_pairs += st.n_pairs_lvl[lev];
            for (unsigned long long v : hs) st.n_bound += (int64_t)(v & 0xFFFFFFFFull);
            st.n_disc[lev] = (int64_t)h[72 + DEC_DISCARD];
            st.n_refine[lev] = (int64_t)h[72 + DEC_REFINE];
            st.n_conv[lev] = (int64_t)h[72 + DEC_CONV];
            st.n_hmin[lev] = (int64_t)h[72 + DEC_HMIN];
            if (8 * st.n_refine[lev] >= (int64_t)0x7FFFFFFF ||
                st.n_conv[lev] + st.n_hmin[lev] >= (int64_t)0x7FFFFFFF)
                return fail(ctx, TMS_E_INVALID, "level %d too large (32-bit offsets)", lev);
            HIPCK(grow_keep(ctx->leaves, sizeof(tms_leaf) * (size_t)(L + nl), sizeof(tms_leaf) * (size_t)L, s));
            HIPCK(ctx->q[cur ^ 1].ensure(sizeof(int4) * (size_t)std::max<int64_t>(nc, 1)));
            if (reex) HIPCK(ctx->qpar.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nc / 8, 1)));
            {
                TimedScope ts_(ctx, TMS_T_COMPACT);
                HIPCK(launch_level_emit(q, ctx->dec.as<uint8_t>(), nq, lev, ctx->scan_a.as<int32_t>(),
                                        ctx->scan_b.as<int32_t>(), ctx->leaves.as<tms_leaf>(), L,
                                        ctx->q[cur ^ 1].as<int4>(), s, nullptr, nullptr, 0, 0,
                                        nullptr, reex ? ctx->qpar.as<int32_t>() : nullptr));
            }
            L += nl;
            nq_prev = nq;
            nq = nc;
            cur ^= 1;
        }
        HIPCK(ctx->leaves.ensure(sizeof(tms_leaf) * (size_t)std::max<int64_t>(L, 1)));
        HIPCK(ctx->corner_phi.ensure(sizeof(double) * 8 * (size_t)std::max<int64_t>(L, 1)));
        if (nconf > 1) {
            rc = regroup_by_conf(ctx, cells, L);
            if (rc) return rc;
        } else {
            ctx->leaf_off = {0, L};
        }
        // a caller's buffer that holds the result receives the classified
        // leaves (and corner values) directly; ctx then keeps no copy
        direct = leaves_out && cap >= L;
        lres = direct ? leaves_out : ctx->leaves.as<tms_leaf>();
        double *cres = direct && corner_phi_out ? corner_phi_out : ctx->corner_phi.as<double>();
        int64_t nu = 0, ng = 0;
        rc = corner_stage(ctx, cells, ctx->leaves.as<tms_leaf>(), L, lres, cres, &nu, &ng);
        if (rc) return rc;
        st.n_corners = nu;
        st.guard_points = ng;
    }
    if (!direct) lres = ctx->leaves.as<tms_leaf>();
    HIPCK(hipMemsetAsync(ctr + 80, 0, 8, s));
    {
        TimedScope ts_(ctx, TMS_T_COMPACT);
        HIPCK(launch_count_surface(lres, L, ctr + 80, ctr + 256, s));
    }
    unsigned long long ns = 0;
    HIPCK(d2h(ctx, &ns, ctr + 80, 1));
    st.n_leaves = L;
    st.n_surface = (int64_t)ns;
    ctx->n_leaves = L;
    ctx->last_stats = st;
    ctx->last_stats_cells = cells->id;
    for (int l = 0; l < TMS_MAX_LEVELS; ++l) ctx->last_chunks[l] = chunks_lvl[l];
    if (stats) *stats = st;
    *n_leaves = L;
    ctx->leaves_kept = !direct;
    ctx->cphi_kept = !(direct && corner_phi_out);
    if (!leaves_out) return TMS_OK;
    if (cap < L) return fail(ctx, TMS_E_CAPACITY, "leaf capacity %lld < %lld", (long long)cap, (long long)L);
    if (L > 0 && !direct) {
        HIPCK(hipMemcpyAsync(leaves_out, ctx->leaves.p, sizeof(tms_leaf) * (size_t)L,
                             hipMemcpyDeviceToDevice, s));
        if (corner_phi_out)
            HIPCK(hipMemcpyAsync(corner_phi_out, ctx->corner_phi.p, sizeof(double) * 8 * (size_t)L,
                                 hipMemcpyDeviceToDevice, s));
    }
    HIPCK(hipStreamSynchronize(s));
    return TMS_OK;
}

int32_t tms_get_leaves(tms_ctx *ctx, tms_leaf *leaves, double *corner_phi, int64_t cap,
                       int64_t *n_leaves) {
    if (!ctx) return TMS_E_INVALID;
    if (!n_leaves) return fail(ctx, TMS_E_INVALID, "n_leaves is NULL");
    *n_leaves = ctx->n_leaves;
    if (!leaves) return TMS_OK;
    if (!ctx->leaves_kept || (corner_phi && !ctx->cphi_kept))
        return fail(ctx, TMS_E_INVALID,
                    "the last pass wrote its leaves into the caller's buffers and kept no copy");
    if (cap < ctx->n_leaves) return fail(ctx, TMS_E_CAPACITY, "leaf capacity too small");
    HIPCK(hipSetDevice(ctx->device));
    const int64_t L = ctx->n_leaves;
    if (L > 0) {
        HIPCK(hipMemcpyAsync(leaves, ctx->leaves.p, sizeof(tms_leaf) * (size_t)L,
                             hipMemcpyDeviceToDevice, ctx->stream));
        if (corner_phi)
            HIPCK(hipMemcpyAsync(corner_phi, ctx->corner_phi.p, sizeof(double) * 8 * (size_t)L,
                                 hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    return TMS_OK;
}

int32_t tms_extract_cube_vertices(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves,
                                  int64_t n, const double *corner_phi, tms_vertex *out, int64_t cap,
                                  int64_t *n_out) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || !n_out || n < 0 || cap < 0 || (n > 0 && !leaves))
        return fail(ctx, TMS_E_INVALID, "invalid arguments to tms_extract_cube_vertices");
    if (n >= (int64_t)0x7FFFFFFF) return fail(ctx, TMS_E_INVALID, "too many leaves");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const Grid &g = cells->g;
    const tms_leaf *lv = leaves;
    const double *cphi = corner_phi;
    if (n > 0 && !cphi) {
        // evaluate the corners of the given leaves (classes recomputed too)
        HIPCK(ctx->ctmp.ensure((sizeof(tms_leaf) + 8 * sizeof(double)) * (size_t)n + 256));
        tms_leaf *lt = ctx->ctmp.as<tms_leaf>();
        double *ct = reinterpret_cast<double *>(
            (reinterpret_cast<uintptr_t>(lt + n) + 255) & ~(uintptr_t)255);
        int64_t nu = 0, ng = 0;
        int32_t rc = corner_stage(ctx, cells, leaves, n, lt, ct, &nu, &ng);
        if (rc) return rc;
        lv = lt;
        cphi = ct;
    }
    int64_t nv = 0;
    bool vdirect = false;  // vertices written into the caller's buffer
    // edge lattices of every conformation, one block of words each
    // (conformation-major, then level, then axis: the edge-key order)
    const int nconf = cells->nconf;
    std::vector<EdgeLat> etab((size_t)nconf);
    std::vector<int64_t> first_word((size_t)nconf);
    double ebits = 0.0;
    int64_t words = 0;
    for (int b = 0; b < nconf; ++b) {
        const Grid &gb = cells->gh[(size_t)b];
        EdgeLat &el = etab[(size_t)b];
        first_word[(size_t)b] = words;
        for (int lev = 0; lev <= g.K; ++lev)
            for (int a = 0; a < 3; ++a) {
                Lat &l = el.l[lev][a];
                double bits = 1.0;
                for (int k = 0; k < 3; ++k) {
                    l.n[k] = ((int64_t)gb.nr[k] << lev) + 1;
                    bits *= (double)l.n[k];
                }
                l.base = words;
                words += (int64_t)((bits + 63.0) / 64.0);
                ebits += bits;
            }
        el.words = words - first_word[(size_t)b];
    }
    const int64_t lwords = leaf_lattices(etab, cells);
    ctx->n_verts = 0;
    ctx->edge_cells = cells->id;
    ctx->edge_dense = n == 0;
    ctx->vert_off.assign((size_t)nconf + 1, 0);
    if (n > 0 && ebits <= kMaxBitmapBits && 64.0 * (double)lwords <= kMaxBitmapBits &&
        words < (int64_t)0x7FFFFFFF) {
        // edge bitmaps in buffers of their own: the corner bitmap stays
        // valid for the adjoint
        const int64_t nwords = words;
        HIPCK(ctx->etab.ensure(sizeof(EdgeLat) * (size_t)nconf + sizeof(int64_t) * (size_t)(2 * nconf)));
        EdgeLat *et = ctx->etab.as<EdgeLat>();
        int64_t *fw = reinterpret_cast<int64_t *>(et + nconf), *vo = fw + nconf;
        HIPCK(hipMemcpyAsync(et, etab.data(), sizeof(EdgeLat) * (size_t)nconf,
                             hipMemcpyHostToDevice, s));
        HIPCK(hipMemcpyAsync(fw, first_word.data(), sizeof(int64_t) * (size_t)nconf,
                             hipMemcpyHostToDevice, s));
        HIPCK(ctx->ebmap.ensure(sizeof(uint64_t) * (size_t)nwords));
        HIPCK(ctx->ebcnt.ensure(sizeof(int32_t) * (size_t)nwords));
        HIPCK(ctx->eown.ensure(sizeof(uint16_t) * (size_t)n));
        HIPCK(ctx->lbmap.ensure(sizeof(uint64_t) * (size_t)std::max<int64_t>(lwords, 1)));
        HIPCK(ctx->eboff.ensure(sizeof(int32_t) * (size_t)nwords));
        {
            TimedScope ts_(ctx, TMS_T_EXTRACT);
            HIPCK(launch_fill_u64(ctx->ebmap.as<uint64_t>(), 0ull, nwords, s));
            HIPCK(launch_fill_u64(ctx->lbmap.as<uint64_t>(), 0ull, lwords, s));
            HIPCK(launch_leaf_mark(lv, n, et, ctx->lbmap.as<unsigned long long>(), s));
            HIPCK(launch_edge_mark(lv, n, et, ctx->lbmap.as<uint64_t>(),
                                   ctx->ebmap.as<unsigned long long>(), ctx->eown.as<uint16_t>(),
                                   s));
            HIPCK(launch_popc(ctx->ebmap.as<uint64_t>(), nwords, ctx->ebcnt.as<int32_t>(), s));
        }
        int32_t rc = scan_total(ctx, ctx->ebcnt.as<int32_t>(), ctx->eboff.as<int32_t>(), nwords, &nv);
        if (rc) return rc;
        // a caller's buffer that holds the result receives the vertices
        // directly; ctx then keeps no copy
        vdirect = out && cap >= nv;
        if (!vdirect) HIPCK(ctx->verts.ensure(sizeof(tms_vertex) * (size_t)std::max<int64_t>(nv, 1)));
        {
            TimedScope ts_(ctx, TMS_T_EXTRACT);
            HIPCK(launch_edge_write(cells->gtab.as<Grid>(), lv, cphi, n, et,
                                    ctx->ebmap.as<uint64_t>(), ctx->eboff.as<int32_t>(),
                                    ctx->eown.as<uint16_t>(),
                                    vdirect ? out : ctx->verts.as<tms_vertex>(), s));
        }
        // first vertex of every conformation: the rank of its first word
        HIPCK(launch_gather_i32(ctx->eboff.as<int32_t>(), fw, nconf, vo, s));
        HIPCK(d2h(ctx, ctx->vert_off.data(), vo, (size_t)nconf));
        ctx->vert_off[(size_t)nconf] = nv;
        ctx->edge_dense = true;
        ctx->edge_lat = etab[0];
    } else if (n > 0) {
        return fail(ctx, TMS_E_INVALID,
                    "the edge lattices need %.4g bits of bitmap (limit %.4g): split the atoms "
                    "into smaller boxes", std::max(ebits, 64.0 * (double)lwords), kMaxBitmapBits);
    }
    ctx->n_verts = nv;
    ctx->verts_kept = !vdirect;
    *n_out = nv;
    if (!out) {
        HIPCK(hipStreamSynchronize(s));
        return TMS_OK;
    }
    if (cap < nv) {
        HIPCK(hipStreamSynchronize(s));
        return fail(ctx, TMS_E_CAPACITY, "vertex capacity %lld < %lld", (long long)cap, (long long)nv);
    }
    if (nv > 0 && !vdirect)
        HIPCK(hipMemcpyAsync(out, ctx->verts.p, sizeof(tms_vertex) * (size_t)nv,
                             hipMemcpyDeviceToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    return TMS_OK;
}

int32_t tms_stage2_points(tms_ctx *ctx, const tms_cells *cells, const tms_leaf *leaves, int64_t n,
                          const double *corner_phi, tms_s2point *out, int64_t cap,
                          int64_t *n_out, int64_t *n_degenerate) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || n < 0 || !n_out || (n > 0 && (!leaves || !corner_phi)) || cap < 0)
        return fail(ctx, TMS_E_INVALID, "invalid arguments to tms_stage2_points");
    HIPCK(hipSetDevice(ctx->device));
    *n_out = 0;
    if (n_degenerate) *n_degenerate = 0;
    if (n == 0) return TMS_OK;
    hipStream_t s = ctx->stream;
    const Grid *gt = cells->gtab.as<Grid>();
    // leaves in chunks whose record counts (<= 12 per leaf) fit int32 offsets
    constexpr int64_t kChunk = (int64_t)1 << 27;
    HIPCK(ctx->flags.ensure(sizeof(int32_t) * (size_t)n));
    HIPCK(ctx->scan_a.ensure(sizeof(int32_t) * (size_t)n));
    unsigned long long *ndeg = ctx->counters.as<unsigned long long>() + 112;
    HIPCK(launch_fill_u64(reinterpret_cast<uint64_t *>(ndeg), 0ull, 1, s));
    std::vector<int64_t> base;
    int64_t total = 0;
    for (int64_t q0 = 0; q0 < n; q0 += kChunk) {
        const int64_t nq = std::min(kChunk, n - q0);
        {
            TimedScope ts_(ctx, TMS_T_STAGE2);
            HIPCK(launch_s2_count(gt, leaves + q0, corner_phi + 8 * q0, nq,
                                  ctx->flags.as<int32_t>() + q0, ndeg, s));
        }
        int64_t t = 0;
        int32_t rc = scan_total(ctx, ctx->flags.as<int32_t>() + q0, ctx->scan_a.as<int32_t>() + q0,
                                nq, &t);
        if (rc) return rc;
        base.push_back(total);
        total += t;
    }
    unsigned long long nd = 0;
    HIPCK(d2h(ctx, &nd, ndeg, 1));
    *n_out = total;
    if (n_degenerate) *n_degenerate = (int64_t)nd;
    if (!out) return TMS_OK;
    if (cap < total)
        return fail(ctx, TMS_E_CAPACITY, "stage-two output needs %lld records, capacity %lld",
                    (long long)total, (long long)cap);
    // leaf indices in the records count from the start of the whole list
    for (size_t k = 0; k * kChunk < (size_t)n; ++k) {
        const int64_t q0 = (int64_t)k * kChunk, nq = std::min(kChunk, n - q0);
        TimedScope ts_(ctx, TMS_T_STAGE2);
        HIPCK(launch_s2_emit(gt, leaves + q0, corner_phi + 8 * q0, nq,
                             ctx->scan_a.as<int32_t>() + q0, out + base[k], q0, s));
    }
    HIPCK(hipStreamSynchronize(s));
    return TMS_OK;
}

int32_t tms_get_vertices(tms_ctx *ctx, tms_vertex *out, int64_t cap, int64_t *n_out) {
    if (!ctx) return TMS_E_INVALID;
    if (!n_out) return fail(ctx, TMS_E_INVALID, "n_out is NULL");
    *n_out = ctx->n_verts;
    if (!out) return TMS_OK;
    if (!ctx->verts_kept)
        return fail(ctx, TMS_E_INVALID,
                    "the last extraction wrote its vertices into the caller's buffer and kept no copy");
    if (cap < ctx->n_verts) return fail(ctx, TMS_E_CAPACITY, "vertex capacity too small");
    HIPCK(hipSetDevice(ctx->device));
    if (ctx->n_verts > 0)
        HIPCK(hipMemcpyAsync(out, ctx->verts.p, sizeof(tms_vertex) * (size_t)ctx->n_verts,
                             hipMemcpyDeviceToDevice, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return TMS_OK;
}

int32_t tms_get_corners(tms_ctx *ctx, double *xyz, double *phi, int64_t cap, int64_t *n_out) {
    if (!ctx) return TMS_E_INVALID;
    if (!n_out) return fail(ctx, TMS_E_INVALID, "n_out is NULL");
    const int64_t m = ctx->n_corners;
    *n_out = m;
    if (!xyz && !phi) return TMS_OK;
    if (cap < m) return fail(ctx, TMS_E_CAPACITY, "corner capacity %lld < %lld", (long long)cap, (long long)m);
    HIPCK(hipSetDevice(ctx->device));
    if (m > 0) {
        if (xyz)
            HIPCK(hipMemcpyAsync(xyz, ctx->uniq.p, sizeof(double) * 3 * (size_t)m,
                                 hipMemcpyDeviceToDevice, ctx->stream));
        if (phi)
            HIPCK(hipMemcpyAsync(phi, ctx->uphi.p, sizeof(double) * (size_t)m,
                                 hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    return TMS_OK;
}

int32_t tms_backward(tms_ctx *ctx, const tms_cells *cells, const double *dphi, int64_t m,
                     const double *dt, int64_t nv, double *dxyzr) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || std::find(ctx->cells.begin(), ctx->cells.end(), cells) == ctx->cells.end())
        return fail(ctx, TMS_E_INVALID, "cells handle does not belong to this context");
    if (cells->n > 0 && !dxyzr) return fail(ctx, TMS_E_INVALID, "dxyzr is NULL");
    if (cells->nconf != 1)
        return fail(ctx, TMS_E_INVALID, "tms_backward takes cells of one conformation");
    if (ctx->corner_cells != cells->id || !ctx->corner_dense)
        return fail(ctx, TMS_E_INVALID,
                    "no kept corners of an adaptive pass on these cells (run "
                    "tms_partition_estimate on them first; the uniform grid has no adjoint)");
    if (dphi && m != ctx->n_corners)
        return fail(ctx, TMS_E_INVALID, "dphi holds %lld values, %lld corners are kept",
                    (long long)m, (long long)ctx->n_corners);
    if (dt) {
        if (ctx->edge_cells != cells->id || !ctx->edge_dense)
            return fail(ctx, TMS_E_INVALID,
                        "no kept edge points of these cells (run tms_extract_cube_vertices on the "
                        "kept leaves first)");
        if (nv != ctx->n_verts)
            return fail(ctx, TMS_E_INVALID, "dt holds %lld values, %lld edge points are kept",
                        (long long)nv, (long long)ctx->n_verts);
    }
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const Grid &g = cells->g;
    const int64_t M = ctx->n_corners;
    if (M == 0) {  // no corners: every derivative is zero
        if (cells->n > 0)
            HIPCK(launch_fill_u64(reinterpret_cast<uint64_t *>(dxyzr), 0ull, 4 * cells->n, s));
        HIPCK(hipStreamSynchronize(s));
        return TMS_OK;
    }
    HIPCK(ctx->wbar.ensure(sizeof(double) * (size_t)M));
    unsigned *bad = reinterpret_cast<unsigned *>(ctx->counters.as<unsigned long long>() + 96);
    HIPCK(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    {
        TimedScope ts_(ctx, TMS_T_BACKWARD);
        HIPCK(launch_adjoint_fold(g, g.clat, ctx->bmap.as<uint64_t>(),
                                  ctx->bmoff.as<int32_t>(), ctx->uniq.as<double>(),
                                  ctx->uphi.as<double>(), M, dphi, ctx->edge_lat,
                                  ctx->ebmap.as<uint64_t>(), ctx->eboff.as<int32_t>(), dt,
                                  ctx->wbar.as<double>(), bad, s));
        HIPCK(launch_adjoint_atoms(g, cells->p.precision, g.clat, ctx->bmap.as<uint64_t>(),
                                   ctx->bmoff.as<int32_t>(), ctx->uniq.as<double>(),
                                   ctx->wbar.as<double>(), cells->n, cells->ax.as<double>(),
                                   cells->ay.as<double>(), cells->az.as<double>(),
                                   cells->aw.as<double>(), cells->ar.as<double>(),
                                   cells->aidx.as<int32_t>(), dxyzr, s));
    }
    unsigned hb = 0;
    HIPCK(d2h(ctx, &hb, bad, 1));
    if (hb) return fail(ctx, TMS_E_INVALID, "kept edge points do not end on kept corners");
    return TMS_OK;
}

int32_t tms_batch_counts(tms_ctx *ctx, const tms_cells *cells, int64_t *leaf_offsets,
                         int64_t *vertex_offsets) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || std::find(ctx->cells.begin(), ctx->cells.end(), cells) == ctx->cells.end())
        return fail(ctx, TMS_E_INVALID, "cells handle does not belong to this context");
    const size_t nb = (size_t)cells->nconf + 1;
    if (leaf_offsets) {
        if (ctx->corner_cells != cells->id || ctx->leaf_off.size() != nb)
            return fail(ctx, TMS_E_INVALID, "no kept pass of these cells");
        std::copy(ctx->leaf_off.begin(), ctx->leaf_off.end(), leaf_offsets);
    }
    if (vertex_offsets) {
        if (ctx->edge_cells != cells->id || ctx->vert_off.size() != nb)
            return fail(ctx, TMS_E_INVALID, "no kept per-conformation vertex offsets of these cells");
        std::copy(ctx->vert_off.begin(), ctx->vert_off.end(), vertex_offsets);
    }
    return TMS_OK;
}

int32_t tms_graph_capacity(tms_ctx *ctx, const tms_cells *cells, double margin, int64_t *leaf_cap,
                           int64_t *vert_cap) {
    if (!ctx) return TMS_E_INVALID;
    if (int32_t rc = capture_args(ctx, cells, margin)) return rc;
    if (leaf_cap) *leaf_cap = graph_grow(ctx->last_stats.n_leaves, margin);
    if (vert_cap) *vert_cap = graph_grow(ctx->n_verts, margin);
    return TMS_OK;
}

int32_t tms_graph_capture(tms_ctx *ctx, const tms_cells *cells, double margin) {
    return tms_graph_capture_into(ctx, cells, margin, nullptr, nullptr, 0, nullptr, 0);
}

int32_t tms_graph_capture_into(tms_ctx *ctx, const tms_cells *cells, double margin,
                               tms_leaf *leaves, double *corner_phi, int64_t leaf_cap,
                               tms_vertex *verts, int64_t vert_cap) {
    if (!ctx) return TMS_E_INVALID;
    if (int32_t rc = capture_args(ctx, cells, margin)) return rc;
    const int64_t lneed = graph_grow(ctx->last_stats.n_leaves, margin);
    const int64_t vneed = graph_grow(ctx->n_verts, margin);
    if ((leaves || corner_phi) && leaf_cap < lneed)
        return fail(ctx, TMS_E_CAPACITY, "bound leaf buffers hold %lld entries, the capture needs %lld",
                    (long long)leaf_cap, (long long)lneed);
    if (verts && vert_cap < vneed)
        return fail(ctx, TMS_E_CAPACITY, "bound vertex buffer holds %lld entries, the capture needs %lld",
                    (long long)vert_cap, (long long)vneed);
    HIPCK(hipSetDevice(ctx->device));
    tms_graph_state &G = ctx->graph;
    G.release();
    G.out_leaves = leaves;
    G.out_cphi = corner_phi;
    G.out_verts = verts;
    // the captured pass has private copies of the eager partition's
    // workspace; give that back first (the next eager pass grows it again)
    for (tms::DevBuf *b : {&ctx->q[0], &ctx->q[1], &ctx->abuf, &ctx->ebuf, &ctx->hidx, &ctx->dec,
                           &ctx->ptab, &ctx->chunks, &ctx->chunks2, &ctx->runs})
        b->release();
    int32_t rc = plan_graph(ctx, cells, margin);
    if (rc) {
        G.release();
        return rc;
    }
    HIPCK(hipStreamCreateWithFlags(&G.cap_stream, hipStreamNonBlocking));
    const bool timing = ctx->timing;
    ctx->timing = false;
    hipError_t e = hipStreamBeginCapture(G.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        ctx->timing = timing;
        G.release();
        return hip_fail(ctx, e, "hipStreamBeginCapture");
    }
    rc = record_pass(ctx, cells, G.cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(G.cap_stream, &graph);
    ctx->timing = timing;
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        G.release();
        return rc ? rc : hip_fail(ctx, e, "hipStreamEndCapture");
    }
    G.graph = graph;
    e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        G.release();
        return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    G.cells_id = cells->id;
    G.gh = cells->gh;
    G.n_atoms = cells->n;
    G.atom_off = cells->atom_off;
    cells_buffers(cells, G.cells_buf);
    return TMS_OK;
}

int32_t tms_graph_launch(tms_ctx *ctx, const tms_cells *cells, tms_leaf *leaves,
                         double *corner_phi, int64_t leaf_cap, int64_t *n_leaves,
                         tms_vertex *verts, int64_t vert_cap, int64_t *n_verts,
                         int64_t *leaf_offsets, int64_t *vertex_offsets, tms_stats *stats) {
    if (!ctx) return TMS_E_INVALID;
    tms_graph_state &G = ctx->graph;
    if (!G.exec) return fail(ctx, TMS_E_INVALID, "no captured pass (tms_graph_capture)");
    if (!cells || std::find(ctx->cells.begin(), ctx->cells.end(), cells) == ctx->cells.end())
        return fail(ctx, TMS_E_INVALID, "cells handle does not belong to this context");
    if (cells->id != G.cells_id) {
        // a rebuild keeps the graph valid when geometry, atom counts and
        // buffers are unchanged (the captured launches and the projection
        // table's rows are sized by the atom count)
        const void *p[kCellsBufs];
        cells_buffers(cells, p);
        bool same = cells->gh.size() == G.gh.size() &&
                    memcmp(cells->gh.data(), G.gh.data(), sizeof(Grid) * G.gh.size()) == 0 &&
                    cells->n == G.n_atoms && cells->atom_off == G.atom_off;
        for (int k = 0; k < kCellsBufs && same; ++k) same = p[k] == G.cells_buf[k];
        if (!same)
            return fail(ctx, TMS_E_INVALID,
                        "cells changed geometry, atom count or buffers since the capture; "
                        "capture again");
    }
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    HIPCK(hipGraphLaunch(G.exec, s));
    const int nconf = G.nconf, K = G.nlev - 1;
    std::vector<int32_t> hs(kSz64);
    std::vector<int64_t> h64((size_t)(16 + 2 * (nconf + 1)));
    std::vector<unsigned long long> hc(kCtSurf + 1);
    HIPCK(hipMemcpyAsync(hs.data(), G.sz.p, sizeof(int32_t) * kSz64, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(h64.data(), G.sz.as<int32_t>() + kSz64, sizeof(int64_t) * h64.size(),
                         hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(hc.data(), G.ctr.p, sizeof(unsigned long long) * hc.size(),
                         hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    const int64_t L = h64[0];
    const int64_t nv = hs[kSzNv];
    if (n_leaves) *n_leaves = L;
    if (n_verts) *n_verts = nv;
    if ((h64[1] & 0xFFFFFFFFll) != 0)
        return fail(ctx, TMS_E_CAPACITY,
                    "a count exceeded the captured capacity; capture again with a larger margin");
    tms_stats st;
    memset(&st, 0, sizeof st);
    for (int l = 0; l <= K; ++l) {
        st.n_est[l] = hs[kSzNq + l];
        const unsigned long long *h = hc.data() + kCtHisto + 8 * l;
        st.n_disc[l] = (int64_t)h[DEC_DISCARD];
        st.n_refine[l] = (int64_t)h[DEC_REFINE];
        st.n_conv[l] = (int64_t)h[DEC_CONV];
        st.n_hmin[l] = (int64_t)h[DEC_HMIN];
        for (int k = 0; k < 64; ++k) st.n_pairs_lvl[l] += (int64_t)hc[kCtPairs + 64 * l + k];
        st.n_pairs += st.n_pairs_lvl[l];
        for (int k = 0; k < 2 * kMaxSlices; ++k)
            st.n_bound += (int64_t)(hc[kCtHard + 2 * kMaxSlices * l + k] & 0xFFFFFFFFull);
        st.guard_cubes += hs[kSzNg + l];
    }
    st.n_leaves = L;
    st.n_surface = (int64_t)hc[kCtSurf];
    st.n_corners = hs[kSzNu];
    st.guard_points = cells->p.precision == TMS_PREC_FP32_GUARD ? hs[kSzNgp] : 0;
    if (stats) *stats = st;
    if (leaf_offsets) std::copy(h64.begin() + 16, h64.begin() + 16 + nconf + 1, leaf_offsets);
    if (vertex_offsets) {
        std::copy(h64.begin() + 16 + nconf + 1, h64.begin() + 16 + 2 * nconf + 1, vertex_offsets);
        vertex_offsets[nconf] = nv;
    }
    if ((leaves && leaf_cap < L) || (verts && vert_cap < nv))
        return fail(ctx, TMS_E_CAPACITY, "output capacity too small (%lld leaves, %lld vertices)",
                    (long long)L, (long long)nv);
    // results already in a requested buffer (bound at capture) are not copied
    const tms_leaf *lsrc = G.out_leaves       ? G.out_leaves
                           : G.leaves_in_lsort ? G.lsort.as<tms_leaf>()
                                               : G.leaves.as<tms_leaf>();
    const double *csrc = G.out_cphi ? G.out_cphi : G.cphi.as<double>();
    const tms_vertex *vsrc = G.out_verts ? G.out_verts : G.verts.as<tms_vertex>();
    if (leaves && leaves != lsrc && L > 0)
        HIPCK(hipMemcpyAsync(leaves, lsrc, sizeof(tms_leaf) * (size_t)L, hipMemcpyDeviceToDevice, s));
    if (corner_phi && corner_phi != csrc && L > 0)
        HIPCK(hipMemcpyAsync(corner_phi, csrc, sizeof(double) * 8 * (size_t)L,
                             hipMemcpyDeviceToDevice, s));
    if (verts && verts != vsrc && nv > 0)
        HIPCK(hipMemcpyAsync(verts, vsrc, sizeof(tms_vertex) * (size_t)nv,
                             hipMemcpyDeviceToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    return TMS_OK;
}

int32_t tms_set_tuning(tms_ctx *ctx, const tms_tuning *t) {
    if (!ctx) return TMS_E_INVALID;
    if (!t) return fail(ctx, TMS_E_INVALID, "tuning is NULL");
    if (t->slice_cubes < 4096) return fail(ctx, TMS_E_INVALID, "slice_cubes < 4096");
    if (t->tiled_min_level < 0 || t->tiled_min_level > 4)
        return fail(ctx, TMS_E_INVALID, "tiled_min_level outside 0..4");
    if (t->tile_atoms != 8 && t->tile_atoms != 16 && t->tile_atoms != 32)
        return fail(ctx, TMS_E_INVALID, "tile_atoms must be 8, 16 or 32");
    if (t->proj_table != 0 && t->proj_table != 1)
        return fail(ctx, TMS_E_INVALID, "proj_table must be 0 or 1");
    if (t->tiled_persistent != 0 && t->tiled_persistent != 1)
        return fail(ctx, TMS_E_INVALID, "tiled_persistent must be 0 or 1");
    if (t->tiled_half < 0 || t->tiled_half > 2)
        return fail(ctx, TMS_E_INVALID, "tiled_half must be 0, 1 or 2");
    if (t->corner_groups < 0 || t->corner_groups > 8)
        return fail(ctx, TMS_E_INVALID, "corner_groups outside 0..8");
    if (t->corner_reach < 1 || t->corner_reach > 64)
        return fail(ctx, TMS_E_INVALID, "corner_reach outside 1..64");
    ctx->slice_cubes = t->slice_cubes;
    ctx->tiled_min_level = t->tiled_min_level;
    ctx->tile_atoms = t->tile_atoms;
    ctx->proj_table = t->proj_table;
    ctx->tiled_dyn = t->tiled_persistent != 0;
    ctx->tiled_half = t->tiled_half;
    ctx->corner_groups = t->corner_groups;
    ctx->corner_reach = t->corner_reach;
    return TMS_OK;
}

int32_t tms_get_tuning(tms_ctx *ctx, tms_tuning *t) {
    if (!ctx || !t) return TMS_E_INVALID;
    t->slice_cubes = ctx->slice_cubes;
    t->tiled_min_level = ctx->tiled_min_level;
    t->tile_atoms = ctx->tile_atoms;
    t->proj_table = ctx->proj_table;
    t->tiled_persistent = ctx->tiled_dyn ? 1 : 0;
    t->tiled_half = ctx->tiled_half;
    t->corner_groups = ctx->corner_groups;
    t->corner_reach = ctx->corner_reach;
    t->reserved = 0;
    return TMS_OK;
}

int32_t tms_autotune(tms_ctx *ctx, const tms_cells *cells, tms_tuning *best, double *best_ms,
                     int32_t *n_tried) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells) return fail(ctx, TMS_E_INVALID, "cells is NULL");
    tms_tuning cur{};
    tms_get_tuning(ctx, &cur);
    int64_t ref_leaves = -1, ref_est = -1;
    int tried = 0;
    // one timed count-only pass under tuning t
    auto run = [&](const tms_tuning &t, double *ms) -> int32_t {
        int32_t rc = tms_set_tuning(ctx, &t);
        if (rc) return rc;
        tms_stats st;
        int64_t nl = 0;
        const auto t0 = std::chrono::steady_clock::now();
        rc = tms_partition_estimate(ctx, cells, nullptr, 0, &nl, nullptr, &st);
        const auto t1 = std::chrono::steady_clock::now();
        if (rc) return rc;
        ++tried;
        int64_t est = 0;
        for (int l = 0; l < TMS_MAX_LEVELS; ++l) est += st.n_est[l];
        if (ref_leaves < 0) {
            ref_leaves = nl;
            ref_est = est;
        } else if (nl != ref_leaves || est != ref_est) {
            return fail(ctx, TMS_E_DEVICE, "tuning changed the result (%lld vs %lld leaves)",
                        (long long)nl, (long long)ref_leaves);
        }
        *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        return TMS_OK;
    };
    double ms = 0.0, bms = 0.0;
    int32_t rc = run(cur, &ms);  // warm-up (buffers grow to size)
    if (rc) return rc;
    rc = run(cur, &bms);
    if (rc) return rc;
    tms_tuning b = cur;
    auto consider = [&](tms_tuning t) -> int32_t {
        int32_t r = run(t, &ms);
        if (r) return r;
        if (ms < bms) {
            bms = ms;
            b = t;
        }
        return TMS_OK;
    };
    for (int ch : {8, 16, 32}) {
        if (ch == b.tile_atoms) continue;
        tms_tuning t = b;
        t.tile_atoms = ch;
        if ((rc = consider(t))) return rc;
    }
    {
        tms_tuning t = b;
        t.proj_table = 1 - b.proj_table;
        if ((rc = consider(t))) return rc;
    }
    {
        tms_tuning t = b;
        t.tiled_persistent = 1 - b.tiled_persistent;
        if ((rc = consider(t))) return rc;
    }
    const tms_tuning bh = b;
    for (int h : {0, 1, 2}) {
        if (h == bh.tiled_half) continue;
        tms_tuning t = bh;
        t.tiled_half = h;
        if ((rc = consider(t))) return rc;
    }
    const tms_tuning bch = b;
    for (int lv : {0, 1, 2, 3}) {
        if (lv == bch.tiled_min_level) continue;
        tms_tuning t = bch;
        t.tiled_min_level = lv;
        if ((rc = consider(t))) return rc;
    }
    const tms_tuning blv = b;
    for (int64_t sc : {(int64_t)1 << 23, (int64_t)1 << 24, (int64_t)1 << 25, (int64_t)1 << 26,
                       (int64_t)1 << 27}) {
        if (sc == blv.slice_cubes) continue;
        tms_tuning t = blv;
        t.slice_cubes = sc;
        if ((rc = consider(t))) return rc;
    }
    tms_set_tuning(ctx, &b);
    if (best) *best = b;
    if (best_ms) *best_ms = bms;
    if (n_tried) *n_tried = tried;
    return TMS_OK;
}

int32_t tms_set_timing(tms_ctx *ctx, int32_t enable) {
    if (!ctx) return TMS_E_INVALID;
    timing_flush(ctx);
    ctx->timing = enable != 0;
    return TMS_OK;
}

int32_t tms_get_timing(tms_ctx *ctx, tms_timing *out, int32_t reset) {
    if (!ctx || !out) return TMS_E_INVALID;
    timing_flush(ctx);
    for (int i = 0; i < TMS_T_SLOTS; ++i) {
        out->ms[i] = ctx->t_ms[i];
        out->launches[i] = ctx->t_launch[i];
        if (reset) {
            ctx->t_ms[i] = 0;
            ctx->t_launch[i] = 0;
        }
    }
    return TMS_OK;
}

int32_t tms_debug_tensor(tms_ctx *ctx, const tms_cells *cells, const int32_t *cubes, int64_t n,
                         int32_t precision, double *A, double *S) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || n < 0 || (n > 0 && (!cubes || !A)) ||
        (precision != TMS_PREC_FP64 && precision != TMS_PREC_FP32_GUARD))
        return fail(ctx, TMS_E_INVALID, "invalid arguments to tms_debug_tensor");
    if (cells->p.mode != TMS_MODE_ADAPTIVE)
        return fail(ctx, TMS_E_INVALID, "tensors need cells built in adaptive mode");
    if (n == 0) return TMS_OK;
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const Grid &g = cells->g;
    std::vector<int32_t> hc(4 * (size_t)n);
    HIPCK(d2h(ctx, hc.data(), cubes, 4 * (size_t)n));
    std::vector<int4> hq((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int lev = hc[4 * i];
        if (lev < 0 || lev > g.K) return fail(ctx, TMS_E_INVALID, "cube level out of range");
        for (int a = 0; a < 3; ++a) {
            int v = hc[4 * i + 1 + a];
            if (v < 0 || v >= (g.nr[a] << lev)) return fail(ctx, TMS_E_INVALID, "cube index out of range");
        }
        hq[(size_t)i] = make_int4(hc[4 * i + 1], hc[4 * i + 2], hc[4 * i + 3], 0);
    }
    HIPCK(ctx->q[0].ensure(sizeof(int4) * (size_t)n));
    HIPCK(ctx->ebuf.ensure(sizeof(double) * (size_t)n));
    HIPCK(ctx->idx.ensure(sizeof(int32_t) * (size_t)n));
    HIPCK(hipMemcpyAsync(ctx->q[0].p, hq.data(), sizeof(int4) * (size_t)n, hipMemcpyHostToDevice, s));
    for (int lev = 0; lev <= g.K; ++lev) {
        std::vector<int32_t> sub;
        for (int64_t i = 0; i < n; ++i)
            if (hc[4 * i] == lev) sub.push_back((int32_t)i);
        if (sub.empty()) continue;
        HIPCK(hipMemcpyAsync(ctx->idx.p, sub.data(), sizeof(int32_t) * sub.size(),
                             hipMemcpyHostToDevice, s));
        HIPCK(launch_estimate(g, cells->gtab.as<Grid>(), lev, precision, ctx->q[0].as<int4>(),
                              (int64_t)sub.size(),
                              ctx->idx.as<int32_t>(), cells->root_start.as<int32_t>(),
                              cells->root_atoms.as<int32_t>(), cells->ax.as<double>(),
                              cells->ay.as<double>(), cells->az.as<double>(), cells->aw.as<double>(),
                              A, ctx->ebuf.as<double>(), nullptr, s));
        HIPCK(hipStreamSynchronize(s));
    }
    if (S) HIPCK(hipMemcpyAsync(S, ctx->ebuf.p, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    return TMS_OK;
}

int32_t tms_debug_phi_pairs(tms_ctx *ctx, const tms_cells *cells, const double *pts, int64_t m,
                            int64_t *pairs) {
    if (!ctx) return TMS_E_INVALID;
    if (!cells || m < 0 || !pairs || (m > 0 && !pts))
        return fail(ctx, TMS_E_INVALID, "invalid arguments to tms_debug_phi_pairs");
    if (cells->nconf != 1)
        return fail(ctx, TMS_E_INVALID, "tms_debug_phi_pairs takes cells of one conformation");
    HIPCK(hipSetDevice(ctx->device));
    unsigned long long *ctr = ctx->counters.as<unsigned long long>() + 113;
    HIPCK(launch_fill_u64(reinterpret_cast<uint64_t *>(ctr), 0ull, 1, ctx->stream));
    HIPCK(launch_phi_pairs(cells->gtab.as<Grid>(), pts, m, cells->cell_start.as<int32_t>(),
                           cells->axw.as<double4>(), ctr, ctx->stream));
    unsigned long long h = 0;
    HIPCK(d2h(ctx, &h, ctr, 1));
    *pairs = (int64_t)h;
    return TMS_OK;
}

int32_t tms_debug_fast_exp(tms_ctx *ctx, const double *x, int64_t n, double *y) {
    if (!ctx) return TMS_E_INVALID;
    if (n < 0 || (n > 0 && (!x || !y))) return fail(ctx, TMS_E_INVALID, "invalid arguments");
    HIPCK(hipSetDevice(ctx->device));
    HIPCK(launch_fast_exp_debug(x, n, y, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return TMS_OK;
}

int32_t tms_debug_bound(tms_ctx *ctx, const double *A, const double *band, int64_t n,
                        double *out) {
    if (!ctx) return TMS_E_INVALID;
    if (n < 0 || (n > 0 && (!A || !out))) return fail(ctx, TMS_E_INVALID, "invalid arguments");
    HIPCK(hipSetDevice(ctx->device));
    HIPCK(launch_bound_debug(A, band, n, out, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return TMS_OK;
}

}  // extern "C"
