// Adaptive partition and estimation kernels (Section 2.2, Steps 1-3) for
// gfx950.
//
//   roots      Q_0: root cubes with a non-empty neighbourhood, raster order
//   estimate   per cube: A = sum_i w_i a~x (x) a~y (x) a~z over the atoms within
//              R_c of the cube (eqs. polynew, tensor1, tensor2); its epilogue
//              takes the decisions that need no bound (Step 3's stopping
//              rule 2E <= tau for children; sampled values of P on both sides
//              of c) and appends the other cubes to a dense "hard" list
//   bound      per hard cube: Step 2's test L <= c <= U with the nested-SVD
//              bound, then leaf / divide
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

// queue entry (ix, iy, iz, conformation) of every root with atoms nearby;
// roots of the batch in conformation order, each in raster order (x fastest)
__global__ void k_roots_emit(const Grid *__restrict__ gt, int nconf, const int32_t *__restrict__ f,
                             const int32_t *__restrict__ off, int64_t nroots,
                             int4 *__restrict__ q) {
    int64_t r = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (r >= nroots || !f[r]) return;
    const int b = conf_of_root(gt, nconf, r);
    const Grid &g = gt[b];
    const int64_t rl = r - g.root_base;
    int rx = (int)(rl % g.nr[0]), ry = (int)((rl / g.nr[0]) % g.nr[1]),
        rz = (int)(rl / ((int64_t)g.nr[0] * g.nr[1]));
    q[off[r]] = make_int4(rx, ry, rz, b);
}

// wavefront sum of a 64-bit counter, one atomic per wavefront, striped over
// 64 slots (the host adds them) so that wavefronts do not queue on one address
__device__ __forceinline__ void wave_add(unsigned long long *ctr, unsigned long long v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0 && v)
        atomicAdd(ctr + ((blockIdx.x * (kBS / 64) + (threadIdx.x >> 6)) & 63), v);
}

// ---------------------------------------------------------------------------
// Estimate epilogue: the decisions that need no bound, and the hard list.
// ---------------------------------------------------------------------------
struct EstOut {
    uint8_t *dec;        // [n] decision per queue entry (255: in the hard list)
    double *hardA;       // tensors of hard cubes, entry pairs outermost: the
                         // pair (A[2 e], A[2 e + 1]) of slot k at double2 e * hs + k
    double *hardE;       // [cap] their error bounds (0 for exact exponentials)
    int32_t *hardIdx;    // [cap] their queue indices
    unsigned *hardCount; // device counter (reset by the host per pass)
    const int32_t *ncount;  // device count of entries (or chunks) when the
                            // launch is sized by a capacity; null: the launch size
    unsigned *tick = nullptr;  // [8] zeroed slot counters (persistent tiled grid)
    unsigned *ovf = nullptr;   // set when a capacity-sized tiled grid is short of chunks
    double *allA = nullptr;    // every entry's tensor (children re-expanded from
                               // their parents' next level), or null: pair e
                               // of entry k at double2 e * as + k
    int64_t hs = 0;            // slots of the hard list (its stride)
    int64_t as = 0;            // entries of allA (its stride)
};

constexpr uint8_t DEC_HARD = 255;

// slot of this lane in a list appended by the whole wavefront
__device__ __forceinline__ unsigned wave_append(unsigned *ctr, bool want) {
    const unsigned long long m = __ballot(want);
    const int lane = threadIdx.x & 63;
    unsigned base = 0;
    const int leader = __ffsll((long long)m) - 1;
    if (m && lane == leader) base = atomicAdd(ctr, (unsigned)__popcll(m));
    base = __shfl(base, leader < 0 ? 0 : leader, 64);
    return base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
}

// l1 mass of the entries of degree above one (Step 3) and of all entries
__device__ __forceinline__ void masses(const double *A, double &E, double &asum) {
    E = 0.0;
    asum = 0.0;
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
}

// l1 error band of A: the accumulated bound of the FAST exponentials plus a
// floor for double-precision rounding; zero for exact exponentials (no guard)
__device__ __forceinline__ double error_band(bool fast, double EA, double asum) {
    return fast ? EA + 1e-13 * asum : 0.0;
}

__device__ __forceinline__ uint8_t keep_code(const Grid &g, int level) {
    return (level == g.K) ? DEC_HMIN : DEC_REFINE;
}

// Decisions without the bound; DEC_HARD when the bound is needed.
__device__ __forceinline__ uint8_t easy_decision(const Grid &g, int level, bool fast,
                                                 const double *A, double EA) {
    double E, asum;
    masses(A, E, asum);
    const double band = error_band(fast, EA, asum);
    if (level >= 1) {
        // Step 3: higher-order mass under the user bound -> trilinear leaf
        if (band > 0.0 && fabs(2.0 * E - g.tau) <= 2.0 * band) return DEC_GUARD;
        if (2.0 * E <= g.tau) return DEC_CONV;
    }
    // two sampled values of P on either side of c imply L <= c <= U for every
    // valid enclosure [L, U] of P, so Step 2 keeps the cube
    double slo, shi;
    sample_range(A, slo, shi);
    const double tiny = 1e-12 * asum + band;
    if (slo <= g.c - tiny && shi >= g.c + tiny) return keep_code(g, level);
    return DEC_HARD;
}

__device__ __forceinline__ void epilogue(const Grid &g, int level, bool fast, const double *A,
                                         double EA, int64_t qi, bool valid, const EstOut &o) {
    const uint8_t d = valid ? easy_decision(g, level, fast, A, EA) : (uint8_t)0;
    if (o.allA && valid) {
        double2 *dst = reinterpret_cast<double2 *>(o.allA) + qi;
#pragma unroll
        for (int e = 0; e < 32; ++e) dst[e * o.as] = make_double2(A[2 * e], A[2 * e + 1]);
    }
    const bool hard = valid && d == DEC_HARD;
    const unsigned slot = wave_append(o.hardCount, hard);
    if (hard) {
        // a wavefront's slots are consecutive: each pair is one contiguous
        // run of stores across its lanes
        double2 *dst = reinterpret_cast<double2 *>(o.hardA) + slot;
#pragma unroll
        for (int e = 0; e < 32; ++e) dst[e * o.hs] = make_double2(A[2 * e], A[2 * e + 1]);
        o.hardE[slot] = EA;
        o.hardIdx[slot] = (int32_t)qi;
    }
    if (valid) o.dec[qi] = d;
}

// First interval of an atom's row of the projection table along one axis:
// one below the interval holding x - R_c.  Every kernel evaluates this same
// expression (a multiplication when h is a power of two: then exact).
__device__ __forceinline__ int proj_first(const Grid &g, int axis, double x, double rc, double h,
                                          int level) {
    const double u = x - g.o[axis] - rc;
    return (int)floor(g.inv_h0 != 0.0 ? u * ldexp(g.inv_h0, level) : u / h) - 1;
}

// Projection of atom i on interval j along `axis` from the table, when the
// interval has a slot in the atom's row (it always has when it lies within
// R_c); false: not tabulated, project in place.  The table and the
// in-place projection agree bit for bit (lo + s, the interval's midpoint,
// is the same double for the lattice index j).
__device__ __forceinline__ bool tab_proj(const ProjTab &P, int axis, int64_t i, int j, int first,
                                         double a[4], double &err) {
    const int64_t ia = (int64_t)axis * P.n + i;
    const int slot = j - first;
    if (slot < 0 || slot >= P.ns) return false;
    const double2 *src = reinterpret_cast<const double2 *>(P.t + 6 * (ia * P.ns + slot));
    const double2 u0 = src[0], u1 = src[1], u2 = src[2];
    a[0] = u0.x;
    a[1] = u0.y;
    a[2] = u1.x;
    a[3] = u1.y;
    err = u2.x;
    return true;
}

// ---------------------------------------------------------------------------
// Tensor estimate, one thread per cube.  The thread walks its root's
// neighbourhood list (threads of a wavefront usually share a root, so the
// list loads are uniform), keeps the atoms within R_c of its own cube,
// projects the three Gaussian factors and accumulates the 4x4x4 rank-one
// update in double precision.  With FAST exponentials it also accumulates the
// l1 error bound of the tensor: a perturbation da of a factor moves
// w a (x) b (x) c by at most w (|da| |b| |c| + |a| |db| |c| + |a| |b| |dc|).
// Used for the shallow levels (few cubes per root) and the debug hook.
// ---------------------------------------------------------------------------
template <bool FAST, int QH, bool EPI>
__global__ __launch_bounds__(kBS) void k_estimate_thread(
    const Grid *__restrict__ gt, int level, GLRule<double> R, const int4 *__restrict__ q, int64_t n,
    const int32_t *__restrict__ subset, const int32_t *__restrict__ root_start,
    const int32_t *__restrict__ root_atoms, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ az, const double *__restrict__ aw,
    double *__restrict__ Aout, double *__restrict__ Eout, EstOut o,
    unsigned long long *__restrict__ pairs, ProjTab P) {
    const int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    unsigned long long np = 0;
    const int64_t n_ = o.ncount ? min((int64_t)*o.ncount, n) : n;
    const bool valid = t < n_;
    const int64_t qi = valid ? (subset ? subset[t] : t) : 0;
    const int4 c = valid ? q[qi] : make_int4(0, 0, 0, 0);
    const Grid &g = gt[c.w];
    double A[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) A[e] = 0.0;
    double EA = 0.0;
    if (valid) {
        const double h = ldexp(g.h0, -level);
        const double lo[3] = {g.o[0] + c.x * h, g.o[1] + c.y * h, g.o[2] + c.z * h};
        const double hi[3] = {lo[0] + h, lo[1] + h, lo[2] + h};
        const double mid[3] = {lo[0] + 0.5 * h, lo[1] + 0.5 * h, lo[2] + 0.5 * h};
        const double s = 0.5 * h;
        const int64_t root = g.root_base +
            ((int64_t)(c.z >> level) * g.nr[1] + (c.y >> level)) * g.nr[0] + (c.x >> level);
        const double rc2 = g.rc2, rc = sqrt(rc2);
        const int b = root_start[root], e_ = root_start[root + 1];
        // exact instantiation: the list is walked with its loads ahead of
        // use (the index two atoms ahead, the coordinates and weight one atom
        // ahead), so an atom's step waits on its table entries alone; the
        // FAST one has no registers to spare for that and loads in place
        int i1 = 0, i2 = 0;
        double nx_ = 0.0, ny_ = 0.0, nz_ = 0.0, nw_ = 0.0;
        if (!FAST && b < e_) {
            i1 = root_atoms[b];
            i2 = b + 1 < e_ ? root_atoms[b + 1] : 0;
            nx_ = ax[i1];
            ny_ = ay[i1];
            nz_ = az[i1];
            nw_ = aw[i1];
        }
        for (int p = b; p < e_; ++p) {
            int i;
            double x, y, z, w;
            if constexpr (FAST) {
                i = root_atoms[p];
                x = ax[i];
                y = ay[i];
                z = az[i];
                w = aw[i];
            } else {
                i = i1;
                x = nx_;
                y = ny_;
                z = nz_;
                w = nw_;
                i1 = i2;
                if (p + 2 < e_) i2 = root_atoms[p + 2];
                if (p + 1 < e_) {
                    nx_ = ax[i1];
                    ny_ = ay[i1];
                    nz_ = az[i1];
                    nw_ = aw[i1];
                }
            }
            const double dx = fmax(fmax(lo[0] - x, x - hi[0]), 0.0);
            const double dy = fmax(fmax(lo[1] - y, y - hi[1]), 0.0);
            const double dz = fmax(fmax(lo[2] - z, z - hi[2]), 0.0);
            if (dx * dx + dy * dy + dz * dz > rc2) continue;
            ++np;
            double px[4], py[4], pz[4], ex, ey, ez;
            if (!P.t || !tab_proj(P, 0, i, c.x, proj_first(g, 0, x, rc, h, level), px, ex))
                project<FAST, QH>(R, g.D, s, mid[0] - x, g.deg, px, ex);
            if (!P.t || !tab_proj(P, 1, i, c.y, proj_first(g, 1, y, rc, h, level), py, ey))
                project<FAST, QH>(R, g.D, s, mid[1] - y, g.deg, py, ey);
            if (!P.t || !tab_proj(P, 2, i, c.z, proj_first(g, 2, z, rc, h, level), pz, ez))
                project<FAST, QH>(R, g.D, s, mid[2] - z, g.deg, pz, ez);
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
    }
    if (EPI) {
        epilogue(g, level, FAST, A, EA, qi, valid, o);
    } else if (valid) {
        double *dst = Aout + 64 * qi;
#pragma unroll
        for (int e = 0; e < 64; ++e) dst[e] = A[e];
        Eout[qi] = EA;
    }
    if (pairs) wave_add(pairs, np);
}

// ---------------------------------------------------------------------------
// Tensor estimate for deep levels: one 64-lane workgroup per chunk of at most
// 64 consecutive queue entries (or entries of a sorted subset of the queue)
// of one root (a root's cubes are contiguous in refinement order).
//
// The root's neighbourhood list is first filtered, 64 atoms at a time, down
// to the atoms within R_c of the chunk's bounding box, kept in list order in
// an LDS buffer; tiles of CH such atoms are then staged.  For a tile, each
// 1-D projection (atom, axis, interval) is put once into LDS and shared by
// every cube of the chunk on that interval; each lane then applies the
// per-cube R_c test and the rank-one update of its cube.  Same arithmetic,
// in the same atom order, as the per-thread kernel.
//
// A projection is needed only if some cube of the chunk on that interval can
// be within R_c of the atom: its 1-D distance squared plus the chunk's
// bounding-box distances squared on the other two axes, summed in the order
// of the per-cube test, must not exceed R_c^2 (floating-point addition is
// monotone, so the per-cube sum is at least that).  With a projection table
// the needed entries go from the table straight into LDS (global-to-LDS
// loads: no registers, many in flight); they are bit-identical to the
// projections computed here (same lattice points, same routine).
// ---------------------------------------------------------------------------

// The tiled kernels run one wavefront per workgroup: their lanes exchange data
// through LDS with no workgroup barrier (wave_lds_sync).  A workgroup
// barrier's fence would also wait for the global-to-LDS copies still in
// flight, which the pipelined tiles overlap with the updates.

constexpr int64_t kXcdBlock = 256;  // consecutive chunks per XCD turn

// Bijection of [0, n): slot v = 8 j + x (x: the XCD the slot lands on) maps
// to block (j / B) * 8 + x, offset j % B, for the slots below the last whole
// group of 8 blocks; the remaining slots map to themselves.
__device__ __forceinline__ int64_t xcd_chunk(int64_t v, int64_t n) {
    const int64_t nf = n - n % (8 * kXcdBlock);
    if (v >= nf) return v;
    const int64_t j = v >> 3, x = v & 7;
    return ((j / kXcdBlock) * 8 + x) * kXcdBlock + j % kXcdBlock;
}

constexpr int kTileIv = 8;  // intervals per axis a chunk may span (levels <= 3)
constexpr int64_t kStrideGrid = 2048;  // workgroups of the persistent tiled grid (tuning option)
// workgroups (one wavefront each) of a grouped launch whose chunk count is on
// the device: many more than are resident, so the hardware balances them,
// each striding over the chunk groups
constexpr int64_t kGroupedGrid = 65536;
                                       // (about the resident count: 256 CUs x 8)

template <bool FAST, int QH, int CH, bool DYN>
__global__ __launch_bounds__(64, 2) void k_estimate_tiled(
    const Grid *__restrict__ gt, int level, GLRule<double> R, const int4 *__restrict__ q,
    const int32_t *__restrict__ subset, const int2 *__restrict__ chunks, int64_t nch_cap,
    const int32_t *__restrict__ root_start,
    const int32_t *__restrict__ root_atoms, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ az, const double *__restrict__ aw,
    EstOut o, unsigned long long *__restrict__ pairs, ProjTab P) {
    // Two sets of WS projection items: the table rows of the next tile are
    // copied into one set while the rank-one updates of the current tile
    // read the other.  A tile holds as many atoms as the chunk's items fit
    // (WS / (intervals the chunk spans on the three axes)); the atom buffer
    // holds a tile plus one refill of at most 64.
    constexpr int WS = CH * 16;
    constexpr int NA = WS / 3;  // most atoms in a tile
    // the atom buffer is a ring of NB slots (a power of two >= NA + 64)
    constexpr int NB = (NA + 64 <= 128) ? 128 : ((NA + 64 <= 256) ? 256 : 512);
    // item w = a * per_atom + (axis offset) + interval: {a0, a1}, {a2, a3},
    // {err, squared 1-D distance}; a tile's atom weights alongside
    __shared__ double2 s0_01[WS], s0_23[WS], s0_ed[WS];
    __shared__ double2 s1_01[WS], s1_23[WS], s1_ed[WS];
    __shared__ double s0_w[NA], s1_w[NA];
    __shared__ int b_i[NB];
    __shared__ int b_lo[NB][3];  // first table interval per axis
    __shared__ double b_w[NB];
    __shared__ double b_x[NB][3];
    const int lane = threadIdx.x;
    using lds_ptr = __attribute__((address_space(3))) void *;
    // XCD-aware assignment: the hardware deals workgroups round-robin to the
    // 8 XCDs, each with its own L2, and neighbouring chunks read the same atoms
    // and table rows.  Workgroup slot v (v % 8 = its XCD) takes chunk
    // xcd_chunk(v): blocks of kXcdBlock consecutive chunks are dealt to the
    // XCDs in turn, so an XCD works through one block at a time while the
    // blocks of all XCDs interleave over the queue (balanced work).
    //
    // Slots: DYN = false, one per workgroup (the grid covers the chunks, or
    // with a device count their capacity); DYN = true, a fixed persistent
    // grid (a multiple of 8, o.tick zeroed; a tuning option):
    // the workgroups on XCD x = blockIdx % 8 draw slots 8 t + x from their own
    // counter tick[x] (drawn one chunk ahead), so each XCD walks its slots in
    // order however long single chunks take.  Every workgroup stops at its
    // first slot past the end; the counters only grow.
    const int64_t nch = o.ncount ? min((int64_t)*o.ncount, nch_cap) : nch_cap;
    // a capacity-sized grid of one workgroup per chunk that is too small for
    // the device's chunk count reports it (the results are then not used)
    if (!DYN && o.ovf && o.ncount && blockIdx.x == 0 && lane == 0 && *o.ncount > (int)gridDim.x)
        atomicOr(o.ovf, 1u);
    const unsigned xq = blockIdx.x & 7u;
    unsigned tdraw = 0;
    if (DYN && lane == 0) tdraw = atomicAdd(o.tick + xq, 1u);
    int64_t v = DYN ? 8 * (int64_t)__shfl(tdraw, 0, 64) + xq : (int64_t)blockIdx.x;
    while (v < nch) {
    if (DYN && lane == 0) tdraw = atomicAdd(o.tick + xq, 1u);
    const int64_t cix = xcd_chunk(v, nch);
    const int2 ch = chunks[cix];
    const bool valid = lane < ch.y;
    const int64_t pos = (int64_t)ch.x + (valid ? lane : 0);
    const int64_t qi = subset ? subset[pos] : pos;
    const int4 c = q[qi];
    const int4 c0 = q[subset ? subset[ch.x] : ch.x];
    const Grid &g = gt[c0.w];  // one root, hence one conformation, per chunk
    const double rc2 = g.rc2, D = g.D, rc = sqrt(rc2);
    const double h = ldexp(g.h0, -level);
    const double s = 0.5 * h;
    const int rxyz[3] = {c0.x >> level, c0.y >> level, c0.z >> level};
    const int64_t root = g.root_base + ((int64_t)rxyz[2] * g.nr[1] + rxyz[1]) * g.nr[0] + rxyz[0];
    // local interval indices of this lane's cube, and the chunk's range
    const int li[3] = {c.x - (rxyz[0] << level), c.y - (rxyz[1] << level),
                       c.z - (rxyz[2] << level)};
    int mn[3], mx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int vlo = valid ? li[a] : 1 << 20, vhi = valid ? li[a] : -1;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            vlo = min(vlo, __shfl_xor(vlo, d, 64));
            vhi = max(vhi, __shfl_xor(vhi, d, 64));
        }
        // wave-uniform: held in scalar registers, so the tile loops are too
        mn[a] = __builtin_amdgcn_readfirstlane(vlo);
        mx[a] = __builtin_amdgcn_readfirstlane(vhi);
    }
    const int nv[3] = {mx[0] - mn[0] + 1, mx[1] - mn[1] + 1, mx[2] - mn[2] + 1};
    double base[3], blo[3], bhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        base[a] = g.o[a] + (double)(rxyz[a] << level) * h;
        blo[a] = base[a] + mn[a] * h;
        bhi[a] = base[a] + (mx[a] + 1) * h;
    }
    const int per_atom = nv[0] + nv[1] + nv[2];
    const int tile = WS / per_atom;  // atoms per tile for this chunk
    // this lane's items in a tile: x, y, z interval of its cube
    const int ox = li[0] - mn[0], oy = nv[0] + li[1] - mn[1], oz = nv[0] + nv[1] + li[2] - mn[2];
    const int re = root_start[root + 1];
    int head = root_start[root], nbuf = 0, bs = 0;  // ring: atoms [bs, bs + nbuf)
    double A[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) A[e] = 0.0;
    double EA = 0.0;
    unsigned long long np = 0;

    // refill: atoms of the list within R_c of the chunk's box, in order,
    // until a tile is buffered or the list ends
    auto refill = [&]() {
        while (nbuf < tile && head < re) {
            const int p = head + lane;
            bool use = false;
            int i = 0;
            double x[3] = {0.0, 0.0, 0.0};
            if (p < re) {
                i = root_atoms[p];
                x[0] = ax[i];
                x[1] = ay[i];
                x[2] = az[i];
                double d2 = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double d = fmax(fmax(blo[a] - x[a], x[a] - bhi[a]), 0.0);
                    d2 += d * d;
                }
                use = d2 <= rc2;
            }
            const unsigned long long m = __ballot(use);
            if (use) {
                const int at = (bs + nbuf + __popcll(m & ((1ull << lane) - 1ull))) & (NB - 1);
                b_i[at] = i;
                b_w[at] = aw[i];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    b_x[at][a] = x[a];
                    b_lo[at][a] = proj_first(g, a, x[a], rc, h, level);
                }
            }
            nbuf += __popcll(m);
            head += 64;
        }
        wave_lds_sync();
    };
    // projections of the first na buffered atoms on the chunk's intervals
    // into one item set: table rows by global-to-LDS copies (issued, not
    // waited for), pruned and in-place items by LDS stores; the atoms then
    // leave the ring
    auto stage = [&](int na, double2 *t01, double2 *t23, double2 *ted, double *tw) {
        const int nw = na * per_atom;
        for (int k0 = 0; k0 < nw; k0 += 64) {
            const int w = k0 + lane;
            const double *src = nullptr;
            if (w < nw) {
                const int a_loc = w / per_atom;
                const int a_idx = (bs + a_loc) & (NB - 1);
                int r = w - a_loc * per_atom, axis = 0;
                if (r >= nv[0]) {
                    r -= nv[0];
                    axis = 1;
                    if (r >= nv[1]) {
                        r -= nv[1];
                        axis = 2;
                    }
                }
                const double xa = b_x[a_idx][axis];
                const double lo = base[axis] + (mn[axis] + r) * h, hi = lo + h;
                const double d = fmax(fmax(lo - xa, xa - hi), 0.0);
                const double dd = d * d;
                // no cube of the chunk on this interval is in range: only the
                // distance is read
                double b[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double e = fmax(fmax(blo[a] - b_x[a_idx][a], b_x[a_idx][a] - bhi[a]), 0.0);
                    b[a] = a == axis ? dd : e * e;
                }
                const int slot = (rxyz[axis] << level) + mn[axis] + r - b_lo[a_idx][axis];
                if (b[0] + b[1] + b[2] > rc2) {
                    ted[w] = make_double2(0.0, dd);
                } else if (P.t && slot >= 0 && slot < P.ns) {
                    src = P.t + 6 * (((int64_t)axis * P.n + b_i[a_idx]) * P.ns + slot);
                } else {
                    double pr[4], err;
                    project<FAST, QH>(R, D, s, (lo + s) - xa, g.deg, pr, err);
                    t01[w] = make_double2(pr[0], pr[1]);
                    t23[w] = make_double2(pr[2], pr[3]);
                    ted[w] = make_double2(err, dd);
                }
            }
            if (src) {  // lane w's 16-byte pieces land at [k0 + lane] = [w]
                __builtin_amdgcn_global_load_lds(src, (lds_ptr)(t01 + k0), 16, 0, 0);
                __builtin_amdgcn_global_load_lds(src + 2, (lds_ptr)(t23 + k0), 16, 0, 0);
                __builtin_amdgcn_global_load_lds(src + 4, (lds_ptr)(ted + k0), 16, 0, 0);
            }
        }
        // a tile holds up to NA atoms (more than 64 with 32-atom tiles)
        for (int a = lane; a < na; a += 64) tw[a] = b_w[(bs + a) & (NB - 1)];
        // keep the copies issued here ahead of the update that follows
        __builtin_amdgcn_sched_barrier(0);
        bs = (bs + na) & (NB - 1);
        nbuf -= na;
        wave_lds_sync();
    };
    // the per-cube R_c test and the rank-one updates of a staged tile
    auto update = [&](int na, const double2 *t01, const double2 *t23, const double2 *ted,
                      const double *tw) {
        if (!valid) return;
        for (int a = 0; a < na; ++a) {
            const int ba = a * per_atom;
            const double2 ex = ted[ba + ox], ey = ted[ba + oy], ez = ted[ba + oz];
            if (ex.y + ey.y + ez.y > rc2) continue;
            ++np;
            const double2 x01 = t01[ba + ox], x23 = t23[ba + ox];
            const double2 y01 = t01[ba + oy], y23 = t23[ba + oy];
            const double2 z01 = t01[ba + oz], z23 = t23[ba + oz];
            const double px[4] = {x01.x, x01.y, x23.x, x23.y};
            const double py[4] = {y01.x, y01.y, y23.x, y23.y};
            const double pz[4] = {z01.x, z01.y, z23.x, z23.y};
            const double wgt = tw[a];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double wx = wgt * px[j];
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
                EA += wgt * ((ex.x * ny + nx * ey.x) * nz + nx * ny * ez.x);
            }
        }
    };

    // software pipeline over tiles: while tile t is summed from one item set,
    // the copies of tile t + 1 land in the other.  Before a set is refilled,
    // every copy issued so far is waited for (those into it were issued a
    // whole tile earlier)
    refill();
    int na_cur = min(tile, nbuf);
    stage(na_cur, s0_01, s0_23, s0_ed, s0_w);
    while (na_cur > 0) {
        refill();
        int na_nxt = min(tile, nbuf);
        __builtin_amdgcn_s_waitcnt(0);  // the current set's copies have landed
        wave_lds_sync();
        stage(na_nxt, s1_01, s1_23, s1_ed, s1_w);
        update(na_cur, s0_01, s0_23, s0_ed, s0_w);
        wave_lds_sync();
        na_cur = na_nxt;
        if (na_cur == 0) break;
        refill();
        na_nxt = min(tile, nbuf);
        __builtin_amdgcn_s_waitcnt(0);
        wave_lds_sync();
        stage(na_nxt, s0_01, s0_23, s0_ed, s0_w);
        update(na_cur, s1_01, s1_23, s1_ed, s1_w);
        wave_lds_sync();
        na_cur = na_nxt;
    }
    __builtin_amdgcn_s_waitcnt(0);  // no copy outlives the chunk
    epilogue(g, level, FAST, A, EA, qi, valid, o);
    if (pairs) wave_add(pairs, np);
    if (!DYN) break;
    v = 8 * (int64_t)__shfl(tdraw, 0, 64) + xq;
    }
}

// ---------------------------------------------------------------------------
// Tensor estimate with several chunks per wavefront: 64 / GL groups of GL
// lanes, each taking one chunk of at most GL cubes of one root (level 1,
// where a root holds at most 2 x 2 x 2 cubes, and optionally level 0, where
// it is one cube: GL = 8; deeper levels optionally in half-wave chunks,
// GL = 32).  Every group runs the steps of
// the tiled kernel on its own -- filters its root's list to the atoms within
// R_c of its cubes' box (in list order), stages CH of them, puts each needed
// projection once into LDS (from the projection table when there is one) and
// lets each lane apply the per-cube test and update -- and the wavefront
// loops while any group has atoms left.  IV bounds the intervals per axis a
// chunk spans.  Same arithmetic, in the same atom order per cube, as the
// per-thread kernel.
// ---------------------------------------------------------------------------
template <bool FAST, int QH, int CH, int GL, int IV>
__global__ __launch_bounds__(64, 2) void k_estimate_groups(
    const Grid *__restrict__ gt, int level, GLRule<double> R, const int4 *__restrict__ q,
    const int2 *__restrict__ chunks, int64_t nch_cap, const int32_t *__restrict__ root_start,
    const int32_t *__restrict__ root_atoms, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ az, const double *__restrict__ aw,
    EstOut o, unsigned long long *__restrict__ pairs, ProjTab P) {
    constexpr int NG = 64 / GL;                          // groups per wavefront
    constexpr int PA = 3 * IV;                           // items per atom, at most
    constexpr int WI = (CH * PA + GL - 1) / GL * GL;     // items per group (multiple of GL)
    constexpr int NB = CH + GL;                          // atom buffer per group
    constexpr unsigned long long GM = GL == 64 ? ~0ull : (1ull << GL) - 1ull;
    // item w of group gr sits at (w / GL) * 64 + gr * GL + w % GL, so the GL
    // items of all groups handled in one step are 64 consecutive slots
    __shared__ double2 t01[WI * NG], t23[WI * NG], ted[WI * NG];
    __shared__ int b_i[NG][NB];
    __shared__ int b_lo[NG][NB][3];
    __shared__ double b_w[NG][NB];
    __shared__ double b_x[NG][NB][3];
    const int lane = threadIdx.x, gr = lane / GL, gl = lane % GL;
    using lds_ptr = __attribute__((address_space(3))) void *;
    const int64_t nch = o.ncount ? min((int64_t)*o.ncount, nch_cap) : nch_cap;
    for (int64_t wv = blockIdx.x; wv * NG < nch; wv += gridDim.x) {
    const int64_t cix = wv * NG + gr;
    const int2 ch = cix < nch ? chunks[cix] : make_int2(0, 0);
    const bool valid = gl < ch.y;
    const int64_t qi = (int64_t)ch.x + (valid ? gl : 0);
    const int4 c = q[qi];
    const int4 c0 = q[ch.x];
    const Grid &g = gt[c0.w];  // one root, hence one conformation, per group
    const double rc2 = g.rc2, D = g.D, rc = sqrt(rc2);
    const double h = ldexp(g.h0, -level);
    const double s = 0.5 * h;
    const int rxyz[3] = {c0.x >> level, c0.y >> level, c0.z >> level};
    const int64_t root = g.root_base + ((int64_t)rxyz[2] * g.nr[1] + rxyz[1]) * g.nr[0] + rxyz[0];
    const int li[3] = {c.x - (rxyz[0] << level), c.y - (rxyz[1] << level),
                       c.z - (rxyz[2] << level)};
    int mn[3], mx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int vlo = valid ? li[a] : 1 << 20, vhi = valid ? li[a] : -1;
#pragma unroll
        for (int d = GL / 2; d > 0; d >>= 1) {  // within the group
            vlo = min(vlo, __shfl_xor(vlo, d, 64));
            vhi = max(vhi, __shfl_xor(vhi, d, 64));
        }
        mn[a] = vlo;
        mx[a] = vhi;
    }
    const bool gact = ch.y > 0;  // the group has cubes
    int nv[3];
    double base[3], blo[3], bhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nv[a] = gact ? mx[a] - mn[a] + 1 : 0;
        base[a] = g.o[a] + (double)(rxyz[a] << level) * h;
        blo[a] = base[a] + mn[a] * h;
        bhi[a] = base[a] + (mx[a] + 1) * h;
    }
    const int per_atom = nv[0] + nv[1] + nv[2];
    const int ox = li[0] - mn[0], oy = nv[0] + li[1] - mn[1], oz = nv[0] + nv[1] + li[2] - mn[2];
    const int re = gact ? root_start[root + 1] : 0;
    int head = gact ? root_start[root] : 0, nbuf = 0;
    double A[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) A[e] = 0.0;
    double EA = 0.0;
    unsigned long long np = 0;
    for (;;) {
        // refill each group's buffer, 8 atoms of its list per step
        for (;;) {
            const bool need = nbuf < CH && head < re;
            if (!__any(need)) break;
            const int p = head + gl;
            bool use = false;
            int i = 0;
            double x[3] = {0.0, 0.0, 0.0};
            if (need && p < re) {
                i = root_atoms[p];
                x[0] = ax[i];
                x[1] = ay[i];
                x[2] = az[i];
                double d2 = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double d = fmax(fmax(blo[a] - x[a], x[a] - bhi[a]), 0.0);
                    d2 += d * d;
                }
                use = d2 <= rc2;
            }
            const unsigned long long gm = (__ballot(use) >> (GL * gr)) & GM;
            if (use) {
                const int at = nbuf + __popcll(gm & ((1ull << gl) - 1ull));
                b_i[gr][at] = i;
                b_w[gr][at] = aw[i];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    b_x[gr][at][a] = x[a];
                    b_lo[gr][at][a] = proj_first(g, a, x[a], rc, h, level);
                }
            }
            if (need) {
                nbuf += __popcll(gm);
                head += GL;
            }
        }
        __syncthreads();
        const int na = min(CH, nbuf);
        if (!__any(na > 0)) break;
        // projections of each group's staged atoms on its intervals
        const int nw = na * per_atom;
        int nw_max = nw;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) nw_max = max(nw_max, __shfl_xor(nw_max, d, 64));
        for (int k0 = 0; k0 < nw_max; k0 += GL) {
            const int w = k0 + gl;
            const int slot_lds = (k0 / GL) * 64 + lane;
            const double *src = nullptr;
            if (w < nw) {
                const int a_idx = w / per_atom;
                int r = w - a_idx * per_atom, axis = 0;
                if (r >= nv[0]) {
                    r -= nv[0];
                    axis = 1;
                    if (r >= nv[1]) {
                        r -= nv[1];
                        axis = 2;
                    }
                }
                const double xa = b_x[gr][a_idx][axis];
                const double lo = base[axis] + (mn[axis] + r) * h, hi = lo + h;
                const double d = fmax(fmax(lo - xa, xa - hi), 0.0);
                const double dd = d * d;
                double b[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double e =
                        fmax(fmax(blo[a] - b_x[gr][a_idx][a], b_x[gr][a_idx][a] - bhi[a]), 0.0);
                    b[a] = a == axis ? dd : e * e;
                }
                const int slot = (rxyz[axis] << level) + mn[axis] + r - b_lo[gr][a_idx][axis];
                if (b[0] + b[1] + b[2] > rc2) {
                    ted[slot_lds] = make_double2(0.0, dd);
                } else if (P.t && slot >= 0 && slot < P.ns) {
                    src = P.t + 6 * (((int64_t)axis * P.n + b_i[gr][a_idx]) * P.ns + slot);
                } else {
                    double pr[4], err;
                    project<FAST, QH>(R, D, s, (lo + s) - xa, g.deg, pr, err);
                    t01[slot_lds] = make_double2(pr[0], pr[1]);
                    t23[slot_lds] = make_double2(pr[2], pr[3]);
                    ted[slot_lds] = make_double2(err, dd);
                }
            }
            if (src) {  // lane's 16-byte pieces land at [(k0 / GL) * 64 + lane]
                const int blk = (k0 / GL) * 64;
                __builtin_amdgcn_global_load_lds(src, (lds_ptr)(t01 + blk), 16, 0, 0);
                __builtin_amdgcn_global_load_lds(src + 2, (lds_ptr)(t23 + blk), 16, 0, 0);
                __builtin_amdgcn_global_load_lds(src + 4, (lds_ptr)(ted + blk), 16, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int gofs = gr * GL;
        int na_max = na;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) na_max = max(na_max, __shfl_xor(na_max, d, 64));
        for (int a = 0; a < na_max; ++a) {
            if (!valid || a >= na) continue;
            const int wa = a * per_atom;
            const int ix = ((wa + ox) / GL) * 64 + gofs + (wa + ox) % GL;
            const int iy = ((wa + oy) / GL) * 64 + gofs + (wa + oy) % GL;
            const int iz = ((wa + oz) / GL) * 64 + gofs + (wa + oz) % GL;
            const double2 ex = ted[ix], ey = ted[iy], ez = ted[iz];
            if (ex.y + ey.y + ez.y > rc2) continue;
            ++np;
            const double2 x01 = t01[ix], x23 = t23[ix];
            const double2 y01 = t01[iy], y23 = t23[iy];
            const double2 z01 = t01[iz], z23 = t23[iz];
            const double px[4] = {x01.x, x01.y, x23.x, x23.y};
            const double py[4] = {y01.x, y01.y, y23.x, y23.y};
            const double pz[4] = {z01.x, z01.y, z23.x, z23.y};
            const double wgt = b_w[gr][a];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double wx = wgt * px[j];
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
                EA += wgt * ((ex.x * ny + nx * ey.x) * nz + nx * ny * ez.x);
            }
        }
        __syncthreads();
        // move each group's atoms not yet staged (fewer than GL) to the front
        const int rest = nbuf - na;
        int mi = 0, ml[3] = {0, 0, 0};
        double mw = 0.0, mx3[3] = {0.0, 0.0, 0.0};
        if (gl < rest) {
            mi = b_i[gr][na + gl];
            mw = b_w[gr][na + gl];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ml[a] = b_lo[gr][na + gl][a];
                mx3[a] = b_x[gr][na + gl][a];
            }
        }
        __syncthreads();
        if (gl < rest) {
            b_i[gr][gl] = mi;
            b_w[gr][gl] = mw;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b_lo[gr][gl][a] = ml[a];
                b_x[gr][gl][a] = mx3[a];
            }
        }
        nbuf = rest;
    }
    epilogue(g, level, FAST, A, EA, qi, valid, o);
    if (pairs) wave_add(pairs, np);
    }
}

// ---------------------------------------------------------------------------
// Projection table of one level: one thread per (axis, atom, slot).  A row
// (axis, atom) starts at proj_first and holds ceil(2 R_c / h) + 3 intervals,
// so every interval within R_c of the atom along the axis has a slot (the
// tiled kernel still checks, and projects in place on a miss).  An entry is
// {a0, a1, a2, a3, err, squared 1-D distance}.  Lattice points are exact
// multiples of the finest spacing, so an interval's bounds are the same
// doubles here and in the estimate kernels.
// ---------------------------------------------------------------------------
template <bool FAST, int QH>
__global__ void k_proj_table(const Grid *__restrict__ gt, int nconf, int level, GLRule<double> R,
                             const double *__restrict__ ax, const double *__restrict__ ay,
                             const double *__restrict__ az, int64_t n, int ns,
                             double *__restrict__ T) {
    const int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t >= 3 * n * ns) return;
    const int64_t ia = t / ns;  // axis * n + atom
    const int slot = (int)(t - ia * ns);
    const int axis = (int)(ia / n);
    const int64_t i = ia - axis * n;
    const Grid &g = gt[conf_of_atom(gt, nconf, i)];
    const double x = axis == 0 ? ax[i] : (axis == 1 ? ay[i] : az[i]);
    const double h = ldexp(g.h0, -level), s = 0.5 * h;
    const int first = proj_first(g, axis, x, sqrt(g.rc2), h, level);
    const double lo = g.o[axis] + (double)(first + slot) * h, hi = lo + h;
    const double d = fmax(fmax(lo - x, x - hi), 0.0);
    double pr[4] = {0.0, 0.0, 0.0, 0.0}, err = 0.0;
    if (d * d <= g.rc2) project<FAST, QH>(R, g.D, s, (lo + s) - x, g.deg, pr, err);
    double2 *dst = reinterpret_cast<double2 *>(T + 6 * t);
    dst[0] = make_double2(pr[0], pr[1]);
    dst[1] = make_double2(pr[2], pr[3]);
    dst[2] = make_double2(err, d * d);
}

// ---------------------------------------------------------------------------
// Step 2 on the hard list: nested-SVD bound, keep iff L <= c <= U.  For
// tensors built with FAST exponentials, a decision whose margin |L - c| or
// |U - c| lies within kKappa * band * amp plus the rank-flip cap becomes
// DEC_GUARD and is redone with exact exponentials.
// The list length is read on the device.
// ---------------------------------------------------------------------------

// Safety factor on the first-order perturbation estimate band * amp of the
// bound (measured deviations of bounds from FAST tensors stay below
// 0.25 band * amp).
constexpr double kKappa = 8.0;

template <bool FAST>
__global__ __launch_bounds__(kBS, 2) void k_bound(Grid g, int level, EstOut o) {
    __shared__ double wsh[36 * kBS];
    const int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t >= (int64_t)*o.hardCount) return;
    double A[64];
    const double2 *src = reinterpret_cast<const double2 *>(o.hardA) + t;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        const double2 v = src[e * o.hs];
        A[2 * e] = v.x;
        A[2 * e + 1] = v.y;
    }
    double E, asum;
    masses(A, E, asum);
    const double band = error_band(FAST, o.hardE[t], asum);
    const BoundResult B = nested_bound<FAST>(A, band, wsh + threadIdx.x, kBS);
    uint8_t d;
    const double tol = kKappa * band * B.amp + B.jump;
    if (band > 0.0 && (fabs(B.L - g.c) <= tol || fabs(B.U - g.c) <= tol))
        d = DEC_GUARD;
    else
        d = (B.L <= g.c && g.c <= B.U) ? keep_code(g, level) : DEC_DISCARD;
    o.dec[o.hardIdx[t]] = d;
}

// chunking of a level queue into runs of one root, at most 64 entries each
__device__ __forceinline__ int64_t root_of(const Grid *__restrict__ gt, int level, int4 c) {
    const Grid &g = gt[c.w];
    return g.root_base +
           ((int64_t)(c.z >> level) * g.nr[1] + (c.y >> level)) * g.nr[0] + (c.x >> level);
}

__global__ void k_run_flags(const Grid *__restrict__ gt, int level, const int4 *__restrict__ q,
                            const int32_t *__restrict__ subset, int64_t n,
                            const int32_t *__restrict__ nd, int32_t *__restrict__ f) {
    const int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    if (nd && i >= (int64_t)*nd) {  // capacity-sized launch: zero the tail for the scan
        f[i] = 0;
        return;
    }
    if (i == 0) {
        f[i] = 1;
        return;
    }
    const int4 a = q[subset ? subset[i] : i], b = q[subset ? subset[i - 1] : i - 1];
    f[i] = (root_of(gt, level, a) != root_of(gt, level, b)) ? 1 : 0;
}

__global__ void k_run_starts(const int32_t *__restrict__ f, const int32_t *__restrict__ off,
                             int64_t n, int32_t *__restrict__ starts) {
    const int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i < n && f[i]) starts[off[i]] = (int32_t)i;
}

__global__ void k_run_chunk_counts(const int32_t *__restrict__ starts, int64_t nruns, int64_t n,
                                   const int32_t *__restrict__ nrd, const int32_t *__restrict__ nd,
                                   int cmax, int32_t *__restrict__ cnt) {
    const int64_t r = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (r >= nruns) return;
    const int64_t R = nrd ? min((int64_t)*nrd, nruns) : nruns, N = nd ? (int64_t)*nd : n;
    if (r >= R) {
        cnt[r] = 0;
        return;
    }
    const int64_t len = ((r + 1 < R) ? starts[r + 1] : N) - starts[r];
    cnt[r] = (int32_t)((len + cmax - 1) / cmax);
}

__global__ void k_run_chunk_emit(const int32_t *__restrict__ starts, int64_t nruns, int64_t n,
                                 const int32_t *__restrict__ nrd, const int32_t *__restrict__ nd,
                                 int cmax, const int32_t *__restrict__ coff,
                                 int2 *__restrict__ chunks) {
    const int64_t r = blockIdx.x * (int64_t)kBS + threadIdx.x;
    const int64_t R = nrd ? min((int64_t)*nrd, nruns) : nruns, N = nd ? (int64_t)*nd : n;
    if (r >= R) return;
    const int64_t b = starts[r], len = ((r + 1 < R) ? starts[r + 1] : N) - b;
    int2 *o = chunks + coff[r];
    for (int64_t k = 0; k * cmax < len; ++k)
        o[k] = make_int2((int32_t)(b + cmax * k), (int32_t)min<int64_t>(cmax, len - cmax * k));
}

// Chunks reordered by the length of their root's atom list, longest first, in
// buckets of 8 atoms: a wavefront of the grouped kernel then holds groups of
// like length, which loop about equally long.  A counting sort: per-workgroup
// bucket counts (LDS atomics), one scan over (bucket, workgroup), then each
// workgroup scatters its chunks from its own offsets (the order inside a
// workgroup's bucket is that of its LDS atomics).  Each chunk's result is its
// own, so the order changes no value.
__device__ __forceinline__ int chunk_len_bucket(const Grid *__restrict__ gt, int level,
                                                const int4 *__restrict__ q, int2 ch,
                                                const int32_t *__restrict__ root_start) {
    const int4 c = q[ch.x];
    const Grid &g = gt[c.w];
    const int64_t root = g.root_base +
        ((int64_t)(c.z >> level) * g.nr[1] + (c.y >> level)) * g.nr[0] + (c.x >> level);
    const int len = root_start[root + 1] - root_start[root];
    return kLenBuckets - 1 - min(len >> 3, kLenBuckets - 1);
}

// bcnt[b * gridDim.x + block]: chunks of workgroup `block` in bucket b
__global__ __launch_bounds__(kLenBuckets) void k_chunk_len_hist(
    const Grid *__restrict__ gt, int level, const int4 *__restrict__ q,
    const int2 *__restrict__ chunks, int64_t n, const int32_t *__restrict__ ncount,
    const int32_t *__restrict__ root_start, int32_t *__restrict__ bkt, int32_t *__restrict__ bcnt) {
    __shared__ int h[kLenBuckets];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)kLenBuckets + t;
    const int64_t nn = ncount ? min((int64_t)*ncount, n) : n;
    if (i < nn) {
        const int b = chunk_len_bucket(gt, level, q, chunks[i], root_start);
        bkt[i] = b;
        atomicAdd(&h[b], 1);
    }
    __syncthreads();
    bcnt[(int64_t)t * gridDim.x + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(kLenBuckets) void k_chunk_len_scatter(
    const int2 *__restrict__ chunks, int64_t n, const int32_t *__restrict__ ncount,
    const int32_t *__restrict__ bkt, const int32_t *__restrict__ boff, int2 *__restrict__ out) {
    __shared__ int h[kLenBuckets];
    const int t = threadIdx.x;
    h[t] = boff[(int64_t)t * gridDim.x + blockIdx.x];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)kLenBuckets + t;
    const int64_t nn = ncount ? min((int64_t)*ncount, n) : n;
    if (i < nn) out[atomicAdd(&h[bkt[i]], 1)] = chunks[i];
}

// Chunks starting in each bin of kChunkBin queue entries of a level (the
// chunks of one slice, ascending starts relative to the slice at queue
// position off): one thread per bin the slice touches, two binary searches.
__global__ void k_chunk_bins(const int2 *__restrict__ chunks, int64_t n, int64_t off, int64_t len,
                             int32_t *__restrict__ hist) {
    const int64_t b0 = off / kChunkBin;
    const int64_t j = b0 + blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (j * kChunkBin >= off + len) return;
    // chunk starts in [lo, hi) relative to the slice
    const int64_t lo = max((int64_t)0, j * kChunkBin - off), hi = min(len, (j + 1) * kChunkBin - off);
    auto lower = [&](int64_t v) {
        int64_t a = 0, b = n;
        while (a < b) {
            const int64_t m = (a + b) >> 1;
            if ((int64_t)chunks[m].x < v) a = m + 1;
            else b = m;
        }
        return a;
    };
    hist[j] += (int32_t)(lower(hi) - lower(lo));
}

__global__ void k_level_counts(const uint8_t *__restrict__ dec, int64_t n,
                               const int32_t *__restrict__ nd, int32_t *__restrict__ lc,
                               int32_t *__restrict__ cc) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n) return;
    if (nd && i >= (int64_t)*nd) {
        lc[i] = 0;
        cc[i] = 0;
        return;
    }
    const uint8_t d = dec[i];
    lc[i] = (d == DEC_CONV || d == DEC_HMIN) ? 1 : 0;
    cc[i] = (d == DEC_REFINE) ? 8 : 0;
}

// Capacity-sized launches (nd given) read the leaf base from *lbd and guard
// the leaf and child capacities (setting *ovf instead of writing past them).
__global__ void k_level_emit(const int4 *__restrict__ q, const uint8_t *__restrict__ dec, int64_t n,
                             int level, const int32_t *__restrict__ loff,
                             const int32_t *__restrict__ coff, tms_leaf *__restrict__ leaves,
                             int64_t leaf_base, int4 *__restrict__ qn, const int32_t *__restrict__ nd,
                             const int64_t *__restrict__ lbd, int64_t lcap, int64_t qcap,
                             unsigned *__restrict__ ovf, int32_t *__restrict__ qpar) {
    int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n || (nd && i >= (int64_t)*nd)) return;
    const uint8_t d = dec[i];
    const int4 c = q[i];
    if (nd) {
        const int64_t li = *lbd + loff[i];
        if (((d == DEC_CONV || d == DEC_HMIN) && li >= lcap) ||
            (d == DEC_REFINE && (int64_t)coff[i] + 8 > qcap)) {
            atomicOr(ovf, 1u);
            return;
        }
        leaf_base = *lbd;
    }
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
        // the children's parent: next-level entries 8 j .. 8 j + 7 come from
        // this entry
        if (qpar) qpar[coff[i] >> 3] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// Child tensors by re-expansion (Section 2.2.3, eq. childtensor): the parent's
// polynomial written in the Legendre basis of the child.  Along one axis the
// child covers parent coordinates u = (t + s)/2, t in [-1,1], s = -1 (lower
// half) or +1 (upper half), and
//   L0(u) = L0,  L1(u) = s/2 L0 + 1/2 L1,  L2(u) = 3s/4 L1 + 1/4 L2,
//   L3(u) = -s/8 L0 + 3/8 L1 + 5s/8 L2 + 1/8 L3
// (from (t + s)^2 = t^2 + 2 s t + 1, (t + s)^3 = t^3 + 3 s t^2 + 3 t + s and
// t^2 = (2 L2 + L0)/3, t^3 = (2 L3 + 3 L1)/5), so a series p becomes
//   x0 = p0 + s/2 p1 - s/8 p3,  x1 = 1/2 p1 + 3s/4 p2 + 3/8 p3,
//   x2 = 1/4 p2 + 5s/8 p3,      x3 = 1/8 p3
// along each axis in turn.  Then the decisions of the estimate epilogue.
// One thread per child; entries 8 j .. 8 j + 7 of the level (the children of
// parent qpar[j]) are consecutive, its octant the low bits of its coordinates.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void half_series(double p0, double p1, double p2, double p3, double s,
                                            double x[4]) {
    x[0] = p0 + (0.5 * s) * p1 - (0.125 * s) * p3;
    x[1] = 0.5 * p1 + (0.75 * s) * p2 + 0.375 * p3;
    x[2] = 0.25 * p2 + (0.625 * s) * p3;
    x[3] = 0.125 * p3;
}

__global__ __launch_bounds__(kBS) void k_reexpand(Grid g, int level, const int4 *__restrict__ q,
                                                  int64_t n, int64_t off,
                                                  const double *__restrict__ Apar, int64_t aps,
                                                  const int32_t *__restrict__ qpar, EstOut o) {
    const int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    const bool valid = t < n;  // every lane reaches the epilogue (wave append)
    double A[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) A[e] = 0.0;
    if (valid) {
        const int4 c = q[t];
        const double2 *src = reinterpret_cast<const double2 *>(Apar) + qpar[(off + t) >> 3];
#pragma unroll
        for (int e = 0; e < 32; ++e) {
            const double2 v = src[e * aps];
            A[2 * e] = v.x;
            A[2 * e + 1] = v.y;
        }
        const double sx = (c.x & 1) ? 1.0 : -1.0, sy = (c.y & 1) ? 1.0 : -1.0,
                     sz = (c.z & 1) ? 1.0 : -1.0;
        double x[4];
#pragma unroll
        for (int kl = 0; kl < 16; ++kl) {  // along x: index 16 j + kl
            half_series(A[kl], A[16 + kl], A[32 + kl], A[48 + kl], sx, x);
#pragma unroll
            for (int j = 0; j < 4; ++j) A[16 * j + kl] = x[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int l = 0; l < 4; ++l) {  // along y: index 16 j + 4 k + l
                const int b = 16 * j + l;
                half_series(A[b], A[b + 4], A[b + 8], A[b + 12], sy, x);
#pragma unroll
                for (int k = 0; k < 4; ++k) A[b + 4 * k] = x[k];
            }
#pragma unroll
        for (int jk = 0; jk < 16; ++jk) {  // along z: index 4 jk + l
            half_series(A[4 * jk], A[4 * jk + 1], A[4 * jk + 2], A[4 * jk + 3], sz, x);
#pragma unroll
            for (int l = 0; l < 4; ++l) A[4 * jk + l] = x[l];
        }
    }
    epilogue(g, level, false, A, 0.0, t, valid, o);
}

// A batch's leaves come out level by level, conformations in order inside a
// level.  Segment (level, conformation) heads, then a move that regroups the
// leaves conformation by conformation (order inside a segment kept).
__global__ void k_leaf_seg_heads(const tms_leaf *__restrict__ lv, int64_t n, int nconf,
                                 const int64_t *__restrict__ nd, int64_t *__restrict__ src) {
    const int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n || (nd && i >= *nd)) return;
    const int seg = lv[i].level * nconf + lv[i].conf;
    if (i == 0 || seg != lv[i - 1].level * nconf + lv[i - 1].conf) src[seg] = i;
}

__global__ void k_leaf_seg_move(const tms_leaf *__restrict__ lv, int64_t n, int nconf,
                                const int64_t *__restrict__ nd, const int64_t *__restrict__ src,
                                const int64_t *__restrict__ dst, tms_leaf *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (i >= n || (nd && i >= *nd)) return;
    const tms_leaf L = lv[i];
    const int seg = L.level * nconf + L.conf;
    out[dst[seg] + (i - src[seg])] = L;
}

// decision histogram in two passes (block partials, then one block), with
// no atomics on shared addresses
constexpr int kHistoBlocks = 1024;

__global__ void k_level_histo(const uint8_t *__restrict__ dec, int64_t n,
                              const int32_t *__restrict__ nd,
                              unsigned long long *__restrict__ part) {
    __shared__ unsigned long long sh[5][kBS];
    unsigned long long c[5] = {0, 0, 0, 0, 0};
    if (nd) n = min(n, (int64_t)*nd);
    for (int64_t i = blockIdx.x * (int64_t)kBS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBS) {
        const uint8_t d = dec[i];
        if (d < 5) c[d] += 1;
    }
#pragma unroll
    for (int b = 0; b < 5; ++b) sh[b][threadIdx.x] = c[b];
    __syncthreads();
    for (int st = kBS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int b = 0; b < 5; ++b) sh[b][threadIdx.x] += sh[b][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 5) part[5 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// one wavefront: lanes sum strided blocks, then a wavefront reduction
// (integer sums: the order does not matter)
__global__ void k_level_histo_final(const unsigned long long *__restrict__ part, int nb,
                                    unsigned long long *__restrict__ out) {
    const int lane = threadIdx.x;
    unsigned long long t[5] = {0, 0, 0, 0, 0};
    for (int b = lane; b < nb; b += 64)
#pragma unroll
        for (int k = 0; k < 5; ++k) t[k] += part[5 * b + k];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) t[k] += __shfl_xor(t[k], d, 64);
        if (lane == k) out[k] = t[k];
    }
}

__global__ __launch_bounds__(kBS) void k_bound_debug(const double *__restrict__ Ain,
                                                     const double *__restrict__ band, int64_t n,
                                                     double *__restrict__ out) {
    __shared__ double wsh[36 * kBS];
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t >= n) return;
    double A[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) A[e] = Ain[64 * t + e];
    BoundResult B = nested_bound(A, band ? band[t] : 0.0, wsh + threadIdx.x, kBS);
    out[6 * t + 0] = B.L;
    out[6 * t + 1] = B.U;
    out[6 * t + 2] = B.rho;
    out[6 * t + 3] = (double)B.r;
    out[6 * t + 4] = B.jump;
    out[6 * t + 5] = B.amp;
}

__global__ void k_fast_exp_debug(const double *__restrict__ x, int64_t n, double *__restrict__ y) {
    int64_t t = blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (t < n) y[t] = expn<true>(x[t]);
}

template <bool FAST, int QH>
hipError_t estimate_thread_t(const Grid *g, int level, const int4 *q, int64_t n,
                             const int32_t *subset, const int32_t *rs, const int32_t *ra,
                             const double *ax, const double *ay, const double *az, const double *aw,
                             double *A, double *E, const EstOut *o, unsigned long long *pairs,
                             const ProjTab &P, hipStream_t s) {
    GLRule<double> R = gl_rule<double>(QH);
    if (o)
        hipLaunchKernelGGL((k_estimate_thread<FAST, QH, true>), dim3(nblk(n)), dim3(kBS), 0, s, g,
                           level, R, q, n, subset, rs, ra, ax, ay, az, aw, A, E, *o, pairs, P);
    else
        hipLaunchKernelGGL((k_estimate_thread<FAST, QH, false>), dim3(nblk(n)), dim3(kBS), 0, s, g,
                           level, R, q, n, subset, rs, ra, ax, ay, az, aw, A, E, EstOut{}, pairs,
                           P);
    return hipGetLastError();
}

template <bool FAST, int QH>
hipError_t estimate_tiled_t(int ch, const Grid *g, int level, const int4 *q, const int32_t *subset,
                            const int2 *chunks, int64_t nchunks, const int32_t *rs,
                            const int32_t *ra, const double *ax, const double *ay, const double *az,
                            const double *aw, const EstOut &o, unsigned long long *pairs,
                            const ProjTab &P, hipStream_t s) {
    GLRule<double> R = gl_rule<double>(QH);
    // with slot counters a fixed grid (a multiple of 8) draws chunks from
    // per-XCD counters; otherwise one workgroup per chunk (with the count on
    // the device: nchunks is the capacity, and a shortfall is flagged)
    const bool dyn = o.tick != nullptr;
    const unsigned grid = (unsigned)(dyn ? std::min<int64_t>((nchunks + 7) / 8 * 8, kStrideGrid)
                                         : nchunks);
    // atoms staged per LDS tile (a tuning knob; the arithmetic is the same)
#define TMS_TILED_LAUNCH(C, D)                                                                   \
    hipLaunchKernelGGL((k_estimate_tiled<FAST, QH, C, D>), dim3(grid), dim3(64), 0, s, g, level, R, \
                       q, subset, chunks, nchunks, rs, ra, ax, ay, az, aw, o, pairs, P)
    switch (ch) {
    case 8:
        if (dyn) TMS_TILED_LAUNCH(8, true); else TMS_TILED_LAUNCH(8, false);
        break;
    case 32:
        if (dyn) TMS_TILED_LAUNCH(32, true); else TMS_TILED_LAUNCH(32, false);
        break;
    default:
        if (dyn) TMS_TILED_LAUNCH(16, true); else TMS_TILED_LAUNCH(16, false);
    }
#undef TMS_TILED_LAUNCH
    return hipGetLastError();
}

// several chunks per wavefront, tiles of 8 atoms (the LDS footprint of larger
// tiles would cost occupancy): level 1 in 8-lane groups (roots of <= 8
// cubes); levels 2-3 in half-wave groups of chunks of <= 32 cubes
template <bool FAST, int QH>
hipError_t estimate_groups_t(const Grid *g, int level, const int4 *q, const int2 *chunks,
                             int64_t nchunks, const int32_t *rs, const int32_t *ra,
                             const double *ax, const double *ay, const double *az,
                             const double *aw, const EstOut &o, unsigned long long *pairs,
                             const ProjTab &P, hipStream_t s) {
    GLRule<double> R = gl_rule<double>(QH);
    const int gl = level <= 1 ? 8 : 32;
    const int64_t waves = (nchunks + 64 / gl - 1) / (64 / gl);
    const unsigned grid = (unsigned)(o.ncount ? std::min<int64_t>(waves, kGroupedGrid) : waves);
    if (level == 0)
        hipLaunchKernelGGL((k_estimate_groups<FAST, QH, 8, 8, 1>), dim3(grid), dim3(64), 0, s, g,
                           level, R, q, chunks, nchunks, rs, ra, ax, ay, az, aw, o, pairs, P);
    else if (level == 1)
        hipLaunchKernelGGL((k_estimate_groups<FAST, QH, 8, 8, 2>), dim3(grid), dim3(64), 0, s, g,
                           level, R, q, chunks, nchunks, rs, ra, ax, ay, az, aw, o, pairs, P);
    else if (level == 2)
        hipLaunchKernelGGL((k_estimate_groups<FAST, QH, 8, 32, 4>), dim3(grid), dim3(64), 0, s, g,
                           level, R, q, chunks, nchunks, rs, ra, ax, ay, az, aw, o, pairs, P);
    else if (level == 3)
        hipLaunchKernelGGL((k_estimate_groups<FAST, QH, 8, 32, 8>), dim3(grid), dim3(64), 0, s, g,
                           level, R, q, chunks, nchunks, rs, ra, ax, ay, az, aw, o, pairs, P);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

#define TMS_QH_SWITCH(qh, CALL)                    \
    switch (qh) {                                  \
    case 4: { constexpr int QH = 4; return CALL; } \
    case 5: { constexpr int QH = 5; return CALL; } \
    case 6: { constexpr int QH = 6; return CALL; } \
    case 8: { constexpr int QH = 8; return CALL; } \
    default: return hipErrorInvalidValue;          \
    }

template <bool FAST>
hipError_t thread_dispatch(int qh, const Grid *g, int level, const int4 *q, int64_t n,
                           const int32_t *subset, const int32_t *rs, const int32_t *ra,
                           const double *ax, const double *ay, const double *az, const double *aw,
                           double *A, double *E, const EstOut *o, unsigned long long *pairs,
                           const ProjTab &P, hipStream_t s) {
    TMS_QH_SWITCH(qh, (estimate_thread_t<FAST, QH>(g, level, q, n, subset, rs, ra, ax, ay, az, aw,
                                                   A, E, o, pairs, P, s)))
}

template <bool FAST>
hipError_t tiled_dispatch(int qh, int ch, const Grid *g, int level, const int4 *q,
                          const int32_t *subset, const int2 *chunks, int64_t nchunks,
                          const int32_t *rs, const int32_t *ra, const double *ax, const double *ay,
                          const double *az, const double *aw, const EstOut &o,
                          unsigned long long *pairs, const ProjTab &P, bool half, hipStream_t s) {
    if (!subset && (level <= 1 || (half && level <= 3)))
        TMS_QH_SWITCH(qh, (estimate_groups_t<FAST, QH>(g, level, q, chunks, nchunks, rs, ra, ax,
                                                       ay, az, aw, o, pairs, P, s)))
    TMS_QH_SWITCH(qh, (estimate_tiled_t<FAST, QH>(ch, g, level, q, subset, chunks, nchunks, rs, ra,
                                                  ax, ay, az, aw, o, pairs, P, s)))
}

template <bool FAST, int QH>
hipError_t proj_table_t(const Grid *gt, int nconf, int level, const double *ax, const double *ay,
                        const double *az, int64_t n, int ns, double *t, hipStream_t s) {
    GLRule<double> R = gl_rule<double>(QH);
    hipLaunchKernelGGL((k_proj_table<FAST, QH>), dim3(nblk(3 * n * ns)), dim3(kBS), 0, s, gt, nconf,
                       level, R, ax, ay, az, n, ns, t);
    return hipGetLastError();
}

template <bool FAST>
hipError_t proj_table_dispatch(int qh, const Grid *gt, int nconf, int level, const double *ax,
                               const double *ay, const double *az, int64_t n, int ns, double *t,
                               hipStream_t s) {
    TMS_QH_SWITCH(qh, (proj_table_t<FAST, QH>(gt, nconf, level, ax, ay, az, n, ns, t, s)))
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

hipError_t launch_roots_emit(const Grid *gt, int nconf, const int32_t *flags, const int32_t *off,
                             int64_t nroots, int4 *q, hipStream_t s) {
    if (nroots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_roots_emit, dim3(nblk(nroots)), dim3(kBS), 0, s, gt, nconf, flags, off,
                       nroots, q);
    return hipGetLastError();
}

static int qh_for(const Grid &g, int level) {
    return gl_half_nodes(0.5 * ldexp(g.h0, -level) * sqrt(g.D), false);
}

hipError_t launch_estimate(const Grid &g, const Grid *gt, int level, int precision, const int4 *q,
                           int64_t n,
                           const int32_t *subset, const int32_t *root_start,
                           const int32_t *root_atoms, const double *ax, const double *ay,
                           const double *az, const double *aw, double *A, double *S,
                           int64_t *pairs, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int qh = qh_for(g, level);
    auto *pc = reinterpret_cast<unsigned long long *>(pairs);
    if (precision == TMS_PREC_FP32_GUARD)
        return thread_dispatch<true>(qh, gt, level, q, n, subset, root_start, root_atoms, ax, ay,
                                     az, aw, A, S, nullptr, pc, ProjTab{}, s);
    return thread_dispatch<false>(qh, gt, level, q, n, subset, root_start, root_atoms, ax, ay, az,
                                  aw, A, S, nullptr, pc, ProjTab{}, s);
}

hipError_t launch_estimate_decide(const Grid &g, const Grid *gt, int level, int precision,
                                  const int4 *q, int64_t n,
                                  const int32_t *subset, const int2 *chunks, int64_t nchunks,
                                  const int32_t *root_start, const int32_t *root_atoms,
                                  const double *ax, const double *ay, const double *az,
                                  const double *aw, uint8_t *dec, double *hardA, double *hardE,
                                  int32_t *hardIdx, unsigned *hardCount, int64_t *pairs,
                                  int tile_atoms, hipStream_t s, const int32_t *ncount,
                                  const ProjTab &pt, unsigned *tick, bool half, unsigned *ovf,
                                  double *allA, int64_t hs, int64_t as) {
    if (n <= 0) return hipSuccess;
    if (hs < n) return hipErrorInvalidValue;  // the hard list holds every entry
    const int qh = qh_for(g, level);
    const bool fast = precision == TMS_PREC_FP32_GUARD;
    auto *pc = reinterpret_cast<unsigned long long *>(pairs);
    EstOut o{dec, hardA, hardE, hardIdx, hardCount, ncount, tick, ovf, allA, hs, as};
    if (chunks) {
        if (nchunks <= 0) return hipSuccess;
        if (fast)
            return tiled_dispatch<true>(qh, tile_atoms, gt, level, q, subset, chunks, nchunks,
                                        root_start, root_atoms, ax, ay, az, aw, o, pc, pt, half,
                                        s);
        return tiled_dispatch<false>(qh, tile_atoms, gt, level, q, subset, chunks, nchunks,
                                     root_start, root_atoms, ax, ay, az, aw, o, pc, pt, half, s);
    }
    if (fast)
        return thread_dispatch<true>(qh, gt, level, q, n, subset, root_start, root_atoms, ax, ay,
                                     az, aw, nullptr, nullptr, &o, pc, pt, s);
    return thread_dispatch<false>(qh, gt, level, q, n, subset, root_start, root_atoms, ax, ay, az,
                                  aw, nullptr, nullptr, &o, pc, pt, s);
}

int proj_table_slots(const tms_cells *cells, int level) {
    double rc2 = 0.0;
    for (const Grid &gb : cells->gh) rc2 = std::max(rc2, gb.rc2);
    const double h = ldexp(cells->g.h0, -level);
    return (int)std::ceil(2.0 * std::sqrt(rc2) / h) + 3;
}

hipError_t launch_proj_table(const Grid &g, const Grid *gt, int nconf, int level, int precision,
                             const double *ax, const double *ay, const double *az, int64_t n,
                             int ns, double *t, hipStream_t s) {
    if (n <= 0 || ns <= 0) return hipSuccess;
    const int qh = qh_for(g, level);
    if (precision == TMS_PREC_FP32_GUARD)
        return proj_table_dispatch<true>(qh, gt, nconf, level, ax, ay, az, n, ns, t, s);
    return proj_table_dispatch<false>(qh, gt, nconf, level, ax, ay, az, n, ns, t, s);
}

hipError_t launch_reexpand(const Grid &g, int level, const int4 *q, int64_t n, int64_t off,
                          const double *Apar, int64_t aps, const int32_t *qpar, uint8_t *dec,
                          double *hardA, double *hardE, int32_t *hardIdx, unsigned *hardCount,
                          double *allA, hipStream_t s, int64_t hs, int64_t as) {
    if (n <= 0) return hipSuccess;
    if (hs < n) return hipErrorInvalidValue;
    EstOut o{dec, hardA, hardE, hardIdx, hardCount, nullptr};
    o.allA = allA;
    o.hs = hs;
    o.as = as;
    hipLaunchKernelGGL(k_reexpand, dim3(nblk(n)), dim3(kBS), 0, s, g, level, q, n, off, Apar, aps,
                       qpar, o);
    return hipGetLastError();
}

hipError_t launch_bound(const Grid &g, int level, int precision, int64_t max_n, uint8_t *dec,
                        double *hardA, double *hardE, int32_t *hardIdx, unsigned *hardCount,
                        hipStream_t s, int64_t hs) {
    if (max_n <= 0) return hipSuccess;
    if (hs < max_n) return hipErrorInvalidValue;
    EstOut o{dec, hardA, hardE, hardIdx, hardCount, nullptr};
    o.hs = hs;
    if (precision == TMS_PREC_FP32_GUARD)
        hipLaunchKernelGGL(k_bound<true>, dim3(nblk(max_n)), dim3(kBS), 0, s, g, level, o);
    else
        hipLaunchKernelGGL(k_bound<false>, dim3(nblk(max_n)), dim3(kBS), 0, s, g, level, o);
    return hipGetLastError();
}

hipError_t launch_run_flags(const Grid *gt, int level, const int4 *q, const int32_t *subset,
                            int64_t n, int32_t *f, hipStream_t s, const int32_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_run_flags, dim3(nblk(n)), dim3(kBS), 0, s, gt, level, q, subset, n, nd, f);
    return hipGetLastError();
}

hipError_t launch_run_starts(const int32_t *f, const int32_t *off, int64_t n, int32_t *starts,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_run_starts, dim3(nblk(n)), dim3(kBS), 0, s, f, off, n, starts);
    return hipGetLastError();
}

hipError_t launch_run_chunk_counts(const int32_t *starts, int64_t nruns, int64_t n, int32_t *cnt,
                                   hipStream_t s, const int32_t *nrd, const int32_t *nd, int cmax) {
    if (nruns <= 0) return hipSuccess;
    if (cmax < 1 || cmax > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_run_chunk_counts, dim3(nblk(nruns)), dim3(kBS), 0, s, starts, nruns, n, nrd,
                       nd, cmax, cnt);
    return hipGetLastError();
}

hipError_t launch_run_chunk_emit(const int32_t *starts, int64_t nruns, int64_t n,
                                 const int32_t *coff, int2 *chunks, hipStream_t s,
                                 const int32_t *nrd, const int32_t *nd, int cmax) {
    if (nruns <= 0) return hipSuccess;
    if (cmax < 1 || cmax > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_run_chunk_emit, dim3(nblk(nruns)), dim3(kBS), 0, s, starts, nruns, n, nrd,
                       nd, cmax, coff, chunks);
    return hipGetLastError();
}

hipError_t launch_chunk_bins(const int2 *chunks, int64_t n, int64_t off, int64_t len,
                             int32_t *hist, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    const int64_t nb = (off + len - 1) / kChunkBin - off / kChunkBin + 1;
    hipLaunchKernelGGL(k_chunk_bins, dim3(nblk(nb)), dim3(kBS), 0, s, chunks, n, off, len, hist);
    return hipGetLastError();
}

int64_t chunks_by_length_scratch(int64_t n) {
    return (int64_t)kLenBuckets * ((n + kLenBuckets - 1) / kLenBuckets);
}

hipError_t launch_chunks_by_length(const Grid *gt, int level, const int4 *q, const int2 *chunks,
                                   int64_t n, const int32_t *ncount, const int32_t *root_start,
                                   int32_t *bkt, int32_t *bcnt, int32_t *boff, void *tmp,
                                   int2 *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kLenBuckets - 1) / kLenBuckets;
    hipLaunchKernelGGL(k_chunk_len_hist, dim3((unsigned)nb), dim3(kLenBuckets), 0, s, gt, level, q,
                       chunks, n, ncount, root_start, bkt, bcnt);
    hipError_t e = exclusive_scan(bcnt, boff, nb * kLenBuckets, nullptr, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chunk_len_scatter, dim3((unsigned)nb), dim3(kLenBuckets), 0, s, chunks, n,
                       ncount, bkt, boff, out);
    return hipGetLastError();
}

hipError_t launch_level_counts(const uint8_t *dec, int64_t n, int32_t *lc, int32_t *cc,
                               hipStream_t s, const int32_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_counts, dim3(nblk(n)), dim3(kBS), 0, s, dec, n, nd, lc, cc);
    return hipGetLastError();
}

hipError_t launch_level_emit(const int4 *q, const uint8_t *dec, int64_t n, int level,
                             const int32_t *loff, const int32_t *coff, tms_leaf *leaves,
                             int64_t leaf_base, int4 *qn, hipStream_t s, const int32_t *nd,
                             const int64_t *lbd, int64_t lcap, int64_t qcap, unsigned *ovf,
                             int32_t *qpar) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_emit, dim3(nblk(n)), dim3(kBS), 0, s, q, dec, n, level, loff, coff,
                       leaves, leaf_base, qn, nd, lbd, lcap, qcap, ovf, qpar);
    return hipGetLastError();
}

hipError_t launch_level_histo(const uint8_t *dec, int64_t n, unsigned long long *h,
                              unsigned long long *part, hipStream_t s, const int32_t *nd) {
    if (n <= 0) return hipSuccess;
    const int nb = (int)std::min<int64_t>(kHistoBlocks, (n + kBS - 1) / kBS);
    hipLaunchKernelGGL(k_level_histo, dim3(nb), dim3(kBS), 0, s, dec, n, nd, part);
    hipLaunchKernelGGL(k_level_histo_final, dim3(1), dim3(64), 0, s, part, nb, h);
    return hipGetLastError();
}

hipError_t launch_fast_exp_debug(const double *x, int64_t n, double *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fast_exp_debug, dim3(nblk(n)), dim3(kBS), 0, s, x, n, y);
    return hipGetLastError();
}

hipError_t launch_leaf_seg_heads(const tms_leaf *leaves, int64_t n, int nconf, int64_t *src,
                                 hipStream_t s, const int64_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaf_seg_heads, dim3(nblk(n)), dim3(kBS), 0, s, leaves, n, nconf, nd, src);
    return hipGetLastError();
}

hipError_t launch_leaf_seg_move(const tms_leaf *leaves, int64_t n, int nconf, const int64_t *src,
                                const int64_t *dst, tms_leaf *out, hipStream_t s,
                                const int64_t *nd) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaf_seg_move, dim3(nblk(n)), dim3(kBS), 0, s, leaves, n, nconf, nd, src,
                       dst, out);
    return hipGetLastError();
}

hipError_t launch_bound_debug(const double *A, const double *band, int64_t n, double *out,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bound_debug, dim3(nblk(n)), dim3(kBS), 0, s, A, band, n, out);
    return hipGetLastError();
}

}  // namespace tms
