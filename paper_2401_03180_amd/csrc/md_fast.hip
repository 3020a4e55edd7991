// md_fast.hip -- pairs of "fast" atoms between neighbour builds (arXiv 2401.03180,
// section II.A Eq. 2 and Eq. 8, section II.B cutoff; same pair predicate and
// potential as the list kernels).
//
// The per-atom lists hold every partner within rc + skin at the last build, so a pair
// whose two atoms have each moved at most skin/2 since then is in them.  An atom that
// has moved farther ("fast": flagged by the first velocity-Verlet half step) is staged
// like a padding slot by the list kernels, and every pair it takes part in is
// evaluated here, in FP64 with the exact predicate:
//   * fast_self: one work-group per fast atom f scans, in the columns within
//     rc + skin/2 of f, the z bins within that distance (every other atom sits in
//     the bin of its build position, which is within skin/2 of where it is now),
//     reading the slot-ordered positions (NaN for fast atoms and padding), and then
//     every other fast atom; it writes F_f and the energy of f's pairs (pairs with
//     another fast atom count one half from each side);
//   * fast_nbr: one work-group per column adds, to each non-fast atom of the
//     column, the forces of the fast atoms within reach, in fast-list order.
// No atomics on forces: every result is written by one thread in a fixed order.
#include "md_device.h"
#include "md_internal.h"
#include "md_launch.h"

namespace md {

constexpr int kFastBlock = 256;
constexpr int kFastRanges = 256;     // (column, z range) pairs per sweep of fast_self
constexpr int kFastU = 4;            // items per thread whose loads are issued together

struct FastArgs {
    const double *x, *y, *z;       // caller positions (current)
    const int8_t* q;               // caller charges (current)
    const uint8_t* atype;          // types in caller order (build time)
    const int32_t* sys_of_atom;
    const int64_t* sys_off;
    const GridSys* grid;
    int B;
    const int64_t* col_pre;
    const int32_t* bin_start;
    const int32_t* perm;
    const double* xs;              // slot-order positions (SoA, stride cap_slots)
    const int8_t* qs;
    const uint8_t* ts;
    int64_t cap_slots;
    const double* kappa;
    int64_t S1;
    const double *c6, *c12;
    int T;
    double rc2, reach;             // rc^2; column search radius rc + skin/2
    int screen_lj;
    const double* hyb64;           // hybrid screening rows (NULL: Debye)
    int hyb_q;
    const double* qlj;             // charge-scaled LJ radii (Eq. 11), kQljLen, or NULL
    const int32_t* excl_off;       // LJ exclusions per caller atom (NULL: none)
    const int32_t* excl;
    const uint8_t* fast_flag;
    const int32_t* fast_list;
    double* fast_e;
    DevScalars* dsc;
    double *fx, *fy, *fz;
    int2* emit;
    int64_t emit_max;
};

// d = p_a - p_b (minimum image) and its squared length, in FP64 in a fixed order:
// the exact membership test of the pair.
__device__ inline double pair_r2_fp64(const GridSys& gs, double xa, double ya, double za,
                                      double xb, double yb, double zb, double* dx, double* dy,
                                      double* dz)
{
#pragma clang fp contract(off)
    double ex = xa - xb, ey = ya - yb, ez = za - zb;
    if (gs.periodic) {
        ex = ex - gs.L[0] * rint(ex * gs.invL[0]);
        ey = ey - gs.L[1] * rint(ey * gs.invL[1]);
        ez = ez - gs.L[2] * rint(ez * gs.invL[2]);
    }
    double r2 = ex * ex + ey * ey;
    r2 = r2 + ez * ez;
    *dx = ex; *dy = ey; *dz = ez;
    return r2;
}

// Exact membership and FP64 pair terms for d = p_a - p_b (minimum image); returns
// false when the pair is outside the cutoff.  f multiplies d for the force on a.
// hrow: hybrid-screening coefficient rows of the system and step (NULL: Debye).
// ia, ib: caller indices of the two atoms (for the LJ exclusions).
// FULL: hybrid screening, charge-scaled LJ or LJ exclusions may be bound (the plain
// instantiation leaves their code, and its registers, out).
template <bool FULL>
__device__ inline bool pair_fp64(const FastArgs& A, const GridSys& gs, double kap,
                                 const double* hrow, int ia, int ib, double xa, double ya,
                                 double za, int qa, int ta, double xb, double yb, double zb,
                                 int qb, int tb, double* dx, double* dy, double* dz, double* f,
                                 double* e)
{
    const double r2 = pair_r2_fp64(gs, xa, ya, za, xb, yb, zb, dx, dy, dz);
    if (!(r2 < A.rc2)) return false;
    double c6 = A.c6[ta * A.T + tb], c12 = A.c12[ta * A.T + tb];
    if (FULL && A.excl_off) {
        for (int x = A.excl_off[ia]; x < A.excl_off[ia + 1]; ++x)
            if (A.excl[x] == ib) { c6 = 0.0; c12 = 0.0; break; }
    }
    if (FULL && A.qlj) qlj_scale64(A.qlj, ta, tb, qa, qb, &c6, &c12);
    if (FULL && hrow) {
        pair_terms_hybrid64(r2, kap, qa, qb, c6, c12, A.screen_lj != 0, hrow, A.hyb_q, f, e);
        return true;
    }
    const double r = sqrt(r2);
    const double rinv2 = 1.0 / r2;
    const double rinv6 = rinv2 * rinv2 * rinv2;
    const double s = exp_nonpos64(-kap * r);
    const double uc = kKe * (double)qa * (double)qb / r;
    const double l12 = c12 * rinv6 * rinv6, l6 = c6 * rinv6;
    if (A.screen_lj) {
        const double uu = uc + (l12 - l6);
        *f = ((uc + 12.0 * l12 - 6.0 * l6) + uu * (kap * r)) * s * rinv2;
        *e = uu * s;
    } else {
        *f = (uc + uc * (kap * r)) * s * rinv2 + (12.0 * l12 - 6.0 * l6) * rinv2;
        *e = uc * s + (l12 - l6);
    }
    return true;
}

__device__ inline void emit_one(const FastArgs& A, int a, int b)
{
    const unsigned long long p = atomicAdd(&A.dsc->pair_count, 1ull);
    if ((int64_t)p < A.emit_max) A.emit[p] = make_int2(min(a, b), max(a, b));
}

// The four sums over the work-group in one pass (each in a fixed order); the
// results are valid in every thread.
__device__ inline void block_sum4(double& a, double& b, double& c, double& d,
                                  double (*s)[kFastBlock / 64])
{
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
        c += __shfl_xor(c, off, 64);
        d += __shfl_xor(d, off, 64);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        s[0][w] = a; s[1][w] = b; s[2][w] = c; s[3][w] = d;
    }
    __syncthreads();
    a = b = c = d = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
        a += s[0][k]; b += s[1][k]; c += s[2][k]; d += s[3][k];
    }
}

__device__ inline int64_t clamp_step_fast(const FastArgs& A)
{
    int64_t s = A.dsc->step;
    return s < 0 ? 0 : (s >= A.S1 ? A.S1 - 1 : s);
}

// Exclusive prefix of one int per thread over the work-group, in thread order; the
// block sum goes to *total.  s holds one int per wave.  Starts with a barrier, so
// LDS read before the call may be overwritten after it.
__device__ inline int block_excl_scan(int v, int* s, int* total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    __syncthreads();
    if (lane == 63) s[wv] = inc;
    __syncthreads();
    int off = inc - v, t = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < wv) off += s[k];
        t += s[k];
    }
    *total = t;
    return off;
}

// Work-group fi of the fast-atom pass: all pairs of fast atom fi.  Each thread takes
// kFastU items per trip and issues their loads together (the pass is latency-bound);
// its items keep the order k, k + blockDim, ... of a plain strided loop.
template <bool ENERGY, bool EMIT, bool FULL>
__device__ void fast_self(const FastArgs& A, int fi)
{
    static_assert(kFastRanges == kFastBlock, "one (column, z range) pair per thread");
    __shared__ double s_red4[4][kFastBlock / 64];
    __shared__ int s_ws[kFastBlock / 64];
    __shared__ int64_t s_r0[kFastRanges];
    __shared__ int s_pre[kFastRanges + 1];
    const int nf = A.dsc->n_fast;
    if (fi >= nf) return;
    const int f = A.fast_list[fi];
    const int b = A.sys_of_atom[f];
    const GridSys gs = A.grid[b];
    const int64_t step = clamp_step_fast(A);
    const double kap = A.kappa[(int64_t)b * A.S1 + step];
    const double* hrow = A.hyb64 ? A.hyb64 + ((int64_t)b * A.S1 + step) * A.hyb_q * 4 : nullptr;
    const double xf = A.x[f], yf = A.y[f], zf = A.z[f];
    const int qf = A.q[f], tf = A.atype[f];
    double Fx = 0.0, Fy = 0.0, Fz = 0.0, E = 0.0;
    int cx0, cx1, cy0, cy1;
    col_range(gs, 0, xf, A.reach, &cx0, &cx1);
    col_range(gs, 1, yf, A.reach, &cy0, &cy1);
    int zr0[2], zr1[2];
    const int nzr = zbin_ranges(gs, zf, A.reach, zr0, zr1);
    const int64_t cs = A.cap_slots;
    const int64_t n_slots = A.dsc->n_slots;
    // slot ranges of every (column, z range) pair within reach, one per thread, then
    // swept by the whole work-group as one flattened list
    const int ncy = cy1 - cy0 + 1;
    const int npairs = max(0, (cx1 - cx0 + 1) * ncy * nzr);
    // the other fast atoms of the same system (by their current positions) are items of
    // the last sweep after its slots, so their loads overlap the slots'
    const int64_t a0 = A.sys_off[b], a1 = A.sys_off[b + 1];
    for (int p0 = 0; p0 == 0 || p0 < npairs; p0 += kFastRanges) {
        const int np = max(0, min(kFastRanges, npairs - p0));
        const int nextra = p0 + kFastRanges >= npairs ? nf : 0;
        const int t = threadIdx.x;
        int64_t r0 = 0;
        int len = 0;
        if (t < np) {
            const int p = p0 + t;
            const int r = p % nzr, cc = p / nzr;
            const int cx = cx0 + cc / ncy, cy = cy0 + cc % ncy;
            const int wx = gs.periodic ? ((cx % gs.n[0]) + gs.n[0]) % gs.n[0] : cx;
            const int wy = gs.periodic ? ((cy % gs.n[1]) + gs.n[1]) % gs.n[1] : cy;
            const int col = gs.col_off + wx * gs.n[1] + wy;
            const int64_t slot0 = (int64_t)col_first_cluster(A.col_pre, col) * kCluster;
            const int bin0 = gs.bin_off + (col - gs.col_off) * gs.n[2];
            const int a_col = A.bin_start[bin0];
            // the column's atoms are in bin order from slot0 on
            const int64_t s0 = slot0 + (A.bin_start[bin0 + zr0[r]] - a_col);
            const int64_t s1 = min(slot0 + (A.bin_start[bin0 + zr1[r] + 1] - a_col), n_slots);
            r0 = s0;
            len = (int)max((int64_t)0, s1 - s0);
        }
        int total;
        const int off = block_excl_scan(len, s_ws, &total);   // the previous sweep is done
        if (t < np) {
            s_r0[t] = r0;
            s_pre[t] = off;
        }
        __syncthreads();
        const int nitems = total + nextra;
        for (int k0 = t; k0 < nitems; k0 += kFastU * kFastBlock) {
            int64_t sl[kFastU];
            int gg[kFastU];
#pragma unroll
            for (int u = 0; u < kFastU; ++u) {
                const int k = k0 + u * kFastBlock;
                sl[u] = -1;
                gg[u] = -1;
                if (k < total) {
                    int lo = 0, hi = np - 1;            // last range with s_pre <= k
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= k) lo = mid; else hi = mid - 1;
                    }
                    sl[u] = s_r0[lo] + (k - s_pre[lo]);
                } else if (k < nitems) {
                    gg[u] = A.fast_list[k - total];
                }
            }
            double px[kFastU], py[kFastU], pz[kFastU];
            int pq[kFastU], pt[kFastU], pa[kFastU];
#pragma unroll
            for (int u = 0; u < kFastU; ++u) {
                const int64_t s = sl[u];
                const int g = gg[u];
                px[u] = NAN; py[u] = 0.0; pz[u] = 0.0; pq[u] = 0; pt[u] = 0; pa[u] = -1;
                if (s >= 0) {
                    px[u] = A.xs[s];
                    py[u] = A.xs[cs + s];
                    pz[u] = A.xs[2 * cs + s];
                    pq[u] = A.qs[s];
                    pt[u] = A.ts[s];
                    pa[u] = A.perm[s];
                } else if (g >= 0 && g != f && g >= a0 && g < a1) {
                    px[u] = A.x[g]; py[u] = A.y[g]; pz[u] = A.z[g];
                    pq[u] = A.q[g]; pt[u] = A.atype[g];
                    pa[u] = g;
                }
            }
#pragma unroll
            for (int u = 0; u < kFastU; ++u) {
                // a fast atom or padding slot (NaN), no item, or a fast atom that is f
                // itself or in another system
                if (px[u] != px[u] || pa[u] < 0) continue;
                const bool other_fast = gg[u] >= 0;
                double dx, dy, dz, fp, e;
                if (pair_fp64<FULL>(A, gs, kap, hrow, f, pa[u], xf, yf, zf, qf, tf, px[u], py[u],
                                    pz[u], pq[u], pt[u], &dx, &dy, &dz, &fp, &e)) {
                    Fx += fp * dx; Fy += fp * dy; Fz += fp * dz;
                    // a pair of two fast atoms counts one half from each side
                    if (ENERGY) E += other_fast ? 0.5 * e : e;
                    if (EMIT && (!other_fast || f < pa[u])) emit_one(A, f, pa[u]);
                }
            }
        }
    }
    block_sum4(Fx, Fy, Fz, E, s_red4);
    if (threadIdx.x == 0) {
        A.fx[f] = Fx;
        A.fy[f] = Fy;
        A.fz[f] = Fz;
        if (ENERGY) A.fast_e[fi] = E;
    }
}

// System of a global column: the last system whose first column is <= c.
__device__ inline int sys_of_col(const GridSys* grid, int B, int c)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (grid[mid].col_off <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Distance along z from coordinate z to the interval [lo, hi] (all wrapped into
// [0, L) for a periodic system, where the nearer image counts); +inf for an empty
// interval.
__device__ inline double wave_z_gap(double z, double lo, double hi, const GridSys& gs)
{
    if (!(lo <= hi)) return INFINITY;
    const double g0 = fmax(0.0, fmax(lo - z, z - hi));
    if (!gs.periodic) return g0;
    const double g1 = fmax(0.0, fmax(lo - (z + gs.L[2]), (z + gs.L[2]) - hi));
    const double g2 = fmax(0.0, fmax(lo - (z - gs.L[2]), (z - gs.L[2]) - hi));
    return fmin(g0, fmin(g1, g2));
}

constexpr int kFastLocal = 1024;     // fast atoms near one column (indices in LDS)
constexpr int kFastChunk = kFastBlock;   // their positions staged in LDS per chunk

// Column `col` of the fast-atom pass: forces of nearby fast atoms on its other atoms.
template <bool FULL>
__device__ void fast_nbr(const FastArgs& A, int col)
{
    __shared__ int s_loc[kFastLocal];
    __shared__ int s_ws[kFastBlock / 64];
    __shared__ double s_px[kFastChunk], s_py[kFastChunk], s_pz[kFastChunk];
    __shared__ int s_pg[kFastChunk], s_pq[kFastChunk], s_pt[kFastChunk];
    __shared__ double s_pzw[kFastChunk];
    const int nf = A.dsc->n_fast;
    if (nf == 0 || col >= A.dsc->n_cols) return;
    const int b = sys_of_col(A.grid, A.B, col);
    const GridSys gs = A.grid[b];
    const int lc = col - gs.col_off;
    const int cx = lc / gs.n[1], cy = lc % gs.n[1];
    // column rectangle (edge columns of a vacuum grid extend outward: binning clamps)
    double lo[2], hi[2];
    const int cc[2] = {cx, cy};
    for (int d = 0; d < 2; ++d) {
        const double o = gs.periodic ? 0.0 : gs.origin[d];
        lo[d] = o + cc[d] * gs.w[d];
        hi[d] = o + (cc[d] + 1) * gs.w[d];
        if (!gs.periodic && cc[d] == 0) lo[d] = -INFINITY;
        if (!gs.periodic && cc[d] == gs.n[d] - 1) hi[d] = INFINITY;
    }
    const int64_t a0 = A.sys_off[b], a1 = A.sys_off[b + 1];
    const double R2 = A.reach * A.reach;
    // fast atoms of this system within reach of the column, in fast-list order: each
    // thread tests kFastU consecutive list entries (loads issued together)
    int total = 0;
    for (int base = 0; base < nf; base += kFastU * kFastBlock) {
        const int kb = base + threadIdx.x * kFastU;
        int gg[kFastU];
#pragma unroll
        for (int u = 0; u < kFastU; ++u) gg[u] = kb + u < nf ? A.fast_list[kb + u] : -1;
        double px[kFastU], py[kFastU];
#pragma unroll
        for (int u = 0; u < kFastU; ++u) {
            px[u] = 0.0; py[u] = 0.0;
            if (gg[u] >= a0 && gg[u] < a1) { px[u] = A.x[gg[u]]; py[u] = A.y[gg[u]]; }
        }
        unsigned takes = 0u;
        int c = 0;
#pragma unroll
        for (int u = 0; u < kFastU; ++u) {
            if (!(gg[u] >= a0 && gg[u] < a1)) continue;
            double qx = px[u], qy = py[u];
            if (gs.periodic) {
                qx -= gs.L[0] * floor(qx * gs.invL[0]);
                qy -= gs.L[1] * floor(qy * gs.invL[1]);
            }
            const double gx = axis_gap(qx, lo[0], hi[0], gs.periodic, gs.L[0]);
            const double gy = axis_gap(qy, lo[1], hi[1], gs.periodic, gs.L[1]);
            if (gx * gx + gy * gy < R2) { takes |= 1u << u; ++c; }
        }
        int add;
        int pos = total + block_excl_scan(c, s_ws, &add);
#pragma unroll
        for (int u = 0; u < kFastU; ++u) {
            if (((takes >> u) & 1u) == 0u) continue;
            if (pos < kFastLocal) s_loc[pos] = gg[u];
            ++pos;
        }
        total += add;
    }
    if (total == 0) return;
    if (total > kFastLocal) {
        if (threadIdx.x == 0) set_flag(A.dsc, MD_FLAG_LIST_OVERFLOW);
        total = kFastLocal;
    }
    const int64_t step = clamp_step_fast(A);
    const double kap = A.kappa[(int64_t)b * A.S1 + step];
    const double* hrow = A.hyb64 ? A.hyb64 + ((int64_t)b * A.S1 + step) * A.hyb_q * 4 : nullptr;
    const int64_t s0 = (int64_t)col_first_cluster(A.col_pre, col) * kCluster;
    const int64_t s1 = min((int64_t)col_first_cluster(A.col_pre, col + 1) * kCluster,
                           (int64_t)A.dsc->n_slots);
    const int64_t cs = A.cap_slots;
    // a wave skips a fast atom only when its z gap exceeds rc by a margin far above
    // the rounding of the wrapped coordinates
    const double zskip = sqrt(A.rc2) * (1.0 + 1e-9) + 1e-9;
    // the nearby fast atoms c0 .. c0 + nc - 1 into LDS (positions, wrapped z, charge,
    // type); when they fit one chunk (the common case) they are staged once for all
    // of the column's slot passes
    auto stage = [&](int c0, int nc) {
        if ((int)threadIdx.x < nc) {
            const int g = s_loc[c0 + threadIdx.x];
            s_pg[threadIdx.x] = g;
            s_px[threadIdx.x] = A.x[g];
            s_py[threadIdx.x] = A.y[g];
            s_pz[threadIdx.x] = A.z[g];
            s_pq[threadIdx.x] = A.q[g];
            s_pt[threadIdx.x] = A.atype[g];
            const double zg = s_pz[threadIdx.x];
            s_pzw[threadIdx.x] = gs.periodic ? zg - gs.L[2] * floor(zg * gs.invL[2]) : zg;
        }
    };
    const bool one_chunk = total <= kFastChunk;          // uniform
    if (one_chunk) {
        __syncthreads();                                 // s_loc written
        stage(0, total);
        __syncthreads();
    }
    for (int64_t sb = s0; sb < s1; sb += kFastBlock) {
        const int64_t s = sb + threadIdx.x;
        double xa = NAN, ya = 0.0, za = 0.0;
        int qa = 0, ta = 0, ia = -1;
        if (s < s1) {
            xa = A.xs[s]; ya = A.xs[cs + s]; za = A.xs[2 * cs + s];
            qa = A.qs[s]; ta = A.ts[s]; ia = A.perm[s];
        }
        const bool live = xa == xa;                    // not fast, padding or past the end
        // z extent of the wave's live atoms (a column's slots are in z-bin order, so
        // a wave covers a short stretch of it): fast atoms farther than rc from it in
        // z are skipped by the whole wave
        double zl = INFINITY, zh = -INFINITY;
        if (live) {
            const double zw = gs.periodic ? za - gs.L[2] * floor(za * gs.invL[2]) : za;
            zl = zw;
            zh = zw;
        }
        for (int off = 32; off > 0; off >>= 1) {
            zl = fmin(zl, __shfl_xor(zl, off, 64));
            zh = fmax(zh, __shfl_xor(zh, off, 64));
        }
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        bool any = false;
        for (int c0 = 0; c0 < total; c0 += kFastChunk) {
            const int nc = min(kFastChunk, total - c0);
            if (!one_chunk) {
                __syncthreads();                       // the previous chunk is consumed
                stage(c0, nc);
                __syncthreads();
            }
            if (!live) continue;
            // membership first (cheap), then the pair terms of this lane's partners
            // only, in ascending k: a wave no longer runs the terms for every k that
            // one of its lanes needs
            for (int k0 = 0; k0 < nc; k0 += 64) {
                const int kn = min(64, nc - k0);
                unsigned long long hit = 0ull;
                for (int kk = 0; kk < kn; ++kk) {
                    const int k = k0 + kk;
                    if (wave_z_gap(s_pzw[k], zl, zh, gs) > zskip) continue;    // wave-uniform
                    double dx, dy, dz;
                    const double r2 = pair_r2_fp64(gs, xa, ya, za, s_px[k], s_py[k], s_pz[k], &dx,
                                                   &dy, &dz);
                    if (r2 < A.rc2) hit |= 1ull << kk;
                }
                while (hit != 0ull) {
                    const int k = k0 + __builtin_ctzll(hit);
                    hit &= hit - 1ull;
                    double dx, dy, dz, fp, e;
                    if (pair_fp64<FULL>(A, gs, kap, hrow, ia, s_pg[k], xa, ya, za, qa, ta, s_px[k],
                                        s_py[k], s_pz[k], s_pq[k], s_pt[k], &dx, &dy, &dz, &fp,
                                        &e)) {
                        Fx += fp * dx; Fy += fp * dy; Fz += fp * dz;
                        any = true;
                    }
                }
            }
        }
        if (any) {
            A.fx[ia] += Fx;
            A.fy[ia] += Fy;
            A.fz[ia] += Fz;
        }
    }
}

// The pass as one launch: work-groups [0, fast_cap) take one fast atom each (its own
// pairs), the following ones one column each (the fast atoms' forces on the column's
// other atoms); the two halves write disjoint atoms, so they need no ordering.
template <bool ENERGY, bool EMIT, bool FULL>
__global__ void __launch_bounds__(kFastBlock) k_fast(FastArgs A, int fast_cap)
{
    if ((int)blockIdx.x < fast_cap) fast_self<ENERGY, EMIT, FULL>(A, blockIdx.x);
    else fast_nbr<FULL>(A, blockIdx.x - fast_cap);
}

// The same pass as two launches, one kernel per half: each half alone fits 128 VGPRs
// (4 waves per SIMD), while the one kernel holding both takes 171 (2 waves), which
// halves the work-groups in flight of this latency-bound pass.  The second launch costs
// a kernel boundary, so it pays only on a large grid (see launch_fast).
template <bool ENERGY, bool EMIT, bool FULL>
__global__ void __launch_bounds__(kFastBlock) k_fast_self(FastArgs A)
{
    fast_self<ENERGY, EMIT, FULL>(A, blockIdx.x);
}

template <bool FULL>
__global__ void __launch_bounds__(kFastBlock) k_fast_nbr(FastArgs A)
{
    fast_nbr<FULL>(A, blockIdx.x);
}

void launch_fast(Ctx* c, const double* x, const double* y, const double* z, const int8_t* q,
                 double* fx, double* fy, double* fz, bool energy, int2* emit, int64_t emit_max,
                 hipStream_t st)
{
    FastArgs A;
    A.x = x; A.y = y; A.z = z; A.q = q; A.atype = c->d_atype;
    A.sys_of_atom = c->d_sys_of_atom; A.sys_off = c->d_sys_off; A.grid = c->d_grid; A.B = c->B;
    A.col_pre = c->d_col_pre; A.bin_start = c->d_bin_start; A.perm = c->d_perm;
    A.xs = c->d_xs; A.qs = c->d_qs; A.ts = c->d_ts; A.cap_slots = c->cap_slots;
    A.kappa = c->d_kappa; A.S1 = c->n_steps + 1;
    A.c6 = c->d_c6; A.c12 = c->d_c12; A.T = c->T_lj;
    A.qlj = c->ff_qlj ? c->d_qlj : nullptr;
    A.excl_off = c->ff_excl ? c->d_excl_off : nullptr; A.excl = c->d_excl;
    A.rc2 = c->cfg.rc * c->cfg.rc;
    A.reach = c->cfg.rc + 0.5 * c->cfg.skin;
    A.screen_lj = c->cfg.screen_lj;
    A.hyb64 = c->hybrid ? c->d_hyb64 : nullptr;
    A.hyb_q = c->hyb_q;
    A.fast_flag = c->d_fast_flag; A.fast_list = c->d_fast_list; A.fast_e = c->d_fast_e;
    A.dsc = c->dsc; A.fx = fx; A.fy = fy; A.fz = fz; A.emit = emit; A.emit_max = emit_max;
    const int fc = std::max(c->fast_cap, 1);
    const int64_t ncol = std::max<int64_t>(c->cap_cols, 1);
    const dim3 bs(kFastBlock);
    const bool full = A.hyb64 || A.qlj || A.excl_off;
    // one launch while the whole grid fits about eight rounds of the one-kernel form (two
    // work-groups per CU); beyond that the two-kernel form, whose halves run four per CU.
    // Measured per step: 98,304-atom box (786 work-groups) one launch 4 % faster; protein
    // crystal (2,624) one launch 0.4 % faster; 4.19 M-atom box (8,598) two launches 0.5 %
    // faster; 256 methane clusters (~216 k, most exiting at once) two launches 1.1 % faster
    if ((int64_t)fc + ncol <= 16 * (int64_t)c->n_cu) {
        const dim3 gs((unsigned)(fc + ncol));
        if (full) {
            if (emit) {
                if (energy) hipLaunchKernelGGL((k_fast<true, true, true>), gs, bs, 0, st, A, fc);
                else hipLaunchKernelGGL((k_fast<false, true, true>), gs, bs, 0, st, A, fc);
            } else {
                if (energy) hipLaunchKernelGGL((k_fast<true, false, true>), gs, bs, 0, st, A, fc);
                else hipLaunchKernelGGL((k_fast<false, false, true>), gs, bs, 0, st, A, fc);
            }
        } else if (emit) {
            if (energy) hipLaunchKernelGGL((k_fast<true, true, false>), gs, bs, 0, st, A, fc);
            else hipLaunchKernelGGL((k_fast<false, true, false>), gs, bs, 0, st, A, fc);
        } else {
            if (energy) hipLaunchKernelGGL((k_fast<true, false, false>), gs, bs, 0, st, A, fc);
            else hipLaunchKernelGGL((k_fast<false, false, false>), gs, bs, 0, st, A, fc);
        }
        return;
    }
    const dim3 gf((unsigned)fc), gc((unsigned)ncol);
    if (full) {
        if (emit) {
            if (energy) hipLaunchKernelGGL((k_fast_self<true, true, true>), gf, bs, 0, st, A);
            else hipLaunchKernelGGL((k_fast_self<false, true, true>), gf, bs, 0, st, A);
        } else {
            if (energy) hipLaunchKernelGGL((k_fast_self<true, false, true>), gf, bs, 0, st, A);
            else hipLaunchKernelGGL((k_fast_self<false, false, true>), gf, bs, 0, st, A);
        }
        hipLaunchKernelGGL((k_fast_nbr<true>), gc, bs, 0, st, A);
    } else {
        if (emit) {
            if (energy) hipLaunchKernelGGL((k_fast_self<true, true, false>), gf, bs, 0, st, A);
            else hipLaunchKernelGGL((k_fast_self<false, true, false>), gf, bs, 0, st, A);
        } else {
            if (energy) hipLaunchKernelGGL((k_fast_self<true, false, false>), gf, bs, 0, st, A);
            else hipLaunchKernelGGL((k_fast_self<false, false, false>), gf, bs, 0, st, A);
        }
        hipLaunchKernelGGL((k_fast_nbr<false>), gc, bs, 0, st, A);
    }
}

}  // namespace md
