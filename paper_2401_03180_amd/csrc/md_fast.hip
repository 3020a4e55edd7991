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
    const double* invz64;          // 1/Z per type when the LJ radius scales with charge
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

// Exact membership and FP64 pair terms for d = p_a - p_b (minimum image); returns
// false when the pair is outside the cutoff.  f multiplies d for the force on a.
// hrow: hybrid-screening coefficient rows of the system and step (NULL: Debye).
// ia, ib: caller indices of the two atoms (for the LJ exclusions).
__device__ inline bool pair_fp64(const FastArgs& A, const GridSys& gs, double kap,
                                 const double* hrow, int ia, int ib, double xa, double ya,
                                 double za, int qa, int ta, double xb, double yb, double zb,
                                 int qb, int tb, double* dx, double* dy, double* dz, double* f,
                                 double* e)
{
    double r2;
    {
#pragma clang fp contract(off)
        double ex = xa - xb, ey = ya - yb, ez = za - zb;
        if (gs.periodic) {
            ex = ex - gs.L[0] * rint(ex * gs.invL[0]);
            ey = ey - gs.L[1] * rint(ey * gs.invL[1]);
            ez = ez - gs.L[2] * rint(ez * gs.invL[2]);
        }
        r2 = ex * ex + ey * ey;
        r2 = r2 + ez * ez;
        *dx = ex; *dy = ey; *dz = ez;
    }
    if (!(r2 < A.rc2)) return false;
    double c6 = A.c6[ta * A.T + tb], c12 = A.c12[ta * A.T + tb];
    if (A.excl_off) {
        for (int x = A.excl_off[ia]; x < A.excl_off[ia + 1]; ++x)
            if (A.excl[x] == ib) { c6 = 0.0; c12 = 0.0; break; }
    }
    if (A.invz64) {
#pragma clang fp contract(off)
        const double ca = 1.0 - (double)qa * A.invz64[ta];
        const double cb = 1.0 - (double)qb * A.invz64[tb];
        const double sc = 0.5 * (ca + cb);
        const double s6 = sc * sc * sc * sc * sc * sc;
        c6 = c6 * s6;
        c12 = c12 * s6 * s6;
    }
    if (hrow) {
        pair_terms_hybrid64(r2, kap, qa, qb, c6, c12, A.screen_lj != 0, hrow, A.hyb_q, f, e);
        return true;
    }
    const double r = sqrt(r2);
    const double rinv2 = 1.0 / r2;
    const double rinv6 = rinv2 * rinv2 * rinv2;
    const double s = exp(-kap * r);
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

__device__ inline double block_sum(double v, double* s)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += s[k];
    return t;
}

__device__ inline int64_t clamp_step_fast(const FastArgs& A)
{
    int64_t s = A.dsc->step;
    return s < 0 ? 0 : (s >= A.S1 ? A.S1 - 1 : s);
}

// Work-group fi of the fast-atom pass: all pairs of fast atom fi.
template <bool ENERGY, bool EMIT>
__device__ void fast_self(const FastArgs& A, int fi)
{
    __shared__ double s_red[kFastBlock / 64];
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
    // slot ranges of every (column, z range) pair within reach, computed by one
    // thread each, then swept by the whole work-group as one flattened list
    __shared__ int64_t s_r0[kFastRanges];
    __shared__ int s_len[kFastRanges], s_pre[kFastRanges + 1];
    const int ncy = cy1 - cy0 + 1;
    const int npairs = (cx1 - cx0 + 1) * ncy * nzr;
    for (int p0 = 0; p0 < npairs; p0 += kFastRanges) {
        const int np = min(kFastRanges, npairs - p0);
        __syncthreads();
        for (int t = threadIdx.x; t < np; t += blockDim.x) {
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
            s_r0[t] = s0;
            s_len[t] = (int)max((int64_t)0, s1 - s0);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int t = 0; t < np; ++t) { s_pre[t] = acc; acc += s_len[t]; }
            s_pre[np] = acc;
        }
        __syncthreads();
        const int total = s_pre[np];
        for (int k = threadIdx.x; k < total; k += blockDim.x) {
            int lo = 0, hi = np - 1;                // last range with s_pre <= k
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= k) lo = mid; else hi = mid - 1;
            }
            const int64_t s = s_r0[lo] + (k - s_pre[lo]);
            const double xa = A.xs[s];
            if (xa != xa) continue;                // fast atom or padding
            double dx, dy, dz, fp, e;
            if (pair_fp64(A, gs, kap, hrow, f, A.perm[s], xf, yf, zf, qf, tf, xa, A.xs[cs + s],
                          A.xs[2 * cs + s],
                          A.qs[s], A.ts[s], &dx, &dy, &dz, &fp, &e)) {
                Fx += fp * dx; Fy += fp * dy; Fz += fp * dz;
                if (ENERGY) E += e;
                if (EMIT) emit_one(A, f, A.perm[s]);
            }
        }
    }
    // other fast atoms of the same system, by their current positions
    const int64_t a0 = A.sys_off[b], a1 = A.sys_off[b + 1];
    for (int k = threadIdx.x; k < nf; k += blockDim.x) {
        const int g = A.fast_list[k];
        if (g == f || g < a0 || g >= a1) continue;
        double dx, dy, dz, fp, e;
        if (pair_fp64(A, gs, kap, hrow, f, g, xf, yf, zf, qf, tf, A.x[g], A.y[g], A.z[g], A.q[g],
                      A.atype[g], &dx, &dy, &dz, &fp, &e)) {
            Fx += fp * dx; Fy += fp * dy; Fz += fp * dz;
            if (ENERGY) E += 0.5 * e;
            if (EMIT && f < g) emit_one(A, f, g);
        }
    }
    Fx = block_sum(Fx, s_red);
    Fy = block_sum(Fy, s_red);
    Fz = block_sum(Fz, s_red);
    if (ENERGY) E = block_sum(E, s_red);
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

constexpr int kFastLocal = 1024;     // fast atoms near one column held in LDS

// Column `col` of the fast-atom pass: forces of nearby fast atoms on its other atoms.
__device__ void fast_nbr(const FastArgs& A, int col)
{
    __shared__ int s_loc[kFastLocal];
    __shared__ int s_cnt[kFastBlock / 64];
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
    // fast atoms of this system within reach of the column, in fast-list order
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int total = 0;
    for (int base = 0; base < nf; base += blockDim.x) {
        const int k = base + threadIdx.x;
        bool take = false;
        if (k < nf) {
            const int g = A.fast_list[k];
            if (g >= a0 && g < a1) {
                double px = A.x[g], py = A.y[g];
                if (gs.periodic) {
                    px -= gs.L[0] * floor(px * gs.invL[0]);
                    py -= gs.L[1] * floor(py * gs.invL[1]);
                }
                const double gx = axis_gap(px, lo[0], hi[0], gs.periodic, gs.L[0]);
                const double gy = axis_gap(py, lo[1], hi[1], gs.periodic, gs.L[1]);
                take = gx * gx + gy * gy < R2;
            }
        }
        const unsigned long long bal = __ballot(take);
        if (lane == 0) s_cnt[w] = __popcll(bal);
        __syncthreads();
        int off = total;
        for (int v = 0; v < w; ++v) off += s_cnt[v];
        int add = 0;
        for (int v = 0; v < (int)(blockDim.x >> 6); ++v) add += s_cnt[v];
        if (take) {
            const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
            if (pos < kFastLocal) s_loc[pos] = A.fast_list[k];
        }
        total += add;
        __syncthreads();
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
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const double xa = A.xs[s];
        if (xa != xa) continue;                    // fast atom or padding
        const double ya = A.xs[cs + s], za = A.xs[2 * cs + s];
        const int qa = A.qs[s], ta = A.ts[s];
        const int ia = A.perm[s];
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        bool any = false;
        for (int k = 0; k < total; ++k) {
            const int g = s_loc[k];
            double dx, dy, dz, fp, e;
            if (pair_fp64(A, gs, kap, hrow, ia, g, xa, ya, za, qa, ta, A.x[g], A.y[g], A.z[g],
                          A.q[g],
                          A.atype[g], &dx, &dy, &dz, &fp, &e)) {
                Fx += fp * dx; Fy += fp * dy; Fz += fp * dz;
                any = true;
            }
        }
        if (any) {
            const int a = A.perm[s];
            A.fx[a] += Fx;
            A.fy[a] += Fy;
            A.fz[a] += Fz;
        }
    }
}

// One launch: work-groups [0, fast_cap) take one fast atom each (its own pairs),
// the following ones one column each (the fast atoms' forces on the column's other
// atoms); the two halves write disjoint atoms, so they need no ordering.
template <bool ENERGY, bool EMIT>
__global__ void __launch_bounds__(kFastBlock) k_fast(FastArgs A, int fast_cap)
{
    if ((int)blockIdx.x < fast_cap) fast_self<ENERGY, EMIT>(A, blockIdx.x);
    else fast_nbr(A, blockIdx.x - fast_cap);
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
    A.invz64 = c->ff_qlj ? c->d_invz64 : nullptr;
    A.excl_off = c->ff_excl ? c->d_excl_off : nullptr; A.excl = c->d_excl;
    A.rc2 = c->cfg.rc * c->cfg.rc;
    A.reach = c->cfg.rc + 0.5 * c->cfg.skin;
    A.screen_lj = c->cfg.screen_lj;
    A.hyb64 = c->hybrid ? c->d_hyb64 : nullptr;
    A.hyb_q = c->hyb_q;
    A.fast_flag = c->d_fast_flag; A.fast_list = c->d_fast_list; A.fast_e = c->d_fast_e;
    A.dsc = c->dsc; A.fx = fx; A.fy = fy; A.fz = fz; A.emit = emit; A.emit_max = emit_max;
    const int fc = std::max(c->fast_cap, 1);
    const dim3 gs((unsigned)(fc + std::max<int64_t>(c->cap_cols, 1))), bs(kFastBlock);
    if (emit) {
        if (energy) hipLaunchKernelGGL((k_fast<true, true>), gs, bs, 0, st, A, fc);
        else hipLaunchKernelGGL((k_fast<false, true>), gs, bs, 0, st, A, fc);
    } else {
        if (energy) hipLaunchKernelGGL((k_fast<true, false>), gs, bs, 0, st, A, fc);
        else hipLaunchKernelGGL((k_fast<false, false>), gs, bs, 0, st, A, fc);
    }
}

}  // namespace md
