// md_build.hip -- neighbour search.
//
// The screening-reduced cutoff (arXiv 2401.03180, section II.B) bounds the pairs
// that are ever evaluated.  A build turns caller-ordered positions into
//   1. a per-system grid of x-y columns with fine z bins; a counting sort puts
//      the atoms of every column in z order (ties by atom index, so the order is
//      deterministic);
//   2. clusters of 8 consecutive atoms of a column ("slots"; the last cluster of a
//      column is padded) with FP64 bounding boxes;
//   3. groups of up to G consecutive clusters of a column; for each group the
//      candidate table of (cluster, periodic shift) entries whose bounding box
//      lies within rc + skin of the group's box;
//   4. for every atom a compacted list of 16-bit codes naming the staged
//      candidate atoms within rc + skin (entry * 8 + lane | type << 13).
// The lists stay valid while no atom moves more than skin/2 from its build
// position.
#include "md_internal.h"
#include "md_launch.h"

namespace md {


__device__ inline int find_sys_by_col(const GridSys* grid, int B, int c)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (grid[mid].col_off <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// largest k in [0, n] with arr[k] <= v (arr non-decreasing, arr[0] <= v)
__device__ inline int upper_index(const int32_t* arr, int n, int v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (arr[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// End of a candidate-table build: the per-atom lists are now pending (the next
// force evaluation rebuilds them), the displacement reference is the new one.
__global__ void k_build_done(DevScalars* d, const int32_t* gate)
{
    if (gate && *gate == 0) return;
    d->need_rebuild = 0;
    d->lists_pending = 1;
    d->disp2_bits = 0ull;
    d->n_fast = 0;
    d->n_fast_raw = 0;
    d->n_builds += 1;
}

// Every build kernel takes `gate`: NULL runs it unconditionally (forced build);
// otherwise it returns at once unless *gate (the device rebuild request) is set.
__device__ inline bool gated_off(const int32_t* gate) { return gate && *gate == 0; }

__device__ inline int col_cl0(const int64_t* pre, int c) { return (int)(pre[c] & 0xFFFFFFFFll); }
__device__ inline int col_grp0(const int64_t* pre, int c) { return (int)(pre[c] >> 32); }

// ---------------------------------------------------------------- vacuum grids

__global__ void __launch_bounds__(256) k_sys_bbox(const double* x, const double* y,
                                                  const double* z, const int64_t* sys_off,
                                                  double* lo, double* hi, DevScalars* dsc,
                                                  const int32_t* gate)
{
    if (gated_off(gate)) return;
    __shared__ double s_v[6][4];
    const int b = blockIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t a = sys_off[b] + threadIdx.x; a < sys_off[b + 1]; a += blockDim.x) {
        const double p[3] = {x[a], y[a], z[a]};
        for (int k = 0; k < 3; ++k) {
            if (!isfinite(p[k])) { bad = true; continue; }
            mn[k] = fmin(mn[k], p[k]);
            mx[k] = fmax(mx[k], p[k]);
        }
    }
    if (bad) set_flag(dsc, MD_FLAG_NONFINITE);
    for (int k = 0; k < 3; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            mn[k] = fmin(mn[k], __shfl_xor(mn[k], off, 64));
            mx[k] = fmax(mx[k], __shfl_xor(mx[k], off, 64));
        }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 3; ++k) { s_v[k][wv] = mn[k]; s_v[3 + k][wv] = mx[k]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) {
            double a = s_v[k][0], c = s_v[3 + k][0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
                a = fmin(a, s_v[k][w]);
                c = fmax(c, s_v[3 + k][w]);
            }
            if (!(a <= c)) { a = 0.0; c = 0.0; }     // empty system
            lo[b * 3 + k] = a;
            hi[b * 3 + k] = c;
        }
    }
}

// One block: grid dimensions of every vacuum system (columns of about 8 atoms'
// cross-section, z bins a quarter of that), bounded by per-system budgets so the
// totals never exceed the capacities; then the global column / bin offsets.
__global__ void __launch_bounds__(256) k_grid_vacuum(const double* lo, const double* hi,
                                                     const int64_t* sys_off, int B,
                                                     GridSys* grid, DevScalars* dsc,
                                                     const int32_t* gate)
{
    if (gated_off(gate)) return;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const int64_t nb = sys_off[b + 1] - sys_off[b];
        GridSys g;
        double ext[3];
        for (int k = 0; k < 3; ++k) {
            const double e = hi[b * 3 + k] - lo[b * 3 + k];
            const double margin = 1e-6 * (1.0 + e);
            ext[k] = fmax(e, 1e-3) + 2.0 * margin;
            g.origin[k] = lo[b * 3 + k] - margin;
            g.L[k] = 0.0;
            g.invL[k] = 0.0;
        }
        const double vol = ext[0] * ext[1] * ext[2];
        const double rho = (double)(nb > 0 ? nb : 1) / vol;
        double wt = cbrt(8.0 / rho);
        const int64_t col_budget = nb / 8 + 1;
        int nx, ny;
        for (;;) {
            nx = max(1, (int)(ext[0] / wt));
            ny = max(1, (int)(ext[1] / wt));
            if ((int64_t)nx * ny <= col_budget) break;
            wt *= 1.25;
        }
        const int64_t bin_budget = 2 * nb + 16;
        int nz = max(1, (int)(ext[2] / (0.25 * wt)));
        while ((int64_t)nx * ny * nz > bin_budget && nz > 1) nz = max(1, nz / 2);
        g.n[0] = nx; g.n[1] = ny; g.n[2] = nz;
        g.w[0] = ext[0] / nx; g.w[1] = ext[1] / ny; g.w[2] = ext[2] / nz;
        for (int k = 0; k < 3; ++k) g.inv_w[k] = 1.0 / g.w[k];
        g.periodic = 0;
        g.col_off = nx * ny;            // counts for now; offsets below
        g.bin_off = nx * ny * nz;
        grid[b] = g;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int cols = 0, bins = 0;
        for (int b = 0; b < B; ++b) {
            const int nc = grid[b].col_off, nbn = grid[b].bin_off;
            grid[b].col_off = cols;
            grid[b].bin_off = bins;
            cols += nc;
            bins += nbn;
        }
        dsc->n_cols = cols;
        dsc->n_bins = bins;
    }
}

// ---------------------------------------------------------------- binning + sort

struct BinArgs {
    int64_t N;
    const double *x, *y, *z;
    const int32_t* sys_of_atom;
    const GridSys* grid;
    int32_t* bin_cnt;
    int32_t* key;
    int32_t* rank;
    int32_t* img;
    double* xref;
    uint8_t* fast_flag;
    int64_t cap_bins;
    DevScalars* dsc;
    const int32_t* gate;
};

__device__ inline void bin_one(const BinArgs& A, int64_t a)
{
    const GridSys g = A.grid[A.sys_of_atom[a]];
    const double p[3] = {A.x[a], A.y[a], A.z[a]};
    int c[3], im[3] = {0, 0, 0};
    bool bad = false;
    for (int k = 0; k < 3; ++k) {
        double v = p[k];
        if (!isfinite(v)) { bad = true; v = 0.0; }
        double w;
        if (g.periodic) {
            const double kk = floor(v * g.invL[k]);
            if (fabs(kk) > 500.0) bad = true;
            im[k] = (int)fmin(fmax(kk, -500.0), 500.0);
            w = v - (double)im[k] * g.L[k];
        } else {
            w = v - g.origin[k];
        }
        const double cf = fmin(fmax(floor(w * g.inv_w[k]), 0.0), (double)(g.n[k] - 1));
        c[k] = (int)cf;
    }
    if (bad) set_flag(A.dsc, MD_FLAG_NONFINITE);
    int bin = g.bin_off + (c[0] * g.n[1] + c[1]) * g.n[2] + c[2];
    if (bin >= A.cap_bins) { set_flag(A.dsc, MD_FLAG_CELL_OVERFLOW); bin = (int)A.cap_bins - 1; }
    A.rank[a] = atomicAdd(&A.bin_cnt[bin], 1);
    A.key[a] = bin;
    A.img[a] = pack_img(im[0], im[1], im[2]);
    A.xref[a] = p[0];
    A.xref[A.N + a] = p[1];
    A.xref[2 * A.N + a] = p[2];
    A.fast_flag[a] = 0;
}

__global__ void __launch_bounds__(256) k_bin(BinArgs A)
{
    if (gated_off(A.gate)) return;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t a = gid; a < A.N; a += (int64_t)gridDim.x * blockDim.x)
        bin_one(A, a);
}


// Scatter atoms into bin order, and count clusters / groups per column (packed
// as ngroups << 32 | nclusters so one 64-bit scan yields both prefixes).
struct ScatterArgs {
    int64_t N;
    const int32_t* key;
    const int32_t* rank;
    const int32_t* bin_start;
    int32_t* sorted;
    const GridSys* grid;
    int B;
    int64_t* col_cnt;
    int64_t cap_cols;
    int G;
    const DevScalars* dsc;
    const int32_t* gate;
};

__global__ void __launch_bounds__(256) k_scatter_cols(ScatterArgs A)
{
    if (gated_off(A.gate)) return;
    const int ncols = A.dsc->n_cols;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t a = gid; a < A.N; a += stride)
        A.sorted[A.bin_start[A.key[a]] + A.rank[a]] = (int32_t)a;
    for (int64_t c = gid; c <= A.cap_cols; c += stride) {
        int ncl = 0;
        if (c < ncols) {
            const int b = find_sys_by_col(A.grid, A.B, (int)c);
            const GridSys& g = A.grid[b];
            const int nz = g.n[2];
            const int bin0 = g.bin_off + ((int)c - g.col_off) * nz;
            const int natoms = A.bin_start[bin0 + nz] - A.bin_start[bin0];
            ncl = (natoms + kCluster - 1) / kCluster;
        }
        const int ngrp = (ncl + A.G - 1) / A.G;
        A.col_cnt[c] = ((int64_t)ngrp << 32) | (int64_t)ncl;
    }
}

// Order the atoms of each bin by caller index (bins hold a few atoms), and clear
// the bin counters for the next build.
__global__ void __launch_bounds__(256) k_bin_sort(const int32_t* bin_start, int32_t* sorted,
                                                  int32_t* bin_cnt, int64_t cap_bins,
                                                  const DevScalars* dsc, const int32_t* gate)
{
    if (gated_off(gate)) return;
    const int nbins = dsc->n_bins;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < cap_bins;
         b += (int64_t)gridDim.x * blockDim.x) {
        bin_cnt[b] = 0;
        if (b >= nbins) continue;
        const int s = bin_start[b], e = bin_start[b + 1];
        if (e - s < 2 || e - s > 128) continue;
        for (int i = s + 1; i < e; ++i) {
            const int v = sorted[i];
            int j = i - 1;
            while (j >= s && sorted[j] > v) { sorted[j + 1] = sorted[j]; --j; }
            sorted[j + 1] = v;
        }
    }
}

struct ClusterArgs {
    const double *x, *y, *z;
    const uint8_t* type;
    const GridSys* grid;
    int B;
    const int32_t* bin_start;
    const int32_t* sorted;
    const int64_t* col_pre;
    const int32_t* img;
    int32_t* perm;
    int32_t* inv_perm;
    int32_t* slot_img;
    uint8_t* ts;
    uint8_t* atype;
    double* xs;
    int64_t cap_slots;
    double* cl_lo;
    double* cl_hi;
    Group* groups;
    int32_t* sys_grp0;
    int64_t cap_clusters;
    int G;
    int T;
    DevScalars* dsc;
    const int32_t* gate;
};

// largest column c in [0, n] whose first cluster index is <= v
__device__ inline int column_of_cluster(const int64_t* pre, int n, int v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (col_cl0(pre, mid) <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_clusters(ClusterArgs A)
{
    if (gated_off(A.gate)) return;
    const int ncols = A.dsc->n_cols;
    int total = col_cl0(A.col_pre, ncols);
    const int ngroups = col_grp0(A.col_pre, ncols);
    const int64_t gid0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (gid0 == 0) {
        if (total > A.cap_clusters) set_flag(A.dsc, MD_FLAG_CELL_OVERFLOW);
        A.dsc->n_clusters = min((int64_t)total, A.cap_clusters);
        A.dsc->n_groups = min((int64_t)ngroups, A.cap_clusters);
        A.dsc->n_slots = kCluster * min((int64_t)total, A.cap_clusters);
        A.sys_grp0[A.B] = min((int64_t)ngroups, A.cap_clusters);
    }
    for (int64_t b = gid0; b < A.B; b += stride)
        A.sys_grp0[b] = min(col_grp0(A.col_pre, A.grid[b].col_off), (int)A.cap_clusters);
    total = (int)min((int64_t)total, A.cap_clusters);
    for (int64_t cl = gid0; cl < total; cl += stride) {
        const int c = column_of_cluster(A.col_pre, ncols, (int)cl);
        const int b = find_sys_by_col(A.grid, A.B, c);
        const GridSys& g = A.grid[b];
        const int nz = g.n[2];
        const int bin0 = g.bin_off + (c - g.col_off) * nz;
        const int k = (int)cl - col_cl0(A.col_pre, c);
        const int abeg = A.bin_start[bin0] + kCluster * k;
        const int aend = A.bin_start[bin0 + nz];
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int l = 0; l < kCluster; ++l) {
            const int64_t slot = cl * kCluster + l;
            const int src = abeg + l;
            if (src < aend) {
                const int a = A.sorted[src];
                const int32_t im = A.img[a];
                A.perm[slot] = a;
                A.inv_perm[a] = (int32_t)slot;
                A.slot_img[slot] = im;
                int ty = A.type[a];
                if (ty >= A.T) { set_flag(A.dsc, MD_FLAG_BAD_INPUT); ty = A.T - 1; }
                A.ts[slot] = (uint8_t)ty;
                A.atype[a] = (uint8_t)ty;
                const double p[3] = {A.x[a], A.y[a], A.z[a]};
                for (int d = 0; d < 3; ++d) A.xs[d * A.cap_slots + slot] = p[d];
                for (int d = 0; d < 3; ++d) {
                    const double w = g.periodic ? p[d] - (double)unpack_img(im, d) * g.L[d] : p[d];
                    lo[d] = fmin(lo[d], w);
                    hi[d] = fmax(hi[d], w);
                }
            } else {
                A.perm[slot] = -1;
                A.slot_img[slot] = 0;
                A.ts[slot] = 0;
                for (int d = 0; d < 3; ++d) A.xs[d * A.cap_slots + slot] = NAN;
            }
        }
        for (int d = 0; d < 3; ++d) {
            A.cl_lo[cl * 3 + d] = lo[d];
            A.cl_hi[cl * 3 + d] = hi[d];
        }
        if (k % A.G == 0) {
            const int ncl_col = col_cl0(A.col_pre, c + 1) - col_cl0(A.col_pre, c);
            const int grp = col_grp0(A.col_pre, c) + k / A.G;
            if (grp < A.cap_clusters) {
                A.groups[grp].cl0 = (int)cl;
                A.groups[grp].ncl = min(A.G, ncl_col - k);
                A.groups[grp].sys = b;
                A.groups[grp].nent = 0;
            }
        }
    }
}

// ---------------------------------------------------------------- group candidate tables

struct EntryArgs {
    const GridSys* grid;
    const int64_t* col_pre;
    const double* cl_lo;
    const double* cl_hi;
    Group* groups;
    uint32_t* ent;
    uint8_t* ent_mask;
    int E_cap;
    double rlist;
    DevScalars* dsc;
    const int32_t* gate;
};

// One work-group (4 waves) per group.  The candidate columns are dealt round-robin
// to the waves; each wave appends its passing (cluster, shift) candidates in a
// fixed order with a ballot prefix, and the four wave lists are concatenated in
// wave order, so the table is deterministic.
constexpr int kEntryWaves = 4;

__global__ void __launch_bounds__(64 * kEntryWaves) k_group_entries(EntryArgs A)
{
    if (gated_off(A.gate)) return;
    extern __shared__ uint32_t s_eb[];                     // [waves][E_cap] entries
    uint8_t* s_mb = reinterpret_cast<uint8_t*>(s_eb + kEntryWaves * A.E_cap);  // masks
    __shared__ int s_cnt[kEntryWaves];
    __shared__ double s_cb[kMaxGroup][6];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ngroups = A.dsc->n_groups;
    const double rl = A.rlist, rl2 = rl * rl;
    for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const Group gr = A.groups[g];
        const GridSys gs = A.grid[gr.sys];
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = lane < gr.ncl ? A.cl_lo[(gr.cl0 + lane) * 3 + d] : INFINITY;
            hi[d] = lane < gr.ncl ? A.cl_hi[(gr.cl0 + lane) * 3 + d] : -INFINITY;
            for (int off = 32; off > 0; off >>= 1) {
                lo[d] = fmin(lo[d], __shfl_xor(lo[d], off, 64));
                hi[d] = fmax(hi[d], __shfl_xor(hi[d], off, 64));
            }
        }
        // an empty or non-finite box (non-finite positions are flagged by the binning)
        // gets no candidates
        bool finite_box = true;
        for (int d = 0; d < 3; ++d) finite_box = finite_box && isfinite(lo[d]) && isfinite(hi[d]);
        int cr[2][2] = {{0, -1}, {0, -1}};
        if (finite_box) {
            for (int d = 0; d < 2; ++d) {
                const double o = gs.periodic ? 0.0 : gs.origin[d];
                const double f0 = floor((lo[d] - rl - o) * gs.inv_w[d]);
                const double f1 = floor((hi[d] + rl - o) * gs.inv_w[d]);
                // images -1, 0, +1 only (the box edge is at least 2 (rc + skin))
                const double lim0 = gs.periodic ? -gs.n[d] : 0.0;
                const double lim1 = gs.periodic ? 2.0 * gs.n[d] - 1.0 : gs.n[d] - 1.0;
                cr[d][0] = (int)fmax(f0, lim0);
                cr[d][1] = (int)fmin(f1, lim1);
            }
        }
        const int ncy = cr[1][1] - cr[1][0] + 1;
        const int ncol = (cr[0][1] - cr[0][0] + 1) * max(ncy, 0);
        uint32_t* my_e = s_eb + w * A.E_cap;
        uint8_t* my_m = s_mb + w * A.E_cap;
        // bounding boxes of the group's own clusters (for the reach masks)
        if (threadIdx.x < gr.ncl * 6) {
            const int c = threadIdx.x / 6, d = threadIdx.x % 6;
            s_cb[c][d] = d < 3 ? A.cl_lo[(gr.cl0 + c) * 3 + d] : A.cl_hi[(gr.cl0 + c) * 3 + d - 3];
        }
        __syncthreads();
        int count = 0;
        for (int ci = w; ci < ncol; ci += kEntryWaves) {
            const int cx = cr[0][0] + ci / ncy, cy = cr[1][0] + ci % ncy;
            const int cxw = ((cx % gs.n[0]) + gs.n[0]) % gs.n[0];
            const int sx = (cx - cxw) / gs.n[0];
            const int cyw = ((cy % gs.n[1]) + gs.n[1]) % gs.n[1];
            const int sy = (cy - cyw) / gs.n[1];
            if (sx < -1 || sx > 1 || sy < -1 || sy > 1) continue;
            const int col = gs.col_off + cxw * gs.n[1] + cyw;
            const int j0 = col_cl0(A.col_pre, col), j1 = col_cl0(A.col_pre, col + 1);
            const double shx = gs.periodic ? sx * gs.L[0] : 0.0;
            const double shy = gs.periodic ? sy * gs.L[1] : 0.0;
            for (int base = j0; base < j1; base += 64) {
                // each lane tests one cluster J of the column for every z image
                const int J = base + lane;
                double jlo[3] = {0, 0, 0}, jhi[3] = {0, 0, 0};
                double dxy2 = INFINITY;
                if (J < j1) {
                    for (int d = 0; d < 3; ++d) {
                        jlo[d] = A.cl_lo[(int64_t)J * 3 + d];
                        jhi[d] = A.cl_hi[(int64_t)J * 3 + d];
                    }
                    jlo[0] += shx; jhi[0] += shx;
                    jlo[1] += shy; jhi[1] += shy;
                    const double gx = fmax(0.0, fmax(jlo[0] - hi[0], lo[0] - jhi[0]));
                    const double gy = fmax(0.0, fmax(jlo[1] - hi[1], lo[1] - jhi[1]));
                    dxy2 = gx * gx + gy * gy;
                }
                for (int sz = gs.periodic ? -1 : 0; sz <= (gs.periodic ? 1 : 0); ++sz) {
                    const double shz = gs.periodic ? sz * gs.L[2] : 0.0;
                    const double zl = jlo[2] + shz, zh = jhi[2] + shz;
                    const double gz = fmax(0.0, fmax(zl - hi[2], lo[2] - zh));
                    const bool pass = dxy2 + gz * gz < rl2;
                    const unsigned long long bal = __ballot(pass);
                    if (bal == 0ull) continue;
                    uint32_t cmask = 0u;
                    if (pass) {
                        // which clusters of the group this candidate can reach
                        for (int c = 0; c < gr.ncl; ++c) {
                            const double ax = fmax(0.0, fmax(jlo[0] - s_cb[c][3], s_cb[c][0] - jhi[0]));
                            const double ay = fmax(0.0, fmax(jlo[1] - s_cb[c][4], s_cb[c][1] - jhi[1]));
                            const double az = fmax(0.0, fmax(zl - s_cb[c][5], s_cb[c][2] - zh));
                            if (ax * ax + ay * ay + az * az < rl2) cmask |= 1u << c;
                        }
                        const int pos = count + __popcll(bal & ((1ull << lane) - 1ull));
                        if (pos < A.E_cap) {
                            my_e[pos] = (uint32_t)J | ((uint32_t)(sx + 1) << 26) |
                                        ((uint32_t)(sy + 1) << 28) | ((uint32_t)(sz + 1) << 30);
                            my_m[pos] = (uint8_t)cmask;
                        }
                    }
                    count += __popcll(bal);
                }
            }
        }
        if (lane == 0) s_cnt[w] = count;
        __syncthreads();
        int off = 0, total = 0;
        for (int v = 0; v < kEntryWaves; ++v) {
            if (v < w) off += s_cnt[v];
            total += s_cnt[v];
        }
        const int mine = min(count, A.E_cap);
        for (int i = lane; i < mine; i += 64) {
            const int pos = off + i;
            if (pos < A.E_cap) {
                A.ent[(int64_t)g * A.E_cap + pos] = my_e[i];
                A.ent_mask[(int64_t)g * A.E_cap + pos] = my_m[i];
            }
        }
        if (threadIdx.x == 0) {
            for (int d = 0; d < 3; ++d) {
                if (!finite_box) { lo[d] = 0.0; hi[d] = 0.0; }
                A.groups[g].lo[d] = lo[d];
                A.groups[g].hi[d] = hi[d];
                A.groups[g].c[d] = 0.5 * (lo[d] + hi[d]);
            }
            A.groups[g].nent = min(total, A.E_cap);
            A.groups[g].nent_raw = total;
            if (total > A.E_cap) set_flag(A.dsc, MD_FLAG_LIST_OVERFLOW);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- orchestration

void launch_build(Ctx* c, const double* x, const double* y, const double* z,
                  const uint8_t* type, bool force, hipStream_t st)
{
    const int64_t N = c->N;
    const int32_t* gate = force ? nullptr : &c->dsc->need_rebuild;
    const int wide = std::max(1, c->n_cu * 8);
    if (!c->cfg.periodic) {
        hipLaunchKernelGGL(k_sys_bbox, dim3(c->B), dim3(256), 0, st, x, y, z, c->d_sys_off,
                           c->d_sys_lo, c->d_sys_hi, c->dsc, gate);
        hipLaunchKernelGGL(k_grid_vacuum, dim3(1), dim3(256), 0, st, c->d_sys_lo, c->d_sys_hi,
                           c->d_sys_off, c->B, c->d_grid, c->dsc, gate);
    }
    {
        BinArgs A{N, x, y, z, c->d_sys_of_atom, c->d_grid, c->d_bin_cnt, c->d_key, c->d_rank,
                  c->d_img, c->d_xref, c->d_fast_flag, c->cap_bins, c->dsc, gate};
        const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(div_up(N, 256), wide));
        hipLaunchKernelGGL(k_bin, dim3(nb), dim3(256), 0, st, A);
    }
    launch_scan(c->d_bin_cnt, c->d_bin_start, c->cap_bins + 1,
                reinterpret_cast<int32_t*>(c->d_scan_tmp), gate, st);
    {
        ScatterArgs A{N, c->d_key, c->d_rank, c->d_bin_start, c->d_sorted, c->d_grid, c->B,
                      c->d_col_cnt, c->cap_cols, c->G, c->dsc, gate};
        const int nb = (int)std::max<int64_t>(
            1, std::min<int64_t>(div_up(std::max<int64_t>(N, c->cap_cols + 1), 256), wide));
        hipLaunchKernelGGL(k_scatter_cols, dim3(nb), dim3(256), 0, st, A);
    }
    {
        const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(div_up(c->cap_bins, 256), wide));
        hipLaunchKernelGGL(k_bin_sort, dim3(nb), dim3(256), 0, st, c->d_bin_start, c->d_sorted,
                           c->d_bin_cnt, c->cap_bins, c->dsc, gate);
    }
    launch_scan64(c->d_col_cnt, c->d_col_pre, c->cap_cols + 1, c->d_scan_tmp, gate, st);
    {
        ClusterArgs A{x, y, z, type, c->d_grid, c->B, c->d_bin_start, c->d_sorted, c->d_col_pre,
                      c->d_img, c->d_perm, c->d_inv_perm, c->d_slot_img, c->d_ts, c->d_atype,
                      c->d_xs,
                      c->cap_slots, c->d_cl_lo, c->d_cl_hi, c->d_groups, c->d_sys_grp0,
                      c->cap_clusters, c->G, c->T, c->dsc, gate};
        const int nb = (int)std::max<int64_t>(
            1, std::min<int64_t>(div_up(std::max<int64_t>(c->cap_clusters, c->B), 256), wide));
        hipLaunchKernelGGL(k_clusters, dim3(nb), dim3(256), 0, st, A);
    }
    {
        EntryArgs A{c->d_grid, c->d_col_pre, c->d_cl_lo, c->d_cl_hi, c->d_groups, c->d_ent,
                    c->d_ent_mask, c->E_cap, c->rlist, c->dsc, gate};
        const size_t lds = (size_t)kEntryWaves * c->E_cap * (sizeof(uint32_t) + 1);
        const int nb = (int)std::min<int64_t>(c->cap_groups, (int64_t)c->n_cu * 4);
        hipLaunchKernelGGL(k_group_entries, dim3(std::max(nb, 1)), dim3(64 * kEntryWaves), lds,
                           st, A);
    }
    hipLaunchKernelGGL(k_build_done, dim3(1), dim3(1), 0, st, c->dsc, gate);
}

__global__ void k_skin_check(DevScalars* d)
{
    if (d->need_rebuild) d->flags |= MD_FLAG_SKIN;
}

void launch_skin_check(Ctx* c, hipStream_t st)
{
    hipLaunchKernelGGL(k_skin_check, dim3(1), dim3(1), 0, st, c->dsc);
}


}  // namespace md
