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
#include "md_device.h"
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
__device__ inline void ph_build_done(DevScalars* d)
{
    d->need_rebuild = 0;
    d->lists_pending = 1;
    d->disp2_bits = 0ull;
    d->n_fast = 0;
    d->n_fast_raw = 0;
    d->n_builds += 1;
}

__global__ void k_build_done(DevScalars* d, const int32_t* gate)
{
    if (gate && *gate == 0) return;
    ph_build_done(d);
}

// Every build kernel takes `gate`: NULL runs it unconditionally (forced build);
// otherwise it returns at once unless *gate (the device rebuild request) is set.
__device__ inline bool gated_off(const int32_t* gate) { return gate && *gate == 0; }

__device__ inline int col_cl0(const int64_t* pre, int c) { return (int)(pre[c] & 0xFFFFFFFFll); }
__device__ inline int col_grp0(const int64_t* pre, int c) { return (int)(pre[c] >> 32); }

// ---------------------------------------------------------------- vacuum grids

// Bounding box of every vacuum system b = bid, bid + nblk, ... (one block each, up
// to 1024 threads).
__device__ void ph_sys_bbox(const double* x, const double* y, const double* z,
                            const int64_t* sys_off, int B, double* lo, double* hi,
                            DevScalars* dsc, int bid, int nblk)
{
    __shared__ double s_v[6][16];
    for (int b = bid; b < B; b += nblk) {
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
    __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_sys_bbox(const double* x, const double* y,
                                                  const double* z, const int64_t* sys_off, int B,
                                                  double* lo, double* hi, DevScalars* dsc,
                                                  const int32_t* gate)
{
    if (gated_off(gate)) return;
    ph_sys_bbox(x, y, z, sys_off, B, lo, hi, dsc, blockIdx.x, gridDim.x);
}

// One block: grid dimensions of every vacuum system (columns of about 8 atoms'
// cross-section, z bins a quarter of that), bounded by per-system budgets so the
// totals never exceed the capacities; then the global column / bin offsets.
__device__ void ph_grid_vacuum(const double* lo, const double* hi, const int64_t* sys_off, int B,
                               GridSys* grid, DevScalars* dsc)
{
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

__global__ void __launch_bounds__(256) k_grid_vacuum(const double* lo, const double* hi,
                                                     const int64_t* sys_off, int B,
                                                     GridSys* grid, DevScalars* dsc,
                                                     const int32_t* gate)
{
    if (gated_off(gate)) return;
    ph_grid_vacuum(lo, hi, sys_off, B, grid, dsc);
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

__device__ inline void ph_bin(const BinArgs& A, int64_t gid, int64_t stride)
{
    for (int64_t a = gid; a < A.N; a += stride) bin_one(A, a);
}

__global__ void __launch_bounds__(256) k_bin(BinArgs A)
{
    if (gated_off(A.gate)) return;
    ph_bin(A, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
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

__device__ void ph_scatter_cols(const ScatterArgs& A, int64_t gid, int64_t stride)
{
    const int ncols = A.dsc->n_cols;
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

__global__ void __launch_bounds__(256) k_scatter_cols(ScatterArgs A)
{
    if (gated_off(A.gate)) return;
    ph_scatter_cols(A, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                    (int64_t)gridDim.x * blockDim.x);
}

// Order the atoms of each bin by caller index (bins hold a few atoms), and clear
// the bin counters for the next build.  Every bin is sorted, whatever its size (a
// vacuum grid stretched by a few far ions can put hundreds of atoms in one bin), so
// the slot order, and with it every summation order, never depends on the order of
// the binning atomics.
// In-place heap sort of a[0 .. m), ascending, by one thread: m log m steps where an
// insertion sort takes ~m^2 / 4 (bins of a few dozen atoms: the dense cores of vacuum
// grids).
__device__ inline void heap_sort_i32(int32_t* a, int m)
{
    // move a[root]'s value down the max-heap a[0 .. end) to its place
    auto sift = [&](int root, int end) {
        const int32_t v = a[root];
        int i = root;
        for (;;) {
            int c = 2 * i + 1;
            if (c >= end) break;
            int32_t cv = a[c];
            if (c + 1 < end) {
                const int32_t c2 = a[c + 1];
                if (c2 > cv) { ++c; cv = c2; }
            }
            if (cv <= v) break;
            a[i] = cv;
            i = c;
        }
        a[i] = v;
    };
    for (int r = m / 2 - 1; r >= 0; --r) sift(r, m);
    for (int end = m - 1; end > 0; --end) {
        const int32_t t = a[0];
        a[0] = a[end];
        a[end] = t;
        sift(0, end);
    }
}

constexpr int kBinInsertionMax = 32;     // above this, the heap sort
constexpr int kBinThreadMax = 128;       // above this, the whole work-group (rank sort)
constexpr int kRankTile = 1024;          // values of the bin staged in LDS at a time
constexpr int kRankPer = 4;              // values ranked per thread and pass
constexpr int kSortBlockMax = 1024;      // largest work-group calling ph_bin_sort

// Sort a[0 .. m) (distinct values) by the whole work-group: each value's place is the
// number of smaller values (counted against LDS tiles of the bin), written to tmp and
// copied back.  m^2 / blockDim compares per thread: a bin of thousands of atoms (a
// vacuum grid stretched by a far ion keeps a whole cluster in one bin) takes tens of
// microseconds where one thread's heap sort took milliseconds.  Called by every thread
// of the work-group; returns after a barrier.
__device__ void block_rank_sort(int32_t* a, int32_t* tmp, int m, int32_t* s_tile)
{
    const int nt = blockDim.x;
    for (int e0 = 0; e0 < m; e0 += nt * kRankPer) {
        int32_t v[kRankPer];
        int cnt[kRankPer];
#pragma unroll
        for (int u = 0; u < kRankPer; ++u) {
            const int e = e0 + u * nt + (int)threadIdx.x;
            v[u] = e < m ? a[e] : INT_MAX;
            cnt[u] = 0;
        }
        for (int j0 = 0; j0 < m; j0 += kRankTile) {
            const int nj = min(kRankTile, m - j0);
            __syncthreads();                              // the previous tile is consumed
            for (int j = threadIdx.x; j < nj; j += nt) s_tile[j] = a[j0 + j];
            __syncthreads();
            for (int j = 0; j < nj; ++j) {
                const int32_t w = s_tile[j];
#pragma unroll
                for (int u = 0; u < kRankPer; ++u) cnt[u] += w < v[u] ? 1 : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kRankPer; ++u) {
            const int e = e0 + u * nt + (int)threadIdx.x;
            if (e < m) tmp[cnt[u]] = v[u];
        }
    }
    __syncthreads();                                      // every place written
    for (int e = threadIdx.x; e < m; e += nt) a[e] = tmp[e];
    __syncthreads();
}

// Every bin's atoms in index order (deterministic slot order), bins dealt to the
// work-group's threads in tiles of blockDim.x: up to 8 atoms a sorting network in
// registers, up to kBinInsertionMax an insertion sort, up to kBinThreadMax a heap sort,
// larger bins by the whole work-group after its tile.  tmp: N scratch words (the
// binning ranks, free once the atoms are scattered).  gid - threadIdx.x and stride must
// be multiples of blockDim.x (every thread of a work-group takes the same tiles).
__device__ void ph_bin_sort(const int32_t* bin_start, int32_t* sorted, int32_t* tmp,
                            int32_t* bin_cnt, int64_t cap_bins, const DevScalars* dsc,
                            int64_t gid, int64_t stride)
{
    __shared__ int32_t s_big[kSortBlockMax];
    __shared__ int32_t s_tile[kRankTile];
    __shared__ int s_nbig;
    const int nbins = dsc->n_bins;
    for (int64_t base = gid - threadIdx.x; base < cap_bins; base += stride) {
        if (threadIdx.x == 0) s_nbig = 0;
        __syncthreads();
        const int64_t b = base + threadIdx.x;
        if (b < cap_bins) {
            bin_cnt[b] = 0;
            const int s = b < nbins ? bin_start[b] : 0, e = b < nbins ? bin_start[b + 1] : 0;
            if (e - s > kBinThreadMax) {
                s_big[atomicAdd(&s_nbig, 1)] = (int32_t)b;    // sorted below
            } else if (e - s > kBinInsertionMax) {
                heap_sort_i32(sorted + s, e - s);
            } else if (e - s > 8) {
                for (int i = s + 1; i < e; ++i) {
                    const int v = sorted[i];
                    int j = i - 1;
                    while (j >= s && sorted[j] > v) { sorted[j + 1] = sorted[j]; --j; }
                    sorted[j + 1] = v;
                }
            } else if (e - s >= 2) {
                // the common case (a bin holds ~2 atoms): all loads at once, a sorting
                // network in registers (Batcher's odd-even merge for 8 inputs), all stores
                constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3},
                                             {4, 6}, {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5},
                                             {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4},
                                             {5, 6}};
                int v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = s + i < e ? sorted[s + i] : INT_MAX;
#pragma unroll
                for (int c = 0; c < 19; ++c) {
                    const int lo = min(v[kNet[c][0]], v[kNet[c][1]]);
                    const int hi = max(v[kNet[c][0]], v[kNet[c][1]]);
                    v[kNet[c][0]] = lo;
                    v[kNet[c][1]] = hi;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (s + i < e) sorted[s + i] = v[i];
            }
        }
        __syncthreads();
        const int nbig = s_nbig;
        for (int i = 0; i < nbig; ++i) {
            const int bb = s_big[i];
            const int s = bin_start[bb], e = bin_start[bb + 1];
            block_rank_sort(sorted + s, tmp + s, e - s, s_tile);
        }
    }
}

__global__ void __launch_bounds__(256) k_bin_sort(const int32_t* bin_start, int32_t* sorted,
                                                  int32_t* tmp, int32_t* bin_cnt,
                                                  int64_t cap_bins, const DevScalars* dsc,
                                                  const int32_t* gate)
{
    if (gated_off(gate)) return;
    ph_bin_sort(bin_start, sorted, tmp, bin_cnt, cap_bins, dsc,
                blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
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

__device__ void ph_clusters(const ClusterArgs& A, int64_t gid0, int64_t stride)
{
    const int ncols = A.dsc->n_cols;
    int total = col_cl0(A.col_pre, ncols);
    const int ngroups = col_grp0(A.col_pre, ncols);
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
    // one thread per slot; the kCluster threads of a cluster are adjacent lanes (the
    // stride is a multiple of 64), which reduce the cluster's bounding box by shuffles
    for (int64_t slot = gid0; slot < (int64_t)total * kCluster; slot += stride) {
        const int64_t cl = slot / kCluster;
        const int l = (int)(slot % kCluster);
        const int c = column_of_cluster(A.col_pre, ncols, (int)cl);
        const int b = find_sys_by_col(A.grid, A.B, c);
        const GridSys& g = A.grid[b];
        const int nz = g.n[2];
        const int bin0 = g.bin_off + (c - g.col_off) * nz;
        const int k = (int)cl - col_cl0(A.col_pre, c);
        const int abeg = A.bin_start[bin0] + kCluster * k;
        const int aend = A.bin_start[bin0 + nz];
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        {
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
        for (int d = 0; d < 3; ++d)
            for (int o = 1; o < kCluster; o <<= 1) {
                lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
                hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
            }
        if (l != 0) continue;
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

__global__ void __launch_bounds__(256) k_clusters(ClusterArgs A)
{
    if (gated_off(A.gate)) return;
    ph_clusters(A, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                (int64_t)gridDim.x * blockDim.x);
}

// ---------------------------------------------------------------- group candidate tables

struct EntryArgs {
    const GridSys* grid;
    const int64_t* col_pre;
    const int32_t* bin_start;     // first sorted atom of each bin (columns' z bins)
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

// kEntryWaves waves per group (one: measured fastest, since this latency-bound phase
// gains more from groups in flight than from lanes per group); a work-group of
// 64 kEntryWaves k threads works on k groups at once.  The candidate columns of a
// group are listed in LDS with, per z image, the range of their clusters that holds
// an atom inside the group's z window widened by rc + skin (found from the column's
// z bins: a cluster with no atom in that window has no pair within reach), and the
// clusters of all ranges are dealt to the group's lanes as one flat sequence (so
// every lane has work and the loads of many clusters are in flight together); each
// wave appends its passing (cluster, shift) candidates in a fixed order with a
// ballot prefix, and the wave lists are concatenated in wave order, so the table is
// deterministic.
constexpr int kEntryWaves = 1;
constexpr int kEntryMaxSub = 16;          // groups at once per work-group (1024 threads)
constexpr int kEntryMaxCols = 64;         // candidate columns listed per group (else per column)
constexpr int kEntrySeg = 3;              // cluster ranges per listed column (z images -1, 0, 1)
static_assert(kEntryMaxCols <= 64 * kEntryWaves, "one thread per listed column");

// s_eb: dynamic LDS of blockDim / 64 * E_cap * 5 bytes.
__device__ void ph_group_entries(const EntryArgs& A, uint32_t* s_eb, int bid, int nblk)
{
    const int nsub = blockDim.x / (64 * kEntryWaves);
    const int sub = threadIdx.x / (64 * kEntryWaves);
    const int ltid = threadIdx.x % (64 * kEntryWaves);
    uint8_t* s_mb = reinterpret_cast<uint8_t*>(s_eb + nsub * kEntryWaves * A.E_cap) +
                    sub * kEntryWaves * A.E_cap;                       // masks
    s_eb += sub * kEntryWaves * A.E_cap;
    __shared__ int s_cnt_all[kEntryMaxSub][kEntryWaves];
    __shared__ double s_cb_all[kEntryMaxSub][kMaxGroup][6];
    // per (listed column, z image) range: first cluster, prefix of the cluster counts,
    // shifts (sx + 1) | (sy + 1) << 2 | (sz + 1) << 4
    __shared__ int s_cj0_all[kEntryMaxSub][kEntrySeg * kEntryMaxCols];
    __shared__ int s_cpre_all[kEntryMaxSub][kEntrySeg * kEntryMaxCols + 1];
    __shared__ uint8_t s_csh_all[kEntryMaxSub][kEntrySeg * kEntryMaxCols];
    int* s_cnt = s_cnt_all[sub];
    double (*s_cb)[6] = s_cb_all[sub];
    int* s_cj0 = s_cj0_all[sub];
    int* s_cpre = s_cpre_all[sub];
    uint8_t* s_csh = s_csh_all[sub];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(ltid >> 6);
    const int ngroups = A.dsc->n_groups;
    const double rl = A.rlist, rl2 = rl * rl;
    // every sub-group of the work-group takes the same number of trips (the
    // work-group barriers below are shared); idle ones skip the work
    for (int k = 0; (k * nblk + bid) * nsub < ngroups; ++k) {
        const int g = (k * nblk + bid) * nsub + sub;
        const bool active = g < ngroups;
        const Group gr = active ? A.groups[g] : Group{};
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
        const bool flat = ncol <= kEntryMaxCols;          // the same for the whole group
        uint32_t* my_e = s_eb + w * A.E_cap;
        uint8_t* my_m = s_mb + w * A.E_cap;
        // candidate column ci: global column and periodic shifts (valid: images -1..1)
        auto column = [&](int ci, int* col, int* sx, int* sy) -> bool {
            const int cx = cr[0][0] + ci / ncy, cy = cr[1][0] + ci % ncy;
            const int cxw = ((cx % gs.n[0]) + gs.n[0]) % gs.n[0];
            const int cyw = ((cy % gs.n[1]) + gs.n[1]) % gs.n[1];
            *sx = (cx - cxw) / gs.n[0];
            *sy = (cy - cyw) / gs.n[1];
            *col = gs.col_off + cxw * gs.n[1] + cyw;
            return *sx >= -1 && *sx <= 1 && *sy >= -1 && *sy <= 1;
        };
        // bounding boxes of the group's own clusters (for the reach masks) and the
        // list of candidate columns with their cluster counts
        if (active && ltid < gr.ncl * 6) {
            const int c = ltid / 6, d = ltid % 6;
            s_cb[c][d] = d < 3 ? A.cl_lo[(gr.cl0 + c) * 3 + d] : A.cl_hi[(gr.cl0 + c) * 3 + d - 3];
        }
        const int nseg = kEntrySeg * ncol;
        if (flat && ltid < ncol) {
            int col, sx, sy;
            const bool ok = column(ltid, &col, &sx, &sy);
            const int nz = gs.n[2];
            const int bin0 = gs.bin_off + (col - gs.col_off) * nz;
            const int j0 = ok ? col_cl0(A.col_pre, col) : 0;
            const int a0 = ok ? A.bin_start[bin0] : 0;
            const double oz = gs.periodic ? 0.0 : gs.origin[2];
            const double eps = 1e-6 * (1.0 + rl);   // beyond any rounding of the bin edges
            for (int q = 0; q < kEntrySeg; ++q) {
                const int sz = q - 1;
                int k0 = 0, nk = 0;
                if (ok && (gs.periodic || sz == 0)) {
                    // the window in the binning coordinate of this image, then its bins
                    // (bin index is monotone in z, clamped at the ends like the binning)
                    const double shz = gs.periodic ? sz * gs.L[2] : 0.0;
                    const double z0 = lo[2] - rl - eps - shz - oz;
                    const double z1 = hi[2] + rl + eps - shz - oz;
                    const double f0 = floor(z0 * gs.inv_w[2]), f1 = floor(z1 * gs.inv_w[2]);
                    if (f1 >= 0.0 && f0 <= (double)(nz - 1)) {
                        const int b0 = (int)fmax(f0, 0.0), b1 = (int)fmin(f1, (double)(nz - 1));
                        const int s0 = A.bin_start[bin0 + b0] - a0;
                        const int s1 = A.bin_start[bin0 + b1 + 1] - a0;
                        if (s1 > s0) {
                            k0 = s0 / kCluster;
                            nk = (s1 - 1) / kCluster - k0 + 1;
                        }
                    }
                }
                const int i = kEntrySeg * ltid + q;
                s_cj0[i] = j0 + k0;
                s_cpre[i + 1] = nk;
                s_csh[i] = (uint8_t)((sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4));
            }
        }
        __syncthreads();
        if (flat && ltid < 64) {                 // prefix of the counts (one wave)
            int carry = 0;
            for (int base = 0; base < nseg; base += 64) {
                const int i = base + lane;
                const int v = i < nseg ? s_cpre[i + 1] : 0;
                int inc = v;
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(inc, o, 64);
                    if (lane >= o) inc += y;
                }
                if (i < nseg) s_cpre[i + 1] = carry + inc;
                carry += __shfl(inc, 63, 64);
            }
            if (lane == 0) s_cpre[0] = 0;
        }
        __syncthreads();
        int count = 0;
        // test cluster J (this lane's, when `has`) under the column shifts and the z
        // images sz0 .. sz1; append the passing ones in (image, lane) order
        // (jlo, jhi: the box of J, read by the caller when `has`)
        auto test_append = [&](bool has, int J, int sx, int sy, int sz0, int sz1, double* jlo,
                               double* jhi) {
            const double shx = gs.periodic ? sx * gs.L[0] : 0.0;
            const double shy = gs.periodic ? sy * gs.L[1] : 0.0;
            double dxy2 = INFINITY;
            if (has) {
                jlo[0] += shx; jhi[0] += shx;
                jlo[1] += shy; jhi[1] += shy;
                const double gx = fmax(0.0, fmax(jlo[0] - hi[0], lo[0] - jhi[0]));
                const double gy = fmax(0.0, fmax(jlo[1] - hi[1], lo[1] - jhi[1]));
                dxy2 = gx * gx + gy * gy;
            }
            for (int sz = sz0; sz <= sz1; ++sz) {
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
        };
        // the box of cluster J (when `has`)
        auto load_box = [&](bool has, int J, double* jlo, double* jhi) {
            for (int d = 0; d < 3; ++d) {
                jlo[d] = has ? A.cl_lo[(int64_t)J * 3 + d] : 0.0;
                jhi[d] = has ? A.cl_hi[(int64_t)J * 3 + d] : 0.0;
            }
        };
        if (flat) {
            const int ntot = s_cpre[nseg];
            // item t: its range (the last ci with s_cpre[ci] <= t), cluster and shifts;
            // the next item's box is read before this one is tested (the loads' latency
            // overlaps the tests)
            auto item = [&](int t, int* J, int* sh) {
                int a = 0, b = nseg - 1;
                while (a < b) {
                    const int m = (a + b + 1) >> 1;
                    if (s_cpre[m] <= t) a = m; else b = m - 1;
                }
                *sh = s_csh[a];
                *J = s_cj0[a] + (t - s_cpre[a]);
            };
            int nJ = 0, nsh = 0;
            double nlo[3], nhi[3];
            const int t_first = w * 64 + lane;
            if (w * 64 < ntot) item(t_first, &nJ, &nsh);
            load_box(t_first < ntot, nJ, nlo, nhi);
            for (int t0 = w * 64; t0 < ntot; t0 += kEntryWaves * 64) {
                const int t = t0 + lane;
                const bool has = t < ntot;
                const int J = nJ, sh = nsh;
                double jlo[3], jhi[3];
                for (int d = 0; d < 3; ++d) { jlo[d] = nlo[d]; jhi[d] = nhi[d]; }
                const int tn = t + kEntryWaves * 64;
                if (t0 + kEntryWaves * 64 < ntot) {
                    item(tn, &nJ, &nsh);
                    load_box(tn < ntot, nJ, nlo, nhi);
                }
                const int sz = ((sh >> 4) & 3) - 1;
                test_append(has, J, (sh & 3) - 1, ((sh >> 2) & 3) - 1, sz, sz, jlo, jhi);
            }
        } else {
            for (int ci = w; ci < ncol; ci += kEntryWaves) {
                int col, sx, sy;
                if (!column(ci, &col, &sx, &sy)) continue;
                const int j0 = col_cl0(A.col_pre, col), j1 = col_cl0(A.col_pre, col + 1);
                for (int base = j0; base < j1; base += 64) {
                    double jlo[3], jhi[3];
                    load_box(base + lane < j1, base + lane, jlo, jhi);
                    test_append(base + lane < j1, base + lane, sx, sy, gs.periodic ? -1 : 0,
                                gs.periodic ? 1 : 0, jlo, jhi);
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
        if (active && ltid == 0) {
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

__global__ void __launch_bounds__(64 * kEntryWaves) k_group_entries(EntryArgs A)
{
    if (gated_off(A.gate)) return;
    extern __shared__ uint32_t s_eb[];                     // [waves][E_cap] entries
    ph_group_entries(A, s_eb, blockIdx.x, gridDim.x);
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
                           c->B, c->d_sys_lo, c->d_sys_hi, c->dsc, gate);
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
                           c->d_rank, c->d_bin_cnt, c->cap_bins, c->dsc, gate);
    }
    launch_scan64(c->d_col_cnt, c->d_col_pre, c->cap_cols + 1, c->d_scan_tmp, gate, st);
    {
        ClusterArgs A{x, y, z, type, c->d_grid, c->B, c->d_bin_start, c->d_sorted, c->d_col_pre,
                      c->d_img, c->d_perm, c->d_inv_perm, c->d_slot_img, c->d_ts, c->d_atype,
                      c->d_xs,
                      c->cap_slots, c->d_cl_lo, c->d_cl_hi, c->d_groups, c->d_sys_grp0,
                      c->cap_clusters, c->G, c->T, c->dsc, gate};
        const int nb = (int)std::max<int64_t>(
            1, std::min<int64_t>(div_up(std::max<int64_t>(c->cap_slots, c->B), 256), wide));
        hipLaunchKernelGGL(k_clusters, dim3(nb), dim3(256), 0, st, A);
    }
    {
        EntryArgs A{c->d_grid, c->d_col_pre, c->d_bin_start, c->d_cl_lo, c->d_cl_hi, c->d_groups, c->d_ent,
                    c->d_ent_mask, c->E_cap, c->rlist, c->dsc, gate};
        const size_t lds = (size_t)kEntryWaves * c->E_cap * (sizeof(uint32_t) + 1);
        const int nb = (int)std::min<int64_t>(c->cap_groups, (int64_t)c->n_cu * 4);
        hipLaunchKernelGGL(k_group_entries, dim3(std::max(nb, 1)), dim3(64 * kEntryWaves), lds,
                           st, A);
    }
    hipLaunchKernelGGL(k_build_done, dim3(1), dim3(1), 0, st, c->dsc, gate);
}

// ---------------------------------------------------------------- fused per-step build

// Exclusive scan of in[0..n) into out[0..n) by all blocks of a persistent grid:
// each block sums a contiguous chunk, waits for the others, offsets its chunk by
// the totals of the chunks before it and scans it in tiles.  tot holds nblk values.
template <class T>
__device__ bool ph_scan(const T* in, T* out, int64_t n, T* tot, int bid, int nblk,
                        GridBarrier& gb, DevScalars* d)
{
    __shared__ T s_w[16];
    const int64_t chunk = (n + nblk - 1) / nblk;
    const int64_t c0 = min(n, (int64_t)bid * chunk), c1 = min(n, c0 + chunk);
    T t = 0;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) t += in[i];
    t = block_sum_all(t, s_w);
    if (threadIdx.x == 0) tot[bid] = t;
    if (!grid_barrier(gb, d)) return false;
    T off = 0;
    for (int k = threadIdx.x; k < bid; k += blockDim.x) off += tot[k];
    off = block_sum_all(off, s_w);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t base = c0; base < c1; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const T v = i < c1 ? in[i] : (T)0;
        T inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const T y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        __syncthreads();
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        T wofs = 0, ttot = 0;
        for (int k = 0; k < nw; ++k) {
            if (k < wv) wofs += s_w[k];
            ttot += s_w[k];
        }
        if (i < c1) out[i] = off + wofs + inc - v;
        off += ttot;
    }
    return grid_barrier(gb, d);
}

// Exclusive scan of a short array computed by every block on its own (no grid
// barrier): each block writes the same values, so every block can read the result
// right away (its own writes are visible to it).  n must be small (the column
// counts), since every block reads and writes all of it.
template <class T>
__device__ void ph_scan_local(const T* in, T* out, int64_t n)
{
    __shared__ T s_w[16];
    __shared__ T s_carry;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    for (int64_t base = 0; base < n; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const T v = i < n ? in[i] : (T)0;
        T inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const T y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        __syncthreads();
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        T wofs = 0, ttot = 0;
        for (int k = 0; k < nw; ++k) {
            if (k < wv) wofs += s_w[k];
            ttot += s_w[k];
        }
        const T carry = s_carry;
        if (i < n) out[i] = carry + wofs + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + ttot;
    }
    __syncthreads();
}

constexpr int64_t kLocalScanMax = 4096;   // column counts up to this are scanned per block

struct StepBuildArgs {
    FastJoinArgs join;
    int force;                   // rebuild whatever the displacements
    int periodic;
    const double *x, *y, *z;
    const int64_t* sys_off;
    int B;
    double *sys_lo, *sys_hi;
    GridSys* grid;
    BinArgs bin;
    ScatterArgs sc;
    ClusterArgs cl;
    EntryArgs en;
    int32_t* bin_cnt;
    int32_t* bin_start;
    int64_t n_bin_scan;          // cap_bins + 1
    int64_t* col_cnt;
    int64_t* col_pre;
    int64_t n_col_scan;          // cap_cols + 1
    int64_t* scan_tmp;           // >= grid blocks
    int32_t* sorted;
    int64_t cap_bins;
    RepackArgs rp;
    uint32_t* bar_arrive;        // >= grid blocks
    DevScalars* dsc;
};

// The build half of one step in one persistent launch (all blocks resident): gather
// positions and charges into the current slot order for the force kernels, join the
// fast-atom lists of phase 0 of the integrator and advance the step counter; when a
// rebuild is due (more fast atoms than the capacity, a pending request, or `force`),
// run the whole build with grid barriers between its phases and gather again into
// the new slot order.  On a step without rebuild this replaces a dozen launches by one.
// 1024 threads per work-group: one work-group per CU fits (registers), which gives
// the latency-bound phases 16 waves per CU and each grid barrier one release per CU.
constexpr int kBuildStepThreads = 1024;
static_assert(kBuildStepThreads <= kSortBlockMax, "the bin sort lists one large bin per thread");

__global__ void __launch_bounds__(kBuildStepThreads) k_build_step(StepBuildArgs S)
{
    extern __shared__ uint32_t s_dyn[];
    __shared__ int s_i[16];
    DevScalars* d = S.dsc;
    const int bid = blockIdx.x, nblk = gridDim.x;
    const int64_t gid = bid * (int64_t)blockDim.x + threadIdx.x;
    const int64_t gstride = (int64_t)nblk * blockDim.x;
    // every block takes the decision from the same inputs (no one writes them here)
    const int pending = d->need_rebuild;
    // unless a rebuild is already requested, the slot repack for the current lists
    // runs first, before the decision is known (a rebuild rewrites everything it
    // writes, after several grid barriers; the binning of a rebuild may clear the fast
    // flags while another work-group's repack still reads them, which only changes
    // values that are rewritten).  The last work-group joins the fast-atom lists
    // instead (when there are others).
    if (!S.force && !pending && (nblk == 1 || bid < nblk - 1))
        repack_range<4>(S.rp, gid, (int64_t)(nblk > 1 ? nblk - 1 : 1) * blockDim.x, false);
    int cnt = 0;
    for (int k = threadIdx.x; k < S.join.nblocks; k += blockDim.x) cnt += S.join.fast_cnt[k];
    const int total = block_sum_all(cnt, s_i);
    const bool rebuild = S.force || pending || total > S.join.fast_cap;
    // the generation word cannot move before every block has arrived at the first
    // barrier, so all blocks read the same starting value here
    GridBarrier gb{S.bar_arrive, &d->bar_gen, (unsigned)nblk,
                   __hip_atomic_load(&d->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
    if (bid == nblk - 1) fast_join_block(S.join);
    if (!rebuild) return;
    if (!S.periodic) {
        ph_sys_bbox(S.x, S.y, S.z, S.sys_off, S.B, S.sys_lo, S.sys_hi, d, bid, nblk);
        if (!grid_barrier(gb, d)) return;
        if (bid == 0) ph_grid_vacuum(S.sys_lo, S.sys_hi, S.sys_off, S.B, S.grid, d);
        if (!grid_barrier(gb, d)) return;
    }
    ph_bin(S.bin, gid, gstride);
    if (!grid_barrier(gb, d)) return;
    if (!ph_scan<int32_t>(S.bin_cnt, S.bin_start, S.n_bin_scan,
                          reinterpret_cast<int32_t*>(S.scan_tmp), bid, nblk, gb, d))
        return;
    ph_scatter_cols(S.sc, gid, gstride);
    if (!grid_barrier(gb, d)) return;
    ph_bin_sort(S.bin_start, S.sorted, S.bin.rank, S.bin_cnt, S.cap_bins, d, gid, gstride);
    if (!grid_barrier(gb, d)) return;
    if (S.n_col_scan <= kLocalScanMax) {
        ph_scan_local<int64_t>(S.col_cnt, S.col_pre, S.n_col_scan);
    } else if (!ph_scan<int64_t>(S.col_cnt, S.col_pre, S.n_col_scan, S.scan_tmp, bid, nblk, gb,
                                 d)) {
        return;
    }
    ph_clusters(S.cl, gid, gstride);
    if (!grid_barrier(gb, d)) return;
    // candidate tables and the slot repack read disjoint data: no barrier between
    ph_group_entries(S.en, s_dyn, bid, nblk);
    repack_range<4>(S.rp, gid, gstride, false);
    if (bid == 0 && threadIdx.x == 0) ph_build_done(d);
}

constexpr int kBuildStepPerCu = 1;

size_t build_step_lds_bytes(int E_cap)
{
    return (size_t)(kBuildStepThreads / (64 * kEntryWaves)) * kEntryWaves * E_cap *
           (sizeof(uint32_t) + 1);
}

hipError_t build_step_setup(Ctx* c)
{
    int occ = 0;
    (void)hipFuncSetAttribute((const void*)k_build_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)build_step_lds_bytes(c->E_cap));
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, (const void*)k_build_step, kBuildStepThreads, build_step_lds_bytes(c->E_cap));
    if (e != hipSuccess) {
        c->bs_blocks = 0;
        return e;
    }
    // one resident work-group of 1024 threads per CU: every grid barrier costs one
    // release (an L2 write-back) per work-group, while the latency-bound phases want
    // many waves (with 256-thread work-groups a forced-rebuild step took 0.70 ms at two
    // per CU, 0.79 ms at four, 0.75 ms at one)
    c->bs_blocks = occ > 0 ? std::min(c->n_cu * std::min(occ, kBuildStepPerCu), c->cap_bar) : 0;
    return hipSuccess;
}

void launch_build_step(Ctx* c, const double* x, const double* y, const double* z,
                       const uint8_t* type, const int8_t* q, bool force, hipStream_t st)
{
    StepBuildArgs S;
    const int nvb = vv_blocks(c->N);
    S.join = FastJoinArgs{c->d_partial + nvb + c->B + 1, c->d_fast_cnt, c->d_fast_loc,
                          c->d_fast_list, c->fast_cap, nvb, vv_block_size(), c->dsc};
    S.force = force ? 1 : 0;
    S.periodic = c->cfg.periodic;
    S.x = x; S.y = y; S.z = z;
    S.sys_off = c->d_sys_off; S.B = c->B; S.sys_lo = c->d_sys_lo; S.sys_hi = c->d_sys_hi;
    S.grid = c->d_grid;
    S.bin = BinArgs{c->N, x, y, z, c->d_sys_of_atom, c->d_grid, c->d_bin_cnt, c->d_key,
                    c->d_rank, c->d_img, c->d_xref, c->d_fast_flag, c->cap_bins, c->dsc, nullptr};
    S.sc = ScatterArgs{c->N, c->d_key, c->d_rank, c->d_bin_start, c->d_sorted, c->d_grid, c->B,
                       c->d_col_cnt, c->cap_cols, c->G, c->dsc, nullptr};
    S.cl = ClusterArgs{x, y, z, type, c->d_grid, c->B, c->d_bin_start, c->d_sorted,
                       c->d_col_pre, c->d_img, c->d_perm, c->d_inv_perm, c->d_slot_img, c->d_ts,
                       c->d_atype, c->d_xs, c->cap_slots, c->d_cl_lo, c->d_cl_hi, c->d_groups,
                       c->d_sys_grp0, c->cap_clusters, c->G, c->T, c->dsc, nullptr};
    S.en = EntryArgs{c->d_grid, c->d_col_pre, c->d_bin_start, c->d_cl_lo, c->d_cl_hi, c->d_groups, c->d_ent,
                     c->d_ent_mask, c->E_cap, c->rlist, c->dsc, nullptr};
    S.bin_cnt = c->d_bin_cnt; S.bin_start = c->d_bin_start; S.n_bin_scan = c->cap_bins + 1;
    S.col_cnt = c->d_col_cnt; S.col_pre = c->d_col_pre; S.n_col_scan = c->cap_cols + 1;
    S.scan_tmp = c->d_scan_tmp; S.sorted = c->d_sorted; S.cap_bins = c->cap_bins;
    S.rp = RepackArgs{x, y, z, q, c->d_perm, c->d_fast_flag, c->d_xs, c->d_qs, c->cap_slots,
                      c->dsc, c->d_slot_img, c->d_cl_lo, c->d_grid, c->d_sys_of_atom, c->B,
                      c->d_xo};
    S.bar_arrive = c->d_bar_arrive;
    S.dsc = c->dsc;
    hipLaunchKernelGGL(k_build_step, dim3(c->bs_blocks), dim3(kBuildStepThreads),
                       build_step_lds_bytes(c->E_cap), st, S);
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
