// md_rdf.hip -- pair-distance histograms for the radial distribution functions
// g_ab(r) behind the partial structure factors (arXiv 2401.03180, section II.C,
// Eq. 18).
//
// Counts every unordered pair {i, j} of one system whose minimum-image distance
// (the FP64 expression of the cutoff predicate) is below r_max, in bin k when
// (k dr)^2 <= r^2 < ((k + 1) dr)^2, under the element pair (min, max).  Exact
// integer counts, independent of the launch configuration.
//
// The search reuses the last neighbour build: every atom sits in the z bin of its
// build position.  An atom that has moved at most skin/2 since the build is found
// by scanning, around the other atom's current position, the bins within
// r_max + skin/2; pairs with an atom that has moved farther ("moved" here, judged
// from the positions passed in) are counted by a brute-force pass over its system.
// The current positions are first gathered into slot order (NaN for moved atoms and
// padding), so that the scans of neighbouring slots read the same cache lines.
#include <mutex>

#include "md_device.h"
#include "md_internal.h"
#include "md_launch.h"

namespace md {

// Workspace of the no-allocation histogram entry point: one fixed array per device
// (the code object's copy on that device), held until the process ends.  Host code
// never takes this name as an address: rdf_scratch_setup asks the runtime for the
// array's device address once per device and the launch passes that pointer.
static __device__ __align__(256) unsigned char scratch[kRdfScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
bool g_scratch_done[kScratchDevices] = {};
}  // namespace

size_t rdf_scratch_bytes(int64_t N, int64_t cap_slots)
{
    const size_t xr = ((size_t)cap_slots * 3 * sizeof(double) + 255) & ~(size_t)255;
    const size_t er = ((size_t)cap_slots + 255) & ~(size_t)255;
    return xr + er + (size_t)N;
}

hipError_t rdf_scratch_setup(int device)
{
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return g_scratch_ptr[device] ? hipSuccess : hipErrorInvalidSymbol;
    g_scratch_done[device] = true;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void* rdf_scratch(int device)
{
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

constexpr int kRdfBlock = 256;
constexpr int kRdfSplit = 8;         // threads sharing one slot's scan (latency hiding)

struct RdfArgs {
    const double *x, *y, *z;       // current positions (caller order)
    const uint8_t* elem;
    const double* xref;            // build positions, SoA stride N
    const int32_t* sys_of_atom;
    const int64_t* sys_off;
    const GridSys* grid;
    const int64_t* col_pre;
    const int32_t* bin_start;
    const int32_t* perm;
    DevScalars* dsc;
    int64_t N;
    int E;
    int n_bins;
    double dr;                     // r_max / n_bins
    double reach;                  // r_max + skin/2
    double thr2;                   // (skin/2)^2
    uint8_t* moved;                // per atom
    double* xr;                    // slot-order current positions (SoA, stride cap_slots)
    uint8_t* er;                   // slot-order elements
    int64_t cap_slots;
    unsigned long long* hist;      // [B][E][E][n_bins]
    int lds_hist;                  // per-block LDS histogram when the block is one system
};

// Squared bin edges e2[k] = (k dr)^2, k = 0 .. n, in LDS.
__device__ inline void fill_edges(double* e2, int n, double dr)
{
#pragma clang fp contract(off)
    for (int k = threadIdx.x; k <= n; k += blockDim.x) {
        const double e = (double)k * dr;
        e2[k] = e * e;
    }
}

// Bin of r2 (0 <= r2 < e2[n]): k with e2[k] <= r2 < e2[k + 1].
__device__ inline int rdf_bin(double r2, const double* e2, int n, double inv_dr)
{
    int k = (int)(sqrt(r2) * inv_dr);
    k = min(max(k, 0), n - 1);
    while (k > 0 && r2 < e2[k]) --k;
    while (k < n - 1 && r2 >= e2[k + 1]) ++k;
    return k;
}

__device__ inline int64_t hist_index(const RdfArgs& A, int b, int ea, int eb, int k)
{
    const int lo = min(ea, eb), hi = max(ea, eb);
    return (((int64_t)b * A.E + lo) * A.E + hi) * A.n_bins + k;
}

// Per slot: the atom's "moved" flag (farther than skin/2 from its build position,
// or a position that is not finite) and its current position in slot order (NaN
// when moved, and for padding slots).
__global__ void __launch_bounds__(kRdfBlock) k_rdf_gather(RdfArgs A)
{
#pragma clang fp contract(off)
    const int64_t s = blockIdx.x * (int64_t)kRdfBlock + threadIdx.x;
    if (s >= A.cap_slots) return;
    const int a = s < A.dsc->n_slots ? A.perm[s] : -1;
    double p[3] = {NAN, NAN, NAN};
    uint8_t e = 0;
    if (a >= 0) {
        p[0] = A.x[a]; p[1] = A.y[a]; p[2] = A.z[a];
        const double ex = p[0] - A.xref[a];
        const double ey = p[1] - A.xref[A.N + a];
        const double ez = p[2] - A.xref[2 * A.N + a];
        double d2 = ex * ex + ey * ey;
        d2 = d2 + ez * ez;
        const uint8_t mv = (d2 <= A.thr2) ? 0 : 1;
        A.moved[a] = mv;
        if (mv) p[0] = p[1] = p[2] = NAN;
        e = A.elem[a];
    }
    A.xr[s] = p[0];
    A.xr[A.cap_slots + s] = p[1];
    A.xr[2 * A.cap_slots + s] = p[2];
    A.er[s] = e;
}

// Pairs of two atoms that have not moved: kRdfSplit threads per slot i share the
// scan of the bins within reach of i (each takes every kRdfSplit-th candidate) and
// count partners in slots j > i (a moved or padding slot has a NaN position, so its
// distances fail the range test).
__global__ void __launch_bounds__(kRdfBlock) k_rdf_grid(RdfArgs A)
{
    extern __shared__ double s_dyn[];
    double* e2 = s_dyn;                                              // n_bins + 1
    unsigned* s_h = reinterpret_cast<unsigned*>(s_dyn + A.n_bins + 1); // E*E*n_bins
    const int n = A.n_bins;
    const int64_t n_slots = A.dsc->n_slots;
    constexpr int kSlotsPerBlock = kRdfBlock / kRdfSplit;
    const int64_t s0b = blockIdx.x * (int64_t)kSlotsPerBlock;
    if (s0b >= n_slots) return;                                      // block-uniform
    const int64_t i = s0b + threadIdx.x / kRdfSplit;
    const int sub = threadIdx.x % kRdfSplit;
    // the block's system when all its slots belong to one (slots are system-major)
    const int64_t last = min(s0b + kSlotsPerBlock, n_slots) - 1;
    int pf = -1, pl = -1;
    for (int64_t t = s0b; t <= last && pf < 0; ++t) pf = A.perm[t];
    for (int64_t t = last; t >= s0b && pl < 0; --t) pl = A.perm[t];
    const int bfirst = pf >= 0 ? A.sys_of_atom[pf] : 0, blast = pl >= 0 ? A.sys_of_atom[pl] : 0;
    const bool lds = A.lds_hist && bfirst == blast;                  // block-uniform
    const int nh = A.E * A.E * n;
    fill_edges(e2, n, A.dr);
    if (lds)
        for (int k = threadIdx.x; k < nh; k += blockDim.x) s_h[k] = 0u;
    __syncthreads();
    const double inv_dr = 1.0 / A.dr;
    const double r2max = e2[n];
    const int64_t cs = A.cap_slots;
    const double xi = i < n_slots ? A.xr[i] : NAN;
    const bool live = xi == xi;
    int b = 0, ei = 0;
    double yi = 0.0, zi = 0.0;
    GridSys gs{};
    int cx0 = 0, cx1 = -1, cy0 = 0, cy1 = -1, nzr = 0;
    int zr0[2] = {0, 0}, zr1[2] = {-1, -1};
    if (live) {
        b = A.sys_of_atom[A.perm[i]];
        gs = A.grid[b];
        ei = A.er[i];
        yi = A.xr[cs + i]; zi = A.xr[2 * cs + i];
        col_range(gs, 0, xi, A.reach, &cx0, &cx1);
        col_range(gs, 1, yi, A.reach, &cy0, &cy1);
        nzr = zbin_ranges(gs, zi, A.reach, zr0, zr1);
    }
    const int ncy = cy1 - cy0 + 1;
    const int npairs = live ? (cx1 - cx0 + 1) * ncy * nzr : 0;
    for (int p = 0; p < npairs; ++p) {
        const int r = p % nzr, cc = p / nzr;
        const int cx = cx0 + cc / ncy, cy = cy0 + cc % ncy;
        const int wx = gs.periodic ? ((cx % gs.n[0]) + gs.n[0]) % gs.n[0] : cx;
        const int wy = gs.periodic ? ((cy % gs.n[1]) + gs.n[1]) % gs.n[1] : cy;
        const int col = gs.col_off + wx * gs.n[1] + wy;
        const int64_t slot0 = (int64_t)col_first_cluster(A.col_pre, col) * kCluster;
        const int bin0 = gs.bin_off + (col - gs.col_off) * gs.n[2];
        const int a_col = A.bin_start[bin0];
        const int64_t s0 = max(slot0 + (A.bin_start[bin0 + zr0[r]] - a_col), i + 1);
        const int64_t s1 = min(slot0 + (A.bin_start[bin0 + zr1[r] + 1] - a_col), n_slots);
        for (int64_t s = s0 + sub; s < s1; s += kRdfSplit) {   // each pair once: slot j > slot i
            const double r2 = pair_r2_exact(xi, yi, zi, A.xr[s], A.xr[cs + s], A.xr[2 * cs + s], gs);
            if (!(r2 < r2max)) continue;                 // also NaN: moved or padding
            const int k = rdf_bin(r2, e2, n, inv_dr);
            const int ej = A.er[s];
            if (lds)
                atomicAdd(&s_h[(min(ei, ej) * A.E + max(ei, ej)) * n + k], 1u);
            else
                atomicAdd(&A.hist[hist_index(A, b, ei, ej, k)], 1ull);
        }
    }
    if (lds) {
        __syncthreads();
        for (int k = threadIdx.x; k < nh; k += blockDim.x)
            if (s_h[k]) atomicAdd(&A.hist[(int64_t)bfirst * nh + k], (unsigned long long)s_h[k]);
    }
}

// Pairs with at least one moved atom: the moved atoms of this block, one after
// another, each against every atom of its system (a pair of two moved atoms is
// counted by the smaller index).
__global__ void __launch_bounds__(kRdfBlock) k_rdf_moved(RdfArgs A)
{
    extern __shared__ double s_dyn[];
    double* e2 = s_dyn;
    __shared__ int s_list[kRdfBlock];
    __shared__ int s_cnt[kRdfBlock / 64];
    const int n = A.n_bins;
    const int64_t i0 = blockIdx.x * (int64_t)kRdfBlock + threadIdx.x;
    const bool mv = i0 < A.N && A.moved[i0];
    const unsigned long long bal = __ballot(mv);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_cnt[w] = __popcll(bal);
    __syncthreads();
    int pos = __popcll(bal & ((1ull << lane) - 1ull)), nm = 0;
    for (int v = 0; v < (int)(blockDim.x >> 6); ++v) {
        if (v < w) pos += s_cnt[v];
        nm += s_cnt[v];
    }
    if (nm == 0) return;                                 // block-uniform
    if (mv) s_list[pos] = (int)i0;
    fill_edges(e2, n, A.dr);
    __syncthreads();
    const double inv_dr = 1.0 / A.dr;
    const double r2max = e2[n];
    for (int t = 0; t < nm; ++t) {
        const int i = s_list[t];
        const int b = A.sys_of_atom[i];
        const GridSys gs = A.grid[b];
        const int ei = A.elem[i];
        const double xi = A.x[i], yi = A.y[i], zi = A.z[i];
        const int64_t j0 = A.sys_off[b], j1 = A.sys_off[b + 1];
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            if (j == i || (A.moved[j] && j < i)) continue;
            const double r2 = pair_r2_exact(xi, yi, zi, A.x[j], A.y[j], A.z[j], gs);
            if (!(r2 < r2max)) continue;
            const int k = rdf_bin(r2, e2, n, inv_dr);
            atomicAdd(&A.hist[hist_index(A, b, ei, A.elem[j], k)], 1ull);
        }
    }
}

size_t rdf_lds_bytes(int E, int n_bins, bool with_hist)
{
    return (size_t)(n_bins + 1) * sizeof(double) +
           (with_hist ? (size_t)E * E * n_bins * sizeof(unsigned) : 0);
}

void launch_rdf(Ctx* c, const double* x, const double* y, const double* z, const uint8_t* elem,
                double r_max, int n_bins, unsigned long long* hist, uint8_t* moved, double* xr,
                uint8_t* er, hipStream_t st)
{
    RdfArgs A;
    A.x = x; A.y = y; A.z = z; A.elem = elem; A.xref = c->d_xref;
    A.sys_of_atom = c->d_sys_of_atom; A.sys_off = c->d_sys_off; A.grid = c->d_grid;
    A.col_pre = c->d_col_pre; A.bin_start = c->d_bin_start; A.perm = c->d_perm; A.dsc = c->dsc;
    A.N = c->N; A.E = c->E; A.n_bins = n_bins;
    A.dr = r_max / (double)n_bins;
    A.reach = r_max + 0.5 * c->cfg.skin;
    A.thr2 = 0.25 * c->cfg.skin * c->cfg.skin;
    A.moved = moved;
    A.xr = xr;
    A.er = er;
    A.cap_slots = c->cap_slots;
    A.hist = hist;
    const size_t with = rdf_lds_bytes(c->E, n_bins, true);
    A.lds_hist = with <= kRdfLdsMax ? 1 : 0;
    const int nb = (int)div_up(c->N, kRdfBlock);
    const int ns = (int)div_up(c->cap_slots, kRdfBlock);
    const int ng = (int)div_up(c->cap_slots, kRdfBlock / kRdfSplit);
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_rdf_gather, dim3(ns), dim3(kRdfBlock), 0, st, A);
    hipLaunchKernelGGL(k_rdf_grid, dim3(ng), dim3(kRdfBlock),
                       A.lds_hist ? with : rdf_lds_bytes(c->E, n_bins, false), st, A);
    hipLaunchKernelGGL(k_rdf_moved, dim3(nb), dim3(kRdfBlock), rdf_lds_bytes(c->E, n_bins, false),
                       st, A);
}

}  // namespace md
