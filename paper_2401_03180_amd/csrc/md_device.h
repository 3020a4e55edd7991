// md_device.h -- device routines shared by the stand-alone kernels and the fused
// per-step build kernel (inline, so every translation unit has its own copy).
#pragma once

#include "md_internal.h"

namespace md {

// Grid-wide barrier for a persistent launch whose blocks are all resident at once.
// Every block publishes its writes (agent-scope release) and stores the barrier's
// epoch into its own arrival word (no contended atomics); the threads of block 0
// watch all arrival words, then store the epoch into the generation word, which
// the other blocks watch.  Epochs are gen0 + 1, gen0 + 2, ... where gen0 is the
// generation read at kernel start.  Waits are bounded (about half a second): a
// block that gives up latches MD_FLAG_BARRIER and the caller leaves the kernel,
// so no launch can hang; later barriers time out the same way.
struct GridBarrier {
    uint32_t* arrive;              // one word per block
    uint32_t* gen;
    unsigned nblk;
    unsigned epoch;                // epoch of the last barrier passed
};

__device__ inline bool bar_wait_ok(unsigned spins) { return spins <= (1u << 22); }

__device__ inline bool grid_barrier(GridBarrier& B, DevScalars* d)
{
    __shared__ int s_ok;
    const unsigned ep = B.epoch + 1u;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                          // release this block's writes
        __hip_atomic_store(&B.arrive[blockIdx.x], ep, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    if (blockIdx.x == 0) {
        // every thread watches a share of the arrival words
        unsigned spins = 0;
        for (unsigned k = threadIdx.x; k < B.nblk; k += blockDim.x) {
            while (__hip_atomic_load(&B.arrive[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                   ep) {
                __builtin_amdgcn_s_sleep(2);
                if (!bar_wait_ok(++spins)) { ok = 0; break; }
            }
            if (!ok) break;
        }
        ok = __syncthreads_and(ok);
        if (threadIdx.x == 0) {
            __threadfence();
            if (ok) __hip_atomic_store(B.gen, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(B.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep) {
            __builtin_amdgcn_s_sleep(4);
            if (!bar_wait_ok(++spins)) { ok = 0; break; }
        }
        __threadfence();                          // acquire the others' writes
    }
    if (threadIdx.x == 0) {
        if (!ok) atomicOr(&d->flags, MD_FLAG_BARRIER);
        s_ok = ok;
    }
    __syncthreads();
    B.epoch = ep;
    return s_ok != 0;
}

// exp(x) for x <= 0, the screening factor exp(-kappa r) of the FP64 pair terms, without
// the overflow handling of the general exp (Cody and Waite's method): x = n ln2 + t with
// n = rint(x / ln2) and ln2 in two parts (a head of 32 significant bits, so n ln2_hi is
// exact for |n| < 2^21), so |t| <= ln2 / 2; exp(t) from the degree-11 polynomial that
// interpolates exp at the 12 Chebyshev nodes of [-ln2/2, ln2/2] (interpolation error
// below 1e-17; the coefficients were computed in 60-digit arithmetic and rounded once);
// then one ldexp, which gives a subnormal or 0 below 2^-1022.  Within 0.8 ulp of exp
// on a dense sample of [-745, 0]; exp(-0) = exp(0) = 1 exactly.
__device__ inline double exp_nonpos64(double x)
{
    const double n = rint(x * 1.4426950408889634);
    double t = fma(-n, 0.6931471803691238, x);
    t = fma(-n, 1.9082149292705877e-10, t);
    double p = 2.5110037605963777e-08;
    p = fma(p, t, 2.763263963904103e-07);
    p = fma(p, t, 2.755724091857897e-06);
    p = fma(p, t, 2.4801485482328494e-05);
    p = fma(p, t, 0.00019841269890047113);
    p = fma(p, t, 0.0013888888952314775);
    p = fma(p, t, 0.008333333333319601);
    p = fma(p, t, 0.0416666666664881);
    p = fma(p, t, 0.1666666666666668);
    p = fma(p, t, 0.5000000000000019);
    p = fma(p, t, 1.0);
    p = fma(p, t, 1.0);
    return ldexp(p, (int)n);
}

// Hybrid ion-sphere / Debye potential of an ion of charge Q (section II.A, Eq. 4-7):
// h = {r', c1, c2, c3}; inside r' the ion-sphere form Q/r + c1 - c2 r^2, outside the
// Debye form c3 exp(-kappa r)/r (s = exp(-kappa r) is passed in).  Returns phi and
// w = -r dphi/dr.
__device__ inline void hyb_phi_w(double Q, const double* h, double kap, double r, double s,
                                 double& phi, double& w)
{
#pragma clang fp contract(off)
    if (r < h[0]) {
        phi = Q / r + h[1] - h[2] * r * r;
        w = Q / r + 2.0 * h[2] * r * r;
    } else {
        const double e = s / r;
        phi = h[3] * e;
        w = h[3] * e * (1.0 + kap * r);
    }
}

// FP64 pair terms with the hybrid Coulomb term k_e (q_b phi_a + q_a phi_b) / 2 and the
// Lennard-Jones term (screened by exp(-kappa r) when screen_lj): f multiplies
// d = p_a - p_b for the force on a; e is the pair energy.  hrow: the coefficient rows
// of charges 0 .. qn - 1 for this system and step.
__device__ inline void pair_terms_hybrid64(double r2, double kap, int qa, int qb, double c6,
                                           double c12, bool screen_lj, const double* hrow,
                                           int qn, double* f, double* e)
{
#pragma clang fp contract(off)
    const double r = sqrt(r2);
    const double rinv2 = 1.0 / r2;
    const double rinv6 = rinv2 * rinv2 * rinv2;
    const double s = exp_nonpos64(-kap * r);
    double pa = 0.0, wa = 0.0, pb = 0.0, wb = 0.0;
    if (qa > 0) hyb_phi_w((double)qa, hrow + 4 * min(qa, qn - 1), kap, r, s, pa, wa);
    if (qb > 0) hyb_phi_w((double)qb, hrow + 4 * min(qb, qn - 1), kap, r, s, pb, wb);
    const double uc = 0.5 * kKe * ((double)qb * pa + (double)qa * pb);
    const double wc = 0.5 * kKe * ((double)qb * wa + (double)qa * wb);
    const double l12 = c12 * rinv6 * rinv6, l6 = c6 * rinv6;
    const double ulj = l12 - l6, wlj = 12.0 * l12 - 6.0 * l6;
    if (screen_lj) {
        *e = uc + ulj * s;
        *f = (wc + (wlj + ulj * (kap * r)) * s) * rinv2;
    } else {
        *e = uc + ulj;
        *f = (wc + wlj) * rinv2;
    }
}

// Charge-scaled LJ radii (section II.B, Eq. 11) in FP64: each radius shrinks to
// c sigma with c = 1 - q/Z and the pair radius is the mean of the two, so c6 and c12
// scale by s^6 and s^12 with s = (c_a sigma_a + c_b sigma_b)/(sigma_a + sigma_b);
// no scaling when both radii are 0 (no LJ term).  tab: the kQljLen table.
__device__ inline void qlj_scale64(const double* tab, int ta, int tb, int qa, int qb, double* c6,
                                   double* c12)
{
#pragma clang fp contract(off)
    const double sa = tab[kQljSig + ta], sb = tab[kQljSig + tb];
    const double sum = sa + sb;
    if (!(sum > 0.0)) return;
    const double ca = 1.0 - (double)qa * tab[kQljInvZ + ta];
    const double cb = 1.0 - (double)qb * tab[kQljInvZ + tb];
    const double sc = (ca * sa + cb * sb) / sum;
    const double s6 = sc * sc * sc * sc * sc * sc;
    *c6 = *c6 * s6;
    *c12 = *c12 * s6 * s6;
}

// ---- the build grid: columns (x, y) with z bins, per system

__device__ inline int col_first_cluster(const int64_t* pre, int c)
{
    return (int)(pre[c] & 0xFFFFFFFFll);
}

// Distance from the point p to the interval [lo, hi] along one axis; periodic axes
// take the nearest image of p.
__device__ inline double axis_gap(double p, double lo, double hi, bool periodic, double L)
{
    double g = fmax(0.0, fmax(lo - p, p - hi));
    if (periodic) {
        g = fmin(g, fmax(0.0, fmax(lo - (p + L), (p + L) - hi)));
        g = fmin(g, fmax(0.0, fmax(lo - (p - L), (p - L) - hi)));
    }
    return g;
}

// Column index range along axis d (x or y) within `reach` of coordinate p.  Periodic
// ranges are in unwrapped column numbers (callers wrap them) and become every column
// when they would cover the axis (also for a non-finite p); vacuum ranges are clamped
// to the grid.  The range length never exceeds the column count.
__device__ inline void col_range(const GridSys& g, int d, double p, double reach, int* c0, int* c1)
{
    if (g.periodic) {
        const double w = p - g.L[d] * floor(p * g.invL[d]);
        const double a = floor((w - reach) * g.inv_w[d]);
        const double b = floor((w + reach) * g.inv_w[d]);
        if (!(b - a + 1.0 < (double)g.n[d]) || !(fabs(a) < 1e6) || !(fabs(b) < 1e6)) {
            *c0 = 0; *c1 = g.n[d] - 1;
        } else {
            *c0 = (int)a; *c1 = (int)b;
        }
    } else {
        const double w = p - g.origin[d];
        const double a = fmin(fmax(floor((w - reach) * g.inv_w[d]), 0.0), (double)(g.n[d] - 1));
        const double b = fmin(fmax(floor((w + reach) * g.inv_w[d]), 0.0), (double)(g.n[d] - 1));
        *c0 = (int)a; *c1 = (int)b;
    }
}

// z-bin ranges (up to two, for a periodic wrap) of column-local bins within
// `reach` of coordinate p; returns the number of ranges.
__device__ inline int zbin_ranges(const GridSys& g, double p, double reach, int r0[2], int r1[2])
{
    const int nz = g.n[2];
    if (g.periodic) {
        const double w = p - g.L[2] * floor(p * g.invL[2]);
        const double a = floor((w - reach) * g.inv_w[2]);
        const double b = floor((w + reach) * g.inv_w[2]);
        if (!(b - a + 1.0 < (double)nz) || !(fabs(a) < 1e6) || !(fabs(b) < 1e6)) {
            r0[0] = 0; r1[0] = nz - 1;
            return 1;
        }
        int lo = (int)a, hi = (int)b;
        if (lo < 0) {
            r0[0] = 0; r1[0] = hi;
            r0[1] = lo + nz; r1[1] = nz - 1;
            return 2;
        }
        if (hi >= nz) {
            r0[0] = lo; r1[0] = nz - 1;
            r0[1] = 0; r1[1] = hi - nz;
            return 2;
        }
        r0[0] = lo; r1[0] = hi;
        return 1;
    }
    const double w = p - g.origin[2];
    r0[0] = (int)fmin(fmax(floor((w - reach) * g.inv_w[2]), 0.0), (double)(nz - 1));
    r1[0] = (int)fmin(fmax(floor((w + reach) * g.inv_w[2]), 0.0), (double)(nz - 1));
    return 1;
}

// Sum of v over the block (every thread receives it); s holds one value per wave.
template <class T>
__device__ inline T block_sum_all(T v, T* s)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    T t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += s[k];
    return t;
}

// After phase 0 of velocity Verlet: join the per-block fast-atom lists (block
// order = ascending atom index) into the capped dense list, record the counts and
// the largest displacement, and advance the step counter.  One block (any size that
// is a multiple of 64, at most 1024).  Returns the uncapped fast count.
struct FastJoinArgs {
    const double* disp_partial;
    const int32_t* fast_cnt;
    const int32_t* fast_loc;       // per-block lists, stride loc_stride
    int32_t* fast_list;
    int fast_cap;
    int nblocks;
    int loc_stride;
    DevScalars* dsc;
};

__device__ inline int fast_join_block(const FastJoinArgs& A)
{
    __shared__ int s_w[16];
    __shared__ double s_m[16];
    const int nt = blockDim.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = nt >> 6;
    const int chunk = (A.nblocks + nt - 1) / nt;
    const int k0 = threadIdx.x * chunk, k1 = min(A.nblocks, k0 + chunk);
    double m = 0.0;
    int n = 0;
    for (int k = k0; k < k1; ++k) {
        m = fmax(m, A.disp_partial[k]);
        n += A.fast_cnt[k];
    }
    // exclusive prefix of the per-thread counts in thread order (= atom order)
    int inc = n;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wv] = inc;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) s_m[wv] = m;
    __syncthreads();
    int off = inc - n, total = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < wv) off += s_w[k];
        total += s_w[k];
    }
    for (int k = k0; k < k1 && off < A.fast_cap; ++k) {
        const int cnt = A.fast_cnt[k];
        for (int i = 0; i < cnt && off < A.fast_cap; ++i, ++off)
            A.fast_list[off] = A.fast_loc[(int64_t)k * A.loc_stride + i];
    }
    if (threadIdx.x == 0) {
        double mm = s_m[0];
        for (int k = 1; k < nt / 64; ++k) mm = fmax(mm, s_m[k]);
        const double prev = __longlong_as_double((long long)A.dsc->disp2_bits);
        A.dsc->disp2_bits = (unsigned long long)__double_as_longlong(fmax(prev, mm));
        A.dsc->n_fast_raw = total;
        A.dsc->n_fast = min(total, A.fast_cap);
        A.dsc->step += 1;
    }
    __syncthreads();
    return total;
}

// Gather positions and charges into slot order for the force kernels; fast atoms
// (moved more than skin/2 since the build) and padding slots get NaN positions.
struct RepackArgs {
    const double *x, *y, *z;
    const int8_t* q;
    const int32_t* perm;
    const uint8_t* fast_flag;
    double* xs;
    int8_t* qs;
    int64_t cap_slots;
    DevScalars* dsc;
    // FP32 staging copy: the position in the frame of the build (image removed) less
    // the low corner of the slot's cluster box, and the charge
    const int32_t* slot_img;
    const double* cl_lo;
    const GridSys* grid;
    const int32_t* sys_of_atom;    // (not read for a single system)
    int B;
    float4* xo;
};

// check_skin: latch MD_FLAG_SKIN when a rebuild is still pending (stale lists).
// U slots per thread and pass, each step's loads issued for all U together (the
// gathers through the permutation are latency-bound where few threads run).
template <int U>
__device__ inline void repack_range(const RepackArgs& A, int64_t gtid, int64_t gstride,
                                    bool check_skin)
{
    const int64_t n = A.dsc->n_slots;
    if (gtid == 0) {
        A.dsc->work_force = 0u;
        if (check_skin && A.dsc->need_rebuild) atomicOr(&A.dsc->flags, MD_FLAG_SKIN);
    }
    for (int64_t s0 = gtid; s0 < n; s0 += U * gstride) {
        int a[U];
        bool live[U];
        double p[U][3];
        int8_t qa[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t s = s0 + u * gstride;
            a[u] = s < n ? A.perm[s] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            live[u] = a[u] >= 0 && !A.fast_flag[a[u]];
            qa[u] = a[u] >= 0 ? A.q[a[u]] : (int8_t)0;
            p[u][0] = live[u] ? A.x[a[u]] : NAN;
            p[u][1] = live[u] ? A.y[a[u]] : NAN;
            p[u][2] = live[u] ? A.z[a[u]] : NAN;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t s = s0 + u * gstride;
            if (s >= n) break;
            A.xs[s] = p[u][0];
            A.xs[A.cap_slots + s] = p[u][1];
            A.xs[2 * A.cap_slots + s] = p[u][2];
            A.qs[s] = qa[u];
            if (live[u]) {
                const GridSys& g = A.grid[A.B == 1 ? 0 : A.sys_of_atom[a[u]]];
                const int32_t im = A.slot_img[s];
                const double* lo = A.cl_lo + (s / kCluster) * 3;
                float o[3];
                for (int d = 0; d < 3; ++d) {
                    const double w =
                        g.periodic ? p[u][d] - (double)unpack_img(im, d) * g.L[d] : p[u][d];
                    o[d] = (float)(w - lo[d]);
                }
                A.xo[s] = make_float4(o[0], o[1], o[2], (float)qa[u]);
            } else {
                // x alone marks the slot empty (the force kernel's staging tests it)
                A.xo[s] = make_float4(NAN, 0.0f, 0.0f, (float)qa[u]);
            }
        }
    }
}

// One block after the force kernels: the per-system energy as the sum of the group
// energies and of the fast atoms' pair energies in a fixed order (deterministic),
// and the end of a pending list rebuild.
struct ForceFinalizeArgs {
    const double* grp_epot;
    double* epot;                  // NULL: no energy requested
    const int32_t* sys_grp0;
    int B;
    const int32_t* fast_list;
    const double* fast_e;
    const int64_t* sys_off;
    DevScalars* dsc;
    const double* bond_e;          // per-atom bonded energies (NULL: no bonded terms)
    const double* bond_blk;        // their sums per work-group of bonded_block atoms
    int bonded_block;
    int64_t N;
};

// Work-groups that sum the per-system energies of a batch (one per system up to this
// many; each takes every kFinMax-th system): one work-group took ~2.8 us per system
// in turn, 0.7 ms per step for 256 systems.
constexpr int kFinMax = 64;
inline __host__ __device__ int fin_blocks(int B) { return B < 1 ? 1 : (B < kFinMax ? B : kFinMax); }

// b_first, b_stride: the systems this work-group sums (several work-groups share a
// batch of many systems; each system's sum is the same whichever takes it).
__device__ inline void force_finalize_block(const ForceFinalizeArgs& F, int b_first = 0,
                                            int b_stride = 1)
{
    __shared__ double s_red[16];
    if (F.epot) {
        const int nf = F.dsc->n_fast;
        const int nw = blockDim.x >> 6;
        for (int b = b_first; b < F.B; b += b_stride) {
            const int g0 = F.sys_grp0[b], g1 = F.sys_grp0[b + 1];
            // the group energies in passes of 16 per thread (16 loads in flight
            // together) into 16 partial sums, then the rest one at a time; combined
            // in a fixed order
            constexpr int U = 16;
            double tu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) tu[u] = 0.0;
            const int nt = blockDim.x;
            int g = g0 + threadIdx.x;
            for (; g + (U - 1) * nt < g1; g += U * nt) {
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = F.grp_epot[g + u * nt];
#pragma unroll
                for (int u = 0; u < U; ++u) tu[u] += v[u];
            }
            double rest = 0.0;
            for (; g < g1; g += nt) rest += F.grp_epot[g];
#pragma unroll
            for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
                for (int u = 0; u < w; ++u) tu[u] += tu[u + w];
            double t = tu[0] + rest;
            const int64_t a0 = F.sys_off[b], a1 = F.sys_off[b + 1];
            for (int k = threadIdx.x; k < nf; k += blockDim.x) {
                const int f = F.fast_list[k];
                if (f >= a0 && f < a1) t += F.fast_e[k];
            }
            if (F.bond_e && a1 > a0) {
                // whole bonded work-groups inside the system by their sums, the (at
                // most two) that straddle its ends atom by atom
                const int64_t bb = F.bonded_block;
                for (int64_t k = a0 / bb + threadIdx.x; k <= (a1 - 1) / bb; k += blockDim.x) {
                    const int64_t lo = k * bb, hi = min(lo + bb, F.N);
                    if (lo >= a0 && hi <= a1) {
                        t += F.bond_blk[k];
                    } else {
                        for (int64_t a = max(lo, a0); a < min(hi, a1); ++a) t += F.bond_e[a];
                    }
                }
            }
            for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
            __syncthreads();
            if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = t;
            __syncthreads();
            if (threadIdx.x == 0) {
                double e = 0.0;
                for (int w = 0; w < nw; ++w) e += s_red[w];
                F.epot[b] = e;
            }
        }
    }
    if (threadIdx.x == 0 && b_first == 0) F.dsc->lists_pending = 0;
}

}  // namespace md
