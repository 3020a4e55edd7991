// md_step.hip -- element-wise per-step kernels: ionization, velocity Verlet,
// slot repacking, and the generic scan / fill utilities used by the build.
#include "md_device.h"
#include "md_internal.h"
#include "md_launch.h"

namespace md {

// ------------------------------------------------------------------ utilities

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>(div_up(n, 256), 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, st, p, n, v);
}

// Exclusive prefix sum within a block of kScanBlock threads, kScanPerThread values
// per thread.  Returns the block total.
template <class T>
__device__ T block_scan_exclusive(T (&v)[kScanPerThread], T* s_warp)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    T t = 0;
    for (int k = 0; k < kScanPerThread; ++k) { T x = v[k]; v[k] = t; t += x; }
    // inclusive scan of per-thread totals across the wave
    T inc = t;
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) s_warp[wv] = inc;
    __syncthreads();
    if (wv == 0) {
        int nw = blockDim.x >> 6;
        T x = lane < nw ? s_warp[lane] : (T)0;
        T xi = x;
        for (int off = 1; off < 64; off <<= 1) {
            T y = __shfl_up(xi, off, 64);
            if (lane >= off) xi += y;
        }
        if (lane < nw) s_warp[lane] = xi - x;       // exclusive wave offsets
        if (lane == nw - 1) s_warp[64] = xi;         // block total
    }
    __syncthreads();
    T base = s_warp[wv] + (inc - t);
    for (int k = 0; k < kScanPerThread; ++k) v[k] += base;
    T total = s_warp[64];
    __syncthreads();
    return total;
}

// `gate` (device int, may be NULL): the scan kernels do nothing when *gate == 0.
template <class T>
__global__ void __launch_bounds__(kScanBlock) k_scan_local(const T* in, T* out, int64_t n,
                                                           T* block_sums, const int32_t* gate)
{
    if (gate && *gate == 0) return;
    __shared__ T s_warp[65];
    T v[kScanPerThread];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    for (int k = 0; k < kScanPerThread; ++k) v[k] = (base + k < n) ? in[base + k] : (T)0;
    T total = block_scan_exclusive<T>(v, s_warp);
    for (int k = 0; k < kScanPerThread; ++k)
        if (base + k < n) out[base + k] = v[k];
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

template <class T>
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(T* block_sums, int nb,
                                                          const int32_t* gate)
{
    if (gate && *gate == 0) return;
    __shared__ T s_warp[65];
    T v[kScanPerThread];
    int base = threadIdx.x * kScanPerThread;
    for (int k = 0; k < kScanPerThread; ++k) v[k] = (base + k < nb) ? block_sums[base + k] : (T)0;
    block_scan_exclusive<T>(v, s_warp);
    for (int k = 0; k < kScanPerThread; ++k)
        if (base + k < nb) block_sums[base + k] = v[k];
}

template <class T>
__global__ void __launch_bounds__(kScanBlock) k_scan_add(T* out, int64_t n, const T* block_sums,
                                                         const int32_t* gate)
{
    if (gate && *gate == 0) return;
    T add = block_sums[blockIdx.x];
    if (add == 0) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    for (int k = 0; k < kScanPerThread; ++k)
        if (base + k < n) out[base + k] += add;
}

// Exclusive scan of in[0..n) into out[0..n).  n <= kScanTile^2; tmp holds kScanTile
// values of type T.
template <class T>
static void scan_impl(const T* in, T* out, int64_t n, T* tmp, const int32_t* gate, hipStream_t st)
{
    if (n <= 0) return;
    int nb = (int)div_up(n, kScanTile);
    hipLaunchKernelGGL(k_scan_local<T>, dim3(nb), dim3(kScanBlock), 0, st, in, out, n, tmp, gate);
    if (nb > 1) {
        hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanBlock), 0, st, tmp, nb, gate);
        hipLaunchKernelGGL(k_scan_add<T>, dim3(nb), dim3(kScanBlock), 0, st, out, n, tmp, gate);
    }
}

void launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, const int32_t* gate,
                 hipStream_t st)
{
    scan_impl<int32_t>(in, out, n, tmp, gate, st);
}

void launch_scan64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, const int32_t* gate,
                   hipStream_t st)
{
    scan_impl<int64_t>(in, out, n, tmp, gate, st);
}

// ------------------------------------------------------------------ Philox4x32-10

// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of
// two 32x32->64 multiplications with the round key bumped by the Weyl constants
// between rounds.  Returns word 0 of the output block.
__device__ inline uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
        const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0; c1 = loB; c2 = n2; c3 = loA;
        k0 += kWeylA; k1 += kWeylB;
    }
    return c0;
}

// ------------------------------------------------------------------ ionization

struct IonArgs {
    int64_t N;
    const int32_t* sys_of_atom;
    const uint8_t* elem;
    const uint32_t* atom_id;
    int8_t* q;
    const int8_t* qmax;
    const double* base;
    int32_t E, Q;
    const double* g;
    int64_t S1;
    const uint64_t* seeds;
    DevScalars* dsc;
};

// Ionization of atom a at step s (1 <= s < S1).
__device__ inline void ionize_one(const IonArgs& A, int64_t a, int64_t s)
{
    const int e = A.elem[a];
    const int qa = A.q[a];
    if (e >= A.E || qa < 0 || qa >= A.Q) {
        set_flag(A.dsc, MD_FLAG_BAD_INPUT);
        return;
    }
    if (qa >= A.qmax[e]) return;
    const int b = A.sys_of_atom[a];
    double p = A.base[e * A.Q + qa] * A.g[b * A.S1 + s];
    p = p > 1.0 ? 1.0 : p;
    const uint64_t thresh = (uint64_t)floor(p * 4294967296.0);
    const uint64_t seed = A.seeds[b];
    const uint32_t u = philox_word0(A.atom_id[a], (uint32_t)s, (uint32_t)b, 0u, (uint32_t)seed,
                                    (uint32_t)(seed >> 32));
    if ((uint64_t)u < thresh) A.q[a] = (int8_t)(qa + 1);
}

__global__ void __launch_bounds__(256) k_ionize(IonArgs A)
{
    const int64_t s = A.dsc->step;
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= A.N) return;
    if (s < 1 || s >= A.S1) {
        if (a == 0) set_flag(A.dsc, MD_FLAG_STEP);
        return;
    }
    ionize_one(A, a, s);
}

static IonArgs ion_args(Ctx* c, const uint8_t* elem, const uint32_t* atom_id, int8_t* q)
{
    return IonArgs{c->N, c->d_sys_of_atom, elem, atom_id, q, c->d_qmax, c->d_base, c->E, c->Q,
                   c->d_g, c->n_steps + 1, c->d_seeds, c->dsc};
}

void launch_ionize(Ctx* c, const uint8_t* elem, const uint32_t* atom_id, int8_t* q,
                   hipStream_t st)
{
    if (c->N == 0) return;
    hipLaunchKernelGGL(k_ionize, dim3(div_up(c->N, 256)), dim3(256), 0, st,
                       ion_args(c, elem, atom_id, q));
}

// ------------------------------------------------------------------ velocity Verlet


struct VvArgs {
    int64_t N;
    double dt, hdt, thr2;
    const double* inv_mass;
    const double *fx, *fy, *fz;
    double *x, *y, *z, *vx, *vy, *vz;
    const double* xref;          // N*3 build positions
    double* partial;             // nblocks + B (kinetic-energy partials)
    unsigned long long* ek_slots;   // the same as atomic words (fused phase 1), or NULL
    double* disp_partial;        // nblocks (displacement maxima)
    double* ekin;
    const int64_t* sys_off;
    const int32_t* sys_of_atom;
    int B;
    DevScalars* dsc;
    uint8_t* fast_flag;          // N
    int32_t* fast_loc;           // nblocks * kVvBlock
    int32_t* fast_cnt;           // nblocks
    int32_t* fast_list;          // fast_cap
    int fast_cap;
};

__device__ double block_sum_d(double v, double* s)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += s[k];
    return t;   // valid in thread 0
}

// Langevin coupling tables and per-atom inputs (phase 0 only).
struct LgArgs {
    const double* c1;              // B*E
    const double* kt;              // B*S1
    int E;
    int64_t S1;
    const uint8_t* elem;
    const uint32_t* atom_id;
    const uint64_t* seeds;
    const int32_t* sys_of_atom;
};

// Three standard normals for (atom_id, step s, system b): Philox4x32-10 with counter
// (atom_id, s, b, 1), Box-Muller in FP64 on words (0, 1) and (2, 3).
__device__ inline void langevin_normals(uint32_t id, uint32_t s, uint32_t b, uint64_t seed,
                                        double z[3])
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
    uint32_t c0 = id, c1 = s, c2 = b, c3 = 1u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
        const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0; c1 = loB; c2 = n2; c3 = loA;
        k0 += kWeylA; k1 += kWeylB;
    }
    const double two_pi = 6.283185307179586;
    const double scale = 2.3283064365386963e-10;
    const double u0 = ((double)c0 + 0.5) * scale, u1 = ((double)c1 + 0.5) * scale;
    const double u2 = ((double)c2 + 0.5) * scale, u3 = ((double)c3 + 0.5) * scale;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    z[0] = r0 * cos(two_pi * u1);
    z[1] = r0 * sin(two_pi * u1);
    z[2] = r1 * cos(two_pi * u3);
}

constexpr unsigned long long kEkSlotEmpty = ~0ull;   // a NaN no arithmetic produces


// Phase 1 of the fused step: an extra work-group sums the kinetic-energy partials of
// its systems (b_first, b_first + b_stride, ...) in the order of the finalize kernel
// (so the result is the same), waiting for each block's word, and empties the words
// for the next launch (the systems' words are disjoint).  A wait that does not end
// latches MD_FLAG_BARRIER (the step's results are then not to be trusted, as after any
// latched error).
__device__ void ekin_from_slots(const VvArgs& A, double* s_red, int b_first, int b_stride)
{
    for (int b = b_first; b < A.B; b += b_stride) {
        const int64_t s0 = A.sys_off[b], s1 = A.sys_off[b + 1];
        double t = 0.0;
        if (s1 > s0) {
            const int64_t k0 = s0 / kVvBlock, k1 = (s1 - 1) / kVvBlock;
            // 16 words per thread read together (whole passes; the rest one at a
            // time), then each one waited for in turn and added in the same order as
            // one at a time
            constexpr int U = 16;
            for (int64_t kb = k0 + threadIdx.x; kb <= k1; kb += U * kVvBlock) {
                const int nu = kb + (U - 1) * kVvBlock <= k1 ? U : 1;
                unsigned long long v[U];
                if (nu == U) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        v[u] = __hip_atomic_load(A.ek_slots + kb + u * kVvBlock + b,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t k = kb + u * kVvBlock;
                    if (k > k1) break;
                    unsigned long long* w = A.ek_slots + k + b;
                    if (nu != U)
                        v[u] = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    unsigned spins = 0;
                    while (v[u] == kEkSlotEmpty) {
                        __builtin_amdgcn_s_sleep(2);
                        v[u] = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (++spins > (1u << 22)) {
                            atomicOr(&A.dsc->flags, MD_FLAG_BARRIER);
                            v[u] = 0ull;
                            break;
                        }
                    }
                    t += __longlong_as_double((long long)v[u]);
                    __hip_atomic_store(w, kEkSlotEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        t = block_sum_d(t, s_red);
        if (threadIdx.x == 0) A.ekin[b] = t;
    }
}

// IONIZE (phase 0 only): also the ionization of the step this phase starts (the
// step counter is advanced after this kernel), as md_step issues it.  FIN (phase 1
// only): fin_blocks(B) extra work-groups (the first) run the force finalize of the
// step, each for its share of the systems.  LANGEVIN (phase 0 only): the drift is split
// around the exact friction + noise velocity update.
template <int PHASE, bool EKIN, bool IONIZE = false, bool FIN = false, bool LANGEVIN = false>
__global__ void __launch_bounds__(kVvBlock) k_vv(VvArgs A, IonArgs I, ForceFinalizeArgs F,
                                                 LgArgs L)
{
#pragma clang fp contract(off)
    __shared__ double s_red[kVvBlock / 64];
    // FIN: the first work-groups (dispatched first) sum the group energies of their
    // systems while the others integrate, then wait for those systems' kinetic-energy
    // words; the others take the atoms
    const int nfin = FIN ? fin_blocks(A.B) : 0;
    if (FIN && (int)blockIdx.x < nfin) {
        force_finalize_block(F, (int)blockIdx.x, nfin);
        if (EKIN && A.ek_slots) ekin_from_slots(A, s_red, (int)blockIdx.x, nfin);
        return;
    }
    const int bi = (int)blockIdx.x - nfin;                           // atom block
    const int64_t a = bi * (int64_t)kVvBlock + threadIdx.x;
    double d2 = 0.0, ke = 0.0;
    if (IONIZE && a < A.N) {
        const int64_t s = A.dsc->step + 1;
        if (s >= 1 && s < I.S1) ionize_one(I, a, s);
        else if (a == 0) set_flag(A.dsc, MD_FLAG_STEP);
    }
    if (a < A.N) {
        const double h = A.hdt * A.inv_mass[a];
        double vx = A.vx[a] + h * A.fx[a];
        double vy = A.vy[a] + h * A.fy[a];
        double vz = A.vz[a] + h * A.fz[a];
        if (PHASE == 0 && LANGEVIN) {
            const int b = L.sys_of_atom[a];
            const int64_t s = A.dsc->step + 1;
            const int64_t sk = s < 0 ? 0 : (s >= L.S1 ? L.S1 - 1 : s);
            const double c1 = L.c1[b * L.E + L.elem[a]];
            const double sig = sqrt(L.kt[b * L.S1 + sk] * (1.0 - c1 * c1) * A.inv_mass[a]);
            double g[3];
            langevin_normals(L.atom_id[a], (uint32_t)s, (uint32_t)b, L.seeds[b], g);
            double p[3] = {A.x[a], A.y[a], A.z[a]};
            double v[3] = {vx, vy, vz};
            for (int d = 0; d < 3; ++d) {
                p[d] = p[d] + A.hdt * v[d];
                v[d] = c1 * v[d] + sig * g[d];
                p[d] = p[d] + A.hdt * v[d];
            }
            vx = v[0]; vy = v[1]; vz = v[2];
            A.x[a] = p[0]; A.y[a] = p[1]; A.z[a] = p[2];
        }
        A.vx[a] = vx; A.vy[a] = vy; A.vz[a] = vz;
        if (PHASE == 0) {
            double x, y, z;
            if (LANGEVIN) {
                x = A.x[a]; y = A.y[a]; z = A.z[a];
            } else {
                x = A.x[a] + A.dt * vx;
                y = A.y[a] + A.dt * vy;
                z = A.z[a] + A.dt * vz;
                A.x[a] = x; A.y[a] = y; A.z[a] = z;
            }
            const double ex = x - A.xref[a], ey = y - A.xref[A.N + a], ez = z - A.xref[2 * A.N + a];
            d2 = ex * ex + ey * ey + ez * ez;
            A.fast_flag[a] = d2 > A.thr2 ? 1 : 0;
        } else if (EKIN) {
            double v2 = vx * vx + vy * vy;
            v2 = v2 + vz * vz;
            ke = 0.5 * v2 / A.inv_mass[a];
        }
    }
    if (PHASE == 0) {
        // this block's fast atoms in atom order, and the block maximum of the squared
        // displacement since the last build
        __shared__ int s_n[kVvBlock / 64];
        const bool fast = a < A.N && d2 > A.thr2;
        const unsigned long long bal = __ballot(fast);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) s_n[wv] = __popcll(bal);
        for (int off = 32; off > 0; off >>= 1) d2 = fmax(d2, __shfl_xor(d2, off, 64));
        if (lane == 0) s_red[wv] = d2;
        __syncthreads();
        int pos = __popcll(bal & ((1ull << lane) - 1ull));
        for (int k = 0; k < wv; ++k) pos += s_n[k];
        if (fast) A.fast_loc[(int64_t)bi * kVvBlock + pos] = (int32_t)a;
        if (threadIdx.x == 0) {
            double m = s_red[0];
            int n = s_n[0];
            for (int k = 1; k < kVvBlock / 64; ++k) { m = fmax(m, s_red[k]); n += s_n[k]; }
            A.disp_partial[bi] = m;
            A.fast_cnt[bi] = n;
        }
    }
    if (PHASE == 1 && EKIN) {
        // per-system partial of this block, stored at index block + system
        const int64_t a0 = (int64_t)bi * kVvBlock;
        const int64_t a1 = min(A.N, a0 + kVvBlock) - 1;
        const int b0 = A.sys_of_atom[a0], b1 = A.sys_of_atom[a1];
        const int myb = a < A.N ? A.sys_of_atom[a] : -1;
        for (int b = b0; b <= b1; ++b) {
            double t = block_sum_d(myb == b ? ke : 0.0, s_red);
            if (threadIdx.x == 0) {
                if (A.ek_slots) {
                    // the partial travels as one atomic word: no separate ready flag,
                    // hence no release fence (an L2 write-back) per work-group
                    unsigned long long v = (unsigned long long)__double_as_longlong(t);
                    if (v == kEkSlotEmpty) v = 0x7FF8000000000000ull;
                    __hip_atomic_store(A.ek_slots + bi + b, v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    A.partial[bi + b] = t;
                }
            }
        }
    }
}

// One block: after phase 0, fold the displacement partials (rebuild request) and
// advance the step counter; after phase 1, sum the kinetic-energy partials of each
// system in a fixed order.
template <int PHASE>
__global__ void __launch_bounds__(kVvBlock) k_vv_finalize(VvArgs A, int nblocks)
{
    __shared__ double s_red[kVvBlock / 64];
    if (PHASE == 0) {
        // fast list: the blocks' lists concatenated in block order (ascending atom
        // index), up to the capacity; a rebuild is due when more atoms are fast
        FastJoinArgs J{A.disp_partial, A.fast_cnt, A.fast_loc, A.fast_list, A.fast_cap, nblocks,
                       kVvBlock, A.dsc};
        const int total = fast_join_block(J);
        if (threadIdx.x == 0 && total > A.fast_cap) A.dsc->need_rebuild = 1;
        return;
    }
    // phase 1: the systems of this work-group (fin_blocks(B) of them share a batch)
    for (int b = (int)blockIdx.x; b < A.B; b += (int)gridDim.x) {
        const int64_t s0 = A.sys_off[b], s1 = A.sys_off[b + 1];
        double t = 0.0;
        if (s1 > s0) {
            const int64_t k0 = s0 / kVvBlock, k1 = (s1 - 1) / kVvBlock;
            for (int64_t k = k0 + threadIdx.x; k <= k1; k += kVvBlock) t += A.partial[k + b];
        }
        t = block_sum_d(t, s_red);
        if (threadIdx.x == 0) A.ekin[b] = t;
    }
}

static LgArgs lg_args(Ctx* c, const uint8_t* elem, const uint32_t* atom_id)
{
    return LgArgs{c->d_lg_c1, c->d_lg_kt, c->E, c->n_steps + 1, elem, atom_id, c->d_seeds,
                  c->d_sys_of_atom};
}

static VvArgs vv_args(Ctx* c, int phase, double dt, const double* inv_mass, const double* fx,
                      const double* fy, const double* fz, double* x, double* y, double* z,
                      double* vx, double* vy, double* vz, double* ekin)
{
    (void)phase;
    VvArgs A;
    A.N = c->N; A.dt = dt; A.hdt = 0.5 * dt;
    const double half_skin = 0.5 * c->cfg.skin;
    A.thr2 = half_skin * half_skin;
    A.inv_mass = inv_mass; A.fx = fx; A.fy = fy; A.fz = fz;
    A.x = x; A.y = y; A.z = z; A.vx = vx; A.vy = vy; A.vz = vz;
    A.xref = c->d_xref; A.partial = c->d_partial; A.ek_slots = nullptr; A.ekin = ekin;
    const int nb = (int)div_up(c->N, kVvBlock);
    A.disp_partial = c->d_partial + nb + c->B + 1;
    A.sys_off = c->d_sys_off; A.sys_of_atom = c->d_sys_of_atom; A.B = c->B; A.dsc = c->dsc;
    A.fast_flag = c->d_fast_flag; A.fast_loc = c->d_fast_loc; A.fast_cnt = c->d_fast_cnt;
    A.fast_list = c->d_fast_list; A.fast_cap = c->fast_cap;
    return A;
}

void launch_vv(Ctx* c, int phase, double dt, const double* inv_mass, const double* fx,
               const double* fy, const double* fz, double* x, double* y, double* z, double* vx,
               double* vy, double* vz, double* ekin, hipStream_t st)
{
    const VvArgs A = vv_args(c, phase, dt, inv_mass, fx, fy, fz, x, y, z, vx, vy, vz, ekin);
    const int nb = (int)div_up(c->N, kVvBlock);
    const IonArgs I{};
    const ForceFinalizeArgs F{};
    const LgArgs L{};
    if (phase == 0) {
        if (nb > 0)
            hipLaunchKernelGGL((k_vv<0, false>), dim3(nb), dim3(kVvBlock), 0, st, A, I, F, L);
        hipLaunchKernelGGL((k_vv_finalize<0>), dim3(1), dim3(kVvBlock), 0, st, A, nb);
    } else if (ekin) {
        if (nb > 0)
            hipLaunchKernelGGL((k_vv<1, true>), dim3(nb), dim3(kVvBlock), 0, st, A, I, F, L);
        hipLaunchKernelGGL((k_vv_finalize<1>), dim3(fin_blocks(c->B)), dim3(kVvBlock), 0, st, A,
                           nb);
    } else if (nb > 0) {
        hipLaunchKernelGGL((k_vv<1, false>), dim3(nb), dim3(kVvBlock), 0, st, A, I, F, L);
    }
}

void launch_vv1_finalize(Ctx* c, double dt, const double* inv_mass, const double* fx,
                         const double* fy, const double* fz, double* vx, double* vy, double* vz,
                         double* ekin, double* epot, hipStream_t st)
{
    VvArgs A = vv_args(c, 1, dt, inv_mass, fx, fy, fz, nullptr, nullptr, nullptr, vx, vy, vz,
                       ekin);
    const int nb = (int)div_up(c->N, kVvBlock);
    const IonArgs I{};
    const ForceFinalizeArgs F = force_finalize_args(c, epot);
    const LgArgs L{};
    const int nf = fin_blocks(c->B);
    if (ekin && nb > 0) {
        // the extra work-groups also sum the kinetic energies (no separate launch)
        A.ek_slots = c->d_ek_slots;
        hipLaunchKernelGGL((k_vv<1, true, false, true>), dim3(nb + nf), dim3(kVvBlock), 0, st,
                           A, I, F, L);
    } else if (ekin) {
        hipLaunchKernelGGL((k_vv<1, true, false, true>), dim3(nb + nf), dim3(kVvBlock), 0, st,
                           A, I, F, L);
        hipLaunchKernelGGL((k_vv_finalize<1>), dim3(nf), dim3(kVvBlock), 0, st, A, nb);
    } else {
        hipLaunchKernelGGL((k_vv<1, false, false, true>), dim3(nb + nf), dim3(kVvBlock), 0, st,
                           A, I, F, L);
    }
}

void launch_vv0_ionize(Ctx* c, double dt, const double* inv_mass, const double* fx,
                       const double* fy, const double* fz, double* x, double* y, double* z,
                       double* vx, double* vy, double* vz, const uint8_t* elem,
                       const uint32_t* atom_id, int8_t* q, hipStream_t st)
{
    const VvArgs A = vv_args(c, 0, dt, inv_mass, fx, fy, fz, x, y, z, vx, vy, vz, nullptr);
    const int nb = (int)div_up(c->N, kVvBlock);
    if (nb <= 0) return;
    if (c->langevin)
        hipLaunchKernelGGL((k_vv<0, false, true, false, true>), dim3(nb), dim3(kVvBlock), 0, st, A,
                           ion_args(c, elem, atom_id, q), ForceFinalizeArgs{},
                           lg_args(c, elem, atom_id));
    else
        hipLaunchKernelGGL((k_vv<0, false, true>), dim3(nb), dim3(kVvBlock), 0, st, A,
                           ion_args(c, elem, atom_id, q), ForceFinalizeArgs{}, LgArgs{});
}

void launch_vv0_langevin(Ctx* c, double dt, const double* inv_mass, const uint8_t* elem,
                         const uint32_t* atom_id, const double* fx, const double* fy,
                         const double* fz, double* x, double* y, double* z, double* vx,
                         double* vy, double* vz, hipStream_t st)
{
    const VvArgs A = vv_args(c, 0, dt, inv_mass, fx, fy, fz, x, y, z, vx, vy, vz, nullptr);
    const int nb = (int)div_up(c->N, kVvBlock);
    if (nb > 0)
        hipLaunchKernelGGL((k_vv<0, false, false, false, true>), dim3(nb), dim3(kVvBlock), 0, st,
                           A, IonArgs{}, ForceFinalizeArgs{}, lg_args(c, elem, atom_id));
    hipLaunchKernelGGL((k_vv_finalize<0>), dim3(1), dim3(kVvBlock), 0, st, A, nb);
}

int vv_blocks(int64_t N) { return (int)div_up(N, kVvBlock); }
int vv_block_size() { return kVvBlock; }

int64_t vv_partials_needed(int64_t N, int B) { return 2 * (div_up(N, kVvBlock) + B + 1); }

// ------------------------------------------------------------------ device scalars

__global__ void k_set_step(DevScalars* d, int64_t step) { d->step = step; }
// Clear the error word and re-arm the fused build kernel's barrier (a timed-out
// barrier can leave arrival words ahead of the generation).
__global__ void k_clear_flags(DevScalars* d, uint32_t* bar_arrive, int n)
{
    for (int k = threadIdx.x; k < n; k += blockDim.x) bar_arrive[k] = 0u;
    if (threadIdx.x == 0) {
        d->flags = 0u;
        d->bar_gen = 0u;
    }
}

void launch_set_step(Ctx* c, int64_t step, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, st, c->dsc, step);
}

void launch_clear_flags(Ctx* c, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(256), 0, st, c->dsc, c->d_bar_arrive,
                       c->cap_bar);
}

}  // namespace md
