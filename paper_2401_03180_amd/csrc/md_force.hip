// md_force.hip -- screened pair forces (arXiv 2401.03180, section II.A: Eq. 2
// Debye-screened Coulomb between integer charges, Eq. 8 Lennard-Jones modulated
// by the same exp(-r / lambda_D); section II.B: plain truncation at rc).
//
// Work decomposition (full neighbour lists, no atomics, deterministic):
//   * a persistent work-group pulls cluster groups from a queue;
//   * it stages every candidate atom of the group's table in LDS as FP32 coordinates
//     relative to the group's centre: per table entry the FP64 offset of the
//     cluster's box corner (with the entry's periodic shift), rounded once, plus the
//     atom's FP32 offset from that corner (written by the repack), charge in .w;
//   * each 64-lane wave owns one 8-atom i-cluster: lane = 8 * i + k walks codes
//     k, k+8, ... of atom i's compacted list, so all 64 lanes evaluate distinct
//     pairs; the 8 partial sums of an atom are combined at the end.
// FP32 path: pair arithmetic in FP32; per-lane sums in FP32 over chunks of 16 terms,
// folded into a Kahan (sum, compensation) pair; cross-lane combination and the
// output in FP64.  Membership uses an FP32 distance whose rounding error is
// bounded; pairs inside the error band are re-decided with the FP64 expression,
// so the pair set equals the FP64 definition.
// FP64 path: the plain comparison form, every pair in FP64 from the caller's
// positions with the exact membership expression.
// HYBRID: the Coulomb term of a pair is k_e (q_j phi_i + q_i phi_j) / 2 with phi_Q the
// hybrid ion-sphere / Debye potential of a charge-Q ion (section II.A, Eq. 4-7),
// whose coefficients {r', c1, c2, c3} per (system, step, charge) are tabulated on the
// host; the Lennard-Jones term is unchanged.
// QLJ: the LJ radius of each atom shrinks to c sigma with c = 1 - q/Z (section II.B,
// Eq. 11) and a pair's radius is the mean of the two scaled radii, so the pair's
// c6 -> c6 s^6, c12 -> c12 s^12 with s = (c_i sigma_i + c_j sigma_j)/(sigma_i +
// sigma_j).  LJ-excluded pairs (bonded 1-2 and 1-3 partners) carry the all-zero
// pseudo-type in their list codes.
#include "md_device.h"
#include "md_internal.h"
#include "md_launch.h"

namespace md {

constexpr float kFarF = 1.0e4f;
constexpr int kMaxWpc = 2;        // waves per i-cluster (FP32 kernel): one per half-list
constexpr int kForceBlockMax = 64 * kMaxGroup * kMaxWpc;

// ------------------------------------------------------------------ repack (per step)

// Gather positions and charges into slot order; reset the force work queue;
// latch MD_FLAG_SKIN if the lists are stale.  Fast atoms (moved more than skin/2
// since the build) get NaN positions like padding slots: the list kernels skip
// them and their pairs are evaluated by the fast-atom kernels.
__global__ void __launch_bounds__(256) k_repack(RepackArgs A)
{
    repack_range<1>(A, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                 (int64_t)gridDim.x * blockDim.x, true);
}

void launch_repack(Ctx* c, const double* x, const double* y, const double* z, const int8_t* q,
                   hipStream_t st)
{
    const int nb = (int)std::min<int64_t>(div_up(c->cap_slots, 256), (int64_t)c->n_cu * 8);
    const RepackArgs A{x, y, z, q, c->d_perm, c->d_fast_flag, c->d_xs, c->d_qs, c->cap_slots,
                       c->dsc, c->d_slot_img, c->d_cl_lo, c->d_grid, c->d_sys_of_atom, c->B,
                       c->d_xo};
    hipLaunchKernelGGL(k_repack, dim3(std::max(nb, 1)), dim3(256), 0, st, A);
}

// ------------------------------------------------------------------ shared pieces

struct ForceArgs {
    const Group* groups;
    const uint32_t* ent;
    uint16_t* nb;
    int32_t* cl_nt;
    const int32_t* perm;
    const int32_t* slot_img;
    const double* xs;            // slot-order FP64 positions (SoA, stride cap_slots)
    const float4* xo;            // slot-order FP32 offsets from the cluster box corner, charge
    const double* cl_lo;         // cluster box corners (the offsets' origins)
    const int8_t* qs;
    const uint8_t* ts;
    const GridSys* grid;
    const double* kappa;         // B * S1
    int64_t S1;
    const float* lj32;           // T*T (c6, c12)
    const double* c6;
    const double* c12;
    int T;
    double rc2;                  // rc * rc (FP64, rounded once)
    int E_cap;
    int64_t cap_slots;
    double *fx, *fy, *fz;
    double* grp_epot;
    double* epot;
    const int32_t* sys_grp0;
    int B;
    DevScalars* dsc;
    int2* emit;
    int64_t emit_max;
    int wpc;
    int stage64;                 // FP64 kernel: the group table is staged in LDS
    // list (re)build inside the FP32 kernel
    int32_t* cl_len;
    const uint8_t* ent_mask;
    int nb_cap_h;
    float thr2;                  // ((rc + skin)(1 + 1e-5))^2
    // hybrid screening rows, [(b * S1 + step) * hyb_q + q]
    const float4* hyb32;
    const double* hyb64;
    int hyb_q;
    // force-field terms
    const double* qlj;           // charge-scaled LJ radii (QLJ): the kQljLen table
    const int32_t* excl_off;     // LJ exclusions per caller atom (NULL: none)
    const int32_t* excl;
    int t_excl;                  // pseudo-type of excluded pairs
    const int32_t* inv_perm;     // slot of each caller atom (current build)
    double* e_atom;              // debug (EMIT) launches: per-atom energies, or NULL
};

constexpr int kExclRegs = 8;     // excluded partners per atom held in registers

__global__ void __launch_bounds__(256) k_force_finalize(ForceFinalizeArgs F)
{
    force_finalize_block(F, (int)blockIdx.x, (int)gridDim.x);   // fin_blocks(B) of them
}

template <class T>
__device__ inline const __attribute__((address_space(1))) T* gbl(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}

// Global load at a 32-bit byte offset from a base pointer (the base stays scalar).
template <class T>
__device__ inline T ld_off(const T* p, uint32_t byte_off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
}

// Global store at a 32-bit byte offset from a base pointer (the base stays scalar).
template <class T>
__device__ inline void st_off(T* p, uint32_t byte_off, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + byte_off) = v;
}

__device__ inline int64_t slot_of_code(const uint32_t* ent_g, uint32_t idx)
{
    const uint32_t en = ent_g[idx >> 3];
    return (int64_t)(en & kEntClusterMask) * kCluster + (idx & 7u);
}

// FP64 re-decision of one pair (rare path of the FP32 kernel).
__device__ __noinline__ int recheck_pair(const uint32_t* ent_g, const double* xs, int64_t cs,
                                         int64_t slot_i, uint32_t idx, const GridSys* gsp,
                                         double rc2)
{
    const int64_t slot_j = slot_of_code(ent_g, idx);
    const GridSys gs = *gsp;
    const double r2 = pair_r2_exact(xs[slot_i], xs[cs + slot_i], xs[2 * cs + slot_i], xs[slot_j],
                                    xs[cs + slot_j], xs[2 * cs + slot_j], gs);
    return r2 < rc2 ? 1 : 0;
}

// Debug export: every lane whose pair is inside the cutoff with ai < aj appends
// (ai, aj); one atomic per wave reserves the slots.
__device__ __noinline__ void emit_pairs(bool in, const uint32_t* ent_g, const int32_t* perm,
                                        int ai, uint32_t idx, unsigned long long* counter,
                                        int2* out, int64_t max)
{
    int aj = -1;
    if (in) aj = perm[slot_of_code(ent_g, idx)];
    const bool take = in && ai < aj;
    const unsigned long long bal = __builtin_amdgcn_ballot_w64(take);
    if (bal == 0ull) return;
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    const int leader = __builtin_ctzll(bal);
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(bal));
    base = __shfl(base, leader, 64);
    if (take) {
        const unsigned long long p = base + __popcll(bal & ((1ull << lane) - 1ull));
        if ((int64_t)p < max) out[p] = make_int2(ai, aj);
    }
}

// Step counter clamped to the bound schedule (MD_FLAG_STEP latched otherwise).
__device__ inline int64_t clamp_step(const ForceArgs& A)
{
    int64_t s = A.dsc->step;
    if (s < 0 || s >= A.S1) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&A.dsc->flags, MD_FLAG_STEP);
        s = s < 0 ? 0 : A.S1 - 1;
    }
    return s;
}

__device__ inline void kahan_add(float& s, float& c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Combine the 8 lanes of one atom (lanes 8i .. 8i+7) in FP64.
__device__ inline double reduce8(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

// Place of list position p in its row of 32 codes: p = 32 r + 8 a + k is stored at
// 32 r + 4 k + a, so lane k of an atom reads positions k, k + 8, k + 16, k + 24 with
// one 8-byte load, and at each step the atom's 8 lanes read 8 consecutive positions
// (mostly neighbouring candidates of one entry: fewer LDS bank conflicts).
__device__ inline int row_place(int p)
{
    return (p & ~31) | ((p & 7) << 2) | ((p >> 3) & 3);
}

// 8-code columns of a half-list's last row that hold codes (1..4; 0 without rows):
// lane k of an atom takes positions 32 r + 8 a + k of row r, and past the longest
// list of the cluster (len codes) every position is the sentinel, whose terms are
// exact zeros, so the FP64 kernel skips the columns a >= tail_cols of the last row.
// (The FP32 kernel walks whole rows: splitting off its last row measured slower.)
__device__ inline int tail_cols(int len, int nrow)
{
    return nrow > 0 ? min(4, max(1, (len - 32 * (nrow - 1) + 7) >> 3)) : 0;
}

// Rebuild the half-list `half` of cluster I from the candidates staged in LDS
// (during a rebuild their .w holds the type): the codes (staged index | type << 13)
// of partners within rc + skin, compacted per atom in entry order.  Each atom's
// half-list is contiguous (nb_cap_h codes), padded with the sentinel to whole rows
// of 32 codes.  s_mask[e] holds the clusters of the group entry e can reach (low
// byte) and the cluster whose own unshifted entry it is (high byte).  Returns the
// row count.
// EXCL: LJ exclusions are bound (a separate instantiation keeps their per-candidate
// test out of the plain builder's loop).
template <bool EXCL>
__device__ int build_half_list_t(const ForceArgs& A, int I, int half, int cw, int il, int k,
                                 int ai, float xi, float yi, float zi, int nent, const float4* s_j,
                                 const uint16_t* s_mask, int sentinel, const uint32_t* ent_g)
{
    const int lane = threadIdx.x & 63;
    // this half-list block of the cluster (wave-uniform base) and the lane's atom row
    // in it (a 32-bit byte offset, so the stores keep a scalar base)
    uint16_t* outw = A.nb + ((int64_t)I * 2 + half) * kCluster * A.nb_cap_h;
    const uint32_t lrow = (uint32_t)(il * A.nb_cap_h);
    const bool live = ai >= 0;
    // on the cluster's own entry the lane whose candidate is its own atom (k == il)
    // compares against a negative threshold: one compare decides every lane
    const float thr_own = k == il ? -1.0f : A.thr2;
    const uint32_t below = (1u << k) - 1u;      // lanes of this atom before this one
    const float thr2 = A.thr2;
    const int cap = A.nb_cap_h;
    int cnt = 0;
    // the LJ-excluded partners of this lane's atom as slots of the current build (the
    // first kExclRegs in registers; any others are looked up by atom below)
    int exs[kExclRegs];
    int x0 = 0, x1 = 0;
    if (EXCL && live) {
        x0 = A.excl_off[ai];
        x1 = A.excl_off[ai + 1];
    }
#pragma unroll
    for (int x = 0; x < kExclRegs; ++x) exs[x] = x0 + x < x1 ? A.inv_perm[A.excl[x0 + x]] : -1;
    // candidate entry e (its atom k staged as pj): test, compact in entry order, store
    auto emit = [&](int e, bool own, const float4& pj) {
        const int j = e * kCluster + k;
        const float dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        // no test of the i-atom itself: padding and fast i-atoms sit at -kFarF and
        // padding candidates at +kFarF, far outside every cutoff
        const bool pass = r2 < (own ? thr_own : thr2);
        const uint64_t bal = __builtin_amdgcn_ballot_w64(pass);
        const uint32_t mine = (uint32_t)(bal >> (il * 8)) & 0xFFu;
        const int pos = cnt + __popc(mine & below);
        int tcode = __float_as_int(pj.w);
        if (EXCL && pass) {                   // LJ-excluded partner: the pseudo-type
            const int slot_j =
                (int)((__builtin_amdgcn_readfirstlane(ent_g[e]) & kEntClusterMask) * kCluster) + k;
            bool exc = false;
#pragma unroll
            for (int x = 0; x < kExclRegs; ++x) exc |= exs[x] == slot_j;
            if (!exc && x1 - x0 > kExclRegs) {
                const int aj = A.perm[slot_j];
                for (int x = x0 + kExclRegs; x < x1; ++x) exc |= A.excl[x] == aj;
            }
            if (exc) tcode = A.t_excl;
        }
        if (pass && pos < cap)
            st_off(outw, (lrow + (uint32_t)row_place(pos)) * 2u,
                   (uint16_t)(j | (tcode << kCodeIdxBits)));
        cnt += __popc(mine);
    };
    // the entries of this half (e = half, half + 2, ...) that reach this cluster, 64
    // at a time: one lane reads each mask, a ballot lists the reaching ones, and the
    // wave walks them two at a time (both candidate reads in flight together)
    for (int eb = half; eb < nent; eb += 128) {
        const int el = eb + 2 * lane;
        const uint32_t mk = el < nent ? (uint32_t)s_mask[el] : 0u;
        uint64_t todo = __builtin_amdgcn_ballot_w64(((mk >> cw) & 1u) != 0u);
        const uint64_t ownb = __builtin_amdgcn_ballot_w64(((mk >> (8 + cw)) & 1u) != 0u);
        while (todo != 0ull) {
            const int l0 = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            const int e0 = eb + 2 * l0;
            const float4 p0 = s_j[e0 * kCluster + k];
            if (todo != 0ull) {
                const int l1 = __builtin_ctzll(todo);
                todo &= todo - 1ull;
                const int e1 = eb + 2 * l1;
                const float4 p1 = s_j[e1 * kCluster + k];
                emit(e0, ((ownb >> l0) & 1ull) != 0ull, p0);
                emit(e1, ((ownb >> l1) & 1ull) != 0ull, p1);
            } else {
                emit(e0, ((ownb >> l0) & 1ull) != 0ull, p0);
            }
        }
    }
    int mx = cnt;
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
    const int nrow = min((mx + 31) >> 5, cap >> 5);
    for (int pos = cnt + k; pos < nrow * 32; pos += 8)
        st_off(outw, (lrow + (uint32_t)row_place(pos)) * 2u, (uint16_t)sentinel);
    if (lane == 0) {
        A.cl_nt[(int64_t)I * 2 + half] = nrow;
        A.cl_len[(int64_t)I * 2 + half] = mx;
        if (mx > cap) atomicOr(&A.dsc->flags, MD_FLAG_LIST_OVERFLOW);
    }
    return nrow;
}

__device__ inline int build_half_list(const ForceArgs& A, int I, int half, int cw, int il, int k,
                                      int ai, float xi, float yi, float zi, int nent,
                                      const float4* s_j, const uint16_t* s_mask, int sentinel,
                                      const uint32_t* ent_g)
{
    if (A.excl_off)
        return build_half_list_t<true>(A, I, half, cw, il, k, ai, xi, yi, zi, nent, s_j, s_mask,
                                       sentinel, ent_g);
    return build_half_list_t<false>(A, I, half, cw, il, k, ai, xi, yi, zi, nent, s_j, s_mask,
                                    sentinel, ent_g);
}

// ------------------------------------------------------------------ FP32 kernel

// LISTS: only (re)build the per-atom lists, for the FP64 kernel; does nothing
// unless a rebuild is pending.  HYBRID: hybrid screening of the Coulomb term.
template <bool ENERGY, bool EMIT, bool SCREEN_LJ, bool LISTS = false, bool HYBRID = false,
          bool QLJ = false>
__global__ void __launch_bounds__(kForceBlockMax) k_force32(ForceArgs A)
{
    extern __shared__ float4 s_j[];
    __shared__ float2 s_lj[MD_MAX_TYPES * MD_MAX_TYPES];
    __shared__ float s_m[kForceBlockMax / 64];
    __shared__ double s_part[kForceBlockMax / 64][kCluster][4];
    __shared__ int s_g;
    const int tid = threadIdx.x, lane = tid & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index (uniform)
    const int wpc = A.wpc;                     // waves per i-cluster
    const int cw = w / wpc, half = w - cw * wpc;
    const int il = lane >> 3, k8 = lane & 7;
    const int64_t step = clamp_step(A);
    const int ngroups = A.dsc->n_groups;
    // candidate tables were rebuilt: (re)build the per-atom half-lists first
    const bool rebuild = __builtin_amdgcn_readfirstlane(A.dsc->lists_pending) != 0;
    if (LISTS && !rebuild) return;
    for (int i = tid; i < A.T * A.T; i += blockDim.x)
        s_lj[i] = make_float2(A.lj32[2 * i], A.lj32[2 * i + 1]);
    __shared__ double s_qlj[QLJ ? kQljLen : 1];
    if (QLJ)
        for (int i = tid; i < kQljLen; i += blockDim.x) s_qlj[i] = A.qlj[i];
    const int sentinel = A.E_cap * kCluster;
    uint16_t* s_mask = reinterpret_cast<uint16_t*>(s_j + sentinel + 1);
    // hybrid screening: {r', c1, c2, c3} per charge state, after the masks (dynamic LDS
    // sized by the bound charge states)
    float4* s_hyb = reinterpret_cast<float4*>(
        reinterpret_cast<char*>(s_mask) + ((A.E_cap * sizeof(uint16_t) + 15) & ~(size_t)15));
    if (tid == 0) s_j[sentinel] = make_float4(kFarF, kFarF, kFarF, 0.0f);
    const float rc2f = (float)A.rc2;
    const int64_t cs = A.cap_slots;

    // the first group of every work-group is its own index; later ones come from a
    // shared counter (no burst of same-address atomics at launch)
    for (int g = blockIdx.x; g < ngroups;) {
        // the next group is claimed now (its atomic's latency overlaps this group)
        unsigned claim = 0u;
        if (!LISTS && tid == 0) claim = atomicAdd(&A.dsc->work_force, 1u);
        const Group gr = A.groups[g];
        const GridSys gs = A.grid[gr.sys];
        const double kap = A.kappa[(int64_t)gr.sys * A.S1 + step];
        const auto ent_gl = gbl(A.ent + (int64_t)g * A.E_cap);
        if (HYBRID) {
            const float4* hr = A.hyb32 + ((int64_t)gr.sys * A.S1 + step) * A.hyb_q;
            for (int q = tid; q < A.hyb_q; q += blockDim.x) s_hyb[q] = hr[q];
        }

        // ---- stage the candidate atoms in the group frame, in batches of 64 entries
        //      per wave: (a) one lane per entry computes the FP64 offset of the
        //      entry's cluster box corner from the group centre (with its periodic
        //      shift), rounded once, and parks it with the cluster index in the slot
        //      of the entry's atom (e & 7); (b) one lane per atom (an entry's 8 atoms in
        //      adjacent lanes of the same wave, so LDS program order makes the corner
        //      visible) adds its FP32 offset from the corner (written by the repack)
        //      and stores the candidate.  Padding and fast atoms (offset x NaN) go far
        //      away, outside every cutoff; their NaNs do not enter m (max ignores a NaN
        //      operand).
        float m = 0.0f;                        // largest |staged coordinate| or |offset|
        const int nent = gr.nent;
        const uint32_t gbase = (uint32_t)g * (uint32_t)A.E_cap;
        for (int eb = w * 64; eb < nent; eb += nw * 64) {
            {
                const int e = eb + lane;
                if (e < nent) {
                    // 32-bit byte offsets keep the load bases scalar
                    const uint32_t en = ld_off(A.ent, (gbase + (uint32_t)e) * 4u);
                    const uint32_t cl = en & kEntClusterMask;
                    const uint32_t cb = cl * 24u;                  // 24 bytes per corner
                    float b[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        double bd = ld_off(A.cl_lo, cb + 8u * (uint32_t)d) - gr.c[d];
                        if (gs.periodic) {
                            const int sh = (int)((en >> (26 + 2 * d)) & 3u) - 1;
                            bd = fma((double)sh, gs.L[d], bd);
                        }
                        b[d] = (float)bd;
                    }
                    s_j[e * kCluster + (e & 7)] =
                        make_float4(b[0], b[1], b[2], __int_as_float((int)cl));
                    if (rebuild) {
                        const int c = (int)cl - gr.cl0;
                        const uint32_t own = ((en >> 26) == 0x15u && c >= 0 && c < gr.ncl)
                                                 ? (1u << (8 + c)) : 0u;
                        s_mask[e] = (uint16_t)(A.ent_mask[(int64_t)g * A.E_cap + e] | own);
                    }
                }
            }
            // 4 loads in flight before any use.  A lane past the last entry stores
            // nothing and loads from cluster 0 (the corner slot it would read may
            // already hold a staged atom: no cluster index)
            auto atoms = [&](int a0, auto reb_c) {
                constexpr bool REB = decltype(reb_c)::value;
                float4 bb[4], o[4];
                uint32_t tv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int e = min(eb + (a0 + a) * 8 + (lane >> 3), nent - 1);
                    bb[a] = s_j[e * kCluster + (e & 7)];
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const bool here = eb + (a0 + a) * 8 + (lane >> 3) < nent;
                    const uint32_t cl = here ? (uint32_t)__float_as_int(bb[a].w) : 0u;
                    const uint32_t slot = cl * kCluster + (lane & 7);
                    o[a] = ld_off(A.xo, slot * (uint32_t)sizeof(float4));
                    // while the lists are rebuilt .w carries the type (the charges are
                    // put back before the pair loop)
                    if (REB) tv[a] = ld_off(A.ts, slot);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int e = eb + (a0 + a) * 8 + (lane >> 3);
                    if (e < nent) {
                        const float r0 = bb[a].x + o[a].x, r1 = bb[a].y + o[a].y,
                                    r2 = bb[a].z + o[a].z;
                        m = fmaxf(m, fmaxf(fabsf(r0), fabsf(o[a].x)));
                        m = fmaxf(m, fmaxf(fabsf(r1), fabsf(o[a].y)));
                        m = fmaxf(m, fmaxf(fabsf(r2), fabsf(o[a].z)));
                        const float wv = REB ? __int_as_float((int)tv[a]) : o[a].w;
                        s_j[e * kCluster + (lane & 7)] =
                            make_float4(o[a].x != o[a].x ? kFarF : r0, r1, r2, wv);
                    }
                }
            };
            for (int a0 = 0; a0 < 8; a0 += 4) {
                if (rebuild) atoms(a0, std::true_type{});
                else atoms(a0, std::false_type{});
            }
        }
        // this wave's i-atoms (slot-indexed): the loads are issued before the barrier,
        // so their latency overlaps the wait
        const bool act = cw < gr.ncl;              // wave-uniform
        const int I = gr.cl0 + cw;
        const int64_t slot_i = (int64_t)I * kCluster + il;
        int ai = -1, im_i = 0, q_i = 0, t_i = 0, nr = 0;
        double pxi[3] = {0.0, 0.0, 0.0};
        if (act) {
            ai = A.perm[slot_i];
            for (int d = 0; d < 3; ++d) pxi[d] = A.xs[d * cs + slot_i];
            im_i = A.slot_img[slot_i];
            q_i = A.qs[slot_i];
            t_i = A.ts[slot_i];
            if (!rebuild) nr = A.cl_nt[(int64_t)I * 2 + half];
        }
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        if (lane == 0) s_m[w] = m;
        __syncthreads();
        m = s_m[0];
        for (int k = 1; k < nw; ++k) m = fmaxf(m, s_m[k]);
        // Rounding bound of the FP32 r^2 near the cutoff (u = 2^-24, m as above): a
        // staged candidate coordinate fl(fl(b) + fl(o)) carries <= u (|b| + |o| + |x|)
        // <= 4 u m error (|b| <= |x| + |o|), the i-atom coordinate <= u m, so
        // |d32 - d| <= u (5m + |d|) per axis and |r2_32 - r2| <= 2 sqrt(3) rc u (5m + rc)
        // + 3 u rc^2; doubled for margin.
        const float u = 5.9604645e-8f;
        const float rcf = sqrtf(rc2f);
        const float band = 2.0f * (3.4641016f * rcf * u * (5.0f * m + rcf) + 3.0f * u * rc2f) +
                           1e-12f;
        const float lo2 = rc2f - band, hi2 = rc2f + band;

        double Fx = 0.0, Fy = 0.0, Fz = 0.0, Ea = 0.0;
        float xi = -kFarF, yi = -kFarF, zi = -kFarF, qike = 0.0f, qif = 0.0f;
        float4 hi = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        double ci = 0.0;                       // QLJ: the scaled radius c_i sigma_i
        const double* rs_row = s_qlj + kQljRs; // QLJ: 1/(sigma_i + sigma_j) of this atom
        int tb = 0;
        // a fast atom (NaN position) takes no part, like padding: its pairs and its
        // force come from the fast-atom kernels
        if (act && ai >= 0 && pxi[0] == pxi[0]) {
            float r[3];
            for (int d = 0; d < 3; ++d) {
                double v = pxi[d];
                if (gs.periodic) v = v - (double)unpack_img(im_i, d) * gs.L[d];
                r[d] = (float)(v - gr.c[d]);
            }
            xi = r[0]; yi = r[1]; zi = r[2];
            qike = (float)(kKe * (double)q_i);
            tb = t_i * A.T;
            if (QLJ) {
                ci = fma(-(double)q_i, s_qlj[kQljSigZ + t_i], s_qlj[kQljSig + t_i]);
                rs_row = s_qlj + kQljRs + t_i * MD_MAX_TYPES;
            }
            if (HYBRID) {
                qif = (float)q_i;
                hi = s_hyb[min(max(q_i, 0), A.hyb_q - 1)];
            }
        }
        if (rebuild) {
            if (act)
                nr = build_half_list(A, I, half, cw, il, k8, ai, xi, yi, zi, gr.nent, s_j, s_mask,
                                     sentinel, A.ent + (int64_t)g * A.E_cap);
            if (LISTS) {              // static group order (the force queue is not used)
                __syncthreads();
                g += gridDim.x;
                continue;
            }
            // the lists are read back only inside this work-group: the barrier's
            // work-group-scope ordering suffices (an agent-scope fence would write
            // back the L2)
            __syncthreads();
            for (int idx = tid; idx < nent * kCluster; idx += blockDim.x) {   // charges back
                const uint32_t en = ent_gl[idx >> 3];
                const float qv = (float)A.qs[(int64_t)(en & kEntClusterMask) * kCluster + (idx & 7)];
                reinterpret_cast<float*>(s_j + idx)[3] = qv;
            }
            __syncthreads();
        }
        if (act) {
            const float kapf = (float)kap;
            const float nkl2 = (float)(-kap * 1.4426950408889634);   // -kappa log2(e)
            const float hke = (float)(0.5 * kKe);
            const int qn1 = A.hyb_q - 1;
            // wave-uniform row count and list base (scalar loop control / addressing);
            // each lane reads its next 4 codes with one 8-byte load, two rows ahead
            nr = __builtin_amdgcn_readfirstlane(nr);
            // lane (i, k) takes codes 4k .. 4k + 3 of every 32-code row of atom i
            const auto cp = gbl(reinterpret_cast<const uint64_t*>(
                                A.nb + (((int64_t)I * 2 + half) * kCluster + il) * A.nb_cap_h)) +
                            k8;
            const uint32_t* ent_g = A.ent + (int64_t)g * A.E_cap;
            const GridSys* gsp = A.grid + gr.sys;
            float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
            float ax = 0.f, ay = 0.f, az = 0.f, ea = 0.f;
            double eacc = 0.0;
            // one row = 4 codes per lane: the 4 candidate reads are issued together,
            // then the 4 distances, one ballot for the rare FP64 re-decisions, and the
            // 4 pair terms, summed in code order
            const float2* lj_row = s_lj + tb;           // this atom's row of the LJ table
            auto row = [&](uint64_t codes) {
                uint32_t idx[4];
                int tj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // one bit-field extract per field from the 32-bit half
                    const uint32_t wd = (uint32_t)(codes >> (32 * (u >> 1)));
                    const uint32_t sh = 16u * (uint32_t)(u & 1);
                    idx[u] = __builtin_amdgcn_ubfe(wd, sh, kCodeIdxBits);
                    tj[u] = (int)__builtin_amdgcn_ubfe(wd, sh + kCodeIdxBits, 16 - kCodeIdxBits);
                }
                float4 pj[4];
                float2 lj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) pj[u] = s_j[idx[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) lj[u] = lj_row[tj[u]];
                if (QLJ) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        // in FP64 (full rate here): c sigma cancels as q nears Z and
                        // the scale enters as s^12
                        const double cj = fma(-(double)pj[u].w, s_qlj[kQljSigZ + tj[u]],
                                              s_qlj[kQljSig + tj[u]]);
                        const double sc = (ci + cj) * rs_row[tj[u]];
                        const double s2 = sc * sc, s6 = s2 * s2 * s2;
                        lj[u].x = (float)((double)lj[u].x * s6);
                        lj[u].y = (float)((double)lj[u].y * (s6 * s6));
                    }
                }
                float dx[4], dy[4], dz[4], r2[4];
                bool in[4], amb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    dx[u] = xi - pj[u].x;
                    dy[u] = yi - pj[u].y;
                    dz[u] = zi - pj[u].z;
                    r2[u] = fmaf(dz[u], dz[u], fmaf(dy[u], dy[u], dx[u] * dx[u]));
                    // in: surely inside; below hi2 but not in: within the band, where
                    // the FP64 test decides (two compares, combined on the scalar unit)
                    in[u] = r2[u] < lo2;
                    amb[u] = r2[u] <= hi2;
                }
                uint64_t band_any = 0ull;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    band_any |= __builtin_amdgcn_ballot_w64(amb[u]) &
                                ~__builtin_amdgcn_ballot_w64(in[u]);
                if (__builtin_expect(band_any != 0ull, 0)) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (amb[u] && !in[u])
                            in[u] = recheck_pair(ent_g, A.xs, cs, slot_i, idx[u], gsp, A.rc2) != 0;
                }
                if (EMIT) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        emit_pairs(in[u], ent_g, A.perm, ai, idx[u], &A.dsc->pair_count, A.emit,
                                   A.emit_max);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float rinv = in[u] ? __builtin_amdgcn_rsqf(r2[u]) : 0.0f;
                    const float r = r2[u] * rinv;
                    const float s = __builtin_amdgcn_exp2f(r * nkl2);
                    const float rinv2 = rinv * rinv;
                    const float rinv6 = rinv2 * rinv2 * rinv2;
                    const float uc = qike * pj[u].w * rinv;
                    const float l6 = lj[u].x * rinv6;
                    const float l12 = lj[u].y * rinv6 * rinv6;
                    const float kr = r * kapf;
                    float f, e;
                    if (HYBRID) {
                        // potentials of ions i and j at r (ion-sphere form inside r',
                        // Debye form outside) and w = -r dphi/dr
                        const float qj = pj[u].w;
                        const float4 hj = s_hyb[min(max((int)qj, 0), qn1)];
                        const float so = s * rinv, kr1 = 1.0f + kr;
                        const bool ii = r < hi.x, jj = r < hj.x;
                        const float pI = ii ? fmaf(qif, rinv, fmaf(-hi.z, r2[u], hi.y)) : hi.w * so;
                        const float wI = ii ? fmaf(2.0f * hi.z, r2[u], qif * rinv) : hi.w * so * kr1;
                        const float pJ = jj ? fmaf(qj, rinv, fmaf(-hj.z, r2[u], hj.y)) : hj.w * so;
                        const float wJ = jj ? fmaf(2.0f * hj.z, r2[u], qj * rinv) : hj.w * so * kr1;
                        const float uC = in[u] ? hke * fmaf(qj, pI, qif * pJ) : 0.0f;
                        const float wC = in[u] ? hke * fmaf(qj, wI, qif * wJ) : 0.0f;
                        const float ulj = l12 - l6, wlj = fmaf(-6.0f, l6, 12.0f * l12);
                        if (SCREEN_LJ) {
                            f = fmaf(fmaf(ulj, kr, wlj), s, wC) * rinv2;
                            e = fmaf(ulj, s, uC);
                        } else {
                            f = (wC + wlj) * rinv2;
                            e = uC + ulj;
                        }
                        (void)uc;
                    } else if (SCREEN_LJ) {
                        const float uu = uc + (l12 - l6);
                        const float wv = fmaf(-6.0f, l6, fmaf(12.0f, l12, uc));
                        f = fmaf(uu, kr, wv) * s * rinv2;
                        e = uu * s;
                    } else {
                        const float wl = fmaf(-6.0f, l6, 12.0f * l12);
                        f = fmaf(uc * s, 1.0f + kr, wl) * rinv2;
                        e = fmaf(uc, s, l12 - l6);
                    }
                    if (HYBRID) {
                        // recomputed here: holding the 4 separations across the pair terms
                        // spills registers in this variant
                        ax = fmaf(f, xi - pj[u].x, ax);
                        ay = fmaf(f, yi - pj[u].y, ay);
                        az = fmaf(f, zi - pj[u].z, az);
                    } else {
                        ax = fmaf(f, dx[u], ax);
                        ay = fmaf(f, dy[u], ay);
                        az = fmaf(f, dz[u], az);
                    }
                    if (ENERGY) ea += e;
                }
            };
            const uint64_t sent4 = 0x0001000100010001ull * (uint64_t)sentinel;
            uint64_t v0 = nr > 0 ? (uint64_t)cp[0] : sent4;
            uint64_t v1 = nr > 1 ? (uint64_t)cp[8] : sent4;
            for (int r = 0; r < nr; ++r) {
                const uint64_t cur = v0;
                v0 = v1;
                if (r + 2 < nr) v1 = cp[(r + 2) * 8];
                row(cur);
                if ((r & 3) == 3) {      // fold every 16 terms into the compensated sums
                    kahan_add(sx, cx, ax); kahan_add(sy, cy, ay); kahan_add(sz, cz, az);
                    if (ENERGY) eacc += (double)ea;
                    ax = ay = az = ea = 0.0f;
                }
            }
            if (ENERGY) eacc += (double)ea;
            kahan_add(sx, cx, ax); kahan_add(sy, cy, ay); kahan_add(sz, cz, az);
            // true per-lane sum = s - c; combine the atom's 8 lanes in FP64
            Fx = reduce8((double)sx - (double)cx);
            Fy = reduce8((double)sy - (double)cy);
            Fz = reduce8((double)sz - (double)cz);
            if (ENERGY) Ea = reduce8(eacc);
        }
        // combine the waves of each cluster in a fixed order (deterministic)
        if ((lane & 7) == 0) {
            s_part[w][il][0] = Fx;
            s_part[w][il][1] = Fy;
            s_part[w][il][2] = Fz;
            s_part[w][il][3] = Ea;
        }
        __syncthreads();
        if (half == 0 && (lane & 7) == 0 && ai >= 0) {
            double F[3] = {0.0, 0.0, 0.0};
            for (int h = 0; h < wpc; ++h)
                for (int d = 0; d < 3; ++d) F[d] += s_part[w + h][il][d];
            A.fx[ai] = F[0];
            A.fy[ai] = F[1];
            A.fz[ai] = F[2];
            if (EMIT && ENERGY && A.e_atom) {
                double e = 0.0;
                for (int h = 0; h < wpc; ++h) e += s_part[w + h][il][3];
                A.e_atom[ai] = 0.5 * e;    // each pair is visited from both atoms
            }
        }
        if (ENERGY && tid == 0) {
            double t = 0.0;
            for (int k = 0; k < nw; ++k)
                for (int i = 0; i < kCluster; ++i) t += s_part[k][i][3];
            A.grp_epot[g] = 0.5 * t;       // each pair is visited from both atoms
        }
        if (tid == 0) s_g = (int)(gridDim.x + claim);
        __syncthreads();
        g = s_g;
    }
}

// ------------------------------------------------------------------ FP64 kernel

// The FP64 kernel stages a group's candidates in LDS as the caller's FP64 positions
// (unchanged values, so every pair's distance is the exact membership expression)
// and their charges; a group table too large for one work-group's LDS is read from
// global memory instead (same values, same order).  Each i-cluster takes wpc waves:
// the two half-lists, each split by alternate rows (one wave takes both in turn).
// Candidates without a position
// (the sentinel, padding, fast atoms: NaN in the slot arrays) are staged at the
// origin with the charge kAbsentQ, which no pair test accepts.
constexpr int kForce64Block = 512;
constexpr int16_t kAbsentQ = 0x4000;

__host__ __device__ inline int64_t force64_stage_slots(int E_cap)
{
    return (int64_t)E_cap * kCluster + 1;          // + the sentinel
}

size_t force64_lds_bytes(int E_cap)
{
    const int64_t S = force64_stage_slots(E_cap);
    return (size_t)S * 3 * sizeof(double) + (size_t)((S * 2 + 15) & ~(int64_t)15);
}

template <bool ENERGY, bool EMIT, bool SCREEN_LJ, bool HYBRID = false, bool QLJ = false>
__global__ void __launch_bounds__(kForce64Block) k_force64(ForceArgs A)
{
    extern __shared__ double s_x[];
    __shared__ double2 s_c[MD_MAX_TYPES * MD_MAX_TYPES];
    __shared__ double s_part[kForce64Block / 64][kCluster][4];
    __shared__ int s_g;
    const int tid = threadIdx.x, lane = tid & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpc = A.wpc;                          // waves per i-cluster (even)
    const int cw = w / wpc, sub = w - cw * wpc;
    // two or more waves per cluster: wave sub takes half-list sub & 1, rows sub >> 1,
    // + wpc / 2, ...; one wave per cluster (groups of 8): both half-lists in turn
    const int half = wpc > 1 ? (sub & 1) : 0, nhalf = wpc > 1 ? 1 : 2;
    const int rp = sub >> 1, nrp = wpc > 1 ? wpc >> 1 : 1;
    const int il = lane >> 3, k8 = lane & 7;
    const int64_t step = clamp_step(A);
    const int ngroups = A.dsc->n_groups;
    const uint32_t sentinel = (uint32_t)(A.E_cap * kCluster);
    const int64_t cs = A.cap_slots;
    const bool staged = A.stage64 != 0;              // uniform
    const int64_t S = force64_stage_slots(A.E_cap);
    double* s_y = s_x + S;
    double* s_z = s_x + 2 * S;
    int16_t* s_q = reinterpret_cast<int16_t*>(s_x + 3 * S);
    for (int i = tid; i < A.T * A.T; i += blockDim.x) s_c[i] = make_double2(A.c6[i], A.c12[i]);
    if (staged && tid == 0) {                        // the sentinel: never inside
        s_x[sentinel] = 0.0; s_y[sentinel] = 0.0; s_z[sentinel] = 0.0;
        s_q[sentinel] = kAbsentQ;
    }
    for (int g = blockIdx.x; g < ngroups;) {
        unsigned claim = 0u;
        if (tid == 0) claim = atomicAdd(&A.dsc->work_force, 1u);
        const Group gr = A.groups[g];
        const GridSys gs = A.grid[gr.sys];
        const double kap = A.kappa[(int64_t)gr.sys * A.S1 + step];
        const double* hrow = HYBRID ? A.hyb64 + ((int64_t)gr.sys * A.S1 + step) * A.hyb_q * 4
                                    : nullptr;
        const uint32_t* ent_g = A.ent + (int64_t)g * A.E_cap;
        const int nent = gr.nent;
        // ---- stage: candidate t = 8 e + k is atom k of entry e's cluster (consecutive
        //      threads read consecutive slots); four candidates per thread and pass,
        //      each step's loads issued for all four together (candidates past the end
        //      load the last one and store nothing)
        if (staged) {
            const int nst = nent * kCluster;
            for (int t0 = tid; t0 < nst; t0 += 4 * (int)blockDim.x) {
                int64_t slot[4];
                double px[4], py[4], pz[4];
                int16_t qv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = min(t0 + u * (int)blockDim.x, nst - 1);
                    slot[u] = (int64_t)(ent_g[t >> 3] & kEntClusterMask) * kCluster + (t & 7);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    px[u] = A.xs[slot[u]];
                    py[u] = A.xs[cs + slot[u]];
                    pz[u] = A.xs[2 * cs + slot[u]];
                    qv[u] = A.qs[slot[u]];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = t0 + u * (int)blockDim.x;
                    if (t < nst) {
                        const bool here = px[u] == px[u];
                        s_x[t] = here ? px[u] : 0.0;
                        s_y[t] = here ? py[u] : 0.0;
                        s_z[t] = here ? pz[u] : 0.0;
                        s_q[t] = here ? qv[u] : kAbsentQ;
                    }
                }
            }
        }
        const bool act = cw < gr.ncl;                 // wave-uniform
        const int I = gr.cl0 + cw;
        const int64_t slot_i = (int64_t)I * kCluster + il;
        int ai = -1, ti = 0, qi_n = 0, nr = 0;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        if (act) {
            ai = A.perm[slot_i];
            if (ai >= 0) {
                xi = A.xs[slot_i]; yi = A.xs[cs + slot_i]; zi = A.xs[2 * cs + slot_i];
                qi_n = A.qs[slot_i];
                ti = A.ts[slot_i];
            }
        }
        // a fast i-atom (NaN position) takes no part: its force comes from the
        // fast-atom kernels
        const bool live = ai >= 0 && xi == xi;
        if (!live) xi = yi = zi = 0.0;
        __syncthreads();
        double Fx = 0.0, Fy = 0.0, Fz = 0.0, eacc = 0.0;
        if (act) {
            const double qi = kKe * (double)qi_n;
            const double2* c_row = s_c + ti * A.T;
            // one row of 4 candidates (NU in the last row): distances by the exact
            // membership expression (the sentinel and padding i-atoms, at finite
            // placeholder positions, are never inside), then the pair terms of all 4
            // without branches (a pair outside the cutoff is evaluated at r^2 = 1 and its
            // terms dropped), so the 4 evaluations interleave.  ST: staged table; PER:
            // periodic system (both uniform, fixed per loop, so no branch on them sits
            // inside the row)
            auto row = [&](uint64_t codes, auto st_c, auto per_c,
                           auto nu_c) __attribute__((always_inline)) {
                constexpr bool ST = decltype(st_c)::value;
                constexpr bool PER = decltype(per_c)::value;
                constexpr int NU = decltype(nu_c)::value;
                uint32_t idx[4];
                int tj[4], qj[4];
                double dx[4], dy[4], dz[4], r2[4];
                bool in[4];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const uint32_t code = (uint32_t)(codes >> (16 * u)) & 0xFFFFu;
                    idx[u] = code & kCodeIdxMask;
                    tj[u] = (int)(code >> kCodeIdxBits);
                    double xj, yj, zj;
                    if constexpr (ST) {
                        xj = s_x[idx[u]]; yj = s_y[idx[u]]; zj = s_z[idx[u]];
                        qj[u] = s_q[idx[u]];
                    } else {
                        xj = yj = zj = 0.0;
                        qj[u] = kAbsentQ;
                        if (idx[u] != sentinel) {
                            const int64_t slot_j = slot_of_code(ent_g, idx[u]);
                            const double px = A.xs[slot_j];
                            if (px == px) {
                                xj = px; yj = A.xs[cs + slot_j]; zj = A.xs[2 * cs + slot_j];
                                qj[u] = A.qs[slot_j];
                            }
                        }
                    }
                    {
#pragma clang fp contract(off)
                        dx[u] = xi - xj;
                        dy[u] = yi - yj;
                        dz[u] = zi - zj;
                        if (PER) {
                            dx[u] = dx[u] - gs.L[0] * rint(dx[u] * gs.invL[0]);
                            dy[u] = dy[u] - gs.L[1] * rint(dy[u] * gs.invL[1]);
                            dz[u] = dz[u] - gs.L[2] * rint(dz[u] * gs.invL[2]);
                        }
                        r2[u] = dx[u] * dx[u] + dy[u] * dy[u];
                        r2[u] = r2[u] + dz[u] * dz[u];
                    }
                    in[u] = live && qj[u] != kAbsentQ && r2[u] < A.rc2;
                }
                if (EMIT) {
#pragma unroll
                    for (int u = 0; u < NU; ++u)
                        emit_pairs(in[u], ent_g, A.perm, ai, in[u] ? idx[u] : 0u,
                                   &A.dsc->pair_count, A.emit, A.emit_max);
                }
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const double rr = in[u] ? r2[u] : 1.0;
                    const int qq = (HYBRID || QLJ) && !in[u] ? 0 : qj[u];
                    double c6 = c_row[tj[u]].x, c12 = c_row[tj[u]].y;
                    if (QLJ) qlj_scale64(A.qlj, ti, tj[u], qi_n, qq, &c6, &c12);
                    double f, e;
                    if (HYBRID) {
                        pair_terms_hybrid64(rr, kap, qi_n, qq, c6, c12, SCREEN_LJ, hrow,
                                            A.hyb_q, &f, &e);
                    } else {
                        // 1/r from one reciprocal square root; r, 1/r^2, q_i q_j / r follow
                        const double rinv = rsqrt(rr);
                        const double r = rr * rinv;
                        const double rinv2 = rinv * rinv;
                        const double rinv6 = rinv2 * rinv2 * rinv2;
                        const double s = exp_nonpos64(-kap * r);
                        const double uc = qi * (double)qq * rinv;
                        const double l12 = c12 * rinv6 * rinv6, l6 = c6 * rinv6;
                        if (SCREEN_LJ) {
                            const double uu = uc + (l12 - l6);
                            f = ((uc + 12.0 * l12 - 6.0 * l6) + uu * (kap * r)) * s * rinv2;
                            e = uu * s;
                        } else {
                            f = (uc + uc * (kap * r)) * s * rinv2 +
                                (12.0 * l12 - 6.0 * l6) * rinv2;
                            e = uc * s + (l12 - l6);
                        }
                    }
                    // (finite separations: a dropped pair adds exact zeros)
                    const double fi = in[u] ? f : 0.0;
                    Fx += fi * dx[u];
                    Fy += fi * dy[u];
                    Fz += fi * dz[u];
                    if (ENERGY) eacc += in[u] ? e : 0.0;
                }
            };
            // lane (i, k) takes codes 4k .. 4k + 3 of rows rp, rp + nrp, ... of atom i's
            // half-list (one 8-byte load per row, the next one issued a row ahead)
            using C1 = std::integral_constant<int, 1>;
            using C2 = std::integral_constant<int, 2>;
            using C3 = std::integral_constant<int, 3>;
            using C4 = std::integral_constant<int, 4>;
            for (int hh = half; hh < half + nhalf; ++hh) {
                nr = __builtin_amdgcn_readfirstlane(A.cl_nt[(int64_t)I * 2 + hh]);
                const int nt = __builtin_amdgcn_readfirstlane(
                    tail_cols(A.cl_len[(int64_t)I * 2 + hh], nr));
                const auto cp = gbl(reinterpret_cast<const uint64_t*>(
                                    A.nb + (((int64_t)I * 2 + hh) * kCluster + il) * A.nb_cap_h)) +
                                k8;
                auto rows = [&](auto st_c, auto per_c) {
                    uint64_t nxt = rp < nr ? (uint64_t)cp[rp * 8] : 0ull;
                    int r = rp;
                    for (; r < nr - 1; r += nrp) {
                        const uint64_t cur = nxt;
                        if (r + nrp < nr) nxt = cp[(r + nrp) * 8];
                        row(cur, st_c, per_c, C4{});
                    }
                    if (r == nr - 1) {   // the last row (in nxt): its columns in use only
                        if (nt >= 4) row(nxt, st_c, per_c, C4{});
                        else if (nt == 3) row(nxt, st_c, per_c, C3{});
                        else if (nt == 2) row(nxt, st_c, per_c, C2{});
                        else row(nxt, st_c, per_c, C1{});
                    }
                };
                using T_ = std::true_type;
                using F_ = std::false_type;
                if (staged) {
                    if (gs.periodic) rows(T_{}, T_{});
                    else rows(T_{}, F_{});
                } else {
                    if (gs.periodic) rows(F_{}, T_{});
                    else rows(F_{}, F_{});
                }
            }
            Fx = reduce8(Fx);
            Fy = reduce8(Fy);
            Fz = reduce8(Fz);
            if (ENERGY) eacc = reduce8(eacc);
        }
        // combine the waves of each cluster in a fixed order (deterministic)
        if (k8 == 0) {
            s_part[w][il][0] = Fx;
            s_part[w][il][1] = Fy;
            s_part[w][il][2] = Fz;
            s_part[w][il][3] = eacc;
        }
        __syncthreads();
        if (sub == 0 && k8 == 0 && ai >= 0) {
            double F[4] = {0.0, 0.0, 0.0, 0.0};
            for (int h = 0; h < wpc; ++h)
                for (int d = 0; d < 4; ++d) F[d] += s_part[w + h][il][d];
            A.fx[ai] = F[0];
            A.fy[ai] = F[1];
            A.fz[ai] = F[2];
            if (EMIT && ENERGY && A.e_atom) A.e_atom[ai] = 0.5 * F[3];
        }
        if (ENERGY && tid == 0) {
            double t = 0.0;
            for (int k = 0; k < nw; ++k)
                for (int i = 0; i < kCluster; ++i) t += s_part[k][i][3];
            A.grp_epot[g] = 0.5 * t;        // each pair is visited from both atoms
        }
        if (tid == 0) s_g = (int)(gridDim.x + claim);
        __syncthreads();
        g = s_g;
    }
}

// ------------------------------------------------------------------ launch

size_t force32_lds_bytes(int E_cap, int hyb_q)
{
    // staged candidates (+ the far sentinel), the per-entry reach / self masks and the
    // hybrid-screening rows of the bound charge states
    return (size_t)(E_cap * kCluster + 1) * sizeof(float4) +
           (size_t)((E_cap * sizeof(uint16_t) + 15) & ~(size_t)15) +
           (size_t)hyb_q * sizeof(float4);
}

template <bool E, bool M, bool S>
static void set_lds_attr(size_t lds)
{
    (void)hipFuncSetAttribute((const void*)k_force32<E, M, S>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int lds_h = (int)(lds + MD_MAX_CHARGE_STATES * sizeof(float4));
    (void)hipFuncSetAttribute((const void*)k_force32<E, M, S, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_h);
    (void)hipFuncSetAttribute((const void*)k_force32<E, M, S, false, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_force32<E, M, S, false, true, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_h);
}

template <bool E, bool M, bool S>
static void set_lds_attr64(size_t lds)
{
    (void)hipFuncSetAttribute((const void*)k_force64<E, M, S, false, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_force64<E, M, S, true, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_force64<E, M, S, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_force64<E, M, S, true, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t force_kernel_setup(Ctx* c)
{
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, (const void*)k_force32<true, false, true>) == hipSuccess)
        c->force32_static_lds = fa.sharedSizeBytes;
    if (hipFuncGetAttributes(&fa, (const void*)k_force32<true, false, true, false, true, true>) ==
        hipSuccess)
        c->force32_static_lds_h = fa.sharedSizeBytes;      // the largest variant
    const size_t lds = force32_lds_bytes(c->E_cap);
    set_lds_attr<false, false, false>(lds); set_lds_attr<false, false, true>(lds);
    set_lds_attr<true, false, false>(lds);  set_lds_attr<true, false, true>(lds);
    set_lds_attr<false, true, false>(lds);  set_lds_attr<false, true, true>(lds);
    set_lds_attr<true, true, false>(lds);   set_lds_attr<true, true, true>(lds);
    (void)hipFuncSetAttribute((const void*)k_force32<false, false, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    // FP64 kernel: staged tables when they fit one work-group's LDS
    if (hipFuncGetAttributes(&fa, (const void*)k_force64<true, true, true, true, true>) ==
        hipSuccess)
        c->force64_static_lds = fa.sharedSizeBytes;
    const size_t lds64 = force64_lds_bytes(c->E_cap);
    c->stage64 = lds64 + c->force64_static_lds <= c->max_lds;
    if (c->stage64) {
        set_lds_attr64<false, false, false>(lds64); set_lds_attr64<false, false, true>(lds64);
        set_lds_attr64<true, false, false>(lds64);  set_lds_attr64<true, false, true>(lds64);
        set_lds_attr64<false, true, false>(lds64);  set_lds_attr64<false, true, true>(lds64);
        set_lds_attr64<true, true, false>(lds64);   set_lds_attr64<true, true, true>(lds64);
    }
    return hipGetLastError();
}

// FP64 kernel launch shape: work-groups per CU as the LDS allows (at most 4), waves
// per i-cluster (even: whole half-lists per pair of waves; one for groups of 8) for
// up to 16 waves per CU within the 512-thread work-group.  Work-groups of 512
// threads leave each wave 256 VGPRs, so the four pairs of a row overlap their FP64
// chains: faster than 1,024 threads at 128 VGPRs (10.3 against 11.2 ms per launch
// on the 4.19 M-atom box, one work-group per CU either way, limited by the LDS).
static void force64_shape(const Ctx* c, int* per_cu, int* wpc)
{
    const size_t lds = (c->stage64 ? force64_lds_bytes(c->E_cap) : 0) + c->force64_static_lds;
    const int p = (int)std::min<size_t>(4, std::max<size_t>(1, c->lds_per_cu / lds));
    const int wmax = std::max(1, kForce64Block / 64 / c->G);
    int w = std::max(1, std::min(wmax, 16 / (c->G * p)));
    if (w > 1) w &= ~1;
    *per_cu = std::max(1, std::min(p, 16 / (c->G * w)));
    *wpc = w;
}

template <bool E, bool M, bool S, bool H, bool Q>
static void launch_one(Ctx* c, md_precision prec, const ForceArgs& A, int blocks, hipStream_t st)
{
    if (prec == MD_FP32_KAHAN)
        hipLaunchKernelGGL((k_force32<E, M, S, false, H, Q>), dim3(blocks),
                           dim3(64 * c->G * A.wpc), force32_lds_bytes(c->E_cap, H ? c->hyb_q : 0),
                           st, A);
    else
        hipLaunchKernelGGL((k_force64<E, M, S, H, Q>), dim3(blocks), dim3(64 * c->G * A.wpc),
                           c->stage64 ? force64_lds_bytes(c->E_cap) : 0, st, A);
}

template <bool E, bool M, bool S>
static void launch_sh(Ctx* c, md_precision prec, const ForceArgs& A, int blocks, hipStream_t st)
{
    if (c->hybrid) {
        if (c->ff_qlj) launch_one<E, M, S, true, true>(c, prec, A, blocks, st);
        else launch_one<E, M, S, true, false>(c, prec, A, blocks, st);
    } else {
        if (c->ff_qlj) launch_one<E, M, S, false, true>(c, prec, A, blocks, st);
        else launch_one<E, M, S, false, false>(c, prec, A, blocks, st);
    }
}

ForceFinalizeArgs force_finalize_args(Ctx* c, double* epot)
{
    return ForceFinalizeArgs{c->d_grp_epot, epot, c->d_sys_grp0, c->B, c->d_fast_list,
                             c->d_fast_e, c->d_sys_off, c->dsc,
                             c->n_bonds + c->n_angles > 0 ? c->d_bond_e : nullptr,
                             c->d_bond_blk, kBondedBlock, c->N};
}

hipError_t launch_forces(Ctx* c, md_precision prec, const double* x, const double* y,
                         const double* z, const int8_t* q, double* fx, double* fy, double* fz,
                         double* epot, int2* emit, int64_t emit_max, hipStream_t st,
                         hipEvent_t ev0, hipEvent_t ev1, bool finalize)
{
    ForceArgs A;
    A.groups = c->d_groups; A.ent = c->d_ent; A.nb = c->d_nb; A.cl_nt = c->d_cl_nt;
    A.perm = c->d_perm; A.slot_img = c->d_slot_img; A.xs = c->d_xs; A.qs = c->d_qs; A.ts = c->d_ts;
    A.xo = c->d_xo; A.cl_lo = c->d_cl_lo;
    A.grid = c->d_grid; A.kappa = c->d_kappa; A.S1 = c->n_steps + 1;
    A.lj32 = c->d_lj32; A.c6 = c->d_c6; A.c12 = c->d_c12; A.T = c->T_lj;
    A.rc2 = c->cfg.rc * c->cfg.rc;
    A.E_cap = c->E_cap; A.cap_slots = c->cap_slots;
    A.fx = fx; A.fy = fy; A.fz = fz;
    A.grp_epot = c->d_grp_epot; A.epot = epot; A.sys_grp0 = c->d_sys_grp0; A.B = c->B;
    A.dsc = c->dsc; A.emit = emit; A.emit_max = emit_max;
    A.wpc = kMaxWpc; A.stage64 = 0;
    A.cl_len = c->d_cl_len; A.ent_mask = c->d_ent_mask; A.nb_cap_h = c->nb_cap_h;
    A.hyb32 = c->d_hyb32; A.hyb64 = c->d_hyb64; A.hyb_q = c->hyb_q;
    A.qlj = c->d_qlj;
    A.excl_off = c->ff_excl ? c->d_excl_off : nullptr; A.excl = c->d_excl; A.t_excl = c->T;
    A.inv_perm = c->d_inv_perm;
    A.e_atom = emit ? c->dbg_e_atom : nullptr;
    {
        const double m = c->rlist * (1.0 + 1e-5);
        A.thr2 = (float)(m * m);
    }
    // persistent grid: as many work-groups as fit on every CU at once (LDS, waves)
    int per_cu32;
    {
        const size_t lds = force32_lds_bytes(c->E_cap, c->hybrid ? c->hyb_q : 0) +
                           (c->hybrid ? c->force32_static_lds_h : c->force32_static_lds);
        per_cu32 = (int)std::max<size_t>(1, c->lds_per_cu / lds);
        per_cu32 = std::min(per_cu32, std::max(1, 32 / (c->G * A.wpc)));
    }
    int per_cu = per_cu32;
    if (prec == MD_FP64) {
        // the FP32 kernel's list builder, alone (the FP32 force kernel builds its own)
        const int lb = (int)std::max<int64_t>(
            1, std::min<int64_t>(c->cap_groups, (int64_t)c->n_cu * per_cu32));
        hipLaunchKernelGGL((k_force32<false, false, false, true>), dim3(lb),
                           dim3(64 * c->G * A.wpc), force32_lds_bytes(c->E_cap), st, A);
        force64_shape(c, &per_cu, &A.wpc);
        A.stage64 = c->stage64 ? 1 : 0;
    }
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>(c->cap_groups, (int64_t)c->n_cu * per_cu));
    const bool E = epot != nullptr, M = emit != nullptr, S = c->cfg.screen_lj != 0;
    if (ev0) {
        const hipError_t e = hipEventRecord(ev0, st);
        if (e != hipSuccess) return e;
    }
    if (E) {
        if (M) { if (S) launch_sh<true, true, true>(c, prec, A, blocks, st); else launch_sh<true, true, false>(c, prec, A, blocks, st); }
        else   { if (S) launch_sh<true, false, true>(c, prec, A, blocks, st); else launch_sh<true, false, false>(c, prec, A, blocks, st); }
    } else {
        if (M) { if (S) launch_sh<false, true, true>(c, prec, A, blocks, st); else launch_sh<false, true, false>(c, prec, A, blocks, st); }
        else   { if (S) launch_sh<false, false, true>(c, prec, A, blocks, st); else launch_sh<false, false, false>(c, prec, A, blocks, st); }
    }
    if (ev1) {
        const hipError_t e = hipEventRecord(ev1, st);
        if (e != hipSuccess) return e;
    }
    if (c->fast_cap > 0) launch_fast(c, x, y, z, q, fx, fy, fz, E, emit, emit_max, st);
    if (c->n_bonds + c->n_angles > 0) launch_bonded(c, x, y, z, q, fx, fy, fz, st);
    if (finalize)
        hipLaunchKernelGGL(k_force_finalize, dim3(fin_blocks(c->B)), dim3(256), 0, st,
                           force_finalize_args(c, epot));
    return hipGetLastError();
}

}  // namespace md
