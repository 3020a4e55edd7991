// md_internal.h -- context layout, constants and device helpers shared by the
// library's translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <vector>

#include "md.h"

namespace md {

// Coulomb constant 1/(4 pi eps0) in kJ mol^-1 nm e^-2 (CODATA 2018 e, N_A, eps0).
constexpr double kKe = 138.935457644382;

constexpr int kCluster = 8;          // atoms per cluster (one i-cluster per 64-lane wave)
constexpr int kWave = 64;
constexpr int kMaxGroup = 8;         // i-clusters per force work-group
constexpr int kCodeIdxBits = 13;     // neighbour code: staged-atom index | type << 13
constexpr uint32_t kCodeIdxMask = (1u << kCodeIdxBits) - 1u;
constexpr int kMaxGroupEntries = (1 << kCodeIdxBits) / kCluster - 1;   // 1023
constexpr uint32_t kEntClusterMask = (1u << 26) - 1u;                  // group entry: J | shift << 26
constexpr int kScanBlock = 1024;
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kScanBlock * kScanPerThread;

// Per-system grid used to bin atoms into columns (x, y) and fine z bins.
struct GridSys {
    double origin[3];
    double w[3];        // column widths in x, y; z-bin width in z
    double inv_w[3];
    double L[3];        // periodic box lengths (0 when vacuum)
    double invL[3];
    int32_t n[3];       // columns in x, y; bins in z
    int32_t col_off;    // first global column of this system
    int32_t bin_off;    // first global bin
    int32_t periodic;
};

// A work-group's set of i-clusters: consecutive clusters of one column.
struct Group {
    double lo[3], hi[3];    // bounding box of its atoms at build time (wrapped frame)
    double c[3];            // frame origin (box centre)
    int32_t cl0, ncl;       // first cluster, number of clusters (<= cluster_group)
    int32_t sys;
    int32_t nent;           // candidate (cluster, shift) entries kept (<= capacity)
    int32_t nent_raw;       // candidates found (a larger value means overflow)
    int32_t pad_;
};

// Device-resident scalars (one allocation).
struct DevScalars {
    int64_t step;               // index of the latest force evaluation
    uint32_t flags;             // MD_FLAG_* error word
    int32_t need_rebuild;       // set when a displacement exceeds skin/2
    int32_t lists_pending;      // candidate tables rebuilt; per-atom lists not yet rebuilt
    unsigned long long disp2_bits;  // max squared displacement since build (double bits)
    int32_t n_cols, n_bins, n_clusters, n_groups;
    int32_t n_slots;
    int64_t n_builds;
    uint32_t work_force;        // work-queue counter of the force kernel
    unsigned long long pair_count;  // debug pair export counter
    int32_t n_fast;             // atoms beyond skin/2 of their build position (<= capacity)
    int32_t n_fast_raw;         // the same, uncapped (above the capacity a rebuild is due)
    uint32_t bar_gen, bar_pad_;     // grid barrier generation of the fused build kernel
};

struct Ctx {
    md_config cfg;
    int B = 0;
    int64_t N = 0;
    std::string err;
    bool tables_bound = false;
    bool built = false;
    int device = 0;
    int n_cu = 0;
    size_t max_lds = 65536;        // per work-group
    size_t lds_per_cu = 65536;
    size_t force32_static_lds = 8192;
    int bs_blocks = 0;             // grid of the fused build kernel (0: not usable)
    // Langevin coupling (bound by md_bind_langevin)
    bool langevin = false;
    double lg_dt = 0.0;
    double* d_lg_c1 = nullptr;     // B*E: exp(-gamma dt)
    double* d_lg_kt = nullptr;     // B*(S+1): k_B T_e, kJ/mol
    // hybrid ion-sphere / Debye screening (bound by md_bind_hybrid): per (system,
    // step, charge) the coefficients {r', c1, c2, c3}
    bool hybrid = false;
    size_t force32_static_lds_h = 0;   // static LDS of the hybrid FP32 force kernel
    size_t force64_static_lds = 0;     // static LDS of the FP64 force kernel
    bool stage64 = false;              // FP64 kernel: group tables fit the LDS
    int32_t hyb_q = 0;             // charges tabulated (0 .. hyb_q - 1)
    double* d_hyb64 = nullptr;     // B*(S+1)*hyb_q*4
    float4* d_hyb32 = nullptr;     // B*(S+1)*hyb_q
    uint8_t* d_rdf_moved = nullptr;   // N: atoms beyond skin/2 of the build (histogram pass)
    // force-field terms (bound by md_bind_forcefield)
    int32_t T_lj = 0;              // stride of the LJ tables: T, or T + 1 with exclusions
                                   // (type T is the "LJ excluded" pseudo-type, all zero)
    bool ff_qlj = false;           // LJ radii scaled with the charge
    double* d_qlj = nullptr;       // kQljLen (0 for the pseudo-type)
    bool ff_excl = false;
    int32_t* d_excl_off = nullptr; // N+1: per-atom LJ-excluded partners (CSR, sorted)
    int32_t* d_excl = nullptr;
    int64_t n_bonds = 0, n_angles = 0;
    int32_t* d_bonds = nullptr;    double* d_bond_par = nullptr;      // [n][2], [n][3]
    int32_t* d_angles = nullptr;   double* d_angle_par = nullptr;     // [n][3], [n][2]
    int32_t* d_bt_off = nullptr;   // N+1: per-atom incident bonded terms (CSR)
    int32_t* d_bt = nullptr;       // term id * 2 + kind (0 bond, 1 angle)
    double* d_bond_e = nullptr;    // N: energy of the bonded terms whose first atom is a
    double* d_bond_blk = nullptr;  // per bonded work-group: the sum of its atoms' d_bond_e
    double* d_rdf_xr = nullptr;       // cap_slots*3: slot-order current positions
    uint8_t* d_rdf_er = nullptr;      // cap_slots: slot-order elements
    int cap_bar = 0;               // arrival words of its barrier
    uint32_t* d_bar_arrive = nullptr;
    // per-atom energies e_i = 1/2 sum_j phi_ij written by the debug force launch
    // (md_debug_pairs), NULL otherwise
    double* dbg_e_atom = nullptr;
    // force-kernel launch timer: event pairs recorded around the next t_cap launches
    std::vector<hipEvent_t> t_ev;
    int t_cap = 0, t_n = 0;

    // host copies
    std::vector<int64_t> sys_off;
    std::vector<double> box;       // B*3 (periodic)
    std::vector<double> lambda_d;  // B*(S+1) Debye lengths as bound (nm; +inf: unscreened)
    std::vector<double> h_c6, h_c12;   // T*T as bound
    int64_t n_steps = 0;
    int32_t T = 0, E = 0, Q = 0;
    int32_t G = 4;                 // i-clusters per group
    int32_t E_cap = 0;             // entries per group
    int32_t nb_cap = 0;            // per-atom list capacity (both halves)
    int32_t nb_cap_h = 0;          // per-atom capacity of one half-list (multiple of 32)
    double rlist = 0.0;            // rc + skin

    // capacities
    int64_t cap_cols = 0, cap_bins = 0, cap_clusters = 0, cap_slots = 0, cap_groups = 0;
    int64_t cap_partials = 0;

    // device buffers
    DevScalars* dsc = nullptr;
    int64_t* d_sys_off = nullptr;        // B+1
    int32_t* d_sys_of_atom = nullptr;    // N
    GridSys* d_grid = nullptr;           // B
    double* d_sys_lo = nullptr;          // B*3 (vacuum bounding boxes)
    double* d_sys_hi = nullptr;
    int32_t* d_sys_grp0 = nullptr;       // B+1 first group per system
    // tables
    double* d_c6 = nullptr;   double* d_c12 = nullptr;     // T*T
    float* d_lj32 = nullptr;                               // T*T*2 (c6, c12) float
    int8_t* d_qmax = nullptr;                              // E
    double* d_kappa = nullptr;                             // B*(S+1)
    double* d_base = nullptr;                              // E*Q
    double* d_g = nullptr;                                 // B*(S+1)
    uint64_t* d_seeds = nullptr;                           // B
    // binning
    int32_t* d_key = nullptr;      // N bin of each atom
    int32_t* d_rank = nullptr;     // N rank inside the bin
    int32_t* d_img = nullptr;      // N packed periodic image of each atom at build
    int32_t* d_bin_cnt = nullptr;  // cap_bins + 1
    int32_t* d_bin_start = nullptr;// cap_bins + 1
    int32_t* d_sorted = nullptr;   // N atoms in bin order
    int64_t* d_scan_tmp = nullptr; // block sums for the scans
    // columns: (groups << 32 | clusters) per column and its exclusive prefix
    int64_t* d_col_cnt = nullptr;  int64_t* d_col_pre = nullptr;       // cap_cols + 1
    // clusters / slots
    double* d_cl_lo = nullptr;     double* d_cl_hi = nullptr;          // cap_clusters*3
    int32_t* d_cl_nt = nullptr;    // cap_clusters * 2: rows (32 codes per atom) of each half-list
    int32_t* d_cl_len = nullptr;   // cap_clusters * 2: longest half-list of the cluster (stats)
    int32_t* d_perm = nullptr;     // cap_slots: caller atom of each slot (-1 = padding)
    int32_t* d_slot_img = nullptr; // cap_slots: packed image of the slot's atom
    int32_t* d_inv_perm = nullptr; // N
    double* d_xs = nullptr;        // cap_slots*3 positions in slot order (SoA x|y|z)
    float4* d_xo = nullptr;        // cap_slots: offsets from the cluster's box corner, charge
    int8_t* d_qs = nullptr;        // cap_slots charges in slot order
    uint8_t* d_ts = nullptr;       // cap_slots types in slot order (build time)
    // groups and lists
    Group* d_groups = nullptr;     // cap_groups
    uint32_t* d_ent = nullptr;     // cap_groups * E_cap
    uint8_t* d_ent_mask = nullptr; // cap_groups * E_cap: group clusters each entry can reach
    uint16_t* d_nb = nullptr;      // cap_clusters * 2 * 8 * nb_cap_h: (cluster, half, atom) lists
    double* d_grp_epot = nullptr;  // cap_groups
    // integrator
    double* d_xref = nullptr;      // N*3 build positions
    double* d_partial = nullptr;   // cap_partials (kinetic-energy block partials)
    // the same partials for the fused step, each published as one device-scope atomic
    // word (kEkSlotEmpty when not yet written; the reader empties them again)
    unsigned long long* d_ek_slots = nullptr;   // cap_partials
    // atoms that moved more than skin/2 since the last build
    int32_t fast_cap = 0;
    uint8_t* d_fast_flag = nullptr;   // N
    int32_t* d_fast_loc = nullptr;    // vv blocks * block size: per-block lists
    int32_t* d_fast_cnt = nullptr;    // vv blocks
    int32_t* d_fast_list = nullptr;   // fast_cap, ascending atom index
    double* d_fast_e = nullptr;       // fast_cap: energy of each fast atom's pairs
    uint8_t* d_atype = nullptr;       // N: types in caller order (build time)
};

// Table of the charge-scaled LJ radii (section II.B, Eq. 11): the radius of atom i
// shrinks to c_i sigma_i with c_i = 1 - q_i/Z_i, a pair's radius is the mean of the
// two, so its LJ radius scales by s = (c_i sigma_i + c_j sigma_j)/(sigma_i + sigma_j).
// FP64 (both paths evaluate the scale in FP64: sigma - q sigma/Z cancels when q
// approaches Z, and s enters as s^12): [1/Z_t | sigma_t | sigma_t/Z_t |
// 1/(sigma_i + sigma_j) (0 when both are 0), row stride MD_MAX_TYPES].
constexpr int kQljInvZ = 0, kQljSig = MD_MAX_TYPES, kQljSigZ = 2 * MD_MAX_TYPES;
constexpr int kQljRs = 3 * MD_MAX_TYPES;
constexpr int kQljLen = 3 * MD_MAX_TYPES + MD_MAX_TYPES * MD_MAX_TYPES;

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- device helpers

// Packed periodic image (kx, ky, kz), 10 signed bits each.
__host__ __device__ inline int32_t pack_img(int kx, int ky, int kz)
{
    return ((kx & 1023) << 20) | ((ky & 1023) << 10) | (kz & 1023);
}
__host__ __device__ inline int unpack_img(int32_t v, int axis)
{
    int s = (axis == 0) ? 20 : (axis == 1 ? 10 : 0);
    int t = (v >> s) & 1023;
    return (t & 512) ? t - 1024 : t;
}

__device__ inline void set_flag(DevScalars* d, uint32_t f)
{
    atomicOr(&d->flags, f);
}

// Minimum-image squared distance with every operation a separately rounded FP64
// operation in this order (no contraction): d = a - b; d -= L rint(d * (1/L));
// r2 = (dx*dx + dy*dy) + dz*dz.  This is the membership test of the pair set.
__device__ inline double pair_r2_exact(double xi, double yi, double zi, double xj, double yj,
                                       double zj, const GridSys& g)
{
#pragma clang fp contract(off)
    double dx = xi - xj;
    double dy = yi - yj;
    double dz = zi - zj;
    if (g.periodic) {
        dx = dx - g.L[0] * rint(dx * g.invL[0]);
        dy = dy - g.L[1] * rint(dy * g.invL[1]);
        dz = dz - g.L[2] * rint(dz * g.invL[2]);
    }
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    return r2;
}

}  // namespace md
