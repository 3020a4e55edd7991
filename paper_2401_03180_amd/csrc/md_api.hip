// md_api.hip -- host side of the C ABI declared in include/md.h: argument
// validation, workspace sizing and allocation, table upload and launch order.
#include <math.h>
#include <string.h>
#include <stdarg.h>

#include <algorithm>
#include <utility>
#include <vector>
#include <cstdio>
#include <new>

#include "md_internal.h"
#include "md_launch.h"

using namespace md;

struct md_ctx {
    Ctx c;
};

namespace {

thread_local std::string g_create_err;

md_status fail(Ctx* c, md_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_create_err = buf;
    return s;
}

#define HIP_TRY(c, expr)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((c), MD_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

template <class T>
hipError_t dalloc(T** p, int64_t count)
{
    if (count <= 0) count = 1;
    return hipMalloc((void**)p, sizeof(T) * (size_t)count);
}

void free_all(Ctx* c)
{
    void* ptrs[] = {c->dsc, c->d_sys_off, c->d_sys_of_atom, c->d_grid, c->d_sys_lo, c->d_sys_hi,
                    c->d_sys_grp0, c->d_c6, c->d_c12, c->d_lj32, c->d_qmax, c->d_kappa,
                    c->d_base, c->d_g, c->d_seeds, c->d_key, c->d_rank, c->d_img,
                    c->d_bin_cnt, c->d_bin_start, c->d_sorted, c->d_scan_tmp, c->d_col_cnt,
                    c->d_col_pre, c->d_cl_lo, c->d_cl_hi,
                    c->d_cl_nt, c->d_cl_len, c->d_perm, c->d_slot_img, c->d_inv_perm, c->d_xs, c->d_xo, c->d_qs,
                    c->d_ts, c->d_groups, c->d_ent, c->d_ent_mask, c->d_nb, c->d_grp_epot, c->d_xref,
                    c->d_partial, c->d_ek_slots, c->d_fast_flag, c->d_fast_loc, c->d_fast_cnt,
                    c->d_fast_list, c->d_fast_e, c->d_atype, c->d_bar_arrive,
                    c->d_lg_c1, c->d_lg_kt, c->d_hyb64, c->d_hyb32, c->d_rdf_moved,
                    c->d_rdf_xr, c->d_rdf_er, c->d_qlj, c->d_excl_off,
                    c->d_excl, c->d_bonds, c->d_bond_par, c->d_angles, c->d_angle_par,
                    c->d_bt_off, c->d_bt, c->d_bond_e, c->d_bond_blk};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

bool null_any(std::initializer_list<const void*> ps)
{
    for (const void* p : ps)
        if (!p) return true;
    return false;
}

hipStream_t S(md_stream s) { return reinterpret_cast<hipStream_t>(s); }

void free_timer(Ctx* c)
{
    for (hipEvent_t e : c->t_ev)
        if (e) (void)hipEventDestroy(e);
    c->t_ev.clear();
    c->t_cap = c->t_n = 0;
}

// Events for the next timed force launch, if the timer has room and the stream is
// not being captured into a graph.
void next_timer_events(Ctx* c, hipStream_t st, hipEvent_t* e0, hipEvent_t* e1)
{
    *e0 = *e1 = nullptr;
    if (c->t_n >= c->t_cap) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    *e0 = c->t_ev[2 * c->t_n];
    *e1 = c->t_ev[2 * c->t_n + 1];
    ++c->t_n;
}

}  // namespace

extern "C" {

const char* md_last_error(const md_ctx* ctx)
{
    return ctx ? ctx->c.err.c_str() : g_create_err.c_str();
}

md_status md_create(const md_config* cfg, const int64_t* sys_offsets, md_ctx** out)
{
    if (!out) return fail(nullptr, MD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || !sys_offsets) return fail(nullptr, MD_ERR_ARG, "cfg or sys_offsets is NULL");
    if (cfg->n_systems < 1) return fail(nullptr, MD_ERR_ARG, "n_systems must be >= 1");
    if (cfg->n_types < 1 || cfg->n_types > MD_MAX_TYPES)
        return fail(nullptr, MD_ERR_CAPACITY, "n_types must be in [1, %d]", MD_MAX_TYPES);
    if (cfg->n_elements < 1 || cfg->n_elements > MD_MAX_ELEMENTS)
        return fail(nullptr, MD_ERR_CAPACITY, "n_elements must be in [1, %d]", MD_MAX_ELEMENTS);
    if (cfg->n_charge_states < 1 || cfg->n_charge_states > MD_MAX_CHARGE_STATES)
        return fail(nullptr, MD_ERR_CAPACITY, "n_charge_states must be in [1, %d]",
                    MD_MAX_CHARGE_STATES);
    if (!(cfg->rc > 0.0) || !(cfg->skin > 0.0) || !isfinite(cfg->rc) || !isfinite(cfg->skin))
        return fail(nullptr, MD_ERR_ARG, "rc and skin must be finite and > 0");
    const int G = cfg->cluster_group ? cfg->cluster_group : 4;
    if (G != 1 && G != 2 && G != 4 && G != 8)
        return fail(nullptr, MD_ERR_ARG, "cluster_group must be 1, 2, 4 or 8");
    if (cfg->fast_capacity < -1 || cfg->fast_capacity > 65536)
        return fail(nullptr, MD_ERR_ARG, "fast_capacity must be in [-1, 65536]");
    if (sys_offsets[0] != 0) return fail(nullptr, MD_ERR_ARG, "sys_offsets[0] must be 0");
    for (int b = 0; b < cfg->n_systems; ++b)
        if (sys_offsets[b + 1] < sys_offsets[b])
            return fail(nullptr, MD_ERR_ARG, "sys_offsets must be non-decreasing");
    const int64_t N = sys_offsets[cfg->n_systems];
    if (N > cfg->capacity_atoms)
        return fail(nullptr, MD_ERR_CAPACITY, "%lld atoms exceed capacity_atoms %lld",
                    (long long)N, (long long)cfg->capacity_atoms);
    if (N >= (int64_t)1 << 30) return fail(nullptr, MD_ERR_CAPACITY, "at most 2^30 atoms");
    md_ctx* ctx = new (std::nothrow) md_ctx();
    if (!ctx) return fail(nullptr, MD_ERR_CAPACITY, "host allocation failed");
    Ctx* c = &ctx->c;
    c->cfg = *cfg;
    c->B = cfg->n_systems;
    c->N = N;
    c->G = G;
    c->sys_off.assign(sys_offsets, sys_offsets + c->B + 1);
    c->rlist = cfg->rc + cfg->skin;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount,
                                                   c->device);
    // the device address of the no-allocation histogram's fixed workspace, once per
    // device (its failure only disables that entry point)
    if (e == hipSuccess) (void)rdf_scratch_setup(c->device);
    int lds = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, MD_ERR_HIP, "no HIP device: %s", hipGetErrorString(e));
    }
    c->max_lds = (size_t)lds;
    int lds_cu = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              c->device) != hipSuccess || lds_cu <= 0)
        lds_cu = lds;
    c->lds_per_cu = (size_t)std::max(lds_cu, lds);
    *out = ctx;
    return MD_OK;
}

md_status md_destroy(md_ctx* ctx)
{
    if (!ctx) return MD_OK;
    (void)hipDeviceSynchronize();
    free_timer(&ctx->c);
    free_all(&ctx->c);
    delete ctx;
    return MD_OK;
}

static md_status upload_lj(Ctx* c, int stride);

static md_status size_and_allocate(Ctx* c)
{
    const md_config& cfg = c->cfg;
    const int64_t N = c->N;
    const int B = c->B;
    const double rl = c->rlist;
    // sizing density: the hint, else 1.1 x the densest periodic box, else 130 / nm^3
    double rho = cfg.density_hint;
    if (!(rho > 0.0)) {
        rho = 130.0;
        if (cfg.periodic) {
            double mx = 0.0;
            for (int b = 0; b < B; ++b) {
                const double* L = &c->box[3 * b];
                mx = std::max(mx, (double)(c->sys_off[b + 1] - c->sys_off[b]) /
                                      (L[0] * L[1] * L[2]));
            }
            rho = std::max(1.1 * mx, 1.0);
        }
    }
    const double a = cbrt(8.0 / rho);

    // periodic grids are fixed by the boxes
    std::vector<GridSys> grids(B);
    int64_t cols = 0, bins = 0;
    if (cfg.periodic) {
        for (int b = 0; b < B; ++b) {
            GridSys g{};
            const double* L = &c->box[3 * b];
            const double vol = L[0] * L[1] * L[2];
            const int64_t nb = c->sys_off[b + 1] - c->sys_off[b];
            const double wt = nb > 0 ? cbrt(8.0 * vol / (double)nb) : std::max({L[0], L[1], L[2]});
            g.n[0] = std::max(1, (int)(L[0] / wt));
            g.n[1] = std::max(1, (int)(L[1] / wt));
            g.n[2] = std::max(1, (int)(L[2] / (0.25 * wt)));
            for (int k = 0; k < 3; ++k) {
                g.origin[k] = 0.0;
                g.L[k] = L[k];
                g.invL[k] = 1.0 / L[k];
                g.w[k] = L[k] / g.n[k];
                g.inv_w[k] = 1.0 / g.w[k];
            }
            g.periodic = 1;
            g.col_off = (int32_t)cols;
            g.bin_off = (int32_t)bins;
            cols += (int64_t)g.n[0] * g.n[1];
            bins += (int64_t)g.n[0] * g.n[1] * g.n[2];
            grids[b] = g;
        }
        c->cap_cols = cols;
        c->cap_bins = bins;
    } else {
        c->cap_cols = N / 8 + B + 1;
        c->cap_bins = 2 * N + 16 * (int64_t)B + 1;
    }
    if (c->cap_bins >= ((int64_t)kScanTile * kScanTile - 1) || c->cap_bins >= INT32_MAX / 2)
        return fail(c, MD_ERR_CAPACITY, "grid too large (%lld bins)", (long long)c->cap_bins);
    c->cap_clusters = N / kCluster + c->cap_cols + B + 1;
    c->cap_slots = c->cap_clusters * kCluster;
    c->cap_groups = c->cap_clusters;

    // group candidate-table capacity from the rounded-box volume around a group; the
    // force and list kernels stage one group's candidates in LDS, so the capacity is
    // also bounded by the LDS of one work-group (the group size shrinks if needed)
    int G = c->G;
    int E_cap = 0;
    for (;;) {
        const double X = 2.0 * a, Y = 2.0 * a, Z = (G + 1) * a;
        const double V = X * Y * Z + 2.0 * rl * (X * Y + X * Z + Y * Z) +
                         M_PI * rl * rl * (X + Y + Z) + 4.0 / 3.0 * M_PI * rl * rl * rl;
        // vacuum grids follow each system's bounding box, whose columns widen as a
        // cluster expands (ions leaving it stretch the box): more headroom there.  A
        // group of 8 clusters often spans two columns: on a periodic water box its
        // table reached 1.4 times the box volume's count (groups of 4: 1.25); more
        // headroom would pass the 1,023 entries a list code can index
        const double safety = cfg.periodic ? (G >= 8 ? 1.6 : 1.35) : 2.4;
        const int est = (int)(V * rho / kCluster * safety) + 16;
        E_cap = std::min(est, kMaxGroupEntries);
        while (E_cap > 32 &&
               force32_lds_bytes(E_cap, MD_MAX_CHARGE_STATES) + 8192 > c->max_lds)
            E_cap -= 8;
        if (E_cap >= est || G == 1) break;
        G /= 2;
    }
    if (E_cap < 32) return fail(c, MD_ERR_CAPACITY, "LDS too small for the candidate table");
    // the force kernel addresses the candidate tables and the slot arrays with 32-bit
    // byte offsets
    if ((uint64_t)c->cap_groups * (uint64_t)E_cap * 4u >= ((uint64_t)1 << 32) ||
        (uint64_t)c->cap_slots * 16u >= ((uint64_t)1 << 32))
        return fail(c, MD_ERR_CAPACITY, "system too large for the force kernel's 32-bit offsets "
                    "(%lld groups x %d entries)", (long long)c->cap_groups, E_cap);
    c->G = G;
    c->E_cap = E_cap;
    int nb_cap = cfg.max_neighbors;
    if (nb_cap <= 0) nb_cap = (int)(4.0 / 3.0 * M_PI * rl * rl * rl * rho * 1.2) + 16;
    nb_cap = (nb_cap + 7) & ~7;
    c->nb_cap = nb_cap;
    // two half-lists per atom (entries of even / odd index), each with some slack
    c->nb_cap_h = ((nb_cap / 2 + nb_cap / 16 + 8) + 31) & ~31;     // rows of 32 codes
    c->cap_partials = vv_partials_needed(N, B);
    // fast-atom capacity: beyond it a rebuild is due (-1: rebuild on the first fast atom)
    if (cfg.fast_capacity < 0) c->fast_cap = 0;
    else if (cfg.fast_capacity > 0) c->fast_cap = cfg.fast_capacity;
    else c->fast_cap = (int)std::min<int64_t>(1024, std::max<int64_t>(64, N / 96));

    // allocation
    HIP_TRY(c, dalloc(&c->dsc, 1));
    HIP_TRY(c, dalloc(&c->d_sys_off, B + 1));
    HIP_TRY(c, dalloc(&c->d_sys_of_atom, N));
    HIP_TRY(c, dalloc(&c->d_grid, B));
    HIP_TRY(c, dalloc(&c->d_sys_lo, 3 * B));
    HIP_TRY(c, dalloc(&c->d_sys_hi, 3 * B));
    HIP_TRY(c, dalloc(&c->d_sys_grp0, B + 1));
    HIP_TRY(c, dalloc(&c->d_key, N));
    HIP_TRY(c, dalloc(&c->d_rank, N));
    HIP_TRY(c, dalloc(&c->d_img, N));
    HIP_TRY(c, dalloc(&c->d_bin_cnt, c->cap_bins + 1));
    HIP_TRY(c, dalloc(&c->d_bin_start, c->cap_bins + 1));
    HIP_TRY(c, dalloc(&c->d_sorted, N));
    HIP_TRY(c, dalloc(&c->d_scan_tmp, kScanTile + 64));
    HIP_TRY(c, dalloc(&c->d_col_cnt, c->cap_cols + 1));
    HIP_TRY(c, dalloc(&c->d_col_pre, c->cap_cols + 1));
    HIP_TRY(c, dalloc(&c->d_cl_lo, 3 * c->cap_clusters));
    HIP_TRY(c, dalloc(&c->d_cl_hi, 3 * c->cap_clusters));
    HIP_TRY(c, dalloc(&c->d_cl_nt, 2 * c->cap_clusters));
    HIP_TRY(c, dalloc(&c->d_cl_len, 2 * c->cap_clusters));
    HIP_TRY(c, dalloc(&c->d_perm, c->cap_slots));
    HIP_TRY(c, dalloc(&c->d_slot_img, c->cap_slots));
    HIP_TRY(c, dalloc(&c->d_inv_perm, N));
    HIP_TRY(c, dalloc(&c->d_xs, 3 * c->cap_slots));
    HIP_TRY(c, dalloc(&c->d_xo, c->cap_slots));
    HIP_TRY(c, dalloc(&c->d_qs, c->cap_slots));
    HIP_TRY(c, dalloc(&c->d_ts, c->cap_slots));
    HIP_TRY(c, dalloc(&c->d_groups, c->cap_groups));
    HIP_TRY(c, dalloc(&c->d_ent, c->cap_groups * (int64_t)E_cap));
    HIP_TRY(c, dalloc(&c->d_ent_mask, c->cap_groups * (int64_t)E_cap));
    HIP_TRY(c, dalloc(&c->d_nb, c->cap_clusters * 2 * kCluster * (int64_t)c->nb_cap_h));
    HIP_TRY(c, dalloc(&c->d_grp_epot, c->cap_groups));
    HIP_TRY(c, dalloc(&c->d_xref, 3 * N));
    HIP_TRY(c, dalloc(&c->d_partial, c->cap_partials));
    HIP_TRY(c, dalloc(&c->d_ek_slots, c->cap_partials));
    HIP_TRY(c, hipMemset(c->d_ek_slots, 0xFF, sizeof(unsigned long long) * c->cap_partials));
    {
        // per integrator work-group: its fast atoms (kVvBlock slots) and their count
        const int64_t nvb = div_up(std::max<int64_t>(N, 1), kVvBlock);
        HIP_TRY(c, dalloc(&c->d_fast_flag, std::max<int64_t>(N, 1)));
        HIP_TRY(c, dalloc(&c->d_fast_loc, nvb * kVvBlock));
        HIP_TRY(c, dalloc(&c->d_fast_cnt, nvb));
        HIP_TRY(c, dalloc(&c->d_fast_list, std::max(c->fast_cap, 1)));
        HIP_TRY(c, dalloc(&c->d_fast_e, std::max(c->fast_cap, 1)));
        HIP_TRY(c, dalloc(&c->d_atype, std::max<int64_t>(N, 1)));
        c->cap_bar = 8 * std::max(c->n_cu, 1);
        HIP_TRY(c, dalloc(&c->d_bar_arrive, c->cap_bar));
    }

    // initial contents
    DevScalars h{};
    h.need_rebuild = 1;
    h.n_cols = (int32_t)(cfg.periodic ? cols : 0);
    h.n_bins = (int32_t)(cfg.periodic ? bins : 0);
    HIP_TRY(c, hipMemcpy(c->dsc, &h, sizeof h, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_sys_off, c->sys_off.data(), sizeof(int64_t) * (B + 1),
                         hipMemcpyHostToDevice));
    {
        std::vector<int32_t> soa(std::max<int64_t>(N, 1));
        for (int b = 0; b < B; ++b)
            for (int64_t i = c->sys_off[b]; i < c->sys_off[b + 1]; ++i) soa[i] = b;
        HIP_TRY(c, hipMemcpy(c->d_sys_of_atom, soa.data(), sizeof(int32_t) * std::max<int64_t>(N, 1),
                             hipMemcpyHostToDevice));
    }
    if (cfg.periodic)
        HIP_TRY(c, hipMemcpy(c->d_grid, grids.data(), sizeof(GridSys) * B, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemset(c->d_perm, 0xFF, sizeof(int32_t) * c->cap_slots));
    HIP_TRY(c, hipMemset(c->d_bin_cnt, 0, sizeof(int32_t) * (c->cap_bins + 1)));
    HIP_TRY(c, hipMemset(c->d_cl_nt, 0, sizeof(int32_t) * 2 * c->cap_clusters));
    HIP_TRY(c, hipMemset(c->d_cl_len, 0, sizeof(int32_t) * 2 * c->cap_clusters));
    HIP_TRY(c, hipMemset(c->d_groups, 0, sizeof(Group) * c->cap_groups));
    HIP_TRY(c, hipMemset(c->d_xref, 0, sizeof(double) * 3 * std::max<int64_t>(N, 1)));
    HIP_TRY(c, hipMemset(c->d_sys_grp0, 0, sizeof(int32_t) * (B + 1)));
    HIP_TRY(c, hipMemset(c->d_grp_epot, 0, sizeof(double) * c->cap_groups));
    HIP_TRY(c, hipMemset(c->d_fast_flag, 0, std::max<int64_t>(N, 1)));
    HIP_TRY(c, hipMemset(c->d_atype, 0, std::max<int64_t>(N, 1)));
    HIP_TRY(c, hipMemset(c->d_bar_arrive, 0, sizeof(uint32_t) * c->cap_bar));
    HIP_TRY(c, hipMemset(c->d_fast_cnt, 0,
                         sizeof(int32_t) * div_up(std::max<int64_t>(N, 1), kVvBlock)));
    HIP_TRY(c, force_kernel_setup(c));
    HIP_TRY(c, build_step_setup(c));
    return MD_OK;
}

md_status md_bind_tables(md_ctx* ctx, const double* box, const double* c6, const double* c12,
                         const int8_t* qmax, const double* lambda_d, const double* base,
                         const double* g, const uint64_t* seeds, int64_t n_steps)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (null_any({c6, c12, qmax, lambda_d, base, g, seeds}))
        return fail(c, MD_ERR_ARG, "a table pointer is NULL");
    if (n_steps < 0) return fail(c, MD_ERR_ARG, "n_steps must be >= 0");
    if (c->cfg.periodic && !box) return fail(c, MD_ERR_ARG, "periodic systems need box");
    const int B = c->B, T = c->cfg.n_types, E = c->cfg.n_elements, Q = c->cfg.n_charge_states;
    if (c->cfg.periodic) {
        for (int b = 0; b < B; ++b)
            for (int k = 0; k < 3; ++k) {
                const double L = box[3 * b + k];
                if (!(L > 0.0) || !isfinite(L))
                    return fail(c, MD_ERR_ARG, "box[%d][%d] must be finite and > 0", b, k);
                if (L < 2.0 * c->rlist * (1.0 + 1e-4))
                    return fail(c, MD_ERR_GEOMETRY,
                                "box edge %.6g < 2 (rc + skin) = %.6g: images would overlap", L,
                                2.0 * c->rlist);
            }
    }
    for (int i = 0; i < T; ++i)
        for (int j = 0; j < T; ++j)
            if (c6[i * T + j] != c6[j * T + i] || c12[i * T + j] != c12[j * T + i])
                return fail(c, MD_ERR_ARG, "c6/c12 tables must be symmetric");
    for (int e = 0; e < E; ++e)
        if (qmax[e] < 0) return fail(c, MD_ERR_ARG, "qmax must be >= 0");
    if (c->tables_bound) {
        (void)hipDeviceSynchronize();
        free_timer(c);
        free_all(c);
        Ctx fresh;
        fresh.cfg = c->cfg; fresh.B = c->B; fresh.N = c->N; fresh.G = c->cfg.cluster_group ? c->cfg.cluster_group : 4;
        fresh.sys_off = c->sys_off; fresh.rlist = c->rlist; fresh.device = c->device;
        fresh.n_cu = c->n_cu; fresh.max_lds = c->max_lds; fresh.lds_per_cu = c->lds_per_cu;
        fresh.force32_static_lds = c->force32_static_lds;
        fresh.force32_static_lds_h = c->force32_static_lds_h;
        fresh.force64_static_lds = c->force64_static_lds;
        *c = fresh;
    }
    c->box.assign(c->cfg.periodic ? box : nullptr, c->cfg.periodic ? box + 3 * B : nullptr);
    c->n_steps = n_steps;
    c->T = T; c->E = E; c->Q = Q;
    md_status s = size_and_allocate(c);
    if (s != MD_OK) return s;
    const int64_t S1 = n_steps + 1;
    c->lambda_d.assign(lambda_d, lambda_d + (size_t)B * S1);
    std::vector<double> kappa((size_t)B * S1);
    for (size_t i = 0; i < kappa.size(); ++i) {
        const double lam = lambda_d[i];
        if (!(lam > 0.0)) return fail(c, MD_ERR_ARG, "lambda_d must be > 0 (+inf: unscreened)");
        kappa[i] = isinf(lam) ? 0.0 : 1.0 / lam;
    }
    c->h_c6.assign(c6, c6 + T * T);
    c->h_c12.assign(c12, c12 + T * T);
    constexpr int TT = MD_MAX_TYPES * MD_MAX_TYPES;     // room for the padded layout
    HIP_TRY(c, dalloc(&c->d_c6, TT));
    HIP_TRY(c, dalloc(&c->d_c12, TT));
    HIP_TRY(c, dalloc(&c->d_lj32, 2 * TT));
    HIP_TRY(c, dalloc(&c->d_qmax, E));
    HIP_TRY(c, dalloc(&c->d_kappa, B * S1));
    HIP_TRY(c, dalloc(&c->d_base, (int64_t)E * Q));
    HIP_TRY(c, dalloc(&c->d_g, B * S1));
    HIP_TRY(c, dalloc(&c->d_seeds, B));
    {
        const md_status ls = upload_lj(c, T);
        if (ls != MD_OK) return ls;
    }
    HIP_TRY(c, hipMemcpy(c->d_qmax, qmax, E, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_kappa, kappa.data(), sizeof(double) * B * S1, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_base, base, sizeof(double) * E * Q, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_g, g, sizeof(double) * B * S1, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_seeds, seeds, sizeof(uint64_t) * B, hipMemcpyHostToDevice));
    HIP_TRY(c, hipDeviceSynchronize());
    c->tables_bound = true;
    c->built = false;
    return MD_OK;
}

md_status md_set_step(md_ctx* ctx, int64_t step, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    launch_set_step(c, step, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_get_step(md_ctx* ctx, int64_t* step, md_stream stream)
{
    if (!ctx || !step) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    HIP_TRY(c, hipStreamSynchronize(S(stream)));
    HIP_TRY(c, hipMemcpy(step, &c->dsc->step, sizeof(int64_t), hipMemcpyDeviceToHost));
    return MD_OK;
}

md_status md_build_cells(md_ctx* ctx, const double* x, const double* y, const double* z,
                         const uint8_t* type, int32_t mode, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (null_any({x, y, z, type}) && c->N > 0) return fail(c, MD_ERR_ARG, "NULL array");
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    if (mode != MD_BUILD_AUTO && mode != MD_BUILD_FORCE && mode != MD_BUILD_CHECK)
        return fail(c, MD_ERR_ARG, "unknown build mode %d", mode);
    if (mode == MD_BUILD_CHECK && c->built) {
        launch_skin_check(c, S(stream));
    } else if (mode == MD_BUILD_FORCE || !c->built) {
        launch_build(c, x, y, z, type, true, S(stream));
        c->built = true;
    } else {
        // device-gated: the build kernels run only when the rebuild request is set
        launch_build(c, x, y, z, type, false, S(stream));
    }
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_ionize_step(md_ctx* ctx, const uint8_t* elem, const uint32_t* atom_id, int8_t* q,
                         md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (null_any({elem, atom_id, q}) && c->N > 0) return fail(c, MD_ERR_ARG, "NULL array");
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    launch_ionize(c, elem, atom_id, q, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_screened_forces(md_ctx* ctx, md_precision prec, const double* x, const double* y,
                             const double* z, const int8_t* q, const uint8_t* type, double* fx,
                             double* fy, double* fz, double* epot, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (null_any({x, y, z, q, type, fx, fy, fz}) && c->N > 0)
        return fail(c, MD_ERR_ARG, "NULL array");
    if (prec != MD_FP64 && prec != MD_FP32_KAHAN) return fail(c, MD_ERR_ARG, "unknown precision");
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    if (!c->built) return fail(c, MD_ERR_STATE, "md_build_cells has not run");
    hipEvent_t e0, e1;
    next_timer_events(c, S(stream), &e0, &e1);
    launch_repack(c, x, y, z, q, S(stream));
    HIP_TRY(c, launch_forces(c, prec, x, y, z, q, fx, fy, fz, epot, nullptr, 0, S(stream), e0,
                             e1));
    return MD_OK;
}

md_status md_force_timer_start(md_ctx* ctx, int32_t capacity)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (capacity < 0) return fail(c, MD_ERR_ARG, "capacity must be >= 0");
    (void)hipDeviceSynchronize();      // no recorded event may still be pending
    free_timer(c);
    if (capacity == 0) return MD_OK;
    c->t_ev.assign(2 * (size_t)capacity, nullptr);
    for (auto& e : c->t_ev) {
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) {
            free_timer(c);
            return fail(c, MD_ERR_HIP, "event creation failed: %s", hipGetErrorString(err));
        }
    }
    c->t_cap = capacity;
    return MD_OK;
}

md_status md_force_timer_read(md_ctx* ctx, float* ms, int32_t max, int32_t* n)
{
    if (!ctx || !n || (max > 0 && !ms) || max < 0) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    *n = c->t_n;
    for (int i = 0; i < c->t_n && i < max; ++i) {
        hipError_t err = hipEventSynchronize(c->t_ev[2 * i + 1]);
        float v = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&v, c->t_ev[2 * i], c->t_ev[2 * i + 1]);
        if (err != hipSuccess) return fail(c, MD_ERR_HIP, "timer read: %s", hipGetErrorString(err));
        ms[i] = v;
    }
    return MD_OK;
}

md_status md_integrate_vv(md_ctx* ctx, int32_t phase, double dt, const double* inv_mass,
                          const double* fx, const double* fy, const double* fz, double* x,
                          double* y, double* z, double* vx, double* vy, double* vz,
                          double* ekin, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (phase != 0 && phase != 1) return fail(c, MD_ERR_ARG, "phase must be 0 or 1");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, MD_ERR_ARG, "dt must be finite and > 0");
    if (null_any({inv_mass, fx, fy, fz, x, y, z, vx, vy, vz}) && c->N > 0)
        return fail(c, MD_ERR_ARG, "NULL array");
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    launch_vv(c, phase, dt, inv_mass, fx, fy, fz, x, y, z, vx, vy, vz, ekin, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_bind_langevin(md_ctx* ctx, const double* gamma, const double* kt, double dt)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    if (!gamma) {
        c->langevin = false;
        return MD_OK;
    }
    if (!kt) return fail(c, MD_ERR_ARG, "kt is NULL");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, MD_ERR_ARG, "dt must be finite and > 0");
    const int64_t BE = (int64_t)c->B * c->E, BS = (int64_t)c->B * (c->n_steps + 1);
    std::vector<double> c1((size_t)std::max<int64_t>(BE, 1));
    for (int64_t i = 0; i < BE; ++i) {
        if (!(gamma[i] >= 0.0) || !isfinite(gamma[i]))
            return fail(c, MD_ERR_ARG, "gamma[%lld] must be finite and >= 0", (long long)i);
        c1[i] = exp(-gamma[i] * dt);
    }
    for (int64_t i = 0; i < BS; ++i)
        if (!(kt[i] >= 0.0) || !isfinite(kt[i]))
            return fail(c, MD_ERR_ARG, "kt[%lld] must be finite and >= 0", (long long)i);
    if (!c->d_lg_c1) {
        HIP_TRY(c, dalloc(&c->d_lg_c1, BE));
        HIP_TRY(c, dalloc(&c->d_lg_kt, BS));
    }
    HIP_TRY(c, hipDeviceSynchronize());      // no step may still read the old tables
    HIP_TRY(c, hipMemcpy(c->d_lg_c1, c1.data(), sizeof(double) * c1.size(), hipMemcpyHostToDevice));
    if (BS > 0)
        HIP_TRY(c, hipMemcpy(c->d_lg_kt, kt, sizeof(double) * BS, hipMemcpyHostToDevice));
    c->lg_dt = dt;
    c->langevin = true;
    return MD_OK;
}

// Device LJ tables with row stride `stride` (T, or T + 1 with the all-zero
// pseudo-type T that marks LJ-excluded pairs in the neighbour lists).
static md_status upload_lj(Ctx* c, int stride)
{
    const int T = c->T;
    std::vector<double> a6((size_t)stride * stride, 0.0), a12((size_t)stride * stride, 0.0);
    std::vector<float> lj32(2 * (size_t)stride * stride, 0.0f);
    for (int i = 0; i < T; ++i)
        for (int j = 0; j < T; ++j) {
            const size_t d = (size_t)i * stride + j;
            a6[d] = c->h_c6[(size_t)i * T + j];
            a12[d] = c->h_c12[(size_t)i * T + j];
            lj32[2 * d] = (float)a6[d];
            lj32[2 * d + 1] = (float)a12[d];
        }
    HIP_TRY(c, hipMemcpy(c->d_c6, a6.data(), sizeof(double) * a6.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_c12, a12.data(), sizeof(double) * a12.size(),
                         hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_lj32, lj32.data(), sizeof(float) * lj32.size(),
                         hipMemcpyHostToDevice));
    c->T_lj = stride;
    return MD_OK;
}

md_status md_bind_forcefield(md_ctx* ctx, const int8_t* z_type, const double* sigma_type,
                             const int32_t* excl, int64_t n_excl, const int32_t* bonds,
                             const double* bond_par,
                             int64_t n_bonds, const int32_t* angles, const double* angle_par,
                             int64_t n_angles)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    if (n_excl < 0 || n_bonds < 0 || n_angles < 0) return fail(c, MD_ERR_ARG, "negative count");
    if ((n_excl && !excl) || (n_bonds && (!bonds || !bond_par)) ||
        (n_angles && (!angles || !angle_par)))
        return fail(c, MD_ERR_ARG, "NULL array");
    const int64_t N = c->N;
    const int T = c->T;
    if (n_excl > 0 && T >= MD_MAX_TYPES)
        return fail(c, MD_ERR_ARG, "LJ exclusions need n_types <= %d", MD_MAX_TYPES - 1);
    std::vector<int32_t> soa(N);
    for (int b = 0; b < c->B; ++b)
        for (int64_t a = c->sys_off[b]; a < c->sys_off[b + 1]; ++a) soa[a] = b;
    auto check_term = [&](const int32_t* at, int n, const char* what, int64_t t) -> md_status {
        for (int k = 0; k < n; ++k) {
            if (at[k] < 0 || at[k] >= N)
                return fail(c, MD_ERR_ARG, "%s %lld: atom %d out of range", what, (long long)t,
                            at[k]);
            if (soa[at[k]] != soa[at[0]])
                return fail(c, MD_ERR_ARG, "%s %lld spans two systems", what, (long long)t);
            for (int l = 0; l < k; ++l)
                if (at[l] == at[k])
                    return fail(c, MD_ERR_ARG, "%s %lld repeats atom %d", what, (long long)t,
                                at[k]);
        }
        return MD_OK;
    };
    for (int64_t t = 0; t < n_excl; ++t) {
        const md_status s = check_term(excl + 2 * t, 2, "exclusion", t);
        if (s != MD_OK) return s;
    }
    for (int64_t t = 0; t < n_bonds; ++t) {
        const md_status s = check_term(bonds + 2 * t, 2, "bond", t);
        if (s != MD_OK) return s;
        for (int k = 0; k < 3; ++k)
            if (!isfinite(bond_par[3 * t + k]))
                return fail(c, MD_ERR_ARG, "bond %lld: parameter not finite", (long long)t);
    }
    for (int64_t t = 0; t < n_angles; ++t) {
        const md_status s = check_term(angles + 3 * t, 3, "angle", t);
        if (s != MD_OK) return s;
        for (int k = 0; k < 2; ++k)
            if (!isfinite(angle_par[2 * t + k]))
                return fail(c, MD_ERR_ARG, "angle %lld: parameter not finite", (long long)t);
    }
    if ((z_type == nullptr) != (sigma_type == nullptr))
        return fail(c, MD_ERR_ARG, "z_type and sigma_type go together");
    if (z_type)
        for (int t = 0; t < T; ++t) {
            if (z_type[t] < 1) return fail(c, MD_ERR_ARG, "Z of type %d must be >= 1", t);
            if (!(sigma_type[t] >= 0.0) || !isfinite(sigma_type[t]))
                return fail(c, MD_ERR_ARG, "sigma of type %d must be finite and >= 0", t);
        }
    HIP_TRY(c, hipDeviceSynchronize());          // no launch may still read the old data
    auto csr = [&](std::vector<std::pair<int32_t, int32_t>>& e, int32_t** off, int32_t** lst)
        -> md_status {
        std::sort(e.begin(), e.end());
        e.erase(std::unique(e.begin(), e.end()), e.end());
        std::vector<int32_t> o(N + 1, 0), l(std::max<size_t>(e.size(), 1));
        for (auto& p : e) ++o[p.first + 1];
        for (int64_t a = 0; a < N; ++a) o[a + 1] += o[a];
        for (size_t k = 0; k < e.size(); ++k) l[k] = e[k].second;
        if (*off) { (void)hipFree(*off); *off = nullptr; }
        if (*lst) { (void)hipFree(*lst); *lst = nullptr; }
        HIP_TRY(c, dalloc(off, N + 1));
        HIP_TRY(c, dalloc(lst, (int64_t)l.size()));
        HIP_TRY(c, hipMemcpy(*off, o.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(*lst, l.data(), sizeof(int32_t) * l.size(), hipMemcpyHostToDevice));
        return MD_OK;
    };
    // LJ exclusions: both directions, sorted, in the list build's pseudo-type
    const bool had_excl = c->ff_excl;
    c->ff_excl = n_excl > 0;
    if (c->ff_excl) {
        std::vector<std::pair<int32_t, int32_t>> e;
        e.reserve(2 * n_excl);
        for (int64_t t = 0; t < n_excl; ++t) {
            e.emplace_back(excl[2 * t], excl[2 * t + 1]);
            e.emplace_back(excl[2 * t + 1], excl[2 * t]);
        }
        const md_status s = csr(e, &c->d_excl_off, &c->d_excl);
        if (s != MD_OK) return s;
    }
    {
        const md_status s = upload_lj(c, c->ff_excl ? T + 1 : T);
        if (s != MD_OK) return s;
    }
    if (had_excl || c->ff_excl) {
        // the neighbour lists carry the exclusions: rebuild them at the next build
        const int32_t one = 1;
        HIP_TRY(c, hipMemcpy(&c->dsc->need_rebuild, &one, sizeof one, hipMemcpyHostToDevice));
    }
    // charge scaling of the LJ radii (Eq. 11)
    c->ff_qlj = z_type != nullptr;
    if (c->ff_qlj) {
        double tab[kQljLen] = {};
        for (int t = 0; t < T; ++t) {
            tab[kQljInvZ + t] = 1.0 / (double)z_type[t];
            tab[kQljSig + t] = sigma_type[t];
            tab[kQljSigZ + t] = sigma_type[t] / (double)z_type[t];
        }
        for (int a = 0; a < T; ++a)
            for (int b = 0; b < T; ++b) {
                const double sum = sigma_type[a] + sigma_type[b];
                tab[kQljRs + a * MD_MAX_TYPES + b] = sum > 0.0 ? 1.0 / sum : 0.0;
            }
        if (!c->d_qlj) HIP_TRY(c, dalloc(&c->d_qlj, kQljLen));
        HIP_TRY(c, hipMemcpy(c->d_qlj, tab, sizeof tab, hipMemcpyHostToDevice));
    }
    // bonded terms and, per atom, the terms it takes part in
    for (void* p : {(void*)c->d_bonds, (void*)c->d_bond_par, (void*)c->d_angles,
                    (void*)c->d_angle_par})
        if (p) (void)hipFree(p);
    c->d_bonds = nullptr; c->d_bond_par = nullptr; c->d_angles = nullptr; c->d_angle_par = nullptr;
    c->n_bonds = n_bonds;
    c->n_angles = n_angles;
    if (n_bonds + n_angles > 0) {
        HIP_TRY(c, dalloc(&c->d_bonds, 2 * n_bonds));
        HIP_TRY(c, dalloc(&c->d_bond_par, 3 * n_bonds));
        HIP_TRY(c, dalloc(&c->d_angles, 3 * n_angles));
        HIP_TRY(c, dalloc(&c->d_angle_par, 2 * n_angles));
        if (n_bonds) {
            HIP_TRY(c, hipMemcpy(c->d_bonds, bonds, sizeof(int32_t) * 2 * n_bonds,
                                 hipMemcpyHostToDevice));
            HIP_TRY(c, hipMemcpy(c->d_bond_par, bond_par, sizeof(double) * 3 * n_bonds,
                                 hipMemcpyHostToDevice));
        }
        if (n_angles) {
            HIP_TRY(c, hipMemcpy(c->d_angles, angles, sizeof(int32_t) * 3 * n_angles,
                                 hipMemcpyHostToDevice));
            HIP_TRY(c, hipMemcpy(c->d_angle_par, angle_par, sizeof(double) * 2 * n_angles,
                                 hipMemcpyHostToDevice));
        }
        std::vector<std::pair<int32_t, int32_t>> inc;
        inc.reserve(2 * n_bonds + 3 * n_angles);
        for (int64_t t = 0; t < n_bonds; ++t)
            for (int k = 0; k < 2; ++k) inc.emplace_back(bonds[2 * t + k], (int32_t)(t * 2));
        for (int64_t t = 0; t < n_angles; ++t)
            for (int k = 0; k < 3; ++k) inc.emplace_back(angles[3 * t + k], (int32_t)(t * 2 + 1));
        const md_status s = csr(inc, &c->d_bt_off, &c->d_bt);
        if (s != MD_OK) return s;
        if (!c->d_bond_e) {
            HIP_TRY(c, dalloc(&c->d_bond_e, N));
            HIP_TRY(c, dalloc(&c->d_bond_blk, div_up(N, kBondedBlock)));
        }
    }
    return MD_OK;
}

// Coefficients {r', c1, c2, c3} of the hybrid potential of a charge-Q ion (Q >= 1):
// R from Eq. 4, r' from Eq. 7; eliminating c2 between the slope and curvature
// conditions at r' gives c3 = 3Q / (r'^3 u0 (t^2 + t/r' + 1/r'^2)) with
// u0 = exp(-r'/lambda)/r' and t = 1/lambda + 1/r'; the slope condition gives c2 and
// the value condition c1.  An infinite Debye length leaves the bare charge.
static void hybrid_coeffs(double Q, double lambda, double ne, double h[4])
{
    if (isinf(lambda)) {
        h[0] = 0.0; h[1] = 0.0; h[2] = 0.0; h[3] = Q;
        return;
    }
    const double R = cbrt(3.0 * Q / (4.0 * M_PI * ne));
    const double a = R / lambda;
    const double rp = lambda * (cbrt(a * a * a + 1.0) - 1.0);
    const double u0 = exp(-rp / lambda) / rp;
    const double t = 1.0 / lambda + 1.0 / rp;
    const double c3 = 3.0 * Q / (rp * rp * rp * u0 * (t * t + t / rp + 1.0 / (rp * rp)));
    const double c2 = (c3 * u0 * t - Q / (rp * rp)) / (2.0 * rp);
    const double c1 = c3 * u0 - Q / rp + c2 * rp * rp;
    h[0] = rp; h[1] = c1; h[2] = c2; h[3] = c3;
}

md_status md_bind_hybrid(md_ctx* ctx, const double* ne)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    if (!ne) {
        c->hybrid = false;
        return MD_OK;
    }
    const int64_t S1 = c->n_steps + 1, BS = (int64_t)c->B * S1;
    const int nq = std::max(c->Q, 1);
    std::vector<double> h64((size_t)std::max<int64_t>(BS * nq * 4, 4), 0.0);
    std::vector<float4> h32((size_t)std::max<int64_t>(BS * nq, 1));
    for (int64_t i = 0; i < BS; ++i) {
        if (!(ne[i] > 0.0) || !isfinite(ne[i]))
            return fail(c, MD_ERR_ARG, "ne[%lld] must be finite and > 0", (long long)i);
        for (int q = 1; q < nq; ++q) {
            double* h = &h64[(size_t)(i * nq + q) * 4];
            hybrid_coeffs((double)q, c->lambda_d[i], ne[i], h);
            for (int k = 0; k < 4; ++k)
                if (!isfinite(h[k]))
                    return fail(c, MD_ERR_ARG,
                                "hybrid coefficients not finite at entry %lld, charge %d "
                                "(lambda_d %.6g nm, ne %.6g nm^-3)",
                                (long long)i, q, c->lambda_d[i], ne[i]);
        }
    }
    for (size_t k = 0; k < h32.size(); ++k)
        h32[k] = make_float4((float)h64[4 * k], (float)h64[4 * k + 1], (float)h64[4 * k + 2],
                             (float)h64[4 * k + 3]);
    if (!c->d_hyb64) {
        HIP_TRY(c, dalloc(&c->d_hyb64, (int64_t)h64.size()));
        HIP_TRY(c, dalloc(&c->d_hyb32, (int64_t)h32.size()));
    }
    HIP_TRY(c, hipDeviceSynchronize());      // no step may still read the old tables
    HIP_TRY(c, hipMemcpy(c->d_hyb64, h64.data(), sizeof(double) * h64.size(),
                         hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_hyb32, h32.data(), sizeof(float4) * h32.size(),
                         hipMemcpyHostToDevice));
    c->hyb_q = nq;
    c->hybrid = true;
    return MD_OK;
}

md_status md_rdf_histogram(md_ctx* ctx, const double* x, const double* y, const double* z,
                           const uint8_t* elem, double r_max, int32_t n_bins, uint64_t* hist,
                           md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound || !c->built)
        return fail(c, MD_ERR_STATE, "build cells before the histogram");
    if (!(r_max > 0.0) || !(r_max <= c->cfg.rc))
        return fail(c, MD_ERR_ARG, "r_max must be in (0, rc]");
    if (n_bins < 1 || n_bins > kRdfMaxBins)
        return fail(c, MD_ERR_ARG, "n_bins must be in [1, %d]", kRdfMaxBins);
    if (null_any({x, y, z, elem, hist}) && c->N > 0) return fail(c, MD_ERR_ARG, "NULL array");
    if (!c->d_rdf_moved) {
        HIP_TRY(c, dalloc(&c->d_rdf_moved, c->N));
        HIP_TRY(c, dalloc(&c->d_rdf_xr, 3 * c->cap_slots));
        HIP_TRY(c, dalloc(&c->d_rdf_er, c->cap_slots));
    }
    launch_rdf(c, x, y, z, elem, r_max, n_bins, reinterpret_cast<unsigned long long*>(hist),
               c->d_rdf_moved, c->d_rdf_xr, c->d_rdf_er, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_rdf_histogram_noalloc(md_ctx* ctx, const double* x, const double* y,
                                   const double* z, const uint8_t* elem, double r_max,
                                   int32_t n_bins, uint64_t* hist, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound || !c->built)
        return fail(c, MD_ERR_STATE, "build cells before the histogram");
    if (!(r_max > 0.0) || !(r_max <= c->cfg.rc))
        return fail(c, MD_ERR_ARG, "r_max must be in (0, rc]");
    if (n_bins < 1 || n_bins > kRdfMaxBins)
        return fail(c, MD_ERR_ARG, "n_bins must be in [1, %d]", kRdfMaxBins);
    if (null_any({x, y, z, elem, hist}) && c->N > 0) return fail(c, MD_ERR_ARG, "NULL array");
    const size_t need = rdf_scratch_bytes(c->N, c->cap_slots);
    if (need > kRdfScratchBytes)
        return fail(c, MD_ERR_CAPACITY,
                    "the no-allocation histogram needs %zu bytes of workspace (%lld atoms, "
                    "%lld slots); its fixed device array holds %zu",
                    need, (long long)c->N, (long long)c->cap_slots, kRdfScratchBytes);
    unsigned char* p = static_cast<unsigned char*>(rdf_scratch(c->device));
    if (!p) return fail(c, MD_ERR_HIP, "device address of the histogram workspace unavailable");
    double* xr = reinterpret_cast<double*>(p);
    uint8_t* er = p + (((size_t)c->cap_slots * 3 * sizeof(double) + 255) & ~(size_t)255);
    uint8_t* moved = er + (((size_t)c->cap_slots + 255) & ~(size_t)255);
    launch_rdf(c, x, y, z, elem, r_max, n_bins, reinterpret_cast<unsigned long long*>(hist),
               moved, xr, er, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_rdf_normalize(int32_t n_bins, double r_max, const uint64_t* counts, int64_t n_a,
                           int64_t n_b, int32_t same, double volume, double* g)
{
    if (n_bins < 1 || !(r_max > 0.0) || !counts || !g || !(volume > 0.0) || n_a < 0 || n_b < 0)
        return MD_ERR_ARG;
    const double pairs = same ? 0.5 * (double)n_a * (double)(n_a - 1) : (double)n_a * (double)n_b;
    const double dr = r_max / (double)n_bins;
    for (int k = 0; k < n_bins; ++k) {
        const double r0 = (double)k * dr, r1 = (double)(k + 1) * dr;
        const double shell = 4.0 / 3.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
        const double ideal = pairs / volume * shell;
        g[k] = ideal > 0.0 ? (double)counts[k] / ideal : 0.0;
    }
    return MD_OK;
}

md_status md_structure_factor(int32_t n_bins, double r_max, const double* g, double rho0,
                              int32_t n_q, const double* q, double* S)
{
    if (n_bins < 1 || !(r_max > 0.0) || !g || n_q < 0 || (n_q > 0 && (!q || !S)))
        return MD_ERR_ARG;
    const double dr = r_max / (double)n_bins;
    for (int m = 0; m < n_q; ++m) {
        if (!(q[m] > 0.0)) return MD_ERR_ARG;
        double acc = 0.0;
        for (int k = 0; k < n_bins; ++k) {
            const double r = ((double)k + 0.5) * dr;
            acc += r * (g[k] - 1.0) * sin(q[m] * r);
        }
        S[m] = 1.0 + 4.0 * M_PI * rho0 / q[m] * acc * dr;
    }
    return MD_OK;
}

md_status md_integrate_langevin(md_ctx* ctx, double dt, const double* inv_mass,
                                const uint8_t* elem, const uint32_t* atom_id, const double* fx,
                                const double* fy, const double* fz, double* x, double* y,
                                double* z, double* vx, double* vy, double* vz, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return fail(c, MD_ERR_STATE, "tables not bound");
    if (!c->langevin) return fail(c, MD_ERR_STATE, "Langevin coupling not bound");
    if (dt != c->lg_dt) return fail(c, MD_ERR_ARG, "dt differs from the bound one");
    if (null_any({inv_mass, elem, atom_id, fx, fy, fz, x, y, z, vx, vy, vz}) && c->N > 0)
        return fail(c, MD_ERR_ARG, "NULL array");
    launch_vv0_langevin(c, dt, inv_mass, elem, atom_id, fx, fy, fz, x, y, z, vx, vy, vz, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_sync_check(md_ctx* ctx, md_stream stream, uint32_t* flags)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) {
        if (flags) *flags = 0;
        return MD_OK;
    }
    HIP_TRY(c, hipStreamSynchronize(S(stream)));
    uint32_t f = 0;
    HIP_TRY(c, hipMemcpy(&f, &c->dsc->flags, sizeof f, hipMemcpyDeviceToHost));
    if (flags) *flags = f;
    if (f) return fail(c, MD_ERR_DEVICE, "device error word 0x%x", f);
    return MD_OK;
}

md_status md_clear_flags(md_ctx* ctx, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (!c->tables_bound) return MD_OK;
    launch_clear_flags(c, S(stream));
    HIP_TRY(c, hipGetLastError());
    return MD_OK;
}

md_status md_debug_pairs(md_ctx* ctx, md_precision prec, const double* x, const double* y,
                         const double* z, const int8_t* q, int64_t* n_pairs, int32_t* ij,
                         int64_t max, double* e_atom, md_stream stream)
{
    if (!ctx) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    if (null_any({x, y, z, q, n_pairs}) || (max > 0 && !ij))
        return fail(c, MD_ERR_ARG, "NULL argument");
    if (max < 0) return fail(c, MD_ERR_ARG, "max must be >= 0");
    if (!c->tables_bound || !c->built) return fail(c, MD_ERR_STATE, "no build");
    hipStream_t st = S(stream);
    if (e_atom) {
        // per-atom energies come from the list kernels alone: no atom may be fast
        HIP_TRY(c, hipStreamSynchronize(st));
        int32_t nf = 0, pend = 0;
        HIP_TRY(c, hipMemcpy(&nf, &c->dsc->n_fast_raw, sizeof nf, hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(&pend, &c->dsc->need_rebuild, sizeof pend, hipMemcpyDeviceToHost));
        if (nf != 0 || pend != 0)
            return fail(c, MD_ERR_STATE, "per-atom energies need a build at the current "
                                         "positions (%d atoms beyond skin/2)", nf);
    }
    int2* buf = nullptr;
    double* f = nullptr;
    HIP_TRY(c, dalloc(&buf, std::max<int64_t>(max, 1)));
    // forces (3N), per-atom energies (N) and per-system energies (B)
    hipError_t e = dalloc(&f, 4 * std::max<int64_t>(c->N, 1) + c->B);
    if (e != hipSuccess) { (void)hipFree(buf); return fail(c, MD_ERR_HIP, "allocation failed"); }
    e = hipMemsetAsync(&c->dsc->pair_count, 0, sizeof(unsigned long long), st);
    if (e == hipSuccess && e_atom)
        e = hipMemsetAsync(f + 3 * c->N, 0, sizeof(double) * c->N, st);
    if (e == hipSuccess) {
        c->dbg_e_atom = e_atom ? f + 3 * c->N : nullptr;
        launch_repack(c, x, y, z, q, st);
        e = launch_forces(c, prec, x, y, z, q, f, f + c->N, f + 2 * c->N,
                          e_atom ? f + 4 * c->N : nullptr, buf, max, st);
        c->dbg_e_atom = nullptr;
    }
    unsigned long long cnt = 0;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = hipMemcpy(&cnt, &c->dsc->pair_count, sizeof cnt, hipMemcpyDeviceToHost);
    if (e == hipSuccess && max > 0)
        e = hipMemcpy(ij, buf, sizeof(int2) * std::min<int64_t>((int64_t)cnt, max),
                      hipMemcpyDeviceToHost);
    if (e == hipSuccess && e_atom)
        e = hipMemcpy(e_atom, f + 3 * c->N, sizeof(double) * c->N, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    (void)hipFree(f);
    if (e != hipSuccess) return fail(c, MD_ERR_HIP, "debug pair export: %s", hipGetErrorString(e));
    *n_pairs = (int64_t)cnt;
    return MD_OK;
}

md_status md_get_stats(md_ctx* ctx, md_stats* out, md_stream stream)
{
    if (!ctx || !out) return MD_ERR_ARG;
    Ctx* c = &ctx->c;
    memset(out, 0, sizeof *out);
    out->n_atoms = c->N;
    out->cluster_group = c->G;
    out->list_capacity = c->nb_cap_h;
    out->group_entry_capacity = c->E_cap;
    if (!c->tables_bound) return MD_OK;
    HIP_TRY(c, hipStreamSynchronize(S(stream)));
    DevScalars h;
    HIP_TRY(c, hipMemcpy(&h, c->dsc, sizeof h, hipMemcpyDeviceToHost));
    out->n_clusters = h.n_clusters;
    out->n_groups = h.n_groups;
    out->n_builds = h.n_builds;
    out->n_fast = h.n_fast;
    out->n_fast_raw = h.n_fast_raw;
    out->flags = h.flags;
    int64_t ne = 0, max_e = 0, codes = 0, max_l = 0;
    if (h.n_groups > 0) {
        std::vector<Group> gr(h.n_groups);
        HIP_TRY(c, hipMemcpy(gr.data(), c->d_groups, sizeof(Group) * h.n_groups,
                             hipMemcpyDeviceToHost));
        for (const Group& x : gr) {
            ne += x.nent;
            max_e = std::max<int64_t>(max_e, x.nent_raw);
        }
    }
    if (h.n_clusters > 0) {
        // list lengths: rows give the code count up to padding; the longest half-list per
        // cluster is kept exactly
        std::vector<int32_t> len(2 * (size_t)h.n_clusters), nt(2 * (size_t)h.n_clusters);
        HIP_TRY(c, hipMemcpy(len.data(), c->d_cl_len, sizeof(int32_t) * len.size(),
                             hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(nt.data(), c->d_cl_nt, sizeof(int32_t) * nt.size(),
                             hipMemcpyDeviceToHost));
        for (size_t i = 0; i < len.size(); ++i) {
            max_l = std::max<int64_t>(max_l, len[i]);
            codes += (int64_t)nt[i] * 32 * kCluster;    // padded code slots
        }
    }
    out->n_list_codes = codes;
    out->max_list_len = max_l;
    out->max_group_entries = max_e;
    out->n_entries = ne;
    return MD_OK;
}

double md_debye_length_nm(double te_ev, double ne_m3)
{
    // lambda_D = sqrt(eps0 k_B T_e / (n_e e^2)) with k_B T_e = T_e[eV] * e
    const double eps0 = 8.8541878128e-12, e = 1.602176634e-19;
    if (!(te_ev > 0.0) || !(ne_m3 > 0.0)) return NAN;
    return sqrt(eps0 * te_ev / (ne_m3 * e)) * 1e9;
}

md_status md_rates_from_fractions(int64_t S, int32_t Z, const double* P, double* p)
{
    if (!P || !p || S < 0 || Z < 0) return MD_ERR_ARG;
    const int32_t nq = Z + 1;
    for (int32_t q = 0; q < nq; ++q) p[q] = 0.0;
    for (int64_t s = 1; s <= S; ++s) {
        const double* prev = P + (s - 1) * nq;
        const double* cur = P + s * nq;
        // flux out of charge q = growth of every higher charge state
        double above = 0.0;
        for (int32_t q = Z; q >= 0; --q) {
            double v = 0.0;
            if (q < Z && prev[q] > 0.0) v = above / prev[q];
            p[s * nq + q] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            above += cur[q] - prev[q];
        }
    }
    return MD_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ full step and graphs

struct md_graph {
    md_ctx* ctx;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

static md_status step_impl(md_ctx* ctx, const md_step_args* a, int32_t build_mode, md_stream st)
{
    Ctx* c = &ctx->c;
    const bool fused = (build_mode == MD_BUILD_AUTO || build_mode == MD_BUILD_FORCE) &&
                       c->bs_blocks > 0 && c->tables_bound && c->built && c->N > 0;
    if (fused) {
        // the same sequence in four launches: phase 0 + ionization; fast-list join,
        // step counter, rebuild when due and slot repack; forces; phase 1
        if (!(a->dt > 0.0) || !isfinite(a->dt)) return fail(c, MD_ERR_ARG, "dt must be > 0");
        if (null_any({a->x, a->y, a->z, a->vx, a->vy, a->vz, a->fx, a->fy, a->fz, a->inv_mass,
                      a->elem, a->type, a->atom_id, a->q}))
            return fail(c, MD_ERR_ARG, "NULL array");
        if (a->prec != MD_FP64 && a->prec != MD_FP32_KAHAN)
            return fail(c, MD_ERR_ARG, "unknown precision");
        if (c->langevin && a->dt != c->lg_dt)
            return fail(c, MD_ERR_ARG, "dt differs from the one the coupling was bound with");
        hipStream_t hs = S(st);
        launch_vv0_ionize(c, a->dt, a->inv_mass, a->fx, a->fy, a->fz, a->x, a->y, a->z, a->vx,
                          a->vy, a->vz, a->elem, a->atom_id, a->q, hs);
        launch_build_step(c, a->x, a->y, a->z, a->type, a->q, build_mode == MD_BUILD_FORCE, hs);
        hipEvent_t e0, e1;
        next_timer_events(c, hs, &e0, &e1);
        HIP_TRY(c, launch_forces(c, a->prec, a->x, a->y, a->z, a->q, a->fx, a->fy, a->fz,
                                 a->epot, nullptr, 0, hs, e0, e1, false));
        launch_vv1_finalize(c, a->dt, a->inv_mass, a->fx, a->fy, a->fz, a->vx, a->vy, a->vz,
                            a->ekin, a->epot, hs);
        HIP_TRY(c, hipGetLastError());
        return MD_OK;
    }
    md_status s = c->langevin
                      ? md_integrate_langevin(ctx, a->dt, a->inv_mass, a->elem, a->atom_id, a->fx,
                                              a->fy, a->fz, a->x, a->y, a->z, a->vx, a->vy, a->vz,
                                              st)
                      : md_integrate_vv(ctx, 0, a->dt, a->inv_mass, a->fx, a->fy, a->fz, a->x,
                                        a->y, a->z, a->vx, a->vy, a->vz, nullptr, st);
    if (s == MD_OK) s = md_ionize_step(ctx, a->elem, a->atom_id, a->q, st);
    if (s == MD_OK) s = md_build_cells(ctx, a->x, a->y, a->z, a->type, build_mode, st);
    if (s == MD_OK)
        s = md_screened_forces(ctx, a->prec, a->x, a->y, a->z, a->q, a->type, a->fx, a->fy, a->fz,
                               a->epot, st);
    if (s == MD_OK)
        s = md_integrate_vv(ctx, 1, a->dt, a->inv_mass, a->fx, a->fy, a->fz, a->x, a->y, a->z,
                            a->vx, a->vy, a->vz, a->ekin, st);
    return s;
}

md_status md_step(md_ctx* ctx, const md_step_args* args, int32_t build_mode, md_stream stream)
{
    if (!ctx || !args) return MD_ERR_ARG;
    return step_impl(ctx, args, build_mode, stream);
}

md_status md_graph_create(md_ctx* ctx, const md_step_args* args, int32_t build_mode,
                          md_stream stream, md_graph** out)
{
    if (!ctx || !args || !out) return MD_ERR_ARG;
    *out = nullptr;
    Ctx* c = &ctx->c;
    if (!stream) return fail(c, MD_ERR_ARG, "graph capture needs a non-null stream");
    if (!c->built) return fail(c, MD_ERR_STATE, "build cells before capturing a step");
    hipStream_t st = S(stream);
    HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const md_status s = step_impl(ctx, args, build_mode, stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != MD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(c, MD_ERR_HIP, "capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(c, MD_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e2));
    }
    md_graph* g = new (std::nothrow) md_graph{ctx, graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(c, MD_ERR_CAPACITY, "host allocation failed");
    }
    *out = g;
    return MD_OK;
}

md_status md_graph_launch(md_graph* graph, md_stream stream)
{
    if (!graph) return MD_ERR_ARG;
    const hipError_t e = hipGraphLaunch(graph->exec, S(stream));
    if (e != hipSuccess)
        return fail(&graph->ctx->c, MD_ERR_HIP, "graph launch failed: %s", hipGetErrorString(e));
    return MD_OK;
}

md_status md_graph_destroy(md_graph* graph)
{
    if (!graph) return MD_OK;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
    return MD_OK;
}

}  // extern "C"
