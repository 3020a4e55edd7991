/*
 * md.h -- C ABI of the MI355X screened-force + ionization step library (libmd_hip.so).
 *
 * The library advances atoms that interact through spherically symmetric two-body
 * potentials: a Debye-screened Coulomb term between integer-charged ions and a
 * Lennard-Jones term modulated by the same screening factor, both truncated at a
 * cutoff (arXiv 2401.03180, section II.A Eq. 2 and Eq. 8; section II.B on the
 * screening-reduced cutoff).  Every step the integer charges change stochastically
 * (section II.A: charges are assigned stochastically so that ensemble averages
 * follow the collisional-radiative charge-state fractions; section II.B: no partial
 * charges), and Newton's equation is integrated (section II.B, Eq. 12).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Units: nm, ps, amu, kJ/mol, elementary charge.  Forces in kJ mol^-1 nm^-1.
 *  Atoms of B independent systems are concatenated; system b owns atoms
 *  [sys_offsets[b], sys_offsets[b+1]).  Per-atom arrays are structure-of-arrays
 *  in the caller's atom order, contiguous, in device memory (hipMalloc'd or torch
 *  CUDA tensors) unless a parameter says "host".  The caller owns every per-atom
 *  array; the library owns only its context workspace, allocated by
 *  md_bind_tables (no device allocation happens in the per-step calls; only
 *  md_debug_pairs allocates), so the asynchronous calls can be captured in a HIP
 *  graph.
 *  `stream` is a hipStream_t (0 = the null stream).  Asynchronous calls enqueue
 *  work on `stream` and return after argument validation; errors found on the
 *  device are latched in a device error word (MD_FLAG_*) and reported by
 *  md_sync_check.  No call aborts or throws; every failure is a status code with a
 *  message available from md_last_error.  One context serves one stream at a time
 *  and is not thread-safe.
 *
 *  Step counter: the context keeps a device step counter k = index of the latest
 *  force evaluation.  k = 0 selects kappa[.][0] for the initial forces; phase 0 of
 *  md_integrate_vv advances it to s = k + 1; md_ionize_step and the following
 *  md_screened_forces use s; phase 1 leaves it unchanged.
 */
#ifndef MD_H
#define MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx md_ctx;           /* opaque, library-owned */
typedef void* md_stream;                /* a hipStream_t */

typedef enum md_status {
    MD_OK = 0,
    MD_ERR_ARG = -1,        /* null pointer, size or enum out of range */
    MD_ERR_HIP = -2,        /* a HIP runtime call failed */
    MD_ERR_CAPACITY = -3,   /* more atoms/types/elements than the context was sized for */
    MD_ERR_GEOMETRY = -4,   /* periodic box too small for the cutoff (need L >= 2 (rc + skin)) */
    MD_ERR_DEVICE = -5,     /* the device error word is non-zero (see MD_FLAG_*) */
    MD_ERR_STATE = -6       /* call out of order (e.g. forces before tables or cells) */
} md_status;

typedef enum md_precision {
    MD_FP64 = 0,            /* plain FP64 pair arithmetic and accumulation */
    MD_FP32_KAHAN = 1       /* FP32 pair arithmetic, FP32 + compensated per-atom sums */
} md_precision;

/* Device error word bits (latched until md_clear_flags). */
#define MD_FLAG_CELL_OVERFLOW 0x1u   /* grid/cluster capacity exceeded during a build */
#define MD_FLAG_LIST_OVERFLOW 0x2u   /* neighbour-list capacity exceeded: pairs may be missing
                                        (the per-atom lists are written by the first
                                        md_screened_forces after a build, which latches it) */
#define MD_FLAG_SKIN 0x4u            /* forces were evaluated (or MD_BUILD_CHECK ran) while some
                                        atom had moved more than skin/2 since the last build */
#define MD_FLAG_NONFINITE 0x8u       /* non-finite position seen by a build, or one more than
                                        500 box lengths from a periodic box (binned at the
                                        500th image) */
#define MD_FLAG_STEP 0x10u           /* step counter outside the bound schedule tables */
#define MD_FLAG_BAD_INPUT 0x20u      /* a type, element or charge outside its table (the entry
                                        was clamped or skipped) */
#define MD_FLAG_BARRIER 0x40u        /* a grid-wide wait of the fused step kernel timed out: the
                                        step's results are invalid (md_clear_flags resets it) */

#define MD_MAX_TYPES 8
#define MD_MAX_ELEMENTS 8
#define MD_MAX_CHARGE_STATES 128

typedef struct md_config {
    int32_t n_systems;          /* B >= 1 */
    int32_t n_types;            /* Lennard-Jones types, 1..MD_MAX_TYPES */
    int32_t n_elements;         /* ionizable elements, 1..MD_MAX_ELEMENTS */
    int32_t n_charge_states;    /* Q: row length of the base[] table, 1..MD_MAX_CHARGE_STATES */
    int32_t periodic;           /* 1: rectangular periodic box per system; 0: vacuum */
    int32_t screen_lj;          /* 1: LJ multiplied by exp(-r/lambda_D) (Eq. 8); 0: plain LJ */
    double rc;                  /* cutoff, nm (pairs with r^2 < rc^2 interact) */
    double skin;                /* Verlet buffer, nm (> 0) */
    int64_t capacity_atoms;     /* >= sys_offsets[B]; every workspace is sized from it */
    int32_t cluster_group;      /* i-clusters per force work-group: 1, 2, 4 or 8 (0 = 4);
                                   halved at md_create while the group's candidate table
                                   would not fit one work-group's LDS at density_hint
                                   (md_stats.cluster_group is the size in use) */
    int32_t max_neighbors;      /* per-atom neighbour-list capacity (0 = derived) */
    double density_hint;        /* upper bound on atoms per nm^3 used for sizing the grid,
                                   the group tables and the per-atom lists (0: 1.1 x the
                                   mean density of the densest periodic box, 130 for
                                   vacuum); a region much denser than it overflows the
                                   lists (MD_FLAG_LIST_OVERFLOW) */
    int32_t fast_capacity;      /* atoms allowed beyond skin/2 of their build position before a
                                   rebuild is due; their pairs are evaluated separately, exactly
                                   (0 = min(1024, max(64, N/96)); -1 = none: rebuild as soon as
                                   one atom is that far; at most 65536) */
    int32_t reserved;           /* 0 */
} md_config;

/* Build modes of md_build_cells. */
#define MD_BUILD_AUTO 0         /* device-decided: the build kernels are enqueued but do their
                                   work only if phase 0 of md_integrate_vv found more than
                                   fast_capacity atoms that moved more than skin/2 since the
                                   last build (no host round trip, graph-capturable); the
                                   first build always runs */
#define MD_BUILD_FORCE 1        /* rebuild now */
#define MD_BUILD_CHECK 2        /* never rebuild; latch MD_FLAG_SKIN if a rebuild was due */

/* Create a context for B systems.  sys_offsets: host int64[B+1], non-decreasing,
 * sys_offsets[0] = 0, sys_offsets[B] <= capacity_atoms.  Validates the
 * configuration and binds the context to the current HIP device; the device
 * workspace is allocated by md_bind_tables.  On failure *out is NULL. */
md_status md_create(const md_config* cfg, const int64_t* sys_offsets, md_ctx** out);

/* Release the context and its device workspace (synchronizes the device). */
md_status md_destroy(md_ctx* ctx);

/* Message describing the last non-MD_OK status returned for ctx (never NULL;
 * ctx may be NULL for errors of md_create). */
const char* md_last_error(const md_ctx* ctx);

/* Copy the per-run tables (all HOST arrays, FP64 unless stated) into the context
 * and size / allocate its device workspace (a second call re-allocates):
 *   box       [B*3]  periodic box lengths per system (NULL when vacuum);
 *   c6, c12   [T*T]  Lennard-Jones coefficients, symmetric (c6 = 4 eps sigma^6,
 *                    c12 = 4 eps sigma^12);
 *   qmax      int8 [E]  highest charge reachable per element;
 *   lambda_d  [B*(S+1)] Debye length per system and force evaluation k = 0..S
 *                    (section II.A, Eq. 3); +inf means unscreened.  The library stores
 *                    kappa = 1/lambda_d;
 *   base      [E*Q]  per-(element, charge) per-step ionization probability scale;
 *   g         [B*(S+1)] per-system pulse envelope for ionization steps s = 1..S
 *                    (entry 0 unused);
 *   seeds     uint64 [B] per-system random seeds;
 *   n_steps   S >= 0.
 * Synchronous.  Resets the step counter to 0 and the error word to 0.  Fails with
 * MD_ERR_GEOMETRY when a periodic box edge is below 2 (rc + skin), and with
 * MD_ERR_CAPACITY when the workspace would exceed a kernel's limits (the candidate
 * tables and slot arrays are addressed with 32-bit byte offsets: tens of millions of
 * atoms per context). */
md_status md_bind_tables(md_ctx* ctx, const double* box, const double* c6, const double* c12,
                         const int8_t* qmax, const double* lambda_d, const double* base,
                         const double* g, const uint64_t* seeds, int64_t n_steps);

/* Set the device step counter (asynchronous, graph-capturable). */
md_status md_set_step(md_ctx* ctx, int64_t step, md_stream stream);

/* Read the device step counter (synchronizes `stream`). */
md_status md_get_step(md_ctx* ctx, int64_t* step, md_stream stream);

/* Neighbour search (section II.B: the screening-reduced cutoff bounds the pairs
 * that are evaluated).  x, y, z: device FP64 [N] current positions (never
 * wrapped by the library); type: uint8 [N] Lennard-Jones types (the same array
 * must be passed to md_screened_forces).  Builds the grid binning, the 8-atom
 * clusters, the cluster-group candidate tables and the per-atom neighbour codes
 * covering every pair within rc + skin, and records the build positions for the
 * displacement test (the largest displacement is tracked by phase 0 of
 * md_integrate_vv).  `mode` is one of MD_BUILD_*.  Asynchronous. */
md_status md_build_cells(md_ctx* ctx, const double* x, const double* y, const double* z,
                         const uint8_t* type, int32_t mode, md_stream stream);


/* Stochastic integer ionization for the current step s (>= 1, the device step
 * counter).  Section II.A assigns every atom an integer charge, drawn at random so
 * that averages over atoms and runs follow the collisional-radiative charge-state
 * populations; section II.B keeps charges integer (no partial charges).  Reading
 * (the paper gives no mechanism): a sequential +1 process, every atom a of system b
 * with element e = elem[a] and charge q[a] < qmax[e] gains +1 iff
 *   u < floor(min(1, base[e][q] * g[b][s]) * 2^32),
 * where u is word 0 of Philox4x32-10 with counter (atom_id[a], s, b, 0) and key
 * (low, high 32 bits of seeds[b]) (Salmon et al., SC'11), so the charges depend
 * only on (seeds, tables, ids), never on positions or the neighbour structure.
 * elem: uint8 [N]; atom_id: uint32 [N] (the atom's index inside its system); q:
 * int8 [N], updated in place (device, caller-owned).  Errors: MD_ERR_ARG for a NULL
 * array, MD_ERR_STATE before md_bind_tables; an element or charge outside its table
 * latches MD_FLAG_BAD_INPUT, a step outside the tables MD_FLAG_STEP.
 * Asynchronous. */
md_status md_ionize_step(md_ctx* ctx, const uint8_t* elem, const uint32_t* atom_id, int8_t* q,
                         md_stream stream);

/* Screened pair forces (section II.A Eq. 2 + Eq. 8).  For every pair (i, j) of one
 * system whose minimum-image separation d = x_i - x_j has
 * r^2 = (dx*dx + dy*dy) + dz*dz < rc*rc (FP64, exactly as written), with
 * s = exp(-kappa r), kappa = 1/lambda_d[b][k] at the current step k:
 *   phi = (k_e q_i q_j / r + c12/r^12 - c6/r^6) s,   F_i = -F_j = f d,
 *   f = ((k_e q_i q_j / r + 12 c12/r^12 - 6 c6/r^6) + (phi/s) kappa r) s / r^2.
 * x, y, z: FP64 [N]; q: int8 [N]; type: uint8 [N] (< n_types).  fx, fy, fz: FP64 [N]
 * outputs, overwritten in caller order.  epot: device FP64 [B] (sum of phi per
 * system) or NULL.  Requires a prior md_build_cells on positions within skin/2.
 * MD_FP32_KAHAN decides membership with an error-bounded FP32 test and re-decides
 * every pair inside the error band with the FP64 expression above, so the set of
 * interacting pairs is identical for both precisions. */
md_status md_screened_forces(md_ctx* ctx, md_precision prec, const double* x, const double* y,
                             const double* z, const int8_t* q, const uint8_t* type, double* fx,
                             double* fy, double* fz, double* epot, md_stream stream);

/* Velocity-Verlet half steps (section II.B, Eq. 12), FP64, element-wise with no
 * contraction, h = (0.5 dt) * inv_mass[a]:
 *   phase 0: v += h F; x += dt v; then advance the step counter; also tracks the
 *            largest displacement since the last build;
 *   phase 1: v += h F; if ekin != NULL, ekin[b] = sum 1/2 m v^2 per system.
 * inv_mass, fx, fy, fz: FP64 [N]; x..vz: FP64 [N] in/out; ekin: device FP64 [B]. */
md_status md_integrate_vv(md_ctx* ctx, int32_t phase, double dt, const double* inv_mass,
                          const double* fx, const double* fy, const double* fz, double* x,
                          double* y, double* z, double* vx, double* vy, double* vz,
                          double* ekin, md_stream stream);

/* Synchronize `stream`; return MD_ERR_DEVICE if the error word is non-zero.
 * flags (host, may be NULL) receives the word. */
md_status md_sync_check(md_ctx* ctx, md_stream stream, uint32_t* flags);

/* Clear the device error word (asynchronous). */
md_status md_clear_flags(md_ctx* ctx, md_stream stream);

/* Debug export of the interacting pair set exactly as md_screened_forces decides
 * it for `prec` at positions x, y, z with charges q (runs the same force kernel):
 * writes up to max pairs (i, j), i < j, as caller indices into ij (HOST int32
 * [2*max], unordered) and their count into *n_pairs (max = 0: count only).
 * e_atom (HOST FP64 [N], or NULL) receives the per-atom energies e_i = 1/2 sum_j
 * phi_ij (section II.A, Eq. 2 and Eq. 8) of the same evaluation; it needs lists
 * built at the current positions (no atom beyond skin/2 of the last build, e.g.
 * right after md_build_cells with MD_BUILD_FORCE), else MD_ERR_STATE.
 * Synchronous; allocates temporary device buffers. */
md_status md_debug_pairs(md_ctx* ctx, md_precision prec, const double* x, const double* y,
                         const double* z, const int8_t* q, int64_t* n_pairs, int32_t* ij,
                         int64_t max, double* e_atom, md_stream stream);

/* Every array a full step touches (all device pointers, caller order). */
typedef struct md_step_args {
    md_precision prec;
    double dt;
    double *x, *y, *z, *vx, *vy, *vz;
    double *fx, *fy, *fz;           /* forces of the current positions (in/out) */
    const double* inv_mass;
    const uint8_t* elem;
    const uint8_t* type;
    const uint32_t* atom_id;
    int8_t* q;
    double* epot;                   /* device FP64 [B] or NULL */
    double* ekin;                   /* device FP64 [B] or NULL */
} md_step_args;

/* One full step in the order of the method: md_integrate_vv phase 0 (kick + drift,
 * step counter s = k + 1), md_ionize_step (step s), md_build_cells(build_mode),
 * md_screened_forces (kappa of step s), md_integrate_vv phase 1 (kick); while the
 * Langevin coupling is bound, md_integrate_langevin replaces phase 0 (args->dt must
 * then equal the bound dt, else MD_ERR_ARG).  The forces
 * in fx, fy, fz must be those of the current positions on entry (call
 * md_screened_forces once before the first step).  Asynchronous. */
md_status md_step(md_ctx* ctx, const md_step_args* args, int32_t build_mode, md_stream stream);

/* HIP-graph form of md_step: records one step with the given MD_BUILD_* mode on
 * `stream` (not the null stream) into an executable graph, without executing it.
 * Replaying it runs the step with no host work; the step counter, schedules,
 * random streams and (with MD_BUILD_AUTO) list rebuilds advance on the device.
 * The pointers in args, and whether the Langevin coupling is bound, are baked into
 * the graph (the coupling's tables are read at replay time). */
typedef struct md_graph md_graph;
md_status md_graph_create(md_ctx* ctx, const md_step_args* args, int32_t build_mode,
                          md_stream stream, md_graph** out);
md_status md_graph_launch(md_graph* graph, md_stream stream);
md_status md_graph_destroy(md_graph* graph);

/* Measurement helper: time the main force kernel of each of the next `capacity`
 * force evaluations issued by md_screened_forces or md_step outside graph capture.
 * Two HIP events are recorded on the launch stream, immediately before and after
 * that kernel (the slot repack before it and the energy reduction after it fall
 * outside the interval).  A new call discards earlier records (it synchronizes the
 * device first); capacity 0 stops recording and frees the events.  Launches beyond
 * the capacity are not timed. */
md_status md_force_timer_start(md_ctx* ctx, int32_t capacity);

/* Number of timed launches so far in *n, and the first min(*n, max) kernel
 * durations, in milliseconds and launch order, in the host array ms.  Waits for
 * those launches to finish. */
md_status md_force_timer_read(md_ctx* ctx, float* ms, int32_t max, int32_t* n);

typedef struct md_stats {
    int64_t n_atoms, n_clusters, n_groups, n_entries;   /* from the last build */
    int64_t n_list_codes;                               /* sum of per-atom list lengths */
    int64_t max_list_len, list_capacity;                /* per atom */
    int64_t max_group_entries, group_entry_capacity;
    int64_t n_builds;                                   /* builds executed on the device */
    int64_t n_fast, n_fast_raw;                         /* fast atoms now (capped, found) */
    int32_t cluster_group;                              /* i-clusters per work-group in use */
    uint32_t flags;
} md_stats;

/* Synchronize `stream` and report build statistics. */
md_status md_get_stats(md_ctx* ctx, md_stats* out, md_stream stream);

/* Langevin electron-ion coupling (section II.B, Eq. 13 and Eq. 14): friction
 * -m gamma v and a Gaussian random force with <f(t) f(t')> = 2 m gamma k_B T_e delta(t - t')
 * on every atom.  Binds HOST tables: gamma [B*E] (ps^-1, per system and element; the
 * paper's gamma = rho_N g_e-ion, constant over a run), kt [B*(S+1)] (k_B T_e in kJ/mol per
 * system and step, read every step), and the time step dt they will be used with (the
 * library tabulates c1 = exp(-gamma dt)).  gamma NULL unbinds; md_bind_tables unbinds
 * too (the step count may change).  Errors: MD_ERR_STATE before md_bind_tables,
 * MD_ERR_ARG for kt NULL, dt not finite and > 0, or a gamma or kt entry negative or
 * not finite.  Synchronous. */
md_status md_bind_langevin(md_ctx* ctx, const double* gamma, const double* kt, double dt);

/* Phase 0 of the integrator with the coupling bound by md_bind_langevin (a reading:
 * the paper gives no discretization): for the step s = k + 1 this phase starts,
 *   v += h F;  x += (dt/2) v;  v = c1 v + sqrt(kT (1 - c1^2) / m) z;  x += (dt/2) v,
 * then the step counter advances as in md_integrate_vv phase 0 (displacement
 * tracking included).  z: three normals from Philox4x32-10 with counter
 * (atom_id, s, b, 1) and key (seed low, high), Box-Muller in FP64 on words (0, 1) and
 * (2, 3) with u = (w + 1/2) 2^-32.  elem: uint8 [N]; atom_id: uint32 [N]; the other
 * arrays as in md_integrate_vv.  dt must equal the bound one.  md_step uses this phase
 * automatically while the coupling is bound.  Asynchronous. */
md_status md_integrate_langevin(md_ctx* ctx, double dt, const double* inv_mass,
                                const uint8_t* elem, const uint32_t* atom_id, const double* fx,
                                const double* fy, const double* fz, double* x, double* y,
                                double* z, double* vx, double* vy, double* vz, md_stream stream);

/* Hybrid ion-sphere / Debye screening (section II.A, Eq. 4-7; a reading: the paper
 * gives the form but not the pair rule).  Binds the free-electron density ne
 * [B*(S+1)] (HOST array, nm^-3, per system and step, > 0) to go with the Debye
 * lengths of md_bind_tables.  From then on the Coulomb term of every pair is
 *   k_e (q_j phi_{q_i}(r) + q_i phi_{q_j}(r)) / 2,
 * where phi_Q is the potential of a charge-Q ion: Q/r + c1 - c2 r^2 inside r' (the
 * ion-sphere form of Eq. 5), c3 exp(-r/lambda_D)/r outside (the Debye form of
 * Eq. 2), with R = (3Q / (4 pi ne))^(1/3) (Eq. 4), r' from Eq. 7 and c1, c2, c3
 * matching value, slope and curvature at r'.  An infinite Debye length leaves the
 * bare Coulomb term.  The Lennard-Jones term, the cutoff and the pair set are
 * unchanged.  The library tabulates the coefficients for every (system, step,
 * charge < n_charge_states) on the host (FP64, and FP32 for the FP32 path).  ne
 * NULL unbinds; md_bind_tables unbinds too.  Applies to md_screened_forces,
 * md_step and graphs captured after the call.  Errors: MD_ERR_STATE before
 * md_bind_tables; MD_ERR_ARG for an ne entry not finite and > 0, or coefficients
 * that overflow (an ion sphere so large against lambda_D that exp(-r'/lambda_D)
 * underflows).  Synchronous. */
md_status md_bind_hybrid(md_ctx* ctx, const double* ne);

/* Force-field terms of section II.B (readings: the paper names the terms; the forms
 * of Eq. 9 and Eq. 10 are garbled).  Binds, replacing what was bound before (HOST
 * arrays, global atom indices of the batch):
 *   z_type [n_types], sigma_type [n_types]  atomic number and neutral Lennard-Jones
 *                      radius (nm, >= 0) per type, both or neither (NULL): the
 *                      radius of an atom shrinks to c sigma with c = 1 - q/Z
 *                      (Eq. 11) and a pair's radius is the mean of the two scaled
 *                      radii (the Lorentz rule of the c6/c12 tables), so at the
 *                      current charges c6 -> c6 s^6 and c12 -> c12 s^12 with
 *                      s = (c_i sigma_i + c_j sigma_j)/(sigma_i + sigma_j) (no
 *                      scaling for a pair of two zero radii);
 *   excl [n_excl][2]   pairs whose LJ term is omitted (the bonded 1-2 and 1-3
 *                      partners); their screened Coulomb term stays; needs
 *                      n_types <= 7 (excluded pairs carry type n_types in the
 *                      neighbour lists, which are rebuilt at the next build);
 *   bonds [n_bonds][2] with bond_par [n_bonds][3] = (D_e kJ/mol, beta nm^-1, b_e nm):
 *                      Morse bonds c D_e (1 - exp(-beta (r - b_e)))^2;
 *   angles [n_angles][3] (middle atom second) with angle_par [n_angles][2] =
 *                      (k kJ/mol/rad^2, theta0 rad): c k/2 (theta - theta0)^2;
 * where c = max(0, 1 - (sum of the term's charges)/(its atom count)) (Eq. 9).
 * md_screened_forces and md_step then add the bonded forces (FP64, one thread per
 * atom over its terms: no atomics) and their energies to epot.  Every count may be
 * 0 (that part is off).  Errors: MD_ERR_STATE before md_bind_tables; MD_ERR_ARG for
 * an atom index out of range, a term whose atoms are in different systems or repeat,
 * a parameter that is not finite, Z < 1, a negative radius, only one of z_type and
 * sigma_type, or exclusions with n_types > 7.  Graphs
 * captured before the call hold the previous arrays: capture again.  Synchronous. */
md_status md_bind_forcefield(md_ctx* ctx, const int8_t* z_type, const double* sigma_type,
                             const int32_t* excl, int64_t n_excl, const int32_t* bonds,
                             const double* bond_par, int64_t n_bonds, const int32_t* angles,
                             const double* angle_par, int64_t n_angles);

/* Pair-distance histogram for the radial distribution functions g_ab(r) behind the
 * partial structure factors of section II.C (Eq. 18).  Adds to hist (DEVICE uint64
 * [B][E][E][n_bins], not cleared: the caller zeroes it, or accumulates frames)
 * the count of every unordered pair {i, j} of one system whose minimum-image
 * distance r (the FP64 r^2 of the cutoff predicate) is below r_max, under
 * [b][min(e_i, e_j)][max(e_i, e_j)][k] with k such that (k dr)^2 <= r^2 < ((k+1) dr)^2,
 * dr = r_max / n_bins (squared edges evaluated as (k * dr) * (k * dr) in FP64).
 * Counts are exact.  Uses the last md_build_cells for the search (any positions
 * are accepted; atoms farther than skin/2 from their build position are handled by
 * a brute-force pass over their system, so many of them make the call slow).
 * Errors: MD_ERR_STATE before a build; MD_ERR_ARG for r_max outside (0, rc],
 * n_bins outside [1, 2048] or a NULL array.  The first call allocates about
 * 26 bytes per slot of workspace (do not capture it into a graph).  Asynchronous. */
md_status md_rdf_histogram(md_ctx* ctx, const double* x, const double* y, const double* z,
                           const uint8_t* elem, double r_max, int32_t n_bins, uint64_t* hist,
                           md_stream stream);

/* No-allocation form of md_rdf_histogram, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and the same counts, bit for bit; the search workspace
 * (25 bytes per slot of the context plus one per atom, about 28 bytes per atom) lives
 * in a fixed device array of MD_RDF_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends, instead of the context workspace that
 * md_rdf_histogram allocates on its first call.  Nothing is allocated and nothing
 * synchronizes, so the call can be captured.  Every call on one device shares that
 * device's array and leaves its contents behind: calls that overlap on one GPU (two
 * streams, contexts or threads) race and give wrong counts, so serialize them.
 * Errors: as md_rdf_histogram; MD_ERR_CAPACITY when the context needs more workspace
 * than the array holds; MD_ERR_HIP when the array's device address could not be
 * found.  Asynchronous. */
#define MD_RDF_SCRATCH_BYTES (32u << 20)
md_status md_rdf_histogram_noalloc(md_ctx* ctx, const double* x, const double* y,
                                   const double* z, const uint8_t* elem, double r_max,
                                   int32_t n_bins, uint64_t* hist, md_stream stream);

/* g_ab for one element pair from its n_bins counts (HOST arrays, FP64, no device
 * work): g[k] = counts[k] / (P / volume * 4/3 pi (r_{k+1}^3 - r_k^3)) with r_k = k dr
 * and P = n_a n_b pairs (same = 0) or n_a (n_a - 1) / 2 (same = 1: a = b).  The ideal
 * gas gives g = 1.  MD_ERR_ARG for bad sizes or volume <= 0. */
md_status md_rdf_normalize(int32_t n_bins, double r_max, const uint64_t* counts, int64_t n_a,
                           int64_t n_b, int32_t same, double volume, double* g);

/* Partial structure factor of section II.C, Eq. 18, from a binned g (HOST arrays):
 * S(q) = 1 + 4 pi rho0 / q * sum_k r_k (g_k - 1) sin(q r_k) dr with bin centres
 * r_k = (k + 1/2) dr, i.e. the midpoint rule of the integral truncated at r_max
 * (rho0 in nm^-3, q in nm^-1, q > 0).  MD_ERR_ARG for bad sizes or q <= 0. */
md_status md_structure_factor(int32_t n_bins, double r_max, const double* g, double rho0,
                              int32_t n_q, const double* q, double* S);

/* Host helpers for the per-step schedules (FP64, no device work). */

/* Debye length (section II.A, Eq. 3) in nm for electron temperature te_ev (eV) and
 * free-electron density ne_m3 (m^-3). */
double md_debye_length_nm(double te_ev, double ne_m3);

/* Per-step ionization probabilities of a sequential +1 process from charge-state
 * fractions (reading of section II.A: the stochastic integer charges average to
 * the CR fractions).  P: host [(S+1)*(Z+1)] fractions per step s and charge q;
 * p: host [(S+1)*(Z+1)] output, p[s][q] = (sum_{q'>q} P[s][q'] - P[s-1][q']) /
 * P[s-1][q] clamped to [0, 1] (0 where P[s-1][q] == 0, for q == Z and for s == 0). */
md_status md_rates_from_fractions(int64_t S, int32_t Z, const double* P, double* p);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
