/*
 * md_oracle.c -- plain FP64 CPU oracle for the screened-force + ionization step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
 * this file: only the tests, the smoke check and the benchmark's CPU-baseline leg
 * use it.  It shares no code, header, table or constant generator with the GPU
 * library.
 *
 * Build:  gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * Every floating-point operation is a separately rounded IEEE-754 binary64
 * operation in the order written (contraction is disabled), so the pair set,
 * the ionization draws and the integrator updates are bit-reproducible.
 *
 * What it computes (arXiv 2401.03180):
 *  - kappa = 1/lambda_D per force evaluation; Debye length from (T_e, n_e)
 *    (section II.A, Eq. 3).
 *  - The pair set S: all pairs inside one system whose minimum-image distance is
 *    below the cutoff rc (section II.B: cutoff chosen where the screened force is
 *    negligible; plain truncation).  Brute force over all pairs.
 *  - Pair potential phi = (k_e q_i q_j / r + c12/r^12 - c6/r^6) exp(-r/lambda_D)
 *    (section II.A, Eq. 2 screened Coulomb; Eq. 8 screened Lennard-Jones) and the
 *    force -d(phi)/dr along the pair axis.
 *  - Stochastic integer charges (section II.A: charges are integers assigned
 *    stochastically so that ensemble averages follow the CR charge-state
 *    fractions; section II.B: no partial charges).  Reading used: each step every
 *    atom below its maximum charge gains +1 with probability
 *    p = min(1, base[e][q] * g[b][s]), decided by a Philox4x32-10 draw keyed by
 *    (atom, step, system) and the system seed.
 *  - The ionization-probability table from CR charge-state fractions for a
 *    sequential +1 process (reading of section II.A's statement that the
 *    stochastic charges average to the CR fractions).
 *  - Velocity-Verlet integration of Newton's equation (section II.B, Eq. 12;
 *    the paper uses leap-frog, which yields the same positions).
 *  - Langevin coupling of the ions to the free electrons (section II.B, Eq. 13-14):
 *    friction and a random force of matching variance, integrated exactly over a
 *    step between two half drifts (a reading: the paper gives no discretization).
 *  - Hybrid ion-sphere / Debye potential (section II.A, Eq. 4-7), a reading: the
 *    ion-sphere form Q/r + c1 - c2 r^2 inside r', Debye form c3 exp(-r/lambda)/r
 *    outside, r' from Eq. 7, c1..c3 from matching value, slope and curvature at r';
 *    the energy of a pair is the mean of (charge j in the potential of ion i) and
 *    (charge i in the potential of ion j).
 *  - Force-field terms of section II.B (readings): Lennard-Jones radii scaled with
 *    the charge (Eq. 11), LJ omitted between atoms joined by a bond or an angle
 *    (screened Coulomb kept), Morse bonds and harmonic angles scaled by the mean
 *    charge of their atoms (Eq. 9, Eq. 10).
 *  - Radial distribution functions and partial structure factors (section II.C,
 *    Eq. 18): brute-force pair-distance histograms per element pair, their
 *    normalization against the ideal gas, and the sine transform of Eq. 18.
 *
 * Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KE 138.935457644382   /* 1/(4 pi eps0) in kJ mol^-1 nm e^-2 */

/* ------------------------------------------------------------------------ */
/* Schedules (section II.A, Eq. 3)                                          */
/* ------------------------------------------------------------------------ */

/* kappa = 1/lambda_D; an infinite Debye length means no screening. */
void orc_kappa_from_lambda(int64_t n, const double* lambda_d, double* kappa)
{
    for (int64_t k = 0; k < n; ++k)
        kappa[k] = isinf(lambda_d[k]) ? 0.0 : 1.0 / lambda_d[k];
}

/* Debye length lambda_D = sqrt(eps0 k_B T_e / (n_e e^2)) with T_e in eV
 * (k_B T_e = T_e * e joule) and n_e in m^-3; returned in nm. */
double orc_debye_length_nm(double te_ev, double ne_m3)
{
    const double eps0 = 8.8541878128e-12;     /* F/m (CODATA 2018) */
    const double e = 1.602176634e-19;         /* C (exact) */
    double kt = te_ev * e;                    /* joule */
    double lam = sqrt(eps0 * kt / (ne_m3 * e * e));
    return lam * 1e9;
}

/* Per-step ionization probabilities for a sequential +1 process from
 * charge-state fractions P[s][q], s = 0..S, q = 0..Z:
 *   flux out of charge q during step s  J_q(s) = sum_{q'>q} (P_q'(s) - P_q'(s-1)),
 *   p_q(s) = J_q(s) / P_q(s-1)  (0 where P_q(s-1) == 0), clamped to [0, 1].
 * Output p[s][q] for s = 1..S (row 0 is set to 0). */
void orc_rates_from_fractions(int64_t S, int32_t Z, const double* P, double* p)
{
    int32_t nq = Z + 1;
    for (int32_t q = 0; q < nq; ++q) p[q] = 0.0;
    for (int64_t s = 1; s <= S; ++s) {
        const double* prev = P + (s - 1) * nq;
        const double* cur = P + s * nq;
        double* out = p + s * nq;
        for (int32_t q = 0; q < nq; ++q) {
            double flux = 0.0;
            for (int32_t qq = q + 1; qq < nq; ++qq) flux += cur[qq] - prev[qq];
            double v = prev[q] > 0.0 ? flux / prev[q] : 0.0;
            if (v < 0.0) v = 0.0;
            if (v > 1.0) v = 1.0;
            out[q] = (q == Z) ? 0.0 : v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pair predicate and pair force (section II.A Eq. 2 and Eq. 8, II.B cutoff) */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t periodic;
    double L[3], invL[3];
    double rc2;
} orc_geom;

static void geom_init(orc_geom* g, int periodic, const double* box, double rc)
{
    g->periodic = periodic;
    for (int k = 0; k < 3; ++k) {
        g->L[k] = periodic ? box[k] : 0.0;
        g->invL[k] = periodic ? 1.0 / box[k] : 0.0;
    }
    g->rc2 = rc * rc;
}

/* Minimum-image separation d = x_i - x_j and r2 = (dx*dx + dy*dy) + dz*dz. */
static inline double pair_r2(const orc_geom* g, const double* x, const double* y,
                             const double* z, int64_t i, int64_t j, double d[3])
{
    d[0] = x[i] - x[j];
    d[1] = y[i] - y[j];
    d[2] = z[i] - z[j];
    if (g->periodic) {
        for (int k = 0; k < 3; ++k) d[k] = d[k] - g->L[k] * rint(d[k] * g->invL[k]);
    }
    double r2 = d[0] * d[0] + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    return r2;
}

/* ------------------------------------------------------------------------ */
/* Hybrid ion-sphere / Debye potential (section II.A, Eq. 4-7)               */
/* ------------------------------------------------------------------------ */

/* Coefficients of the potential of one ion of charge Q in an electron gas of
 * density ne (nm^-3) with Debye length lambda (nm):
 *   phi(r) = Q/r + c1 - c2 r^2          for r <  r'   (ion sphere, Eq. 5 form)
 *   phi(r) = c3 exp(-r/lambda) / r      for r >= r'   (Debye, Eq. 2 form)
 * with the ion-sphere radius R = (3Q / (4 pi ne))^(1/3) (Eq. 4), the transition
 * radius r' = lambda (((R/lambda)^3 + 1)^(1/3) - 1) (Eq. 7), and c1, c2, c3 the
 * solution of the three linear conditions that phi, phi' and phi'' agree at r'.
 * out = {r', c1, c2, c3}.  Q <= 0: no potential (all zero).  lambda = +inf (no
 * screening): r' = 0 and c3 = Q, the bare Coulomb potential. */
void orc_hybrid_coeffs(double Q, double lambda, double ne, double out[4])
{
    if (!(Q > 0.0)) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    if (isinf(lambda)) {
        out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = Q;
        return;
    }
    const double pi = 3.14159265358979323846;
    double R = cbrt(3.0 * Q / (4.0 * pi * ne));
    double a = R / lambda;
    double rp = lambda * (cbrt(a * a * a + 1.0) - 1.0);
    double kap = 1.0 / lambda;
    /* u(r) = exp(-kap r)/r and its first two derivatives at r' */
    double u0 = exp(-kap * rp) / rp;
    double t = kap + 1.0 / rp;
    double u1 = -u0 * t;
    double u2 = u0 * (t * t + 1.0 / (rp * rp));
    /* unknowns (c1, c2, c3):
     *   value:      c1 - rp^2 c2 - u0 c3 = -Q/rp
     *   slope:         -2 rp c2  - u1 c3 =  Q/rp^2
     *   curvature:     -2 c2     - u2 c3 = -2Q/rp^3
     * solved by Gaussian elimination with partial pivoting */
    double M[3][4] = {{1.0, -rp * rp, -u0, -Q / rp},
                      {0.0, -2.0 * rp, -u1, Q / (rp * rp)},
                      {0.0, -2.0, -u2, -2.0 * Q / (rp * rp * rp)}};
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        for (int k = 0; k < 4; ++k) {
            double tmp = M[c][k];
            M[c][k] = M[p][k];
            M[p][k] = tmp;
        }
        for (int r = c + 1; r < 3; ++r) {
            double m = M[r][c] / M[c][c];
            for (int k = c; k < 4; ++k) M[r][k] = M[r][k] - m * M[c][k];
        }
    }
    double x[3];
    for (int c = 2; c >= 0; --c) {
        double s = M[c][3];
        for (int k = c + 1; k < 3; ++k) s = s - M[c][k] * x[k];
        x[c] = s / M[c][c];
    }
    out[0] = rp;
    out[1] = x[0];
    out[2] = x[1];
    out[3] = x[2];
}

/* The potential phi of an ion of charge Q with coefficients h = {r', c1, c2, c3}
 * (orc_hybrid_coeffs) at distance r, and w = -r dphi/dr. */
void orc_hybrid_phi(double Q, const double h[4], double kappa, double r, double* phi, double* w)
{
    if (r < h[0]) {
        *phi = Q / r + h[1] - h[2] * r * r;
        *w = Q / r + 2.0 * h[2] * r * r;
    } else {
        double e = exp(-kappa * r) / r;
        *phi = h[3] * e;
        *w = h[3] * e * (1.0 + kappa * r);
    }
}

/* Pair energy and scalar force with the hybrid Coulomb term:
 * phi = k_e (q_j phi_i(r) + q_i phi_j(r)) / 2 + LJ (screened as in Eq. 8). */
static void pair_phi_f_hybrid(double r2, int qi, int qj, const double* hi, const double* hj,
                              double c6, double c12, double kappa, int screen_lj, double* phi,
                              double* f)
{
    double r = sqrt(r2);
    double rinv2 = 1.0 / r2;
    double rinv6 = rinv2 * rinv2 * rinv2;
    double s = exp(-kappa * r);
    double pi_ = 0.0, wi = 0.0, pj = 0.0, wj = 0.0;
    if (qi > 0) orc_hybrid_phi((double)qi, hi, kappa, r, &pi_, &wi);
    if (qj > 0) orc_hybrid_phi((double)qj, hj, kappa, r, &pj, &wj);
    double uc = 0.5 * ORC_KE * ((double)qj * pi_ + (double)qi * pj);
    double wc = 0.5 * ORC_KE * ((double)qj * wi + (double)qi * wj);
    double lj12 = c12 * rinv6 * rinv6;
    double lj6 = c6 * rinv6;
    double ulj = lj12 - lj6;
    double wlj = 12.0 * lj12 - 6.0 * lj6;
    if (screen_lj) {
        *phi = uc + ulj * s;
        *f = (wc + (wlj + ulj * (kappa * r)) * s) * rinv2;
    } else {
        *phi = uc + ulj;
        *f = (wc + wlj) * rinv2;
    }
}

/* Screened pair energy phi and scalar force f (F_i = f * d, F_j = -f * d). */
static inline void pair_phi_f(double r2, double qiqj_ke, double c6, double c12,
                              double kappa, int screen_lj, double* phi, double* f)
{
    double r = sqrt(r2);
    double rinv2 = 1.0 / r2;
    double rinv6 = rinv2 * rinv2 * rinv2;
    double s = exp(-kappa * r);
    double uc = qiqj_ke / r;
    double lj12 = c12 * rinv6 * rinv6;
    double lj6 = c6 * rinv6;
    double ulj = lj12 - lj6;
    double wlj = 12.0 * lj12 - 6.0 * lj6;           /* -r d(uLJ)/dr */
    if (screen_lj) {
        *phi = (uc + ulj) * s;
        *f = ((uc + wlj) + (uc + ulj) * (kappa * r)) * s * rinv2;
    } else {
        *phi = uc * s + ulj;
        *f = (uc + uc * (kappa * r)) * s * rinv2 + wlj * rinv2;
    }
}

/* Optional force-field terms of the pair loop (NULL members: off).
 *   inv_z[t], sigma[t]  1/Z and the neutral Lennard-Jones radius of type t: the
 *              radius of atom i shrinks with its charge to c_i sigma_i, c_i =
 *              1 - q_i / Z_i (Eq. 11), and a pair's radius is the arithmetic mean of
 *              the two scaled radii (the tables' Lorentz rule), so the pair's LJ
 *              radius is scaled by s = (c_i sigma_i + c_j sigma_j) / (sigma_i +
 *              sigma_j): c6 -> c6 s^6, c12 -> c12 s^12 (no scaling when both radii
 *              are zero: such a pair has no LJ term);
 *   excl_off, excl  per-atom sorted lists (CSR over global atom indices) of the
 *              partners whose LJ term is omitted (bonded 1-2 and 1-3 pairs). */
typedef struct {
    const double* inv_z;
    const double* sigma;
    const int64_t* excl_off;
    const int64_t* excl;
} orc_ff;

static int excluded(const orc_ff* ff, int64_t i, int64_t j)
{
    if (!ff || !ff->excl_off) return 0;
    for (int64_t k = ff->excl_off[i]; k < ff->excl_off[i + 1]; ++k)
        if (ff->excl[k] == j) return 1;
    return 0;
}

/* c6, c12 of pair (i, j) after exclusion and charge scaling. */
static void pair_lj(const orc_ff* ff, int64_t i, int64_t j, const int8_t* q, const uint8_t* type,
                    int32_t n_types, const double* c6, const double* c12, double* a6, double* a12)
{
    int tt = type[i] * n_types + type[j];
    *a6 = c6[tt];
    *a12 = c12[tt];
    if (excluded(ff, i, j)) {
        *a6 = 0.0;
        *a12 = 0.0;
        return;
    }
    if (ff && ff->inv_z && ff->sigma) {
        double si = ff->sigma[type[i]], sj = ff->sigma[type[j]];
        double ci = 1.0 - (double)q[i] * ff->inv_z[type[i]];
        double cj = 1.0 - (double)q[j] * ff->inv_z[type[j]];
        double sum = si + sj;
        if (!(sum > 0.0)) return;
        double s = (ci * si + cj * sj) / sum;
        double s6 = s * s * s * s * s * s;
        *a6 = *a6 * s6;
        *a12 = *a12 * s6 * s6;
    }
}

/* Brute-force forces and energies over all i<j pairs of every system.
 *   kappa[b]  screening constant of system b for this force evaluation.
 *   e_atom[i] = 1/2 sum_j phi_ij ;  a_atom[i] = sum_j |f_ij| r_ij ;
 *   epot[b]   = sum over pairs of system b.
 * Any of e_atom, a_atom, epot may be NULL.  Returns |S|. */
int64_t orc_forces(int64_t n_sys, const int64_t* sys_off, int32_t periodic,
                   const double* box, double rc, const double* x, const double* y,
                   const double* z, const int8_t* q, const uint8_t* type, int32_t n_types,
                   const double* c6, const double* c12, const double* kappa,
                   int32_t screen_lj, double* fx, double* fy, double* fz,
                   double* e_atom, double* a_atom, double* epot, const double* hyb,
                   int32_t n_q, const double* inv_z, const double* sigma,
                   const int64_t* excl_off,
                   const int64_t* excl)
{
    orc_ff ffv = {inv_z, sigma, excl_off, excl};
    const orc_ff* ff = &ffv;
    int64_t npairs = 0;
    int64_t n = sys_off[n_sys];
    for (int64_t i = 0; i < n; ++i) {
        fx[i] = fy[i] = fz[i] = 0.0;
        if (e_atom) e_atom[i] = 0.0;
        if (a_atom) a_atom[i] = 0.0;
    }
    for (int64_t b = 0; b < n_sys; ++b) {
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, rc);
        double esum = 0.0;
        for (int64_t i = sys_off[b]; i < sys_off[b + 1]; ++i) {
            for (int64_t j = i + 1; j < sys_off[b + 1]; ++j) {
                double d[3];
                double r2 = pair_r2(&g, x, y, z, i, j, d);
                if (!(r2 < g.rc2)) continue;
                if (r2 <= 0.0) abort();   /* coincident atoms: undefined */
                double a6, a12;
                pair_lj(ff, i, j, q, type, n_types, c6, c12, &a6, &a12);
                double qq = ORC_KE * ((double)q[i] * (double)q[j]);
                double phi, f;
                if (hyb)
                    pair_phi_f_hybrid(r2, q[i], q[j], hyb + 4 * (b * n_q + q[i]),
                                      hyb + 4 * (b * n_q + q[j]), a6, a12, kappa[b],
                                      screen_lj, &phi, &f);
                else
                    pair_phi_f(r2, qq, a6, a12, kappa[b], screen_lj, &phi, &f);
                fx[i] += f * d[0]; fy[i] += f * d[1]; fz[i] += f * d[2];
                fx[j] -= f * d[0]; fy[j] -= f * d[1]; fz[j] -= f * d[2];
                if (e_atom) { e_atom[i] += 0.5 * phi; e_atom[j] += 0.5 * phi; }
                if (a_atom) {
                    double mag = fabs(f) * sqrt(r2);
                    a_atom[i] += mag; a_atom[j] += mag;
                }
                esum += phi;
                ++npairs;
            }
        }
        if (epot) epot[b] = esum;
    }
    return npairs;
}

/* Rows mode: for the listed atoms i, F_i, e_i and A_i against every j of the same
 * system (full j loop, so rows are independent; OpenMP over rows).
 * sys_of_row[r] is the system of row r.  Used for sub-box checks of large
 * systems and for the CPU timing baseline.  row_hits[r] (may be NULL) receives the
 * number of partners of row r.  Returns the number of (i, j) hits. */
int64_t orc_forces_rows(int64_t n_rows, const int64_t* rows, const int64_t* sys_of_row,
                        const int64_t* sys_off, int32_t periodic, const double* box, double rc,
                        const double* x, const double* y, const double* z, const int8_t* q,
                        const uint8_t* type, int32_t n_types, const double* c6,
                        const double* c12, const double* kappa, int32_t screen_lj,
                        double* fx, double* fy, double* fz, double* e_atom, double* a_atom,
                        int64_t* row_hits, int32_t n_threads, const double* hyb, int32_t n_q,
                        const double* inv_z, const double* sigma, const int64_t* excl_off,
                        const int64_t* excl)
{
    orc_ff ffv = {inv_z, sigma, excl_off, excl};
    const orc_ff* ff = &ffv;
    int64_t hits = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : hits)
#endif
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = rows[r];
        int64_t b = sys_of_row[r];
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, rc);
        double F[3] = {0.0, 0.0, 0.0}, e = 0.0, a = 0.0;
        int64_t h = 0;
        for (int64_t j = sys_off[b]; j < sys_off[b + 1]; ++j) {
            if (j == i) continue;
            double d[3];
            double r2 = pair_r2(&g, x, y, z, i, j, d);
            if (!(r2 < g.rc2)) continue;
            double a6, a12;
            pair_lj(ff, i, j, q, type, n_types, c6, c12, &a6, &a12);
            double qq = ORC_KE * ((double)q[i] * (double)q[j]);
            double phi, f;
            if (hyb)
                pair_phi_f_hybrid(r2, q[i], q[j], hyb + 4 * (b * n_q + q[i]),
                                  hyb + 4 * (b * n_q + q[j]), a6, a12, kappa[b], screen_lj,
                                  &phi, &f);
            else
                pair_phi_f(r2, qq, a6, a12, kappa[b], screen_lj, &phi, &f);
            F[0] += f * d[0]; F[1] += f * d[1]; F[2] += f * d[2];
            e += 0.5 * phi;
            a += fabs(f) * sqrt(r2);
            ++h;
        }
        hits += h;
        if (row_hits) row_hits[r] = h;
        fx[r] = F[0]; fy[r] = F[1]; fz[r] = F[2];
        if (e_atom) e_atom[r] = e;
        if (a_atom) a_atom[r] = a;
    }
    return hits;
}

/* The pair set S as (i, j) with i < j (global caller indices), in i-major order.
 * Writes at most max pairs; returns |S|. */
int64_t orc_pairs(int64_t n_sys, const int64_t* sys_off, int32_t periodic, const double* box,
                  double rc, const double* x, const double* y, const double* z,
                  int64_t* out_i, int64_t* out_j, int64_t max)
{
    int64_t cnt = 0;
    for (int64_t b = 0; b < n_sys; ++b) {
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, rc);
        for (int64_t i = sys_off[b]; i < sys_off[b + 1]; ++i)
            for (int64_t j = i + 1; j < sys_off[b + 1]; ++j) {
                double d[3];
                double r2 = pair_r2(&g, x, y, z, i, j, d);
                if (r2 < g.rc2) {
                    if (cnt < max) { out_i[cnt] = i; out_j[cnt] = j; }
                    ++cnt;
                }
            }
    }
    return cnt;
}

/* Rows mode of the pair set: for each listed atom i (rows[r], system sys_of_row[r]),
 * every partner j != i of its system with r2 < rc2, ascending in j.  Partners of
 * row r go to out_j[off[r] .. off[r + 1]), where off (n_rows + 1) is computed here
 * from the counts; at most max partners are written in total.  Returns the total. */
int64_t orc_pairs_rows(int64_t n_rows, const int64_t* rows, const int64_t* sys_of_row,
                       const int64_t* sys_off, int32_t periodic, const double* box, double rc,
                       const double* x, const double* y, const double* z, int64_t* off,
                       int64_t* out_j, int64_t max, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t r = 0; r < n_rows; ++r) {         /* count */
        int64_t i = rows[r], b = sys_of_row[r], h = 0;
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, rc);
        for (int64_t j = sys_off[b]; j < sys_off[b + 1]; ++j) {
            double d[3];
            if (j != i && pair_r2(&g, x, y, z, i, j, d) < g.rc2) ++h;
        }
        off[r + 1] = h;
    }
    off[0] = 0;
    for (int64_t r = 0; r < n_rows; ++r) off[r + 1] += off[r];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t r = 0; r < n_rows; ++r) {         /* fill */
        int64_t i = rows[r], b = sys_of_row[r], k = off[r];
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, rc);
        for (int64_t j = sys_off[b]; j < sys_off[b + 1]; ++j) {
            double d[3];
            if (j != i && pair_r2(&g, x, y, z, i, j, d) < g.rc2) {
                if (k < max) out_j[k] = j;
                ++k;
            }
        }
    }
    return off[n_rows];
}

/* ------------------------------------------------------------------------ */
/* Bonded terms (section II.B, Eq. 9 and Eq. 10; readings)                  */
/* ------------------------------------------------------------------------ */

/* Minimum-image separation a - b of two atoms of system geometry g. */
static void bond_vec(const orc_geom* g, const double* x, const double* y, const double* z,
                     int64_t a, int64_t b, double d[3])
{
    d[0] = x[a] - x[b];
    d[1] = y[a] - y[b];
    d[2] = z[a] - z[b];
    if (g->periodic)
        for (int k = 0; k < 3; ++k) d[k] = d[k] - g->L[k] * rint(d[k] * g->invL[k]);
}

/* Scale of a bonded term over n atoms: c = 1 - (sum of their charges)/n, clamped to
 * [0, 1] (Eq. 9: 1 for neutral atoms, 0 once the mean charge reaches 1). */
static double bonded_scale(const int8_t* q, const int32_t* atoms, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += (double)q[atoms[k]];
    double c = 1.0 - s / (double)n;
    return c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
}

/* Morse bonds V = c D_e (1 - exp(-beta (r - b_e)))^2 (Eq. 10 read as the standard
 * Morse form) and harmonic angles V = c k/2 (theta - theta0)^2 with theta the angle
 * at the middle atom.  Forces are ADDED to fx, fy, fz; the energy of every term is
 * added to epot of the system of its first atom (epot may be NULL). */
void orc_bonded(int64_t n_sys, const int64_t* sys_off, int32_t periodic, const double* box,
                const double* x, const double* y, const double* z, const int8_t* q,
                int64_t n_bonds, const int32_t* bonds, const double* bond_par,
                int64_t n_angles, const int32_t* angles, const double* angle_par,
                double* fx, double* fy, double* fz, double* epot)
{
    for (int64_t t = 0; t < n_bonds; ++t) {
        const int32_t* at = bonds + 2 * t;
        int64_t i = at[0], j = at[1];
        int64_t b = 0;
        while (b + 1 < n_sys && sys_off[b + 1] <= i) ++b;
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, 0.0);
        double d[3];
        bond_vec(&g, x, y, z, i, j, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double De = bond_par[3 * t], beta = bond_par[3 * t + 1], be = bond_par[3 * t + 2];
        double c = bonded_scale(q, at, 2);
        double ex = exp(-beta * (r - be));
        double u = 1.0 - ex;
        double V = c * De * u * u;
        double dVdr = c * 2.0 * De * u * beta * ex;
        /* F_i = -dV/dr * d/r, F_j = -F_i */
        for (int k = 0; k < 3; ++k) {
            double fk = -dVdr * d[k] / r;
            double* F = k == 0 ? fx : (k == 1 ? fy : fz);
            F[i] += fk;
            F[j] -= fk;
        }
        if (epot) epot[b] += V;
    }
    for (int64_t t = 0; t < n_angles; ++t) {
        const int32_t* at = angles + 3 * t;
        int64_t i = at[0], j = at[1], k = at[2];
        int64_t b = 0;
        while (b + 1 < n_sys && sys_off[b + 1] <= i) ++b;
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, 0.0);
        double a[3], e[3];
        bond_vec(&g, x, y, z, i, j, a);
        bond_vec(&g, x, y, z, k, j, e);
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        double cs = (a[0] * e[0] + a[1] * e[1] + a[2] * e[2]) / (la * le);
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double th = acos(cs);
        double kth = angle_par[2 * t], th0 = angle_par[2 * t + 1];
        double c = bonded_scale(q, at, 3);
        double V = 0.5 * c * kth * (th - th0) * (th - th0);
        double dVdth = c * kth * (th - th0);
        double sn = sqrt(1.0 - cs * cs);
        if (epot) epot[b] += V;
        if (sn < 1e-12) continue;          /* collinear: the gradient is undefined */
        /* d(theta)/d(a) = -(e/(|a||e|) - cos a/|a|^2) / sin, likewise for e */
        double Fi[3], Fk[3];
        for (int m = 0; m < 3; ++m) {
            Fi[m] = dVdth / sn * (e[m] / (la * le) - cs * a[m] / (la * la));
            Fk[m] = dVdth / sn * (a[m] / (la * le) - cs * e[m] / (le * le));
        }
        double* F[3] = {fx, fy, fz};
        for (int m = 0; m < 3; ++m) {
            F[m][i] += Fi[m];
            F[m][k] += Fk[m];
            F[m][j] -= Fi[m] + Fk[m];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Radial distribution functions and structure factors (section II.C, Eq. 18) */
/* ------------------------------------------------------------------------ */

/* Histogram of the minimum-image distances of all unordered pairs of each system
 * below r_max: pair {i, j} goes to hist[b][min(e_i,e_j)][max(e_i,e_j)][k] (added to)
 * with k such that (k dr)^2 <= r^2 < ((k+1) dr)^2, dr = r_max / n_bins, and r^2 the
 * expression of the cutoff predicate.  Brute force over all pairs (OpenMP over i,
 * with per-thread histograms summed at the end: integer counts, so the result does
 * not depend on the thread count). */
void orc_rdf_histogram(int64_t n_sys, const int64_t* sys_off, int32_t periodic,
                       const double* box, const double* x, const double* y, const double* z,
                       const uint8_t* elem, int32_t E, double r_max, int32_t n_bins,
                       uint64_t* hist)
{
    size_t per_sys = (size_t)E * (size_t)E * (size_t)n_bins;
    double dr = r_max / (double)n_bins;
    double* e2 = (double*)malloc(sizeof(double) * (size_t)(n_bins + 1));
    for (int32_t k = 0; k <= n_bins; ++k) {
        double e = (double)k * dr;
        e2[k] = e * e;
    }
    for (int64_t b = 0; b < n_sys; ++b) {
        orc_geom g;
        geom_init(&g, periodic, periodic ? box + 3 * b : NULL, r_max);
        uint64_t* hb = hist + (size_t)b * per_sys;
#ifdef _OPENMP
#pragma omp parallel
#endif
        {
            uint64_t* mine = (uint64_t*)calloc(per_sys, sizeof(uint64_t));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t i = sys_off[b]; i < sys_off[b + 1]; ++i)
                for (int64_t j = i + 1; j < sys_off[b + 1]; ++j) {
                    double d[3];
                    double r2 = pair_r2(&g, x, y, z, i, j, d);
                    if (!(r2 < e2[n_bins])) continue;
                    /* largest k with e2[k] <= r2 (binary search; e2[0] = 0 <= r2) */
                    int32_t lo = 0, hi = n_bins - 1;
                    while (lo < hi) {
                        int32_t mid = (lo + hi + 1) / 2;
                        if (e2[mid] <= r2) lo = mid; else hi = mid - 1;
                    }
                    int ea = elem[i] < elem[j] ? elem[i] : elem[j];
                    int eb = elem[i] < elem[j] ? elem[j] : elem[i];
                    mine[((size_t)ea * E + eb) * n_bins + lo] += 1;
                }
#ifdef _OPENMP
#pragma omp critical
#endif
            for (size_t k = 0; k < per_sys; ++k) hb[k] += mine[k];
            free(mine);
        }
    }
    free(e2);
}

/* g(r) of one element pair: counts over the ideal-gas expectation, P / V times the
 * shell volume 4/3 pi (r_{k+1}^3 - r_k^3), with P = n_a n_b pairs of distinct
 * elements or n_a (n_a - 1) / 2 pairs of one element. */
void orc_rdf_normalize(int32_t n_bins, double r_max, const uint64_t* counts, int64_t n_a,
                       int64_t n_b, int32_t same, double volume, double* g)
{
    const double pi = 3.14159265358979323846;
    double P = same ? (double)n_a * (double)(n_a - 1) / 2.0 : (double)n_a * (double)n_b;
    double dr = r_max / (double)n_bins;
    for (int32_t k = 0; k < n_bins; ++k) {
        double r0 = k * dr, r1 = (k + 1) * dr;
        double expect = P / volume * (4.0 * pi / 3.0) * (r1 * r1 * r1 - r0 * r0 * r0);
        g[k] = expect > 0.0 ? (double)counts[k] / expect : 0.0;
    }
}

/* Eq. 18 with the integral over [0, r_max] by the midpoint rule on the bins:
 * S(q) = 1 + (4 pi rho0 / q) sum_k r_k (g_k - 1) sin(q r_k) dr, r_k = (k + 1/2) dr. */
void orc_structure_factor(int32_t n_bins, double r_max, const double* g, double rho0,
                          int32_t n_q, const double* q, double* S)
{
    const double pi = 3.14159265358979323846;
    double dr = r_max / (double)n_bins;
    for (int32_t m = 0; m < n_q; ++m) {
        double integral = 0.0;
        for (int32_t k = 0; k < n_bins; ++k) {
            double r = (k + 0.5) * dr;
            integral += r * (g[k] - 1.0) * sin(q[m] * r) * dr;
        }
        S[m] = 1.0 + 4.0 * pi * rho0 / q[m] * integral;
    }
}

/* Squared minimum-image distance of one pair (for adversarial predicate tests). */
double orc_pair_r2(int32_t periodic, const double* box, const double* x, const double* y,
                   const double* z, int64_t i, int64_t j)
{
    orc_geom g;
    geom_init(&g, periodic, box, 0.0);
    double d[3];
    return pair_r2(&g, x, y, z, i, j, d);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11)                                     */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Ionization update                                                        */
/* ------------------------------------------------------------------------ */

/* One ionization step s >= 1 for every atom.  g_step[b] = g[b][s].  An atom of
 * element e with charge q < qmax[e] gains +1 iff u < floor(p * 2^32), where
 * p = min(1, base[e*Q + q] * g_step[b]) and u is word 0 of
 * Philox4x32-10(counter = (atom_id, s, b, 0), key = (seed_b low, seed_b high)).
 * Returns the number of atoms that were ionized. */
int64_t orc_ionize(int64_t n_sys, const int64_t* sys_off, const uint8_t* elem,
                   const uint32_t* atom_id, int8_t* q, const int8_t* qmax, int32_t Q,
                   const double* base, const double* g_step, const uint64_t* seeds,
                   int64_t step)
{
    int64_t jumps = 0;
    for (int64_t b = 0; b < n_sys; ++b) {
        uint32_t key[2] = {(uint32_t)(seeds[b] & 0xFFFFFFFFu), (uint32_t)(seeds[b] >> 32)};
        for (int64_t a = sys_off[b]; a < sys_off[b + 1]; ++a) {
            int e = elem[a];
            int qa = q[a];
            if (qa >= qmax[e]) continue;
            double p = base[e * Q + qa] * g_step[b];
            if (p > 1.0) p = 1.0;
            uint64_t thresh = (uint64_t)floor(p * 4294967296.0);
            uint32_t ctr[4] = {atom_id[a], (uint32_t)step, (uint32_t)b, 0u};
            uint32_t r[4];
            orc_philox4x32_10(ctr, key, r);
            if ((uint64_t)r[0] < thresh) {
                q[a] = (int8_t)(qa + 1);
                ++jumps;
            }
        }
    }
    return jumps;
}

/* ------------------------------------------------------------------------ */
/* Velocity Verlet (section II.B, Eq. 12)                                   */
/* ------------------------------------------------------------------------ */

/* phase 0: v += h F ; x += dt v.   phase 1: v += h F.   h = (0.5 dt) / m. */
void orc_vv(int64_t n, int32_t phase, double dt, const double* inv_mass, const double* fx,
            const double* fy, const double* fz, double* x, double* y, double* z, double* vx,
            double* vy, double* vz)
{
    double hdt = 0.5 * dt;
    for (int64_t a = 0; a < n; ++a) {
        double h = hdt * inv_mass[a];
        vx[a] = vx[a] + h * fx[a];
        vy[a] = vy[a] + h * fy[a];
        vz[a] = vz[a] + h * fz[a];
        if (phase == 0) {
            x[a] = x[a] + dt * vx[a];
            y[a] = y[a] + dt * vy[a];
            z[a] = z[a] + dt * vz[a];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Langevin electron-ion coupling (section II.B, Eq. 13 and Eq. 14)          */
/* ------------------------------------------------------------------------ */

/* Three standard normals for atom `atom_id` of system b at step s: Philox4x32-10
 * with counter (atom_id, s, b, 1) and key (seed low, seed high), Box-Muller in FP64
 * on output words (0, 1) and (2, 3) with u = (w + 1/2) 2^-32:
 * z = sqrt(-2 ln u_a) cos(2 pi u_b), sqrt(-2 ln u_a) sin(2 pi u_b), and the cosine
 * of the second pair. */
void orc_langevin_normals(uint32_t atom_id, int64_t s, int64_t b, uint64_t seed, double z[3])
{
    const uint32_t ctr[4] = {atom_id, (uint32_t)s, (uint32_t)b, 1u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const double two_pi = 6.283185307179586;
    double u0 = ((double)w[0] + 0.5) * 2.3283064365386963e-10;
    double u1 = ((double)w[1] + 0.5) * 2.3283064365386963e-10;
    double u2 = ((double)w[2] + 0.5) * 2.3283064365386963e-10;
    double u3 = ((double)w[3] + 0.5) * 2.3283064365386963e-10;
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    z[0] = r0 * cos(two_pi * u1);
    z[1] = r0 * sin(two_pi * u1);
    z[2] = r1 * cos(two_pi * u3);
}

/* Phase 0 of the integrator with the coupling, for step s (the step this phase
 * starts): the friction -m gamma v and the random force of variance 2 m gamma kT
 * integrated exactly over dt between two half drifts:
 *   v += h F;  x += (dt/2) v;  v = c1 v + sqrt(kT (1 - c1^2) / m) z;  x += (dt/2) v,
 * with h = (dt/2)/m, c1 = c1_tab[b * E + e] (= exp(-gamma dt), tabulated by the caller)
 * and kT = kt[b * S1 + s] (k_B T_e in kJ/mol).  Phase 1 is the plain kick. */
void orc_vv_langevin(int64_t n_sys, const int64_t* sys_off, const uint8_t* elem, int32_t E,
                     const uint32_t* atom_id, const double* c1_tab, const double* kt, int64_t S1,
                     int64_t s, const uint64_t* seeds, double dt, const double* inv_mass,
                     const double* fx, const double* fy, const double* fz, double* x, double* y,
                     double* z, double* vx, double* vy, double* vz)
{
    double hdt = 0.5 * dt;
    for (int64_t b = 0; b < n_sys; ++b) {
        double kT = kt[b * S1 + s];
        for (int64_t a = sys_off[b]; a < sys_off[b + 1]; ++a) {
            double h = hdt * inv_mass[a];
            double c1 = c1_tab[b * E + elem[a]];
            double sig = sqrt(kT * (1.0 - c1 * c1) * inv_mass[a]);
            double g[3];
            orc_langevin_normals(atom_id[a], s, b, seeds[b], g);
            double v[3] = {vx[a] + h * fx[a], vy[a] + h * fy[a], vz[a] + h * fz[a]};
            double* p[3] = {&x[a], &y[a], &z[a]};
            for (int d = 0; d < 3; ++d) {
                *p[d] = *p[d] + hdt * v[d];
                v[d] = c1 * v[d] + sig * g[d];
                *p[d] = *p[d] + hdt * v[d];
            }
            vx[a] = v[0];
            vy[a] = v[1];
            vz[a] = v[2];
        }
    }
}

/* Kinetic energy per system: 1/2 sum m v^2. */
void orc_ekin(int64_t n_sys, const int64_t* sys_off, const double* inv_mass, const double* vx,
              const double* vy, const double* vz, double* ekin)
{
    for (int64_t b = 0; b < n_sys; ++b) {
        double s = 0.0;
        for (int64_t a = sys_off[b]; a < sys_off[b + 1]; ++a) {
            double v2 = vx[a] * vx[a] + vy[a] * vy[a];
            v2 = v2 + vz[a] * vz[a];
            s += 0.5 * v2 / inv_mass[a];
        }
        ekin[b] = s;
    }
}
