// md_bonded.hip -- bonded terms of the force field (arXiv 2401.03180, section II.B):
// Morse bonds between atoms bonded in the native structure (Eq. 10, read as the
// standard Morse form D_e (1 - exp(-beta (r - b_e)))^2) and harmonic angle terms
// k/2 (theta - theta0)^2, each scaled by c = max(0, 1 - mean charge of its atoms)
// (Eq. 9), in FP64 with minimum-image bond vectors.
//
// One thread per atom evaluates every term the atom takes part in (per-atom CSR
// built on the host) and adds its own share of the force, so no atomics are needed
// and the result is deterministic; a term's energy is booked on its first atom and
// summed per system by the force finalize.  Runs after the pair kernels.
#include "md_internal.h"
#include "md_launch.h"

namespace md {

struct BondedArgs {
    const double *x, *y, *z;
    const int8_t* q;
    const int32_t* sys_of_atom;
    const GridSys* grid;
    int64_t N;
    const int32_t* bt_off;
    const int32_t* bt;
    const int32_t* bonds;
    const double* bond_par;
    const int32_t* angles;
    const double* angle_par;
    double *fx, *fy, *fz;
    double* bond_e;
    double* bond_blk;
};

__device__ inline void min_image(const GridSys& g, const double* x, const double* y,
                                 const double* z, int a, int b, double d[3])
{
#pragma clang fp contract(off)
    d[0] = x[a] - x[b];
    d[1] = y[a] - y[b];
    d[2] = z[a] - z[b];
    if (g.periodic)
        for (int k = 0; k < 3; ++k) d[k] = d[k] - g.L[k] * rint(d[k] * g.invL[k]);
}

__device__ inline double term_scale(const int8_t* q, const int32_t* at, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += (double)q[at[k]];
    const double c = 1.0 - s / (double)n;
    return c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
}

// The forces on atom a from every bonded term it takes part in (added to fx, fy,
// fz) and the energy of the terms it is the first atom of (returned, and stored).
__device__ inline double bonded_atom(const BondedArgs& A, int64_t a)
{
#pragma clang fp contract(off)
    const GridSys g = A.grid[A.sys_of_atom[a]];
    double F[3] = {0.0, 0.0, 0.0}, e = 0.0;
    for (int t = A.bt_off[a]; t < A.bt_off[a + 1]; ++t) {
        const int code = A.bt[t];
        const int id = code >> 1;
        if ((code & 1) == 0) {
            const int32_t* at = A.bonds + 2 * id;
            const double* p = A.bond_par + 3 * id;
            double d[3];
            min_image(g, A.x, A.y, A.z, at[0], at[1], d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double c = term_scale(A.q, at, 2);
            const double ex = exp(-p[1] * (r - p[2]));
            const double u = 1.0 - ex;
            const double dVdr = c * 2.0 * p[0] * u * p[1] * ex;
            // force on the first atom -dV/dr d/r, on the second its opposite
            const double sg = at[0] == a ? 1.0 : -1.0;
            for (int k = 0; k < 3; ++k) F[k] += sg * (-dVdr * d[k] / r);
            if (at[0] == a) e += c * p[0] * u * u;
        } else {
            const int32_t* at = A.angles + 3 * id;
            const double* p = A.angle_par + 2 * id;
            double va[3], vb[3];
            min_image(g, A.x, A.y, A.z, at[0], at[1], va);
            min_image(g, A.x, A.y, A.z, at[2], at[1], vb);
            const double la = sqrt(va[0] * va[0] + va[1] * va[1] + va[2] * va[2]);
            const double lb = sqrt(vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2]);
            double cs = (va[0] * vb[0] + va[1] * vb[1] + va[2] * vb[2]) / (la * lb);
            cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
            const double th = acos(cs);
            const double c = term_scale(A.q, at, 3);
            const double dVdth = c * p[0] * (th - p[1]);
            if (at[0] == a) e += 0.5 * c * p[0] * (th - p[1]) * (th - p[1]);
            const double sn = sqrt(1.0 - cs * cs);
            if (sn < 1e-12) continue;            // collinear: no defined gradient
            for (int k = 0; k < 3; ++k) {
                const double fa = dVdth / sn * (vb[k] / (la * lb) - cs * va[k] / (la * la));
                const double fb = dVdth / sn * (va[k] / (la * lb) - cs * vb[k] / (lb * lb));
                if (at[0] == a) F[k] += fa;
                else if (at[2] == a) F[k] += fb;
                else F[k] -= fa + fb;
            }
        }
    }
    A.fx[a] += F[0];
    A.fy[a] += F[1];
    A.fz[a] += F[2];
    A.bond_e[a] = e;
    return e;
}

__global__ void __launch_bounds__(kBondedBlock) k_bonded(BondedArgs A)
{
    __shared__ double s_e[kBondedBlock / 64];
    const int64_t a = blockIdx.x * (int64_t)kBondedBlock + threadIdx.x;
    double e = a < A.N ? bonded_atom(A, a) : 0.0;
    // the work-group's energy, in a fixed order (the finalize uses it for work-groups
    // that lie inside one system)
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if ((threadIdx.x & 63) == 0) s_e[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBondedBlock / 64; ++w) t += s_e[w];
        A.bond_blk[blockIdx.x] = t;
    }
}

void launch_bonded(Ctx* c, const double* x, const double* y, const double* z, const int8_t* q,
                   double* fx, double* fy, double* fz, hipStream_t st)
{
    const BondedArgs A{x, y, z, q, c->d_sys_of_atom, c->d_grid, c->N, c->d_bt_off, c->d_bt,
                       c->d_bonds, c->d_bond_par, c->d_angles, c->d_angle_par, fx, fy, fz,
                       c->d_bond_e, c->d_bond_blk};
    const int nb = (int)div_up(c->N, kBondedBlock);
    if (nb > 0) hipLaunchKernelGGL(k_bonded, dim3(nb), dim3(kBondedBlock), 0, st, A);
}

}  // namespace md
