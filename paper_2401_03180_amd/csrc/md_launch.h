// md_launch.h -- host-side launchers implemented in the kernel translation units.
#pragma once

#include "md_internal.h"

namespace md {

constexpr int kVvBlock = 512;       // threads per work-group of the integrator kernels (measured: 512 beats 128, 256, 1024)

// md_step.hip
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, const int32_t* gate,
                 hipStream_t st);
void launch_scan64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, const int32_t* gate,
                   hipStream_t st);
void launch_ionize(Ctx* c, const uint8_t* elem, const uint32_t* atom_id, int8_t* q,
                   hipStream_t st);
void launch_vv(Ctx* c, int phase, double dt, const double* inv_mass, const double* fx,
               const double* fy, const double* fz, double* x, double* y, double* z, double* vx,
               double* vy, double* vz, double* ekin, hipStream_t st);
int64_t vv_partials_needed(int64_t N, int B);
// phase 0 of velocity Verlet with the ionization of the step it starts (md_step)
void launch_vv0_ionize(Ctx* c, double dt, const double* inv_mass, const double* fx,
                       const double* fy, const double* fz, double* x, double* y, double* z,
                       double* vx, double* vy, double* vz, const uint8_t* elem,
                       const uint32_t* atom_id, int8_t* q, hipStream_t st);
// phase 1 of velocity Verlet with the force finalize of the step (md_step)
void launch_vv1_finalize(Ctx* c, double dt, const double* inv_mass, const double* fx,
                         const double* fy, const double* fz, double* vx, double* vy, double* vz,
                         double* ekin, double* epot, hipStream_t st);
// phase 0 with the Langevin coupling (md_integrate_langevin)
void launch_vv0_langevin(Ctx* c, double dt, const double* inv_mass, const uint8_t* elem,
                         const uint32_t* atom_id, const double* fx, const double* fy,
                         const double* fz, double* x, double* y, double* z, double* vx,
                         double* vy, double* vz, hipStream_t st);
int vv_blocks(int64_t N);
// bonded terms (md_bonded.hip): forces added to fx, fy, fz; energies per atom and
// per work-group of kBondedBlock atoms
constexpr int kBondedBlock = 256;
void launch_bonded(Ctx* c, const double* x, const double* y, const double* z, const int8_t* q,
                   double* fx, double* fy, double* fz, hipStream_t st);
// pair-distance histograms (md_rdf.hip)
constexpr size_t kRdfLdsMax = 48 * 1024;
constexpr int kRdfMaxBins = 2048;
// moved (N bytes), xr (3 * cap_slots doubles), er (cap_slots bytes): the search
// workspace, every byte of it written before it is read
void launch_rdf(Ctx* c, const double* x, const double* y, const double* z, const uint8_t* elem,
                double r_max, int n_bins, unsigned long long* hist, uint8_t* moved, double* xr,
                uint8_t* er, hipStream_t st);
// the same workspace in the fixed per-device array of the no-allocation entry point:
// rdf_scratch_setup looks its device address up once per device (with that device
// current); rdf_scratch returns it (NULL if the lookup failed or never ran)
constexpr size_t kRdfScratchBytes = MD_RDF_SCRATCH_BYTES;
size_t rdf_scratch_bytes(int64_t N, int64_t cap_slots);
hipError_t rdf_scratch_setup(int device);
void* rdf_scratch(int device);
int vv_block_size();
void launch_set_step(Ctx* c, int64_t step, hipStream_t st);
void launch_clear_flags(Ctx* c, hipStream_t st);

// md_build.hip
// md_step's fused build: fast-list join, step counter, rebuild when due, slot repack
void launch_build_step(Ctx* c, const double* x, const double* y, const double* z,
                       const uint8_t* type, const int8_t* q, bool force, hipStream_t st);
hipError_t build_step_setup(Ctx* c);
void launch_build(Ctx* c, const double* x, const double* y, const double* z, const uint8_t* type,
                  bool force, hipStream_t st);
void launch_skin_check(Ctx* c, hipStream_t st);

// md_force.hip
void launch_repack(Ctx* c, const double* x, const double* y, const double* z, const int8_t* q,
                   hipStream_t st);
// ev0 / ev1 (optional) are recorded on st immediately before / after the main force
// kernel, so their interval times that kernel alone
// finalize = false leaves the energy reduction and the end of a pending list
// rebuild to the caller (md_step folds them into phase 1 of the integrator).
hipError_t launch_forces(Ctx* c, md_precision prec, const double* x, const double* y,
                         const double* z, const int8_t* q, double* fx, double* fy, double* fz,
                         double* epot, int2* emit, int64_t emit_max, hipStream_t st,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool finalize = true);
struct ForceFinalizeArgs;
ForceFinalizeArgs force_finalize_args(Ctx* c, double* epot);
// dynamic LDS of the FP32 force kernel (hyb_q: bound hybrid charge states, else 0)
size_t force32_lds_bytes(int E_cap, int hyb_q = 0);

// md_fast.hip
void launch_fast(Ctx* c, const double* x, const double* y, const double* z, const int8_t* q,
                 double* fx, double* fy, double* fz, bool energy, int2* emit, int64_t emit_max,
                 hipStream_t st);
hipError_t force_kernel_setup(Ctx* c);

}  // namespace md
