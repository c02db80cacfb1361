// Host-side launchers of the HIP kernels (implemented in the .hip files).
#pragma once

#include "common.hpp"

namespace shh {

enum { RES_INIT = 0, RES_RECOMPUTE = 1, RES_FINAL = 2 };
enum { PH_ITER = 0, PH_MEAN = 2, PH_RESID = 3 };

// field.hip (single slot per launch; d_slot is the device copy of the slot)
hipError_t launch_field(SlotDev *d_slot, int n, int nb, hipStream_t st);
int reduce_blocks(long long nn);
hipError_t launch_select_hard(SlotDev *d_slot, long long nn, long long k, hipStream_t st);
hipError_t launch_minmax_d(SlotDev *d_slot, long long nn, hipStream_t st);
hipError_t launch_bisect_steps(SlotDev *d_slot, long long nn, int steps, hipStream_t st);
hipError_t launch_occupancy(SlotDev *d_slot, long long nn, double *beta_out, hipStream_t st);
// e_dtype 0: 1-byte solid/void code (E = Es where nonzero, else Ev); 1: float; 2: double
hipError_t launch_moduli_copy(SlotDev *d_slot, long long nn, const void *E, int e_dtype, double Es, double Ev,
                              hipStream_t st);
hipError_t launch_dinv(SlotDev *d_slot, long long nn, int prec, hipStream_t st);

// stencil.hip (segments of (slot, load case, tile)); the PCG launch is one
// whole CG iteration of every listed load case
hipError_t launch_stencil_pcg(const LaunchArgs &la, int prec, hipStream_t st);
hipError_t launch_stencil_resid(const LaunchArgs &la, int prec, hipStream_t st);
hipError_t launch_stencil_apply(const LaunchArgs &la, int prec, hipStream_t st);
// multigrid voxel-level passes (op: SMG_DIR, SMG_STEP1, SMG_POST, SMG_LAST, SMG_RES, SMG_POST1)
hipError_t launch_stencil_mg(const LaunchArgs &la, int prec, int op, hipStream_t st);

// cg.hip (segments of (slot, load case, chunk); fold/zero use one case per slot)
hipError_t launch_finish_resid(const LaunchArgs &la, int prec, hipStream_t st);
hipError_t launch_scalar(const LaunchArgs &la, int phase, hipStream_t st);
hipError_t launch_fold(const LaunchArgs &la, int prec, hipStream_t st);
hipError_t launch_zero_vectors(const LaunchArgs &la, int prec, hipStream_t st);

// energy.hip
hipError_t launch_energy(SlotDev *d_slot, long long nn, hipStream_t st);
hipError_t launch_energy_sens(SlotDev *d_slot, long long nn, const double *d_G36, double *d_out,
                              hipStream_t st);
// device scratch (bytes) the adjoint needs for an n^3 grid at truncation order K
size_t adjoint_scratch_bytes(int n, int K);
// d_out [N][4] (dL/dx, dL/dy, dL/dz, dL/dq); d_alpha_out [(K+1)^3] and d_t_out
// [1] (either may be null) receive dL/dalpha and dL/dt
hipError_t launch_adjoint(SlotDev *d_slot, int n, int nb, int N, int K, const double *d_gE, double gV,
                          double *d_scratch, double *d_out, double *d_alpha_out, double *d_t_out,
                          hipStream_t st);

// the field's trig coefficient tensor alone; dL/d(charges, alpha) from dL/dcoef
hipError_t launch_coef(SlotDev *d_slot, int nb, hipStream_t st);
hipError_t launch_coef_adjoint(SlotDev *d_slot, int N, int K, const double *d_dcoef, double *d_out,
                               double *d_alpha_out, hipStream_t st);
// the field and its gradient at arbitrary points, and dL/dcoef from dL/dF there
hipError_t launch_points_field(SlotDev *d_slot, int nb, int npts, const double *d_pts, double *d_F,
                               double *d_G, hipStream_t st);
hipError_t launch_points_dcoef(int nb, int npts, const double *d_pts, const double *d_gF, double *d_basis,
                               double *d_dcoef, hipStream_t st);

// device address of the current device's shh_homogenize_noalloc scratch
int noalloc_scratch(void **out);

}  // namespace shh
