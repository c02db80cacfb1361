// Selective (active-set) solve of Sec. 4.2 on compact node lists.
//
// Active voxels are those with beta_e > eps (eps = 1e-3, Sec. 4.2.3); an
// active voxel carries K_e = E beta_e K_0, a culled one nothing.  The unknowns
// live on the active nodes (vertices of at least one active voxel), numbered
// in ascending (z, y, x) order -- the order of their packed 32-bit
// coordinates (z << 20) | (y << 10) | x -- so that consecutive threads touch
// consecutive nodes of one x-run.  A dense int32 map gives the compact index
// of every grid node (-1 when culled); the element whose lower corner is a
// node stores its modulus at that node's index (every active element's lower
// corner is an active node).
//
// The operator is node-centric: row i of K is the 27-point stencil
// sum_r A_i(r) u_{i+r}, whose 3 x 3 blocks are assembled in registers from the
// eight moduli around the node.  With the trilinear element's 1D integrals,
// every entry of A_i(r) is a constant (a function of r, lambda, mu) times a
// signed sum of those moduli: per axis, a fixed element slice where r moves
// along it, and either the sum or the difference of the two slices where it
// does not.  The 64 such sums come from a three-stage transform.
#pragma once

#include "shellhom.h"
#include "common.hpp"

namespace shh {

constexpr double SEL_EPS = 1e-3;   // active set: beta > eps (Sec. 4.2.3)
constexpr int SEL_PS = 8;          // doubles per workgroup partial
constexpr int SEL_THREADS = 256;
constexpr int SEL_CHUNK = 1024;    // grid nodes per workgroup of the compaction scan

// device descriptor of one selective solve
struct SelDev {
  int n;
  int na;                 // active nodes
  int nparts;             // workgroups of the compact kernels
  int prec;               // SHH_PREC_FP64 / SHH_PREC_MIXED
  int nchunks;            // compaction chunks
  int pad_;
  long long nn;           // n^3
  double lam, mu;         // Lame parameters at E = 1
  double rtol, ffloor;
  int max_iter;
  int pad2_;
  // f0[k][a][c]: component c at corner a of K_0 chi^k (E = 1), the element
  // force of unit strain k; a node's load is -sum_a E_a f0[k][a]
  double f0[NRHS][8][3];
  double kop[KOP_N];      // the element operator's constants (E = 1), for the energy sensitivity
  const double *E64;      // dense culled moduli [n^3] (input of the compaction)
  int *map;               // [n^3] compact index or -1
  unsigned *coord;        // [na] packed coordinates, ascending
  int *counts;            // [nchunks + 1] active nodes per chunk, then exclusive offsets; [nchunks] = na
  void *Ec;               // [na] moduli in the working precision
  double *Ec64;           // [na] FP64 moduli (== Ec for the FP64 path)
  void *Dinv;             // [na] inverse Jacobi diagonal (same for the 3 components)
  void *r, *p, *q, *x;    // [6][3][na] working precision
  double *x64;            // [6][3][na] FP64 solution accumulator (mixed); == x for FP64
  double *partials;       // [6][nparts][SEL_PS]
  CgState *st;
  // multigrid preconditioner (mg != 0): the voxel level's V-cycle steps run on
  // the compact lists, the coarse levels on the dense hierarchy built from the
  // culled moduli.  Chebyshev coefficients of the voxel level, the V-cycle's
  // vectors (node-major, working precision) and the first coarse level's
  // right-hand side and iterate ([6][3][n1^3], dense)
  int mg;
  int n1;
  long long nn1;
  double inv_theta, c1, c2;
  void *d0, *d1, *xv, *rv;
  void *b1, *x1;
};

// operator pass flavours
enum { SOP_PCG = 0, SOP_RESID = 1, SOP_ENERGY = 2, SOP_APPLY = 3 };
// scalar phases
enum { SSC_ITER = 0, SSC_MEAN = 1, SSC_RESID_INIT = 2, SSC_RESID_REPLACE = 3, SSC_RESID_FINAL = 4,
       SSC_ENERGY = 5, SSC_MG_ALPHA = 6, SSC_MG_BETA = 7, SSC_MG_RESTART = 8, SSC_MG_REPLACE = 9 };
// voxel-level passes of the multigrid-preconditioned solve (input vector -> epilogue)
enum { SMO_PQ = 0, SMO_STEP1 = 1, SMO_RES = 2, SMO_POST = 3, SMO_LAST = 4,
       SMO_POST1 = 5 };  // POST1: degree-1 post-smoothing, z = x + D (b - K x) / theta

// One launch covers up to SEL_MAXB slots (grid y = slot) of one precision.
constexpr int SEL_MAXB = 16;
struct SelBatch {
  SelDev *d[SEL_MAXB];    // device descriptors
  int count;
  int prec;
  int parts_max;          // largest nparts of the batch
  int chunks_max;         // largest nchunks
  long long nn1_max;      // largest first-coarse-level node count (multigrid)
};

hipError_t sel_launch_compact(const SelBatch &B, hipStream_t st);   // map, coord, counts (na)
hipError_t sel_launch_gather(const SelBatch &B, hipStream_t st);    // Ec, Ec64, Dinv
hipError_t sel_launch_op(const SelBatch &B, int mode, hipStream_t st);
hipError_t sel_launch_scalar(const SelBatch &B, int phase, hipStream_t st);
hipError_t sel_launch_update(const SelBatch &B, hipStream_t st);     // x, r, p after alpha, beta
hipError_t sel_launch_dir0(const SelBatch &B, hipStream_t st);       // p = D^-1 r
hipError_t sel_launch_fold(const SelBatch &B, int all, hipStream_t st);  // x64 += x32, x32 = 0
hipError_t sel_launch_finish(const SelBatch &B, int rmode, hipStream_t st);  // r -= mean; rho, rr partials
hipError_t sel_launch_zero(const SelBatch &B, hipStream_t st);       // x, x64, p = 0
// multigrid: operator pass with a V-cycle epilogue; the CG update fused with
// the first Chebyshev direction (restart: no update); the CG direction;
// restriction to and prolongation from the first coarse level
hipError_t sel_launch_mg_op(const SelBatch &B, int mode, hipStream_t st);
hipError_t sel_launch_mg_s1(const SelBatch &B, int restart, hipStream_t st);
hipError_t sel_launch_mg_dir(const SelBatch &B, hipStream_t st);
hipError_t sel_launch_mg_restrict(const SelBatch &B, hipStream_t st);
hipError_t sel_launch_mg_prolong(const SelBatch &B, hipStream_t st);
// dL/dE_e over the dense voxel grid (zero on culled voxels) from the solution
// of one solved design and the folded weights g21 of dL/dC^H
hipError_t sel_launch_energy_sens(const SelBatch &B, long long nn, const double *d_g21, double *d_gE, hipStream_t st);

}  // namespace shh
