// Geometric multigrid preconditioner for the periodic voxel elasticity system
// (the solver family of Sec. 4.2, here as a V-cycle inside CG).
//
// Levels: level 0 is the voxel grid (matrix-free operator of the stencil
// kernel); level l + 1 halves every axis of level l while it is even.  Coarse
// operators are Galerkin products A_{l+1} = P^T A_l P with trilinear periodic
// prolongation P.  Because P restricted to one coarse element is the
// trilinear interpolation inside it, the product is element-local: a coarse
// element matrix is the sum over its 8 children f of Q_f^T K_f Q_f (Q_f maps
// the coarse element's 8 corner values to child f's corners), and on level 1
// K_f = E_f K_0, so K_E = sum_f E_f G_f with G_f = Q_f^T K_0 Q_f.  Coarse
// element matrices are assembled into 27-point nodal stencils of 3 x 3 blocks
// for the smoother and residual sweeps.  Smoothing is Chebyshev (degree 2)
// on D^-1 A over [h / 33, h], h an upper bound of lambda_max: on the voxel
// level the element bound lambda_max(diag(K_0)^-1 K_0), on coarse levels
// 1.2 x a power-iteration estimate; the coarsest level (at most 8^3 nodes) is
// solved with a dense inverse of its operator made nonsingular on the three
// rigid translations, assembled and inverted on the device.
#pragma once

#include "common.hpp"

namespace shh {

constexpr int MG_MAXL = 10;          // levels including the voxel grid
constexpr int MG_MAX_COARSE = 8;     // coarsest grid at most 8^3 nodes
// A coarse operator is symmetric, so a node stores the 3 x 3 blocks of the 14
// neighbour offsets w = 13..26 of the 27 (w = 9 (dz + 1) + 3 (dy + 1) + dx + 1;
// 13 is the node itself); the block of offset w < 13 is the transpose of the
// block the neighbour at that offset stores for offset 26 - w.
constexpr int MG_HALF = 14;
constexpr int MG_STENCIL = MG_HALF * 9;  // stored values per node

struct MgLevel {
  int n;
  int nchunks;          // CHUNK-node chunks of the level (vector kernels)
  long long nn;
  // levels >= 1: nodal stencil [14 * 9][nn] (block of offset w >= 13, entry (c, c')
  // at ((w - 13) * 9 + 3 c + c') * nn),
  // inverse diagonal [3][nn]; level 0 uses the slot's matrix-free operator and D^-1 [nn]
  void *S, *Dinv;
  // V-cycle vectors [NRHS][3][nn]: right-hand side, iterate, residual,
  // Chebyshev direction, operator output (on levels >= 1 the fused sweeps
  // keep the next direction and the post-smoothing iterate there).  Level 0 aliases the slot's CG
  // vectors (b = r[0], x = r[1] (z), r = q[1], q = q[0]) except d, which
  // has a buffer of its own (the CG direction alternates between p[0] and p[1]).
  void *b, *x, *r, *d, *q;
  void *Ke;             // setup only: element matrices [nn][24][24] (levels >= 1)
  double inv_theta, c1, c2;  // Chebyshev coefficients
  double lmax;               // lambda_max(D^-1 A) estimate (setup: running max of Rayleigh quotients)
  double pw_scale;           // setup: 1 / ||D^-1 A x|| of the last power step
};

struct MgDev {
  int L;                // index of the coarsest level
  int ndof_c;           // 3 n_L^3
  void *G;              // [8][24][24] child Galerkin matrices of K_0 (T)
  double *Mc;           // [ndof_c][ndof_c] coarsest inverse (FP64), dof 3 node + c
  MgLevel lv[MG_MAXL];
};

// One launch of a V-cycle kernel covers up to MG_MAXB slots (grid z = slot).
constexpr int MG_MAXB = 16;
struct MgBatch {
  const SlotDev *slot[MG_MAXB];
  const MgDev *mg[MG_MAXB];
  int count;
};

// CG scalar phases
enum { MGS_RESTART = 0, MGS_ALPHA = 1, MGS_BETA = 2, MGS_REPLACE = 3 };
// coarse-level operator passes with the Chebyshev sweep that follows them
// fused into their output stage (see mg_epilogue)
enum { MGE_NONE = 0, MGE_STEP1 = 1, MGE_RES = 2, MGE_POST = 3, MGE_LAST = 4 };

// Number of levels for an n^3 grid (coarsening while even and above 4^3, so
// the dense coarsest solve stays at most 8^3 and usually 3^3 or 4^3), or 0
// when the coarsest grid would exceed MG_MAX_COARSE.
inline int mg_num_levels(int n) {
  int L = 1;
  while (n % 2 == 0 && n > 4 && L < MG_MAXL) {
    n /= 2;
    ++L;
  }
  return n <= MG_MAX_COARSE ? L : 0;
}

}  // namespace shh
