// The 8-node hexahedral element stiffness of a fully solid unit voxel
// (K_0 of Eq. (7)) applied in the per-axis Walsh-Hadamard basis.
//
// For trilinear shape functions the 1D factors of K_0 are the mass matrix
// M = [[1/3, 1/6], [1/6, 1/3]], the stiffness S = [[1, -1], [-1, 1]] and the
// mixed G_ab = int phi_a' phi_b.  In the basis h_s = (1, 1), h_d = (-1, 1) of
// each axis these become M -> diag(1, 1/3), S -> diag(0, 4), and G has the
// single entry (d, s) = 2.  The isotropic element matrix
//   K^{ij} = lambda int d_i N d_j N + mu int d_j N d_i N + mu delta_ij int grad N . grad N
// is therefore diagonal within each displacement component plus, for each
// pair of components (i, j), four couplings per mode of the third axis: 45
// nonzeros instead of 576.  With Hhat the 8x8 (unnormalized) transform per
// component, K_0 = Hhat^T Khat Hhat / 64; the 1/64 is folded into the constants.
// By the symmetry of the cube under axis permutations the 21 nonzero diagonal
// entries take 5 distinct values, so the operator needs 10 constants.
//
// Mode index m = s_x | s_y << 1 | s_z << 2 with s = 0 (sum) or 1 (difference).
#pragma once

#include "common.hpp"

namespace shh {

//
// The all-sum mode m = 0 of each component is a rigid translation: its
// diagonal entry is zero (every term carries S along some axis) and no
// coupling touches it, so h[c][0] is never read and y[c][0] is exactly zero.
template <typename T, typename KP>
__host__ __device__ __forceinline__ void hex_apply(KP kop, const T (&h)[3][8], T (&y)[3][8], T e) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    y[c][0] = T(0);
#pragma unroll
    for (int m = 1; m < 8; ++m) {
      const int sc = (m >> c) & 1;
      const int so = ((m >> ((c + 1) % 3)) & 1) + ((m >> ((c + 2) % 3)) & 1);
      y[c][m] = kop[sc * 3 + so] * h[c][m];
    }
  }
  // couplings of components (i, j) with third axis k:
  //   y_i(i=d, j=s) += 4 lam M_k h_j(i=s, j=d)   y_i(i=s, j=d) += 4 mu M_k h_j(i=d, j=s)
  //   y_j(i=s, j=d) += 4 lam M_k h_i(i=d, j=s)   y_j(i=d, j=s) += 4 mu M_k h_i(i=s, j=d)
#define SHH_COUPLE(I, J, KK)                                                   \
  _Pragma("unroll") for (int mk = 0; mk < 2; ++mk) {                           \
    const T cl = kop[6 + mk], cm = kop[8 + mk];                                \
    const int a = (1 << (I)) | (mk << (KK));                                   \
    const int b = (1 << (J)) | (mk << (KK));                                   \
    y[I][a] += cl * h[J][b];                                                   \
    y[I][b] += cm * h[J][a];                                                   \
    y[J][b] += cl * h[I][a];                                                   \
    y[J][a] += cm * h[I][b];                                                   \
  }
  SHH_COUPLE(0, 1, 2)
  SHH_COUPLE(0, 2, 1)
  SHH_COUPLE(1, 2, 0)
#undef SHH_COUPLE
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 1; m < 8; ++m) y[c][m] *= e;
}

// Hadamard coefficients of the unit-strain test displacement chi^k
// (corner a displaced by eps^k a): 4 eps^k_{cd} on the mode with a single
// difference along axis d (the all-sum mode is a rigid translation and is
// annihilated by K_0, so it is left out).
template <typename T>
__device__ __forceinline__ void add_chi(int k, T (&h)[3][8]) {
  switch (k) {
    case 0: h[0][1] += T(4); break;                       // eps_11 = 1
    case 1: h[1][2] += T(4); break;                       // eps_22 = 1
    case 2: h[2][4] += T(4); break;                       // eps_33 = 1
    case 3: h[1][4] += T(2); h[2][2] += T(2); break;      // eps_23 = eps_32 = 1/2
    case 4: h[0][4] += T(2); h[2][1] += T(2); break;      // eps_13 = eps_31 = 1/2
    default: h[0][2] += T(2); h[1][1] += T(2); break;     // eps_12 = eps_21 = 1/2
  }
}

// 8-point Hadamard transform of corner values v[a], a = ax | ay << 1 | az << 2:
// out[m] = sum_a prod_axis (s ? 1 : 2 a_axis - 1) v[a]
template <typename T>
__device__ __forceinline__ void hadamard8(const T (&v)[8], T (&out)[8]) {
  T t[8];
#pragma unroll
  for (int yz = 0; yz < 4; ++yz) {  // x
    t[2 * yz] = v[2 * yz] + v[2 * yz + 1];
    t[2 * yz + 1] = v[2 * yz + 1] - v[2 * yz];
  }
  T u[8];
#pragma unroll
  for (int z = 0; z < 2; ++z)  // y
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      u[4 * z + x] = t[4 * z + x] + t[4 * z + 2 + x];
      u[4 * z + 2 + x] = t[4 * z + 2 + x] - t[4 * z + x];
    }
#pragma unroll
  for (int xy = 0; xy < 4; ++xy) {  // z
    out[xy] = u[xy] + u[4 + xy];
    out[4 + xy] = u[4 + xy] - u[xy];
  }
}

}  // namespace shh
