// Matrix-free periodic stiffness operator q = K p, K = sum_e E_e P_e^T K_0 P_e
// (Sec. 4.1, Eq. (7)-(8)), for one load case per workgroup.
//
// A workgroup owns a TX x TY tile of nodes in the x-y plane (64 x 6 for FP32
// compute, 32 x 8 for FP64) and marches up a run of tz planes in z.  Per
// element layer it
//   1. stages the next node plane (tile + one-node periodic halo) in LDS,
//   2. forms, for each of the (TX+1)(TY+1) element columns, the Hadamard
//      coefficients of the element's 24 nodal values (x-y from the 2x2 node
//      block in LDS, z from the previous plane kept in registers),
//   3. applies E_e K_0 in that basis (hexop.hpp) and transforms back along z
//      (the half for the lower node plane completes it; the upper half is
//      carried to the next layer in registers),
//   4. transforms the lower node plane's share back to the four x-y corners,
//      exchanges them through LDS and sums four per output node.
// Thread t < TX*TY both stages and outputs interior node (t % TX, t / TX) of
// the tile; the ring of halo nodes around the tile is staged by the remaining
// threads (and, past those, by a second slot of the first threads).  Every
// global access is a coalesced x-row of one buffer resource; the periodic
// wrap is an index map on the halo only.
//
// Modes
//   PCG   : one whole Jacobi-PCG iteration of the load case per pass.  Pass j
//           reads r_{j-1}, q_{j-1}, p_{j-1} (set pcur) and, at every staged
//           node, forms
//             r_j = r_{j-1} - alpha q_{j-1},  z_j = D^-1 r_j,
//             p_j = z_j + beta p_{j-1}
//           with the alpha, beta left by the scalar kernel after pass j-1.
//           At owned nodes it writes r_j, p_j (other set) and
//           x_j = x_{j-1} + alpha p_{j-1}, and sums r_j . z_j and r_j . r_j;
//           at the outputs it writes q_j = K p_j (other set) and sums
//           p_j . q_j, q_j . z_j and q_j . D^-1 q_j (all sums FP64).
//           The scalar kernel turns these into alpha_j and, by expanding
//           (r_j - alpha_j q_j) . D^-1 (r_j - alpha_j q_j), the next rho and
//           beta: standard PCG whose x, r update is carried into the next
//           pass instead of a pass of its own.  Both p buffers and both q
//           buffers are zeroed when a solve starts and stay finite, so
//           alpha = beta = 0 needs no special case.
//   RESID : FP64 arithmetic on the FP64 solution x: r = -K (x + chi^k), i.e.
//           f - K x with f = -sum_e E_e P_e^T K_0 chi^k added at the element;
//           stored in the vector precision into the current r, with FP64
//           sums of r for the mean projection.  Flag 0 (initial) treats x as
//           zero.
//   APPLY : plain q = K p (component entry point and tests).
#include <type_traits>

#include "common.hpp"
#include "hexop.hpp"
#include "kernels.hpp"

namespace shh {

enum { MODE_PCG = 0, MODE_RESID = 1, MODE_APPLY = 2, MODE_MGDIR = 3, MODE_MGSTEP1 = 4, MODE_MGPOST = 5,
       MODE_MGLAST = 6, MODE_MGRES = 7, MODE_MGPOST1 = 8 };

#ifndef SHH_STENCIL_WAVES_PER_EU
#define SHH_STENCIL_WAVES_PER_EU 1
#endif
#ifndef SHH_CARRY_DB
#define SHH_CARRY_DB 0
#endif

// Halo-tile index of ring node j: the bottom row, the top row, then the left
// and right columns between them.
template <int HX, int HY>
__device__ __forceinline__ int ring_h(int j) {
  if (j < HX) return j;
  if (j < 2 * HX) return (HY - 1) * HX + (j - HX);
  if (j < 2 * HX + (HY - 2)) return (1 + j - 2 * HX) * HX;
  return (2 + j - 2 * HX - (HY - 2)) * HX - 1;
}

template <typename TC, typename TS, int MODE>
__global__ __launch_bounds__(Tile<TC>::THREADS) __attribute__((amdgpu_waves_per_eu(SHH_STENCIL_WAVES_PER_EU)))
void stencil_kernel(LaunchArgs la) {
  // tile geometry of this compute precision
  using TT = Tile<TC>;
  constexpr int TX = TT::X, TY = TT::Y, HX = TT::HX, HY = TT::HY, EXC = TT::EXC, EYC = TT::EYC;
  constexpr int NHALO = TT::NHALO, NELEMC = TT::NELEMC, STENCIL_THREADS = TT::THREADS;
  constexpr int NINT = TT::NINT, NRING = TT::NRING;
  constexpr int TW = tiling_of<TC>();
  __shared__ TC nbuf[2][3][NHALO];
  __shared__ TC ebuf[2][12][NELEMC];
  __shared__ TC mbuf[2][NHALO];  // element moduli, by the halo slot of the element's lower corner
  __shared__ double red[5 * 16];

  Work w;
  if (!decode_work(la, w)) return;
  const SHH_CONST SlotDev *s = to_const(w.slot);
  const SHH_CONST CgState *st = to_const(s->st);
  const int rhs = w.rhs;
  // load cases whose CG has stopped are skipped (Sec. 4.2.2: per-right-hand-
  // side convergence); the multigrid passes likewise
  if ((MODE == MODE_PCG || MODE >= MODE_MGDIR) && !st->active[rhs]) return;
  if (MODE == MODE_RESID) {
    if (w.flag == RES_RECOMPUTE && !st->active[rhs]) return;
    if (w.flag == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
  }

  // n <= 512: every byte offset into one load case's [3][n^3] vector fits in
  // 32 bits.  Per-lane offsets are fixed per thread; plane and component
  // offsets are wave-uniform scalars.
  const int n = s->n;
  const uint32_t plane = (uint32_t)n * (uint32_t)n;
  const long long nn = s->nn;
  const int tile = w.tile;
  const int tix = tile % s->tiles_x[TW];
  const int tiy = (tile / s->tiles_x[TW]) % s->tiles_y[TW];
  const int tiz = tile / (s->tiles_x[TW] * s->tiles_y[TW]);
  const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * s->tz;
  const int z1 = min(z0 + s->tz, n);
  const int tid = threadIdx.x;

  using TL = typename std::conditional<MODE == MODE_RESID, double, TS>::type;
  constexpr uint32_t SL = sizeof(TL), SS = sizeof(TS), SC = sizeof(TC);

  // element-column role
  const bool is_elem = tid < NELEMC;
  const int ecx = tid % EXC, ecy = tid / EXC;
  // output role (also the owner of the node in the PCG update)
  const int ox = tid % TX, oy = tid / TX;
  const bool is_out = tid < NINT && x0 + ox < n && y0 + oy < n;
  const uint32_t ooff = ((uint32_t)(y0 + oy) * n + (uint32_t)(x0 + ox)) * SS;
  // staging role: slot 0 of thread t < NINT is its own interior node; ring
  // nodes fill the remaining slot-0 threads and then slot 1 of the first ones
  // The element moduli of a layer are staged with a node plane: element
  // column (ecx, ecy) is the voxel whose lower corner is halo node (ecx, ecy),
  // so the thread staging that node loads the voxel's E_e at the same offset
  // (hel).  Keeping every global load in the staging batch means the element
  // work never waits on the memory counter, which retires in issue order.
  bool hval[2], hel[2];
  int hslot[2];
  uint32_t hoS[2], hoL[2], hoC[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    int h;
    if (k == 0 && tid < NINT) {
      h = (oy + 1) * HX + ox + 1;
      hval[k] = true;
    } else {
      const int j = k == 0 ? tid - NINT : tid + STENCIL_THREADS - NINT;
      hval[k] = j < NRING;
      h = hval[k] ? ring_h<HX, HY>(j) : 0;
    }
    hslot[k] = h;
    const int hx = h % HX, hy = h / HX;
    const uint32_t o = (uint32_t)wrapi(y0 - 1 + hy, n) * n + (uint32_t)wrapi(x0 - 1 + hx, n);
    hoS[k] = o * SS;
    hoL[k] = o * SL;
    hoC[k] = o * SC;
    hel[k] = hval[k] && hx < EXC && hy < EYC;
  }

  const SHH_CONST TC *kop;
  if constexpr (sizeof(TC) == 8) kop = (const SHH_CONST TC *)s->kop64;
  else kop = (const SHH_CONST TC *)s->kop32;
  // one resource for the moduli and, in the CG pass, D^-1 behind them (the two
  // arrays are adjacent in the slot, D^-1 at byte offset dOff)
  const char *Ebase;
  if constexpr (sizeof(TC) == 8) Ebase = (const char *)s->E64;
  else Ebase = (const char *)s->E32;
  constexpr bool MGF = MODE >= MODE_MGSTEP1;  // a Chebyshev sweep fused behind the operator
  // operand staged as D^-1 v / theta (v = b or r: the direction is not stored)
  constexpr bool MG_SCALED = MODE == MODE_MGSTEP1 || MODE == MODE_MGLAST;
  constexpr bool MG_NEED_D = MG_SCALED || MODE == MODE_MGPOST1;  // D^-1 at the owned nodes
  constexpr bool WITH_D = MODE == MODE_PCG || MG_NEED_D;
  const uint32_t dOff = WITH_D ? (uint32_t)((const char *)s->Dinv - Ebase) : 0u;
  const rsrc_t rE = make_rsrc(Ebase, WITH_D ? (uint64_t)dOff + (uint64_t)nn * SS : (uint64_t)nn * SC);

  // component c of a load case's vector starts c * n^3 elements in
  const uint32_t cS[3] = {0u, (uint32_t)nn * SS, 2u * (uint32_t)nn * SS};
  const uint32_t cL[3] = {0u, (uint32_t)nn * SL, 2u * (uint32_t)nn * SL};
  const long long vbase = (long long)rhs * 3 * nn;
  const uint64_t vbytesS = 3ull * nn * SS, vbytesL = 3ull * nn * SL;
  // PCG: rA = r_{j-1}, rB = q_{j-1}, rC = p_{j-1}; rR, rQ, rP the new set; rX
  // RESID: rA = FP64 x, rQ = current r.  APPLY: rA = p, rQ = q (or the pair the flag names).
  // MGDIR (the multigrid CG's direction pass): rA = z, rC = p_{j-1}, rP = p_j, rQ = q.
  // Fused voxel-level Chebyshev sweeps (q = K v is consumed, not stored); rA
  // the vector staged over the halo, rAux the owned-node inputs, rR, rP, rX
  // the outputs:
  //   STEP1: b (r[0]) staged as d0 = D b / theta;  r = b - q,
  //          d1 = c1 d0 + c2 D r, x = d0 + d1 -> r (q[1]), d1 (mgd), x (r[1])
  //          (degree 1: r and x = d0 only)
  //   POST:  x (r[1]) staged as is; aux b;  r = b - q -> q[1]
  //   RES:   d1 (mgd) staged as is; aux r (q[1]);  r - q -> q[1] (the
  //          residual the restriction takes)
  //   LAST:  r (q[1]) staged as d = D r / theta; aux b, x;
  //          x + (1 + c1) d + c2 D (r - q) -> r[1], partials b . x, b . b
  //          (the post-smoother's x + d folded into the last update)
  //   POST1 (degree-1 smoothing): x (r[1]) staged as is; aux b;
  //          z = x + D (b - q) / theta -> mgd, partials b . z, b . b
  constexpr int NAUX = MODE == MODE_MGLAST ? 2 : 1;
  constexpr int NLOAD = MODE == MODE_MGSTEP1 ? 0 : NAUX;  // auxiliary vectors read
  rsrc_t rA, rB, rC, rR, rQ, rP, rX, rAux[NAUX];
  TC alpha = TC(0), beta = TC(0);
  TC ith = TC(0), c1 = TC(0), c2 = TC(0);
  if constexpr (MGF) {
    ith = (TC)s->mgc[0];
    c1 = (TC)s->mgc[1];
    c2 = (TC)s->mgc[2];
    if constexpr (MODE == MODE_MGSTEP1) {
      rA = make_rsrc((const TS *)s->r[0] + vbase, vbytesS);
      rR = make_rsrc((const TS *)s->q[1] + vbase, vbytesS);
      rP = make_rsrc((const TS *)s->mgd + vbase, vbytesS);
      rX = make_rsrc((const TS *)s->r[1] + vbase, vbytesS);
    } else if constexpr (MODE == MODE_MGPOST || MODE == MODE_MGRES) {
      rA = make_rsrc((const TS *)(MODE == MODE_MGPOST ? s->r[1] : s->mgd) + vbase, vbytesS);
      rAux[0] = make_rsrc((const TS *)(MODE == MODE_MGPOST ? s->r[0] : s->q[1]) + vbase, vbytesS);
      rR = make_rsrc((const TS *)s->q[1] + vbase, vbytesS);
    } else if constexpr (MODE == MODE_MGPOST1) {
      rA = make_rsrc((const TS *)s->r[1] + vbase, vbytesS);
      rAux[0] = make_rsrc((const TS *)s->r[0] + vbase, vbytesS);
      rX = make_rsrc((const TS *)s->mgd + vbase, vbytesS);
    } else {
      rA = make_rsrc((const TS *)s->q[1] + vbase, vbytesS);
      rAux[0] = make_rsrc((const TS *)s->r[0] + vbase, vbytesS);
      rAux[NAUX - 1] = make_rsrc((const TS *)s->r[1] + vbase, vbytesS);
      rX = make_rsrc((const TS *)s->r[1] + vbase, vbytesS);
    }
  } else if constexpr (MODE == MODE_MGDIR) {
    const int pc = st->mgpar[rhs];
    // z: the last post-smoothing pass leaves it in r[1] (degree 2) or mgd
    rA = make_rsrc((const TS *)(SHH_MG_DEG0 == 1 ? s->mgd : s->r[1]) + vbase, vbytesS);
    rC = make_rsrc((const TS *)s->p[pc] + vbase, vbytesS);
    rP = make_rsrc((const TS *)s->p[pc ^ 1] + vbase, vbytesS);
    rQ = make_rsrc((const TS *)s->q[0] + vbase, vbytesS);
    beta = (TC)st->beta[rhs];
  } else if constexpr (MODE == MODE_PCG) {
    const int pc = st->pcur[rhs];
    rA = make_rsrc((const TS *)s->r[pc] + vbase, vbytesS);
    rB = make_rsrc((const TS *)s->q[pc] + vbase, vbytesS);
    rC = make_rsrc((const TS *)s->p[pc] + vbase, vbytesS);
    rR = make_rsrc((const TS *)s->r[pc ^ 1] + vbase, vbytesS);
    rQ = make_rsrc((const TS *)s->q[pc ^ 1] + vbase, vbytesS);
    rP = make_rsrc((const TS *)s->p[pc ^ 1] + vbase, vbytesS);
    rX = make_rsrc((const TS *)s->x + vbase, vbytesS);
    alpha = (TC)st->alpha[rhs];
    beta = (TC)st->beta[rhs];
  } else if constexpr (MODE == MODE_RESID) {
    rA = make_rsrc(s->x64 + vbase, vbytesL);
    rQ = make_rsrc((const TS *)s->r[st->pcur[rhs]] + vbase, vbytesS);
  } else {
    // flag 0: p[0] -> q[0]; otherwise 1 + src + 8 dst over (r0, r1, p0, p1, q0, q1, x, mgd)
    const void *src = s->p[0];
    void *dst = s->q[0];
    if (w.flag > 0) {
      auto pick = [&](int i) -> void * {
        switch (i) {
          case 0: return s->r[0];
          case 1: return s->r[1];
          case 2: return s->p[0];
          case 3: return s->p[1];
          case 4: return s->q[0];
          case 5: return s->q[1];
          case 6: return s->x;
          default: return s->mgd;
        }
      };
      src = pick((w.flag - 1) & 7);
      dst = pick(((w.flag - 1) >> 3) & 7);
    }
    rA = make_rsrc((const TS *)src + vbase, vbytesL);
    rQ = make_rsrc((const TS *)dst + vbase, vbytesS);
  }
  const bool zero_x = (MODE == MODE_RESID) && (w.flag == RES_INIT);

  // FP64 partial sums: PCG r.z, r.r, p.q, q.z, q.D^-1 q; RESID sums of r
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // owned-node values kept from staging to output (two steps later), by
  // parity of the step that staged them: z, D^-1 and p of the node
  TC own_z[2][3], own_p[2][3], own_d[2];
  // fused sweeps: the owned node's auxiliary inputs, by the same parity
  TC own_aux[2][NAUX][3];

  // ---- plane staging, split into issue (loads into registers), finish
  //      (combine, store to LDS) and commit (store owned values) so that the
  //      loads of a plane are in flight during the previous plane's element
  //      work.
  //      Node planes z0-1 .. z1 are touched, so a single wrap suffices.
  TL raw_a[2][3];
  TS raw_b[2][3], raw_c[2][3], raw_d[2], raw_x[3], raw_aux[NAUX][3];
  TC raw_e[2];
  // node plane z, and the element layer z - 1 below it
  auto issue = [&](int z) {
    const uint32_t pz = (uint32_t)wrap1(z, n) * plane;
    const uint32_t pe = (uint32_t)wrap1(z - 1, n) * plane;
    const bool ownz = z >= z0 && z < z1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!hval[k]) continue;
      if (hel[k]) raw_e[k] = bload<TC>(rE, hoC[k], pe * SC);
      if constexpr (MODE == MODE_PCG) {
        raw_d[k] = bload<TS>(rE, hoS[k], dOff + pz * SS);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          raw_a[k][c] = bload<TS>(rA, hoS[k], pz * SS + cS[c]);
          raw_b[k][c] = bload<TS>(rB, hoS[k], pz * SS + cS[c]);
          raw_c[k][c] = bload<TS>(rC, hoS[k], pz * SS + cS[c]);
        }
        if (k == 0 && is_out && ownz) {
#pragma unroll
          for (int c = 0; c < 3; ++c) raw_x[c] = bload<TS>(rX, hoS[0], pz * SS + cS[c]);
        }
      } else if constexpr (MODE == MODE_RESID) {
#pragma unroll
        for (int c = 0; c < 3; ++c) raw_a[k][c] = zero_x ? 0.0 : bload<TL>(rA, hoL[k], pz * SL + cL[c]);
      } else if constexpr (MGF) {
        if constexpr (MG_NEED_D) raw_d[k] = bload<TS>(rE, hoS[k], dOff + pz * SS);
#pragma unroll
        for (int c = 0; c < 3; ++c) raw_a[k][c] = bload<TS>(rA, hoS[k], pz * SS + cS[c]);
        if (k == 0 && is_out && ownz) {
#pragma unroll
          for (int a = 0; a < NLOAD; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) raw_aux[a][c] = bload<TS>(rAux[a], hoS[0], pz * SS + cS[c]);
        }
      } else if constexpr (MODE == MODE_MGDIR) {
        // beta = 0 starts a new direction: the old one is not read
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          raw_a[k][c] = bload<TS>(rA, hoS[k], pz * SS + cS[c]);
          raw_c[k][c] = beta != TC(0) ? bload<TS>(rC, hoS[k], pz * SS + cS[c]) : TS(0);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) raw_a[k][c] = bload<TL>(rA, hoL[k], pz * SL + cL[c]);
      }
    }
  };
  // the owned node's new r, p, x, written by commit() after the next plane's
  // loads are issued (so that waiting for those loads never waits for these
  // stores: the memory counter retires in issue order)
  TS out_r[3], out_p[3], out_x[3];
  auto commit = [&](int z) {
    if constexpr (MODE == MODE_PCG) {
      const uint32_t pz = (uint32_t)wrap1(z, n) * plane;
      const bool ownz = z >= z0 && z < z1;
      if (is_out && ownz) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const uint32_t so = pz * SS + cS[c];
          bstore<TS>(out_r[c], rR, hoS[0], so);
          bstore<TS>(out_p[c], rP, hoS[0], so);
          bstore<TS>(out_x[c], rX, hoS[0], so);
        }
      }
    } else if constexpr (MODE == MODE_MGDIR) {
      const uint32_t pz = (uint32_t)wrap1(z, n) * plane;
      const bool ownz = z >= z0 && z < z1;
      if (is_out && ownz) {
#pragma unroll
        for (int c = 0; c < 3; ++c) bstore<TS>(out_p[c], rP, hoS[0], pz * SS + cS[c]);
      }
    }
  };
  auto finish = [&](int z, auto bc) {
    constexpr int b = decltype(bc)::value;
    const uint32_t pz = (uint32_t)wrap1(z, n) * plane;
    const bool ownz = z >= z0 && z < z1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!hval[k]) continue;
      if (hel[k]) mbuf[b][hslot[k]] = raw_e[k];
      if constexpr (MODE == MODE_PCG) {
        const TC dk = (TC)raw_d[k];
        TC rn[3], zn[3], pn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          rn[c] = (TC)raw_a[k][c] - alpha * (TC)raw_b[k][c];
          zn[c] = dk * rn[c];
          pn[c] = beta * (TC)raw_c[k][c] + zn[c];
          nbuf[b][c][hslot[k]] = pn[c];
        }
        if (k == 0 && is_out && ownz) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            out_r[c] = (TS)rn[c];
            out_p[c] = (TS)pn[c];
            out_x[c] = (TS)((TC)raw_x[c] + alpha * (TC)raw_c[0][c]);
            const double r64 = (double)rn[c];
            acc[0] += r64 * (double)zn[c];
            acc[1] += r64 * r64;
            own_z[b][c] = zn[c];
            own_p[b][c] = pn[c];
          }
          own_d[b] = dk;
        }
      } else if constexpr (MGF) {
        TC v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          v[c] = (TC)raw_a[k][c];
          if constexpr (MG_SCALED) v[c] = (TC)raw_d[k] * v[c] * ith;
          nbuf[b][c][hslot[k]] = v[c];
        }
        if (k == 0 && is_out && ownz) {
          // own_p: the staged value, own_z: the vector it came from
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            own_p[b][c] = v[c];
            own_z[b][c] = (TC)raw_a[0][c];
          }
          if constexpr (MG_NEED_D) own_d[b] = (TC)raw_d[0];
#pragma unroll
          for (int a = 0; a < NLOAD; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) own_aux[b][a][c] = (TC)raw_aux[a][c];
        }
      } else if constexpr (MODE == MODE_MGDIR) {
        TC pn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pn[c] = (TC)raw_a[k][c] + beta * (TC)raw_c[k][c];
          nbuf[b][c][hslot[k]] = pn[c];
        }
        if (k == 0 && is_out && ownz) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            out_p[c] = (TS)pn[c];
            own_p[b][c] = pn[c];
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) nbuf[b][c][hslot[k]] = (TC)raw_a[k][c];
      }
    }
  };
  // x-y Hadamard coefficients of the 2x2 node block of this element column
  auto xy_hadamard = [&](auto bc, TC (&A)[3][4]) {
    constexpr int b = decltype(bc)::value;
    const int i00 = ecy * HX + ecx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const TC p00 = nbuf[b][c][i00], p10 = nbuf[b][c][i00 + 1];
      const TC p01 = nbuf[b][c][i00 + HX], p11 = nbuf[b][c][i00 + HX + 1];
      const TC sx0 = p00 + p10, dx0 = p10 - p00, sx1 = p01 + p11, dx1 = p11 - p01;
      A[c][0] = sx0 + sx1;
      A[c][1] = dx0 + dx1;
      A[c][2] = sx1 - sx0;
      A[c][3] = dx1 - dx0;
    }
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;

  // Values carried from one element layer to the next: the x-y Hadamard
  // coefficients of the lower node plane (A) and the upper-plane half of the
  // layer below (Bc).  With SHH_CARRY_DB (FP32 only) they
  // are double-buffered by layer parity (index b of the step that reads them),
  // which spares the register copies of the two-step unrolled loop at the
  // cost of 24 more registers.
  constexpr int NB = (SHH_CARRY_DB && sizeof(TC) == 4) ? 2 : 1;
  TC A[NB][3][4], Bc[NB][3][4];

  // prologue: planes z0-1 and z0 staged, plane z0+1 in flight
  issue(z0 - 1);
  finish(z0 - 1, B0{});
  issue(z0);
  commit(z0 - 1);
  __syncthreads();
  if (is_elem) {
    xy_hadamard(B0{}, A[0]);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 4; ++m) Bc[0][c][m] = TC(0);
  }
  finish(z0, B1{});
  const int S = z1 - z0 + 1;  // element layers z0-1 .. z1-1
  if (S > 1) issue(z0 + 1);
  commit(z0);
  __syncthreads();

  // one element layer: kk = z0 - 1 + sl lies between node planes kk and kk+1;
  // the layer's node planes sit in nbuf[b] and nbuf[b ^ 1] with b = sl & 1
  auto step = [&](const int sl, auto bc) {
    constexpr int b = decltype(bc)::value;
    constexpr int bn = b ^ 1;
    using BN = std::integral_constant<int, bn>;
    const int kk = z0 - 1 + sl;
    // the owned values of output plane kk (staged two steps ago, same parity)
    // before this step's staging replaces them
    TC oz[3], op[3], od = TC(0), oa[NAUX][3];
    if constexpr (MODE == MODE_PCG) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        oz[c] = own_z[b][c];
        op[c] = own_p[b][c];
      }
      od = own_d[b];
    } else if constexpr (MODE == MODE_MGDIR) {
#pragma unroll
      for (int c = 0; c < 3; ++c) op[c] = own_p[b][c];
    } else if constexpr (MGF) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        op[c] = own_p[b][c];
        oz[c] = own_z[b][c];
      }
      if constexpr (MG_NEED_D) od = own_d[b];
#pragma unroll
      for (int a = 0; a < NLOAD; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) oa[a][c] = own_aux[b][a][c];
    }
    if (is_elem) {
      constexpr int ib = NB == 2 ? b : 0, ibn = NB == 2 ? bn : 0;
      const TC (&Ac)[3][4] = A[ib];
      TC An[3][4];
      xy_hadamard(BN{}, An);
      // layer kk's modulus was staged with node plane kk+1
      const TC e = mbuf[bn][ecy * HX + ecx];
      TC h[3][8], y[3][8];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h[c][0] = TC(0);  // rigid mode: not read by hex_apply
#pragma unroll
        for (int m = 1; m < 4; ++m) h[c][m] = Ac[c][m] + An[c][m];
#pragma unroll
        for (int m = 0; m < 4; ++m) h[c][m + 4] = An[c][m] - Ac[c][m];
      }
      if constexpr (MODE == MODE_RESID) add_chi<TC>(rhs, h);
      hex_apply<TC>(kop, h, y, e);
      if (sl > 0) {
        // lower node plane kk: this layer's lower half completes the upper
        // half carried from the layer below; store its four x-y corners
        const TC (&Bacc)[3][4] = Bc[ib];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const TC L0 = Bacc[c][0] - y[c][4];  // y[c][0] == 0
          const TC L1 = Bacc[c][1] + (y[c][1] - y[c][5]);
          const TC L2 = Bacc[c][2] + (y[c][2] - y[c][6]);
          const TC L3 = Bacc[c][3] + (y[c][3] - y[c][7]);
          const TC u0 = L0 - L1, u1 = L0 + L1, v0 = L2 - L3, v1 = L2 + L3;
          ebuf[b][c * 4 + 0][tid] = u0 - v0;
          ebuf[b][c * 4 + 1][tid] = u1 - v1;
          ebuf[b][c * 4 + 2][tid] = u0 + v0;
          ebuf[b][c * 4 + 3][tid] = u1 + v1;
        }
      }
      TC (&Bnew)[3][4] = Bc[ibn];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Bnew[c][0] = y[c][4];
#pragma unroll
        for (int m = 1; m < 4; ++m) Bnew[c][m] = y[c][m] + y[c][m + 4];
#pragma unroll
        for (int m = 0; m < 4; ++m) A[ibn][c][m] = An[c][m];
      }
    }
    // stage node plane kk+2 (its loads were issued a step ago), issue kk+3
    if (sl + 1 < S) finish(z0 + sl + 1, bc);
    if (sl + 2 < S) issue(z0 + sl + 2);
    if (sl + 1 < S) commit(z0 + sl + 1);
    __syncthreads();
    if (sl > 0 && is_out) {
      // node (x0+ox, y0+oy, kk) is corner (ax, ay) of element column
      // (ox + 1 - ax, oy + 1 - ay)
      const int e00 = (oy + 1) * EXC + ox + 1;
      TC qv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        qv[c] = (ebuf[b][c * 4 + 0][e00] + ebuf[b][c * 4 + 1][e00 - 1]) +
                (ebuf[b][c * 4 + 2][e00 - EXC] + ebuf[b][c * 4 + 3][e00 - EXC - 1]);
      const uint32_t pk = (uint32_t)kk * plane * SS;
      if constexpr (MODE == MODE_PCG) {
        const double d64 = (double)od;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          bstore<TS>((TS)qv[c], rQ, ooff, pk + cS[c]);
          const double q64 = (double)qv[c];
          acc[2] += (double)op[c] * q64;
          acc[3] += (double)oz[c] * q64;
          acc[4] += d64 * q64 * q64;
        }
      } else if constexpr (MODE == MODE_MGDIR) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          bstore<TS>((TS)qv[c], rQ, ooff, pk + cS[c]);
          acc[0] += (double)op[c] * (double)qv[c];
        }
      } else if constexpr (MODE == MODE_MGSTEP1) {
        // op = d0, oz = b
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const TC rv = oz[c] - qv[c];
          bstore<TS>((TS)rv, rR, ooff, pk + cS[c]);
          if constexpr (SHH_MG_DEG0 == 1) {
            bstore<TS>((TS)op[c], rX, ooff, pk + cS[c]);  // one step: x = d0
          } else {
            const TC d1 = c1 * op[c] + c2 * od * rv;
            bstore<TS>((TS)d1, rP, ooff, pk + cS[c]);
            bstore<TS>((TS)(op[c] + d1), rX, ooff, pk + cS[c]);
          }
        }
      } else if constexpr (MODE == MODE_MGPOST || MODE == MODE_MGRES) {
        // oa[0] = b (POST) or r (RES)
#pragma unroll
        for (int c = 0; c < 3; ++c) bstore<TS>((TS)(oa[0][c] - qv[c]), rR, ooff, pk + cS[c]);
      } else if constexpr (MODE == MODE_MGPOST1) {
        // op = x, oa = b
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const TC zv = op[c] + od * (oa[0][c] - qv[c]) * ith;
          bstore<TS>((TS)zv, rX, ooff, pk + cS[c]);
          const double b64 = (double)oa[0][c];
          acc[0] += b64 * (double)zv;
          acc[1] += b64 * b64;
        }
      } else if constexpr (MODE == MODE_MGLAST) {
        // op = d, oz = r, oa = b, x
        const TC c1p = TC(1) + c1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const TC xv = oa[1][c] + c1p * op[c] + c2 * od * (oz[c] - qv[c]);
          bstore<TS>((TS)xv, rX, ooff, pk + cS[c]);
          const double b64 = (double)oa[0][c];
          acc[0] += b64 * (double)xv;
          acc[1] += b64 * b64;
        }
      } else if constexpr (MODE == MODE_RESID) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const TS rv = (TS)(-qv[c]);
          bstore<TS>(rv, rQ, ooff, pk + cS[c]);
          acc[c] += (double)rv;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) bstore<TS>((TS)qv[c], rQ, ooff, pk + cS[c]);
      }
    }
  };
  int sl = 0;
  for (; sl + 1 < S; sl += 2) {
    step(sl, B0{});
    step(sl + 1, B1{});
  }
  if (sl < S) step(sl, B0{});

  // workgroup partials only; the scalar kernel that follows reduces them
  double *parts = w.slot->partials + ((long long)rhs * s->maxparts + tile) * PSTRIDE;
  if constexpr (MODE == MODE_PCG) {
    block_sum<5>(acc, red, STENCIL_THREADS);
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < 5; ++i) parts[i] = acc[i];
    }
  } else if constexpr (MODE == MODE_MGLAST || MODE == MODE_MGPOST1) {
    double a2[2] = {acc[0], acc[1]};
    block_sum<2>(a2, red, STENCIL_THREADS);
    if (tid == 0) {
      parts[0] = a2[0];
      parts[1] = a2[1];
    }
  } else if constexpr (MODE == MODE_MGDIR) {
    double a1[1] = {acc[0]};
    block_sum<1>(a1, red, STENCIL_THREADS);
    if (tid == 0) parts[0] = a1[0];
  } else if constexpr (MODE == MODE_RESID) {
    double a3[3] = {acc[0], acc[1], acc[2]};
    block_sum<3>(a3, red, STENCIL_THREADS);
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) parts[i] = a3[i];
    }
  }
}

static int padded_grid(int total) { return ((total + 7) / 8) * 8; }

hipError_t launch_stencil_pcg(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE_PCG><<<g, Tile<double>::THREADS, 0, st>>>(la);
  else stencil_kernel<float, float, MODE_PCG><<<g, Tile<float>::THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_stencil_resid(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE_RESID><<<g, Tile<double>::THREADS, 0, st>>>(la);
  else stencil_kernel<double, float, MODE_RESID><<<g, Tile<double>::THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_stencil_apply(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE_APPLY><<<g, Tile<double>::THREADS, 0, st>>>(la);
  else stencil_kernel<float, float, MODE_APPLY><<<g, Tile<float>::THREADS, 0, st>>>(la);
  return hipGetLastError();
}

template <int MODE>
static void launch_mg_mode(const LaunchArgs &la, int prec, hipStream_t st) {
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE><<<g, Tile<double>::THREADS, 0, st>>>(la);
  else stencil_kernel<float, float, MODE><<<g, Tile<float>::THREADS, 0, st>>>(la);
}

// Voxel-level passes of the multigrid-preconditioned CG, in the vector
// precision: SMG_DIR the CG direction p_j = z + beta p_{j-1} (into the other
// p buffer), q = K p_j and per-tile partials p_j . q; SMG_STEP1 / SMG_POST /
// SMG_LAST / SMG_RES / SMG_POST1 the operator with the Chebyshev sweep that
// consumes its output (LAST and POST1: per-tile partials b . z, b . b).
hipError_t launch_stencil_mg(const LaunchArgs &la, int prec, int op, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  switch (op) {
    case SMG_DIR: launch_mg_mode<MODE_MGDIR>(la, prec, st); break;
    case SMG_STEP1: launch_mg_mode<MODE_MGSTEP1>(la, prec, st); break;
    case SMG_POST: launch_mg_mode<MODE_MGPOST>(la, prec, st); break;
    case SMG_LAST: launch_mg_mode<MODE_MGLAST>(la, prec, st); break;
    case SMG_RES: launch_mg_mode<MODE_MGRES>(la, prec, st); break;
    case SMG_POST1: launch_mg_mode<MODE_MGPOST1>(la, prec, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace shh
