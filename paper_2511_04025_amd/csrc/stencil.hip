// Matrix-free periodic stiffness operator q = K p, K = sum_e E_e P_e^T K_0 P_e
// (Sec. 4.1, Eq. (7)-(8)), for one load case per workgroup.
//
// A workgroup owns a TX x TY tile of nodes in the x-y plane and marches up a
// run of tz planes in z.  Per element layer it
//   1. stages the next node plane (tile + one-node periodic halo) in LDS,
//   2. forms, for each of the (TX+1)(TY+1) element columns, the Hadamard
//      coefficients of the element's 24 nodal values (x-y from the 2x2 node
//      block in LDS, z from the previous plane kept in registers),
//   3. applies E_e K_0 in that basis (hexop.hpp) and transforms back along z
//      (the half for the lower node plane completes it; the upper half is
//      carried to the next layer in registers),
//   4. transforms back along x-y through LDS and writes one output node per
//      thread.
// Every global access is a coalesced x-row; the periodic wrap is an index
// map on the halo only.
//
// Modes
//   PCG   : the node values are p_new = D^-1 r + beta p_old (the CG direction
//           update, fused); owned nodes store p_new into the other p buffer;
//           output q = K p_new and the FP64 partial p_new . q (alpha is formed
//           by the scalar kernel that follows).
//   RESID : FP64 arithmetic on the FP64 solution x: r = -K (x + chi^k), i.e.
//           f - K x with f = -sum_e E_e P_e^T K_0 chi^k added at the element;
//           stored in the vector precision, with FP64 sums of r for the
//           mean projection.  Flag 0 (initial) treats x as zero.
//   APPLY : plain q = K p (component entry point and tests).
#include <type_traits>

#include "common.hpp"
#include "hexop.hpp"
#include "kernels.hpp"

namespace shh {

enum { MODE_PCG = 0, MODE_RESID = 1, MODE_APPLY = 2 };

#ifndef SHH_STENCIL_WAVES_PER_EU
#define SHH_STENCIL_WAVES_PER_EU 1
#endif

template <typename TC, typename TS, int MODE>
__global__ __launch_bounds__(STENCIL_THREADS) __attribute__((amdgpu_waves_per_eu(SHH_STENCIL_WAVES_PER_EU)))
void stencil_kernel(LaunchArgs la) {
  __shared__ TC nbuf[2][3][NHALO];
  __shared__ TC ebuf[2][12][NELEMC];
  __shared__ double red[3 * 16];

  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  CgState *st = s->st;
  const int rhs = w.rhs;
  if (MODE == MODE_PCG && !st->active[rhs]) return;
  if (MODE == MODE_RESID) {
    if (w.flag == RES_RECOMPUTE && !st->active[rhs]) return;
    if (w.flag == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
  }

  const int n = s->n;
  const long long nn = s->nn;
  const long long plane = (long long)n * n;
  const int tile = w.tile;
  const int tix = tile % s->tiles_x;
  const int tiy = (tile / s->tiles_x) % s->tiles_y;
  const int tiz = tile / (s->tiles_x * s->tiles_y);
  const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * s->tz;
  const int z1 = min(z0 + s->tz, n);
  const int tid = threadIdx.x;

  // element-column role
  const bool is_elem = tid < NELEMC;
  const int ecx = tid % EXC, ecy = tid / EXC;
  const long long eoff = (long long)wrapi(y0 - 1 + ecy, n) * n + wrapi(x0 - 1 + ecx, n);
  // output role
  const int ox = tid % TX, oy = tid / TX;
  const bool is_out = tid < TX * TY && x0 + ox < n && y0 + oy < n;
  const long long ooff = (long long)(y0 + oy) * n + (x0 + ox);
  // element columns (ecx, ecy) = (ox + 1, oy + 1) is the one whose 2x2 node
  // block has this output node at its lower corner: the output thread reads
  // its own p from that block's position in the node buffer
  const int own_h = (oy + 1) * HX + ox + 1;
  // halo-load role: up to two halo nodes per thread
  bool hval[2], hown[2];
  long long hoff[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int h = tid + k * STENCIL_THREADS;
    hval[k] = h < NHALO;
    const int hx = h % HX, hy = h / HX;
    hoff[k] = (long long)wrapi(y0 - 1 + hy, n) * n + wrapi(x0 - 1 + hx, n);
    hown[k] = hval[k] && hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && x0 + hx - 1 < n &&
              y0 + hy - 1 < n;
  }

  const TC *__restrict__ kop;
  if constexpr (sizeof(TC) == 8) kop = (const TC *)s->kop64; else kop = (const TC *)s->kop32;
  const TC *__restrict__ E;
  if constexpr (sizeof(TC) == 8) E = (const TC *)s->E64; else E = (const TC *)s->E32;

  const long long vbase = (long long)rhs * 3 * nn;
  const TS *__restrict__ rin = nullptr;
  const TS *__restrict__ pold = nullptr;
  const TS *__restrict__ dinv = nullptr;
  const TS *__restrict__ pin = nullptr;
  const double *__restrict__ xin = nullptr;
  TS *__restrict__ pnew = nullptr;
  TS *__restrict__ qout = nullptr;
  TC beta = TC(0);
  if constexpr (MODE == MODE_PCG) {
    const int pc = st->pcur[rhs];
    rin = (const TS *)s->r + vbase;
    pold = (const TS *)(pc ? s->p1 : s->p0) + vbase;
    pnew = (TS *)(pc ? s->p0 : s->p1) + vbase;
    dinv = (const TS *)s->Dinv;
    qout = (TS *)s->q + vbase;
    beta = (TC)st->beta[rhs];
  } else if constexpr (MODE == MODE_RESID) {
    xin = s->x64 + vbase;
    qout = (TS *)s->r + vbase;
  } else {
    pin = (const TS *)s->p0 + vbase;
    qout = (TS *)s->q + vbase;
  }
  const bool zero_x = (MODE == MODE_RESID) && (w.flag == RES_INIT);
  const bool use_pold = beta != TC(0);

  // ---- plane staging, split into issue (global loads into registers) and
  //      finish (combine, store owned p, store to LDS) so that the loads of a
  //      plane are in flight during the previous plane's element work
  using TL = typename std::conditional<MODE == MODE_RESID, double, TS>::type;
  TL raw_a[2][3], raw_b[2][3];
  TS raw_d[2];
  auto issue = [&](int z) {
    const long long pb = (long long)wrapi(z, n) * plane;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!hval[k]) continue;
      const long long i = pb + hoff[k];
      if constexpr (MODE == MODE_PCG) {
        raw_d[k] = dinv[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          raw_a[k][c] = rin[c * nn + i];
          raw_b[k][c] = use_pold ? pold[c * nn + i] : TS(0);
        }
      } else if constexpr (MODE == MODE_RESID) {
#pragma unroll
        for (int c = 0; c < 3; ++c) raw_a[k][c] = zero_x ? 0.0 : xin[c * nn + i];
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) raw_a[k][c] = pin[c * nn + i];
      }
    }
  };
  auto finish = [&](int z, int b) {
    const long long pb = (long long)wrapi(z, n) * plane;
    const bool ownz = z >= z0 && z < z1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!hval[k]) continue;
      const int hslot = tid + k * STENCIL_THREADS;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        TC v;
        if constexpr (MODE == MODE_PCG) {
          const TC zc = (TC)raw_d[k] * (TC)raw_a[k][c];
          v = beta * (TC)raw_b[k][c] + zc;
          if (hown[k] && ownz) pnew[c * nn + pb + hoff[k]] = (TS)v;
        } else {
          v = (TC)raw_a[k][c];
        }
        nbuf[b][c][hslot] = v;
      }
    }
  };
  // x-y Hadamard coefficients of the 2x2 node block of this element column
  auto xy_hadamard = [&](int b, TC (&A)[3][4]) {
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

  TC A[3][4], Bacc[3][4];
  TC pc_next[3] = {TC(0), TC(0), TC(0)};
  TC pc_cur[3] = {TC(0), TC(0), TC(0)};
  double acc[3] = {0.0, 0.0, 0.0};

  // prologue: planes z0-1 and z0 staged, plane z0+1 in flight
  issue(z0 - 1);
  finish(z0 - 1, 0);
  issue(z0);
  TC e_next = is_elem ? E[(long long)wrapi(z0 - 1, n) * plane + eoff] : TC(0);
  __syncthreads();
  if (is_elem) {
    xy_hadamard(0, A);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 4; ++m) Bacc[c][m] = TC(0);
  }
  finish(z0, 1);
  const int S = z1 - z0 + 1;  // element layers z0-1 .. z1-1
  if (S > 1) issue(z0 + 1);
  __syncthreads();

  for (int sl = 0; sl < S; ++sl) {
    const int kk = z0 - 1 + sl;  // element layer between node planes kk and kk+1
    const int b = sl & 1;
    const TC e = e_next;
    if (is_elem && sl + 1 < S) e_next = E[(long long)wrapi(kk + 1, n) * plane + eoff];
    if constexpr (MODE == MODE_PCG) {
      // this thread's p at the next output plane (node plane kk+1, in nbuf[b ^ 1])
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pc_cur[c] = pc_next[c];
        if (is_out) pc_next[c] = nbuf[b ^ 1][c][own_h];
      }
    }
    if (is_elem) {
      TC An[3][4];
      xy_hadamard(b ^ 1, An);
      TC h[3][8], y[3][8];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          h[c][m] = A[c][m] + An[c][m];
          h[c][m + 4] = An[c][m] - A[c][m];
        }
      if constexpr (MODE == MODE_RESID) add_chi<TC>(rhs, h);
      hex_apply<TC>(kop, h, y, e);
      if (sl > 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int m = 0; m < 4; ++m) ebuf[b][c * 4 + m][tid] = Bacc[c][m] + (y[c][m] - y[c][m + 4]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          Bacc[c][m] = y[c][m] + y[c][m + 4];
          A[c][m] = An[c][m];
        }
    }
    // stage node plane kk+2 (its loads were issued a step ago), issue kk+3
    if (sl + 1 < S) finish(z0 + sl + 1, b);
    if (sl + 2 < S) issue(z0 + sl + 2);
    __syncthreads();
    if (sl > 0 && is_out) {
      // node (x0+ox, y0+oy, kk) gathers the element columns at offsets
      // (ax, ay) in {0,1}^2: column index (ox + 1 - ax, oy + 1 - ay)
      const int e00 = (oy + 1) * EXC + ox + 1, e10 = e00 - 1, e01 = e00 - EXC, e11 = e01 - 1;
      TC qv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const TC *B0 = ebuf[b][c * 4 + 0], *B1 = ebuf[b][c * 4 + 1], *B2 = ebuf[b][c * 4 + 2],
                 *B3 = ebuf[b][c * 4 + 3];
        const TC a00 = (B0[e00] - B1[e00]) - (B2[e00] - B3[e00]);
        const TC a10 = (B0[e10] + B1[e10]) - (B2[e10] + B3[e10]);
        const TC a01 = (B0[e01] - B1[e01]) + (B2[e01] - B3[e01]);
        const TC a11 = (B0[e11] + B1[e11]) + (B2[e11] + B3[e11]);
        qv[c] = (a00 + a10) + (a01 + a11);
      }
      const long long i = (long long)kk * plane + ooff;
      if constexpr (MODE == MODE_PCG) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          qout[c * nn + i] = (TS)qv[c];
          acc[0] += (double)pc_cur[c] * (double)qv[c];
        }
      } else if constexpr (MODE == MODE_RESID) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const TS rv = (TS)(-qv[c]);
          qout[c * nn + i] = rv;
          acc[c] += (double)rv;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) qout[c * nn + i] = (TS)qv[c];
      }
    }
  }

  // workgroup partials only; the scalar kernel that follows reduces them
  if constexpr (MODE == MODE_PCG) {
    double a1[1] = {acc[0]};
    block_sum<1>(a1, red, STENCIL_THREADS);
    double *parts = s->partials + (long long)rhs * s->maxparts * 4;
    if (tid == 0) parts[4 * tile] = a1[0];
  } else if constexpr (MODE == MODE_RESID) {
    block_sum<3>(acc, red, STENCIL_THREADS);
    double *parts = s->partials + (long long)rhs * s->maxparts * 4;
    if (tid == 0) {
      parts[4 * tile + 0] = acc[0];
      parts[4 * tile + 1] = acc[1];
      parts[4 * tile + 2] = acc[2];
    }
  }
}

static int padded_grid(int total) { return ((total + 7) / 8) * 8; }

hipError_t launch_stencil_pcg(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE_PCG><<<g, STENCIL_THREADS, 0, st>>>(la);
  else stencil_kernel<float, float, MODE_PCG><<<g, STENCIL_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_stencil_resid(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE_RESID><<<g, STENCIL_THREADS, 0, st>>>(la);
  else stencil_kernel<double, float, MODE_RESID><<<g, STENCIL_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_stencil_apply(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  const int g = padded_grid(la.total);
  if (prec == 0) stencil_kernel<double, double, MODE_APPLY><<<g, STENCIL_THREADS, 0, st>>>(la);
  else stencil_kernel<float, float, MODE_APPLY><<<g, STENCIL_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

}  // namespace shh
