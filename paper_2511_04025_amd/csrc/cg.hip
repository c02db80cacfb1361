// CG vector kernels of the six-load-case Jacobi-PCG: streaming, one load
// case and one CHUNK of nodes (3 components) per workgroup, FP64 dot products
// written as per-workgroup partials; a scalar kernel per phase reduces them in
// a fixed order and updates the load case's scalars on the device.
#include "common.hpp"
#include "kernels.hpp"

namespace shh {

// x += alpha p; r -= alpha q; rho' = r . D^-1 r, ||r||^2; then beta, convergence.
// Each thread owns NPT nodes (stride VEC_THREADS); all loads are issued before
// any store so that a wave keeps NPT * 13 loads in flight.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void update_kernel(LaunchArgs la) {
  __shared__ double red[2 * 16];
  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  CgState *st = s->st;
  const int rhs = w.rhs;
  if (!st->active[rhs]) return;
  const long long nn = s->nn;
  const long long i0 = (long long)w.tile * CHUNK;
  const T a = (T)st->alpha[rhs];
  const long long vb = (long long)rhs * 3 * nn;
  T *__restrict__ x = (T *)s->x + vb;
  T *__restrict__ r = (T *)s->r + vb;
  const T *__restrict__ q = (const T *)s->q + vb;
  const T *__restrict__ p = (const T *)(st->pcur[rhs] ? s->p1 : s->p0) + vb;
  const T *__restrict__ dinv = (const T *)s->Dinv;
  constexpr int NPT = CHUNK / VEC_THREADS;
  T dv[NPT], pv[NPT][3], xv[NPT][3], rv[NPT][3], qv[NPT][3];
  bool ok[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const long long i = i0 + threadIdx.x + (long long)k * VEC_THREADS;
    ok[k] = i < nn;
    const long long ii = ok[k] ? i : 0;
    dv[k] = dinv[ii];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv[k][c] = p[c * nn + ii];
      xv[k][c] = x[c * nn + ii];
      rv[k][c] = r[c * nn + ii];
      qv[k][c] = q[c * nn + ii];
    }
  }
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if (!ok[k]) continue;
    const long long i = i0 + threadIdx.x + (long long)k * VEC_THREADS;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c * nn + i] = xv[k][c] + a * pv[k][c];
      const T rn = rv[k][c] - a * qv[k][c];
      r[c * nn + i] = rn;
      const T zv = dv[k] * rn;
      acc[0] += (double)rn * (double)zv;
      acc[1] += (double)rn * (double)rn;
    }
  }
  block_sum<2>(acc, red, VEC_THREADS);
  double *parts = s->partials + (long long)rhs * s->maxparts * 4;
  if (threadIdx.x == 0) {
    parts[4 * w.tile + 0] = acc[0];
    parts[4 * w.tile + 1] = acc[1];
  }
}

// After the FP64 residual stencil: r -= mean (per component), rho = r . D^-1 r,
// ||r||^2, and the scalar update for the initial / periodic / final residual.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void finish_resid_kernel(LaunchArgs la) {
  __shared__ double red[2 * 16];
  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  CgState *st = s->st;
  const int rhs = w.rhs;
  const int mode = w.flag;
  if (mode == RES_RECOMPUTE && !st->active[rhs]) return;
  if (mode == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
  const long long nn = s->nn;
  const long long i0 = (long long)w.tile * CHUNK;
  const long long vb = (long long)rhs * 3 * nn;
  T *__restrict__ r = (T *)s->r + vb;
  const T *__restrict__ dinv = (const T *)s->Dinv;
  const double m0 = st->mean[rhs][0], m1 = st->mean[rhs][1], m2 = st->mean[rhs][2];
  constexpr int NPT = CHUNK / VEC_THREADS;
  T dv[NPT], rv[NPT][3];
  bool ok[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const long long i = i0 + threadIdx.x + (long long)k * VEC_THREADS;
    ok[k] = i < nn;
    const long long ii = ok[k] ? i : 0;
    dv[k] = dinv[ii];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[k][c] = r[c * nn + ii];
  }
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if (!ok[k]) continue;
    const long long i = i0 + threadIdx.x + (long long)k * VEC_THREADS;
    const double d = (double)dv[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double mc = c == 0 ? m0 : (c == 1 ? m1 : m2);
      const T rn = (T)((double)rv[k][c] - mc);
      r[c * nn + i] = rn;
      acc[0] += (double)rn * d * (double)rn;
      acc[1] += (double)rn * (double)rn;
    }
  }
  block_sum<2>(acc, red, VEC_THREADS);
  double *parts = s->partials + (long long)rhs * s->maxparts * 4;
  if (threadIdx.x == 0) {
    parts[4 * w.tile + 0] = acc[0];
    parts[4 * w.tile + 1] = acc[1];
  }
}

// ---- scalar phase: one workgroup per (design, load case) --------------------
// Reduces the partials of the kernel just before it in a fixed order and
// updates the load case's CG scalars.  Kernel boundaries order it with the
// producers, so no fences or atomics are needed and the result is
// deterministic.  Skip rules repeat the producers' so both see the same set.
__global__ __launch_bounds__(VEC_THREADS) void scalar_kernel(LaunchArgs la, int phase) {
  __shared__ double red[3 * 16];
  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  CgState *st = s->st;
  const int rhs = w.rhs;
  const int mode = w.flag;
  const double *parts = s->partials + (long long)rhs * s->maxparts * 4;
  if (phase == PH_ALPHA) {  // after the PCG stencil: alpha = rho / (p . K p)
    if (!st->active[rhs]) return;
    double tot[1];
    sum_partials<1>(parts, s->ntiles, tot, red, VEC_THREADS);
    if (threadIdx.x == 0) {
      const double sigma = tot[0];
      if (!(sigma > 0.0) || !isfinite(sigma)) {
        st->status[rhs] = ST_BREAKDOWN;
        st->active[rhs] = 0;
      } else {
        st->alpha[rhs] = st->rho[rhs] / sigma;
      }
      st->pcur[rhs] ^= 1;
    }
  } else if (phase == PH_BETA) {  // after the update: beta, convergence
    if (!st->active[rhs]) return;
    double tot[2];
    sum_partials<2>(parts, s->nchunks, tot, red, VEC_THREADS);
    if (threadIdx.x == 0) {
      const double rho = tot[0], rr = tot[1];
      st->iters[rhs] += 1;
      st->rho_prev[rhs] = st->rho[rhs];
      st->beta[rhs] = rho / st->rho[rhs];
      st->rho[rhs] = rho;
      st->rr[rhs] = rr;
      const double rel = sqrt(rr / st->ff[rhs]);
      st->rel[rhs] = rel;
      if (!isfinite(rho) || rho < 0.0) {
        st->status[rhs] = ST_BREAKDOWN;
        st->active[rhs] = 0;
      } else if (rel <= s->rtol) {
        st->status[rhs] = ST_CONVERGED;
        st->active[rhs] = 0;
      } else if (st->iters[rhs] >= s->max_iter) {
        st->status[rhs] = ST_MAXIT;
        st->active[rhs] = 0;
      }
    }
  } else if (phase == PH_MEAN) {  // after the residual stencil: component means
    if (mode == RES_RECOMPUTE && !st->active[rhs]) return;
    if (mode == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
    double tot[3];
    sum_partials<3>(parts, s->ntiles, tot, red, VEC_THREADS);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) st->mean[rhs][c] = tot[c] / double(s->nn);
    }
  } else {  // PH_RESID, after finish_resid: initial / replaced / final residual
    if (mode == RES_RECOMPUTE && !st->active[rhs]) return;
    if (mode == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
    double tot[2];
    sum_partials<2>(parts, s->nchunks, tot, red, VEC_THREADS);
    if (threadIdx.x != 0) return;
    const double rho = tot[0], rr = tot[1];
    if (mode == RES_INIT) {
      st->ff[rhs] = rr;
      st->rho[rhs] = rho;
      st->rho_prev[rhs] = rho;
      st->beta[rhs] = 0.0;
      st->alpha[rhs] = 0.0;
      st->iters[rhs] = 0;
      st->pcur[rhs] = 0;
      st->rr[rhs] = rr;
      if (sqrt(rr) <= s->ffloor) {  // zero load: u = 0 solves it
        st->active[rhs] = 0;
        st->status[rhs] = ST_CONVERGED;
        st->rel[rhs] = 0.0;
        st->rel_true[rhs] = 0.0;
      } else {
        st->active[rhs] = s->max_iter > 0 ? 1 : 0;
        st->status[rhs] = s->max_iter > 0 ? ST_RUNNING : ST_MAXIT;
        st->rel[rhs] = 1.0;
        st->rel_true[rhs] = 1.0;
      }
    } else {
      // residual replacement: keep p, restart the rho recurrence from the true residual
      st->rho[rhs] = rho;
      st->beta[rhs] = rho / st->rho_prev[rhs];
      st->rr[rhs] = rr;
      const double rel = sqrt(rr / st->ff[rhs]);
      st->rel[rhs] = rel;
      st->rel_true[rhs] = rel;
      if (st->status[rhs] == ST_BREAKDOWN) {
        st->active[rhs] = 0;
      } else if (!isfinite(rel)) {
        st->status[rhs] = ST_BREAKDOWN;
        st->active[rhs] = 0;
      } else if (rel <= s->rtol) {
        st->status[rhs] = ST_CONVERGED;
        st->active[rhs] = 0;
      } else if (st->iters[rhs] >= s->max_iter) {
        st->status[rhs] = ST_MAXIT;
        st->active[rhs] = 0;
      } else {
        st->status[rhs] = ST_RUNNING;
        st->active[rhs] = 1;
      }
    }
  }
}

// Mixed precision: x64 += x32, x32 = 0 for all six load cases of a chunk.
__global__ __launch_bounds__(VEC_THREADS) void fold_kernel(LaunchArgs la) {
  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  const long long nn = s->nn;
  const long long i0 = (long long)w.tile * CHUNK;
  const long long i1 = min(i0 + CHUNK, nn);
  float *x32 = (float *)s->x;
  double *x64 = s->x64;
  for (int f = 0; f < 3 * NRHS; ++f) {
    for (long long i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
      const long long j = f * nn + i;
      x64[j] += (double)x32[j];
      x32[j] = 0.0f;
    }
  }
}

// Zero x, both p buffers, q (and x64) of every load case before a solve.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void zero_kernel(LaunchArgs la) {
  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  const long long nn = s->nn;
  const long long i0 = (long long)w.tile * CHUNK;
  const long long i1 = min(i0 + CHUNK, nn);
  T *x = (T *)s->x, *p0 = (T *)s->p0, *p1 = (T *)s->p1, *q = (T *)s->q;
  for (int f = 0; f < 3 * NRHS; ++f) {
    for (long long i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
      const long long j = f * nn + i;
      x[j] = T(0);
      p0[j] = T(0);
      p1[j] = T(0);
      q[j] = T(0);
      if (s->prec == 1) s->x64[j] = 0.0;
    }
  }
}

static int padded_grid(int total) { return ((total + 7) / 8) * 8; }

hipError_t launch_update(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  if (prec == 0) update_kernel<double><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  else update_kernel<float><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_finish_resid(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  if (prec == 0) finish_resid_kernel<double><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  else finish_resid_kernel<float><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_scalar(const LaunchArgs &la, int phase, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  scalar_kernel<<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la, phase);
  return hipGetLastError();
}

hipError_t launch_fold(const LaunchArgs &la, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  fold_kernel<<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_zero_vectors(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  if (prec == 0) zero_kernel<double><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  else zero_kernel<float><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

}  // namespace shh
