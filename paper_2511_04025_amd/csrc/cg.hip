// CG vector and scalar kernels of the six-load-case Jacobi-PCG (the CG pass
// itself is the PCG mode of the stencil kernel).  Streaming kernels take one
// load case and one CHUNK of nodes (3 components) per workgroup and write FP64
// per-workgroup partials; a scalar kernel per phase reduces them in a fixed
// order and updates the load case's scalars on the device.
#include "common.hpp"
#include "kernels.hpp"

namespace shh {

// After the FP64 residual stencil: r -= mean (per component), rho = r . D^-1 r,
// ||r||^2, for the initial / periodic / final residual.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void finish_resid_kernel(LaunchArgs la) {
  __shared__ double red[2 * 16];
  Work w;
  if (!decode_work(la, w)) return;
  const SHH_CONST SlotDev *s = to_const(w.slot);
  const SHH_CONST CgState *st = to_const(s->st);
  const int rhs = w.rhs;
  const int mode = w.flag;
  if (mode == RES_RECOMPUTE && !st->active[rhs]) return;
  if (mode == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
  const long long nn = s->nn;
  constexpr uint32_t SZ = sizeof(T);
  const uint32_t i0 = (uint32_t)w.tile * CHUNK;
  const uint32_t base = i0 * SZ;
  const uint32_t cS[3] = {0u, (uint32_t)nn * SZ, 2u * (uint32_t)nn * SZ};
  const long long vb = (long long)rhs * 3 * nn;
  const rsrc_t rR = make_rsrc((const T *)s->r[st->pcur[rhs]] + vb, 3ull * nn * SZ);
  const rsrc_t rD = make_rsrc(s->Dinv, (uint64_t)nn * SZ);
  const double mean[3] = {st->mean[rhs][0], st->mean[rhs][1], st->mean[rhs][2]};
  constexpr int NPT = CHUNK / VEC_THREADS;
  T dv[NPT], rv[NPT][3];
  bool ok[NPT];
  uint32_t vo[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const uint32_t l = threadIdx.x + k * VEC_THREADS;
    ok[k] = (long long)(i0 + l) < nn;
    vo[k] = ok[k] ? l * SZ : 0u;  // the chunk's first node stands in past the end
    dv[k] = bload<T>(rD, vo[k], base);
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[k][c] = bload<T>(rR, vo[k], base + cS[c]);
  }
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if (!ok[k]) continue;
    const double d = (double)dv[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T rn = (T)((double)rv[k][c] - mean[c]);
      bstore<T>(rn, rR, vo[k], base + cS[c]);
      acc[0] += (double)rn * d * (double)rn;
      acc[1] += (double)rn * (double)rn;
    }
  }
  block_sum<2>(acc, red, VEC_THREADS);
  double *parts = w.slot->partials + ((long long)rhs * s->maxparts + w.tile) * PSTRIDE;
  if (threadIdx.x == 0) {
    parts[0] = acc[0];
    parts[1] = acc[1];
  }
}

// ---- scalar phase: one workgroup per (design, load case) --------------------
// Reduces the partials of the kernel just before it in a fixed order and
// updates the load case's CG scalars.  Kernel boundaries order it with the
// producers, so no fences or atomics are needed and the result is
// deterministic.  Skip rules repeat the producers' so both see the same set.
__global__ __launch_bounds__(VEC_THREADS) void scalar_kernel(LaunchArgs la, int phase) {
  __shared__ double red[5 * 16];
  Work w;
  if (!decode_work(la, w)) return;
  SlotDev *s = w.slot;
  CgState *st = s->st;
  const int rhs = w.rhs;
  const int mode = w.flag;
  const double *parts = s->partials + (long long)rhs * s->maxparts * PSTRIDE;
  if (phase == PH_ITER) {
    // after CG pass j: the pass's sums r.z, r.r, p.q, q.z, q.D^-1 q
    if (!st->active[rhs]) return;
    double tot[5];
    sum_partials<5, PSTRIDE>(parts, s->ntiles[s->prec], tot, red, VEC_THREADS);
    if (threadIdx.x != 0) return;
    const double rho = tot[0], rr = tot[1], sigma = tot[2], tau = tot[3], mu = tot[4];
    st->iters[rhs] += 1;
    st->pcur[rhs] ^= 1;  // the pass wrote r_j, p_j, q_j into the other set
    st->rho[rhs] = rho;
    st->rr[rhs] = rr;
    const double rel = sqrt(rr / st->ff[rhs]);
    st->rel[rhs] = rel;
    const bool ok = isfinite(rho) && rho >= 0.0 && isfinite(sigma) && sigma > 0.0;
    // alpha_j = rho_j / p_j.K p_j, still to be applied to x and r
    const double a = ok ? rho / sigma : 0.0;
    st->alpha[rhs] = a;
    if (ok) {
      // rho_{j+1} = (r_j - a q_j) . D^-1 (r_j - a q_j), expanded with this
      // pass's sums (rounding can only push a vanishing value below zero)
      const double rho_next = fmax(rho - 2.0 * a * tau + a * a * mu, 0.0);
      st->beta[rhs] = rho > 0.0 ? rho_next / rho : 0.0;
    }
    if (rel <= s->rtol) {
      st->status[rhs] = ST_CONVERGED;
      st->active[rhs] = 0;
    } else if (!ok || !isfinite(rel)) {
      st->status[rhs] = ST_BREAKDOWN;
      st->active[rhs] = 0;
      st->alpha[rhs] = 0.0;
    } else if (st->iters[rhs] >= s->max_iter) {
      st->status[rhs] = ST_MAXIT;
      st->active[rhs] = 0;
    }
  } else if (phase == PH_MEAN) {  // after the residual stencil: component means
    if (mode == RES_RECOMPUTE && !st->active[rhs]) return;
    if (mode == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
    double tot[3];
    sum_partials<3, PSTRIDE>(parts, s->ntiles[0], tot, red, VEC_THREADS);  // FP64 residual tiles
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) st->mean[rhs][c] = tot[c] / double(s->nn);
    }
  } else {  // PH_RESID, after finish_resid: initial / replaced / final residual
    if (mode == RES_RECOMPUTE && !st->active[rhs]) return;
    if (mode == RES_FINAL && !(st->ff[rhs] > s->ffloor * s->ffloor)) return;
    double tot[2];
    sum_partials<2, PSTRIDE>(parts, s->nchunks, tot, red, VEC_THREADS);
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
      st->mgpar[rhs] = 0;
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
      // residual replacement: the fold has applied the pending update to x;
      // keep p and restart the recurrences from the true residual
      st->rho_prev[rhs] = st->rho[rhs];
      st->beta[rhs] = st->rho[rhs] > 0.0 ? rho / st->rho[rhs] : 0.0;
      st->alpha[rhs] = 0.0;
      st->rho[rhs] = rho;
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

// Before a residual replacement (flag RES_RECOMPUTE) or the final check
// (RES_FINAL): apply each selected load case's pending update x += alpha p
// (selection as in the residual kernels that follow, whose scalar phase then
// clears alpha), and in mixed precision move the FP32 x into the FP64
// accumulator: x64 += x32 (+ alpha p), x32 = 0.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void fold_kernel(LaunchArgs la) {
  Work w;
  if (!decode_work(la, w)) return;
  const SHH_CONST SlotDev *s = to_const(w.slot);
  const SHH_CONST CgState *st = to_const(s->st);
  const int mode = w.flag;
  const long long nn = s->nn;
  const long long i0 = (long long)w.tile * CHUNK;
  const long long i1 = min(i0 + CHUNK, nn);
  for (int k = 0; k < NRHS; ++k) {
    const bool sel = mode == RES_RECOMPUTE ? st->active[k] != 0 : st->ff[k] > s->ffloor * s->ffloor;
    const double a = sel ? st->alpha[k] : 0.0;
    const T *p = (const T *)s->p[st->pcur[k]] + (long long)k * 3 * nn;
    T *x = (T *)s->x + (long long)k * 3 * nn;
    double *x64 = s->x64 + (long long)k * 3 * nn;
    for (int c = 0; c < 3; ++c) {
      for (long long i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
        const long long j = c * nn + i;
        if constexpr (sizeof(T) == 4) {
          x64[j] += (double)x[j] + a * (double)p[j];
          x[j] = T(0);
        } else {
          x[j] += a * p[j];  // FP64: x is the accumulator
        }
      }
    }
  }
}

// Zero x, both p and both q buffers (and x64) of every load case before a solve.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void zero_kernel(LaunchArgs la) {
  Work w;
  if (!decode_work(la, w)) return;
  const SHH_CONST SlotDev *s = to_const(w.slot);
  const long long nn = s->nn;
  const long long i0 = (long long)w.tile * CHUNK;
  const long long i1 = min(i0 + CHUNK, nn);
  T *x = (T *)s->x, *p0 = (T *)s->p[0], *p1 = (T *)s->p[1], *q0 = (T *)s->q[0], *q1 = (T *)s->q[1];
  double *x64 = s->x64;
  const bool mixed = s->prec == 1;
  for (int f = 0; f < 3 * NRHS; ++f) {
    for (long long i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
      const long long j = f * nn + i;
      x[j] = T(0);
      p0[j] = T(0);
      p1[j] = T(0);
      q0[j] = T(0);
      q1[j] = T(0);
      if (mixed) x64[j] = 0.0;
    }
  }
}

static int padded_grid(int total) { return ((total + 7) / 8) * 8; }

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

hipError_t launch_fold(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  if (prec == 0) fold_kernel<double><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  else fold_kernel<float><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

hipError_t launch_zero_vectors(const LaunchArgs &la, int prec, hipStream_t st) {
  if (la.total == 0) return hipSuccess;
  if (prec == 0) zero_kernel<double><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  else zero_kernel<float><<<padded_grid(la.total), VEC_THREADS, 0, st>>>(la);
  return hipGetLastError();
}

}  // namespace shh
