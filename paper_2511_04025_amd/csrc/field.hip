// Steps 1-2 of the path: the periodic charge field of Eq. (6) on the voxel
// centers, the distance and occupancy of Eq. (7), the thickness rule, the
// element moduli E_e and the Jacobi diagonal.
//
// Field evaluation is the exact regrouping of Eq. (6): expanding
//   cos 2 pi h (x - x_j) = cos 2 pi h x cos 2 pi h x_j + sin 2 pi h x sin 2 pi h x_j
// in all three axes turns the charge sum into a tensor of (2K+1)^3 real
// coefficients over the 1D basis {1, cos 2 pi h s, sin 2 pi h s}, which a
// workgroup contracts with the basis values of one z plane (a (2K+1)^2 plane
// tensor in LDS) and then with its x and y basis values.  FP64 throughout, so
// the hard threshold decides voxel for voxel like the FP64 oracle.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace shh {

// basis index u: 0 -> 1; 2h-1 -> cos(2 pi h s); 2h -> sin(2 pi h s)
__device__ __forceinline__ int basis_h(int u) { return (u + 1) >> 1; }

// ---- trig coefficient tensor of the field -----------------------------------
__global__ void coef_kernel(SlotDev *s) {
  const int K = s->K, nb = s->nb, N = s->N, K1 = K + 1;
  const int total = nb * nb * nb;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int u = e / (nb * nb), v = (e / nb) % nb, w = e % nb;
    const int h = basis_h(u), k = basis_h(v), l = basis_h(w);
    double out = 0.0;
    if (h + k + l > 0) {
      const int zeros = (h == 0) + (k == 0) + (l == 0);
      const double wgt = zeros == 0 ? 1.0 : (zeros == 1 ? 0.5 : 0.25);
      const double a = s->alpha ? s->alpha[(h * K1 + k) * K1 + l] : 1.0;
      const double c = a * wgt / double(h * h + k * k + l * l);
      double acc = 0.0;
      for (int j = 0; j < N; ++j) {
        const double *ch = s->charges + 4 * j;
        double tx = 1.0, ty = 1.0, tz = 1.0, sn, cs;
        if (u > 0) { sincospi(2.0 * h * ch[0], &sn, &cs); tx = (u & 1) ? cs : sn; }
        if (v > 0) { sincospi(2.0 * k * ch[1], &sn, &cs); ty = (v & 1) ? cs : sn; }
        if (w > 0) { sincospi(2.0 * l * ch[2], &sn, &cs); tz = (w & 1) ? cs : sn; }
        acc += ch[3] * tx * ty * tz;
      }
      out = c * acc;
    }
    s->coef[e] = out;
  }
}

// basis value and derivative at voxel center (i + 1/2)/n
__device__ __forceinline__ void basis_at(int u, int i, int n, double &val, double &der) {
  if (u == 0) { val = 1.0; der = 0.0; return; }
  const int h = basis_h(u);
  double sn, cs;
  sincospi(double(h) * double(2 * i + 1) / double(n), &sn, &cs);
  const double w = 2.0 * M_PI * h;
  if (u & 1) { val = cs; der = -w * sn; } else { val = sn; der = w * cs; }
}

// ---- field + gradient on one z plane; 64 x 4 voxels per workgroup ------------
__global__ __launch_bounds__(256) void field_kernel(SlotDev *s) {
  __shared__ double P[MAXB * MAXB], Pz[MAXB * MAXB];
  __shared__ double Xv[64][MAXB], Xd[64][MAXB], Yv[4][MAXB], Yd[4][MAXB];
  __shared__ double red[16];
  const int n = s->n, nb = s->nb;
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 4, z = blockIdx.z;
  const int tid = threadIdx.x;
  // plane tensors P[u][v] = sum_w coef[u][v][w] Z_w(z), Pz with Z_w'(z)
  for (int e = tid; e < nb * nb; e += 256) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < nb; ++w) {
      double zv, zd;
      basis_at(w, z, n, zv, zd);
      const double c = s->coef[e * nb + w];
      a += c * zv;
      b += c * zd;
    }
    P[e] = a;
    Pz[e] = b;
  }
  for (int e = tid; e < 64 * nb; e += 256) {
    const int i = e / nb, u = e % nb;
    double v = 0.0, d = 0.0;
    if (x0 + i < n) basis_at(u, x0 + i, n, v, d);
    Xv[i][u] = v;
    Xd[i][u] = d;
  }
  if (tid < 4 * nb) {
    const int j = tid / nb, u = tid % nb;
    double v = 0.0, d = 0.0;
    if (y0 + j < n) basis_at(u, y0 + j, n, v, d);
    Yv[j][u] = v;
    Yd[j][u] = d;
  }
  __syncthreads();
  const int i = tid & 63, j = tid >> 6;
  const int x = x0 + i, y = y0 + j;
  double gn = 0.0;
  if (x < n && y < n) {
    double F = 0.0, Gx = 0.0, Gy = 0.0, Gz = 0.0;
    for (int u = 0; u < nb; ++u) {
      double t = 0.0, ty = 0.0, tz = 0.0;
      for (int v = 0; v < nb; ++v) {
        const double pv = P[u * nb + v];
        t += pv * Yv[j][v];
        ty += pv * Yd[j][v];
        tz += Pz[u * nb + v] * Yv[j][v];
      }
      F += Xv[i][u] * t;
      Gx += Xd[i][u] * t;
      Gy += Xv[i][u] * ty;
      Gz += Xv[i][u] * tz;
    }
    const long long idx = ((long long)z * n + y) * n + x;
    s->F[idx] = F;
    s->G[idx] = Gx;
    s->G[s->nn + idx] = Gy;
    s->G[2 * s->nn + idx] = Gz;
    gn = sqrt(Gx * Gx + Gy * Gy + Gz * Gz);
  }
  // workgroup max, then a bitwise atomic max (non-negative doubles order as integers)
  for (int off = 32; off > 0; off >>= 1) gn = fmax(gn, __shfl_xor(gn, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = gn;
  __syncthreads();
  if (tid == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(&s->st->gmax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

// ---- distance d = |F - c| / max(||grad F||, 1e-12 max ||grad F||) ------------
__global__ __launch_bounds__(256) void distance_kernel(SlotDev *s) {
  const long long nn = s->nn;
  const double gmax = __longlong_as_double((long long)s->st->gmax_bits);
  const double gmin = 1e-12 * gmax;
  const int mode = s->dist_mode;
  const double iso = s->iso;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const double num = fabs(s->F[i] - iso);
    double d;
    if (mode == 1) {
      d = num;
    } else {
      const double gx = s->G[i], gy = s->G[nn + i], gz = s->G[2 * nn + i];
      const double den = fmax(sqrt(gx * gx + gy * gy + gz * gz), gmin);
      d = num > 0.0 ? num / den : 0.0;  // 0/0 -> 0; num/0 -> +inf
    }
    s->d[i] = d;
  }
}

// ---- hard step: k-th smallest distance by a 16-way search over bit patterns --
// Non-negative doubles (and +inf) order like their bit patterns.  Two searches
// run together: the k1-th and k2-th smallest values (1-based), each the
// smallest pattern v with count(d <= v) >= k inside its range [lo, hi].  Each
// launch counts the elements at or below 15 pivots splitting each range into
// 16 parts and keeps the part that holds the answer; a range of width w
// leaves at most w / 16 + 1, so 17 launches finish the 63-bit start.
constexpr int SEL_WAYS = 16, SEL_LAUNCHES = 18;

__device__ __forceinline__ unsigned long long sel_pivot(unsigned long long lo, unsigned long long w, int i) {
  // lo + floor(w (i + 1) / 16) without overflow
  return lo + (w / SEL_WAYS) * (i + 1) + ((w % SEL_WAYS) * (i + 1)) / SEL_WAYS;
}

__global__ __launch_bounds__(256) void select_count_kernel(SlotDev *s, long long k1, long long k2,
                                                           int nblocks) {
  constexpr int NP = SEL_WAYS - 1;
  __shared__ double red[2 * NP * 16];
  __shared__ int lastflag;
  CgState *st = s->st;
  const unsigned long long lo[2] = {st->sel_lo[0], st->sel_lo[1]};
  const unsigned long long hi[2] = {st->sel_hi[0], st->sel_hi[1]};
  if (lo[0] >= hi[0] && lo[1] >= hi[1]) return;  // both found (every workgroup sees the same)
  unsigned long long m[2][NP];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < NP; ++i) m[j][i] = sel_pivot(lo[j], hi[j] - lo[j], i);
  unsigned c[2][NP];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < NP; ++i) c[j][i] = 0u;
  const long long nn = s->nn;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)nblocks * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(s->d[e]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) c[j][i] += b <= m[j][i] ? 1u : 0u;
  }
  double v[2 * NP];  // exact: counts stay far below 2^53
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < NP; ++i) v[j * NP + i] = double(c[j][i]);
  block_sum<2 * NP>(v, red, 256);
  double *parts = s->partials;
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < 2 * NP; ++i) parts[32 * blockIdx.x + i] = v[i];
  if (!arrive_last(&st->cnt[6], nblocks, &lastflag)) return;
  double tot[2 * NP];
  sum_partials<2 * NP, 32>(parts, nblocks, tot, red, 256);
  if (threadIdx.x == 0) {
    const double kk[2] = {double(k1), double(k2)};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (lo[j] >= hi[j]) continue;
      // the first pivot whose count reaches k bounds the answer from above;
      // the pivot before it (or lo) from below
      unsigned long long nlo = lo[j], nhi = hi[j];
      bool found = false;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (found) continue;
        if (tot[j * NP + i] >= kk[j]) {
          nhi = m[j][i];
          found = true;
        } else {
          nlo = m[j][i] + 1;
        }
      }
      st->sel_lo[j] = nlo;
      st->sel_hi[j] = nhi;
    }
    st->cnt[6] = 0;
  }
}

// t from the two order statistics; k = round(vf n^3).
__global__ void select_finish_kernel(SlotDev *s, long long k) {
  CgState *st = s->st;
  const double v1 = __longlong_as_double((long long)st->sel_lo[0]);
  const double v2 = __longlong_as_double((long long)st->sel_lo[1]);
  double t;
  if (k <= 0) t = 0.5 * v1;                 // v1 = smallest
  else if (k >= s->nn) t = 2.0 * v2 + 1.0;  // v2 = largest
  else t = 0.5 * (v1 + v2);
  st->t = t;
}

// ---- logistic: bisection on t until |V(t) - target| <= 1e-12 ------------------
__global__ __launch_bounds__(256) void minmax_d_kernel(SlotDev *s) {
  // reuses sel_lo[0] / sel_hi[0] as min / max bit patterns
  const long long nn = s->nn;
  unsigned long long mn = ~0ull, mx = 0ull;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(s->d[i]);
    mn = b < mn ? b : mn;
    mx = b > mx ? b : mx;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a = __shfl_xor(mn, off, 64), c = __shfl_xor(mx, off, 64);
    mn = a < mn ? a : mn;
    mx = c > mx ? c : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s->st->sel_lo[0], mn);
    atomicMax(&s->st->sel_hi[0], mx);
  }
}

__global__ void bisect_init_kernel(SlotDev *s) {
  CgState *st = s->st;
  const double dmin = __longlong_as_double((long long)st->sel_lo[0]);
  const double dmax = __longlong_as_double((long long)st->sel_hi[0]);
  st->bis_lo = dmin - 40.0 / s->kappa;
  st->bis_hi = dmax + 40.0 / s->kappa;
  st->bis_done = 0;
  st->t = 0.5 * (st->bis_lo + st->bis_hi);
}

__device__ __forceinline__ double logistic(double kappa, double t, double d) {
  // 1 / (1 + exp(-kappa (t - d))), stable for both signs
  const double a = kappa * (t - d);
  if (a >= 0.0) return 1.0 / (1.0 + exp(-a));
  const double e = exp(a);
  return e / (1.0 + e);
}

__global__ __launch_bounds__(256) void bisect_step_kernel(SlotDev *s, int nblocks) {
  __shared__ double red[16];
  __shared__ int lastflag;
  CgState *st = s->st;
  if (st->bis_done) return;
  const double t = 0.5 * (st->bis_lo + st->bis_hi);
  const double kappa = s->kappa;
  const long long nn = s->nn;
  double v[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)nblocks * blockDim.x)
    v[0] += logistic(kappa, t, s->d[i]);
  block_sum<1>(v, red, 256);
  if (threadIdx.x == 0) s->partials[4 * blockIdx.x] = v[0];
  if (!arrive_last(&st->cnt[6], nblocks, &lastflag)) return;
  double tot[1];
  sum_partials<1>(s->partials, nblocks, tot, red, 256);
  if (threadIdx.x == 0) {
    const double V = tot[0] / double(nn);
    st->t = t;
    st->bis_V = V;
    if (fabs(V - s->target_vf) <= 1e-12) st->bis_done = 1;
    else if (V < s->target_vf) st->bis_lo = t;
    else st->bis_hi = t;
    st->cnt[6] = 0;
  }
}

// ---- occupancy, element moduli and volume fraction ---------------------------
__global__ __launch_bounds__(256) void occupancy_kernel(SlotDev *s, double *beta_out, int nblocks) {
  __shared__ double red[16];
  __shared__ int lastflag;
  CgState *st = s->st;
  const double t = st->t, kappa = s->kappa, E = s->E, Ev = s->E_void;
  const long long nn = s->nn;
  double v[1] = {0.0};  // V = mean beta over every voxel, culled or not
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)nblocks * blockDim.x) {
    const double d = s->d[i];
    const double b = kappa == 0.0 ? (d < t ? 1.0 : 0.0) : logistic(kappa, t, d);
    const double e = s->cull > 0.0 ? (b > s->cull ? E * b : 0.0) : Ev + (E - Ev) * b;
    s->E64[i] = e;
    if (s->E32) s->E32[i] = (float)e;
    if (beta_out) beta_out[i] = b;
    v[0] += b;
  }
  block_sum<1>(v, red, 256);
  if (threadIdx.x == 0) s->partials[4 * blockIdx.x] = v[0];
  if (!arrive_last(&st->cnt[6], nblocks, &lastflag)) return;
  double tot[1];
  sum_partials<1>(s->partials, nblocks, tot, red, 256);
  if (threadIdx.x == 0) {
    st->V = tot[0] / double(nn);
    st->cnt[6] = 0;
  }
}

// Moduli given directly (solver-only entries).  The source grid is one of
//   DT = 0: a 1-byte solid/void code, E_e = E where the code is nonzero, else E_void
//   DT = 1: float moduli,  DT = 2: double moduli.
template <int DT>
__device__ __forceinline__ double decode_modulus(const void *E, long long i, double Es, double Ev) {
  if constexpr (DT == 0) return ((const unsigned char *)E)[i] ? Es : Ev;
  else if constexpr (DT == 1) return (double)((const float *)E)[i];
  else return ((const double *)E)[i];
}

// Copy, round, and record the volume fraction: the solid share of the code
// (DT = 0), else mean(E) / max(E) (the bitwise max is taken beforehand).
template <int DT>
__global__ __launch_bounds__(256) void moduli_copy_kernel(SlotDev *s, const void *E, double Es, double Ev,
                                                          int nblocks) {
  __shared__ double red[16];
  __shared__ int lastflag;
  CgState *st = s->st;
  const long long nn = s->nn;
  double v[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)nblocks * blockDim.x) {
    const double e = decode_modulus<DT>(E, i, Es, Ev);
    s->E64[i] = e;
    if (s->E32) s->E32[i] = (float)e;
    if constexpr (DT == 0) v[0] += ((const unsigned char *)E)[i] ? 1.0 : 0.0;
    else v[0] += e;
  }
  block_sum<1>(v, red, 256);
  if (threadIdx.x == 0) s->partials[4 * blockIdx.x] = v[0];
  if (!arrive_last(&st->cnt[6], nblocks, &lastflag)) return;
  double tot[1];
  sum_partials<1>(s->partials, nblocks, tot, red, 256);
  if (threadIdx.x == 0) {
    const double emax = __longlong_as_double((long long)st->gmax_bits);
    st->Emax = emax;
    if constexpr (DT == 0) st->V = tot[0] / double(nn);
    else st->V = emax > 0.0 ? tot[0] / double(nn) / emax : 0.0;
    st->t = 0.0;
    st->cnt[6] = 0;
  }
}

template <int DT>
__global__ __launch_bounds__(256) void max_bits_kernel(SlotDev *s, const void *E, double Es, double Ev) {
  const long long nn = s->nn;
  unsigned long long mx = 0ull;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const double e = decode_modulus<DT>(E, i, Es, Ev);
    const unsigned long long b = e > 0.0 ? (unsigned long long)__double_as_longlong(e) : 0ull;
    mx = b > mx ? b : mx;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long c = __shfl_xor(mx, off, 64);
    mx = c > mx ? c : mx;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(&s->st->gmax_bits, mx);
}

// ---- inverse Jacobi diagonal: ((lambda + 4 mu)/9 * sum of the 8 incident E_e)^-1 --
template <typename T>
__global__ __launch_bounds__(256) void dinv_kernel(SlotDev *s) {
  const int n = s->n;
  const long long nn = s->nn;
  const double c = (s->lam + 4.0 * s->mu) / 9.0;
  T *Dinv = (T *)s->Dinv;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = int(i % n), y = int((i / n) % n), z = int(i / ((long long)n * n));
    const int xm = x == 0 ? n - 1 : x - 1, ym = y == 0 ? n - 1 : y - 1, zm = z == 0 ? n - 1 : z - 1;
    const double *E = s->E64;
    auto at = [&](int a, int b, int cc) { return E[((long long)cc * n + b) * n + a]; };
    const double sum = ((at(x, y, z) + at(xm, y, z)) + (at(x, ym, z) + at(xm, ym, z))) +
                       ((at(x, y, zm) + at(xm, y, zm)) + (at(x, ym, zm) + at(xm, ym, zm)));
    const double dg = c * sum;
    Dinv[i] = (T)(dg > 0.0 ? 1.0 / dg : 0.0);
  }
}

// ---- host launchers ------------------------------------------------------------
static int grid_for(long long nn, int cap) {
  long long g = (nn + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return int(g);
}

hipError_t launch_field(SlotDev *d_slot, int n, int nb, hipStream_t st) {
  coef_kernel<<<(nb * nb * nb + 255) / 256, 256, 0, st>>>(d_slot);
  dim3 g((n + 63) / 64, (n + 3) / 4, n);
  field_kernel<<<g, 256, 0, st>>>(d_slot);
  const long long nn = (long long)n * n * n;
  distance_kernel<<<grid_for(nn, 8192), 256, 0, st>>>(d_slot);
  return hipGetLastError();
}

int reduce_blocks(long long nn) { return grid_for(nn, 1024); }

hipError_t launch_select_hard(SlotDev *d_slot, long long nn, long long k, hipStream_t st) {
  // 32 elements per thread: fewer partials for the last workgroup to sum
  const int nbk = (int)std::max(1LL, std::min(2048LL, (nn + 8191) / 8192));
  const long long k1 = k <= 0 ? 1 : (k >= nn ? nn : k);
  const long long k2 = k <= 0 ? 1 : (k >= nn ? nn : k + 1);
  for (int it = 0; it < SEL_LAUNCHES; ++it) select_count_kernel<<<nbk, 256, 0, st>>>(d_slot, k1, k2, nbk);
  select_finish_kernel<<<1, 1, 0, st>>>(d_slot, k);
  return hipGetLastError();
}

hipError_t launch_minmax_d(SlotDev *d_slot, long long nn, hipStream_t st) {
  minmax_d_kernel<<<grid_for(nn, 1024), 256, 0, st>>>(d_slot);
  bisect_init_kernel<<<1, 1, 0, st>>>(d_slot);
  return hipGetLastError();
}

hipError_t launch_bisect_steps(SlotDev *d_slot, long long nn, int steps, hipStream_t st) {
  const int nbk = reduce_blocks(nn);
  for (int it = 0; it < steps; ++it) bisect_step_kernel<<<nbk, 256, 0, st>>>(d_slot, nbk);
  return hipGetLastError();
}

hipError_t launch_occupancy(SlotDev *d_slot, long long nn, double *beta_out, hipStream_t st) {
  const int nbk = reduce_blocks(nn);
  occupancy_kernel<<<nbk, 256, 0, st>>>(d_slot, beta_out, nbk);
  return hipGetLastError();
}

hipError_t launch_moduli_copy(SlotDev *d_slot, long long nn, const void *E, int e_dtype, double Es, double Ev,
                              hipStream_t st) {
  const int g = grid_for(nn, 1024), nbk = reduce_blocks(nn);
  if (e_dtype == 0) {
    max_bits_kernel<0><<<g, 256, 0, st>>>(d_slot, E, Es, Ev);
    moduli_copy_kernel<0><<<nbk, 256, 0, st>>>(d_slot, E, Es, Ev, nbk);
  } else if (e_dtype == 1) {
    max_bits_kernel<1><<<g, 256, 0, st>>>(d_slot, E, Es, Ev);
    moduli_copy_kernel<1><<<nbk, 256, 0, st>>>(d_slot, E, Es, Ev, nbk);
  } else {
    max_bits_kernel<2><<<g, 256, 0, st>>>(d_slot, E, Es, Ev);
    moduli_copy_kernel<2><<<nbk, 256, 0, st>>>(d_slot, E, Es, Ev, nbk);
  }
  return hipGetLastError();
}

hipError_t launch_dinv(SlotDev *d_slot, long long nn, int prec, hipStream_t st) {
  if (prec == 0) dinv_kernel<double><<<grid_for(nn, 8192), 256, 0, st>>>(d_slot);
  else dinv_kernel<float><<<grid_for(nn, 8192), 256, 0, st>>>(d_slot);
  return hipGetLastError();
}

hipError_t launch_coef(SlotDev *d_slot, int nb, hipStream_t st) {
  coef_kernel<<<(nb * nb * nb + 255) / 256, 256, 0, st>>>(d_slot);
  return hipGetLastError();
}

}  // namespace shh
