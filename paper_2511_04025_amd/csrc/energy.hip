// Step 4 and the adjoint.
//
// C^H_ij = (1/n^3) sum_e E_e (chi^i + u^i_e)^T K_0 (chi^j + u^j_e)  (Eq. (8)),
// evaluated per element in the Walsh-Hadamard basis (hexop.hpp) in FP64 with a
// deterministic two-stage reduction of the 21 distinct entries.
//
// Adjoint (Eq. (9)): every u^k is at equilibrium, so
//   dC_ij/dE_e = (1/n^3) (chi^i + u^i_e)^T K_0 (chi^j + u^j_e)   (no extra solve);
// chained through E_e = E_void + (E - E_void) beta_e, the logistic occupancy,
// d = |F - c| / ||grad F|| and Eq. (6).  The pull-back onto the charges uses the
// same separable trig basis as the field synthesis: the voxel sensitivities
// are projected onto the (2K+1)^3 coefficient tensor one axis at a time
// (x-rows, then y, then z), and the coefficient tensor's derivative with
// respect to each charge position and value closes the chain.
#include "common.hpp"
#include "hexop.hpp"
#include <algorithm>

#include "kernels.hpp"

namespace shh {

__device__ __forceinline__ void element_hadamard(const double *u, long long nn, const long long (&node)[8],
                                                 int k, double (&h)[3][8]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = u[((long long)k * 3 + c) * nn + node[a]];
    hadamard8<double>(v, h[c]);
  }
  add_chi<double>(k, h);
}

__host__ __device__ constexpr int pair_index(int i, int j) {  // i <= j, row-major upper triangle
  return i * 6 - (i * (i - 1)) / 2 + (j - i);
}

// MODE 0: per-workgroup sums of E_e e_ij (21 values) -> st->C.
// MODE 1: out[e] = sum_{i<=j} Gs_ij e_ij / n^3 (dL/dE_e for a symmetric-folded Gs).
template <int MODE>
__global__ __launch_bounds__(256) void energy_kernel(SlotDev *s, int nblocks, const double *Gs,
                                                     double *out) {
  __shared__ double red[21 * 16];
  __shared__ int lastflag;
  const int n = s->n;
  const long long nn = s->nn;
  const double *u = s->x64;
  const double *kop = s->kop64;
  double acc[21];
#pragma unroll
  for (int t = 0; t < 21; ++t) acc[t] = 0.0;
  double g[21];
  if (MODE == 1) {
#pragma unroll
    for (int t = 0; t < 21; ++t) g[t] = Gs[t];
  }
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (long long)nblocks * blockDim.x) {
    const int x = int(e % n), y = int((e / n) % n), z = int(e / ((long long)n * n));
    const int xp = x + 1 == n ? 0 : x + 1, yp = y + 1 == n ? 0 : y + 1, zp = z + 1 == n ? 0 : z + 1;
    long long node[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = (a & 1) ? xp : x, ay = (a & 2) ? yp : y, az = (a & 4) ? zp : z;
      node[a] = ((long long)az * n + ay) * n + ax;
    }
    const double Ee = s->E64[e];
    double sens = 0.0;
#pragma unroll
    for (int j = 0; j < NRHS; ++j) {
      double hj[3][8], wj[3][8];
      element_hadamard(u, nn, node, j, hj);
      hex_apply<double>(kop, hj, wj, 1.0);
#pragma unroll
      for (int i = 0; i <= j; ++i) {
        double hi[3][8];
        if (i == j) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int m = 0; m < 8; ++m) hi[c][m] = hj[c][m];
        } else {
          element_hadamard(u, nn, node, i, hi);
        }
        double eij = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int m = 0; m < 8; ++m) eij += hi[c][m] * wj[c][m];
        if (MODE == 0) acc[pair_index(i, j)] += Ee * eij;
        else sens += g[pair_index(i, j)] * eij;
      }
    }
    if (MODE == 1) out[e] = sens / double(nn);
  }
  if (MODE == 1) return;
  block_sum<21>(acc, red, 256);
  double *parts = s->partials;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < 21; ++t) parts[21 * blockIdx.x + t] = acc[t];
  }
  if (!arrive_last(&s->st->cnt[7], nblocks, &lastflag)) return;
  double tot[21];
  sum_partials<21, 21>(parts, nblocks, tot, red, 256);
  if (threadIdx.x == 0) {
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j) {
        const double c = tot[pair_index(i, j)] / double(nn);
        s->st->C[i * 6 + j] = c;
        s->st->C[j * 6 + i] = c;
      }
    s->st->cnt[7] = 0;
  }
}

hipError_t launch_energy(SlotDev *d_slot, long long nn, hipStream_t st) {
  const int nbk = reduce_blocks(nn);
  energy_kernel<0><<<nbk, 256, 0, st>>>(d_slot, nbk, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_energy_sens(SlotDev *d_slot, long long nn, const double *d_G21, double *d_out,
                              hipStream_t st) {
  long long g = (nn + 255) / 256;
  if (g > 8192) g = 8192;
  energy_kernel<1><<<int(g), 256, 0, st>>>(d_slot, int(g), d_G21, d_out);
  return hipGetLastError();
}

// ---- adjoint: voxel sensitivities ---------------------------------------------
__device__ __forceinline__ double logistic_d(double kappa, double t, double d) {
  const double a = kappa * (t - d);
  if (a >= 0.0) return 1.0 / (1.0 + exp(-a));
  const double e = exp(a);
  return e / (1.0 + e);
}

// gF = dL/dF_e, gG = dL/d(grad F)_e  (layout [4][nn]); per workgroup the
// partial sum of dL/dt = sum_e dL/dbeta_e kappa beta_e (1 - beta_e) (t free)
__global__ __launch_bounds__(256) void voxel_adjoint_kernel(SlotDev *s, const double *gE, double gV,
                                                            double *gout, double *t_parts) {
  __shared__ double red[16];
  const long long nn = s->nn;
  const CgState *st = s->st;
  const double t = st->t, kappa = s->kappa, dE = s->E - s->E_void, iso = s->iso;
  const double gmax = __longlong_as_double((long long)st->gmax_bits);
  const double gmin = 1e-12 * gmax;
  double gt[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const double d = s->d[i];
    const double b = logistic_d(kappa, t, d);
    const double gbeta = gE[i] * dE + gV / double(nn);
    const double gd = gbeta * (-kappa * b * (1.0 - b));
    gt[0] -= gd;
    const double diff = s->F[i] - iso;
    const double sgn = diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0);
    double gF, gx = 0.0, gy = 0.0, gz = 0.0;
    if (s->dist_mode == 1) {
      gF = gd * sgn;
    } else {
      const double Gx = s->G[i], Gy = s->G[nn + i], Gz = s->G[2 * nn + i];
      const double gn = sqrt(Gx * Gx + Gy * Gy + Gz * Gz);
      const bool clamped = gn < gmin;
      const double den = clamped ? gmin : gn;
      gF = gd * sgn / den;
      if (!clamped) {
        const double f = -gd * fabs(diff) / (den * den * den);
        gx = f * Gx;
        gy = f * Gy;
        gz = f * Gz;
      }
    }
    gout[i] = gF;
    gout[nn + i] = gx;
    gout[2 * nn + i] = gy;
    gout[3 * nn + i] = gz;
  }
  block_sum<1>(gt, red, 256);
  if (threadIdx.x == 0) t_parts[blockIdx.x] = gt[0];
}

// dL/dt: the workgroup partials of voxel_adjoint_kernel in a fixed order
__global__ __launch_bounds__(256) void adj_thickness_kernel(const double *t_parts, int count, double *out) {
  __shared__ double red[16];
  double tot[1];
  sum_partials<1, 1>(t_parts, count, tot, red, 256);
  if (threadIdx.x == 0) *out = tot[0];
}

// dL/dalpha_hkl from dL/dcoef: coef[u][v][w] = sum_hkl alpha_hkl w_hkl / (h^2+k^2+l^2)
// sum_j q_j T_u(x_j) T_v(y_j) T_w(z_j), the charge-side basis T pairing cos
// with cos and sin with sin, so dL/dalpha_hkl sums dL/dcoef over the (at most
// 8) basis triples of mode (h, k, l) against the charges' products.  One
// thread per mode.
__global__ __launch_bounds__(256) void adj_alpha_kernel(SlotDev *s, const double *dcoef, double *out) {
  const int K = s->K, K1 = K + 1, nb = s->nb, N = s->N;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= K1 * K1 * K1) return;
  const int h = m / (K1 * K1), k = (m / K1) % K1, l = m % K1;
  if (h + k + l == 0) {
    out[m] = 0.0;
    return;
  }
  const int zeros = (h == 0) + (k == 0) + (l == 0);
  const double wgt = (zeros == 0 ? 1.0 : (zeros == 1 ? 0.5 : 0.25)) / double(h * h + k * k + l * l);
  // basis indices of the mode per axis: u = 0 (h = 0), else 2h - 1 (cos) and 2h (sin)
  const int hu[3] = {h, k, l};
  double acc = 0.0;
  for (int j = 0; j < N; ++j) {
    const double *ch = s->charges + 4 * j;
    double T[3][2];
    int nu_[3], u0[3];
    for (int ax = 0; ax < 3; ++ax) {
      if (hu[ax] == 0) {
        nu_[ax] = 1;
        u0[ax] = 0;
        T[ax][0] = 1.0;
      } else {
        nu_[ax] = 2;
        u0[ax] = 2 * hu[ax] - 1;
        double sn, cs;
        sincospi(2.0 * hu[ax] * ch[ax], &sn, &cs);
        T[ax][0] = cs;
        T[ax][1] = sn;
      }
    }
    double sj = 0.0;
    for (int a = 0; a < nu_[0]; ++a)
      for (int b = 0; b < nu_[1]; ++b)
        for (int c = 0; c < nu_[2]; ++c)
          sj += dcoef[((u0[0] + a) * nb + (u0[1] + b)) * nb + (u0[2] + c)] * T[0][a] * T[1][b] * T[2][c];
    acc += ch[3] * sj;
  }
  out[m] = wgt * acc;
}

// 1D basis table at the voxel centers: val[i][u], der[i][u]
__global__ void basis_table_kernel(int n, int nb, double *val, double *der) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nb) return;
  const int i = e / nb, u = e % nb;
  if (u == 0) { val[e] = 1.0; der[e] = 0.0; return; }
  const int h = (u + 1) >> 1;
  double sn, cs;
  sincospi(double(h) * double(2 * i + 1) / double(n), &sn, &cs);
  const double w = 2.0 * M_PI * h;
  if (u & 1) { val[e] = cs; der[e] = -w * sn; } else { val[e] = sn; der[e] = w * cs; }
}

// one wave per x-row (y, z): rows[row][0..nb) = sum_x gF X_u + gGx X'_u,
// [nb..2nb) = sum_x gGy X_u, [2nb..3nb) = sum_x gGz X_u
__global__ __launch_bounds__(256) void adj_rows_kernel(int n, int nb, const double *g, const double *val,
                                                       const double *der, double *rows) {
  const long long nn = (long long)n * n * n;
  const int lane = threadIdx.x & 63;
  const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (long long)n * n) return;
  double a[MAXB], b[MAXB], c[MAXB];
  for (int u = 0; u < nb; ++u) { a[u] = 0.0; b[u] = 0.0; c[u] = 0.0; }
  for (int x = lane; x < n; x += 64) {
    const long long i = row * n + x;
    const double gF = g[i], gx = g[nn + i], gy = g[2 * nn + i], gz = g[3 * nn + i];
    for (int u = 0; u < nb; ++u) {
      const double X = val[x * nb + u], Xd = der[x * nb + u];
      a[u] += gF * X + gx * Xd;
      b[u] += gy * X;
      c[u] += gz * X;
    }
  }
  for (int u = 0; u < nb; ++u) {
    for (int off = 32; off > 0; off >>= 1) {
      a[u] += __shfl_xor(a[u], off, 64);
      b[u] += __shfl_xor(b[u], off, 64);
      c[u] += __shfl_xor(c[u], off, 64);
    }
  }
  if (lane == 0) {
    double *o = rows + row * 3 * nb;
    for (int u = 0; u < nb; ++u) { o[u] = a[u]; o[nb + u] = b[u]; o[2 * nb + u] = c[u]; }
  }
}

// per z plane: P[z][u][v] = sum_y a[u] Y_v + b[u] Y'_v;  Pz[z][u][v] = sum_y c[u] Y_v
__global__ void adj_planes_kernel(int n, int nb, const double *rows, const double *val,
                                  const double *der, double *planes) {
  const int z = blockIdx.x;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int u = e / nb, v = e % nb;
    double P = 0.0, Pz = 0.0;
    for (int y = 0; y < n; ++y) {
      const double *r = rows + ((long long)z * n + y) * 3 * nb;
      P += r[u] * val[y * nb + v] + r[nb + u] * der[y * nb + v];
      Pz += r[2 * nb + u] * val[y * nb + v];
    }
    planes[((long long)z * 2 + 0) * nb * nb + e] = P;
    planes[((long long)z * 2 + 1) * nb * nb + e] = Pz;
  }
}

// dL/dcoef[u][v][w] = sum_z P[z][u][v] Z_w + Pz[z][u][v] Z'_w
__global__ void adj_coef_kernel(int n, int nb, const double *planes, const double *val,
                                const double *der, double *dcoef) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * nb * nb) return;
  const int uv = e / nb, w = e % nb;
  double acc = 0.0;
  for (int z = 0; z < n; ++z)
    acc += planes[((long long)z * 2) * nb * nb + uv] * val[z * nb + w] +
           planes[((long long)z * 2 + 1) * nb * nb + uv] * der[z * nb + w];
  dcoef[e] = acc;
}

// per charge: dL/dq_j and dL/d(x_j, y_j, z_j) from dL/dcoef
__global__ void adj_charges_kernel(SlotDev *s, const double *dcoef, double *out) {
  const int j = blockIdx.x;
  const int K = s->K, nb = s->nb, K1 = K + 1;
  const double *ch = s->charges + 4 * j;
  // charge-side basis values and derivatives per axis
  __shared__ double tv[3][MAXB], td[3][MAXB];
  __shared__ double red[4 * 16];
  if (threadIdx.x < 3 * nb) {
    const int ax = threadIdx.x / nb, u = threadIdx.x % nb;
    if (u == 0) { tv[ax][u] = 1.0; td[ax][u] = 0.0; }
    else {
      const int h = (u + 1) >> 1;
      double sn, cs;
      sincospi(2.0 * h * ch[ax], &sn, &cs);
      const double w = 2.0 * M_PI * h;
      if (u & 1) { tv[ax][u] = cs; td[ax][u] = -w * sn; } else { tv[ax][u] = sn; td[ax][u] = w * cs; }
    }
  }
  __syncthreads();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int total = nb * nb * nb;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int u = e / (nb * nb), v = (e / nb) % nb, w = e % nb;
    const int h = (u + 1) >> 1, k = (v + 1) >> 1, l = (w + 1) >> 1;
    if (h + k + l == 0) continue;
    const int zeros = (h == 0) + (k == 0) + (l == 0);
    const double wgt = zeros == 0 ? 1.0 : (zeros == 1 ? 0.5 : 0.25);
    const double a = s->alpha ? s->alpha[(h * K1 + k) * K1 + l] : 1.0;
    const double c = a * wgt / double(h * h + k * k + l * l) * dcoef[e];
    acc[0] += c * tv[0][u] * tv[1][v] * tv[2][w];
    acc[1] += c * td[0][u] * tv[1][v] * tv[2][w];
    acc[2] += c * tv[0][u] * td[1][v] * tv[2][w];
    acc[3] += c * tv[0][u] * tv[1][v] * td[2][w];
  }
  block_sum<4>(acc, red, blockDim.x);
  if (threadIdx.x == 0) {
    const double q = ch[3];
    out[4 * j + 0] = q * acc[1];
    out[4 * j + 1] = q * acc[2];
    out[4 * j + 2] = q * acc[3];
    out[4 * j + 3] = acc[0];
  }
}

size_t adjoint_scratch_bytes(int n, int K) {
  const long long nn = (long long)n * n * n;
  const long long nb = 2 * K + 1;
  const long long parts = std::min((nn + 255) / 256, 8192LL);  // voxel_adjoint_kernel workgroups
  const long long doubles = 4 * nn + 2 * n * nb + (long long)n * n * 3 * nb + (long long)n * 2 * nb * nb +
                            nb * nb * nb + parts;
  return size_t(doubles) * sizeof(double);
}

hipError_t launch_adjoint(SlotDev *d_slot, int n, int nb, int N, int K, const double *d_gE, double gV,
                          double *d_scratch, double *d_out, double *d_alpha_out, double *d_t_out,
                          hipStream_t st) {
  const long long nn = (long long)n * n * n;
  double *g = d_scratch;                          // [4][nn]
  double *val = g + 4 * nn;                       // [n][nb]
  double *der = val + (long long)n * nb;          // [n][nb]
  double *rows = der + (long long)n * nb;         // [n*n][3 nb]
  double *planes = rows + (long long)n * n * 3 * nb;  // [n][2][nb*nb]
  double *dcoef = planes + (long long)n * 2 * nb * nb;  // [nb^3]
  double *t_parts = dcoef + (long long)nb * nb * nb;    // [<= 8192]
  long long gg = (nn + 255) / 256;
  if (gg > 8192) gg = 8192;
  voxel_adjoint_kernel<<<int(gg), 256, 0, st>>>(d_slot, d_gE, gV, g, t_parts);
  if (d_t_out) adj_thickness_kernel<<<1, 256, 0, st>>>(t_parts, int(gg), d_t_out);
  basis_table_kernel<<<(n * nb + 255) / 256, 256, 0, st>>>(n, nb, val, der);
  const long long nrows = (long long)n * n;
  adj_rows_kernel<<<int((nrows + 3) / 4), 256, 0, st>>>(n, nb, g, val, der, rows);
  adj_planes_kernel<<<n, 64, 0, st>>>(n, nb, rows, val, der, planes);
  adj_coef_kernel<<<(nb * nb * nb + 127) / 128, 128, 0, st>>>(n, nb, planes, val, der, dcoef);
  adj_charges_kernel<<<N, 256, 0, st>>>(d_slot, dcoef, d_out);
  const int K1 = K + 1;
  if (d_alpha_out) adj_alpha_kernel<<<(K1 * K1 * K1 + 255) / 256, 256, 0, st>>>(d_slot, dcoef, d_alpha_out);
  return hipGetLastError();
}

// dL/d(charges, alpha) from dL/dcoef alone (the point-field adjoint)
hipError_t launch_coef_adjoint(SlotDev *d_slot, int N, int K, const double *d_dcoef, double *d_out,
                               double *d_alpha_out, hipStream_t st) {
  adj_charges_kernel<<<N, 256, 0, st>>>(d_slot, d_dcoef, d_out);
  const int K1 = K + 1;
  if (d_alpha_out) adj_alpha_kernel<<<(K1 * K1 * K1 + 255) / 256, 256, 0, st>>>(d_slot, d_dcoef, d_alpha_out);
  return hipGetLastError();
}

}  // namespace shh
