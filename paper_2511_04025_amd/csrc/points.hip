// The charge field of Eq. (6) at arbitrary points (not voxel centers), and the
// adjoint of a functional of those values: the pieces the fitting objective of
// Eq. (10) needs.  Both go through the trig coefficient tensor of the field
// (see field.hip): F(p) = sum_uvw coef[u][v][w] T_u(x) T_v(y) T_w(z), with
// T_0 = 1, T_{2h-1} = cos 2 pi h s, T_{2h} = sin 2 pi h s.  FP64.
#include "common.hpp"
#include "kernels.hpp"

namespace shh {

namespace {

__device__ __forceinline__ void point_basis(double s, int nb, double *val, double *der) {
  val[0] = 1.0;
  der[0] = 0.0;
  for (int u = 1; u < nb; ++u) {
    const int h = (u + 1) >> 1;
    double sn, cs;
    sincospi(2.0 * h * s, &sn, &cs);
    const double w = 2.0 * M_PI * h;
    if (u & 1) { val[u] = cs; der[u] = -w * sn; } else { val[u] = sn; der[u] = w * cs; }
  }
}

}  // namespace

// one thread per point; the coefficient tensor is staged in LDS
__global__ __launch_bounds__(256) void points_field_kernel(const SlotDev *s, int npts, const double *pts,
                                                           double *F, double *G) {
  __shared__ double coef[MAXB * MAXB * MAXB];
  const int nb = s->nb;
  const int total = nb * nb * nb;
  for (int e = threadIdx.x; e < total; e += blockDim.x) coef[e] = s->coef[e];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  double tv[3][MAXB], td[3][MAXB];
  for (int ax = 0; ax < 3; ++ax) point_basis(pts[3 * i + ax], nb, tv[ax], td[ax]);
  double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int u = 0; u < nb; ++u)
    for (int v = 0; v < nb; ++v) {
      double a = 0.0, b = 0.0;
      const double *c = coef + (u * nb + v) * nb;
      for (int w = 0; w < nb; ++w) {
        a += c[w] * tv[2][w];
        b += c[w] * td[2][w];
      }
      f += tv[0][u] * tv[1][v] * a;
      gx += td[0][u] * tv[1][v] * a;
      gy += tv[0][u] * td[1][v] * a;
      gz += tv[0][u] * tv[1][v] * b;
    }
  F[i] = f;
  if (G) {
    G[i] = gx;
    G[npts + i] = gy;
    G[2 * npts + i] = gz;
  }
}

// basis values per point: [npts][3][nb]
__global__ __launch_bounds__(256) void points_basis_kernel(int nb, int npts, const double *pts, double *basis) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  double val[MAXB], der[MAXB];
  for (int ax = 0; ax < 3; ++ax) {
    point_basis(pts[3 * i + ax], nb, val, der);
    for (int u = 0; u < nb; ++u) basis[((long long)i * 3 + ax) * nb + u] = val[u];
  }
}

// dL/dcoef[u][v][w] = sum_i dL/dF_i T_u(x_i) T_v(y_i) T_w(z_i): one workgroup
// per coefficient, a fixed-order reduction over the points
__global__ __launch_bounds__(256) void points_dcoef_kernel(int nb, int npts, const double *basis, const double *gF,
                                                           double *dcoef) {
  __shared__ double red[16];
  const int e = blockIdx.x;
  const int u = e / (nb * nb), v = (e / nb) % nb, w = e % nb;
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < npts; i += blockDim.x) {
    const double *b = basis + (long long)i * 3 * nb;
    acc[0] += gF[i] * b[u] * b[nb + v] * b[2 * nb + w];
  }
  block_sum<1>(acc, red, 256);
  if (threadIdx.x == 0) dcoef[e] = acc[0];
}

hipError_t launch_points_field(SlotDev *d_slot, int nb, int npts, const double *d_pts, double *d_F, double *d_G,
                               hipStream_t st) {
  (void)nb;
  points_field_kernel<<<(npts + 255) / 256, 256, 0, st>>>(d_slot, npts, d_pts, d_F, d_G);
  return hipGetLastError();
}

hipError_t launch_points_dcoef(int nb, int npts, const double *d_pts, const double *d_gF, double *d_basis,
                               double *d_dcoef, hipStream_t st) {
  points_basis_kernel<<<(npts + 255) / 256, 256, 0, st>>>(nb, npts, d_pts, d_basis);
  points_dcoef_kernel<<<nb * nb * nb, 256, 0, st>>>(nb, npts, d_basis, d_gF, d_dcoef);
  return hipGetLastError();
}

}  // namespace shh
