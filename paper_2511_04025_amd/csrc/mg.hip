// Kernels of the geometric multigrid preconditioner (see mg.hpp): setup
// (Galerkin element matrices, nodal stencils, diagonals, power iteration) and
// the V-cycle and CG sweeps.  T is the working precision of the slot.
#include "kernels.hpp"
#include "mg.hpp"

namespace shh {

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

// Level-1 element matrices: K_E = sum_f E_f G_f over the 8 voxels of coarse
// element E.  One thread per (element, row).
template <typename T>
__global__ __launch_bounds__(256) void mg_elem1_kernel(const SlotDev *s, const MgDev *mg) {
  const MgLevel &c = mg->lv[1];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= c.nn * 24) return;
  const long long E = t / 24;
  const int i = int(t % 24);
  const int nc = c.n, nf = s->n;
  const int X = int(E % nc), Y = int((E / nc) % nc), Z = int(E / ((long long)nc * nc));
  const double *Ef = s->E64;
  const T *G = (const T *)mg->G;
  double row[24];
#pragma unroll
  for (int j = 0; j < 24; ++j) row[j] = 0.0;
  for (int f = 0; f < 8; ++f) {
    const int fx = f & 1, fy = (f >> 1) & 1, fz = f >> 2;
    const long long fe = ((long long)(2 * Z + fz) * nf + (2 * Y + fy)) * nf + (2 * X + fx);
    const double e = Ef[fe];
    const T *g = G + (f * 24 + i) * 24;
#pragma unroll
    for (int j = 0; j < 24; ++j) row[j] += e * (double)g[j];
  }
  T *K = (T *)c.Ke + E * 576 + i * 24;
#pragma unroll
  for (int j = 0; j < 24; ++j) K[j] = (T)row[j];
}

// Trilinear weight of coarse corner a at fine corner b of child f (per axis:
// fine position (f + b) / 2 in the coarse element).
__device__ __forceinline__ double qweight(int f, int b, int a) {
  double w = 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int pos2 = ((f >> d) & 1) + ((b >> d) & 1);  // 0, 1 or 2 halves
    const int ad = (a >> d) & 1;
    const double p = 0.5 * pos2;
    w *= ad ? p : 1.0 - p;
  }
  return w;
}

// Level l + 1 element matrices from level l: K_E = sum_f Q_f^T K_f Q_f.
// One thread per (coarse element, row i = 3 a + c).
template <typename T>
__global__ __launch_bounds__(256) void mg_elemc_kernel(const MgDev *mg, int l) {
  const MgLevel &fl = mg->lv[l];
  const MgLevel &cl = mg->lv[l + 1];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cl.nn * 24) return;
  const long long E = t / 24;
  const int i = int(t % 24);
  const int a = i / 3, ci = i % 3;
  const int nc = cl.n, nf = fl.n;
  const int X = int(E % nc), Y = int((E / nc) % nc), Z = int(E / ((long long)nc * nc));
  const T *Kf = (const T *)fl.Ke;
  double row[24];
#pragma unroll
  for (int j = 0; j < 24; ++j) row[j] = 0.0;
  for (int f = 0; f < 8; ++f) {
    const int fx = f & 1, fy = (f >> 1) & 1, fz = f >> 2;
    const long long fe = ((long long)(2 * Z + fz) * nf + (2 * Y + fy)) * nf + (2 * X + fx);
    const T *K = Kf + fe * 576;
    // w = Q_f[:, i]^T K_f: rows 3 b' + ci of K_f weighted by q(f, b', a)
    double w[24];
#pragma unroll
    for (int j = 0; j < 24; ++j) w[j] = 0.0;
    for (int bp = 0; bp < 8; ++bp) {
      const double q = qweight(f, bp, a);
      if (q == 0.0) continue;
      const T *kr = K + (3 * bp + ci) * 24;
#pragma unroll
      for (int j = 0; j < 24; ++j) w[j] += q * (double)kr[j];
    }
    // row += w Q_f: column 3 a' + c of the result sums w[3 b + c] q(f, b, a')
    for (int ap = 0; ap < 8; ++ap) {
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double q = qweight(f, b, ap);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) row[3 * ap + cc] += q * w[3 * b + cc];
      }
    }
  }
  T *out = (T *)cl.Ke + E * 576 + i * 24;
#pragma unroll
  for (int j = 0; j < 24; ++j) out[j] = (T)row[j];
}

// Nodal stencil of level l from its element matrices (the 14 stored offsets),
// and D^-1.  Node v is corner a of element v - a; entry (v, v - a + b)
// gathers K_e[a][b].
template <typename T>
__global__ __launch_bounds__(256) void mg_stencil_kernel(const MgDev *mg, int l) {
  const MgLevel &L = mg->lv[l];
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= L.nn) return;
  const int n = L.n;
  const int x = int(v % n), y = int((v / n) % n), z = int(v / ((long long)n * n));
  const T *Ke = (const T *)L.Ke;
  T *S = (T *)L.S;
  for (int k = 0; k < MG_STENCIL; ++k) S[k * L.nn + v] = T(0);
  double diag[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const long long e = ((long long)wrapi(z - az, n) * n + wrapi(y - ay, n)) * n + wrapi(x - ax, n);
    const T *K = Ke + e * 576;
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      const int w = ((bz - az + 1) * 3 + (by - ay + 1)) * 3 + (bx - ax + 1);
      if (w < 13) continue;  // stored by the neighbour, transposed
      for (int c = 0; c < 3; ++c)
        for (int cp = 0; cp < 3; ++cp) {
          const T kv = K[(3 * a + c) * 24 + 3 * b + cp];
          T *dst = S + ((w - 13) * 9 + 3 * c + cp) * L.nn + v;
          *dst = *dst + kv;
          if (b == a && cp == c) diag[c] += (double)kv;
        }
    }
  }
  T *Dinv = (T *)L.Dinv;
  for (int c = 0; c < 3; ++c) Dinv[c * L.nn + v] = diag[c] > 0.0 ? (T)(1.0 / diag[c]) : T(0);
}

// ---------------------------------------------------------------------------
// operator, transfer and coarsest solve (levels >= 1)
// ---------------------------------------------------------------------------

// q = A_l v (v = x or d of the level) for RHS load cases per thread: RHS =
// NRHS (one thread per node; the stencil is read once for all load cases) on
// large levels of odd size (even ones take the pair form below), RHS = 1 (one
// thread per node and load case: six times the threads, so latency overlaps)
// on small ones.
// The coarse-level Chebyshev sweep that follows an operator pass, applied
// to q = A_l v at node v, load case k (entry j = (3 k + c) nn + v):
//   MGE_NONE:  q = A v
//   MGE_STEP1: (v = d0) r = b - q;  d1 = c1 d0 + c2 D^-1 r;  x = d0 + d1;  d1 into q
//   MGE_RES:   (v = d1, in q) r -= q: the residual the restriction takes
//   MGE_POST:  (v = x) r = b - q;  d = D^-1 r / theta;  x + d into q
//   MGE_LAST:  (v = d) x = (x + d, in q) + c1 d + c2 D^-1 (r - q)
// No pass writes the vector its operator reads.
// The level's vectors and coefficients, read once per thread into scalar
// registers: a field read after a store would be read again (the store might
// have changed it), behind a wait for the store.
template <typename T>
struct MgEpi {
  SHH_GLOBAL T *q, *r, *x, *d;
  const SHH_GLOBAL T *b;
  T c1, c2, inv_theta;
};
template <typename T>
__device__ __forceinline__ MgEpi<T> mg_epi(const MgLevel &L) {
  MgEpi<T> E;
  E.q = to_global((T *)L.q);
  E.r = to_global((T *)L.r);
  E.x = to_global((T *)L.x);
  E.d = to_global((T *)L.d);
  E.b = to_global((const T *)L.b);
  E.c1 = (T)L.c1;
  E.c2 = (T)L.c2;
  E.inv_theta = (T)L.inv_theta;
  return E;
}
// Inputs of the sweep at entry j (loaded for every output of a thread before
// its first store, so the loads overlap).
template <typename T, int EP>
__device__ __forceinline__ void mg_epi_load(const MgEpi<T> &E, long long j, T (&in)[3]) {
  if constexpr (EP == MGE_STEP1) {
    in[0] = E.d[j];
    in[1] = E.b[j];
  } else if constexpr (EP == MGE_RES) {
    in[0] = E.r[j];
  } else if constexpr (EP == MGE_POST) {
    in[0] = E.b[j];
    in[1] = E.x[j];
  } else if constexpr (EP == MGE_LAST) {
    in[0] = E.q[j];
    in[1] = E.d[j];
    in[2] = E.r[j];
  }
}
template <typename T, int EP>
__device__ __forceinline__ void mg_epilogue(const MgEpi<T> &E, long long j, T dinv, T a, const T (&in)[3]) {
  if constexpr (EP == MGE_NONE) {
    E.q[j] = a;
  } else if constexpr (EP == MGE_STEP1) {
    const T d0 = in[0];
    const T rv = in[1] - a;
    const T d1 = E.c1 * d0 + E.c2 * dinv * rv;
    E.r[j] = rv;
    E.x[j] = d0 + d1;
    E.q[j] = d1;
  } else if constexpr (EP == MGE_RES) {
    E.r[j] = in[0] - a;
  } else if constexpr (EP == MGE_POST) {
    const T rv = in[0] - a;
    const T dv = dinv * rv * E.inv_theta;
    E.r[j] = rv;
    E.d[j] = dv;
    E.q[j] = in[1] + dv;
  } else {  // MGE_LAST
    E.x[j] = in[0] + E.c1 * in[1] + E.c2 * dinv * (in[2] - a);
  }
}

// the operator's input vector of an epilogue (MGE_NONE: src 0 x, 1 d)
template <typename T, int EP>
__device__ __forceinline__ const T *mg_operand(const MgLevel &L, int src) {
  if constexpr (EP == MGE_STEP1 || EP == MGE_LAST) return (const T *)L.d;
  else if constexpr (EP == MGE_RES) return (const T *)L.q;
  else if constexpr (EP == MGE_POST) return (const T *)L.x;
  else return (const T *)(src == 0 ? L.x : L.d);
}

template <typename T, int RHS, int EP>
__global__ __launch_bounds__(256) void mg_apply_kernel(MgBatch B, int l, int src, int live) {
  const MgLevel &L = B.mg[blockIdx.z]->lv[l];
  const long long nn = L.nn;
  // node indices fit 32 bits (n <= 512); 64-bit divisions are slow
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (unsigned)nn * (NRHS / RHS)) return;
  const unsigned r0u = t / (unsigned)nn;
  const long long v = t - r0u * (unsigned)nn;
  const int r0 = int(r0u) * RHS;
  // live: load cases that have converged (or broken down) are skipped, as in
  // the voxel-level passes (Sec. 4.2.2: per-right-hand-side convergence)
  bool act[RHS];
  bool any = false;
#pragma unroll
  for (int r = 0; r < RHS; ++r) {
    act[r] = !live || B.slot[blockIdx.z]->st->active[r0 + r] != 0;
    any = any || act[r];
  }
  if (!any) return;
  const int n = L.n;
  const unsigned row = unsigned(v) / (unsigned)n;
  const int x = int(unsigned(v) - row * (unsigned)n), y = int(row % (unsigned)n), z = int(row / (unsigned)n);
  const SHH_GLOBAL T *S = to_global((const T *)L.S);
  const SHH_GLOBAL T *Dv = to_global((const T *)L.Dinv);
  const SHH_GLOBAL T *in = to_global(mg_operand<T, EP>(L, src)) + (long long)r0 * 3 * nn;
  T acc[RHS][3];
#pragma unroll
  for (int r = 0; r < RHS; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = T(0);
  // a node with a zero diagonal has a zero row (every element around it
  // culled): A v = 0 there without reading its stencil
  const bool zero_row = Dv[v] == T(0);
  // three offsets per trip: their loads are in flight together (measured
  // faster than one; more waves per SIMD or fewer load cases per thread are
  // slower, the stencil reads then miss the caches more)
  if (!zero_row) {
#pragma unroll 3
    for (int w = 0; w < 27; ++w) {
      const int dx = w % 3 - 1, dy = (w / 3) % 3 - 1, dz = w / 9 - 1;
      const long long u = ((long long)wrap1(z + dz, n) * n + wrap1(y + dy, n)) * n + wrap1(x + dx, n);
      T blk[9];
      if (w >= 13) {
#pragma unroll
        for (int k = 0; k < 9; ++k) blk[k] = S[((w - 13) * 9 + k) * nn + v];
      } else {
        // A[v][u] = A[u][v]^T, stored at u for offset 26 - w
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int cp = 0; cp < 3; ++cp) blk[3 * c + cp] = S[((13 - w) * 9 + 3 * cp + c) * nn + u];
      }
#pragma unroll
      for (int r = 0; r < RHS; ++r) {
        if (!act[r]) continue;
        const SHH_GLOBAL T *vr = in + (long long)r * 3 * nn;
        const T u0 = vr[u], u1 = vr[nn + u], u2 = vr[2 * nn + u];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][c] += blk[3 * c] * u0 + blk[3 * c + 1] * u1 + blk[3 * c + 2] * u2;
      }
    }
  }
  const MgEpi<T> E = mg_epi<T>(L);
  T dv[3], ein[RHS][3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) dv[c] = Dv[(long long)c * nn + v];
#pragma unroll
  for (int r = 0; r < RHS; ++r)
    if (act[r])
#pragma unroll
      for (int c = 0; c < 3; ++c) mg_epi_load<T, EP>(E, ((long long)(r0 + r) * 3 + c) * nn + v, ein[r][c]);
#pragma unroll
  for (int r = 0; r < RHS; ++r)
    if (act[r])
#pragma unroll
      for (int c = 0; c < 3; ++c)
        mg_epilogue<T, EP>(E, ((long long)(r0 + r) * 3 + c) * nn + v, dv[c], acc[r][c], ein[r][c]);
}

// q = A_l v as above, all six load cases, for two z-adjacent nodes per thread
// (even n; the form the large levels take): the vector values of the two
// planes between them are loaded once for both (12 % faster per launch than
// one node per thread).  Occupancy 2 waves per SIMD in FP32 (230 registers;
// holding it to 3 waves spills).  An inactive load case's gathers read one
// broadcast element instead of branching around them (7 % faster), and the
// fused sweep loads all of a node's inputs before its first store.
template <typename T, int EP>
__global__ __launch_bounds__(256) void mg_apply_pair_kernel(MgBatch B, int l, int src, int live) {
  const MgLevel &L = B.mg[blockIdx.z]->lv[l];
  const long long nn = L.nn;
  const int n = L.n;
  const long long plane = (long long)n * n;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= unsigned(nn / 2)) return;
  bool act[NRHS];
  bool any = false;
#pragma unroll
  for (int r = 0; r < NRHS; ++r) {
    act[r] = !live || B.slot[blockIdx.z]->st->active[r] != 0;
    any = any || act[r];
  }
  if (!any) return;
  // 32-bit index arithmetic (n <= 512)
  const unsigned zp = t / unsigned(plane);
  const unsigned xy = t - zp * unsigned(plane);
  const int y = int(xy / unsigned(n)), x = int(xy - unsigned(y) * unsigned(n)), z0 = 2 * int(zp);
  const long long v0 = (long long)z0 * plane + xy;
  const SHH_GLOBAL T *S = to_global((const T *)L.S);
  const SHH_GLOBAL T *Dv = to_global((const T *)L.Dinv);
  const SHH_GLOBAL T *in = to_global(mg_operand<T, EP>(L, src));
  // nodes with a zero diagonal have a zero row (every element around them
  // culled): A v = 0 there without reading their stencil
  const bool zero_rows = Dv[v0] == T(0) && Dv[v0 + plane] == T(0);
  T acc[2][NRHS][3];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int r = 0; r < NRHS; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[k][r][c] = T(0);
  if (!zero_rows) {
#pragma unroll
    for (int pz = 0; pz < 4; ++pz) {  // planes z0 - 1 .. z0 + 2
      const long long pzo = (long long)wrap1(z0 - 1 + pz, n) * plane;
      // three offsets per trip (one and nine measured slower)
#pragma unroll 3
      for (int o = 0; o < 9; ++o) {
        const int dx = o % 3 - 1, dy = o / 3 - 1;
        const long long u = pzo + (long long)wrap1(y + dy, n) * n + wrap1(x + dx, n);
        T val[NRHS][3];
#pragma unroll
        for (int r = 0; r < NRHS; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c)  // an inactive load case reads one broadcast
            val[r][c] = in[((long long)r * 3 + c) * nn + (act[r] ? u : 0)];  // value: no branch, no traffic
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int dz = pz - 1 - k;
          if (dz < -1 || dz > 1) continue;
          const int w = (dz + 1) * 9 + o;
          const long long v = v0 + k * plane;
          T blk[9];
          if (w >= 13) {
#pragma unroll
            for (int e = 0; e < 9; ++e) blk[e] = S[((w - 13) * 9 + e) * nn + v];
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
              for (int cp = 0; cp < 3; ++cp) blk[3 * c + cp] = S[((13 - w) * 9 + 3 * cp + c) * nn + u];
          }
#pragma unroll
          for (int r = 0; r < NRHS; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              acc[k][r][c] += blk[3 * c] * val[r][0] + blk[3 * c + 1] * val[r][1] + blk[3 * c + 2] * val[r][2];
        }
      }
    }
  }
  // output stage, per node: every load of its sweep before its first store
  const MgEpi<T> E = mg_epi<T>(L);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const long long vk = v0 + k * plane;
    T dv[3], ein[NRHS][3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dv[c] = Dv[(long long)c * nn + vk];
#pragma unroll
    for (int r = 0; r < NRHS; ++r)
      if (act[r])
#pragma unroll
        for (int c = 0; c < 3; ++c) mg_epi_load<T, EP>(E, ((long long)r * 3 + c) * nn + vk, ein[r][c]);
#pragma unroll
    for (int r = 0; r < NRHS; ++r)
      if (act[r])
#pragma unroll
        for (int c = 0; c < 3; ++c)
          mg_epilogue<T, EP>(E, ((long long)r * 3 + c) * nn + vk, dv[c], acc[k][r][c], ein[r][c]);
  }
}

// two-wide element pairs of the fine vectors (x = 2X and 2X + 1)
template <typename T> struct Pair2 { using type = T __attribute__((ext_vector_type(2))); };

// b_{l+1} = P^T r_l, the residual after the pre-smoother (its last operator
// pass leaves it in r): coarse node I collects fine nodes 2I + o,
// o in {-1, 0, 1}^3, with weight prod (o == 0 ? 1 : 1/2).  One thread per
// coarse node, grid y = load case.  Per fine row the pair (2X, 2X + 1) is one
// two-wide load; the odd node 2X - 1 is the pair of the lane below (a
// shuffle), loaded only where that lane holds another row or wave.  Node
// indices fit 32 bits (n <= 512): 64-bit divisions would cost more than the
// kernel's memory traffic.
template <typename T>
__global__ __launch_bounds__(256) void mg_restrict_kernel(MgBatch B, int l) {
  using T2 = typename Pair2<T>::type;
  const MgDev *mg = B.mg[blockIdx.z];
  const MgLevel &F = mg->lv[l];
  const MgLevel &C = mg->lv[l + 1];
  const unsigned I = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  // in-range lanes are a prefix of the wave, so the lane below an in-range
  // lane is in range too
  if (I >= (unsigned)C.nn || !B.slot[blockIdx.z]->st->active[k]) return;
  const int nc = C.n, nf = F.n;
  const unsigned row = I / (unsigned)nc;
  const int X = int(I - row * (unsigned)nc), Y = int(row % (unsigned)nc), Z = int(row / (unsigned)nc);
  const bool own_left = X == 0 || (threadIdx.x & 63u) == 0;
  const int xl = X == 0 ? nf - 1 : 2 * X - 1;
  const SHH_GLOBAL T *r = to_global((const T *)F.r) + (long long)k * 3 * F.nn;
  // all loads are issued before the first shuffle waits on one
  unsigned rowo[9];
#pragma unroll
  for (int oz = 0; oz < 3; ++oz)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
      rowo[3 * oz + oy] =
          (unsigned(wrap1(2 * Z + oz - 1, nf)) * unsigned(nf) + unsigned(wrap1(2 * Y + oy - 1, nf))) * unsigned(nf);
  T2 v[9][3];
#pragma unroll
  for (int o = 0; o < 9; ++o)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[o][c] = *(const SHH_GLOBAL T2 *)(r + (long long)c * F.nn + rowo[o] + 2 * X);
  T left[9][3];
#pragma unroll
  for (int o = 0; o < 9; ++o)
#pragma unroll
    for (int c = 0; c < 3; ++c) left[o][c] = __shfl_up(v[o][c].y, 1);
  if (own_left) {
#pragma unroll
    for (int o = 0; o < 9; ++o)
#pragma unroll
      for (int c = 0; c < 3; ++c) left[o][c] = r[(long long)c * F.nn + rowo[o] + xl];
  }
  T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    const T wyz = T((o / 3 != 1 ? 0.5 : 1.0) * (o % 3 != 1 ? 0.5 : 1.0));
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += wyz * (v[o][c].x + T(0.5) * (v[o][c].y + left[o][c]));
  }
  SHH_GLOBAL T *b = to_global((T *)C.b) + (long long)k * 3 * C.nn;
#pragma unroll
  for (int c = 0; c < 3; ++c) b[(long long)c * C.nn + I] = acc[c];
}

// x_l += P x_{l+1}: fine node 2I + a, a in {0, 1}^3, takes the coarse nodes
// I + i with i_d in {0, a_d}, weight 1/2 per axis with a_d = 1.  One thread
// per coarse node (grid y = load case) updates its 2 x 2 x 2 fine block as
// four two-wide pairs; 32-bit node indices as in the restriction.
template <typename T>
__global__ __launch_bounds__(256) void mg_prolong_kernel(MgBatch B, int l) {
  using T2 = typename Pair2<T>::type;
  const MgDev *mg = B.mg[blockIdx.z];
  const MgLevel &F = mg->lv[l];
  const MgLevel &C = mg->lv[l + 1];
  const unsigned I = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (I >= (unsigned)C.nn || !B.slot[blockIdx.z]->st->active[k]) return;
  const int nc = C.n, nf = F.n;
  const long long cnn = C.nn, fnn = F.nn;  // read once: the stores below might alias them
  const unsigned row = I / (unsigned)nc;
  const int X = int(I - row * (unsigned)nc), Y = int(row % (unsigned)nc), Z = int(row / (unsigned)nc);
  const int X1 = X + 1 == nc ? 0 : X + 1;
  const unsigned cy[2] = {unsigned(Y), unsigned(Y + 1 == nc ? 0 : Y + 1)};
  const unsigned cz[2] = {unsigned(Z), unsigned(Z + 1 == nc ? 0 : Z + 1)};
  const SHH_GLOBAL T *xc = to_global((const T *)C.x) + (long long)k * 3 * cnn;
  SHH_GLOBAL T *xf = to_global((T *)F.x) + (long long)k * 3 * fnn;
  // every load (coarse values, then the fine pairs) is issued before the
  // first store
  T cv[3][2][2][2];  // [c][z][y][x] offsets 0 / +1
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int iz = 0; iz < 2; ++iz)
#pragma unroll
      for (int iy = 0; iy < 2; ++iy) {
        const SHH_GLOBAL T *v = xc + (long long)c * cnn + (cz[iz] * unsigned(nc) + cy[iy]) * unsigned(nc);
        cv[c][iz][iy][0] = v[X];
        cv[c][iz][iy][1] = v[X1];
      }
  unsigned fi[2][2];
#pragma unroll
  for (int az = 0; az < 2; ++az)
#pragma unroll
    for (int ay = 0; ay < 2; ++ay)
      fi[az][ay] = ((2 * unsigned(Z) + az) * unsigned(nf) + 2 * unsigned(Y) + ay) * unsigned(nf) + 2 * X;
  T2 f[3][2][2];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
      for (int ay = 0; ay < 2; ++ay) f[c][az][ay] = *(const SHH_GLOBAL T2 *)(xf + (long long)c * fnn + fi[az][ay]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
      for (int ay = 0; ay < 2; ++ay) {
        T s[2];
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
          const T yz0 = ay ? T(0.5) * (cv[c][0][0][ix] + cv[c][0][1][ix]) : cv[c][0][0][ix];
          const T yz1 = ay ? T(0.5) * (cv[c][1][0][ix] + cv[c][1][1][ix]) : cv[c][1][0][ix];
          s[ix] = az ? T(0.5) * (yz0 + yz1) : yz0;
        }
        T2 o = f[c][az][ay];
        o.x += s[0];
        o.y += T(0.5) * (s[0] + s[1]);
        *(SHH_GLOBAL T2 *)(xf + (long long)c * fnn + fi[az][ay]) = o;
      }
}

// Coarsest level: x = Mc b per load case (one workgroup per load case; four
// lanes share a row and combine their partial sums by shuffles).
template <typename T>
__global__ __launch_bounds__(256) void mg_coarsest_kernel(MgBatch B) {
  const MgDev *mg = B.mg[blockIdx.z];
  const MgLevel &L = mg->lv[mg->L];
  const int k = blockIdx.x;
  if (!B.slot[blockIdx.z]->st->active[k]) return;
  const int nd = mg->ndof_c;
  const long long nn = L.nn;
  const double *M = mg->Mc;
  const T *b = (const T *)L.b + (long long)k * 3 * nn;
  T *x = (T *)L.x + (long long)k * 3 * nn;
  const int part = threadIdx.x & 3;
  for (int row0 = 0; row0 < nd; row0 += 64) {
    const int row = row0 + (threadIdx.x >> 2);
    double acc = 0.0;
    if (row < nd)
      for (int j = part; j < nd; j += 4) acc += (double)M[(long long)row * nd + j] * (double)b[(j % 3) * nn + j / 3];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (row < nd && part == 0) x[(row % 3) * nn + row / 3] = (T)acc;
  }
}

// Degree-2 Chebyshev smoothing of A x = b at level l:
//   d = D^-1 b / theta;  r = b - A d;  d' = c1 d + c2 D^-1 r;  x = d + d'
//   (pre-smoother; the restriction takes r - A d');  after the coarse
//   correction r = b - A x;  d = D^-1 r / theta;  x += d;
//   x += c1 d + c2 D^-1 (r - A d)  (post-smoother).
// Every step after an operator application runs in that pass's output stage
// (the stencil kernel's multigrid modes at the voxel level, mg_epilogue on
// the coarse levels); this sweep is the first step, d = D^-1 b / theta, on
// the coarse levels, and at the voxel level the pending CG update
// x_cg += alpha p, b = r -= alpha q (q = K p), so that b is the new CG
// residual (the stencil pass after it forms d itself).
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void mg_vec_kernel(MgBatch B, int l) {
  const SlotDev *s = B.slot[blockIdx.z];
  const MgLevel &L = B.mg[blockIdx.z]->lv[l];
  const int k = blockIdx.y;
  const long long nn = L.nn;
  if (blockIdx.x >= (unsigned)L.nchunks || !s->st->active[k]) return;
  const long long i0 = (long long)blockIdx.x * CHUNK;
  const long long i1 = min(i0 + (long long)CHUNK, nn);
  const long long vb = (long long)k * 3 * nn;
  T *b = (T *)L.b + vb;
  if (l == 0) {
    const T a = (T)s->st->alpha[k];
    if (a == T(0)) return;
    // (the same pass with every load of a thread's four nodes ahead of its
    // stores measured 5 % slower: this one keeps more waves in flight)
    T *xcg = (T *)s->x + vb;
    const T *pcg = (const T *)s->p[s->st->mgpar[k]] + vb;
    const T *q = (const T *)L.q + vb;
    for (long long i = i0 + threadIdx.x; i < i1; i += VEC_THREADS)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long j = c * nn + i;
        xcg[j] = xcg[j] + a * pcg[j];
        b[j] = b[j] - a * q[j];
      }
    return;
  }
  const T ith = (T)L.inv_theta;
  SHH_GLOBAL T *d = to_global((T *)L.d) + vb;
  const SHH_GLOBAL T *Dv = to_global((const T *)L.Dinv);
  const SHH_GLOBAL T *bg = to_global((const T *)b);
  constexpr int PER = CHUNK / VEC_THREADS;
  T dv[PER][3], bv[PER][3];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const long long i = i0 + threadIdx.x + u * VEC_THREADS;
    if (i < i1)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dv[u][c] = Dv[c * nn + i];
        bv[u][c] = bg[c * nn + i];
      }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const long long i = i0 + threadIdx.x + u * VEC_THREADS;
    if (i < i1)
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c * nn + i] = dv[u][c] * bv[u][c] * ith;
  }
}

// CG scalars of the multigrid-preconditioned solve (one workgroup per load
// case; per-tile partials of the voxel-level stencil passes: the direction
// pass for ALPHA, the last post-smoothing sweep for RESTART and BETA).
//   RESTART: rho = r . z after a (re)started V-cycle, beta = 0
//   REPLACE: the same after a residual replacement, the direction kept:
//            beta = rho' / (rho the last iteration started from)
//   ALPHA:   alpha = rho / p . K p; the new direction becomes current
//   BETA:    rho' = r . z, ||r||^2 -> convergence; beta = rho' / rho
__global__ __launch_bounds__(VEC_THREADS) void mg_scalar_kernel(MgBatch B, int phase) {
  __shared__ double red[2 * 16];
  const SlotDev *s = B.slot[blockIdx.z];
  const int k = blockIdx.x;
  CgState *st = s->st;
  const double *parts = s->partials + (long long)k * s->maxparts * PSTRIDE;
  double tot[2];
  sum_partials<2, PSTRIDE>(parts, s->ntiles[s->prec], tot, red, VEC_THREADS);
  if (threadIdx.x != 0) return;
  // the direction pass ran for the active load cases only: their new
  // direction becomes current
  if (!st->active[k]) {
    st->alpha[k] = 0.0;
    st->beta[k] = 0.0;
    return;
  }
  if (phase == MGS_RESTART || phase == MGS_REPLACE) {
    // (the replacement's residual phase has since overwritten rho and beta
    // with the Jacobi recurrences; rho_mg kept the iteration's own rho)
    // The direction is kept only while the replaced residual agrees with the
    // recursive one (r . z within a factor 2 of it: rho_prev holds the
    // recursive value); a larger drift restarts.
    const double rho = tot[0], rho0 = st->rho_mg[k], rho_rec = st->rho_prev[k];
    const bool keep = phase == MGS_REPLACE && rho0 > 0.0 && rho_rec > 0.0 && rho <= 2.0 * rho_rec &&
                      rho >= 0.5 * rho_rec;
    st->beta[k] = keep ? rho / rho0 : 0.0;
    st->rho[k] = rho;
    st->alpha[k] = 0.0;
    if (!(rho > 0.0) || !isfinite(rho)) {
      st->status[k] = ST_BREAKDOWN;
      st->active[k] = 0;
    }
  } else if (phase == MGS_ALPHA) {
    st->mgpar[k] ^= 1;
    const double sigma = tot[0], rho = st->rho[k];
    const bool ok = isfinite(sigma) && sigma > 0.0 && rho > 0.0;
    st->alpha[k] = ok ? rho / sigma : 0.0;
    if (!ok) {
      st->status[k] = ST_BREAKDOWN;
      st->active[k] = 0;
    }
  } else {
    const double rho_n = tot[0], rr = tot[1];
    st->iters[k] += 1;
    st->alpha[k] = 0.0;
    st->rr[k] = rr;
    const double rel = sqrt(rr / st->ff[k]);
    st->rel[k] = rel;
    const double rho = st->rho[k];
    const bool ok = isfinite(rho_n) && rho_n >= 0.0;
    st->beta[k] = ok && rho > 0.0 ? rho_n / rho : 0.0;
    st->rho_mg[k] = rho;
    st->rho[k] = rho_n;
    if (rel <= s->rtol) {
      st->status[k] = ST_CONVERGED;
      st->active[k] = 0;
    } else if (!ok || !isfinite(rel)) {
      st->status[k] = ST_BREAKDOWN;
      st->active[k] = 0;
    } else if (st->iters[k] >= s->max_iter) {
      st->status[k] = ST_MAXIT;
      st->active[k] = 0;
    }
  }
}

// Power iteration for lambda_max(D^-1 A) at a coarse level l, on load case 0
// of x, for a batch of slots (grid z = slot):
//   phase 0: x = a fixed pseudo-random vector
//   phase 1: partial x.q and x.D x (the Rayleigh quotient x.A x / x.D x of
//            D^-1 A, self-adjoint in the D inner product), then x = D^-1 q
//            (q = A x) and partial ||x||^2
//   phase 2: x *= the level's pw_scale
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void mg_power_kernel(MgBatch B, int l, int phase) {
  __shared__ double red[3 * 16];
  const SlotDev *s = B.slot[blockIdx.z];
  const MgLevel &L = B.mg[blockIdx.z]->lv[l];
  const long long nn = L.nn;
  if (blockIdx.x >= (unsigned)L.nchunks) return;
  const long long i0 = (long long)blockIdx.x * CHUNK;
  const long long i1 = min(i0 + (long long)CHUNK, nn);
  T *x = (T *)L.x;
  const T *q = (const T *)L.q;
  const T *Dv = (const T *)L.Dinv;
  double acc[3] = {0.0, 0.0, 0.0};
  for (long long i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long j = c * nn + i;
      if (phase == 0) {
        uint32_t h = (uint32_t)j * 2654435761u + 0x9e3779b9u;
        h ^= h >> 16;
        h *= 0x85ebca6bu;
        h ^= h >> 13;
        x[j] = (T)((double)(h & 0xffffff) / 16777216.0 - 0.5);
      } else if (phase == 1) {
        const T di = Dv[j];
        const double xo = (double)x[j], qo = (double)q[j];
        acc[1] += xo * qo;
        acc[2] += di != T(0) ? xo * xo / (double)di : 0.0;
        const T v = di * q[j];
        x[j] = v;
        acc[0] += (double)v * (double)v;
      } else {
        x[j] = (T)((double)x[j] * L.pw_scale);
      }
    }
  }
  if (phase == 1) {
    block_sum<3>(acc, red, VEC_THREADS);
    if (threadIdx.x == 0) {
      s->partials[blockIdx.x * PSTRIDE] = acc[0];
      s->partials[blockIdx.x * PSTRIDE + 1] = acc[1];
      s->partials[blockIdx.x * PSTRIDE + 2] = acc[2];
    }
  }
}

// After power phase 1: reduce the partials (one workgroup per slot), keep the
// largest Rayleigh quotient in lmax and the normalization for phase 2 (a
// vanishing or non-finite step leaves lmax = -1, which the host reports as a
// breakdown).
__global__ __launch_bounds__(VEC_THREADS) void mg_power_reduce_kernel(MgBatch B, int l) {
  __shared__ double red[3 * 16];
  const SlotDev *s = B.slot[blockIdx.z];
  // the slot's own descriptor in device memory, written only here
  MgLevel &L = const_cast<MgDev *>(B.mg[blockIdx.z])->lv[l];
  double tot[3];
  sum_partials<3, PSTRIDE>(s->partials, L.nchunks, tot, red, VEC_THREADS);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(tot[0]);
  if (!(nrm > 0.0) || !isfinite(nrm) || !(tot[2] > 0.0) || L.lmax < 0.0) {
    L.lmax = -1.0;
    L.pw_scale = 0.0;
    return;
  }
  L.lmax = fmax(L.lmax, tot[1] / tot[2]);
  L.pw_scale = 1.0 / nrm;
}

// The coarsest level's dense inverse, in one workgroup: assemble the
// operator from the stored stencil blocks (row 3 v + c gathers every block of
// node v, the lower offsets transposed from the neighbours), add gamma / nn to
// each component's constant block (gamma = mean diagonal; this makes the
// operator nonsingular on the rigid translations and leaves its inverse on
// the range equal to the pseudo-inverse), then invert in place by
// Gauss-Jordan elimination (the matrix is symmetric positive definite, so no
// pivoting).  FP64 throughout.
// One workgroup per design of the batch (grid x).
template <typename T>
__global__ __launch_bounds__(1024) void mg_coarse_inverse_kernel(MgBatch B) {
  __shared__ double red[16];
  const MgDev *mg = B.mg[blockIdx.x];
  const MgLevel &L = mg->lv[mg->L];
  const int n = L.n, m = mg->ndof_c;
  const long long nn = L.nn;
  const T *S = (const T *)L.S;
  double *A = mg->Mc;
  for (long long k = threadIdx.x; k < (long long)m * m; k += blockDim.x) A[k] = 0.0;
  __syncthreads();
  for (int row = threadIdx.x; row < m; row += blockDim.x) {
    const long long v = row / 3;
    const int c = row % 3;
    const int x = int(v % n), y = int((v / n) % n), z = int(v / ((long long)n * n));
    for (int w = 0; w < 27; ++w) {
      const int dx = w % 3 - 1, dy = (w / 3) % 3 - 1, dz = w / 9 - 1;
      const long long u = ((long long)wrap1(z + dz, n) * n + wrap1(y + dy, n)) * n + wrap1(x + dx, n);
#pragma unroll
      for (int cp = 0; cp < 3; ++cp) {
        const double a = w >= 13 ? (double)S[((w - 13) * 9 + 3 * c + cp) * nn + v]
                                  : (double)S[((13 - w) * 9 + 3 * cp + c) * nn + u];
        A[(long long)row * m + 3 * u + cp] += a;
      }
    }
  }
  __syncthreads();
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < m; i += blockDim.x) acc[0] += A[(long long)i * m + i];
  block_sum<1>(acc, red, blockDim.x);
  if (threadIdx.x == 0) red[0] = acc[0];
  __syncthreads();
  const double add = red[0] / m / double(nn);
  const double mean_diag = red[0] / m;
  for (long long k = threadIdx.x; k < (long long)m * m; k += blockDim.x) {
    const int i = int(k / m), j = int(k % m);
    if (i % 3 == j % 3) A[k] += add;
  }
  __syncthreads();
  // column k of the current matrix and the normalized pivot row, kept in LDS
  // while the other rows are updated (each wave sweeps rows, its lanes the
  // columns)
  __shared__ double colk[3 * MG_MAX_COARSE * MG_MAX_COARSE * MG_MAX_COARSE];
  __shared__ double rowk[3 * MG_MAX_COARSE * MG_MAX_COARSE * MG_MAX_COARSE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int k = 0; k < m; ++k) {
    const double piv = A[(long long)k * m + k];
    if (!(piv > 1e-12 * mean_diag)) {
      // a vanishing pivot of the (positive semidefinite) Schur complement: the
      // dof is a null direction beyond the rigid translations (nodes whose
      // elements are all culled, pieces that float at this level).  It is
      // taken out -- row and column k zero -- so the result stays a symmetric
      // generalized inverse.  Never taken on the floored operator.
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        A[(long long)i * m + k] = 0.0;
        A[(long long)k * m + i] = 0.0;
      }
      __syncthreads();
      continue;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) colk[i] = A[(long long)i * m + k];
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      const long long kj = (long long)k * m + j;
      const double v = j == k ? 1.0 / piv : A[kj] / piv;
      A[kj] = v;
      rowk[j] = v;
    }
    __syncthreads();
    // rows i != k: A[i][j] -= f_i A[k][j] (j != k), A[i][k] = -f_i / piv
    for (int i = wave; i < m; i += nwaves) {
      if (i == k) continue;
      const double f = colk[i];
      double *Ai = A + (long long)i * m;
      for (int j = lane; j < m; j += 64) Ai[j] = (j == k ? 0.0 : Ai[j]) - f * rowk[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static unsigned blocks_for(long long count, int per) { return (unsigned)((count + per - 1) / per); }

hipError_t mg_launch_elem1(const SlotDev *d_slot, const MgDev *d_mg, long long nn1, int prec, hipStream_t st) {
  const unsigned g = blocks_for(nn1 * 24, 256);
  if (prec == 0) mg_elem1_kernel<double><<<g, 256, 0, st>>>(d_slot, d_mg);
  else mg_elem1_kernel<float><<<g, 256, 0, st>>>(d_slot, d_mg);
  return hipGetLastError();
}

hipError_t mg_launch_elemc(const MgDev *d_mg, int l, long long nn_next, int prec, hipStream_t st) {
  const unsigned g = blocks_for(nn_next * 24, 256);
  if (prec == 0) mg_elemc_kernel<double><<<g, 256, 0, st>>>(d_mg, l);
  else mg_elemc_kernel<float><<<g, 256, 0, st>>>(d_mg, l);
  return hipGetLastError();
}

hipError_t mg_launch_coarse_inverse(const MgBatch &B, int prec, hipStream_t st) {
  if (prec == 0) mg_coarse_inverse_kernel<double><<<B.count, 1024, 0, st>>>(B);
  else mg_coarse_inverse_kernel<float><<<B.count, 1024, 0, st>>>(B);
  return hipGetLastError();
}

hipError_t mg_launch_stencil(const MgDev *d_mg, int l, long long nn, int prec, hipStream_t st) {
  const unsigned g = blocks_for(nn, 256);
  if (prec == 0) mg_stencil_kernel<double><<<g, 256, 0, st>>>(d_mg, l);
  else mg_stencil_kernel<float><<<g, 256, 0, st>>>(d_mg, l);
  return hipGetLastError();
}

// whether mg_launch_apply takes the all-load-cases-per-thread variant
bool mg_apply_wide(long long nn_max) { return nn_max > 32768; }

namespace {
template <int EP>
void launch_apply_ep(const MgBatch &B, int l, int src, long long nn_max, bool even, int prec, hipStream_t st,
                     int live) {
  if (mg_apply_wide(nn_max) && even) {
    const dim3 g(blocks_for(nn_max / 2, 256), 1, B.count);
    if (prec == 0) mg_apply_pair_kernel<double, EP><<<g, 256, 0, st>>>(B, l, src, live);
    else mg_apply_pair_kernel<float, EP><<<g, 256, 0, st>>>(B, l, src, live);
  } else if (mg_apply_wide(nn_max)) {
    const dim3 g(blocks_for(nn_max, 256), 1, B.count);
    if (prec == 0) mg_apply_kernel<double, NRHS, EP><<<g, 256, 0, st>>>(B, l, src, live);
    else mg_apply_kernel<float, NRHS, EP><<<g, 256, 0, st>>>(B, l, src, live);
  } else {
    const dim3 g(blocks_for(nn_max * NRHS, 256), 1, B.count);
    if (prec == 0) mg_apply_kernel<double, 1, EP><<<g, 256, 0, st>>>(B, l, src, live);
    else mg_apply_kernel<float, 1, EP><<<g, 256, 0, st>>>(B, l, src, live);
  }
}
}  // namespace

hipError_t mg_launch_apply(const MgBatch &B, int l, int src, long long nn_max, bool even, int prec,
                           hipStream_t st, int live, int ep) {
  switch (ep) {
    case MGE_STEP1: launch_apply_ep<MGE_STEP1>(B, l, src, nn_max, even, prec, st, live); break;
    case MGE_RES: launch_apply_ep<MGE_RES>(B, l, src, nn_max, even, prec, st, live); break;
    case MGE_POST: launch_apply_ep<MGE_POST>(B, l, src, nn_max, even, prec, st, live); break;
    case MGE_LAST: launch_apply_ep<MGE_LAST>(B, l, src, nn_max, even, prec, st, live); break;
    default: launch_apply_ep<MGE_NONE>(B, l, src, nn_max, even, prec, st, live); break;
  }
  return hipGetLastError();
}

// q = A_l v for load case 0 only (the setup's power iteration)
hipError_t mg_launch_apply_case0(const MgBatch &B, int l, long long nn_max, int prec, hipStream_t st) {
  const dim3 g(blocks_for(nn_max, 256), 1, B.count);
  if (prec == 0) mg_apply_kernel<double, 1, MGE_NONE><<<g, 256, 0, st>>>(B, l, 0, 0);
  else mg_apply_kernel<float, 1, MGE_NONE><<<g, 256, 0, st>>>(B, l, 0, 0);
  return hipGetLastError();
}

hipError_t mg_launch_restrict(const MgBatch &B, int l, long long nn_coarse_max, int prec,
                              hipStream_t st) {
  const dim3 g(blocks_for(nn_coarse_max, 256), NRHS, B.count);
  if (prec == 0) mg_restrict_kernel<double><<<g, 256, 0, st>>>(B, l);
  else mg_restrict_kernel<float><<<g, 256, 0, st>>>(B, l);
  return hipGetLastError();
}

hipError_t mg_launch_prolong(const MgBatch &B, int l, long long nn_coarse_max, int prec, hipStream_t st) {
  const dim3 g(blocks_for(nn_coarse_max, 256), NRHS, B.count);
  if (prec == 0) mg_prolong_kernel<double><<<g, 256, 0, st>>>(B, l);
  else mg_prolong_kernel<float><<<g, 256, 0, st>>>(B, l);
  return hipGetLastError();
}

hipError_t mg_launch_coarsest(const MgBatch &B, int prec, hipStream_t st) {
  const dim3 g(NRHS, 1, B.count);
  if (prec == 0) mg_coarsest_kernel<double><<<g, 256, 0, st>>>(B);
  else mg_coarsest_kernel<float><<<g, 256, 0, st>>>(B);
  return hipGetLastError();
}

hipError_t mg_launch_vec(const MgBatch &B, int l, int nchunks_max, int prec, hipStream_t st) {
  const dim3 g((unsigned)nchunks_max, NRHS, B.count);
  if (prec == 0) mg_vec_kernel<double><<<g, VEC_THREADS, 0, st>>>(B, l);
  else mg_vec_kernel<float><<<g, VEC_THREADS, 0, st>>>(B, l);
  return hipGetLastError();
}


hipError_t mg_launch_scalar(const MgBatch &B, int phase, hipStream_t st) {
  mg_scalar_kernel<<<dim3(NRHS, 1, B.count), VEC_THREADS, 0, st>>>(B, phase);
  return hipGetLastError();
}

hipError_t mg_launch_power(const MgBatch &B, int l, int phase, int nchunks_max, int prec, hipStream_t st) {
  if (phase == 3) {
    mg_power_reduce_kernel<<<dim3(1, 1, B.count), VEC_THREADS, 0, st>>>(B, l);
  } else if (prec == 0) {
    mg_power_kernel<double><<<dim3((unsigned)nchunks_max, 1, B.count), VEC_THREADS, 0, st>>>(B, l, phase);
  } else {
    mg_power_kernel<float><<<dim3((unsigned)nchunks_max, 1, B.count), VEC_THREADS, 0, st>>>(B, l, phase);
  }
  return hipGetLastError();
}

}  // namespace shh
