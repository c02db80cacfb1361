// Kernels of the selective (active-set) solve: compaction of the active nodes,
// the node-centric operator on the compact lists, and the CG vector and scalar
// phases.  See sel.hpp for the layout and the operator's construction.
#include "hexop.hpp"
#include "sel.hpp"

namespace shh {

namespace {

__device__ __forceinline__ int wrap_dec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int n) { return v + 1 == n ? 0 : v + 1; }

// Vectors are node-major: the 18 values (load case k, component c at 3 k + c)
// of one node are contiguous, so a neighbour's values come in nine 8- or
// 16-byte loads (the row of node j starts at 72 j or 144 j bytes).
template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

template <typename TV, typename TE>
__device__ __forceinline__ void load_row(const TV *u, long long j, TE (&v)[3 * NRHS]) {
  using P2 = typename Pair<TV>::type;
  const P2 *p = reinterpret_cast<const P2 *>(u + j * (3 * NRHS));
#pragma unroll
  for (int t = 0; t < 3 * NRHS / 2; ++t) {
    const P2 w = p[t];
    v[2 * t] = (TE)w.x;
    v[2 * t + 1] = (TE)w.y;
  }
}

template <typename TV, typename TE>
__device__ __forceinline__ void store_row(TV *u, long long j, const TE (&v)[3 * NRHS]) {
  using P2 = typename Pair<TV>::type;
  P2 *p = reinterpret_cast<P2 *>(u + j * (3 * NRHS));
#pragma unroll
  for (int t = 0; t < 3 * NRHS / 2; ++t) {
    P2 w;
    w.x = (TV)v[2 * t];
    w.y = (TV)v[2 * t + 1];
    p[t] = w;
  }
}

// node (x, y, z) is active if one of the eight voxels it is a corner of --
// lower corners (x - ax, y - ay, z - az) -- carries stiffness
__device__ __forceinline__ bool node_active(const double *E, int n, int x, int y, int z) {
  const int xm = wrap_dec(x, n), ym = wrap_dec(y, n), zm = wrap_dec(z, n);
  const long long n2 = (long long)n * n;
  const long long z0 = (long long)z * n2, z1 = (long long)zm * n2;
  const long long y0 = (long long)y * n, y1 = (long long)ym * n;
  return E[z0 + y0 + x] > 0.0 || E[z0 + y0 + xm] > 0.0 || E[z0 + y1 + x] > 0.0 || E[z0 + y1 + xm] > 0.0 ||
         E[z1 + y0 + x] > 0.0 || E[z1 + y0 + xm] > 0.0 || E[z1 + y1 + x] > 0.0 || E[z1 + y1 + xm] > 0.0;
}

// exclusive prefix sum over the 256 threads of a workgroup
__device__ __forceinline__ int block_exclusive_scan(int v, int *s, int *total) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < SEL_THREADS; off <<= 1) {
    const int add = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const int incl = s[t];
  if (total) *total = s[SEL_THREADS - 1];
  __syncthreads();
  return incl - v;
}

}  // namespace

// ---- compaction ---------------------------------------------------------------
// Chunk b covers grid nodes [b * 1024, (b + 1) * 1024), four consecutive nodes
// per thread; nodes keep their linear (z, y, x) order.
__global__ __launch_bounds__(SEL_THREADS) void sel_count_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nchunks) return;
  __shared__ int s[SEL_THREADS];
  const int n = S->n;
  const long long nn = S->nn;
  int cnt = 0;
  const long long base = (long long)blockIdx.x * SEL_CHUNK + 4 * threadIdx.x;
  for (int j = 0; j < 4; ++j) {
    const long long i = base + j;
    if (i < nn) {
      const int x = int(i % n), y = int((i / n) % n), z = int(i / ((long long)n * n));
      cnt += node_active(S->E64, n, x, y, z) ? 1 : 0;
    }
  }
  int total;
  block_exclusive_scan(cnt, s, &total);
  if (threadIdx.x == 0) S->counts[blockIdx.x] = total;
}

// exclusive offsets of the chunk counts (one workgroup of 1024 threads, each
// summing a contiguous run); counts[nchunks] receives the total
__global__ __launch_bounds__(1024) void sel_scan_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  __shared__ long long s[1024];
  const int nc = S->nchunks;
  const int per = (nc + 1023) / 1024;
  const int lo = threadIdx.x * per, hi = min(lo + per, nc);
  long long sum = 0;
  for (int b = lo; b < hi; ++b) sum += S->counts[b];
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  long long run = s[threadIdx.x] - sum;
  for (int b = lo; b < hi; ++b) {
    const int c = S->counts[b];
    S->counts[b] = int(run);
    run += c;
  }
  if (threadIdx.x == 1023) S->counts[nc] = int(s[1023]);
}

__global__ __launch_bounds__(SEL_THREADS) void sel_write_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nchunks) return;
  __shared__ int s[SEL_THREADS];
  const int n = S->n;
  const long long nn = S->nn;
  const long long base = (long long)blockIdx.x * SEL_CHUNK + 4 * threadIdx.x;
  bool act[4];
  int cnt = 0;
  for (int j = 0; j < 4; ++j) {
    const long long i = base + j;
    act[j] = false;
    if (i < nn) {
      const int x = int(i % n), y = int((i / n) % n), z = int(i / ((long long)n * n));
      act[j] = node_active(S->E64, n, x, y, z);
    }
    cnt += act[j] ? 1 : 0;
  }
  int idx = S->counts[blockIdx.x] + block_exclusive_scan(cnt, s, nullptr);
  for (int j = 0; j < 4; ++j) {
    const long long i = base + j;
    if (i >= nn) break;
    if (act[j]) {
      const int x = int(i % n), y = int((i / n) % n), z = int(i / ((long long)n * n));
      S->map[i] = idx;
      S->coord[idx] = ((unsigned)z << 20) | ((unsigned)y << 10) | (unsigned)x;
      ++idx;
    } else {
      S->map[i] = -1;
    }
  }
}

// moduli and Jacobi diagonal on the compact list
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_gather_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int n = S->n, na = S->na;
  const double c = (S->lam + 4.0 * S->mu) / 9.0;
  const double *E = S->E64;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    const unsigned cd = S->coord[i];
    const int x = int(cd & 1023u), y = int((cd >> 10) & 1023u), z = int(cd >> 20);
    const int xm = wrap_dec(x, n), ym = wrap_dec(y, n), zm = wrap_dec(z, n);
    auto at = [&](int a, int b, int cc) { return E[((long long)cc * n + b) * n + a]; };
    const double e = at(x, y, z);
    const double sum = ((e + at(xm, y, z)) + (at(x, ym, z) + at(xm, ym, z))) +
                       ((at(x, y, zm) + at(xm, y, zm)) + (at(x, ym, zm) + at(xm, ym, zm)));
    ((T *)S->Ec)[i] = (T)e;
    S->Ec64[i] = e;
    ((T *)S->Dinv)[i] = (T)(1.0 / (c * sum));
  }
}

// ---- the node-centric operator ------------------------------------------------
// Block A(r) of the row of node i for the neighbour at offset r, from the
// moduli E[a] of the eight elements around i (element with lower corner i - a,
// a = ax + 2 ay + 4 az).  Element a contains both nodes when a_d = 0 for
// r_d = +1, a_d = 1 for r_d = -1 (either for r_d = 0).  The integrals of the
// trilinear shape functions give, per axis, 1/3 (same corner) or 1/6 (other
// corner) for the mass factor, +1 / -1 for the stiffness factor, and +-1/2
// for the mixed factor, whose sign is -1 at corner 0 and +1 at corner 1.
// Hence:
//   A_cc  = [(lam + mu) T_c + mu (T_x + T_y + T_z)] * sum_shared E
//   A_cc' = (1/4) M_d * { -(lam + mu) r_c r_c' sumE       both axes move
//                         (lam - mu) r_c' D_c              c free, c' moves
//                         (mu - lam) r_c D_c'              c moves, c' free
//                         (lam + mu) D_cc' }               both free
// with T_c = S_c prod_{d != c} M_d, d the third axis, D_c the sum over the
// shared elements of E times sigma_c (+1 where a_c = 1, -1 where a_c = 0).
template <int RX, int RY, int RZ, typename TE>
__device__ __forceinline__ TE shared_sum(const TE (&E)[8], int sx, int sy, int sz) {
  // sx: weight mode on x for free axes: 0 sum, 1 sigma
  TE acc = TE(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    if (RX == 1 && ax != 0) continue;
    if (RX == -1 && ax != 1) continue;
    if (RY == 1 && ay != 0) continue;
    if (RY == -1 && ay != 1) continue;
    if (RZ == 1 && az != 0) continue;
    if (RZ == -1 && az != 1) continue;
    int sg = 1;
    if (RX == 0 && sx) sg *= ax ? 1 : -1;
    if (RY == 0 && sy) sg *= ay ? 1 : -1;
    if (RZ == 0 && sz) sg *= az ? 1 : -1;
    acc = sg > 0 ? acc + E[a] : acc - E[a];
  }
  return acc;
}

template <int R>
__device__ constexpr double mass1(void) { return R == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
template <int R>
__device__ constexpr double stiff1(void) { return R == 0 ? 1.0 : -1.0; }

template <int RX, int RY, int RZ, typename TE>
__device__ __forceinline__ void block_of(const TE (&E)[8], TE lam, TE mu, TE (&A)[3][3]) {
  constexpr int r[3] = {RX, RY, RZ};
  constexpr double M[3] = {mass1<RX>(), mass1<RY>(), mass1<RZ>()};
  constexpr double Sd[3] = {stiff1<RX>(), stiff1<RY>(), stiff1<RZ>()};
  constexpr double Tc[3] = {Sd[0] * M[1] * M[2], Sd[1] * M[0] * M[2], Sd[2] * M[0] * M[1]};
  const TE sE = shared_sum<RX, RY, RZ>(E, 0, 0, 0);
  const TE lpm = lam + mu, lmm = lam - mu;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    A[c][c] = (lpm * TE(Tc[c]) + mu * TE(Tc[0] + Tc[1] + Tc[2])) * sE;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int cp = 0; cp < 3; ++cp) {
      if (c == cp) continue;
      const int d = 3 - c - cp;
      const TE q = TE(0.25 * M[d]);
      TE v;
      if (r[c] != 0 && r[cp] != 0) {
        v = -q * TE(r[c] * r[cp]) * lpm * sE;
      } else if (r[c] == 0 && r[cp] != 0) {
        v = q * TE(r[cp]) * lmm * shared_sum<RX, RY, RZ>(E, c == 0, c == 1, c == 2);
      } else if (r[c] != 0 && r[cp] == 0) {
        v = -q * TE(r[c]) * lmm * shared_sum<RX, RY, RZ>(E, cp == 0, cp == 1, cp == 2);
      } else {
        v = q * lpm * shared_sum<RX, RY, RZ>(E, c == 0 || cp == 0, c == 1 || cp == 1, c == 2 || cp == 2);
      }
      A[c][cp] = v;
    }
  }
}

// q[k] += A(r) u_j[k] for the active load cases
template <int RX, int RY, int RZ, typename TE, typename TV>
__device__ __forceinline__ void accumulate(const TE (&E)[8], TE lam, TE mu, int j, const TV *u, int na,
                                           const unsigned act, TE (&q)[NRHS][3]) {
  // a culled neighbour shares no stiffness with the node.  (Reading row 0
  // against a zero block instead of this branch, so that all 27 neighbours'
  // loads form one block, measured 7 % slower: more registers, and the
  // culled neighbours' loads still take issue slots.)
  if (j < 0) return;
  TE A[3][3];
  block_of<RX, RY, RZ>(E, lam, mu, A);
  TE v[3 * NRHS];
  load_row(u, j, v);
#pragma unroll
  for (int k = 0; k < NRHS; ++k) {
    if (!((act >> k) & 1u)) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) q[k][c] += A[c][0] * v[3 * k] + A[c][1] * v[3 * k + 1] + A[c][2] * v[3 * k + 2];
  }
}

// q[k] += A(r) u_j[k] for the three neighbours of one x-row (dy, dz): one
// branch for the row (skipped when all three are culled), the three rows'
// loads in flight together; a culled one reads row 0 against a zero block
template <int RY, int RZ, typename TE, typename TV>
__device__ __forceinline__ void accumulate_xrow(const TE (&E)[8], TE lam, TE mu, const int *nb, const TV *u,
                                                const unsigned act, TE (&q)[NRHS][3]) {
  const int j0 = nb[0], j1 = nb[1], j2 = nb[2];
  if ((j0 & j1 & j2) < 0) return;  // all three culled (negative)
  TE A[3][3][3];
  block_of<-1, RY, RZ>(E, lam, mu, A[0]);
  block_of<0, RY, RZ>(E, lam, mu, A[1]);
  block_of<1, RY, RZ>(E, lam, mu, A[2]);
  const int jj[3] = {j0, j1, j2};
  TE v[3][3 * NRHS];
#pragma unroll
  for (int x = 0; x < 3; ++x) load_row(u, jj[x] < 0 ? 0 : jj[x], v[x]);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const TE live = jj[x] < 0 ? TE(0) : TE(1);
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
      if (!((act >> k) & 1u)) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        q[k][c] += live * (A[x][c][0] * v[x][3 * k] + A[x][c][1] * v[x][3 * k + 1] + A[x][c][2] * v[x][3 * k + 2]);
    }
  }
}

// K u at node i: the 27 offsets, unrolled at compile time.  FP32 takes the
// neighbours by x-rows (one branch and three loads in flight per row: the
// selective multigrid's operator passes 17-20 % faster than one branch per
// neighbour); FP64 one by one (by rows it would need more registers than a
// wave has: the FP64 residual pass was 19 % slower).
template <typename TE, typename TV>
__device__ __forceinline__ void apply_row(const TE (&E)[8], TE lam, TE mu, const int (&nb)[27], const TV *u,
                                          int na, unsigned act, TE (&q)[NRHS][3]) {
  constexpr bool XROW = sizeof(TE) == 4;
#define SEL_ACC(dx, dy, dz) accumulate<dx, dy, dz>(E, lam, mu, nb[((dz) + 1) * 9 + ((dy) + 1) * 3 + (dx) + 1], u, na, act, q)
#define SEL_ROW(dy, dz)                                                                    \
  if constexpr (XROW) {                                                                    \
    accumulate_xrow<dy, dz>(E, lam, mu, &nb[((dz) + 1) * 9 + ((dy) + 1) * 3], u, act, q); \
  } else {                                                                                 \
    SEL_ACC(-1, dy, dz);                                                                   \
    SEL_ACC(0, dy, dz);                                                                    \
    SEL_ACC(1, dy, dz);                                                                    \
  }
#define SEL_PLANE(dz) SEL_ROW(-1, dz); SEL_ROW(0, dz); SEL_ROW(1, dz)
  SEL_PLANE(-1);
  SEL_PLANE(0);
  SEL_PLANE(1);
#undef SEL_PLANE
#undef SEL_ROW
#undef SEL_ACC
}

// neighbour indices (offset index (dz + 1) 9 + (dy + 1) 3 + dx + 1) and the
// eight element moduli of node i
template <typename TE>
__device__ __forceinline__ void node_frame(const SelDev *S, int i, const TE *Ec, int (&nb)[27], TE (&E)[8]) {
  const int n = S->n;
  const unsigned cd = S->coord[i];
  const int x = int(cd & 1023u), y = int((cd >> 10) & 1023u), z = int(cd >> 20);
  const int xs[3] = {wrap_dec(x, n), x, wrap_inc(x, n)};
  const int ys[3] = {wrap_dec(y, n), y, wrap_inc(y, n)};
  const int zs[3] = {wrap_dec(z, n), z, wrap_inc(z, n)};
  const int *map = S->map;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const long long row = ((long long)zs[dz] * n + ys[dy]) * n;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) nb[dz * 9 + dy * 3 + dx] = map[row + xs[dx]];
    }
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const int j = nb[(1 - az) * 9 + (1 - ay) * 3 + (1 - ax)];
    E[a] = j >= 0 ? Ec[j] : TE(0);
  }
}

// load cases a residual pass covers: replacement passes only the running ones,
// the initial and final passes every load case with a nonzero load
__device__ __forceinline__ unsigned resid_cases(const CgState *st, int rmode, double ffloor) {
  unsigned m = 0;
  for (int k = 0; k < NRHS; ++k) {
    bool on;
    if (rmode == 0) on = true;                                   // initial
    else if (rmode == 1) on = st->active[k] != 0;                // replacement
    else on = st->ff[k] > ffloor * ffloor;                       // final
    if (on) m |= 1u << k;
  }
  return m;
}

// PCG: q = K p for the running load cases and the per-workgroup sums
//   p.q, r.D^-1 r, q.D^-1 r, q.D^-1 q, r.r, q.r, q.q
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_op_pcg_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  __shared__ double red[7 * 16];
  const int na = S->na;
  const CgState *st = S->st;
  unsigned act = 0;
  for (int k = 0; k < NRHS; ++k)
    if (st->active[k]) act |= 1u << k;
  if (!act) return;
  const T lam = (T)S->lam, mu = (T)S->mu;
  const T *P = (const T *)S->p, *Rv = (const T *)S->r, *Dv = (const T *)S->Dinv;
  T *Q = (T *)S->q;
  // one node per thread (the grid covers the list), so the sums below need
  // no accumulators across nodes
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  T q[NRHS][3];
#pragma unroll
  for (int k = 0; k < NRHS; ++k) q[k][0] = q[k][1] = q[k][2] = T(0);
  double dv = 0.0;
  T pr[3 * NRHS], rr[3 * NRHS];
  if (i < na) {
    int nb[27];
    T E[8];
    node_frame<T>(S, i, (const T *)S->Ec, nb, E);
    apply_row<T, T>(E, lam, mu, nb, P, na, act, q);
    dv = (double)Dv[i];
    T qr[3 * NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) qr[3 * k + c] = q[k][c];
    store_row(Q, i, qr);
    load_row(P, i, pr);
    load_row(Rv, i, rr);
  }
  double *parts = S->partials;
  const int np = S->nparts;
#pragma unroll
  for (int k = 0; k < NRHS; ++k) {
    if (!((act >> k) & 1u)) continue;
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < na) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double qv = (double)q[k][c], pv = (double)pr[3 * k + c], rv = (double)rr[3 * k + c];
        v[0] += pv * qv;
        v[1] += rv * dv * rv;
        v[2] += qv * dv * rv;
        v[3] += qv * dv * qv;
        v[4] += rv * rv;
        v[5] += qv * rv;
        v[6] += qv * qv;
      }
    }
    block_sum<7>(v, red, SEL_THREADS);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int s = 0; s < 7; ++s) parts[((long long)k * np + blockIdx.x) * SEL_PS + s] = v[s];
    }
  }
}

// r = f - K u in FP64 (u = the FP64 solution), stored in the working
// precision; per-workgroup component sums of r (for the mean removal).
// f at node i is -sum_a E_a (K_0 chi^k)_a.
template <typename TV>
__global__ __launch_bounds__(SEL_THREADS) void sel_op_resid_kernel(const SelBatch B, int rmode) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  __shared__ double red[3 * 16];
  const int na = S->na;
  const unsigned act = resid_cases(S->st, rmode, S->ffloor);
  if (!act) return;
  const double lam = S->lam, mu = S->mu;
  const double *U = S->x64;
  TV *Rv = (TV *)S->r;
  double acc[NRHS][3];
#pragma unroll
  for (int k = 0; k < NRHS; ++k) acc[k][0] = acc[k][1] = acc[k][2] = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    int nb[27];
    double E[8];
    node_frame<double>(S, i, S->Ec64, nb, E);
    double q[NRHS][3];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) q[k][0] = q[k][1] = q[k][2] = 0.0;
    apply_row<double, double>(E, lam, mu, nb, U, na, act, q);
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
      if (!((act >> k) & 1u)) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double f = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) f -= E[a] * S->f0[k][a][c];
        const double rv = f - q[k][c];
        Rv[(long long)i * (3 * NRHS) + 3 * k + c] = (TV)rv;
        acc[k][c] += rv;
      }
    }
  }
  double *parts = S->partials;
  const int np = S->nparts;
#pragma unroll
  for (int k = 0; k < NRHS; ++k) {
    if (!((act >> k) & 1u)) continue;
    double v[3] = {acc[k][0], acc[k][1], acc[k][2]};
    block_sum<3>(v, red, SEL_THREADS);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) parts[((long long)k * np + blockIdx.x) * SEL_PS + c] = v[c];
    }
  }
}

// the energy form of Eq. (8) on the compact lists: with u^k at equilibrium,
//   sum_e E_e (chi^i + u^i_e)^T K_0 (chi^j + u^j_e)
//     = (sum_e E_e) D_ij - f^i . u^j - f^j . u^i + u^i . K u^j,
// since chi^i^T K_0 chi^j = D_ij and f^i = -sum_e P_e^T E_e K_0 chi^i.
// Per workgroup: the 21 sums S_ij (i <= j) and sum_e E_e.
__global__ __launch_bounds__(SEL_THREADS) void sel_op_energy_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  __shared__ double red[22 * 16];
  const int na = S->na;
  const double lam = S->lam, mu = S->mu;
  const double *U = S->x64;
  double acc[22];
#pragma unroll
  for (int s = 0; s < 22; ++s) acc[s] = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    int nb[27];
    double E[8];
    node_frame<double>(S, i, S->Ec64, nb, E);
    double q[NRHS][3];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) q[k][0] = q[k][1] = q[k][2] = 0.0;
    apply_row<double, double>(E, lam, mu, nb, U, na, 0x3Fu, q);
    double u[NRHS][3], f[NRHS][3];
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u[k][c] = U[(long long)i * (3 * NRHS) + 3 * k + c];
        double fv = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) fv -= E[a] * S->f0[k][a][c];
        f[k][c] = fv;
      }
    int s = 0;
#pragma unroll
    for (int a = 0; a < NRHS; ++a)
#pragma unroll
      for (int b = a; b < NRHS; ++b) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) v += u[a][c] * q[b][c] - f[a][c] * u[b][c] - f[b][c] * u[a][c];
        acc[s++] += v;
      }
    acc[21] += E[0];  // the element whose lower corner is node i
  }
  block_sum<22>(acc, red, SEL_THREADS);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < 22; ++s) S->partials[(long long)s * S->nparts + blockIdx.x] = acc[s];
  }
}

// plain q = K p for every load case (operator parity tests)
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_op_apply_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na;
  const T lam = (T)S->lam, mu = (T)S->mu;
  const T *P = (const T *)S->p;
  T *Q = (T *)S->q;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    int nb[27];
    T E[8];
    node_frame<T>(S, i, (const T *)S->Ec, nb, E);
    T q[NRHS][3];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) q[k][0] = q[k][1] = q[k][2] = T(0);
    apply_row<T, T>(E, lam, mu, nb, P, na, 0x3Fu, q);
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) Q[(long long)i * (3 * NRHS) + 3 * k + c] = q[k][c];
  }
}

// ---- vector phases ------------------------------------------------------------
// x += alpha p, r -= alpha q, p = D^-1 r + beta p for the load cases the
// scalar phase gave a step (alpha != 0)
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_update_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na;
  const CgState *st = S->st;
  T *X = (T *)S->x, *Rv = (T *)S->r, *P = (T *)S->p;
  const T *Q = (const T *)S->q, *Dv = (const T *)S->Dinv;
  T a[NRHS], b[NRHS];
  unsigned step = 0;
  for (int k = 0; k < NRHS; ++k) {
    a[k] = (T)st->alpha[k];
    b[k] = (T)st->beta[k];
    if (st->alpha[k] != 0.0) step |= 1u << k;
  }
  if (!step) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    const T d = Dv[i];
    T x[3 * NRHS], r[3 * NRHS], p[3 * NRHS], q[3 * NRHS];
    load_row(X, i, x);
    load_row(Rv, i, r);
    load_row(P, i, p);
    load_row(Q, i, q);
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
      if (!((step >> k) & 1u)) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int o = 3 * k + c;
        const T pv = p[o];
        const T rv = r[o] - a[k] * q[o];
        x[o] += a[k] * pv;
        r[o] = rv;
        p[o] = d * rv + b[k] * pv;
      }
    }
    store_row(X, i, x);
    store_row(Rv, i, r);
    store_row(P, i, p);
  }
}

// p = D^-1 r (start of the iteration) for every load case still running
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_dir0_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na;
  const CgState *st = S->st;
  T *P = (T *)S->p;
  const T *Rv = (const T *)S->r, *Dv = (const T *)S->Dinv;
  for (int k = 0; k < NRHS; ++k) {
    if (!st->active[k]) continue;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = (long long)i * (3 * NRHS) + 3 * k + c;
        P[o] = Dv[i] * Rv[o];
      }
  }
}

// mixed: x64 += x32, x32 = 0 (every load case, or the running ones)
__global__ __launch_bounds__(SEL_THREADS) void sel_fold_kernel(const SelBatch B, int all) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na;
  const CgState *st = S->st;
  float *X = (float *)S->x;
  double *X64 = S->x64;
  for (int k = 0; k < NRHS; ++k) {
    if (!all && !st->active[k]) continue;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = (long long)i * (3 * NRHS) + 3 * k + c;
        X64[o] += (double)X[o];
        X[o] = 0.0f;
      }
  }
}

// the recomputed residual: remove its component means (rigid translations of
// the whole active set), then the sums r.D^-1 r and r.r
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_finish_kernel(const SelBatch B, int rmode) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  __shared__ double red[2 * 16];
  const int na = S->na;
  const CgState *st = S->st;
  const unsigned act = resid_cases(st, rmode, S->ffloor);
  T *Rv = (T *)S->r;
  const T *Dv = (const T *)S->Dinv;
  for (int k = 0; k < NRHS; ++k) {
    if (!((act >> k) & 1u)) continue;
    const T m[3] = {(T)st->mean[k][0], (T)st->mean[k][1], (T)st->mean[k][2]};
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
      const double d = (double)Dv[i];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long o = (long long)i * (3 * NRHS) + 3 * k + c;
        const T rv = Rv[o] - m[c];
        Rv[o] = rv;
        const double r64 = (double)rv;
        v[0] += r64 * d * r64;
        v[1] += r64 * r64;
      }
    }
    block_sum<2>(v, red, SEL_THREADS);
    if (threadIdx.x == 0) {
      S->partials[((long long)k * S->nparts + blockIdx.x) * SEL_PS + 0] = v[0];
      S->partials[((long long)k * S->nparts + blockIdx.x) * SEL_PS + 1] = v[1];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_zero_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const long long m = (long long)NRHS * 3 * S->na;
  T *X = (T *)S->x, *P = (T *)S->p;
  double *X64 = S->x64;
  const bool mixed = S->prec == SHH_PREC_MIXED;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (long long)S->nparts * blockDim.x) {
    X[i] = T(0);
    P[i] = T(0);
    if (mixed) X64[i] = 0.0;
  }
}

// ---- scalar phases (one workgroup per load case; one in total for C^H) --------
// a residual replacement keeps the CG direction while the new r . z is within
// this factor of the recursive one (and until the case has stalled once)
#ifndef SHH_KEEP_DIR_RATIO
#define SHH_KEEP_DIR_RATIO 2.0
#endif
__global__ __launch_bounds__(SEL_THREADS) void sel_scalar_kernel(const SelBatch B, int phase) {
  SelDev *S = B.d[blockIdx.y];
  __shared__ double red[22 * 16];
  CgState *st = S->st;
  const int np = S->nparts;
  if (phase == SSC_ENERGY) {
    double tot[22];
    for (int s = 0; s < 22; ++s) tot[s] = 0.0;
    for (int b = threadIdx.x; b < np; b += SEL_THREADS)
      for (int s = 0; s < 22; ++s) tot[s] += S->partials[(long long)s * np + b];
    block_sum<22>(tot, red, SEL_THREADS);
    if (threadIdx.x != 0) return;
    const double lam = S->lam, mu = S->mu, sumE = tot[21], inv = 1.0 / double(S->nn);
    int s = 0;
    for (int a = 0; a < NRHS; ++a)
      for (int b = a; b < NRHS; ++b) {
        double D = 0.0;
        if (a < 3 && b < 3) D = a == b ? lam + 2.0 * mu : lam;
        else if (a == b) D = mu;
        const double c = (sumE * D + tot[s++]) * inv;
        st->C[a * 6 + b] = c;
        st->C[b * 6 + a] = c;
      }
    return;
  }
  const int k = blockIdx.x;
  const double *parts = S->partials + (long long)k * np * SEL_PS;
  if (phase == SSC_MG_ALPHA) {  // alpha = rho / p . K p
    if (!st->active[k]) {
      if (threadIdx.x == 0) st->alpha[k] = 0.0;
      return;
    }
    double tot[1];
    sum_partials<1, SEL_PS>(parts, np, tot, red, SEL_THREADS);
    if (threadIdx.x != 0) return;
    const double pq = tot[0];
    if (!(pq > 0.0) || !(st->rho[k] > 0.0)) {
      st->alpha[k] = 0.0;
      st->active[k] = 0;
      st->status[k] = ST_STALLED;
      st->no_keep[k] = 1;
      return;
    }
    st->alpha[k] = st->rho[k] / pq;
    return;
  }
  // rho' = r . z, ||r||, and beta: after an iteration rho' / rho; after a
  // restart 0; after a residual replacement (r replaced by f - K u, z = V r
  // recomputed) the direction is kept, beta' = beta rho' / rho = rho' over
  // the rho the last iteration started from, while rho' is within a factor 2
  // of the recursive rho (a larger drift restarts)
  if (phase == SSC_MG_BETA || phase == SSC_MG_RESTART || phase == SSC_MG_REPLACE) {
    if (!st->active[k]) return;
    double tot[2];
    sum_partials<2, SEL_PS>(parts, np, tot, red, SEL_THREADS);
    if (threadIdx.x != 0) return;
    const double rho1 = tot[0], rr = tot[1];
    st->rr[k] = rr;
    const double rel = sqrt(rr / st->ff[k]);
    st->rel[k] = rel;
    if (phase == SSC_MG_BETA) st->iters[k] += 1;
    if (rel <= S->rtol) {
      st->active[k] = 0;
      st->status[k] = ST_CONVERGED;
    } else if (!(rho1 > 0.0)) {  // r . V r > 0 unless the cycle lost definiteness
      st->active[k] = 0;
      st->status[k] = phase == SSC_MG_RESTART ? ST_BREAKDOWN : ST_STALLED;
      st->no_keep[k] = 1;
    } else if (st->iters[k] >= S->max_iter) {
      st->active[k] = 0;
      st->status[k] = ST_MAXIT;
    }
    if (phase == SSC_MG_RESTART) st->beta[k] = 0.0;
    else if (phase == SSC_MG_REPLACE)
      st->beta[k] = !st->no_keep[k] && rho1 <= SHH_KEEP_DIR_RATIO * st->rho[k] &&
                            rho1 * SHH_KEEP_DIR_RATIO >= st->rho[k]
                        ? st->beta[k] * rho1 / st->rho[k]
                        : 0.0;
    else st->beta[k] = rho1 / st->rho[k];
    st->rho[k] = rho1;
    return;
  }
  if (phase == SSC_ITER) {
    if (!st->active[k]) {
      if (threadIdx.x == 0) st->alpha[k] = 0.0;
      return;
    }
    double tot[7];
    sum_partials<7, SEL_PS>(parts, np, tot, red, SEL_THREADS);
    if (threadIdx.x != 0) return;
    const double pq = tot[0], rho = tot[1], qzr = tot[2], qzq = tot[3], rr = tot[4], qr = tot[5], qq = tot[6];
    if (!(pq > 0.0) || !(rho >= 0.0)) {  // breakdown (or NaN)
      st->alpha[k] = 0.0;
      st->active[k] = 0;
      st->status[k] = ST_BREAKDOWN;
      return;
    }
    const double a = rho / pq;
    const double rho1 = rho - 2.0 * a * qzr + a * a * qzq;
    const double rr1 = fmax(rr - 2.0 * a * qr + a * a * qq, 0.0);
    st->alpha[k] = a;
    st->beta[k] = rho > 0.0 ? rho1 / rho : 0.0;
    st->rho[k] = rho1;
    st->rr[k] = rr1;
    st->iters[k] += 1;
    const double rel = sqrt(rr1 / st->ff[k]);
    st->rel[k] = rel;
    if (rel <= S->rtol) {
      st->active[k] = 0;
      st->status[k] = ST_CONVERGED;
    } else if (st->iters[k] >= S->max_iter) {
      st->active[k] = 0;
      st->status[k] = ST_MAXIT;
    }
    return;
  }
  // residual phases: rmode 0 initial, 1 replacement, 2 final
  const int rmode = phase == SSC_RESID_INIT ? 0 : (phase == SSC_RESID_REPLACE ? 1 : 2);
  if (phase == SSC_MEAN) return;  // launched through sel_launch_scalar_mean
  const unsigned act = resid_cases(st, rmode, S->ffloor);
  if (!((act >> k) & 1u)) return;
  double tot[2];
  sum_partials<2, SEL_PS>(parts, np, tot, red, SEL_THREADS);
  if (threadIdx.x != 0) return;
  const double rho = tot[0], rr = tot[1];
  if (rmode == 0) {
    st->ff[k] = rr;
    st->rr[k] = rr;
    st->rho[k] = rho;
    st->alpha[k] = 0.0;
    st->beta[k] = 0.0;
    st->iters[k] = 0;
    st->rel_min[k] = 1.0;
    st->no_keep[k] = 0;
    st->stag[k] = 0;
    if (sqrt(rr) <= S->ffloor) {  // zero load: u = 0
      st->active[k] = 0;
      st->status[k] = ST_CONVERGED;
      st->rel[k] = st->rel_true[k] = 0.0;
    } else {
      st->active[k] = S->max_iter > 0 ? 1 : 0;
      st->status[k] = S->max_iter > 0 ? ST_RUNNING : ST_MAXIT;
      st->rel[k] = st->rel_true[k] = 1.0;
    }
  } else if (rmode == 1) {
    st->rr[k] = rr;
    const double rel = sqrt(rr / st->ff[k]);
    // a true residual twice the smallest one so far: the kept directions
    // have drifted; this case restarts after every replacement from now on
    if (rel > 2.0 * st->rel_min[k]) st->no_keep[k] = 1;
    // 50 replacements without a 1 % gain: the precision's floor is above the
    // tolerance (FP32 vectors on a nearly singular culled system); stop
    st->stag[k] = rel < 0.99 * st->rel_min[k] ? 0 : st->stag[k] + 1;
    if (st->stag[k] >= 50) {
      st->active[k] = 0;
      st->status[k] = ST_MAXIT;
    }
    st->rel_min[k] = fmin(st->rel_min[k], rel);
    st->rel_true[k] = rel;
  } else {
    st->rr[k] = rr;
    const double rel = sqrt(rr / st->ff[k]);
    st->rel_true[k] = rel;
    if (rel <= S->rtol) {
      st->active[k] = 0;
      st->status[k] = ST_CONVERGED;
    } else if (st->status[k] != ST_BREAKDOWN && st->status[k] != ST_MAXIT && st->iters[k] < S->max_iter) {
      st->active[k] = 1;  // the recursive residual was optimistic, or the case stalled: resume
      st->status[k] = ST_RUNNING;
    } else if (st->status[k] != ST_BREAKDOWN) {
      st->active[k] = 0;
      st->status[k] = ST_MAXIT;
    }
  }
}

// component means of the recomputed residual
__global__ __launch_bounds__(SEL_THREADS) void sel_mean_kernel(const SelBatch B, int rmode) {
  SelDev *S = B.d[blockIdx.y];
  __shared__ double red[3 * 16];
  CgState *st = S->st;
  const int k = blockIdx.x;
  const unsigned act = resid_cases(st, rmode, S->ffloor);
  if (!((act >> k) & 1u)) return;
  double tot[3];
  sum_partials<3, SEL_PS>(S->partials + (long long)k * S->nparts * SEL_PS, S->nparts, tot, red, SEL_THREADS);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) st->mean[k][c] = tot[c] / double(S->na);
}

// ---- the multigrid-preconditioned solve: voxel-level V-cycle steps ------------
// The same degree-2 Chebyshev smoothing on D^-1 A as the dense path (interval
// [h/33, h], h the element bound of lambda_max): with b the CG residual,
//   pre:  d0 = D^-1 b / theta;  r1 = b - A d0;  d1 = c1 d0 + c2 D^-1 r1;
//         x = d0 + d1;  r2 = r1 - A d1            (restricted to level 1)
//   post: x += P x1;  r = b - A x;  d0 = D^-1 r / theta;  x += d0;
//         r' = r - A d0;  d1 = c1 d0 + c2 D^-1 r';  z = x + d1.
// Each operator pass fuses the element-wise step after it, and none writes
// the vector its operator reads (a neighbour's input).
__device__ __forceinline__ unsigned active_mask(const CgState *st) {
  unsigned act = 0;
  for (int k = 0; k < NRHS; ++k)
    if (st->active[k]) act |= 1u << k;
  return act;
}

template <typename T, int MODE>
__global__ __launch_bounds__(SEL_THREADS) void sel_mg_op_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  __shared__ double red[2 * 16];
  const int na = S->na;
  const unsigned act = active_mask(S->st);
  if (!act) return;
  const T lam = (T)S->lam, mu = (T)S->mu;
  const T *in = (const T *)(MODE == SMO_PQ ? S->p : MODE == SMO_STEP1 ? S->d0 : MODE == SMO_RES ? S->d1
                           : (MODE == SMO_POST || MODE == SMO_POST1) ? S->xv : S->d0);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  T q[NRHS][3];
#pragma unroll
  for (int k = 0; k < NRHS; ++k) q[k][0] = q[k][1] = q[k][2] = T(0);
  double acc[NRHS][2];
#pragma unroll
  for (int k = 0; k < NRHS; ++k) acc[k][0] = acc[k][1] = 0.0;
  if (i < na) {
    int nb[27];
    T E[8];
    node_frame<T>(S, i, (const T *)S->Ec, nb, E);
    apply_row<T, T>(E, lam, mu, nb, in, na, act, q);
    const T dv = ((const T *)S->Dinv)[i];
    const T it = (T)S->inv_theta, c1 = (T)S->c1, c2 = (T)S->c2;
    if constexpr (MODE == SMO_PQ) {
      T pr[3 * NRHS], qr[3 * NRHS];
      load_row((const T *)S->p, i, pr);
#pragma unroll
      for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          qr[3 * k + c] = q[k][c];
          acc[k][0] += (double)pr[3 * k + c] * (double)q[k][c];
        }
      store_row((T *)S->q, i, qr);
    } else if constexpr (MODE == SMO_STEP1) {
      T b[3 * NRHS], d0[3 * NRHS], r1[3 * NRHS], d1[3 * NRHS], x[3 * NRHS];
      load_row((const T *)S->r, i, b);
      load_row((const T *)S->d0, i, d0);
#pragma unroll
      for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int o = 3 * k + c;
          r1[o] = b[o] - q[k][c];
          d1[o] = c1 * d0[o] + c2 * dv * r1[o];
          x[o] = d0[o] + d1[o];
        }
      store_row((T *)S->rv, i, r1);
      if constexpr (SHH_SEL_DEG0 != 1) store_row((T *)S->d1, i, d1);  // degree 1: d1 = 0, unused
      store_row((T *)S->xv, i, x);
    } else if constexpr (MODE == SMO_RES) {
      T r[3 * NRHS];
      load_row((const T *)S->rv, i, r);
#pragma unroll
      for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) r[3 * k + c] -= q[k][c];
      store_row((T *)S->rv, i, r);
    } else if constexpr (MODE == SMO_POST) {
      // x is this pass's operand: the updated x goes to d1 (free after the
      // restriction), not over the neighbours' input
      T b[3 * NRHS], x[3 * NRHS], r[3 * NRHS], d0[3 * NRHS];
      load_row((const T *)S->r, i, b);
      load_row((const T *)S->xv, i, x);
#pragma unroll
      for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int o = 3 * k + c;
          r[o] = b[o] - q[k][c];
          d0[o] = it * dv * r[o];
          x[o] += d0[o];
        }
      store_row((T *)S->rv, i, r);
      store_row((T *)S->d0, i, d0);
      store_row((T *)S->d1, i, x);
    } else if constexpr (MODE == SMO_POST1) {
      // degree 1: z = x + D (b - K x) / theta into d1 (x is the operand),
      // and the sums b . z, b . b
      T b[3 * NRHS], x[3 * NRHS];
      load_row((const T *)S->r, i, b);
      load_row((const T *)S->xv, i, x);
#pragma unroll
      for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int o = 3 * k + c;
          x[o] += it * dv * (b[o] - q[k][c]);
          acc[k][0] += (double)b[o] * (double)x[o];
          acc[k][1] += (double)b[o] * (double)b[o];
        }
      store_row((T *)S->d1, i, x);
    } else {  // SMO_LAST: z = x + d1 into xv, and the sums b . z, b . b
      T b[3 * NRHS], x[3 * NRHS], r[3 * NRHS], d0[3 * NRHS];
      load_row((const T *)S->r, i, b);
      load_row((const T *)S->d1, i, x);
      load_row((const T *)S->rv, i, r);
      load_row((const T *)S->d0, i, d0);
#pragma unroll
      for (int k = 0; k < NRHS; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int o = 3 * k + c;
          const T r2 = r[o] - q[k][c];
          x[o] += c1 * d0[o] + c2 * dv * r2;
          acc[k][0] += (double)b[o] * (double)x[o];
          acc[k][1] += (double)b[o] * (double)b[o];
        }
      store_row((T *)S->xv, i, x);
    }
  }
  if constexpr (MODE == SMO_PQ || MODE == SMO_LAST || MODE == SMO_POST1) {
    double *parts = S->partials;
    const int np = S->nparts;
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
      if (!((act >> k) & 1u)) continue;
      double v[2] = {acc[k][0], acc[k][1]};
      block_sum<2>(v, red, SEL_THREADS);
      if (threadIdx.x == 0) {
        parts[((long long)k * np + blockIdx.x) * SEL_PS + 0] = v[0];
        parts[((long long)k * np + blockIdx.x) * SEL_PS + 1] = v[1];
      }
    }
  }
}

// the CG update x += alpha p, r -= alpha q (not on a restart), then the first
// Chebyshev direction d0 = D^-1 r / theta
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_mg_s1_kernel(const SelBatch B, int restart) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na;
  const CgState *st = S->st;
  T a[NRHS];
  for (int k = 0; k < NRHS; ++k) a[k] = restart ? T(0) : (T)st->alpha[k];
  const T it = (T)S->inv_theta;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    const T dv = ((const T *)S->Dinv)[i];
    T x[3 * NRHS], r[3 * NRHS], p[3 * NRHS], q[3 * NRHS], d0[3 * NRHS];
    load_row((const T *)S->r, i, r);
    if (!restart) {
      load_row((const T *)S->x, i, x);
      load_row((const T *)S->p, i, p);
      load_row((const T *)S->q, i, q);
    }
#pragma unroll
    for (int k = 0; k < NRHS; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int o = 3 * k + c;
        if (!restart && a[k] != T(0)) {
          x[o] += a[k] * p[o];
          r[o] -= a[k] * q[o];
        }
        d0[o] = it * dv * r[o];
      }
    if (!restart) {
      store_row((T *)S->x, i, x);
      store_row((T *)S->r, i, r);
    }
    store_row((T *)S->d0, i, d0);
  }
}

// p = z + beta p for the running load cases (beta = 0 after a restart)
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_mg_dir_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na;
  const unsigned act = active_mask(S->st);
  if (!act) return;
  T b[NRHS];
  for (int k = 0; k < NRHS; ++k) b[k] = (T)S->st->beta[k];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    T z[3 * NRHS], p[3 * NRHS];
    load_row((const T *)(SHH_SEL_DEG0 == 1 ? S->d1 : S->xv), i, z);  // where post-smoothing left z
    load_row((const T *)S->p, i, p);
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
      if (!((act >> k) & 1u)) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) p[3 * k + c] = z[3 * k + c] + b[k] * p[3 * k + c];
    }
    store_row((T *)S->p, i, p);
  }
}

// b1 = P^T r2: coarse node I collects the fine nodes 2 I + o, o in {-1, 0, 1}^3,
// with weight prod (o == 0 ? 1 : 1/2); culled fine nodes hold zero
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_mg_restrict_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  const int n = S->n, n1 = S->n1;
  const long long nn1 = S->nn1;
  const unsigned I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= (unsigned)nn1) return;
  const unsigned row = I / (unsigned)n1;  // 32-bit: n <= 512
  const int X = int(I - row * (unsigned)n1), Y = int(row % (unsigned)n1), Z = int(row / (unsigned)n1);
  T acc[3 * NRHS];
#pragma unroll
  for (int o = 0; o < 3 * NRHS; ++o) acc[o] = T(0);
  const T *rv = (const T *)S->rv;
  // the 27 map entries first, all in flight together
  int jf[27];
  bool any = false;
#pragma unroll
  for (int f = 0; f < 27; ++f) {
    const int ox = f % 3 - 1, oy = (f / 3) % 3 - 1, oz = f / 9 - 1;
    const int fx = wrap1(2 * X + ox, n), fy = wrap1(2 * Y + oy, n), fz = wrap1(2 * Z + oz, n);
    jf[f] = S->map[((long long)fz * n + fy) * n + fx];
  }
#pragma unroll
  for (int f = 0; f < 27; ++f) any = any || jf[f] >= 0;
  // then the rows.  FP32: without a branch per fine node (a culled one reads
  // row 0 at weight 0), so the loads of all 27 overlap (the transfer passes
  // 6 % faster than with the branch); FP64 would not fit the registers that
  // way and skips culled nodes by a branch.
  constexpr bool STRAIGHT = sizeof(T) == 4;
  if (any) {
#pragma unroll
    for (int f = 0; f < 27; ++f) {
      if (!STRAIGHT && jf[f] < 0) continue;
      const int ox = f % 3 - 1, oy = (f / 3) % 3 - 1, oz = f / 9 - 1;
      const T w = jf[f] >= 0 ? T((ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0)) : T(0);
      T v[3 * NRHS];
      load_row(rv, jf[f] >= 0 ? jf[f] : 0, v);
#pragma unroll
      for (int o = 0; o < 3 * NRHS; ++o) acc[o] += w * v[o];
    }
  }
  T *b1 = (T *)S->b1;
#pragma unroll
  for (int o = 0; o < 3 * NRHS; ++o) b1[(long long)o * nn1 + I] = acc[o];
}

// z += P x1 at the active nodes: per axis, an even fine index has one coarse
// parent (weight 1), an odd one two (weight 1/2 each)
template <typename T>
__global__ __launch_bounds__(SEL_THREADS) void sel_mg_prolong_kernel(const SelBatch B) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int na = S->na, n1 = S->n1;
  const long long nn1 = S->nn1;
  const T *x1 = (const T *)S->x1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += S->nparts * blockDim.x) {
    const unsigned cd = S->coord[i];
    const int c3[3] = {int(cd & 1023u), int((cd >> 10) & 1023u), int(cd >> 20)};
    int par[3][2];
    T wt[3][2];
    int cnt[3];
    for (int a = 0; a < 3; ++a) {
      if ((c3[a] & 1) == 0) {
        par[a][0] = c3[a] >> 1;
        wt[a][0] = T(1);
        cnt[a] = 1;
      } else {
        par[a][0] = c3[a] >> 1;
        par[a][1] = (c3[a] >> 1) + 1 == n1 ? 0 : (c3[a] >> 1) + 1;
        wt[a][0] = wt[a][1] = T(0.5);
        cnt[a] = 2;
      }
    }
    T z[3 * NRHS];
    load_row((const T *)S->xv, i, z);
    for (int kz = 0; kz < cnt[2]; ++kz)
      for (int ky = 0; ky < cnt[1]; ++ky)
        for (int kx = 0; kx < cnt[0]; ++kx) {
          const long long I = ((long long)par[2][kz] * n1 + par[1][ky]) * n1 + par[0][kx];
          const T w = wt[0][kx] * wt[1][ky] * wt[2][kz];
#pragma unroll
          for (int o = 0; o < 3 * NRHS; ++o) z[o] += w * x1[(long long)o * nn1 + I];
        }
    store_row((T *)S->xv, i, z);
  }
}

// ---- energy sensitivity (the adjoint of Eq. (9) on the culled system) --------
// With u^k at equilibrium, dC_ij / dE_e = (chi^i + u^i_e)^T K_0 (chi^j + u^j_e) / n^3
// (the solve's own dependence drops out by self-adjointness), so
// dL/dE_e = sum_{i<=j} g_ij e_ij / n^3 with g the symmetric fold of dL/dC.
// One thread per active node: the element whose lower corner it is, when that
// element carries stiffness (its eight corners are then active nodes); culled
// elements keep the zero of the fill.
__global__ __launch_bounds__(SEL_THREADS) void sel_fill_kernel(double *out, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = 0.0;
}

__global__ __launch_bounds__(SEL_THREADS) void sel_energy_sens_kernel(const SelBatch B, const double *g21,
                                                                      double *out) {
  SelDev *S = B.d[blockIdx.y];
  if (blockIdx.x >= (unsigned)S->nparts) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S->na) return;
  if (!(S->Ec64[i] > 0.0)) return;
  const int n = S->n;
  const unsigned cd = S->coord[i];
  const int x = int(cd & 1023u), y = int((cd >> 10) & 1023u), z = int(cd >> 20);
  const int xs[2] = {x, wrap_inc(x, n)}, ys[2] = {y, wrap_inc(y, n)}, zs[2] = {z, wrap_inc(z, n)};
  int node[8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
    node[a] = S->map[((long long)zs[a >> 2] * n + ys[(a >> 1) & 1]) * n + xs[a & 1]];
  const double *U = S->x64;
  double g[21];
#pragma unroll
  for (int t = 0; t < 21; ++t) g[t] = g21[t];
  // element Hadamard coefficients of chi^k + u^k for every load case
  auto coeffs = [&](int k, double (&h)[3][8]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) v[a] = U[(long long)node[a] * (3 * NRHS) + 3 * k + c];
      hadamard8<double>(v, h[c]);
    }
    add_chi<double>(k, h);
  };
  double sens = 0.0;
  int t = 0;
  for (int a = 0; a < NRHS; ++a) {
    double ha[3][8];
    coeffs(a, ha);
    for (int b = a; b < NRHS; ++b) {
      double hb[3][8], wb[3][8];
      coeffs(b, hb);
      hex_apply<double>(S->kop, hb, wb, 1.0);
      double e = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 8; ++m) e += ha[c][m] * wb[c][m];
      sens += g[t++] * e;
    }
  }
  out[((long long)z * n + y) * n + x] = sens / double(S->nn);
}

// ---- launchers ----------------------------------------------------------------
// Every launch covers the batch's slots (grid y = slot); workgroups past a
// slot's own count return at once.
namespace {
dim3 parts_grid(const SelBatch &B) { return dim3((unsigned)std::max(B.parts_max, 1), (unsigned)B.count); }
}  // namespace

#define SEL_PREC_LAUNCH(kern, grid, ...)                                                  \
  do {                                                                                  \
    if (B.prec == SHH_PREC_FP64) kern<double><<<grid, SEL_THREADS, 0, st>>>(__VA_ARGS__); \
    else kern<float><<<grid, SEL_THREADS, 0, st>>>(__VA_ARGS__);                        \
  } while (0)

hipError_t sel_launch_compact(const SelBatch &B, hipStream_t st) {
  const dim3 g((unsigned)std::max(B.chunks_max, 1), (unsigned)B.count);
  sel_count_kernel<<<g, SEL_THREADS, 0, st>>>(B);
  sel_scan_kernel<<<dim3(1, B.count), 1024, 0, st>>>(B);
  sel_write_kernel<<<g, SEL_THREADS, 0, st>>>(B);
  return hipGetLastError();
}

hipError_t sel_launch_gather(const SelBatch &B, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_gather_kernel, parts_grid(B), B);
  return hipGetLastError();
}

hipError_t sel_launch_op(const SelBatch &B, int mode, hipStream_t st) {
  const dim3 g = parts_grid(B);
  if (mode == SOP_PCG) {
    SEL_PREC_LAUNCH(sel_op_pcg_kernel, g, B);
  } else if (mode == SOP_ENERGY) {
    sel_op_energy_kernel<<<g, SEL_THREADS, 0, st>>>(B);
  } else if (mode == SOP_APPLY) {
    SEL_PREC_LAUNCH(sel_op_apply_kernel, g, B);
  } else {
    const int rmode = mode - 10;  // SOP_RESID + rmode: 10 initial, 11 replacement, 12 final
    SEL_PREC_LAUNCH(sel_op_resid_kernel, g, B, rmode);
  }
  return hipGetLastError();
}

hipError_t sel_launch_scalar(const SelBatch &B, int phase, hipStream_t st) {
  if (phase == SSC_ENERGY) sel_scalar_kernel<<<dim3(1, B.count), SEL_THREADS, 0, st>>>(B, phase);
  else if (phase >= 100) sel_mean_kernel<<<dim3(NRHS, B.count), SEL_THREADS, 0, st>>>(B, phase - 100);
  else sel_scalar_kernel<<<dim3(NRHS, B.count), SEL_THREADS, 0, st>>>(B, phase);
  return hipGetLastError();
}

hipError_t sel_launch_update(const SelBatch &B, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_update_kernel, parts_grid(B), B);
  return hipGetLastError();
}

hipError_t sel_launch_dir0(const SelBatch &B, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_dir0_kernel, parts_grid(B), B);
  return hipGetLastError();
}

hipError_t sel_launch_fold(const SelBatch &B, int all, hipStream_t st) {
  if (B.prec == SHH_PREC_MIXED) sel_fold_kernel<<<parts_grid(B), SEL_THREADS, 0, st>>>(B, all);
  return hipGetLastError();
}

hipError_t sel_launch_finish(const SelBatch &B, int rmode, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_finish_kernel, parts_grid(B), B, rmode);
  return hipGetLastError();
}

hipError_t sel_launch_zero(const SelBatch &B, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_zero_kernel, parts_grid(B), B);
  return hipGetLastError();
}

hipError_t sel_launch_mg_op(const SelBatch &B, int mode, hipStream_t st) {
  const bool f64 = B.prec == SHH_PREC_FP64;
  const dim3 g = parts_grid(B);
#define SEL_MG_OP(M)                                                                 \
  if (f64) sel_mg_op_kernel<double, M><<<g, SEL_THREADS, 0, st>>>(B);                \
  else sel_mg_op_kernel<float, M><<<g, SEL_THREADS, 0, st>>>(B)
  switch (mode) {
    case SMO_PQ: SEL_MG_OP(SMO_PQ); break;
    case SMO_STEP1: SEL_MG_OP(SMO_STEP1); break;
    case SMO_RES: SEL_MG_OP(SMO_RES); break;
    case SMO_POST: SEL_MG_OP(SMO_POST); break;
    case SMO_POST1: SEL_MG_OP(SMO_POST1); break;
    default: SEL_MG_OP(SMO_LAST); break;
  }
#undef SEL_MG_OP
  return hipGetLastError();
}

hipError_t sel_launch_mg_s1(const SelBatch &B, int restart, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_mg_s1_kernel, parts_grid(B), B, restart);
  return hipGetLastError();
}

hipError_t sel_launch_mg_dir(const SelBatch &B, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_mg_dir_kernel, parts_grid(B), B);
  return hipGetLastError();
}

hipError_t sel_launch_mg_restrict(const SelBatch &B, hipStream_t st) {
  const dim3 g((unsigned)((B.nn1_max + SEL_THREADS - 1) / SEL_THREADS), (unsigned)B.count);
  SEL_PREC_LAUNCH(sel_mg_restrict_kernel, g, B);
  return hipGetLastError();
}

hipError_t sel_launch_mg_prolong(const SelBatch &B, hipStream_t st) {
  SEL_PREC_LAUNCH(sel_mg_prolong_kernel, parts_grid(B), B);
  return hipGetLastError();
}

hipError_t sel_launch_energy_sens(const SelBatch &B, long long nn, const double *d_g21, double *d_gE,
                                  hipStream_t st) {
  sel_fill_kernel<<<(unsigned)std::min<long long>((nn + SEL_THREADS - 1) / SEL_THREADS, 4096), SEL_THREADS, 0, st>>>(
      d_gE, nn);
  sel_energy_sens_kernel<<<parts_grid(B), SEL_THREADS, 0, st>>>(B, d_g21, d_gE);
  return hipGetLastError();
}

#undef SEL_PREC_LAUNCH

}  // namespace shh
