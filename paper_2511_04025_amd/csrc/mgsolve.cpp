// Host side of the multigrid-preconditioned CG (see mg.hpp): memory carving,
// setup (Galerkin hierarchy, coarsest inverse, Chebyshev bounds) and the
// V-cycle / CG launch sequence of one iteration.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <vector>

#include "hexop.hpp"
#include "kernels.hpp"
#include "runtime.hpp"

namespace shh {

#define SHH_HIP(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return SHH_HIP_ERROR;      \
  } while (0)

hipError_t mg_launch_elem1(const SlotDev *d_slot, const MgDev *d_mg, long long nn1, int prec, hipStream_t st);
hipError_t mg_launch_elemc(const MgDev *d_mg, int l, long long nn_next, int prec, hipStream_t st);
hipError_t mg_launch_stencil(const MgDev *d_mg, int l, long long nn, int prec, hipStream_t st);
hipError_t mg_launch_coarse_inverse(const MgBatch &B, int prec, hipStream_t st);
// live = 1: skip the load cases whose CG has stopped (state read on the device)
// ep: the Chebyshev sweep fused into the output stage (MGE_*)
hipError_t mg_launch_apply(const MgBatch &B, int l, int src, long long nn_max, bool even, int prec,
                           hipStream_t st, int live, int ep);
hipError_t mg_launch_apply_case0(const MgBatch &B, int l, long long nn_max, int prec, hipStream_t st);
bool mg_apply_wide(long long nn_max);
hipError_t mg_launch_restrict(const MgBatch &B, int l, long long nn_coarse_max, int prec,
                              hipStream_t st);
hipError_t mg_launch_prolong(const MgBatch &B, int l, long long nn_coarse_max, int prec, hipStream_t st);
hipError_t mg_launch_coarsest(const MgBatch &B, int prec, hipStream_t st);
hipError_t mg_launch_vec(const MgBatch &B, int l, int nchunks_max, int prec, hipStream_t st);
hipError_t mg_launch_scalar(const MgBatch &B, int phase, hipStream_t st);
hipError_t mg_launch_power(const MgBatch &B, int l, int phase, int nchunks_max, int prec, hipStream_t st);

namespace {

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int POWER_ITERS = 30;  // power steps per coarse level
// Chebyshev interval [hi / SHH_CHEB_RATIO, hi]; hi is the voxel level's
// element bound times SHH_CHEB_BOUND0, and SHH_CHEB_COARSE times the power
// estimate on coarse levels (compile-time, for A/B builds)
#ifndef SHH_CHEB_RATIO
#define SHH_CHEB_RATIO 33.0
#endif
#ifndef SHH_CHEB_BOUND0
#define SHH_CHEB_BOUND0 1.0
#endif
#ifndef SHH_CHEB_COARSE
#define SHH_CHEB_COARSE 1.2
#endif

// Lay out the multigrid region at `base` (nullptr: sizing only).  Fills the
// level descriptors' persistent buffers, G and Mc.
size_t carve(char *base, int n, int prec, MgDev *mg, char **d_mgdev) {
  const size_t ts = prec == SHH_PREC_FP64 ? 8 : 4;
  const int count = mg_num_levels(n);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = a256(off + bytes);
    return base ? base + o : nullptr;
  };
  char *dev = take(sizeof(MgDev));
  char *G = take(8 * 576 * ts);
  // the voxel level's stored Chebyshev direction (its other V-cycle vectors
  // alias CG vectors)
  char *d0 = take((size_t)NRHS * 3 * (size_t)n * n * n * ts);
  if (mg) {
    mg->L = count - 1;
    mg->G = G;
    mg->lv[0].d = d0;
  }
  if (d_mgdev) *d_mgdev = dev;
  long long nl = n;
  for (int l = 1; l < count; ++l) {
    nl /= 2;
    const long long nn = nl * nl * nl;
    char *S = take(MG_STENCIL * nn * ts);
    char *D = take(3 * nn * ts);
    char *v[5];
    for (int k = 0; k < 5; ++k) v[k] = take((size_t)NRHS * 3 * nn * ts);
    if (mg) {
      MgLevel &L = mg->lv[l];
      L.n = int(nl);
      L.nn = nn;
      L.nchunks = int((nn + CHUNK - 1) / CHUNK);
      L.S = S;
      L.Dinv = D;
      L.b = v[0];
      L.x = v[1];
      L.r = v[2];
      L.d = v[3];
      L.q = v[4];
    }
  }
  const long long nc = nl * nl * nl;
  char *Mc = take((size_t)(3 * nc) * (3 * nc) * sizeof(double));
  if (mg) {
    mg->ndof_c = int(3 * nc);
    mg->Mc = (double *)Mc;
  }
  return off;
}

// Dense K_0 (DOF 3 a + c, corner a = ax + 2 ay + 4 az) of the factored operator:
// K_0 v = H^T hex_apply(H v) with H[m][a] = prod_axis (m bit ? 2 a bit - 1 : 1).
void dense_k0(const double kop[KOP_N], double K0[24][24]) {
  auto H = [](int m, int a) {
    int s = 1;
    for (int d = 0; d < 3; ++d)
      if ((m >> d) & 1) s *= ((a >> d) & 1) ? 1 : -1;
    return double(s);
  };
  for (int j = 0; j < 24; ++j) {
    double h[3][8] = {}, y[3][8] = {};
    const int aj = j / 3, cj = j % 3;
    for (int m = 0; m < 8; ++m) h[cj][m] = H(m, aj);
    hex_apply<double>(kop, h, y, 1.0);
    for (int a = 0; a < 8; ++a)
      for (int c = 0; c < 3; ++c) {
        double v = 0.0;
        for (int m = 0; m < 8; ++m) v += H(m, a) * y[c][m];
        K0[3 * a + c][j] = v;
      }
  }
}

// lambda_max(diag(K_0)^-1 K_0): since K = sum_e E_e K_0 with D = sum_e E_e
// diag(K_0), x^T K x <= this value times x^T D x, so it bounds
// lambda_max(D^-1 K) on the voxel grid whatever the moduli.  It is the
// largest eigenvalue of the symmetric D_0^-1/2 K_0 D_0^-1/2, found by cyclic
// Jacobi rotations (converged to rounding; a power iteration's Rayleigh
// quotient would only approach it from below).
double element_bound(const double K0[24][24]) {
  constexpr int N = 24;
  double A[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) A[i][j] = K0[i][j] / std::sqrt(K0[i][i] * K0[j][j]);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < N; ++i) {
      diag += A[i][i] * A[i][i];
      for (int j = i + 1; j < N; ++j) off += A[i][j] * A[i][j];
    }
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q) {
        if (A[p][q] == 0.0) continue;
        // rotation that zeroes A[p][q] (Golub & Van Loan, symmetric Schur)
        const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < N; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  double lam = A[0][0];
  for (int i = 1; i < N; ++i) lam = std::max(lam, A[i][i]);
  return lam;
}

double qweight(int f, int b, int a) {
  double w = 1.0;
  for (int d = 0; d < 3; ++d) {
    const double p = 0.5 * (((f >> d) & 1) + ((b >> d) & 1));
    w *= ((a >> d) & 1) ? p : 1.0 - p;
  }
  return w;
}

// G_f = Q_f^T K_0 Q_f for the 8 children f of a coarse element.
void child_galerkin(const double K0[24][24], std::vector<double> &G) {
  G.assign(8 * 576, 0.0);
  for (int f = 0; f < 8; ++f) {
    double Q[24][24] = {};
    for (int b = 0; b < 8; ++b)
      for (int a = 0; a < 8; ++a)
        for (int c = 0; c < 3; ++c) Q[3 * b + c][3 * a + c] = qweight(f, b, a);
    double T[24][24] = {};
    for (int i = 0; i < 24; ++i)
      for (int k = 0; k < 24; ++k) {
        double v = 0.0;
        for (int j = 0; j < 24; ++j) v += K0[i][j] * Q[j][k];
        T[i][k] = v;
      }
    for (int i = 0; i < 24; ++i)
      for (int k = 0; k < 24; ++k) {
        double v = 0.0;
        for (int j = 0; j < 24; ++j) v += Q[j][i] * T[j][k];
        G[(f * 24 + i) * 24 + k] = v;
      }
  }
}

// The constants of one element operator (a Poisson ratio): the voxel-level
// bound and the child Galerkin matrices, computed once per process and kept
// for the last few operators seen.
void nu_constants(const double kop[KOP_N], double &bound0, std::vector<double> &G) {
  struct Entry {
    double kop[KOP_N];
    double bound0;
    std::vector<double> G;
  };
  static std::mutex mu;
  static std::deque<Entry> cache;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry &e : cache)
      if (std::memcmp(e.kop, kop, sizeof(e.kop)) == 0) {
        bound0 = e.bound0;
        G = e.G;
        return;
      }
  }
  double K0[24][24];
  dense_k0(kop, K0);
  bound0 = element_bound(K0);
  child_galerkin(K0, G);
  std::lock_guard<std::mutex> lock(mu);
  Entry e;
  std::memcpy(e.kop, kop, sizeof(e.kop));
  e.bound0 = bound0;
  e.G = G;
  cache.push_back(std::move(e));
  if (cache.size() > 8) cache.pop_front();
}

template <typename T>
int upload_as(const std::vector<double> &src, void *dst, hipStream_t st) {
  std::vector<T> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
  SHH_HIP(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, st));
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int upload(const std::vector<double> &src, void *dst, int prec, hipStream_t st) {
  return prec == SHH_PREC_FP64 ? upload_as<double>(src, dst, st) : upload_as<float>(src, dst, st);
}

MgBatch batch_of(const std::vector<Slot *> &slots) {
  MgBatch B;
  std::memset(&B, 0, sizeof(B));
  B.count = int(slots.size());
  for (int i = 0; i < B.count; ++i) {
    B.slot[i] = slots[i]->d_slot;
    B.mg[i] = slots[i]->d_mg;
  }
  return B;
}

// One V-cycle from level l down, for slots that all have at least l + 1
// levels; slots whose coarsest level is l take the dense solve there.
int vcycle(const std::vector<Slot *> &slots, int l, hipStream_t st, Solver *timer, const MgApply0 &apply0) {
  const int prec = slots[0]->host.prec;
  std::vector<Slot *> coarse, smooth;
  for (Slot *s : slots) (s->mg.L == l ? coarse : smooth).push_back(s);
  if (!coarse.empty()) SHH_HIP(mg_launch_coarsest(batch_of(coarse), prec, st));
  if (smooth.empty()) return SHH_OK;
  const MgBatch B = batch_of(smooth);
  long long nn_max = 0, nn_next_max = 0;
  int nch_max = 0;
  bool all_even = true;  // the two-nodes-per-thread operator form needs even n
  for (Slot *s : smooth) {
    nn_max = std::max(nn_max, s->mg.lv[l].nn);
    nn_next_max = std::max(nn_next_max, s->mg.lv[l + 1].nn);
    nch_max = std::max(nch_max, s->mg.lv[l].nchunks);
    all_even = all_even && s->mg.lv[l].n % 2 == 0;
  }
  int rc;
  // when profiling, the voxel level's launches and the first coarse level's
  // operator are timed by kernel family (the rest is small)
  hipEvent_t e0 = nullptr;
  auto tb = [&](bool on) -> int { return (on && timer) ? timer->timed_begin(&e0) : (e0 = nullptr, 0); };
  auto te = [&](int kind) -> int { return (e0 && timer) ? timer->timed_end(e0, kind) : 0; };
  auto vec = [&]() -> int {
    if ((rc = tb(l == 0))) return rc;
    SHH_HIP(mg_launch_vec(B, l, nch_max, prec, st));
    return te(SHH_PROF_MG_UPDATE);
  };
  // an operator pass with the Chebyshev sweep after it fused in: the voxel
  // level's stencil passes, the coarse levels' stored-stencil passes
  auto app = [&](int src0, int ep) -> int {
    if (l == 0) return apply0(smooth, src0);
    if ((rc = tb(l == 1))) return rc;
    SHH_HIP(mg_launch_apply(B, l, 0, nn_max, all_even, prec, st, 1, ep));
    return te(SHH_PROF_MG_APPLY1);
  };
  // pre-smoother (at the voxel level INIT also applies the pending CG
  // update); with degree 2 the second pass leaves r - A d1, the residual to
  // restrict, in r.  Degree-1 smoothing at the voxel level: the first step
  // alone (its r is the residual to restrict), and after the correction one
  // pass that leaves z = x + D r / theta
  const bool deg1 = l == 0 && SHH_MG_DEG0 == 1;
  if ((rc = vec()) || (rc = app(MG_SRC_STEP1, MGE_STEP1)) || (!deg1 && (rc = app(MG_SRC_RES, MGE_RES)))) return rc;
  // coarse-grid correction
  if ((rc = tb(l == 0))) return rc;
  SHH_HIP(mg_launch_restrict(B, l, nn_next_max, prec, st));
  if ((rc = te(SHH_PROF_MG_RESTRICT))) return rc;
  if ((rc = vcycle(smooth, l + 1, st, timer, apply0))) return rc;
  if ((rc = tb(l == 0))) return rc;
  SHH_HIP(mg_launch_prolong(B, l, nn_next_max, prec, st));
  if ((rc = te(SHH_PROF_MG_PROLONG))) return rc;
  // post-smoother
  if (deg1) return app(MG_SRC_POST1, MGE_NONE);
  if ((rc = app(MG_SRC_POST, MGE_POST)) || (rc = app(MG_SRC_LAST, MGE_LAST))) return rc;
  return SHH_OK;
}

}  // namespace

size_t mg_region_bytes(int n, int prec) {
  if (mg_num_levels(n) < 2) return 0;
  return carve(nullptr, n, prec, nullptr, nullptr);
}

namespace {

// Setup of one slot up to the power iteration: level descriptors, the
// nu-dependent constants, element matrices, stencils, D^-1 of every coarse
// level and the coarsest inverse (all on the stream, no read-back).
int mg_setup_levels(Slot &s, hipStream_t st, double &bound0) {
  SlotDev &h = s.host;
  const int n = h.n, prec = h.prec;
  const int count = mg_num_levels(n);
  if (count < 2 || s.lay.mg == 0 || !s.lay.vectors) return SHH_UNSUPPORTED;
  const size_t ts = prec == SHH_PREC_FP64 ? 8 : 4;
  std::memset(&s.mg, 0, sizeof(s.mg));
  char *dev = nullptr;
  carve(s.base + s.lay.mg, n, prec, &s.mg, &dev);
  s.d_mg = (MgDev *)dev;
  MgDev &mg = s.mg;
  MgLevel &L0 = mg.lv[0];
  L0.n = n;
  L0.nn = h.nn;
  L0.nchunks = h.nchunks;
  L0.Dinv = h.Dinv;
  L0.b = h.r[0];
  L0.x = h.r[1];
  L0.r = h.q[1];
  L0.q = h.q[0];
  h.mgd = L0.d;
  SHH_HIP(hipMemcpyAsync(&s.d_slot->mgd, &h.mgd, sizeof(h.mgd), hipMemcpyHostToDevice, st));
  // element matrices of levels >= 1 live in the (not yet used) CG vector region
  {
    char *ke = s.base + s.lay.vec;
    size_t used = 0;
    for (int l = 1; l < count; ++l) {
      mg.lv[l].Ke = ke + used;
      used = a256(used + (size_t)mg.lv[l].nn * 576 * ts);
    }
    if (used > 7 * s.lay.vec_bytes) return SHH_WORKSPACE_TOO_SMALL;
  }
  // child Galerkin matrices of this Poisson ratio's K_0 and the voxel-level
  // Chebyshev bound (host work of about 1 ms, kept per element operator)
  std::vector<double> G;
  nu_constants(h.kop64, bound0, G);
  int rc;
  if ((rc = upload(G, mg.G, prec, st))) return rc;
  SHH_HIP(hipMemcpyAsync(s.d_mg, &mg, sizeof(MgDev), hipMemcpyHostToDevice, st));
  SHH_HIP(mg_launch_elem1(s.d_slot, s.d_mg, mg.lv[1].nn, prec, st));
  for (int l = 1; l + 1 < count; ++l) SHH_HIP(mg_launch_elemc(s.d_mg, l, mg.lv[l + 1].nn, prec, st));
  for (int l = 1; l < count; ++l) SHH_HIP(mg_launch_stencil(s.d_mg, l, mg.lv[l].nn, prec, st));
  return SHH_OK;  // the coarsest inverse follows, batched over the slots (mg_setup)
}

// Chebyshev coefficients of every smoothing level from the estimates, and
// their upload.
int mg_setup_coefficients(Slot &s, const MgDev &est, double bound0, hipStream_t st) {
  SlotDev &h = s.host;
  MgDev &mg = s.mg;
  for (int l = 0; l < mg.L; ++l) {
    MgLevel &W = mg.lv[l];
    // Chebyshev interval [hi/33, hi]: above lambda_max, or the smoother
    // amplifies the top of the spectrum and the V-cycle stops being positive
    // definite.  The voxel level takes the rigorous element bound
    // lambda_max(diag(K_0)^-1 K_0) >= lambda_max(D^-1 K) (its power estimates
    // on the headline designs, 3.0 to 4.2, sit well below it); the Rayleigh
    // quotients of a coarse level bound its lambda_max from below, so those
    // levels take 1.2 x the estimate (1.5 cost 5-9 % more iterations on the
    // headline designs; neither broke down on 64 random designs of 16^3 to
    // 128^3 with either solver).
    const double lam = l == 0 ? bound0 : est.lv[l].lmax;
    if (!(lam > 0.0) || !std::isfinite(lam)) return SHH_BREAKDOWN;
    W.lmax = lam;
    if (std::getenv("SHH_MG_VERBOSE"))
      std::fprintf(stderr, "mg setup: n=%d level %d (n=%d) lambda_max %.5f%s\n", h.n, l, W.n, lam,
                   l == 0 ? " (bound)" : "");
    const double hi = l == 0 ? SHH_CHEB_BOUND0 * bound0 : SHH_CHEB_COARSE * lam, lo = hi / SHH_CHEB_RATIO;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sigma = theta / delta, rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
    W.inv_theta = 1.0 / theta;
    W.c1 = rho1 * rho0;
    W.c2 = 2.0 * rho1 / delta;
    // one step, x = D b / theta, where the voxel level smooths with degree 1
    // (the selective solve takes these coefficients for its own voxel level)
    if (l == 0 && (is_selective(s.opts.solver) ? SHH_SEL_DEG0 : SHH_MG_DEG0) == 1) W.c1 = W.c2 = 0.0;
  }
  // the fused voxel-level sweeps read the coefficients from the slot
  h.mgc[0] = mg.lv[0].inv_theta;
  h.mgc[1] = mg.lv[0].c1;
  h.mgc[2] = mg.lv[0].c2;
  SHH_HIP(hipMemcpyAsync(&s.d_slot->mgc, h.mgc, sizeof(h.mgc), hipMemcpyHostToDevice, st));
  SHH_HIP(hipMemcpyAsync(s.d_mg, &mg, sizeof(MgDev), hipMemcpyHostToDevice, st));
  s.mg_restart = true;
  return SHH_OK;
}

}  // namespace

int mg_setup(const std::vector<Slot *> &all, hipStream_t st, std::vector<int> *rcs) {
  if (rcs) rcs->assign(all.size(), SHH_OK);
  if (all.empty()) return SHH_OK;
  const int prec = all[0]->host.prec;
  // a slot's own failure is recorded (when asked) and the slot left out;
  // HIP errors end the setup of all
  auto fail = [&](size_t i, int rc) { return (!rcs || rc == SHH_HIP_ERROR) ? rc : ((*rcs)[i] = rc, 0); };
  std::vector<Slot *> slots;
  std::vector<size_t> idx;
  std::vector<double> bound0;
  int rc;
  int max_l = 0;
  for (size_t i = 0; i < all.size(); ++i) {
    double b0 = 0.0;
    if ((rc = mg_setup_levels(*all[i], st, b0))) {
      if ((rc = fail(i, rc))) return rc;
      continue;
    }
    slots.push_back(all[i]);
    idx.push_back(i);
    bound0.push_back(b0);
    max_l = std::max(max_l, all[i]->mg.L);
  }
  if (slots.empty()) return SHH_OK;
  // the coarsest levels' dense inverses, one workgroup per slot (a launch
  // per slot ran them one after another: 1.8 ms each)
  for (size_t b0 = 0; b0 < slots.size(); b0 += MG_MAXB) {
    const std::vector<Slot *> part(slots.begin() + b0, slots.begin() + std::min(slots.size(), b0 + MG_MAXB));
    SHH_HIP(mg_launch_coarse_inverse(batch_of(part), prec, st));
  }
  // lambda_max(D^-1 A) of every coarse smoothing level by power iteration
  // on load case 0, entirely on the device and batched over the slots that
  // have the level (phase 0 start, then per step: apply, phase 1 sweep,
  // reduction, phase 2 normalization); one read-back at the end.  The voxel
  // level needs none: it takes the rigorous bound.
  for (int l = 1; l < max_l; ++l) {
    std::vector<Slot *> at;
    for (Slot *s : slots)
      if (s->mg.L > l) at.push_back(s);
    for (size_t b0 = 0; b0 < at.size(); b0 += MG_MAXB) {
      const std::vector<Slot *> part(at.begin() + b0, at.begin() + std::min(at.size(), b0 + MG_MAXB));
      const MgBatch B = batch_of(part);
      long long nn = 0;
      int nch = 0;
      for (Slot *s : part) {
        nn = std::max(nn, s->mg.lv[l].nn);
        nch = std::max(nch, s->mg.lv[l].nchunks);
      }
      SHH_HIP(mg_launch_power(B, l, 0, nch, prec, st));
      for (int it = 0; it < POWER_ITERS; ++it) {
        SHH_HIP(mg_launch_apply_case0(B, l, nn, prec, st));
        SHH_HIP(mg_launch_power(B, l, 1, nch, prec, st));
        SHH_HIP(mg_launch_power(B, l, 3, nch, prec, st));
        SHH_HIP(mg_launch_power(B, l, 2, nch, prec, st));
      }
    }
  }
  std::vector<MgDev> est(slots.size());
  for (size_t i = 0; i < slots.size(); ++i)
    SHH_HIP(hipMemcpyAsync(&est[i], slots[i]->d_mg, sizeof(MgDev), hipMemcpyDeviceToHost, st));
  SHH_HIP(hipStreamSynchronize(st));
  for (size_t i = 0; i < slots.size(); ++i)
    if ((rc = mg_setup_coefficients(*slots[i], est[i], bound0[i], st)) && (rc = fail(idx[i], rc))) return rc;
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int mg_setup(Slot &s, hipStream_t st) { return mg_setup(std::vector<Slot *>{&s}, st); }

int mg_vcycle_coarse(const std::vector<Slot *> &slots, hipStream_t st) {
  for (Slot *s : slots)
    if (s->mg.L < 1) return SHH_UNSUPPORTED;
  // levels >= 1 never call the voxel-level operator
  const MgApply0 none = [](const std::vector<Slot *> &, int) { return SHH_UNSUPPORTED; };
  int rc;
  for (size_t b0 = 0; b0 < slots.size(); b0 += MG_MAXB) {
    const std::vector<Slot *> part(slots.begin() + b0, slots.begin() + std::min(slots.size(), b0 + MG_MAXB));
    if ((rc = vcycle(part, 1, st, nullptr, none))) return rc;
  }
  return SHH_OK;
}

int mg_apply_level(Slot &s, int l, const void *d_v, void *d_q, hipStream_t st) {
  if (l < 1 || l > s.mg.L) return SHH_INVALID_ARG;
  const MgLevel &L = s.mg.lv[l];
  const size_t bytes = (size_t)NRHS * 3 * L.nn * (s.host.prec == SHH_PREC_FP64 ? 8 : 4);
  SHH_HIP(hipMemcpyAsync(L.x, d_v, bytes, hipMemcpyDeviceToDevice, st));
  SHH_HIP(mg_launch_apply(batch_of({&s}), l, 0, L.nn, L.n % 2 == 0, s.host.prec, st, 0, MGE_NONE));
  SHH_HIP(hipMemcpyAsync(d_q, L.q, bytes, hipMemcpyDeviceToDevice, st));
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int mg_iterate(const std::vector<Slot *> &all, hipStream_t st, Solver *timer, const MgApply0 &apply0) {
  if (all.empty()) return SHH_OK;
  int rc;
  for (size_t b0 = 0; b0 < all.size(); b0 += MG_MAXB) {
    const std::vector<Slot *> slots(all.begin() + b0, all.begin() + std::min(all.size(), b0 + MG_MAXB));
    // slots with a new residual: z = V r, rho = r . z, and beta = 0 (a
    // restart: the direction pass then starts from p = z) or, after a
    // residual replacement, beta rho' / rho (the direction is kept)
    std::vector<Slot *> rs, restart, keep;
    for (Slot *s : slots)
      if (s->mg_restart) {
        rs.push_back(s);
        (s->mg_keep_dir ? keep : restart).push_back(s);
      }
    if (!rs.empty()) {
      if ((rc = vcycle(rs, 0, st, timer, apply0))) return rc;
      if (!restart.empty()) SHH_HIP(mg_launch_scalar(batch_of(restart), MGS_RESTART, st));
      if (!keep.empty()) SHH_HIP(mg_launch_scalar(batch_of(keep), MGS_REPLACE, st));
      for (Slot *s : rs) s->mg_restart = s->mg_keep_dir = false;
    }
    const MgBatch B = batch_of(slots);
    // p = z + beta p, q = K p, partials p . q in one pass; alpha
    if ((rc = apply0(slots, MG_SRC_DIR))) return rc;
    SHH_HIP(mg_launch_scalar(B, MGS_ALPHA, st));
    // the V-cycle's first sweep applies x += alpha p, r -= alpha q
    if ((rc = vcycle(slots, 0, st, timer, apply0))) return rc;
    SHH_HIP(mg_launch_scalar(B, MGS_BETA, st));
  }
  return SHH_OK;
}

}  // namespace shh
