// Host driver of the selective (active-set) solve of Sec. 4.2: compaction of
// the active nodes, CG on the compact lists preconditioned by a multigrid
// V-cycle (voxel level on the active nodes, coarse levels the Galerkin grids
// of the culled operator) or by Jacobi (FP32 or FP64 vectors, FP64 dot
// products, FP64 residual replacement every R iterations in the mixed path),
// the energy form of C^H.
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"
#include "sel.hpp"

namespace shh {

namespace {

#define SEL_HIP(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return SHH_HIP_ERROR;      \
  } while (0)

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

// 1D integrals of the linear shape functions phi_0 = 1 - s, phi_1 = s on [0, 1]:
// value-value, derivative-derivative, and derivative-value products
double int1(int a, int b, int da, int db) {
  const double sa = a ? 1.0 : -1.0, sb = b ? 1.0 : -1.0;
  if (!da && !db) return a == b ? 1.0 / 3.0 : 1.0 / 6.0;
  if (da && db) return sa * sb;
  return da ? 0.5 * sa : 0.5 * sb;
}

// K_0 entry (corner a, component c; corner b, component c') of the unit
// voxel at E = 1: int lam d_c N_a d_c' N_b + mu d_c' N_a d_c N_b
// + mu delta_cc' grad N_a . grad N_b over the cube
double k0_entry(int a, int c, int b, int cp, double lam, double mu) {
  auto grad_pair = [&](int ca, int cb) {  // int d_ca N_a d_cb N_b
    double v = 1.0;
    for (int d = 0; d < 3; ++d) v *= int1((a >> d) & 1, (b >> d) & 1, d == ca, d == cb);
    return v;
  };
  double v = lam * grad_pair(c, cp) + mu * grad_pair(cp, c);
  if (c == cp) v += mu * (grad_pair(0, 0) + grad_pair(1, 1) + grad_pair(2, 2));
  return v;
}

// f0[k][a][c] = (K_0 chi^k) at corner a, component c; chi^k displaces corner b
// by eps^k b, eps^k the unit strain k in Voigt order with engineering shear
void element_forces(double lam, double mu, double (&f0)[NRHS][8][3]) {
  double eps[NRHS][3][3] = {};
  eps[0][0][0] = eps[1][1][1] = eps[2][2][2] = 1.0;
  const int pr[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  for (int k = 3; k < 6; ++k) eps[k][pr[k - 3][0]][pr[k - 3][1]] = eps[k][pr[k - 3][1]][pr[k - 3][0]] = 0.5;
  for (int k = 0; k < NRHS; ++k)
    for (int a = 0; a < 8; ++a)
      for (int c = 0; c < 3; ++c) {
        double v = 0.0;
        for (int b = 0; b < 8; ++b) {
          const double xb[3] = {double(b & 1), double((b >> 1) & 1), double((b >> 2) & 1)};
          for (int cp = 0; cp < 3; ++cp) {
            double chi = 0.0;
            for (int d = 0; d < 3; ++d) chi += eps[k][cp][d] * xb[d];
            v += k0_entry(a, c, b, cp, lam, mu) * chi;
          }
        }
        f0[k][a][c] = v;
      }
}

struct SelRun {
  SelDev h;
  SelDev *d = nullptr;
  hipStream_t st;
  bool timing = false;  // shh_profile_enable: HIP events around the timed launches
  std::vector<hipEvent_t> pool;
  struct Timed {
    hipEvent_t e0, e1;
    int kind;
  };
  std::vector<Timed> timed;
  ~SelRun() {
    resolve();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
  // launch `fn` bracketed by events when timing (family `kind`)
  template <typename F>
  int run_timed(int kind, F fn) {
    hipEvent_t e0 = timing ? event() : nullptr, e1 = timing ? event() : nullptr;
    if (e0 && e1) SEL_HIP(hipEventRecord(e0, st));
    SEL_HIP(fn());
    if (e0 && e1) {
      SEL_HIP(hipEventRecord(e1, st));
      timed.push_back({e0, e1, kind});
    } else {
      if (e0) pool.push_back(e0);
      if (e1) pool.push_back(e1);
    }
    return SHH_OK;
  }
  // after a synchronization: add the timed launches to the process-wide counters
  void resolve() {
    for (auto &t : timed) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.e0, t.e1) == hipSuccess) profile_add(t.kind, ms);
      pool.push_back(t.e0);
      pool.push_back(t.e1);
    }
    timed.clear();
  }
  int read_state(Slot &s) {
    SEL_HIP(hipMemcpyAsync(&s.state, s.d_state, sizeof(CgState), hipMemcpyDeviceToHost, st));
    SEL_HIP(hipStreamSynchronize(st));
    resolve();
    return SHH_OK;
  }
  // recompute r = f - K x64 for the cases of rmode (0 initial, 1 replacement, 2 final)
  int residual(int rmode) {
    if (rmode != 0) SEL_HIP(sel_launch_fold(d, h, rmode == 2 ? 1 : 0, st));
    int rc;
    if ((rc = run_timed(SHH_PROF_SEL_RESID, [&] { return sel_launch_op(d, h, 10 + rmode, st); }))) return rc;
    SEL_HIP(sel_launch_scalar(d, 100 + rmode, st));
    SEL_HIP(sel_launch_finish(d, h, rmode, st));
    SEL_HIP(sel_launch_scalar(d, rmode == 0 ? SSC_RESID_INIT : (rmode == 1 ? SSC_RESID_REPLACE : SSC_RESID_FINAL),
                              st));
    return SHH_OK;
  }
};

bool all_stopped(const CgState &c) {
  for (int k = 0; k < NRHS; ++k)
    if (c.active[k]) return false;
  return true;
}

}  // namespace

size_t sel_descriptor_bytes() { return sizeof(SelDev); }

int sel_solve(Slot &s, hipStream_t st) {
  const Layout &L = s.lay;
  const SlotDev &sd = s.host;
  const int n = sd.n;
  const long long nn = sd.nn;
  const int prec = sd.prec;
  const size_t ts = prec == SHH_PREC_FP64 ? 8 : 4;
  char *base = s.base;
  char *vec = base + L.vec;
  const size_t vb = L.vec_bytes;
  SelRun run;
  run.st = st;
  run.timing = s.timing && profile_on();
  SelDev &h = run.h;
  std::memset(&h, 0, sizeof(h));
  h.n = n;
  h.nn = nn;
  h.prec = prec;
  h.nchunks = int((nn + SEL_CHUNK - 1) / SEL_CHUNK);
  h.lam = sd.lam;
  h.mu = sd.mu;
  h.rtol = sd.rtol;
  h.ffloor = sd.ffloor;
  h.max_iter = sd.max_iter;
  element_forces(sd.lam, sd.mu, h.f0);
  h.E64 = sd.E64;
  h.st = sd.st;
  // compact arrays in the dense CG vector region (seven [6][3][n^3] vectors):
  // the map, coordinates, counts, moduli and diagonal in vectors 0-1, r, p,
  // q, x in vectors 2, 3, 4, 6, the partials in vector 5; the descriptor in
  // the slot's small parameter block
  h.r = vec + 2 * vb;
  h.p = vec + 3 * vb;
  h.q = vec + 4 * vb;
  h.x = vec + 6 * vb;
  h.x64 = prec == SHH_PREC_MIXED ? (double *)(base + L.x64) : (double *)h.x;
  char *aux = vec;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = aux + off;
    off = al256(off + bytes);
    return p;
  };
  h.map = (int *)take(sizeof(int) * nn);
  h.coord = (unsigned *)take(sizeof(unsigned) * nn);
  h.counts = (int *)take(sizeof(int) * (h.nchunks + 1));
  h.Ec = take(ts * nn);
  h.Ec64 = prec == SHH_PREC_FP64 ? (double *)h.Ec : (double *)take(sizeof(double) * nn);
  h.Dinv = take(ts * nn);
  if (off > 2 * vb) return SHH_WORKSPACE_TOO_SMALL;
  h.partials = (double *)(vec + 5 * vb);
  static_assert(sizeof(SelDev) <= 4096, "descriptor fits the parameter block");
  run.d = (SelDev *)(base + L.segs);
  int rc;
  // multigrid hierarchy of the culled operator (Galerkin levels from the
  // culled moduli; its element matrices use the vector region as scratch, so
  // it is built before the compaction writes there)
  if (s.opts.solver == SHH_SOLVER_SELECTIVE && L.mg && mg_num_levels(n) >= 2) {
    rc = mg_setup(s, st);
    if (rc == SHH_HIP_ERROR) return rc;
    h.mg = rc == SHH_OK ? 1 : 0;  // otherwise (a failed estimate) Jacobi
  }
  if (h.mg) {
    const MgDev &M = s.mg;
    h.inv_theta = M.lv[0].inv_theta;
    h.c1 = M.lv[0].c1;
    h.c2 = M.lv[0].c2;
    h.n1 = M.lv[1].n;
    h.nn1 = M.lv[1].nn;
    h.b1 = M.lv[1].b;
    h.x1 = M.lv[1].x;
    h.d0 = M.lv[0].d;  // the dense level-0 direction buffer: [6][3][n^3] >= [n_a][18]
  }
  if (s.ev[1]) SEL_HIP(hipEventRecord(s.ev[1], st));
  SEL_HIP(hipMemcpyAsync(run.d, &h, sizeof(SelDev), hipMemcpyHostToDevice, st));
  SEL_HIP(sel_launch_compact(run.d, h, st));
  int na = 0;
  SEL_HIP(hipMemcpyAsync(&na, h.counts + h.nchunks, sizeof(int), hipMemcpyDeviceToHost, st));
  SEL_HIP(hipStreamSynchronize(st));
  h.na = na;
  h.nparts = std::max(1, (na + SEL_THREADS - 1) / SEL_THREADS);
  const size_t pbytes = al256((size_t)NRHS * h.nparts * SEL_PS * sizeof(double));
  if (pbytes > vb || 22ull * h.nparts * sizeof(double) > vb) return SHH_WORKSPACE_TOO_SMALL;
  if (h.mg) {
    // three more [n_a][18] vectors of the V-cycle's voxel level: after the
    // compact arrays in vectors 0-1, then after the partials in vector 5
    const size_t vbytes = al256((size_t)na * 3 * NRHS * ts);
    char *arena[2] = {aux + off, vec + 5 * vb + pbytes};
    size_t room[2] = {2 * vb - off, vb - pbytes};
    void **dst[3] = {&h.d1, &h.xv, &h.rv};
    for (void **v : dst) {
      const int a = room[0] >= vbytes ? 0 : (room[1] >= vbytes ? 1 : -1);
      if (a < 0) {
        h.mg = 0;  // a nearly full design: no room, Jacobi
        break;
      }
      *v = arena[a];
      arena[a] += vbytes;
      room[a] -= vbytes;
    }
  }
  SEL_HIP(hipMemcpyAsync(run.d, &h, sizeof(SelDev), hipMemcpyHostToDevice, st));
  s.sel_active_nodes = na;
  if (na == 0) {  // everything culled: no stiffness, C^H = 0
    SEL_HIP(hipMemcpyAsync(&s.state, s.d_state, sizeof(CgState), hipMemcpyDeviceToHost, st));
    SEL_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < 36; ++i) s.state.C[i] = 0.0;
    for (int k = 0; k < NRHS; ++k) {
      s.state.iters[k] = 0;
      s.state.rel_true[k] = 0.0;
      s.state.status[k] = ST_CONVERGED;
    }
    s.status = SHH_OK;
    s.finished = true;
    return SHH_OK;
  }
  SEL_HIP(sel_launch_gather(run.d, h, st));
  SEL_HIP(sel_launch_zero(run.d, h, st));
  if ((rc = run.residual(0))) return rc;
  // multigrid-preconditioned CG (the V-cycle: a Chebyshev pre-smoothing of
  // the CG residual at the voxel level, restriction to level 1, the coarse
  // levels' V-cycle, prolongation, post-smoothing):
  //   restart:   z = V r, rho = r . z, beta = 0
  //   iteration: p = z + beta p; q = K p; alpha = rho / p . q;
  //              x += alpha p, r -= alpha q; z = V r; rho' = r . z; beta
  auto vcycle = [&](int restart) -> int {
    if ((rc = run.run_timed(SHH_PROF_SEL_MG_VEC, [&] { return sel_launch_mg_s1(run.d, h, restart, st); })))
      return rc;
    for (int m : {SMO_STEP1, SMO_RES}) {
      if ((rc = run.run_timed(SHH_PROF_SEL_MG_SMOOTH, [&] { return sel_launch_mg_op(run.d, h, m, st); })))
        return rc;
    }
    if ((rc = run.run_timed(SHH_PROF_SEL_MG_TRANSFER, [&] { return sel_launch_mg_restrict(run.d, h, st); })))
      return rc;
    if ((rc = mg_vcycle_coarse(s, st))) return rc;
    if ((rc = run.run_timed(SHH_PROF_SEL_MG_TRANSFER, [&] { return sel_launch_mg_prolong(run.d, h, st); })))
      return rc;
    for (int m : {SMO_POST, SMO_LAST}) {
      if ((rc = run.run_timed(SHH_PROF_SEL_MG_SMOOTH, [&] { return sel_launch_mg_op(run.d, h, m, st); })))
        return rc;
    }
    return SHH_OK;
  };
  auto restart = [&]() -> int {
    if ((rc = vcycle(1))) return rc;
    SEL_HIP(sel_launch_scalar(run.d, SSC_MG_RESTART, st));
    return SHH_OK;
  };
  if (h.mg) {
    if ((rc = restart())) return rc;
  } else {
    SEL_HIP(sel_launch_dir0(run.d, h, st));
  }
  if (s.ev[2]) SEL_HIP(hipEventRecord(s.ev[2], st));
  const int R = prec == SHH_PREC_MIXED ? s.opts.recompute_every : 0;
  const int check = std::max(1, s.opts.check_every);
  long long launched = 0;
  const long long guard = 4LL * s.opts.max_iter + 64LL * check + 1024;
  int finals = 0;
  if ((rc = run.read_state(s))) return rc;
  while (!all_stopped(s.state)) {
    for (int j = 0; j < check; ++j) {
      if (h.mg) {
        if ((rc = run.run_timed(SHH_PROF_SEL_MG_VEC, [&] { return sel_launch_mg_dir(run.d, h, st); }))) return rc;
        if ((rc = run.run_timed(SHH_PROF_SEL_MG_PQ, [&] { return sel_launch_mg_op(run.d, h, SMO_PQ, st); })))
          return rc;
        SEL_HIP(sel_launch_scalar(run.d, SSC_MG_ALPHA, st));
        if ((rc = vcycle(0))) return rc;
        SEL_HIP(sel_launch_scalar(run.d, SSC_MG_BETA, st));
      } else {
        if ((rc = run.run_timed(SHH_PROF_SEL_OP, [&] { return sel_launch_op(run.d, h, SOP_PCG, st); }))) return rc;
        SEL_HIP(sel_launch_scalar(run.d, SSC_ITER, st));
        if ((rc = run.run_timed(SHH_PROF_SEL_UPDATE, [&] { return sel_launch_update(run.d, h, st); }))) return rc;
      }
      ++launched;
      if (R > 0 && launched % R == 0) {
        if ((rc = run.residual(1))) return rc;
        if (h.mg && (rc = restart())) return rc;  // the V-cycle of the replaced residual
      }
    }
    if ((rc = run.read_state(s))) return rc;
    if (all_stopped(s.state)) {
      // the true residual decides: a case whose recursive residual was
      // optimistic resumes (at most 8 times)
      if ((rc = run.residual(2))) return rc;
      ++finals;
      if ((rc = run.read_state(s))) return rc;
      if (finals >= 8) break;
      if (h.mg && !all_stopped(s.state) && (rc = restart())) return rc;
    }
    if (launched > guard) break;
  }
  if (!all_stopped(s.state) || finals == 0) {
    if ((rc = run.residual(2))) return rc;
  }
  if (s.ev[3]) SEL_HIP(hipEventRecord(s.ev[3], st));
  SEL_HIP(sel_launch_fold(run.d, h, 1, st));
  SEL_HIP(sel_launch_op(run.d, h, SOP_ENERGY, st));
  SEL_HIP(sel_launch_scalar(run.d, SSC_ENERGY, st));
  if (s.ev[4]) SEL_HIP(hipEventRecord(s.ev[4], st));
  if ((rc = run.read_state(s))) return rc;
  float a = 0.f;
  for (int k = 0; k < 4; ++k)
    if (s.ev[k] && s.ev[k + 1] && hipEventElapsedTime(&a, s.ev[k], s.ev[k + 1]) == hipSuccess) s.ms[k] = a;
  if (s.ev[0] && s.ev[4] && hipEventElapsedTime(&a, s.ev[0], s.ev[4]) == hipSuccess) s.ms[4] = a;
  int status = SHH_OK;
  for (int k = 0; k < NRHS; ++k) {
    if (s.state.status[k] == ST_BREAKDOWN) status = SHH_BREAKDOWN;
    else if (status == SHH_OK && s.state.status[k] != ST_CONVERGED) status = SHH_NOT_CONVERGED;
  }
  s.status = status;
  s.finished = true;
  return SHH_OK;
}

}  // namespace shh
