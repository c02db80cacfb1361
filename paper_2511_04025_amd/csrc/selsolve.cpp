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

}  // namespace

// Where one design's selective solve stands, kept with its slot between the
// steps of a batch call or of the engine: the host copy of the descriptor, the
// device copy, the preconditioner, and the iteration and check counts.
struct SelHost {
  SelDev h;
  SelDev *d = nullptr;
  size_t aux = 0;        // bytes of the compact arrays in vectors 0-1
  bool mg = false;       // multigrid-preconditioned (else Jacobi)
  bool done = false;     // converged (true residual checked), or given up
  int finals = 0;        // final residual checks so far
  long long launched = 0;  // CG iterations launched
};

namespace {

SelHost &H(Slot *s) { return *s->sel; }

SelBatch batch_of(const std::vector<Slot *> &v) {
  SelBatch B;
  std::memset(&B, 0, sizeof(B));
  B.count = int(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    const SelHost &x = H(v[i]);
    B.d[i] = x.d;
    B.prec = x.h.prec;
    B.parts_max = std::max(B.parts_max, x.h.nparts);
    B.chunks_max = std::max(B.chunks_max, x.h.nchunks);
    B.nn1_max = std::max(B.nn1_max, x.h.nn1);
  }
  return B;
}

bool all_stopped(const CgState &c) {
  for (int k = 0; k < NRHS; ++k)
    if (c.active[k]) return false;
  return true;
}

// the slots in launches of at most SEL_MAXB
template <typename F>
int chunked(const std::vector<Slot *> &v, F fn) {
  int rc;
  for (size_t b0 = 0; b0 < v.size(); b0 += SEL_MAXB) {
    const std::vector<Slot *> part(v.begin() + b0, v.begin() + std::min(v.size(), b0 + SEL_MAXB));
    if ((rc = fn(part))) return rc;
  }
  return SHH_OK;
}

struct SelRun {
  hipStream_t st;
  bool timing = false;  // shh_profile_enable: HIP events around the timed launches
  std::vector<hipEvent_t> pool;
  struct Timed {
    hipEvent_t e0, e1;
    int kind;
  };
  std::vector<Timed> timed;
  SelRun(hipStream_t s, const std::vector<Slot *> &v) : st(s) {
    timing = !v.empty() && v[0]->timing && profile_on();
  }
  ~SelRun() {
    (void)hipStreamSynchronize(st);
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
  int read_state(const std::vector<Slot *> &v) {
    for (Slot *s : v) SEL_HIP(hipMemcpyAsync(&s->state, s->d_state, sizeof(CgState), hipMemcpyDeviceToHost, st));
    SEL_HIP(hipStreamSynchronize(st));
    resolve();
    return SHH_OK;
  }
  void record(const std::vector<Slot *> &v, int k) {
    for (Slot *s : v)
      if (s->ev[k]) (void)hipEventRecord(s->ev[k], st);
  }
  // recompute r = f - K x64 for the cases of rmode (0 initial, 1 replacement, 2 final)
  int residual(const std::vector<Slot *> &v, int rmode) {
    return chunked(v, [&](const std::vector<Slot *> &part) {
      const SelBatch B = batch_of(part);
      if (rmode != 0) SEL_HIP(sel_launch_fold(B, rmode == 2 ? 1 : 0, st));
      int rc;
      if ((rc = run_timed(SHH_PROF_SEL_RESID, [&] { return sel_launch_op(B, 10 + rmode, st); }))) return rc;
      SEL_HIP(sel_launch_scalar(B, 100 + rmode, st));
      SEL_HIP(sel_launch_finish(B, rmode, st));
      SEL_HIP(sel_launch_scalar(
          B, rmode == 0 ? SSC_RESID_INIT : (rmode == 1 ? SSC_RESID_REPLACE : SSC_RESID_FINAL), st));
      return SHH_OK;
    });
  }
  // multigrid-preconditioned CG (the V-cycle: a Chebyshev pre-smoothing of
  // the CG residual at the voxel level, restriction to level 1, the coarse
  // levels' V-cycle, prolongation, post-smoothing):
  //   restart:   z = V r, rho = r . z, beta = 0
  //   iteration: p = z + beta p; q = K p; alpha = rho / p . q;
  //              x += alpha p, r -= alpha q; z = V r; rho' = r . z; beta
  int vcycle(const SelBatch &B, const std::vector<Slot *> &ss, int restart) {
    int rc;
    if ((rc = run_timed(SHH_PROF_SEL_MG_VEC, [&] { return sel_launch_mg_s1(B, restart, st); }))) return rc;
    // degree-1 smoothing (build option SHH_SEL_DEG0): one pass before the
    // restriction and one after the prolongation
    const std::vector<int> pre = SHH_SEL_DEG0 == 1 ? std::vector<int>{SMO_STEP1} : std::vector<int>{SMO_STEP1, SMO_RES};
    const std::vector<int> post = SHH_SEL_DEG0 == 1 ? std::vector<int>{SMO_POST1} : std::vector<int>{SMO_POST, SMO_LAST};
    for (int m : pre)
      if ((rc = run_timed(SHH_PROF_SEL_MG_SMOOTH, [&] { return sel_launch_mg_op(B, m, st); }))) return rc;
    if ((rc = run_timed(SHH_PROF_SEL_MG_TRANSFER, [&] { return sel_launch_mg_restrict(B, st); }))) return rc;
    if ((rc = mg_vcycle_coarse(ss, st))) return rc;
    if ((rc = run_timed(SHH_PROF_SEL_MG_TRANSFER, [&] { return sel_launch_mg_prolong(B, st); }))) return rc;
    for (int m : post)
      if ((rc = run_timed(SHH_PROF_SEL_MG_SMOOTH, [&] { return sel_launch_mg_op(B, m, st); }))) return rc;
    return SHH_OK;
  }
  // z = V r of a new residual: a restart (beta = 0), or after a residual
  // replacement with the direction kept (SSC_MG_REPLACE)
  int restart(const std::vector<Slot *> &v, int phase = SSC_MG_RESTART) {
    return chunked(v, [&](const std::vector<Slot *> &part) {
      const SelBatch B = batch_of(part);
      int rc;
      if ((rc = vcycle(B, part, 1))) return rc;
      SEL_HIP(sel_launch_scalar(B, phase, st));
      return SHH_OK;
    });
  }
  int iteration(const std::vector<Slot *> &v, bool mg) {
    return chunked(v, [&](const std::vector<Slot *> &part) {
      const SelBatch B = batch_of(part);
      int rc;
      if (mg) {
        if ((rc = run_timed(SHH_PROF_SEL_MG_VEC, [&] { return sel_launch_mg_dir(B, st); }))) return rc;
        if ((rc = run_timed(SHH_PROF_SEL_MG_PQ, [&] { return sel_launch_mg_op(B, SMO_PQ, st); }))) return rc;
        SEL_HIP(sel_launch_scalar(B, SSC_MG_ALPHA, st));
        if ((rc = vcycle(B, part, 0))) return rc;
        SEL_HIP(sel_launch_scalar(B, SSC_MG_BETA, st));
      } else {
        if ((rc = run_timed(SHH_PROF_SEL_OP, [&] { return sel_launch_op(B, SOP_PCG, st); }))) return rc;
        SEL_HIP(sel_launch_scalar(B, SSC_ITER, st));
        if ((rc = run_timed(SHH_PROF_SEL_UPDATE, [&] { return sel_launch_update(B, st); }))) return rc;
      }
      return SHH_OK;
    });
  }
};

// Descriptor of one slot before the compaction: the compact arrays in the
// dense CG vector region (seven [6][3][n^3] vectors): the map, coordinates,
// counts, moduli and diagonal in vectors 0-1, r, p, q, x in vectors 2, 3, 4,
// 6, the partials in vector 5; the descriptor in the slot's small parameter
// block.
int describe(Slot &s) {
  SelHost &x = *s.sel;
  const Layout &L = s.lay;
  const SlotDev &sd = s.host;
  SelDev &h = x.h;
  const size_t ts = sd.prec == SHH_PREC_FP64 ? 8 : 4;
  char *base = s.base;
  char *vec = base + L.vec;
  const size_t vb = L.vec_bytes;
  std::memset(&h, 0, sizeof(h));
  h.n = sd.n;
  h.nn = sd.nn;
  h.prec = sd.prec;
  h.nchunks = int((sd.nn + SEL_CHUNK - 1) / SEL_CHUNK);
  h.lam = sd.lam;
  h.mu = sd.mu;
  h.rtol = sd.rtol;
  h.ffloor = sd.ffloor;
  h.max_iter = sd.max_iter;
  element_forces(sd.lam, sd.mu, h.f0);
  for (int c = 0; c < KOP_N; ++c) h.kop[c] = sd.kop64[c];
  h.E64 = sd.E64;
  h.st = sd.st;
  h.r = vec + 2 * vb;
  h.p = vec + 3 * vb;
  h.q = vec + 4 * vb;
  h.x = vec + 6 * vb;
  h.x64 = sd.prec == SHH_PREC_MIXED ? (double *)(base + L.x64) : (double *)h.x;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = vec + off;
    off = al256(off + bytes);
    return p;
  };
  h.map = (int *)take(sizeof(int) * sd.nn);
  h.coord = (unsigned *)take(sizeof(unsigned) * sd.nn);
  h.counts = (int *)take(sizeof(int) * (h.nchunks + 1));
  h.Ec = take(ts * sd.nn);
  h.Ec64 = sd.prec == SHH_PREC_FP64 ? (double *)h.Ec : (double *)take(sizeof(double) * sd.nn);
  h.Dinv = take(ts * sd.nn);
  if (off > 2 * vb) return SHH_WORKSPACE_TOO_SMALL;
  h.partials = (double *)(vec + 5 * vb);
  static_assert(sizeof(SelDev) <= 4096, "descriptor fits the parameter block");
  x.d = (SelDev *)(base + L.segs);
  x.aux = off;
  return SHH_OK;
}

// After the compaction (n_a known): workgroup count, partial room, and the
// multigrid's three extra [n_a][18] vectors after the compact arrays in
// vectors 0-1, then after the partials in vector 5 (Jacobi when a nearly full
// design leaves no room for them).
int place(Slot &s) {
  SelHost &x = *s.sel;
  SelDev &h = x.h;
  const size_t ts = h.prec == SHH_PREC_FP64 ? 8 : 4;
  char *vec = s.base + s.lay.vec;
  const size_t vb = s.lay.vec_bytes;
  h.nparts = std::max(1, (h.na + SEL_THREADS - 1) / SEL_THREADS);
  const size_t pbytes = al256((size_t)NRHS * h.nparts * SEL_PS * sizeof(double));
  if (pbytes > vb || 22ull * h.nparts * sizeof(double) > vb) return SHH_WORKSPACE_TOO_SMALL;
  if (h.mg) {
    const size_t vbytes = al256((size_t)h.na * 3 * NRHS * ts);
    char *arena[2] = {vec + x.aux, vec + 5 * vb + pbytes};
    size_t room[2] = {2 * vb - x.aux, vb - pbytes};
    void **dst[3] = {&h.d1, &h.xv, &h.rv};
    for (void **v : dst) {
      const int a = room[0] >= vbytes ? 0 : (room[1] >= vbytes ? 1 : -1);
      if (a < 0) {
        h.mg = 0;
        break;
      }
      *v = arena[a];
      arena[a] += vbytes;
      room[a] -= vbytes;
    }
  }
  x.mg = h.mg != 0;
  return SHH_OK;
}

void finish(Slot &s, int status) {
  s.status = status;
  s.finished = true;
  s.sel->done = true;
}

}  // namespace

size_t sel_descriptor_bytes() { return sizeof(SelDev); }

int sel_energy_gradient(Slot &s, const double g21[21], double **d_gE, hipStream_t st) {
  // the compact lists and the FP64 solution of the forward call are still in
  // the workspace (save_for_backward); the descriptor is rebuilt from the
  // layout, n_a read back from the compaction counts
  s.sel = std::make_shared<SelHost>();
  int rc;
  if ((rc = describe(s))) return rc;
  SelHost &x = *s.sel;
  SelDev &h = x.h;
  SEL_HIP(hipMemcpyAsync(&h.na, h.counts + h.nchunks, sizeof(int), hipMemcpyDeviceToHost, st));
  SEL_HIP(hipStreamSynchronize(st));
  h.nparts = std::max(1, (h.na + SEL_THREADS - 1) / SEL_THREADS);
  // dL/dE_e (n^3 doubles) and the weights after the compact arrays in vectors 0-1
  char *vec = s.base + s.lay.vec;
  if (x.aux + al256(sizeof(double) * (size_t)h.nn) + 256 > 2 * s.lay.vec_bytes) return SHH_WORKSPACE_TOO_SMALL;
  *d_gE = (double *)(vec + x.aux);
  double *d_g21 = (double *)(vec + x.aux + al256(sizeof(double) * (size_t)h.nn));
  SEL_HIP(hipMemcpyAsync(x.d, &h, sizeof(SelDev), hipMemcpyHostToDevice, st));
  SEL_HIP(hipMemcpyAsync(d_g21, g21, 21 * sizeof(double), hipMemcpyHostToDevice, st));
  SEL_HIP(sel_launch_energy_sens(batch_of({&s}), h.nn, d_g21, *d_gE, st));
  // the weights' host copy must outlive the asynchronous upload
  SEL_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int sel_start(const std::vector<Slot *> &in, hipStream_t st) {
  if (in.empty()) return SHH_OK;
  SelRun run(st, in);
  std::vector<Slot *> slots, mgc;
  int rc;
  for (Slot *s : in) {
    s->sel = std::make_shared<SelHost>();
    if ((rc = describe(*s))) {
      finish(*s, rc);
      continue;
    }
    slots.push_back(s);
    if (s->opts.solver == SHH_SOLVER_SELECTIVE && s->lay.mg && mg_num_levels(s->host.n) >= 2) mgc.push_back(s);
  }
  // multigrid hierarchies of the culled operators (Galerkin levels from the
  // culled moduli; their element matrices use the vector region as scratch,
  // so they are built before the compaction writes there), batched
  if (!mgc.empty()) {
    std::vector<int> rcs;
    if ((rc = mg_setup(mgc, st, &rcs))) return rc;
    for (size_t j = 0; j < mgc.size(); ++j) {
      if (rcs[j] != SHH_OK) continue;  // a failed estimate: Jacobi
      const MgDev &M = mgc[j]->mg;
      SelDev &h = H(mgc[j]).h;
      h.mg = 1;
      h.inv_theta = M.lv[0].inv_theta;
      h.c1 = M.lv[0].c1;
      h.c2 = M.lv[0].c2;
      h.n1 = M.lv[1].n;
      h.nn1 = M.lv[1].nn;
      h.b1 = M.lv[1].b;
      h.x1 = M.lv[1].x;
      h.d0 = M.lv[0].d;  // the dense level-0 direction buffer: [6][3][n^3] >= [n_a][18]
    }
  }
  run.record(slots, 1);
  for (Slot *s : slots) SEL_HIP(hipMemcpyAsync(H(s).d, &H(s).h, sizeof(SelDev), hipMemcpyHostToDevice, st));
  if ((rc = chunked(slots, [&](const std::vector<Slot *> &part) {
         SEL_HIP(sel_launch_compact(batch_of(part), st));
         return SHH_OK;
       })))
    return rc;
  std::vector<int> na(slots.size(), 0);
  for (size_t i = 0; i < slots.size(); ++i)
    SEL_HIP(hipMemcpyAsync(&na[i], H(slots[i]).h.counts + H(slots[i]).h.nchunks, sizeof(int),
                           hipMemcpyDeviceToHost, st));
  SEL_HIP(hipStreamSynchronize(st));
  std::vector<Slot *> gm, gj, empty;
  for (size_t i = 0; i < slots.size(); ++i) {
    Slot *s = slots[i];
    SelHost &x = H(s);
    x.h.na = na[i];
    s->sel_active_nodes = na[i];
    if ((rc = place(*s))) {
      finish(*s, rc);
      continue;
    }
    SEL_HIP(hipMemcpyAsync(x.d, &x.h, sizeof(SelDev), hipMemcpyHostToDevice, st));
    (na[i] == 0 ? empty : (x.mg ? gm : gj)).push_back(s);
  }
  // everything culled: no stiffness, C^H = 0
  if (!empty.empty() && (rc = run.read_state(empty))) return rc;
  for (Slot *s : empty) {
    for (int i = 0; i < 36; ++i) s->state.C[i] = 0.0;
    for (int k = 0; k < NRHS; ++k) {
      s->state.iters[k] = 0;
      s->state.rel_true[k] = 0.0;
      s->state.status[k] = ST_CONVERGED;
    }
    finish(*s, SHH_OK);
  }
  for (const std::vector<Slot *> *g : {&gm, &gj}) {
    if (g->empty()) continue;
    if ((rc = chunked(*g, [&](const std::vector<Slot *> &part) {
           const SelBatch B = batch_of(part);
           SEL_HIP(sel_launch_gather(B, st));
           SEL_HIP(sel_launch_zero(B, st));
           return SHH_OK;
         })))
      return rc;
    if ((rc = run.residual(*g, 0))) return rc;
    if (g == &gm) {
      if ((rc = run.restart(gm))) return rc;
    } else if ((rc = chunked(gj, [&](const std::vector<Slot *> &part) {
                  SEL_HIP(sel_launch_dir0(batch_of(part), st));
                  return SHH_OK;
                }))) {
      return rc;
    }
  }
  std::vector<Slot *> started(gm);
  started.insert(started.end(), gj.begin(), gj.end());
  run.record(started, 2);
  return run.read_state(started);
}

int sel_step(const std::vector<Slot *> &in, int iters, hipStream_t st) {
  std::vector<Slot *> live;
  for (Slot *s : in)
    if (s->sel && !s->sel->done) live.push_back(s);
  if (live.empty()) return SHH_OK;
  SelRun run(st, live);
  int rc;
  // iterate: each preconditioner's slots together; each slot replaces its
  // residual by the FP64 one every R of its own iterations
  for (const bool mg : {true, false}) {
    std::vector<Slot *> g;
    for (Slot *s : live)
      if (H(s).mg == mg && !all_stopped(s->state)) g.push_back(s);
    for (int j = 0; j < iters && !g.empty(); ++j) {
      if ((rc = run.iteration(g, mg))) return rc;
      std::vector<Slot *> due;
      for (Slot *s : g) {
        SelHost &x = H(s);
        ++x.launched;
        const int R = s->host.prec == SHH_PREC_MIXED ? s->opts.recompute_every : 0;
        if (R > 0 && x.launched % R == 0) due.push_back(s);
      }
      if (!due.empty()) {
        if ((rc = run.residual(due, 1))) return rc;
        if (mg && (rc = run.restart(due, SSC_MG_REPLACE))) return rc;  // z of the replaced residual
      }
    }
  }
  if ((rc = run.read_state(live))) return rc;
  // slots whose every load case has stopped: the true residual decides (a
  // case whose recursive residual was optimistic, or that stalled, resumes
  // from a restart, at most 8 times); a slot past the iteration guard stops
  std::vector<Slot *> check, done;
  for (Slot *s : live) {
    const long long guard = 4LL * s->opts.max_iter + 64LL * std::max(1, s->opts.check_every) + 1024;
    if (all_stopped(s->state) || H(s).launched > guard) check.push_back(s);
  }
  if (!check.empty()) {
    if ((rc = run.residual(check, 2))) return rc;
    if ((rc = run.read_state(check))) return rc;
    std::vector<Slot *> resumed;
    for (Slot *s : check) {
      SelHost &x = H(s);
      ++x.finals;
      const long long guard = 4LL * s->opts.max_iter + 64LL * std::max(1, s->opts.check_every) + 1024;
      if (all_stopped(s->state) || x.finals >= 8 || x.launched > guard) {
        done.push_back(s);
        continue;
      }
      // resume; the replacement schedule follows the device iteration count,
      // so that the arithmetic does not depend on when the host polled
      int m = 0;
      for (int k = 0; k < NRHS; ++k) m = std::max(m, s->state.iters[k]);
      x.launched = m;
      resumed.push_back(s);
    }
    std::vector<Slot *> rmg;
    for (Slot *s : resumed)
      if (H(s).mg) rmg.push_back(s);
    if (!rmg.empty() && (rc = run.restart(rmg))) return rc;
  }
  if (done.empty()) return SHH_OK;
  // C^H of the finished slots
  run.record(done, 3);
  if ((rc = chunked(done, [&](const std::vector<Slot *> &part) {
         const SelBatch B = batch_of(part);
         SEL_HIP(sel_launch_fold(B, 1, st));
         SEL_HIP(sel_launch_op(B, SOP_ENERGY, st));
         SEL_HIP(sel_launch_scalar(B, SSC_ENERGY, st));
         return SHH_OK;
       })))
    return rc;
  run.record(done, 4);
  if ((rc = run.read_state(done))) return rc;
  for (Slot *s : done) {
    float a = 0.f;
    for (int k = 0; k < 4; ++k)
      if (s->ev[k] && s->ev[k + 1] && hipEventElapsedTime(&a, s->ev[k], s->ev[k + 1]) == hipSuccess) s->ms[k] = a;
    if (s->ev[0] && s->ev[4] && hipEventElapsedTime(&a, s->ev[0], s->ev[4]) == hipSuccess) s->ms[4] = a;
    int status = SHH_OK;
    for (int k = 0; k < NRHS; ++k) {
      // a case still stalled after its restarts counts as broken down
      if (s->state.status[k] == ST_BREAKDOWN || s->state.status[k] == ST_STALLED) status = SHH_BREAKDOWN;
      else if (status == SHH_OK && s->state.status[k] != ST_CONVERGED) status = SHH_NOT_CONVERGED;
    }
    finish(*s, status);
  }
  return SHH_OK;
}

int sel_solve(const std::vector<Slot *> &all, hipStream_t st) {
  int rc;
  if ((rc = sel_start(all, st))) return rc;
  for (;;) {
    std::vector<Slot *> live;
    for (Slot *s : all)
      if (!s->sel->done) live.push_back(s);
    if (live.empty()) return SHH_OK;
    if ((rc = sel_step(live, std::max(1, live[0]->opts.check_every), st))) return rc;
  }
}

}  // namespace shh
