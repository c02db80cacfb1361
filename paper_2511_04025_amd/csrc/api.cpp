// extern "C" entry points of libshellhom (declared in include/shellhom.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

using namespace shh;

#define SHH_HIP(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return SHH_HIP_ERROR;      \
  } while (0)
#define SHH_TRY(call)                                \
  do {                                               \
    int rc_ = (call);                                \
    if (rc_ < 0) return rc_;                         \
  } while (0)

namespace {

constexpr int MAX_BATCH = 64;

// Segment tables of one solve live in a fixed block of the first workspace.
size_t seg_region() { return Solver::seg_bytes(MAX_BATCH); }

// The multigrid solver needs n = m 2^k, k >= 1, m <= 8, n >= 6;
// SHH_SOLVER_AUTO resolves here, per grid, to it or to Jacobi.
int check_solver(int n, shh_opts *o) {
  if (o->solver == SHH_SOLVER_AUTO) o->solver = mg_num_levels(n) >= 2 ? SHH_SOLVER_MG : SHH_SOLVER_JACOBI;
  if (o->solver == SHH_SOLVER_MG && mg_num_levels(n) < 2) return SHH_UNSUPPORTED;
  return SHH_OK;
}

size_t ws_bytes_for(const shh_design *d, const shh_opts *o) {
  const Layout L = make_layout(d->n, charge_count(d), d->K, o->precision, o->save_for_backward != 0, true,
                               o->solver);
  return L.total + seg_region() + 256;
}

char *aligned(void *p) {
  const uintptr_t v = (uintptr_t)p;
  return (char *)((v + 255) & ~uintptr_t(255));
}

struct Events {
  Slot *s;
  explicit Events(Slot *slot) : s(slot) {
    for (auto &e : s->ev) (void)hipEventCreate(&e);
  }
  ~Events() {
    for (auto &e : s->ev) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
  }
};

int prepare_slot(Slot &s, const shh_design *d, const shh_opts *o, void *d_ws, size_t ws_bytes,
                 char **seg_mem, bool vectors = true) {
  copy_design(d, s.design);
  s.opts = *o;
  SHH_TRY(check_solver(d->n, &s.opts));
  o = &s.opts;
  s.lay = make_layout(d->n, charge_count(d), d->K, o->precision, o->save_for_backward != 0, vectors,
                      vectors ? o->solver : SHH_SOLVER_JACOBI);
  if (!d_ws) return SHH_INVALID_ARG;
  char *base = aligned(d_ws);
  const size_t need = s.lay.total + seg_region() + size_t(base - (char *)d_ws);
  if (ws_bytes < need) return SHH_WORKSPACE_TOO_SMALL;
  s.base = base;
  if (seg_mem) *seg_mem = base + s.lay.total;
  s.R = o->recompute_every;
  return SHH_OK;
}

// Run the PCG of already-set-up slots to completion.
int solve_all(Solver &sv, std::vector<Slot *> slots, int check_every, int max_iter) {
  SHH_TRY(sv.start(slots));
  long long guard = 0;
  const long long guard_max = (long long)max_iter * 4 + 64 * (long long)check_every + 1024;
  while (!slots.empty()) {
    SHH_TRY(sv.iterate(slots, check_every));
    std::vector<Slot *> done;
    SHH_TRY(sv.poll(slots, done));
    std::vector<Slot *> rest;
    for (Slot *s : slots)
      if (!s->finished) rest.push_back(s);
    slots.swap(rest);
    guard += check_every;
    if (guard > guard_max) {
      for (Slot *s : slots) s->status = SHH_NOT_CONVERGED;
      break;
    }
  }
  return SHH_OK;
}

}  // namespace

extern "C" {

int32_t shh_version(void) { return 10000; }

const char *shh_strerror(int32_t code) {
  switch (code) {
    case SHH_OK: return "ok";
    case SHH_NOT_CONVERGED: return "not converged: residual above rtol after max_iter";
    case SHH_INVALID_ARG: return "invalid argument";
    case SHH_WORKSPACE_TOO_SMALL: return "workspace too small";
    case SHH_HIP_ERROR: return "HIP runtime error";
    case SHH_OVER_BUDGET: return "request footprint exceeds the engine arena";
    case SHH_UNSUPPORTED: return "unsupported (hard-step gradient, or a grid the multigrid solver cannot coarsen)";
    case SHH_BREAKDOWN: return "CG breakdown (p^T K p <= 0 or NaN)";
    case SHH_NOT_FOUND: return "unknown request id";
    case SHH_SCRATCH_TOO_SMALL:
      return "design needs more workspace than the fixed device scratch of shh_homogenize_noalloc";
    default: return "unknown status";
  }
}

int32_t shh_workspace_bytes(const shh_design *design, const shh_opts *opts, size_t *bytes) {
  SHH_TRY(validate_design(design));
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  if (!bytes) return SHH_INVALID_ARG;
  SHH_TRY(check_solver(design->n, &o));
  *bytes = ws_bytes_for(design, &o);
  return SHH_OK;
}

}  // extern "C"

namespace {

// The path for `count` designs; `timed` false creates no HIP events (result
// timings stay zero), which keeps the no-allocation entry point free of them.
int homogenize_run(const shh_design *designs, int32_t count, const shh_opts *opts, void *const *d_ws,
                   const size_t *ws_bytes, void *hip_stream, shh_result *out, bool timed) {
  if (count < 1 || count > MAX_BATCH || !designs || !d_ws || !ws_bytes || !out) return SHH_INVALID_ARG;
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  for (int i = 0; i < count; ++i) SHH_TRY(validate_design(&designs[i]));
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<std::unique_ptr<Events>> evs;
  char *seg_mem = nullptr;
  for (int i = 0; i < count; ++i) {
    slots.emplace_back(new Slot());
    SHH_TRY(prepare_slot(*slots.back(), &designs[i], &o, d_ws[i], ws_bytes[i], i == 0 ? &seg_mem : nullptr));
    if (timed) evs.emplace_back(new Events(slots.back().get()));
  }
  for (auto &s : slots) {
    if (s->ev[0]) SHH_HIP(hipEventRecord(s->ev[0], st));
    SHH_TRY(slot_init(*s, s->base, st));
    SHH_TRY(slot_setup_field(*s, nullptr, st));
    s->timing = timed;
  }
  if (is_selective(o.solver)) {
    std::vector<Slot *> ptrs;
    for (auto &s : slots) ptrs.push_back(s.get());
    SHH_TRY(sel_solve(ptrs, st));  // the batch shares every launch
    int worst = SHH_OK;
    for (int i = 0; i < count; ++i) {
      fill_result(*slots[i], &out[i]);
      const int s = slots[i]->status;
      if (s < 0 && (worst >= 0 || s < worst)) worst = s;
      else if (s > 0 && worst == SHH_OK) worst = s;
    }
    return worst;
  }
  Solver sv(st);
  sv.set_timing(timed);
  sv.set_segment_memory(seg_mem, seg_region());
  std::vector<Slot *> ptrs;
  for (auto &s : slots) ptrs.push_back(s.get());
  SHH_TRY(solve_all(sv, ptrs, o.check_every, o.max_iter));
  int worst = SHH_OK;
  for (int i = 0; i < count; ++i) {
    fill_result(*slots[i], &out[i]);
    const int s = slots[i]->status;
    if (s < 0 && (worst >= 0 || s < worst)) worst = s;
    else if (s > 0 && worst == SHH_OK) worst = s;
  }
  return worst;
}

}  // namespace

extern "C" {

int32_t shh_homogenize_batch(const shh_design *designs, int32_t count, const shh_opts *opts,
                             void *const *d_ws, const size_t *ws_bytes, void *hip_stream,
                             shh_result *out) {
  return homogenize_run(designs, count, opts, d_ws, ws_bytes, hip_stream, out, true);
}

int32_t shh_homogenize(const shh_design *design, const shh_opts *opts, void *d_ws, size_t ws_bytes,
                       void *hip_stream, shh_result *out) {
  return shh_homogenize_batch(design, 1, opts, &d_ws, &ws_bytes, hip_stream, out);
}

int32_t shh_homogenize_noalloc(const shh_design *design, const shh_opts *opts, void *hip_stream,
                               shh_result *out) {
  if (!design || !out) return SHH_INVALID_ARG;
  size_t need = 0;
  SHH_TRY(shh_workspace_bytes(design, opts, &need));
  if (need > SHH_NOALLOC_SCRATCH_BYTES) return SHH_SCRATCH_TOO_SMALL;
  void *ws = nullptr;
  SHH_TRY(noalloc_scratch(&ws));
  const size_t cap = SHH_NOALLOC_SCRATCH_BYTES;
  return homogenize_run(design, 1, opts, &ws, &cap, hip_stream, out, false);
}

int32_t shh_field(const shh_design *design, void *d_ws, size_t ws_bytes, double *d_F, double *d_G,
                  double *d_d, double *d_beta, void *hip_stream, shh_result *out) {
  SHH_TRY(validate_design(design));
  shh_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = SHH_PREC_FP64;
  o.rtol = 1e-10;
  o.max_iter = 1;
  SHH_TRY(normalize_opts(&o, &o));
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  SHH_TRY(prepare_slot(s, design, &o, d_ws, ws_bytes, nullptr));
  SHH_TRY(slot_init(s, s.base, st));
  SHH_TRY(slot_setup_field(s, d_beta, st));
  const size_t nb = sizeof(double) * (size_t)s.host.nn;
  if (d_F) SHH_HIP(hipMemcpyAsync(d_F, s.host.F, nb, hipMemcpyDeviceToDevice, st));
  if (d_G) SHH_HIP(hipMemcpyAsync(d_G, s.host.G, 3 * nb, hipMemcpyDeviceToDevice, st));
  if (d_d) SHH_HIP(hipMemcpyAsync(d_d, s.host.d, nb, hipMemcpyDeviceToDevice, st));
  SHH_HIP(hipMemcpyAsync(&s.state, s.d_state, sizeof(CgState), hipMemcpyDeviceToHost, st));
  SHH_HIP(hipStreamSynchronize(st));
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->vol_frac = s.state.V;
    out->t_used = s.state.t;
  }
  return SHH_OK;
}

// ---- solver-only and component entry points ---------------------------------

static shh_design stiffness_design(int32_t n, double nu) {
  static const double zero3[3] = {0.0, 0.0, 0.0};
  static const double one = 1.0;
  shh_design d;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.num_charges = 1;
  d.pos = zero3;
  d.q = &one;
  d.K = 1;
  d.thickness = 0.0;
  d.E = 1.0;
  d.nu = nu;
  d.E_void = 0.0;
  return d;
}

int32_t shh_workspace_bytes_stiffness(int32_t n, const shh_opts *opts, size_t *bytes) {
  if (n < 2 || n > 512 || !bytes) return SHH_INVALID_ARG;
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  o.save_for_backward = 0;
  const shh_design d = stiffness_design(n, 0.3);
  SHH_TRY(check_solver(n, &o));
  *bytes = ws_bytes_for(&d, &o);
  return SHH_OK;
}

int32_t shh_workspace_bytes_operator(int32_t n, int32_t precision, size_t *bytes) {
  if (n < 2 || n > 512 || !bytes || (precision != SHH_PREC_FP64 && precision != SHH_PREC_MIXED))
    return SHH_INVALID_ARG;
  const shh_design d = stiffness_design(n, 0.3);
  const Layout L = make_layout(d.n, d.num_charges, d.K, precision, false, false);
  *bytes = L.total + seg_region() + 256;
  return SHH_OK;
}

// Slot over a workspace with moduli copied from d_E (scale taken from max E).
static int moduli_slot(Slot &s, int32_t n, const void *d_E, double nu, const shh_opts *o, void *d_ws,
                       size_t ws_bytes, hipStream_t st, char **seg_mem, bool vectors,
                       int e_dtype = SHH_EDTYPE_F64, double Es = 0.0, double Ev = 0.0) {
  if (n < 2 || n > 512 || !d_E || !(nu > -1.0 && nu < 0.5)) return SHH_INVALID_ARG;
  if (e_dtype != SHH_EDTYPE_U8 && e_dtype != SHH_EDTYPE_F32 && e_dtype != SHH_EDTYPE_F64) return SHH_INVALID_ARG;
  if (e_dtype == SHH_EDTYPE_U8 && !(Es > 0.0 && std::isfinite(Es) && Ev >= 0.0 && Ev <= Es)) return SHH_INVALID_ARG;
  shh_opts oo = *o;
  oo.save_for_backward = 0;
  const shh_design d = stiffness_design(n, nu);
  SHH_TRY(prepare_slot(s, &d, &oo, d_ws, ws_bytes, seg_mem, vectors));
  SHH_TRY(slot_init(s, s.base, st));
  // a culled voxel of the selective solve carries nothing, whatever E_void says
  SHH_TRY(slot_setup_moduli(s, d_E, e_dtype, Es, is_selective(oo.solver) ? 0.0 : Ev, st));
  SHH_HIP(hipMemcpyAsync(&s.state, s.d_state, sizeof(CgState), hipMemcpyDeviceToHost, st));
  SHH_HIP(hipStreamSynchronize(st));
  const double emax = s.state.Emax;
  // the selective solve culls zero moduli; an all-zero grid is an empty cell
  const bool sel = is_selective(oo.solver);
  if (!std::isfinite(emax) || !(emax > 0.0 || (sel && emax == 0.0))) return SHH_INVALID_ARG;
  s.host.E = emax;
  s.host.ffloor = 1e-12 * emax * std::sqrt(3.0 * double(s.host.nn));
  SHH_HIP(hipMemcpyAsync(s.d_slot, &s.host, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int32_t shh_homogenize_stiffness(int32_t n, const double *d_E, double nu, const shh_opts *opts,
                                 void *d_ws, size_t ws_bytes, void *hip_stream, shh_result *out) {
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  if (!out) return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  char *seg_mem = nullptr;
  Events ev(&s);
  SHH_HIP(hipEventRecord(s.ev[0], st));
  SHH_TRY(moduli_slot(s, n, d_E, nu, &o, d_ws, ws_bytes, st, &seg_mem, true));
  if (is_selective(o.solver)) {
    SHH_TRY(sel_solve(s, st));
  } else {
    Solver sv(st);
    sv.set_segment_memory(seg_mem, seg_region());
    SHH_TRY(solve_all(sv, {&s}, o.check_every, o.max_iter));
  }
  fill_result(s, out);
  return s.status;
}

int32_t shh_homogenize_field(int32_t n, const void *d_E, int32_t e_dtype, double E, double E_void, double nu,
                             const shh_opts *opts, void *d_ws, size_t ws_bytes, void *hip_stream,
                             shh_result *out) {
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  if (!out || n < 2 || n > 512 || !d_E || !(nu > -1.0 && nu < 0.5)) return SHH_INVALID_ARG;
  if (e_dtype != SHH_EDTYPE_U8 && e_dtype != SHH_EDTYPE_F32 && e_dtype != SHH_EDTYPE_F64) return SHH_INVALID_ARG;
  if (e_dtype == SHH_EDTYPE_U8 && !(E > 0.0 && std::isfinite(E) && E_void >= 0.0 && E_void <= E))
    return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  char *seg_mem = nullptr;
  Events ev(&s);
  SHH_HIP(hipEventRecord(s.ev[0], st));
  SHH_TRY(moduli_slot(s, n, d_E, nu, &o, d_ws, ws_bytes, st, &seg_mem, true, e_dtype, E, E_void));
  if (is_selective(o.solver)) {
    SHH_TRY(sel_solve(s, st));
  } else {
    Solver sv(st);
    sv.set_segment_memory(seg_mem, seg_region());
    SHH_TRY(solve_all(sv, {&s}, o.check_every, o.max_iter));
  }
  fill_result(s, out);
  return s.status;
}

int32_t shh_apply_stiffness(int32_t n, int32_t precision, const double *d_E, double nu, int32_t nrhs,
                            const void *d_p, void *d_q, void *d_ws, size_t ws_bytes, void *hip_stream) {
  if (nrhs < 1 || nrhs > NRHS || !d_p || !d_q) return SHH_INVALID_ARG;
  shh_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = precision;
  o.rtol = 1e-10;
  o.max_iter = 1;
  SHH_TRY(normalize_opts(&o, &o));
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  char *seg_mem = nullptr;
  SHH_TRY(moduli_slot(s, n, d_E, nu, &o, d_ws, ws_bytes, st, &seg_mem, false));
  s.host.p[0] = const_cast<void *>(d_p);
  s.host.q[0] = d_q;
  SHH_HIP(hipMemcpyAsync(s.d_slot, &s.host, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  Segment g;
  std::memset(&g, 0, sizeof(g));
  g.slot = s.d_slot;
  g.first = 0;
  g.nrhs = nrhs;
  for (int r = 0; r < nrhs; ++r) g.rhs[r] = r;
  g.nblocks = s.host.ntiles[precision == SHH_PREC_MIXED ? 1 : 0] * nrhs;
  SHH_HIP(hipMemcpyAsync(seg_mem, &g, sizeof(g), hipMemcpyHostToDevice, st));
  LaunchArgs la{(const Segment *)seg_mem, 1, g.nblocks};
  SHH_HIP(launch_stencil_apply(la, precision, st));
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int32_t shh_mg_operator(int32_t n, int32_t precision, const double *d_E, double nu, int32_t level,
                        const void *d_v, void *d_q, void *d_ws, size_t ws_bytes, void *hip_stream) {
  if (!d_v || !d_q) return SHH_INVALID_ARG;
  shh_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = precision;
  o.rtol = 1e-10;
  o.max_iter = 1;
  o.solver = SHH_SOLVER_MG;
  SHH_TRY(normalize_opts(&o, &o));
  SHH_TRY(check_solver(n, &o));
  if (level < 1 || level >= mg_num_levels(n)) return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  char *seg_mem = nullptr;
  SHH_TRY(moduli_slot(s, n, d_E, nu, &o, d_ws, ws_bytes, st, &seg_mem, true));
  SHH_TRY(mg_setup(s, st));
  return mg_apply_level(s, level, d_v, d_q, st);
}

int32_t shh_load_vectors(int32_t n, const double *d_E, double nu, double *d_f, void *d_ws, size_t ws_bytes,
                         void *hip_stream) {
  if (!d_f) return SHH_INVALID_ARG;
  shh_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = SHH_PREC_FP64;
  o.rtol = 1e-10;
  o.max_iter = 1;
  SHH_TRY(normalize_opts(&o, &o));
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  char *seg_mem = nullptr;
  SHH_TRY(moduli_slot(s, n, d_E, nu, &o, d_ws, ws_bytes, st, &seg_mem, false));
  s.host.r[0] = d_f;
  SHH_HIP(hipMemcpyAsync(s.d_slot, &s.host, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  Segment g;
  std::memset(&g, 0, sizeof(g));
  g.slot = s.d_slot;
  g.nrhs = NRHS;
  for (int r = 0; r < NRHS; ++r) g.rhs[r] = r;
  g.nblocks = s.host.ntiles[0] * NRHS;  // FP64 residual kernel
  g.flag = RES_INIT;
  SHH_HIP(hipMemcpyAsync(seg_mem, &g, sizeof(g), hipMemcpyHostToDevice, st));
  LaunchArgs la{(const Segment *)seg_mem, 1, g.nblocks};
  SHH_HIP(launch_stencil_resid(la, SHH_PREC_FP64, st));
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int32_t shh_energy(int32_t n, const double *d_E, double nu, const double *d_u, double CH[36], void *d_ws,
                   size_t ws_bytes, void *hip_stream) {
  if (!d_u || !CH) return SHH_INVALID_ARG;
  shh_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = SHH_PREC_FP64;
  o.rtol = 1e-10;
  o.max_iter = 1;
  SHH_TRY(normalize_opts(&o, &o));
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  SHH_TRY(moduli_slot(s, n, d_E, nu, &o, d_ws, ws_bytes, st, nullptr, false));
  s.host.x64 = const_cast<double *>(d_u);
  SHH_HIP(hipMemcpyAsync(s.d_slot, &s.host, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  SHH_HIP(launch_energy(s.d_slot, s.host.nn, st));
  SHH_HIP(hipMemcpyAsync(&s.state, s.d_state, sizeof(CgState), hipMemcpyDeviceToHost, st));
  SHH_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < 36; ++i) CH[i] = s.state.C[i];
  return SHH_OK;
}

// ---- adjoint -------------------------------------------------------------------

namespace {

// Enqueue the adjoint of one forward run (its workspace kept with
// save_for_backward); the results land in the slot's partials region:
// [N][4] charge gradients, then dL/dalpha [(K+1)^3] and dL/dt.
struct GradJob {
  Slot s;
  double *d_out = nullptr;
  int N = 0, nalpha = 0;        // N: charges after the fundamental volume's expansion
  int sym = 0, nfbv = 0;        // the caller's symmetry mode and charge count
  std::vector<double> host;
};

int grad_enqueue(GradJob &job, const shh_design *design, const shh_opts *opts, void *d_ws, size_t ws_bytes,
                 const double dL_dCH[36], double dL_dV, hipStream_t st) {
  SHH_TRY(validate_design(design));
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  if (!dL_dCH || !std::isfinite(dL_dV)) return SHH_INVALID_ARG;
  if (!(design->kappa > 0.0)) return SHH_UNSUPPORTED;
  if (!o.save_for_backward) return SHH_INVALID_ARG;
  for (int i = 0; i < 36; ++i)
    if (!std::isfinite(dL_dCH[i])) return SHH_INVALID_ARG;
  Slot &s = job.s;
  SHH_TRY(prepare_slot(s, design, &o, d_ws, ws_bytes, nullptr));
  // the device descriptor written by the forward call is still in place; read it back
  SHH_HIP(hipMemcpyAsync(&s.host, (SlotDev *)(s.base + s.lay.slotdev), sizeof(SlotDev),
                         hipMemcpyDeviceToHost, st));
  SHH_HIP(hipStreamSynchronize(st));
  s.d_slot = (SlotDev *)(s.base + s.lay.slotdev);
  if (s.host.n != design->n || s.host.N != charge_count(design) || s.host.prec != o.precision ||
      s.host.K != design->K)
    return SHH_INVALID_ARG;
  job.sym = design->symmetry;
  job.nfbv = design->num_charges;
  // dL/dE_e weights: symmetric fold of dL/dC over the 21 distinct entries
  double g21[21];
  int t = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) g21[t++] = (i == j) ? dL_dCH[i * 6 + i] : dL_dCH[i * 6 + j] + dL_dCH[j * 6 + i];
  job.N = s.host.N;
  const int K1 = s.host.K + 1;
  job.nalpha = K1 * K1 * K1;
  double *d_g21 = (double *)(s.base + s.lay.segs);
  job.d_out = s.host.partials;  // free after the forward
  const size_t outd = 4 * (size_t)job.N + job.nalpha + 1;
  if (sizeof(double) * outd > sizeof(double) * NRHS * (size_t)s.lay.maxparts * PSTRIDE)
    return SHH_WORKSPACE_TOO_SMALL;
  double *d_gE = (double *)s.host.r[0];  // n^3 doubles
  double *d_scr = (double *)(s.base + s.lay.adj);  // sized for the adjoint by the layout
  job.host.assign(outd, 0.0);
  std::memcpy(job.host.data(), g21, sizeof(g21));
  if (is_selective(o.solver)) {
    // the culled system: dL/dE_e from the compact solution (culled voxels 0)
    SHH_TRY(sel_energy_gradient(s, g21, &d_gE, st));
  } else {
    SHH_HIP(hipMemcpyAsync(d_g21, job.host.data(), sizeof(g21), hipMemcpyHostToDevice, st));
    SHH_HIP(launch_energy_sens(s.d_slot, s.host.nn, d_g21, d_gE, st));
  }
  SHH_HIP(launch_adjoint(s.d_slot, s.host.n, s.host.nb, job.N, s.host.K, d_gE, dL_dV, d_scr, job.d_out,
                         job.d_out + 4 * job.N, job.d_out + 4 * job.N + job.nalpha, st));
  SHH_HIP(hipMemcpyAsync(job.host.data(), job.d_out, sizeof(double) * outd, hipMemcpyDeviceToHost, st));
  return SHH_OK;
}

void grad_unpack(const GradJob &job, double *dL_dpos, double *dL_dq, double *dL_dalpha, double *dL_dt) {
  // expanded charge j * G + g is image g of given charge j: fold its gradient back
  const int G = sym_images(job.sym);
  for (int j = 0; j < job.nfbv; ++j) {
    double gp[3] = {0.0, 0.0, 0.0}, gq = 0.0;
    for (int g = 0; g < G; ++g) {
      const double *h = &job.host[4 * ((size_t)j * G + g)];
      sym_fold(g, h, gp);
      gq += h[3];
    }
    dL_dpos[3 * j] = gp[0];
    dL_dpos[3 * j + 1] = gp[1];
    dL_dpos[3 * j + 2] = gp[2];
    dL_dq[j] = gq;
  }
  if (dL_dalpha)
    for (int m = 0; m < job.nalpha; ++m) dL_dalpha[m] = job.host[4 * job.N + m];
  if (dL_dt) *dL_dt = job.host[4 * job.N + job.nalpha];
}

}  // namespace

int32_t shh_grad(const shh_design *design, const shh_opts *opts, void *d_ws, size_t ws_bytes,
                 const double dL_dCH[36], double dL_dV, double *dL_dpos, double *dL_dq, double *dL_dalpha,
                 double *dL_dt, void *hip_stream) {
  if (!dL_dpos || !dL_dq) return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  GradJob job;
  SHH_TRY(grad_enqueue(job, design, opts, d_ws, ws_bytes, dL_dCH, dL_dV, st));
  SHH_HIP(hipStreamSynchronize(st));
  grad_unpack(job, dL_dpos, dL_dq, dL_dalpha, dL_dt);
  return SHH_OK;
}

int32_t shh_grad_batch(const shh_design *designs, int32_t count, const shh_opts *opts, void *const *d_ws,
                       const size_t *ws_bytes, const double *dL_dCH, const double *dL_dV, double *dL_dpos,
                       double *dL_dq, double *dL_dalpha, double *dL_dt, void *hip_stream) {
  if (count < 1 || !designs || !d_ws || !ws_bytes || !dL_dCH || !dL_dV || !dL_dpos || !dL_dq)
    return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  // every design's adjoint is enqueued before the one synchronization
  std::vector<std::unique_ptr<GradJob>> jobs;
  for (int i = 0; i < count; ++i) {
    jobs.emplace_back(new GradJob());
    SHH_TRY(grad_enqueue(*jobs.back(), &designs[i], opts, d_ws[i], ws_bytes[i], dL_dCH + 36 * i, dL_dV[i], st));
  }
  SHH_HIP(hipStreamSynchronize(st));
  size_t off = 0, aoff = 0;
  for (int i = 0; i < count; ++i) {
    grad_unpack(*jobs[i], dL_dpos + 3 * off, dL_dq + off, dL_dalpha ? dL_dalpha + aoff : nullptr,
                dL_dt ? dL_dt + i : nullptr);
    off += designs[i].num_charges;
    aoff += jobs[i]->nalpha;
  }
  return SHH_OK;
}

}  // extern "C"

namespace {

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

// Byte sizes of the point-field workspace: a field-only slot (no grid), then
// the per-point basis table, dL/dcoef and the charge/alpha gradients.
struct PointsLayout {
  size_t slot, basis, dcoef, out, total;
};

PointsLayout points_layout(const shh_design *d, int npts) {
  const Layout L = make_layout(2, charge_count(d), d->K, SHH_PREC_FP64, false, false);
  const size_t nb = 2 * (size_t)d->K + 1, K1 = (size_t)d->K + 1;
  PointsLayout P;
  P.slot = al256(L.total + seg_region() + 256);
  P.basis = al256(sizeof(double) * (size_t)npts * 3 * nb);
  P.dcoef = al256(sizeof(double) * nb * nb * nb);
  P.out = al256(sizeof(double) * (4 * (size_t)charge_count(d) + K1 * K1 * K1));
  P.total = P.slot + P.basis + P.dcoef + P.out;
  return P;
}

// The point field reads only the charges, alpha, K and the symmetry mode:
// the rest of the design is replaced by valid placeholders before validation.
shh_design points_design(const shh_design *in) {
  shh_design d = *in;
  d.n = 2;
  d.iso = 0.0;
  d.thickness = 0.0;
  d.target_vf = 0.0;
  d.kappa = 0.0;
  d.dist_mode = 0;
  d.E = 1.0;
  d.nu = 0.3;
  d.E_void = 0.0;
  return d;
}

int points_slot(Slot &s, const shh_design *design, int npts, void *d_ws, size_t ws_bytes, PointsLayout &P,
                hipStream_t st) {
  if (!design) return SHH_INVALID_ARG;
  shh_design d = points_design(design);
  SHH_TRY(validate_design(&d));
  if (npts < 1 || npts > (1 << 26) || !d_ws) return SHH_INVALID_ARG;
  P = points_layout(&d, npts);
  if (ws_bytes < P.total) return SHH_WORKSPACE_TOO_SMALL;
  shh_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = SHH_PREC_FP64;
  o.rtol = 1e-10;
  o.max_iter = 1;
  SHH_TRY(normalize_opts(&o, &o));
  SHH_TRY(prepare_slot(s, &d, &o, d_ws, ws_bytes, nullptr, false));
  SHH_TRY(slot_init(s, s.base, st));
  return SHH_OK;
}

}  // namespace

extern "C" {

int32_t shh_workspace_bytes_points(const shh_design *design, int32_t npts, size_t *bytes) {
  if (!design) return SHH_INVALID_ARG;
  const shh_design d = points_design(design);
  SHH_TRY(validate_design(&d));
  if (npts < 1 || npts > (1 << 26) || !bytes) return SHH_INVALID_ARG;
  *bytes = points_layout(&d, npts).total;
  return SHH_OK;
}

int32_t shh_field_points(const shh_design *design, int32_t npts, const double *d_pts, double *d_F, double *d_G,
                         void *d_ws, size_t ws_bytes, void *hip_stream) {
  if (!d_pts || !d_F) return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  PointsLayout P;
  SHH_TRY(points_slot(s, design, npts, d_ws, ws_bytes, P, st));
  SHH_HIP(launch_coef(s.d_slot, s.host.nb, st));
  SHH_HIP(launch_points_field(s.d_slot, s.host.nb, npts, d_pts, d_F, d_G, st));
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int32_t shh_field_points_grad(const shh_design *design, int32_t npts, const double *d_pts, const double *d_dL_dF,
                              double *dL_dpos, double *dL_dq, double *dL_dalpha, void *d_ws, size_t ws_bytes,
                              void *hip_stream) {
  if (!d_pts || !d_dL_dF || !dL_dpos || !dL_dq) return SHH_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  Slot s;
  PointsLayout P;
  SHH_TRY(points_slot(s, design, npts, d_ws, ws_bytes, P, st));
  char *base = (char *)d_ws;
  base = (char *)(((uintptr_t)base + 255) & ~uintptr_t(255));
  double *d_basis = (double *)(base + P.slot);
  double *d_dcoef = (double *)(base + P.slot + P.basis);
  double *d_out = (double *)(base + P.slot + P.basis + P.dcoef);
  const int Nx = s.host.N, K1 = s.host.K + 1;
  SHH_HIP(launch_points_dcoef(s.host.nb, npts, d_pts, d_dL_dF, d_basis, d_dcoef, st));
  SHH_HIP(launch_coef_adjoint(s.d_slot, Nx, s.host.K, d_dcoef, d_out, d_out + 4 * Nx, st));
  GradJob job;
  job.N = Nx;
  job.nalpha = K1 * K1 * K1;
  job.sym = design->symmetry;
  job.nfbv = design->num_charges;
  job.host.assign(4 * (size_t)Nx + job.nalpha + 1, 0.0);
  SHH_HIP(hipMemcpyAsync(job.host.data(), d_out, sizeof(double) * (4 * (size_t)Nx + job.nalpha),
                         hipMemcpyDeviceToHost, st));
  SHH_HIP(hipStreamSynchronize(st));
  grad_unpack(job, dL_dpos, dL_dq, dL_dalpha, nullptr);
  return SHH_OK;
}

int32_t shh_profile_enable(int32_t on) {
  profile_enable(on != 0);
  return SHH_OK;
}

int32_t shh_profile_read(int32_t kind, int64_t *launches, double *ms_total) {
  long long l = 0;
  double m = 0.0;
  SHH_TRY(profile_read(kind, &l, &m));
  if (launches) *launches = l;
  if (ms_total) *ms_total = m;
  return SHH_OK;
}

}  // extern "C"

// ---- serving engine ---------------------------------------------------------------

struct shh_engine {
  hipStream_t st = nullptr;
  char *arena = nullptr;
  size_t bytes = 0;
  size_t header = 0;
  int max_slots = 0;
  int prec = -1;
  // free list of [begin, end) byte ranges inside the arena
  std::map<size_t, size_t> free_ranges;
  struct Pending {
    uint64_t id;
    DesignCopy design;
    shh_opts opts;
  };
  std::deque<Pending> queue;
  std::vector<std::unique_ptr<Slot>> resident;
  std::vector<size_t> resident_off;
  std::deque<std::pair<uint64_t, shh_result>> completed;
  std::unique_ptr<Solver> solver;

  bool alloc(size_t need, size_t &off) {
    need = (need + 255) & ~size_t(255);
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      const size_t b = it->first, e = it->second;
      if (e - b >= need) {
        off = b;
        free_ranges.erase(it);
        if (e - b > need) free_ranges[b + need] = e;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t need) {
    need = (need + 255) & ~size_t(255);
    size_t b = off, e = off + need;
    auto nx = free_ranges.lower_bound(b);
    if (nx != free_ranges.end() && nx->first == e) {
      e = nx->second;
      nx = free_ranges.erase(nx);
    }
    if (nx != free_ranges.begin()) {
      auto pv = std::prev(nx);
      if (pv->second == b) {
        b = pv->first;
        free_ranges.erase(pv);
      }
    }
    free_ranges[b] = e;
  }
};

extern "C" {

int32_t shh_engine_footprint(const shh_design *design, const shh_opts *opts, size_t *bytes) {
  SHH_TRY(validate_design(design));
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  if (!bytes) return SHH_INVALID_ARG;
  SHH_TRY(check_solver(design->n, &o));
  const Layout L = make_layout(design->n, charge_count(design), design->K, o.precision, o.save_for_backward != 0,
                               true, o.solver);
  *bytes = (L.total + 255) & ~size_t(255);
  return SHH_OK;
}

int32_t shh_engine_create(void *d_arena, size_t arena_bytes, int32_t max_slots, void *hip_stream,
                          shh_engine **out) {
  if (!d_arena || !out || max_slots < 1 || max_slots > 4096) return SHH_INVALID_ARG;
  shh_engine *e = new (std::nothrow) shh_engine();
  if (!e) return SHH_INVALID_ARG;
  e->st = (hipStream_t)hip_stream;
  e->arena = aligned(d_arena);
  const size_t lost = size_t(e->arena - (char *)d_arena);
  if (arena_bytes <= lost) {
    delete e;
    return SHH_WORKSPACE_TOO_SMALL;
  }
  e->bytes = arena_bytes - lost;
  e->max_slots = max_slots;
  e->header = (Solver::seg_bytes(max_slots) + 255) & ~size_t(255);
  if (e->header >= e->bytes) {
    delete e;
    return SHH_WORKSPACE_TOO_SMALL;
  }
  e->free_ranges[e->header] = e->bytes;
  e->solver.reset(new Solver(e->st));
  e->solver->set_segment_memory(e->arena, e->header);
  *out = e;
  return SHH_OK;
}

int32_t shh_engine_submit(shh_engine *eng, const shh_design *design, const shh_opts *opts, uint64_t request_id) {
  if (!eng) return SHH_INVALID_ARG;
  SHH_TRY(validate_design(design));
  shh_opts o;
  SHH_TRY(normalize_opts(opts, &o));
  if (eng->prec >= 0 && o.precision != eng->prec) return SHH_INVALID_ARG;
  SHH_TRY(check_solver(design->n, &o));  // SHH_SOLVER_AUTO: multigrid or Jacobi for this grid
  size_t need = 0;
  SHH_TRY(shh_engine_footprint(design, &o, &need));
  if (need > eng->bytes - eng->header) return SHH_OVER_BUDGET;
  eng->prec = o.precision;
  shh_engine::Pending p;
  p.id = request_id;
  copy_design(design, p.design);
  p.opts = o;
  eng->queue.push_back(std::move(p));
  return SHH_OK;
}

static int engine_admit(shh_engine *eng, std::vector<Slot *> &fresh) {
  while (!eng->queue.empty() && (int)eng->resident.size() < eng->max_slots) {
    shh_engine::Pending &p = eng->queue.front();
    const Layout L = make_layout(p.design.d.n, p.design.d.num_charges, p.design.d.K, p.opts.precision,
                                 p.opts.save_for_backward != 0, true, p.opts.solver);
    size_t off = 0;
    if (!eng->alloc(L.total, off)) break;  // first in line waits for memory
    std::unique_ptr<Slot> s(new Slot());
    s->design = std::move(p.design);
    s->design.d.pos = s->design.pos.data();
    s->design.d.q = s->design.q.data();
    s->design.d.alpha = s->design.alpha.empty() ? nullptr : s->design.alpha.data();
    s->opts = p.opts;
    s->lay = L;
    s->R = p.opts.recompute_every;
    s->id = p.id;
    for (auto &ev : s->ev) (void)hipEventCreate(&ev);
    eng->queue.pop_front();
    SHH_HIP(hipEventRecord(s->ev[0], eng->st));
    int rc = slot_init(*s, eng->arena + off, eng->st);
    if (rc == SHH_OK) rc = slot_setup_field(*s, nullptr, eng->st);
    if (rc != SHH_OK) {
      eng->release(off, L.total);
      shh_result r;
      std::memset(&r, 0, sizeof(r));
      r.status = rc;
      eng->completed.emplace_back(s->id, r);
      for (auto &ev : s->ev) (void)hipEventDestroy(ev);
      continue;
    }
    fresh.push_back(s.get());
    eng->resident.push_back(std::move(s));
    eng->resident_off.push_back(off);
  }
  return SHH_OK;
}

static void engine_retire(shh_engine *eng, size_t idx) {
  Slot *s = eng->resident[idx].get();
  for (auto &ev : s->ev) {
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
  }
  eng->release(eng->resident_off[idx], s->lay.total);
  eng->resident.erase(eng->resident.begin() + idx);
  eng->resident_off.erase(eng->resident_off.begin() + idx);
}

int32_t shh_engine_step(shh_engine *eng, int32_t iters, int32_t *n_resident, int32_t *n_queued) {
  if (!eng || iters < 0) return SHH_INVALID_ARG;
  std::vector<Slot *> fresh, failed, fresh_sel;
  SHH_TRY(engine_admit(eng, fresh));
  // selective requests run their own solve (compact lists, culled hierarchy)
  // beside the dense ones, one launch per step for all of them
  for (size_t i = fresh.size(); i-- > 0;)
    if (is_selective(fresh[i]->opts.solver)) {
      fresh_sel.push_back(fresh[i]);
      fresh.erase(fresh.begin() + i);
    }
  // a request whose own setup fails completes with its status; the others go on
  SHH_TRY(eng->solver->start(fresh, &failed));
  SHH_TRY(sel_start(fresh_sel, eng->st));
  std::vector<Slot *> done;
  for (Slot *s : fresh_sel)
    if (s->finished) (s->status < 0 ? failed : done).push_back(s);  // setup failure, or all culled
  for (Slot *f : failed) {
    shh_result r;
    std::memset(&r, 0, sizeof(r));
    r.status = f->status;
    eng->completed.emplace_back(f->id, r);
  }
  std::vector<Slot *> live, live_sel;
  for (auto &s : eng->resident)
    if (!s->finished) (is_selective(s->opts.solver) ? live_sel : live).push_back(s.get());
  if (iters > 0) {
    if (!live.empty()) {
      SHH_TRY(eng->solver->iterate(live, iters));
      SHH_TRY(eng->solver->poll(live, done));
    }
    if (!live_sel.empty()) {
      SHH_TRY(sel_step(live_sel, iters, eng->st));
      for (Slot *s : live_sel)
        if (s->finished) done.push_back(s);
    }
  }
  for (Slot *d : done) {
    shh_result r;
    fill_result(*d, &r);
    eng->completed.emplace_back(d->id, r);
  }
  if (!failed.empty() || !done.empty()) {
    SHH_HIP(hipStreamSynchronize(eng->st));  // their memory may still be in use
    for (size_t i = eng->resident.size(); i-- > 0;)
      if (eng->resident[i]->finished) engine_retire(eng, i);
  }
  if (n_resident) *n_resident = (int32_t)eng->resident.size();
  if (n_queued) *n_queued = (int32_t)eng->queue.size();
  return SHH_OK;
}

int32_t shh_engine_poll(shh_engine *eng, shh_result *out, uint64_t *ids, int32_t max, int32_t *n_out) {
  if (!eng || !n_out || max < 0 || (max > 0 && (!out || !ids))) return SHH_INVALID_ARG;
  int k = 0;
  while (k < max && !eng->completed.empty()) {
    ids[k] = eng->completed.front().first;
    out[k] = eng->completed.front().second;
    eng->completed.pop_front();
    ++k;
  }
  *n_out = k;
  return SHH_OK;
}

int32_t shh_engine_cancel(shh_engine *eng, uint64_t request_id) {
  if (!eng) return SHH_INVALID_ARG;
  for (auto it = eng->queue.begin(); it != eng->queue.end(); ++it) {
    if (it->id == request_id) {
      eng->queue.erase(it);
      return SHH_OK;
    }
  }
  for (size_t i = 0; i < eng->resident.size(); ++i) {
    if (eng->resident[i]->id == request_id) {
      SHH_HIP(hipStreamSynchronize(eng->st));  // its memory may still be in use
      engine_retire(eng, i);
      return SHH_OK;
    }
  }
  return SHH_NOT_FOUND;
}

void shh_engine_destroy(shh_engine *eng) {
  if (!eng) return;
  (void)hipStreamSynchronize(eng->st);
  while (!eng->resident.empty()) engine_retire(eng, eng->resident.size() - 1);
  delete eng;
}

}  // extern "C"
