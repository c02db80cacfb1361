// Host runtime of libshellhom: validation, slot layout and setup, and the
// batched PCG driver shared by the single-design entry points, the batch
// entry points and the serving engine.
#include "runtime.hpp"
#include "sel.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "kernels.hpp"

namespace shh {

#define SHH_HIP(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return SHH_HIP_ERROR;      \
  } while (0)

namespace {
std::atomic<bool> g_prof_on{false};
std::mutex g_prof_mu;
long long g_prof_launches[SHH_PROF_NKIND] = {};
double g_prof_ms[SHH_PROF_NKIND] = {};
}  // namespace

void profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on;
  if (on) {
    for (int k = 0; k < SHH_PROF_NKIND; ++k) {
      g_prof_launches[k] = 0;
      g_prof_ms[k] = 0.0;
    }
  }
}
bool profile_on() { return g_prof_on.load(); }
int profile_read(int kind, long long *launches, double *ms) {
  if (kind < 0 || kind >= SHH_PROF_NKIND) return SHH_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (launches) *launches = g_prof_launches[kind];
  if (ms) *ms = g_prof_ms[kind];
  return SHH_OK;
}
void profile_add(int kind, double ms) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_launches[kind] += 1;
  g_prof_ms[kind] += ms;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

static bool finite(double v) { return std::isfinite(v); }

int sym_images(int sym) { return sym == SHH_SYM_MIRROR ? 8 : (sym == SHH_SYM_CUBIC ? 48 : 1); }

// Image g of a point under the fundamental volume's group: the axes permuted
// (permutation g / 8 of six, cubic only), then reflected x_d -> 1 - x_d for
// the bits of g % 8.
static const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

void sym_image(int g, const double *p, double *v) {
  const int *pm = kPerm[g / 8];
  for (int d = 0; d < 3; ++d) {
    v[d] = p[pm[d]];
    if ((g >> d) & 1) v[d] = 1.0 - v[d];
  }
}

// dL/dp of a given charge accumulates dL/dv of its image g (the transpose of
// the image map's linear part)
void sym_fold(int g, const double *gv, double *gp) {
  const int *pm = kPerm[g / 8];
  for (int d = 0; d < 3; ++d) gp[pm[d]] += ((g >> d) & 1) ? -gv[d] : gv[d];
}

int charge_count(const shh_design *d) { return d->num_charges * sym_images(d->symmetry); }

int validate_design(const shh_design *d) {
  if (!d) return SHH_INVALID_ARG;
  if (d->n < 2 || d->n > 512) return SHH_INVALID_ARG;  // 32-bit byte offsets per vector
  if (d->num_charges < 1 || !d->pos || !d->q) return SHH_INVALID_ARG;
  if (d->symmetry < SHH_SYM_NONE || d->symmetry > SHH_SYM_CUBIC) return SHH_INVALID_ARG;
  if ((long long)d->num_charges * sym_images(d->symmetry) > 4096) return SHH_INVALID_ARG;
  if (d->K < 1 || d->K > MAXK) return SHH_INVALID_ARG;
  for (int j = 0; j < d->num_charges; ++j) {
    if (!finite(d->pos[3 * j]) || !finite(d->pos[3 * j + 1]) || !finite(d->pos[3 * j + 2]) ||
        !finite(d->q[j]))
      return SHH_INVALID_ARG;
  }
  if (d->alpha) {
    const int K1 = d->K + 1;
    for (int i = 0; i < K1 * K1 * K1; ++i)
      if (!finite(d->alpha[i])) return SHH_INVALID_ARG;
  }
  if (!finite(d->iso)) return SHH_INVALID_ARG;
  if (!finite(d->thickness)) return SHH_INVALID_ARG;
  if (d->thickness < 0 && !(d->target_vf > 0.0 && d->target_vf < 1.0)) return SHH_INVALID_ARG;
  if (!(d->kappa >= 0.0) || !finite(d->kappa)) return SHH_INVALID_ARG;
  if (d->dist_mode != 0 && d->dist_mode != 1) return SHH_INVALID_ARG;
  if (!(d->E > 0.0) || !finite(d->E)) return SHH_INVALID_ARG;
  if (!(d->nu > -1.0 && d->nu < 0.5)) return SHH_INVALID_ARG;
  if (!(d->E_void >= 0.0 && d->E_void <= d->E)) return SHH_INVALID_ARG;
  return SHH_OK;
}

int normalize_opts(const shh_opts *in, shh_opts *out) {
  if (!in) return SHH_INVALID_ARG;
  *out = *in;
  if (out->precision != SHH_PREC_FP64 && out->precision != SHH_PREC_MIXED) return SHH_INVALID_ARG;
  if (!(out->rtol > 0.0 && out->rtol < 1.0)) return SHH_INVALID_ARG;
  if (out->max_iter < 0 || out->recompute_every < 0 || out->check_every < 0) return SHH_INVALID_ARG;
  if (out->solver != SHH_SOLVER_JACOBI && out->solver != SHH_SOLVER_MG && out->solver != SHH_SOLVER_AUTO &&
      !is_selective(out->solver))
    return SHH_INVALID_ARG;
  // the selective multigrid solve replaces its FP32 residual five times as
  // often: its V-cycle puts large components along the culled operator's
  // (near-)null modes, which the FP32 recursion turns into residual drift
  if (out->recompute_every == 0 && out->precision == SHH_PREC_MIXED)
    out->recompute_every = out->solver == SHH_SOLVER_SELECTIVE ? 10 : 50;
  if (out->check_every == 0) out->check_every = 16;
  return SHH_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

#ifndef SHH_TZ
#define SHH_TZ 32
#endif
// z planes per stencil workgroup (the z-march length)
static int tz_for(int n) { return n < SHH_TZ ? n : SHH_TZ; }

Layout make_layout(int n, int N, int K, int prec, bool save, bool vectors, int solver) {
  Layout L{};
  L.vectors = vectors;
  const long long nn = (long long)n * n * n;
  const int nb = 2 * K + 1;
  const int tz_runs = (n + tz_for(n) - 1) / tz_for(n);
  const int tiles = std::max(((n + Tile<float>::X - 1) / Tile<float>::X) * ((n + Tile<float>::Y - 1) / Tile<float>::Y),
                             ((n + Tile<double>::X - 1) / Tile<double>::X) * ((n + Tile<double>::Y - 1) / Tile<double>::Y)) *
                    tz_runs;
  const int chunks = int((nn + CHUNK - 1) / CHUNK);
  L.maxparts = std::max(std::max(tiles, chunks), 1024);
  const size_t ts = prec == SHH_PREC_FP64 ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.slotdev = take(sizeof(SlotDev));
  L.state = take(sizeof(CgState));
  L.charges = take(sizeof(double) * 4 * (size_t)N);
  L.alpha = take(sizeof(double) * (size_t)(K + 1) * (K + 1) * (K + 1));
  L.coef = take(sizeof(double) * (size_t)nb * nb * nb);
  L.partials = take(sizeof(double) * (size_t)NRHS * L.maxparts * PSTRIDE);
  L.segs = take(4096);
  L.E64 = take(sizeof(double) * nn);
  L.E32 = prec == SHH_PREC_MIXED ? take(sizeof(float) * nn) : 0;
  L.Dinv = take(ts * nn);
  if (!vectors) {  // the operator calls bring their own vectors
    L.total = off;
    return L;
  }
  L.x64 = prec == SHH_PREC_MIXED ? take(sizeof(double) * NRHS * 3 * nn) : 0;
  L.vec_bytes = align256(ts * NRHS * 3 * nn);
  L.vec = take(7 * L.vec_bytes);  // r[2], p[2], q[2], x
  // after a forward with save, the adjoint takes r[0] for dL/dE and p[0], p[1],
  // q[0], q[1] as scratch -- or a region of its own on grids too small for
  // that, so that the solution (x, or x64) survives for further calls
  if (save) {
    const size_t adj = align256(adjoint_scratch_bytes(n, K));
    L.adj = adj <= 4 * L.vec_bytes ? L.vec + 2 * L.vec_bytes : take(adj);
  }
  L.field = save ? take(sizeof(double) * 5 * nn) : L.vec;  // F, G[3], d (aliased unless saved)
  // the selective solve takes the same multigrid region for its coarse levels
  if (solver == SHH_SOLVER_MG || solver == SHH_SOLVER_SELECTIVE) L.mg = take(mg_region_bytes(n, prec));
  L.total = off;
  return L;
}

void copy_design(const shh_design *src, DesignCopy &dst) {
  dst.d = *src;
  const int N = src->num_charges, G = sym_images(src->symmetry);
  dst.sym = src->symmetry;
  dst.nfbv = N;
  // the fundamental volume's charges and their images, charge by charge
  dst.pos.resize(3 * (size_t)N * G);
  dst.q.resize((size_t)N * G);
  for (int j = 0; j < N; ++j)
    for (int g = 0; g < G; ++g) {
      sym_image(g, src->pos + 3 * j, &dst.pos[3 * ((size_t)j * G + g)]);
      dst.q[(size_t)j * G + g] = src->q[j];
    }
  dst.d.num_charges = N * G;
  dst.d.symmetry = SHH_SYM_NONE;
  if (src->alpha) {
    const int K1 = src->K + 1;
    dst.alpha.assign(src->alpha, src->alpha + K1 * K1 * K1);
    dst.d.alpha = dst.alpha.data();
  } else {
    dst.alpha.clear();
    dst.d.alpha = nullptr;
  }
  dst.d.pos = dst.pos.data();
  dst.d.q = dst.q.data();
}

static void element_operator(double nu, double kop[KOP_N]) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double Mh[2] = {1.0, 1.0 / 3.0}, Sh[2] = {0.0, 4.0};
  // diagonal entry of component c at mode m depends on s_c and s_o1 + s_o2 only
  for (int sc = 0; sc < 2; ++sc)
    for (int so = 0; so < 3; ++so) {
      const int s1 = so > 0 ? 1 : 0, s2 = so > 1 ? 1 : 0;
      kop[sc * 3 + so] = ((lam + 2.0 * mu) * Sh[sc] * Mh[s1] * Mh[s2] +
                          mu * Mh[sc] * (Sh[s1] * Mh[s2] + Mh[s1] * Sh[s2])) / 64.0;
    }
  for (int mk = 0; mk < 2; ++mk) {
    kop[6 + mk] = 4.0 * lam * Mh[mk] / 64.0;
    kop[8 + mk] = 4.0 * mu * Mh[mk] / 64.0;
  }
}

int slot_init(Slot &s, char *base, hipStream_t st) {
  const shh_design &d = s.design.d;
  const int prec = s.opts.precision;
  s.base = base;
  const Layout &L = s.lay;
  SlotDev &h = s.host;
  std::memset(&h, 0, sizeof(h));
  const int n = d.n;
  h.n = n;
  h.prec = prec;
  h.nn = (long long)n * n * n;
  h.tz = tz_for(n);
  h.tiles_z = (n + h.tz - 1) / h.tz;
  h.tiles_x[0] = (n + Tile<double>::X - 1) / Tile<double>::X;
  h.tiles_y[0] = (n + Tile<double>::Y - 1) / Tile<double>::Y;
  h.tiles_x[1] = (n + Tile<float>::X - 1) / Tile<float>::X;
  h.tiles_y[1] = (n + Tile<float>::Y - 1) / Tile<float>::Y;
  for (int w = 0; w < 2; ++w) h.ntiles[w] = h.tiles_x[w] * h.tiles_y[w] * h.tiles_z;
  h.nchunks = int((h.nn + CHUNK - 1) / CHUNK);
  h.K = d.K;
  h.nb = 2 * d.K + 1;
  h.N = d.num_charges;
  h.dist_mode = d.dist_mode;
  h.maxparts = L.maxparts;
  h.mode_t = d.thickness >= 0 ? 0 : (d.kappa == 0.0 ? 1 : 2);
  h.lam = d.nu / ((1.0 + d.nu) * (1.0 - 2.0 * d.nu));
  h.mu = 1.0 / (2.0 * (1.0 + d.nu));
  h.E = d.E;
  h.E_void = is_selective(s.opts.solver) ? 0.0 : d.E_void;  // the culled system has no floor: E_e = E beta
  h.iso = d.iso;
  h.kappa = d.kappa;
  h.t_given = d.thickness;
  h.target_vf = d.target_vf;
  h.rtol = s.opts.rtol;
  h.max_iter = s.opts.max_iter;
  h.ffloor = 1e-12 * d.E * std::sqrt(3.0 * double(h.nn));
  h.cull = is_selective(s.opts.solver) ? SEL_EPS : 0.0;
  element_operator(d.nu, h.kop64);
  for (int i = 0; i < KOP_N; ++i) h.kop32[i] = (float)h.kop64[i];
  h.charges = (double *)(base + L.charges);
  h.alpha = d.alpha ? (double *)(base + L.alpha) : nullptr;
  h.coef = (double *)(base + L.coef);
  h.F = L.vectors ? (double *)(base + L.field) : nullptr;
  h.G = L.vectors ? h.F + h.nn : nullptr;
  h.d = L.vectors ? h.F + 4 * h.nn : nullptr;
  h.E64 = (double *)(base + L.E64);
  h.E32 = prec == SHH_PREC_MIXED ? (float *)(base + L.E32) : nullptr;
  h.Dinv = base + L.Dinv;
  if (L.vectors) {
    for (int b = 0; b < 2; ++b) {
      h.r[b] = base + L.vec + (0 + b) * L.vec_bytes;
      h.p[b] = base + L.vec + (2 + b) * L.vec_bytes;
      h.q[b] = base + L.vec + (4 + b) * L.vec_bytes;
    }
    h.x = base + L.vec + 6 * L.vec_bytes;
    h.x64 = prec == SHH_PREC_MIXED ? (double *)(base + L.x64) : (double *)h.x;
  }  // else: left null; each operator call sets the vectors it uses
  h.partials = (double *)(base + L.partials);
  h.st = (CgState *)(base + L.state);
  s.d_slot = (SlotDev *)(base + L.slotdev);
  s.d_state = h.st;
  std::vector<double> ch(4 * (size_t)h.N);
  for (int j = 0; j < h.N; ++j) {
    ch[4 * j] = d.pos[3 * j];
    ch[4 * j + 1] = d.pos[3 * j + 1];
    ch[4 * j + 2] = d.pos[3 * j + 2];
    ch[4 * j + 3] = d.q[j];
  }
  CgState init;
  std::memset(&init, 0, sizeof(init));
  init.t = d.thickness;
  if (h.mode_t == 2) {
    // min / max of the distance bit patterns, reduced with atomicMin / atomicMax
    init.sel_lo[0] = ~0ull;
    init.sel_hi[0] = 0ull;
  } else {
    // bisection range of the order-statistic search: [0, +inf]
    init.sel_lo[0] = init.sel_lo[1] = 0ull;
    init.sel_hi[0] = init.sel_hi[1] = 0x7FF0000000000000ull;
  }
  SHH_HIP(hipMemcpyAsync(s.d_slot, &h, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  SHH_HIP(hipMemcpyAsync(s.d_state, &init, sizeof(CgState), hipMemcpyHostToDevice, st));
  SHH_HIP(hipMemcpyAsync(h.charges, ch.data(), sizeof(double) * ch.size(), hipMemcpyHostToDevice, st));
  if (h.alpha) {
    const int K1 = d.K + 1;
    SHH_HIP(hipMemcpyAsync(h.alpha, d.alpha, sizeof(double) * K1 * K1 * K1, hipMemcpyHostToDevice, st));
  }
  // the host vectors above are released at return: wait for the copies
  SHH_HIP(hipStreamSynchronize(st));
  return SHH_OK;
}

int slot_setup_field(Slot &s, double *beta_out, hipStream_t st) {
  const SlotDev &h = s.host;
  SHH_HIP(launch_field(s.d_slot, h.n, h.nb, st));
  if (h.mode_t == 1) {
    const long long k = (long long)std::floor(h.target_vf * double(h.nn) + 0.5);
    SHH_HIP(launch_select_hard(s.d_slot, h.nn, k, st));
  } else if (h.mode_t == 2) {
    SHH_HIP(launch_minmax_d(s.d_slot, h.nn, st));
    SHH_HIP(launch_bisect_steps(s.d_slot, h.nn, 200, st));
  }
  SHH_HIP(launch_occupancy(s.d_slot, h.nn, beta_out, st));
  SHH_HIP(launch_dinv(s.d_slot, h.nn, h.prec, st));
  return SHH_OK;
}

int slot_setup_moduli(Slot &s, const void *d_E, int e_dtype, double Es, double Ev, hipStream_t st) {
  const SlotDev &h = s.host;
  SHH_HIP(launch_moduli_copy(s.d_slot, h.nn, d_E, e_dtype, Es, Ev, st));
  SHH_HIP(launch_dinv(s.d_slot, h.nn, h.prec, st));
  return SHH_OK;
}

// ---------------------------------------------------------------------------
// batched solver
// ---------------------------------------------------------------------------

size_t Solver::seg_bytes(int max_slots) {
  return align256(sizeof(Segment) * (size_t)std::max(max_slots, 1)) * K_NKIND;
}

void Solver::set_segment_memory(char *d_mem, size_t bytes) {
  seg_mem_ = d_mem;
  seg_cap_ = bytes / K_NKIND;
  for (auto &v : host_segs_) v.clear();
}

int Solver::build(Kind k, const std::vector<Slot *> &slots, int flag, bool all_rhs, LaunchArgs &la) {
  std::vector<Segment> segs;
  int first = 0;
  for (Slot *s : slots) {
    Segment g;
    std::memset(&g, 0, sizeof(g));
    g.slot = s->d_slot;
    g.first = first;
    g.flag = flag;
    const bool mg_apply = (k >= K_MG_DIR && k <= K_MG_LAST);
    const bool per_tile = (k == K_STENCIL || k == K_RESID || mg_apply);
    const bool scalar = (k == K_SCAL_IT || k == K_SCAL_RES);
    // the CG pass and the operator compute in the vector precision, the residual always in FP64
    const int tiling = (k == K_STENCIL || mg_apply) ? s->host.prec : 0;
    const int units = scalar ? 1 : (per_tile ? s->host.ntiles[tiling] : s->host.nchunks);
    if (k == K_FOLD || k == K_ZERO) {
      g.nrhs = 1;
      g.rhs[0] = 0;
    } else {
      g.nrhs = 0;
      for (int r = 0; r < NRHS; ++r) {
        // skip load cases known (from the last read-back) to be finished, unless asked for all
        const bool live = all_rhs || s->state.active[r];
        if (live) g.rhs[g.nrhs++] = r;
      }
      if (g.nrhs == 0) continue;
    }
    g.nblocks = units * g.nrhs;
    first += g.nblocks;
    segs.push_back(g);
  }
  la.nseg = int(segs.size());
  la.total = first;
  const size_t bytes = sizeof(Segment) * segs.size();
  if (bytes > seg_cap_) return SHH_WORKSPACE_TOO_SMALL;
  Segment *dst = (Segment *)(seg_mem_ + (size_t)k * seg_cap_);
  la.segs = dst;
  if (segs.empty()) return SHH_OK;
  auto &prev = host_segs_[k];
  const bool same = prev.size() == segs.size() &&
                    std::memcmp(prev.data(), segs.data(), bytes) == 0;
  if (!same) {
    SHH_HIP(hipMemcpyAsync(dst, segs.data(), bytes, hipMemcpyHostToDevice, st_));
    SHH_HIP(hipStreamSynchronize(st_));
    prev = segs;
  }
  return SHH_OK;
}

// Residual f - K x in FP64 (mode RES_INIT: x = 0), mean projection and the
// scalar update for the given slots.
int Solver::residual(const std::vector<Slot *> &slots, int mode) {
  if (slots.empty()) return SHH_OK;
  const int prec = slots[0]->host.prec;
  const bool all = mode != RES_RECOMPUTE;
  LaunchArgs la;
  int rc;
  if (mode != RES_INIT) {
    // apply the pending x update (and, mixed, move x into the FP64 accumulator)
    if ((rc = build(K_FOLD, slots, mode, true, la))) return rc;
    SHH_HIP(launch_fold(la, prec, st_));
  }
  if ((rc = build(K_RESID, slots, mode, all, la))) return rc;
  hipEvent_t e0 = nullptr;
  if (la.total > 0 && (rc = timed_begin(&e0))) return rc;
  SHH_HIP(launch_stencil_resid(la, prec, st_));
  if ((rc = timed_end(e0, SHH_PROF_RESID64))) return rc;
  LaunchArgs ls;
  if ((rc = build(K_SCAL_RES, slots, mode, all, ls))) return rc;
  SHH_HIP(launch_scalar(ls, PH_MEAN, st_));
  if ((rc = build(K_FINISH, slots, mode, all, la))) return rc;
  SHH_HIP(launch_finish_resid(la, prec, st_));
  SHH_HIP(launch_scalar(ls, PH_RESID, st_));
  // a multigrid-preconditioned CG takes z = V r of the new residual: a
  // restart after the first and the final residual, the direction kept after
  // a replacement (reliable updates)
  for (Slot *s : slots) {
    s->mg_restart = true;
    s->mg_keep_dir = mode == RES_RECOMPUTE;
  }
  return SHH_OK;
}

int Solver::start(const std::vector<Slot *> &in, std::vector<Slot *> *failed) {
  if (in.empty()) return SHH_OK;
  const int prec = in[0]->host.prec;
  LaunchArgs la;
  int rc;
  // multigrid hierarchies first: their setup borrows the CG vector region
  std::vector<Slot *> mgs;
  for (Slot *s : in)
    if (s->opts.solver == SHH_SOLVER_MG) mgs.push_back(s);
  std::vector<int> rcs;
  if ((rc = mg_setup(mgs, st_, failed ? &rcs : nullptr))) return rc;
  std::vector<Slot *> slots;
  for (Slot *s : in) {
    bool ok = true;
    for (size_t i = 0; i < rcs.size(); ++i)
      if (mgs[i] == s && rcs[i] != SHH_OK) {
        s->finished = true;
        s->status = rcs[i];
        failed->push_back(s);
        ok = false;
      }
    if (ok) slots.push_back(s);
  }
  if (slots.empty()) return SHH_OK;
  if ((rc = build(K_ZERO, slots, 0, true, la))) return rc;
  SHH_HIP(launch_zero_vectors(la, prec, st_));
  for (Slot *s : slots) if (s->ev[1]) SHH_HIP(hipEventRecord(s->ev[1], st_));
  if ((rc = residual(slots, RES_INIT))) return rc;
  for (Slot *s : slots) {
    if (s->ev[2]) SHH_HIP(hipEventRecord(s->ev[2], st_));
    for (int r = 0; r < NRHS; ++r) s->state.active[r] = 1;  // refreshed at the next read-back
    s->launched = 0;
  }
  return SHH_OK;
}

Solver::~Solver() {
  resolve_events();
  for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
}

hipEvent_t Solver::get_event() {
  if (!ev_pool_.empty()) {
    hipEvent_t e = ev_pool_.back();
    ev_pool_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Call only after the stream has been synchronized.
void Solver::resolve_events() {
  for (auto &tk : ev_timed_) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, tk.e0, tk.e1) == hipSuccess) profile_add(tk.kind, ms);
    ev_pool_.push_back(tk.e0);
    ev_pool_.push_back(tk.e1);
  }
  ev_timed_.clear();
}

int Solver::iterate(const std::vector<Slot *> &all, int iters) {
  if (all.empty()) return SHH_OK;
  std::vector<Slot *> slots, mgs;
  for (Slot *s : all) (s->opts.solver == SHH_SOLVER_MG ? mgs : slots).push_back(s);
  int rc;
  if (!mgs.empty() && (rc = iterate_mg(mgs, iters))) return rc;
  if (slots.empty()) return SHH_OK;
  const int prec = slots[0]->host.prec;
  LaunchArgs la_s;
  if ((rc = build(K_STENCIL, slots, 0, false, la_s))) return rc;
  LaunchArgs la_c;
  if ((rc = build(K_SCAL_IT, slots, 0, false, la_c))) return rc;
  for (int it = 0; it < iters; ++it) {
    hipEvent_t e0 = nullptr;
    if (la_s.total > 0 && (rc = timed_begin(&e0))) return rc;
    SHH_HIP(launch_stencil_pcg(la_s, prec, st_));
    if ((rc = timed_end(e0, SHH_PROF_CG_PASS))) return rc;
    SHH_HIP(launch_scalar(la_c, PH_ITER, st_));
    std::vector<Slot *> due;
    for (Slot *s : slots) {
      s->launched += 1;
      if (s->R > 0 && s->launched % s->R == 0) due.push_back(s);
    }
    if (!due.empty()) {
      if ((rc = residual(due, RES_RECOMPUTE))) return rc;
    }
  }
  return SHH_OK;
}

// Multigrid-preconditioned CG: one launch sequence per slot and iteration.
int Solver::iterate_mg(const std::vector<Slot *> &slots, int iters) {
  int rc;
  // voxel-level operator over all the given slots, one launch
  MgApply0 apply0 = [this](const std::vector<Slot *> &ss, int src) -> int {
    // (the degree-1 post-smoothing pass takes the last sweep's segments and
    // profile kind: it replaces it)
    static const Kind kinds[6] = {K_MG_DIR, K_MG_RES, K_MG_STEP1, K_MG_POST, K_MG_LAST, K_MG_LAST};
    static const int ops[6] = {SMG_DIR, SMG_RES, SMG_STEP1, SMG_POST, SMG_LAST, SMG_POST1};
    static const int prof[6] = {SHH_PROF_MG_DIR, SHH_PROF_MG_RES, SHH_PROF_MG_STEP1, SHH_PROF_MG_POST,
                                SHH_PROF_MG_LAST, SHH_PROF_MG_LAST};
    if (src < 0 || src > MG_SRC_POST1) return SHH_INVALID_ARG;
    LaunchArgs la;
    int r;
    // segments of the load cases still running at the last read-back; the
    // kernels also skip those that stopped since
    if ((r = build(kinds[src], ss, 0, false, la))) return r;
    if (la.total == 0) return SHH_OK;
    hipEvent_t e0 = nullptr;
    if ((r = timed_begin(&e0))) return r;
    SHH_HIP(launch_stencil_mg(la, ss[0]->host.prec, ops[src], st_));
    return timed_end(e0, prof[src]);
  };
  for (int it = 0; it < iters; ++it) {
    if ((rc = mg_iterate(slots, st_, this, apply0))) return rc;
    std::vector<Slot *> due;
    for (Slot *s : slots) {
      s->launched += 1;
      if (s->R > 0 && s->launched % s->R == 0) due.push_back(s);
    }
    if (!due.empty() && (rc = residual(due, RES_RECOMPUTE))) return rc;
  }
  return SHH_OK;
}

int Solver::timed_begin(hipEvent_t *e0) {
  *e0 = nullptr;
  if (!timing_ || !profile_on()) return SHH_OK;
  *e0 = get_event();
  if (*e0) SHH_HIP(hipEventRecord(*e0, st_));
  return SHH_OK;
}

int Solver::timed_end(hipEvent_t e0, int kind) {
  if (!e0) return SHH_OK;
  hipEvent_t e1 = get_event();
  if (!e1) {
    ev_pool_.push_back(e0);
    return SHH_OK;
  }
  SHH_HIP(hipEventRecord(e1, st_));
  ev_timed_.push_back({e0, e1, kind});
  return SHH_OK;
}

int Solver::read_states(const std::vector<Slot *> &slots) {
  for (Slot *s : slots)
    SHH_HIP(hipMemcpyAsync(&s->state, s->d_state, sizeof(CgState), hipMemcpyDeviceToHost, st_));
  SHH_HIP(hipStreamSynchronize(st_));
  resolve_events();
  return SHH_OK;
}

int Solver::sync() {
  SHH_HIP(hipStreamSynchronize(st_));
  resolve_events();
  return SHH_OK;
}

static bool all_inactive(const CgState &c) {
  for (int r = 0; r < NRHS; ++r)
    if (c.active[r]) return false;
  return true;
}

int Solver::final_check(const std::vector<Slot *> &slots) {
  if (slots.empty()) return SHH_OK;
  int rc;
  if ((rc = residual(slots, RES_FINAL))) return rc;
  for (Slot *s : slots) s->finals += 1;
  return read_states(slots);
}

int Solver::poll(const std::vector<Slot *> &slots, std::vector<Slot *> &done) {
  int rc;
  if ((rc = read_states(slots))) return rc;
  std::vector<Slot *> cand;
  for (Slot *s : slots)
    if (!s->finished && all_inactive(s->state)) cand.push_back(s);
  if (cand.empty()) return SHH_OK;
  for (Slot *s : cand) if (s->ev[3]) SHH_HIP(hipEventRecord(s->ev[3], st_));
  if ((rc = final_check(cand))) return rc;
  std::vector<Slot *> fin;
  for (Slot *s : cand) {
    if (!all_inactive(s->state) && s->finals < 8) {
      // true residual above rtol: resume.  Align the recompute schedule with
      // the device iteration count so that a design's arithmetic does not
      // depend on when the host happened to poll it.
      int m = 0;
      for (int r = 0; r < NRHS; ++r) m = std::max(m, s->state.iters[r]);
      s->launched = m;
      continue;
    }
    fin.push_back(s);
  }
  for (Slot *s : fin) {
    SHH_HIP(launch_energy(s->d_slot, s->host.nn, st_));
    if (s->ev[4]) SHH_HIP(hipEventRecord(s->ev[4], st_));
  }
  if (!fin.empty()) {
    if ((rc = read_states(fin))) return rc;
  }
  for (Slot *s : fin) {
    s->finished = true;
    int status = SHH_OK;
    for (int r = 0; r < NRHS; ++r) {
      if (s->state.status[r] == ST_BREAKDOWN) status = SHH_BREAKDOWN;
      else if (status == SHH_OK && s->state.status[r] != ST_CONVERGED) status = SHH_NOT_CONVERGED;
    }
    s->status = status;
    float a = 0.f;
    if (s->ev[0] && hipEventElapsedTime(&a, s->ev[0], s->ev[1]) == hipSuccess) s->ms[0] = a;
    if (s->ev[1] && hipEventElapsedTime(&a, s->ev[1], s->ev[2]) == hipSuccess) s->ms[1] = a;
    if (s->ev[2] && hipEventElapsedTime(&a, s->ev[2], s->ev[3]) == hipSuccess) s->ms[2] = a;
    if (s->ev[3] && hipEventElapsedTime(&a, s->ev[3], s->ev[4]) == hipSuccess) s->ms[3] = a;
    if (s->ev[0] && hipEventElapsedTime(&a, s->ev[0], s->ev[4]) == hipSuccess) s->ms[4] = a;
    done.push_back(s);
  }
  return SHH_OK;
}

void fill_result(const Slot &s, shh_result *out) {
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < 36; ++i) out->CH[i] = s.state.C[i];
  out->vol_frac = s.state.V;
  out->t_used = s.state.t;
  for (int r = 0; r < NRHS; ++r) {
    out->iters[r] = s.state.iters[r];
    out->rel_res[r] = s.state.rel_true[r];
  }
  for (int i = 0; i < 5; ++i) out->ms[i] = s.ms[i];
  out->status = s.status;
  out->active_nodes = is_selective(s.opts.solver) ? s.sel_active_nodes : int32_t(s.host.nn);
}

}  // namespace shh
