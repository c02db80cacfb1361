// Host runtime of libshellhom: slot layout and setup, the batched six-load-case
// PCG driver, and the serving engine.  Everything here is host C++; the
// arithmetic of the path runs in the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <memory>
#include <vector>

#include "shellhom.h"
#include "common.hpp"
#include "mg.hpp"

namespace shh {

// Byte offsets of one design's buffers inside its device region.
struct Layout {
  size_t slotdev, state, charges, alpha, coef, partials, segs;
  size_t E64, E32, Dinv, x64, vec, field;
  size_t adj;         // adjoint scratch (save_for_backward only)
  size_t vec_bytes;   // one [6][3][n^3] vector
  size_t mg;          // multigrid region (0 bytes unless the multigrid solver is used)
  size_t total;
  int maxparts;
  bool vectors;       // false: operator-only slot (no CG vectors, no field arrays)
};

struct DesignCopy {
  shh_design d;                 // pointers below point into the vectors; charges expanded
                                // over the fundamental volume's images (d.symmetry = 0)
  std::vector<double> pos, q, alpha;
  int sym = 0;                  // the caller's symmetry mode
  int nfbv = 0;                 // the caller's charge count
};

struct SelHost;  // selective solve state of a slot (selsolve.cpp)

struct Slot {
  DesignCopy design;
  shh_opts opts;
  Layout lay;
  char *base = nullptr;         // device region
  SlotDev host;                 // host image of the device descriptor
  SlotDev *d_slot = nullptr;
  CgState *d_state = nullptr;
  CgState state;                // last copy read back
  int launched = 0;             // CG iterations launched while resident
  int finals = 0;               // final-residual checks done
  int R = 0;                    // recompute period (0: never)
  bool finished = false;
  int status = SHH_OK;
  uint64_t id = 0;
  double t_arrive_ms = 0.0;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double ms[5] = {0, 0, 0, 0, 0};
  // multigrid solver (opts.solver == SHH_SOLVER_MG)
  MgDev mg;                     // host image of the level descriptors
  MgDev *d_mg = nullptr;
  bool mg_restart = false;      // next iteration starts from z = V r, p = z
  bool mg_keep_dir = false;     // ... or, after a residual replacement, p = z + beta p
  int sel_active_nodes = 0;     // selective solve: active nodes
  std::shared_ptr<SelHost> sel; // selective solve: descriptor and progress between steps
  bool timing = true;           // launch timing allowed (false: the no-allocation entry point)
};

// the culled solve of Sec. 4.2 (either preconditioner)
inline bool is_selective(int solver) {
  return solver == SHH_SOLVER_SELECTIVE || solver == SHH_SOLVER_SELECTIVE_JACOBI;
}
int validate_design(const shh_design *d);
// fundamental bounding volumes (shh_design.symmetry): image count, image g of a
// point, gradient fold of image g, charges after expansion
int sym_images(int sym);
void sym_image(int g, const double *p, double *v);
void sym_fold(int g, const double *gv, double *gp);
int charge_count(const shh_design *d);
int normalize_opts(const shh_opts *in, shh_opts *out);
Layout make_layout(int n, int N, int K, int prec, bool save, bool vectors = true, int solver = 0);
// bytes of the multigrid region of an n^3 slot (levels >= 1, coarsest inverse, descriptors)
size_t mg_region_bytes(int n, int prec);
// multigrid setup of a slot whose moduli and D^-1 are in place (before the CG
// vectors are zeroed: the element matrices use the vector region as scratch)
int mg_setup(Slot &s, hipStream_t st);
// the same for several slots at once (their power iterations batched).  With
// `rcs` null the first failure is returned; otherwise (*rcs)[i] receives slot
// i's own status (a slot that fails is left out of the remaining steps) and
// only HIP errors are returned.
int mg_setup(const std::vector<Slot *> &slots, hipStream_t st, std::vector<int> *rcs = nullptr);
// Voxel-level operator launches of the multigrid iteration: the CG direction
// pass (p_j = z + beta p_{j-1} into the other p buffer, q[0] = K p_j, partials
// p_j . q); r - K d for the stored Chebyshev direction (the residual the
// restriction takes, in place of r); the operator fused with the Chebyshev
// sweep after it (pre-smoother step 1, post-smoother steps 1 and 2)
enum { MG_SRC_DIR = 0, MG_SRC_RES = 1, MG_SRC_STEP1 = 2, MG_SRC_POST = 3, MG_SRC_LAST = 4, MG_SRC_POST1 = 5 };
class Solver;
using MgApply0 = std::function<int(const std::vector<Slot *> &, int)>;
// one multigrid-preconditioned CG iteration of every load case of the slots
// (timer: when profiling, the largest coarse level's operator launches are
// timed with their algorithmic bytes)
int mg_iterate(const std::vector<Slot *> &slots, hipStream_t st, Solver *timer, const MgApply0 &apply0);
// the V-cycle of set-up slots from level 1 down: lv[1].b in, lv[1].x out
// (the selective solve runs the voxel level itself); batched launches
int mg_vcycle_coarse(const std::vector<Slot *> &slots, hipStream_t st);
// q = A_l v for the Galerkin operator of level l >= 1 of a set-up slot (all six
// load cases, [6][3][n_l^3] in the slot's precision)
int mg_apply_level(Slot &s, int l, const void *d_v, void *d_q, hipStream_t st);
void copy_design(const shh_design *src, DesignCopy &dst);

// Fill the slot descriptor for a region and upload it (+ charges, alpha, zeroed state).
int slot_init(Slot &s, char *base, hipStream_t st);
// Field, distance, thickness, occupancy, Jacobi diagonal (steps 1-2).
int slot_setup_field(Slot &s, double *beta_out, hipStream_t st);
// Moduli given directly instead of steps 1-2 (e_dtype as SHH_EDTYPE_*; Es, Ev
// the solid and void moduli of the byte code).
int slot_setup_moduli(Slot &s, const void *d_E, int e_dtype, double Es, double Ev, hipStream_t st);

// Batched solver over a set of slots sharing one stream.
class Solver {
 public:
  explicit Solver(hipStream_t st) : st_(st) {}
  // Device memory for the segment tables (must hold seg_bytes(max_slots)).
  void set_segment_memory(char *d_mem, size_t bytes);
  static size_t seg_bytes(int max_slots);
  // zero vectors + initial residual for newly set-up slots.  With `failed`
  // null the first failure is returned; otherwise a slot whose own setup fails
  // (e.g. a multigrid hierarchy without a positive spectrum estimate) is marked
  // finished with that status, appended to *failed and left out, and the
  // others start; only HIP errors are returned then.
  int start(const std::vector<Slot *> &slots, std::vector<Slot *> *failed = nullptr);
  // run `iters` CG iterations over the resident slots (recomputes as due)
  int iterate(const std::vector<Slot *> &slots, int iters);
  // read back states; for slots whose load cases are all inactive run the final
  // residual check and, if it holds, the C^H reduction. Returns slots finished now.
  int poll(const std::vector<Slot *> &slots, std::vector<Slot *> &done);
  int sync();
  // bracket one launch on the solver's stream with events when profiling is
  // on (kind: SHH_PROF_*); resolved at the next synchronization
  int timed_begin(hipEvent_t *e0);
  int timed_end(hipEvent_t e0, int kind);
  // false: no HIP events are created for launch timing (the no-allocation
  // entry point), whatever shh_profile_enable says
  void set_timing(bool on) { timing_ = on; }

 private:
  bool timing_ = true;
  enum Kind { K_STENCIL = 0, K_RESID, K_FINISH, K_FOLD, K_ZERO, K_SCAL_IT, K_SCAL_RES, K_MG_DIR, K_MG_RES,
              K_MG_STEP1, K_MG_POST, K_MG_LAST,
              K_NKIND };
  int residual(const std::vector<Slot *> &slots, int mode);
  int iterate_mg(const std::vector<Slot *> &slots, int iters);
  int build(Kind k, const std::vector<Slot *> &slots, int flag, bool all_rhs, LaunchArgs &la);
  int read_states(const std::vector<Slot *> &slots);
  int final_check(const std::vector<Slot *> &slots);
  hipStream_t st_;
  char *seg_mem_ = nullptr;
  size_t seg_cap_ = 0;
  std::vector<Segment> host_segs_[K_NKIND];
  // events bracketing timed launches, resolved at the next synchronization
  std::vector<hipEvent_t> ev_pool_;
  struct Timed {
    hipEvent_t e0, e1;
    int kind;
  };
  std::vector<Timed> ev_timed_;
  hipEvent_t get_event();
  void resolve_events();

 public:
  ~Solver();
};

// process-wide launch timing by kernel family (shh_profile_*, SHH_PROF_*)
void profile_enable(bool on);
bool profile_on();
int profile_read(int kind, long long *launches, double *ms);
void profile_add(int kind, double ms);

double now_ms();
// the selective solve of slots whose culled moduli are in place (field setup
// or given moduli): compaction, CG on the active nodes, C^H; the slots share
// every launch (same precision and solver option).  sel_start sets up a set
// of slots (compaction, hierarchy, first residual); sel_step runs `iters`
// iterations of the unfinished ones, checks those that stopped and finishes
// them (C^H, status, s.finished); sel_solve runs both to the end.
int sel_start(const std::vector<Slot *> &slots, hipStream_t st);
int sel_step(const std::vector<Slot *> &slots, int iters, hipStream_t st);
int sel_solve(const std::vector<Slot *> &slots, hipStream_t st);
inline int sel_solve(Slot &s, hipStream_t st) { return sel_solve(std::vector<Slot *>{&s}, st); }
// the selective solve's dL/dE_e (dense [n^3], zero on culled voxels) for the
// folded weights g21 of dL/dC^H, from a slot solved with save_for_backward;
// *d_gE points into the slot's workspace
int sel_energy_gradient(Slot &s, const double g21[21], double **d_gE, hipStream_t st);
void fill_result(const Slot &s, shh_result *out);

}  // namespace shh
