// Shared definitions of the HIP kernels and the host runtime of libshellhom.
//
// One "slot" is one design resident on the GPU: its voxel grid, its six-load-
// case CG vectors and a small device-resident state block (CG scalars,
// reduction counters, results).  Every kernel works on a list of slots at
// once; a launch covers "segments" (slot, active load cases, tiles) and each
// workgroup decodes its (slot, load case, tile) from its block index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shh {

constexpr int NRHS = 6;       // Voigt unit-strain load cases (Eq. (8))
constexpr int KOP_N = 10;     // constants of the factored element operator
constexpr int MAXK = 6;       // largest truncation order supported
constexpr int MAXB = 2 * MAXK + 1;  // 1D basis functions per axis: 1, cos, sin up to K

// ---- stencil tiling ----
// A stencil workgroup owns an X x Y tile of nodes in the x-y plane and marches
// up tz planes in z.  Kernels that compute in FP32 use a wide 64 x 6 tile: its
// halo ring has 12 side-column nodes per 384 outputs (each of those pulls a
// whole 128-byte line), 8 waves per workgroup, 2 workgroups per CU.  Kernels
// that compute in FP64 hold twice the bytes in LDS per node and use 32 x 8.
#ifndef SHH_F32_TILE_X
#define SHH_F32_TILE_X 64
#endif
#ifndef SHH_F32_TILE_Y
#define SHH_F32_TILE_Y 6
#endif
#ifndef SHH_F64_TILE_X
#define SHH_F64_TILE_X 32
#endif
#ifndef SHH_F64_TILE_Y
#define SHH_F64_TILE_Y 8
#endif

template <typename TC> struct TileDims;
template <> struct TileDims<float> { static constexpr int X = SHH_F32_TILE_X, Y = SHH_F32_TILE_Y; };
template <> struct TileDims<double> { static constexpr int X = SHH_F64_TILE_X, Y = SHH_F64_TILE_Y; };

// Index of a compute precision's tiling in the per-slot tile counts.
template <typename TC> constexpr int tiling_of() { return sizeof(TC) == 4 ? 1 : 0; }

template <typename TC>
struct Tile {
  static constexpr int X = TileDims<TC>::X, Y = TileDims<TC>::Y;
  static constexpr int HX = X + 2, HY = Y + 2;        // node halo tile
  static constexpr int EXC = X + 1, EYC = Y + 1;      // element columns needed by the tile
  static constexpr int NHALO = HX * HY;
  static constexpr int NELEMC = EXC * EYC;
  // one thread per element column, rounded up to whole waves
  static constexpr int THREADS = ((NELEMC + 63) / 64) * 64;
  static constexpr int NINT = X * Y;                  // interior (owned) nodes
  static constexpr int NRING = NHALO - NINT;          // halo ring: 2 (X + 2) + 2 Y nodes
  static_assert(2 * THREADS >= NHALO, "each thread stages at most two halo nodes");
  static_assert(NINT <= THREADS, "one output node per thread");
  static_assert(THREADS <= 1024, "one workgroup");
};

// ---- vector-update chunking ----
constexpr int CHUNK = 1024;         // nodes per workgroup in the update kernels (4 per thread)
constexpr int VEC_THREADS = 256;
constexpr int PSTRIDE = 8;          // doubles per workgroup partial of the CG kernels

// ---- per-slot device state ----
// ST_STALLED: the selective multigrid CG lost definiteness after keeping its
// direction across a residual replacement; the case waits for the design's
// final residual check, which resumes it from a restart, and restarts after
// every later replacement
enum SolveStatus : int { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXIT = 2, ST_STALLED = 3, ST_BREAKDOWN = -6 };

struct CgState {
  double rho[NRHS];       // r^T D^-1 r of the current residual
  double rho_prev[NRHS];  // the previous one (for a replaced residual's beta)
  double rho_mg[NRHS];    // multigrid CG: r . z at the start of the last iteration
  double alpha[NRHS];     // step length of the update still to be applied to x, r
  double beta[NRHS];      // coefficient of the next direction update
  double rr[NRHS];        // ||r||^2 (recursive, or true after a recompute)
  double ff[NRHS];        // ||f||^2
  double rel[NRHS];       // ||r|| / ||f|| last seen
  double rel_true[NRHS];  // ||f - K u|| / ||f|| at the last recompute
  double rel_min[NRHS];   // selective multigrid CG: the smallest of those so far
  double mean[NRHS][3];   // mean of the recomputed residual per component
  int active[NRHS];       // 1 while load case k iterates
  int status[NRHS];
  int iters[NRHS];
  int pcur[NRHS];         // which of the two r, p, q buffer sets is current
  int mgpar[NRHS];        // multigrid CG: which p buffer holds the current direction
  int no_keep[NRHS];      // selective multigrid CG: restart after every replacement (set by a stall)
  int stag[NRHS];         // selective CG: replacements since the true residual last fell by 1 %
  unsigned cnt[8];        // last-workgroup counters (0..5 per load case, 6, 7 misc)
  double V;               // volume fraction
  double t;               // half-thickness used
  double gmax;            // max ||grad F|| (stored as bits for atomicMax)
  unsigned long long gmax_bits;
  double Emax;
  double C[36];           // homogenized tensor
  // thickness selection state
  unsigned long long sel_lo[2], sel_hi[2];  // bisection over distance bit patterns
  double bis_lo, bis_hi, bis_V;             // logistic bisection on t
  int bis_done;
  int pad_;
};

struct SlotDev {
  int n;
  int prec;             // 0 FP64, 1 mixed
  long long nn;         // n^3
  int tiles_x[2], tiles_y[2], ntiles[2];  // by tiling: [0] FP64-compute, [1] FP32-compute kernels
  int tiles_z, tz;
  int nchunks;
  int K, nb, N;
  int dist_mode;
  int maxparts;
  int mode_t;           // 0: thickness given, 1: hard-step selection, 2: logistic bisection
  double lam, mu;       // Lame parameters at E = 1
  double E, E_void, iso, kappa, t_given, target_vf;
  double rtol;
  double ffloor;        // ||f|| at or below this counts as a zero load
  double cull;          // > 0: selective solve, voxels with beta <= cull carry no
                        // stiffness and the others E beta (Sec. 4.2); 0: the
                        // stiffness floor E_void + (E - E_void) beta
  int max_iter;
  int pad_;
  // element operator in the per-axis Walsh-Hadamard basis, already scaled by
  // 1/64: the diagonal entry of component c at mode m depends only on s_c and
  // on the number of difference modes among the two other axes (6 classes,
  // index 3 s_c + s_o1 + s_o2), then the couplings 4 lambda Mhat[s|d] / 64
  // and 4 mu Mhat[s|d] / 64
  double kop64[KOP_N];
  float kop32[KOP_N];
  // buffers
  double *charges;      // [N][4]: x, y, z, q
  double *alpha;        // [(K+1)^3]
  double *coef;         // [nb^3] trig coefficient tensor of the field
  double *F, *G, *d;    // field, gradient [3][nn], distance
  double *E64;          // element moduli
  float *E32;           // element moduli rounded to float (mixed)
  void *Dinv;           // inverse Jacobi diagonal (float mixed / double FP64)
  // CG vectors [6][3][nn] (float mixed / double FP64).  r, p and q are double
  // buffered: a CG pass reads set pcur[k] of load case k and writes the other
  void *r[2], *p[2], *q[2], *x;
  // multigrid, voxel level: the pre-smoother's second Chebyshev direction
  // [6][3][nn] (the only one stored) and the coefficients 1 / theta, c1, c2
  void *mgd;
  double mgc[3];
  double *x64;          // FP64 solution accumulator (mixed); == x for FP64
  double *partials;     // [NRHS][maxparts][PSTRIDE]
  CgState *st;
};

// A launch segment: `nblocks` consecutive logical workgroups for one slot.
// Logical block L in [first, first + nblocks) maps to
//   local = L - first, case index = local % nrhs, tile = local / nrhs.
struct Segment {
  SlotDev *slot;
  int first;
  int nblocks;
  int nrhs;             // load cases in this segment (6, or 1 for per-slot kernels)
  int rhs[NRHS];        // which load cases
  int flag;             // kernel-specific (e.g. recompute mode)
  int pad_;
};

// Fused voxel-level passes of the multigrid-preconditioned CG (stencil kernel)
enum { SMG_DIR = 0, SMG_STEP1 = 1, SMG_POST = 2, SMG_LAST = 3, SMG_RES = 4, SMG_POST1 = 5 };
// Chebyshev degree of the voxel level's smoother (1 or 2; the coarse levels
// take 2).  Dense multigrid (SHH_MG_DEG0): degree 1 costs about 1 % more CG
// iterations at 128^3 and saves two of the five voxel-level operator passes
// of an iteration (20 % faster).  Selective solve (SHH_SEL_DEG0): degree 2,
// since with degree 1 the FP32 culled solve of some designs stalls above the
// tolerance (FP64 converges).  The other degree is a build option.
#ifndef SHH_MG_DEG0
#define SHH_MG_DEG0 1
#endif
#ifndef SHH_SEL_DEG0
#define SHH_SEL_DEG0 2
#endif

struct LaunchArgs {
  const Segment *segs;
  int nseg;
  int total;            // logical workgroups (before padding to a multiple of 8)
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Give each XCD a contiguous run of logical workgroups so that
// neighbouring tiles (shared halos) and the six load cases of one tile (shared
// moduli) meet in the same L2.
__device__ __forceinline__ int logical_block(int b, int grid) {
  const int per = grid >> 3;  // grid is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

struct Work {
  SlotDev *slot;
  int rhs;
  int tile;
  int flag;
  int seg;
};

// Segments, slot descriptors and (within one kernel) the CG scalars are never
// written while a kernel reads them: reading them through the constant address
// space lets the compiler use scalar loads and keep them in scalar registers.
#define SHH_CONST __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const SHH_CONST T *to_const(const T *p) {
  return (const SHH_CONST T *)p;
}

__device__ __forceinline__ bool decode_work(const LaunchArgs &a, Work &w) {
  const int L = logical_block(blockIdx.x, gridDim.x);
  if (L >= a.total) return false;
  const SHH_CONST Segment *segs = to_const(a.segs);
  int lo = 0, hi = a.nseg - 1;
  while (lo < hi) {  // last segment with first <= L
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= L) lo = mid; else hi = mid - 1;
  }
  const SHH_CONST Segment &s = segs[lo];
  const int local = L - s.first;
  if (local >= s.nblocks) return false;
  w.slot = s.slot;
  w.rhs = s.rhs[local % s.nrhs];
  w.tile = local / s.nrhs;
  w.flag = s.flag;
  w.seg = lo;
  return true;
}

// ---- deterministic block reductions in FP64 ----
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red, int nthreads) {
  // red: shared scratch of NV * 16 doubles
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (nthreads + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * 16 + wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[i * 16 + w];
      v[i] = s;
    }
  }
}

// Publish a workgroup partial and find out whether this workgroup is the last
// of `total` to arrive; the last one then sees every partial.  Thread 0 must
// have stored this workgroup's partials before the call.
__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned total, int *flag_smem) {
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    *flag_smem = (prev == total - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *flag_smem != 0;
  if (last) __threadfence();
  return last;
}

// Sum `count` partials of NV values each (stride 4 doubles) in a fixed order:
// thread t adds partials t, t + nthreads, ...; then a fixed-tree block sum.
template <int NV, int STRIDE = 4>
__device__ __forceinline__ void sum_partials(const double *parts, int count, double (&out)[NV],
                                             double *red, int nthreads) {
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = 0.0;
  for (int k = threadIdx.x; k < count; k += nthreads) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] += parts[STRIDE * k + i];
  }
  block_sum<NV>(out, red, nthreads);
}

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Periodic wrap of an index known to lie in [-n, 2n).
__device__ __forceinline__ int wrap1(int v, int n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// ---- global-memory access ----
// Slot buffers are reached through pointers stored in device memory, which the
// compiler would otherwise treat as generic (FLAT) addresses.  FLAT loads count
// against the LDS wait counter as well, so every LDS wait would also wait for
// the prefetched HBM loads.  The hot kernels therefore address global memory
// through address-space-1 pointers held in scalar registers, with 32-bit byte
// offsets (the "saddr + voffset" form of global_load / global_store).
#define SHH_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ SHH_GLOBAL T *to_global(T *p) {
  // the pointer is the same for every lane: keep it in scalar registers
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (SHH_GLOBAL T *)(((uint64_t)hi << 32) | lo);
}

// ---- buffer access (the streaming arrays of the stencil and CG kernels) ----
// A buffer resource holds the base address and byte size of one array in
// scalar registers; each access adds a per-lane 32-bit byte offset (fixed per
// thread: its place in the tile or chunk) and a wave-uniform scalar offset
// (plane and component), so the hot loops do no per-lane address arithmetic.
// Every array covered by one resource is below 4 GiB (n <= 512).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;  // gfx9: 32-bit data format, raw access

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)(uint32_t)bytes,
                                           RSRC_WORD3);
}

template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t voff, uint32_t soff) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit elements");
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Cache policy of the streaming stores (CPol bits: 2 = non-temporal on gfx950):
// the CG vectors written by one pass are read back only by the next, long
// after they would have left the L2, so they are streamed past it.
#ifndef SHH_STORE_AUX
#define SHH_STORE_AUX 2
#endif

template <typename T>
__device__ __forceinline__ void bstore(T v, rsrc_t r, uint32_t voff, uint32_t soff) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit elements");
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, SHH_STORE_AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(uint32_t __attribute__((ext_vector_type(2))), v), r, voff, soff, SHH_STORE_AUX);
}

template <typename T>
__device__ __forceinline__ T gld(const SHH_GLOBAL T *base, uint32_t byte_off) {
  return *(const SHH_GLOBAL T *)((const SHH_GLOBAL char *)base + byte_off);
}

template <typename T>
__device__ __forceinline__ void gst(SHH_GLOBAL T *base, uint32_t byte_off, T v) {
  *(SHH_GLOBAL T *)((SHH_GLOBAL char *)base + byte_off) = v;
}

}  // namespace shh
