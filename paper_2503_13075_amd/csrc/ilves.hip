// Device kernels and the C ABI of the constraint solver (gfx950 / CDNA4).
//
// Method (Supplement section 2.3 and 3 of the ILVES paper, with lambda
// entering as r' = r_u - M^{-1} G(r)^T lambda, see include/ilves.h):
//   r'(lambda) = r_u - M^{-1} G(r)^T lambda                     (Eq. 6)
//   Newton: A(r', r) z = g(r'), lambda += z, A = G(r') M^{-1} G(r)^T (Eq. defA)
//   chord:  the same with the constant A(r, r)                   (ILVES-F)
//   stop when max |g_k| / d_k^2 <= tol                            (Supplement section 4)
//
// GPU design.  One workgroup solves one molecule; the whole Newton loop runs
// inside the kernel.  The iteration works in constraint space: with e_k the
// old bond vector and u_k the unconstrained one, the current bond vector is
//   e'_k = u_k - sum_j C_kj lambda_j e_j,
//   C_kk = 1/m_a + 1/m_b,  C_kj = s_kx s_jx / m_x  (x the shared atom),
// which is the position map of Eq. 6 taken along constraint k, so no atom
// positions are formed until the end.  The Newton matrix has the same
// pattern: A_kj = C_kj (e'_k . e_j).
//
// The LU is an up-looking factorisation scheduled by elimination level:
// rows are numbered level by level, and the entries owned by the rows of one
// level (their diagonal and upper entries, plus the transposed lower ones)
// are independent.  A diagonal entry gathers over its row's lower pattern
// (and performs the forward substitution for its row at the same time) and
// stores 1/U_jj in place of A_jj; an upper entry (j, m) and its transpose
// (m, j) run over the planned list of rows coupled to both.  The backward
// substitution walks the levels down.  Everything one level needs -- the
// slot structure (column, transpose link, update lists) and the factor
// values -- is kept in LDS when it fits, so a level costs a few dependent
// LDS accesses plus one barrier; data used once per iteration (old and
// unconstrained bond vectors, couplings, lambda) stays in a per-molecule
// workspace in global memory, where it is L2 resident.  No atomics: every value has one writer, so results are bitwise
// reproducible.
//
// Precision: FP64 throughout, or mixed (matrix, factor and triangular solves
// in FP32 while e', g, lambda and positions stay FP64), which makes Newton
// an iterative refinement that still reaches FP64 accuracy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ilves.h"
#include "device_plan.hpp"
#include "inputs.hpp"
#include "md.hpp"
#include "plan.hpp"
#include "warmstart.hpp"

using namespace ilves_dev;

namespace {

thread_local std::string g_last_error;

ilves_status_t fail(ilves_status_t s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ILVES_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

// ---------------------------------------------------------------------------
// device plan layout: see device_plan.hpp

struct SolveArgs {
  const double* r;
  const double* r_u;
  const double* mass;
  double* r_out;
  double* lambda;
  int32_t* iters;
  int32_t* status;
  int32_t* fallback;  // per molecule (learned warm start), may be null
  unsigned char* ws;
  double tol;
  int32_t n_atoms;
  int32_t max_iter;
  int32_t warm;      // 0: lambda_0 = 0, 1: read lambda, 2: read the network's lambda (with fallback),
                     // 3: each constraint's decoupled solution (with fallback)
  int32_t chord;     // 0: Newton, 1: chord
  int32_t wait_limit;  // polls of a split molecule's barrier wait before it gives up
  int32_t project;   // 1: velocity projection (r_u holds velocities, residual e_k . p_k, chord)
  double* hist;      // per molecule [hist_len]: max relative violation before each linear solve, may be null
  int32_t hist_len;
};

// FP64 workspace of a molecule: per row {e, lambda} (4n), {u, C_kk} (4n) and
// {1/m_a, 1/m_b} (2n), 1/m per atom (s + 1)
__host__ __device__ inline size_t ws_vec_bytes(int32_t n, int32_t s, int32_t, int32_t) {
  return align16(8 * (10 * static_cast<size_t>(n) + s + 1));
}
// factor values: F (off-diagonal slots), D (diagonal, then 1/U_jj), y
template <typename T>
__host__ __device__ inline size_t value_bytes(int32_t n, int32_t n_up, int32_t n_l) {
  return align16(sizeof(T) * (static_cast<size_t>(n_up) + n_l + 2 * static_cast<size_t>(n)));
}

// packed structure records: 2 or 4 indices in one LDS/global access
__device__ inline void ld2(const uint16_t* p, int32_t& a, int32_t& b) {
  const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
  a = static_cast<int32_t>(v & 0xffffu);
  b = static_cast<int32_t>(v >> 16);
}
__device__ inline void ld2(const int32_t* p, int32_t& a, int32_t& b) {
  const int2 v = *reinterpret_cast<const int2*>(p);
  a = v.x;
  b = v.y;
}
__device__ inline void ld4(const uint16_t* p, int32_t& a, int32_t& b, int32_t& c, int32_t& d) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  a = static_cast<int32_t>(v.x & 0xffffu);
  b = static_cast<int32_t>(v.x >> 16);
  c = static_cast<int32_t>(v.y & 0xffffu);
  d = static_cast<int32_t>(v.y >> 16);
}
__device__ inline void ld4(const int32_t* p, int32_t& a, int32_t& b, int32_t& c, int32_t& d) {
  const int4 v = *reinterpret_cast<const int4*>(p);
  a = v.x;
  b = v.y;
  c = v.z;
  d = v.w;
}

// Values that are the same in every lane (read from LDS or from a
// wave-uniform address) made explicit to the compiler: they move to scalar
// registers, so indexing, loop bounds and branches on them run on the scalar
// unit and free vector registers (occupancy).
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = static_cast<uint64_t>(v);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int32_t>(u)));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int32_t>(u >> 32)));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ double uni(double v) {
  return __longlong_as_double(static_cast<long long>(uni(static_cast<int64_t>(__double_as_longlong(v)))));
}
__device__ __forceinline__ MolDesc uni(const MolDesc& m) {
  MolDesc r;
  r.n = uni(m.n);
  r.s = uni(m.s);
  r.n_up = uni(m.n_up);
  r.n_l = uni(m.n_l);
  r.n_upd = uni(m.n_upd);
  r.n_levels = uni(m.n_levels);
  r.n_pl = uni(m.n_pl);
  r.wide = uni(m.wide);
  r.ix_off = uni(m.ix_off);
  r.coef_off = uni(m.coef_off);
  r.row_off = uni(m.row_off);
  r.atom_off = uni(m.atom_off);
  r.incp_off = uni(m.incp_off);
  r.inc_off = uni(m.inc_off);
  r.ws_off = uni(m.ws_off);
  return r;
}

__device__ __forceinline__ SplitPart uni(const SplitPart& p) {
  SplitPart r;
  r.desc = uni(p.desc);
  r.report = uni(p.report);
  r.part = uni(p.part);
  r.n_parts = uni(p.n_parts);
  r.n_int = uni(p.n_int);
  r.h_int = uni(p.h_int);
  r.s_own = uni(p.s_own);
  r.m = uni(p.m);
  r.bsep_off = uni(p.bsep_off);
  r.ext_off = uni(p.ext_off);
  r.sep_off = uni(p.sep_off);
  r.ew_off = uni(p.ew_off);
  r.xch = uni(p.xch);
  r.lds_extra[0] = uni(p.lds_extra[0]);
  r.lds_extra[1] = uni(p.lds_extra[1]);
  r.ew_total = uni(p.ew_total);
  r.n_sadj = uni(p.n_sadj);
  r.bw = uni(p.bw);
  r.pad = 0;
  return r;
}

// Data one workgroup of a split molecule writes and another reads (the
// exchange area, lambdas of rows coupled across parts) is read with
// device-coherent loads, which fetch past the caches of the reading
// compute unit and XCD; everything a part reads only of its own stays
// cacheable (no cache invalidation at the barriers).
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_coh(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier of the workgroups of one split molecule (all resident: the
// launch never holds more of them than fit on the device at once).  Every
// wave first writes its global data back device-wide (release); one lane
// per workgroup arrives on the counter, the last arrival resets it and
// advances the generation, the others wait for the generation to change.
// Readers use ld_coh for data written by other workgroups, so no acquire
// invalidation is needed.  The wait is bounded: after wait_limit polls
// (2^22 by default, seconds) the workgroup marks the molecule poisoned,
// which also releases every other waiter, and reports false.
__device__ bool grid_barrier(uint32_t* bar, int32_t n_parts, int32_t wait_limit, int32_t* flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t good = __hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    if (good) {
      const uint32_t g = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);  // the generation is read before arriving
      const uint32_t a = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (a == static_cast<uint32_t>(n_parts - 1)) {
        __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        for (int32_t i = 0; __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g; ++i) {
          if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            good = 0;
            break;
          }
          if (i >= wait_limit) {
            __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            good = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    *flag = good;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*flag) != 0;
}

// per-row record of the workspace: old bond vector and lambda, read with
// two 16-byte loads
struct Rec {
  double x, y, z, l;
};
__device__ __forceinline__ Rec ld_rec(const double* p) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  return Rec{a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ void st_rec(double* p, double x, double y, double z, double l) {
  *reinterpret_cast<double2*>(p) = make_double2(x, y);
  *reinterpret_cast<double2*>(p + 2) = make_double2(z, l);
}
// entries gathered per batch: row neighbours (global memory, FP64),
// lower / upper entries of the factor, factor updates.  kBatchNWide
// neighbours per batch for launches whose workgroups need more than half
// of a CU's LDS, and for the parts of split molecules whose structure is
// read from global memory: one of them runs per CU whatever its registers,
// so the wider batch (more loads in flight, more registers) costs no
// occupancy.
constexpr int kBatchN = 2;
constexpr int kBatchNWide = 4;
constexpr int kBatch = 2;
constexpr int kBatchU = 1;

// 1/a from the hardware reciprocal refined by Newton steps (one in FP32,
// two in FP64): a few dependent operations instead of a full division; the
// result is within an ulp or two, which the factorisation does not notice
// (Newton on the constraints converges the same with a slightly perturbed
// Jacobian).
__device__ __forceinline__ float recip(float a) {
  const float r = __builtin_amdgcn_rcpf(a);
  return __builtin_fmaf(__builtin_fmaf(-a, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
  return __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
}

// Decoupled start: the multiplier of constraint k taken alone, the root
// nearest 0 of |u - lambda cd e|^2 = d^2, i.e. a l^2 + b l + c = 0 with
// a = cd^2 |e|^2, b = -2 cd (u . e), c = |u|^2 - d^2, in the cancellation-free
// form c / q, q = (-b + sqrt(b^2 - 4ac)) / 2; without a real root (or with
// u . e <= 0) the Newton step from 0, -c / b (0 if b = 0).
__device__ inline double decoupled_lambda(double u0, double u1, double u2, double e0, double e1, double e2,
                                          double cd, double d2) {
  const double c = u0 * u0 + u1 * u1 + u2 * u2 - d2;
  const double b = -2.0 * cd * (u0 * e0 + u1 * e1 + u2 * e2);
  const double a = cd * cd * (e0 * e0 + e1 * e1 + e2 * e2);
  const double disc = b * b - 4.0 * a * c;
  if (b < 0.0 && disc >= 0.0) return c / (0.5 * (-b + sqrt(disc)));
  return b != 0.0 ? -c / b : 0.0;
}

// C_kj of a slot of row k from its coupling code (see kFillCode) and the
// inverse masses of k's atoms
__device__ __forceinline__ double coupling(uint32_t code, double ima, double imb) {
  const double v = (code & 2u) ? imb : ima;
  return (code & kFillCode) ? 0.0 : ((code & 1u) ? -v : v);
}

// integer min by value (no reference to a temporary, which would keep
// small arrays out of registers)
__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

template <typename T> __device__ inline T pivot_eps();
template <> __device__ inline double pivot_eps<double>() { return 1e-13; }
template <> __device__ inline float pivot_eps<float>() { return 1e-6f; }

// ---------------------------------------------------------------------------
// the solve kernel: one workgroup per molecule

//
// SPLIT: one workgroup per part of a molecule split across workgroups
// (block-bordered LU).  A part holds its interior rows and its border rows
// (the separator rows touching its atoms), ordered so that the border rows
// come last in levels of their own.  Per Newton iteration every part forms
// its residuals (a border row also gathers the coupled rows that other parts
// hold), factors its rows with the forward substitution fused, and takes
// from the border block of its factors the Schur contribution
//   E_i = L_BB U_BB - A_BB = -A_BI A_II^-1 A_IB
// and the reduced right-hand side contribution w_i = g_B - L_BB y_B =
// A_BI A_II^-1 g_I.  After a barrier every workgroup reads all parts'
// violations (the same convergence decision everywhere), assembles the
// dense separator system (A_SS + sum E_i) z_S = g_S - sum w_i from the
// published border data in the same order, and solves it; each part then
// sets its border unknowns to z_S, substitutes backward through its interior
// levels and updates lambda; a second barrier publishes the new lambdas.
template <typename T, typename Idx, int MODE, int BLOCK, bool SPLIT = false, int NB = kBatchN>
__global__ void __launch_bounds__(BLOCK) solve_kernel(const DevPlan P, const int32_t* __restrict__ mols,
                                                      const int32_t count, int32_t* __restrict__ counter,
                                                      const SolveArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  // factor entries / updates per batch: wider where the structure is read
  // from global memory, so that several of its records are in flight
  constexpr bool kStructGlobal = MODE == VALUES_LDS || MODE == GLOBAL;
  constexpr int KB = kStructGlobal ? 4 : kBatch;
  constexpr int KU = (kStructGlobal || MODE == PAIRS_GLOBAL) ? 8 : kBatchU;
  __shared__ double red[BLOCK / 64];
  __shared__ double red0[BLOCK / 64];
  __shared__ int32_t singular;
  __shared__ int32_t next_slot;

  const int tid = threadIdx.x;
  // persistent workgroup: take molecules (largest first) from the queue
  // until it is empty; every wave of the workgroup leaves together
  for (;;) {
  int32_t slot;
  if constexpr (SPLIT) {
    slot = uni(mols[blockIdx.x]);  // the launch's parts
  } else {
    if (tid == 0) next_slot = atomicAdd(counter, 1);
    __syncthreads();
    slot = uni(next_slot);
    if (slot >= count) break;
  }
  SplitPart sp{};
  if constexpr (SPLIT) sp = uni(P.split[slot]);
  const int32_t m_idx = SPLIT ? sp.desc : uni(mols[slot]);
  const int32_t report = SPLIT ? sp.report : m_idx;
  const MolDesc md = uni(P.mol[m_idx]);
  const int32_t n = md.n, s = md.s, n_up = md.n_up, n_l = md.n_l, n_upd = md.n_upd, H = md.n_levels;
  const int32_t n_pl = md.n_pl;
  const int32_t S = A.n_atoms;

  // ---- structure (LDS copy unless GLOBAL)
  const Layout Lo = struct_layout(n, H, n_up, n_l, n_pl, n_upd, static_cast<int>(sizeof(Idx)));
  const unsigned char* gst = P.ix + md.ix_off;
  const unsigned char* st;
  // bytes of the structure block held in LDS (PAIRS_GLOBAL: up to the pair
  // tasks, rounded up to whole 16-byte copies)
  const int64_t st_lds = MODE == PAIRS_GLOBAL ? align_to(Lo.prec, 16) : Lo.total;
  if (MODE == GLOBAL || MODE == VALUES_LDS) {
    st = gst;
  } else {
    const int64_t nvec = st_lds / 16;  // blocks are 16-byte aligned and padded
    const int4* gv = reinterpret_cast<const int4*>(gst);
    int4* lv = reinterpret_cast<int4*>(smem);
    // four 16-byte loads in flight per lane before their stores
    int64_t i = tid;
    for (; i + 3 * BLOCK < nvec; i += 4 * BLOCK) {
      const int4 v0 = gv[i], v1 = gv[i + BLOCK], v2 = gv[i + 2 * BLOCK], v3 = gv[i + 3 * BLOCK];
      lv[i] = v0;
      lv[i + BLOCK] = v1;
      lv[i + 2 * BLOCK] = v2;
      lv[i + 3 * BLOCK] = v3;
    }
    for (; i < nvec; i += BLOCK) lv[i] = gv[i];
    st = smem;
  }
  const Idx* __restrict__ up_start = reinterpret_cast<const Idx*>(st + Lo.up_start);
  const Idx* __restrict__ l_start = reinterpret_cast<const Idx*>(st + Lo.l_start);
  const Idx* __restrict__ ucol = reinterpret_cast<const Idx*>(st + Lo.ucol);
  const Idx* __restrict__ lvh = reinterpret_cast<const Idx*>(st + Lo.lvh);
  const Idx* __restrict__ lvc = reinterpret_cast<const Idx*>(st + Lo.lvc);
  // lower-slot records are indexed by the F index t in [n_up, n_up + n_l)
  const Idx* __restrict__ lpair = reinterpret_cast<const Idx*>(st + Lo.lpair) - 2 * static_cast<int64_t>(n_up);
  const uint8_t* __restrict__ ccode = reinterpret_cast<const uint8_t*>(st + Lo.ccode);  // per slot (F index)
  const unsigned char* stp = MODE == PAIRS_GLOBAL ? gst : st;  // pair tasks and updates
  const Idx* __restrict__ prec = reinterpret_cast<const Idx*>(stp + Lo.prec);
  const Idx* __restrict__ upd = reinterpret_cast<const Idx*>(stp + Lo.upd);
  const Idx* __restrict__ updi = reinterpret_cast<const Idx*>(stp + Lo.updi);

  // ---- workspace and values
  unsigned char* wsb = A.ws + md.ws_off;
  double* __restrict__ er = reinterpret_cast<double*>(wsb);  // per row {e_x, e_y, e_z, lambda}
  double* __restrict__ uc = er + 4 * static_cast<int64_t>(n);  // per row {u_x, u_y, u_z, C_kk}
  double* __restrict__ im2 = uc + 4 * static_cast<int64_t>(n);  // per row {1/m_a, 1/m_b}
  double* __restrict__ invm = im2 + 2 * static_cast<int64_t>(n);
  T* __restrict__ F;
  if (MODE == ALL_LDS) F = reinterpret_cast<T*>(smem + Lo.total);
  else if (MODE == PAIRS_GLOBAL) F = reinterpret_cast<T*>(smem + st_lds);
  else if (MODE == VALUES_LDS) F = reinterpret_cast<T*>(smem);
  else F = reinterpret_cast<T*>(wsb + ws_vec_bytes(n, s, n_up, n_l));
  T* __restrict__ D = F + n_up + n_l;
  T* __restrict__ y = D + n;

  // split parts: exchange area of the molecule and the LDS scratch
  const int32_t ni = SPLIT ? sp.n_int : n;  // interior rows
  const int32_t nb = n - ni;                // border rows
  const int32_t ms = SPLIT ? sp.m : 0;      // separator rows
  unsigned char* xb = A.ws + (SPLIT ? sp.xch : 0);
  uint32_t* bar = reinterpret_cast<uint32_t*>(xb);
  PartX* pxa = reinterpret_cast<PartX*>(xb + 64);
  SepX* sxa = reinterpret_cast<SepX*>(xb + xch_sepx(SPLIT ? sp.n_parts : 0));
  double* xd = reinterpret_cast<double*>(xb);
  double* ew = xd + (SPLIT ? sp.ew_off : 0);  // this part's E (nb x nb), then w (nb)
  double* Sm = reinterpret_cast<double*>(smem + (SPLIT ? sp.lds_extra[sizeof(T) == 4 ? 1 : 0] : 0));  // [ms][ms + 1]
  double* zs = Sm + ms * (ms + 1);
  double* gB = zs + ms;
  double* Ab = gB + nb;
  double* Lb = Ab + nb * nb;
  double* Ub = Lb + nb * nb;
  double* amax = Ub + nb * nb;  // row maxima of the separator matrix, then 1/pivot per row
  double* xs = amax + ms;       // copy of SepX[ms] (8 doubles each) then the E/w blocks
  const int32_t ew_total = SPLIT ? sp.ew_total : 0;
  SepRow* srow = reinterpret_cast<SepRow*>(xs + 8 * ms + ew_total);
  int32_t* sadj_l = reinterpret_cast<int32_t*>(srow + ms);
  const int32_t ew_base = static_cast<int32_t>(xch_ew(SPLIT ? sp.n_parts : 0, ms) / 8);

  const int32_t* __restrict__ atom_gid = P.atom_gid + md.atom_off;
  const int32_t* __restrict__ cid = P.cid + md.row_off;
  const double* __restrict__ d2 = P.d2 + md.row_off;
  const double* __restrict__ rx = A.r;
  const double* __restrict__ ux = A.r_u;

  // ---- set-up: 1/m, old and unconstrained bond vectors, lambda_0, the
  //      inverse masses of each row's atoms (the slot couplings C_kj are
  //      taken from them and the slot's code), coordinate magnitude
  // (the loops read input atom indices prepared with the plan, so each
  // entry takes one round of gathers)
  double rmax = 0.0;
  // atoms four per lane at a time (index, then mass and position gathers
  // in flight together)
  for (int32_t a0 = tid; a0 < s; a0 += 4 * BLOCK) {
    int32_t g[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = atom_gid[imin(a0 + i * BLOCK, s - 1)];
    double m[4], x[4], yv[4], z[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      m[i] = A.mass[g[i]];
      x[i] = ux[g[i]];
      yv[i] = ux[S + g[i]];
      z[i] = ux[2 * S + g[i]];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (a0 + i * BLOCK < s) {
        invm[a0 + i * BLOCK] = 1.0 / m[i];
        rmax = fmax(rmax, fmax(fabs(x[i]), fmax(fabs(yv[i]), fabs(z[i]))));
      }
    }
  }
  if (tid == 0) {
    invm[s] = 0.0;  // fill entries point here: zero coupling
    singular = 0;
  }
  const int32_t* __restrict__ rga = P.ga + md.row_off;
  const int32_t* __restrict__ rgb = P.gb + md.row_off;
  double v0 = 0.0;  // max relative violation at lambda = 0 (learned start fallback test)
  // rows RS per lane at a time (kernels of workgroups alone on their CU,
  // whose registers cost no occupancy): the gathers of all of them in flight
  // together
  constexpr int RS = NB == kBatchNWide ? 2 : 1;
  for (int32_t k0 = tid; k0 < n; k0 += RS * BLOCK) {
    int32_t ga[RS], gb[RS];
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int32_t k = imin(k0 + i * BLOCK, n - 1);
      ga[i] = rga[k];
      gb[i] = rgb[k];
    }
    double ua[RS][3], ub[RS][3], ra_[RS][3], rb_[RS][3], ma[RS], mb[RS];
#pragma unroll
    for (int i = 0; i < RS; ++i) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ua[i][c] = ux[c * S + ga[i]];
        ub[i][c] = ux[c * S + gb[i]];
        ra_[i][c] = rx[c * S + ga[i]];
        rb_[i][c] = rx[c * S + gb[i]];
      }
      ma[i] = A.mass[ga[i]];
      mb[i] = A.mass[gb[i]];
    }
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int32_t k = k0 + i * BLOCK;
      if (k >= n) break;
      const double a0 = ua[i][0] - ub[i][0], a1 = ua[i][1] - ub[i][1], a2 = ua[i][2] - ub[i][2];
      const double e0 = ra_[i][0] - rb_[i][0], e1 = ra_[i][1] - rb_[i][1], e2 = ra_[i][2] - rb_[i][2];
      const double ima = 1.0 / ma[i], imb = 1.0 / mb[i];
      const double cdk = ima + imb;
      const double lam0 = A.warm == 3 ? decoupled_lambda(a0, a1, a2, e0, e1, e2, cdk, d2[k])
                                      : (A.warm ? A.lambda[cid[k]] : 0.0);
      st_rec(er + 4 * k, e0, e1, e2, lam0);
      if constexpr (SPLIT) {
        if (k >= ni) {
          const int32_t v = P.bsep[sp.bsep_off + (k - ni)];
          if (v >> 30) {
            SepX& X = sxa[v & 0x3fffffff];
            X.e[0] = e0;
            X.e[1] = e1;
            X.e[2] = e2;
          }
        }
      }
      st_rec(uc + 4 * k, a0, a1, a2, cdk);
      *reinterpret_cast<double2*>(im2 + 2 * k) = make_double2(ima, imb);
      v0 = fmax(v0, fabs(a0 * a0 + a1 * a1 + a2 * a2 - d2[k]) / (2.0 * d2[k]));
    }
  }
  int32_t adj0 = 0;  // first separator coupling of the molecule
  if constexpr (SPLIT) {
    // separator rows and couplings of the molecule into LDS (plan data)
    const int32_t* src = reinterpret_cast<const int32_t*>(P.sep + sp.sep_off);
    int32_t* dst = reinterpret_cast<int32_t*>(srow);
    constexpr int kw = static_cast<int>(sizeof(SepRow) / 4);
    for (int32_t i = tid; i < ms * kw; i += BLOCK) dst[i] = src[i];
    adj0 = uni(P.sep[sp.sep_off].adj_off);
    for (int32_t i = tid; i < 2 * sp.n_sadj; i += BLOCK) sadj_l[i] = P.sadj[2 * adj0 + i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
    v0 = fmax(v0, __shfl_xor(v0, off, 64));
  }
  if ((tid & 63) == 0) {
    red[tid >> 6] = rmax;
    red0[tid >> 6] = v0;
  }
  __syncthreads();
  // Rounding r' to doubles moves each output coordinate by at most
  // |r'| 2^-53, so a bond vector formed from the returned positions differs
  // from the one iterated here by at most delta = sqrt(3) rmax 2^-52.  The
  // convergence test adds the resulting bound on |g| so that the returned
  // positions themselves satisfy the tolerance.
  double gr = red[0], rel_zero = red0[0];
#pragma unroll
  for (int w = 1; w < BLOCK / 64; ++w) {
    gr = fmax(gr, red[w]);
    rel_zero = fmax(rel_zero, red0[w]);
  }
  gr = uni(gr);
  rel_zero = uni(rel_zero);
  const double delta = 1.7320508075688772 * gr * 0x1.0p-52;
  const double delta2 = 0.5 * delta * delta;
  __syncthreads();

  const int32_t level1 = uni(static_cast<int32_t>(lvh[1]));  // end row of level 0
  // diagonal of row k from the bond-vector product: level-0 rows have no
  // lower entries, so their factorisation is just the inverted pivot
  auto set_diag = [&](int32_t k, T akk) {
    if (k < level1) {
      if (!(fabs(akk) > T(0))) singular = 1;
      D[k] = recip(akk);
    } else {
      D[k] = akk;
    }
  };
  // the off-diagonal slots of a row, upper ones then lower ones: entry idx
  // -> slot and column
  auto slot_of = [&](int32_t idx, int32_t q0, int32_t nq, int32_t t0, int32_t& sl, int32_t& j) {
    if (idx < nq) {
      sl = q0 + idx;
      j = ucol[sl];
    } else {
      sl = t0 + (idx - nq);
      j = lpair[2 * sl];
    }
  };
  // row k of A(x, r), x having bond vector (px, py, pz).  Entries are taken
  // NB at a time (indices clamped to the last entry, extra lanes of a
  // batch discarded) so that their loads are issued together.
  auto build_row = [&](int32_t k, double px, double py, double pz) {
    const Rec ek = ld_rec(er + 4 * k);
    const double2 mk = *reinterpret_cast<const double2*>(im2 + 2 * k);
    set_diag(k, static_cast<T>(uc[4 * k + 3] * (px * ek.x + py * ek.y + pz * ek.z)));
    const int32_t q0 = up_start[k], nq = up_start[k + 1] - q0;
    const int32_t t0 = l_start[k], tot = nq + (l_start[k + 1] - t0);
    for (int32_t b = 0; b < tot; b += NB) {
      int32_t sb[NB];
      Rec nb[NB];
      double cb[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        int32_t j;
        slot_of(imin(b + i, tot - 1), q0, nq, t0, sb[i], j);
        nb[i] = ld_rec(er + 4 * j);
        cb[i] = coupling(ccode[sb[i]], mk.x, mk.y);
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (b + i < tot) F[sb[i]] = static_cast<T>(cb[i] * (px * nb[i].x + py * nb[i].y + pz * nb[i].z));
    }
  };

  // one elimination level: diagonal entries (forward substitution fused
  // when FORWARD) and, when FACTOR, the upper entries with updates.  A lane
  // takes every G-th entry of its item, KB (updates KU) at a time, indices
  // clamped to the last entry and the extra lanes of a batch discarded, so
  // that the loads of a batch are issued together; the G lanes of an item
  // then add their partial sums.
  auto factor_level = [&](int32_t h, auto factor_tag, auto forward_tag) {
    constexpr bool FACTOR = decltype(factor_tag)::value;
    constexpr bool FORWARD = decltype(forward_tag)::value;
    int32_t r0, r1, p0, p1;
    ld4(lvh + 4 * h, r0, r1, p0, p1);
    r0 = uni(r0);
    r1 = uni(r1);
    p0 = uni(p0);
    p1 = uni(p1);
    const int32_t nr = r1 - r0;
    const int32_t np = FACTOR ? p1 - p0 : 0;
    const int32_t lg = uni(static_cast<int32_t>(lvc[2 * h]));
    // the row items are padded to a whole number of waves, so that no wave
    // holds both kinds of item: a wave with rows and pair tasks would run the
    // two code paths one after the other
    if (!SPLIT || lg == 0) {  // one lane per item (whole molecules: always)
      const int32_t nrp = FACTOR ? (nr + 63) & ~63 : nr;
      const int32_t items = nrp + np;
      for (int32_t idx = tid; idx < items; idx += BLOCK) {
        if (idx < nrp) {
          if (idx >= nr) continue;
          const int32_t j = r0 + idx;
          T acc = D[j], yj = y[j];
          const T a0 = acc;
          const int32_t t0 = l_start[j], nt = l_start[j + 1] - t0;
          for (int32_t b = 0; b < nt; b += KB) {
            int32_t ii[KB], ss[KB];
            T f[KB], di[KB], fs[KB], yi[KB];
#pragma unroll
            for (int i = 0; i < KB; ++i) ld2(lpair + 2 * (t0 + imin(b + i, nt - 1)), ii[i], ss[i]);
#pragma unroll
            for (int i = 0; i < KB; ++i) {
              f[i] = F[t0 + imin(b + i, nt - 1)];
              di[i] = D[ii[i]];
              if (FACTOR) fs[i] = F[ss[i]];
              if (FORWARD) yi[i] = y[ii[i]];
            }
#pragma unroll
            for (int i = 0; i < KB; ++i) {
              if (b + i < nt) {
                const T l = f[i] * di[i];
                if (FACTOR) acc -= l * fs[i];
                if (FORWARD) yj -= l * yi[i];
              }
            }
          }
          if (FACTOR) {
            if (!(fabs(acc) > pivot_eps<T>() * fabs(a0))) singular = 1;
            D[j] = recip(acc);
          }
          if (FORWARD) y[j] = yj;
        } else if (FACTOR) {
          int32_t q, tr, u0, nu;
          ld4(prec + 4 * (p0 + idx - nrp), q, tr, u0, nu);
          T au = F[q], aw = F[tr];
          for (int32_t b = 0; b < nu; b += KU) {
            int32_t pa[KU], pb[KU], s1[KU], s2[KU], ui[KU];
#pragma unroll
            for (int i = 0; i < KU; ++i) {
              const int32_t u = u0 + imin(b + i, nu - 1);
              ld4(upd + 4 * u, pa[i], pb[i], s1[i], s2[i]);
              ui[i] = updi[u];
            }
            T fa[KU], fb[KU], f1[KU], f2[KU], di[KU];
#pragma unroll
            for (int i = 0; i < KU; ++i) {
              fa[i] = F[pa[i]];
              fb[i] = F[pb[i]];
              f1[i] = F[s1[i]];
              f2[i] = F[s2[i]];
              di[i] = D[ui[i]];
            }
#pragma unroll
            for (int i = 0; i < KU; ++i) {
              if (b + i < nu) {
                au -= fa[i] * di[i] * f1[i];
                aw -= fb[i] * di[i] * f2[i];
              }
            }
          }
          F[q] = au;
          F[tr] = aw;
        }
      }
      return;
    }
    const int32_t G = 1 << lg;
    const int32_t nrl = nr << lg;
    const int32_t nrp = FACTOR ? (nrl + 63) & ~63 : nrl;
    const int32_t lanes = nrp + (np << lg);
    // whole waves per pass, so that every lane of a wave takes part in the
    // shuffles of its items
    for (int32_t base = tid & ~63; base < lanes; base += BLOCK) {
      const int32_t idx = base + (tid & 63);
      const int32_t sub = idx & (G - 1);
      if (base < nrp) {
        const bool valid = idx < nrl;
        const int32_t j = r0 + (valid ? idx >> lg : 0);
        const T a0 = D[j], y0 = y[j];  // loaded with the item's first records
        const int32_t t0 = l_start[j], nt = valid ? l_start[j + 1] - t0 : 0;
        T sf = T(0), sy = T(0);
        for (int32_t b = sub; b < nt; b += KB * G) {
          int32_t ii[KB], ss[KB];
          T f[KB], di[KB], fs[KB], yi[KB];
#pragma unroll
          for (int i = 0; i < KB; ++i) ld2(lpair + 2 * (t0 + imin(b + i * G, nt - 1)), ii[i], ss[i]);
#pragma unroll
          for (int i = 0; i < KB; ++i) {
            f[i] = F[t0 + imin(b + i * G, nt - 1)];
            di[i] = D[ii[i]];
            if (FACTOR) fs[i] = F[ss[i]];
            if (FORWARD) yi[i] = y[ii[i]];
          }
#pragma unroll
          for (int i = 0; i < KB; ++i) {
            if (b + i * G < nt) {
              const T l = f[i] * di[i];
              if (FACTOR) sf += l * fs[i];
              if (FORWARD) sy += l * yi[i];
            }
          }
        }
        for (int32_t o = G >> 1; o > 0; o >>= 1) {
          if (FACTOR) sf += __shfl_xor(sf, o, 64);
          if (FORWARD) sy += __shfl_xor(sy, o, 64);
        }
        if (valid && sub == 0) {
          if (FACTOR) {
            const T acc = a0 - sf;
            if (!(fabs(acc) > pivot_eps<T>() * fabs(a0))) singular = 1;
            D[j] = recip(acc);
          }
          if (FORWARD) y[j] = y0 - sy;
        }
      } else if (FACTOR) {
        const int32_t pl = idx - nrp;
        const bool valid = pl < (np << lg);
        int32_t q, tr, u0, nu;
        ld4(prec + 4 * (p0 + (valid ? pl >> lg : 0)), q, tr, u0, nu);
        if (!valid) nu = 0;
        const T au = F[q], aw = F[tr];
        T sa = T(0), sw = T(0);
        for (int32_t b = sub; b < nu; b += KU * G) {
          int32_t pa[KU], pb[KU], s1[KU], s2[KU], ui[KU];
#pragma unroll
          for (int i = 0; i < KU; ++i) {
            const int32_t u = u0 + imin(b + i * G, nu - 1);
            ld4(upd + 4 * u, pa[i], pb[i], s1[i], s2[i]);
            ui[i] = updi[u];
          }
          T fa[KU], fb[KU], f1[KU], f2[KU], di[KU];
#pragma unroll
          for (int i = 0; i < KU; ++i) {
            fa[i] = F[pa[i]];
            fb[i] = F[pb[i]];
            f1[i] = F[s1[i]];
            f2[i] = F[s2[i]];
            di[i] = D[ui[i]];
          }
#pragma unroll
          for (int i = 0; i < KU; ++i) {
            if (b + i * G < nu) {
              sa += fa[i] * di[i] * f1[i];
              sw += fb[i] * di[i] * f2[i];
            }
          }
        }
        for (int32_t o = G >> 1; o > 0; o >>= 1) {
          sa += __shfl_xor(sa, o, 64);
          sw += __shfl_xor(sw, o, 64);
        }
        if (valid && sub == 0) {
          F[q] = au - sa;
          F[tr] = aw - sw;
        }
      }
    }
  };
  auto factor_sweep = [&](auto factor_tag, auto forward_tag) {
    for (int32_t h = 1; h < H; ++h) {
      factor_level(h, factor_tag, forward_tag);
      __syncthreads();
    }
  };
  // backward substitution, levels h_top-1 .. 0 (G lanes per row as in the
  // factorisation, from the level's longest row of upper entries)
  auto back_sweep = [&](int32_t h_top) {
    for (int32_t h = h_top - 1; h >= 0; --h) {
      const int32_t k0 = uni(static_cast<int32_t>(lvh[4 * h])), k1 = uni(static_cast<int32_t>(lvh[4 * h + 1]));
      const int32_t nr = k1 - k0;
      const int32_t lg = uni(static_cast<int32_t>(lvc[2 * h + 1]));
      if (!SPLIT || lg == 0) {  // one lane per row (whole molecules: always)
        for (int32_t k = k0 + tid; k < k1; k += BLOCK) {
          T acc = y[k];
          const T dk = D[k];
          const int32_t q0 = up_start[k], nq = up_start[k + 1] - q0;
          for (int32_t b = 0; b < nq; b += KB) {
            int32_t c[KB];
            T f[KB], yc[KB];
#pragma unroll
            for (int i = 0; i < KB; ++i) c[i] = ucol[q0 + imin(b + i, nq - 1)];
#pragma unroll
            for (int i = 0; i < KB; ++i) {
              f[i] = F[q0 + imin(b + i, nq - 1)];
              yc[i] = y[c[i]];
            }
#pragma unroll
            for (int i = 0; i < KB; ++i)
              if (b + i < nq) acc -= f[i] * yc[i];
          }
          y[k] = acc * dk;
        }
        __syncthreads();
        continue;
      }
      const int32_t G = 1 << lg;
      const int32_t nrl = nr << lg;
      for (int32_t base = tid & ~63; base < nrl; base += BLOCK) {
        const int32_t idx = base + (tid & 63);
        const int32_t sub = idx & (G - 1);
        const bool valid = idx < nrl;
        const int32_t k = k0 + (valid ? idx >> lg : 0);
        const T yk = y[k], dk = D[k];
        const int32_t q0 = up_start[k], nq = valid ? up_start[k + 1] - q0 : 0;
        T sacc = T(0);
        for (int32_t b = sub; b < nq; b += KB * G) {
          int32_t c[KB];
          T f[KB], yc[KB];
#pragma unroll
          for (int i = 0; i < KB; ++i) c[i] = ucol[q0 + imin(b + i * G, nq - 1)];
#pragma unroll
          for (int i = 0; i < KB; ++i) {
            f[i] = F[q0 + imin(b + i * G, nq - 1)];
            yc[i] = y[c[i]];
          }
#pragma unroll
          for (int i = 0; i < KB; ++i)
            if (b + i * G < nq) sacc += f[i] * yc[i];
        }
        for (int32_t o = G >> 1; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, 64);
        if (valid && sub == 0) y[k] = (yk - sacc) * dk;
      }
      __syncthreads();
    }
  };


  // ---- split parts: border block, Schur contribution, separator system
  // border block of the matrix (rows built, not yet factored), one thread
  // per border row
  auto save_border = [&]() {
    for (int32_t i = tid; i < nb * nb; i += BLOCK) Ab[i] = 0.0;
    __syncthreads();
    for (int32_t j = tid; j < nb; j += BLOCK) {
      const int32_t k = ni + j;
      Ab[j * nb + j] = static_cast<double>(D[k]);
      for (int32_t q = up_start[k]; q < up_start[k + 1]; ++q) Ab[j * nb + (ucol[q] - ni)] = static_cast<double>(F[q]);
      for (int32_t t = l_start[k]; t < l_start[k + 1]; ++t) {
        const int32_t i = lpair[2 * t];
        if (i >= ni) Ab[j * nb + (i - ni)] = static_cast<double>(F[t]);
      }
    }
    __syncthreads();
  };
  // factors of the border block (after the factorisation) and, with schur,
  // the contribution E = L_BB U_BB - A_BB to the exchange area
  auto border_factors = [&](bool schur) {
    for (int32_t i = tid; i < nb * nb; i += BLOCK) {
      Lb[i] = 0.0;
      Ub[i] = 0.0;
    }
    __syncthreads();
    for (int32_t j = tid; j < nb; j += BLOCK) {
      const int32_t k = ni + j;
      Lb[j * nb + j] = 1.0;
      Ub[j * nb + j] = 1.0 / static_cast<double>(D[k]);
      for (int32_t q = up_start[k]; q < up_start[k + 1]; ++q) Ub[j * nb + (ucol[q] - ni)] = static_cast<double>(F[q]);
      for (int32_t t = l_start[k]; t < l_start[k + 1]; ++t) {
        const int32_t i = lpair[2 * t];
        if (i >= ni) Lb[j * nb + (i - ni)] = static_cast<double>(F[t]) * static_cast<double>(D[i]);
      }
    }
    __syncthreads();
    if (schur)
      for (int32_t i = tid; i < nb * nb; i += BLOCK) {
        const int32_t p = i / nb, q = i - p * nb;
        double acc = 0.0;
        for (int32_t t = 0; t <= (p < q ? p : q); ++t) acc += Lb[p * nb + t] * Ub[t * nb + q];
        ew[i] = acc - Ab[i];
      }
  };
  // reduced right-hand side contribution w = g_B - L_BB y_B (after the
  // forward substitution)
  auto border_rhs = [&]() {
    for (int32_t p = tid; p < nb; p += BLOCK) {
      double acc = static_cast<double>(y[ni + p]);
      for (int32_t t = 0; t < p; ++t) acc += Lb[p * nb + t] * static_cast<double>(y[ni + t]);
      ew[nb * nb + p] = gB[p] - acc;
    }
  };
  // the exchange area's SepX records and E/w blocks into LDS, one round of
  // device-coherent loads
  auto stage = [&]() {
    const double* src = reinterpret_cast<const double*>(xb + xch_sepx(sp.n_parts));
    for (int32_t i = tid; i < 8 * ms + ew_total; i += BLOCK) xs[i] = ld_coh(src + i);
    __syncthreads();
  };
  // separator matrix A_SS (at the owners' bond vectors e', or e for the
  // chord) plus the parts' contributions, into Sm[:, :ms] (from the staged
  // copies)
  auto assemble = [&](bool at_e) {
    for (int32_t i = tid; i < ms * (ms + 1); i += BLOCK) Sm[i] = 0.0;
    __syncthreads();
    for (int32_t b = tid; b < ms; b += BLOCK) {
      const SepRow& R = srow[b];
      const double* X = xs + 8 * b;  // e'[3], g, e[3]
      const double p0 = at_e ? X[4] : X[0], p1 = at_e ? X[5] : X[1], p2 = at_e ? X[6] : X[2];
      Sm[b * (ms + 1) + b] = (1.0 / A.mass[R.ga] + 1.0 / A.mass[R.gb]) * (p0 * X[4] + p1 * X[5] + p2 * X[6]);
      for (int32_t a = 0; a < R.adj_cnt; ++a) {
        const int32_t c = sadj_l[2 * (R.adj_off - adj0 + a)], cc = sadj_l[2 * (R.adj_off - adj0 + a) + 1];
        const double* Y = xs + 8 * c;
        Sm[b * (ms + 1) + c] = ((cc & 1) ? -1.0 : 1.0) / A.mass[cc >> 1] * (p0 * Y[4] + p1 * Y[5] + p2 * Y[6]);
      }
    }
    __syncthreads();
    const double* E = xs + 8 * ms - ew_base;  // indexed by doubles from the exchange area
    for (int32_t i = tid; i < ms * ms; i += BLOCK) {
      const int32_t b = i / (ms > 0 ? ms : 1), c = i - b * ms;  // (ms > 0 whenever this runs)
      const SepRow& Rb = srow[b];
      const SepRow& Rc = srow[c];
      double acc = Sm[b * (ms + 1) + c];
      for (int u = 0; u < 2; ++u) {
        const int32_t g = u ? Rb.part1 : Rb.part0, lb = u ? Rb.loc1 : Rb.loc0;
        const int32_t eo = u ? Rb.ew1 : Rb.ew0, nbg = u ? Rb.nb1 : Rb.nb0;
        for (int v = 0; v < 2; ++v)
          if ((v ? Rc.part1 : Rc.part0) == g) acc += E[eo + lb * nbg + (v ? Rc.loc1 : Rc.loc0)];
      }
      Sm[b * (ms + 1) + c] = acc;
    }
    __syncthreads();
  };
  // elimination without pivoting of the first cols columns (ms + 1: with
  // the right-hand side), inside the band of half-width bw that holds every
  // entry and its fill: wave 0 alone, lane i updating row p + 1 + i at step
  // p (LDS accesses of one wave stay in order, so no workgroup barrier per
  // step).  False when a pivot falls below 1e-13 of its row's largest entry
  // before the elimination.
  auto eliminate = [&](int32_t cols) -> bool {
    const int32_t bw = sp.bw;
    for (int32_t p = tid; p < ms; p += BLOCK) {
      double a0 = 0.0;
      for (int32_t c = 0; c < ms; ++c) a0 = fmax(a0, fabs(Sm[p * (ms + 1) + c]));
      amax[p] = a0;
    }
    __syncthreads();
    if (tid < 64) {
      // a step's entries (row r, column cc) sit at lane r * W + cc, W the
      // power of two >= bw + 1 (at most bw columns and the right-hand side)
      int32_t lw = 0;
      while ((1 << lw) < bw + 1) ++lw;
      const int32_t W = 1 << lw;
      int32_t bad = 0;
      for (int32_t p = 0; p < ms; ++p) {
        const double piv = Sm[p * (ms + 1) + p];
        if (!(fabs(piv) > 1e-13 * amax[p])) {
          bad = 1;
          break;
        }
        const double inv = recip(piv);
        if (tid == 0) amax[p] = inv;  // the row maximum is used up: keep 1/pivot for the triangular solves
        // rows p + 1 .. p + nr, columns p + 1 .. c1 (and the right-hand side
        // column): one (row, column) entry per lane; column p and row p are
        // only read in this step, so every entry has one writer
        const int32_t c1 = p + bw < ms - 1 ? p + bw : ms - 1;
        const int32_t nr = c1 - p, w = nr + (cols > ms ? 1 : 0);
        for (int32_t l = tid; l < nr * W; l += 64) {
          const int32_t r = l >> lw, cc = l & (W - 1);
          if (cc < w) {
            const int32_t q = p + 1 + r, c = cc < nr ? p + 1 + cc : ms;
            Sm[q * (ms + 1) + c] -= Sm[q * (ms + 1) + p] * inv * Sm[p * (ms + 1) + c];
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      if (tid == 0) next_slot = bad;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(next_slot) == 0;
  };
  // separator right-hand side g_S - sum_i w_i into zs (and the last column
  // of Sm for the Newton elimination)
  auto sep_rhs = [&]() {
    const double* E = xs + 8 * ms - ew_base;
    for (int32_t b = tid; b < ms; b += BLOCK) {
      const SepRow& R = srow[b];
      const double r = xs[8 * b + 3] - E[R.ew0 + R.nb0 * R.nb0 + R.loc0] - E[R.ew1 + R.nb1 * R.nb1 + R.loc1];
      zs[b] = r;
      Sm[b * (ms + 1) + ms] = r;
    }
    __syncthreads();
  };
  // triangular solves of the eliminated system inside the band: forward
  // (chord: the right-hand side was not eliminated with the matrix) by
  // wave 0, lane i updating row p + 1 + i; backward by lane 0; z in zs
  auto sep_solve = [&](bool forward) {
    const int32_t bw = sp.bw;
    if (tid < 64) {
      if (!forward)
        for (int32_t q = tid; q < ms; q += 64) zs[q] = Sm[q * (ms + 1) + ms];
      __builtin_amdgcn_wave_barrier();
      if (forward)
        for (int32_t p = 0; p < ms; ++p) {
          // rows p + 1 .. p + bw, the wave's lanes striding over them
          for (int32_t i = tid; i < bw; i += 64) {
            const int32_t q = p + 1 + i;
            if (q < ms) zs[q] -= Sm[q * (ms + 1) + p] * amax[p] * zs[p];
          }
          __builtin_amdgcn_wave_barrier();
        }
      if (tid == 0)
        for (int32_t q = ms - 1; q >= 0; --q) {
          double acc = zs[q];
          const int32_t c1 = q + bw < ms - 1 ? q + bw : ms - 1;
          for (int32_t c = q + 1; c <= c1; ++c) acc -= Sm[q * (ms + 1) + c] * zs[c];
          zs[q] = acc * amax[q];
        }
    }
    __syncthreads();
  };

  // maximum over the molecule's parts of their violation (at lambda = 0 with
  // rel0) and OR of their singular flags: the lanes of every wave read the
  // parts' records together (one round of device-coherent loads, not one per
  // part), then reduce within the wave; every wave obtains the same values
  [[maybe_unused]] auto parts_reduce = [&](bool rel0, double& vmax, int32_t& sing) {
    double v = 0.0;
    int32_t sg = 0;
    for (int32_t q = tid & 63; q < sp.n_parts; q += 64) {
      v = fmax(v, ld_coh(rel0 ? &pxa[q].rel0 : &pxa[q].viol));
      sg |= ld_coh(&pxa[q].singular);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v = fmax(v, __shfl_xor(v, off, 64));
      sg |= __shfl_xor(sg, off, 64);
    }
    vmax = v;
    sing = sg;
  };

  // ---- chord: factor A(r, r) once
  if (A.chord) {
    for (int32_t k = tid; k < n; k += BLOCK) {
      const Rec ek = ld_rec(er + 4 * k);
      build_row(k, ek.x, ek.y, ek.z);
    }
    __syncthreads();
    if constexpr (SPLIT) save_border();
    factor_sweep(std::true_type{}, std::false_type{});
    if constexpr (SPLIT) border_factors(true);
  }

  int32_t it = 0;
  int32_t st_code = ILVES_ERR_NOT_CONVERGED;
  int32_t fell_back = 0, rises = 0;
  double prev_gmax = INFINITY;
  bool chord_singular = A.chord && uni(singular);
  if constexpr (SPLIT) {
    // every part's set-up (records, owners' bond vectors, chord factors) is
    // published before anything is read across parts
    if (tid == 0) {
      pxa[sp.part].rel0 = rel_zero;
      pxa[sp.part].singular = singular;
    }
    bool stop = !grid_barrier(bar, sp.n_parts, A.wait_limit, &next_slot);
    if (stop) {
      st_code = ILVES_ERR_TIMEOUT;
    } else {
      int32_t sing = 0;
      parts_reduce(true, rel_zero, sing);
      rel_zero = uni(rel_zero);
      chord_singular = A.chord && uni(sing) != 0;
      if (A.chord && !chord_singular) {
        stage();
        assemble(true);
        chord_singular = !eliminate(ms);
      }
      if (chord_singular) st_code = ILVES_ERR_SINGULAR;
    }
    stop = stop || chord_singular;
    chord_singular = stop;
  }
  if (!SPLIT && chord_singular) st_code = ILVES_ERR_SINGULAR;
  while (!chord_singular) {
    // ---- residual at the current lambda; Newton: rebuild the matrix rows.
    //      The neighbour entries are gathered NB at a time; when a row
    //      has at most NB of them they stay in registers for the build.
    double vmax = 0.0;
    for (int32_t k = tid; k < n; k += BLOCK) {
      const Rec ek = ld_rec(er + 4 * k);
      const Rec uk = ld_rec(uc + 4 * k);
      const double2 mk = *reinterpret_cast<const double2*>(im2 + 2 * k);
      const double lk = ek.l * uk.l;
      double px = uk.x - lk * ek.x;
      double py = uk.y - lk * ek.y;
      double pz = uk.z - lk * ek.z;
      const int32_t q0 = up_start[k], nq = up_start[k + 1] - q0;
      const int32_t t0 = l_start[k], tot = nq + (l_start[k + 1] - t0);
      int32_t sb[NB];
      Rec nb[NB];
      double cb[NB];
      for (int32_t b = 0; b < tot; b += NB) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          int32_t j;
          slot_of(imin(b + i, tot - 1), q0, nq, t0, sb[i], j);
          nb[i] = ld_rec(er + 4 * j);
          cb[i] = coupling(ccode[sb[i]], mk.x, mk.y);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          if (b + i < tot) {
            const double c = cb[i] * nb[i].l;
            px -= c * nb[i].x;
            py -= c * nb[i].y;
            pz -= c * nb[i].z;
          }
        }
      }
      if constexpr (SPLIT) {
        if (k >= ni) {  // couplings to rows held by other parts
          const int32_t e0 = P.ext_ptr[sp.ext_off + (k - ni)], e1 = P.ext_ptr[sp.ext_off + (k - ni) + 1];
          for (int32_t e = e0; e < e1; ++e) {
            const double* hp = reinterpret_cast<const double*>(A.ws) + P.ext_rec[e];
            const Rec h{ld_coh(hp), ld_coh(hp + 1), ld_coh(hp + 2), ld_coh(hp + 3)};
            const int32_t cc = P.ext_coef[e];
            const double c = ((cc & 1) ? -1.0 : 1.0) / A.mass[cc >> 1] * h.l;
            px -= c * h.x;
            py -= c * h.y;
            pz -= c * h.z;
          }
        }
      }
      const double pp = px * px + py * py + pz * pz;
      double g, rel;
      if (A.project) {  // velocity constraint e_k . (v_a - v_b), relative to |e_k| |v_a - v_b|
        g = px * ek.x + py * ek.y + pz * ek.z;
        rel = fabs(g) / fmax(sqrt(pp * (ek.x * ek.x + ek.y * ek.y + ek.z * ek.z)), DBL_MIN);
      } else {
        g = 0.5 * (pp - d2[k]);
        rel = (fabs(g) + sqrt(pp) * delta + delta2) / d2[k];
      }
      if (!(rel <= DBL_MAX)) rel = INFINITY;  // NaN or Inf
      vmax = fmax(vmax, rel);
      y[k] = static_cast<T>(g);
      if constexpr (SPLIT) {
        if (k >= ni) {
          gB[k - ni] = static_cast<double>(static_cast<T>(g));
          const int32_t v = P.bsep[sp.bsep_off + (k - ni)];
          if (v >> 30) {
            SepX& X = sxa[v & 0x3fffffff];
            X.ep[0] = px;
            X.ep[1] = py;
            X.ep[2] = pz;
            X.g = g;
          }
        }
      }
      if (!A.chord) {
        if (tot <= NB) {
          set_diag(k, static_cast<T>(uk.l * (px * ek.x + py * ek.y + pz * ek.z)));
#pragma unroll
          for (int i = 0; i < NB; ++i)
            if (i < tot) F[sb[i]] = static_cast<T>(cb[i] * (px * nb[i].x + py * nb[i].y + pz * nb[i].z));
        } else {
          build_row(k, px, py, pz);
        }
      }
    }
    // workgroup max of the relative violation
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = vmax;
    __syncthreads();
    double gmax = red[0];
#pragma unroll
    for (int w = 1; w < BLOCK / 64; ++w) gmax = fmax(gmax, red[w]);
    gmax = uni(gmax);
    [[maybe_unused]] int32_t sing_all = 0;
    if constexpr (SPLIT) {
      // factor (speculatively: the decision needs every part's violation),
      // publish the border data, then decide from all parts alike
      if (!A.chord) save_border();
      if (A.chord) factor_sweep(std::false_type{}, std::true_type{});
      else factor_sweep(std::true_type{}, std::true_type{});
      if (!A.chord) border_factors(true);
      border_rhs();
      if (tid == 0) {
        pxa[sp.part].viol = gmax;
        pxa[sp.part].singular = singular;
      }
      if (!grid_barrier(bar, sp.n_parts, A.wait_limit, &next_slot)) { st_code = ILVES_ERR_TIMEOUT; break; }
      double gm = 0.0;
      parts_reduce(false, gm, sing_all);
      gmax = uni(gm);
      sing_all = uni(sing_all);
    }
    // convergence history: the maximum violation at iterate it (a restart
    // from 0 after a fallback overwrites the start's entries)
    if (A.hist && tid == 0 && (!SPLIT || sp.part == 0) && it < A.hist_len)
      A.hist[static_cast<int64_t>(report) * A.hist_len + it] = gmax;
    if (A.warm >= 2 && !fell_back) {
      // learned or decoupled start: keep it only while it beats lambda = 0 and the
      // residual does not rise twice in a row; otherwise restart from 0
      rises = (it > 0 && gmax > prev_gmax) ? rises + 1 : 0;
      if ((it == 0 && !(gmax < rel_zero)) || rises >= 2) {
        fell_back = 1;
        prev_gmax = INFINITY;
        for (int32_t k = tid; k < n; k += BLOCK) er[4 * k + 3] = 0.0;
        __syncthreads();
        if constexpr (SPLIT) {
          if (!grid_barrier(bar, sp.n_parts, A.wait_limit, &next_slot)) { st_code = ILVES_ERR_TIMEOUT; break; }
        }
        continue;
      }
      prev_gmax = gmax;
    }
    if (gmax == INFINITY) { st_code = ILVES_ERR_NONFINITE; break; }
    if (gmax <= A.tol) { st_code = ILVES_OK; break; }
    if (it >= A.max_iter) { st_code = ILVES_ERR_NOT_CONVERGED; break; }

    if constexpr (SPLIT) {
      // ---- separator system, then the backward substitution of the
      //      interior levels from the border unknowns z_S
      if (sing_all) { st_code = ILVES_ERR_SINGULAR; break; }
      stage();
      if (!A.chord) assemble(false);
      sep_rhs();
      if (!A.chord && !eliminate(ms + 1)) { st_code = ILVES_ERR_SINGULAR; break; }
      sep_solve(A.chord != 0);
      for (int32_t j = tid; j < nb; j += BLOCK) y[ni + j] = static_cast<T>(zs[P.bsep[sp.bsep_off + j] & 0x3fffffff]);
      __syncthreads();
      back_sweep(sp.h_int);
    } else {
      // ---- factorisation fused with the forward substitution (Newton), or
      //      the forward substitution alone (chord)
      if (A.chord) factor_sweep(std::false_type{}, std::true_type{});
      else factor_sweep(std::true_type{}, std::true_type{});
      if (uni(singular)) { st_code = ILVES_ERR_SINGULAR; break; }

      // ---- backward substitution, then the lambda update
      back_sweep(H);
    }
    // lambda update after the sweep: keeps global traffic out of the levels
    for (int32_t k = tid; k < n; k += BLOCK) er[4 * k + 3] += static_cast<double>(y[k]);
    __syncthreads();
    if constexpr (SPLIT) {
      if (!grid_barrier(bar, sp.n_parts, A.wait_limit, &next_slot)) { st_code = ILVES_ERR_TIMEOUT; break; }
    }
    ++it;
  }

  // ---- outputs: lambda in input order and r' = r_u - M^{-1} G(r)^T lambda
  //      (a part: its interior rows, the separator rows it owns, its atoms)
  for (int32_t k = tid; k < n; k += BLOCK)
    if (!SPLIT || k < ni || (P.bsep[sp.bsep_off + (k - ni)] >> 30)) A.lambda[cid[k]] = er[4 * k + 3];
  const int32_t* __restrict__ inc_ptr = P.inc_ptr + md.incp_off;
  const int32_t* __restrict__ inc = P.inc + md.inc_off;
  const int32_t s_out = SPLIT ? sp.s_own : s;
  for (int32_t a = tid; a < s_out; a += BLOCK) {
    // the atom's own data first, then its constraints two at a time, so
    // that each round of loads is issued together
    const int32_t g = atom_gid[a];
    const double im = invm[a];
    const double u0 = ux[g], u1 = ux[S + g], u2 = ux[2 * S + g];
    const int32_t q0 = inc_ptr[a], q1 = inc_ptr[a + 1];
    double dx = 0.0, dy = 0.0, dz = 0.0;
    for (int32_t q = q0; q < q1; q += 2) {
      const int32_t e0 = inc[q], e1 = inc[imin(q + 1, q1 - 1)];
      const Rec r0 = ld_rec(er + 4 * (e0 >> 1));
      const Rec r1 = ld_rec(er + 4 * (e1 >> 1));
      const double l0 = (e0 & 1) ? -r0.l : r0.l;
      dx += l0 * r0.x;
      dy += l0 * r0.y;
      dz += l0 * r0.z;
      if (q + 1 < q1) {
        const double l1 = (e1 & 1) ? -r1.l : r1.l;
        dx += l1 * r1.x;
        dy += l1 * r1.y;
        dz += l1 * r1.z;
      }
    }
    A.r_out[g] = u0 - im * dx;
    A.r_out[S + g] = u1 - im * dy;
    A.r_out[2 * S + g] = u2 - im * dz;
  }
  if (tid == 0 && (!SPLIT || sp.part == 0)) {
    A.iters[report] = it;
    A.status[report] = st_code;
    if (A.fallback) A.fallback[report] = fell_back;
  }
  __syncthreads();  // LDS and next_slot are reused by the next molecule
  if constexpr (SPLIT) break;
  }
}

// ---------------------------------------------------------------------------
// small molecules (at most 3 constraints on at most 4 atoms): one thread per
// molecule, the same constraint-space Newton iteration in FP64 registers,
// the dense system solved by elimination without pivoting.  A connected
// molecule of that size has one of five shapes; the plan numbers its atoms
// and constraints in the shape's canonical order (SmallTopo) and groups the
// molecules by shape, so each shape runs code with the atom of every
// constraint end and every coupling known at compile time.  G(r) does not
// depend on which end of a constraint comes first (e_k and the signs of its
// row flip together), so the canonical orientation changes nothing.

// Canonical constraints (A[k], B[k]) of each shape: 0 one bond; 1 two bonds
// at atom 0; 2 triangle; 3 three bonds at atom 0; 4 chain 0-1-2-3.
template <int CLS> struct SmallTopo;
template <> struct SmallTopo<0> { static constexpr int NC = 1, NA = 2; static constexpr int A[3] = {0, 0, 0}, B[3] = {1, 1, 1}; };
template <> struct SmallTopo<1> { static constexpr int NC = 2, NA = 3; static constexpr int A[3] = {0, 0, 0}, B[3] = {1, 2, 2}; };
template <> struct SmallTopo<2> { static constexpr int NC = 3, NA = 3; static constexpr int A[3] = {0, 0, 1}, B[3] = {1, 2, 2}; };
template <> struct SmallTopo<3> { static constexpr int NC = 3, NA = 4; static constexpr int A[3] = {0, 0, 0}, B[3] = {1, 2, 3}; };
template <> struct SmallTopo<4> { static constexpr int NC = 3, NA = 4; static constexpr int A[3] = {0, 1, 2}, B[3] = {1, 2, 3}; };

// sigma_{k,x}: +1 if atom x is A[k], -1 if it is B[k], else 0
template <int CLS>
__device__ constexpr int small_sigma(int k, int x) {
  return SmallTopo<CLS>::A[k] == x ? 1 : (SmallTopo<CLS>::B[k] == x ? -1 : 0);
}
// the atom constraints k != j share, or -1
template <int CLS>
__device__ constexpr int small_shared(int k, int j) {
  using T = SmallTopo<CLS>;
  return k == j ? -1
         : (T::A[k] == T::A[j] || T::A[k] == T::B[j]) ? T::A[k]
         : (T::B[k] == T::A[j] || T::B[k] == T::B[j]) ? T::B[k]
                                                      : -1;
}

// PROJECT: velocity projection (residual e_k . p_k; compiled apart so that
// the solve keeps its registers)
template <int CLS, bool PROJECT>
__device__ __forceinline__ void small_solve(const SmallMol& M, const SolveArgs& A) {
  using Tp = SmallTopo<CLS>;
  constexpr int NC = Tp::NC, NA = Tp::NA;
  const int32_t S = A.n_atoms;
  double invm[NA], ru[NA][3];
  double rmax = 0.0;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int32_t g = M.atom[i];
    invm[i] = 1.0 / A.mass[g];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ru[i][c] = A.r_u[c * S + g];
      rmax = fmax(rmax, fabs(ru[i][c]));
    }
  }
  // u_k is formed from r_u where it is needed rather than kept
  auto ucomp = [&](int k, int c) { return ru[Tp::A[k]][c] - ru[Tp::B[k]][c]; };
  double e[NC][3], lam[NC], cdiag[NC], id2[NC];
  double v0 = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int32_t ga = M.atom[Tp::A[k]], gb = M.atom[Tp::B[k]];
#pragma unroll
    for (int c = 0; c < 3; ++c) e[k][c] = A.r[c * S + ga] - A.r[c * S + gb];
    cdiag[k] = invm[Tp::A[k]] + invm[Tp::B[k]];
    id2[k] = 1.0 / M.d2[k];
    const double u0 = ucomp(k, 0), u1 = ucomp(k, 1), u2 = ucomp(k, 2);
    lam[k] = A.warm == 3 ? decoupled_lambda(u0, u1, u2, e[k][0], e[k][1], e[k][2], cdiag[k], M.d2[k])
             : A.warm ? A.lambda[M.cid[k]] : 0.0;
    v0 = fmax(v0, fabs(u0 * u0 + u1 * u1 + u2 * u2 - M.d2[k]) * (0.5 * id2[k]));
  }
  // C_kj for k != j: sigma(k, x) sigma(j, x) / m_x for the shared atom x
  auto coup = [&](int k, int j) {
    const int x = small_shared<CLS>(k, j);
    const double w = invm[x < 0 ? 0 : x];
    return small_sigma<CLS>(k, x < 0 ? 0 : x) * small_sigma<CLS>(j, x < 0 ? 0 : x) > 0 ? w : -w;
  };
  const double delta = 1.7320508075688772 * rmax * 0x1.0p-52;
  const double delta2 = 0.5 * delta * delta;
  int32_t it = 0, st_code = ILVES_ERR_NOT_CONVERGED, fell_back = 0, rises = 0;
  double prev = INFINITY;
  for (;;) {
    double ep[NC][3], g[NC];
    double gmax = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double x = ucomp(k, c) - cdiag[k] * lam[k] * e[k][c];
#pragma unroll
        for (int j = 0; j < NC; ++j)
          if (small_shared<CLS>(k, j) >= 0) x -= coup(k, j) * lam[j] * e[j][c];
        ep[k][c] = x;
      }
      const double pp = ep[k][0] * ep[k][0] + ep[k][1] * ep[k][1] + ep[k][2] * ep[k][2];
      double rel;
      if (PROJECT) {
        g[k] = ep[k][0] * e[k][0] + ep[k][1] * e[k][1] + ep[k][2] * e[k][2];
        rel = fabs(g[k]) / fmax(sqrt(pp * (e[k][0] * e[k][0] + e[k][1] * e[k][1] + e[k][2] * e[k][2])), DBL_MIN);
      } else {
        g[k] = 0.5 * (pp - M.d2[k]);
        rel = (fabs(g[k]) + sqrt(pp) * delta + delta2) * id2[k];
      }
      if (!(rel <= DBL_MAX)) rel = INFINITY;
      gmax = fmax(gmax, rel);
    }
    if (A.hist && it < A.hist_len) A.hist[static_cast<int64_t>(M.mol) * A.hist_len + it] = gmax;
    if (A.warm >= 2 && !fell_back) {
      rises = (it > 0 && gmax > prev) ? rises + 1 : 0;
      if ((it == 0 && !(gmax < v0)) || rises >= 2) {
        fell_back = 1;
        prev = INFINITY;
#pragma unroll
        for (int k = 0; k < NC; ++k) lam[k] = 0.0;
        continue;
      }
      prev = gmax;
    }
    if (gmax == INFINITY) { st_code = ILVES_ERR_NONFINITE; break; }
    if (gmax <= A.tol) { st_code = ILVES_OK; break; }
    if (it >= A.max_iter) { st_code = ILVES_ERR_NOT_CONVERGED; break; }
    // A_kj = C_kj (e'_k . e_j), zero where k and j share no atom
    double m[NC][NC + 1];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const double* xk = A.chord ? e[k] : ep[k];  // chord: the constant A(r, r)
        const double dot = xk[0] * e[j][0] + xk[1] * e[j][1] + xk[2] * e[j][2];
        m[k][j] = k == j ? cdiag[k] * dot : (small_shared<CLS>(k, j) >= 0 ? coup(k, j) * dot : 0.0);
      }
      m[k][NC] = g[k];
    }
    bool sing = false;
#pragma unroll
    for (int p = 0; p < NC; ++p) {
      if (!(fabs(m[p][p]) > 1e-13 * fabs(cdiag[p] * (e[p][0] * e[p][0] + e[p][1] * e[p][1] + e[p][2] * e[p][2]))))
        sing = true;
      // 1 / pivot from the hardware reciprocal refined by Newton steps,
      // kept in the pivot's slot for the back substitution
      const double inv = recip(m[p][p]);
#pragma unroll
      for (int q = p + 1; q < NC; ++q) {
        const double f = m[q][p] * inv;
#pragma unroll
        for (int j = p; j <= NC; ++j) m[q][j] -= f * m[p][j];
      }
      m[p][p] = inv;
    }
    if (sing) { st_code = ILVES_ERR_SINGULAR; break; }
    double z[NC];
#pragma unroll
    for (int p = NC - 1; p >= 0; --p) {
      double acc = m[p][NC];
#pragma unroll
      for (int j = p + 1; j < NC; ++j) acc -= m[p][j] * z[j];
      z[p] = acc * m[p][p];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) lam[k] += z[k];
    ++it;
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) A.lambda[M.cid[k]] = lam[k];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int sg = small_sigma<CLS>(k, i);
      if (sg == 0) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] += (sg > 0 ? lam[k] : -lam[k]) * e[k][c];
    }
    const int32_t gi = M.atom[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) A.r_out[c * S + gi] = ru[i][c] - invm[i] * d[c];
  }
  A.iters[M.mol] = it;
  A.status[M.mol] = st_code;
  if (A.fallback) A.fallback[M.mol] = fell_back;
}

// the shape of a record, from its canonical numbering (small_shape on the
// host): a star and a chain both have three constraints on four atoms and
// differ in the first atom of constraint 1
__device__ __forceinline__ int small_class(const SmallMol& M) {
  return M.nc == 1 ? 0 : M.nc == 2 ? 1 : M.na == 3 ? 2 : (M.a[1] == 0 ? 3 : 4);
}

template <bool PROJECT>
__global__ void __launch_bounds__(256) small_kernel(const SmallMol* __restrict__ sm, int32_t count,
                                                   const SolveArgs A) {
  const int32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= count) return;
  const SmallMol M = sm[t];
  switch (small_class(M)) {
    case 0: small_solve<0, PROJECT>(M, A); break;
    case 1: small_solve<1, PROJECT>(M, A); break;
    case 2: small_solve<2, PROJECT>(M, A); break;
    case 3: small_solve<3, PROJECT>(M, A); break;
    default: small_solve<4, PROJECT>(M, A); break;
  }
}

__global__ void reset_counters(int32_t* __restrict__ c, int32_t n) {
  const int i = threadIdx.x;
  if (i < n) c[i] = 0;
}

__global__ void copy_free_atoms(const int32_t* __restrict__ idx, int32_t n_free, int32_t S,
                                const double* __restrict__ r_u, double* __restrict__ r_out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_free) {
    const int32_t g = idx[i];
    r_out[g] = r_u[g];
    r_out[S + g] = r_u[S + g];
    r_out[2 * S + g] = r_u[2 * S + g];
  }
}

using KernelFn = void (*)(DevPlan, const int32_t*, int32_t, int32_t*, SolveArgs);

template <typename T, typename Idx, int MODE>
KernelFn pick_block(int block) {
  switch (block) {
    case 64: return solve_kernel<T, Idx, MODE, 64>;
    case 128: return solve_kernel<T, Idx, MODE, 128>;
    case 256: return solve_kernel<T, Idx, MODE, 256>;
    case 512: return solve_kernel<T, Idx, MODE, 512>;
    default: return solve_kernel<T, Idx, MODE, 1024>;
  }
}

template <typename T, typename Idx, int MODE>
KernelFn pick_big(int block) {
  return block <= 512 ? solve_kernel<T, Idx, MODE, 512> : solve_kernel<T, Idx, MODE, 1024>;
}

// Block size a kernel is compiled for: every launch uses exactly this.
int kernel_block(int mode, bool wide, int block) {
  if (mode == ALL_LDS && !wide) return block <= 64 ? 64 : block <= 128 ? 128 : block <= 256 ? 256 : block <= 512 ? 512 : 1024;
  if (mode == VALUES_LDS && !wide) return block <= 256 ? 256 : block <= 512 ? 512 : 1024;
  return block <= 512 ? 512 : 1024;
}

template <typename T>
KernelFn pick_mode(int mode, bool wide, int block, bool heavy) {
  if (heavy && mode == ALL_LDS && !wide && block == 512) return solve_kernel<T, uint16_t, ALL_LDS, 512, false, kBatchNWide>;
  if (wide) return mode == VALUES_LDS ? pick_big<T, int32_t, VALUES_LDS>(block) : pick_big<T, int32_t, GLOBAL>(block);
  if (mode == ALL_LDS) return pick_block<T, uint16_t, ALL_LDS>(block);
  if (mode == STRUCT_LDS) return pick_big<T, uint16_t, STRUCT_LDS>(block);
  if (mode == VALUES_LDS) return block <= 256 ? solve_kernel<T, uint16_t, VALUES_LDS, 256> : pick_big<T, uint16_t, VALUES_LDS>(block);
  return pick_big<T, uint16_t, GLOBAL>(block);
}

KernelFn pick_kernel(bool fp32, int mode, bool wide, int block, bool heavy = false) {
  return fp32 ? pick_mode<float>(mode, wide, block, heavy) : pick_mode<double>(mode, wide, block, heavy);
}

// parts of split molecules (16-bit indices): structure and values in LDS,
// the values and the per-row structure, or the values only
constexpr int kSplitBlock = 512;
KernelFn pick_split(bool fp32, int mode) {
  if (mode == ALL_LDS)
    return fp32 ? solve_kernel<float, uint16_t, ALL_LDS, kSplitBlock, true>
                : solve_kernel<double, uint16_t, ALL_LDS, kSplitBlock, true>;
  if (mode == PAIRS_GLOBAL)
    return fp32 ? solve_kernel<float, uint16_t, PAIRS_GLOBAL, kSplitBlock, true, kBatchNWide>
                : solve_kernel<double, uint16_t, PAIRS_GLOBAL, kSplitBlock, true, kBatchNWide>;
  return fp32 ? solve_kernel<float, uint16_t, VALUES_LDS, kSplitBlock, true, kBatchNWide>
              : solve_kernel<double, uint16_t, VALUES_LDS, kSplitBlock, true, kBatchNWide>;
}

constexpr int kLdsMax = 160 * 1024 - 1024;  // dynamic LDS a molecule may use
constexpr int kCuLds = 160 * 1024;          // LDS of a CU
constexpr int kStreams = 4;                 // concurrent launch groups

struct Group {
  int block = 256;
  int mode = ALL_LDS;
  bool wide = false;
  int lds_bytes = 0;
  int32_t first = 0;  // into the device molecule-list array
  int32_t count = 0;
  int32_t grid = 0;   // persistent workgroups
  int32_t counter = 0;  // index of the group's queue counter
  int stream = 0;       // index into the plan's streams
  int64_t work = 0;     // sum over its molecules of rows + off-diagonal slots
  bool heavy = false;   // largest trees, 512 threads: the wide-batch kernel
};
constexpr int kMaxGroups = 64;

// One launch of split-molecule parts: whole molecules, at most as many
// parts as can be resident on the device at once (their barriers need it).
struct SplitLaunch {
  int32_t first = 0, count = 0;  // parts: a range of the precision's part order (d_split_order)
  int lds_bytes = 0;
  int stream = 0;
  int mode = ALL_LDS;            // placement of every part of the launch
};

}  // namespace

// ---------------------------------------------------------------------------
// the plan object

struct ilves_plan {
  int device = 0;
  int32_t n_atoms = 0, n_con = 0;
  ilves_options_t opt{};
  std::vector<ilves::MolPlan> mols;   // host copy, in plan order
  DevPlan dp{};
  void* d_buf = nullptr;
  size_t buf_bytes = 0;
  unsigned char* d_ws = nullptr;
  size_t ws_bytes = 0;
  int32_t* d_free = nullptr;
  int32_t n_free = 0;
  int32_t* d_lists = nullptr;          // molecule lists of every group, both precisions
  int32_t* d_counters = nullptr;       // queue counters of the groups (kMaxGroups per precision)
  int n_cu = 0;
  int32_t band_block[5] = {64, 128, 256, 512, 1024};  // block size per LDS band (tunable)
  std::vector<Group> groups[2];        // [0] FP64, [1] mixed
  std::vector<ilves::SplitPlan> splits;  // molecules split across workgroups
  std::vector<int32_t> split_mol;        // their molecule indices
  std::vector<int32_t> split_first;      // first part (device part index) of each
  std::vector<int64_t> split_xch;        // workspace byte offset of each one's exchange area
  std::vector<int> split_lds[2];         // per part: dynamic LDS bytes
  std::vector<int> split_mode[2];        // per split molecule: ALL_LDS, PAIRS_GLOBAL or VALUES_LDS
  std::vector<SplitLaunch> split_launch[2];
  const int32_t* d_split_order[2] = {nullptr, nullptr};  // per precision: parts grouped by placement
  int32_t chunk_first[2] = {0, 0};     // row chunks of the feature passes, by index width
  int32_t chunk_count[2] = {0, 0};
  const int2* d_chunks = nullptr;      // {molecule, first row} pairs in d_buf
  const SmallMol* d_small = nullptr;   // small-molecule records in d_buf
  int32_t n_small = 0;
  int small_stream = 0;                // stream of the small-molecule kernel
  int split_stream[2] = {0, 0};        // stream of the split-molecule launches
  int32_t wait_limit = 1 << 22;        // polls of a split barrier's wait
  float* d_mlp = nullptr;              // network parameters then normalisation block
  float* d_feat = nullptr;             // [n_constraints][16] features (plan row order)
  float* d_w = nullptr;                // [n_constraints] 1/m_a + 1/m_b
  hipStream_t streams[kStreams] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kStreams] = {};
  int64_t stats[ILVES_STAT_COUNT] = {};
};

namespace {

template <typename V>
size_t push_array(std::vector<unsigned char>& blob, const std::vector<V>& v) {
  size_t off = (blob.size() + 255) & ~static_cast<size_t>(255);
  blob.resize(off + v.size() * sizeof(V));
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(V));
  return off;
}

// Ends of constraint k of a small-molecule shape (the canonical order of
// SmallTopo): end 0 is A[k], end 1 is B[k].
int small_topo_end(int shape, int k, int end) {
  switch (shape) {
    case 0: return end == 0 ? SmallTopo<0>::A[k] : SmallTopo<0>::B[k];
    case 1: return end == 0 ? SmallTopo<1>::A[k] : SmallTopo<1>::B[k];
    case 2: return end == 0 ? SmallTopo<2>::A[k] : SmallTopo<2>::B[k];
    case 3: return end == 0 ? SmallTopo<3>::A[k] : SmallTopo<3>::B[k];
    default: return end == 0 ? SmallTopo<4>::A[k] : SmallTopo<4>::B[k];
  }
}

// Shape of a molecule of at most kSmallCons constraints on kSmallAtoms
// atoms and its canonical numbering: atom[a] is the molecule's local atom
// that takes canonical number a, con[k] the local constraint that takes
// canonical number k.  Returns -1 when the molecule has none of the shapes
// (a connected molecule of that size always has one).
int small_shape(const ilves::MolPlan& M, int32_t atom[kSmallAtoms], int32_t con[kSmallCons]) {
  const int nc = M.n, na = M.s;
  int deg[kSmallAtoms] = {0, 0, 0, 0};
  for (int k = 0; k < nc; ++k) {
    if (M.ra[k] < 0 || M.ra[k] >= na || M.rb[k] < 0 || M.rb[k] >= na) return -1;
    ++deg[M.ra[k]];
    ++deg[M.rb[k]];
  }
  auto other = [&](int k, int x) { return M.ra[k] == x ? M.rb[k] : M.ra[k]; };
  auto find = [&](int x, int y) {
    for (int k = 0; k < nc; ++k)
      if ((M.ra[k] == x && M.rb[k] == y) || (M.ra[k] == y && M.rb[k] == x)) return k;
    return -1;
  };
  auto center = [&](int d) {
    for (int x = 0; x < na; ++x)
      if (deg[x] == d) return x;
    return -1;
  };
  int shape = -1;
  for (int a = 0; a < kSmallAtoms; ++a) atom[a] = 0;
  for (int k = 0; k < kSmallCons; ++k) con[k] = 0;
  if (nc == 1 && na == 2) {
    shape = 0;
    atom[0] = M.ra[0];
    atom[1] = M.rb[0];
  } else if (nc == 2 && na == 3) {
    const int c = center(2);
    if (c < 0) return -1;
    shape = 1;
    atom[0] = c;
    atom[1] = other(0, c);
    atom[2] = other(1, c);
    con[1] = 1;
  } else if (nc == 3 && na == 3) {
    shape = 2;
    for (int a = 0; a < 3; ++a) atom[a] = a;
  } else if (nc == 3 && na == 4) {
    const int c = center(3);
    if (c >= 0) {
      shape = 3;
      atom[0] = c;
      for (int k = 0; k < 3; ++k) atom[k + 1] = other(k, c);
    } else {
      const int p0 = center(1);
      if (p0 < 0) return -1;
      shape = 4;
      atom[0] = p0;
      for (int a = 1; a < 4; ++a) {  // walk the chain
        int next = -1;
        for (int k = 0; k < nc; ++k) {
          const int y = M.ra[k] == atom[a - 1] ? M.rb[k] : (M.rb[k] == atom[a - 1] ? M.ra[k] : -1);
          if (y >= 0 && (a < 2 || y != atom[a - 2])) next = y;
        }
        if (next < 0) return -1;
        atom[a] = next;
      }
    }
  } else {
    return -1;
  }
  // every canonical constraint is one of the molecule's, each used once
  bool used[kSmallCons] = {false, false, false};
  for (int k = 0; k < nc; ++k) {
    const int q = find(atom[small_topo_end(shape, k, 0)], atom[small_topo_end(shape, k, 1)]);
    if (q < 0 || used[q]) return -1;
    used[q] = true;
    con[k] = q;
  }
  return shape;
}

template <typename V>
void append(std::vector<V>& dst, const std::vector<int32_t>& src) {
  for (int32_t x : src) dst.push_back(static_cast<V>(x));
}

// lanes per item (log2) of level h: in the factorisation from its longest
// chain (lower entries of a row, updates of a pair task), in the backward
// substitution from its longest row of upper entries
void level_lanes(const ilves::MolPlan& M, int32_t h, int32_t& lg_factor, int32_t& lg_backward) {
  int32_t cf = 0, cb = 0;
  for (int32_t j = M.lvl_row[h]; j < M.lvl_row[h + 1]; ++j) {
    cf = std::max(cf, M.l_start[j + 1] - M.l_start[j]);
    cb = std::max(cb, M.up_start[j + 1] - M.up_start[j]);
  }
  for (int32_t pi = M.pl_start[h]; pi < M.pl_start[h + 1]; ++pi)
    cf = std::max(cf, M.ustart[M.plist[pi] + 1] - M.ustart[M.plist[pi]]);
  const int32_t nr = M.lvl_row[h + 1] - M.lvl_row[h], np = M.pl_start[h + 1] - M.pl_start[h];
  lg_factor = item_lanes_log2(cf, nr, np, true);
  lg_backward = item_lanes_log2(cb, nr, 0, false);
}

// Appends a molecule's structure block (see struct_layout) to the pool and
// returns its byte offset (-1 if a slot's shared atom is not one of its
// row's atoms, which a consistent plan never has).
template <typename Idx>
int64_t pack_struct(const ilves::MolPlan& M, std::vector<unsigned char>& pool) {
  const int32_t n_pl = static_cast<int32_t>(M.plist.size());
  const Layout Lo = struct_layout(M.n, M.n_levels, M.n_up, M.n_l, n_pl, M.n_upd, static_cast<int>(sizeof(Idx)));
  const int64_t off = align_to(static_cast<int64_t>(pool.size()), 16);
  pool.resize(static_cast<size_t>(off + Lo.total), 0);
  auto put = [&](int64_t sec, int64_t idx, int32_t v) {
    const Idx x = static_cast<Idx>(v);
    std::memcpy(pool.data() + off + sec + idx * static_cast<int64_t>(sizeof(Idx)), &x, sizeof(Idx));
  };
  for (int32_t k = 0; k <= M.n; ++k) {
    put(Lo.up_start, k, M.up_start[k]);
    put(Lo.l_start, k, M.l_start[k]);
  }
  for (int32_t q = 0; q < M.n_up; ++q) put(Lo.ucol, q, M.ucol[q]);
  for (int32_t h = 0; h < M.n_levels; ++h) {
    put(Lo.lvh, 4 * h + 0, M.lvl_row[h]);
    put(Lo.lvh, 4 * h + 1, M.lvl_row[h + 1]);
    put(Lo.lvh, 4 * h + 2, M.pl_start[h]);
    put(Lo.lvh, 4 * h + 3, M.pl_start[h + 1]);
  }
  for (int32_t h = 0; h < M.n_levels; ++h) {
    int32_t lf, lb;
    level_lanes(M, h, lf, lb);
    put(Lo.lvc, 2 * h + 0, lf);
    put(Lo.lvc, 2 * h + 1, lb);
  }
  for (int32_t t = 0; t < M.n_l; ++t) {
    put(Lo.lpair, 2 * t + 0, M.lcol[t]);
    put(Lo.lpair, 2 * t + 1, M.ltr[t]);
  }
  // coupling codes: the shared atom of every slot is one of its row's atoms
  unsigned char* cc = pool.data() + off + Lo.ccode;
  bool bad = false;
  auto code = [&](int32_t k, int32_t c) -> unsigned char {
    const int32_t x = c >> 1;
    if (x >= M.s) return kFillCode;
    if (x != M.ra[k] && x != M.rb[k]) bad = true;
    return static_cast<unsigned char>((x == M.rb[k] ? 2 : 0) | (c & 1));
  };
  for (int32_t k = 0; k < M.n; ++k) {
    for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q) cc[q] = code(k, M.ucoef[q]);
    for (int32_t t = M.l_start[k]; t < M.l_start[k + 1]; ++t) cc[t] = code(k, M.lcoef[t - M.n_up]);
  }
  if (bad) return -1;
  for (int32_t pi = 0; pi < n_pl; ++pi) {
    const int32_t q = M.plist[pi];
    put(Lo.prec, 4 * pi + 0, q);
    put(Lo.prec, 4 * pi + 1, M.utr[q]);
    put(Lo.prec, 4 * pi + 2, M.ustart[q]);
    put(Lo.prec, 4 * pi + 3, M.ustart[q + 1] - M.ustart[q]);
  }
  for (int32_t u = 0; u < M.n_upd; ++u) {
    const int32_t pa = M.upd_a[u], pb = M.upd_b[u];
    put(Lo.upd, 4 * u + 0, pa);
    put(Lo.upd, 4 * u + 1, pb);
    put(Lo.upd, 4 * u + 2, M.ltr[pb - M.n_up]);  // slot (i, m)
    put(Lo.upd, 4 * u + 3, M.ltr[pa - M.n_up]);  // slot (i, j)
    put(Lo.updi, u, M.lcol[pa - M.n_up]);        // row i
  }
  return off;
}

// placement of one molecule for value type T: mode and LDS bytes
// (prefer everything in LDS; else the factor values, whose accesses form
// the dependent chain of each level; else the structure; else nothing)
template <typename T>
std::pair<int, int> placement(const ilves::MolPlan& M, bool wide, int64_t lds_limit) {
  const size_t vb = value_bytes<T>(M.n, M.n_up, M.n_l);
  if (wide) return static_cast<int64_t>(vb) <= lds_limit ? std::make_pair(static_cast<int>(VALUES_LDS), static_cast<int>(vb))
                                                        : std::make_pair(static_cast<int>(GLOBAL), 0);
  const size_t sb = static_cast<size_t>(struct_layout(M.n, M.n_levels, M.n_up, M.n_l,
                                                      static_cast<int32_t>(M.plist.size()), M.n_upd, 2).total);
  if (static_cast<int64_t>(sb + vb) <= lds_limit) return {ALL_LDS, static_cast<int>(sb + vb)};
  if (static_cast<int64_t>(vb) <= lds_limit) return {VALUES_LDS, static_cast<int>(vb)};
  if (static_cast<int64_t>(sb) <= lds_limit) return {STRUCT_LDS, static_cast<int>(sb)};
  return {GLOBAL, 0};
}

ilves_status_t build_device_plan(ilves_plan* P) {
  const int32_t nm = static_cast<int32_t>(P->mols.size());
  int32_t n_parts = 0;
  for (const auto& sp : P->splits) n_parts += static_cast<int32_t>(sp.parts.size());
  std::vector<MolDesc> desc(nm + n_parts);
  std::vector<unsigned char> pool;
  std::vector<int32_t> coef, ra, rb, cid, atom_gid, inc_ptr, inc, gcoef, gra, grb;
  std::vector<double> d2;
  std::vector<char> wide(nm + n_parts, 0);
  int64_t fill = 0, work = 0, maxlev = 0, sumlev = 0, nslots = 0, natoms = 0, ncon = 0;
  size_t ws = 0;
  // descriptors: the molecules, then the parts of the split molecules
  std::vector<const ilves::MolPlan*> plans;
  for (const auto& M : P->mols) plans.push_back(&M);
  for (const auto& sp : P->splits)
    for (const auto& M : sp.parts) plans.push_back(&M);
  for (int32_t i = 0; i < nm + n_parts; ++i) {
    const ilves::MolPlan& M = *plans[i];
    MolDesc& D = desc[i];
    D.n = M.n;
    D.s = M.s;
    D.n_up = M.n_up;
    D.n_l = M.n_l;
    D.n_upd = M.n_upd;
    D.n_levels = M.n_levels;
    D.n_pl = static_cast<int32_t>(M.plist.size());
    const int64_t total = static_cast<int64_t>(M.n_up) + M.n_l;
    wide[i] = (total >= 65535 || M.n >= 65535 || M.n_upd >= 65535) ? 1 : 0;
    D.wide = wide[i];
    D.ix_off = wide[i] ? pack_struct<int32_t>(M, pool) : pack_struct<uint16_t>(M, pool);
    if (D.ix_off < 0) return fail(ILVES_ERR_TOPOLOGY, "plan: a coupling's shared atom is not an atom of its row");
    D.coef_off = static_cast<int32_t>(coef.size());
    coef.insert(coef.end(), M.ucoef.begin(), M.ucoef.end());
    coef.insert(coef.end(), M.lcoef.begin(), M.lcoef.end());
    for (const std::vector<int32_t>* cv : {&M.ucoef, &M.lcoef})
      for (int32_t c : *cv) gcoef.push_back((c >> 1) >= M.s ? -1 : ((M.atom_gid[c >> 1] << 1) | (c & 1)));
    for (int32_t k = 0; k < M.n; ++k) {
      gra.push_back(M.atom_gid[M.ra[k]]);
      grb.push_back(M.atom_gid[M.rb[k]]);
    }
    D.row_off = static_cast<int32_t>(ra.size());
    ra.insert(ra.end(), M.ra.begin(), M.ra.end());
    rb.insert(rb.end(), M.rb.begin(), M.rb.end());
    cid.insert(cid.end(), M.cid.begin(), M.cid.end());
    d2.insert(d2.end(), M.d2.begin(), M.d2.end());
    D.atom_off = static_cast<int32_t>(atom_gid.size());
    atom_gid.insert(atom_gid.end(), M.atom_gid.begin(), M.atom_gid.end());
    D.incp_off = static_cast<int32_t>(inc_ptr.size());
    inc_ptr.insert(inc_ptr.end(), M.inc_ptr.begin(), M.inc_ptr.end());
    D.inc_off = static_cast<int32_t>(inc.size());
    inc.insert(inc.end(), M.inc.begin(), M.inc.end());
    D.ws_off = static_cast<int64_t>(ws);
    ws += (ws_vec_bytes(M.n, M.s, M.n_up, M.n_l) + value_bytes<double>(M.n, M.n_up, M.n_l) + 255) &
          ~static_cast<size_t>(255);
    if (i >= nm) continue;  // statistics count whole molecules
    fill += M.fill;
    work += M.n_upd;
    maxlev = std::max<int64_t>(maxlev, M.n_levels);
    sumlev += M.n_levels;
    nslots += total + M.n;
    natoms += M.s;
    ncon += M.n;
  }
  // launch order: largest structure first
  std::vector<int32_t> ord(nm);
  for (int32_t i = 0; i < nm; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    return static_cast<int64_t>(desc[x].n_up) + desc[x].n_l + desc[x].n >
           static_cast<int64_t>(desc[y].n_up) + desc[y].n_l + desc[y].n;
  });
  // small molecules go to the one-thread-per-molecule kernel, numbered in
  // their shape's canonical order and grouped by shape (the kernel branches
  // on the shape, so a wave should hold one)
  std::vector<char> small(nm, 0);
  std::vector<SmallMol> smalls;
  std::vector<int> shapes;
  for (int32_t i = 0; i < nm; ++i) {
    const ilves::MolPlan& M = P->mols[i];
    if (M.n > kSmallCons || M.s > kSmallAtoms || M.n < 1) continue;
    int32_t atom[kSmallAtoms], con[kSmallCons];
    const int shape = small_shape(M, atom, con);
    if (shape < 0) continue;  // not one of the five shapes: the general path
    small[i] = 1;
    SmallMol r{};
    for (int a = 0; a < kSmallAtoms; ++a) r.atom[a] = M.atom_gid[atom[a < M.s ? a : 0]];
    for (int k = 0; k < kSmallCons; ++k) {
      const bool used = k < M.n;
      r.cid[k] = M.cid[used ? con[k] : con[0]];
      r.a[k] = static_cast<uint8_t>(used ? small_topo_end(shape, k, 0) : 0);
      r.b[k] = static_cast<uint8_t>(used ? small_topo_end(shape, k, 1) : 0);
      r.d2[k] = used ? M.d2[con[k]] : 1.0;
    }
    r.mol = i;
    r.nc = static_cast<uint8_t>(M.n);
    r.na = static_cast<uint8_t>(M.s);
    smalls.push_back(r);
    shapes.push_back(shape);
  }
  {
    std::vector<int32_t> so(smalls.size());
    for (size_t q = 0; q < so.size(); ++q) so[q] = static_cast<int32_t>(q);
    std::stable_sort(so.begin(), so.end(), [&](int32_t x, int32_t y) { return shapes[x] < shapes[y]; });
    std::vector<SmallMol> sorted;
    sorted.reserve(smalls.size());
    for (int32_t q : so) sorted.push_back(smalls[q]);
    smalls.swap(sorted);
  }
  ord.erase(std::remove_if(ord.begin(), ord.end(), [&](int32_t i) { return small[i] != 0; }), ord.end());
  std::vector<char> is_split(nm, 0);
  for (int32_t i : P->split_mol) is_split[i] = 1;
  std::vector<int32_t> ord_solve;  // molecules solved by the per-molecule kernels
  for (int32_t i : ord)
    if (!is_split[i]) ord_solve.push_back(i);

  // split molecules: part records, separator tables, exchange areas
  std::vector<SplitPart> sparts;
  std::vector<SepRow> seprows;
  std::vector<int32_t> sadj, bsep, ext_ptr, ext_coef;
  std::vector<int64_t> ext_rec;
  P->split_first.clear();
  P->split_xch.clear();
  for (int prec = 0; prec < 2; ++prec) {
    P->split_lds[prec].clear();
    P->split_mode[prec].clear();
  }
  int64_t max_sep = 0;
  {
    int32_t d0 = nm;  // descriptor of the first part of the current molecule
    for (size_t si = 0; si < P->splits.size(); ++si) {
      const ilves::SplitPlan& SPL = P->splits[si];
      const int32_t G = static_cast<int32_t>(SPL.parts.size()), m = SPL.m;
      max_sep = std::max<int64_t>(max_sep, m);
      ws = (ws + 255) & ~static_cast<size_t>(255);
      const int64_t xch = static_cast<int64_t>(ws);
      std::vector<int32_t> ew_off(G);
      int64_t xsz = xch_ew(G, m);
      for (int32_t g = 0; g < G; ++g) {
        ew_off[g] = static_cast<int32_t>(xsz / 8);
        const int64_t nbg = SPL.parts[g].n - SPL.parts[g].n_int;
        xsz += 8 * (nbg * nbg + nbg);
      }
      ws += static_cast<size_t>((xsz + 255) & ~static_cast<int64_t>(255));
      const int32_t ew_total = static_cast<int32_t>((xsz - xch_ew(G, m)) / 8);
      const int32_t n_sadj = static_cast<int32_t>(SPL.sadj_col.size());
      const int32_t sep_off = static_cast<int32_t>(seprows.size());
      for (int32_t b = 0; b < m; ++b) {
        SepRow R{};
        R.part0 = SPL.sep_part[2 * b];
        R.part1 = SPL.sep_part[2 * b + 1];
        R.loc0 = SPL.sep_loc[2 * b];
        R.loc1 = SPL.sep_loc[2 * b + 1];
        R.ga = SPL.sep_ga[b];
        R.gb = SPL.sep_gb[b];
        R.adj_off = static_cast<int32_t>(sadj.size() / 2);
        R.adj_cnt = SPL.sadj_ptr[b + 1] - SPL.sadj_ptr[b];
        for (int32_t a = SPL.sadj_ptr[b]; a < SPL.sadj_ptr[b + 1]; ++a) {
          sadj.push_back(SPL.sadj_col[a]);
          sadj.push_back(SPL.sadj_coef[a]);
        }
        R.ew0 = ew_off[R.part0];
        R.ew1 = ew_off[R.part1];
        R.nb0 = SPL.parts[R.part0].n - SPL.parts[R.part0].n_int;
        R.nb1 = SPL.parts[R.part1].n - SPL.parts[R.part1].n_int;
        seprows.push_back(R);
      }
      P->split_first.push_back(static_cast<int32_t>(sparts.size()));
      P->split_xch.push_back(xch);
      // placement per precision: structure and values in LDS when every part
      // fits, else the values with the per-row structure (pair tasks and
      // updates read from global memory), else the values only
      for (int prec = 0; prec < 2; ++prec) {
        bool all = true, rows = true;
        for (int32_t g = 0; g < G; ++g) {
          const ilves::MolPlan& M = SPL.parts[g];
          const Layout Lo = struct_layout(M.n, M.n_levels, M.n_up, M.n_l, static_cast<int32_t>(M.plist.size()),
                                          M.n_upd, 2);
          const int64_t vb = prec == 0 ? value_bytes<double>(M.n, M.n_up, M.n_l) : value_bytes<float>(M.n, M.n_up, M.n_l);
          const int64_t scr = split_lds_bytes(m, M.n - M.n_int, ew_total, n_sadj);
          if (static_cast<int64_t>(align16(Lo.total + vb)) + scr > kLdsMax) all = false;
          if (static_cast<int64_t>(align16(align_to(Lo.prec, 16) + vb)) + scr > kLdsMax) rows = false;
        }
        P->split_mode[prec].push_back(all ? ALL_LDS : rows ? PAIRS_GLOBAL : VALUES_LDS);
      }
      for (int32_t g = 0; g < G; ++g) {
        const ilves::MolPlan& M = SPL.parts[g];
        const int32_t nbg = M.n - M.n_int;
        SplitPart X{};
        X.desc = d0 + g;
        X.report = P->split_mol[si];
        X.part = g;
        X.n_parts = G;
        X.n_int = M.n_int;
        X.h_int = M.h_int;
        X.s_own = M.s_own;
        X.m = m;
        X.bsep_off = static_cast<int32_t>(bsep.size());
        for (int32_t j = 0; j < nbg; ++j) {
          int32_t v = -1;
          for (int32_t b = 0; b < m && v < 0; ++b)
            for (int u = 0; u < 2; ++u)
              if (SPL.sep_part[2 * b + u] == g && SPL.sep_loc[2 * b + u] == j) v = b | (u == 0 ? (1 << 30) : 0);
          if (v < 0) return fail(ILVES_ERR_ARG, "internal: border row without separator row");
          bsep.push_back(v);
        }
        X.ext_off = static_cast<int32_t>(ext_ptr.size());
        for (int32_t j = 0; j <= nbg; ++j) ext_ptr.push_back(static_cast<int32_t>(ext_rec.size()) + SPL.ext_ptr[g][j]);
        for (size_t e = 0; e < SPL.ext_part[g].size(); ++e)
          ext_coef.push_back(SPL.ext_coef[g][e]);
        for (size_t e = 0; e < SPL.ext_part[g].size(); ++e)
          ext_rec.push_back(desc[d0 + SPL.ext_part[g][e]].ws_off / 8 + 4 * static_cast<int64_t>(SPL.ext_row[g][e]));
        X.sep_off = sep_off;
        X.ew_off = ew_off[g];
        X.xch = xch;
        X.ew_total = ew_total;
        X.n_sadj = n_sadj;
        X.bw = SPL.bw;
        // LDS: the structure block (ALL_LDS) or its per-row part
        // (PAIRS_GLOBAL), then the values, then the split scratch
        const Layout Lo = struct_layout(M.n, M.n_levels, M.n_up, M.n_l, static_cast<int32_t>(M.plist.size()),
                                        M.n_upd, 2);
        for (int prec = 0; prec < 2; ++prec) {
          const int64_t vb = prec == 0 ? value_bytes<double>(M.n, M.n_up, M.n_l) : value_bytes<float>(M.n, M.n_up, M.n_l);
          const int mode = P->split_mode[prec].back();
          const int64_t base = mode == ALL_LDS        ? static_cast<int64_t>(align16(Lo.total + vb))
                               : mode == PAIRS_GLOBAL ? static_cast<int64_t>(align16(align_to(Lo.prec, 16) + vb))
                                                      : static_cast<int64_t>(align16(vb));
          X.lds_extra[prec] = static_cast<int32_t>(base);
          P->split_lds[prec].push_back(static_cast<int>(base + split_lds_bytes(m, nbg, ew_total, n_sadj)));
        }
        sparts.push_back(X);
      }
      d0 += G;
    }
  }
  std::vector<int32_t> lists;
  int64_t in_lds = 0, in_ws = 0;
  for (int prec = 0; prec < 2; ++prec) {
    P->groups[prec].clear();
    // launch groups: LDS-resident molecules in bands of LDS size (block
    // size grows with the band), structure-only and global molecules apart
    // Launch groups.  Every workgroup of a group allocates the group's
    // largest LDS need, and groups beyond the number of streams run one after
    // another, so the molecules held wholly in LDS are split, in order of
    // their LDS need, into at most as many groups as there are streams left,
    // at the split points that minimise the sum over groups of (allocated
    // LDS) x (sum of the planner's cost estimates): the LDS-time product that
    // bounds how many molecules are resident per CU.  Molecules with only
    // part of their data in LDS form groups of their own by size.
    struct Key { int mode; bool wide; int band; };
    std::vector<std::pair<Key, std::vector<int32_t>>> buckets;
    std::vector<int> lds_of(nm, 0);
    std::vector<int32_t> in_lds_list;
    for (int32_t i : ord_solve) {
      const ilves::MolPlan& M = P->mols[i];
      auto pl = prec == 0 ? placement<double>(M, wide[i], P->opt.lds_limit)
                          : placement<float>(M, wide[i], P->opt.lds_limit);
      lds_of[i] = pl.second;
      if (prec == 1) {
        if (pl.first == ALL_LDS) ++in_lds; else ++in_ws;
      }
      if (pl.first == ALL_LDS && !wide[i]) {
        in_lds_list.push_back(i);
        continue;
      }
      Key key{pl.first, wide[i] != 0, M.n <= 4096 ? 3 : 4};
      bool found = false;
      for (auto& b : buckets)
        if (b.first.mode == key.mode && b.first.wide == key.wide && b.first.band == key.band) {
          b.second.push_back(i);
          found = true;
          break;
        }
      if (!found) buckets.push_back({key, std::vector<int32_t>{i}});
    }
    if (!in_lds_list.empty()) {
      // classes of LDS need in 256-byte steps (at most kLdsMax / 256 of them)
      std::stable_sort(in_lds_list.begin(), in_lds_list.end(),
                       [&](int32_t x, int32_t y) { return lds_of[x] < lds_of[y]; });
      std::vector<int32_t> cls_end;  // end index (into in_lds_list) of each class
      std::vector<double> cls_cost;
      for (size_t t = 0; t < in_lds_list.size(); ++t) {
        const int32_t q = (lds_of[in_lds_list[t]] + 255) / 256;
        if (cls_end.empty() || (lds_of[in_lds_list[t - 1]] + 255) / 256 != q) {
          cls_end.push_back(0);
          cls_cost.push_back(0.0);
        }
        cls_end.back() = static_cast<int32_t>(t + 1);
        cls_cost.back() += std::max(1.0, P->mols[in_lds_list[t]].cost);
      }
      const int32_t C = static_cast<int32_t>(cls_end.size());
      const int K = std::max(1, std::min<int>(kStreams - static_cast<int>(buckets.size()), C));
      std::vector<double> pre(C + 1, 0.0);
      for (int32_t c = 0; c < C; ++c) pre[c + 1] = pre[c] + cls_cost[c];
      // best[k][e]: least cost of splitting the first e classes into k groups
      const double INF = 1e300;
      std::vector<std::vector<double>> best(K + 1, std::vector<double>(C + 1, INF));
      std::vector<std::vector<int32_t>> from(K + 1, std::vector<int32_t>(C + 1, 0));
      best[0][0] = 0.0;
      for (int k = 1; k <= K; ++k)
        for (int32_t e = 1; e <= C; ++e) {
          const double alloc = static_cast<double>(lds_of[in_lds_list[cls_end[e - 1] - 1]]);
          for (int32_t b = k - 1; b < e; ++b) {
            if (best[k - 1][b] >= INF) continue;
            const double c = best[k - 1][b] + alloc * (pre[e] - pre[b]);
            if (c < best[k][e]) {
              best[k][e] = c;
              from[k][e] = b;
            }
          }
        }
      int kb = 1;
      for (int k = 2; k <= K; ++k)
        if (best[k][C] < best[kb][C]) kb = k;
      std::vector<int32_t> cut{C};
      for (int k = kb, e = C; k > 0; --k) {
        e = from[k][e];
        cut.push_back(e);
      }
      std::reverse(cut.begin(), cut.end());  // 0 = cut[0] < ... < cut[kb] = C (class indices)
      for (int k = kb - 1; k >= 0; --k) {     // largest first
        const int32_t t0 = cut[k] == 0 ? 0 : cls_end[cut[k] - 1], t1 = cls_end[cut[k + 1] - 1];
        const int mx = lds_of[in_lds_list[t1 - 1]];
        const int band = mx <= 8192 ? 0 : mx <= 24576 ? 1 : mx <= 65536 ? 2 : 3;
        std::vector<int32_t> mem(in_lds_list.begin() + t0, in_lds_list.begin() + t1);
        std::stable_sort(mem.begin(), mem.end(), [&](int32_t x, int32_t y) {
          return static_cast<int64_t>(desc[x].n_up) + desc[x].n_l + desc[x].n >
                 static_cast<int64_t>(desc[y].n_up) + desc[y].n_l + desc[y].n;
        });
        buckets.push_back({Key{ALL_LDS, false, band}, mem});
      }
    }
    if (buckets.size() > static_cast<size_t>(kMaxGroups)) return fail(ILVES_ERR_ARG, "internal: too many launch groups");
    const int32_t* band_block = P->band_block;
    const int cap = P->opt.block_threads > 0 ? P->opt.block_threads : 1024;
    for (auto& b : buckets) {
      Group g;
      g.mode = b.first.mode;
      g.wide = b.first.wide;
      // molecules outside LDS run with 512 or 1024 threads whatever the cap
      g.block = kernel_block(g.mode, g.wide, std::min(band_block[b.first.band], cap));
      int mx = 0;
      for (int32_t i : b.second) mx = std::max(mx, lds_of[i]);
      g.lds_bytes = mx;
      g.first = static_cast<int32_t>(lists.size());
      g.count = static_cast<int32_t>(b.second.size());
      g.counter = prec * kMaxGroups + static_cast<int32_t>(P->groups[prec].size());
      g.grid = g.count;  // refined from the occupancy once the kernels are known
      for (int32_t i : b.second) g.work += static_cast<int64_t>(desc[i].n) + desc[i].n_up + desc[i].n_l;
      lists.insert(lists.end(), b.second.begin(), b.second.end());
      P->groups[prec].push_back(g);
    }
    // streams: longest processing time first -- each group, by decreasing
    // work, joins the stream with the least work so far (launch order is
    // the group order, so within a stream larger groups go first)
    std::vector<Group>& gs = P->groups[prec];
    std::stable_sort(gs.begin(), gs.end(), [](const Group& a, const Group& b) { return a.work > b.work; });
    int64_t load[kStreams] = {};
    for (Group& g : gs) {
      int best = 0;
      for (int i = 1; i < kStreams; ++i)
        if (load[i] < load[best]) best = i;
      g.stream = best;
      load[best] += g.work;
    }
    // the group of the smallest molecules runs last on the stream of the
    // group of the largest: started beside the large trees it takes CUs
    // that lengthen their critical path, chained behind them its many
    // short molecules fill the CUs the trees release as they finish (the
    // same shortest-last rule as the order inside each group)
    if (gs.size() >= 3) {
      size_t big = 0, small = 0;
      for (size_t i = 1; i < gs.size(); ++i) {
        if (gs[i].lds_bytes > gs[big].lds_bytes) big = i;
        if (gs[i].lds_bytes < gs[small].lds_bytes) small = i;
      }
      if (big != small) {
        Group sg = gs[small];
        load[sg.stream] -= sg.work;
        sg.stream = gs[big].stream;
        load[sg.stream] += sg.work;
        gs.erase(gs.begin() + static_cast<std::ptrdiff_t>(small));
        if (small < big) --big;
        gs.insert(gs.begin() + static_cast<std::ptrdiff_t>(big + 1), sg);
      }
    }
    auto least_loaded = [&]() {
      int least = 0;
      for (int i = 1; i < kStreams; ++i)
        if (load[i] < load[least]) least = i;
      return least;
    };
    // split molecules (every launch of them on one stream), then the small ones
    int64_t split_work = 0;
    for (size_t i = nm; i < plans.size(); ++i) split_work += static_cast<int64_t>(plans[i]->n) + plans[i]->n_up + plans[i]->n_l;
    P->split_stream[prec] = least_loaded();
    load[P->split_stream[prec]] += split_work;
    P->small_stream = least_loaded();
  }
  // row chunks of the feature passes, narrow molecules then wide ones
  std::vector<int32_t> chunks;
  for (int wdt = 0; wdt < 2; ++wdt) {
    P->chunk_first[wdt] = static_cast<int32_t>(chunks.size() / 2);
    for (int32_t i : ord)
      if (wide[i] == wdt)
        for (int32_t r0 = 0; r0 < P->mols[i].n; r0 += ilves_ws::kChunk) {
          chunks.push_back(i);
          chunks.push_back(r0);
        }
    P->chunk_count[wdt] = static_cast<int32_t>(chunks.size() / 2) - P->chunk_first[wdt];
  }
  if (chunks.empty()) chunks.resize(2, 0);
  if (pool.empty()) pool.resize(16, 0);
  std::vector<unsigned char> blob;
  const size_t o_desc = push_array(blob, desc);
  const size_t o_pool = push_array(blob, pool);
  const size_t o_coef = push_array(blob, coef);
  const size_t o_gcoef = push_array(blob, gcoef);
  const size_t o_gra = push_array(blob, gra);
  const size_t o_grb = push_array(blob, grb);
  const size_t o_ra = push_array(blob, ra);
  const size_t o_rb = push_array(blob, rb);
  const size_t o_cid = push_array(blob, cid);
  const size_t o_d2 = push_array(blob, d2);
  const size_t o_atom = push_array(blob, atom_gid);
  const size_t o_incp = push_array(blob, inc_ptr);
  const size_t o_inc = push_array(blob, inc);
  const size_t o_lists = push_array(blob, lists);
  const size_t o_chunks = push_array(blob, chunks);
  const size_t o_small = push_array(blob, smalls);
  if (sparts.empty()) sparts.resize(1);
  if (seprows.empty()) seprows.resize(1);
  if (sadj.empty()) sadj.resize(2, 0);
  if (bsep.empty()) bsep.resize(1, 0);
  if (ext_ptr.empty()) ext_ptr.resize(1, 0);
  if (ext_rec.empty()) ext_rec.resize(1, 0);
  if (ext_coef.empty()) ext_coef.resize(1, 0);
  const size_t o_sparts = push_array(blob, sparts);
  const size_t o_seprows = push_array(blob, seprows);
  const size_t o_sadj = push_array(blob, sadj);
  const size_t o_bsep = push_array(blob, bsep);
  const size_t o_extp = push_array(blob, ext_ptr);
  const size_t o_extr = push_array(blob, ext_rec);
  const size_t o_extc = push_array(blob, ext_coef);
  // per precision: the parts of the split molecules grouped by placement (the
  // order the split launches take them in, one range per launch, so that
  // molecules of different placements do not cut a launch into pieces)
  std::vector<int32_t> split_order[2];
  for (int prec = 0; prec < 2; ++prec)
    for (int mode : {ALL_LDS, PAIRS_GLOBAL, VALUES_LDS})
      for (size_t si = 0; si < P->splits.size(); ++si)
        if (P->split_mode[prec][si] == mode)
          for (size_t g = 0; g < P->splits[si].parts.size(); ++g)
            split_order[prec].push_back(P->split_first[si] + static_cast<int32_t>(g));
  const size_t o_sord0 = push_array(blob, split_order[0]);
  const size_t o_sord1 = push_array(blob, split_order[1]);
  blob.resize(blob.size() + 256);

  HIP_TRY(hipMalloc(&P->d_buf, blob.size()));
  HIP_TRY(hipMemcpy(P->d_buf, blob.data(), blob.size(), hipMemcpyHostToDevice));
  P->buf_bytes = blob.size();
  unsigned char* b = static_cast<unsigned char*>(P->d_buf);
  P->dp.mol = reinterpret_cast<const MolDesc*>(b + o_desc);
  P->dp.ix = b + o_pool;
  P->dp.coef = reinterpret_cast<const int32_t*>(b + o_coef);
  P->dp.gcoef = reinterpret_cast<const int32_t*>(b + o_gcoef);
  P->dp.ga = reinterpret_cast<const int32_t*>(b + o_gra);
  P->dp.gb = reinterpret_cast<const int32_t*>(b + o_grb);
  P->dp.ra = reinterpret_cast<const int32_t*>(b + o_ra);
  P->dp.rb = reinterpret_cast<const int32_t*>(b + o_rb);
  P->dp.cid = reinterpret_cast<const int32_t*>(b + o_cid);
  P->dp.d2 = reinterpret_cast<const double*>(b + o_d2);
  P->dp.atom_gid = reinterpret_cast<const int32_t*>(b + o_atom);
  P->dp.inc_ptr = reinterpret_cast<const int32_t*>(b + o_incp);
  P->dp.inc = reinterpret_cast<const int32_t*>(b + o_inc);
  P->d_lists = reinterpret_cast<int32_t*>(b + o_lists);
  P->d_chunks = reinterpret_cast<const int2*>(b + o_chunks);
  P->d_small = reinterpret_cast<const SmallMol*>(b + o_small);
  P->dp.split = reinterpret_cast<const SplitPart*>(b + o_sparts);
  P->d_split_order[0] = reinterpret_cast<const int32_t*>(b + o_sord0);
  P->d_split_order[1] = reinterpret_cast<const int32_t*>(b + o_sord1);
  P->dp.sep = reinterpret_cast<const SepRow*>(b + o_seprows);
  P->dp.sadj = reinterpret_cast<const int32_t*>(b + o_sadj);
  P->dp.bsep = reinterpret_cast<const int32_t*>(b + o_bsep);
  P->dp.ext_ptr = reinterpret_cast<const int32_t*>(b + o_extp);
  P->dp.ext_rec = reinterpret_cast<const int64_t*>(b + o_extr);
  P->dp.ext_coef = reinterpret_cast<const int32_t*>(b + o_extc);
  P->n_small = static_cast<int32_t>(smalls.size());
  if (ws > 0) {
    HIP_TRY(hipMalloc(&P->d_ws, ws));
    HIP_TRY(hipMemset(P->d_ws, 0, ws));  // barrier counters of split molecules start at zero
    P->ws_bytes = ws;
  }
  P->stats[0] = nm;
  P->stats[1] = ncon;
  P->stats[2] = natoms;
  P->stats[3] = nslots;
  P->stats[4] = fill;
  P->stats[5] = work;
  P->stats[6] = maxlev;
  P->stats[7] = sumlev;
  P->stats[8] = in_lds;
  P->stats[9] = in_ws;
  P->stats[10] = static_cast<int64_t>(ws);
  P->stats[11] = static_cast<int64_t>(blob.size());
  P->stats[12] = static_cast<int64_t>(P->splits.size());
  P->stats[13] = n_parts;
  P->stats[14] = max_sep;
  P->stats[15] = std::count(P->split_mode[0].begin(), P->split_mode[0].end(), static_cast<int>(VALUES_LDS));
  P->stats[16] = std::count(P->split_mode[1].begin(), P->split_mode[1].end(), static_cast<int>(PAIRS_GLOBAL));
  int64_t shared = 0;  // levels of the parts that share items over several lanes
  for (const auto& sp : P->splits)
    for (const auto& M : sp.parts)
      for (int32_t h = 0; h < M.n_levels; ++h) {
        int32_t lf, lb;
        level_lanes(M, h, lf, lb);
        if (lf > 0 || lb > 0) ++shared;
      }
  P->stats[17] = shared;
  return ILVES_OK;
}

// Kernel attributes and persistent grid sizes of the launch groups.
ilves_status_t finalize_groups(ilves_plan* P) {
  for (int prec = 0; prec < 2; ++prec) {
    int lds_top = 0;
    for (const Group& g : P->groups[prec]) lds_top = std::max(lds_top, g.lds_bytes);
    for (Group& g : P->groups[prec]) {
      g.heavy = false;
      const void* k = reinterpret_cast<const void*>(pick_kernel(prec == 1, g.mode, g.wide, g.block));
      // the attribute is per kernel and process-wide: always raise it to the
      // largest size any plan may use, never lower it
      if (g.lds_bytes > 0) HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax));
      int per_cu = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, g.block, static_cast<size_t>(g.lds_bytes)));
      if (per_cu < 1) return fail(ILVES_ERR_HIP, "a solve kernel cannot be resident on a compute unit");
      // The group of the largest trees, one workgroup per CU by LDS, has its
      // CU to itself when no group running beside it (on another stream)
      // fits in the LDS it leaves; the group chained behind it runs after it.
      // It then runs 1024 threads whatever the tuning (not above the plan's
      // cap on threads per workgroup), which halves its passes over the rows
      // (set-up, residual, outputs).  Otherwise, or should that kernel not
      // fit, the 512-thread wide-batch kernel (four row neighbours per batch)
      // takes it.  Other one-per-CU groups keep the lean kernel: a CU holding
      // one of their workgroups has LDS left for smaller molecules, which
      // extra registers would keep out.
      bool alone = true;
      for (const Group& o : P->groups[prec])
        if (o.stream != g.stream && o.lds_bytes + g.lds_bytes <= kCuLds) alone = false;
      if (per_cu == 1 && g.lds_bytes == lds_top && g.mode == ALL_LDS && !g.wide) {
        int per_cu_t = 0;
        if (alone && (P->opt.block_threads <= 0 || P->opt.block_threads >= 1024)) {
          const void* kt = reinterpret_cast<const void*>(pick_kernel(prec == 1, g.mode, g.wide, 1024));
          HIP_TRY(hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax));
          HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_t, kt, 1024, static_cast<size_t>(g.lds_bytes)));
        }
        if (per_cu_t >= 1) {
          g.block = 1024;
          per_cu = per_cu_t;
        } else if (g.block == 512) {
          const void* kh = reinterpret_cast<const void*>(pick_kernel(prec == 1, g.mode, g.wide, g.block, true));
          HIP_TRY(hipFuncSetAttribute(kh, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax));
          int per_cu_h = 0;
          HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_h, kh, g.block, static_cast<size_t>(g.lds_bytes)));
          if (per_cu_h >= 1) g.heavy = true;
        }
      }
      g.grid = static_cast<int32_t>(std::min<int64_t>(g.count, static_cast<int64_t>(per_cu) * P->n_cu));
    }
  }
  // split molecules: launches of whole molecules whose parts can all be
  // resident at once (the barriers of a molecule wait for all its parts)
  for (int prec = 0; prec < 2; ++prec) {
    P->split_launch[prec].clear();
    if (P->splits.empty()) continue;
    int32_t pos = 0;  // position in the precision's part order (d_split_order)
    for (int mode : {ALL_LDS, PAIRS_GLOBAL, VALUES_LDS}) {
    const void* k = reinterpret_cast<const void*>(pick_split(prec == 1, mode));
    HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax));
    auto capacity = [&](int lds, int64_t& cap) -> ilves_status_t {
      int per_cu = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kSplitBlock, static_cast<size_t>(lds)));
      cap = static_cast<int64_t>(per_cu) * P->n_cu;
      return ILVES_OK;
    };
    SplitLaunch cur;
    cur.stream = P->split_stream[prec];
    cur.mode = mode;
    for (size_t si = 0; si < P->splits.size(); ++si) {
      if (P->split_mode[prec][si] != mode) continue;
      const int32_t first = pos;
      const int32_t G = static_cast<int32_t>(P->splits[si].parts.size());
      pos += G;
      int lds = 0;
      for (int32_t g = 0; g < G; ++g) lds = std::max(lds, P->split_lds[prec][P->split_first[si] + g]);
      int64_t cap_alone = 0, cap_joined = 0;
      ilves_status_t st = capacity(lds, cap_alone);
      if (st != ILVES_OK) return st;
      if (cap_alone < G) return fail(ILVES_ERR_UNSUPPORTED, "a split molecule has more parts than can be resident");
      st = capacity(std::max(lds, cur.lds_bytes), cap_joined);
      if (st != ILVES_OK) return st;
      if (cur.count > 0 && cur.count + G > cap_joined) {
        P->split_launch[prec].push_back(cur);
        cur.first = first;
        cur.count = 0;
        cur.lds_bytes = 0;
      }
      if (cur.count == 0) cur.first = first;
      cur.count += G;
      cur.lds_bytes = std::max(cur.lds_bytes, lds);
    }
    if (cur.count > 0) P->split_launch[prec].push_back(cur);
    }
  }
  return ILVES_OK;
}

void release_device_plan(ilves_plan* P) {
  if (P->d_buf) (void)hipFree(P->d_buf);
  if (P->d_ws) (void)hipFree(P->d_ws);
  P->d_buf = nullptr;
  P->d_ws = nullptr;
  P->dp = DevPlan{};
  P->d_lists = nullptr;
  P->d_chunks = nullptr;
  P->d_small = nullptr;
  P->n_small = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

void ilves_default_options(ilves_options_t* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = ILVES_PREC_FP64;
  opt->variant = ILVES_VARIANT_NEWTON;
  opt->max_iter = 0;
  opt->warm_start = ILVES_WARM_ZERO;
  opt->block_threads = 0;
  opt->lds_limit = 0;
  opt->ordering = 0;
}

const char* ilves_version(void) { return "ilves-mi355x 0.1 (gfx950)"; }

const char* ilves_last_error(void) { return g_last_error.c_str(); }

const char* ilves_status_string(ilves_status_t s) {
  switch (s) {
    case ILVES_OK: return "ok";
    case ILVES_ERR_ARG: return "invalid argument";
    case ILVES_ERR_TOPOLOGY: return "invalid topology";
    case ILVES_ERR_HIP: return "HIP runtime error";
    case ILVES_ERR_NOMEM: return "out of memory";
    case ILVES_ERR_SINGULAR: return "singular Newton matrix";
    case ILVES_ERR_NOT_CONVERGED: return "not converged";
    case ILVES_ERR_NONFINITE: return "non-finite values";
    case ILVES_ERR_UNSUPPORTED: return "unsupported option";
    case ILVES_ERR_TIMEOUT: return "workgroups of a split molecule did not meet";
  }
  return "unknown status";
}

ilves_status_t ilves_plan_create(int32_t n_atoms, int32_t n_constraints, const int32_t* pairs, const double* d,
                                 const ilves_options_t* opt, ilves_plan_t* out) {
  if (!out) return fail(ILVES_ERR_ARG, "out must not be NULL");
  *out = nullptr;
  if (n_atoms <= 0 || n_constraints < 0) return fail(ILVES_ERR_ARG, "sizes must be positive");
  std::string msg = ilves::validate_topology(n_atoms, n_constraints, pairs, d);
  if (!msg.empty()) return fail(ILVES_ERR_TOPOLOGY, msg);
  std::unique_ptr<ilves_plan> P(new (std::nothrow) ilves_plan());
  if (!P) return fail(ILVES_ERR_NOMEM, "host allocation failed");
  if (opt) P->opt = *opt; else ilves_default_options(&P->opt);
  if (P->opt.lds_limit <= 0 || P->opt.lds_limit > kLdsMax) P->opt.lds_limit = kLdsMax;
  if (P->opt.block_threads != 0 && P->opt.block_threads != 64 && P->opt.block_threads != 128 &&
      P->opt.block_threads != 256 && P->opt.block_threads != 512 && P->opt.block_threads != 1024)
    return fail(ILVES_ERR_ARG, "block_threads must be 0, 64, 128, 256, 512 or 1024");
  P->n_atoms = n_atoms;
  P->n_con = n_constraints;
  HIP_TRY(hipGetDevice(&P->device));
  std::vector<int32_t> free_atoms;
  std::vector<std::vector<int32_t>> mols = ilves::split_molecules(n_atoms, n_constraints, pairs, free_atoms);
  ilves::PlanOptions po;
  po.ordering = P->opt.ordering;
  P->mols.reserve(mols.size());
  // molecules above split_rows constraints are split across workgroups
  // when every part's factor values then fit in LDS with 16-bit indices
  const int32_t split_rows = P->opt.split_rows == 0 ? 4096 : P->opt.split_rows;
  const int32_t part_rows = P->opt.split_part_rows;  // <= 0: automatic
  try {
    for (const auto& c : mols) P->mols.push_back(ilves::plan_molecule(c, pairs, d, po));
    for (size_t i = 0; i < mols.size(); ++i) {
      if (split_rows < 0 || static_cast<int32_t>(mols[i].size()) <= split_rows) continue;
      ilves::SplitPlan sp;
      if (!ilves::plan_split_auto(mols[i], pairs, d, po, part_rows, sp)) continue;
      bool fits = true;
      int32_t ew_total = 0;
      for (const auto& M : sp.parts) ew_total += (M.n - M.n_int) * (M.n - M.n_int + 1);
      for (const auto& M : sp.parts) {
        const int32_t nb = M.n - M.n_int;
        const bool wide = static_cast<int64_t>(M.n_up) + M.n_l >= 65535 || M.n >= 65535 || M.n_upd >= 65535;
        if (wide || static_cast<int64_t>(align16(value_bytes<double>(M.n, M.n_up, M.n_l))) +
                            split_lds_bytes(sp.m, nb, ew_total, static_cast<int32_t>(sp.sadj_col.size())) > kLdsMax)
          fits = false;
      }
      if (!fits) continue;
      P->splits.push_back(std::move(sp));
      P->split_mol.push_back(static_cast<int32_t>(i));
    }
  } catch (const std::bad_alloc&) {
    return fail(ILVES_ERR_NOMEM, "host allocation failed while planning");
  }
  HIP_TRY(hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, P->device));
  ilves_status_t st = build_device_plan(P.get());
  if (st != ILVES_OK) return st;
  st = finalize_groups(P.get());
  if (st != ILVES_OK) return st;
  P->n_free = static_cast<int32_t>(free_atoms.size());
  if (P->n_free > 0) {
    HIP_TRY(hipMalloc(&P->d_free, free_atoms.size() * sizeof(int32_t)));
    HIP_TRY(hipMemcpy(P->d_free, free_atoms.data(), free_atoms.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMalloc(&P->d_counters, sizeof(int32_t) * 2 * kMaxGroups));
  HIP_TRY(hipMemset(P->d_counters, 0, sizeof(int32_t) * 2 * kMaxGroups));
  for (int i = 0; i < kStreams; ++i) {
    HIP_TRY(hipStreamCreateWithFlags(&P->streams[i], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&P->ev_join[i], hipEventDisableTiming));
  }
  HIP_TRY(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
  *out = P.release();
  return ILVES_OK;
}

ilves_status_t ilves_plan_destroy(ilves_plan_t P) {
  if (!P) return ILVES_OK;
  for (int i = 0; i < kStreams; ++i) {
    if (P->streams[i]) (void)hipStreamDestroy(P->streams[i]);
    if (P->ev_join[i]) (void)hipEventDestroy(P->ev_join[i]);
  }
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  release_device_plan(P);
  if (P->d_free) (void)hipFree(P->d_free);
  if (P->d_counters) (void)hipFree(P->d_counters);
  if (P->d_mlp) (void)hipFree(P->d_mlp);
  if (P->d_feat) (void)hipFree(P->d_feat);
  if (P->d_w) (void)hipFree(P->d_w);
  (void)hipGetLastError();  // the codes above are ignored: leave no error state behind
  delete P;
  return ILVES_OK;
}

ilves_status_t ilves_perturb_normal(const double* r, int32_t n_atoms, double sigma, uint64_t seed,
                                    const uint64_t* step, double* r_u, void* hip_stream) {
  if (n_atoms < 0) return fail(ILVES_ERR_ARG, "n_atoms must be >= 0");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(ILVES_ERR_ARG, "sigma must be finite and >= 0");
  if (n_atoms == 0) return ILVES_OK;
  if (!r || !r_u || !step) return fail(ILVES_ERR_ARG, "null argument");
  const hipError_t e = ilves_in::launch_perturb(r, n_atoms, sigma, seed, step, r_u, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(ILVES_ERR_HIP, std::string("perturb kernel: ") + hipGetErrorString(e));
  return ILVES_OK;
}

ilves_status_t ilves_counter_add(uint64_t* counter, uint64_t delta, void* hip_stream) {
  if (!counter) return fail(ILVES_ERR_ARG, "null argument");
  const hipError_t e = ilves_in::launch_counter_add(counter, delta, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(ILVES_ERR_HIP, std::string("counter kernel: ") + hipGetErrorString(e));
  return ILVES_OK;
}

ilves_status_t ilves_md_kick_drift(const double* r, double* v, const double* f, const double* mass, double h,
                                   int32_t n_atoms, double* r_u, void* hip_stream) {
  if (n_atoms < 0 || !(h > 0.0) || !std::isfinite(h)) return fail(ILVES_ERR_ARG, "need n_atoms >= 0 and h > 0");
  if (n_atoms == 0) return ILVES_OK;
  if (!r || !v || !f || !mass || !r_u) return fail(ILVES_ERR_ARG, "null argument");
  const hipError_t e = ilves_md::launch_kick_drift(r, v, f, mass, h, n_atoms, r_u, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(ILVES_ERR_HIP, std::string("kick/drift kernel: ") + hipGetErrorString(e));
  return ILVES_OK;
}

ilves_status_t ilves_md_finish(double* r, const double* r_new, double h, int32_t n_atoms, double* v,
                               void* hip_stream) {
  if (n_atoms < 0 || !(h > 0.0) || !std::isfinite(h)) return fail(ILVES_ERR_ARG, "need n_atoms >= 0 and h > 0");
  if (n_atoms == 0) return ILVES_OK;
  if (!r || !r_new || !v) return fail(ILVES_ERR_ARG, "null argument");
  const hipError_t e = ilves_md::launch_finish(r, r_new, h, n_atoms, v, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(ILVES_ERR_HIP, std::string("finish kernel: ") + hipGetErrorString(e));
  return ILVES_OK;
}

ilves_status_t ilves_plan_get_tuning(ilves_plan_t P, ilves_tuning_t* t) {
  if (!P || !t) return fail(ILVES_ERR_ARG, "null argument");
  std::memset(t, 0, sizeof(*t));
  for (int b = 0; b < 5; ++b) t->band_block[b] = P->band_block[b];
  t->lds_limit = P->opt.lds_limit;
  return ILVES_OK;
}

ilves_status_t ilves_plan_tune(ilves_plan_t P, const ilves_tuning_t* t) {
  if (!P || !t) return fail(ILVES_ERR_ARG, "null argument");
  for (int b = 0; b < 5; ++b) {
    const int v = t->band_block[b];
    if (v != 64 && v != 128 && v != 256 && v != 512 && v != 1024)
      return fail(ILVES_ERR_ARG, "band block sizes must be 64, 128, 256, 512 or 1024");
  }
  if (t->lds_limit < 0) return fail(ILVES_ERR_ARG, "lds_limit must be >= 0");
  HIP_TRY(hipDeviceSynchronize());
  for (int b = 0; b < 5; ++b) P->band_block[b] = t->band_block[b];
  P->opt.lds_limit = (t->lds_limit <= 0 || t->lds_limit > kLdsMax) ? kLdsMax : t->lds_limit;
  release_device_plan(P);
  ilves_status_t st = build_device_plan(P);
  if (st != ILVES_OK) return st;
  return finalize_groups(P);
}

int32_t ilves_plan_num_molecules(ilves_plan_t P) { return P ? static_cast<int32_t>(P->mols.size()) : -1; }

ilves_status_t ilves_plan_set_wait_limit(ilves_plan_t P, int32_t polls) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  if (polls < 0) return fail(ILVES_ERR_ARG, "polls must be >= 0");
  P->wait_limit = polls;
  return ILVES_OK;
}

ilves_status_t ilves_plan_reset_barriers(ilves_plan_t P) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device) return fail(ILVES_ERR_ARG, "plan was created on another device");
  HIP_TRY(hipDeviceSynchronize());
  for (int64_t xch : P->split_xch) HIP_TRY(hipMemset(P->d_ws + xch, 0, 64));
  HIP_TRY(hipDeviceSynchronize());
  return ILVES_OK;
}

ilves_status_t ilves_plan_stats(ilves_plan_t P, int64_t* stats) {
  if (!P || !stats) return fail(ILVES_ERR_ARG, "plan and stats must not be NULL");
  std::memcpy(stats, P->stats, sizeof(P->stats));
  return ILVES_OK;
}

ilves_status_t ilves_plan_molecules(ilves_plan_t P, int32_t* n_con, int32_t* n_atoms, int32_t* n_levels,
                                    int32_t* first_constraint) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  for (size_t i = 0; i < P->mols.size(); ++i) {
    const auto& M = P->mols[i];
    if (n_con) n_con[i] = M.n;
    if (n_atoms) n_atoms[i] = M.s;
    if (n_levels) n_levels[i] = M.n_levels;
    if (first_constraint) first_constraint[i] = *std::min_element(M.cid.begin(), M.cid.end());
  }
  return ILVES_OK;
}

}  // extern "C"

namespace {

ilves_status_t check_solve_args(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                                int32_t precision, int32_t variant, double* r_out, double* lambda, int32_t* iters,
                                int32_t* status) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  if (!r || !r_u || !mass || !r_out) return fail(ILVES_ERR_ARG, "position and mass pointers must not be NULL");
  if (P->n_con > 0 && (!lambda || !iters || !status)) return fail(ILVES_ERR_ARG, "lambda/iters/status must not be NULL");
  if (!(tol >= 0.0)) return fail(ILVES_ERR_ARG, "tol must be >= 0");
  if (precision != ILVES_PREC_FP64 && precision != ILVES_PREC_MIXED) return fail(ILVES_ERR_ARG, "bad precision");
  if (variant != ILVES_VARIANT_NEWTON && variant != ILVES_VARIANT_CHORD) return fail(ILVES_ERR_ARG, "bad variant");
  if (r_out == r || r_out == r_u) return fail(ILVES_ERR_ARG, "r_out must not alias r or r_u");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device) return fail(ILVES_ERR_ARG, "plan was created on another device");
  return ILVES_OK;
}

// features of every row into the plan's buffers (or the given ones)
ilves_status_t run_features(ilves_plan_t P, const double* r, const double* r_u, const double* mass, float* feat,
                            float* w, hipStream_t stream) {
  for (int wdt = 0; wdt < 2; ++wdt) {
    hipError_t e = ilves_ws::launch_features(P->dp, P->d_chunks + P->chunk_first[wdt], P->chunk_count[wdt], wdt == 1,
                                             r, r_u, mass, P->n_atoms, P->d_ws, feat, w, stream);
    if (e != hipSuccess) return fail(ILVES_ERR_HIP, std::string("features kernel: ") + hipGetErrorString(e));
  }
  return ILVES_OK;
}

ilves_status_t solve_impl(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                          int32_t precision, int32_t variant, int32_t warm, int32_t max_iter, double* r_out,
                          double* lambda, int32_t* iters, int32_t* status, int32_t* fallback, hipStream_t stream,
                          int32_t project = 0, double* hist = nullptr, int32_t hist_len = 0) {
  // an error left by an earlier, unrelated runtime call (already returned to
  // its caller, or ignored) must not be reported as this solve's launch error
  (void)hipGetLastError();
  SolveArgs A;
  A.hist = hist_len > 0 ? hist : nullptr;
  A.hist_len = hist_len > 0 ? hist_len : 0;
  A.r = r;
  A.r_u = r_u;
  A.mass = mass;
  A.r_out = r_out;
  A.lambda = lambda;
  A.iters = iters;
  A.status = status;
  A.fallback = fallback;
  A.ws = P->d_ws;
  A.tol = tol;
  A.n_atoms = P->n_atoms;
  A.max_iter = max_iter > 0 ? max_iter
                            : (precision == ILVES_PREC_FP64 && variant == ILVES_VARIANT_NEWTON ? 20 : 40);
  A.warm = warm;
  A.chord = variant == ILVES_VARIANT_CHORD ? 1 : 0;
  A.wait_limit = P->wait_limit;
  A.project = project;
  if (P->n_free > 0) {
    const int tb = 256;
    hipLaunchKernelGGL(copy_free_atoms, dim3((P->n_free + tb - 1) / tb), dim3(tb), 0, stream, P->d_free, P->n_free,
                       P->n_atoms, r_u, r_out);
    HIP_TRY(hipGetLastError());
  }
  const std::vector<Group>& groups = P->groups[precision == ILVES_PREC_MIXED ? 1 : 0];
  if (groups.empty() && P->n_small == 0 && P->splits.empty()) return ILVES_OK;
  // fork: the groups run concurrently on the plan's streams, joined back
  // into the caller's stream (also valid under graph capture)
  int32_t* counters = P->d_counters + (precision == ILVES_PREC_MIXED ? kMaxGroups : 0);
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(kMaxGroups), 0, stream, counters, kMaxGroups);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(P->ev_fork, stream));
  const int pr = precision == ILVES_PREC_MIXED ? 1 : 0;
  int ns = P->n_small > 0 ? P->small_stream + 1 : 1;
  for (const Group& g : groups) ns = std::max(ns, g.stream + 1);
  for (const SplitLaunch& l : P->split_launch[pr]) ns = std::max(ns, l.stream + 1);
  for (int i = 0; i < ns; ++i) HIP_TRY(hipStreamWaitEvent(P->streams[i], P->ev_fork, 0));
  // split molecules first: their parts wait for each other, so they should
  // be dispatched before the persistent groups fill the device
  for (const SplitLaunch& l : P->split_launch[pr]) {
    KernelFn k = pick_split(pr == 1, l.mode);
    DevPlan dp = P->dp;
    const int32_t* list = P->d_split_order[pr] + l.first;
    int32_t count = l.count;
    int32_t* counter = nullptr;
    SolveArgs a = A;
    void* args[] = {&dp, &list, &count, &counter, &a};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(l.count), dim3(kSplitBlock), args,
                            static_cast<size_t>(l.lds_bytes), P->streams[l.stream]));
  }
  // the group of the largest trees (and the group chained behind it) runs on
  // the caller's stream: its launch follows the counter reset in the same
  // queue, while the forked streams first wait for the fork event, so its
  // workgroups take whole CUs before the other groups spread over them
  // (with every group forked, eager launches left that to the order in
  // which the hardware serves the queues).  Not with split molecules: their
  // parts are dispatched first.
  int origin = -1;
  if (!groups.empty() && P->split_launch[pr].empty()) {
    size_t big = 0;
    for (size_t gi = 1; gi < groups.size(); ++gi)
      if (groups[gi].lds_bytes > groups[big].lds_bytes) big = gi;
    origin = groups[big].stream;
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    KernelFn k = pick_kernel(precision == ILVES_PREC_MIXED, g.mode, g.wide, g.block, g.heavy);
    hipStream_t s = g.stream == origin ? stream : P->streams[g.stream];
    DevPlan dp = P->dp;
    const int32_t* list = P->d_lists + g.first;
    int32_t count = g.count;
    int32_t* counter = P->d_counters + g.counter;
    SolveArgs a = A;
    void* args[] = {&dp, &list, &count, &counter, &a};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(g.grid), dim3(g.block), args,
                            static_cast<size_t>(g.lds_bytes), s));
  }
  if (P->n_small > 0) {
    if (A.project)
      hipLaunchKernelGGL(small_kernel<true>, dim3((P->n_small + 255) / 256), dim3(256), 0,
                         P->streams[P->small_stream], P->d_small, P->n_small, A);
    else
      hipLaunchKernelGGL(small_kernel<false>, dim3((P->n_small + 255) / 256), dim3(256), 0,
                         P->streams[P->small_stream], P->d_small, P->n_small, A);
    HIP_TRY(hipGetLastError());
  }
  for (int i = 0; i < ns; ++i) {
    HIP_TRY(hipEventRecord(P->ev_join[i], P->streams[i]));
    HIP_TRY(hipStreamWaitEvent(stream, P->ev_join[i], 0));
  }
  return ILVES_OK;
}

ilves_status_t predict_impl(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double* lambda,
                            hipStream_t stream) {
  if (!P->d_mlp) return fail(ILVES_ERR_UNSUPPORTED, "no network loaded: call ilves_mlp_load first");
  ilves_status_t st = run_features(P, r, r_u, mass, P->d_feat, P->d_w, stream);
  if (st != ILVES_OK) return st;
  hipError_t e = ilves_ws::launch_mlp_infer(P->d_mlp, P->d_mlp + ilves_ws::N_PARAMS, P->d_feat, P->d_w, P->dp.cid,
                                            P->n_con, lambda, stream);
  if (e != hipSuccess) return fail(ILVES_ERR_HIP, std::string("network kernel: ") + hipGetErrorString(e));
  return ILVES_OK;
}

}  // namespace

extern "C" {

ilves_status_t ilves_solve_ex(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                              int32_t precision, int32_t variant, int32_t warm_start, int32_t max_iter,
                              double* r_out, double* lambda, int32_t* iters, int32_t* status, double* history,
                              int32_t history_len, void* hip_stream) {
  ilves_status_t st = check_solve_args(P, r, r_u, mass, tol, precision, variant, r_out, lambda, iters, status);
  if (st != ILVES_OK) return st;
  if (history_len < 0 || (history_len > 0 && !history)) return fail(ILVES_ERR_ARG, "bad history buffer");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  if (warm_start != ILVES_WARM_ZERO && warm_start != ILVES_WARM_CALLER && warm_start != ILVES_WARM_DECOUPLED &&
      warm_start != ILVES_WARM_MLP)
    return fail(ILVES_ERR_ARG, "bad warm_start");
  if (warm_start == ILVES_WARM_MLP && P->n_con > 0) {
    st = predict_impl(P, r, r_u, mass, lambda, stream);
    if (st != ILVES_OK) return st;
  }
  const int32_t warm = warm_start == ILVES_WARM_CALLER ? 1
                       : warm_start == ILVES_WARM_DECOUPLED ? 3
                       : (warm_start == ILVES_WARM_MLP && P->n_con > 0) ? 2 : 0;
  return solve_impl(P, r, r_u, mass, tol, precision, variant, warm, max_iter, r_out, lambda, iters, status, nullptr,
                    stream, 0, history, history_len);
}

ilves_status_t ilves_solve_learned(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                                   int32_t precision, int32_t variant, int32_t max_iter, double* r_out,
                                   double* lambda, int32_t* iters, int32_t* status, int32_t* fallback,
                                   void* hip_stream) {
  ilves_status_t st = check_solve_args(P, r, r_u, mass, tol, precision, variant, r_out, lambda, iters, status);
  if (st != ILVES_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  if (P->n_con == 0) return solve_impl(P, r, r_u, mass, tol, precision, variant, 0, max_iter, r_out, lambda, iters,
                                       status, fallback, stream);
  st = predict_impl(P, r, r_u, mass, lambda, stream);
  if (st != ILVES_OK) return st;
  return solve_impl(P, r, r_u, mass, tol, precision, variant, 2, max_iter, r_out, lambda, iters, status, fallback,
                    stream);
}

ilves_status_t ilves_project_velocities(ilves_plan_t P, const double* r, const double* v, const double* mass,
                                        double tol, int32_t precision, double* v_out, double* mu, int32_t* iters,
                                        int32_t* status, void* hip_stream) {
  ilves_status_t st = check_solve_args(P, r, v, mass, tol, precision, ILVES_VARIANT_CHORD, v_out, mu, iters, status);
  if (st != ILVES_OK) return st;
  return solve_impl(P, r, v, mass, tol, precision, ILVES_VARIANT_CHORD, 0, 0, v_out, mu, iters, status, nullptr,
                    static_cast<hipStream_t>(hip_stream), 1);
}

ilves_status_t ilves_mlp_predict(ilves_plan_t P, const double* r, const double* r_u, const double* mass,
                                 double* lambda, void* hip_stream) {
  if (!P || !r || !r_u || !mass || (P->n_con > 0 && !lambda)) return fail(ILVES_ERR_ARG, "null argument");
  if (P->n_con == 0) return ILVES_OK;
  return predict_impl(P, r, r_u, mass, lambda, static_cast<hipStream_t>(hip_stream));
}

ilves_status_t ilves_features(ilves_plan_t P, const double* r, const double* r_u, const double* mass, float* feat,
                              float* w, void* hip_stream) {
  if (!P || !r || !r_u || !mass || (P->n_con > 0 && (!feat || !w))) return fail(ILVES_ERR_ARG, "null argument");
  return run_features(P, r, r_u, mass, feat, w, static_cast<hipStream_t>(hip_stream));
}

ilves_status_t ilves_plan_row_constraints(ilves_plan_t P, int32_t* cid) {
  if (!P || (P->n_con > 0 && !cid)) return fail(ILVES_ERR_ARG, "null argument");
  int64_t off = 0;
  for (const auto& M : P->mols) {
    std::memcpy(cid + off, M.cid.data(), M.cid.size() * sizeof(int32_t));
    off += static_cast<int64_t>(M.cid.size());
  }
  return ILVES_OK;
}

int32_t ilves_mlp_param_count(void) { return ilves_ws::N_PARAMS; }
int32_t ilves_mlp_norm_count(void) { return ilves_ws::N_NORM; }

ilves_status_t ilves_mlp_load(ilves_plan_t P, const float* params, int32_t n_params, const float* norm,
                              int32_t n_norm) {
  if (!P || !params || !norm) return fail(ILVES_ERR_ARG, "null argument");
  if (n_params != ilves_ws::N_PARAMS)
    return fail(ILVES_ERR_ARG, "n_params must be ilves_mlp_param_count() = " + std::to_string(ilves_ws::N_PARAMS));
  if (n_norm != ilves_ws::N_NORM)
    return fail(ILVES_ERR_ARG, "n_norm must be ilves_mlp_norm_count() = " + std::to_string(ilves_ws::N_NORM));
  for (int i = 0; i < ilves_ws::N_PARAMS + ilves_ws::N_NORM; ++i)
    if (!std::isfinite(i < ilves_ws::N_PARAMS ? params[i] : norm[i - ilves_ws::N_PARAMS]))
      return fail(ILVES_ERR_ARG, "network parameters and normalisation must be finite");
  for (int i = 0; i < ilves_ws::N_FEAT; ++i)
    if (!(norm[ilves_ws::N_FEAT + i] > 0.0f)) return fail(ILVES_ERR_ARG, "feature scales must be positive");
  if (!P->d_mlp) HIP_TRY(hipMalloc(&P->d_mlp, sizeof(float) * (ilves_ws::N_PARAMS + ilves_ws::N_NORM)));
  if (!P->d_feat && P->n_con > 0) {
    HIP_TRY(hipMalloc(&P->d_feat, sizeof(float) * ilves_ws::N_FEAT * static_cast<size_t>(P->n_con)));
    HIP_TRY(hipMalloc(&P->d_w, sizeof(float) * static_cast<size_t>(P->n_con)));
  }
  HIP_TRY(hipMemcpy(P->d_mlp, params, sizeof(float) * ilves_ws::N_PARAMS, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P->d_mlp + ilves_ws::N_PARAMS, norm, sizeof(float) * ilves_ws::N_NORM, hipMemcpyHostToDevice));
  return ILVES_OK;
}

ilves_status_t ilves_mlp_forward_f32(const float* params, const float* x, int32_t n, float* out, void* hip_stream) {
  if (!params || (n > 0 && (!x || !out)) || n < 0) return fail(ILVES_ERR_ARG, "bad argument");
  hipError_t e = ilves_ws::launch_mlp_forward_f32(params, x, n, out, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ILVES_OK : fail(ILVES_ERR_HIP, hipGetErrorString(e));
}

int64_t ilves_mlp_grad_workspace(int32_t n) {
  return n <= 0 ? 0 : static_cast<int64_t>((n + ilves_ws::TRAIN_BS - 1) / ilves_ws::TRAIN_BS) * (ilves_ws::N_PARAMS + 1);
}

ilves_status_t ilves_mlp_grad_f32(const float* params, const float* x, const float* y, int32_t n, float* grad,
                                  float* loss, float* work, int64_t work_floats, void* hip_stream) {
  if (!params || !x || !y || !grad || !loss || !work || n <= 0) return fail(ILVES_ERR_ARG, "bad argument");
  if (work_floats < ilves_mlp_grad_workspace(n)) return fail(ILVES_ERR_ARG, "workspace too small");
  hipError_t e = ilves_ws::launch_mlp_grad_f32(params, x, y, n, grad, loss, work, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ILVES_OK : fail(ILVES_ERR_HIP, hipGetErrorString(e));
}

ilves_status_t ilves_mlp_grad_f32_static(const float* params, const float* x, const float* y, int32_t n, float* grad,
                                         float* loss, void* hip_stream) {
  static_assert(ILVES_MLP_GRAD_STATIC_MAX_SAMPLES == ilves_ws::kStaticGradBlocks * ilves_ws::TRAIN_BS,
                "header limit and device array size disagree");
  if (!params || !x || !y || !grad || !loss || n <= 0) return fail(ILVES_ERR_ARG, "bad argument");
  if (n > ILVES_MLP_GRAD_STATIC_MAX_SAMPLES)
    return fail(ILVES_ERR_ARG, "n = " + std::to_string(n) + " exceeds ILVES_MLP_GRAD_STATIC_MAX_SAMPLES (" +
                                   std::to_string(ILVES_MLP_GRAD_STATIC_MAX_SAMPLES) +
                                   "); use ilves_mlp_grad_f32 with a workspace");
  hipError_t e = ilves_ws::launch_mlp_grad_f32_static(params, x, y, n, grad, loss, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ILVES_OK : fail(ILVES_ERR_HIP, hipGetErrorString(e));
}

ilves_status_t ilves_mlp_adam_f32(float* params, const float* grad, float* m, float* v, int32_t n, float lr,
                                  float beta1, float beta2, float eps, int32_t step, void* hip_stream) {
  if (!params || !grad || !m || !v || n <= 0 || step < 1) return fail(ILVES_ERR_ARG, "bad argument");
  hipError_t e = ilves_ws::launch_mlp_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step,
                                           static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ILVES_OK : fail(ILVES_ERR_HIP, hipGetErrorString(e));
}

ilves_status_t ilves_solve(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                           double* r_out, double* lambda, int32_t* iters, int32_t* status, void* hip_stream) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  return ilves_solve_ex(P, r, r_u, mass, tol, P->opt.precision, P->opt.variant, P->opt.warm_start,
                        P->opt.max_iter, r_out, lambda, iters, status, nullptr, 0, hip_stream);
}

}  // extern "C"
