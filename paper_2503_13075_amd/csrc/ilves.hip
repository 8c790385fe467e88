// Device kernels and the C ABI of the constraint solver (gfx950 / CDNA4).
//
// Method (Supplement section 2.3 and 3 of the ILVES paper, spec sign
// convention, see include/ilves.h):
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
// pattern: A_kj = C_kj (e'_k . e_j).  Per molecule the vectors e, lambda,
// 1/m and the LU factor live in LDS when they fit (a global workspace, L2
// resident in practice, otherwise).  The LU is an up-looking factorisation
// scheduled by elimination-tree level (all entries owned by the nodes of one
// level are independent); the forward substitution is fused into it; the
// backward substitution walks the levels down.  No atomics: every value has
// one writer, so results are bitwise reproducible.
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
#include <vector>

#include "../../include/ilves.h"
#include "plan.hpp"

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
// device plan layout

struct MolDesc {
  int32_t n, s, nslots, n_levels;
  int32_t row_off;    // per-row arrays (ra, rb, d2, cid, row_nup)
  int32_t rowp_off;   // row_start, n + 1 entries
  int32_t slot_off;   // slot_col, slot_coef
  int32_t atom_off;   // atom_gid
  int32_t incp_off;   // inc_ptr, s + 1 entries
  int32_t inc_off;    // inc
  int32_t task_off;   // tasks
  int32_t upd_off;    // upd4, updd
  int32_t lvl_off;    // lvl_task and lvl_node, n_levels + 1 entries each
  int32_t node_off;   // nodes
  int64_t ws_off;     // byte offset of the molecule's arena in the workspace
};

struct DevPlan {
  const MolDesc* mol;
  const int32_t* atom_gid;
  const int32_t* inc_ptr;
  const int32_t* inc;
  const int32_t* row_start;
  const int32_t* row_nup;
  const int32_t* ra;
  const int32_t* rb;
  const double* d2;
  const int32_t* cid;
  const int32_t* slot_col;
  const int32_t* slot_coef;
  const int4* tasks;
  const int4* upd4;
  const int32_t* updd;
  const int32_t* lvl_task;
  const int32_t* lvl_node;
  const int32_t* nodes;
};

struct SolveArgs {
  const double* r;
  const double* r_u;
  const double* mass;
  double* r_out;
  double* lambda;
  int32_t* iters;
  int32_t* status;
  unsigned char* ws;
  double tol;
  int32_t n_atoms;
  int32_t max_iter;
  int32_t warm;      // 0: lambda_0 = 0, 1: read lambda
  int32_t chord;     // 0: Newton, 1: chord
};

template <typename T>
__host__ __device__ constexpr size_t arena_bytes(int32_t n, int32_t s, int32_t nslots) {
  return (static_cast<size_t>(8) * (4 * static_cast<size_t>(n) + s + 1) +
          sizeof(T) * (static_cast<size_t>(n) + nslots) + 15) & ~static_cast<size_t>(15);
}

template <typename T> __device__ inline T pivot_eps();
template <> __device__ inline double pivot_eps<double>() { return 1e-13; }
template <> __device__ inline float pivot_eps<float>() { return 1e-6f; }

// ---------------------------------------------------------------------------
// the solve kernel: one workgroup per molecule

template <typename T, bool IN_LDS, int BLOCK>
__global__ void __launch_bounds__(BLOCK) solve_kernel(const DevPlan P, const int32_t* __restrict__ mols,
                                                      const SolveArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[BLOCK / 64];
  __shared__ int32_t singular;

  const int tid = threadIdx.x;
  const int32_t m = mols[blockIdx.x];
  const MolDesc md = P.mol[m];
  const int32_t n = md.n, s = md.s;
  unsigned char* base = IN_LDS ? smem : (A.ws + md.ws_off);
  double* __restrict__ ex = reinterpret_cast<double*>(base);
  double* __restrict__ ey = ex + n;
  double* __restrict__ ez = ey + n;
  double* __restrict__ lam = ez + n;
  double* __restrict__ invm = lam + n;
  T* __restrict__ y = reinterpret_cast<T*>(invm + s + 1);
  T* __restrict__ F = y + n;

  const int32_t* __restrict__ atom_gid = P.atom_gid + md.atom_off;
  const int32_t* __restrict__ ra = P.ra + md.row_off;
  const int32_t* __restrict__ rb = P.rb + md.row_off;
  const double* __restrict__ d2 = P.d2 + md.row_off;
  const int32_t* __restrict__ cid = P.cid + md.row_off;
  const int32_t* __restrict__ row_nup = P.row_nup + md.row_off;
  const int32_t* __restrict__ row_start = P.row_start + md.rowp_off;
  const int32_t* __restrict__ slot_col = P.slot_col + md.slot_off;
  const int32_t* __restrict__ slot_coef = P.slot_coef + md.slot_off;
  const int4* __restrict__ tasks = P.tasks + md.task_off;
  const int4* __restrict__ upd4 = P.upd4 + md.upd_off;
  const int32_t* __restrict__ updd = P.updd + md.upd_off;
  const int32_t* __restrict__ lvl_task = P.lvl_task + md.lvl_off;
  const int32_t* __restrict__ lvl_node = P.lvl_node + md.lvl_off;
  const int32_t* __restrict__ nodes = P.nodes + md.node_off;
  const int32_t S = A.n_atoms;
  const double* __restrict__ rx = A.r;
  const double* __restrict__ ux = A.r_u;

  // ---- set-up: 1/m, old bond vectors, lambda_0, coordinate magnitude
  double rmax = 0.0;
  for (int32_t a = tid; a < s; a += BLOCK) {
    const int32_t g = atom_gid[a];
    invm[a] = 1.0 / A.mass[g];
    rmax = fmax(rmax, fmax(fabs(ux[g]), fmax(fabs(ux[S + g]), fabs(ux[2 * S + g]))));
  }
  if (tid == 0) {
    invm[s] = 0.0;  // fill entries point here: zero coupling
    singular = 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = rmax;
  for (int32_t k = tid; k < n; k += BLOCK) {
    const int32_t ga = atom_gid[ra[k]], gb = atom_gid[rb[k]];
    ex[k] = rx[ga] - rx[gb];
    ey[k] = rx[S + ga] - rx[S + gb];
    ez[k] = rx[2 * S + ga] - rx[2 * S + gb];
    lam[k] = A.warm ? A.lambda[cid[k]] : 0.0;
  }
  __syncthreads();
  // Rounding r' to doubles moves each output coordinate by at most
  // |r'| 2^-53, so a bond vector formed from the returned positions differs
  // from the one iterated here by at most delta = sqrt(3) rmax 2^-52.  The
  // convergence test adds the resulting bound on |g| so that the returned
  // positions themselves satisfy the tolerance.
  double gr = red[0];
#pragma unroll
  for (int w = 1; w < BLOCK / 64; ++w) gr = fmax(gr, red[w]);
  const double delta = 1.7320508075688772 * gr * 0x1.0p-52;
  const double delta2 = 0.5 * delta * delta;
  __syncthreads();

  const int32_t H = md.n_levels;

  // ---- chord: factor A(r, r) once
  if (A.chord) {
    for (int32_t k = tid; k < n; k += BLOCK) {
      const double w = invm[ra[k]] + invm[rb[k]];
      const double ekx = ex[k], eky = ey[k], ekz = ez[k];
      const int32_t q0 = row_start[k], q1 = row_start[k + 1];
      F[q0] = static_cast<T>(w * (ekx * ekx + eky * eky + ekz * ekz));
      for (int32_t q = q0 + 1; q < q1; ++q) {
        const int32_t j = slot_col[q];
        const int32_t cf = slot_coef[q];
        const double c = (cf & 1) ? -invm[cf >> 1] : invm[cf >> 1];
        F[q] = static_cast<T>(c * (ekx * ex[j] + eky * ey[j] + ekz * ez[j]));
      }
    }
    __syncthreads();
    for (int32_t h = 0; h < H; ++h) {
      for (int32_t t = lvl_task[h] + tid; t < lvl_task[h + 1]; t += BLOCK) {
        const int4 tk = tasks[t];
        if (tk.y < 0) {
          T acc = F[tk.x];
          const T a0 = acc;
          for (int32_t u = tk.z; u < tk.w; ++u) {
            const int4 q = upd4[u];
            acc -= F[q.x] * F[updd[u]] * F[q.y];
          }
          if (!(fabs(acc) > pivot_eps<T>() * fabs(a0))) singular = 1;
          F[tk.x] = T(1) / acc;
        } else {
          T au = F[tk.x], aw = F[tk.y];
          for (int32_t u = tk.z; u < tk.w; ++u) {
            const int4 q = upd4[u];
            const T dinv = F[updd[u]];
            au -= F[q.x] * dinv * F[q.y];
            aw -= F[q.z] * dinv * F[q.w];
          }
          F[tk.x] = au;
          F[tk.y] = aw;
        }
      }
      __syncthreads();
    }
  }

  int32_t it = 0;
  int32_t st = ILVES_ERR_NOT_CONVERGED;
  const bool chord_singular = A.chord && singular;
  if (chord_singular) st = ILVES_ERR_SINGULAR;
  while (!chord_singular) {
    // ---- residual at the current lambda; Newton: rebuild the matrix rows
    double vmax = 0.0;
    for (int32_t k = tid; k < n; k += BLOCK) {
      const int32_t la = ra[k], lb = rb[k];
      const int32_t ga = atom_gid[la], gb = atom_gid[lb];
      const double w = invm[la] + invm[lb];
      const double lk = lam[k] * w;
      const double ekx = ex[k], eky = ey[k], ekz = ez[k];
      double px = ux[ga] - ux[gb] - lk * ekx;
      double py = ux[S + ga] - ux[S + gb] - lk * eky;
      double pz = ux[2 * S + ga] - ux[2 * S + gb] - lk * ekz;
      const int32_t q0 = row_start[k], q1 = row_start[k + 1];
      for (int32_t q = q0 + 1; q < q1; ++q) {
        const int32_t j = slot_col[q];
        const int32_t cf = slot_coef[q];
        const double c = ((cf & 1) ? -invm[cf >> 1] : invm[cf >> 1]) * lam[j];
        px -= c * ex[j];
        py -= c * ey[j];
        pz -= c * ez[j];
      }
      const double pp = px * px + py * py + pz * pz;
      const double g = 0.5 * (pp - d2[k]);
      double rel = (fabs(g) + sqrt(pp) * delta + delta2) / d2[k];
      if (!(rel <= DBL_MAX)) rel = INFINITY;  // NaN or Inf
      vmax = fmax(vmax, rel);
      y[k] = static_cast<T>(g);
      if (!A.chord) {
        F[q0] = static_cast<T>(w * (px * ekx + py * eky + pz * ekz));
        for (int32_t q = q0 + 1; q < q1; ++q) {
          const int32_t j = slot_col[q];
          const int32_t cf = slot_coef[q];
          const double c = (cf & 1) ? -invm[cf >> 1] : invm[cf >> 1];
          F[q] = static_cast<T>(c * (px * ex[j] + py * ey[j] + pz * ez[j]));
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
    if (gmax == INFINITY) { st = ILVES_ERR_NONFINITE; break; }
    if (gmax <= A.tol) { st = ILVES_OK; break; }
    if (it >= A.max_iter) { st = ILVES_ERR_NOT_CONVERGED; break; }

    // ---- factorisation fused with the forward substitution (Newton), or
    //      the forward substitution alone (chord)
    for (int32_t h = 0; h < H; ++h) {
      for (int32_t t = lvl_task[h] + tid; t < lvl_task[h + 1]; t += BLOCK) {
        const int4 tk = tasks[t];
        if (tk.y < 0) {
          const int32_t j = -tk.y - 1;
          T yj = y[j];
          if (A.chord) {
            for (int32_t u = tk.z; u < tk.w; ++u) {
              const int4 q = upd4[u];
              yj -= F[q.x] * F[updd[u]] * y[q.z];
            }
          } else {
            T acc = F[tk.x];
            const T a0 = acc;
            for (int32_t u = tk.z; u < tk.w; ++u) {
              const int4 q = upd4[u];
              const T l = F[q.x] * F[updd[u]];
              acc -= l * F[q.y];
              yj -= l * y[q.z];
            }
            if (!(fabs(acc) > pivot_eps<T>() * fabs(a0))) singular = 1;
            F[tk.x] = T(1) / acc;
          }
          y[j] = yj;
        } else if (!A.chord) {
          T au = F[tk.x], aw = F[tk.y];
          for (int32_t u = tk.z; u < tk.w; ++u) {
            const int4 q = upd4[u];
            const T dinv = F[updd[u]];
            au -= F[q.x] * dinv * F[q.y];
            aw -= F[q.z] * dinv * F[q.w];
          }
          F[tk.x] = au;
          F[tk.y] = aw;
        }
      }
      __syncthreads();
    }
    if (singular) { st = ILVES_ERR_SINGULAR; break; }

    // ---- backward substitution and lambda update
    for (int32_t h = H - 1; h >= 0; --h) {
      for (int32_t i = lvl_node[h] + tid; i < lvl_node[h + 1]; i += BLOCK) {
        const int32_t k = nodes[i];
        const int32_t q0 = row_start[k];
        T acc = y[k];
        for (int32_t q = q0 + 1; q <= q0 + row_nup[k]; ++q) acc -= F[q] * y[slot_col[q]];
        const T z = acc * F[q0];
        y[k] = z;
        lam[k] += static_cast<double>(z);
      }
      __syncthreads();
    }
    ++it;
  }

  // ---- outputs: lambda in input order and r' = r_u - M^{-1} G(r)^T lambda
  for (int32_t k = tid; k < n; k += BLOCK) A.lambda[cid[k]] = lam[k];
  const int32_t* __restrict__ inc_ptr = P.inc_ptr + md.incp_off;
  const int32_t* __restrict__ inc = P.inc + md.inc_off;
  for (int32_t a = tid; a < s; a += BLOCK) {
    double dx = 0.0, dy = 0.0, dz = 0.0;
    for (int32_t q = inc_ptr[a]; q < inc_ptr[a + 1]; ++q) {
      const int32_t e = inc[q];
      const int32_t k = e >> 1;
      const double l = (e & 1) ? -lam[k] : lam[k];
      dx += l * ex[k];
      dy += l * ey[k];
      dz += l * ez[k];
    }
    const int32_t g = atom_gid[a];
    const double im = invm[a];
    A.r_out[g] = ux[g] - im * dx;
    A.r_out[S + g] = ux[S + g] - im * dy;
    A.r_out[2 * S + g] = ux[2 * S + g] - im * dz;
  }
  if (tid == 0) {
    A.iters[m] = it;
    A.status[m] = st;
  }
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

using KernelFn = void (*)(DevPlan, const int32_t*, SolveArgs);

template <typename T, bool L>
KernelFn pick_block(int block) {
  switch (block) {
    case 64: return solve_kernel<T, L, 64>;
    case 128: return solve_kernel<T, L, 128>;
    case 256: return solve_kernel<T, L, 256>;
    case 512: return solve_kernel<T, L, 512>;
    default: return solve_kernel<T, L, 1024>;
  }
}

KernelFn pick_kernel(bool fp32, bool lds, int block) {
  if (fp32) return lds ? pick_block<float, true>(block) : pick_block<float, false>(block);
  return lds ? pick_block<double, true>(block) : pick_block<double, false>(block);
}

constexpr int kLdsMax = 160 * 1024 - 1024;  // dynamic LDS a molecule may use
constexpr int kStreams = 4;                 // concurrent launch groups

struct Group {
  int block = 256;
  bool lds = true;
  int lds_bytes = 0;
  int32_t first = 0;  // into the device molecule-list array
  int32_t count = 0;
};

}  // namespace

// ---------------------------------------------------------------------------
// the plan object

struct ilves_plan {
  int device = 0;
  int32_t n_atoms = 0, n_con = 0;
  ilves_options_t opt{};
  std::vector<ilves::MolPlan> mols;   // host copy, in plan order
  std::vector<int32_t> order;         // launch order (largest first)
  DevPlan dp{};
  void* d_buf = nullptr;
  size_t buf_bytes = 0;
  unsigned char* d_ws = nullptr;
  size_t ws_bytes = 0;
  int32_t* d_free = nullptr;
  int32_t n_free = 0;
  int32_t* d_lists = nullptr;          // molecule lists of every group, both precisions
  std::vector<Group> groups[2];        // [0] FP64, [1] mixed
  hipStream_t streams[kStreams] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kStreams] = {};
  int64_t stats[ILVES_STAT_COUNT] = {};
};

namespace {

int auto_block(int32_t n, int32_t cap) {
  int b = n <= 64 ? 64 : n <= 256 ? 128 : n <= 1024 ? 256 : 512;
  return std::min(b, cap);
}

template <typename V>
size_t push_array(std::vector<unsigned char>& blob, const std::vector<V>& v) {
  size_t off = (blob.size() + 255) & ~static_cast<size_t>(255);
  blob.resize(off + v.size() * sizeof(V));
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(V));
  return off;
}

ilves_status_t build_device_plan(ilves_plan* P) {
  const int32_t nm = static_cast<int32_t>(P->mols.size());
  std::vector<MolDesc> desc(nm);
  std::vector<int32_t> atom_gid, inc_ptr, inc, row_start, row_nup, ra, rb, cid, slot_col, slot_coef,
      updd, lvl_task, lvl_node, nodes;
  std::vector<double> d2;
  std::vector<int4> tasks, upd4;
  int64_t fill = 0, nupd = 0, maxlev = 0, sumlev = 0, nslots = 0, natoms = 0, ncon = 0;
  size_t ws = 0;
  int64_t in_lds = 0, in_ws = 0;
  for (int32_t i = 0; i < nm; ++i) {
    const ilves::MolPlan& M = P->mols[i];
    MolDesc& D = desc[i];
    D.n = M.n;
    D.s = M.s;
    D.nslots = M.nslots;
    D.n_levels = M.n_levels;
    D.row_off = static_cast<int32_t>(ra.size());
    D.rowp_off = static_cast<int32_t>(row_start.size());
    D.slot_off = static_cast<int32_t>(slot_col.size());
    D.atom_off = static_cast<int32_t>(atom_gid.size());
    D.incp_off = static_cast<int32_t>(inc_ptr.size());
    D.inc_off = static_cast<int32_t>(inc.size());
    D.task_off = static_cast<int32_t>(tasks.size());
    D.upd_off = static_cast<int32_t>(upd4.size());
    D.lvl_off = static_cast<int32_t>(lvl_task.size());
    D.node_off = static_cast<int32_t>(nodes.size());
    atom_gid.insert(atom_gid.end(), M.atom_gid.begin(), M.atom_gid.end());
    inc_ptr.insert(inc_ptr.end(), M.inc_ptr.begin(), M.inc_ptr.end());
    inc.insert(inc.end(), M.inc.begin(), M.inc.end());
    row_start.insert(row_start.end(), M.row_start.begin(), M.row_start.end());
    row_nup.insert(row_nup.end(), M.row_nup.begin(), M.row_nup.end());
    ra.insert(ra.end(), M.ra.begin(), M.ra.end());
    rb.insert(rb.end(), M.rb.begin(), M.rb.end());
    d2.insert(d2.end(), M.d2.begin(), M.d2.end());
    cid.insert(cid.end(), M.cid.begin(), M.cid.end());
    slot_col.insert(slot_col.end(), M.slot_col.begin(), M.slot_col.end());
    slot_coef.insert(slot_coef.end(), M.slot_coef.begin(), M.slot_coef.end());
    for (const auto& t : M.tasks) tasks.push_back(make_int4(t.out0, t.out1, t.u0, t.u1));
    for (const auto& u : M.upd) {
      upd4.push_back(make_int4(u.a, u.b, u.c, u.e));
      updd.push_back(u.d);
    }
    lvl_task.insert(lvl_task.end(), M.lvl_task.begin(), M.lvl_task.end());
    lvl_node.insert(lvl_node.end(), M.lvl_node.begin(), M.lvl_node.end());
    nodes.insert(nodes.end(), M.nodes.begin(), M.nodes.end());
    const size_t a64 = arena_bytes<double>(M.n, M.s, M.nslots);
    if (static_cast<int64_t>(a64) > P->opt.lds_limit) {
      D.ws_off = static_cast<int64_t>(ws);
      ws += (a64 + 255) & ~static_cast<size_t>(255);
    } else {
      D.ws_off = -1;
    }
    fill += M.fill;
    nupd += static_cast<int64_t>(M.upd.size());
    maxlev = std::max<int64_t>(maxlev, M.n_levels);
    sumlev += M.n_levels;
    nslots += M.nslots;
    natoms += M.s;
    ncon += M.n;
  }
  // launch groups per precision: molecules sorted by FP64 arena size
  // (largest first), grouped by block size and LDS residency
  std::vector<int32_t> ord(nm);
  for (int32_t i = 0; i < nm; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    return arena_bytes<double>(desc[x].n, desc[x].s, desc[x].nslots) >
           arena_bytes<double>(desc[y].n, desc[y].s, desc[y].nslots);
  });
  P->order = ord;
  std::vector<int32_t> lists;
  for (int prec = 0; prec < 2; ++prec) {
    P->groups[prec].clear();
    // key: (lds, block); bucket the LDS size by powers of two to keep occupancy
    struct Key { bool lds; int block; int bucket; };
    std::vector<std::pair<Key, std::vector<int32_t>>> buckets;
    for (int32_t i : ord) {
      const MolDesc& D = desc[i];
      const size_t a = prec == 0 ? arena_bytes<double>(D.n, D.s, D.nslots) : arena_bytes<float>(D.n, D.s, D.nslots);
      const bool lds = static_cast<int64_t>(a) <= P->opt.lds_limit;
      if (!lds && D.ws_off < 0) return fail(ILVES_ERR_ARG, "internal: molecule without workspace");
      const int cap = P->opt.block_threads > 0 ? P->opt.block_threads : 1024;
      const int block = auto_block(D.n, cap);
      int bucket = 0;
      if (lds) {
        size_t lim = 1024;
        while (lim < a) { lim <<= 1; ++bucket; }
      }
      bool found = false;
      for (auto& b : buckets)
        if (b.first.lds == lds && b.first.block == block && b.first.bucket == bucket) {
          b.second.push_back(i);
          found = true;
          break;
        }
      if (!found) buckets.push_back({Key{lds, block, bucket}, std::vector<int32_t>{i}});
    }
    for (auto& b : buckets) {
      Group g;
      g.block = b.first.block;
      g.lds = b.first.lds;
      int mx = 0;
      for (int32_t i : b.second) {
        const MolDesc& D = desc[i];
        const size_t a = prec == 0 ? arena_bytes<double>(D.n, D.s, D.nslots) : arena_bytes<float>(D.n, D.s, D.nslots);
        mx = std::max<int>(mx, static_cast<int>(a));
      }
      g.lds_bytes = g.lds ? mx : 0;
      g.first = static_cast<int32_t>(lists.size());
      g.count = static_cast<int32_t>(b.second.size());
      lists.insert(lists.end(), b.second.begin(), b.second.end());
      P->groups[prec].push_back(g);
    }
  }
  for (int32_t i = 0; i < nm; ++i) {
    if (desc[i].ws_off < 0) ++in_lds; else ++in_ws;
  }

  std::vector<unsigned char> blob;
  const size_t o_desc = push_array(blob, desc);
  const size_t o_atom = push_array(blob, atom_gid);
  const size_t o_incp = push_array(blob, inc_ptr);
  const size_t o_inc = push_array(blob, inc);
  const size_t o_rows = push_array(blob, row_start);
  const size_t o_nup = push_array(blob, row_nup);
  const size_t o_ra = push_array(blob, ra);
  const size_t o_rb = push_array(blob, rb);
  const size_t o_d2 = push_array(blob, d2);
  const size_t o_cid = push_array(blob, cid);
  const size_t o_scol = push_array(blob, slot_col);
  const size_t o_scoef = push_array(blob, slot_coef);
  const size_t o_tasks = push_array(blob, tasks);
  const size_t o_upd4 = push_array(blob, upd4);
  const size_t o_updd = push_array(blob, updd);
  const size_t o_lt = push_array(blob, lvl_task);
  const size_t o_ln = push_array(blob, lvl_node);
  const size_t o_nodes = push_array(blob, nodes);
  const size_t o_lists = push_array(blob, lists);
  blob.resize(blob.size() + 256);

  HIP_TRY(hipMalloc(&P->d_buf, blob.size()));
  HIP_TRY(hipMemcpy(P->d_buf, blob.data(), blob.size(), hipMemcpyHostToDevice));
  P->buf_bytes = blob.size();
  unsigned char* b = static_cast<unsigned char*>(P->d_buf);
  P->dp.mol = reinterpret_cast<const MolDesc*>(b + o_desc);
  P->dp.atom_gid = reinterpret_cast<const int32_t*>(b + o_atom);
  P->dp.inc_ptr = reinterpret_cast<const int32_t*>(b + o_incp);
  P->dp.inc = reinterpret_cast<const int32_t*>(b + o_inc);
  P->dp.row_start = reinterpret_cast<const int32_t*>(b + o_rows);
  P->dp.row_nup = reinterpret_cast<const int32_t*>(b + o_nup);
  P->dp.ra = reinterpret_cast<const int32_t*>(b + o_ra);
  P->dp.rb = reinterpret_cast<const int32_t*>(b + o_rb);
  P->dp.d2 = reinterpret_cast<const double*>(b + o_d2);
  P->dp.cid = reinterpret_cast<const int32_t*>(b + o_cid);
  P->dp.slot_col = reinterpret_cast<const int32_t*>(b + o_scol);
  P->dp.slot_coef = reinterpret_cast<const int32_t*>(b + o_scoef);
  P->dp.tasks = reinterpret_cast<const int4*>(b + o_tasks);
  P->dp.upd4 = reinterpret_cast<const int4*>(b + o_upd4);
  P->dp.updd = reinterpret_cast<const int32_t*>(b + o_updd);
  P->dp.lvl_task = reinterpret_cast<const int32_t*>(b + o_lt);
  P->dp.lvl_node = reinterpret_cast<const int32_t*>(b + o_ln);
  P->dp.nodes = reinterpret_cast<const int32_t*>(b + o_nodes);
  P->d_lists = reinterpret_cast<int32_t*>(b + o_lists);
  if (ws > 0) {
    HIP_TRY(hipMalloc(&P->d_ws, ws));
    P->ws_bytes = ws;
  }
  P->stats[0] = nm;
  P->stats[1] = ncon;
  P->stats[2] = natoms;
  P->stats[3] = nslots;
  P->stats[4] = fill;
  P->stats[5] = nupd;
  P->stats[6] = maxlev;
  P->stats[7] = sumlev;
  P->stats[8] = in_lds;
  P->stats[9] = in_ws;
  P->stats[10] = static_cast<int64_t>(ws);
  P->stats[11] = static_cast<int64_t>(blob.size());
  return ILVES_OK;
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
  try {
    for (const auto& c : mols) P->mols.push_back(ilves::plan_molecule(c, pairs, d, po));
  } catch (const std::bad_alloc&) {
    return fail(ILVES_ERR_NOMEM, "host allocation failed while planning");
  }
  ilves_status_t st = build_device_plan(P.get());
  if (st != ILVES_OK) return st;
  P->n_free = static_cast<int32_t>(free_atoms.size());
  if (P->n_free > 0) {
    HIP_TRY(hipMalloc(&P->d_free, free_atoms.size() * sizeof(int32_t)));
    HIP_TRY(hipMemcpy(P->d_free, free_atoms.data(), free_atoms.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  // allow every kernel this plan launches its dynamic LDS size
  for (int prec = 0; prec < 2; ++prec)
    for (const Group& g : P->groups[prec])
      if (g.lds_bytes > 0)
        HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(pick_kernel(prec == 1, g.lds, g.block)),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, g.lds_bytes));
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
  if (P->d_buf) (void)hipFree(P->d_buf);
  if (P->d_ws) (void)hipFree(P->d_ws);
  if (P->d_free) (void)hipFree(P->d_free);
  delete P;
  return ILVES_OK;
}

int32_t ilves_plan_num_molecules(ilves_plan_t P) { return P ? static_cast<int32_t>(P->mols.size()) : -1; }

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

ilves_status_t ilves_solve_ex(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                              int32_t precision, int32_t variant, int32_t warm_start, int32_t max_iter,
                              double* r_out, double* lambda, int32_t* iters, int32_t* status, void* hip_stream) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  if (!r || !r_u || !mass || !r_out) return fail(ILVES_ERR_ARG, "position and mass pointers must not be NULL");
  if (P->n_con > 0 && (!lambda || !iters || !status)) return fail(ILVES_ERR_ARG, "lambda/iters/status must not be NULL");
  if (!(tol >= 0.0)) return fail(ILVES_ERR_ARG, "tol must be >= 0");
  if (precision != ILVES_PREC_FP64 && precision != ILVES_PREC_MIXED) return fail(ILVES_ERR_ARG, "bad precision");
  if (variant != ILVES_VARIANT_NEWTON && variant != ILVES_VARIANT_CHORD) return fail(ILVES_ERR_ARG, "bad variant");
  if (warm_start == ILVES_WARM_MLP) return fail(ILVES_ERR_UNSUPPORTED, "no network loaded for the learned warm start");
  if (warm_start != ILVES_WARM_ZERO && warm_start != ILVES_WARM_CALLER) return fail(ILVES_ERR_ARG, "bad warm_start");
  if (r_out == r || r_out == r_u) return fail(ILVES_ERR_ARG, "r_out must not alias r or r_u");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device) return fail(ILVES_ERR_ARG, "plan was created on another device");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  SolveArgs A;
  A.r = r;
  A.r_u = r_u;
  A.mass = mass;
  A.r_out = r_out;
  A.lambda = lambda;
  A.iters = iters;
  A.status = status;
  A.ws = P->d_ws;
  A.tol = tol;
  A.n_atoms = P->n_atoms;
  A.max_iter = max_iter > 0 ? max_iter
                            : (precision == ILVES_PREC_FP64 && variant == ILVES_VARIANT_NEWTON ? 20 : 40);
  A.warm = warm_start == ILVES_WARM_CALLER ? 1 : 0;
  A.chord = variant == ILVES_VARIANT_CHORD ? 1 : 0;
  if (P->n_free > 0) {
    const int tb = 256;
    hipLaunchKernelGGL(copy_free_atoms, dim3((P->n_free + tb - 1) / tb), dim3(tb), 0, stream, P->d_free, P->n_free,
                       P->n_atoms, r_u, r_out);
    HIP_TRY(hipGetLastError());
  }
  const std::vector<Group>& groups = P->groups[precision == ILVES_PREC_MIXED ? 1 : 0];
  if (groups.empty()) return ILVES_OK;
  // fork: the groups run concurrently on the plan's streams, joined back
  // into the caller's stream (also valid under graph capture)
  HIP_TRY(hipEventRecord(P->ev_fork, stream));
  const int ns = std::min<int>(kStreams, static_cast<int>(groups.size()));
  for (int i = 0; i < ns; ++i) HIP_TRY(hipStreamWaitEvent(P->streams[i], P->ev_fork, 0));
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    KernelFn k = pick_kernel(precision == ILVES_PREC_MIXED, g.lds, g.block);
    hipStream_t s = P->streams[gi % ns];
    DevPlan dp = P->dp;
    const int32_t* list = P->d_lists + g.first;
    SolveArgs a = A;
    void* args[] = {&dp, &list, &a};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(g.count), dim3(g.block), args,
                            static_cast<size_t>(g.lds_bytes), s));
  }
  for (int i = 0; i < ns; ++i) {
    HIP_TRY(hipEventRecord(P->ev_join[i], P->streams[i]));
    HIP_TRY(hipStreamWaitEvent(stream, P->ev_join[i], 0));
  }
  return ILVES_OK;
}

ilves_status_t ilves_solve(ilves_plan_t P, const double* r, const double* r_u, const double* mass, double tol,
                           double* r_out, double* lambda, int32_t* iters, int32_t* status, void* hip_stream) {
  if (!P) return fail(ILVES_ERR_ARG, "plan must not be NULL");
  return ilves_solve_ex(P, r, r_u, mass, tol, P->opt.precision, P->opt.variant, P->opt.warm_start,
                        P->opt.max_iter, r_out, lambda, iters, status, hip_stream);
}

}  // extern "C"
