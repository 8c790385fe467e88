// Device-side layout of a plan, shared by the solve and warm-start kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ilves_dev {

// Placement of a molecule's per-level data:
//   ALL_LDS:    slot structure and factor values in LDS
//   STRUCT_LDS: slot structure in LDS, factor values in the workspace
//   VALUES_LDS: factor values in LDS, slot structure read from global memory
//   GLOBAL:     both read from global memory (molecules too large for LDS)
enum { ALL_LDS = 0, STRUCT_LDS = 1, GLOBAL = 2, VALUES_LDS = 3 };

struct MolDesc {
  int32_t n, s, n_up, n_l, n_upd, n_levels, n_pl;
  int32_t wide;       // 0: 16-bit structure indices, 1: 32-bit
  int64_t ix_off;     // byte offset of the structure block in the structure pool
  int32_t coef_off;   // ucoef then lcoef
  int32_t row_off;    // ra, rb, cid, d2 (also the global row index of row 0)
  int32_t atom_off;   // atom_gid
  int32_t incp_off;   // inc_ptr, s + 1 entries
  int32_t inc_off;    // inc
  int64_t ws_off;     // byte offset of the molecule's workspace
};

// Structure block of one molecule (index type of isz bytes, 2 or 4), as
// byte offsets from the block start (16-byte aligned):
//   up_start[n+1], l_start[n+1], ucol[n_up]          per row / upper slot
//   lvh[H]      level header {first row, end row, first pair task, end}
//   lpair[n_l]  lower slot t: {column i, slot of the transpose (i, k)}
//   prec[n_pl]  pair task: {upper slot q, slot of (m, j), first update, count}
//   upd[n_upd]  update: {slot (j,i), slot (m,i), slot (i,m), slot (i,j)}
//   updi[n_upd] row i of the update
struct Layout {
  int64_t up_start, l_start, ucol, lvh, lpair, prec, upd, updi, total;
};

__host__ __device__ inline int64_t align_to(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline Layout struct_layout(int32_t n, int32_t H, int32_t n_up, int32_t n_l, int32_t n_pl,
                                                int32_t n_upd, int isz) {
  Layout L;
  L.up_start = 0;
  L.l_start = L.up_start + static_cast<int64_t>(isz) * (n + 1);
  L.ucol = L.l_start + static_cast<int64_t>(isz) * (n + 1);
  L.lvh = align_to(L.ucol + static_cast<int64_t>(isz) * n_up, 4 * isz);
  L.lpair = L.lvh + static_cast<int64_t>(4 * isz) * H;
  L.prec = align_to(L.lpair + static_cast<int64_t>(2 * isz) * n_l, 4 * isz);
  L.upd = L.prec + static_cast<int64_t>(4 * isz) * n_pl;
  L.updi = L.upd + static_cast<int64_t>(4 * isz) * n_upd;
  L.total = align_to(L.updi + static_cast<int64_t>(isz) * n_upd, 16);
  return L;
}

struct DevPlan {
  const MolDesc* mol;
  const unsigned char* ix;    // structure pool (16-byte aligned blocks)
  const int32_t* coef;
  const int32_t* ra;
  const int32_t* rb;
  const int32_t* cid;
  const double* d2;
  const int32_t* atom_gid;
  const int32_t* inc_ptr;
  const int32_t* inc;
  const int32_t* ga;     // per row: input index of atom a_k (same offsets as ra)
  const int32_t* gb;     // per row: input index of atom b_k
  const int32_t* gcoef;  // per slot: (input index of the shared atom << 1) | (sign < 0), -1 for fill
};

// A molecule of at most kSmallCons constraints on at most kSmallAtoms atoms,
// solved by one thread with the whole Newton loop in registers (water-,
// diatomic- or triatomic-like molecules).  64 bytes.
constexpr int kSmallCons = 3;
constexpr int kSmallAtoms = 4;
struct SmallMol {
  int32_t atom[kSmallAtoms];  // input atom indices (unused entries repeat atom[0])
  int32_t cid[kSmallCons];    // input constraint indices
  int32_t mol;                // molecule index (iters / status / fallback slot)
  uint8_t a[kSmallCons], b[kSmallCons];  // local atoms of each constraint
  uint8_t nc, na;
  double d2[kSmallCons];
};
static_assert(sizeof(SmallMol) == 64, "SmallMol is one 64-byte record");

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

}  // namespace ilves_dev
