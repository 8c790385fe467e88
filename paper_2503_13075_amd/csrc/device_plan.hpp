// Device-side layout of a plan, shared by the solve and warm-start kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ilves_dev {

// Placement of a molecule's per-level data:
//   ALL_LDS:    slot structure and factor values in LDS
//   STRUCT_LDS: slot structure in LDS, factor values in the workspace
//   GLOBAL:     both read from global memory (molecules too large for LDS)
enum { ALL_LDS = 0, STRUCT_LDS = 1, GLOBAL = 2 };

struct MolDesc {
  int32_t n, s, n_up, n_l, n_upd, n_levels, n_pl;
  int32_t wide;       // 0: 16-bit structure indices, 1: 32-bit
  int32_t ix_off;     // structure block in the index pool of its width
  int32_t coef_off;   // ucoef then lcoef
  int32_t row_off;    // ra, rb, cid, d2 (also the global row index of row 0)
  int32_t atom_off;   // atom_gid
  int32_t incp_off;   // inc_ptr, s + 1 entries
  int32_t inc_off;    // inc
  int64_t ws_off;     // byte offset of the molecule's workspace
};

// Structure block of one molecule, in this order:
//   up_start[n+1] l_start[n+1] lvl_row[H+1] pl_start[H+1] ustart[n_up+1]
//   ucol[n_up] utr[n_up] lcol[n_l] ltr[n_l] upd_a[n_upd] upd_b[n_upd]
//   plist[n_pl]
__host__ __device__ inline int64_t struct_elems(int32_t n, int32_t H, int32_t n_up, int32_t n_l, int32_t n_upd,
                                                int32_t n_pl) {
  return 2 * (static_cast<int64_t>(n) + 1) + 2 * (static_cast<int64_t>(H) + 1) + 3 * static_cast<int64_t>(n_up) + 1 +
         2 * static_cast<int64_t>(n_l) + 2 * static_cast<int64_t>(n_upd) + n_pl;
}

struct DevPlan {
  const MolDesc* mol;
  const uint16_t* ix16;
  const int32_t* ix32;
  const int32_t* coef;
  const int32_t* ra;
  const int32_t* rb;
  const int32_t* cid;
  const double* d2;
  const int32_t* atom_gid;
  const int32_t* inc_ptr;
  const int32_t* inc;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

}  // namespace ilves_dev
