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
//   PAIRS_GLOBAL: factor values and the per-row structure (row starts,
//               upper columns, level headers, lower-slot records) in LDS; the
//               pair tasks and their update lists read from global memory
enum { ALL_LDS = 0, STRUCT_LDS = 1, GLOBAL = 2, VALUES_LDS = 3, PAIRS_GLOBAL = 4 };

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
//   lvc[H]      per level {lg of the factorisation, lg of the backward
//               substitution}: 2^lg lanes per item (see item_lanes_log2)
//   lpair[n_l]  lower slot t: {column i, slot of the transpose (i, k)}
//   ccode[n_up + n_l]  one byte per slot (F index): coupling code, see
//               kFillCode
//   prec[n_pl]  pair task: {upper slot q, slot of (m, j), first update, count}
//   upd[n_upd]  update: {slot (j,i), slot (m,i), slot (i,m), slot (i,j)}
//   updi[n_upd] row i of the update
struct Layout {
  int64_t up_start, l_start, ucol, lvh, lvc, lpair, ccode, prec, upd, updi, total;
};

// Lanes per item of an elimination level.  Where a level's longest chain
// (the most lower entries of a row or updates of a pair task in the
// factorisation, the most upper entries of a row in the backward
// substitution) is long, G = 2^lg lanes share each item's entries and add
// their partial sums with lane shuffles: the largest G <= kMaxItemLanes that
// leaves each lane at least kLaneEntries entries of that chain while the
// level's items (rows padded to whole waves when pair tasks follow, then
// pair tasks) fit kItemLaneBudget lanes.  It depends on the plan only, not
// on the launch tuning, so a tuning never changes the arithmetic.  Only the
// kernel of the parts of split molecules has the shared-lane path (the long
// chains are theirs: angle constraints fill the factor); whole molecules
// always take one lane per item, which keeps that kernel's code lean.
constexpr int kMaxItemLanes = 16;
constexpr int kLaneEntries = 4;
constexpr int kItemLaneBudget = 512;
__host__ __device__ inline int32_t item_lanes_log2(int32_t chain, int32_t nr, int32_t np, bool pad) {
  int32_t lg = 0;
  while ((1 << (lg + 1)) <= kMaxItemLanes && (chain >> (lg + 1)) >= kLaneEntries) {
    const int32_t nrl = nr << (lg + 1);
    if ((pad ? (nrl + 63) & ~63 : nrl) + (np << (lg + 1)) > kItemLaneBudget) break;
    ++lg;
  }
  return lg;
}

// Coupling code of the slot (k, j): C_kj = sign / m_x, x the atom that
// constraints k and j share, which is one of k's two atoms.  Bit 1: x is
// b_k (else a_k); bit 0: negative sign; kFillCode: a fill entry of the
// factor (k and j share no atom, C_kj = 0).
constexpr uint8_t kFillCode = 4;

__host__ __device__ inline int64_t align_to(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline Layout struct_layout(int32_t n, int32_t H, int32_t n_up, int32_t n_l, int32_t n_pl,
                                                int32_t n_upd, int isz) {
  Layout L;
  L.up_start = 0;
  L.l_start = L.up_start + static_cast<int64_t>(isz) * (n + 1);
  L.ucol = L.l_start + static_cast<int64_t>(isz) * (n + 1);
  L.lvh = align_to(L.ucol + static_cast<int64_t>(isz) * n_up, 4 * isz);
  L.lvc = L.lvh + static_cast<int64_t>(4 * isz) * H;
  L.lpair = align_to(L.lvc + static_cast<int64_t>(2 * isz) * H, 4 * isz);
  L.ccode = L.lpair + static_cast<int64_t>(2 * isz) * n_l;
  L.prec = align_to(L.ccode + static_cast<int64_t>(n_up) + n_l, 4 * isz);
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
  const int32_t* gcoef;  // per slot: (input index of the shared atom << 1) | (sign < 0), -1 for fill (feature passes)
  // molecules split across workgroups (one workgroup per part)
  const struct SplitPart* split;  // per part, in launch order
  const struct SepRow* sep;       // separator rows of every split molecule
  const int32_t* sadj;            // separator couplings: {other separator row, coupling} pairs
  const int32_t* bsep;            // per border row: separator row | (1 << 30 when the part owns it)
  const int32_t* ext_ptr;         // per border row: first external coupling (CSR, one extra entry per part)
  const int64_t* ext_rec;         // external coupling: offset (doubles) of the holder's record in the workspace
  const int32_t* ext_coef;        // external coupling: (input atom << 1) | (sign < 0)
};

// One part of a split molecule (block-bordered LU, see the solve kernel).
struct SplitPart {
  int32_t desc;     // descriptor of the part's rows (MolDesc index)
  int32_t report;   // molecule index for iters / status / fallback
  int32_t part, n_parts;
  int32_t n_int;    // interior rows [0, n_int), border rows [n_int, n)
  int32_t h_int;    // levels [0, h_int) hold the interior rows
  int32_t s_own;    // local atoms [0, s_own) are the part's own
  int32_t m;        // separator rows of the molecule
  int32_t bsep_off;  // into bsep (n - n_int entries)
  int32_t ext_off;   // into ext_ptr (n - n_int + 1 entries)
  int32_t sep_off;   // first SepRow of the molecule
  int32_t ew_off;    // doubles from the exchange area to this part's E block (nb*nb, then w: nb)
  int64_t xch;       // byte offset of the molecule's exchange area in the workspace
  int32_t lds_extra[2];  // byte offset of the split scratch in dynamic LDS (FP64, FP32 values)
  int32_t ew_total;  // doubles of the molecule's E/w blocks (all parts)
  int32_t n_sadj;    // separator couplings of the molecule
  int32_t bw;        // half-bandwidth of the separator matrix with its fill
  int32_t pad;
};
static_assert(sizeof(SplitPart) == 80, "SplitPart is one 80-byte record");

// A separator row: the two parts holding it as a border row (part0 owns
// it), its border index in each, its atoms and its separator couplings.
struct SepRow {
  int32_t part0, part1;  // part indices within the molecule
  int32_t loc0, loc1;
  int32_t ga, gb;
  int32_t adj_off, adj_cnt;  // into sadj (pairs)
  int32_t ew0, ew1;          // E/w blocks of the two parts (doubles from the exchange area)
  int32_t nb0, nb1;          // border rows of the two parts
};

// Exchange area of a split molecule in the workspace (byte offsets):
//   [0, 64)          barrier: arrival count, generation, poisoned flag
//   PartX[n_parts]   per part: max relative violation, violation at
//                    lambda = 0, singular flag
//   SepX[m]          per separator row (owner writes): bond vector e', g, e
//   E/w blocks       per part: Schur contribution E (nb x nb), reduced
//                    right-hand side contribution w (nb)
struct PartX {
  double viol, rel0;
  int32_t singular, pad[3];
};
struct SepX {
  double ep[3], g, e[3], pad;
};
__host__ __device__ inline int64_t xch_partx(int32_t) { return 64; }
__host__ __device__ inline int64_t xch_sepx(int32_t n_parts) { return 64 + 32 * static_cast<int64_t>(n_parts); }
__host__ __device__ inline int64_t xch_ew(int32_t n_parts, int32_t m) { return xch_sepx(n_parts) + 64 * static_cast<int64_t>(m); }

// Split scratch in LDS after the factor values (doubles): the separator
// system [m][m + 1], its solution z[m], per border row the saved residual
// gB[nb]; the border block of the matrix, the unit-lower and the upper
// factors ([nb][nb] each); the row maxima of the separator matrix [m]; a
// copy of the exchange area's SepX records and E/w blocks [8m + ew_total];
// the molecule's SepRow records [m] and separator couplings [n_sadj pairs].
__host__ __device__ inline int64_t split_lds_bytes(int32_t m, int32_t nb, int32_t ew_total, int32_t n_sadj) {
  return 8 * (static_cast<int64_t>(m) * (m + 1) + m + nb + 3 * static_cast<int64_t>(nb) * nb + m + 8 * m + ew_total) +
         static_cast<int64_t>(sizeof(SepRow)) * m + 8 * static_cast<int64_t>(n_sadj);
}

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
