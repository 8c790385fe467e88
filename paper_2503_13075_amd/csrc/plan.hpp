// Host-side planner: molecules, line graph, ordering, symbolic LU, level
// schedule, and the packed device layout the solve kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ilves {

// Plan of one molecule.  Rows (constraints) are numbered in elimination
// order, grouped by elimination level: level h holds rows
// [lvl_row[h], lvl_row[h+1]).  The diagonal of row j has its own entry
// (index j of the diagonal array); every off-diagonal entry of the filled
// LU pattern has one "slot" (an index into the value array F):
//   * upper slots [0, n_up): row j owns [up_start[j], up_start[j+1]) =
//     its entries (j, m), m > j, ascending in m;
//   * lower slots [n_up, n_up + n_l): row k owns [l_start[k], l_start[k+1])
//     = its entries (k, i), i < k, ascending in i.
// utr / ltr link an entry to its transpose.  The factor update of an upper
// entry (j, m) and of its transpose (m, j) runs over the rows i < j that
// are coupled to both j and m; the pairs (slot (j, i), slot (m, i)) of
// those rows are listed in upd_a / upd_b over [ustart[q], ustart[q+1]) for
// upper slot q.  Level h's upper slots that have at least one update are
// listed in plist[pl_start[h] .. pl_start[h+1]); the others keep their
// matrix value.  Level 0 holds exactly the rows without lower entries, whose
// factorisation is just 1/A_jj.  *coef hold
// the coupling of an original entry: (shared atom << 1) | (sign < 0), or
// (s << 1) for a fill entry.
struct MolPlan {
  int32_t n = 0, s = 0, n_levels = 0, n_up = 0, n_l = 0, n_upd = 0;
  std::vector<int32_t> cid;        // row -> input constraint index
  std::vector<int32_t> atom_gid;   // local atom -> input atom index
  std::vector<int32_t> ra, rb;     // row -> local atoms a_k, b_k
  std::vector<double> d2;          // row -> d_k^2
  std::vector<int32_t> up_start, l_start;            // n + 1 each
  std::vector<int32_t> ucol, utr, ucoef;             // n_up each
  std::vector<int32_t> ustart;                       // n_up + 1
  std::vector<int32_t> lcol, ltr, lcoef;             // n_l each
  std::vector<int32_t> upd_a, upd_b;                 // n_upd each
  std::vector<int32_t> lvl_row;    // n_levels + 1
  std::vector<int32_t> pl_start;   // n_levels + 1
  std::vector<int32_t> plist;      // upper slots with updates, level by level
  std::vector<int32_t> inc_ptr;    // s + 1
  std::vector<int32_t> inc;        // (row << 1) | (atom is b_k)
  int64_t fill = 0;
  int ordering = 0;                // 1 minimum fill, 2 nested dissection
  double cost = 0.0;               // critical-path estimate of one Newton iteration (planner units)
  // Parts of a split molecule (plan_split): rows [0, n_int) are the part's
  // interior constraints, rows [n_int, n) its border constraints, which
  // occupy levels [h_int, n_levels) alone; local atoms [0, s_own) belong to
  // the part (their positions are its output).  A whole molecule has
  // n_int = n, h_int = n_levels, s_own = s.
  int32_t n_int = 0, h_int = 0, s_own = 0;
};

// A part of a split molecule: the constraints, interior ones first, with
// n_tail border constraints at the end, and the input atoms the part owns
// (sorted).
struct PartSpec {
  int32_t n_tail = 0;
  const std::vector<int32_t>* owned = nullptr;
};

// A molecule split across several workgroups (block-bordered form).  The
// atoms are partitioned into groups; a constraint inside a group is an
// interior row of that group's part, a constraint joining two groups is a
// separator row and a border row of both parts.  After ordering every
// part's interior rows before its border rows, the Newton matrix is
//   [A_11         A_1S]
//   [      ...    ... ]     A_SS - sum_i A_Si A_ii^-1 A_iS = Schur complement
//   [A_S1  ...    A_SS]
// and each part's LU of its own rows yields its contribution to the Schur
// complement and to the reduced right-hand side.
struct SplitPlan {
  std::vector<MolPlan> parts;
  int32_t m = 0;                        // separator rows (ordered by their two parts)
  int32_t bw = 0;                       // half-bandwidth of the separator matrix with its fill
  std::vector<int32_t> sep_cid;         // [m] input constraint
  std::vector<int32_t> sep_ga, sep_gb;  // [m] input atoms a_b, b_b
  std::vector<int32_t> sep_part;        // [2m] the two parts holding row b (owner first)
  std::vector<int32_t> sep_loc;         // [2m] its border index (local row - n_int) in each
  std::vector<int32_t> sadj_ptr;        // [m + 1] CSR: separator rows coupled to b
  std::vector<int32_t> sadj_col;        //   other separator row
  std::vector<int32_t> sadj_coef;       //   coupling (input atom << 1) | (sign < 0)
  // per part, per border row (CSR): coupled rows not held by the part, as
  // (holding part, local row there, coupling)
  std::vector<std::vector<int32_t>> ext_ptr, ext_part, ext_row, ext_coef;
};

constexpr int32_t kSplitMaxParts = 64;    // workgroups of one split molecule
constexpr int32_t kSplitMaxSep = 64;      // separator rows of one split molecule
constexpr int32_t kSplitMaxBorder = 24;   // border rows of one part

struct PlanOptions {
  int ordering = 0;      // 0 auto, 1 MD, 2 ND
  int nd_leaf = 48;      // ND stops splitting below this many vertices
};

// Validates a topology and splits it into molecules.  Returns an empty
// string on success or a message describing the first problem.
std::string validate_topology(int32_t n_atoms, int32_t n_con, const int32_t* pairs, const double* d);

// Connected components: for each molecule the (sorted) input constraint
// indices.  free_atoms receives atoms that appear in no constraint.
std::vector<std::vector<int32_t>> split_molecules(int32_t n_atoms, int32_t n_con, const int32_t* pairs,
                                                  std::vector<int32_t>& free_atoms);

// Builds the plan of one molecule (or, with part, of one part of a split
// molecule) from its input constraint indices.
MolPlan plan_molecule(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d,
                      const PlanOptions& opt, const PartSpec* part = nullptr);

// Splits a molecule into parts of about part_rows constraints.  Returns false
// (out untouched) when the split would exceed the limits above or leave a
// part without interior constraints.
bool plan_split(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d, const PlanOptions& opt,
                int32_t part_rows, SplitPlan& out);

// Split with an automatic part size when part_rows <= 0: about twelve parts
// (measured best: fewer parts leave long per-part sweeps, more parts a large
// separator system), 384 to 1,024 constraints each, then 1.5x larger parts
// while the split exceeds the limits.
bool plan_split_auto(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d,
                     const PlanOptions& opt, int32_t part_rows, SplitPlan& out);

// Orderings of a graph given as sorted adjacency lists (exposed for tests).
std::vector<int32_t> order_min_degree(const std::vector<std::vector<int32_t>>& adj);
std::vector<int32_t> order_nested_dissection(const std::vector<std::vector<int32_t>>& adj, int leaf);

}  // namespace ilves
