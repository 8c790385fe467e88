// Host-side planner: molecules, line graph, ordering, symbolic LU, level
// schedule, and the packed device layout the solve kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ilves {

// One factorisation task.  Diagonal task: out0 = diagonal slot of row j,
// out1 = -(j + 1).  Pair task for (j, m), m > j: out0 = slot of U_jm in row
// j, out1 = slot of W_mj in row m.  Updates are [u0, u1).
struct Task {
  int32_t out0, out1, u0, u1;
};

// Update of a diagonal task: acc -= W[s_wji] * D[s_dii] * U[s_uij], and the
// forward solve y_j -= W[s_wji] * D[s_dii] * y[i].
// Update of a pair task: U_jm -= W[a] * D[d] * U[b];  W_mj -= W[c] * D[d] * U[e].
struct Update {
  int32_t a, b, c, e;   // diag: a = slot(j,i), b = slot(i,j), c = i, e unused
  int32_t d;            // diagonal slot of row i (holds 1/U_ii once factored)
};

// Plan of one molecule (all indices local to it; rows in elimination order).
struct MolPlan {
  int32_t n = 0, s = 0, n_levels = 0, nslots = 0;
  std::vector<int32_t> cid;        // row -> input constraint index
  std::vector<int32_t> atom_gid;   // local atom -> input atom index
  std::vector<int32_t> ra, rb;     // row -> local atoms a_k, b_k
  std::vector<double> d2;          // row -> d_k^2
  std::vector<int32_t> row_start;  // n + 1; row k = [diag][upper (cols > k)][lower (cols < k)]
  std::vector<int32_t> row_nup;    // number of upper entries of row k
  std::vector<int32_t> slot_col;   // slot -> column (row index)
  std::vector<int32_t> slot_coef;  // slot -> (shared atom << 1) | (sign < 0); fill: (s << 1)
  std::vector<int32_t> inc_ptr;    // s + 1
  std::vector<int32_t> inc;        // (row << 1) | (atom is b_k)
  std::vector<int32_t> lvl_task;   // n_levels + 1 pointers into tasks
  std::vector<Task> tasks;
  std::vector<Update> upd;
  std::vector<int32_t> lvl_node;   // n_levels + 1 pointers into nodes
  std::vector<int32_t> nodes;      // rows sorted by level
  int64_t fill = 0;
  int ordering = 0;                // 1 minimum degree, 2 nested dissection
};

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

// Builds the plan of one molecule from its input constraint indices.
MolPlan plan_molecule(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d,
                      const PlanOptions& opt);

// Orderings of a graph given as sorted adjacency lists (exposed for tests).
std::vector<int32_t> order_min_degree(const std::vector<std::vector<int32_t>>& adj);
std::vector<int32_t> order_nested_dissection(const std::vector<std::vector<int32_t>>& adj, int leaf);

}  // namespace ilves
