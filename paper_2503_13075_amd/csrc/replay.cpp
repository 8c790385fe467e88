// Host replay of the device schedule (planner diagnostics).
//
// Executes, on the host and in the same order of operations, the level
// schedule that the solve kernel runs on the GPU: residual and matrix rows,
// level-by-level up-looking LU with the fused forward substitution, backward
// substitution, lambda update.  It exists so that the planner (ordering,
// symbolic factorisation, task lists) can be tested without a GPU; the solve
// entry points never call it.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ilves.h"
#include "plan.hpp"

namespace {

thread_local std::string g_replay_error;

template <typename T>
int32_t replay_molecule(const ilves::MolPlan& M, int32_t S, const double* mass, const double* r, const double* ru,
                        double tol, bool chord, int32_t max_iter, double* r_out, double* lambda, int32_t* iters) {
  const int32_t n = M.n, s = M.s;
  std::vector<double> ex(n), ey(n), ez(n), lam(n, 0.0), invm(s + 1, 0.0);
  std::vector<T> y(n), F(M.nslots);
  double rmax = 0.0;
  for (int32_t a = 0; a < s; ++a) {
    const int32_t g = M.atom_gid[a];
    invm[a] = 1.0 / mass[g];
    rmax = std::fmax(rmax, std::fmax(std::fabs(ru[g]), std::fmax(std::fabs(ru[S + g]), std::fabs(ru[2 * S + g]))));
  }
  const double delta = 1.7320508075688772 * rmax * 0x1.0p-52;
  const double delta2 = 0.5 * delta * delta;
  for (int32_t k = 0; k < n; ++k) {
    const int32_t ga = M.atom_gid[M.ra[k]], gb = M.atom_gid[M.rb[k]];
    ex[k] = r[ga] - r[gb];
    ey[k] = r[S + ga] - r[S + gb];
    ez[k] = r[2 * S + ga] - r[2 * S + gb];
  }
  const T eps = sizeof(T) == 8 ? T(1e-13) : T(1e-6);
  bool singular = false;
  auto coef = [&](int32_t cf) { return (cf & 1) ? -invm[cf >> 1] : invm[cf >> 1]; };
  auto factor_level = [&](int32_t h, bool with_forward, bool with_factor) {
    for (int32_t t = M.lvl_task[h]; t < M.lvl_task[h + 1]; ++t) {
      const ilves::Task& tk = M.tasks[t];
      if (tk.out1 < 0) {
        const int32_t j = -tk.out1 - 1;
        T yj = y[j];
        T acc = F[tk.out0];
        const T a0 = acc;
        for (int32_t u = tk.u0; u < tk.u1; ++u) {
          const ilves::Update& q = M.upd[u];
          const T l = F[q.a] * F[q.d];
          if (with_factor) acc -= l * F[q.b];
          if (with_forward) yj -= l * y[q.c];
        }
        if (with_factor) {
          if (!(std::fabs(acc) > eps * std::fabs(a0))) singular = true;
          F[tk.out0] = T(1) / acc;
        }
        if (with_forward) y[j] = yj;
      } else if (with_factor) {
        T au = F[tk.out0], aw = F[tk.out1];
        for (int32_t u = tk.u0; u < tk.u1; ++u) {
          const ilves::Update& q = M.upd[u];
          const T dinv = F[q.d];
          au -= F[q.a] * dinv * F[q.b];
          aw -= F[q.c] * dinv * F[q.e];
        }
        F[tk.out0] = au;
        F[tk.out1] = aw;
      }
    }
  };
  if (chord) {
    for (int32_t k = 0; k < n; ++k) {
      const double w = invm[M.ra[k]] + invm[M.rb[k]];
      const int32_t q0 = M.row_start[k], q1 = M.row_start[k + 1];
      F[q0] = static_cast<T>(w * (ex[k] * ex[k] + ey[k] * ey[k] + ez[k] * ez[k]));
      for (int32_t q = q0 + 1; q < q1; ++q) {
        const int32_t j = M.slot_col[q];
        F[q] = static_cast<T>(coef(M.slot_coef[q]) * (ex[k] * ex[j] + ey[k] * ey[j] + ez[k] * ez[j]));
      }
    }
    for (int32_t h = 0; h < M.n_levels; ++h) factor_level(h, false, true);
  }
  int32_t it = 0, st = ILVES_ERR_NOT_CONVERGED;
  if (singular) st = ILVES_ERR_SINGULAR;
  while (!singular) {
    double vmax = 0.0;
    for (int32_t k = 0; k < n; ++k) {
      const int32_t la = M.ra[k], lb = M.rb[k];
      const int32_t ga = M.atom_gid[la], gb = M.atom_gid[lb];
      const double w = invm[la] + invm[lb];
      const double lk = lam[k] * w;
      double px = ru[ga] - ru[gb] - lk * ex[k];
      double py = ru[S + ga] - ru[S + gb] - lk * ey[k];
      double pz = ru[2 * S + ga] - ru[2 * S + gb] - lk * ez[k];
      const int32_t q0 = M.row_start[k], q1 = M.row_start[k + 1];
      for (int32_t q = q0 + 1; q < q1; ++q) {
        const int32_t j = M.slot_col[q];
        const double c = coef(M.slot_coef[q]) * lam[j];
        px -= c * ex[j];
        py -= c * ey[j];
        pz -= c * ez[j];
      }
      const double pp = px * px + py * py + pz * pz;
      const double g = 0.5 * (pp - M.d2[k]);
      double rel = (std::fabs(g) + std::sqrt(pp) * delta + delta2) / M.d2[k];
      if (!(rel <= DBL_MAX)) rel = INFINITY;
      vmax = std::fmax(vmax, rel);
      y[k] = static_cast<T>(g);
      if (!chord) {
        F[q0] = static_cast<T>(w * (px * ex[k] + py * ey[k] + pz * ez[k]));
        for (int32_t q = q0 + 1; q < q1; ++q) {
          const int32_t j = M.slot_col[q];
          F[q] = static_cast<T>(coef(M.slot_coef[q]) * (px * ex[j] + py * ey[j] + pz * ez[j]));
        }
      }
    }
    if (vmax == INFINITY) { st = ILVES_ERR_NONFINITE; break; }
    if (vmax <= tol) { st = ILVES_OK; break; }
    if (it >= max_iter) { st = ILVES_ERR_NOT_CONVERGED; break; }
    for (int32_t h = 0; h < M.n_levels; ++h) factor_level(h, true, !chord);
    if (singular) { st = ILVES_ERR_SINGULAR; break; }
    for (int32_t h = M.n_levels - 1; h >= 0; --h)
      for (int32_t i = M.lvl_node[h]; i < M.lvl_node[h + 1]; ++i) {
        const int32_t k = M.nodes[i];
        const int32_t q0 = M.row_start[k];
        T acc = y[k];
        for (int32_t q = q0 + 1; q <= q0 + M.row_nup[k]; ++q) acc -= F[q] * y[M.slot_col[q]];
        const T z = acc * F[q0];
        y[k] = z;
        lam[k] += static_cast<double>(z);
      }
    ++it;
  }
  for (int32_t k = 0; k < n; ++k) lambda[M.cid[k]] = lam[k];
  for (int32_t a = 0; a < s; ++a) {
    double dx = 0, dy = 0, dz = 0;
    for (int32_t q = M.inc_ptr[a]; q < M.inc_ptr[a + 1]; ++q) {
      const int32_t e = M.inc[q];
      const int32_t k = e >> 1;
      const double l = (e & 1) ? -lam[k] : lam[k];
      dx += l * ex[k];
      dy += l * ey[k];
      dz += l * ez[k];
    }
    const int32_t g = M.atom_gid[a];
    r_out[g] = ru[g] - invm[a] * dx;
    r_out[S + g] = ru[S + g] - invm[a] * dy;
    r_out[2 * S + g] = ru[2 * S + g] - invm[a] * dz;
  }
  *iters = it;
  return st;
}

}  // namespace

extern "C" {

ilves_status_t ilves_plan_replay_host(int32_t n_atoms, int32_t n_constraints, const int32_t* pairs, const double* d,
                                      const ilves_options_t* opt, const double* mass, const double* r,
                                      const double* r_u, double tol, int32_t precision, int32_t variant,
                                      int32_t max_iter, double* r_out, double* lambda, int32_t* iters,
                                      int32_t* status, int32_t* n_molecules, int64_t* schedule_stats) {
  if (n_atoms <= 0 || n_constraints < 0 || !mass || !r || !r_u || !r_out || !n_molecules) {
    g_replay_error = "bad argument";
    return ILVES_ERR_ARG;
  }
  std::string msg = ilves::validate_topology(n_atoms, n_constraints, pairs, d);
  if (!msg.empty()) {
    g_replay_error = msg;
    return ILVES_ERR_TOPOLOGY;
  }
  ilves::PlanOptions po;
  if (opt) po.ordering = opt->ordering;
  std::vector<int32_t> free_atoms;
  auto mols = ilves::split_molecules(n_atoms, n_constraints, pairs, free_atoms);
  *n_molecules = static_cast<int32_t>(mols.size());
  for (int32_t g : free_atoms) {
    r_out[g] = r_u[g];
    r_out[n_atoms + g] = r_u[n_atoms + g];
    r_out[2 * n_atoms + g] = r_u[2 * n_atoms + g];
  }
  const int32_t cap = max_iter > 0 ? max_iter : (precision == ILVES_PREC_FP64 && variant == 0 ? 20 : 40);
  int64_t nslots = 0, nupd = 0, maxlev = 0, fill = 0;
  for (size_t i = 0; i < mols.size(); ++i) {
    ilves::MolPlan M = ilves::plan_molecule(mols[i], pairs, d, po);
    nslots += M.nslots;
    nupd += static_cast<int64_t>(M.upd.size());
    maxlev = std::max<int64_t>(maxlev, M.n_levels);
    fill += M.fill;
    int32_t it = 0;
    int32_t st = precision == ILVES_PREC_MIXED
                     ? replay_molecule<float>(M, n_atoms, mass, r, r_u, tol, variant == 1, cap, r_out, lambda, &it)
                     : replay_molecule<double>(M, n_atoms, mass, r, r_u, tol, variant == 1, cap, r_out, lambda, &it);
    if (iters) iters[i] = it;
    if (status) status[i] = st;
  }
  if (schedule_stats) {
    schedule_stats[0] = static_cast<int64_t>(mols.size());
    schedule_stats[1] = nslots;
    schedule_stats[2] = nupd;
    schedule_stats[3] = maxlev;
    schedule_stats[4] = fill;
  }
  return ILVES_OK;
}

}  // extern "C"
