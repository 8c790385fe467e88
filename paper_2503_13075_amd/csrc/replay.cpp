// Host replay of the device schedule (planner diagnostics).
//
// Executes on the host, level by level and with the same arithmetic, the
// schedule that the solve kernel runs on the GPU: residual and matrix rows,
// up-looking LU by elimination level with the fused forward substitution
// (each upper entry merges the lower patterns of its two rows), backward
// substitution, lambda update.  It exists so that the planner (ordering,
// symbolic factorisation, slot links) can be tested without a GPU; the solve
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
  const int32_t n = M.n, s = M.s, nu = M.n_up;
  std::vector<double> ex(n), ey(n), ez(n), ux(n), uy(n), uz(n), lam(n, 0.0), cd(n), invm(s + 1, 0.0);
  std::vector<double> cf(M.n_up + M.n_l);
  std::vector<T> y(n), D(n), F(M.n_up + M.n_l);
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
    ux[k] = ru[ga] - ru[gb];
    uy[k] = ru[S + ga] - ru[S + gb];
    uz[k] = ru[2 * S + ga] - ru[2 * S + gb];
    cd[k] = invm[M.ra[k]] + invm[M.rb[k]];
  }
  auto coupling = [&](int32_t c) { return (c & 1) ? -invm[c >> 1] : invm[c >> 1]; };
  for (int32_t q = 0; q < M.n_up; ++q) cf[q] = coupling(M.ucoef[q]);
  for (int32_t t = 0; t < M.n_l; ++t) cf[nu + t] = coupling(M.lcoef[t]);
  const T eps = sizeof(T) == 8 ? T(1e-13) : T(1e-6);
  bool singular = false;
  // one elimination level: factor entries (unless chord) and forward solve
  auto factor_level = [&](int32_t h, bool with_forward, bool with_factor) {
    const int32_t r0 = M.lvl_row[h], r1 = M.lvl_row[h + 1];
    for (int32_t j = r0; j < r1; ++j) {
      T acc = D[j], yj = y[j];
      const T a0 = acc;
      for (int32_t t = M.l_start[j]; t < M.l_start[j + 1]; ++t) {
        const int32_t i = M.lcol[t - nu];
        const T l = F[t] * D[i];
        if (with_factor) acc -= l * F[M.ltr[t - nu]];
        if (with_forward) yj -= l * y[i];
      }
      if (with_factor) {
        if (!(std::fabs(acc) > eps * std::fabs(a0))) singular = true;
        D[j] = T(1) / acc;
      }
      if (with_forward) y[j] = yj;
    }
    if (!with_factor) return;
    for (int32_t pi = M.pl_start[h]; pi < M.pl_start[h + 1]; ++pi) {
      const int32_t q = M.plist[pi];
      const int32_t tr = M.utr[q];
      T au = F[q], aw = F[tr];
      for (int32_t u = M.ustart[q]; u < M.ustart[q + 1]; ++u) {
        const int32_t pa = M.upd_a[u], pb = M.upd_b[u];
        const T di = D[M.lcol[pa - nu]];
        au -= F[pa] * di * F[M.ltr[pb - nu]];
        aw -= F[pb] * di * F[M.ltr[pa - nu]];
      }
      F[q] = au;
      F[tr] = aw;
    }
  };
  // row k of A(x, r), x having bond vector p
  // (level-0 rows have no lower entries: their pivot is inverted here)
  auto build_row = [&](int32_t k, double px, double py, double pz) {
    const T akk = static_cast<T>(cd[k] * (px * ex[k] + py * ey[k] + pz * ez[k]));
    if (k < M.lvl_row[1]) {
      if (!(std::fabs(akk) > T(0))) singular = true;
      D[k] = T(1) / akk;
    } else {
      D[k] = akk;
    }
    for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q) {
      const int32_t j = M.ucol[q];
      F[q] = static_cast<T>(cf[q] * (px * ex[j] + py * ey[j] + pz * ez[j]));
    }
    for (int32_t t = M.l_start[k]; t < M.l_start[k + 1]; ++t) {
      const int32_t j = M.lcol[t - nu];
      F[t] = static_cast<T>(cf[t] * (px * ex[j] + py * ey[j] + pz * ez[j]));
    }
  };
  if (chord) {
    for (int32_t k = 0; k < n; ++k) build_row(k, ex[k], ey[k], ez[k]);
    for (int32_t h = 1; h < M.n_levels; ++h) factor_level(h, false, true);
  }
  int32_t it = 0, st = ILVES_ERR_NOT_CONVERGED;
  if (singular) st = ILVES_ERR_SINGULAR;
  while (!singular) {
    double vmax = 0.0;
    for (int32_t k = 0; k < n; ++k) {
      const double lk = lam[k] * cd[k];
      double px = ux[k] - lk * ex[k];
      double py = uy[k] - lk * ey[k];
      double pz = uz[k] - lk * ez[k];
      for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q) {
        const int32_t j = M.ucol[q];
        const double c = cf[q] * lam[j];
        px -= c * ex[j];
        py -= c * ey[j];
        pz -= c * ez[j];
      }
      for (int32_t t = M.l_start[k]; t < M.l_start[k + 1]; ++t) {
        const int32_t j = M.lcol[t - nu];
        const double c = cf[t] * lam[j];
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
      if (!chord) build_row(k, px, py, pz);
    }
    if (vmax == INFINITY) { st = ILVES_ERR_NONFINITE; break; }
    if (vmax <= tol) { st = ILVES_OK; break; }
    if (it >= max_iter) { st = ILVES_ERR_NOT_CONVERGED; break; }
    for (int32_t h = 1; h < M.n_levels; ++h) factor_level(h, true, !chord);
    if (singular) { st = ILVES_ERR_SINGULAR; break; }
    for (int32_t h = M.n_levels - 1; h >= 0; --h)
      for (int32_t k = M.lvl_row[h]; k < M.lvl_row[h + 1]; ++k) {
        T acc = y[k];
        for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q) acc -= F[q] * y[M.ucol[q]];
        const T z = acc * D[k];
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
  int64_t nslots = 0, work = 0, maxlev = 0, fill = 0;
  for (size_t i = 0; i < mols.size(); ++i) {
    ilves::MolPlan M = ilves::plan_molecule(mols[i], pairs, d, po);
    nslots += static_cast<int64_t>(M.n) + M.n_up + M.n_l;
    work += M.n_upd;
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
    schedule_stats[2] = work;
    schedule_stats[3] = maxlev;
    schedule_stats[4] = fill;
  }
  return ILVES_OK;
}

}  // extern "C"
