// Host replay of the device schedule (planner diagnostics).
//
// Executes on the host, level by level and with the same arithmetic, the
// schedule that the solve kernels run on the GPU: residual and matrix rows,
// up-looking LU by elimination level with the fused forward substitution
// (each upper entry merges the lower patterns of its two rows), backward
// substitution, lambda update -- and, for a molecule split across several
// workgroups, the block-bordered scheme: every part factors its interior and
// border rows, contributes to the Schur complement on the separator rows,
// the small dense separator system is solved, and every part finishes its
// backward substitution from the separator solution.  It exists so that the
// planner (ordering, symbolic factorisation, slot links, splits) can be
// tested without a GPU; the solve entry points never call it.  The sums of
// an item run in entry order here; in the levels where the device shares an
// item over several lanes (parts of split molecules with long chains) it
// adds per-lane partial sums instead, so the two agree to rounding there.
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

// State of one molecule, or of one part of a split molecule.
template <typename T>
struct Rep {
  const ilves::MolPlan& M;
  const int32_t S;
  const double* mass;
  const double* ru;
  int32_t n, s, nu;
  std::vector<double> ex, ey, ez, ux, uy, uz, lam, cd, invm, cf;
  std::vector<T> y, D, F;
  double delta = 0.0, delta2 = 0.0;
  bool singular = false;
  T eps;

  Rep(const ilves::MolPlan& M_, int32_t S_, const double* mass_, const double* r, const double* ru_)
      : M(M_), S(S_), mass(mass_), ru(ru_), n(M_.n), s(M_.s), nu(M_.n_up) {
    ex.resize(n); ey.resize(n); ez.resize(n); ux.resize(n); uy.resize(n); uz.resize(n);
    lam.assign(n, 0.0); cd.resize(n); invm.assign(s + 1, 0.0); cf.resize(M.n_up + M.n_l);
    y.resize(n); D.resize(n); F.resize(M.n_up + M.n_l);
    eps = sizeof(T) == 8 ? T(1e-13) : T(1e-6);
    double rmax = 0.0;
    for (int32_t a = 0; a < s; ++a) {
      const int32_t g = M.atom_gid[a];
      invm[a] = 1.0 / mass[g];
      rmax = std::fmax(rmax, std::fmax(std::fabs(ru[g]), std::fmax(std::fabs(ru[S + g]), std::fabs(ru[2 * S + g]))));
    }
    delta = 1.7320508075688772 * rmax * 0x1.0p-52;
    delta2 = 0.5 * delta * delta;
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
    for (int32_t q = 0; q < M.n_up; ++q) cf[q] = coupling(M.ucoef[q]);
    for (int32_t t = 0; t < M.n_l; ++t) cf[nu + t] = coupling(M.lcoef[t]);
  }
  double coupling(int32_t c) const { return (c & 1) ? -invm[c >> 1] : invm[c >> 1]; }

  // one elimination level: factor entries (unless chord) and forward solve
  void factor_level(int32_t h, bool with_forward, bool with_factor) {
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
  }
  void factor_sweep(bool with_forward, bool with_factor) {
    for (int32_t h = 1; h < M.n_levels; ++h) factor_level(h, with_forward, with_factor);
  }
  // row k of A(x, r), x having bond vector p
  // (level-0 rows have no lower entries: their pivot is inverted here)
  void build_row(int32_t k, double px, double py, double pz) {
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
  }
  // bond vector of row k at the current lambda (rows held here only)
  void bond(int32_t k, double& px, double& py, double& pz) const {
    const double lk = lam[k] * cd[k];
    px = ux[k] - lk * ex[k];
    py = uy[k] - lk * ey[k];
    pz = uz[k] - lk * ez[k];
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
  }
  // relative violation of row k with bond vector p; y[k] = g
  double violation(int32_t k, double px, double py, double pz) {
    const double pp = px * px + py * py + pz * pz;
    const double g = 0.5 * (pp - M.d2[k]);
    double rel = (std::fabs(g) + std::sqrt(pp) * delta + delta2) / M.d2[k];
    if (!(rel <= DBL_MAX)) rel = INFINITY;
    y[k] = static_cast<T>(g);
    return rel;
  }
  // backward substitution over levels h_top-1 .. 0 (rows above keep y)
  void back(int32_t h_top) {
    for (int32_t h = h_top - 1; h >= 0; --h)
      for (int32_t k = M.lvl_row[h]; k < M.lvl_row[h + 1]; ++k) {
        T acc = y[k];
        for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q) acc -= F[q] * y[M.ucol[q]];
        y[k] = acc * D[k];
      }
  }
  void update() {
    for (int32_t k = 0; k < n; ++k) lam[k] += static_cast<double>(y[k]);
  }
  // r' of the local atoms [0, s_own); lambda of the rows k with keep(k)
  template <class Keep>
  void outputs(double* r_out, double* lambda, Keep keep) const {
    for (int32_t k = 0; k < n; ++k)
      if (keep(k)) lambda[M.cid[k]] = lam[k];
    for (int32_t a = 0; a < M.s_own; ++a) {
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
  }
};

template <typename T>
int32_t replay_molecule(const ilves::MolPlan& M, int32_t S, const double* mass, const double* r, const double* ru,
                        double tol, bool chord, int32_t max_iter, double* r_out, double* lambda, int32_t* iters) {
  Rep<T> R(M, S, mass, r, ru);
  const int32_t n = M.n;
  if (chord) {
    for (int32_t k = 0; k < n; ++k) R.build_row(k, R.ex[k], R.ey[k], R.ez[k]);
    R.factor_sweep(false, true);
  }
  int32_t it = 0, st = ILVES_ERR_NOT_CONVERGED;
  if (R.singular) st = ILVES_ERR_SINGULAR;
  while (!R.singular) {
    double vmax = 0.0;
    for (int32_t k = 0; k < n; ++k) {
      double px, py, pz;
      R.bond(k, px, py, pz);
      vmax = std::fmax(vmax, R.violation(k, px, py, pz));
      if (!chord) R.build_row(k, px, py, pz);
    }
    if (vmax == INFINITY) { st = ILVES_ERR_NONFINITE; break; }
    if (vmax <= tol) { st = ILVES_OK; break; }
    if (it >= max_iter) { st = ILVES_ERR_NOT_CONVERGED; break; }
    R.factor_sweep(true, !chord);
    if (R.singular) { st = ILVES_ERR_SINGULAR; break; }
    R.back(M.n_levels);
    R.update();
    ++it;
  }
  R.outputs(r_out, lambda, [](int32_t) { return true; });
  *iters = it;
  return st;
}

// Block-bordered solve of a split molecule, in the order of the device
// scheme (every part's phase completes before the next phase starts).
template <typename T>
int32_t replay_split(const ilves::SplitPlan& SP, int32_t S, const double* mass, const double* r, const double* ru,
                     double tol, bool chord, int32_t max_iter, double* r_out, double* lambda, int32_t* iters) {
  const int32_t G = static_cast<int32_t>(SP.parts.size()), m = SP.m;
  std::vector<Rep<T>> R;
  R.reserve(G);
  for (int32_t g = 0; g < G; ++g) R.emplace_back(SP.parts[g], S, mass, r, ru);
  auto nb = [&](int32_t g) { return SP.parts[g].n - SP.parts[g].n_int; };
  auto gcoup = [&](int32_t c) { return ((c & 1) ? -1.0 : 1.0) / mass[c >> 1]; };
  // per part, border block (row-major nb x nb): matrix, unit-lower and
  // upper factors, Schur contribution E; w and g of the border rows
  std::vector<std::vector<double>> Ab(G), Lb(G), Ub(G), E(G), w(G), gB(G);
  for (int32_t g = 0; g < G; ++g) {
    const int32_t b = nb(g);
    Ab[g].assign(b * b, 0.0); Lb[g].assign(b * b, 0.0); Ub[g].assign(b * b, 0.0);
    E[g].assign(b * b, 0.0); w[g].assign(b, 0.0); gB[g].assign(b, 0.0);
  }
  auto border_matrix = [&](int32_t g) {
    const ilves::MolPlan& M = SP.parts[g];
    Rep<T>& P = R[g];
    const int32_t b = nb(g), ni = M.n_int;
    std::fill(Ab[g].begin(), Ab[g].end(), 0.0);
    for (int32_t j = 0; j < b; ++j) {
      const int32_t k = ni + j;
      Ab[g][j * b + j] = static_cast<double>(P.D[k]);
      for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q)
        Ab[g][j * b + (M.ucol[q] - ni)] = static_cast<double>(P.F[q]);
      for (int32_t t = M.l_start[k]; t < M.l_start[k + 1]; ++t)
        if (M.lcol[t - M.n_up] >= ni) Ab[g][j * b + (M.lcol[t - M.n_up] - ni)] = static_cast<double>(P.F[t]);
    }
  };
  auto border_factors = [&](int32_t g) {  // after the factorisation
    const ilves::MolPlan& M = SP.parts[g];
    Rep<T>& P = R[g];
    const int32_t b = nb(g), ni = M.n_int;
    std::fill(Lb[g].begin(), Lb[g].end(), 0.0);
    std::fill(Ub[g].begin(), Ub[g].end(), 0.0);
    for (int32_t j = 0; j < b; ++j) {
      const int32_t k = ni + j;
      Lb[g][j * b + j] = 1.0;
      Ub[g][j * b + j] = 1.0 / static_cast<double>(P.D[k]);
      for (int32_t q = M.up_start[k]; q < M.up_start[k + 1]; ++q)
        Ub[g][j * b + (M.ucol[q] - ni)] = static_cast<double>(P.F[q]);
      for (int32_t t = M.l_start[k]; t < M.l_start[k + 1]; ++t) {
        const int32_t i = M.lcol[t - M.n_up];
        if (i >= ni) Lb[g][j * b + (i - ni)] = static_cast<double>(P.F[t]) * static_cast<double>(P.D[i]);
      }
    }
    for (int32_t p = 0; p < b; ++p)
      for (int32_t q = 0; q < b; ++q) {
        double acc = 0.0;
        for (int32_t t = 0; t <= std::min(p, q); ++t) acc += Lb[g][p * b + t] * Ub[g][t * b + q];
        E[g][p * b + q] = acc - Ab[g][p * b + q];
      }
  };
  auto border_rhs = [&](int32_t g) {  // after the forward substitution
    const int32_t b = nb(g), ni = SP.parts[g].n_int;
    for (int32_t p = 0; p < b; ++p) {
      double acc = static_cast<double>(R[g].y[ni + p]);
      for (int32_t t = 0; t < p; ++t) acc += Lb[g][p * b + t] * static_cast<double>(R[g].y[ni + t]);
      w[g][p] = gB[g][p] - acc;
    }
  };
  // separator rows: bond vectors and residuals from their owners
  std::vector<double> ep(3 * m), es(3 * m), gs(m), cds(m);
  for (int32_t b = 0; b < m; ++b) {
    const int32_t o = SP.sep_part[2 * b], k = SP.parts[o].n_int + SP.sep_loc[2 * b];
    es[3 * b] = R[o].ex[k]; es[3 * b + 1] = R[o].ey[k]; es[3 * b + 2] = R[o].ez[k];
    cds[b] = 1.0 / mass[SP.sep_ga[b]] + 1.0 / mass[SP.sep_gb[b]];
  }
  std::vector<double> Sm(m * (m + 1)), z(m);
  auto assemble = [&](const std::vector<double>& pv) {
    for (int32_t b = 0; b < m; ++b) {
      for (int32_t c = 0; c <= m; ++c) Sm[b * (m + 1) + c] = 0.0;
      Sm[b * (m + 1) + b] = cds[b] * (pv[3 * b] * es[3 * b] + pv[3 * b + 1] * es[3 * b + 1] + pv[3 * b + 2] * es[3 * b + 2]);
      for (int32_t a = SP.sadj_ptr[b]; a < SP.sadj_ptr[b + 1]; ++a) {
        const int32_t c = SP.sadj_col[a];
        Sm[b * (m + 1) + c] = gcoup(SP.sadj_coef[a]) *
                              (pv[3 * b] * es[3 * c] + pv[3 * b + 1] * es[3 * c + 1] + pv[3 * b + 2] * es[3 * c + 2]);
      }
    }
    for (int32_t b = 0; b < m; ++b)
      for (int32_t c = 0; c < m; ++c)
        for (int32_t u = 0; u < 2; ++u) {
          const int32_t g = SP.sep_part[2 * b + u];
          for (int32_t v = 0; v < 2; ++v)
            if (SP.sep_part[2 * c + v] == g)
              Sm[b * (m + 1) + c] += E[g][SP.sep_loc[2 * b + u] * nb(g) + SP.sep_loc[2 * c + v]];
        }
  };
  // no pivoting; false if a pivot falls below 1e-13 of its row's largest
  // entry before the elimination
  auto eliminate = [&](int32_t cols) {
    std::vector<double> amax(m, 0.0);
    for (int32_t p = 0; p < m; ++p)
      for (int32_t c = 0; c < m; ++c) amax[p] = std::fmax(amax[p], std::fabs(Sm[p * (m + 1) + c]));
    for (int32_t p = 0; p < m; ++p) {
      const double piv = Sm[p * (m + 1) + p];
      if (!(std::fabs(piv) > 1e-13 * amax[p])) return false;
      const double inv = 1.0 / piv;
      for (int32_t q = p + 1; q < m; ++q) {
        const double f = Sm[q * (m + 1) + p] * inv;
        for (int32_t c = p + 1; c < cols; ++c) Sm[q * (m + 1) + c] -= f * Sm[p * (m + 1) + c];
      }
    }
    return true;
  };
  auto sep_solve = [&](std::vector<double> rhs, bool forward) {
    if (forward)
      for (int32_t p = 0; p < m; ++p)
        for (int32_t q = p + 1; q < m; ++q) rhs[q] -= Sm[q * (m + 1) + p] / Sm[p * (m + 1) + p] * rhs[p];
    for (int32_t q = m - 1; q >= 0; --q) {
      double acc = rhs[q];
      for (int32_t c = q + 1; c < m; ++c) acc -= Sm[q * (m + 1) + c] * z[c];
      z[q] = acc / Sm[q * (m + 1) + q];
    }
  };
  auto residuals = [&](bool build) {
    double vmax = 0.0;
    for (int32_t g = 0; g < G; ++g) {
      const ilves::MolPlan& M = SP.parts[g];
      Rep<T>& P = R[g];
      for (int32_t k = 0; k < M.n; ++k) {
        double px, py, pz;
        P.bond(k, px, py, pz);
        if (k >= M.n_int) {
          const int32_t j = k - M.n_int;
          for (int32_t e = SP.ext_ptr[g][j]; e < SP.ext_ptr[g][j + 1]; ++e) {
            const Rep<T>& H = R[SP.ext_part[g][e]];
            const int32_t i = SP.ext_row[g][e];
            const double c = gcoup(SP.ext_coef[g][e]) * H.lam[i];
            px -= c * H.ex[i];
            py -= c * H.ey[i];
            pz -= c * H.ez[i];
          }
        }
        vmax = std::fmax(vmax, P.violation(k, px, py, pz));
        if (k >= M.n_int) {
          gB[g][k - M.n_int] = static_cast<double>(P.y[k]);
          for (int32_t b = 0; b < m; ++b)  // owners publish
            if (SP.sep_part[2 * b] == g && SP.sep_loc[2 * b] == k - M.n_int) {
              ep[3 * b] = px; ep[3 * b + 1] = py; ep[3 * b + 2] = pz;
              gs[b] = 0.5 * (px * px + py * py + pz * pz - M.d2[k]);
            }
        }
        if (build) P.build_row(k, px, py, pz);
      }
    }
    return vmax;
  };

  int32_t it = 0, st = ILVES_ERR_NOT_CONVERGED;
  bool sing = false;
  if (chord) {
    for (int32_t g = 0; g < G; ++g) {
      Rep<T>& P = R[g];
      for (int32_t k = 0; k < P.n; ++k) P.build_row(k, P.ex[k], P.ey[k], P.ez[k]);
      border_matrix(g);
      P.factor_sweep(false, true);
      sing = sing || P.singular;
      border_factors(g);
    }
    if (!sing) {
      assemble(es);
      sing = !eliminate(m);
    }
    if (sing) st = ILVES_ERR_SINGULAR;
  }
  while (!sing) {
    const double gmax = residuals(!chord);
    if (gmax == INFINITY) { st = ILVES_ERR_NONFINITE; break; }
    if (gmax <= tol) { st = ILVES_OK; break; }
    if (it >= max_iter) { st = ILVES_ERR_NOT_CONVERGED; break; }
    for (int32_t g = 0; g < G; ++g) {
      if (!chord) border_matrix(g);
      R[g].factor_sweep(true, !chord);
      if (R[g].singular) sing = true;
      if (!chord) border_factors(g);
      border_rhs(g);
    }
    if (!sing && !chord) {
      assemble(ep);
      sing = !eliminate(m);
    }
    if (sing) { st = ILVES_ERR_SINGULAR; break; }
    std::vector<double> rhs(m);
    for (int32_t b = 0; b < m; ++b)
      rhs[b] = gs[b] - w[SP.sep_part[2 * b]][SP.sep_loc[2 * b]] - w[SP.sep_part[2 * b + 1]][SP.sep_loc[2 * b + 1]];
    sep_solve(rhs, true);
    for (int32_t g = 0; g < G; ++g) {
      const ilves::MolPlan& M = SP.parts[g];
      for (int32_t b = 0; b < m; ++b)
        for (int32_t u = 0; u < 2; ++u)
          if (SP.sep_part[2 * b + u] == g) R[g].y[M.n_int + SP.sep_loc[2 * b + u]] = static_cast<T>(z[b]);
      R[g].back(M.h_int);
      R[g].update();
    }
    ++it;
  }
  for (int32_t g = 0; g < G; ++g) {
    const ilves::MolPlan& M = SP.parts[g];
    std::vector<char> own(M.n, 0);
    for (int32_t k = 0; k < M.n_int; ++k) own[k] = 1;
    for (int32_t b = 0; b < m; ++b)
      if (SP.sep_part[2 * b] == g) own[M.n_int + SP.sep_loc[2 * b]] = 1;
    R[g].outputs(r_out, lambda, [&](int32_t k) { return own[k] != 0; });
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
  int32_t split_rows = 4096, part_rows = 0;
  if (opt) {
    po.ordering = opt->ordering;
    if (opt->split_rows != 0) split_rows = opt->split_rows;
    part_rows = opt->split_part_rows;
  }
  std::vector<int32_t> free_atoms;
  auto mols = ilves::split_molecules(n_atoms, n_constraints, pairs, free_atoms);
  *n_molecules = static_cast<int32_t>(mols.size());
  for (int32_t g : free_atoms) {
    r_out[g] = r_u[g];
    r_out[n_atoms + g] = r_u[n_atoms + g];
    r_out[2 * n_atoms + g] = r_u[2 * n_atoms + g];
  }
  const int32_t cap = max_iter > 0 ? max_iter : (precision == ILVES_PREC_FP64 && variant == 0 ? 20 : 40);
  const bool chord = variant == ILVES_VARIANT_CHORD;
  int64_t nslots = 0, work = 0, maxlev = 0, fill = 0, n_split = 0;
  for (size_t i = 0; i < mols.size(); ++i) {
    int32_t it = 0, st = 0;
    ilves::SplitPlan SP;
    if (split_rows > 0 && static_cast<int32_t>(mols[i].size()) > split_rows &&
        ilves::plan_split_auto(mols[i], pairs, d, po, part_rows, SP)) {
      ++n_split;
      for (const auto& M : SP.parts) {
        nslots += static_cast<int64_t>(M.n) + M.n_up + M.n_l;
        work += M.n_upd;
        maxlev = std::max<int64_t>(maxlev, M.n_levels);
        fill += M.fill;
      }
      st = precision == ILVES_PREC_MIXED
               ? replay_split<float>(SP, n_atoms, mass, r, r_u, tol, chord, cap, r_out, lambda, &it)
               : replay_split<double>(SP, n_atoms, mass, r, r_u, tol, chord, cap, r_out, lambda, &it);
    } else {
      ilves::MolPlan M = ilves::plan_molecule(mols[i], pairs, d, po);
      nslots += static_cast<int64_t>(M.n) + M.n_up + M.n_l;
      work += M.n_upd;
      maxlev = std::max<int64_t>(maxlev, M.n_levels);
      fill += M.fill;
      st = precision == ILVES_PREC_MIXED
               ? replay_molecule<float>(M, n_atoms, mass, r, r_u, tol, chord, cap, r_out, lambda, &it)
               : replay_molecule<double>(M, n_atoms, mass, r, r_u, tol, chord, cap, r_out, lambda, &it);
    }
    if (iters) iters[i] = it;
    if (status) status[i] = st;
  }
  if (schedule_stats) {
    schedule_stats[0] = static_cast<int64_t>(mols.size());
    schedule_stats[1] = nslots;
    schedule_stats[2] = work;
    schedule_stats[3] = maxlev;
    schedule_stats[4] = fill;
    schedule_stats[5] = n_split;
  }
  return ILVES_OK;
}

}  // extern "C"
