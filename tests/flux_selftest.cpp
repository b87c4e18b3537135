// Host self-check of the reverse flux products in dg_flux.h: for random states and random
// output adjoints, the transposed-Jacobian product must equal the central finite difference of
// <adjoint, flux> along every input coordinate.  Prints one line per function with the largest
// relative mismatch and returns non-zero if any exceeds the tolerance.
#define DGFN inline
#include "../paper_1910_02858_amd/csrc/dg_flux.h"

#include <cstdio>
#include <cstdlib>
#include <random>

using namespace dgf;

static std::mt19937_64 rng(7);
static double urand(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static P rand_prim(double mach) {
  P q;
  q.r = urand(0.6, 1.6);
  q.p = urand(0.6, 1.6);
  q.u = urand(-1, 1) * mach; q.v = urand(-1, 1) * mach; q.w = urand(-1, 1) * mach;
  q.ir = 1.0 / q.r;
  return q;
}
static void to_cons(const P &q, double gamma, double *U) {
  U[0] = q.r; U[1] = q.r * q.u; U[2] = q.r * q.v; U[3] = q.r * q.w;
  U[4] = q.p / (gamma - 1) + 0.5 * q.r * (q.u * q.u + q.v * q.v + q.w * q.w);
}
static double *comp(P &q, int j) { return j == 0 ? &q.r : j == 1 ? &q.u : j == 2 ? &q.v : j == 3 ? &q.w : &q.p; }
static double comp(const PA &a, int j) { return j == 0 ? a.r : j == 1 ? a.u : j == 2 ? a.v : j == 3 ? a.w : a.p; }
// q with component j moved by h (the cached reciprocal density follows)
static P moved(P q, int j, double h) {
  *comp(q, j) += h;
  q.ir = 1.0 / q.r;
  return q;
}

static int failures = 0;
static void report(const char *name, double err, double tol) {
  std::printf("%-28s max rel err %.3e %s\n", name, err, err <= tol ? "ok" : "FAIL");
  if (!(err <= tol)) ++failures;
}

template <class F> static double fd_dir(F f, double h) { return (f(h) - f(-h)) / (2 * h); }
// fourth-order central difference (the log means of states far apart have large third derivatives)
template <class F> static double fd4_dir(F f, double h) {
  return (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h);
}

int main() {
  const double gamma = 1.4, gm1 = gamma - 1, g1 = gamma / gm1, tol = 2e-7;
  double worst;
  // Euler flux
  worst = 0;
  for (int it = 0; it < 200; ++it) {
    P q = rand_prim(0.8);
    double nv[3] = {urand(-1, 1), urand(-1, 1), urand(-1, 1)}, Fb[5];
    for (double &x : Fb) x = urand(-1, 1);
    PA a = zero_pa();
    euler_flux_adj(q, nv, g1, Fb, a);
    for (int j = 0; j < 5; ++j) {
      auto f = [&](double h) { P t = moved(q, j, h); double F[5]; euler_flux(t, nv, g1, F);
                               double s = 0; for (int v = 0; v < 5; ++v) s += Fb[v] * F[v]; return s; };
      double fd = fd_dir(f, 1e-6), an = comp(a, j);
      worst = std::max(worst, std::fabs(fd - an) / (std::fabs(an) + 1e-3));
    }
  }
  report("euler_flux_adj", worst, tol);
  // logarithmic mean: value against the logarithms away from a = b, derivatives against central
  // differences on both branches
  worst = 0;
  for (int it = 0; it < 400; ++it) {
    const double a = urand(0.3, 3.0), b = it % 2 ? a * (1.0 + urand(-1e-3, 1e-3)) : urand(0.3, 3.0);
    double L, La, Lb;
    logmean_d(a, b, L, La, Lb);
    if (std::fabs(a - b) > 0.05 * a) worst = std::max(worst, std::fabs(L - (a - b) / (std::log(a) - std::log(b))) / L);
    auto fa = [&](double h) { double l, x, y; logmean_d(a + h, b, l, x, y); return l; };
    auto fb = [&](double h) { double l, x, y; logmean_d(a, b + h, l, x, y); return l; };
    worst = std::max(worst, std::fabs(fd_dir(fa, 1e-7) - La) / std::fabs(La));
    worst = std::max(worst, std::fabs(fd_dir(fb, 1e-7) - Lb) / std::fabs(Lb));
  }
  report("logmean_d", worst, tol);
  // two-point fluxes (EC also with nearly equal states, the series branch of the log means)
  for (int vf : {0, 1, 2, 3}) {
    worst = 0;
    for (int it = 0; it < 200; ++it) {
      P A = rand_prim(0.8), B = rand_prim(0.8);
      if (vf == 3) {
        B = A;
        B.r *= 1.0 + urand(-2e-3, 2e-3); B.p *= 1.0 + urand(-2e-3, 2e-3); B.ir = 1.0 / B.r;
      }
      double nv[3] = {urand(-1, 1), urand(-1, 1), urand(-1, 1)}, Fb[5];
      for (double &x : Fb) x = urand(-1, 1);
      PA aA = zero_pa(), aB = zero_pa();
      pair_flux_adj(vf == 3 ? 1 : vf, A, B, nv, g1, Fb, aA, aB);
      for (int side = 0; side < 2; ++side)
        for (int j = 0; j < 5; ++j) {
          auto f = [&](double h) { P a = side ? A : moved(A, j, h), b = side ? moved(B, j, h) : B; double F[5];
                                   pair_flux(vf == 3 ? 1 : vf, a, b, nv, g1, F);
                                   double s = 0; for (int v = 0; v < 5; ++v) s += Fb[v] * F[v]; return s; };
          double fd = fd4_dir(f, 1e-4), an = comp(side ? aB : aA, j);
          worst = std::max(worst, std::fabs(fd - an) / (std::fabs(an) + 1e-3));
        }
    }
    report(vf == 0 ? "kep_flux_adj" : vf == 1 ? "ec_flux_adj" : vf == 2 ? "central_flux_adj" : "ec_flux_adj near-equal",
           worst, tol);
  }
  // Roe dissipation
  worst = 0;
  for (int it = 0; it < 300; ++it) {
    P L = rand_prim(0.5), R = rand_prim(0.5);  // away from sonic points, where |u_n -+ c| has kinks
    double nh[3] = {urand(-1, 1), urand(-1, 1), urand(-1, 1)};
    double nn = std::sqrt(nh[0] * nh[0] + nh[1] * nh[1] + nh[2] * nh[2]);
    for (double &x : nh) x /= nn;
    double Db[5];
    for (double &x : Db) x = urand(-1, 1);
    PA aL = zero_pa(), aR = zero_pa();
    roe_diss_adj(L, R, nh, gm1, g1, Db, aL, aR);
    for (int side = 0; side < 2; ++side)
      for (int j = 0; j < 5; ++j) {
        auto f = [&](double h) { P a = side ? L : moved(L, j, h), b = side ? moved(R, j, h) : R; double D[5];
                                 roe_diss(a, b, nh, gm1, g1, D);
                                 double s = 0; for (int v = 0; v < 5; ++v) s += Db[v] * D[v]; return s; };
        double fd = fd_dir(f, 1e-5), an = comp(side ? aR : aL, j);
        worst = std::max(worst, std::fabs(fd - an) / (std::fabs(an) + 1e-3));
      }
  }
  report("roe_diss_adj", worst, tol);
  // full Riemann solvers in conservative variables (case 4: EC two-point flux + Roe dissipation)
  for (int rc : {0, 1, 3, 4}) {
    const int rs = rc == 4 ? 3 : rc, vf = rc == 4 ? 1 : 0;
    worst = 0;
    for (int it = 0; it < 200; ++it) {
      P L = rand_prim(0.5), R = rand_prim(0.5);
      double UL[5], UR[5];
      to_cons(L, gamma, UL); to_cons(R, gamma, UR);
      double nh[3] = {urand(-1, 1), urand(-1, 1), urand(-1, 1)};
      double nn = std::sqrt(nh[0] * nh[0] + nh[1] * nh[1] + nh[2] * nh[2]);
      for (double &x : nh) x /= nn;
      double Fb[5];
      for (double &x : Fb) x = urand(-1, 1);
      double ULb[5] = {0, 0, 0, 0, 0}, URb[5] = {0, 0, 0, 0, 0};
      riemann_adj(rs, vf, L, R, UL, UR, nh, gamma, Fb, ULb, URb);
      for (int side = 0; side < 2; ++side)
        for (int j = 0; j < 5; ++j) {
          auto f = [&](double h) { double a[5], b[5]; for (int v = 0; v < 5; ++v) { a[v] = UL[v]; b[v] = UR[v]; }
                                   (side ? b : a)[j] += h;
                                   P pa = prim(a, gm1), pb = prim(b, gm1); double F[5];
                                   riemann(rs, vf, pa, pb, a, b, nh, gamma, F);
                                   double s = 0; for (int v = 0; v < 5; ++v) s += Fb[v] * F[v]; return s; };
          double fd = fd_dir(f, 1e-5), an = (side ? URb : ULb)[j];
          worst = std::max(worst, std::fabs(fd - an) / (std::fabs(an) + 1e-3));
        }
    }
    report(rc == 0 ? "riemann_adj llf" : rc == 1 ? "riemann_adj roe" : rc == 3 ? "riemann_adj kep+roe" : "riemann_adj ec+roe",
           worst, tol);
  }
  // viscous flux (state and gradient) and lifted variables
  worst = 0;
  for (int it = 0; it < 200; ++it) {
    P q = rand_prim(0.8);
    double g[12], nv[3] = {urand(-1, 1), urand(-1, 1), urand(-1, 1)}, Fb[5];
    for (double &x : g) x = urand(-1, 1);
    for (double &x : Fb) x = urand(-1, 1);
    const double mu = 0.013, kappa = 0.021;
    PA a = zero_pa();
    double gb[12] = {0};
    visc_flux_adj(q, g, mu, kappa, nv, Fb, a, gb);
    for (int j = 0; j < 5 + 12; ++j) {
      auto f = [&](double h) { P t = q; double gg[12]; for (int c = 0; c < 12; ++c) gg[c] = g[c];
                               if (j < 5) t = moved(t, j, h); else gg[j - 5] += h;
                               double F[5]; visc_flux(t, gg, mu, kappa, nv, F);
                               double s = 0; for (int v = 0; v < 5; ++v) s += Fb[v] * F[v]; return s; };
      double fd = fd_dir(f, 1e-6), an = j < 5 ? comp(a, j) : gb[j - 5];
      worst = std::max(worst, std::fabs(fd - an) / (std::fabs(an) + 1e-3));
    }
  }
  report("visc_flux_adj", worst, tol);
  // primitive -> conservative adjoint map
  worst = 0;
  for (int it = 0; it < 200; ++it) {
    P q = rand_prim(0.8);
    double U[5];
    to_cons(q, gamma, U);
    PA a;
    a.r = urand(-1, 1); a.u = urand(-1, 1); a.v = urand(-1, 1); a.w = urand(-1, 1); a.p = urand(-1, 1);
    double Ub[5] = {0, 0, 0, 0, 0};
    cons_adj(q, gm1, a, Ub);
    for (int j = 0; j < 5; ++j) {
      auto f = [&](double h) { double V[5]; for (int v = 0; v < 5; ++v) V[v] = U[v]; V[j] += h;
                               P t = prim(V, gm1);
                               return a.r * t.r + a.u * t.u + a.v * t.v + a.w * t.w + a.p * t.p; };
      double fd = fd_dir(f, 1e-6);
      worst = std::max(worst, std::fabs(fd - Ub[j]) / (std::fabs(Ub[j]) + 1e-3));
    }
  }
  report("cons_adj", worst, tol);
  // conservative adjoint carried through primitive space and back
  worst = 0;
  for (int it = 0; it < 200; ++it) {
    P q = rand_prim(0.8);
    double Ub[5], back[5] = {0, 0, 0, 0, 0};
    for (double &x : Ub) x = urand(-1, 1);
    PA a = zero_pa();
    prim_adj_of_cons(q, gm1, Ub, a);
    cons_adj(q, gm1, a, back);
    for (int j = 0; j < 5; ++j) worst = std::max(worst, std::fabs(back[j] - Ub[j]) / (std::fabs(Ub[j]) + 1e-3));
  }
  report("prim_adj_of_cons round trip", worst, 1e-13);
  return failures ? 1 : 0;
}
