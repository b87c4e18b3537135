// Pointwise fluxes of the compressible Euler / Navier-Stokes equations and their reverse
// (transposed-Jacobian) products, written in primitive variables (rho, u, v, w, p).
// Used by the vector-Jacobian-product kernels; plain C++ arithmetic, so the same header
// also compiles on the host for the finite-difference self-check.
//
// Conventions: every *_adj function ADDS the transposed-Jacobian product of the given
// output adjoint into the argument adjoints.  Derivative of |x| is 0 when |x| is within
// 1e-12 of the local sound speed (the kink), and max(a,b) splits its derivative evenly
// when the two arguments agree to 1e-12 relative.
#pragma once
#include <math.h>

#ifndef DGFN
#define DGFN __host__ __device__ __forceinline__
#endif

namespace dgf {

struct P {  // primitive state; ir = 1/r is kept so that no function divides by the density
  double r, u, v, w, p, ir;
};
struct PA {  // adjoint of a primitive state
  double r, u, v, w, p;
};

DGFN P prim(const double *U, double gm1) {
  P q;
  q.r = U[0];
  const double ir = 1.0 / U[0];
  q.ir = ir;
  q.u = U[1] * ir; q.v = U[2] * ir; q.w = U[3] * ir;
  q.p = gm1 * (U[4] - 0.5 * (U[1] * q.u + U[2] * q.v + U[3] * q.w));
  return q;
}

DGFN PA zero_pa() {
  PA a;
  a.r = a.u = a.v = a.w = a.p = 0.0;
  return a;
}

// conservative adjoint += (d prim / d U)^T a, for U = (rho, m, E), u = m/rho,
// p = (gamma-1)(E - |m|^2/(2 rho))
DGFN void cons_adj(const P &q, double gm1, const PA &a, double *Ub) {
  const double ir = q.ir;
  const double q2 = q.u * q.u + q.v * q.v + q.w * q.w;
  Ub[0] += a.r - (a.u * q.u + a.v * q.v + a.w * q.w) * ir + a.p * gm1 * 0.5 * q2;
  Ub[1] += a.u * ir - a.p * gm1 * q.u;
  Ub[2] += a.v * ir - a.p * gm1 * q.v;
  Ub[3] += a.w * ir - a.p * gm1 * q.w;
  Ub[4] += a.p * gm1;
}

// a conservative adjoint Ub expressed as a primitive adjoint: a += (dU/dP)^T Ub, so that
// cons_adj maps it back to Ub (U = (rho, rho u, rho v, rho w, p/(gamma-1) + rho |u|^2/2))
DGFN void prim_adj_of_cons(const P &q, double gm1, const double *Ub, PA &a) {
  const double q2 = q.u * q.u + q.v * q.v + q.w * q.w;
  a.r += Ub[0] + q.u * Ub[1] + q.v * Ub[2] + q.w * Ub[3] + 0.5 * q2 * Ub[4];
  a.u += q.r * (Ub[1] + q.u * Ub[4]);
  a.v += q.r * (Ub[2] + q.v * Ub[4]);
  a.w += q.r * (Ub[3] + q.w * Ub[4]);
  a.p += Ub[4] / gm1;
}

// total enthalpy H = g1 p / rho + |u|^2 / 2 with g1 = gamma / (gamma - 1)
DGFN double enthalpy(const P &q, double g1) { return g1 * q.p * q.ir + 0.5 * (q.u * q.u + q.v * q.v + q.w * q.w); }

DGFN void enthalpy_adj(const P &q, double g1, double Hb, PA &a) {
  const double k = Hb * g1 * q.ir;
  a.p += k;
  a.r -= k * q.p * q.ir;
  a.u += Hb * q.u; a.v += Hb * q.v; a.w += Hb * q.w;
}

DGFN double sound_speed(const P &q, double gamma) { return sqrt(gamma * q.p * q.ir); }

DGFN void sound_speed_adj(const P &q, double gamma, double c, double cb, PA &a) {
  // c = sqrt(gamma p / rho)
  const double k = cb * 0.5 / c * gamma * q.ir;
  a.p += k;
  a.r -= k * q.p * q.ir;
}

DGFN double kink_sign(double x, double scale) {
  if (fabs(x) <= 1e-12 * scale) return 0.0;
  return x > 0.0 ? 1.0 : -1.0;
}

// Euler flux along nv: (rho u_n, rho u u_n + p n, rho H u_n)
DGFN void euler_flux(const P &q, const double *nv, double g1, double *F) {
  const double un = q.u * nv[0] + q.v * nv[1] + q.w * nv[2];
  const double H = enthalpy(q, g1);
  F[0] = q.r * un;
  F[1] = q.r * q.u * un + q.p * nv[0];
  F[2] = q.r * q.v * un + q.p * nv[1];
  F[3] = q.r * q.w * un + q.p * nv[2];
  F[4] = q.r * H * un;
}

DGFN void euler_flux_adj(const P &q, const double *nv, double g1, const double *Fb, PA &a) {
  const double un = q.u * nv[0] + q.v * nv[1] + q.w * nv[2];
  const double H = enthalpy(q, g1);
  const double s = Fb[0] + Fb[1] * q.u + Fb[2] * q.v + Fb[3] * q.w + Fb[4] * H;  // coefficient of rho u_n
  a.r += s * un;
  a.u += q.r * nv[0] * s + q.r * un * Fb[1];
  a.v += q.r * nv[1] * s + q.r * un * Fb[2];
  a.w += q.r * nv[2] * s + q.r * un * Fb[3];
  a.p += Fb[1] * nv[0] + Fb[2] * nv[1] + Fb[3] * nv[2];
  enthalpy_adj(q, g1, Fb[4] * q.r * un, a);
}

// kinetic-energy preserving two-point flux: {rho}{u.n}, {u} F_rho + {p} n, F_rho {H}
DGFN void kep_flux(const P &A, const P &B, const double *nv, double g1, double *F) {
  const double um = 0.5 * (A.u + B.u), vm = 0.5 * (A.v + B.v), wm = 0.5 * (A.w + B.w);
  const double umn = um * nv[0] + vm * nv[1] + wm * nv[2];
  const double f0 = 0.5 * (A.r + B.r) * umn;
  const double pm = 0.5 * (A.p + B.p);
  F[0] = f0;
  F[1] = f0 * um + pm * nv[0];
  F[2] = f0 * vm + pm * nv[1];
  F[3] = f0 * wm + pm * nv[2];
  F[4] = f0 * 0.5 * (enthalpy(A, g1) + enthalpy(B, g1));
}

// reverse of kep_flux with the two total enthalpies given: the adjoints of the enthalpies are
// accumulated into hA, hB (enthalpy_adj maps them to the states)
DGFN void kep_flux_adj_h(const P &A, const P &B, double HA, double HB, const double *nv, const double *Fb, PA &aA,
                         PA &aB, double &hA, double &hB) {
  const double um = 0.5 * (A.u + B.u), vm = 0.5 * (A.v + B.v), wm = 0.5 * (A.w + B.w);
  const double umn = um * nv[0] + vm * nv[1] + wm * nv[2];
  const double rm = 0.5 * (A.r + B.r);
  const double f0 = rm * umn;
  const double Hm = 0.5 * (HA + HB);
  const double g0 = Fb[0] + Fb[1] * um + Fb[2] * vm + Fb[3] * wm + Fb[4] * Hm;  // adjoint of f0
  const double bu = Fb[1] * f0 + g0 * rm * nv[0];
  const double bv = Fb[2] * f0 + g0 * rm * nv[1];
  const double bw = Fb[3] * f0 + g0 * rm * nv[2];
  const double br = g0 * umn;
  const double bp = Fb[1] * nv[0] + Fb[2] * nv[1] + Fb[3] * nv[2];
  const double bH = Fb[4] * f0;
  aA.r += 0.5 * br; aA.u += 0.5 * bu; aA.v += 0.5 * bv; aA.w += 0.5 * bw; aA.p += 0.5 * bp;
  aB.r += 0.5 * br; aB.u += 0.5 * bu; aB.v += 0.5 * bv; aB.w += 0.5 * bw; aB.p += 0.5 * bp;
  hA += 0.5 * bH;
  hB += 0.5 * bH;
}

DGFN void kep_flux_adj(const P &A, const P &B, const double *nv, double g1, const double *Fb, PA &aA, PA &aB) {
  double hA = 0.0, hB = 0.0;
  kep_flux_adj_h(A, B, enthalpy(A, g1), enthalpy(B, g1), nv, Fb, aA, aB, hA, hB);
  enthalpy_adj(A, g1, hA, aA);
  enthalpy_adj(B, g1, hB, aB);
}

// mean of the two Euler fluxes
DGFN void central_flux(const P &A, const P &B, const double *nv, double g1, double *F) {
  double Fa[5], Fb_[5];
  euler_flux(A, nv, g1, Fa);
  euler_flux(B, nv, g1, Fb_);
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (Fa[v] + Fb_[v]);
}

DGFN void central_flux_adj(const P &A, const P &B, const double *nv, double g1, const double *Fb, PA &aA, PA &aB) {
  double h[5];
  for (int v = 0; v < 5; ++v) h[v] = 0.5 * Fb[v];
  euler_flux_adj(A, nv, g1, h, aA);
  euler_flux_adj(B, nv, g1, h, aB);
}

// logarithmic mean (a - b)/(ln a - ln b) of two positive numbers and its partial derivatives;
// for u = ((a - b)/(a + b))^2 below 1e-4 from the series of artanh(f)/f = 1 + u/3 + u^2/5 + u^3/7
// (f = (a - b)/(a + b)), where the difference of logarithms loses its accuracy
DGFN void logmean_d(double a, double b, double &L, double &La, double &Lb) {
  const double s = a + b, d = a - b, is = 1.0 / s, f = d * is, u = f * f;
  if (u < 1e-4) {
    const double h = 1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)));
    const double hu = 1.0 / 3.0 + u * (2.0 / 5.0 + u * (3.0 / 7.0));  // dh/du
    const double ih = 1.0 / h;
    L = 0.5 * s * ih;
    // L = s / (2 h(u)); du/da = 4 b d / s^3, du/db = -4 a d / s^3
    const double c = 2.0 * s * hu * ih * ih * d * is * is * is;
    La = 0.5 * ih - c * b;
    Lb = 0.5 * ih + c * a;
  } else {
    const double il = 1.0 / (log(a) - log(b));
    L = d * il;
    La = (1.0 - L / a) * il;
    Lb = (L / b - 1.0) * il;
  }
}

// entropy-conserving two-point flux (Chandrashekar) along nv, with beta = rho / (2 p):
// F_rho = rho^ln {u}.n, F_m = F_rho {u} + {rho}/(2 {beta}) n,
// F_E = F_rho (1 / (2 (gamma-1) beta^ln) - {|u|^2}/2) + {u}.F_m   (g1 = gamma / (gamma-1))
DGFN void ec_flux(const P &A, const P &B, const double *nv, double g1, double *F) {
  const double kg = g1 - 1.0;  // 1 / (gamma - 1)
  const double ba = 0.5 * A.r / A.p, bb = 0.5 * B.r / B.p;
  double rl, bl, t0, t1;
  logmean_d(A.r, B.r, rl, t0, t1);
  logmean_d(ba, bb, bl, t0, t1);
  const double um[3] = {0.5 * (A.u + B.u), 0.5 * (A.v + B.v), 0.5 * (A.w + B.w)};
  const double umn = um[0] * nv[0] + um[1] * nv[1] + um[2] * nv[2];
  const double ph = 0.5 * (A.r + B.r) / (ba + bb);
  const double q2m = 0.5 * ((A.u * A.u + A.v * A.v + A.w * A.w) + (B.u * B.u + B.v * B.v + B.w * B.w));
  F[0] = rl * umn;
  for (int k = 0; k < 3; ++k) F[1 + k] = F[0] * um[k] + ph * nv[k];
  F[4] = F[0] * (0.5 * kg / bl - 0.5 * q2m) + um[0] * F[1] + um[1] * F[2] + um[2] * F[3];
}

DGFN void ec_flux_adj(const P &A, const P &B, const double *nv, double g1, const double *Fb, PA &aA, PA &aB) {
  const double kg = g1 - 1.0;
  const double ipA = 1.0 / A.p, ipB = 1.0 / B.p;
  const double ba = 0.5 * A.r * ipA, bb = 0.5 * B.r * ipB;
  double rl, rla, rlb, bl, bla, blb;
  logmean_d(A.r, B.r, rl, rla, rlb);
  logmean_d(ba, bb, bl, bla, blb);
  const double um[3] = {0.5 * (A.u + B.u), 0.5 * (A.v + B.v), 0.5 * (A.w + B.w)};
  const double umn = um[0] * nv[0] + um[1] * nv[1] + um[2] * nv[2];
  const double rm = 0.5 * (A.r + B.r), ibm = 2.0 / (ba + bb);  // 1 / {beta}
  const double ph = 0.5 * rm * ibm;
  const double ibl = 1.0 / bl;
  const double q2m = 0.5 * ((A.u * A.u + A.v * A.v + A.w * A.w) + (B.u * B.u + B.v * B.v + B.w * B.w));
  const double F0 = rl * umn;
  const double e = 0.5 * kg * ibl - 0.5 * q2m;
  // reverse sweep
  double bum[3], bF0 = Fb[0] + Fb[4] * e, bph = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double Fm = F0 * um[k] + ph * nv[k];
    const double bFm = Fb[1 + k] + Fb[4] * um[k];  // F_m enters F_E through {u}.F_m
    bum[k] = Fb[4] * Fm + bFm * F0;
    bF0 += bFm * um[k];
    bph += bFm * nv[k];
  }
  const double be = Fb[4] * F0;
  const double brl = bF0 * umn, bumn = bF0 * rl;
  for (int k = 0; k < 3; ++k) bum[k] += bumn * nv[k];
  const double bbl = -be * 0.5 * kg * ibl * ibl;
  const double bq2m = -0.5 * be;
  const double brm = 0.5 * bph * ibm;
  const double bbm = -0.5 * bph * rm * ibm * ibm;
  // densities: {rho} and rho^ln
  aA.r += 0.5 * brm + brl * rla;
  aB.r += 0.5 * brm + brl * rlb;
  // beta = rho / (2 p): {beta} and beta^ln
  const double bba = 0.5 * bbm + bbl * bla, bbb = 0.5 * bbm + bbl * blb;
  aA.r += bba * 0.5 * ipA; aA.p -= bba * ba * ipA;
  aB.r += bbb * 0.5 * ipB; aB.p -= bbb * bb * ipB;
  // velocities: {u} and {|u|^2}
  aA.u += 0.5 * bum[0] + bq2m * A.u; aA.v += 0.5 * bum[1] + bq2m * A.v; aA.w += 0.5 * bum[2] + bq2m * A.w;
  aB.u += 0.5 * bum[0] + bq2m * B.u; aB.v += 0.5 * bum[1] + bq2m * B.v; aB.w += 0.5 * bum[2] + bq2m * B.w;
}

// two-point flux of kind vf (0 KEP, 1 EC, 2 central)
DGFN void pair_flux(int vf, const P &A, const P &B, const double *nv, double g1, double *F) {
  if (vf == 0) kep_flux(A, B, nv, g1, F);
  else if (vf == 1) ec_flux(A, B, nv, g1, F);
  else central_flux(A, B, nv, g1, F);
}
DGFN void pair_flux_adj(int vf, const P &A, const P &B, const double *nv, double g1, const double *Fb, PA &aA,
                        PA &aB) {
  if (vf == 0) kep_flux_adj(A, B, nv, g1, Fb, aA, aB);
  else if (vf == 1) ec_flux_adj(A, B, nv, g1, Fb, aA, aB);
  else central_flux_adj(A, B, nv, g1, Fb, aA, aB);
}

// Roe dissipation sum |lambda_k| alpha_k r_k (no entropy fix), unit normal nh
DGFN void roe_diss(const P &L, const P &R, const double *nh, double gm1, double g1, double *D) {
  const double sL = sqrt(L.r), sR = sqrt(R.r);
  const double is = 1.0 / (sL + sR);
  const double u = (sL * L.u + sR * R.u) * is, v = (sL * L.v + sR * R.v) * is, w = (sL * L.w + sR * R.w) * is;
  const double H = (sL * enthalpy(L, g1) + sR * enthalpy(R, g1)) * is;
  const double q2 = u * u + v * v + w * w;
  const double c2 = gm1 * (H - 0.5 * q2);
  const double c = sqrt(c2);
  const double rt = sL * sR;
  const double un = u * nh[0] + v * nh[1] + w * nh[2];
  const double dr = R.r - L.r, dp = R.p - L.p;
  const double du = R.u - L.u, dv = R.v - L.v, dw = R.w - L.w;
  const double dun = du * nh[0] + dv * nh[1] + dw * nh[2];
  const double ic2 = 1.0 / c2;
  const double a1 = 0.5 * (dp - rt * c * dun) * ic2, a5 = 0.5 * (dp + rt * c * dun) * ic2, a2 = dr - dp * ic2;
  const double l1 = fabs(un - c), l2 = fabs(un), l5 = fabs(un + c);
  const double tu = du - dun * nh[0], tv = dv - dun * nh[1], tw = dw - dun * nh[2];
  const double s1 = l1 * a1, s5 = l5 * a5, s2 = l2 * a2, ss = l2 * rt;
  D[0] = s1 + s2 + s5;
  D[1] = s1 * (u - c * nh[0]) + s2 * u + ss * tu + s5 * (u + c * nh[0]);
  D[2] = s1 * (v - c * nh[1]) + s2 * v + ss * tv + s5 * (v + c * nh[1]);
  D[3] = s1 * (w - c * nh[2]) + s2 * w + ss * tw + s5 * (w + c * nh[2]);
  D[4] = s1 * (H - un * c) + s2 * 0.5 * q2 + ss * (u * tu + v * tv + w * tw) + s5 * (H + un * c);
}

DGFN void roe_diss_adj(const P &L, const P &R, const double *nh, double gm1, double g1, const double *Db, PA &aL,
                       PA &aR) {
  // forward sweep (same operations as roe_diss)
  const double sL = sqrt(L.r), sR = sqrt(R.r);
  const double is = 1.0 / (sL + sR);
  const double HL = enthalpy(L, g1), HR = enthalpy(R, g1);
  const double nu[3] = {sL * L.u + sR * R.u, sL * L.v + sR * R.v, sL * L.w + sR * R.w};
  const double uu[3] = {nu[0] * is, nu[1] * is, nu[2] * is};
  const double nH = sL * HL + sR * HR;
  const double H = nH * is;
  const double q2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
  const double c2 = gm1 * (H - 0.5 * q2);
  const double c = sqrt(c2);
  const double rt = sL * sR;
  const double un = uu[0] * nh[0] + uu[1] * nh[1] + uu[2] * nh[2];
  const double dr = R.r - L.r, dp = R.p - L.p;
  const double d[3] = {R.u - L.u, R.v - L.v, R.w - L.w};
  const double dun = d[0] * nh[0] + d[1] * nh[1] + d[2] * nh[2];
  const double ic2 = 1.0 / c2;
  const double a1 = 0.5 * (dp - rt * c * dun) * ic2, a5 = 0.5 * (dp + rt * c * dun) * ic2, a2 = dr - dp * ic2;
  const double l1 = fabs(un - c), l2 = fabs(un), l5 = fabs(un + c);
  const double t[3] = {d[0] - dun * nh[0], d[1] - dun * nh[1], d[2] - dun * nh[2]};
  const double s1 = l1 * a1, s5 = l5 * a5, s2 = l2 * a2, ss = l2 * rt;
  const double ut = uu[0] * t[0] + uu[1] * t[1] + uu[2] * t[2];
  // reverse sweep
  double bs1 = Db[0] + Db[4] * (H - un * c), bs5 = Db[0] + Db[4] * (H + un * c), bs2 = Db[0] + Db[4] * 0.5 * q2;
  double bss = Db[4] * ut;
  double bu[3], bt[3];
  double bc = 0.0, bun = 0.0;
  for (int k = 0; k < 3; ++k) {
    bs1 += Db[1 + k] * (uu[k] - c * nh[k]);
    bs5 += Db[1 + k] * (uu[k] + c * nh[k]);
    bs2 += Db[1 + k] * uu[k];
    bss += Db[1 + k] * t[k];
    bu[k] = Db[1 + k] * (s1 + s2 + s5) + Db[4] * (s2 * uu[k] + ss * t[k]);
    bt[k] = Db[1 + k] * ss + Db[4] * ss * uu[k];
    bc += Db[1 + k] * (s5 - s1) * nh[k];
  }
  bc += Db[4] * (s5 - s1) * un;
  bun += Db[4] * (s5 - s1) * c;
  double bH = Db[4] * (s1 + s5);
  // s = l * a
  const double bl1 = bs1 * a1, ba1 = bs1 * l1, bl5 = bs5 * a5, ba5 = bs5 * l5;
  double bl2 = bs2 * a2 + bss * rt;
  const double ba2 = bs2 * l2;
  double brt = bss * l2;
  // |.| with the kink convention (scale c)
  const double g1s = kink_sign(un - c, c), g5s = kink_sign(un + c, c), g2s = kink_sign(un, c);
  bun += bl1 * g1s + bl5 * g5s + bl2 * g2s;
  bc += -bl1 * g1s + bl5 * g5s;
  // tangential jump t = d - (d.n) n
  double bd[3] = {bt[0], bt[1], bt[2]};
  double bdun = -(bt[0] * nh[0] + bt[1] * nh[1] + bt[2] * nh[2]);
  // wave strengths
  double bdp = 0.5 * ba1 * ic2 + 0.5 * ba5 * ic2 - ba2 * ic2;
  const double bdr = ba2;
  brt += 0.5 * (ba5 - ba1) * c * dun * ic2;
  bc += 0.5 * (ba5 - ba1) * rt * dun * ic2;
  bdun += 0.5 * (ba5 - ba1) * rt * c * ic2;
  const double bic2 = ba1 * 0.5 * (dp - rt * c * dun) + ba5 * 0.5 * (dp + rt * c * dun) - ba2 * dp;
  double bc2 = -bic2 * ic2 * ic2 + bc * 0.5 * c * ic2;  // 1/c = c / c^2
  // un = u . n
  for (int k = 0; k < 3; ++k) bu[k] += bun * nh[k];
  // c2 = gm1 (H - q2/2)
  bH += gm1 * bc2;
  const double bq2 = -0.5 * gm1 * bc2;
  for (int k = 0; k < 3; ++k) bu[k] += 2.0 * bq2 * uu[k];
  for (int k = 0; k < 3; ++k) bd[k] += bdun * nh[k];
  // Roe averages
  double bis = bH * nH;
  const double bnH = bH * is;
  double bsL = bnH * HL + brt * sR, bsR = bnH * HR + brt * sL;
  const double bHL = bnH * sL, bHR = bnH * sR;
  const double uL[3] = {L.u, L.v, L.w}, uR[3] = {R.u, R.v, R.w};
  double buL[3], buR[3];
  for (int k = 0; k < 3; ++k) {
    bis += bu[k] * nu[k];
    const double bnu = bu[k] * is;
    bsL += bnu * uL[k];
    bsR += bnu * uR[k];
    buL[k] = bnu * sL - bd[k];
    buR[k] = bnu * sR + bd[k];
  }
  bsL -= bis * is * is;
  bsR -= bis * is * is;
  aL.r += bsL * 0.5 * sL * L.ir - bdr;  // 1/sqrt(rho) = sqrt(rho) / rho
  aR.r += bsR * 0.5 * sR * R.ir + bdr;
  aL.p -= bdp;
  aR.p += bdp;
  aL.u += buL[0]; aL.v += buL[1]; aL.w += buL[2];
  aR.u += buR[0]; aR.v += buR[1]; aR.w += buR[2];
  enthalpy_adj(L, g1, bHL, aL);
  enthalpy_adj(R, g1, bHR, aR);
}

// convective numerical flux f*(L, R, nh): rs 0 LLF, 1 Roe, 2 two-point flux, 3 two-point flux + Roe
// dissipation; UL, UR are the conservative states (LLF dissipates their jump)
DGFN void riemann(int rs, int vf, const P &L, const P &R, const double *UL, const double *UR, const double *nh,
                  double gamma, double *F) {
  const double gm1 = gamma - 1.0, g1 = gamma / gm1;
  if (rs >= 2) {
    pair_flux(vf, L, R, nh, g1, F);
    if (rs == 3) {
      double D[5];
      roe_diss(L, R, nh, gm1, g1, D);
      for (int v = 0; v < 5; ++v) F[v] -= 0.5 * D[v];
    }
    return;
  }
  double FL[5], FR[5];
  euler_flux(L, nh, g1, FL);
  euler_flux(R, nh, g1, FR);
  if (rs == 0) {
    const double cL = sound_speed(L, gamma), cR = sound_speed(R, gamma);
    const double unL = L.u * nh[0] + L.v * nh[1] + L.w * nh[2], unR = R.u * nh[0] + R.v * nh[1] + R.w * nh[2];
    const double lam = fmax(fabs(unL) + cL, fabs(unR) + cR);
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (UR[v] - UL[v]);
    return;
  }
  double D[5];
  roe_diss(L, R, nh, gm1, g1, D);
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

// reverse of riemann: primitive adjoints of both states (accumulated into aL, aR); the LLF
// jump term, linear in the conservative states, enters through (dU/dP)^T
DGFN void riemann_adj_prim(int rs, int vf, const P &L, const P &R, const double *UL, const double *UR,
                           const double *nh, double gamma, const double *Fb, PA &aL, PA &aR) {
  const double gm1 = gamma - 1.0, g1 = gamma / gm1;
  if (rs >= 2) {
    pair_flux_adj(vf, L, R, nh, g1, Fb, aL, aR);
    if (rs == 3) {
      double Dbar[5];
      for (int v = 0; v < 5; ++v) Dbar[v] = -0.5 * Fb[v];
      roe_diss_adj(L, R, nh, gm1, g1, Dbar, aL, aR);
    }
  } else {
    double h[5];
    for (int v = 0; v < 5; ++v) h[v] = 0.5 * Fb[v];
    euler_flux_adj(L, nh, g1, h, aL);
    euler_flux_adj(R, nh, g1, h, aR);
    if (rs == 0) {
      const double cL = sound_speed(L, gamma), cR = sound_speed(R, gamma);
      const double unL = L.u * nh[0] + L.v * nh[1] + L.w * nh[2], unR = R.u * nh[0] + R.v * nh[1] + R.w * nh[2];
      const double xL = fabs(unL) + cL, xR = fabs(unR) + cR;
      const double lam = fmax(xL, xR);
      double blam = 0.0, jL[5], jR[5];
      for (int v = 0; v < 5; ++v) {
        blam -= 0.5 * Fb[v] * (UR[v] - UL[v]);
        jL[v] = 0.5 * lam * Fb[v];
        jR[v] = -0.5 * lam * Fb[v];
      }
      prim_adj_of_cons(L, gm1, jL, aL);
      prim_adj_of_cons(R, gm1, jR, aR);
      double wL, wR;
      if (fabs(xL - xR) <= 1e-12 * fmax(fabs(xL), fabs(xR))) { wL = 0.5; wR = 0.5; }
      else if (xL > xR) { wL = 1.0; wR = 0.0; }
      else { wL = 0.0; wR = 1.0; }
      const double bxL = blam * wL, bxR = blam * wR;
      const double sgL = kink_sign(unL, cL), sgR = kink_sign(unR, cR);
      aL.u += bxL * sgL * nh[0]; aL.v += bxL * sgL * nh[1]; aL.w += bxL * sgL * nh[2];
      aR.u += bxR * sgR * nh[0]; aR.v += bxR * sgR * nh[1]; aR.w += bxR * sgR * nh[2];
      sound_speed_adj(L, gamma, cL, bxL, aL);
      sound_speed_adj(R, gamma, cR, bxR, aR);
    } else {
      double Dbar[5];
      for (int v = 0; v < 5; ++v) Dbar[v] = -0.5 * Fb[v];
      roe_diss_adj(L, R, nh, gm1, g1, Dbar, aL, aR);
    }
  }
}

// reverse of riemann: conservative adjoints of both states (accumulated)
DGFN void riemann_adj(int rs, int vf, const P &L, const P &R, const double *UL, const double *UR, const double *nh,
                      double gamma, const double *Fb, double *ULb, double *URb) {
  PA aL = zero_pa(), aR = zero_pa();
  riemann_adj_prim(rs, vf, L, R, UL, UR, nh, gamma, Fb, aL, aR);
  cons_adj(L, gamma - 1.0, aL, ULb);
  cons_adj(R, gamma - 1.0, aR, URb);
}

// viscous flux along nv (components 0..4, component 0 is zero); g[d*4+c] = dW_c/dx_d with
// W = (u, v, w, T); Newtonian stress with Stokes' hypothesis and Fourier heat flux
DGFN void visc_flux(const P &q, const double *g, double mu, double kappa, const double *nv, double *F) {
  const double div = g[0] + g[5] + g[10];
  const double t00 = mu * (2.0 * g[0] - (2.0 / 3.0) * div);
  const double t11 = mu * (2.0 * g[5] - (2.0 / 3.0) * div);
  const double t22 = mu * (2.0 * g[10] - (2.0 / 3.0) * div);
  const double t01 = mu * (g[4] + g[1]);
  const double t02 = mu * (g[8] + g[2]);
  const double t12 = mu * (g[9] + g[6]);
  F[0] = 0.0;
  F[1] = t00 * nv[0] + t01 * nv[1] + t02 * nv[2];
  F[2] = t01 * nv[0] + t11 * nv[1] + t12 * nv[2];
  F[3] = t02 * nv[0] + t12 * nv[1] + t22 * nv[2];
  F[4] = F[1] * q.u + F[2] * q.v + F[3] * q.w + kappa * (g[3] * nv[0] + g[7] * nv[1] + g[11] * nv[2]);
}

// reverse of visc_flux given its momentum part tn = tau . nv (the flux is linear in the gradients
// and depends on the state only through u in tau . u): a (velocity part) and gb[12] accumulated
DGFN void visc_flux_adj_tn(const P &q, const double *tn, double mu, double kappa, const double *nv, const double *Fb,
                           PA &a, double *gb) {
  a.u += Fb[4] * tn[0];
  a.v += Fb[4] * tn[1];
  a.w += Fb[4] * tn[2];
  const double bm[3] = {Fb[1] + Fb[4] * q.u, Fb[2] + Fb[4] * q.v, Fb[3] + Fb[4] * q.w};
  // tau_ab adjoint = bm_a nv_b ; tau_ab = mu (du_a/dx_b + du_b/dx_a) - 2/3 mu div delta_ab
  double tb[3][3];
  for (int a_ = 0; a_ < 3; ++a_)
    for (int b_ = 0; b_ < 3; ++b_) tb[a_][b_] = bm[a_] * nv[b_];
  const double tr = tb[0][0] + tb[1][1] + tb[2][2];
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) {
      // g[d*4+c] = du_c/dx_d enters tau_cd and tau_dc
      double v = mu * (tb[c][d] + tb[d][c]);
      if (c == d) v -= (2.0 / 3.0) * mu * tr;
      gb[d * 4 + c] += v;
    }
  for (int d = 0; d < 3; ++d) gb[d * 4 + 3] += Fb[4] * kappa * nv[d];
}

// reverse of visc_flux: a (velocity part) and gb[12] accumulated; F[0] has no dependence
DGFN void visc_flux_adj(const P &q, const double *g, double mu, double kappa, const double *nv, const double *Fb,
                        PA &a, double *gb) {
  double Fv[5];
  visc_flux(q, g, mu, kappa, nv, Fv);
  visc_flux_adj_tn(q, Fv + 1, mu, kappa, nv, Fb, a, gb);
}

// lifted variables W = (u, v, w, T = p / (rho R)): adjoint into primitive adjoint
DGFN void lift_vars_adj(const P &q, double Rg, const double *Wb, PA &a) {
  a.u += Wb[0]; a.v += Wb[1]; a.w += Wb[2];
  const double k = Wb[3] * q.ir / Rg;
  a.p += k;
  a.r -= k * q.p * q.ir;
}

}  // namespace dgf
