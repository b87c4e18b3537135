// HIP kernels of the DGSEM operator for gfx950 (one workgroup per element).
//
// Paper map (Krais et al., FLEXI):
//   k_lift  ... BR1 lifting of W = (u,v,w,T): Sec. 3.1, eq. discreteGradient, U* = mean of traces
//   k_main  ... volume integral (weak eq. semiDiscrete / strong eq. semiDiscreteStrong / split
//               flux differencing eq. semiDiscreteSplit), numerical surface flux (Riemann + BR1
//               viscous mean), surface integral, -1/J scaling, and optionally the 2N-storage
//               Runge-Kutta update of Sec. 4.4 fused into the epilogue.
//   k_reduce .. per-element partial sums for the time step (eqs. CFLCondition, DFLCondition),
//               quadrature integrals and the finiteness check, then one final pass.
//
// Layout: U[e][v][k][j][i] (i fastest), Ja[e][i*3+d][node], 1/J[e][node],
// outward normals fn[e][side][d][a + n*b].  Each workgroup stages its element's state in
// LDS; neighbour face values are read straight from global memory (for LGL nodes they are
// volume nodes of the neighbour's face layer; for LG nodes they are interpolated on the fly).
// Both elements sharing a face evaluate the same numerical flux with the master's normal and
// the master's state as the left argument, so the two contributions cancel to rounding.
#include <hip/hip_runtime.h>

#include "dg_internal.h"

// minimum waves per SIMD requested for the split-form kernel: 4 fits two 512-thread
// workgroups per CU at N=7 (128 VGPRs), measured faster than 2-3 waves despite a small spill
#ifndef DG_SPLIT_MINB
#define DG_SPLIT_MINB 4
#endif
// minimum waves per SIMD for the lifting kernel: 6 fits three 512-thread workgroups per CU
#ifndef DG_LIFT_MINB
#define DG_LIFT_MINB 6
#endif
// the lifting of meshes with non-conforming faces: at 80 registers it spills 44 bytes, at 128 (two
// workgroups per CU) none: 0.73 -> 0.65 ms at 16^3 N=7 half refined
#ifndef DG_LIFT_MORTAR_MINB
#define DG_LIFT_MORTAR_MINB 4
#endif

namespace dg {

template <int N> struct Sz {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static constexpr int NT = ((n3 + 63) / 64) * 64;  // threads per workgroup (one node each)
};

// node of the line through face point (a,b) of direction dn at position m along dn
template <int n> __device__ __forceinline__ int line_node(int dn, int a, int b, int m) {
  return dn == 0 ? (m + n * (a + n * b)) : (dn == 1 ? (a + n * (m + n * b)) : (a + n * (b + n * m)));
}

// Symmetry-plane (slip-wall) boundary: the outer side is the mirror image of the inner one across
// the plane with unit normal nh.  mirror3 reflects a 3-vector; mirror_grad reflects gradients
// g[d*4+v] = dW_v/dx_d of W = (u, v, w, T) in the derivative direction and, for the velocity
// block, also in the component.
__device__ __forceinline__ void mirror3(double *x, const double *nh) {
  const double xn = 2.0 * (x[0] * nh[0] + x[1] * nh[1] + x[2] * nh[2]);
  x[0] -= xn * nh[0];
  x[1] -= xn * nh[1];
  x[2] -= xn * nh[2];
}
__device__ __forceinline__ void mirror_grad(double *g, const double *nh) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double c[3] = {g[v], g[4 + v], g[8 + v]};
    mirror3(c, nh);
    g[v] = c[0]; g[4 + v] = c[1]; g[8 + v] = c[2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) mirror3(g + 4 * d, nh);
}
// side s of element e belongs to a non-conforming face (its terms come from the mortar arrays)
__device__ __forceinline__ bool is_mortar(const Geo &g, int e, int s) {
  if (!g.fc) return false;
  const int c = g.fc[(size_t)e * 6 + s];
  return (c & 128) && (c & 7) == FACE_MORTAR;
}
__device__ __forceinline__ void unit3(const double *x, double *nh) {
  const double il = 1.0 / sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  nh[0] = x[0] * il; nh[1] = x[1] * il; nh[2] = x[2] * il;
}

// ----------------------------------------------------------------------------- physics
// Reciprocal from v_rcp_f64 refined by two Newton steps (error well below one ulp of the
// quantities it feeds); used for the two-point fluxes, where IEEE division dominated.
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
struct Pr5 {
  double rho, u, v, w, p;
};

__device__ __forceinline__ Pr5 to_prim(const double *U, double gm1) {
  Pr5 P;
  P.rho = U[0];
  const double ir = frcp(U[0]);
  P.u = U[1] * ir; P.v = U[2] * ir; P.w = U[3] * ir;
  P.p = gm1 * (U[4] - 0.5 * (U[1] * P.u + U[2] * P.v + U[3] * P.w));
  return P;
}

// Euler flux along the (unnormalised) vector nv
__device__ __forceinline__ void flux_c(const double *U, const Pr5 &P, const double *nv, double *F) {
  const double un = P.u * nv[0] + P.v * nv[1] + P.w * nv[2];
  F[0] = U[0] * un;
  F[1] = U[1] * un + P.p * nv[0];
  F[2] = U[2] * un + P.p * nv[1];
  F[3] = U[3] * un + P.p * nv[2];
  F[4] = (U[4] + P.p) * un;
}

// viscous flux along nv; g[d*4+c] = dW_c/dx_d with W = (u, v, w, T)
__device__ __forceinline__ void flux_v(const Pr5 &P, const double *g, const Phys &ph, const double *nv, double *F) {
  const double mu = ph.mu;
  const double div = g[0] + g[5] + g[10];
  // tau[a][b] = mu (du_a/dx_b + du_b/dx_a) - 2/3 mu div delta_ab ; du_a/dx_b = g[b*4+a]
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
  // energy: (tau . u)_d + kappa dT/dx_d, contracted with nv
  F[4] = F[1] * P.u + F[2] * P.v + F[3] * P.w + ph.kappa * (g[3] * nv[0] + g[7] * nv[1] + g[11] * nv[2]);
}

__device__ __forceinline__ double logmean(double a, double b) {
  const double s = a + b;
  const double d = a - b;
  const double f = d / s;
  const double u = f * f;
  if (u < 1e-4) return s / (2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0))));
  // log(a) - log(b) as one logarithm, log1p of the difference over the smaller argument
  const double ad = fabs(d);
  return ad / log1p(ad / fmin(a, b));
}

// two-point flux along nv: vf 0 KEP (Pirozzoli), 1 EC (Chandrashekar), 2 central
__device__ __forceinline__ void flux_2pt(int vf, const double *Ua, const Pr5 &A, const double *Ub, const Pr5 &B,
                                         const double *nv, double gm1, double *F) {
  if (vf == 2) {
    double Fa[5], Fb[5];
    flux_c(Ua, A, nv, Fa);
    flux_c(Ub, B, nv, Fb);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (Fa[v] + Fb[v]);
    return;
  }
  const double um = 0.5 * (A.u + B.u), vm = 0.5 * (A.v + B.v), wm = 0.5 * (A.w + B.w);
  const double umn = um * nv[0] + vm * nv[1] + wm * nv[2];
  if (vf == 0) {
    const double rhom = 0.5 * (A.rho + B.rho);
    const double pm = 0.5 * (A.p + B.p);
    const double Hm = 0.5 * ((Ua[4] + A.p) / A.rho + (Ub[4] + B.p) / B.rho);
    const double f0 = rhom * umn;
    F[0] = f0;
    F[1] = f0 * um + pm * nv[0];
    F[2] = f0 * vm + pm * nv[1];
    F[3] = f0 * wm + pm * nv[2];
    F[4] = f0 * Hm;
    return;
  }
  const double ba = 0.5 * A.rho / A.p, bb = 0.5 * B.rho / B.p;
  const double rholn = logmean(A.rho, B.rho);
  const double betaln = logmean(ba, bb);
  const double phat = 0.25 * (A.rho + B.rho) / (0.5 * (ba + bb));
  const double q2m = 0.5 * ((A.u * A.u + A.v * A.v + A.w * A.w) + (B.u * B.u + B.v * B.v + B.w * B.w));
  const double f0 = rholn * umn;
  F[0] = f0;
  F[1] = f0 * um + phat * nv[0];
  F[2] = f0 * vm + phat * nv[1];
  F[3] = f0 * wm + phat * nv[2];
  F[4] = f0 * (0.5 / (gm1 * betaln) - 0.5 * q2m) + um * F[1] + vm * F[2] + wm * F[3];
}

// Roe dissipation sum |lambda_k| alpha_k r_k, written without a rotated frame:
// shear waves act on the tangential velocity jump du - (du.n) n.
__device__ __forceinline__ void roe_diss(const double *UL, const Pr5 &L, const double *UR, const Pr5 &R,
                                         const double *nh, double gm1, double *D) {
  const double sL = sqrt(L.rho), sR = sqrt(R.rho);
  const double is = 1.0 / (sL + sR);
  const double u = (sL * L.u + sR * R.u) * is;
  const double v = (sL * L.v + sR * R.v) * is;
  const double w = (sL * L.w + sR * R.w) * is;
  const double HL = (UL[4] + L.p) / L.rho, HR = (UR[4] + R.p) / R.rho;
  const double H = (sL * HL + sR * HR) * is;
  const double q2 = u * u + v * v + w * w;
  const double c2 = gm1 * (H - 0.5 * q2);
  const double c = sqrt(c2);
  const double rt = sL * sR;
  const double un = u * nh[0] + v * nh[1] + w * nh[2];
  const double dr = R.rho - L.rho, dp = R.p - L.p;
  const double du = R.u - L.u, dv = R.v - L.v, dw = R.w - L.w;
  const double dun = du * nh[0] + dv * nh[1] + dw * nh[2];
  const double ic2 = 1.0 / c2;
  const double a1 = 0.5 * (dp - rt * c * dun) * ic2;
  const double a5 = 0.5 * (dp + rt * c * dun) * ic2;
  const double a2 = dr - dp * ic2;
  const double l1 = fabs(un - c), l2 = fabs(un), l5 = fabs(un + c);
  const double tu = du - dun * nh[0], tv = dv - dun * nh[1], tw = dw - dun * nh[2];
  const double s1 = l1 * a1, s5 = l5 * a5, s2 = l2 * a2, ss = l2 * rt;
  D[0] = s1 + s2 + s5;
  D[1] = s1 * (u - c * nh[0]) + s2 * u + ss * tu + s5 * (u + c * nh[0]);
  D[2] = s1 * (v - c * nh[1]) + s2 * v + ss * tv + s5 * (v + c * nh[1]);
  D[3] = s1 * (w - c * nh[2]) + s2 * w + ss * tw + s5 * (w + c * nh[2]);
  D[4] = s1 * (H - un * c) + s2 * 0.5 * q2 + ss * (u * tu + v * tv + w * tw) + s5 * (H + un * c);
}

// convective numerical flux f*(UL, UR, nh), nh a unit normal
__device__ __forceinline__ void riemann(const Phys &ph, const double *UL, const double *UR, const double *nh,
                                        double *F) {
  const double gm1 = ph.gamma - 1.0;
  const Pr5 L = to_prim(UL, gm1), R = to_prim(UR, gm1);
  if (ph.rs >= 2) {
    flux_2pt(ph.vf, UL, L, UR, R, nh, gm1, F);
    if (ph.rs == 3) {
      double D[5];
      roe_diss(UL, L, UR, R, nh, gm1, D);
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] -= 0.5 * D[v];
    }
    return;
  }
  double FL[5], FR[5];
  flux_c(UL, L, nh, FL);
  flux_c(UR, R, nh, FR);
  if (ph.rs == 0) {
    const double cL = sqrt(ph.gamma * L.p / L.rho), cR = sqrt(ph.gamma * R.p / R.rho);
    const double unL = L.u * nh[0] + L.v * nh[1] + L.w * nh[2];
    const double unR = R.u * nh[0] + R.v * nh[1] + R.w * nh[2];
    const double lam = fmax(fabs(unL) + cL, fabs(unR) + cR);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (UR[v] - UL[v]);
    return;
  }
  double D[5];
  roe_diss(UL, L, UR, R, nh, gm1, D);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

// riemann() with the solver fixed at compile time (RS = ph.rs)
template <int RS>
__device__ __forceinline__ void riemann_t(const Phys &ph, const double *UL, const double *UR, const double *nh,
                                          double *F) {
  const double gm1 = ph.gamma - 1.0;
  const Pr5 L = to_prim(UL, gm1), R = to_prim(UR, gm1);
  if (RS >= 2) {
    flux_2pt(ph.vf, UL, L, UR, R, nh, gm1, F);
    if (RS == 3) {
      double D[5];
      roe_diss(UL, L, UR, R, nh, gm1, D);
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] -= 0.5 * D[v];
    }
    return;
  }
  double FL[5], FR[5];
  flux_c(UL, L, nh, FL);
  flux_c(UR, R, nh, FR);
  if (RS == 0) {
    const double cL = sqrt(ph.gamma * L.p / L.rho), cR = sqrt(ph.gamma * R.p / R.rho);
    const double unL = L.u * nh[0] + L.v * nh[1] + L.w * nh[2];
    const double unR = R.u * nh[0] + R.v * nh[1] + R.w * nh[2];
    const double lam = fmax(fabs(unL) + cL, fabs(unR) + cR);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (UR[v] - UL[v]);
    return;
  }
  double D[5];
  roe_diss(UL, L, UR, R, nh, gm1, D);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

// numerical flux of the split-form kernel: as riemann(), with the two-point variants (rs 2, 3)
// evaluated by the volume flux VF of the kernel (pair2, defined below)
template <int VF>
__device__ __forceinline__ void riemann_vf(const Phys &ph, const double *UL, const double *UR, const double *nh,
                                           double *F);

__device__ __forceinline__ void grad_prim_to_W(const double *U, double gm1, double Rg, double *W) {
  const Pr5 P = to_prim(U, gm1);
  W[0] = P.u; W[1] = P.v; W[2] = P.w; W[3] = P.p / (P.rho * Rg);
}

// ----------------------------------------------------------------------------- lifting
// LDS sizes (doubles) of one element in the lifting kernel
template <int N> struct LiftLds {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  // the three regions together hold 12 values per node at the end (the staged viscous fluxes of
  // LIFT_DIV)
  static constexpr int W = 4 * n3, JA = 3 * n3, WS = (24 * n2 > 5 * n3) ? 24 * n2 : 5 * n3;
};

// 1D tables of the lifting kernel into LDS (by the first threads of the workgroup)
template <int N>
__device__ __forceinline__ void lift_tables(const Tab *tb, int t, int nthreads, double *sDh, double *sl, double *slh) {
  constexpr int n = N + 1;
  for (int c = t; c < n * n; c += nthreads) sDh[c] = tb->Dh[c];
  if (t < n) {
    sl[t] = tb->lm[t]; sl[n + t] = tb->lp[t];
    slh[t] = tb->lhm[t]; slh[n + t] = tb->lhp[t];
  }
}

// BR1 lifting of element e by the NT threads t of one slot.  valid = false keeps the slot's
// threads in step with the workgroup barriers without touching memory.
// OUT: LIFT_G writes the gradients G[e][d*4+c][node] = dW_c/dx_d (weak and strong forms);
// LIFT_FV writes instead the contravariant viscous fluxes Fv[e][dir*4+c][node] =
// (F^v . Ja^dir)_{1+c} (momentum, energy), which the reverse sweep consumes; LIFT_DIV writes what
// the split-form operator reads, the strong-form divergence Geo::Gd (sums along the lines of D
// times Fv^dir, and the interior part of the surface term) and the face traces Geo::Gf of Fv;
// LIFT_DIVK writes both (the stage kept for a reverse sweep).  LIFT_GT (LG nodes) writes the
// gradients and every side's traces of them, interpolated with l(+-1) (Geo::Gtr), which the
// operator kernel reads at its faces instead of interpolating along the lines of its own and the
// neighbour's element.  On LG nodes the neighbours' traces of W come from k_prolong (Geo::Wtr).
// LIFT_WV (weak form, conforming meshes) writes what the weak-form operator reads: the volume
// term Geo::Gd (sums along the lines of D-hat times Fv^dir) and every side's viscous flux at its
// trace, F^v(U, grad W) . n with the side's own outward normal (Geo::Gf; on a boundary side
// already the BR1 mean with the outer state), and the gradients too when G is not NULL.
// LIFT_SV (strong form on LG nodes, conforming meshes) writes the face fluxes as LIFT_WV and as
// Geo::Gd the strong-form viscous term: sums along the lines of D times Fv^dir minus, for both
// faces of each line, lhat(+-1) times +- the interior viscous flux interpolated to the face (both
// in one contraction with Tab::Ds).
enum { LIFT_G = 0, LIFT_FV = 1, LIFT_DIV = 2, LIFT_DIVK = 3, LIFT_GT = 4, LIFT_WV = 5, LIFT_SV = 6 };

// The node's gradients acc[d*4+c] = dW_c/dx_d become its contravariant viscous fluxes
// acc[dir*4+c] = (F^v . Ja^dir)_{1+c} (momentum, energy): Newtonian stress with Stokes'
// hypothesis and Fourier heat flux, contracted with the metric terms jo[dir*3+d].  Every rounding
// step is spelled out (explicit fma, no contraction), so every kernel that runs the lifting
// produces the same fluxes bit for bit.
__device__ __forceinline__ void contra_visc(double *acc, const double *jo, double u, double v, double w,
                                            const Phys &ph) {
#pragma clang fp contract(off)
  const double mu = ph.mu, div = (acc[0] + acc[5]) + acc[10];
  const double t00 = mu * fma(-2.0 / 3.0, div, 2.0 * acc[0]);
  const double t11 = mu * fma(-2.0 / 3.0, div, 2.0 * acc[5]);
  const double t22 = mu * fma(-2.0 / 3.0, div, 2.0 * acc[10]);
  const double t01 = mu * (acc[4] + acc[1]);
  const double t02 = mu * (acc[8] + acc[2]);
  const double t12 = mu * (acc[9] + acc[6]);
  const double dT0 = acc[3], dT1 = acc[7], dT2 = acc[11];
#pragma unroll
  for (int dir = 0; dir < 3; ++dir) {
    const double *nv = jo + 3 * dir;
    acc[dir * 4] = fma(t02, nv[2], fma(t01, nv[1], t00 * nv[0]));
    acc[dir * 4 + 1] = fma(t12, nv[2], fma(t11, nv[1], t01 * nv[0]));
    acc[dir * 4 + 2] = fma(t22, nv[2], fma(t12, nv[1], t02 * nv[0]));
    const double q = fma(dT2, nv[2], fma(dT1, nv[1], dT0 * nv[0]));
    acc[dir * 4 + 3] = fma(ph.kappa, q, fma(acc[dir * 4 + 2], w, fma(acc[dir * 4 + 1], v, acc[dir * 4] * u)));
  }
}

// LDS slot of node (i, j, k) in one component array of the viscous divergence stage.  For n = 8
// the index bits are swizzled so that the 64 lanes that read the m-th node of 64 different lines
// hit distinct banks in each direction (and in node order): i is XORed with two bits of j and k,
// j with the low bits of k.
template <int n> __device__ __forceinline__ int div_slot(int i, int j, int k) {
  if constexpr (n == 8) return (i ^ ((j >> 2) | ((k & 3) << 1))) + 8 * (j ^ (k & 3)) + 64 * k;
  else return i + n * (j + n * k);
}

// sm: the slot's LiftLds<N> regions, contiguous (W, JA, WS).
template <int N, bool LGL, int OUT, int GEN>
__device__ __forceinline__ void lift_body(const Geo &g, const Phys &ph, int e, bool valid, int t,
                                          const double *__restrict__ U, double *__restrict__ G,
                                          double *__restrict__ Fv, double *sm, const double *sDh,
                                          const double *sl, const double *slh) {
  using S = Sz<N>;
  using L = LiftLds<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, NT = S::NT;
  constexpr bool FVO = OUT == LIFT_FV || OUT == LIFT_DIV || OUT == LIFT_DIVK;  // viscous fluxes formed
  double *sW = sm, *sJa = sm + L::W, *sWs = sm + L::W + L::JA;
  const double gm1 = ph.gamma - 1.0;
  const double *Ue = U + (size_t)e * 5 * n3;
  // the metric terms of the next direction (at most 3 per thread) and, in the last direction, the
  // node's 1/J are loaded one phase ahead
  constexpr int JPT = (3 * n3 + NT - 1) / NT;
  double jn[JPT], sjn = 0.0;
  {
    const double *Jd = g.Ja + (size_t)e * 9 * n3;
#pragma unroll
    for (int r = 0; r < JPT; ++r) jn[r] = (valid && t + r * NT < 3 * n3) ? Jd[t + r * NT] : 0.0;
  }
  // on LGL nodes with one face point per thread, the neighbour's trace is loaded before the
  // first barrier
  constexpr bool PF = LGL && 6 * n2 <= NT;
  double Unp[5];
  if (PF && valid && t < 6 * n2) {
    const int s = t / n2, ab = t - s * n2, a = ab % n, b = ab / n;
    const int nb = g.nbr[(size_t)e * 6 + s];
    const NbFace f = nbr_face<n, (GEN > 0)>(g, e, s, a, b);
    const int qn = GEN ? line_node<n>(f.dn, f.a, f.b, f.plus ? N : 0) : line_node<n>(s >> 1, a, b, (s & 1) ? 0 : N);
    if (!(GEN && f.bnd)) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Unp[v] = U[((size_t)nb * 5 + v) * n3 + qn];
    }
  }
  if (valid && t < n3) {
    double Uq[5], W[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = Ue[v * n3 + t];
    grad_prim_to_W(Uq, gm1, ph.R, W);
#pragma unroll
    for (int v = 0; v < 4; ++v) sW[v * n3 + t] = W[v];
  }
  __syncthreads();
  // W* = mean of the two traces on every face point of the element
  for (int p = valid ? t : 6 * n2; p < 6 * n2; p += NT) {
    const int s = p / n2, ab = p - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
    const bool plus = s & 1;
    const int nb = g.nbr[(size_t)e * 6 + s];
    const NbFace f = nbr_face<n, (GEN > 0)>(g, e, s, a, b);
    const double *Un = U + (size_t)(GEN && f.bnd ? e : nb) * 5 * n3;
    double WL[4], WR[4];
    if (LGL) {
      const int q = line_node<n>(dn, a, b, plus ? N : 0);
      const int qn = GEN ? line_node<n>(f.dn, f.a, f.b, f.plus ? N : 0) : line_node<n>(dn, a, b, plus ? 0 : N);
#pragma unroll
      for (int v = 0; v < 4; ++v) WL[v] = sW[v * n3 + q];
      if (!(GEN && f.bnd)) {
        double Uq[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) Uq[v] = PF ? Unp[v] : Un[v * n3 + qn];
        grad_prim_to_W(Uq, gm1, ph.R, WR);
      }
    } else {
      const double *lo = sl + (plus ? n : 0), *ln = GEN ? sl + (f.plus ? n : 0) : sl + (plus ? 0 : n);
#pragma unroll
      for (int v = 0; v < 4; ++v) { WL[v] = 0.0; WR[v] = 0.0; }
#pragma unroll 1
      for (int m = 0; m < n; ++m) {
        const int q = line_node<n>(dn, a, b, m);
#pragma unroll
        for (int v = 0; v < 4; ++v) WL[v] += lo[m] * sW[v * n3 + q];
      }
      if (!(GEN && f.bnd)) {
        // the neighbour's trace of W on its side of the face, from the prolongation kernel
        const double *wt = g.Wtr + ((size_t)nb * 6 + 2 * f.dn + (f.plus ? 1 : 0)) * 4 * n2 + f.a + n * f.b;
#pragma unroll
        for (int v = 0; v < 4; ++v) WR[v] = wt[v * n2];
      }
    }
    if (GEN && f.bnd && f.kind == DG_BC_STATE) {
      // given outer state
      grad_prim_to_W(ph.ub, gm1, ph.R, WR);
    } else if (GEN && f.bnd && f.kind == DG_BC_WALL) {
      // no-slip wall: velocity reversed, temperature kept
#pragma unroll
      for (int v = 0; v < 3; ++v) WR[v] = -WL[v];
      WR[3] = WL[3];
    } else if (GEN && f.bnd && f.kind == DG_BC_WALL_ISOTHERMAL) {
      // isothermal wall: velocity reversed, mean temperature T_w
#pragma unroll
      for (int v = 0; v < 3; ++v) WR[v] = -WL[v];
      WR[3] = 2.0 * ph.tw - WL[3];
    } else if (GEN && f.bnd && f.kind == DG_BC_OUTFLOW) {
      // pressure outflow: the own trace's density and velocity with p_out (the conservative
      // trace: the face node on LGL nodes, interpolated with l(+-1) on LG nodes)
      double Uq[5];
      if (LGL) {
        const int q = line_node<n>(dn, a, b, plus ? N : 0);
#pragma unroll
        for (int v = 0; v < 5; ++v) Uq[v] = Ue[v * n3 + q];
      } else {
        const double *lo = sl + (plus ? n : 0);
#pragma unroll
        for (int v = 0; v < 5; ++v) Uq[v] = 0.0;
        for (int m = 0; m < n; ++m) {
          const int q = line_node<n>(dn, a, b, m);
#pragma unroll
          for (int v = 0; v < 5; ++v) Uq[v] += lo[m] * Ue[v * n3 + q];
        }
      }
      Uq[4] = ph.pout / gm1 + 0.5 * (Uq[1] * Uq[1] + Uq[2] * Uq[2] + Uq[3] * Uq[3]) / Uq[0];
      grad_prim_to_W(Uq, gm1, ph.R, WR);
    } else if (GEN == 2 && f.bnd && f.kind == FACE_MORTAR) {
      // non-conforming face: the surface term comes from the mortar face array
#pragma unroll
      for (int v = 0; v < 4; ++v) WR[v] = WL[v];
    } else if (GEN && f.bnd) {
      // symmetry plane: the outer W is the inner one with the velocity reflected
      const double *fnp = g.fn + ((size_t)e * 6 + s) * 3 * n2 + ab;
      const double nt[3] = {fnp[0], fnp[n2], fnp[2 * n2]};
      double nh[3];
      unit3(nt, nh);
#pragma unroll
      for (int v = 0; v < 4; ++v) WR[v] = WL[v];
      mirror3(WR, nh);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sWs[(s * 4 + v) * n2 + ab] = 0.5 * (WL[v] + WR[v]);
  }
  double acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = 0.0;
  const int i = t % n, j = (t / n) % n, k = t / n2;
  double jo[9];  // this node's metric terms, kept for the viscous fluxes
  double gd[4] = {0.0, 0.0, 0.0, 0.0};  // the viscous divergence (LIFT_DIV, LIFT_DIVK)
#pragma unroll
  for (int dir = 0; dir < 3; ++dir) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < JPT; ++r)
      if (valid && t + r * NT < 3 * n3) sJa[t + r * NT] = jn[r];
    if (dir < 2) {
      const double *Jd = g.Ja + ((size_t)e * 9 + (dir + 1) * 3) * n3;
#pragma unroll
      for (int r = 0; r < JPT; ++r) jn[r] = (valid && t + r * NT < 3 * n3) ? Jd[t + r * NT] : 0.0;
    }
    if (dir == 2 && valid && t < n3) sjn = g.sJ[(size_t)e * n3 + t];  // for the epilogue
    __syncthreads();
    if ((FVO || OUT == LIFT_WV || OUT == LIFT_SV) && valid && t < n3) {
#pragma unroll
      for (int d = 0; d < 3; ++d) jo[dir * 3 + d] = sJa[d * n3 + t];
    }
    if (valid && t < n3) {
      const int id = dir == 0 ? i : (dir == 1 ? j : k);
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int base = t - id * str;
      // not unrolled: with all of a line's loads in flight the kernel exceeds its register budget
#pragma unroll 1
      for (int m = 0; m < n; ++m) {
        const int qm = base + m * str;
        const double Dh = sDh[id * n + m];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double c1 = Dh * sJa[d * n3 + qm];
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[d * 4 + v] += c1 * sW[v * n3 + qm];
        }
      }
      if (LGL && (id == 0 || id == N)) {
        // surface on the face of this direction through the node: on LGL nodes the outward
        // normal times s-hat is +-Ja^dir at the node itself
        const bool plus = id == N;
        const int s = 2 * dir + (plus ? 1 : 0);
        const double lh = slh[(plus ? n : 0) + id];
        const int a = dir == 0 ? j : i, b = dir == 2 ? j : k;
        const int ab = a + n * b;
        const double sl_ = plus ? lh : -lh;
        if (GEN == 2 && is_mortar(g, e, s)) {
          // non-conforming face: W* s n_d (outward) from the mortar face array
          const double *ml = g.mlift + (size_t)g.mslot[(size_t)e * 6 + s] * 12 * n2 + ab;
#pragma unroll
          for (int c = 0; c < 12; ++c) acc[c] += lh * ml[c * n2];
        } else {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const double c1 = sl_ * sJa[d * n3 + t];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[d * 4 + v] += c1 * sWs[(s * 4 + v) * n2 + ab];
          }
        }
      }
    }
  }
  if (!LGL && valid && t < n3) {
    // surface: lhat(+-1) [W* nt_d] on each side
    for (int s = 0; s < 6; ++s) {
      const int dn = s >> 1;
      const bool plus = s & 1;
      const int id = dn == 0 ? i : (dn == 1 ? j : k);
      const double lh = slh[(plus ? n : 0) + id];
      if (LGL && lh == 0.0) continue;
      const int a = dn == 0 ? j : i, b = dn == 2 ? j : k;
      const int ab = a + n * b;
      if (GEN == 2 && is_mortar(g, e, s)) {
        const double *ml = g.mlift + (size_t)g.mslot[(size_t)e * 6 + s] * 12 * n2 + ab;
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] += lh * ml[c * n2];
        continue;
      }
      const double *nt = g.fn + ((size_t)e * 6 + s) * 3 * n2 + ab;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double c1 = lh * nt[d * n2];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[d * 4 + v] += c1 * sWs[(s * 4 + v) * n2 + ab];
      }
    }
  }
  if (valid && t < n3) {
    const double sj = sjn;
    {
      // the gradients are rounded once, whatever is computed from them (so the three output
      // variants give the same bits)
#pragma clang fp contract(off)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] *= sj;
    }
    if (GEN == 2 && LGL) {
      // face nodes of non-conforming sides keep their gradients for the mortar flux kernel
#pragma unroll
      for (int dir = 0; dir < 3; ++dir) {
        const int id = dir == 0 ? i : (dir == 1 ? j : k);
        if (id != 0 && id != N) continue;
        const int s = 2 * dir + (id == N ? 1 : 0);
        const int slot = g.mslot[(size_t)e * 6 + s];
        if (slot < 0) continue;
        const int ab = (dir == 0 ? j : i) + n * (dir == 2 ? j : k);
        double *mg = g.mg + (size_t)slot * 12 * n2 + ab;
#pragma unroll
        for (int c = 0; c < 12; ++c) mg[c * n2] = acc[c];
      }
    }
    if (OUT == LIFT_G || OUT == LIFT_GT || ((OUT == LIFT_WV || OUT == LIFT_SV || OUT == LIFT_DIV) && G)) {
      double *Ge = G + (size_t)e * 12 * n3;
#pragma unroll
      for (int c = 0; c < 12; ++c) Ge[c * n3 + t] = acc[c];
    }
    if (FVO) {
      contra_visc(acc, jo, sW[t], sW[n3 + t], sW[2 * n3 + t], ph);
      if (OUT == LIFT_FV || OUT == LIFT_DIVK) {
        double *Fe = Fv + (size_t)e * 12 * n3;
#pragma unroll
        for (int c = 0; c < 12; ++c) Fe[c * n3 + t] = acc[c];
      }
      if (OUT == LIFT_DIV || OUT == LIFT_DIVK) {
        // the traces Fv^dir on the element's faces through this node, and their interior part
        // -+lhat(+-1) Fv^dir of the surface term
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
          const int id = dir == 0 ? i : (dir == 1 ? j : k);
          if (id != 0 && id != N) continue;
          const bool plus = id == N;
          const int s = 2 * dir + (plus ? 1 : 0);
          const int ab = (dir == 0 ? j : i) + n * (dir == 2 ? j : k);
          double *gf = g.Gf + ((size_t)e * 6 + s) * 4 * n2 + ab;
          const double lh = slh[(plus ? n : 0) + id];
          const double sl_ = plus ? -lh : lh;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            gf[c * n2] = acc[dir * 4 + c];
            gd[c] = fma(sl_, acc[dir * 4 + c], gd[c]);
          }
        }
      }
    }
  }
  if constexpr (OUT == LIFT_WV || OUT == LIFT_SV) {
    // weak form (and strong form on LG nodes): every side's viscous flux at its trace (LG:
    // gradients interpolated from LDS, U from the prolongation; LGL: the face node's), with the
    // side's own outward normal; on a boundary side the BR1 mean with the outer state as the
    // operator would form it (this side is the master).  The node's contravariant fluxes for the
    // volume term below are formed first.
    double u = 0.0, v = 0.0, w = 0.0;
    if (valid && t < n3) { u = sW[t]; v = sW[n3 + t]; w = sW[2 * n3 + t]; }
    __syncthreads();
    if (valid && t < n3) {
      const int q = div_slot<n>(i, j, k);
#pragma unroll
      for (int c = 0; c < 12; ++c) sm[c * n3 + q] = acc[c];
      // the node's contravariant fluxes now: 12 values held across the face loop instead of the
      // gradients and the metric terms
      contra_visc(acc, jo, u, v, w, ph);
    }
    __syncthreads();
    for (int p = valid ? t : 6 * n2; p < 6 * n2; p += NT) {
      const int s = p / n2, ab = p - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
      const bool plus = s & 1;
      double gq[12], Uq[5];
      if (LGL) {
        const int m = plus ? N : 0;
        const int q = dn == 0 ? div_slot<n>(m, a, b) : (dn == 1 ? div_slot<n>(a, m, b) : div_slot<n>(a, b, m));
#pragma unroll
        for (int c = 0; c < 12; ++c) gq[c] = sm[c * n3 + q];
        const int qn = line_node<n>(dn, a, b, m);
#pragma unroll
        for (int c = 0; c < 5; ++c) Uq[c] = Ue[c * n3 + qn];
      } else {
        const double *lo = sl + (plus ? n : 0);
#pragma unroll
        for (int c = 0; c < 12; ++c) gq[c] = 0.0;
#pragma unroll 1
        for (int m = 0; m < n; ++m) {
          const int q = dn == 0 ? div_slot<n>(m, a, b) : (dn == 1 ? div_slot<n>(a, m, b) : div_slot<n>(a, b, m));
#pragma unroll
          for (int c = 0; c < 12; ++c) gq[c] += lo[m] * sm[c * n3 + q];
        }
        const double *ut = g.Utr + ((size_t)e * 6 + s) * 5 * n2 + ab;
#pragma unroll
        for (int c = 0; c < 5; ++c) Uq[c] = ut[c * n2];
      }
      const double *fnp = g.fn + ((size_t)e * 6 + s) * 3 * n2 + ab;
      const double nt[3] = {fnp[0], fnp[n2], fnp[2 * n2]};
      double Fo[5];
      flux_v(to_prim(Uq, gm1), gq, ph, nt, Fo);
      const NbFace f = nbr_face<n, (GEN > 0)>(g, e, s, a, b);
      if (GEN && f.bnd && f.kind != DG_BC_STATE && f.kind != DG_BC_OUTFLOW) {
        // walls and symmetry planes: the outer state and gradients; a given outer state or
        // outflow takes the outer viscous flux equal to the inner one (the mean is Fo itself)
        const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
        const double ish = 1.0 / sh;
        const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
        double Ux[5], gx[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) gx[c] = gq[c];
        if (f.kind == DG_BC_WALL_ISOTHERMAL || f.kind == DG_BC_WALL) {
          // no-slip wall: velocity reversed; at an adiabatic wall the temperature gradient mirrored
          Ux[0] = Uq[0]; Ux[1] = -Uq[1]; Ux[2] = -Uq[2]; Ux[3] = -Uq[3]; Ux[4] = Uq[4];
          if (f.kind == DG_BC_WALL) {
            double tg[3] = {gq[3], gq[7], gq[11]};
            mirror3(tg, nh);
            gx[3] = tg[0]; gx[7] = tg[1]; gx[11] = tg[2];
          }
        } else {
          // symmetry plane: mirror image of the inner state and gradients
#pragma unroll
          for (int c = 0; c < 5; ++c) Ux[c] = Uq[c];
          mirror3(Ux + 1, nh);
          mirror_grad(gx, nh);
        }
        double Fx[5];
        flux_v(to_prim(Ux, gm1), gx, ph, nt, Fx);
#pragma unroll
        for (int c = 1; c < 5; ++c) Fo[c] = 0.5 * (Fo[c] + Fx[c]);
      } else if (GEN && f.bnd) {
#pragma unroll
        for (int c = 1; c < 5; ++c) Fo[c] = 0.5 * (Fo[c] + Fo[c]);
      }
      double *pv = g.Gf + ((size_t)e * 6 + s) * 4 * n2 + ab;
#pragma unroll
      for (int c = 0; c < 4; ++c) pv[c * n2] = Fo[1 + c];
    }
  }
  if constexpr (OUT == LIFT_DIV || OUT == LIFT_DIVK || OUT == LIFT_WV || OUT == LIFT_SV) {
    // strong-form divergence of the viscous fluxes for the split-form operator:
    // Gd_c = sum_dir (sum_m D_{id,m} Fv^dir_c(m on the line) + [face node] -+lhat(+-1) Fv^dir_c),
    // the interior part of the surface term taken with the volume term; for the weak form
    // (LIFT_WV) Gd_c = sum_dir sum_m Dhat_{id,m} Fv^dir_c(m on the line), for the strong form on LG
    // nodes (LIFT_SV) the same with Tab::Ds.  The three regions are
    // free once every thread is past its last read of them.
    __syncthreads();
    if (valid && t < n3) {
      const int q = div_slot<n>(i, j, k);
#pragma unroll
      for (int c = 0; c < 12; ++c) sm[c * n3 + q] = acc[c];
    }
    __syncthreads();
    // one line, one direction and two components per task: the line's values are read once and
    // its n results written back in place (each LDS value is read once, not n times); the
    // matrix comes from the table through the scalar cache, the same for every lane
    // (LIFT_SV: Tab::Ds, the strong-form derivative with the interior fluxes interpolated to the
    // line's two faces and lifted back, -lhat(+1) l(+1) + lhat(-1) l(-1))
    const __attribute__((address_space(4))) double *Dg = (const __attribute__((address_space(4))) double *)(
        OUT == LIFT_WV ? g.tab->Dh : (OUT == LIFT_SV ? g.tab->Ds : g.tab->D));
    // TPD task slots per direction: 2 n^2 rounded up to whole waves where the three directions
    // then still fit the workgroup in one pass (n = 7: 98 -> 128, 384 lanes), so that every wave
    // works on one direction
    constexpr int TPW = (2 * n2 + 63) / 64 * 64;
    constexpr int TPD = (2 * n2) % 64 != 0 && 3 * TPW <= NT ? TPW : 2 * n2;
    for (int task = valid ? t : 3 * TPD; task < 3 * TPD; task += NT) {
      const int dir = TPD % 64 == 0 ? __builtin_amdgcn_readfirstlane(task / TPD) : task / TPD;
      const int r = task - dir * TPD, cp = r / n2, ln = r - cp * n2;
      if (TPD != 2 * n2 && r >= 2 * n2) continue;  // a padding slot
      const int a = ln % n, b = ln / n;
      double *s0 = sm + (dir * 4 + 2 * cp) * n3, *s1 = s0 + n3;
      double f0[n], f1[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const int q = dir == 0 ? div_slot<n>(m, a, b) : (dir == 1 ? div_slot<n>(a, m, b) : div_slot<n>(a, b, m));
        f0[m] = s0[q];
        f1[m] = s1[q];
      }
#pragma unroll 2
      for (int id = 0; id < n; ++id) {
        double o0 = 0.0, o1 = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) {
          const double D = Dg[id * n + m];
          o0 = fma(D, f0[m], o0);
          o1 = fma(D, f1[m], o1);
        }
        const int q = dir == 0 ? div_slot<n>(id, a, b) : (dir == 1 ? div_slot<n>(a, id, b) : div_slot<n>(a, b, id));
        s0[q] = o0;
        s1[q] = o1;
      }
    }
    __syncthreads();
    if (valid && t < n3) {
      const int q = div_slot<n>(i, j, k);
#pragma unroll
      for (int dir = 0; dir < 3; ++dir) {
#pragma unroll
        for (int c = 0; c < 4; ++c) gd[c] += sm[(dir * 4 + c) * n3 + q];
      }
      double *Gde = g.Gd + (size_t)e * 4 * n3 + t;
#pragma unroll
      for (int c = 0; c < 4; ++c) Gde[c * n3] = gd[c];
    }
  }
  if constexpr (OUT == LIFT_GT) {
    // LG face traces, each face point by one thread: the gradients (staged once the three
    // regions are free), then the conservative state, each summed along the face-normal line
    // with l(+-1) in the order the operator kernel would
    __syncthreads();
    if (valid && t < n3) {
      const int q = div_slot<n>(i, j, k);
#pragma unroll
      for (int c = 0; c < 12; ++c) sm[c * n3 + q] = acc[c];
    }
    __syncthreads();
    for (int p = valid ? t : 6 * n2; p < 6 * n2; p += NT) {
      const int s = p / n2, ab = p - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
      const double *lo = sl + ((s & 1) ? n : 0);
      double gq[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) gq[c] = 0.0;
#pragma unroll 1
      for (int m = 0; m < n; ++m) {
        const int q = dn == 0 ? div_slot<n>(m, a, b) : (dn == 1 ? div_slot<n>(a, m, b) : div_slot<n>(a, b, m));
#pragma unroll
        for (int c = 0; c < 12; ++c) gq[c] += lo[m] * sm[c * n3 + q];
      }
      double *gt = g.Gtr + ((size_t)e * 6 + s) * 12 * n2 + ab;
#pragma unroll
      for (int c = 0; c < 12; ++c) gt[c * n2] = gq[c];
    }
  }
}

// Prolongation on LG nodes (Navier-Stokes): every side's traces of the conservative state and of
// W = (u, v, w, T), each interpolated with l(+-1) along the face-normal lines of the element
// (Utr, Wtr of Geo), so that the lifting and operator kernels read their neighbours' traces
// contiguously instead of the neighbours' whole lines.
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_prolong(Geo g, Phys ph, const double *__restrict__ U) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n, NT = Sz<N>::NT;
  __shared__ double sm[9 * n3];
  __shared__ double sl[2 * n];
  const int t = threadIdx.x;
  if (t < n) { sl[t] = g.tab->lm[t]; sl[n + t] = g.tab->lp[t]; }
  const int e = xcd_element(blockIdx.x, g.K);
  if (e >= g.K) return;
  if (t < n3) {
    const double *Ue = U + (size_t)e * 5 * n3;
    const int q = div_slot<n>(t % n, (t / n) % n, t / n2);
    double Uq[5], W[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Uq[v] = Ue[v * n3 + t];
      sm[v * n3 + q] = Uq[v];
    }
    grad_prim_to_W(Uq, ph.gamma - 1.0, ph.R, W);
#pragma unroll
    for (int v = 0; v < 4; ++v) sm[(5 + v) * n3 + q] = W[v];
  }
  __syncthreads();
  for (int p = t; p < 6 * n2; p += NT) {
    const int s = p / n2, ab = p - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
    const double *lo = sl + ((s & 1) ? n : 0);
    double x[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) x[v] = 0.0;
#pragma unroll 1
    for (int m = 0; m < n; ++m) {
      const int q = dn == 0 ? div_slot<n>(m, a, b) : (dn == 1 ? div_slot<n>(a, m, b) : div_slot<n>(a, b, m));
#pragma unroll
      for (int v = 0; v < 9; ++v) x[v] += lo[m] * sm[v * n3 + q];
    }
    double *ut = g.Utr + ((size_t)e * 6 + s) * 5 * n2 + ab;
    double *wt = g.Wtr + ((size_t)e * 6 + s) * 4 * n2 + ab;
#pragma unroll
    for (int v = 0; v < 5; ++v) ut[v * n2] = x[v];
#pragma unroll
    for (int v = 0; v < 4; ++v) wt[v * n2] = x[5 + v];
  }
}

// waves per SIMD each lifting instantiation is built for (caps its registers)
template <bool LGL, int OUT, int GEN> constexpr int lift_minb() {
  if ((OUT == LIFT_WV || OUT == LIFT_SV) && GEN > 0) return 4;  // boundary code: 128 registers
  if (GEN == 2 && LGL) return DG_LIFT_MORTAR_MINB;
  return (LGL || GEN == 0) ? DG_LIFT_MINB : 2;
}

template <int N, bool LGL, int OUT, int GEN>
__global__ void __launch_bounds__(Sz<N>::NT, (lift_minb<LGL, OUT, GEN>()))
    k_lift(Geo g, Phys ph, const double *__restrict__ U, double *__restrict__ G, double *__restrict__ Fv) {
  using L = LiftLds<N>;
  constexpr int n = L::n;
  __shared__ double sm[L::W + L::JA + L::WS];
  __shared__ double sDh[n * n], sl[2 * n], slh[2 * n];
  lift_tables<N>(g.tab, threadIdx.x, Sz<N>::NT, sDh, sl, slh);
  const int e = xcd_element(blockIdx.x, g.K);
  if (e >= g.K) return;
  lift_body<N, LGL, OUT, GEN>(g, ph, e, true, threadIdx.x, U, G, Fv, sm, sDh, sl, slh);
}

// ----------------------------------------------------------------------------- operator
// waves per SIMD the Navier-Stokes weak- and strong-form operators are built for: 4 (128
// registers, two workgroups per CU at N = 7; no spill on LGL nodes, 84 bytes on LG nodes) against
// the 131-148 registers they take unbounded (one workgroup per CU): at 48^3, N = 7, weak form on
// LG nodes 6.14 -> 5.17 ms.  Degrees below 5 (one or two waves per element) keep their registers,
// and so do the Euler forms (at N = 3 on 96^3 a 128-register budget spills 108 bytes: 5.20 ->
// 6.15 ms).
#ifndef DG_WMAIN_MINB
#define DG_WMAIN_MINB 4
#endif
template <int N, bool LGL, bool NS, int FORM, int GEN> constexpr int main_minb() {
  return (NS && GEN < 2 && N >= 5 && FORM != 1) ? DG_WMAIN_MINB : 1;
}

// FORM: 0 weak, 1 split, 2 strong.  MODE: 0 write U_t, 1 fused RK stage.  GEN: face codes.
// FVM: hybrid DG/FV mesh (Euler): finite-volume elements are left to k_fv_volume, and the sides
// that meet one take their flux from Geo::fvFx.
template <int N, bool LGL, bool NS, int FORM, int MODE, int GEN, bool FVM = false>
__global__ void __launch_bounds__(Sz<N>::NT, (main_minb<N, LGL, NS, FORM, GEN>()))
    k_main(Geo g, Phys ph, const double *__restrict__ U, const double *__restrict__ G, double *__restrict__ out,
           double *__restrict__ R, double ca, double cb, double dt) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, NT = S::NT;
  constexpr int NX = (FORM == 1) ? 8 : 5;
  // WVM: weak form, Navier-Stokes, conforming faces: the lifting kernel has formed the viscous
  // volume term (Geo::Gd) and every side's viscous flux at its trace (Geo::Gf); no gradients
  constexpr bool WVM = NS && FORM == 0 && GEN < 2;
  // SVM: strong form on LGL nodes, Navier-Stokes, conforming faces: as for the split form, the
  // lifting kernel has formed the strong-form viscous divergence (Geo::Gd) and the face traces of
  // the contravariant viscous fluxes (Geo::Gf)
  constexpr bool SVM = NS && FORM == 2 && LGL && GEN < 2;
  // SVL: strong form on LG nodes, Navier-Stokes, conforming faces: the lifting kernel has formed
  // the strong-form viscous volume and interior surface terms (Geo::Gd) and, as for the weak form,
  // every side's viscous flux at its trace (Geo::Gf)
  constexpr bool SVL = NS && FORM == 2 && !LGL && GEN < 2;
  constexpr bool PFM = WVM || SVL;  // face viscous fluxes with each side's own normal
  constexpr bool VH = WVM || SVM || SVL;  // no gradients read
  __shared__ double sU[5 * n3];
  __shared__ double sX[NX * n3];
  __shared__ double sF[6 * 5 * n2];
  __shared__ double sD[n * n], sl[2 * n], slh[2 * n];
  const int e = blockIdx.x;
  const int t = threadIdx.x;
  if (FVM && g.fvflag[e]) return;  // a finite-volume element
  const double gm1 = ph.gamma - 1.0;
  const Tab *tb = g.tab;
  // strong form on LG nodes: the derivative matrix carries the interior flux's interpolation
  // to the line's two faces (Tab::Ds), so the surface terms add the numerical flux alone
  for (int c = t; c < n * n; c += NT) sD[c] = (FORM == 0) ? tb->Dh[c] : ((FORM == 2 && !LGL) ? tb->Ds[c] : tb->D[c]);
  if (t < n) {
    sl[t] = tb->lm[t]; sl[n + t] = tb->lp[t];
    slh[t] = tb->lhm[t]; slh[n + t] = tb->lhp[t];
  }
  const double *Ue = U + (size_t)e * 5 * n3;
  const double *Ge = G + (size_t)e * 12 * n3;
  double Uo[5];
  if (t < n3) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Uo[v] = Ue[v * n3 + t];
      sU[v * n3 + t] = Uo[v];
    }
  }
  __syncthreads();
  // numerical surface flux on the six faces, stored outward for this element
  for (int p = t; p < 6 * n2; p += NT) {
    const int s = p / n2, ab = p - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
    const bool plus = s & 1;
    const int nb = g.nbr[(size_t)e * 6 + s];
    const NbFace f = nbr_face<n, (GEN > 0)>(g, e, s, a, b);
    const bool bnd = GEN && f.bnd;
    if (GEN == 2 && bnd && f.kind == FACE_MORTAR) {
      // non-conforming face: the outward flux from the mortar face array
      const double *mf = g.mflux + (size_t)g.mslot[(size_t)e * 6 + s] * 5 * n2 + ab;
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[(s * 5 + v) * n2 + ab] = mf[v * n2];
      continue;
    }
    if (FVM && g.fvflag[nb]) {
      // face shared with a finite-volume element: the outward flux at the face nodes
      const double *fx = g.fvFx + ((size_t)e * 6 + s) * 5 * n2 + ab;
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[(s * 5 + v) * n2 + ab] = fx[v * n2];
      continue;
    }
    const double *Un = U + (size_t)(bnd ? e : nb) * 5 * n3;
    const double *Gn = G + (size_t)(bnd ? e : nb) * 12 * n3;
    double Uw[5], Ux[5], gw[12], gx[12];  // w: this element's trace, x: neighbour's trace
    if (LGL) {
      const int q = line_node<n>(dn, a, b, plus ? N : 0);
      const int qn = GEN ? line_node<n>(f.dn, f.a, f.b, f.plus ? N : 0) : line_node<n>(dn, a, b, plus ? 0 : N);
#pragma unroll
      for (int v = 0; v < 5; ++v) { Uw[v] = sU[v * n3 + q]; Ux[v] = bnd ? 0.0 : Un[v * n3 + qn]; }
      if (NS && !VH) {
#pragma unroll
        for (int c = 0; c < 12; ++c) { gw[c] = Ge[c * n3 + q]; gx[c] = bnd ? 0.0 : Gn[c * n3 + qn]; }
      }
    } else {
      const double *lo = sl + (plus ? n : 0), *ln = GEN ? sl + (f.plus ? n : 0) : sl + (plus ? 0 : n);
#pragma unroll
      for (int v = 0; v < 5; ++v) { Uw[v] = 0.0; Ux[v] = 0.0; }
      if (NS) {
#pragma unroll
        for (int c = 0; c < 12; ++c) { gw[c] = 0.0; gx[c] = 0.0; }
      }
      if (NS) {
        // Navier-Stokes: the lifting kernel has interpolated every side's traces of U and of the
        // gradients; this side's U trace from LDS, the rest read contiguously
        const double *gt = g.Gtr + ((size_t)e * 6 + s) * 12 * n2 + ab;
        const size_t sn = (size_t)(bnd ? e : nb) * 6 + 2 * f.dn + (f.plus ? 1 : 0);
        const double *utn = g.Utr + sn * 5 * n2 + f.a + n * f.b;
        const double *gtn = g.Gtr + sn * 12 * n2 + f.a + n * f.b;
#pragma unroll 1
        for (int m = 0; m < n; ++m) {
          const int q = line_node<n>(dn, a, b, m);
#pragma unroll
          for (int v = 0; v < 5; ++v) Uw[v] += lo[m] * sU[v * n3 + q];
        }
        if (!VH) {
#pragma unroll
          for (int c = 0; c < 12; ++c) gw[c] = gt[c * n2];
        }
        if (!bnd) {
#pragma unroll
          for (int v = 0; v < 5; ++v) Ux[v] = utn[v * n2];
          if (!VH) {
#pragma unroll
            for (int c = 0; c < 12; ++c) gx[c] = gtn[c * n2];
          }
        }
      } else {
        // a rolled loop: unrolled, the early loads of all n nodes' values spill
#pragma unroll 1
        for (int m = 0; m < n; ++m) {
          const int q = line_node<n>(dn, a, b, m), qn = GEN ? line_node<n>(f.dn, f.a, f.b, m) : q;
#pragma unroll
          for (int v = 0; v < 5; ++v) Uw[v] += lo[m] * sU[v * n3 + q];
          if (!bnd) {
#pragma unroll
            for (int v = 0; v < 5; ++v) Ux[v] += ln[m] * Un[v * n3 + qn];
          }
        }
      }
    }
    // the master's normal and state go first (fn holds the outward normal, the master's
    // negated on the slave side)
    const double *fnp = g.fn + ((size_t)e * 6 + s) * 3 * n2 + ab;
    const bool mst = GEN ? f.master : plus;
    const double sg = mst ? 1.0 : -1.0;
    const double nt[3] = {sg * fnp[0], sg * fnp[n2], sg * fnp[2 * n2]};
    const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    const double ish = 1.0 / sh;
    const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
    const bool given = bnd && (f.kind == DG_BC_STATE || f.kind == DG_BC_OUTFLOW);
    if (given) {
      // given outer state, or the pressure outflow's (inner density and velocity, p_out); the
      // outer viscous flux is taken equal to the inner one below
      if (f.kind == DG_BC_OUTFLOW) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Ux[v] = Uw[v];
        Ux[4] = ph.pout / gm1 + 0.5 * (Uw[1] * Uw[1] + Uw[2] * Uw[2] + Uw[3] * Uw[3]) / Uw[0];
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) Ux[v] = ph.ub[v];
      }
    } else if (bnd && f.kind == DG_BC_WALL_ISOTHERMAL) {
      // isothermal wall: velocity reversed; outer gradient equal to the inner one
      Ux[0] = Uw[0]; Ux[1] = -Uw[1]; Ux[2] = -Uw[2]; Ux[3] = -Uw[3]; Ux[4] = Uw[4];
      if (NS && !VH) {
#pragma unroll
        for (int c = 0; c < 12; ++c) gx[c] = gw[c];
      }
    } else if (bnd && f.kind == DG_BC_WALL) {
      // no-slip wall: velocity reversed; velocity gradient kept, temperature gradient mirrored
      Ux[0] = Uw[0]; Ux[1] = -Uw[1]; Ux[2] = -Uw[2]; Ux[3] = -Uw[3]; Ux[4] = Uw[4];
      if (NS && !VH) {
#pragma unroll
        for (int c = 0; c < 12; ++c) gx[c] = gw[c];
        double tg[3] = {gw[3], gw[7], gw[11]};
        mirror3(tg, nh);
        gx[3] = tg[0]; gx[7] = tg[1]; gx[11] = tg[2];
      }
    } else if (bnd) {
      // symmetry plane: mirror image of the inner state and gradients
#pragma unroll
      for (int v = 0; v < 5; ++v) Ux[v] = Uw[v];
      mirror3(Ux + 1, nh);
      if (NS && !VH) {
#pragma unroll
        for (int c = 0; c < 12; ++c) gx[c] = gw[c];
        mirror_grad(gx, nh);
      }
    }
    const double *UM = mst ? Uw : Ux, *US = mst ? Ux : Uw;
    double F[5];
    riemann(ph, UM, US, nh, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] *= sh;
    if (NS && !VH) {
      const double *gM = mst ? gw : gx, *gS = mst ? gx : gw;
      double FvM[5], FvS[5];
      const Pr5 PM = to_prim(UM, gm1), PS = to_prim(US, gm1);
      flux_v(PM, gM, ph, nt, FvM);
      if (given) {
#pragma unroll
        for (int v = 0; v < 5; ++v) FvS[v] = FvM[v];
      } else {
        flux_v(PS, gS, ph, nt, FvS);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] -= 0.5 * (FvM[v] + FvS[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sF[(s * 5 + v) * n2 + ab] = sg * F[v];
    if (SVM) {
      // minus the BR1 mean of the viscous flux along this side's +xi_dn direction (the split
      // form's reading of the traces and boundary kinds), applied outward
      const double *fo = g.Gf + ((size_t)e * 6 + s) * 4 * n2 + ab;
      double V[4];
      if (given) {
#pragma unroll
        for (int c = 0; c < 4; ++c) V[c] = fo[c * n2];
      } else if (bnd && (f.kind == DG_BC_WALL || f.kind == DG_BC_WALL_ISOTHERMAL)) {
        // no-slip wall: the momentum part of the inner flux; at an isothermal wall the inner heat
        // flux (the energy flux minus the work of the stress)
#pragma unroll
        for (int c = 0; c < 3; ++c) V[c] = fo[c * n2];
        V[3] = f.kind == DG_BC_WALL_ISOTHERMAL
                   ? fo[3 * n2] - (V[0] * Uw[1] + V[1] * Uw[2] + V[2] * Uw[3]) * (1.0 / Uw[0])
                   : 0.0;
      } else if (bnd) {
        // symmetry plane: the normal part of the momentum flux
        const double gm = fo[0] * nh[0] + fo[n2] * nh[1] + fo[2 * n2] * nh[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) V[c] = gm * nh[c];
        V[3] = 0.0;
      } else {
        const double *pn = g.Gf + ((size_t)nb * 6 + 2 * f.dn + (f.plus ? 1 : 0)) * 4 * n2 + f.a + n * f.b;
        const double sn = (GEN && f.plus == plus) ? -1.0 : 1.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) V[c] = 0.5 * (fo[c * n2] + sn * pn[c * n2]);
      }
      const double sp = plus ? 1.0 : -1.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) sF[(s * 5 + 1 + c) * n2 + ab] -= sp * V[c];
    }
    if (PFM) {
      // minus the outward BR1 mean of the viscous flux: each side's flux carries its own outward
      // normal (the two normals of a face are negatives of each other), a boundary side's the
      // mean itself
      const double *po = g.Gf + ((size_t)e * 6 + s) * 4 * n2 + ab;
      if (bnd) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sF[(s * 5 + 1 + c) * n2 + ab] -= po[c * n2];
      } else {
        const double *pn = g.Gf + ((size_t)nb * 6 + 2 * f.dn + (f.plus ? 1 : 0)) * 4 * n2 + f.a + n * f.b;
#pragma unroll
        for (int c = 0; c < 4; ++c) sF[(s * 5 + 1 + c) * n2 + ab] -= 0.5 * (po[c * n2] - pn[c * n2]);
      }
    }
  }
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int i = t % n, j = (t / n) % n, k = t / n2;
  Pr5 Po;
  double go[12];  // the node's lifted gradients, loaded after the face phase
  if (t < n3) {
    if (!VH) Po = to_prim(Uo, gm1);
    if (NS && !VH) {
#pragma unroll
      for (int c = 0; c < 12; ++c) go[c] = Ge[c * n3 + t];
    }
  }
  for (int dir = 0; dir < 3; ++dir) {
    double Fint[5], nv[3];
    __syncthreads();
    if (t < n3) {
      const double *Jd = g.Ja + ((size_t)e * 9 + dir * 3) * n3 + t;
      nv[0] = Jd[0]; nv[1] = Jd[n3]; nv[2] = Jd[2 * n3];
      double Fc[5], Fv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      double Un[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Un[v] = sU[v * n3 + t];
      if (VH) Po = to_prim(Un, gm1);  // recomputed per direction: not held across the phases
      flux_c(Un, Po, nv, Fc);
      if (NS && !VH) flux_v(Po, go, ph, nv, Fv);
#pragma unroll
      for (int v = 0; v < 5; ++v) Fint[v] = Fc[v] - Fv[v];
      if (FORM == 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) sX[d * n3 + t] = nv[d];
#pragma unroll
        for (int v = 0; v < 5; ++v) sX[(3 + v) * n3 + t] = Fv[v];
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) sX[v * n3 + t] = Fint[v];
      }
    }
    __syncthreads();
    if (t < n3) {
      const int id = dir == 0 ? i : (dir == 1 ? j : k);
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int base = t - id * str;
      // at most four nodes' loads in flight: with all n of the last direction's in flight beside
      // the epilogue's loads the LG operators spilled 84 bytes
#pragma unroll 4
      for (int m = 0; m < n; ++m) {
        const int qm = base + m * str;
        const double Dm = sD[id * n + m];
        if (FORM == 1) {
          double Ub[5], F[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) Ub[v] = sU[v * n3 + qm];
          const Pr5 Pb = to_prim(Ub, gm1);
          const double nm[3] = {0.5 * (nv[0] + sX[qm]), 0.5 * (nv[1] + sX[n3 + qm]), 0.5 * (nv[2] + sX[2 * n3 + qm])};
          flux_2pt(ph.vf, Uo, Po, Ub, Pb, nm, gm1, F);
          const double D2 = 2.0 * Dm;
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] += D2 * F[v] - Dm * sX[(3 + v) * n3 + qm];
        } else {
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] += Dm * sX[v * n3 + qm];
        }
      }
      // surface integral of the two faces of this direction
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int s = 2 * dir + sd;
        const double lh = slh[(sd ? n : 0) + id];
        if (LGL && lh == 0.0) continue;
        const int a = dir == 0 ? j : i, b = dir == 2 ? j : k;
        const int ab = a + n * b;
        const double sg = sd ? 1.0 : -1.0;
        // strong and split forms on LGL nodes: minus the face node's own interior flux (on LG
        // nodes its interpolation is part of Tab::Ds)
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          double pen = sF[(s * 5 + v) * n2 + ab];
          if (FORM != 0 && LGL) pen -= sg * Fint[v];
          acc[v] += lh * pen;
        }
      }
    }
  }
  if (t < n3) {
    if (VH) {
      // the viscous volume term, formed by the lifting kernel
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[1 + c] -= g.Gd[((size_t)e * 4 + c) * n3 + t];
    }
    const double sj = g.sJ[(size_t)e * n3 + t];
    if (MODE == 0) {
      double *Oe = out + (size_t)e * 5 * n3;
#pragma unroll
      for (int v = 0; v < 5; ++v) Oe[v * n3 + t] = -acc[v] * sj;
    } else {
      double *Oe = out + (size_t)e * 5 * n3;
      double *Re = R + (size_t)e * 5 * n3;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double ut = -acc[v] * sj;
        // a = 0 (first stage) does not read R, so R may hold anything on entry
        const double r = (ca != 0.0 ? ca * Re[v * n3 + t] : 0.0) + dt * ut;
        Re[v * n3 + t] = r;
        Oe[v * n3 + t] = sU[v * n3 + t] + cb * r;  // the node's state from LDS: not held in registers
      }
    }
  }
}

// ----------------------------------------------------------------------------- split form, LGL
// one Newton step: for ratios that only enter through a correction of relative size < 1e-4
__device__ __forceinline__ double frcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// per-node state of the two-point fluxes: rho, u, v, w, and
//   EC:  b = beta = rho/(2p), q = |u|^2
//   KEP, central: b = p, q = H = (E+p)/rho
struct PS {
  double r, u, v, w, b, q;
};

// Coefficients of f/artanh(f) = 1 + C1 u + C2 u^2 + C3 u^3 + O(u^4), u = f^2 (inverse of the
// series artanh(f)/f = 1 + u/3 + u^2/5 + u^3/7 + ...); the truncation error is below 3e-18
// relative for u < 1e-4.
#define DG_LM_C1 (-1.0 / 3.0)
#define DG_LM_C2 (-4.0 / 45.0)
#define DG_LM_C3 (-44.0 / 945.0)

// Twice the two-point flux of the pair (A, B) contracted with the mean metric, given the
// metric sum nS = Ja(A) + Ja(B) (eq. semiDiscreteSplit: the volume term is 2 D_ij F#(i,j)).
// VF 0: kinetic-energy preserving (Pirozzoli); 1: entropy conserving (Chandrashekar) with the
// logarithmic means f (a+b)/(2 artanh f), f = (a-b)/(a+b), by series for f^2 < 1e-4 and by
// logarithms otherwise; 2: mean of the two Euler fluxes.  kg = 1/(gamma-1).
template <int VF>
__device__ __forceinline__ void pair2(const PS &A, const PS &B, const double *nS, double kg, double *F) {
  const double su = A.u + B.u, sv = A.v + B.v, sw = A.w + B.w;
  if (VF == 2) {
    const double una = A.u * nS[0] + A.v * nS[1] + A.w * nS[2];
    const double unb = B.u * nS[0] + B.v * nS[1] + B.w * nS[2];
    const double ma = 0.5 * A.r * una, mb = 0.5 * B.r * unb, ps = 0.5 * (A.b + B.b);
    F[0] = ma + mb;
    F[1] = fma(ma, A.u, fma(mb, B.u, ps * nS[0]));
    F[2] = fma(ma, A.v, fma(mb, B.v, ps * nS[1]));
    F[3] = fma(ma, A.w, fma(mb, B.w, ps * nS[2]));
    F[4] = fma(ma, A.q, mb * B.q);
    return;
  }
  const double un = su * nS[0] + sv * nS[1] + sw * nS[2];  // 4 {u}.{Ja}
  const double sr = A.r + B.r;
  double f0, pp, e4;
  if (VF == 0) {
    // {rho}{u.Ja}, {u} F_rho + {p}{Ja}, F_rho {H}
    f0 = 0.25 * sr * un;
    pp = 0.5 * (A.b + B.b);
    e4 = 0.5 * (A.q + B.q);
  } else {
    const double dr = A.r - B.r;
    const double fr = dr * frcp1(sr);
    const double ur = fr * fr;
    double rl;  // rho^ln / 2
    // beyond the series, log(a) - log(b) as one logarithm of the larger over the smaller
    // argument (the same bits from either end of the pair)
    if (ur < 1e-4) {
      rl = 0.25 * sr * fma(ur, fma(ur, fma(ur, DG_LM_C3, DG_LM_C2), DG_LM_C1), 1.0);
    } else {
      rl = 0.5 * fabs(dr) / log(fmax(A.r, B.r) * frcp(fmin(A.r, B.r)));
    }
    const double sb = A.b + B.b, db = A.b - B.b;
    const double rb = frcp(sb);
    const double fb = db * rb, ub = fb * fb;
    double eb;  // 1 / (2 (gamma-1) beta^ln)
    if (ub < 1e-4) {
      eb = kg * rb * fma(ub, fma(ub, fma(ub, 1.0 / 7.0, 1.0 / 5.0), 1.0 / 3.0), 1.0);
    } else {
      eb = 0.5 * kg * log(fmax(A.b, B.b) * frcp(fmin(A.b, B.b))) / fabs(db);
    }
    f0 = rl * un;                // 2 rho^ln {u}.{Ja}
    pp = 0.5 * sr * rb;          // {rho} / (2 {beta})
    e4 = eb - 0.25 * (A.q + B.q);
  }
  const double hg = 0.5 * f0;
  F[0] = f0;
  F[1] = fma(hg, su, pp * nS[0]);
  F[2] = fma(hg, sv, pp * nS[1]);
  F[3] = fma(hg, sw, pp * nS[2]);
  if (VF == 0)
    F[4] = f0 * e4;
  else
    F[4] = fma(0.5, su * F[1] + sv * F[2] + sw * F[3], f0 * e4);
}

// partner state from the LDS copy (rho, u, v, w, beta|H); the sixth field is derived:
// |u|^2 for EC, p = ((gamma-1)/gamma) rho (H - |u|^2/2) for KEP and central (gg = (gamma-1)/gamma)
template <int VF>
__device__ __forceinline__ PS load_ps(const double *sS, int n3, int q, double gg) {
  PS s;
  s.r = sS[q]; s.u = sS[n3 + q]; s.v = sS[2 * n3 + q]; s.w = sS[3 * n3 + q];
  const double q2 = s.u * s.u + s.v * s.v + s.w * s.w;
  if (VF == 1) {
    s.b = sS[4 * n3 + q];
    s.q = q2;
  } else {
    s.q = sS[4 * n3 + q];
    s.b = gg * s.r * (s.q - 0.5 * q2);
  }
  return s;
}

template <int VF>
__device__ __forceinline__ void riemann_vf(const Phys &ph, const double *UL, const double *UR, const double *nh,
                                           double *F) {
  if (ph.rs < 2) {
    riemann(ph, UL, UR, nh, F);
    return;
  }
  const double gm1 = ph.gamma - 1.0;
  const Pr5 L = to_prim(UL, gm1), R = to_prim(UR, gm1);
  PS a, b;
  a.r = L.rho; a.u = L.u; a.v = L.v; a.w = L.w;
  b.r = R.rho; b.u = R.u; b.v = R.v; b.w = R.w;
  if (VF == 1) {
    a.b = 0.5 * L.rho / L.p; a.q = L.u * L.u + L.v * L.v + L.w * L.w;
    b.b = 0.5 * R.rho / R.p; b.q = R.u * R.u + R.v * R.v + R.w * R.w;
  } else {
    a.b = L.p; a.q = (UL[4] + L.p) / L.rho;
    b.b = R.p; b.q = (UR[4] + R.p) / R.rho;
  }
  // pair2 along the metric sum nh + nh returns twice the flux along nh
  const double n2[3] = {2.0 * nh[0], 2.0 * nh[1], 2.0 * nh[2]};
  pair2<VF>(a, b, n2, 1.0 / gm1, F);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] *= 0.5;
  if (ph.rs == 3) {
    double D[5];
    roe_diss(UL, L, UR, R, nh, gm1, D);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] -= 0.5 * D[v];
  }
}

// orders this wave's LDS accesses before and after the call (LDS executes one wave's
// instructions in order, so lanes of one wave need no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS sizes (doubles) of one element in the split-form kernel.  Region A first holds the
// contravariant viscous fluxes of the three directions (12 per node), then the two-point state
// (5 per node) and the metric terms Ja^i_d (9 per node); region P first holds the six faces'
// numerical fluxes, then the partner shares of the exchange rounds.
template <int N> struct SplitLds {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static constexpr int A = 14 * n3;
  static constexpr int P = (5 * n3 > 30 * n2) ? 5 * n3 : 30 * n2;
};

template <int N>
__device__ __forceinline__ void split_tables(const Tab *tb, int t, int nthreads, double *sD, double *slh) {
  constexpr int n = N + 1;
  for (int c = t; c < n * n; c += nthreads) sD[c] = tb->D[c];
  if (t < n) { slh[t] = tb->lhm[t]; slh[n + t] = tb->lhp[t]; }
}

// Lane layout of the split-form kernel.  With n = 7 (N = 6) the element's 343 nodes are laid out
// on padded 8 x 8 planes, one k-plane per 64-lane wave (lane i + 8 j + 64 k, lanes with i = 7 or
// j = 7 idle): 448 lanes instead of 384, but the lines of the first two directions then lie
// inside one wave, like those of n = 8.  Other degrees map lane t to node t.
#ifndef DG_SPLIT_PAD7
#define DG_SPLIT_PAD7 1
#endif
template <int N> struct SplitSz {
  static constexpr int n = N + 1;
  static constexpr bool PAD = DG_SPLIT_PAD7 && n == 7;
  static constexpr int NT = PAD ? 64 * n : Sz<N>::NT;
};

// exchange rounds of direction dir stay inside one 64-lane wave: lines of the first two
// directions when n divides 64 and n^2 divides 64 (n = 2, 4, 8) or the planes are padded to
// 8 x 8; every line when the whole element fits one wave
template <int n> __host__ __device__ constexpr bool wave_local(int dir) {
  return (n * n * n <= 64) || (dir < 2 && (n == 2 || n == 4 || n == 8 || SplitSz<n - 1>::PAD));
}

// Split-form operator on LGL nodes (eq. semiDiscreteSplit) for element e by the NT threads t of
// one slot: every unordered pair of nodes on a line is evaluated once; the pair's contribution
// to the other node goes through an LDS accumulator.  Viscous part in strong form, surface
// penalty f* s - F_int.N, -1/J, optional RK update.  Directions whose lines lie inside one wave
// order their exchange rounds with a wave fence instead of a workgroup barrier.
template <int N, bool NS, int VF, int MODE, int GEN, bool FVM = false>
__device__ __forceinline__ void split_body(const Geo &g, const Phys &ph, int e, bool valid, int lane,
                                           const double *__restrict__ U, const double *__restrict__ G,
                                           double *__restrict__ out, double *__restrict__ R, double ca, double cb,
                                           double dt, double *sA, double *sP, const double *sD, const double *slh) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, NT = SplitSz<N>::NT;
  // t: this lane's node (lanes past the element, or on the padding, are idle)
  int t = lane;
  bool inb = lane < n3;
  if constexpr (SplitSz<N>::PAD) {
    const int i = lane & 7, j = (lane >> 3) & 7, k = lane >> 6;
    inb = i < n && j < n && k < n;
    t = i + n * (j + n * k);
  }
  const bool act = valid && inb;
  const double gm1 = ph.gamma - 1.0, kg = 1.0 / gm1, gg = gm1 / ph.gamma;
  const double *Ue = U + (size_t)e * 5 * n3;
  const double *Jae = g.Ja + (size_t)e * 9 * n3;
  double *sS = sA;           // rho, u, v, w, beta (EC) or H (KEP, central) per node
  double *sJ = sA + 5 * n3;  // Ja^i_d at (i*3+d)*n3 + node
  // Navier-Stokes: the lifting kernel has formed the viscous divergence (Geo::Gd) and the face
  // traces of the viscous fluxes (Geo::Gf)
  const double *Gfe = NS ? g.Gf + (size_t)e * 24 * n2 : nullptr;
  // the node's own state is loaded before the face phase, so that its latency overlaps with it
  double Uo[5];
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) Uo[v] = Ue[v * n3 + t];
  }
  // numerical surface flux on the six faces, stored outward for this element
  for (int q = valid ? lane : 6 * n2; q < 6 * n2; q += NT) {
    const int s = q / n2, ab = q - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
    const bool plus = s & 1;
    const int nb = g.nbr[(size_t)e * 6 + s];
    const NbFace f = nbr_face<n, (GEN > 0)>(g, e, s, a, b);
    const bool bnd = GEN && f.bnd;
    if (GEN == 2 && bnd && f.kind == FACE_MORTAR) {
      // non-conforming face: the outward flux from the mortar face array
      const double *mf = g.mflux + (size_t)g.mslot[(size_t)e * 6 + s] * 5 * n2 + ab;
#pragma unroll
      for (int v = 0; v < 5; ++v) sP[(s * 5 + v) * n2 + ab] = mf[v * n2];
      continue;
    }
    if (FVM && g.fvflag[nb]) {
      // face shared with a finite-volume element: the outward flux at the face nodes
      const double *fx = g.fvFx + ((size_t)e * 6 + s) * 5 * n2 + ab;
#pragma unroll
      for (int v = 0; v < 5; ++v) sP[(s * 5 + v) * n2 + ab] = fx[v * n2];
      continue;
    }
    const double *Un = U + (size_t)(bnd ? e : nb) * 5 * n3;
    const int qo = line_node<n>(dn, a, b, plus ? N : 0);
    const int qn = GEN ? line_node<n>(f.dn, f.a, f.b, f.plus ? N : 0) : line_node<n>(dn, a, b, plus ? 0 : N);
    // this side's trace of Fv^dn at the face point (component c at fo[c * n2]) and the
    // neighbour's trace of Fv^{f.dn} on its side of the face (fnb[c * n2])
    const double *fo = NS ? Gfe + s * 4 * n2 + ab : nullptr;
    const double *fnb = NS ? g.Gf + ((size_t)(bnd ? e : nb) * 6 + 2 * f.dn + (f.plus ? 1 : 0)) * 4 * n2 + f.a + n * f.b
                           : nullptr;
    double Uw[5], Ux[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) { Uw[v] = Ue[v * n3 + qo]; Ux[v] = bnd ? Uw[v] : Un[v * n3 + qn]; }
    // normal along +xi_dn scaled by s-hat: Ja^dn at the face node, the master's on the master
    // side and (up to rounding, the metric terms being continuous across the face) on the slave
    const double sg = plus ? 1.0 : -1.0;
    const double nt[3] = {Jae[(dn * 3) * n3 + qo], Jae[(dn * 3 + 1) * n3 + qo], Jae[(dn * 3 + 2) * n3 + qo]};
    const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    const double ish = 1.0 / sh;
    const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
    const bool given = bnd && (f.kind == DG_BC_STATE || f.kind == DG_BC_OUTFLOW);
    const bool iso = bnd && f.kind == DG_BC_WALL_ISOTHERMAL;
    const bool wall = bnd && (f.kind == DG_BC_WALL || iso);
    if (given && f.kind == DG_BC_OUTFLOW) {
      // pressure outflow: the own trace's density and velocity with p_out
      Ux[4] = ph.pout / gm1 + 0.5 * (Uw[1] * Uw[1] + Uw[2] * Uw[2] + Uw[3] * Uw[3]) / Uw[0];
    } else if (given) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Ux[v] = ph.ub[v];  // given outer state
    } else if (wall) {
      Ux[1] = -Uw[1]; Ux[2] = -Uw[2]; Ux[3] = -Uw[3];  // no-slip wall: velocity reversed
    } else if (bnd) {
      mirror3(Ux + 1, nh);  // symmetry plane: mirror image of the inner state
    }
    const double *UM = plus ? Uw : Ux, *US = plus ? Ux : Uw;
    double F[5];
    riemann_vf<VF>(ph, UM, US, nh, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] *= sh;
    if (NS) {
      // BR1 mean of the viscous fluxes along this side's +xi_dn normal Ja^dn: on both sides the
      // contravariant flux of the face's direction (the normal metric of a conforming face is
      // continuous: the neighbour's Ja of its face direction is +-Ja^dn, + where one side is a
      // +xi side and the other a -xi side)
      if (given) {
        // given outer state: the outer viscous flux equals the inner one
#pragma unroll
        for (int c = 0; c < 4; ++c) F[1 + c] -= fo[c * n2];
      } else if (wall) {
        // no-slip wall: the outer momentum flux equals the inner one, the outer energy flux is
        // its negative (reversed velocity, mirrored heat flux), so the mean keeps the momentum;
        // at an isothermal wall the outer gradient is the inner one, so the mean energy flux is
        // the inner heat flux: the inner energy flux minus the work (tau Ja^dn) . u
        double g3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          g3[c] = fo[c * n2];
          F[1 + c] -= g3[c];
        }
        if (iso) {
          const double ir = 1.0 / Uw[0];
          F[4] -= fo[3 * n2] - (g3[0] * Uw[1] + g3[1] * Uw[2] + g3[2] * Uw[3]) * ir;
        }
      } else if (bnd) {
        // symmetry plane: the mirrored outer flux cancels the inner shear and heat flux, the
        // mean keeps the normal part of the momentum flux
        const double gm = fo[0] * nh[0] + fo[n2] * nh[1] + fo[2 * n2] * nh[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) F[1 + c] -= gm * nh[c];
      } else if (GEN) {
        const double sn = (f.plus != plus) ? 1.0 : -1.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) F[1 + c] -= 0.5 * (fo[c * n2] + sn * fnb[c * n2]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) F[1 + c] -= 0.5 * (fo[c * n2] + fnb[c * n2]);
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sP[(s * 5 + v) * n2 + ab] = sg * F[v];
  }
  __syncthreads();
  PS o;
  double p = 0.0;
  if (act) {
    const Pr5 P = to_prim(Uo, gm1);
    p = P.p;
    o.r = P.rho; o.u = P.u; o.v = P.v; o.w = P.w;
    if (VF == 1) {
      o.b = 0.5 * P.rho / P.p;
      o.q = P.u * P.u + P.v * P.v + P.w * P.w;
    } else {
      o.b = P.p;
      o.q = (Uo[4] + P.p) / P.rho;
    }
  }
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int id3[3] = {t % n, (t / n) % n, t / n2};
  if (act) {
    // surface integral, numerical-flux part: lhat(+-1) f* s on the faces through this node
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
      const int id = id3[dir];
      if (id != 0 && id != N) continue;
      const int sd = (id == N) ? 1 : 0;
      const int s = 2 * dir + sd;
      const double lh = slh[(sd ? n : 0) + id];
      const int a = dir == 0 ? id3[1] : id3[0], b = dir == 2 ? id3[1] : id3[2];
      const int ab = a + n * b;
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] += lh * sP[(s * 5 + v) * n2 + ab];
    }
  }
  double ja[9];
  if (act) {
#pragma unroll
    for (int c = 0; c < 9; ++c) ja[c] = Jae[c * n3 + t];
  }
  if (act) {
    sS[t] = o.r; sS[n3 + t] = o.u; sS[2 * n3 + t] = o.v; sS[3 * n3 + t] = o.w;
    sS[4 * n3 + t] = (VF == 1) ? o.b : o.q;
#pragma unroll
    for (int c = 0; c < 9; ++c) sJ[c * n3 + t] = ja[c];
  }
  // the first direction's barrier also separates the face-flux reads above from the partner
  // shares and publishes the staged state of every node
  double Rq[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, sjq = 0.0;
#pragma unroll
  for (int dir = 0; dir < 3; ++dir) {
    if (dir == 2 && act) {
      // the epilogue's loads are issued before the last direction's rounds
      sjq = g.sJ[(size_t)e * n3 + t];
      if (MODE == 1 && ca != 0.0) {
        const double *Re = R + (size_t)e * 5 * n3;
#pragma unroll
        for (int v = 0; v < 5; ++v) Rq[v] = Re[v * n3 + t];
      }
    }
    const bool wl = wave_local<n>(dir);
    if (dir > 0 && wl) wave_sync(); else __syncthreads();
    const double *sJd = sJ + 3 * dir * n3;
    double nvo[3] = {0.0, 0.0, 0.0};
    if (act) { nvo[0] = sJd[t]; nvo[1] = sJd[n3 + t]; nvo[2] = sJd[2 * n3 + t]; }
    const int id = act ? id3[dir] : 0;
    const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
    const int base = t - id * str;
    // pairs (id, id+s mod n), s = 1 .. (n-1)/2: each unordered pair once, both nodes updated
#pragma unroll 1
    for (int sft = 1; sft <= (n - 1) / 2; ++sft) {
      // barriers stay in uniform control flow: only the work is guarded
      if (act) {
        int jp = id + sft;
        if (jp >= n) jp -= n;
        const int qp = base + jp * str;
        const PS bq = load_ps<VF>(sS, n3, qp, gg);
        const double nS[3] = {nvo[0] + sJd[qp], nvo[1] + sJd[n3 + qp], nvo[2] + sJd[2 * n3 + qp]};
        double F[5];
        pair2<VF>(o, bq, nS, kg, F);
        const double Dij = sD[id * n + jp], Dji = sD[jp * n + id];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          acc[v] = fma(Dij, F[v], acc[v]);
          sP[v * n3 + qp] = Dji * F[v];
        }
      }
      // every node receives exactly one partner share per round: collect it in a fixed order
      if (wl) wave_sync(); else __syncthreads();
      if (act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += sP[v * n3 + t];
      }
      if (wl) wave_sync(); else __syncthreads();
    }
    if (act && (n & 1) == 0) {
      // s = n/2 pairs each other twice: each side takes only its own share
      int jp = id + n / 2;
      if (jp >= n) jp -= n;
      const int qp = base + jp * str;
      const PS bq = load_ps<VF>(sS, n3, qp, gg);
      const double nS[3] = {nvo[0] + sJd[qp], nvo[1] + sJd[n3 + qp], nvo[2] + sJd[2 * n3 + qp]};
      double F[5];
      pair2<VF>(o, bq, nS, kg, F);
      const double Dij = sD[id * n + jp];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] = fma(Dij, F[v], acc[v]);
    }
    if (act && (id == 0 || id == N)) {
      // end nodes of the line: diagonal F#(U,U) = F(U).Ja (D_ii is non-zero only there on LGL
      // lines) and the interior convective part - F_int . N_out lhat(+-1) of the surface integral
      const Pr5 P = {o.r, o.u, o.v, o.w, p};
      double Fc[5];
      flux_c(Uo, P, nvo, Fc);
      const double Dii = sD[id * n + id];
      const bool plus = id == N;
      const double lh = slh[(plus ? n : 0) + id];
      const double cd = 2.0 * Dii + (plus ? -lh : lh);
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] += cd * Fc[v];
    }
  }
  if (act) {
    if (NS) {
      // viscous part in strong form, formed by the lifting kernel (loaded here: held through the
      // rounds, these four values push the operator past its register budget)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[1 + c] -= g.Gd[((size_t)e * 4 + c) * n3 + t];
    }
    const double sj = sjq;
    double *Oe = out + (size_t)e * 5 * n3;
    if (MODE == 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Oe[v * n3 + t] = -acc[v] * sj;
    } else {
      double *Re = R + (size_t)e * 5 * n3;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        // a = 0 (first stage) does not read R, so R may hold anything on entry
        const double r = (ca != 0.0 ? ca * Rq[v] : 0.0) + dt * (-acc[v] * sj);
        Re[v * n3 + t] = r;
        Oe[v * n3 + t] = Uo[v] + cb * r;
      }
    }
  }
}

template <int N, bool NS, int VF, int MODE, int GEN, bool FVM = false>
__global__ void __launch_bounds__(SplitSz<N>::NT, DG_SPLIT_MINB) k_split(Geo g, Phys ph, const double *__restrict__ U,
                                                     const double *__restrict__ G, double *__restrict__ out,
                                                     double *__restrict__ R, double ca, double cb, double dt) {
  using L = SplitLds<N>;
  constexpr int n = L::n;
  __shared__ double sA[L::A], sP[L::P];
  __shared__ double sD[n * n], slh[2 * n];
  split_tables<N>(g.tab, threadIdx.x, SplitSz<N>::NT, sD, slh);
  const int e = xcd_element(blockIdx.x, g.K);
  if (e >= g.K) return;
  if (FVM && g.fvflag[e]) return;  // a finite-volume element
  split_body<N, NS, VF, MODE, GEN, FVM>(g, ph, e, true, threadIdx.x, U, G, out, R, ca, cb, dt, sA, sP, sD, slh);
}

// ----------------------------------------------------------------------------- ensemble batch
// Workgroups of the batched kernels walk the concatenated element list of all members of one
// degree; EPB elements share a workgroup (one slot of Sz<N>::NT threads each, SplitSz<N>::NT in
// the split-form kernel, wave aligned).
// Each slot finds its member by bisection of the element prefix sums.
__device__ __forceinline__ int member_of(const int *first, int count, int item) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int N, int EPB, bool GEN>
__global__ void __launch_bounds__(Sz<N>::NT * EPB, DG_LIFT_MINB) k_lift_b(BatchView bv) {
  using L = LiftLds<N>;
  constexpr int n = L::n, NT = Sz<N>::NT, SM = L::W + L::JA + L::WS;
  __shared__ double sm[EPB * SM];
  __shared__ double sDh[n * n], sl[2 * n], slh[2 * n];
  lift_tables<N>(bv.tab, threadIdx.x, NT * EPB, sDh, sl, slh);
  const int nblk = (bv.total + EPB - 1) / EPB;
  const int blk = xcd_element(blockIdx.x, nblk);
  if (blk >= nblk) return;
  const int slot = __builtin_amdgcn_readfirstlane(threadIdx.x / NT);
  const int t = threadIdx.x - slot * NT;
  const int item = blk * EPB + slot;
  const bool valid = item < bv.total;
  const int mi = member_of(bv.first, bv.count, valid ? item : bv.total - 1);
  const Member &M = bv.m[mi];
  lift_body<N, true, LIFT_DIV, GEN>(M.g, M.ph, valid ? item - bv.first[mi] : 0, valid, t, M.U, nullptr, nullptr,
                                    sm + slot * SM, sDh, sl, slh);
}

template <int N, bool NS, int VF, int EPB, bool GEN>
__global__ void __launch_bounds__(SplitSz<N>::NT * EPB, DG_SPLIT_MINB) k_split_b(BatchView bv) {
  using L = SplitLds<N>;
  constexpr int n = L::n, NT = SplitSz<N>::NT;
  __shared__ double sA[EPB * L::A], sP[EPB * L::P];
  __shared__ double sD[n * n], slh[2 * n];
  split_tables<N>(bv.tab, threadIdx.x, NT * EPB, sD, slh);
  const int nblk = (bv.total + EPB - 1) / EPB;
  const int blk = xcd_element(blockIdx.x, nblk);
  if (blk >= nblk) return;
  const int slot = __builtin_amdgcn_readfirstlane(threadIdx.x / NT);
  const int t = threadIdx.x - slot * NT;
  const int item = blk * EPB + slot;
  const bool valid = item < bv.total;
  const int mi = member_of(bv.first, bv.count, valid ? item : bv.total - 1);
  const Member &M = bv.m[mi];
  split_body<N, NS, VF, 1, GEN>(M.g, M.ph, valid ? item - bv.first[mi] : 0, valid, t, M.U, M.G, M.out, M.R, M.a, M.b,
                           M.dt, sA + slot * L::A, sP + slot * L::P, sD, slh);
}

// ----------------------------------------------------------------------------- reductions
// partial[e][0..7]: timestep -> {max sum lambda_c, max sum lambda_v};
// integrals -> {rho, m1, m2, m3, E, KE, entropy, min J}; finite -> {count of non-finite}
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_reduce(Geo g, Phys ph, int what, const double *__restrict__ U,
                                                      double *__restrict__ partial) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, NT = S::NT;
  __shared__ double red[8][NT];
  const int e = blockIdx.x, t = threadIdx.x;
  const double gm1 = ph.gamma - 1.0;
  double val[8];
  const bool isMin[8] = {false, false, false, false, false, false, false, true};
#pragma unroll
  for (int c = 0; c < 8; ++c) val[c] = 0.0;
  if (what == RED_INTEGRALS) val[7] = 1e300;
  if (t < n3) {
    double Uq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = U[((size_t)e * 5 + v) * n3 + t];
    if (what == RED_FINITE) {
      double bad = 0.0;
#pragma unroll
      for (int v = 0; v < 5; ++v) bad += isfinite(Uq[v]) ? 0.0 : 1.0;
      val[0] = bad;
    } else {
      const Pr5 P = to_prim(Uq, gm1);
      const double sj = g.sJ[(size_t)e * n3 + t];
      if (what == RED_TIMESTEP) {
        const double c = sqrt(ph.gamma * P.p / P.rho);
        double sc = 0.0, sv = 0.0;
        for (int dir = 0; dir < 3; ++dir) {
          const double *Jd = g.Ja + ((size_t)e * 9 + dir * 3) * n3 + t;
          const double a0 = Jd[0], a1 = Jd[n3], a2 = Jd[2 * n3];
          const double nn = a0 * a0 + a1 * a1 + a2 * a2;
          sc += (fabs(P.u * a0 + P.v * a1 + P.w * a2) + c * sqrt(nn)) * sj;
          sv += fmax(4.0 / 3.0, ph.gamma / ph.Pr) * (ph.mu / P.rho) * nn * sj * sj;
        }
        val[0] = sc; val[1] = sv;
      } else {
        const int i = t % n, j = (t / n) % n, k = t / n2;
        const double wq = g.tab->w[i] * g.tab->w[j] * g.tab->w[k] / sj;
#pragma unroll
        for (int v = 0; v < 5; ++v) val[v] = wq * Uq[v];
        val[5] = wq * 0.5 * (Uq[1] * P.u + Uq[2] * P.v + Uq[3] * P.w);
        const double s = log(P.p) - ph.gamma * log(P.rho);
        val[6] = wq * (-P.rho * s / gm1);
        val[7] = 1.0 / sj;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) red[c][t] = val[c];
  __syncthreads();
  // fold the block onto its largest power-of-two prefix, then halve
  constexpr int P = (NT & (NT - 1)) == 0 ? NT : (NT >= 512 ? 512 : 256);
  for (int off = P; off > 0; off >>= 1) {
    const int lim = (off == P) ? NT - P : off;
    if (off < P || P < NT) {
      if (t < lim) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const double x = red[c][t], y = red[c][t + off];
          if (what == RED_TIMESTEP) red[c][t] = fmax(x, y);
          else if (what == RED_INTEGRALS && isMin[c]) red[c][t] = fmin(x, y);
          else red[c][t] = x + y;
        }
      }
    }
    __syncthreads();
  }
  if (t < 8) partial[(size_t)e * 8 + t] = red[t][0];
}

// ----------------------------------------------------------------------------- mortars
// Non-conforming faces (Sec. 3.2), one workgroup per face: the big side's traces are
// interpolated to every small side's points (I^L or I^U along each cut face direction), the
// small side's term is evaluated there with the small element's own outward normal and written to
// its face-array slot, and projected back to the big side (P^L, P^U; negated: outward of the big
// element).  The element kernels read these slots for the sides their face codes mark.

// value of the nv-component field X ([e][nv][n^3]) at face point (a,b) of side s of element e:
// the face node on LGL nodes, interpolated along the face normal with l(+-1) on LG nodes
template <int n, bool LGL, int NV>
__device__ __forceinline__ void face_trace(const double *__restrict__ X, int e, int s, int a, int b,
                                           const double *lm, const double *lp, double *out) {
  constexpr int n3 = n * n * n;
  const int dn = s >> 1;
  const bool plus = s & 1;
  const double *Xe = X + (size_t)e * NV * n3;
  if (LGL) {
    const int q = line_node<n>(dn, a, b, plus ? n - 1 : 0);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = Xe[v * n3 + q];
  } else {
    const double *l = plus ? lp : lm;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
#pragma unroll 1
    for (int m = 0; m < n; ++m) {
      const int q = line_node<n>(dn, a, b, m);
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] += l[m] * Xe[v * n3 + q];
    }
  }
}

// lifted variables W = (u, v, w, T) at face point (a,b) of side s of element e: W of the face
// node on LGL nodes; on LG nodes W at every node of the line, interpolated with l(+-1) (as the
// conforming lifting does)
template <int n, bool LGL>
__device__ __forceinline__ void face_trace_W(const double *__restrict__ U, int e, int s, int a, int b,
                                             const double *lm, const double *lp, double gm1, double Rg, double *W) {
  constexpr int n3 = n * n * n;
  const int dn = s >> 1;
  const bool plus = s & 1;
  const double *Ue = U + (size_t)e * 5 * n3;
  double Uq[5];
  if (LGL) {
    const int q = line_node<n>(dn, a, b, plus ? n - 1 : 0);
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = Ue[v * n3 + q];
    grad_prim_to_W(Uq, gm1, Rg, W);
    return;
  }
  const double *l = plus ? lp : lm;
#pragma unroll
  for (int v = 0; v < 4; ++v) W[v] = 0.0;
  for (int m = 0; m < n; ++m) {
    const int q = line_node<n>(dn, a, b, m);
    double Wq[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = Ue[v * n3 + q];
    grad_prim_to_W(Uq, gm1, Rg, Wq);
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] += l[m] * Wq[v];
  }
}

// face point of the big side's sub-face that small-side point (a,b) meets (orientation code o:
// swap if o & 4, then reverse the first index if o & 1, the second if o & 2)
template <int n> __device__ __forceinline__ void sub_point(int o, int a, int b, int &a2, int &b2) {
  const int p = (o & 4) ? b : a, q = (o & 4) ? a : b;
  a2 = (o & 1) ? n - 1 - p : p;
  b2 = (o & 2) ? n - 1 - q : q;
}

// interpolation (proj = false) or projection (proj = true) matrices of sub-face p of a mortar of
// type t along the big side's two face directions, from sM = [IL | IU | PL | PU]; nullptr where
// the face is not cut in that direction
template <int n>
__device__ __forceinline__ void sub_ops(const double *sM, int t, int p, bool proj, const double *&M1,
                                        const double *&M2) {
  const int p1 = t == 1 ? p : (t == 3 ? (p & 1) : -1);
  const int p2 = t == 2 ? p : (t == 3 ? (p >> 1) : -1);
  const double *base = sM + (proj ? 2 * n * n : 0);
  M1 = p1 < 0 ? nullptr : base + p1 * n * n;
  M2 = p2 < 0 ? nullptr : base + p2 * n * n;
}
__device__ __forceinline__ double mcoef(const double *M, int n, int r, int c) {
  return M ? M[r * n + c] : (r == c ? 1.0 : 0.0);
}

// sum over the big side's points (m, l) of M1[r1][m] M2[r2][l] X[v][m + n l], v < NV
template <int n, int NV>
__device__ __forceinline__ void sub_apply(const double *M1, const double *M2, int r1, int r2, const double *X,
                                          double *out) {
  constexpr int n2 = n * n;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = 0.0;
#pragma unroll 1
  for (int l = 0; l < n; ++l) {
    const double c2 = mcoef(M2, n, r2, l);
    if (c2 == 0.0) continue;
#pragma unroll 1
    for (int m = 0; m < n; ++m) {
      const double c1 = mcoef(M1, n, r1, m);
      if (c1 == 0.0) continue;
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] += c1 * (c2 * X[v * n2 + m + n * l]);
    }
  }
}

template <int N, bool LGL>
__global__ void __launch_bounds__(256) k_mortar_lift(Geo g, Phys ph, const MortarDesc *__restrict__ md,
                                                     const double *__restrict__ U) {
  constexpr int n = N + 1, n2 = n * n;
  __shared__ double sM[4 * n * n];    // IL, IU, PL, PU
  __shared__ double sWB[4 * n2];      // W = (u, v, w, T) of the big side's trace
  __shared__ double sT[4 * 12 * n2];  // the small sides' surface terms at their sub-face points
  const int t = threadIdx.x, nth = blockDim.x;
  const Tab *tb = g.tab;
  for (int c = t; c < n * n; c += nth) {
    sM[c] = tb->IL[c]; sM[n * n + c] = tb->IU[c]; sM[2 * n * n + c] = tb->PL[c]; sM[3 * n * n + c] = tb->PU[c];
  }
  const MortarDesc &m = md[blockIdx.x];  // read in place: its arrays are indexed by sub-face
  const double gm1 = ph.gamma - 1.0;
  for (int p = t; p < n2; p += nth) {
    double W[4];
    face_trace_W<n, LGL>(U, m.eb, m.sb, p % n, p / n, tb->lm, tb->lp, gm1, ph.R, W);
#pragma unroll
    for (int v = 0; v < 4; ++v) sWB[v * n2 + p] = W[v];
  }
  __syncthreads();
  const int cnt = m.type == 3 ? 4 : 2;
  for (int q = t; q < cnt * n2; q += nth) {
    const int pos = q / n2, ab = q - pos * n2, a = ab % n, b = ab / n;
    const int es = m.es[pos], ss = m.ss[pos];
    int a2, b2;
    sub_point<n>(m.o[pos], a, b, a2, b2);
    const double *A1, *A2;
    sub_ops<n>(sM, m.type, pos, false, A1, A2);
    double WB[4], Ws[4];
    sub_apply<n, 4>(A1, A2, a2, b2, sWB, WB);
    face_trace_W<n, LGL>(U, es, ss, a, b, tb->lm, tb->lp, gm1, ph.R, Ws);
    const double *fnp = g.fn + ((size_t)es * 6 + ss) * 3 * n2 + ab;
    const double nt[3] = {fnp[0], fnp[n2], fnp[2 * n2]};
    double *ml = g.mlift + (size_t)m.sl[pos] * 12 * n2 + ab;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double tv = nt[d] * (0.5 * (Ws[v] + WB[v]));
        ml[(d * 4 + v) * n2] = tv;
        sT[(pos * 12 + d * 4 + v) * n2 + a2 + n * b2] = tv;
      }
  }
  __syncthreads();
  for (int q = t; q < n2; q += nth) {
    const int i = q % n, j = q / n;
    double acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = 0.0;
    for (int pos = 0; pos < cnt; ++pos) {
      const double *B1, *B2;
      sub_ops<n>(sM, m.type, pos, true, B1, B2);
#pragma unroll 1
      for (int b2 = 0; b2 < n; ++b2) {
        const double c2 = mcoef(B2, n, j, b2);
        if (c2 == 0.0) continue;
#pragma unroll 1
        for (int a2 = 0; a2 < n; ++a2) {
          const double c = mcoef(B1, n, i, a2) * c2;
          if (c == 0.0) continue;
#pragma unroll
          for (int k = 0; k < 12; ++k) acc[k] -= c * sT[(pos * 12 + k) * n2 + a2 + n * b2];
        }
      }
    }
    double *ml = g.mlift + (size_t)m.slot * 12 * n2 + q;
#pragma unroll
    for (int c = 0; c < 12; ++c) ml[c * n2] = acc[c];
  }
}

// G: the lifted gradients [K][12][n^3] (read on LG nodes); on LGL nodes the gradients at the
// mortar sides' points come from Geo::mg, written by the lifting kernel
template <int N, bool LGL, bool NS>
__global__ void __launch_bounds__(256) k_mortar_flux(Geo g, Phys ph, const MortarDesc *__restrict__ md,
                                                     const double *__restrict__ U, const double *__restrict__ G) {
  constexpr int n = N + 1, n2 = n * n;
  __shared__ double sM[4 * n * n];
  __shared__ double sUB[5 * n2];
  __shared__ double sGB[NS ? 12 * n2 : 1];
  __shared__ double sF[4 * 5 * n2];  // the small sides' fluxes at their sub-face points
  const int t = threadIdx.x, nth = blockDim.x;
  const Tab *tb = g.tab;
  for (int c = t; c < n * n; c += nth) {
    sM[c] = tb->IL[c]; sM[n * n + c] = tb->IU[c]; sM[2 * n * n + c] = tb->PL[c]; sM[3 * n * n + c] = tb->PU[c];
  }
  const MortarDesc &m = md[blockIdx.x];  // read in place: its arrays are indexed by sub-face
  const double gm1 = ph.gamma - 1.0;
  for (int p = t; p < n2; p += nth) {
    double Uq[5];
    face_trace<n, LGL, 5>(U, m.eb, m.sb, p % n, p / n, tb->lm, tb->lp, Uq);
#pragma unroll
    for (int v = 0; v < 5; ++v) sUB[v * n2 + p] = Uq[v];
    if (NS) {
      double gq[12];
      if (LGL) {
        const double *mg = g.mg + (size_t)m.slot * 12 * n2 + p;
#pragma unroll
        for (int c = 0; c < 12; ++c) gq[c] = mg[c * n2];
      } else {
        face_trace<n, false, 12>(G, m.eb, m.sb, p % n, p / n, tb->lm, tb->lp, gq);
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) sGB[c * n2 + p] = gq[c];
    }
  }
  __syncthreads();
  const int cnt = m.type == 3 ? 4 : 2;
  for (int q = t; q < cnt * n2; q += nth) {
    const int pos = q / n2, ab = q - pos * n2, a = ab % n, b = ab / n;
    const int es = m.es[pos], ss = m.ss[pos];
    int a2, b2;
    sub_point<n>(m.o[pos], a, b, a2, b2);
    const double *A1, *A2;
    sub_ops<n>(sM, m.type, pos, false, A1, A2);
    // the small side is the master of its part of the face: its own normal, its state first
    double UM[5], US[5];
    face_trace<n, LGL, 5>(U, es, ss, a, b, tb->lm, tb->lp, UM);
    sub_apply<n, 5>(A1, A2, a2, b2, sUB, US);
    const double *fnp = g.fn + ((size_t)es * 6 + ss) * 3 * n2 + ab;
    const double nt[3] = {fnp[0], fnp[n2], fnp[2 * n2]};
    const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    const double ish = 1.0 / sh;
    const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
    double F[5];
    riemann(ph, UM, US, nh, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] *= sh;
    if (NS) {
      // BR1: mean of the two sides' viscous fluxes, the big side's state and gradients interpolated
      double gM[12], gS[12], FvM[5], FvS[5];
      if (LGL) {
        const double *mg = g.mg + (size_t)m.sl[pos] * 12 * n2 + ab;
#pragma unroll
        for (int c = 0; c < 12; ++c) gM[c] = mg[c * n2];
      } else {
        face_trace<n, false, 12>(G, es, ss, a, b, tb->lm, tb->lp, gM);
      }
      sub_apply<n, 12>(A1, A2, a2, b2, sGB, gS);
      const Pr5 PM = to_prim(UM, gm1), PS = to_prim(US, gm1);
      flux_v(PM, gM, ph, nt, FvM);
      flux_v(PS, gS, ph, nt, FvS);
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] -= 0.5 * (FvM[v] + FvS[v]);
    }
    double *mf = g.mflux + (size_t)m.sl[pos] * 5 * n2 + ab;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      mf[v * n2] = F[v];
      sF[(pos * 5 + v) * n2 + a2 + n * b2] = F[v];
    }
  }
  __syncthreads();
  for (int q = t; q < n2; q += nth) {
    const int i = q % n, j = q / n;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int pos = 0; pos < cnt; ++pos) {
      const double *B1, *B2;
      sub_ops<n>(sM, m.type, pos, true, B1, B2);
#pragma unroll 1
      for (int b2 = 0; b2 < n; ++b2) {
        const double c2 = mcoef(B2, n, j, b2);
        if (c2 == 0.0) continue;
#pragma unroll 1
        for (int a2 = 0; a2 < n; ++a2) {
          const double c = mcoef(B1, n, i, a2) * c2;
          if (c == 0.0) continue;
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] -= c * sF[(pos * 5 + v) * n2 + a2 + n * b2];
        }
      }
    }
    double *mf = g.mflux + (size_t)m.slot * 5 * n2 + q;
#pragma unroll
    for (int v = 0; v < 5; ++v) mf[v * n2] = acc[v];
  }
}

// ----------------------------------------------------------------------------- FV subcells
// Shock capturing with finite volumes on (N+1)^3 equal subcells of each troubled element (Sec. 4):
// the element's U then holds subcell means; V = V_DG=>FV converts (eq. FVvdm, dg2fv).  Euler
// equations, conforming meshes without boundary sides.

__device__ __forceinline__ double fv_limit(int lim, double a, double b) {
  if (lim == 0 || a * b <= 0.0) return 0.0;
  if (lim == 1) return fabs(a) < fabs(b) ? a : b;  // minmod
  return 2.0 * a * b / (a + b);                   // van Leer
}
__device__ __forceinline__ void fv_prim(const double *U, double gm1, double *W) {
  const double ir = 1.0 / U[0];
  W[0] = U[0]; W[1] = U[1] * ir; W[2] = U[2] * ir; W[3] = U[3] * ir;
  W[4] = gm1 * (U[4] - 0.5 * U[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]));
}
__device__ __forceinline__ void fv_cons(const double *W, double gm1, double *U) {
  U[0] = W[0]; U[1] = W[0] * W[1]; U[2] = W[0] * W[2]; U[3] = W[0] * W[3];
  U[4] = W[4] / gm1 + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

// reconstructed state of finite-volume element e at its boundary subface (a,b) of side s: the
// limited slope of the adjacent subcell from the next inner subcell and the outer datum Do
template <int n>
__device__ __forceinline__ void fv_recon(const double *__restrict__ U, const FvGeo &f, double gm1, int e, int s, int a,
                                         int b, const double *Do, double *Uf) {
  constexpr int n3 = n * n * n;
  const int dn = s >> 1;
  const bool plus = s & 1;
  const double *Ue = U + (size_t)e * 5 * n3;
  const int q0 = line_node<n>(dn, a, b, plus ? n - 1 : 0), q1 = line_node<n>(dn, a, b, plus ? n - 2 : 1);
  double U0[5], U1[5], W0[5], W1[5], Wo[5], Wf[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) { U0[v] = Ue[v * n3 + q0]; U1[v] = Ue[v * n3 + q1]; }
  fv_prim(U0, gm1, W0);
  fv_prim(U1, gm1, W1);
  fv_prim(Do, gm1, Wo);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double sm = plus ? W0[v] - W1[v] : W0[v] - Wo[v];
    const double sp = plus ? Wo[v] - W0[v] : W1[v] - W0[v];
    const double sg = fv_limit(f.limiter, sm, sp);
    Wf[v] = plus ? W0[v] + 0.5 * sg : W0[v] - 0.5 * sg;
  }
  fv_cons(Wf, gm1, Uf);
}

// (M x M) applied at face point (a,b) of a face field T[v][ia + n jb] (5 fields): sum over jb of
// M[b][jb] (sum over ia of M[a][ia] T[ia + n jb])
template <int n>
__device__ __forceinline__ void face_mm(const double *M, int a, int b, const double *T, double *out) {
  constexpr int n2 = n * n;
  double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int jb = 0; jb < n; ++jb) {
    double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ia = 0; ia < n; ++ia) {
      const double m = M[a * n + ia];
#pragma unroll
      for (int v = 0; v < 5; ++v) c[v] += m * T[v * n2 + ia + n * jb];
    }
    const double m2 = M[b * n + jb];
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] += m2 * c[v];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = r[v];
}

// Work lists of the hybrid operator, rebuilt whenever the element types change: the finite-volume
// elements (count[0] of them in list) and the master sides e*6+s of the faces that touch one
// (count[1] in faces).  The order of either list is arbitrary: every item writes only its own
// outputs.
template <int N> __global__ void k_fv_lists_zero(FvGeo f) {
  if (threadIdx.x == 0) { f.count[0] = 0; f.count[1] = 0; }
}

template <int N, bool GEN>
__global__ void __launch_bounds__(256) k_fv_lists(Geo g, FvGeo f) {
  constexpr int n = N + 1;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= 6 * g.K) return;
  const int e = q / 6, s = q - 6 * e;
  if (s == 0 && f.flag[e]) f.list[atomicAdd(&f.count[0], 1)] = e;
  const int nb = g.nbr[q];
  if (nb < 0) return;
  const NbFace f0 = nbr_face<n, (GEN > 0)>(g, e, s, 0, 0);
  if (f0.master && (f.flag[e] || f.flag[nb])) f.faces[atomicAdd(&f.count[1], 1)] = q;
}

template <int N> struct FvFaceSz {
  static constexpr int NT = ((N + 1) * (N + 1) + 63) / 64 * 64;  // threads: one face point each
};

// Faces that touch a finite-volume element, one workgroup per face of the work list (looping over
// it): the numerical flux at the (N+1)^2 subfaces from both sides' face data (the DG side's trace
// taken to subface means with V in both face directions, the FV side reconstructed); writes both
// sides' outward fluxes (a DG side's back to its face nodes with V^-1) and both sides' view of the
// other's face datum.
template <int N, bool LGL, bool GEN>
__global__ void __launch_bounds__(FvFaceSz<N>::NT) k_fv_face(Geo g, Phys ph, FvGeo f, const double *__restrict__ U) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  __shared__ double sV[n * n], sVi[n * n];
  __shared__ double sTe[5 * n2], sTn[5 * n2];  // DG traces (own / neighbour face coordinates)
  __shared__ double sFe[5 * n2], sFn[5 * n2];  // outward subface fluxes of both sides
  const int t = threadIdx.x;
  for (int c = t; c < n * n; c += blockDim.x) { sV[c] = f.V[c]; sVi[c] = f.Vi[c]; }
  const int nf = f.count[1];
  const double gm1 = ph.gamma - 1.0;
  const Tab *tb = g.tab;
  const bool pt = t < n2;
  const int a = pt ? t % n : 0, b = pt ? t / n : 0;
  for (int it = blockIdx.x; it < nf; it += gridDim.x) {
    const int q = f.faces[it], e = q / 6, s = q - 6 * e;
    const int nb = g.nbr[q];
    const NbFace fm = nbr_face<n, (GEN > 0)>(g, e, s, a, b);
    const int ns = GEN ? 2 * fm.dn + (fm.plus ? 1 : 0) : (s ^ 1);
    const int a2 = fm.a, b2 = fm.b;
    const bool fe = f.flag[e], fn = f.flag[nb];
    __syncthreads();  // the previous face's reads of the LDS fields are done
    if (pt) {
      double tr[5];
      if (!fe) {
        face_trace<n, LGL, 5>(U, e, s, a, b, tb->lm, tb->lp, tr);
#pragma unroll
        for (int v = 0; v < 5; ++v) sTe[v * n2 + t] = tr[v];
      }
      if (!fn) {
        face_trace<n, LGL, 5>(U, nb, ns, a2, b2, tb->lm, tb->lp, tr);
#pragma unroll
        for (int v = 0; v < 5; ++v) sTn[v * n2 + a2 + n * b2] = tr[v];
      }
    }
    __syncthreads();
    if (pt) {
      // face data: the adjacent subcell (FV) or the subface mean of the trace (DG)
      double De[5], Dn[5], Ue[5], Un[5];
      if (fe) {
        const int qe = line_node<n>(s >> 1, a, b, (s & 1) ? n - 1 : 0);
#pragma unroll
        for (int v = 0; v < 5; ++v) De[v] = U[((size_t)e * 5 + v) * n3 + qe];
      } else {
        face_mm<n>(sV, a, b, sTe, De);
      }
      if (fn) {
        const int qn = line_node<n>(ns >> 1, a2, b2, (ns & 1) ? n - 1 : 0);
#pragma unroll
        for (int v = 0; v < 5; ++v) Dn[v] = U[((size_t)nb * 5 + v) * n3 + qn];
      } else {
        face_mm<n>(sV, a2, b2, sTn, Dn);
      }
      double *dxe = f.Dx + ((size_t)e * 6 + s) * 5 * n2 + t;
      double *dxn = f.Dx + ((size_t)nb * 6 + ns) * 5 * n2 + a2 + n * b2;
#pragma unroll
      for (int v = 0; v < 5; ++v) { dxe[v * n2] = Dn[v]; dxn[v * n2] = De[v]; }
      if (fe) {
        fv_recon<n>(U, f, gm1, e, s, a, b, Dn, Ue);
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) Ue[v] = De[v];
      }
      if (fn) {
        fv_recon<n>(U, f, gm1, nb, ns, a2, b2, De, Un);
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) Un[v] = Dn[v];
      }
      // the master's (this side's) face-mean metric, outward
      const bool plus = s & 1;
      const double *Nm = f.Nf + ((((size_t)e * 3 + (s >> 1)) * (n + 1) + (plus ? n : 0)) * n2 + t) * 3;
      const double sgn = plus ? 1.0 : -1.0;
      const double nt[3] = {sgn * Nm[0], sgn * Nm[1], sgn * Nm[2]};
      const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
      const double ish = 1.0 / sh;
      const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
      double F[5];
      riemann(ph, Ue, Un, nh, F);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        sFe[v * n2 + t] = sh * F[v];
        sFn[v * n2 + a2 + n * b2] = -(sh * F[v]);
      }
    }
    __syncthreads();
    if (pt) {
      // thread t writes point t of either side (in that side's own face coordinates)
      double o[5];
      double *fx = f.Fx + ((size_t)e * 6 + s) * 5 * n2 + t;
      if (fe) {
#pragma unroll
        for (int v = 0; v < 5; ++v) o[v] = sFe[v * n2 + t];
      } else {
        face_mm<n>(sVi, a, b, sFe, o);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) fx[v * n2] = o[v];
      fx = f.Fx + ((size_t)nb * 6 + ns) * 5 * n2 + t;
      if (fn) {
#pragma unroll
        for (int v = 0; v < 5; ++v) o[v] = sFn[v * n2 + t];
      } else {
        face_mm<n>(sVi, a, b, sFn, o);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) fx[v * n2] = o[v];
    }
  }
}

// Finite-volume elements of the work list, one workgroup per element (looping over the list):
// second-order subcell update, eq. fv_dof_time_derivative.
template <int N, int MODE, int RS>
__global__ void __launch_bounds__(Sz<N>::NT, 4) k_fv_volume(Geo g, Phys ph, FvGeo f, const double *__restrict__ U,
                                                         double *__restrict__ out, double *__restrict__ R, double ca,
                                                         double cb, double dt) {
  using S = Sz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
  __shared__ double sW[5 * n3];  // primitive subcell means
  __shared__ double sF[5 * n3];  // flux through each subcell's + face (inner faces)
  const int t = threadIdx.x;
  const bool act = t < n3;
  const double gm1 = ph.gamma - 1.0;
  const int nfv = f.count[0];
  for (int it = blockIdx.x; it < nfv; it += gridDim.x) {
    const int e = f.list[it];
    __syncthreads();  // the previous element's reads of the LDS fields are done
    if (act) {
      double Uo[5], W[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Uo[v] = U[((size_t)e * 5 + v) * n3 + t];
      fv_prim(Uo, gm1, W);
#pragma unroll
      for (int v = 0; v < 5; ++v) sW[v * n3 + t] = W[v];
    }
    const int id3[3] = {t % n, (t / n) % n, t / n2};
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int dir = 0; dir < 3; ++dir) {
      __syncthreads();  // sW is complete; the previous direction's reads of sF are done
      const int id = act ? id3[dir] : 0;
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int a = dir == 0 ? id3[1] : id3[0], b = dir == 2 ? id3[1] : id3[2];
      const int ab = a + n * b;
      if (act && id < N) {
        // inner face id + 1/2 between subcells c0 = id and c1 = id + 1 along dir: the two
        // reconstructed states from the stencil c0 - 1 .. c1 + 1, whose ends beyond the element
        // are the outer face data of its sides
        double Wm[5], Wp[5];
        if (id > 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) Wm[v] = sW[v * n3 + t - str];
        } else {
          double Do[5];
          const double *dx = f.Dx + ((size_t)e * 6 + 2 * dir) * 5 * n2 + ab;
#pragma unroll
          for (int v = 0; v < 5; ++v) Do[v] = dx[v * n2];
          fv_prim(Do, gm1, Wm);
        }
        if (id + 1 < N) {
#pragma unroll
          for (int v = 0; v < 5; ++v) Wp[v] = sW[v * n3 + t + 2 * str];
        } else {
          double Do[5];
          const double *dx = f.Dx + ((size_t)e * 6 + 2 * dir + 1) * 5 * n2 + ab;
#pragma unroll
          for (int v = 0; v < 5; ++v) Do[v] = dx[v * n2];
          fv_prim(Do, gm1, Wp);
        }
        double UL[5], UR[5];
        {
          double WL[5], WR[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double w0 = sW[v * n3 + t], w1 = sW[v * n3 + t + str];
            WL[v] = w0 + 0.5 * fv_limit(f.limiter, w0 - Wm[v], w1 - w0);
            WR[v] = w1 - 0.5 * fv_limit(f.limiter, w1 - w0, Wp[v] - w1);
          }
          fv_cons(WL, gm1, UL);
          fv_cons(WR, gm1, UR);
        }
        const double *Nm = f.Nf + ((((size_t)e * 3 + dir) * (n + 1) + id + 1) * n2 + ab) * 3;
        const double sh = sqrt(Nm[0] * Nm[0] + Nm[1] * Nm[1] + Nm[2] * Nm[2]);
        const double ish = 1.0 / sh;
        const double nh[3] = {Nm[0] * ish, Nm[1] * ish, Nm[2] * ish};
        double F[5];
        riemann_t<RS>(ph, UL, UR, nh, F);
        // the subcell's outward flux on its + face; the next subcell's - face reads it from sF
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const double fp = sh * F[v];
          sF[v * n3 + t] = fp;
          acc[v] += fp;
        }
      }
      __syncthreads();
      if (act) {
        const double *fx0 = f.Fx + ((size_t)e * 6 + 2 * dir) * 5 * n2 + ab;
        const double *fx1 = f.Fx + ((size_t)e * 6 + 2 * dir + 1) * 5 * n2 + ab;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          // outward fluxes of the subcell: + face (above for inner faces), then - face
          if (id == N) acc[v] += fx1[v * n2];
          acc[v] += (id > 0) ? -sF[v * n3 + t - str] : fx0[v * n2];
        }
      }
    }
    if (act) {
      const double iwj = 1.0 / (f.w * f.Jbar[(size_t)e * n3 + t]);
      double *Oe = out + (size_t)e * 5 * n3;
      if (MODE == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) Oe[v * n3 + t] = -acc[v] * iwj;
      } else {
        double *Re = R + (size_t)e * 5 * n3;
        const double *Ue = U + (size_t)e * 5 * n3;  // read again (from L2) rather than held
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const double r = (ca != 0.0 ? ca * Re[v * n3 + t] : 0.0) + dt * (-acc[v] * iwj);
          Re[v * n3 + t] = r;
          Oe[v * n3 + t] = Ue[v * n3 + t] + cb * r;
        }
      }
    }
  }
}

// apply the n x n matrix A along all three directions to the 5 fields of sX (in place through sY)
template <int n, int NV = 5>
__device__ __forceinline__ void fv_tensor3(const double *A, double *sX, int t, bool act) {
  constexpr int n2 = n * n, n3 = n2 * n;
  const int i = t % n, j = (t / n) % n, k = t / n2;
  for (int dir = 0; dir < 3; ++dir) {
    double r[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) r[v] = 0.0;
    if (act) {
      const int id = dir == 0 ? i : (dir == 1 ? j : k);
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int base = t - id * str;
      for (int m = 0; m < n; ++m) {
        const double c = A[id * n + m];
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] += c * sX[v * n3 + base + m * str];
      }
    }
    __syncthreads();  // every line is read before any node is overwritten
    if (act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sX[v * n3 + t] = r[v];
    }
    __syncthreads();
  }
}

// troubled-cell indicator (modal decay of rho p) and, with do_switch, the switch with hysteresis in
// place (U <- V U to finite volume above hi, U <- V^-1 U back to DG below lo)
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_fv_switch(Geo g, Phys ph, FvGeo f, double *__restrict__ U,
                                                         int do_switch) {
  using S = Sz<N>;
  constexpr int n = S::n, n3 = S::n3;
  __shared__ double sX[5 * n3], sU[5 * n3];
  __shared__ double sA[3 * n * n];  // V, Vi, Li
  __shared__ double sE[3 * (Sz<N>::NT / 64)];
  __shared__ int sNew;
  const int e = blockIdx.x, t = threadIdx.x;
  const bool act = t < n3;
  for (int c = t; c < n * n; c += blockDim.x) { sA[c] = f.V[c]; sA[n * n + c] = f.Vi[c]; sA[2 * n * n + c] = f.Li[c]; }
  const bool isfv = f.flag[e];
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double u = U[((size_t)e * 5 + v) * n3 + t];
      sU[v * n3 + t] = u;
      sX[v * n3 + t] = u;
    }
  }
  __syncthreads();
  if (isfv) fv_tensor3<n>(sA + n * n, sX, t, act);  // nodal values of the element's DG reading
  if (act) {
    double W[5], Uq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = sX[v * n3 + t];
    fv_prim(Uq, ph.gamma - 1.0, W);
    sX[t] = W[0] * W[4];  // q = rho p in field 0
  }
  __syncthreads();
  fv_tensor3<n, 1>(sA + 2 * n * n, sX, t, act);  // modal coefficients (field 0)
  {
    // energies: of all modes, of those whose largest index is N, of those whose largest index is
    // N-1; summed per wave by a fixed butterfly, then over the waves in order
    double E3[3] = {0.0, 0.0, 0.0};
    if (act) {
      const int i = t % n, j = (t / n) % n, k = t / (n * n);
      const int m = i > j ? (i > k ? i : k) : (j > k ? j : k);
      const double c2 = sX[t] * sX[t];
      E3[0] = c2;
      E3[1] = m == N ? c2 : 0.0;
      E3[2] = m == N - 1 ? c2 : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) E3[c] += __shfl_xor(E3[c], off, 64);
    if ((t & 63) == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sE[3 * (t >> 6) + c] = E3[c];
    }
  }
  __syncthreads();
  if (t == 0) {
    double tot = 0.0, eN = 0.0, eN1 = 0.0;
    for (int w = 0; w < Sz<N>::NT / 64; ++w) { tot += sE[3 * w]; eN += sE[3 * w + 1]; eN1 += sE[3 * w + 2]; }
    const double r1 = eN / fmax(tot, 1e-300);
    const double r2 = eN1 / fmax(tot - eN, 1e-300);
    const double ind = log10(fmax(fmax(r1, r2), 1e-300));
    f.ind[e] = ind;
    int nw = isfv ? 1 : 0;
    if (do_switch) {
      if (!isfv && ind > f.hi) nw = 1;
      if (isfv && ind < f.lo) nw = 0;
    }
    sNew = nw;
  }
  __syncthreads();
  const int nw = sNew;
  if (nw == (isfv ? 1 : 0)) return;  // uniform across the workgroup
  fv_tensor3<n>(nw ? sA : sA + n * n, sU, t, act);
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) U[((size_t)e * 5 + v) * n3 + t] = sU[v * n3 + t];
  }
  if (t == 0) f.flag[e] = (uint8_t)nw;
}

// ----------------------------------------------------------------------------- launchers
#define DG_CHECK_LAUNCH()                                   \
  do {                                                      \
    hipError_t _e = hipGetLastError();                      \
    if (_e != hipSuccess) return DG_ERR_HIP;                \
  } while (0)

template <int N, bool LGL, bool NS, int FORM>
static int launch_main_t(const Geo &g, const Phys &ph, const double *U, const double *G, double *out, double *R,
                         double a, double b, double dt, int mode, hipStream_t st) {
  dim3 grid(g.K), block(Sz<N>::NT);
  const bool gen = g.fc != nullptr;
  if constexpr (!NS) {
    if (g.fvflag) {
      if (mode == 0)
        hipLaunchKernelGGL((k_main<N, LGL, NS, FORM, 0, 1, true>), grid, block, 0, st, g, ph, U, G, out, R, a, b, dt);
      else
        hipLaunchKernelGGL((k_main<N, LGL, NS, FORM, 1, 1, true>), grid, block, 0, st, g, ph, U, G, out, R, a, b, dt);
      DG_CHECK_LAUNCH();
      return DG_OK;
    }
  }
  // GEN: 0 structured, 1 face codes, 2 face codes and non-conforming faces
  const int lev = !gen ? 0 : (g.mslot ? 2 : 1);
#define DG_KM(M_, G_) hipLaunchKernelGGL((k_main<N, LGL, NS, FORM, M_, G_>), grid, block, 0, st, g, ph, U, G, out, R, a, b, dt)
  if (mode == 0) {
    if (lev == 0) DG_KM(0, 0); else if (lev == 1) DG_KM(0, 1); else DG_KM(0, 2);
  } else {
    if (lev == 0) DG_KM(1, 0); else if (lev == 1) DG_KM(1, 1); else DG_KM(1, 2);
  }
#undef DG_KM
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N, bool NS, int VF>
static int launch_split_t(const Geo &g, const Phys &ph, const double *U, const double *G, double *out, double *R,
                          double a, double b, double dt, int mode, hipStream_t st) {
  dim3 grid(xcd_grid(g.K)), block(SplitSz<N>::NT);
  const bool gen = g.fc != nullptr;
  if constexpr (!NS) {
    if (g.fvflag) {
      if (mode == 0)
        hipLaunchKernelGGL((k_split<N, NS, VF, 0, 1, true>), grid, block, 0, st, g, ph, U, G, out, R, a, b, dt);
      else
        hipLaunchKernelGGL((k_split<N, NS, VF, 1, 1, true>), grid, block, 0, st, g, ph, U, G, out, R, a, b, dt);
      DG_CHECK_LAUNCH();
      return DG_OK;
    }
  }
  // GEN: 0 structured, 1 face codes, 2 face codes and non-conforming faces
  const int lev = !gen ? 0 : (g.mslot ? 2 : 1);
#define DG_KS(M_, G_) hipLaunchKernelGGL((k_split<N, NS, VF, M_, G_>), grid, block, 0, st, g, ph, U, G, out, R, a, b, dt)
  if (mode == 0) {
    if (lev == 0) DG_KS(0, 0); else if (lev == 1) DG_KS(0, 1); else DG_KS(0, 2);
  } else {
    if (lev == 0) DG_KS(1, 0); else if (lev == 1) DG_KS(1, 1); else DG_KS(1, 2);
  }
#undef DG_KS
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N, bool LGL, bool NS>
static int launch_form(const Geo &g, const Phys &ph, int form, const double *U, const double *G, double *out,
                       double *R, double a, double b, double dt, int mode, hipStream_t st) {
  if (form == DG_FORM_WEAK) return launch_main_t<N, LGL, NS, 0>(g, ph, U, G, out, R, a, b, dt, mode, st);
  if (form == DG_FORM_STRONG) return launch_main_t<N, LGL, NS, 2>(g, ph, U, G, out, R, a, b, dt, mode, st);
  if (!LGL) return DG_ERR_UNSUPPORTED;
  if (form == DG_FORM_SPLIT) {
    if (ph.vf == DG_VF_EC) return launch_split_t<N, NS, 1>(g, ph, U, G, out, R, a, b, dt, mode, st);
    if (ph.vf == DG_VF_KEP) return launch_split_t<N, NS, 0>(g, ph, U, G, out, R, a, b, dt, mode, st);
    return launch_split_t<N, NS, 2>(g, ph, U, G, out, R, a, b, dt, mode, st);
  }
  return DG_ERR_UNSUPPORTED;
}

template <int N>
int launch_prolong(const Geo &g, const Phys &ph, const double *U, hipStream_t st) {
  hipLaunchKernelGGL((k_prolong<N>), dim3(xcd_grid(g.K)), dim3(Sz<N>::NT), 0, st, g, ph, U);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_lift(const Geo &g, const Phys &ph, bool lgl, int out, const double *U, double *G, double *Fv,
                hipStream_t st) {
  dim3 grid(xcd_grid(g.K)), block(Sz<N>::NT);
  // GEN: 0 structured, 1 face codes, 2 face codes and non-conforming faces
  const int lev = g.fc == nullptr ? 0 : (g.mslot ? 2 : 1);
#define DG_KL(L_, O_) \
  do { \
    if (lev == 0) hipLaunchKernelGGL((k_lift<N, L_, O_, 0>), grid, block, 0, st, g, ph, U, G, Fv); \
    else if (lev == 1) hipLaunchKernelGGL((k_lift<N, L_, O_, 1>), grid, block, 0, st, g, ph, U, G, Fv); \
    else hipLaunchKernelGGL((k_lift<N, L_, O_, 2>), grid, block, 0, st, g, ph, U, G, Fv); \
  } while (0)
  if (out == LIFT_SV) {
    // the strong-form operator of conforming meshes on LG nodes
    if (lev == 2 || lgl) return DG_ERR_UNSUPPORTED;
    if (lev == 0) hipLaunchKernelGGL((k_lift<N, false, LIFT_SV, 0>), grid, block, 0, st, g, ph, U, G, Fv);
    else hipLaunchKernelGGL((k_lift<N, false, LIFT_SV, 1>), grid, block, 0, st, g, ph, U, G, Fv);
  } else if (out == LIFT_WV) {
    // the weak-form operator of conforming meshes
    if (lev == 2) return DG_ERR_UNSUPPORTED;
    if (lgl) {
      if (lev == 0) hipLaunchKernelGGL((k_lift<N, true, LIFT_WV, 0>), grid, block, 0, st, g, ph, U, G, Fv);
      else hipLaunchKernelGGL((k_lift<N, true, LIFT_WV, 1>), grid, block, 0, st, g, ph, U, G, Fv);
    } else {
      if (lev == 0) hipLaunchKernelGGL((k_lift<N, false, LIFT_WV, 0>), grid, block, 0, st, g, ph, U, G, Fv);
      else hipLaunchKernelGGL((k_lift<N, false, LIFT_WV, 1>), grid, block, 0, st, g, ph, U, G, Fv);
    }
  } else if (!lgl) {
    if (out == LIFT_G) DG_KL(false, LIFT_G);
    else if (out == LIFT_GT) DG_KL(false, LIFT_GT);
    else return DG_ERR_UNSUPPORTED;
  } else if (out == LIFT_G) {
    DG_KL(true, LIFT_G);
  } else if (out == LIFT_FV) {
    DG_KL(true, LIFT_FV);
  } else if (out == LIFT_DIV) {
    DG_KL(true, LIFT_DIV);
  } else if (out == LIFT_DIVK) {
    DG_KL(true, LIFT_DIVK);
  } else {
    return DG_ERR_UNSUPPORTED;
  }
#undef DG_KL
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_main(const Geo &g, const Phys &ph, bool lgl, int eqn, int form, const double *U, const double *G,
                double *out, double *R, double a, double b, double dt, int mode, hipStream_t st) {
  const bool ns = (eqn == DG_NAVIER_STOKES);
  if (lgl) {
    if (ns) return launch_form<N, true, true>(g, ph, form, U, G, out, R, a, b, dt, mode, st);
    return launch_form<N, true, false>(g, ph, form, U, G, out, R, a, b, dt, mode, st);
  }
  if (ns) return launch_form<N, false, true>(g, ph, form, U, G, out, R, a, b, dt, mode, st);
  return launch_form<N, false, false>(g, ph, form, U, G, out, R, a, b, dt, mode, st);
}

template <int N, int EPB>
static int launch_batch_lift_t(const BatchView &bv, hipStream_t st) {
  const int nblk = (bv.total + EPB - 1) / EPB;
  if (bv.general)
    hipLaunchKernelGGL((k_lift_b<N, EPB, true>), dim3(xcd_grid(nblk)), dim3(Sz<N>::NT * EPB), 0, st, bv);
  else
    hipLaunchKernelGGL((k_lift_b<N, EPB, false>), dim3(xcd_grid(nblk)), dim3(Sz<N>::NT * EPB), 0, st, bv);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N, bool NS, int VF, int EPB>
static int launch_batch_split_t(const BatchView &bv, hipStream_t st) {
  const int nblk = (bv.total + EPB - 1) / EPB;
  if (bv.general)
    hipLaunchKernelGGL((k_split_b<N, NS, VF, EPB, true>), dim3(xcd_grid(nblk)), dim3(SplitSz<N>::NT * EPB), 0, st,
                       bv);
  else
    hipLaunchKernelGGL((k_split_b<N, NS, VF, EPB, false>), dim3(xcd_grid(nblk)), dim3(SplitSz<N>::NT * EPB), 0, st,
                       bv);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N, bool NS, int EPB>
static int launch_batch_split_vf(const BatchView &bv, int vf, hipStream_t st) {
  if (vf == DG_VF_EC) return launch_batch_split_t<N, NS, 1, EPB>(bv, st);
  if (vf == DG_VF_KEP) return launch_batch_split_t<N, NS, 0, EPB>(bv, st);
  return launch_batch_split_t<N, NS, 2, EPB>(bv, st);
}

template <int N>
int launch_batch_lift(const BatchView &bv, int epb, hipStream_t st) {
  if (bv.total <= 0) return DG_OK;
  if (epb == 1) return launch_batch_lift_t<N, 1>(bv, st);
  if constexpr (batch_max_epb(N) >= 2)
    if (epb == 2) return launch_batch_lift_t<N, 2>(bv, st);
  if constexpr (batch_max_epb(N) >= 4)
    if (epb == 4) return launch_batch_lift_t<N, 4>(bv, st);
  return DG_ERR_UNSUPPORTED;
}

template <int N>
int launch_batch_split(const BatchView &bv, bool ns, int vf, int epb, hipStream_t st) {
  if (bv.total <= 0) return DG_OK;
  if (epb == 1) return ns ? launch_batch_split_vf<N, true, 1>(bv, vf, st) : launch_batch_split_vf<N, false, 1>(bv, vf, st);
  if constexpr (batch_max_epb(N) >= 2)
    if (epb == 2)
      return ns ? launch_batch_split_vf<N, true, 2>(bv, vf, st) : launch_batch_split_vf<N, false, 2>(bv, vf, st);
  if constexpr (batch_max_epb(N) >= 4)
    if (epb == 4)
      return ns ? launch_batch_split_vf<N, true, 4>(bv, vf, st) : launch_batch_split_vf<N, false, 4>(bv, vf, st);
  return DG_ERR_UNSUPPORTED;
}

template <int N>
int launch_fv_face(const Geo &g, const Phys &ph, const FvGeo &f, bool lgl, const double *U, hipStream_t st) {
  const dim3 grid(std::min(3 * g.K, 4096)), block(FvFaceSz<N>::NT);
  const bool gen = g.fc != nullptr;
  if (lgl && gen) hipLaunchKernelGGL((k_fv_face<N, true, true>), grid, block, 0, st, g, ph, f, U);
  else if (lgl) hipLaunchKernelGGL((k_fv_face<N, true, false>), grid, block, 0, st, g, ph, f, U);
  else if (gen) hipLaunchKernelGGL((k_fv_face<N, false, true>), grid, block, 0, st, g, ph, f, U);
  else hipLaunchKernelGGL((k_fv_face<N, false, false>), grid, block, 0, st, g, ph, f, U);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_fv_volume(const Geo &g, const Phys &ph, const FvGeo &f, const double *U, double *out, double *R, double a,
                     double b, double dt, int mode, hipStream_t st) {
  const dim3 grid(std::min(g.K, 1024)), block(Sz<N>::NT);
#define DG_FVV(RS)                                                                                       \
  if (ph.rs == RS) {                                                                                     \
    if (mode == 0) hipLaunchKernelGGL((k_fv_volume<N, 0, RS>), grid, block, 0, st, g, ph, f, U, out, R, a, b, dt); \
    else hipLaunchKernelGGL((k_fv_volume<N, 1, RS>), grid, block, 0, st, g, ph, f, U, out, R, a, b, dt);           \
  }
  DG_FVV(0) DG_FVV(1) DG_FVV(2) DG_FVV(3)
#undef DG_FVV
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_fv_lists(const Geo &g, const FvGeo &f, hipStream_t st) {
  hipLaunchKernelGGL(k_fv_lists_zero<N>, dim3(1), dim3(64), 0, st, f);
  const dim3 grid((6 * g.K + 255) / 256);
  if (g.fc) hipLaunchKernelGGL((k_fv_lists<N, true>), grid, dim3(256), 0, st, g, f);
  else hipLaunchKernelGGL((k_fv_lists<N, false>), grid, dim3(256), 0, st, g, f);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_fv_switch(const Geo &g, const Phys &ph, const FvGeo &f, double *U, int do_switch, hipStream_t st) {
  hipLaunchKernelGGL((k_fv_switch<N>), dim3(g.K), dim3(Sz<N>::NT), 0, st, g, ph, f, U, do_switch);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_mortar_lift(const Geo &g, const Phys &ph, bool lgl, const MortarDesc *md, int nm, const double *U,
                       hipStream_t st) {
  if (nm <= 0) return DG_OK;
  if (lgl) hipLaunchKernelGGL((k_mortar_lift<N, true>), dim3(nm), dim3(256), 0, st, g, ph, md, U);
  else hipLaunchKernelGGL((k_mortar_lift<N, false>), dim3(nm), dim3(256), 0, st, g, ph, md, U);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_mortar_flux(const Geo &g, const Phys &ph, bool lgl, int eqn, const MortarDesc *md, int nm,
                       const double *U, const double *G, hipStream_t st) {
  if (nm <= 0) return DG_OK;
  const bool ns = eqn == DG_NAVIER_STOKES;
  if (lgl && ns) hipLaunchKernelGGL((k_mortar_flux<N, true, true>), dim3(nm), dim3(256), 0, st, g, ph, md, U, G);
  else if (lgl) hipLaunchKernelGGL((k_mortar_flux<N, true, false>), dim3(nm), dim3(256), 0, st, g, ph, md, U, G);
  else if (ns) hipLaunchKernelGGL((k_mortar_flux<N, false, true>), dim3(nm), dim3(256), 0, st, g, ph, md, U, G);
  else hipLaunchKernelGGL((k_mortar_flux<N, false, false>), dim3(nm), dim3(256), 0, st, g, ph, md, U, G);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

template <int N>
int launch_reduce(const Geo &g, const Phys &ph, int what, const double *U, double, double *partial, hipStream_t st) {
  hipLaunchKernelGGL((k_reduce<N>), dim3(g.K), dim3(Sz<N>::NT), 0, st, g, ph, what, U, partial);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

#if !defined(DG_ONLY_N) && !defined(DG_FUSED_BATCH)
// one workgroup folds the per-element partials in a fixed order
__global__ void __launch_bounds__(256) k_final_reduce(int what, const double *__restrict__ partial, int K,
                                                      double *__restrict__ out) {
  __shared__ double red[8][256];
  const int t = threadIdx.x;
  double val[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) val[c] = (what == RED_INTEGRALS && c == 7) ? 1e300 : 0.0;
  for (int e = t; e < K; e += 256) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double x = partial[(size_t)e * 8 + c];
      if (what == RED_TIMESTEP) val[c] = fmax(val[c], x);
      else if (what == RED_INTEGRALS && c == 7) val[c] = fmin(val[c], x);
      else val[c] += x;
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) red[c][t] = val[c];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double x = red[c][t], y = red[c][t + off];
        if (what == RED_TIMESTEP) red[c][t] = fmax(x, y);
        else if (what == RED_INTEGRALS && c == 7) red[c][t] = fmin(x, y);
        else red[c][t] = x + y;
      }
    }
    __syncthreads();
  }
  if (t < 8) out[t] = red[t][0];
}

// quadrature weight of every node: J w_i w_j w_k
__global__ void k_mass(const double *__restrict__ sJ, const double *__restrict__ w, int n, size_t total,
                       double *__restrict__ out) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const int n3 = n * n * n;
  for (; q < total; q += stride) {
    const int node = (int)(q % n3);
    const int i = node % n, j = (node / n) % n, k = node / (n * n);
    out[q] = w[i] * w[j] * w[k] / sJ[q];
  }
}

// y = alpha y + beta x; x may be y
__global__ void k_axpby(double *y, const double *x, double alpha, double beta, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) y[i] = alpha * y[i] + beta * x[i];
}

int launch_final_reduce(int what, const double *partial, int K, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(256), 0, st, what, partial, K, out);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

int launch_mass(const double *sJ, const double *w, int n, size_t total, double *out, hipStream_t st) {
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_mass, dim3((unsigned)blocks), dim3(256), 0, st, sJ, w, n, total, out);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

int launch_axpby(double *y, const double *x, double alpha, double beta, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)blocks), dim3(256), 0, st, y, x, alpha, beta, n);
  DG_CHECK_LAUNCH();
  return DG_OK;
}
#endif

#ifdef DG_FUSED_BATCH
// ----------------------------------------------------------------------------- fused ensemble
// One lifting and one operator launch per stage for the members of every degree (structured
// members): group g of the work takes the workgroups [start[g], start[g+1]) of the grid, each
// workgroup of 512 lanes holds fused_epb elements of its group's degree in slots of the degree's
// own lane count, and the static LDS is the largest degree's, carved per slot.  Lanes past the
// last slot run the per-element code as invalid slots (no memory access, every barrier).
template <int N> constexpr int fused_epb_split() {
  constexpr int by_lanes = 512 / SplitSz<N>::NT;
  constexpr int by_lds = (SplitLds<7>::A + SplitLds<7>::P) / (SplitLds<N>::A + SplitLds<N>::P);
  return by_lanes < by_lds ? by_lanes : by_lds;
}
template <int N> constexpr int fused_epb_lift() {
  constexpr int by_lanes = 512 / Sz<N>::NT;
  constexpr int by_lds = (LiftLds<7>::W + LiftLds<7>::JA + LiftLds<7>::WS) /
                         (LiftLds<N>::W + LiftLds<N>::JA + LiftLds<N>::WS);
  return by_lanes < by_lds ? by_lanes : by_lds;
}

__device__ __forceinline__ int fused_group(const FusedView &fv, int b) {
  int gi = 0;
  while (gi + 1 < fv.ng && b >= fv.start[gi + 1]) ++gi;
  return gi;
}

template <int N, bool NS, int VF>
__device__ __forceinline__ void fused_split_group(const BatchView &bv, int blk, double *smem, double *sD, double *slh) {
  using L = SplitLds<N>;
  constexpr int NT = SplitSz<N>::NT, EPB = fused_epb_split<N>();
  split_tables<N>(bv.tab, threadIdx.x, 512, sD, slh);
  const int raw = __builtin_amdgcn_readfirstlane(threadIdx.x / NT);
  const int slot = raw < EPB ? raw : EPB - 1;
  const int t = threadIdx.x - raw * NT;
  const int item = blk * EPB + slot;
  const bool valid = raw < EPB && item < bv.total;
  const int mi = member_of(bv.first, bv.count, valid ? item : bv.total - 1);
  const Member &M = bv.m[mi];
  split_body<N, NS, VF, 1, false>(M.g, M.ph, valid ? item - bv.first[mi] : 0, valid, t, M.U, M.G, M.out, M.R, M.a,
                                  M.b, M.dt, smem + slot * L::A, smem + EPB * L::A + slot * L::P, sD, slh);
}

template <bool NS, int VF>
__global__ void __launch_bounds__(512, DG_SPLIT_MINB) k_split_f(FusedView fv) {
  __shared__ double smem[SplitLds<7>::A + SplitLds<7>::P];
  __shared__ double sD[64], slh[16];
  const int nb = fv.start[fv.ng];
  const int b = xcd_element(blockIdx.x, nb);
  if (b >= nb) return;
  const int gi = fused_group(fv, b);
  const int lb = b - fv.start[gi];
  switch (fv.N[gi]) {
    case 1: fused_split_group<1, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
    case 2: fused_split_group<2, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
    case 3: fused_split_group<3, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
    case 4: fused_split_group<4, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
    case 5: fused_split_group<5, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
    case 6: fused_split_group<6, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
    default: fused_split_group<7, NS, VF>(fv.v[gi], lb, smem, sD, slh); break;
  }
}

template <int N>
__device__ __forceinline__ void fused_lift_group(const BatchView &bv, int blk, double *smem, double *sDh, double *sl,
                                                 double *slh) {
  using L = LiftLds<N>;
  constexpr int NT = Sz<N>::NT, EPB = fused_epb_lift<N>();
  lift_tables<N>(bv.tab, threadIdx.x, 512, sDh, sl, slh);
  const int raw = __builtin_amdgcn_readfirstlane(threadIdx.x / NT);
  const int slot = raw < EPB ? raw : EPB - 1;
  const int t = threadIdx.x - raw * NT;
  const int item = blk * EPB + slot;
  const bool valid = raw < EPB && item < bv.total;
  const int mi = member_of(bv.first, bv.count, valid ? item : bv.total - 1);
  const Member &M = bv.m[mi];
  lift_body<N, true, LIFT_DIV, false>(M.g, M.ph, valid ? item - bv.first[mi] : 0, valid, t, M.U, nullptr, nullptr,
                                      smem + slot * (L::W + L::JA + L::WS), sDh, sl, slh);
}

__global__ void __launch_bounds__(512, DG_LIFT_MINB) k_lift_f(FusedView fv) {
  __shared__ double smem[LiftLds<7>::W + LiftLds<7>::JA + LiftLds<7>::WS];
  __shared__ double sDh[64], sl[16], slh[16];
  const int nb = fv.start[fv.ng];
  const int b = xcd_element(blockIdx.x, nb);
  if (b >= nb) return;
  const int gi = fused_group(fv, b);
  const int lb = b - fv.start[gi];
  switch (fv.N[gi]) {
    case 1: fused_lift_group<1>(fv.v[gi], lb, smem, sDh, sl, slh); break;
    case 2: fused_lift_group<2>(fv.v[gi], lb, smem, sDh, sl, slh); break;
    case 3: fused_lift_group<3>(fv.v[gi], lb, smem, sDh, sl, slh); break;
    case 4: fused_lift_group<4>(fv.v[gi], lb, smem, sDh, sl, slh); break;
    case 5: fused_lift_group<5>(fv.v[gi], lb, smem, sDh, sl, slh); break;
    case 6: fused_lift_group<6>(fv.v[gi], lb, smem, sDh, sl, slh); break;
    default: fused_lift_group<7>(fv.v[gi], lb, smem, sDh, sl, slh); break;
  }
}

int fused_epb(int N, bool lift) {
  switch (N) {
#define DG_CASE(NN) \
  case NN: return lift ? fused_epb_lift<NN>() : fused_epb_split<NN>();
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7)
#undef DG_CASE
    default: return 0;
  }
}

int launch_fused_lift(const FusedView &fv, hipStream_t st) {
  hipLaunchKernelGGL(k_lift_f, dim3(xcd_grid(fv.start[fv.ng])), dim3(512), 0, st, fv);
  DG_CHECK_LAUNCH();
  return DG_OK;
}

int launch_fused_split(const FusedView &fv, bool ns, int vf, hipStream_t st) {
  const dim3 grid(xcd_grid(fv.start[fv.ng])), block(512);
#define DG_FS(NS_, VF_) hipLaunchKernelGGL((k_split_f<NS_, VF_>), grid, block, 0, st, fv)
  if (ns) {
    if (vf == DG_VF_EC) DG_FS(true, 1);
    else if (vf == DG_VF_KEP) DG_FS(true, 0);
    else DG_FS(true, 2);
  } else {
    if (vf == DG_VF_EC) DG_FS(false, 1);
    else if (vf == DG_VF_KEP) DG_FS(false, 0);
    else DG_FS(false, 2);
  }
#undef DG_FS
  DG_CHECK_LAUNCH();
  return DG_OK;
}
#endif

#ifdef DG_ONLY_N
template int launch_prolong<DG_ONLY_N>(const Geo &, const Phys &, const double *, hipStream_t);
template int launch_lift<DG_ONLY_N>(const Geo &, const Phys &, bool, int, const double *, double *, double *,
                                    hipStream_t);
template int launch_main<DG_ONLY_N>(const Geo &, const Phys &, bool, int, int, const double *, const double *,
                                    double *, double *, double, double, double, int, hipStream_t);
template int launch_reduce<DG_ONLY_N>(const Geo &, const Phys &, int, const double *, double, double *, hipStream_t);
template int launch_mortar_lift<DG_ONLY_N>(const Geo &, const Phys &, bool, const MortarDesc *, int, const double *,
                                           hipStream_t);
template int launch_fv_face<DG_ONLY_N>(const Geo &, const Phys &, const FvGeo &, bool, const double *, hipStream_t);
template int launch_fv_volume<DG_ONLY_N>(const Geo &, const Phys &, const FvGeo &, const double *, double *, double *,
                                         double, double, double, int, hipStream_t);
template int launch_fv_switch<DG_ONLY_N>(const Geo &, const Phys &, const FvGeo &, double *, int, hipStream_t);
template int launch_fv_lists<DG_ONLY_N>(const Geo &, const FvGeo &, hipStream_t);
template int launch_mortar_flux<DG_ONLY_N>(const Geo &, const Phys &, bool, int, const MortarDesc *, int,
                                           const double *, const double *, hipStream_t);
template int launch_batch_lift<DG_ONLY_N>(const BatchView &, int, hipStream_t);
template int launch_batch_split<DG_ONLY_N>(const BatchView &, bool, int, int, hipStream_t);
#endif

}  // namespace dg
