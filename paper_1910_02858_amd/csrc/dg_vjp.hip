// Vector-Jacobian product of the split-form DGSEM operator on LGL nodes (one workgroup per
// element), for Ubar = (dL/dU)^T Utbar.
//
// The forward operator (Krais et al., FLEXI, Sec. 3.3 eq. semiDiscreteSplit with BR1 lifting,
// Sec. 3.1 eq. discreteGradient) is
//   U_t = -(1/J) acc,  acc_q = sum_dir [ sum_m 2 D_im F#(U_q, U_m) - sum_m D_im Fv_m ]
//                            + sum_faces lhat (F_face - sg F_int,q),
//   G = lift(W(U)),    W = (u, v, w, T).
// G holds the contravariant viscous fluxes Fv^dir of the lifting (LIFT_FV): the viscous flux is
// linear in the gradients, so its derivative in U needs only tau . Ja^dir, their momentum part.
// Face normals are Ja^dir at the face node of the element itself, as in the forward kernels.
// With Abar = -(1/J) Utbar (the adjoint of acc) the reverse is:
//   * each unordered pair {q, p} on a line: Fbar = 2 D_qp Abar_q + 2 D_pq Abar_p, then the
//     two-point flux's transposed Jacobian in both arguments (the partner's share goes through
//     LDS, one share per node and round, collected in a fixed order);
//   * viscous volume term: Fvbar_p = -sum_q D_qp Abar_q, then the viscous flux's transposed
//     Jacobian in U and in G;
//   * each face point: the flux enters both elements, so Fbar = lhat (Abar_master - Abar_slave),
//     and every element adds only the derivative with respect to its own trace (the neighbour's
//     Abar is read from global memory, nothing is written into another element);
//   * the lifting transposed: with H = (1/J) Gbar, Wbar = sum_dir Ja^dir . (Dhat^T H) along the
//     lines plus, on each face point, c0 Ja^dn . H (c0 = +-lhat/2) — a term that enters the
//     element's own Wbar and, the face state being the mean of both traces, the neighbour's
//     Wbar at the matching point.  The first kernel does the element's own part and leaves the
//     face terms in a face array; the second adds the neighbours' face terms and W's Jacobian
//     on the face nodes and performs the register update of the 2N scheme.
#include <hip/hip_runtime.h>

#include "dg_flux.h"
#include "dg_internal.h"

// minimum waves per SIMD of the operator's vector-Jacobian kernel (caps its registers)
#ifndef DG_VJP_MINB
#define DG_VJP_MINB 2
#endif
// stage the metric terms and kept viscous fluxes in LDS where they fit
#ifndef DG_VJP_STAGE
#define DG_VJP_STAGE 1
#endif

namespace dg {

template <int N> struct VSz {
  static constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  static constexpr int NT = ((n3 + 63) / 64) * 64;
};

template <int n> __device__ __forceinline__ int vline_node(int dn, int a, int b, int m) {
  return dn == 0 ? (m + n * (a + n * b)) : (dn == 1 ? (a + n * (m + n * b)) : (a + n * (b + n * m)));
}

// ---------------------------------------------------------------------------------- main
// GEN: the mesh has face codes (faces on any side, in any orientation, symmetry planes), and
// every neighbour value is read at the neighbour's matching face point.  The face terms
// themselves need no change: with the two copies of a face flux related by the antisymmetry of
// the surface flux (same-parity sides) or equal (opposite parities), the own-trace derivative of
// both copies is lhat (Abar_own - Abar_nb) times the outward sign of this side in every case.
// A symmetry plane has one copy (Abar_nb = 0) whose outer state is the mirrored own trace: the
// outer argument's adjoint comes back mirrored, and the viscous term keeps only the normal part
// of the own momentum flux.
template <int N, bool NS, bool GEN>
__global__ void __launch_bounds__(VSz<N>::NT, DG_VJP_MINB) k_vjp_main(Geo g, Phys ph, const double *__restrict__ U,
                                                         const double *__restrict__ G,
                                                         const double *__restrict__ Utb, double *__restrict__ Ub,
                                                         double *__restrict__ Pf, double scale, int accumulate) {
  using S = VSz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, NT = S::NT;
  constexpr int NF = NS ? 17 : 5;  // results per face point: primitive adjoint, gradient adjoint
  constexpr int NX = (NF * 6 * n2 > 9 * n3) ? NF * 6 * n2 : 9 * n3;
  __shared__ double sQ[6 * n3];  // primitive state and total enthalpy
  __shared__ double sA[5 * n3];  // Abar = -(1/J) Utbar
  // region X: first the face-point results, then H = (1/J) Gbar (9 per node, Navier-Stokes),
  // then Ja^dir of the current direction (3 per node) and the partner shares of the pair
  // rounds (6 per node: primitive adjoint and enthalpy adjoint)
  static_assert(!NS || NX >= 9 * n3, "region X holds H");
  static_assert(NX >= 9 * n3, "region X holds Ja^dir and the partner shares");
  // where the LDS allows it, all metric terms (9 per node) and the momentum part of the kept
  // viscous fluxes (9 per node) are staged once at the start, so that no later phase waits on a
  // global load after a barrier
  constexpr int NST = 9 + (NS ? 9 : 0);
  constexpr bool STAGE = DG_VJP_STAGE && (11 + NST) * n3 + NX + 2 * n * n <= 160 * 1024 / 8;
  __shared__ double sX[NX];
  __shared__ double sD[n * n], sDh[n * n];
  __shared__ double sM[STAGE ? NST * n3 : 1];  // Ja^i_d at (i*3+d)*n3, then Fv^dir_c at (9+dir*3+c)*n3
  double *sF = sX, *sH = sX, *sJ = sX, *sPA = sX + 3 * n3;
  const int e = xcd_element(blockIdx.x, g.K), t = threadIdx.x;
  if (e >= g.K) return;
  const bool act = t < n3;
  const double gamma = ph.gamma, gm1 = gamma - 1.0, g1 = gamma / gm1;
  const int vf = ph.vf;
  for (int c = t; c < n * n; c += NT) { sD[c] = g.tab->D[c]; sDh[c] = g.tab->Dh[c]; }
  const double lh = g.tab->lhp[N];  // lhat at a face node (the same value at both ends)
  const double *Ue = U + (size_t)e * 5 * n3;
  const double *Ge = G + (size_t)e * 12 * n3;
  const double *Jae = g.Ja + (size_t)e * 9 * n3;
  const double *sJe = g.sJ + (size_t)e * n3;
  // this element's metric term Ja^dir_d and momentum viscous flux Fv^dir_c at a node
  auto JA = [&](int dir, int d, int node) -> double {
    if constexpr (STAGE) return sM[(dir * 3 + d) * n3 + node];
    else return Jae[(dir * 3 + d) * n3 + node];
  };
  auto FV = [&](int dir, int c, int node) -> double {
    if constexpr (STAGE) return sM[(9 + dir * 3 + c) * n3 + node];
    else return Ge[(dir * 4 + c) * n3 + node];
  };
  if (STAGE && act) {
#pragma unroll
    for (int c = 0; c < 9; ++c) sM[c * n3 + t] = Jae[c * n3 + t];
    if (NS) {
#pragma unroll
      for (int dir = 0; dir < 3; ++dir)
#pragma unroll
        for (int c = 0; c < 3; ++c) sM[(9 + dir * 3 + c) * n3 + t] = Ge[(dir * 4 + c) * n3 + t];
    }
  }
  dgf::P q;
  if (act) {
    double Uq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = Ue[v * n3 + t];
    q = dgf::prim(Uq, gm1);
    sQ[t] = q.r; sQ[n3 + t] = q.u; sQ[2 * n3 + t] = q.v; sQ[3 * n3 + t] = q.w; sQ[4 * n3 + t] = q.p;
    sQ[5 * n3 + t] = dgf::enthalpy(q, g1);
    const double sj = sJe[t];
#pragma unroll
    for (int v = 0; v < 5; ++v) sA[v * n3 + t] = -sj * Utb[((size_t)e * 5 + v) * n3 + t];
  }
  __syncthreads();
  // ---- faces: Fbar = lhat (Abar_master - Abar_slave); own-trace derivative only.  All six
  // faces at once, one face point per thread; the results wait in LDS per face point and every
  // node collects its (up to three) face terms in direction order.
  for (int p = t; p < 6 * n2; p += NT) {
    const int s = p / n2, ab = p % n2, a = ab % n, b = ab / n, dn = s >> 1;
    const bool plus = s & 1;
    const int qo = vline_node<n>(dn, a, b, plus ? N : 0);
    int qn, nb;
    bool bnd = false, given = false, wall = false, iso = false, outflow = false;
    if constexpr (GEN) {
      const NbFace f = nbr_face<n, true>(g, e, s, a, b);
      qn = vline_node<n>(f.dn, f.a, f.b, f.plus ? N : 0);
      bnd = f.bnd;
      outflow = bnd && f.kind == DG_BC_OUTFLOW;
      given = bnd && (f.kind == DG_BC_STATE || outflow);
      iso = bnd && f.kind == DG_BC_WALL_ISOTHERMAL;
      wall = bnd && (f.kind == DG_BC_WALL || iso);
      nb = bnd ? e : g.nbr[(size_t)e * 6 + s];  // a boundary side reads nothing of a neighbour
    } else {
      qn = vline_node<n>(dn, a, b, plus ? 0 : N);
      nb = g.nbr[(size_t)e * 6 + s];
    }
    double Uw[5], Ux[5], Aw[5], Ax[5];
    const double sjn = g.sJ[(size_t)nb * n3 + qn];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Uw[v] = Ue[v * n3 + qo];
      Ux[v] = U[((size_t)nb * 5 + v) * n3 + qn];
      Aw[v] = sA[v * n3 + qo];
      Ax[v] = bnd ? 0.0 : -sjn * Utb[((size_t)nb * 5 + v) * n3 + qn];
    }
    // normal along +xi_dn scaled by s-hat: this element's Ja^dn at the face node
    const double nt[3] = {JA(dn, 0, qo), JA(dn, 1, qo), JA(dn, 2, qo)};
    const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    const double ish = 1.0 / sh;
    const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
    if (outflow) {
      // pressure outflow: the own trace's density and velocity with p_out
      Ux[0] = Uw[0]; Ux[1] = Uw[1]; Ux[2] = Uw[2]; Ux[3] = Uw[3];
      Ux[4] = ph.pout / gm1 + 0.5 * (Uw[1] * Uw[1] + Uw[2] * Uw[2] + Uw[3] * Uw[3]) / Uw[0];
    } else if (given) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Ux[v] = ph.ub[v];  // given outer state, independent of U
    } else if (wall) {
      // no-slip wall: the outer state is the own trace with the velocity reversed
      Ux[0] = Uw[0]; Ux[1] = -Uw[1]; Ux[2] = -Uw[2]; Ux[3] = -Uw[3]; Ux[4] = Uw[4];
    } else if (bnd) {
      // symmetry plane: the outer state is the mirrored own trace
      const double mn = 2.0 * (Uw[1] * nh[0] + Uw[2] * nh[1] + Uw[3] * nh[2]);
      Ux[0] = Uw[0]; Ux[4] = Uw[4];
      Ux[1] = Uw[1] - mn * nh[0]; Ux[2] = Uw[2] - mn * nh[1]; Ux[3] = Uw[3] - mn * nh[2];
    }
    double Fb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Fb[v] = lh * (plus ? (Aw[v] - Ax[v]) : (Ax[v] - Aw[v]));
    const double *UM = plus ? Uw : Ux, *US = plus ? Ux : Uw;
    const dgf::P PM = dgf::prim(UM, gm1), PS = dgf::prim(US, gm1);
    double Fbs[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Fbs[v] = Fb[v] * sh;
    // the primitive adjoint of the own trace (the final (dP/dU)^T map of the node applies to it)
    dgf::PA aM = dgf::zero_pa(), aS = dgf::zero_pa();
    dgf::riemann_adj_prim(ph.rs, vf, PM, PS, UM, US, nh, gamma, Fbs, aM, aS);
    dgf::PA pc = plus ? aM : aS;
    const dgf::P Po = plus ? PM : PS;
    if (outflow) {
      // the outer argument's density and velocity are the own trace's, its pressure is fixed
      const dgf::PA ao = plus ? aS : aM;
      pc.r += ao.r; pc.u += ao.u; pc.v += ao.v; pc.w += ao.w;
    } else if (wall) {
      // the outer argument is the own trace with the velocity reversed
      const dgf::PA ao = plus ? aS : aM;
      pc.r += ao.r; pc.p += ao.p;
      pc.u -= ao.u; pc.v -= ao.v; pc.w -= ao.w;
    } else if (bnd && !given) {
      // the outer argument is the mirror image of the own trace: its adjoint comes back mirrored
      const dgf::PA ao = plus ? aS : aM;
      const double an = 2.0 * (ao.u * nh[0] + ao.v * nh[1] + ao.w * nh[2]);
      pc.r += ao.r; pc.p += ao.p;
      pc.u += ao.u - an * nh[0]; pc.v += ao.v - an * nh[1]; pc.w += ao.w - an * nh[2];
    }
    if (NS) {
      // F contains -1/2 Fv(U_own, G_own) . nt; its momentum part along the face's direction is
      // the contravariant viscous flux of that direction from the lifting (G holds those)
      double gbo[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) gbo[c] = 0.0;
      const double tn[3] = {FV(dn, 0, qo), FV(dn, 1, qo), FV(dn, 2, qo)};
      double Fvb[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Fvb[v] = -0.5 * Fb[v];
      if (given) {
        // given outer state: the term is -g, the whole own flux
#pragma unroll
        for (int v = 0; v < 5; ++v) Fvb[v] = -Fb[v];
      } else if (iso) {
        // isothermal wall: the terms are -g_m for the momentum and -(g_E - g_m . u) for the
        // energy, with u this node's velocity
        Fvb[0] = 0.0; Fvb[4] = -Fb[4];
        Fvb[1] = -Fb[1] + Fb[4] * Po.u; Fvb[2] = -Fb[2] + Fb[4] * Po.v; Fvb[3] = -Fb[3] + Fb[4] * Po.w;
        pc.u += Fb[4] * tn[0]; pc.v += Fb[4] * tn[1]; pc.w += Fb[4] * tn[2];
      } else if (wall) {
        // no-slip wall: the term is -g for the momentum, nothing for the energy
        Fvb[0] = 0.0; Fvb[4] = 0.0;
        Fvb[1] = -Fb[1]; Fvb[2] = -Fb[2]; Fvb[3] = -Fb[3];
      } else if (bnd) {
        // symmetry plane: the term is -(g.nh) nh of the own momentum flux g, no energy part
        const double fn_ = Fb[1] * nh[0] + Fb[2] * nh[1] + Fb[3] * nh[2];
        Fvb[0] = 0.0; Fvb[4] = 0.0;
        Fvb[1] = -fn_ * nh[0]; Fvb[2] = -fn_ * nh[1]; Fvb[3] = -fn_ * nh[2];
      }
      dgf::visc_flux_adj_tn(Po, tn, ph.mu, ph.kappa, nt, Fvb, pc, gbo);
#pragma unroll
      for (int c = 0; c < 12; ++c) sF[(5 + c) * 6 * n2 + p] = gbo[c];
    }
    sF[0 * 6 * n2 + p] = pc.r;
    sF[1 * 6 * n2 + p] = pc.u;
    sF[2 * 6 * n2 + p] = pc.v;
    sF[3 * 6 * n2 + p] = pc.w;
    sF[4 * 6 * n2 + p] = pc.p;
  }
  __syncthreads();
  dgf::PA pa = dgf::zero_pa();
  double gbf[12];  // gradient adjoint of the face terms at this node
#pragma unroll
  for (int c = 0; c < 12; ++c) gbf[c] = 0.0;
  const int id3[3] = {t % n, (t / n) % n, t / n2};
  if (act) {
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
      const int id = id3[dir];
      if (id != 0 && id != N) continue;
      const int s = 2 * dir + (id == N ? 1 : 0);
      const int a = dir == 0 ? id3[1] : id3[0], b = dir == 2 ? id3[1] : id3[2];
      const int p = s * n2 + a + n * b;
      pa.r += sF[p]; pa.u += sF[6 * n2 + p]; pa.v += sF[2 * 6 * n2 + p]; pa.w += sF[3 * 6 * n2 + p];
      pa.p += sF[4 * 6 * n2 + p];
      if (NS) {
#pragma unroll
        for (int c = 0; c < 12; ++c) gbf[c] += sF[(5 + c) * 6 * n2 + p];
      }
    }
  }
  double cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // ---- interior convective flux F_int = Fc . Ja on the faces through this node
  if (act) {
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
      const int id = id3[dir];
      if (id != 0 && id != N) continue;
      const double sg = (id == N) ? 1.0 : -1.0;
      const double nv[3] = {JA(dir, 0, t), JA(dir, 1, t), JA(dir, 2, t)};
      double Fib[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Fib[v] = -lh * sg * sA[v * n3 + t];
      dgf::euler_flux_adj(q, nv, g1, Fib, pa);
    }
  }
  // ---- viscous part, all directions before the pair rounds: acc_m -= sum_i D_mi Fv_i gives
  // Fvbar_i = -sum_m D_mi Abar_m; the interior face term -F_int contributes +lhat sg Abar_i.
  // The gradient adjoint of this node is final afterwards.
  double hg[12];  // H = (1/J) scale Gbar of this node
  if (NS && act) {
    double gbo[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) gbo[c] = gbf[c];
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
      const int id = id3[dir];
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int base = t - id * str;
      double fvb[4] = {0.0, 0.0, 0.0, 0.0};
      if (id == 0 || id == N) {
        const double sg = (id == N) ? 1.0 : -1.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) fvb[c] -= -lh * sg * sA[(1 + c) * n3 + t];
      }
      for (int m = 0; m < n; ++m) {
        const int qm = base + m * str;
        const double Dmi = sD[m * n + id];
#pragma unroll
        for (int c = 0; c < 4; ++c) fvb[c] -= Dmi * sA[(1 + c) * n3 + qm];
      }
      const double nv[3] = {JA(dir, 0, t), JA(dir, 1, t), JA(dir, 2, t)};
      const double Fvb[5] = {0.0, fvb[0], fvb[1], fvb[2], fvb[3]};
      const double tn[3] = {FV(dir, 0, t), FV(dir, 1, t), FV(dir, 2, t)};
      dgf::visc_flux_adj_tn(q, tn, ph.mu, ph.kappa, nv, Fvb, pa, gbo);
    }
    const double sj = sJe[t];
#pragma unroll
    for (int c = 0; c < 12; ++c) hg[c] = sj * (scale * gbo[c]);
  }
  // ---- lifting transposed, own part (volume and own face terms); the face terms also go to
  // the face array for the neighbours.  The velocity block of H is symmetric, H_dc = H_cd (every
  // viscous transpose adds mu (T_cd + T_dc) - 2/3 mu tr(T) delta_cd), so region X holds its six
  // distinct entries (00, 11, 22, 01, 02, 12) and the three temperature entries, 9 per node.
  dgf::PA pl = dgf::zero_pa();
  if (NS) {
    __syncthreads();  // every node has collected its face results from region X
    if (act) {
      const double h9[9] = {hg[0], hg[5], hg[10], hg[1], hg[2], hg[6], hg[3], hg[7], hg[11]};
#pragma unroll
      for (int c = 0; c < 9; ++c) sH[c * n3 + t] = h9[c];
    }
    __syncthreads();
    if (act) {
      double Wb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int dir = 0; dir < 3; ++dir) {
        const int id = id3[dir];
        const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
        const int base = t - id * str;
        const double nv[3] = {JA(dir, 0, t), JA(dir, 1, t), JA(dir, 2, t)};
        double hs[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) hs[c] = 0.0;
#pragma unroll 1
        for (int i = 0; i < n; ++i) {
          const int qi = base + i * str;
          const double Dh = sDh[i * n + id];
#pragma unroll
          for (int c = 0; c < 9; ++c) hs[c] += Dh * sH[c * n3 + qi];
        }
        Wb[0] += nv[0] * hs[0] + nv[1] * hs[3] + nv[2] * hs[4];
        Wb[1] += nv[0] * hs[3] + nv[1] * hs[1] + nv[2] * hs[5];
        Wb[2] += nv[0] * hs[4] + nv[1] * hs[5] + nv[2] * hs[2];
        Wb[3] += nv[0] * hs[6] + nv[1] * hs[7] + nv[2] * hs[8];
        if (id == 0 || id == N) {
          const int sd = (id == N) ? 1 : 0;
          const int s = 2 * dir + sd;
          const int a = dir == 0 ? id3[1] : id3[0], b = dir == 2 ? id3[1] : id3[2];
          const double c0 = (sd ? 0.5 : -0.5) * lh;
          double *pf = Pf + ((size_t)e * 6 + s) * 4 * n2 + a + n * b;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double f = c0 * (nv[0] * hg[v] + nv[1] * hg[4 + v] + nv[2] * hg[8 + v]);
            Wb[v] += f;
            pf[v * n2] = f;
          }
        }
      }
      dgf::lift_vars_adj(q, ph.R, Wb, pl);
    }
  }
  // ---- volume: pairs and diagonal, direction by direction.  With the KEP flux the adjoint of
  // this node's total enthalpy is summed over all pairs and mapped once at the end.
  const double Ht = act ? sQ[5 * n3 + t] : 0.0;
  double Htb = 0.0;
  // the epilogue's loads are issued before the rounds
  double *Ube = Ub + (size_t)e * 5 * n3;
  double ub0[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (act && accumulate) {
#pragma unroll
    for (int v = 0; v < 5; ++v) ub0[v] = Ube[v * n3 + t];
  }
  for (int dir = 0; dir < 3; ++dir) {
    double nvo[3] = {0.0, 0.0, 0.0};
    const double *sJd = sJ;
    if constexpr (STAGE) {
      // the metric terms are in LDS already; every exchange round ends with a barrier, so
      // only the first direction needs one (after the last reads of region X)
      if (dir == 0) __syncthreads();
      sJd = sM + dir * 3 * n3;
      if (act) { nvo[0] = sJd[t]; nvo[1] = sJd[n3 + t]; nvo[2] = sJd[2 * n3 + t]; }
    } else {
      __syncthreads();
      if (act) {
        nvo[0] = Jae[(dir * 3) * n3 + t]; nvo[1] = Jae[(dir * 3 + 1) * n3 + t]; nvo[2] = Jae[(dir * 3 + 2) * n3 + t];
        sJ[t] = nvo[0]; sJ[n3 + t] = nvo[1]; sJ[2 * n3 + t] = nvo[2];
      }
      __syncthreads();
    }
    {
      const int id = act ? id3[dir] : 0;
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int base = t - id * str;
      double Ao[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Ao[v] = act ? sA[v * n3 + t] : 0.0;
#pragma unroll 1
      for (int sft = 1; sft <= n / 2; ++sft) {
        if (act) {
          const bool half = (2 * sft == n);  // the pair at distance n/2 is met from both ends
          int jp = id + sft;
          if (jp >= n) jp -= n;
          const int qp = base + jp * str;
          dgf::P r;
          r.r = sQ[qp]; r.u = sQ[n3 + qp]; r.v = sQ[2 * n3 + qp]; r.w = sQ[3 * n3 + qp]; r.p = sQ[4 * n3 + qp];
          const double Hr = sQ[5 * n3 + qp];  // the partner's total enthalpy
          const double nm[3] = {0.5 * (nvo[0] + sJd[qp]), 0.5 * (nvo[1] + sJd[n3 + qp]),
                                0.5 * (nvo[2] + sJd[2 * n3 + qp])};
          const double Dij2 = 2.0 * sD[id * n + jp], Dji2 = 2.0 * sD[jp * n + id];
          double Fb[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) Fb[v] = Dij2 * Ao[v] + (half ? 0.0 : Dji2 * sA[v * n3 + qp]);
          dgf::PA pr = dgf::zero_pa();
          double Hrb = 0.0;
          if (vf == 0) {
            dgf::kep_flux_adj_h(q, r, Ht, Hr, nm, Fb, pa, pr, Htb, Hrb);
          } else {
            r.ir = 1.0 / r.r;  // the central flux's enthalpies need it
            dgf::pair_flux_adj(vf, q, r, nm, g1, Fb, pa, pr);
          }
          // every node receives exactly one partner share per round
          sPA[qp] = pr.r; sPA[n3 + qp] = pr.u; sPA[2 * n3 + qp] = pr.v; sPA[3 * n3 + qp] = pr.w;
          sPA[4 * n3 + qp] = pr.p; sPA[5 * n3 + qp] = Hrb;
        }
        __syncthreads();
        if (act) {
          pa.r += sPA[t]; pa.u += sPA[n3 + t]; pa.v += sPA[2 * n3 + t]; pa.w += sPA[3 * n3 + t];
          pa.p += sPA[4 * n3 + t]; Htb += sPA[5 * n3 + t];
        }
        __syncthreads();
      }
      if (!act) continue;
      const double Dii = sD[id * n + id];
      if (Dii != 0.0) {
        double Fb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) Fb[v] = 2.0 * Dii * Ao[v];
        dgf::euler_flux_adj(q, nvo, g1, Fb, pa);
      }
    }
  }
  if (act) {
    dgf::enthalpy_adj(q, g1, Htb, pa);
    dgf::PA pt;
    pt.r = fma(scale, pa.r, pl.r); pt.u = fma(scale, pa.u, pl.u); pt.v = fma(scale, pa.v, pl.v);
    pt.w = fma(scale, pa.w, pl.w); pt.p = fma(scale, pa.p, pl.p);
    dgf::cons_adj(q, gm1, pt, cb);
#pragma unroll
    for (int v = 0; v < 5; ++v) Ube[v * n3 + t] = ub0[v] + cb[v];
  }
}

// ---------------------------------------------------------------------------------- faces
// Completes Ubar on the face nodes with the neighbours' face terms of the transposed lifting
// (Wbar, then W's Jacobian at the node's state).  With upd != 0 the register of the 2N scheme
// is updated from the final Ubar of every node, Rb = ra Rb + rb Ubar (each node is read and
// written by its own thread only).
template <int N, bool GEN>
__global__ void __launch_bounds__(VSz<N>::NT) k_vjp_face(Geo g, Phys ph, const double *__restrict__ U,
                                                         const double *__restrict__ Pf, double *__restrict__ Ub,
                                                         double *__restrict__ Rb, double ra, double rb, int upd) {
  using S = VSz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
  const int e = xcd_element(blockIdx.x, g.K), t = threadIdx.x;
  if (e >= g.K || t >= n3) return;
  const int id3[3] = {t % n, (t / n) % n, t / n2};
  double Wb[4] = {0.0, 0.0, 0.0, 0.0};
  double tout = 0.0;  // adjoint of outflow sides' outer temperature p_out / (rho R)
  bool face = false;
#pragma unroll
  for (int dir = 0; dir < 3; ++dir) {
    const int id = id3[dir];
    if (id != 0 && id != N) continue;
    const int s = 2 * dir + (id == N ? 1 : 0);
    const int a = dir == 0 ? id3[1] : id3[0], b = dir == 2 ? id3[1] : id3[2];
    // the neighbour's term at its matching face point (structured: side s ^ 1, same index)
    if constexpr (GEN) {
      const NbFace f = nbr_face<n, true>(g, e, s, a, b);
      if (f.bnd && f.kind == DG_BC_OUTFLOW) {
        // pressure outflow: the outer W is (u, v, w, p_out / (rho R)) of this node
        const double *pf = Pf + ((size_t)e * 6 + s) * 4 * n2 + a + n * b;
        Wb[0] += pf[0]; Wb[1] += pf[n2]; Wb[2] += pf[2 * n2];
        tout += pf[3 * n2];
      } else if (f.bnd && f.kind == DG_BC_STATE) {
        // given outer state: W* depends on this element's W only through its own half
      } else if (f.bnd && f.kind == DG_BC_WALL) {
        // no-slip wall: the outer W is the own W with the velocity reversed
        const double *pf = Pf + ((size_t)e * 6 + s) * 4 * n2 + a + n * b;
        Wb[0] -= pf[0]; Wb[1] -= pf[n2]; Wb[2] -= pf[2 * n2];
        Wb[3] += pf[3 * n2];
      } else if (f.bnd && f.kind == DG_BC_WALL_ISOTHERMAL) {
        // isothermal wall: the outer W is (-u, -v, -w, 2 T_w - T)
        const double *pf = Pf + ((size_t)e * 6 + s) * 4 * n2 + a + n * b;
        Wb[0] -= pf[0]; Wb[1] -= pf[n2]; Wb[2] -= pf[2 * n2];
        Wb[3] -= pf[3 * n2];
      } else if (f.bnd) {
        // symmetry plane: the outer W is the mirrored own W, so the element's own face term
        // comes back with its velocity part mirrored
        const double *pf = Pf + ((size_t)e * 6 + s) * 4 * n2 + a + n * b;
        const double *fnp = g.fn + ((size_t)e * 6 + s) * 3 * n2 + a + n * b;
        const double nt[3] = {fnp[0], fnp[n2], fnp[2 * n2]};
        const double il = 1.0 / sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
        const double nh[3] = {nt[0] * il, nt[1] * il, nt[2] * il};
        const double w0 = pf[0], w1 = pf[n2], w2 = pf[2 * n2];
        const double wn = 2.0 * (w0 * nh[0] + w1 * nh[1] + w2 * nh[2]);
        Wb[0] += w0 - wn * nh[0]; Wb[1] += w1 - wn * nh[1]; Wb[2] += w2 - wn * nh[2];
        Wb[3] += pf[3 * n2];
      } else {
        const int nb = g.nbr[(size_t)e * 6 + s];
        const double *pf = Pf + ((size_t)nb * 6 + 2 * f.dn + (f.plus ? 1 : 0)) * 4 * n2 + f.a + n * f.b;
#pragma unroll
        for (int v = 0; v < 4; ++v) Wb[v] += pf[v * n2];
      }
    } else {
      const int nb = g.nbr[(size_t)e * 6 + s];
      const double *pf = Pf + ((size_t)nb * 6 + (s ^ 1)) * 4 * n2 + a + n * b;
#pragma unroll
      for (int v = 0; v < 4; ++v) Wb[v] += pf[v * n2];
    }
    face = true;
  }
  if (!face && !upd) return;
  double *Ube = Ub + (size_t)e * 5 * n3 + t;
  double u[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = Ube[v * n3];
  if (face) {
    double Uq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uq[v] = U[((size_t)e * 5 + v) * n3 + t];
    const dgf::P q = dgf::prim(Uq, ph.gamma - 1.0);
    dgf::PA pa = dgf::zero_pa();
    dgf::lift_vars_adj(q, ph.R, Wb, pa);
    pa.r -= tout * ph.pout * q.ir * q.ir / ph.R;
    double cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    dgf::cons_adj(q, ph.gamma - 1.0, pa, cb);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] += cb[v];
      Ube[v * n3] = u[v];
    }
  }
  if (upd) {
    double *r = Rb + (size_t)e * 5 * n3 + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v * n3] = ra * r[v * n3] + rb * u[v];
  }
}

// ---------------------------------------------------------------------------------- weak form
// Reverse of the weak form (Sec. 3.1, eq. semiDiscreteWeak) for the Euler equations on LG or LGL
// nodes.  The forward operator is
//   U_t,i = -(1/J_i) [ sum_dir sum_m Dhat_{id m} F^dir(U_m) + sum_faces lhat_face(i) f*_face ],
// with F^dir the contravariant Euler flux along Ja^dir_m at node m, f*_face the outward numerical
// flux times the surface element at the face point of node i's line (one value per face, the
// master's, entering the slave negated), evaluated from the two sides' traces prolonged with
// l(+-1) (LG) or read at the face nodes (LGL).  With Abar = -(1/J) Utbar:
//   * volume: Gbar^dir_m = sum_i Dhat_{id_i m} Abar_i along the line, then the flux Jacobian's
//     transpose at node m;
//   * faces: fbar = sg (sum_i lhat(i) Abar_i on this element's line - the same on the
//     neighbour's), the Riemann solver's transposed Jacobian in this element's own trace only
//     (the neighbour does the same for its trace), then the prolongation transposed onto the
//     line (LG) or the face node (LGL); a boundary side's outer state is a function of the own
//     trace and its adjoint comes back through that map.
// Nothing is written into another element.
template <int N, bool LGL, bool GEN>
__global__ void __launch_bounds__(VSz<N>::NT) k_vjp_weak(Geo g, Phys ph, const double *__restrict__ U,
                                                         const double *__restrict__ Utb, double *__restrict__ Ub,
                                                         double scale, int accumulate) {
  using S = VSz<N>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, NT = S::NT;
  __shared__ double sA[5 * n3];   // Abar = -(1/J) Utbar
  __shared__ double sU[5 * n3];   // the element's state
  __shared__ double sT[30 * n2];  // conservative adjoint of the own trace at every face point
  __shared__ double sDh[n * n], sl[2 * n], slh[2 * n];
  const int e = xcd_element(blockIdx.x, g.K), t = threadIdx.x;
  if (e >= g.K) return;
  const bool act = t < n3;
  const double gamma = ph.gamma, gm1 = gamma - 1.0, g1 = gamma / gm1;
  const Tab *tb = g.tab;
  for (int c = t; c < n * n; c += NT) sDh[c] = tb->Dh[c];
  if (t < n) {
    sl[t] = tb->lm[t]; sl[n + t] = tb->lp[t];
    slh[t] = tb->lhm[t]; slh[n + t] = tb->lhp[t];
  }
  const double *Ue = U + (size_t)e * 5 * n3;
  double Uo[5];
  if (act) {
    const double sj = g.sJ[(size_t)e * n3 + t];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Uo[v] = Ue[v * n3 + t];
      sU[v * n3 + t] = Uo[v];
      sA[v * n3 + t] = -sj * Utb[((size_t)e * 5 + v) * n3 + t];
    }
  }
  __syncthreads();
  for (int p = t; p < 6 * n2; p += NT) {
    const int s = p / n2, ab = p - s * n2, a = ab % n, b = ab / n, dn = s >> 1;
    const bool plus = s & 1;
    const NbFace f = nbr_face<n, GEN>(g, e, s, a, b);
    const bool bnd = GEN && f.bnd;
    const int nb = bnd ? e : g.nbr[(size_t)e * 6 + s];
    const int ns = GEN ? 2 * f.dn + (f.plus ? 1 : 0) : (s ^ 1);
    const bool nplus = ns & 1;
    // own and neighbour traces, and the weights of both sides' lines in the face adjoint
    double Uw[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, Ux[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double Ao[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, An[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double *lo = sl + (plus ? n : 0), *ln = sl + (nplus ? n : 0);
    const double *lho = slh + (plus ? n : 0), *lhn = slh + (nplus ? n : 0);
    const double *Un = U + (size_t)nb * 5 * n3;
    const double *Utn = Utb + (size_t)nb * 5 * n3;
    const double *sJn = g.sJ + (size_t)nb * n3;
#pragma unroll 1
    for (int m = 0; m < n; ++m) {
      if (LGL && m != (plus ? N : 0) && m != (nplus ? N : 0)) continue;
      const int q = vline_node<n>(dn, a, b, m);
      if (!LGL || m == (plus ? N : 0)) {
        const double wo = LGL ? 1.0 : lo[m], who = lho[m];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          Uw[v] += wo * sU[v * n3 + q];
          Ao[v] += who * sA[v * n3 + q];
        }
      }
      if (!bnd && (!LGL || m == (nplus ? N : 0))) {
        const int qn = vline_node<n>(f.dn, f.a, f.b, m);
        const double wn = LGL ? 1.0 : ln[m], whn = lhn[m];
        const double sjn = sJn[qn];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          Ux[v] += wn * Un[v * n3 + qn];
          An[v] += whn * (-sjn * Utn[v * n3 + qn]);
        }
      }
    }
    const double *fnp = g.fn + ((size_t)e * 6 + s) * 3 * n2 + ab;
    const bool mst = GEN ? f.master : plus;
    const double sg = mst ? 1.0 : -1.0;
    const double nt[3] = {sg * fnp[0], sg * fnp[n2], sg * fnp[2 * n2]};
    const double sh = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    const double ish = 1.0 / sh;
    const double nh[3] = {nt[0] * ish, nt[1] * ish, nt[2] * ish};
    const bool outflow = bnd && f.kind == DG_BC_OUTFLOW;
    const bool given = bnd && (f.kind == DG_BC_STATE || outflow);
    const bool wall = bnd && (f.kind == DG_BC_WALL || f.kind == DG_BC_WALL_ISOTHERMAL);
    if (outflow) {
      Ux[0] = Uw[0]; Ux[1] = Uw[1]; Ux[2] = Uw[2]; Ux[3] = Uw[3];
      Ux[4] = ph.pout / gm1 + 0.5 * (Uw[1] * Uw[1] + Uw[2] * Uw[2] + Uw[3] * Uw[3]) / Uw[0];
    } else if (given) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Ux[v] = ph.ub[v];
    } else if (wall) {
      Ux[0] = Uw[0]; Ux[1] = -Uw[1]; Ux[2] = -Uw[2]; Ux[3] = -Uw[3]; Ux[4] = Uw[4];
    } else if (bnd) {
      const double mn = 2.0 * (Uw[1] * nh[0] + Uw[2] * nh[1] + Uw[3] * nh[2]);
      Ux[0] = Uw[0]; Ux[4] = Uw[4];
      Ux[1] = Uw[1] - mn * nh[0]; Ux[2] = Uw[2] - mn * nh[1]; Ux[3] = Uw[3] - mn * nh[2];
    }
    // adjoint of the master's flux value (times s-hat): this element enters it with sign sg, the
    // neighbour with -sg
    double Fb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Fb[v] = sg * sh * (Ao[v] - An[v]);
    const double *UM = mst ? Uw : Ux, *US = mst ? Ux : Uw;
    const dgf::P PM = dgf::prim(UM, gm1), PS = dgf::prim(US, gm1);
    double bM[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, bS[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    dgf::riemann_adj(ph.rs, ph.vf, PM, PS, UM, US, nh, gamma, Fb, bM, bS);
    double bw[5], bx[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) { bw[v] = mst ? bM[v] : bS[v]; bx[v] = mst ? bS[v] : bM[v]; }
    if (outflow) {
      // outer state (rho, m, p_out/(gamma-1) + |m|^2/(2 rho)) of the own trace
      const double ir = 1.0 / Uw[0];
      const double k2 = (Uw[1] * Uw[1] + Uw[2] * Uw[2] + Uw[3] * Uw[3]) * ir * ir;
      bw[0] += bx[0] - 0.5 * k2 * bx[4];
      bw[1] += bx[1] + Uw[1] * ir * bx[4];
      bw[2] += bx[2] + Uw[2] * ir * bx[4];
      bw[3] += bx[3] + Uw[3] * ir * bx[4];
    } else if (wall) {
      bw[0] += bx[0]; bw[1] -= bx[1]; bw[2] -= bx[2]; bw[3] -= bx[3]; bw[4] += bx[4];
    } else if (bnd && !given) {
      // mirror image: the reflection is its own transpose
      const double mn = 2.0 * (bx[1] * nh[0] + bx[2] * nh[1] + bx[3] * nh[2]);
      bw[0] += bx[0]; bw[4] += bx[4];
      bw[1] += bx[1] - mn * nh[0]; bw[2] += bx[2] - mn * nh[1]; bw[3] += bx[3] - mn * nh[2];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sT[(s * 5 + v) * n2 + ab] = bw[v];
  }
  __syncthreads();
  if (act) {
    const int id3[3] = {t % n, (t / n) % n, t / n2};
    const dgf::P q = dgf::prim(Uo, gm1);
    dgf::PA pa = dgf::zero_pa();
    double ub[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double *Jae = g.Ja + (size_t)e * 9 * n3;
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
      const int id = id3[dir];
      const int str = dir == 0 ? 1 : (dir == 1 ? n : n2);
      const int base = t - id * str;
      // volume: Gbar = sum over the line of Dhat_{id_i, id} Abar_i
      double Gb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int m = 0; m < n; ++m) {
        const double d = sDh[m * n + id];
#pragma unroll
        for (int v = 0; v < 5; ++v) Gb[v] += d * sA[v * n3 + base + m * str];
      }
      const double nv[3] = {Jae[(dir * 3) * n3 + t], Jae[(dir * 3 + 1) * n3 + t], Jae[(dir * 3 + 2) * n3 + t]};
      dgf::euler_flux_adj(q, nv, g1, Gb, pa);
      // faces of this direction: the own trace's adjoint prolonged back onto this node
      const int fa = dir == 0 ? id3[1] : id3[0], fb = dir == 2 ? id3[1] : id3[2];
      const int ab = fa + n * fb;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int s = 2 * dir + sd;
        double w;
        if (LGL) w = (id == (sd ? N : 0)) ? 1.0 : 0.0;
        else w = sl[(sd ? n : 0) + id];
        if (w == 0.0) continue;
#pragma unroll
        for (int v = 0; v < 5; ++v) ub[v] += w * sT[(s * 5 + v) * n2 + ab];
      }
    }
    dgf::cons_adj(q, gm1, pa, ub);
    double *Ube = Ub + (size_t)e * 5 * n3;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double r = scale * ub[v];
      Ube[v * n3 + t] = accumulate ? Ube[v * n3 + t] + r : r;
    }
  }
}

// ---------------------------------------------------------------------------------- launcher
template <int N>
int launch_vjp(const Geo &g, const Phys &ph, int eqn, int form, bool lgl, const double *U, const double *G, double *Pf,
               const double *Ubar_t, double *Ubar, double scale, int accumulate, double *Rb, double ra, double rb,
               hipStream_t st) {
  const bool gen = g.fc != nullptr;
  if (form == DG_FORM_WEAK) {
    if (eqn != DG_EULER) return DG_ERR_UNSUPPORTED;
    const dim3 grid(xcd_grid(g.K)), block(VSz<N>::NT);
    if (lgl && gen) hipLaunchKernelGGL((k_vjp_weak<N, true, true>), grid, block, 0, st, g, ph, U, Ubar_t, Ubar, scale, accumulate);
    else if (lgl) hipLaunchKernelGGL((k_vjp_weak<N, true, false>), grid, block, 0, st, g, ph, U, Ubar_t, Ubar, scale, accumulate);
    else if (gen) hipLaunchKernelGGL((k_vjp_weak<N, false, true>), grid, block, 0, st, g, ph, U, Ubar_t, Ubar, scale, accumulate);
    else hipLaunchKernelGGL((k_vjp_weak<N, false, false>), grid, block, 0, st, g, ph, U, Ubar_t, Ubar, scale, accumulate);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
  }
  if (form != DG_FORM_SPLIT) return DG_ERR_UNSUPPORTED;
  {
  dim3 grid(xcd_grid(g.K)), block(VSz<N>::NT);
  if (eqn == DG_NAVIER_STOKES) {
    if (gen)
      hipLaunchKernelGGL((k_vjp_main<N, true, true>), grid, block, 0, st, g, ph, U, G, Ubar_t, Ubar, Pf, scale,
                         accumulate);
    else
      hipLaunchKernelGGL((k_vjp_main<N, true, false>), grid, block, 0, st, g, ph, U, G, Ubar_t, Ubar, Pf, scale,
                         accumulate);
    if (hipGetLastError() != hipSuccess) return DG_ERR_HIP;
    if (gen)
      hipLaunchKernelGGL((k_vjp_face<N, true>), grid, block, 0, st, g, ph, U, Pf, Ubar, Rb, ra, rb, Rb ? 1 : 0);
    else
      hipLaunchKernelGGL((k_vjp_face<N, false>), grid, block, 0, st, g, ph, U, Pf, Ubar, Rb, ra, rb, Rb ? 1 : 0);
  } else {
    if (gen)
      hipLaunchKernelGGL((k_vjp_main<N, false, true>), grid, block, 0, st, g, ph, U, G, Ubar_t, Ubar, Pf, scale,
                         accumulate);
    else
      hipLaunchKernelGGL((k_vjp_main<N, false, false>), grid, block, 0, st, g, ph, U, G, Ubar_t, Ubar, Pf, scale,
                         accumulate);
  }
  if (hipGetLastError() != hipSuccess) return DG_ERR_HIP;
  return DG_OK;
  }
}

#ifdef DG_ONLY_N
template int launch_vjp<DG_ONLY_N>(const Geo &, const Phys &, int, int, bool, const double *, const double *, double *,
                                   const double *, double *, double, int, double *, double, double, hipStream_t);
#endif

}  // namespace dg
