// Internal declarations shared by the host setup (dg_host.cpp) and the HIP kernels
// (dg_kernels.hip) of libdgsem.  Not part of the public ABI (include/dgsem.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dgsem.h"

namespace dg {

constexpr int NMAX = 8;  // highest supported polynomial degree

// 1D operators of one node set, packed for the handle's degree (n = N+1):
// D[r*n+s] = l_s'(x_r); Dh[i*n+j] = -(w_j/w_i) D[j*n+i]; l(+-1); lhat(+-1) = l(+-1)/w.
struct Tab {
  double D[(NMAX + 1) * (NMAX + 1)];
  double Dh[(NMAX + 1) * (NMAX + 1)];
  // strong form on LG nodes (eq. semiDiscreteStrong): the volume derivative together with the
  // interior flux interpolated to both faces of the line and lifted back,
  // Ds[i*n+m] = D[i*n+m] - lhat_i(+1) l_m(+1) + lhat_i(-1) l_m(-1), one contraction per line
  double Ds[(NMAX + 1) * (NMAX + 1)];
  double lm[NMAX + 1], lp[NMAX + 1], lhm[NMAX + 1], lhp[NMAX + 1], w[NMAX + 1];
  // mortar operators (Sec. 3.2): interpolation of the big side to its lower / upper half,
  // IL[i*n+m] = l_m((x_i - 1)/2), IU likewise with +1, and the projection back,
  // PL[i*n+a] = l_i((x_a - 1)/2) w_a / w_i, PU likewise
  double IL[(NMAX + 1) * (NMAX + 1)], IU[(NMAX + 1) * (NMAX + 1)];
  double PL[(NMAX + 1) * (NMAX + 1)], PU[(NMAX + 1) * (NMAX + 1)];
};

// Face code kind of a side of a non-conforming face (bits 0-2 of a boundary-flagged code): its
// flux and lifting terms come from the mortar face arrays (Geo::mflux, Geo::mlift).
constexpr int FACE_MORTAR = 7;

// One non-conforming face (Sec. 3.2): the big side and its 2 (types 1, 2) or 4 (type 3) small
// sides, each with its face-array slot.
struct MortarDesc {
  int eb, sb, type, slot;          // big element, side, mortar type 1..3, slot of the big side
  int es[4], ss[4], o[4], sl[4];   // small sides by position: element, side, orientation code, slot
};

// Device-resident geometry of one mesh.
struct Geo {
  const double *Ja;   // [K][9][n3]: Ja^i_d at (i*3+d)
  const double *sJ;   // [K][n3]: 1/J
  const double *fn;   // [K][6][3][n2]: outward scaled normal of each side (the master's, negated on slaves)
  const int32_t *nbr; // [K][6]
  // [K][6] face code of each side, NULL on a structured mesh (every neighbour across side s
  // meets it on side s^1 in the same orientation): bits 0-2 the neighbour's side, bits 3-5
  // the orientation (bit 3+2 swaps the face indices (a,b), then bit 3+0 reverses the first and
  // bit 3+1 the second), bit 6 set where this side is the face's master
  const uint8_t *fc;
  const Tab *tab;
  int K;
  // non-conforming faces (NULL without): slot of every side [K][6] (-1 for conforming sides), and
  // per slot the side's outward numerical flux times the surface element minus the BR1 viscous
  // mean, mflux[slot][5][n^2], its lifting surface term W* s n_d, mlift[slot][d*4+c][n^2], and the
  // lifted gradients at its face points (LGL nodes), mg[slot][d*4+c][n^2]
  const int32_t *mslot;
  double *mflux, *mlift, *mg;
  // hybrid DG/FV operator (NULL without): element types [K] (1 = finite volume) and the outward
  // fluxes [K][6][5][n^2] of the sides of faces that touch a finite-volume element
  const uint8_t *fvflag;
  const double *fvFx;
  // split form, Navier-Stokes (NULL otherwise): the lifting's viscous terms as
  // the operator reads them, the strong-form divergence Gd[e][c][node] = sum_dir (sum_m D_{id,m}
  // Fv^dir_c(node m of the line) -+ lhat(+-1) Fv^dir_c on a +-face node) (c: momentum x, y, z,
  // energy) and every side's face trace Gf[e][s][c][face point] = Fv^{dir(s)}_c at the face node
  double *Gd, *Gf;
  // Navier-Stokes on LG nodes (NULL otherwise): every side's traces interpolated with l(+-1),
  // of the conservative state Utr[e][s][v][face point] and of W = (u, v, w, T)
  // Wtr[e][s][c][face point] (prolongation kernel), and of the lifted gradients
  // Gtr[e][s][d*4+c][face point] (lifting kernel); read at the faces by the lifting and operator
  double *Utr, *Wtr, *Gtr;
};

// Finite-volume subcells (Sec. 4) of one mesh on the device.
struct FvGeo {
  const double *V, *Vi, *Li;  // [n*n]: V_DG=>FV, its inverse, the inverse of Ptilde_k(x_i) (modal)
  const double *Jbar;         // [K][n^3] subcell mean of J
  const double *Nf;           // [K][3][n+1][n^2][3] mean of Ja^dir over subcell face f of direction dir
  uint8_t *flag;              // [K] 1 = finite-volume element (U holds subcell means)
  double *Fx;                 // [K][6][5][n^2] outward flux of sides of faces touching an FV element
  double *Dx;                 // [K][6][5][n^2] the neighbour's face datum at those sides (conservative)
  double *ind;                // [K] last troubled-cell indicator
  int *list;                  // [K] the finite-volume elements (count[0] of them), any order
  int *faces;                 // [3K] master sides e*6+s of faces touching one (count[1]), any order
  int *count;                 // [2]
  int limiter;                // 0 first order, 1 minmod, 2 van Leer
  double w;                   // subcell width 2/(N+1)
  double lo, hi;              // switch to DG below lo, to FV above hi
};

struct Phys {
  double gamma, R, mu, Pr, kappa;  // kappa = mu cp / Pr
  int vf, rs;
  double ub[5];                    // outer state of given-state boundary sides (conservative)
  double tw;                       // wall temperature of isothermal wall sides
  double pout;                     // pressure of outflow sides
};

// Kernel launch entry points, one explicit instantiation per degree.
// prolongation on LG nodes (Navier-Stokes): every side's traces of U and W into Geo::Utr, Wtr
template <int N>
int launch_prolong(const Geo &g, const Phys &ph, const double *U, hipStream_t st);
// lifting: out 0 writes G (gradients), 1 Fv (contravariant viscous fluxes, LGL only), 2 the split
// form's viscous divergence and face traces (Geo::Gd, Gf; LGL only), 3 both 1 and 2, 4 G and its
// LG face traces (Geo::Gtr), 5 the weak form's viscous volume term and face fluxes (Geo::Gd, Gf;
// G too when not NULL; conforming meshes), 6 the strong form's on LG nodes
template <int N>
int launch_lift(const Geo &g, const Phys &ph, bool lgl, int out, const double *U, double *G, double *Fv,
                hipStream_t st);
template <int N>
int launch_main(const Geo &g, const Phys &ph, bool lgl, int eqn, int form, const double *U, const double *G,
                double *out, double *R, double a, double b, double dt, int mode, hipStream_t st);
// Ubar (+)= scale (dL/dU)^T Ubar_t; Pf: face terms of the transposed lifting, [K][6][4][n^2]
// (Navier-Stokes); for Navier-Stokes with Rb != NULL the second reverse kernel then also sets
// Rb = ra Rb + rb Ubar (Euler: the caller updates Rb)
template <int N>
int launch_vjp(const Geo &g, const Phys &ph, int eqn, int form, bool lgl, const double *U, const double *G, double *Pf,
               const double *Ubar_t, double *Ubar, double scale, int accumulate, double *Rb, double ra, double rb,
               hipStream_t st);
template <int N>
int launch_reduce(const Geo &g, const Phys &ph, int what, const double *U, double cfl_unused, double *partial,
                  hipStream_t st);
// hybrid DG/FV (Euler): face fluxes of faces touching FV elements, the FV elements' operator with
// the optional fused RK stage (mode as launch_main), and the indicator with switching in place
template <int N>
int launch_fv_face(const Geo &g, const Phys &ph, const FvGeo &f, bool lgl, const double *U, hipStream_t st);
template <int N>
int launch_fv_volume(const Geo &g, const Phys &ph, const FvGeo &f, const double *U, double *out, double *R, double a,
                     double b, double dt, int mode, hipStream_t st);
template <int N>
int launch_fv_switch(const Geo &g, const Phys &ph, const FvGeo &f, double *U, int do_switch, hipStream_t st);
template <int N>
int launch_fv_lists(const Geo &g, const FvGeo &f, hipStream_t st);
// non-conforming faces: the lifting's surface terms (before the lifting) and the numerical fluxes
// (after it) of every mortar's small and big sides, into Geo::mlift and Geo::mflux
template <int N>
int launch_mortar_lift(const Geo &g, const Phys &ph, bool lgl, const MortarDesc *md, int nm, const double *U,
                       hipStream_t st);
template <int N>
int launch_mortar_flux(const Geo &g, const Phys &ph, bool lgl, int eqn, const MortarDesc *md, int nm,
                       const double *U, const double *G, hipStream_t st);

// One ensemble member as the batched kernels see it (entry of a device-resident table).
struct Member {
  Geo g;
  Phys ph;
  const double *U;  // stage input
  double *G;        // the member's scratch: contravariant viscous fluxes from the lifting
  double *out;      // stage output
  double *R;        // 2N-storage register
  double a, b, dt;  // stage coefficients: R = a R + dt L(U); out = U + b R
};

// All members of one degree N: m[0..count), element prefix sums first[0..count] (device),
// total = first[count]; tab = the 1D tables of degree N (identical for every member).
struct BatchView {
  const Member *m;
  const int *first;
  int count, total;
  const Tab *tab;
  int general;  // some member's mesh has face codes (Geo::fc): launch the kernels that read them
};

// elements per workgroup the batched kernels are built for (1, 2, 4 up to this bound)
__host__ __device__ constexpr int batch_max_epb(int N) { return N <= 3 ? 4 : (N <= 5 ? 2 : 1); }

// element handled by workgroup b of a grid of 8 ceil(K/8) workgroups: the launch hands each XCD
// (workgroups are dealt to the 8 XCDs round-robin) one contiguous range of elements, so face
// neighbours along the first two lattice directions are usually read from the same L2; values
// >= K are past the end
__host__ __device__ inline int xcd_element(int b, int K) {
  const int per = (K + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
__host__ __device__ inline int xcd_grid(int K) { return 8 * ((K + 7) / 8); }

// The neighbour's face point matching face point (a,b) of side s of element e: its direction,
// indices along the other two directions, whether it lies on the neighbour's +xi side, and
// whether side s is the master of the face.  On a structured mesh (no face codes) the neighbour
// meets side s on side s^1 at the same (a,b) and the +xi side is the master.  GEN selects the
// face-code lookup at compile time, so kernels built for structured meshes carry none of it; a
// GEN kernel still treats a mesh without face codes as structured (a batched launch can mix
// both kinds of members).
// A boundary side (bnd) has no neighbour: its outer state is built from the inner one and the
// other fields hold in-range placeholders that no load may use.
struct NbFace {
  int dn, a, b;
  bool plus, master, bnd;
  int kind;  // boundary kind (DG_BC_SYMMETRY, DG_BC_STATE) of a boundary side
};
template <int n, bool GEN> __device__ __forceinline__ NbFace nbr_face(const Geo &g, int e, int s, int a, int b) {
  NbFace f;
  f.bnd = false;
  f.kind = 0;
  if (!GEN || !g.fc) {
    f.dn = s >> 1; f.a = a; f.b = b; f.plus = !(s & 1); f.master = s & 1;
    return f;
  }
  const int c = g.fc[(size_t)e * 6 + s];
  if (c & 128) {
    f.dn = s >> 1; f.a = a; f.b = b; f.plus = !(s & 1); f.master = true; f.bnd = true; f.kind = c & 7;
    return f;
  }
  const int ns = c & 7, o = (c >> 3) & 7;
  const int p = (o & 4) ? b : a, q = (o & 4) ? a : b;
  f.dn = ns >> 1;
  f.a = (o & 1) ? n - 1 - p : p;
  f.b = (o & 2) ? n - 1 - q : q;
  f.plus = ns & 1;
  f.master = (c >> 6) & 1;
  return f;
}

// One launch over the structured members of every degree N <= 7: group g (degree N[g], its own
// view) takes the workgroups [start[g], start[g+1]); start[ng] is the grid's work.
constexpr int FUSED_MAXG = 8;
struct FusedView {
  BatchView v[FUSED_MAXG];
  int N[FUSED_MAXG];
  int start[FUSED_MAXG + 1];
  int ng;
};
int fused_epb(int N, bool lift);  // elements per 512-lane workgroup; 0 where N is not fused
int launch_fused_lift(const FusedView &fv, hipStream_t st);
int launch_fused_split(const FusedView &fv, bool ns, int vf, hipStream_t st);

template <int N>
int launch_batch_lift(const BatchView &bv, int epb, hipStream_t st);
template <int N>
int launch_batch_split(const BatchView &bv, bool ns, int vf, int epb, hipStream_t st);

// what codes for launch_reduce
enum { RED_TIMESTEP = 0, RED_INTEGRALS = 1, RED_FINITE = 2 };

int launch_final_reduce(int what, const double *partial, int K, double *out, hipStream_t st);
// Static scratch of the entry points that allocate nothing (dg_static.hip): doubles per GPU, and
// the once-per-device lookup of its device address, called by dg_init with that device current.
#define DG_NOALLOC_SCRATCH_DOUBLES (1 << 20)
int static_scratch_setup(int device);
int launch_axpby(double *y, const double *x, double alpha, double beta, size_t n, hipStream_t st);
int launch_mass(const double *sJ, const double *w, int n, size_t total, double *out, hipStream_t st);

}  // namespace dg

struct dg_handle {
  int K = 0, N = 0, n = 0, n2 = 0, n3 = 0, node_type = 0;
  int device = -1;  // HIP device current at dg_init
  dg_scheme sc{};
  dg::Phys ph{};
  hipStream_t stream = nullptr;
  // device memory owned by the handle
  double *d_Ja = nullptr, *d_sJ = nullptr, *d_fn = nullptr;
  int32_t *d_nbr = nullptr;
  uint8_t *d_fc = nullptr;      // face codes [K][6], only on meshes that are not structured
  int nm = 0;                   // non-conforming faces (mortars)
  dg::MortarDesc *d_md = nullptr;
  int32_t *d_mslot = nullptr;   // [K][6] face-array slot of every side, -1 if conforming
  bool fv_on = false;           // hybrid DG/FV operator enabled (dg_fv_enable)
  dg::FvGeo fvg{};              // its device tables (owned: the pointers below)
  double *d_fvtab = nullptr, *d_fvJbar = nullptr, *d_fvNf = nullptr, *d_fvFx = nullptr, *d_fvDx = nullptr;
  double *d_fvind = nullptr;
  uint8_t *d_fvflag = nullptr;
  double *d_Gd = nullptr, *d_Gf = nullptr;  // viscous volume term and face traces (Geo::Gd, Gf)
  double *d_Utr = nullptr, *d_Wtr = nullptr, *d_Gtr = nullptr;  // LG face traces of U, W, gradients
  int *d_fvlist = nullptr;  // work lists of the hybrid kernels: [K] elements, [3K] sides, [2] counts
  int *d_fvfaces = nullptr;
  int *d_fvcount = nullptr;
  double *d_mflux = nullptr, *d_mlift = nullptr, *d_mg = nullptr;  // [slots][5|12|12][n^2]
  bool has_boundary = false;    // some side has no neighbour
  bool needs_state = false;     // some boundary side takes the given outer state
  bool state_set = false;       // dg_set_boundary_state has been called
  bool needs_tw = false;        // some boundary side is an isothermal wall
  bool tw_set = false;          // dg_set_wall_temperature has been called
  bool needs_pout = false;      // some boundary side is a pressure outflow
  bool pout_set = false;        // dg_set_outflow_pressure has been called
  dg::Tab *d_tab = nullptr;
  double *d_G = nullptr;        // lifted gradients [K][12][n3] (Navier-Stokes)
  double *d_Pf = nullptr;       // face terms of the transposed lifting [K][6][4][n^2] (first VJP)
  double *d_partial = nullptr;  // [K][8] per-element partial reductions
  double *d_red = nullptr;      // [8] reduction result
  dg::Tab tab{};
  // optional per-kernel timing with HIP events (dg_profile)
  bool prof = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // lift ms, lift launches, main ms, main launches, face-kernel ms and launches (mortar fluxes,
  // DG/FV faces), FV volume-kernel ms and launches
  double prof_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<double> x_nodes;  // solution-node coordinates (host), [K][3][n3]
  std::vector<double> J_nodes;  // Jacobian at the solution nodes (host), [K][n3]
  std::string err;
  dg::Geo geo() const {
    dg::Geo g;
    g.Ja = d_Ja; g.sJ = d_sJ; g.fn = d_fn; g.nbr = d_nbr; g.fc = d_fc; g.tab = d_tab; g.K = K;
    g.mslot = d_mslot; g.mflux = d_mflux; g.mlift = d_mlift; g.mg = d_mg;
    g.fvflag = fv_on ? d_fvflag : nullptr; g.fvFx = fv_on ? d_fvFx : nullptr;
    g.Gd = d_Gd; g.Gf = d_Gf;
    g.Utr = d_Utr; g.Wtr = d_Wtr; g.Gtr = d_Gtr;
    return g;
  }
};
