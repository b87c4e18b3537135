// Host side of libdgsem: argument checks, the one-time geometry setup of dg_init, and the
// C entry points that launch the HIP kernels.  Nothing here computes the operator itself.
//
// Setup (Krais et al., FLEXI, Sec. 3.1):
//   * nodes and weights: roots of P_{N+1} (LG) or +-1 and roots of P_N' (LGL), by Newton;
//   * D_rs = l_s'(x_r) in barycentric form; Dhat_ij = -(w_j/w_i) D_ji, the matrix the volume
//     integral's derivation produces; l(+-1) and lhat(+-1) = l(+-1)/w;
//   * metric terms in curl form (eq. contravariantBasisVectorsCurl), evaluated on the degree-N
//     LGL sample of the mapping and interpolated exactly to LG nodes when those are used;
//   * J = det of the mapping Jacobian from the differentiation matrix at the solution nodes;
//   * face normals: Ja^d on the +xi_d face of the element that owns the face (the master,
//     Sec. 5.1), negated for the neighbour that sees the face as its -xi_d side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <cstddef>
#include <cstdlib>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dg_internal.h"

using dg::NMAX;

namespace {

const char *status_name(int s) {
  switch (s) {
    case DG_OK: return "DG_OK";
    case DG_ERR_ARG: return "DG_ERR_ARG: invalid argument";
    case DG_ERR_MESH: return "DG_ERR_MESH: invalid mesh";
    case DG_ERR_UNSUPPORTED: return "DG_ERR_UNSUPPORTED: valid request the library does not implement";
    case DG_ERR_HIP: return "DG_ERR_HIP: HIP runtime error";
    case DG_ERR_NONFINITE: return "DG_ERR_NONFINITE: non-finite value";
    case DG_ERR_OOM: return "DG_ERR_OOM: device allocation failed";
    default: return "unknown status";
  }
}

int fail(dg_handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

// ---------------------------------------------------------------- 1D basis
// All one-time tables are computed in long double and rounded once to double, so they are
// correctly rounded (up to rare ties) whatever the order of operations used here.
typedef long double xf;

// P_n and P_n' at x via the three-term recurrence
void legendre_pd(int n, xf x, xf &P, xf &dP) {
  xf pm = 1.0L, pc = x;
  if (n == 0) { P = 1.0L; dP = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    const xf pn = ((2.0L * k - 1.0L) * x * pc - (k - 1.0L) * pm) / k;
    pm = pc; pc = pn;
  }
  P = pc;
  // P_n' = n (P_{n-1} - x P_n) / (1 - x^2), valid off +-1
  dP = n * (pm - x * pc) / (1.0L - x * x);
}

void nodes_weights(int N, int type, std::vector<xf> &x, std::vector<xf> &w) {
  const int n = N + 1;
  x.assign(n, 0.0L);
  w.assign(n, 0.0L);
  const xf pi = 3.14159265358979323846264338327950288L;
  if (type == DG_NODES_LG) {
    for (int j = 0; j < n / 2; ++j) {
      // root j of P_n counted from +1, Tricomi-type initial guess
      xf r = std::cos(pi * (4.0L * j + 3.0L) / (4.0L * n + 2.0L));
      for (int it = 0; it < 60; ++it) {
        xf P, dP;
        legendre_pd(n, r, P, dP);
        const xf dr = P / dP;
        r -= dr;
        if (std::fabs(dr) <= 1e-20L) break;
      }
      xf P, dP;
      legendre_pd(n, r, P, dP);
      x[N - j] = r;
      x[j] = -r;
      w[j] = w[N - j] = 2.0L / ((1.0L - r * r) * dP * dP);
    }
    if (n % 2) {
      xf P, dP;
      legendre_pd(n, 0.0L, P, dP);
      x[N / 2] = 0.0L;
      w[N / 2] = 2.0L / (dP * dP);
    }
  } else {
    x[0] = -1.0L;
    x[N] = 1.0L;
    for (int j = 1; j < (n + 1) / 2; ++j) {
      // interior roots of P_N': Newton with P_N'' = (2x P_N' - N(N+1) P_N)/(1-x^2)
      xf r = std::cos(pi * j / N) * (1.0L - 0.05L / (N * N));
      for (int it = 0; it < 80; ++it) {
        xf P, dP;
        legendre_pd(N, r, P, dP);
        const xf d2P = (2.0L * r * dP - N * (N + 1.0L) * P) / (1.0L - r * r);
        const xf dr = dP / d2P;
        r -= dr;
        if (std::fabs(dr) <= 1e-20L) break;
      }
      x[N - j] = r;
      x[j] = -r;
    }
    if (n % 2) x[N / 2] = 0.0L;
    for (int j = 0; j < n; ++j) {
      xf pm = 1.0L, pc = x[j];
      for (int k = 2; k <= N; ++k) {
        const xf pn = ((2.0L * k - 1.0L) * x[j] * pc - (k - 1.0L) * pm) / k;
        pm = pc; pc = pn;
      }
      w[j] = 2.0L / (N * (N + 1.0L) * pc * pc);
    }
  }
}

struct Basis1D {
  int n = 0;
  std::vector<xf> x, w, bw, D, Dh, lm, lp;
};

xf lag_eval(const std::vector<xf> &x, const std::vector<xf> &bw, int j, xf t) {
  const int n = (int)x.size();
  for (int k = 0; k < n; ++k)
    if (t == x[k]) return k == j ? 1.0L : 0.0L;
  xf num = 0.0L, den = 0.0L;
  for (int k = 0; k < n; ++k) {
    const xf c = bw[k] / (t - x[k]);
    den += c;
    if (k == j) num = c;
  }
  return num / den;
}

Basis1D make_basis(int N, int type) {
  Basis1D B;
  const int n = N + 1;
  B.n = n;
  nodes_weights(N, type, B.x, B.w);
  B.bw.assign(n, 1.0L);
  for (int j = 0; j < n; ++j) {
    xf p = 1.0L;
    for (int k = 0; k < n; ++k)
      if (k != j) p *= (B.x[j] - B.x[k]);
    B.bw[j] = 1.0L / p;
  }
  B.D.assign(n * n, 0.0L);
  for (int r = 0; r < n; ++r) {
    xf diag = 0.0L;
    for (int s = 0; s < n; ++s)
      if (s != r) {
        B.D[r * n + s] = (B.bw[s] / B.bw[r]) / (B.x[r] - B.x[s]);
        diag -= B.D[r * n + s];
      }
    B.D[r * n + r] = diag;
  }
  B.Dh.assign(n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B.Dh[i * n + j] = -(B.w[j] / B.w[i]) * B.D[j * n + i];
  B.lm.resize(n);
  B.lp.resize(n);
  for (int j = 0; j < n; ++j) {
    B.lm[j] = lag_eval(B.x, B.bw, j, -1.0L);
    B.lp[j] = lag_eval(B.x, B.bw, j, 1.0L);
  }
  return B;
}

// ---------------------------------------------------------------- geometry
// y[i,j,k] = sum_m A[idx_dir, m] x[.. m ..] for an n x n matrix A along direction dir
void tensor_apply(const xf *A, int n, int dir, const xf *x, xf *y) {
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        xf s = 0.0L;
        const int row = dir == 0 ? i : (dir == 1 ? j : k);
        for (int m = 0; m < n; ++m) {
          const int ii = dir == 0 ? m : i, jj = dir == 1 ? m : j, kk = dir == 2 ? m : k;
          s += A[row * n + m] * x[ii + n * (jj + n * kk)];
        }
        y[i + n * (j + n * k)] = s;
      }
}

// y (n^3) = x (ng^3) interpolated along every direction with the n x ng matrix A
void tensor_interp(const xf *A, int n, int ng, const xf *x, xf *y) {
  std::vector<xf> t1((size_t)n * ng * ng), t2((size_t)n * n * ng);
  for (int c = 0; c < ng; ++c)
    for (int b = 0; b < ng; ++b)
      for (int i = 0; i < n; ++i) {
        xf s = 0.0L;
        for (int a = 0; a < ng; ++a) s += A[i * ng + a] * x[a + ng * (b + ng * c)];
        t1[i + n * (b + ng * c)] = s;
      }
  for (int c = 0; c < ng; ++c)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        xf s = 0.0L;
        for (int b = 0; b < ng; ++b) s += A[j * ng + b] * t1[i + n * (b + ng * c)];
        t2[i + n * (j + n * c)] = s;
      }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        xf s = 0.0L;
        for (int c = 0; c < ng; ++c) s += A[k * ng + c] * t2[i + n * (j + n * c)];
        y[i + n * (j + n * k)] = s;
      }
}

struct HostGeo {
  std::vector<double> Ja, J, sJ, xs, fn;
};

// Face conventions of conforming meshes.  Face point (a,b) of side s (direction d = s/2) is the
// volume node at position 0 (s even) or N (s odd) along d, with a and b the node indices along
// the other two directions in increasing order.  The orientation code o maps it to the
// neighbour's face point: swap (a,b) if o & 4, then reverse the first index if o & 1 and the
// second if o & 2.
inline void face_mate(int o, int N, int a, int b, int &a2, int &b2) {
  const int p = (o & 4) ? b : a, q = (o & 4) ? a : b;
  a2 = (o & 1) ? N - p : p;
  b2 = (o & 2) ? N - q : q;
}
inline int orientation_inverse(int o) { return (o & 4) ? (4 | ((o & 1) << 1) | ((o >> 1) & 1)) : o; }
inline int face_point_node(int n, int s, int a, int b) {
  const int d = s >> 1, m = (s & 1) ? n - 1 : 0;
  return d == 0 ? m + n * (a + n * b) : (d == 1 ? a + n * (m + n * b) : a + n * (b + n * m));
}
// node of the line through face point (ia, jb) of direction dir at position m along dir
inline int face_line_node(int n, int dir, int ia, int jb, int m) {
  return dir == 0 ? m + n * (ia + n * jb) : (dir == 1 ? ia + n * (m + n * jb) : ia + n * (jb + n * m));
}
// master of a face: a boundary side (no neighbour) itself, the +xi side where a +xi side meets
// a -xi side, else the element with the smaller index (the smaller side within one element)
inline bool face_master(int e, int s, int nb, int ns) {
  if (nb < 0) return true;
  if ((s & 1) != (ns & 1)) return (s & 1) != 0;
  return e < nb || (e == nb && s < ns);
}

// xgeo holds the mapping at the LGL nodes of degree ngeo (Sec. 2.1: the geometry degree N_geo is
// independent of N); it is interpolated to the degree-N LGL nodes, where the curl form is taken
inline bool is_mortar_side(const int8_t *mort, int q) { return mort && mort[q] != 0; }

int build_geometry(int K, int N, int ngeo, int type, const double *xgeo, const int32_t *nbr, const int8_t *nside,
                   const int8_t *flip, const int8_t *mort, HostGeo &G, std::string &msg) {
  const int n = N + 1, n2 = n * n, n3 = n2 * n;
  const int ng = ngeo + 1, ng3 = ng * ng * ng;
  const Basis1D L = make_basis(N, DG_NODES_LGL);
  std::vector<xf> Vg;  // degree-ngeo LGL -> degree-N LGL nodes, n x ng
  if (ngeo != N) {
    const Basis1D Bg = make_basis(ngeo, DG_NODES_LGL);
    Vg.resize((size_t)n * ng);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < ng; ++j) Vg[(size_t)i * ng + j] = lag_eval(Bg.x, Bg.bw, j, L.x[i]);
  }
  const Basis1D S = (type == DG_NODES_LGL) ? L : make_basis(N, type);
  std::vector<xf> V(n * n);  // LGL -> solution nodes
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = lag_eval(L.x, L.bw, j, S.x[i]);
  G.Ja.assign((size_t)K * 9 * n3, 0.0);
  G.J.assign((size_t)K * n3, 0.0);
  G.sJ.assign((size_t)K * n3, 0.0);
  G.xs.assign((size_t)K * 3 * n3, 0.0);
  G.fn.assign((size_t)K * 6 * 3 * n2, 0.0);
  // elements are independent: split them over host threads
  unsigned nthr = std::thread::hardware_concurrency();
  if (const char *env = std::getenv("OMP_NUM_THREADS")) nthr = (unsigned)std::max(1, std::atoi(env));
  nthr = std::max(1u, std::min(nthr, 32u));
  if ((size_t)K < 4 * (size_t)nthr) nthr = 1;
  std::vector<int> bad(nthr, -1), badq(nthr, 0);
  std::vector<double> badv(nthr, 0.0);
  auto work = [&](unsigned tid) {
  std::vector<xf> X(3 * n3), dx(9 * n3), prod(3 * n3), c1(n3), c2(n3), JaL(9 * n3), Jas(9 * n3), t1(n3), t2(n3),
      xs(3 * n3), jac(9 * n3), xg(ng3);
  const int e0 = (int)((size_t)K * tid / nthr), e1 = (int)((size_t)K * (tid + 1) / nthr);
  for (int e = e0; e < e1; ++e) {
    // work relative to the element centroid; the curl form is translation invariant and the
    // shift removes the cancellation between the two products of each curl component
    xf c0[3];
    for (int d = 0; d < 3; ++d) {
      xf acc = 0.0L;
      for (int q = 0; q < ng3; ++q) acc += xgeo[((size_t)e * 3 + d) * ng3 + q];
      c0[d] = acc / ng3;
      if (ngeo == N) {
        for (int q = 0; q < n3; ++q) X[d * n3 + q] = xgeo[((size_t)e * 3 + d) * n3 + q] - c0[d];
      } else {
        for (int q = 0; q < ng3; ++q) xg[q] = xgeo[((size_t)e * 3 + d) * ng3 + q] - c0[d];
        tensor_interp(Vg.data(), n, ng, xg.data(), &X[d * n3]);
      }
    }
    // dx[m*3+k] = d x_m / d xi_k on the LGL sample
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 3; ++k) tensor_apply(L.D.data(), n, k, &X[m * n3], &dx[(m * 3 + k) * n3]);
    // curl form, component nn with (nn, m, l) cyclic:
    //   Ja^i_nn = -[curl_xi (x_l grad_xi x_m)]_i
    for (int nn = 0; nn < 3; ++nn) {
      const int m = (nn + 1) % 3, l = (nn + 2) % 3;
      for (int k = 0; k < 3; ++k)
        for (int q = 0; q < n3; ++q) prod[k * n3 + q] = X[l * n3 + q] * dx[(m * 3 + k) * n3 + q];
      for (int i = 0; i < 3; ++i) {
        const int a = (i + 1) % 3, b = (i + 2) % 3;
        tensor_apply(L.D.data(), n, a, &prod[b * n3], c1.data());
        tensor_apply(L.D.data(), n, b, &prod[a * n3], c2.data());
        for (int q = 0; q < n3; ++q) JaL[(i * 3 + nn) * n3 + q] = c2[q] - c1[q];
      }
    }
    if (type == DG_NODES_LGL) {
      Jas = JaL;
      xs = X;
    } else {
      for (int c = 0; c < 9; ++c) {
        tensor_apply(V.data(), n, 0, &JaL[c * n3], t1.data());
        tensor_apply(V.data(), n, 1, t1.data(), t2.data());
        tensor_apply(V.data(), n, 2, t2.data(), &Jas[c * n3]);
      }
      for (int c = 0; c < 3; ++c) {
        tensor_apply(V.data(), n, 0, &X[c * n3], t1.data());
        tensor_apply(V.data(), n, 1, t1.data(), t2.data());
        tensor_apply(V.data(), n, 2, t2.data(), &xs[c * n3]);
      }
    }
    for (int q = 0; q < 9 * n3; ++q) G.Ja[(size_t)e * 9 * n3 + q] = (double)Jas[q];
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < n3; ++q) G.xs[((size_t)e * 3 + d) * n3 + q] = (double)(xs[d * n3 + q] + c0[d]);
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 3; ++k) tensor_apply(S.D.data(), n, k, &xs[m * n3], &jac[(m * 3 + k) * n3]);
    for (int q = 0; q < n3; ++q) {
      const xf a00 = jac[0 * n3 + q], a01 = jac[1 * n3 + q], a02 = jac[2 * n3 + q];
      const xf a10 = jac[3 * n3 + q], a11 = jac[4 * n3 + q], a12 = jac[5 * n3 + q];
      const xf a20 = jac[6 * n3 + q], a21 = jac[7 * n3 + q], a22 = jac[8 * n3 + q];
      const xf det = a00 * (a11 * a22 - a12 * a21) + a01 * (a12 * a20 - a10 * a22) + a02 * (a10 * a21 - a11 * a20);
      if (!(det > 0.0L) || !std::isfinite((double)det)) {
        if (bad[tid] < 0) { bad[tid] = e; badq[tid] = q; badv[tid] = (double)det; }
        return;
      }
      G.J[(size_t)e * n3 + q] = (double)det;
      G.sJ[(size_t)e * n3 + q] = (double)(1.0L / det);
    }
    // outward normal of every master side from the element's own metric: +-Ja^d at the face
    for (int s = 0; s < 6; ++s) {
      const int d = s >> 1;
      // a side of a non-conforming face keeps its own normal (a small side is the master of its
      // part of the face; the big side's flux is projected from the small sides')
      if (!is_mortar_side(mort, e * 6 + s) && !face_master(e, s, nbr[e * 6 + s], nside[e * 6 + s])) continue;
      const std::vector<xf> &l = (s & 1) ? S.lp : S.lm;
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a)
          for (int c = 0; c < 3; ++c) {
            xf v = 0.0L;
            for (int m = 0; m < n; ++m) {
              const int q = d == 0 ? (m + n * (a + n * b)) : (d == 1 ? (a + n * (m + n * b)) : (a + n * (b + n * m)));
              v += l[m] * Jas[(d * 3 + c) * n3 + q];
            }
            G.fn[(((size_t)e * 6 + s) * 3 + c) * n2 + a + n * b] = (double)((s & 1) ? v : -v);
          }
    }
  }
  };
  if (nthr == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nthr; ++t) pool.emplace_back(work, t);
    for (auto &th : pool) th.join();
  }
  for (unsigned t = 0; t < nthr; ++t)
    if (bad[t] >= 0) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "element %d node %d: Jacobian %.3e is not positive", bad[t], badq[t], badv[t]);
      msg = buf;
      return DG_ERR_MESH;
    }
  // slaves: negated normal of the master at the matching face point
  for (int e = 0; e < K; ++e)
    for (int s = 0; s < 6; ++s) {
      const int nb = nbr[e * 6 + s], ns = nside[e * 6 + s], o = flip ? flip[e * 6 + s] : 0;
      if (is_mortar_side(mort, e * 6 + s) || face_master(e, s, nb, ns)) continue;
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          int a2, b2;
          face_mate(o, N, a, b, a2, b2);
          for (int c = 0; c < 3; ++c)
            G.fn[(((size_t)e * 6 + s) * 3 + c) * n2 + a + n * b] = -G.fn[(((size_t)nb * 6 + ns) * 3 + c) * n2 + a2 + n * b2];
        }
    }
  return DG_OK;
}

// face codes for the kernels (see dg::Geo::fc); empty on a structured mesh
std::vector<uint8_t> face_codes(const dg_mesh *mesh) {
  const int K = mesh->n_elems;
  bool structured = true;
  for (int q = 0; q < 6 * K && structured; ++q)
    structured = mesh->nbr_elem[q] >= 0 && mesh->nbr_side[q] == ((q % 6) ^ 1) && (!mesh->flip || mesh->flip[q] == 0) &&
                 !is_mortar_side(mesh->mortar, q);
  std::vector<uint8_t> fc;
  if (structured) return fc;
  fc.resize((size_t)6 * K);
  for (int e = 0; e < K; ++e)
    for (int s = 0; s < 6; ++s) {
      const int q = e * 6 + s, ns = mesh->nbr_side[q], o = mesh->flip ? mesh->flip[q] : 0;
      if (is_mortar_side(mesh->mortar, q))
        fc[q] = (uint8_t)(128 | 64 | dg::FACE_MORTAR);  // fluxes from the mortar face arrays
      else if (mesh->nbr_elem[q] < 0)
        fc[q] = (uint8_t)(128 | 64 | ns);  // boundary of kind ns, its own master
      else
        fc[q] = (uint8_t)(ns | (o << 3) | (face_master(e, s, mesh->nbr_elem[q], ns) ? 64 : 0));
    }
  return fc;
}

int validate_mesh(const dg_mesh *mesh, int N, int node_type) {
  if (!mesh || !mesh->xgeo || !mesh->nbr_elem || !mesh->nbr_side) return DG_ERR_ARG;
  if (N < 1 || N > NMAX) return DG_ERR_UNSUPPORTED;
  if (mesh->n_geo < 1 || mesh->n_geo > 2 * NMAX) return DG_ERR_UNSUPPORTED;
  if (node_type != DG_NODES_LG && node_type != DG_NODES_LGL) return DG_ERR_ARG;
  if (mesh->n_elems < 1) return DG_ERR_ARG;
  const int K = mesh->n_elems;
  // connectivity: every side either is a boundary (neighbour -1, kind in nbr_side:
  // DG_BC_SYMMETRY ... DG_BC_OUTFLOW, orientation 0) or has a neighbour that names it back, on the side and with
  // the inverse orientation it names
  const int8_t *mort = mesh->mortar;
  std::vector<uint8_t> taken;  // positions of every big side named by a small side
  if (mort) taken.assign((size_t)6 * K, 0);
  for (int e = 0; e < K; ++e)
    for (int s = 0; s < 6; ++s) {
      const int q = e * 6 + s, nb = mesh->nbr_elem[q], ns = mesh->nbr_side[q];
      const int o = mesh->flip ? mesh->flip[q] : 0;
      const int mk = mort ? mort[q] : 0;
      if (mk < 0 || mk > 7) return DG_ERR_MESH;
      if (mk >= 1 && mk <= 3) {  // big side of a non-conforming face
        if (nb != -1 || o != 0) return DG_ERR_MESH;
        continue;
      }
      if (mk >= 4) {  // small side at position mk - 4 of the big side (nb, ns)
        if (nb < 0 || nb >= K || ns < 0 || ns > 5 || o < 0 || o > 7 || nb == e) return DG_ERR_MESH;
        const int t = mort[nb * 6 + ns], p = mk - 4;
        if (t < 1 || t > 3 || p >= (t == 3 ? 4 : 2)) return DG_ERR_MESH;
        if (taken[nb * 6 + ns] & (1u << p)) return DG_ERR_MESH;
        taken[nb * 6 + ns] |= (uint8_t)(1u << p);
        continue;
      }
      if (nb == -1) {
        if (ns < DG_BC_SYMMETRY || ns > DG_BC_OUTFLOW) return DG_ERR_UNSUPPORTED;
        if (o != 0) return DG_ERR_MESH;
        continue;
      }
      if (nb < 0 || nb >= K) return DG_ERR_MESH;
      if (ns < 0 || ns > 5 || o < 0 || o > 7 || (nb == e && ns == s)) return DG_ERR_MESH;
      const int qn = nb * 6 + ns;
      if (mesh->nbr_elem[qn] != e || mesh->nbr_side[qn] != s) return DG_ERR_MESH;
      if (mort && mort[qn] != 0) return DG_ERR_MESH;
      if ((mesh->flip ? mesh->flip[qn] : 0) != orientation_inverse(o)) return DG_ERR_MESH;
    }
  if (mort)
    for (int q = 0; q < 6 * K; ++q)
      if (mort[q] >= 1 && mort[q] <= 3 && taken[q] != (mort[q] == 3 ? 15 : 3)) return DG_ERR_MESH;
  // the matched face points coincide up to one translation per face (a periodic shift); the
  // faces are compared at the geometry's own nodes
  const int NG = mesh->n_geo, n = NG + 1, n3 = n * n * n;
  // a small side's points lie on the big side's face polynomial at the points of its sub-face
  std::vector<xf> gIL, gIU;  // geometry-degree interpolation to the lower / upper half
  if (mort) {
    const Basis1D Bg = make_basis(NG, DG_NODES_LGL);
    gIL.resize((size_t)n * n);
    gIU.resize((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m) {
        gIL[i * n + m] = lag_eval(Bg.x, Bg.bw, m, (Bg.x[i] - 1.0L) / 2.0L);
        gIU[i * n + m] = lag_eval(Bg.x, Bg.bw, m, (Bg.x[i] + 1.0L) / 2.0L);
      }
  }
  for (int e = 0; e < K; ++e) {
    const double *xe = mesh->xgeo + (size_t)e * 3 * n3;
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
      double lo = xe[d * n3], hi = lo;
      for (int q = 0; q < n3; ++q) { lo = std::min(lo, xe[d * n3 + q]); hi = std::max(hi, xe[d * n3 + q]); }
      ext = std::max(ext, hi - lo);
    }
    for (int s = 0; s < 6; ++s) {
      const int q = e * 6 + s, nb = mesh->nbr_elem[q], ns = mesh->nbr_side[q], o = mesh->flip ? mesh->flip[q] : 0;
      if (nb < 0) continue;
      const double *xn = mesh->xgeo + (size_t)nb * 3 * n3;
      double shift[3];
      if (mort && mort[q] >= 4) {
        const int t = mort[nb * 6 + ns], p = mort[q] - 4;
        const int p1 = t == 1 ? p : (t == 3 ? (p & 1) : -1), p2 = t == 2 ? p : (t == 3 ? (p >> 1) : -1);
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            int a2, b2;
            face_mate(o, NG, a, b, a2, b2);
            const int qe = face_point_node(n, s, a, b);
            for (int d = 0; d < 3; ++d) {
              xf v = 0.0L;
              for (int l = 0; l < n; ++l)
                for (int m = 0; m < n; ++m) {
                  const xf c1 = p1 < 0 ? (m == a2 ? 1.0L : 0.0L) : (p1 ? gIU : gIL)[a2 * n + m];
                  const xf c2 = p2 < 0 ? (l == b2 ? 1.0L : 0.0L) : (p2 ? gIU : gIL)[b2 * n + l];
                  v += c1 * c2 * xn[d * n3 + face_point_node(n, ns, m, l)];
                }
              const double dx = xe[d * n3 + qe] - (double)v;
              if (a == 0 && b == 0) shift[d] = dx;
              else if (!(std::fabs(dx - shift[d]) <= 1e-9 * ext)) return DG_ERR_MESH;
            }
          }
        continue;
      }
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          int a2, b2;
          face_mate(o, NG, a, b, a2, b2);
          const int qe = face_point_node(n, s, a, b), qn = face_point_node(n, ns, a2, b2);
          for (int d = 0; d < 3; ++d) {
            const double dx = xe[d * n3 + qe] - xn[d * n3 + qn];
            if (a == 0 && b == 0) shift[d] = dx;
            else if (!(std::fabs(dx - shift[d]) <= 1e-9 * ext)) return DG_ERR_MESH;
          }
        }
    }
  }
  return DG_OK;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

template <class T> int dev_alloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return DG_OK;
  if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return DG_ERR_OOM;
  }
  return DG_OK;
}

// lifting of U: out 0 gradients into G, 1 contravariant viscous fluxes into Fv, 2 both
// the kernels read the given outer state of DG_BC_STATE sides from the handle's physics
int state_ready(dg_handle *h) {
  if (h->needs_state && !h->state_set)
    return fail(h, DG_ERR_ARG, "the mesh has given-state boundary sides: call dg_set_boundary_state first");
  if (h->needs_tw && !h->tw_set)
    return fail(h, DG_ERR_ARG, "the mesh has isothermal wall sides: call dg_set_wall_temperature first");
  if (h->needs_pout && !h->pout_set)
    return fail(h, DG_ERR_ARG, "the mesh has outflow sides: call dg_set_outflow_pressure first");
  return DG_OK;
}

int lift_dispatch(dg_handle *h, const double *U, int out, double *G, double *Fv) {
  if (int rc = state_ready(h)) return rc;
  const dg::Geo g = h->geo();
  const bool lgl = h->node_type == DG_NODES_LGL;
  // on LG nodes the traces of U and W are prolonged first (the lifting and the operator read them)
  switch (h->N) {
#define DG_CASE(NN)                                                          \
  case NN:                                                                   \
    if (!lgl) {                                                              \
      const int rc = dg::launch_prolong<NN>(g, h->ph, U, h->stream);         \
      if (rc) return rc;                                                     \
    }                                                                        \
    return dg::launch_lift<NN>(g, h->ph, lgl, out, U, G, Fv, h->stream);
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
}

int main_dispatch(dg_handle *h, const double *U, const double *G, double *out, double *R, double a, double b,
                  double dt, int mode) {
  if (int rc = state_ready(h)) return rc;
  const dg::Geo g = h->geo();
  const bool lgl = h->node_type == DG_NODES_LGL;
  switch (h->N) {
#define DG_CASE(NN) \
  case NN: \
    return dg::launch_main<NN>(g, h->ph, lgl, h->sc.eqn, h->sc.form, U, G, out, R, a, b, dt, mode, h->stream);
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
}

// the kernels of the non-conforming faces: their lifting terms (flux = false) or their numerical
// fluxes (flux = true; G = the lifting output, gradients on LG nodes)
int mortar_dispatch(dg_handle *h, const double *U, const double *G, bool flux) {
  const dg::Geo g = h->geo();
  const bool lgl = h->node_type == DG_NODES_LGL;
  switch (h->N) {
#define DG_CASE(NN)                                                                                       \
  case NN:                                                                                                \
    return flux ? dg::launch_mortar_flux<NN>(g, h->ph, lgl, h->sc.eqn, h->d_md, h->nm, U, G, h->stream) \
                : dg::launch_mortar_lift<NN>(g, h->ph, lgl, h->d_md, h->nm, U, h->stream);
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
}

// the hybrid DG/FV kernels: what 0 the faces touching FV elements, 1 the FV elements' operator,
// 2 the indicator (3: with switching) in place on U, 4 the work lists from the element types
int fv_dispatch(dg_handle *h, int what, const double *U, double *out, double *R, double a, double b, double dt,
                int mode) {
  const dg::Geo g = h->geo();
  const bool lgl = h->node_type == DG_NODES_LGL;
  switch (h->N) {
#define DG_CASE(NN)                                                                                           \
  case NN:                                                                                                    \
    if (what == 0) return dg::launch_fv_face<NN>(g, h->ph, h->fvg, lgl, U, h->stream);                      \
    if (what == 1) return dg::launch_fv_volume<NN>(g, h->ph, h->fvg, U, out, R, a, b, dt, mode, h->stream); \
    if (what == 4) return dg::launch_fv_lists<NN>(g, h->fvg, h->stream);                                    \
    return dg::launch_fv_switch<NN>(g, h->ph, h->fvg, const_cast<double *>(U), what == 3, h->stream);
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
}

// lifting (Navier-Stokes) then the main operator, timed per kernel when profiling is on.  The
// split form takes the strong-form divergence and face traces of the contravariant viscous
// fluxes (Geo::Gd, Gf), the other forms the gradients (in the handle's scratch or, if
// Gkeep != NULL, in Gkeep).  With Gkeep the split form also writes the fluxes there, kept for a
// later reverse sweep.
int rhs_dispatch(dg_handle *h, const double *U, double *out, double *R, double a, double b, double dt, int mode,
                 double *Gkeep = nullptr) {
  const bool ns = h->sc.eqn == DG_NAVIER_STOKES;
  const bool split = h->sc.form == DG_FORM_SPLIT;
  if (h->prof) (void)hipEventRecord(h->ev[0], h->stream);
  if (ns) {
    if (h->nm) {
      // lifting surface terms of the non-conforming faces, read by the lifting kernel
      const int rc = mortar_dispatch(h, U, nullptr, false);
      if (rc) return rc;
    }
    double *dst = Gkeep ? Gkeep : h->d_G;
    // lifting outputs: 0 gradients, 2 divergence, 3 divergence and fluxes, 4 gradients and their
    // face traces (LG nodes), 5 the weak form's viscous volume term and face fluxes (conforming
    // meshes; the gradients too when kept)
    // (the strong form takes the split form's 2 on LGL nodes, 6 on LG nodes: the divergence with
    // the interpolated interior surface term and the face fluxes; with a kept stage the weak and
    // strong forms' liftings also write the gradients)
    const bool lg = h->node_type != DG_NODES_LGL;
    const bool weak_v = h->sc.form == DG_FORM_WEAK && !h->nm;
    const bool strong_v = h->sc.form == DG_FORM_STRONG && !h->nm;
    const int out = split ? (Gkeep ? 3 : 2) : (weak_v ? 5 : (strong_v ? (lg ? 6 : 2) : (lg ? 4 : 0)));
    const int rc = split ? lift_dispatch(h, U, out, nullptr, dst)
                         : lift_dispatch(h, U, out, (weak_v || strong_v) ? Gkeep : dst, nullptr);
    if (rc) return rc;
  }
  if (h->prof) (void)hipEventRecord(h->ev[1], h->stream);
  const double *Gin = (ns && Gkeep) ? Gkeep : h->d_G;
  if (h->fv_on) {
    // hybrid DG/FV (Euler): fluxes of the faces that touch finite-volume elements first
    const int rc = fv_dispatch(h, 0, U, nullptr, nullptr, 0.0, 0.0, 0.0, 0);
    if (rc) return rc;
  }
  if (h->nm) {
    // numerical fluxes of the non-conforming faces, read by the operator kernel
    const int rc = mortar_dispatch(h, U, Gin, true);
    if (rc) return rc;
  }
  if (h->prof) (void)hipEventRecord(h->ev[3], h->stream);
  int rc = main_dispatch(h, U, Gin, out, R, a, b, dt, mode);
  if (rc) return rc;
  if (h->prof) (void)hipEventRecord(h->ev[4], h->stream);
  if (h->fv_on) {
    // the finite-volume elements' subcell operator (the DG kernel leaves them out)
    rc = fv_dispatch(h, 1, U, out, R, a, b, dt, mode);
    if (rc) return rc;
  }
  if (h->prof) {
    (void)hipEventRecord(h->ev[2], h->stream);
    if (hipEventSynchronize(h->ev[2]) != hipSuccess) return DG_ERR_HIP;
    float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
    (void)hipEventElapsedTime(&m0, h->ev[0], h->ev[1]);
    (void)hipEventElapsedTime(&m1, h->ev[3], h->ev[4]);
    (void)hipEventElapsedTime(&m2, h->ev[1], h->ev[3]);
    (void)hipEventElapsedTime(&m3, h->ev[4], h->ev[2]);
    if (ns) { h->prof_ms[0] += m0; h->prof_ms[1] += 1; }
    h->prof_ms[2] += m1; h->prof_ms[3] += 1;
    if (h->nm || h->fv_on) { h->prof_ms[4] += m2; h->prof_ms[5] += 1; }
    if (h->fv_on) { h->prof_ms[6] += m3; h->prof_ms[7] += 1; }
  }
  return DG_OK;
}

int reduce_dispatch(dg_handle *h, int what, const double *U) {
  const dg::Geo g = h->geo();
  int rc;
  switch (h->N) {
#define DG_CASE(NN) \
  case NN: rc = dg::launch_reduce<NN>(g, h->ph, what, U, 0.0, h->d_partial, h->stream); break;
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
  if (rc) return rc;
  return dg::launch_final_reduce(what, h->d_partial, h->K, h->d_red, h->stream);
}

int fetch_red(dg_handle *h, double *out8) {
  if (hipMemcpyAsync(out8, h->d_red, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return fail(h, DG_ERR_HIP, "copy of a reduction result failed");
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, DG_ERR_HIP, "stream synchronisation failed");
  return DG_OK;
}

int check_solution_ptr(dg_handle *h, const void *p, const char *name) {
  if (!p) return fail(h, DG_ERR_ARG, std::string(name) + " is NULL");
  if (!aligned8(p)) return fail(h, DG_ERR_ARG, std::string(name) + " is not 8-byte aligned");
  return DG_OK;
}

bool overlap(const void *a, const void *b, size_t bytes) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + bytes && y < x + bytes;
}

// [a, a + abytes) and [b, b + bbytes) intersect
bool overlap2(const void *a, size_t abytes, const void *b, size_t bbytes) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + bbytes && y < x + abytes;
}

}  // namespace

extern "C" {

const char *dg_status_string(int status) { return status_name(status); }

const char *dg_last_error(const dg_handle *h) { return h ? h->err.c_str() : "no handle"; }

int dg_nodes(int N, int node_type, double *x, double *w) {
  if (N < 1 || N > NMAX || (node_type != DG_NODES_LG && node_type != DG_NODES_LGL) || !x || !w) return DG_ERR_ARG;
  std::vector<xf> xx, ww;
  nodes_weights(N, node_type, xx, ww);
  for (int i = 0; i <= N; ++i) { x[i] = (double)xx[i]; w[i] = (double)ww[i]; }
  return DG_OK;
}

int dg_rk_coefficients(double *a, double *b, double *c) {
  if (!a || !b || !c) return DG_ERR_ARG;
  // Carpenter & Kennedy (1994), five-stage fourth-order 2N-storage scheme
  static const double A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                              -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
  static const double B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                              1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                              2277821191437.0 / 14882151754819.0};
  static const double C[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                              2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};
  for (int s = 0; s < 5; ++s) { a[s] = A[s]; b[s] = B[s]; c[s] = C[s]; }
  return DG_OK;
}

int dg_init(const dg_mesh *mesh, int N, int node_type, const dg_scheme *sc, void *stream, dg_handle **out) {
  if (!out) return DG_ERR_ARG;
  *out = nullptr;
  if (!mesh || !sc) return DG_ERR_ARG;
  if (sc->eqn != DG_EULER && sc->eqn != DG_NAVIER_STOKES) return DG_ERR_ARG;
  if (sc->form < DG_FORM_WEAK || sc->form > DG_FORM_STRONG) return DG_ERR_ARG;
  if (sc->volflux < DG_VF_KEP || sc->volflux > DG_VF_CENTRAL) return DG_ERR_ARG;
  if (sc->riemann < DG_RS_LLF || sc->riemann > DG_RS_VOLFLUX_ROE) return DG_ERR_ARG;
  if (!(sc->gamma > 1.0) || !(sc->R > 0.0) || !(sc->Pr > 0.0) || !(sc->mu >= 0.0)) return DG_ERR_ARG;
  int vrc = validate_mesh(mesh, N, node_type);
  if (vrc) return vrc;
  if (sc->form == DG_FORM_SPLIT && node_type != DG_NODES_LGL) return DG_ERR_UNSUPPORTED;
  const int K = mesh->n_elems;
  dg_handle *h = new (std::nothrow) dg_handle;
  if (!h) return DG_ERR_OOM;
  h->K = K; h->N = N; h->n = N + 1; h->n2 = h->n * h->n; h->n3 = h->n2 * h->n; h->node_type = node_type;
  h->sc = *sc;
  h->stream = (hipStream_t)stream;
  h->ph.gamma = sc->gamma; h->ph.R = sc->R; h->ph.mu = sc->mu; h->ph.Pr = sc->Pr;
  h->ph.kappa = sc->mu * sc->gamma * sc->R / (sc->gamma - 1.0) / sc->Pr;
  h->ph.vf = sc->volflux; h->ph.rs = sc->riemann;
  const int n = h->n, n2 = h->n2, n3 = h->n3;
  // 1D tables
  const Basis1D B = make_basis(N, node_type);
  std::memset(&h->tab, 0, sizeof(h->tab));
  for (int c = 0; c < n * n; ++c) { h->tab.D[c] = (double)B.D[c]; h->tab.Dh[c] = (double)B.Dh[c]; }
  for (int j = 0; j < n; ++j) {
    h->tab.lm[j] = (double)B.lm[j]; h->tab.lp[j] = (double)B.lp[j];
    h->tab.lhm[j] = (double)(B.lm[j] / B.w[j]); h->tab.lhp[j] = (double)(B.lp[j] / B.w[j]);
    h->tab.w[j] = (double)B.w[j];
  }
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m)
      h->tab.Ds[i * n + m] = (double)(B.D[i * n + m] - (B.lp[i] / B.w[i]) * B.lp[m] + (B.lm[i] / B.w[i]) * B.lm[m]);
  // mortar operators of the solution nodes (Sec. 3.2)
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m) {
      h->tab.IL[i * n + m] = (double)lag_eval(B.x, B.bw, m, (B.x[i] - 1.0L) / 2.0L);
      h->tab.IU[i * n + m] = (double)lag_eval(B.x, B.bw, m, (B.x[i] + 1.0L) / 2.0L);
      h->tab.PL[i * n + m] = (double)(lag_eval(B.x, B.bw, i, (B.x[m] - 1.0L) / 2.0L) * B.w[m] / B.w[i]);
      h->tab.PU[i * n + m] = (double)(lag_eval(B.x, B.bw, i, (B.x[m] + 1.0L) / 2.0L) * B.w[m] / B.w[i]);
    }
  if (hipGetDevice(&h->device) != hipSuccess) { delete h; return DG_ERR_HIP; }
  // device address of the static scratch of the allocation-free entry points, once per device
  if (int src = dg::static_scratch_setup(h->device)) { delete h; return src; }
  HostGeo G;
  std::string msg;
  int rc = build_geometry(K, N, mesh->n_geo, node_type, mesh->xgeo, mesh->nbr_elem, mesh->nbr_side, mesh->flip,
                          mesh->mortar, G, msg);
  if (rc) { delete h; return rc; }
  const std::vector<uint8_t> fc = face_codes(mesh);
  for (int q = 0; q < 6 * K; ++q)
    if (mesh->nbr_elem[q] < 0) {
      h->has_boundary = true;
      if (mesh->nbr_side[q] == DG_BC_STATE) h->needs_state = true;
      if (mesh->nbr_side[q] == DG_BC_WALL_ISOTHERMAL) h->needs_tw = true;
      if (mesh->nbr_side[q] == DG_BC_OUTFLOW) h->needs_pout = true;
    }
  // non-conforming faces: one descriptor per big side, one face-array slot per mortar side
  std::vector<dg::MortarDesc> md;
  std::vector<int32_t> mslot;
  if (mesh->mortar) {
    mslot.assign((size_t)6 * K, -1);
    std::vector<int> big_of((size_t)6 * K, -1);
    int slots = 0;
    for (int q = 0; q < 6 * K; ++q)
      if (mesh->mortar[q] >= 1 && mesh->mortar[q] <= 3) {
        dg::MortarDesc d{};
        d.eb = q / 6; d.sb = q % 6; d.type = mesh->mortar[q]; d.slot = slots++;
        mslot[q] = d.slot;
        big_of[q] = (int)md.size();
        md.push_back(d);
      }
    for (int q = 0; q < 6 * K; ++q)
      if (mesh->mortar[q] >= 4) {
        dg::MortarDesc &d = md[big_of[mesh->nbr_elem[q] * 6 + mesh->nbr_side[q]]];
        const int p = mesh->mortar[q] - 4;
        d.es[p] = q / 6; d.ss[p] = q % 6; d.o[p] = mesh->flip ? mesh->flip[q] : 0; d.sl[p] = slots++;
        mslot[q] = d.sl[p];
      }
    h->nm = (int)md.size();
    if (h->nm == 0) mslot.clear();
  }
  const std::vector<double> &sJ = G.sJ;
  h->x_nodes.swap(G.xs);
  h->J_nodes.swap(G.J);
  const bool ns = sc->eqn == DG_NAVIER_STOKES;
  rc = dev_alloc(&h->d_Ja, (size_t)K * 9 * n3);
  if (!rc) rc = dev_alloc(&h->d_sJ, (size_t)K * n3);
  if (!rc) rc = dev_alloc(&h->d_fn, (size_t)K * 18 * n2);
  if (!rc) rc = dev_alloc(&h->d_nbr, (size_t)K * 6);
  if (!rc && !fc.empty()) rc = dev_alloc(&h->d_fc, fc.size());
  if (!rc) rc = dev_alloc(&h->d_tab, 1);
  if (!rc && ns) rc = dev_alloc(&h->d_G, (size_t)K * 12 * n3);
  if (!rc && ns) {
    rc = dev_alloc(&h->d_Gd, (size_t)K * 4 * n3);
    if (!rc) rc = dev_alloc(&h->d_Gf, (size_t)K * 24 * n2);
  }
  if (!rc && ns && node_type != DG_NODES_LGL) {
    rc = dev_alloc(&h->d_Utr, (size_t)K * 30 * n2);
    if (!rc) rc = dev_alloc(&h->d_Wtr, (size_t)K * 24 * n2);
    if (!rc) rc = dev_alloc(&h->d_Gtr, (size_t)K * 72 * n2);
  }
  if (!rc) rc = dev_alloc(&h->d_partial, (size_t)K * 8);
  if (!rc) rc = dev_alloc(&h->d_red, 8);
  if (!rc && h->nm) {
    int slots = 0;
    for (const dg::MortarDesc &d : md) slots += 1 + (d.type == 3 ? 4 : 2);
    rc = dev_alloc(&h->d_md, md.size());
    if (!rc) rc = dev_alloc(&h->d_mslot, mslot.size());
    if (!rc) rc = dev_alloc(&h->d_mflux, (size_t)slots * 5 * n2);
    if (!rc) rc = dev_alloc(&h->d_mlift, (size_t)slots * 12 * n2);
    if (!rc) rc = dev_alloc(&h->d_mg, (size_t)slots * 12 * n2);
  }
  if (rc) { dg_destroy(h); return rc; }
  bool ok = hipMemcpy(h->d_Ja, G.Ja.data(), G.Ja.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(h->d_sJ, sJ.data(), sJ.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(h->d_fn, G.fn.data(), G.fn.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(h->d_nbr, mesh->nbr_elem, (size_t)K * 6 * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
  if (!fc.empty()) ok = ok && hipMemcpy(h->d_fc, fc.data(), fc.size(), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(h->d_tab, &h->tab, sizeof(dg::Tab), hipMemcpyHostToDevice) == hipSuccess;
  if (h->nm) {
    ok = ok && hipMemcpy(h->d_md, md.data(), md.size() * sizeof(dg::MortarDesc), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(h->d_mslot, mslot.data(), mslot.size() * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) { dg_destroy(h); return DG_ERR_HIP; }
  *out = h;
  return DG_OK;
}

int dg_host_geometry(const dg_mesh *mesh, int N, int node_type, double *Ja, double *J, double *fn, double *D,
                     double *Dhat) {
  int rc = validate_mesh(mesh, N, node_type);
  if (rc) return rc;
  const int K = mesh->n_elems, n = N + 1;
  HostGeo G;
  std::string msg;
  rc = build_geometry(K, N, mesh->n_geo, node_type, mesh->xgeo, mesh->nbr_elem, mesh->nbr_side, mesh->flip,
                      mesh->mortar, G, msg);
  if (rc) return rc;
  if (Ja) std::memcpy(Ja, G.Ja.data(), G.Ja.size() * sizeof(double));
  if (J) std::memcpy(J, G.J.data(), G.J.size() * sizeof(double));
  if (fn) std::memcpy(fn, G.fn.data(), G.fn.size() * sizeof(double));
  const Basis1D B = make_basis(N, node_type);
  for (int c = 0; c < n * n; ++c) {
    if (D) D[c] = (double)B.D[c];
    if (Dhat) Dhat[c] = (double)B.Dh[c];
  }
  return DG_OK;
}

int dg_set_stream(dg_handle *h, void *stream) {
  if (!h) return DG_ERR_ARG;
  h->stream = (hipStream_t)stream;
  return DG_OK;
}

int dg_mesh_connect(int n_elems, int n_geo, const double *xgeo, const double period[3], double tol, int bc_kind,
                    int32_t *nbr, int8_t *side, int8_t *flip) {
  if (n_elems < 1 || n_geo < 1 || n_geo > NMAX || !xgeo || !nbr || !side || !flip) return DG_ERR_ARG;
  if (bc_kind < DG_BC_SYMMETRY || bc_kind > DG_BC_OUTFLOW) return DG_ERR_ARG;
  const int K = n_elems, N = n_geo, n = N + 1, n3 = n * n * n;
  double L[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < 3 && period; ++d) {
    if (!(period[d] >= 0.0) || !std::isfinite(period[d])) return DG_ERR_ARG;
    L[d] = period[d];
  }
  // corners of every face, in face-point order (0,0), (N,0), (0,N), (N,N), shifted so that the
  // face centroid lies in [0, L_d) along every periodic direction d
  const int F = 6 * K;
  std::vector<double> corner((size_t)F * 12), cen((size_t)F * 3);
  double hmin = INFINITY;
  for (int e = 0; e < K; ++e) {
    const double *x = xgeo + (size_t)e * 3 * n3;
    for (int d = 0; d < 3; ++d) {
      double lo = x[d * n3], hi = lo;
      for (int q = 0; q < n3; ++q) { lo = std::min(lo, x[d * n3 + q]); hi = std::max(hi, x[d * n3 + q]); }
      if (!std::isfinite(lo) || !std::isfinite(hi)) return DG_ERR_ARG;
      hmin = std::min(hmin, hi - lo);
    }
  }
  if (!(tol > 0.0)) tol = 1e-8 * hmin;
  if (!(tol > 0.0) || !std::isfinite(tol)) return DG_ERR_ARG;  // degenerate elements
  for (int e = 0; e < K; ++e) {
    const double *x = xgeo + (size_t)e * 3 * n3;
    for (int s = 0; s < 6; ++s) {
      const int f = e * 6 + s;
      double c[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < 4; ++k) {
        const int q = face_point_node(n, s, (k & 1) ? N : 0, (k & 2) ? N : 0);
        for (int d = 0; d < 3; ++d) {
          corner[(size_t)f * 12 + k * 3 + d] = x[d * n3 + q];
          c[d] += 0.25 * x[d * n3 + q];
        }
      }
      for (int d = 0; d < 3; ++d) {
        double sh = 0.0;
        if (L[d] > 0.0) sh = std::floor((c[d] + tol) / L[d]) * L[d];
        for (int k = 0; k < 4; ++k) corner[(size_t)f * 12 + k * 3 + d] -= sh;
        cen[(size_t)f * 3 + d] = c[d] - sh;
      }
    }
  }
  // faces binned by centroid on a grid of spacing 4 tol; a partner is searched in the 27 cells
  // around a face's cell
  const double hc = 4.0 * tol;
  auto cell = [&](int f, int d) { return (long long)std::floor(cen[(size_t)f * 3 + d] / hc); };
  auto key = [](long long i, long long j, long long k) {
    return (uint64_t)(i * 73856093LL) ^ (uint64_t)(j * 19349663LL) ^ (uint64_t)(k * 83492791LL);
  };
  std::unordered_multimap<uint64_t, int> bins;
  bins.reserve((size_t)F * 2);
  for (int f = 0; f < F; ++f) bins.emplace(key(cell(f, 0), cell(f, 1), cell(f, 2)), f);
  auto close = [&](int f, int k, int g, int l) {
    for (int d = 0; d < 3; ++d)
      if (!(std::fabs(corner[(size_t)f * 12 + k * 3 + d] - corner[(size_t)g * 12 + l * 3 + d]) <= tol)) return false;
    return true;
  };
  for (int f = 0; f < F; ++f) {
    int partner = -1, code = -1;
    const long long ci = cell(f, 0), cj = cell(f, 1), ck = cell(f, 2);
    for (int di = -1; di <= 1 && partner < 0; ++di)
      for (int dj = -1; dj <= 1 && partner < 0; ++dj)
        for (int dk = -1; dk <= 1 && partner < 0; ++dk) {
          auto range = bins.equal_range(key(ci + di, cj + dj, ck + dk));
          for (auto it = range.first; it != range.second && partner < 0; ++it) {
            const int g = it->second;
            if (g == f) continue;
            // the orientation code whose face map sends every corner of f onto a corner of g
            for (int o = 0; o < 8 && partner < 0; ++o) {
              bool ok = true;
              for (int k = 0; k < 4 && ok; ++k) {
                int a2, b2;
                face_mate(o, N, (k & 1) ? N : 0, (k & 2) ? N : 0, a2, b2);
                ok = close(f, k, g, (a2 ? 1 : 0) + (b2 ? 2 : 0));
              }
              if (ok) { partner = g; code = o; }
            }
          }
        }
    if (partner < 0) {
      nbr[f] = -1; side[f] = (int8_t)bc_kind; flip[f] = 0;
    } else {
      nbr[f] = partner / 6; side[f] = (int8_t)(partner % 6); flip[f] = (int8_t)code;
    }
  }
  return DG_OK;
}

// position of integer point (x0, x1, x2) (each < 2^B) along a 3-D Hilbert curve: Skilling's
// transform of the coordinates to the curve's transposed index (J. Skilling, "Programming the
// Hilbert curve", AIP Conf. Proc. 707, 2004), then the index bits interleaved
static uint64_t hilbert_index(uint32_t x[3], int B) {
  // inverse undo of excess work
  for (uint32_t Q = 1u << (B - 1); Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (x[i] & Q) {
        x[0] ^= P;  // invert the low bits of the first coordinate
      } else {
        const uint32_t t = (x[0] ^ x[i]) & P;  // exchange the low bits of x[0] and x[i]
        x[0] ^= t;
        x[i] ^= t;
      }
    }
  }
  // Gray encode
  for (int i = 1; i < 3; ++i) x[i] ^= x[i - 1];
  uint32_t t = 0;
  for (uint32_t Q = 1u << (B - 1); Q > 1; Q >>= 1)
    if (x[2] & Q) t ^= Q - 1;
  for (int i = 0; i < 3; ++i) x[i] ^= t;
  // interleave: the most significant bit of x[0] first
  uint64_t h = 0;
  for (int b = B - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) h = (h << 1) | ((x[i] >> b) & 1u);
  return h;
}

int dg_mesh_sfc_order(int n_elems, int n_geo, const double *xgeo, int32_t *order) {
  if (n_elems < 1 || n_geo < 1 || n_geo > NMAX || !xgeo || !order) return DG_ERR_ARG;
  const int K = n_elems, n = n_geo + 1, n3 = n * n * n;
  std::vector<double> c((size_t)K * 3);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int e = 0; e < K; ++e)
    for (int d = 0; d < 3; ++d) {
      double acc = 0.0;
      for (int q = 0; q < n3; ++q) acc += xgeo[((size_t)e * 3 + d) * n3 + q];
      acc /= n3;
      if (!std::isfinite(acc)) return DG_ERR_ARG;
      c[(size_t)e * 3 + d] = acc;
      lo[d] = std::min(lo[d], acc);
      hi[d] = std::max(hi[d], acc);
    }
  // centroids mapped onto a 2^21 grid per axis (one scale for all axes keeps the curve's cells
  // cubic), then sorted by their Hilbert index; ties keep the input order
  const int B = 21;
  const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
  const double sc = ((double)((1u << B) - 1)) / ext;
  std::vector<std::pair<uint64_t, int32_t>> key((size_t)K);
  for (int e = 0; e < K; ++e) {
    uint32_t x[3];
    for (int d = 0; d < 3; ++d)
      x[d] = (uint32_t)std::min<double>((double)((1u << B) - 1), std::floor((c[(size_t)e * 3 + d] - lo[d]) * sc + 0.5));
    key[e] = {hilbert_index(x, B), (int32_t)e};
  }
  std::stable_sort(key.begin(), key.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
  for (int i = 0; i < K; ++i) order[i] = key[i].second;
  return DG_OK;
}

int dg_set_outflow_pressure(dg_handle *h, double p_out) {
  if (!h) return DG_ERR_ARG;
  if (!(p_out > 0.0) || !std::isfinite(p_out)) return fail(h, DG_ERR_ARG, "outflow pressure must be positive");
  h->ph.pout = p_out;
  h->pout_set = true;
  return DG_OK;
}

int dg_set_wall_temperature(dg_handle *h, double T_w) {
  if (!h) return DG_ERR_ARG;
  if (!(T_w > 0.0) || !std::isfinite(T_w)) return fail(h, DG_ERR_ARG, "wall temperature must be positive");
  h->ph.tw = T_w;
  h->tw_set = true;
  return DG_OK;
}

int dg_set_boundary_state(dg_handle *h, const double ub[5]) {
  if (!h || !ub) return DG_ERR_ARG;
  for (int v = 0; v < 5; ++v)
    if (!std::isfinite(ub[v])) return fail(h, DG_ERR_ARG, "boundary state is not finite");
  const double p = (h->sc.gamma - 1.0) * (ub[4] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2] + ub[3] * ub[3]) / ub[0]);
  if (!(ub[0] > 0.0) || !(p > 0.0)) return fail(h, DG_ERR_ARG, "boundary state needs positive density and pressure");
  for (int v = 0; v < 5; ++v) h->ph.ub[v] = ub[v];
  h->state_set = true;
  return DG_OK;
}

int dg_info(const dg_handle *h, int64_t out[4]) {
  if (!h || !out) return DG_ERR_ARG;
  out[0] = h->K; out[1] = h->N; out[2] = h->n3; out[3] = h->node_type;
  return DG_OK;
}

int dg_rhs(dg_handle *h, const double *U, double *Ut) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U, "U");
  if (!rc) rc = check_solution_ptr(h, Ut, "Ut");
  if (rc) return rc;
  const size_t bytes = (size_t)h->K * 5 * h->n3 * sizeof(double);
  if (overlap(U, Ut, bytes)) return fail(h, DG_ERR_ARG, "U and Ut overlap");
  rc = rhs_dispatch(h, U, Ut, nullptr, 0.0, 0.0, 0.0, 0);
  if (rc) return fail(h, rc, "launch of the operator failed");
  return DG_OK;
}

int dg_rk_stage(dg_handle *h, const double *U_in, double *U_out, double *R, double a, double b, double dt) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U_in, "U_in");
  if (!rc) rc = check_solution_ptr(h, U_out, "U_out");
  if (!rc) rc = check_solution_ptr(h, R, "R");
  if (rc) return rc;
  const size_t bytes = (size_t)h->K * 5 * h->n3 * sizeof(double);
  if (overlap(U_in, U_out, bytes) || overlap(U_in, R, bytes) || overlap(U_out, R, bytes))
    return fail(h, DG_ERR_ARG, "U_in, U_out and R must be three distinct buffers");
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(dt)) return fail(h, DG_ERR_ARG, "non-finite coefficient");
  rc = rhs_dispatch(h, U_in, U_out, R, a, b, dt, 1);
  if (rc) return fail(h, rc, "launch of the operator failed");
  return DG_OK;
}

int dg_timestep(dg_handle *h, const double *U, double cfl, double dfl, double *dt_out) {
  if (!h || !dt_out) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U, "U");
  if (rc) return rc;
  if (!(cfl > 0.0) || !(dfl > 0.0)) return fail(h, DG_ERR_ARG, "CFL numbers must be positive");
  rc = reduce_dispatch(h, dg::RED_TIMESTEP, U);
  if (rc) return fail(h, rc, "launch of the time-step reduction failed");
  double r[8];
  rc = fetch_red(h, r);
  if (rc) return rc;
  if (!std::isfinite(r[0]) || !(r[0] > 0.0)) return fail(h, DG_ERR_NONFINITE, "invalid signal speed");
  double dt = cfl * 2.0 / ((2.0 * h->N + 1.0) * r[0]);
  if (h->sc.eqn == DG_NAVIER_STOKES && h->sc.mu > 0.0 && r[1] > 0.0)
    dt = std::min(dt, dfl * 4.0 / ((2.0 * h->N + 1.0) * r[1]));
  *dt_out = dt;
  return DG_OK;
}

int dg_integrals(dg_handle *h, const double *U, double out[8]) {
  if (!h || !out) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U, "U");
  if (rc) return rc;
  rc = reduce_dispatch(h, dg::RED_INTEGRALS, U);
  if (rc) return fail(h, rc, "launch of the integral reduction failed");
  return fetch_red(h, out);
}

int dg_check_finite(dg_handle *h, const double *U) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U, "U");
  if (rc) return rc;
  rc = reduce_dispatch(h, dg::RED_FINITE, U);
  if (rc) return fail(h, rc, "launch of the finiteness check failed");
  double r[8];
  rc = fetch_red(h, r);
  if (rc) return rc;
  if (r[0] != 0.0) return fail(h, DG_ERR_NONFINITE, "solution holds NaN or Inf");
  return DG_OK;
}

int dg_mass_weights(dg_handle *h, double *out) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, out, "out");
  if (rc) return rc;
  const double *w = reinterpret_cast<const double *>(reinterpret_cast<const char *>(h->d_tab) + offsetof(dg::Tab, w));
  rc = dg::launch_mass(h->d_sJ, w, h->n, (size_t)h->K * h->n3, out, h->stream);
  if (rc) return fail(h, rc, "launch of the mass-weight kernel failed");
  return DG_OK;
}

int dg_node_coords(dg_handle *h, double *x_host) {
  if (!h || !x_host) return DG_ERR_ARG;
  std::memcpy(x_host, h->x_nodes.data(), h->x_nodes.size() * sizeof(double));
  return DG_OK;
}

int dg_profile(dg_handle *h, int enable) {
  if (!h) return DG_ERR_ARG;
  if (enable && !h->ev[0]) {
    for (int i = 0; i < 5; ++i)
      if (hipEventCreate(&h->ev[i]) != hipSuccess) return fail(h, DG_ERR_HIP, "hipEventCreate failed");
  }
  h->prof = enable != 0;
  for (int i = 0; i < 8; ++i) h->prof_ms[i] = 0.0;
  return DG_OK;
}

int dg_profile_read(const dg_handle *h, double out[4]) {
  if (!h || !out) return DG_ERR_ARG;
  for (int i = 0; i < 4; ++i) out[i] = h->prof_ms[i];
  return DG_OK;
}

int dg_profile_read_ex(const dg_handle *h, double *out, int cap) {
  if (!h || !out || cap < 0) return DG_ERR_ARG;
  for (int i = 0; i < cap && i < 8; ++i) out[i] = h->prof_ms[i];
  return DG_OK;
}

// ---- hybrid DG/finite-volume subcells (Sec. 4)
namespace {
// inverse of an n x n matrix (Gauss-Jordan, partial pivoting, extended precision)
std::vector<xf> invert(std::vector<xf> A, int n) {
  std::vector<xf> I((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0L;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs((double)A[(size_t)r * n + c]) > std::fabs((double)A[(size_t)piv * n + c])) piv = r;
    for (int j = 0; j < n; ++j) {
      std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
      std::swap(I[(size_t)c * n + j], I[(size_t)piv * n + j]);
    }
    const xf d = A[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) { A[(size_t)c * n + j] /= d; I[(size_t)c * n + j] /= d; }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const xf f = A[(size_t)r * n + c];
        for (int j = 0; j < n; ++j) { A[(size_t)r * n + j] -= f * A[(size_t)c * n + j]; I[(size_t)r * n + j] -= f * I[(size_t)c * n + j]; }
      }
  }
  return I;
}
}  // namespace

int dg_fv_enable(dg_handle *h, int limiter, double ind_lo, double ind_hi) {
  if (!h) return DG_ERR_ARG;
  if (h->sc.eqn != DG_EULER) return fail(h, DG_ERR_UNSUPPORTED, "finite-volume subcells are built for the Euler equations");
  if (h->has_boundary || h->nm)
    return fail(h, DG_ERR_UNSUPPORTED, "finite-volume subcells are built for conforming meshes without boundary sides");
  if (limiter < 0 || limiter > 2 || !std::isfinite(ind_lo) || !std::isfinite(ind_hi) || ind_lo > ind_hi)
    return fail(h, DG_ERR_ARG, "limiter must be 0..2 and the thresholds finite with lo <= hi");
  const int K = h->K, N = h->N, n = h->n, n2 = h->n2, n3 = h->n3;
  if (!h->fv_on) {
    const Basis1D B = make_basis(N, h->node_type);
    const xf w = 2.0L / n;
    // V_DG=>FV: subcell means of the Lagrange basis by the scheme's quadrature mapped into each subcell
    std::vector<xf> V((size_t)n * n), L((size_t)n * n);
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i) {
        xf acc = 0.0L;
        for (int l = 0; l < n; ++l) acc += B.w[l] * lag_eval(B.x, B.bw, i, -1.0L + k * w + (B.x[l] + 1.0L) * w / 2.0L);
        V[(size_t)k * n + i] = acc / 2.0L;
      }
    // orthonormal Legendre polynomials at the nodes, L[i][k] = sqrt((2k+1)/2) P_k(x_i)
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        xf P, dP;
        legendre_pd(k, B.x[i], P, dP);
        L[(size_t)i * n + k] = P * std::sqrt((2.0L * k + 1.0L) / 2.0L);
      }
    const std::vector<xf> Vi = invert(V, n), Li = invert(L, n);
    std::vector<double> tab((size_t)3 * n * n);
    for (int c = 0; c < n * n; ++c) { tab[c] = (double)V[c]; tab[n * n + c] = (double)Vi[c]; tab[2 * n * n + c] = (double)Li[c]; }
    // subcell geometry from the metric terms: Jbar = (V x V x V) J, face means of Ja^dir
    std::vector<double> Ja((size_t)K * 9 * n3);
    if (hipMemcpy(Ja.data(), h->d_Ja, Ja.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(h, DG_ERR_HIP, "copy of the metric terms failed");
    std::vector<xf> lf((size_t)(n + 1) * n);
    for (int f = 0; f <= n; ++f)
      for (int m = 0; m < n; ++m) lf[(size_t)f * n + m] = lag_eval(B.x, B.bw, m, -1.0L + f * w);
    std::vector<double> Jbar((size_t)K * n3), Nf((size_t)K * 3 * (n + 1) * n2 * 3);
    // elements are independent: split them over host threads
    unsigned nthr = std::thread::hardware_concurrency();
    if (const char *env = std::getenv("OMP_NUM_THREADS")) nthr = (unsigned)std::max(1, std::atoi(env));
    nthr = std::max(1u, std::min(nthr, 32u));
    if ((size_t)K < 4 * (size_t)nthr) nthr = 1;
    auto work = [&](unsigned tid) {
      std::vector<xf> x(n3), y(n3), gfa((size_t)n2), ga((size_t)n2);
      const int e0 = (int)((size_t)K * tid / nthr), e1 = (int)((size_t)K * (tid + 1) / nthr);
      for (int e = e0; e < e1; ++e) {
        for (int q = 0; q < n3; ++q) x[q] = h->J_nodes[(size_t)e * n3 + q];
        for (int dir = 0; dir < 3; ++dir) {
          tensor_apply(V.data(), n, dir, x.data(), y.data());
          x.swap(y);
        }
        for (int q = 0; q < n3; ++q) Jbar[(size_t)e * n3 + q] = (double)x[q];
        for (int dir = 0; dir < 3; ++dir)
          for (int d = 0; d < 3; ++d) {
            const double *J = Ja.data() + ((size_t)e * 9 + dir * 3 + d) * n3;
            for (int f = 0; f <= n; ++f) {
              // Ja^dir_d on the face position f at face point (ia, jb), then subcell means along the
              // face's first direction and then its second
              for (int jb = 0; jb < n; ++jb)
                for (int ia = 0; ia < n; ++ia) {
                  xf v = 0.0L;
                  for (int m = 0; m < n; ++m) v += lf[(size_t)f * n + m] * J[face_line_node(n, dir, ia, jb, m)];
                  gfa[ia + n * jb] = v;
                }
              for (int jb = 0; jb < n; ++jb)
                for (int aa = 0; aa < n; ++aa) {
                  xf v = 0.0L;
                  for (int ia = 0; ia < n; ++ia) v += V[(size_t)aa * n + ia] * gfa[ia + n * jb];
                  ga[aa + n * jb] = v;
                }
              for (int bb = 0; bb < n; ++bb)
                for (int aa = 0; aa < n; ++aa) {
                  xf v = 0.0L;
                  for (int jb = 0; jb < n; ++jb) v += V[(size_t)bb * n + jb] * ga[aa + n * jb];
                  Nf[((((size_t)e * 3 + dir) * (n + 1) + f) * n2 + aa + n * bb) * 3 + d] = (double)v;
                }
            }
          }
      }
    };
    if (nthr == 1) {
      work(0);
    } else {
      std::vector<std::thread> pool;
      for (unsigned tt = 0; tt < nthr; ++tt) pool.emplace_back(work, tt);
      for (auto &th : pool) th.join();
    }
    int rc = dev_alloc(&h->d_fvtab, tab.size());
    if (!rc) rc = dev_alloc(&h->d_fvJbar, Jbar.size());
    if (!rc) rc = dev_alloc(&h->d_fvNf, Nf.size());
    if (!rc) rc = dev_alloc(&h->d_fvFx, (size_t)K * 30 * n2);
    if (!rc) rc = dev_alloc(&h->d_fvDx, (size_t)K * 30 * n2);
    if (!rc) rc = dev_alloc(&h->d_fvind, (size_t)K);
    if (!rc) rc = dev_alloc(&h->d_fvflag, (size_t)K);
    if (!rc) rc = dev_alloc(&h->d_fvlist, (size_t)K);
    if (!rc) rc = dev_alloc(&h->d_fvfaces, (size_t)3 * K);
    if (!rc) rc = dev_alloc(&h->d_fvcount, (size_t)2);
    if (rc) return fail(h, rc, "allocation of the finite-volume tables failed");
    bool ok = hipMemcpy(h->d_fvtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(h->d_fvJbar, Jbar.data(), Jbar.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(h->d_fvNf, Nf.data(), Nf.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(h->d_fvflag, 0, (size_t)K) == hipSuccess;
    if (!ok) return fail(h, DG_ERR_HIP, "upload of the finite-volume tables failed");
    h->fvg.V = h->d_fvtab; h->fvg.Vi = h->d_fvtab + n * n; h->fvg.Li = h->d_fvtab + 2 * n * n;
    h->fvg.Jbar = h->d_fvJbar; h->fvg.Nf = h->d_fvNf; h->fvg.flag = h->d_fvflag;
    h->fvg.Fx = h->d_fvFx; h->fvg.Dx = h->d_fvDx; h->fvg.ind = h->d_fvind;
    h->fvg.list = h->d_fvlist; h->fvg.faces = h->d_fvfaces; h->fvg.count = h->d_fvcount;
    h->fvg.w = (double)w;
    h->fv_on = true;
    // every element DG: empty work lists
    rc = fv_dispatch(h, 4, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, 0);
    if (!rc && hipStreamSynchronize(h->stream) != hipSuccess) rc = DG_ERR_HIP;
    if (rc) return fail(h, rc, "the finite-volume work lists failed");
  }
  h->fvg.limiter = limiter;
  h->fvg.lo = ind_lo;
  h->fvg.hi = ind_hi;
  return DG_OK;
}

int dg_fv_set_types(dg_handle *h, const uint8_t *types) {
  if (!h || !types) return DG_ERR_ARG;
  if (!h->fv_on) return fail(h, DG_ERR_ARG, "call dg_fv_enable first");
  std::vector<uint8_t> t(types, types + h->K);
  for (uint8_t &c : t)
    if (c > 1) return fail(h, DG_ERR_ARG, "element types are 0 (DG) or 1 (finite volume)");
  if (hipMemcpyAsync(h->d_fvflag, t.data(), t.size(), hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return fail(h, DG_ERR_HIP, "copy of the element types failed");
  const int rc = fv_dispatch(h, 4, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, 0);
  if (rc) return fail(h, rc, "the finite-volume work lists failed");
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, DG_ERR_HIP, "copy of the element types failed");
  return DG_OK;
}

int dg_fv_types(dg_handle *h, uint8_t *types) {
  if (!h || !types) return DG_ERR_ARG;
  if (!h->fv_on) return fail(h, DG_ERR_ARG, "call dg_fv_enable first");
  if (hipMemcpyAsync(types, h->d_fvflag, (size_t)h->K, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(h, DG_ERR_HIP, "copy of the element types failed");
  return DG_OK;
}

int dg_fv_indicator(dg_handle *h, const double *U, double *ind) {
  if (!h || !ind) return DG_ERR_ARG;
  if (!h->fv_on) return fail(h, DG_ERR_ARG, "call dg_fv_enable first");
  int rc = check_solution_ptr(h, U, "U");
  if (rc) return rc;
  rc = fv_dispatch(h, 2, U, nullptr, nullptr, 0.0, 0.0, 0.0, 0);
  if (rc) return fail(h, rc, "launch of the indicator failed");
  if (hipMemcpyAsync(ind, h->d_fvind, (size_t)h->K * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(h, DG_ERR_HIP, "copy of the indicator failed");
  return DG_OK;
}

int dg_fv_switch(dg_handle *h, double *U) {
  if (!h) return DG_ERR_ARG;
  if (!h->fv_on) return fail(h, DG_ERR_ARG, "call dg_fv_enable first");
  int rc = check_solution_ptr(h, U, "U");
  if (rc) return rc;
  rc = fv_dispatch(h, 3, U, nullptr, nullptr, 0.0, 0.0, 0.0, 0);
  if (rc) return fail(h, rc, "launch of the indicator failed");
  rc = fv_dispatch(h, 4, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, 0);
  if (rc) return fail(h, rc, "the finite-volume work lists failed");
  return DG_OK;
}

void dg_destroy(dg_handle *h) {
  if (!h) return;
  for (int i = 0; i < 5; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  (void)hipFree(h->d_Ja); (void)hipFree(h->d_sJ); (void)hipFree(h->d_fn); (void)hipFree(h->d_nbr);
  (void)hipFree(h->d_fc); (void)hipFree(h->d_tab);
  (void)hipFree(h->d_G); (void)hipFree(h->d_Gd); (void)hipFree(h->d_Gf); (void)hipFree(h->d_Utr);
  (void)hipFree(h->d_Wtr); (void)hipFree(h->d_Gtr); (void)hipFree(h->d_Pf); (void)hipFree(h->d_partial); (void)hipFree(h->d_red);
  (void)hipFree(h->d_md); (void)hipFree(h->d_mslot); (void)hipFree(h->d_mflux); (void)hipFree(h->d_mlift);
  (void)hipFree(h->d_mg);
  (void)hipFree(h->d_fvtab); (void)hipFree(h->d_fvJbar); (void)hipFree(h->d_fvNf); (void)hipFree(h->d_fvFx);
  (void)hipFree(h->d_fvDx); (void)hipFree(h->d_fvind); (void)hipFree(h->d_fvflag);
  (void)hipFree(h->d_fvlist); (void)hipFree(h->d_fvfaces); (void)hipFree(h->d_fvcount);
  delete h;
}

namespace {
// Ub (+)= scale (dL/dU)(U)^T Utb; Gin = lifted gradients of U if the caller kept them, else
// they are recomputed into the handle's scratch
int vjp_dispatch(dg_handle *h, const double *U, const double *Utb, double *Ub, double scale, int accumulate,
                 const double *Gin = nullptr, double *Rb = nullptr, double ra = 0.0, double rb = 0.0) {
  const bool weak_euler = h->sc.form == DG_FORM_WEAK && h->sc.eqn == DG_EULER;
  if (!weak_euler && (h->node_type != DG_NODES_LGL || h->sc.form != DG_FORM_SPLIT))
    return fail(h, DG_ERR_UNSUPPORTED,
                "the vector-Jacobian product is built for the split form on LGL nodes and the Euler weak form");
  if (h->nm)
    return fail(h, DG_ERR_UNSUPPORTED, "the vector-Jacobian product is built for conforming meshes");
  if (h->fv_on)
    return fail(h, DG_ERR_UNSUPPORTED, "the vector-Jacobian product is built for the DG operator");
  if (int rc = state_ready(h)) return rc;
  const bool ns = h->sc.eqn == DG_NAVIER_STOKES;
  if (ns && !h->d_Pf) {
    int rc = dev_alloc(&h->d_Pf, (size_t)h->K * 24 * h->n * h->n);
    if (rc) return fail(h, rc, "allocation of the lifting's face adjoint failed");
  }
  if (ns && !Gin) {
    int rc = lift_dispatch(h, U, 1, nullptr, h->d_G);  // forward lifting at U (the reverse needs Fv)
    if (rc) return fail(h, rc, "launch of the lifting kernel failed");
    Gin = h->d_G;
  }
  const dg::Geo g = h->geo();
  int rc;
  switch (h->N) {
#define DG_CASE(NN) \
  case NN: rc = dg::launch_vjp<NN>(g, h->ph, h->sc.eqn, h->sc.form, h->node_type == DG_NODES_LGL, U, Gin, h->d_Pf, \
                                   Utb, Ub, scale, accumulate, \
                                   ns ? Rb : nullptr, ra, rb, h->stream); break;
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: rc = DG_ERR_UNSUPPORTED;
  }
  if (rc) return fail(h, rc, rc == DG_ERR_UNSUPPORTED ? "vector-Jacobian product not built for this degree"
                                                      : "launch of the vector-Jacobian kernels failed");
  if (Rb && !ns) {
    rc = dg::launch_axpby(Rb, Ub, ra, rb, (size_t)h->K * 5 * h->n3, h->stream);
    if (rc) return fail(h, rc, "launch failed");
  }
  return DG_OK;
}
}  // namespace

int dg_rhs_vjp(dg_handle *h, const double *U, const double *Ut_bar, double *U_bar) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U, "U");
  if (!rc) rc = check_solution_ptr(h, Ut_bar, "Ut_bar");
  if (!rc) rc = check_solution_ptr(h, U_bar, "U_bar");
  if (rc) return rc;
  const size_t bytes = (size_t)h->K * 5 * h->n3 * sizeof(double);
  if (overlap(U, U_bar, bytes) || overlap(Ut_bar, U_bar, bytes))
    return fail(h, DG_ERR_ARG, "U_bar must not overlap U or Ut_bar");
  return vjp_dispatch(h, U, Ut_bar, U_bar, 1.0, 0);
}

int dg_rk_stage_vjp(dg_handle *h, const double *U_in, double *U_bar, double *R_bar, double a, double b, double dt) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U_in, "U_in");
  if (!rc) rc = check_solution_ptr(h, U_bar, "U_bar");
  if (!rc) rc = check_solution_ptr(h, R_bar, "R_bar");
  if (rc) return rc;
  const size_t n = (size_t)h->K * 5 * h->n3, bytes = n * sizeof(double);
  if (overlap(U_in, U_bar, bytes) || overlap(U_in, R_bar, bytes) || overlap(U_bar, R_bar, bytes))
    return fail(h, DG_ERR_ARG, "U_in, U_bar and R_bar must be three distinct buffers");
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(dt)) return fail(h, DG_ERR_ARG, "non-finite coefficient");
  // R_bar <- R_bar + b U_bar
  rc = dg::launch_axpby(R_bar, U_bar, 1.0, b, n, h->stream);
  if (rc) return fail(h, rc, "launch failed");
  // U_bar <- U_bar + dt (dL/dU)^T R_bar
  rc = vjp_dispatch(h, U_in, R_bar, U_bar, dt, 1);
  if (rc) return rc;
  // R_bar <- a R_bar
  rc = dg::launch_axpby(R_bar, R_bar, a, 0.0, n, h->stream);
  if (rc) return fail(h, rc, "launch failed");
  return DG_OK;
}

int dg_rk_stage_keep(dg_handle *h, const double *U_in, double *U_out, double *R, double a, double b, double dt,
                     double *G_out) {
  if (!h) return DG_ERR_ARG;
  int rc = check_solution_ptr(h, U_in, "U_in");
  if (!rc) rc = check_solution_ptr(h, U_out, "U_out");
  if (!rc) rc = check_solution_ptr(h, R, "R");
  if (rc) return rc;
  const bool ns = h->sc.eqn == DG_NAVIER_STOKES;
  if (ns && (!G_out || !aligned8(G_out))) return fail(h, DG_ERR_ARG, "G_out is NULL or not 8-byte aligned");
  const size_t bytes = (size_t)h->K * 5 * h->n3 * sizeof(double), gbytes = (size_t)h->K * 12 * h->n3 * sizeof(double);
  if (overlap(U_in, U_out, bytes) || overlap(U_in, R, bytes) || overlap(U_out, R, bytes))
    return fail(h, DG_ERR_ARG, "U_in, U_out and R must be three distinct buffers");
  if (ns && (overlap2(G_out, gbytes, U_in, bytes) || overlap2(G_out, gbytes, U_out, bytes) ||
             overlap2(G_out, gbytes, R, bytes)))
    return fail(h, DG_ERR_ARG, "G_out overlaps a solution buffer");
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(dt)) return fail(h, DG_ERR_ARG, "non-finite coefficient");
  rc = rhs_dispatch(h, U_in, U_out, R, a, b, dt, 1, ns ? G_out : nullptr);
  if (rc) return fail(h, rc, "launch of the operator failed");
  return DG_OK;
}

int dg_rk_steps_vjp(dg_handle *h, int nsteps, const double *const *stage_U, const double *const *stage_G,
                    double *U_bar, double *R_bar, double dt) {
  if (!h) return DG_ERR_ARG;
  if (nsteps < 1) return fail(h, DG_ERR_ARG, "nsteps must be positive");
  if (!stage_U) return fail(h, DG_ERR_ARG, "stage_U is NULL");
  int rc = check_solution_ptr(h, U_bar, "U_bar");
  if (!rc) rc = check_solution_ptr(h, R_bar, "R_bar");
  for (int s = 0; s < 5 * nsteps && !rc; ++s) rc = check_solution_ptr(h, stage_U[s], "stage_U[s]");
  if (rc) return rc;
  const size_t n = (size_t)h->K * 5 * h->n3, bytes = n * sizeof(double);
  if (overlap(U_bar, R_bar, bytes)) return fail(h, DG_ERR_ARG, "U_bar and R_bar overlap");
  for (int s = 0; s < 5 * nsteps; ++s)
    if (overlap(stage_U[s], U_bar, bytes) || overlap(stage_U[s], R_bar, bytes))
      return fail(h, DG_ERR_ARG, "a stage input overlaps U_bar or R_bar");
  if (!std::isfinite(dt)) return fail(h, DG_ERR_ARG, "non-finite time step");
  double A[5], B[5], C[5];
  dg_rk_coefficients(A, B, C);
  // R_bar <- R_bar + b_4 U_bar enters the last stage's reverse; after the reverse of stage s the
  // register update R_bar <- a_s R_bar is merged with the entry of the stage reversed next,
  // R_bar <- a_s R_bar + b_{s-1} U_bar (b_4 across a step boundary, nothing after the last),
  // and done by the reverse kernels themselves
  rc = dg::launch_axpby(R_bar, U_bar, 1.0, B[4], n, h->stream);
  if (rc) return fail(h, rc, "launch failed");
  for (int st = nsteps - 1; st >= 0; --st) {
    for (int s = 4; s >= 0; --s) {
      const int k = 5 * st + s;
      const double *Gs = (stage_G && stage_G[k]) ? stage_G[k] : nullptr;
      const double rb = s > 0 ? B[s - 1] : (st > 0 ? B[4] : 0.0);
      rc = vjp_dispatch(h, stage_U[k], R_bar, U_bar, dt, 1, Gs, R_bar, A[s], rb);
      if (rc) return rc;
    }
  }
  return DG_OK;
}

int dg_rk_step_vjp(dg_handle *h, const double *const *stage_U, const double *const *stage_G, double *U_bar,
                   double *R_bar, double dt) {
  return dg_rk_steps_vjp(h, 1, stage_U, stage_G, U_bar, R_bar, dt);
}



}  // extern "C"
