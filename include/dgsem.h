/*
 * dgsem.h -- C ABI of the MI355X (gfx950) DGSEM operator library, libdgsem.so.
 *
 * The library evaluates the semi-discrete discontinuous Galerkin spectral element
 * operator U -> U_t for the compressible Euler / Navier-Stokes equations on conforming
 * curvilinear hexahedra (Krais et al., "FLEXI", Sec. 3.1, eq. semiDiscrete; strong form
 * eq. semiDiscreteStrong; split form Sec. 3.3, eq. semiDiscreteSplit), with BR1 lifting of
 * the gradients (Sec. 3.1, eq. discreteGradient) and advances it with the two-register
 * low-storage Runge-Kutta scheme (Sec. 4.4).  Every step runs in HIP kernels on the GPU;
 * the host only validates arguments, builds the geometry once in dg_init and launches.
 *
 * Conventions shared by every entry point
 *  - Solution arrays are DEVICE pointers to FP64, owned by the caller, layout
 *    U[e][v][k][j][i] (i fastest), v = (rho, rho u, rho v, rho w, E), n = N+1 nodes per
 *    direction.  Element e's block of one variable is n^3 contiguous doubles.
 *  - Side numbering: side 2d is the face xi_d = -1, side 2d+1 the face xi_d = +1.
 *  - Calls are asynchronous and ordered on the HIP stream given to dg_init (or
 *    dg_set_stream), except the ones marked "synchronous".  A handle is not thread-safe.
 *  - Errors: every int-returning call returns a dg_status; nothing aborts or throws across
 *    the ABI.  Argument checks happen on the host before any launch; a HIP error is
 *    reported as DG_ERR_HIP.  dg_last_error() gives a readable message for the handle.
 *  - Inputs and outputs of one call must not overlap unless stated.
 */
#ifndef DGSEM_H
#define DGSEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_handle dg_handle; /* owns geometry, tables and scratch on the device */
typedef struct dg_batch dg_batch;   /* owns the work list of a batched launch        */

typedef enum {
  DG_OK = 0,
  DG_ERR_ARG = -1,         /* null/misaligned pointer, bad size, aliasing, bad enum value */
  DG_ERR_MESH = -2,        /* J <= 0 somewhere, or inconsistent connectivity               */
  DG_ERR_UNSUPPORTED = -3, /* valid request outside what the library implements           */
  DG_ERR_HIP = -4,         /* a HIP runtime call failed                                    */
  DG_ERR_NONFINITE = -5,   /* NaN or Inf found by dg_check_finite                          */
  DG_ERR_OOM = -6          /* device allocation failed                                     */
} dg_status;

/* interpolation / quadrature nodes (Sec. 3.1: LG or LGL) */
enum { DG_NODES_LG = 0, DG_NODES_LGL = 1 };
/* equation system (Sec. 3.1, eq. 3DconsLaw; viscous part via BR1) */
enum { DG_EULER = 0, DG_NAVIER_STOKES = 1 };
/* discretisation of the volume integral: weak (eq. semiDiscrete), split flux
 * differencing (eq. semiDiscreteSplit, LGL only), strong (eq. semiDiscreteStrong; on LG nodes
 * the interior flux of the surface term is the volume flux interpolated to the face) */
enum { DG_FORM_WEAK = 0, DG_FORM_SPLIT = 1, DG_FORM_STRONG = 2 };
/* two-point volume flux of the split form (Sec. 3.3): kinetic-energy preserving
 * (Pirozzoli), entropy conserving (Chandrashekar), or the mean of the two Euler fluxes */
enum { DG_VF_KEP = 0, DG_VF_EC = 1, DG_VF_CENTRAL = 2 };
/* convective surface flux (Sec. 2.2.3 names LLF and Roe; Sec. 3.3 allows the volume's
 * two-point flux, optionally with Roe-type dissipation) */
enum { DG_RS_LLF = 0, DG_RS_ROE = 1, DG_RS_VOLFLUX = 2, DG_RS_VOLFLUX_ROE = 3 };
/* kind of a boundary side (nbr_elem = -1; the kind goes in nbr_side).  DG_BC_SYMMETRY: a
 * symmetry plane or slip wall, whose outer state and gradient are the mirror images of the inner
 * ones across the face (velocity and, for the gradient, also the derivative direction reflected;
 * Sec. 2 lists slip walls among the boundary conditions).  DG_BC_STATE: a given outer state U_b
 * (far field, inflow; set with dg_set_boundary_state), whose outer viscous flux is taken equal
 * to the inner one.  DG_BC_WALL: a no-slip adiabatic wall (Sec. 2): outer state with the
 * velocity reversed, outer gradient with the velocity gradient kept and the temperature
 * gradient mirrored, so the surface means give zero velocity, no work and no heat flux.
 * DG_BC_WALL_ISOTHERMAL: a no-slip wall at temperature T_w (set with dg_set_wall_temperature):
 * the same outer state, outer (u, v, w, T) = (-u, -v, -w, 2 T_w - T), outer gradient equal to
 * the inner one, so the means give zero velocity, T_w, no work, and the inner heat flux.
 * DG_BC_OUTFLOW: a subsonic pressure outflow: outer state with the inner
 * density and velocity and the pressure p_out (set with dg_set_outflow_pressure), outer viscous
 * flux equal to the inner one. */
enum { DG_BC_SYMMETRY = 0, DG_BC_STATE = 1, DG_BC_WALL = 2, DG_BC_WALL_ISOTHERMAL = 3, DG_BC_OUTFLOW = 4 };

typedef struct {
  int32_t n_elems;         /* K >= 1                                                        */
  int32_t n_geo;           /* polynomial degree N_geo of the geometry, 1..16, independent of N
                              (Sec. 2.1); the mapping is interpolated to the degree-N LGL nodes,
                              where the curl-form metrics are taken                          */
  const double *xgeo;      /* HOST [K][3][(n_geo+1)^3] physical coordinates at the LGL nodes
                              of degree n_geo (node i + n*(j + n*k))                         */
  const int32_t *nbr_elem; /* HOST [K][6] element across each side, -1 on a boundary side     */
  const int8_t *nbr_side;  /* HOST [K][6] side of that neighbour the face lies on, 0..5; on a
                              boundary side the boundary kind (DG_BC_SYMMETRY)                 */
  const int8_t *flip;      /* HOST [K][6] orientation code 0..7 of each face, NULL = all 0
                              (0 on boundary sides)                                            */
  const int8_t *mortar;    /* HOST [K][6] non-conforming faces (Sec. 3.2), NULL = none: 0 a
                              conforming side; 1, 2, 3 the big side of a face cut in half along
                              its first face direction, its second, or both (its nbr_elem -1,
                              nbr_side and flip 0); 4 + p the small side at position p of such a
                              face (p along the cut; p1 + 2 p2 for type 3), whose nbr_elem and
                              nbr_side name the big element and side and whose flip maps its face
                              points onto the big side's sub-face p                            */
} dg_mesh;
/* Faces of conforming meshes (Sec. 5.1: each face has a master and a slave side).  Side 2d is
 * the face xi_d = -1 and side 2d+1 the face xi_d = +1 of direction d.  Face point (a,b) of a
 * side is the node at the face's position along d whose indices along the other two
 * directions, in increasing direction order, are a and b.  flip[e][s] = o maps face point (a,b)
 * of side s of element e to the neighbour's matching face point: swap (a,b) if o & 4, then
 * reverse the first index (x -> N - x) if o & 1 and the second if o & 2.  The neighbour must
 * name e back, on side s, with the inverse code (o itself, or o with bits 0 and 1 exchanged
 * when o & 4), and the matched face points must coincide up to one translation per face (a
 * periodic shift): otherwise DG_ERR_MESH.  The master of a face is the +xi side where a +xi
 * side meets a -xi side, else the element with the smaller index (the smaller side within one
 * element); normals and surface elements are the master's; a boundary side is its own master.
 * A mesh without boundary sides whose every face meets the opposite side with code 0 is
 * structured.  Errors:
 * an unknown boundary kind is DG_ERR_UNSUPPORTED; a neighbour index out of
 * range (other than -1) is DG_ERR_MESH. */

typedef struct {
  int32_t eqn, form, volflux, riemann; /* enums above                                      */
  double gamma;                        /* ratio of specific heats (> 1)                    */
  double R;                            /* gas constant (> 0), T = p/(rho R)                */
  double mu;                           /* dynamic viscosity (>= 0, Navier-Stokes only)     */
  double Pr;                           /* Prandtl number (> 0)                             */
} dg_scheme;

/* Reference nodes and quadrature weights of degree N (n = N+1 values each), host arrays.
 * Sec. 3.1: roots of P_{N+1} (LG) or +-1 and the roots of P_N' (LGL).  Synchronous. */
int dg_nodes(int N, int node_type, double *x, double *w);

/* Carpenter-Kennedy 5-stage 4th-order 2N-storage coefficients a[5], b[5], c[5] (host). */
int dg_rk_coefficients(double *a, double *b, double *c);

/* Build the operator for a mesh (Sec. 3.1: metric terms in curl form, eq.
 * contravariantBasisVectorsCurl; Jacobian; face normals and surface elements from the
 * master side, Sec. 5.1).  Mesh arrays are copied; they may be freed on return.
 * Supported: 1 <= N <= 8, conforming meshes (faces on any side and in any orientation,
 * symmetry-plane, given-state, adiabatic and isothermal wall, and pressure-outflow
 * boundaries; see dg_mesh).  hip_stream is a
 * hipStream_t (NULL = default stream).  Synchronous.  On error *out is NULL. */
int dg_init(const dg_mesh *mesh, int N, int node_type, const dg_scheme *scheme, void *hip_stream,
            dg_handle **out);

/* Mesh preprocessing (Sec. 5.1: the element-to-side connectivity and face orientations a mesh
 * file carries): derives nbr_elem, nbr_side and flip of a conforming hexahedral mesh from its
 * element coordinates alone, in the conventions of dg_mesh.  xgeo is as in dg_mesh (HOST
 * [K][3][(n_geo+1)^3]).  Two faces match when each corner of one lies within tol of a corner of
 * the other (tol <= 0: 1e-8 of the smallest element extent); along every direction d with
 * period[d] > 0 (period may be NULL) coordinates are compared modulo period[d], which joins the
 * opposite faces of a periodic box.  Faces without a match become boundary sides (nbr_elem -1,
 * nbr_side = bc_kind, flip 0).  Outputs are HOST [K][6] arrays owned by the caller.  Host only,
 * synchronous; DG_ERR_ARG for NULL or non-finite input, degenerate (flat) elements, a negative
 * period or an unknown bc_kind.  dg_init validates the result like any other connectivity. */
int dg_mesh_connect(int n_elems, int n_geo, const double *xgeo, const double period[3], double tol, int bc_kind,
                    int32_t *nbr_elem, int8_t *nbr_side, int8_t *flip);

/* Element-package mesh files (Sec. 2.1.1: per element one package of its side connectivity,
 * conforming and non-conforming, and of its nodes' global indices and positions, so that any
 * contiguous range of elements is one contiguous part of the file and is read on its own; a
 * physical node shared by several elements is stored with each and tied by its global index).
 * This library's own little-endian layout: a 64-byte header (magic "DGSEMMSH", int32 version 1,
 * int32 n_geo, int64 K, int32 flags: bit 0 = mortar kinds present), then per element
 * int64 node index [n^3], float64 coordinates [3][n^3], and 6 side records {int32 neighbour
 * element, int8 neighbour side or boundary kind, int8 orientation code, int8 mortar kind, int8 0}
 * in the conventions of dg_mesh.  Host only, synchronous; DG_ERR_ARG for I/O errors, a foreign
 * or damaged file, or a range beyond the file.
 * dg_mesh_file_write: writes K packages (flip and mortar may be NULL: zeros, no mortar flag).
 * dg_mesh_file_info : out = {K, n_geo, flags}.
 * dg_mesh_file_read : elements first .. first+count-1 into caller arrays laid out as in dg_mesh
 *                     (xgeo [count][3][n^3], node_id [count][n^3], the side arrays [count][6]; any
 *                     may be NULL); the neighbour indices are global element indices. */
int dg_mesh_file_write(const char *path, int n_elems, int n_geo, const double *xgeo, const int64_t *node_id,
                       const int32_t *nbr_elem, const int8_t *nbr_side, const int8_t *flip, const int8_t *mortar);
int dg_mesh_file_info(const char *path, int64_t out[3]);
int dg_mesh_file_read(const char *path, int64_t first, int count, double *xgeo, int64_t *node_id, int32_t *nbr_elem,
                      int8_t *nbr_side, int8_t *flip, int8_t *mortar);

/* Conforming connectivity from the global node indices of a mesh file, exactly (no tolerance):
 * two sides whose four corner nodes have the same indices are one face, their orientation codes
 * follow from the corners' order; a side no other side matches becomes a boundary of kind
 * bc_kind (periodic faces, whose nodes differ, must come from the file's side records).
 * node_id HOST [K][(n_geo+1)^3]; outputs HOST [K][6].  DG_ERR_MESH where more than two sides share
 * a face or two matched faces admit no orientation; DG_ERR_ARG for bad arguments. */
int dg_mesh_connect_nodes(int n_elems, int n_geo, const int64_t *node_id, int bc_kind, int32_t *nbr_elem,
                          int8_t *nbr_side, int8_t *flip);

/* Element order along a space-filling curve (Secs. 2.1.1 and 5.2: elements are stored in the
 * order of a space-filling curve, so neighbours are near in memory and in the launch order): order[i]
 * is the element (index into xgeo, HOST [K][3][(n_geo+1)^3]) at position i of the 3-D Hilbert
 * curve through the element centroids.  Renumbering a mesh by it is the caller's (the
 * connectivity arrays refer to element indices).  Host only, synchronous; DG_ERR_ARG for NULL
 * or non-finite input. */
int dg_mesh_sfc_order(int n_elems, int n_geo, const double *xgeo, int32_t *order);

/* The setup dg_init performs, on the host only (no device memory is touched): metric terms
 * Ja [K][9][n^3] (Ja^i_d at i*3+d), J [K][n^3], outward face normals fn [K][6][3][n^2] and the
 * n x n matrices D and Dhat, all host arrays (any may be NULL).  All tables are computed in
 * extended precision and rounded once to double.  For inspection and tests.  Synchronous. */
int dg_host_geometry(const dg_mesh *mesh, int N, int node_type, double *Ja, double *J, double *fn, double *D,
                     double *Dhat);

/* Change the stream later calls are ordered on. */
int dg_set_stream(dg_handle *h, void *hip_stream);

/* Outer state U_b = (rho, rho u, rho v, rho w, E) of the DG_BC_STATE sides (host array of 5).
 * Must be called before the first operator, stage or vector-Jacobian call on a mesh that has
 * such sides (those return DG_ERR_ARG until then) and before the handle joins a batch; may be
 * called again to change the state.  DG_ERR_ARG if rho or the pressure is not positive or a
 * value is not finite.  Synchronous (host only). */
int dg_set_boundary_state(dg_handle *h, const double ub[5]);

/* Wall temperature T_w (> 0, finite; else DG_ERR_ARG) of the DG_BC_WALL_ISOTHERMAL sides.  The
 * same rules as for dg_set_boundary_state: required before launching calls on a mesh with such
 * sides, may be changed later.  Synchronous (host only). */
int dg_set_wall_temperature(dg_handle *h, double T_w);

/* Pressure p_out (> 0, finite; else DG_ERR_ARG) of the DG_BC_OUTFLOW sides, with the same rules
 * as dg_set_boundary_state.  Synchronous (host only). */
int dg_set_outflow_pressure(dg_handle *h, double p_out);

/* U_t = L(U) (eq. semiDiscrete / semiDiscreteStrong / semiDiscreteSplit, BR1 lifting for
 * Navier-Stokes).  U, Ut: device [K][5][n^3]; Ut is overwritten; U and Ut must differ. */
int dg_rhs(dg_handle *h, const double *U, double *Ut);

/* One stage of the 2N-storage Runge-Kutta scheme (Sec. 4.4):
 *   R <- a*R + dt*L(U_in);   U_out <- U_in + b*R.
 * U_in, U_out, R: device [K][5][n^3].  U_in == U_out is rejected (DG_ERR_ARG): neighbours
 * read the old face values of U_in during the stage.  R is read and written in place. */
int dg_rk_stage(dg_handle *h, const double *U_in, double *U_out, double *R, double a, double b, double dt);

/* Vector-Jacobian product of the operator: U_bar = (dL/dU)(U)^T Ut_bar (overwritten).
 * Supported for the split form on LGL nodes (KEP, EC or central volume flux; Euler or
 * Navier-Stokes) and for the weak form of the Euler equations on LG or LGL nodes, on every
 * conforming mesh dg_init accepts, without finite-volume subcells, N = 1..8 (DG_ERR_UNSUPPORTED
 * otherwise); the derivative of |x| at 0 and of max at a tie is the mean of the
 * one-sided derivatives, the log means of the EC flux are differentiated with the forward's
 * branch threshold (series below ((a-b)/(a+b))^2 = 1e-4, logarithms above).  Device arrays [K][5][n^3], pairwise distinct.
 * Not in the paper: the reverse of its operator, for gradients of objectives of U. */
int dg_rhs_vjp(dg_handle *h, const double *U, const double *Ut_bar, double *U_bar);

/* Reverse of dg_rk_stage at the stage input U_in.  On entry U_bar, R_bar hold the
 * adjoints of (U_out, R after the stage); on return they hold the adjoints of
 * (U_in, R before the stage):
 *   R_bar <- R_bar + b*U_bar;  U_bar <- U_bar + dt*(dL/dU)(U_in)^T R_bar;  R_bar <- a*R_bar.
 * Not in the paper: the transpose of one stage of its low-storage Runge-Kutta scheme (Sec. 4.4). */
int dg_rk_stage_vjp(dg_handle *h, const double *U_in, double *U_bar, double *R_bar, double a, double b, double dt);

/* dg_rk_stage that also keeps the lifting output of U_in in G_out (Navier-Stokes: device
 * [K][12][n^3], caller-owned, distinct from the solution buffers; ignored for Euler): for the split
 * form the contravariant viscous fluxes (F^v . Ja^dir), dir*4 + (momentum x, y, z, energy), for the
 * other forms the gradients of (u, v, w, T), d*4 + c.  A reverse sweep over recomputed stages
 * then need not lift again. */
int dg_rk_stage_keep(dg_handle *h, const double *U_in, double *U_out, double *R, double a, double b, double dt,
                     double *G_out);

/* Reverse of one full step of the five-stage scheme of dg_rk_coefficients with time step dt.
 * stage_U[s] (s = 0..4) is the input of stage s; stage_G[s] its lifting output from
 * dg_rk_stage_keep, or NULL (the array or an entry) to recompute it.  On entry U_bar and R_bar
 * hold the adjoints of the step's output state and R; on return those of its input state and
 * of R before the step (zero, as the first stage does not read R).  Same result as the five
 * dg_rk_stage_vjp calls in reverse order, with the register updates of neighbouring stages
 * merged. */
int dg_rk_step_vjp(dg_handle *h, const double *const *stage_U, const double *const *stage_G, double *U_bar,
                   double *R_bar, double dt);

/* Reverse of nsteps >= 1 consecutive steps: stage_U[5*k + s] (and stage_G[5*k + s], or NULL)
 * belong to stage s of the k-th step, in forward order; the steps are reversed from the last.
 * On entry U_bar and R_bar hold the adjoints of the last step's output state and R; on return
 * U_bar holds the adjoint of the first step's input state and R_bar is zero.  Same result, bit
 * for bit, as nsteps dg_rk_step_vjp calls from the last step to the first (the register update
 * between two steps is merged into the reverse kernels, since a_1 = 0 leaves R_bar zero after
 * every reversed step).  DG_ERR_ARG for nsteps < 1, NULL or overlapping arrays or a non-finite
 * dt; the reverse kernels support what dg_rhs_vjp supports (DG_ERR_UNSUPPORTED otherwise).
 * Not in the paper: the reverse of its time integration. */
int dg_rk_steps_vjp(dg_handle *h, int nsteps, const double *const *stage_U, const double *const *stage_G,
                    double *U_bar, double *R_bar, double dt);

/* Largest stable step (eqs. CFLCondition and DFLCondition with gamma_RK = 1, evaluated per
 * reference direction from the metric terms).  Synchronous; result in *dt_out (host). */
int dg_timestep(dg_handle *h, const double *U, double cfl, double dfl, double *dt_out);

/* Quadrature integrals sum_e sum_ijk J w_i w_j w_k X over the mesh (the collocated quadrature
 * of the time-derivative term, Sec. 3.1 eq. discTemp), synchronous, host
 * out[8] = {rho, rho u, rho v, rho w, E, kinetic energy, entropy -rho s/(gamma-1), min J}. */
int dg_integrals(dg_handle *h, const double *U, double out[8]);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the integrals of dg_integrals written to the DEVICE array
 * out_dev[8] (same order, same values bit for bit), asynchronous on the handle's stream.  Calls
 * no hipMalloc, hipFree or allocating routine: the per-element partial sums go to a static
 * device buffer of 2^20 doubles per GPU (8 per element, so at most 131072 elements; larger
 * meshes get DG_ERR_UNSUPPORTED), which each GPU holds until the process ends.  All calls on
 * one GPU share that buffer: calls that overlap in time on one GPU race.  DG_ERR_ARG for NULL
 * or misaligned pointers. */
int dg_integrals_noalloc(dg_handle *h, const double *U, double *out_dev);

/* DG_ERR_NONFINITE if any entry of U is NaN or Inf, DG_OK otherwise.  Synchronous.  Not in the
 * paper: a guard a time loop may call between steps (a blown-up solution is NaN after a few). */
int dg_check_finite(dg_handle *h, const double *U);

/* Quadrature weight of every node, J w_i w_j w_k (the diagonal mass matrix of Sec. 3.1,
 * eq. discTemp), written to the DEVICE array out [K][n^3]. */
int dg_mass_weights(dg_handle *h, double *out);

/* Physical coordinates of the solution nodes, HOST out [K][3][n^3].  Synchronous. */
int dg_node_coords(dg_handle *h, double *x_host);

/* Sizes: out[0] = K, out[1] = N, out[2] = n^3, out[3] = node type. */
int dg_info(const dg_handle *h, int64_t out[4]);

/* Per-kernel timing for performance reports.  With enable != 0 every later dg_rhs /
 * dg_rk_stage records HIP events around the lifting and the main kernel on the handle's
 * stream and waits for them (so calls become synchronous); dg_profile also clears the
 * counters.  dg_profile_read gives {lifting ms, lifting launches, main-kernel ms,
 * main-kernel launches} accumulated since the last dg_profile call. */
int dg_profile(dg_handle *h, int enable);
int dg_profile_read(const dg_handle *h, double out[4]);
/* The same with the kernels of non-conforming faces and finite-volume subcells apart: up to cap
 * of {lifting ms (with the mortars' lifting kernel), launches, operator-kernel ms, launches,
 * face-kernel ms (mortar fluxes, DG/FV faces), launches, finite-volume-kernel ms, launches}. */
int dg_profile_read_ex(const dg_handle *h, double *out, int cap);

/* ---- hybrid DG / finite-volume subcells (Sec. 4: shock capturing) ------------------------
 * A troubled element is advanced by a finite-volume scheme on (N+1)^3 equal subcells of width
 * w = 2/(N+1) in reference space; its entries of every solution array then hold the subcell
 * means of U instead of nodal values (the same storage, eq. dg2fv: U_FV = V U with V the
 * subcell-mean matrix of eq. FVvdm applied along the three directions).  Subcell fluxes use the
 * handle's Riemann solver with a second-order reconstruction of (rho, u, v, w, p) limited per
 * direction; at a face between a DG and an FV element the DG trace is taken to the subcell faces
 * with V, the flux applied to the subcells as is and to the DG nodes through V^-1 (Sec. 4.2).
 * The metric terms of a subcell face are the means of Ja over that face, Jbar the subcell mean of
 * J.  Supported: the Euler equations on meshes without boundary sides or non-conforming faces
 * (DG_ERR_UNSUPPORTED otherwise), every form and node type of the DG operator.
 * dg_fv_enable     : builds the subcell geometry (synchronous, once) and sets the limiter (0 first
 *                    order, 1 minmod, 2 van Leer) and the thresholds of the indicator (lo <= hi).
 *                    Every element starts as DG; afterwards dg_rhs, dg_rk_stage and
 *                    dg_rk_stage_keep evaluate the hybrid operator.  May be called again to change
 *                    the limiter and thresholds.
 * dg_fv_set_types  : element types from a HOST array [K] (0 DG, 1 FV) without converting U.
 * dg_fv_types      : the current types into a HOST array [K].  Synchronous.
 * dg_fv_indicator  : the troubled-cell indicator of every element (Sec. 4.3; modal decay of
 *                    rho p in the orthonormal Legendre basis, log10 max(E_N/E, E_{N-1}/E_{<N}),
 *                    FV elements read through V^-1) into a HOST array [K].  Synchronous.
 * dg_fv_switch     : the indicator and the switch with hysteresis (Fig. fv:indicator): DG
 *                    elements above hi become FV (U <- V U), FV elements below lo become DG
 *                    (U <- V^-1 U), in place on the DEVICE array U.  Asynchronous.
 * dg_integrals and dg_timestep treat every element as DG. */
int dg_fv_enable(dg_handle *h, int limiter, double ind_lo, double ind_hi);
int dg_fv_set_types(dg_handle *h, const uint8_t *types);
int dg_fv_types(dg_handle *h, uint8_t *types);
int dg_fv_indicator(dg_handle *h, const double *U, double *ind);
int dg_fv_switch(dg_handle *h, double *U);

void dg_destroy(dg_handle *h);
const char *dg_status_string(int status);
const char *dg_last_error(const dg_handle *h);

/* ---- batched ensembles ------------------------------------------------------------------
 * Not in the paper: advances many independent handles together so that small meshes fill the
 * GPU.  Every member keeps its own mesh, degree N, viscosity (mu, Pr) and time step; all members
 * share the equations, the volume flux and the Riemann solver, and use the split form on LGL
 * nodes.  A stage launches, for each degree present, one lifting kernel (Navier-Stokes) and one
 * operator kernel over the concatenated elements of all members of that degree, on the stream
 * of members[0] (read at every call).  Members are referenced, not copied: they must outlive
 * the batch, and their gradient scratch is used by the batch's kernels.  Arrays passed below
 * have one entry per member, in the order given to dg_batch_create.
 *
 * dg_batch_create  -> DG_ERR_UNSUPPORTED if a member is not split/LGL, has non-conforming faces or
 *                     finite-volume subcells enabled, or the schemes differ;
 *                     DG_ERR_ARG for NULL entries, a member listed twice, or a member with
 *                     given-state boundary sides whose state is not set.  Members may have
 *                     any mesh dg_init accepts; a later dg_set_boundary_state on a member is
 *                     seen by the next batched call.
 * dg_batch_rk_stage: for every member i, dg_rk_stage(member i, U_in[i], U_out[i], R[i], a[i],
 *                     b_coef[i], dt[i]) (same semantics: a = 0 does not read R; the three
 *                     buffers must be distinct).  Asynchronous.  Descriptor tables of the
 *                     distinct argument sets seen are uploaded once (first use of a set is
 *                     synchronous) and cached (at most 64).
 * dg_batch_step    : one full step of the five-stage scheme of dg_rk_coefficients for every
 *                     member: reads U[i], leaves the new state in U_out[i]; U[i] (overwritten
 *                     with the fourth stage) and R[i] are working storage.  use_graph != 0
 *                     captures the five stages into a HIP graph on first use of an argument set
 *                     and replays it afterwards (ordered after the caller's queued work on the
 *                     members[0] stream, and later work on that stream after it).
 * dg_batch_tune    : times every elements-per-workgroup choice (1, 2, 4 as built for the
 *                     degree) of both kernels of every degree on the states U (read only;
 *                     repeats launches per choice, scratch outputs allocated and freed here) and
 *                     keeps the fastest.  Synchronous.  Without it every choice is 1.
 *                     Where one launch can cover every degree (all N <= 7, no member with face
 *                     codes, at most 8 degrees), it then also times one stage of all members
 *                     with the per-degree launches against one lifting and one operator launch
 *                     for all degrees (512-lane workgroups of the degree's elements, the
 *                     largest degree's LDS) and keeps the faster; the results are the same bits.
 * dg_batch_set_tile: fixes the choices of degree N by hand.
 * dg_batch_set_fused: 1 selects the single pair of launches per stage, 0 the per-degree
 *                     launches (DG_ERR_UNSUPPORTED where one launch cannot cover every degree).
 * dg_batch_fused   : the current choice (0 or 1).
 * dg_batch_info    : writes N, members, elements, elements per workgroup of the lifting and of
 *                     the operator kernel for each degree present (5 ints each, up to cap ints)
 *                     and returns the number of degrees. */
int dg_batch_create(dg_handle *const *members, int n_members, dg_batch **out);
int dg_batch_rk_stage(dg_batch *b, const double *const *U_in, double *const *U_out, double *const *R,
                      const double *a, const double *b_coef, const double *dt);
int dg_batch_step(dg_batch *b, double *const *U, double *const *U_out, double *const *R, const double *dt,
                  int use_graph);
int dg_batch_tune(dg_batch *b, const double *const *U, int repeats);
int dg_batch_set_tile(dg_batch *b, int N, int epb_lift, int epb_main);
int dg_batch_set_fused(dg_batch *b, int fused);
int dg_batch_fused(const dg_batch *b);
int dg_batch_info(const dg_batch *b, int *out, int cap);
const char *dg_batch_last_error(const dg_batch *b);
void dg_batch_destroy(dg_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* DGSEM_H */
