"""Pins of the oracle's full operator (Sec. 3.1 / 3.3 / 4.4) against what the method fixes.

Free-stream preservation on curved meshes, discrete conservation, weak = strong on LGL,
split(central) = strong on affine meshes, zero entropy production of the entropy-
conserving scheme, BR1 exactness for piecewise polynomials, the viscous dissipation rate
of the Taylor-Green vortex, convergence order N+1 on exact solutions, the RK time order,
a brute-force evaluation of the weak form with explicit basis functions, and the dual-
number tangent against finite differences.
"""
import math

import numpy as np
import pytest

from paper_1910_02858_amd import inputs

GAMMA = 1.4


def _mesh(orc, k, N, nodes, curved, kxyz=None, box=None):
    lgl = orc.basis(N, "lgl")["x"]
    kx, ky, kz = kxyz if kxyz else (k, k, k)
    X = inputs.lattice_points(lgl, kx, ky, kz, **({"box": box} if box else {}))
    xg = inputs.warp_sine(X) if curved else X
    nbr, side, _ = inputs.periodic_lattice(kx, ky, kz)
    return orc.OracleMesh(xg, nbr, side, N, nodes)


def _wq(orc, M):
    w = orc.basis(M.N, M.nodes)["w"]
    return np.einsum("k,j,i->kji", w, w, w).ravel()[None, :] * M.geometry()["J"]


SCHEMES = [
    ("euler", "weak", "central", "llf", "lg"),
    ("euler", "weak", "central", "roe", "lgl"),
    ("euler", "split", "ec", "roe", "lgl"),
    ("euler", "split", "kep", "volflux_roe", "lgl"),
    ("ns", "weak", "central", "llf", "lg"),
    ("ns", "split", "kep", "roe", "lgl"),
    ("ns", "split", "ec", "llf", "lgl"),
    ("ns", "strong", "central", "roe", "lgl"),
    ("euler", "strong", "central", "llf", "lg"),
    ("ns", "strong", "central", "roe", "lg"),
]


def _flux_scale(M, U, k):
    F = np.abs(U).max() * 2.0
    h = 2 * math.pi / k
    return F * (M.N + 1) ** 2 / h


@pytest.mark.parametrize("eqn,form,vf,rs,nodes", SCHEMES)
def test_freestream_curved(orc, eqn, form, vf, rs, nodes):
    k, N = 3, 4
    M = _mesh(orc, k, N, nodes, True)
    sc = orc.Scheme(eqn, form, vf, rs, mu=1e-2)
    U = inputs.constant_state(M.K, M.n3)
    Ut = M.rhs(sc, U)
    # tolerance: rounding of the metric identities, 1e-12 of the flux scale |F| (N+1)^2 / h
    assert np.abs(Ut).max() < 1e-12 * _flux_scale(M, U, k)


@pytest.mark.parametrize("eqn,form,vf,rs,nodes", SCHEMES)
def test_conservation_curved(orc, eqn, form, vf, rs, nodes):
    k, N = 3, 3
    M = _mesh(orc, k, N, nodes, True)
    sc = orc.Scheme(eqn, form, vf, rs, mu=5e-2)
    U = inputs.random_perturbation(inputs.taylor_green(M.points(), 1.0, 0.3), 5, 1e-2)
    Ut = M.rhs(sc, U)
    wq = _wq(orc, M)
    tot = np.einsum("eq,evq->v", wq, Ut)
    scale = np.einsum("eq,evq->v", wq, np.abs(Ut))
    assert np.all(np.abs(tot) < 1e-13 * scale)


@pytest.mark.parametrize("nodes", ["lgl", "lg"])
@pytest.mark.parametrize("curved", [False, True])
@pytest.mark.parametrize("eqn", ["euler", "ns"])
def test_weak_equals_strong(orc, eqn, curved, nodes):
    """Sec. 3.1: weak and strong forms agree discretely on LGL nodes, and on LG nodes when the
    strong form's interior surface flux is the volume flux interpolated to the face (the
    summation-by-parts property MD + (MD)^T = l(1)l(1)^T - l(-1)l(-1)^T holds for both)."""
    M = _mesh(orc, 3, 4 if nodes == "lgl" else 3, nodes, curved)
    U = inputs.random_perturbation(inputs.taylor_green(M.points(), 1.0, 0.3), 6, 1e-2)
    a = M.rhs(orc.Scheme(eqn, "weak", "central", "roe", mu=1e-2), U)
    b = M.rhs(orc.Scheme(eqn, "strong", "central", "roe", mu=1e-2), U)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("curved", [False, True])
def test_kinetic_energy_preservation_constant_pressure(orc, curved):
    """Split form with a two-point flux whose momentum part is {u} F_rho + p~ n (Jameson's
    kinetic-energy-preserving structure; both the Pirozzoli and the Chandrashekar flux have it,
    and p~ = p when the pressure is uniform), no surface dissipation, periodic mesh, uniform
    pressure, arbitrary density and velocity: the discrete kinetic energy rate
    sum J w (u . m_t - |u|^2/2 rho_t) vanishes to rounding.  The mean of the Euler fluxes lacks
    that structure and produces kinetic energy."""
    M = _mesh(orc, 3, 4, "lgl", curved)
    rng = np.random.default_rng(21)
    K, n3 = M.K, M.n3
    rho = 1.0 + 0.4 * rng.random((K, n3))
    u = rng.standard_normal((K, 3, n3))
    p = 2.0
    U = np.zeros((K, 5, n3))
    U[:, 0] = rho
    U[:, 1:4] = rho[:, None] * u
    U[:, 4] = p / (GAMMA - 1) + 0.5 * rho * (u * u).sum(axis=1)
    wq = _wq(orc, M)
    rates = {}
    for vf in ("kep", "ec", "central"):
        Ut = M.rhs(orc.Scheme("euler", "split", vf, "volflux"), U)
        dke = (u * Ut[:, 1:4]).sum(axis=1) - 0.5 * (u * u).sum(axis=1) * Ut[:, 0]
        scale = np.sum(wq * (np.abs(u * Ut[:, 1:4]).sum(axis=1) + 0.5 * (u * u).sum(axis=1) * np.abs(Ut[:, 0])))
        rates[vf] = abs(np.sum(wq * dke)) / scale
    assert rates["kep"] < 1e-13 and rates["ec"] < 1e-13, rates
    assert rates["central"] > 1e-4, rates


def test_split_central_equals_strong_affine(orc):
    M = _mesh(orc, 3, 5, "lgl", False)
    U = inputs.random_perturbation(inputs.taylor_green(M.points(), 1.0, 0.3), 7, 1e-2)
    a = M.rhs(orc.Scheme("ns", "split", "central", "llf", mu=1e-2), U)
    b = M.rhs(orc.Scheme("ns", "strong", "central", "llf", mu=1e-2), U)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("curved", [False, True])
def test_entropy_conservation(orc, curved):
    """EC volume flux + EC surface flux: sum J w (w(U) . U_t) = 0; with Roe dissipation <= 0."""
    M = _mesh(orc, 3, 4, "lgl", curved)
    U = inputs.random_perturbation(inputs.taylor_green(M.points(), 1.0, 0.3), 8, 5e-2)
    Ut = M.rhs(orc.Scheme("euler", "split", "ec", "volflux"), U)
    ep = M.entropy_production(U, Ut)
    scale = np.sum(_wq(orc, M) * np.abs(Ut).sum(axis=1)) * 10
    assert abs(ep) < 1e-13 * scale
    for rs in ("roe", "volflux_roe", "llf"):
        Ut = M.rhs(orc.Scheme("euler", "split", "ec", rs), U)
        assert M.entropy_production(U, Ut) < -1e-6 * scale


def _tent(x, h):
    """periodic continuous piecewise-linear function with kinks at element faces"""
    t = np.mod(x, 2 * h) / h
    return np.where(t < 1, t, 2 - t)


def _tent_d(x, xmid, h):
    """derivative of the tent inside the element whose centre is xmid"""
    t = np.mod(xmid, 2 * h) / h
    return np.where(t < 1, 1.0 / h, -1.0 / h)


@pytest.mark.parametrize("nodes", ["lg", "lgl"])
def test_br1_exact_for_continuous_piecewise_polynomials(orc, nodes):
    k, N = 4, 3
    M = _mesh(orc, k, N, nodes, False)
    x = M.points()
    h = 2 * math.pi / k
    xc = x.mean(axis=2, keepdims=True)
    T = [_tent(x[:, d], h) for d in range(3)]
    dT = [np.broadcast_to(_tent_d(x[:, d], xc[:, d], h), T[0].shape) for d in range(3)]
    # W = (u, v, w, T): products of tents (degree <= 1 per direction, continuous everywhere)
    u = 0.1 * T[0] * T[1]
    v = -0.2 * T[1] * T[2]
    w = 0.05 * T[0] * T[2]
    Tt = 1.0 + 0.1 * T[0] * T[1] * T[2]
    grads = {
        0: [0.1 * dT[0] * T[1], 0.1 * T[0] * dT[1], 0 * T[0]],
        1: [0 * T[0], -0.2 * dT[1] * T[2], -0.2 * T[1] * dT[2]],
        2: [0.05 * dT[0] * T[2], 0 * T[0], 0.05 * T[0] * dT[2]],
        3: [0.1 * dT[0] * T[1] * T[2], 0.1 * T[0] * dT[1] * T[2], 0.1 * T[0] * T[1] * dT[2]],
    }
    rho = np.ones_like(u)
    p = rho * Tt  # R = 1
    U = inputs.prim_to_cons(rho, u, v, w, p, GAMMA)
    G = M.lift(U, GAMMA, 1.0).reshape(M.K, 3, 4, M.n3)
    for var in range(4):
        for d in range(3):
            np.testing.assert_allclose(G[:, d, var], grads[var][d], atol=1e-12)


def test_tgv_viscous_dissipation_rate(orc):
    """dKE/dt from the viscous part at t=0 equals -mu * <|omega|^2> * (2pi)^3 = -mu (3/4)(2pi)^3."""
    rates = []
    for k in (2, 4):
        M = _mesh(orc, k, 5, "lgl", False)
        U = inputs.taylor_green(M.points(), 1.0, 0.1)
        wq = _wq(orc, M)

        def dke(mu):
            Ut = M.rhs(orc.Scheme("ns", "split", "kep", "roe", mu=mu), U)
            rho = U[:, 0]
            uu = U[:, 1:4] / rho[:, None]
            return np.sum(wq * (np.einsum("evq,evq->eq", uu, Ut[:, 1:4]) - 0.5 * (uu ** 2).sum(1) * Ut[:, 0]))

        mu = 1.0 / 1600
        rates.append((dke(mu) - dke(0.0)))
    exact = -mu * 0.75 * (2 * math.pi) ** 3
    assert abs(rates[1] / exact - 1) < 2e-3
    assert abs(rates[1] / exact - 1) < abs(rates[0] / exact - 1)


def _quasi1d_wave(M, t):
    x = M.points()
    rho = 1 + 0.2 * np.sin(x[:, 0] - t)
    one, z = np.ones_like(rho), np.zeros_like(rho)
    return inputs.prim_to_cons(rho, one, z, z, one, GAMMA)


def _l2(orc, M, a, b):
    return math.sqrt(np.sum(_wq(orc, M) * (a - b) ** 2))


@pytest.mark.slow
@pytest.mark.parametrize("nodes,form,vf,N", [("lg", "weak", "central", 3), ("lgl", "split", "ec", 3),
                                             ("lgl", "weak", "central", 4)])
def test_density_wave_order(orc, nodes, form, vf, N):
    """Exact Euler density wave: L2 error decays as h^(N+1)."""
    errs = []
    for k in (8, 16, 32):
        M = _mesh(orc, 0, N, nodes, False, kxyz=(k, 1, 1))
        sc = orc.Scheme("euler", form, vf, "roe")
        U0 = _quasi1d_wave(M, 0.0)
        dt = 0.05 * M.timestep(sc, U0, 1.0, 1.0)
        T = 0.5
        ns = int(math.ceil(T / dt))
        U = M.rk(sc, U0, ns, T / ns)
        errs.append(_l2(orc, M, U[:, 0], _quasi1d_wave(M, T)[:, 0]))
    order = math.log2(errs[1] / errs[2])
    assert order > N + 1 - 0.3, errs


@pytest.mark.slow
def test_isentropic_vortex_order(orc):
    """Shu's isentropic vortex (eps=5 on [0,20]^2, extruded in z): order N+1 for the split EC scheme."""
    N = 4
    errs = []
    for k in (5, 10, 20):
        M = _mesh(orc, 0, N, "lgl", False, kxyz=(k, k, 1), box=(20.0, 20.0, 20.0 / k))
        sc = orc.Scheme("euler", "split", "ec", "roe")
        U0 = inputs.isentropic_vortex(M.points())
        dt = 0.2 * M.timestep(sc, U0, 1.0, 1.0)
        T = 0.5
        ns = int(math.ceil(T / dt))
        U = M.rk(sc, U0, ns, T / ns)
        errs.append(_l2(orc, M, U[:, 0], inputs.isentropic_vortex(M.points(), t=T)[:, 0]))
    order = math.log2(errs[1] / errs[2])
    assert order > N + 1 - 0.5, errs


def test_rk_time_order(orc):
    """The oracle's RK loop: halving dt cuts the time error by ~16 (fixed spatial operator)."""
    M = _mesh(orc, 0, 3, "lg", False, kxyz=(4, 1, 1))
    sc = orc.Scheme("euler", "weak", "central", "llf")
    U0 = _quasi1d_wave(M, 0.0)
    T = 0.4
    ref = M.rk(sc, U0, 640, T / 640)
    e = [np.abs(M.rk(sc, U0, ns, T / ns) - ref).max() for ns in (10, 20)]
    assert 13 < e[0] / e[1] < 19, e


# ----------------------------------------------------------------------------- brute force
def _lag(x, j, t):
    v = np.ones_like(t)
    for k in range(len(x)):
        if k != j:
            v = v * (t - x[k]) / (x[j] - x[k])
    return v


def _dlag(x, j, t):
    tot = np.zeros_like(t)
    for m in range(len(x)):
        if m == j:
            continue
        term = np.full_like(t, 1.0 / (x[j] - x[m]))
        for k in range(len(x)):
            if k != j and k != m:
                term = term * (t - x[k]) / (x[j] - x[k])
        tot = tot + term
    return tot


@pytest.mark.parametrize("nodes,N", [("lg", 2), ("lg", 3), ("lgl", 2), ("lgl", 3)])
def test_brute_force_weak_form(orc, nodes, N):
    """Evaluate the weak form (eq. weakFormulation) with explicit basis functions and an
    independent 12-point Gauss rule for the volume and surface integrals; mass matrix by the
    collocated rule (exact for LG, the DGSEM mass lumping for LGL).  Euler, affine 2x1x1 mesh."""

    k = (2, 1, 1)
    M = _mesh(orc, 0, N, nodes, False, kxyz=k)
    b = orc.basis(N, nodes)
    xn, wn = b["x"], b["w"]
    n = N + 1
    rng = np.random.default_rng(21)
    U = inputs.random_perturbation(inputs.constant_state(M.K, M.n3, rho=1.0, u=0.4, v=-0.3, w=0.2, p=1.0), 9, 0.05)
    sc = orc.Scheme("euler", "weak", "central", "llf")
    Ut = M.rhs(sc, U)
    g = M.geometry()
    # LG collocation integrates these polynomials exactly, so an independent exact rule is used;
    # on LGL the scheme is defined by the (inexact) LGL rule itself, so the nodes' rule is used
    # but with explicitly evaluated basis functions and no collocation shortcut
    gx, gw = np.polynomial.legendre.leggauss(12) if nodes == "lg" else (xn, wn)
    L = np.array([_lag(xn, j, gx) for j in range(n)])   # [j][q]
    dL = np.array([_dlag(xn, j, gx) for j in range(n)])
    Lm = np.array([_lag(xn, j, np.array([-1.0]))[0] for j in range(n)])
    Lp = np.array([_lag(xn, j, np.array([1.0]))[0] for j in range(n)])
    Ja = g["Ja"][0, [0, 4, 8], 0]  # diagonal, constant
    Jdet = g["J"][0, 0]
    fn = g["fn"]

    def nodal_flux(e):
        F = np.zeros((3, 5, n, n, n))  # contravariant flux at nodes [dir][v][k][j][i]
        for q in range(M.n3):
            Uq = U[e, :, q]
            for d in range(3):
                nv = np.zeros(3)
                nv[d] = Ja[d]
                F[d, :, q // (n * n), (q // n) % n, q % n] = orc.euler_flux(Uq, nv)
        return F

    def face_state(e, s):
        """polynomial trace of U on side s at the face quadrature nodes [v][b][a] via explicit l_j(+-1)"""
        d = s // 2
        lv = Lp if s % 2 else Lm
        Ue = U[e].reshape(5, n, n, n)
        if d == 0:
            return np.einsum("vkji,i->vkj", Ue, lv)
        if d == 1:
            return np.einsum("vkji,j->vki", Ue, lv)
        return np.einsum("vkji,k->vji", Ue, lv)

    for e in range(M.K):
        F = nodal_flux(e)
        R = np.zeros((5, n, n, n))
        # - <F, grad phi_ijk>: F interpolated (nodal polynomial) times d phi, integrated exactly
        for d in range(3):
            Fd = F[d]  # [v][k][j][i]
            # interpolate F to the Gauss grid
            Fq = np.einsum("vkji,iq,jr,ks->vsrq", Fd, L, L, L)
            for (ii, jj, kk) in np.ndindex(n, n, n):
                phi = [L[ii], L[jj], L[kk]]
                phi[d] = [dL[ii], dL[jj], dL[kk]][d]
                w3 = np.einsum("q,r,s->srq", gw * phi[0], gw * phi[1], gw * phi[2])
                R[:, kk, jj, ii] -= np.einsum("vsrq,srq->v", Fq, w3)
        # + surface integral of phi f* s over the 6 faces (f* at the face nodes, interpolated)
        for s in range(6):
            d = s // 2
            lv = Lp if s % 2 else Lm
            UL = face_state(e, s)
            kx = k[0]
            ex = e % kx
            nbe = ((ex + (1 if s % 2 else -1)) % kx) if d == 0 else e
            UR = face_state(nbe, s ^ 1)
            fs = np.zeros((5, n, n))
            for bb in range(n):
                for aa in range(n):
                    nt = fn[e, s, :, aa + n * bb]
                    sh = np.linalg.norm(nt)
                    if s % 2:
                        fs[:, bb, aa] = orc.riemann("llf", UL[:, bb, aa], UR[:, bb, aa], nt / sh) * sh
                    else:
                        fs[:, bb, aa] = -orc.riemann("llf", UR[:, bb, aa], UL[:, bb, aa], -nt / sh) * sh
            fq = np.einsum("vba,ap,bq->vqp", fs, L, L)
            for (ii, jj, kk) in np.ndindex(n, n, n):
                idx = [ii, jj, kk]
                ta = [x for x in range(3) if x != d]
                pa = L[idx[ta[0]]]
                pb = L[idx[ta[1]]]
                val = np.einsum("vqp,p,q->v", fq, gw * pa, gw * pb) * lv[idx[d]]
                R[:, kk, jj, ii] += val
        # mass matrix: J w_i w_j w_k (collocated); solve <J U_t, phi> = -R
        W3 = np.einsum("k,j,i->kji", wn, wn, wn)
        Ut_bf = (-R / (Jdet * W3[None])).reshape(5, -1)
        np.testing.assert_allclose(Ut[e], Ut_bf, atol=1e-11 * np.abs(Ut_bf).max())


# ----------------------------------------------------------------------------- tangent
@pytest.mark.parametrize("eqn,form,vf,rs", [("ns", "split", "kep", "roe"), ("ns", "split", "ec", "llf"),
                                            ("euler", "weak", "central", "roe")])
def test_tangent_matches_central_differences(orc, eqn, form, vf, rs):
    M = _mesh(orc, 2, 3, "lgl", True)
    sc = orc.Scheme(eqn, form, vf, rs, mu=1e-2)
    U = inputs.taylor_green(M.points(), 1.0, 0.3)
    if rs != "llf":
        # LLF's max(|u_n|+c) has near-ties (gap ~ eps) under random perturbations, where a central
        # difference straddles the kink; the unperturbed field has exact ties instead
        U = inputs.random_perturbation(U, 10, 1e-2)
    dU = inputs.random_directions(U, 1, 1)[0]
    _, jv = M.rhs_jvp(sc, U, dU)
    eps = 1e-6
    fd = (M.rhs(sc, U + eps * dU) - M.rhs(sc, U - eps * dU)) / (2 * eps)
    # LLF at the exact ties of the unperturbed field: the difference quotient straddles the kink of
    # max(|u_n|+c) and carries an O(eps) error there
    tol = 1e-5 if rs == "llf" else 1e-6
    assert np.abs(jv - fd).max() < tol * np.abs(jv).max()
