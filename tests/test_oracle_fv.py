"""Pins of the oracle's finite-volume subcell shock capturing (Sec. 4), Euler equations.

  * V_DG=>FV (eq. FVvdm): rows sum to one, it returns the exact subcell means of polynomials of
    degree <= N (closed-form antiderivatives), and w^T V^-1 = (2/(N+1)) 1^T (the quadrature of
    the DG polynomial equals the sum of the subcell means: eq. fv:cons);
  * on a Cartesian lattice with every element finite-volume, the operator is a textbook MUSCL
    scheme on the uniform grid of all subcells (primitive-variable slopes limited by minmod or
    van Leer, or none), written out here independently with the oracle's Riemann solver only;
  * free stream on a curved mesh, all-FV and mixed DG/FV, every limiter and form;
  * conservation on mixed meshes (the DG elements' quadrature plus the FV elements'
    subcell means times w^3 Jbar);
  * invariance under relabelling the elements' reference axes on a mixed mesh;
  * the indicator: -inf-like for a state whose rho p has degree <= N - 2, large for a jump, and
    the switching's hysteresis and round trip.
"""
import math

import numpy as np
import pytest

from paper_1910_02858_amd import inputs

GAMMA = 1.4


@pytest.mark.parametrize("nodes", ["lg", "lgl"])
@pytest.mark.parametrize("N", [1, 3, 5])
def test_fv_matrices(orc, nodes, N):
    V, Vi = orc.fv_matrices(N, nodes)
    n = N + 1
    w = orc.basis(N, nodes)["w"]
    x = orc.basis(N, nodes)["x"]
    np.testing.assert_allclose(V.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(V @ Vi, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(w @ Vi, np.full(n, 2.0 / n), atol=1e-13)
    edges = -1 + 2.0 * np.arange(n + 1) / n
    for deg in range(N + 1):
        means = (edges[1:] ** (deg + 1) - edges[:-1] ** (deg + 1)) / ((deg + 1) * (2.0 / n))
        np.testing.assert_allclose(V @ x ** deg, means, atol=1e-13)


def _lattice(orc, k, N, nodes, curved, kxyz=None):
    lgl = orc.basis(N, "lgl")["x"]
    kx, ky, kz = kxyz if kxyz else (k, k, k)
    X = inputs.lattice_points(lgl, kx, ky, kz)
    xg = inputs.warp_sine(X) if curved else X
    nbr, side, _ = inputs.periodic_lattice(kx, ky, kz)
    return orc.OracleMesh(xg, nbr, side, N, nodes), xg, nbr, side


def _prim(U):
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]
    p = (GAMMA - 1) * (U[..., 4] - 0.5 * rho * (u * u).sum(-1))
    return np.concatenate([rho[..., None], u, p[..., None]], axis=-1)


def _cons(W):
    rho, u, p = W[..., 0], W[..., 1:4], W[..., 4]
    return np.concatenate([rho[..., None], rho[..., None] * u, (p / (GAMMA - 1) + 0.5 * rho * (u * u).sum(-1))[..., None]],
                          axis=-1)


def _limit(lim, a, b):
    if lim == 0:
        return np.zeros_like(a)
    same = a * b > 0
    if lim == 1:
        return np.where(same, np.where(np.abs(a) < np.abs(b), a, b), 0.0)
    return np.where(same, 2 * a * b / np.where(same, a + b, 1.0), 0.0)


@pytest.mark.parametrize("lim", [0, 1, 2])
@pytest.mark.parametrize("rs", ["llf", "roe"])
def test_fv_equals_muscl_on_uniform_grid(orc, lim, rs):
    N, kx, ky, kz = 2, 3, 2, 2
    n = N + 1
    M, _, _, _ = _lattice(orc, 0, N, "lgl", False, (kx, ky, kz))
    rng = np.random.default_rng(3)
    K = M.K
    gx, gy, gz = kx * n, ky * n, kz * n
    Wg = np.empty((gz, gy, gx, 5))
    Wg[..., 0] = 1.0 + 0.3 * rng.random((gz, gy, gx))
    Wg[..., 1:4] = 0.4 * rng.standard_normal((gz, gy, gx, 3))
    Wg[..., 4] = 1.0 + 0.3 * rng.random((gz, gy, gx))
    Ug = _cons(Wg)
    # element storage of the same field: element (ex,ey,ez), subcell (i,j,k) is global cell
    U = np.empty((K, 5, n ** 3))
    for e in range(K):
        ex, ey, ez = e % kx, (e // kx) % ky, e // (kx * ky)
        blk = Ug[ez * n:(ez + 1) * n, ey * n:(ey + 1) * n, ex * n:(ex + 1) * n]  # [k][j][i][v]
        U[e] = blk.reshape(n ** 3, 5).T
    sc = orc.Scheme("euler", "split", "central", rs)
    Ut = M.fv_rhs(sc, np.ones(K, np.uint8), U, limiter=lim)
    # textbook MUSCL on the periodic uniform grid, cell size h/n
    h = 2 * math.pi / np.array([kx, ky, kz])
    ref = np.zeros_like(Ug)
    for d in range(3):
        ax = 2 - d  # array axis of direction d
        dx = h[d] / n
        Wm, Wp = np.roll(Wg, 1, axis=ax), np.roll(Wg, -1, axis=ax)
        sig = _limit(lim, Wg - Wm, Wp - Wg)
        WL = Wg + 0.5 * sig                         # left state of the face c + 1/2
        WR = np.roll(Wg - 0.5 * sig, -1, axis=ax)   # right state of the face c + 1/2
        UL, UR = _cons(WL), _cons(WR)
        nv = np.zeros(3)
        nv[d] = 1.0
        F = np.empty_like(UL)
        for idx in np.ndindex(*UL.shape[:3]):
            F[idx] = orc.riemann(rs, UL[idx], UR[idx], nv)
        ref -= (F - np.roll(F, 1, axis=ax)) / dx
    got = np.empty_like(Ug)
    for e in range(K):
        ex, ey, ez = e % kx, (e // kx) % ky, e // (kx * ky)
        got[ez * n:(ez + 1) * n, ey * n:(ey + 1) * n, ex * n:(ex + 1) * n] = Ut[e].T.reshape(n, n, n, 5)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


SCHEMES = [("lg", "weak", "central", "llf"), ("lgl", "split", "ec", "roe"), ("lgl", "strong", "central", "roe"),
           ("lgl", "split", "kep", "volflux_roe")]


def _weights(orc, M, fv):
    Jb, _ = M.fv_geometry()
    w1 = orc.basis(M.N, M.nodes)["w"]
    wq = np.einsum("k,j,i->kji", w1, w1, w1).ravel()[None] * M.geometry()["J"]
    return np.where(np.asarray(fv)[:, None] == 1, (2.0 / M.n) ** 3 * Jb, wq)


@pytest.mark.parametrize("lim", [0, 1, 2])
@pytest.mark.parametrize("nodes,form,vf,rs", SCHEMES)
def test_fv_freestream_and_conservation(orc, nodes, form, vf, rs, lim):
    N, k = 3, 3
    M, _, _, _ = _lattice(orc, k, N, nodes, True)
    sc = orc.Scheme("euler", form, vf, rs)
    rng = np.random.default_rng(9)
    for fv in (np.ones(M.K, np.uint8), (rng.random(M.K) < 0.5).astype(np.uint8)):
        Uc = inputs.constant_state(M.K, M.n3)
        assert np.abs(M.fv_rhs(sc, fv, Uc, lim)).max() < 1e-12 * np.abs(Uc).max() * (N + 1) ** 2 * k
        U = inputs.random_perturbation(inputs.taylor_green(M.points(), 1.0, 0.3), 5, 1e-2)
        Ut = M.fv_rhs(sc, fv, U, lim)
        wt = _weights(orc, M, fv)
        tot = np.einsum("eq,evq->v", wt, Ut)
        scale = np.einsum("eq,evq->v", wt, np.abs(Ut))
        assert np.all(np.abs(tot) < 1e-13 * scale), tot / scale


@pytest.mark.parametrize("nodes,form,vf,rs", SCHEMES[:2])
def test_fv_rotation_invariance(orc, nodes, form, vf, rs):
    N, k = 3, 3
    lgl = orc.basis(N, "lgl")["x"]
    X = inputs.warp_sine(inputs.lattice_points(lgl, k, k, k))
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    rot = np.random.default_rng(12).integers(0, 24, k ** 3)
    Xr, nbr2, side2, flip2, maps = inputs.rotate_elements(X, nbr, side, flip, N, rot)
    M0 = orc.OracleMesh(X, nbr, side, N, nodes)
    M1 = orc.OracleMesh(Xr, nbr2, side2, N, nodes, flip=flip2)
    fv = (np.random.default_rng(13).random(M0.K) < 0.5).astype(np.uint8)
    sc = orc.Scheme("euler", form, vf, rs)
    U0 = inputs.random_perturbation(inputs.taylor_green(M0.points(), 1.0, 0.3), 6, 1e-2)
    U1 = np.take_along_axis(U0, maps[:, None, :], axis=2)
    a = np.take_along_axis(M0.fv_rhs(sc, fv, U0), maps[:, None, :], axis=2)
    b = M1.fv_rhs(sc, fv, U1)
    assert np.abs(a - b).max() < 2e-13 * np.abs(a).max()


def test_fv_indicator_and_switching(orc):
    N, k = 4, 2
    M, _, _, _ = _lattice(orc, k, N, "lgl", False)
    x = M.points()
    # rho of degree 2 (<= N - 2) in x, p constant: rho p has no energy in the top two modes
    rho = 1.0 + 0.1 * (x[:, 0] / math.pi - 1) + 0.05 * (x[:, 0] / math.pi - 1) ** 2
    U = inputs.prim_to_cons(rho, 0 * rho + 0.2, 0 * rho, 0 * rho, 0 * rho + 1.0, GAMMA)
    fv0 = np.zeros(M.K, np.uint8)
    ind = M.fv_indicator(fv0, U)
    assert np.all(ind < -20)
    # a density jump at x = 1.3 inside the first column of elements
    rho2 = np.where(x[:, 0] < 1.3, 1.0, 0.125)
    U2 = inputs.prim_to_cons(rho2, 0 * rho2, 0 * rho2, 0 * rho2, np.where(x[:, 0] < 1.3, 1.0, 0.1), GAMMA)
    ind2 = M.fv_indicator(fv0, U2)
    jump = np.array([np.ptp(x[e, 0]) > 0 and x[e, 0].min() < 1.3 < x[e, 0].max() for e in range(M.K)])
    assert np.all(ind2[jump] > -2) and np.all(ind2[~jump] < -20)
    # hysteresis: DG -> FV above hi; FV stays FV between lo and hi; FV -> DG below lo
    hi, lo = -2.5, -6.0
    fv1, U3 = M.fv_switch(fv0, U2, lo, hi)
    assert np.array_equal(fv1.astype(bool), jump)
    V, Vi = orc.fv_matrices(N, "lgl")
    e = int(np.nonzero(jump)[0][0])
    ref = np.einsum("ia,jb,kc,vcba->vkji", V, V, V, U2[e].reshape(5, N + 1, N + 1, N + 1)).reshape(5, -1)
    np.testing.assert_allclose(U3[e], ref, atol=1e-13)
    ind3 = M.fv_indicator(fv1, U3)
    np.testing.assert_allclose(ind3[jump], ind2[jump], atol=1e-9)  # the FV element's DG reading
    fv2, U4 = M.fv_switch(fv1, U3, lo=min(ind2[jump]) - 1, hi=max(ind2[jump]) + 1)
    assert np.array_equal(fv2, fv1) and np.array_equal(U4, U3)
    fv3, U5 = M.fv_switch(fv1, U3, lo=max(ind2[jump]) + 1, hi=max(ind2[jump]) + 2)
    assert not fv3.any()
    np.testing.assert_allclose(U5, U2, atol=1e-12)
