"""Pins of the oracle's 1D basis (Sec. 3.1): nodes, weights, D, Dhat, boundary interpolants.

Every expected value here is a closed form, an exactness property or a brute-force
evaluation written in the test; none comes from the GPU path.
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tikz_lg3.txt")


def test_closed_form_nodes(orc):
    r35 = math.sqrt(3.0 / 5.0)
    cases = {
        (1, "lg"): ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1, 1]),
        (1, "lgl"): ([-1, 1], [1, 1]),
        (2, "lg"): ([-r35, 0, r35], [5 / 9, 8 / 9, 5 / 9]),
        (2, "lgl"): ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
        (3, "lgl"): ([-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
        (4, "lgl"): ([-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1], [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1]),
    }
    a_in = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5))
    a_out = math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    w_in = (18 + math.sqrt(30)) / 36
    w_out = (18 - math.sqrt(30)) / 36
    cases[(3, "lg")] = ([-a_out, -a_in, a_in, a_out], [w_out, w_in, w_in, w_out])
    for (N, t), (x, w) in cases.items():
        b = orc.basis(N, t)
        np.testing.assert_allclose(b["x"], x, atol=2e-16, rtol=0)
        np.testing.assert_allclose(b["w"], w, atol=4e-16, rtol=0)


def test_paper_drawing_lg3_subcell_borders(orc):
    """The paper draws the LG N=3 subcell borders at -1 + w_0 (three decimals)."""
    rows = [ln.split() for ln in open(GOLD) if ln.strip() and not ln.startswith("#")]
    val = {r[0]: float(r[1]) for r in rows}
    w = orc.basis(3, "lg")["w"]
    assert abs((-1 + w[0]) - val["lg3_subcell_border_left"]) < 5e-4
    assert abs((1 - w[-1]) - val["lg3_subcell_border_right"]) < 5e-4
    # and the interior border of the two left subcells is at 0 = -1 + w_0 + w_1
    assert abs(-1 + w[0] + w[1]) < 1e-15
    assert abs(2.0 / 4 - val["fv_equidistant_border"]) < 5e-4


@pytest.mark.parametrize("N", range(1, 9))
@pytest.mark.parametrize("t", ["lg", "lgl"])
def test_quadrature_exactness(orc, N, t):
    b = orc.basis(N, t)
    x, w = b["x"], b["w"]
    exact_deg = 2 * N + 1 if t == "lg" else 2 * N - 1
    for p in range(exact_deg + 1):
        ref = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, x ** p) - ref) < 1e-14
    # one degree higher must fail (even power)
    p = exact_deg + 1
    assert abs(np.dot(w, x ** p) - 2.0 / (p + 1)) > 1e-6


@pytest.mark.parametrize("N", range(1, 9))
@pytest.mark.parametrize("t", ["lg", "lgl"])
def test_derivative_matrix(orc, N, t):
    b = orc.basis(N, t)
    x, D = b["x"], b["D"]
    for p in range(N + 1):
        f = x ** p
        df = p * x ** (p - 1) if p > 0 else np.zeros_like(x)
        np.testing.assert_allclose(D @ f, df, atol=1e-12 * max(1, N * N), rtol=0)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-13)
    if t == "lgl":
        assert abs(D[0, 0] + N * (N + 1) / 4.0) < 1e-12
        assert abs(D[N, N] - N * (N + 1) / 4.0) < 1e-12


@pytest.mark.parametrize("N", range(1, 9))
def test_sbp_and_weak_matrix_lgl(orc, N):
    """LGL: M D + (M D)^T = B, hence Dhat = D - M^{-1} B (this pins the reading of Dhat)."""
    b = orc.basis(N, "lgl")
    M = np.diag(b["w"])
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    Q = M @ b["D"]
    np.testing.assert_allclose(Q + Q.T, B, atol=1e-13)
    np.testing.assert_allclose(b["Dhat"], b["D"] - np.linalg.inv(M) @ B, atol=1e-12 * N * N)


def _lagrange_brute(x, j, t):
    v = 1.0
    for k in range(len(x)):
        if k != j:
            v *= (t - x[k]) / (x[j] - x[k])
    return v


@pytest.mark.parametrize("N", range(1, 9))
@pytest.mark.parametrize("t", ["lg", "lgl"])
def test_boundary_interpolants_and_weak_matrix(orc, N, t):
    b = orc.basis(N, t)
    x = b["x"]
    lm = np.array([_lagrange_brute(x, j, -1.0) for j in range(N + 1)])
    lp = np.array([_lagrange_brute(x, j, 1.0) for j in range(N + 1)])
    np.testing.assert_allclose(b["lm"], lm, atol=1e-13)
    np.testing.assert_allclose(b["lp"], lp, atol=1e-13)
    # Dhat from the volume-integral derivation: <F, d phi_i> / w_i = -sum_m Dhat_im F_m for any F;
    # check with F = x^p and exact integrals of x^p * l_i'(x) evaluated by a 40-point Gauss rule.
    gx, gw = np.polynomial.legendre.leggauss(40)
    for p in range(N + 1):
        Fm = x ** p
        for i in range(N + 1):
            # l_i'(s) by a centred difference of the brute-force Lagrange polynomial is too coarse;
            # use the exact derivative of the product form instead
            def dli(s, i=i):
                tot = 0.0
                for m in range(N + 1):
                    if m == i:
                        continue
                    term = 1.0 / (x[i] - x[m])
                    for k in range(N + 1):
                        if k != i and k != m:
                            term *= (s - x[k]) / (x[i] - x[k])
                    tot += term
                return tot
            # weak-form volume term uses the collocated quadrature of F_interp * l_i'
            integ = sum(b["w"][m] * Fm[m] * dli(x[m]) for m in range(N + 1))
            assert abs(-integ / b["w"][i] - (b["Dhat"][i] @ Fm)) < 1e-11 * (N + 1) ** 2
            if t == "lg" or p + N - 1 <= 2 * N - 1:
                exact = sum(gw[q] * gx[q] ** p * dli(gx[q]) for q in range(40))
                assert abs(integ - exact) < 1e-12 * (N + 1) ** 2


def test_rk_order_conditions(orc):
    """Butcher form of the 2N-storage coefficients meets all conditions up to order 4."""
    A, B, C = orc.rk_coefficients()
    s = 5
    a = np.zeros((s + 1, s))
    for i in range(1, s + 1):
        for j in range(i):
            tot, prod = 0.0, 1.0
            for r in range(j, i):
                if r > j:
                    prod *= A[r]
                tot += B[r] * prod
            a[i, j] = tot
    bb = a[s]
    aa = a[:s]
    c = aa.sum(axis=1)
    np.testing.assert_allclose(c, C, atol=1e-14)
    conds = [
        (bb.sum(), 1.0), (bb @ c, 0.5), (bb @ c ** 2, 1 / 3), (bb @ (aa @ c), 1 / 6),
        (bb @ c ** 3, 0.25), (bb @ (c * (aa @ c)), 1 / 8), (bb @ (aa @ c ** 2), 1 / 12), (bb @ (aa @ (aa @ c)), 1 / 24),
    ]
    for got, ref in conds:
        assert abs(got - ref) < 1e-14
    # stability polynomial of y' = z y agrees with exp(z) through z^4/24: the one-step error
    # shrinks by 2^5 when z is halved
    def err(z):
        y, k = 1.0, 0.0
        for st in range(5):
            k = A[st] * k + z * y
            y = y + B[st] * k
        return abs(y - math.exp(z))
    ratio = err(0.2) / err(0.1)
    assert 28 < ratio < 36
