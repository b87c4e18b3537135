"""Reverse sweep of the weak form (Euler, LG and LGL nodes) and of the split form at degree 8.

* dg_rhs_vjp of the weak form element by element: J^T w against the oracle's Jacobian, assembled
  column by column from its dual-number tangent on a tiny curved lattice and on boxes with every
  boundary kind (symmetry planes with rotated element axes, given state, no-slip wall, pressure
  outflow), 1e-12;
* dot products <J^T w, v> = <w, J v> (J v from the oracle's tangent) for the density-wave
  workload (Euler weak form, LG, N = 3, 4^3) and at every degree 1..8; the split form at degree 8;
* the density-wave workload's checkpointed rollout: reverse sweep against the oracle's tangent
  rollout, 1e-10.
"""
import numpy as np
import pytest

from paper_1910_02858_amd import inputs
from gpu_common import gpu_solver, problem, to_gpu
from test_gpu_general_mesh import box_problem, box_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    from paper_1910_02858_amd import dgsem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def jacobian(M, sc, U0):
    n = U0.size
    J = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        _, col = M.rhs_jvp(sc, U0, e.reshape(U0.shape))
        J[:, j] = col.ravel()
    return J


def check_elementwise(S, J, U0, seed, name):
    rng = np.random.default_rng(seed)
    for _ in range(2):
        w = rng.standard_normal(U0.shape)
        got = S.rhs_vjp(to_gpu(U0), to_gpu(w)).cpu().numpy().ravel()
        ref = J.T @ w.ravel()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"{name}: max-norm relative error of J^T w {err:.2e}")
        assert err <= 1e-12


WEAK = [
    ("lg_llf", dict(nodes="lg", riemann="llf")),
    ("lg_roe", dict(nodes="lg", riemann="roe")),
    ("lgl_roe", dict(nodes="lgl", riemann="roe")),
    ("lg_ec_volflux_roe", dict(nodes="lg", volflux="ec", riemann="volflux_roe")),
    ("lgl_kep_volflux", dict(nodes="lgl", volflux="kep", riemann="volflux")),
]


@pytest.mark.parametrize("name,kw", WEAK, ids=[w[0] for w in WEAK])
def test_weak_vjp_elementwise_against_oracle_jacobian(dg, orc, name, kw):
    print(f"case {name}", flush=True)
    wl = inputs.workload(1, N=2, K1=2, curved=True, **kw)
    M, xgeo, nbr, side, U0 = problem(orc, wl, kxyz=(2, 2, 2), perturb=2e-2, seed=11)
    J = jacobian(M, orc.Scheme.of(wl), U0)
    check_elementwise(gpu_solver(dg, wl, xgeo, nbr, side), J, U0, 3, name)


BOXES = [("symmetry_rotated", 0, 8), ("given_state", 1, None), ("wall", 2, 5), ("outflow", 4, 6)]


@pytest.mark.parametrize("name,kind,seed", BOXES, ids=[b[0] for b in BOXES])
@pytest.mark.parametrize("nodes", ["lg", "lgl"])
def test_weak_vjp_box_elementwise_against_oracle_jacobian(dg, orc, name, kind, seed, nodes):
    print(f"case {name} {nodes}", flush=True)
    wl = inputs.workload(1, N=2, nodes=nodes, riemann="roe", ic="tgv", mach=0.3)
    M, (X, nbr, side, flip), U0 = box_problem(orc, wl, 2, seed=seed, perturb=2e-2, kind=kind)
    J = jacobian(M, orc.Scheme.of(wl), U0)
    check_elementwise(box_solver(dg, wl, X, nbr, side, flip, kind=kind), J, U0, 4, f"{name} {nodes}")


def dot_product(dg, orc, wl, M, S, U0, seed, count=2):
    sc = orc.Scheme.of(wl)
    rng = np.random.default_rng(seed)
    for v in inputs.random_directions(U0, seed + 1, count):
        w = rng.standard_normal(U0.shape)
        _, Jv = M.rhs_jvp(sc, U0, v)
        JTw = S.rhs_vjp(to_gpu(U0), to_gpu(w)).cpu().numpy()
        lhs, rhs = float(np.sum(JTw * v)), float(np.sum(w * Jv))
        scale = float(np.sum(np.abs(JTw * v)))
        print(f"{wl.name} N={wl.N}: <J^T w, v> = {lhs:.15e}  <w, J v> = {rhs:.15e}")
        assert abs(lhs - rhs) <= 1e-12 * scale


def test_weak_vjp_dot_product_density_wave(dg, orc):
    wl = inputs.workload(1)
    M, xgeo, nbr, side, U0 = problem(orc, wl, perturb=1e-3)
    dot_product(dg, orc, wl, M, gpu_solver(dg, wl, xgeo, nbr, side), U0, 40)


@pytest.mark.parametrize("N", [1, 2, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("nodes", ["lg", "lgl"])
def test_weak_vjp_dot_product_degrees(dg, orc, N, nodes):
    wl = inputs.workload(1, N=N, K1=2, nodes=nodes, curved=True)
    M, xgeo, nbr, side, U0 = problem(orc, wl, kxyz=(3, 2, 2), perturb=1e-2, seed=N)
    dot_product(dg, orc, wl, M, gpu_solver(dg, wl, xgeo, nbr, side), U0, 50 + N)


@pytest.mark.parametrize("vf", ["kep", "ec"])
def test_split_vjp_dot_product_degree_8(dg, orc, vf):
    """The split-form reverse kernels at degree 8 (768 lanes per element, no LDS staging)."""
    wl = inputs.workload(5, N=8, K1=2, volflux=vf)
    M, xgeo, nbr, side, U0 = problem(orc, wl, kxyz=(2, 2, 1), curved=True, perturb=1e-2, seed=8)
    dot_product(dg, orc, wl, M, gpu_solver(dg, wl, xgeo, nbr, side), U0, 80)


def test_weak_rollout_dot_product_density_wave(dg, orc):
    wl = inputs.workload(1)
    M, xgeo, nbr, side, U0 = problem(orc, wl, perturb=1e-3)
    sc = orc.Scheme.of(wl)
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    dt = M.timestep(sc, U0, 0.9, 0.9)
    steps = 6
    v = inputs.random_directions(U0, 4, 1)[0]
    _, vT = M.rk_jvp(sc, U0, v, steps, dt)
    w = np.random.default_rng(5).standard_normal(U0.shape)
    _, stage_inputs = dg._rollout_forward(S, to_gpu(U0), steps, dt, keep_stage_inputs=True)
    Ubar = dg._rollout_backward(S, stage_inputs, to_gpu(w), dt).cpu().numpy()
    lhs, rhs = float(np.sum(Ubar * v)), float(np.sum(w * vT))
    scale = float(np.sum(np.abs(Ubar * v)))
    print(f"<Ubar_0, v_0> = {lhs:.15e}  <w, v_T> = {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-10 * scale
