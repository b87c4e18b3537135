"""GPU vector-Jacobian products against the oracle's tangent-linear (dual-number) operator and
against central finite differences.

* dg_rhs_vjp element by element: the oracle's Jacobian is assembled column by column from its
  dual-number tangent on a tiny mesh, and J^T w must match the GPU product (KEP, EC and central
  two-point fluxes, LLF, Roe and two-point surface fluxes, Euler and Navier-Stokes).
* dot-product tests <J^T w, v> = <w, J v> for one operator evaluation at the 12^3 N=5 curved
  workload and at every degree the reverse kernels are built for, and for RK rollouts (GPU
  reverse sweep vs oracle tangent rollout).
* the checkpointed rollout gradient equals the store-everything gradient bit for bit, and the
  stage-by-stage reverse to rounding; the reverse of several steps in one call equals repeated
  single steps bit for bit.
* gradient of the kinetic energy after 50 RK steps (12^3 curved hexes, N=5, checkpoint every 10)
  against central differences (eps = 1e-6) in 20 seeded random directions.
Kink convention: d|x|/dx = 0 and a tie in max splits evenly, also within 1e-12 relative.
"""
import numpy as np
import pytest

from paper_1910_02858_amd import inputs
from gpu_common import gpu_solver, problem, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    from paper_1910_02858_amd import dgsem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


TINY = [
    ("ns_kep_roe", dict(eqn="ns", volflux="kep", riemann="roe")),
    ("ns_central_llf", dict(eqn="ns", volflux="central", riemann="llf")),
    ("euler_kep_volflux_roe", dict(eqn="euler", volflux="kep", riemann="volflux_roe")),
    ("ns_ec_roe", dict(eqn="ns", volflux="ec", riemann="roe")),
    ("euler_ec_volflux", dict(eqn="euler", volflux="ec", riemann="volflux")),
]


@pytest.mark.parametrize("name,kw", TINY, ids=[t[0] for t in TINY])
def test_vjp_elementwise_against_oracle_jacobian(dg, orc, name, kw):
    wl = inputs.workload(2, N=2, K1=2, mach=0.3, **kw)
    M, xgeo, nbr, side, U0 = problem(orc, wl, kxyz=(2, 2, 2), perturb=2e-2, seed=11)
    sc = orc.Scheme.of(wl)
    n = U0.size
    J = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        _, col = M.rhs_jvp(sc, U0, e.reshape(U0.shape))
        J[:, j] = col.ravel()
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    rng = np.random.default_rng(3)
    for _ in range(2):
        w = rng.standard_normal(U0.shape)
        got = S.rhs_vjp(to_gpu(U0), to_gpu(w)).cpu().numpy().ravel()
        ref = J.T @ w.ravel()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"{name}: max-norm relative error of J^T w {err:.2e}")
        assert err <= 1e-12


def test_vjp_dot_product_cfg5_operator(dg, orc):
    wl = inputs.workload(5)
    M, xgeo, nbr, side, U0 = problem(orc, wl, perturb=1e-3)
    sc = orc.Scheme.of(wl)
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    dirs = inputs.random_directions(U0, 1, 3)
    rng = np.random.default_rng(2)
    for v in dirs:
        w = rng.standard_normal(U0.shape)
        _, Jv = M.rhs_jvp(sc, U0, v)
        JTw = S.rhs_vjp(to_gpu(U0), to_gpu(w)).cpu().numpy()
        lhs, rhs = float(np.sum(JTw * v)), float(np.sum(w * Jv))
        scale = float(np.sum(np.abs(JTw * v)))
        print(f"<J^T w, v> = {lhs:.15e}  <w, J v> = {rhs:.15e}")
        assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("N,vf", [(1, "kep"), (3, "kep"), (4, "kep"), (6, "kep"), (7, "kep"), (3, "ec"), (7, "ec")])
def test_vjp_dot_product_degrees(dg, orc, N, vf):
    """<J^T w, v> = <w, J v> for every degree the reverse kernels are built for, on a curved
    ragged 3x2x2 lattice (Navier-Stokes, KEP or EC + Roe + BR1), J v from the oracle's tangent."""
    wl = inputs.workload(5, N=N, K1=2, volflux=vf)
    M, xgeo, nbr, side, U0 = problem(orc, wl, kxyz=(3, 2, 2), curved=True, perturb=1e-2, seed=N)
    sc = orc.Scheme.of(wl)
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    rng = np.random.default_rng(20 + N)
    for v in inputs.random_directions(U0, 30 + N, 2):
        w = rng.standard_normal(U0.shape)
        _, Jv = M.rhs_jvp(sc, U0, v)
        JTw = S.rhs_vjp(to_gpu(U0), to_gpu(w)).cpu().numpy()
        lhs, rhs = float(np.sum(JTw * v)), float(np.sum(w * Jv))
        scale = float(np.sum(np.abs(JTw * v)))
        print(f"N={N} {vf}: <J^T w, v> = {lhs:.15e}  <w, J v> = {rhs:.15e}")
        assert abs(lhs - rhs) <= 1e-12 * scale


def test_rollout_dot_product(dg, orc):
    wl = inputs.workload(5, K1=4)
    M, xgeo, nbr, side, U0 = problem(orc, wl, perturb=1e-3)
    sc = orc.Scheme.of(wl)
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    dt = M.timestep(sc, U0, 0.9, 0.9)
    steps = 6
    v = inputs.random_directions(U0, 4, 1)[0]
    _, vT = M.rk_jvp(sc, U0, v, steps, dt)
    w = np.random.default_rng(5).standard_normal(U0.shape)
    Ug = to_gpu(U0)
    _, stage_inputs = dg._rollout_forward(S, Ug, steps, dt, keep_stage_inputs=True)
    Ubar = dg._rollout_backward(S, stage_inputs, to_gpu(w), dt).cpu().numpy()
    lhs, rhs = float(np.sum(Ubar * v)), float(np.sum(w * vT))
    scale = float(np.sum(np.abs(Ubar * v)))
    print(f"<Ubar_0, v_0> = {lhs:.15e}  <w, v_T> = {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-10 * scale


def test_checkpointed_gradient_equals_store_all(dg, orc):
    import torch
    wl = inputs.workload(5, K1=4)
    M, xgeo, nbr, side, U0 = problem(orc, wl, perturb=0)
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    dt = M.timestep(orc.Scheme.of(wl), U0, 0.9, 0.9)
    wJ = S.mass_weights()
    grads = []
    for ck in (3, 7):
        U = to_gpu(U0).requires_grad_(True)
        ke = dg.kinetic_energy(dg.rollout(S, U, 7, dt, ckpt_every=ck), wJ)
        (g,) = torch.autograd.grad(ke, U)
        grads.append(g.cpu().numpy())
    assert np.array_equal(grads[0], grads[1])


@pytest.mark.parametrize("eqn,ck", [("euler", 4), ("ns", 3)])
def test_rollout_gradient_equals_stage_by_stage_reverse(dg, eqn, ck):
    """The checkpointed rollout (kept last segment, recomputed earlier ones, merged register
    updates) against the plain reverse of every stored stage input with dg_rk_stage_vjp: the
    same products summed with the register updates in another grouping, so equal to 1e-12."""
    import torch
    wl = inputs.workload(5, K1=3, eqn=eqn)
    S, U0 = dg.build_solver(wl)
    U0 = to_gpu(inputs.random_perturbation(U0.cpu().numpy(), 12, 1e-3))
    dt = S.timestep(U0, 0.9, 0.9)
    steps = 7
    w = to_gpu(np.random.default_rng(13).standard_normal(U0.shape))
    U = U0.clone().requires_grad_(True)
    UT = dg.rollout(S, U, steps, dt, ckpt_every=ck)
    (g,) = torch.autograd.grad(UT, U, grad_outputs=w)
    UT2, stage_inputs = dg._rollout_forward(S, U0, steps, dt, keep_stage_inputs=True)
    assert torch.equal(UT.detach(), UT2)
    assert torch.equal(dg.rollout(S, U0, steps, dt, ckpt_every=ck), UT2)  # no gradient wanted
    g2 = dg._rollout_backward(S, stage_inputs, w.clone(), dt)
    rel = float((g - g2).abs().max() / g2.abs().max())
    print(f"{eqn}: checkpointed vs stage-by-stage reverse, max relative difference {rel:.2e}")
    assert rel <= 1e-12


def test_kinetic_energy_gradient_vs_central_differences(dg, orc):
    """12^3 curved hexes, N=5, split KEP + Roe + BR1, TGV; 50 RK steps, checkpoint every 10."""
    import torch
    wl = inputs.workload(5)
    M, xgeo, nbr, side, U0 = problem(orc, wl, perturb=0)
    S = gpu_solver(dg, wl, xgeo, nbr, side)
    dt = M.timestep(orc.Scheme.of(wl), U0, wl.cfl, wl.dfl)
    wJ = S.mass_weights()
    steps = wl.steps
    U = to_gpu(U0).requires_grad_(True)
    ke = dg.kinetic_energy(dg.rollout(S, U, steps, dt, ckpt_every=10), wJ)
    (grad,) = torch.autograd.grad(ke, U)
    grad = grad.cpu().numpy()

    def KE(Ua):
        UT, _ = dg._rollout_forward(S, to_gpu(Ua), steps, dt)
        return float(dg.kinetic_energy(UT, wJ))

    eps = 1e-6
    worst = 0.0
    for d in inputs.random_directions(U0, 1, 20):
        fd = (KE(U0 + eps * d) - KE(U0 - eps * d)) / (2 * eps)
        ad = float(np.sum(grad * d))
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
    print(f"worst relative gap gradient vs central differences over 20 directions: {worst:.2e}")
    assert worst <= 1e-6


def test_step_vjp_matches_stage_vjps(dg):
    """dg_rk_step_vjp (register updates of neighbouring stages merged, kept or recomputed
    gradients) against five dg_rk_stage_vjp calls; dg_rk_stage_keep against dg_rk_stage."""
    import torch
    wl = inputs.workload(5, K1=3)
    S, U0 = dg.build_solver(wl)
    U0 = to_gpu(inputs.random_perturbation(U0.cpu().numpy(), 4, 1e-3))
    dt = S.timestep(U0, 0.9, 0.9)
    a, b, _ = dg.rk_coefficients()
    bufs = [U0.clone()] + [S.empty() for _ in range(5)]
    plain = [U0.clone()] + [S.empty() for _ in range(5)]
    G = [S.empty_grad() for _ in range(5)]
    R, R2 = torch.zeros_like(U0), torch.zeros_like(U0)
    for s in range(5):
        S.rk_stage_keep(bufs[s], bufs[s + 1], R, a[s], b[s], dt, G[s])
        S.rk_stage(plain[s], plain[s + 1], R2, a[s], b[s], dt)
    torch.cuda.synchronize()
    assert torch.equal(bufs[5], plain[5]) and torch.equal(R, R2)
    rng = np.random.default_rng(8)
    w = to_gpu(rng.standard_normal(U0.shape))
    rb = to_gpu(rng.standard_normal(U0.shape))
    Ub1, Rb1 = w.clone(), rb.clone()
    for s in range(4, -1, -1):
        S.rk_stage_vjp(bufs[s], Ub1, Rb1, a[s], b[s], dt)
    Ub2, Rb2 = w.clone(), rb.clone()
    S.rk_step_vjp(bufs[:5], G, Ub2, Rb2, dt)
    Ub3, Rb3 = w.clone(), rb.clone()
    S.rk_step_vjp(bufs[:5], None, Ub3, Rb3, dt)
    torch.cuda.synchronize()
    assert torch.equal(Ub2, Ub3) and torch.equal(Rb2, Rb3)
    rel = float((Ub1 - Ub2).abs().max() / Ub1.abs().max())
    print(f"step VJP vs five stage VJPs: max relative difference {rel:.2e}")
    assert rel <= 1e-13


def test_steps_vjp_equals_repeated_step_vjp(dg):
    """dg_rk_steps_vjp over three steps (register updates merged across step boundaries, some
    lifting outputs kept, some recomputed) equals three dg_rk_step_vjp calls bit for bit."""
    import torch
    wl = inputs.workload(5, K1=3)
    S, U0 = dg.build_solver(wl)
    U0 = to_gpu(inputs.random_perturbation(U0.cpu().numpy(), 6, 1e-3))
    dt = S.timestep(U0, 0.9, 0.9)
    a, b, _ = dg.rk_coefficients()
    nst = 15
    bufs = [U0.clone()] + [S.empty() for _ in range(nst)]
    G = [S.empty_grad() if k % 4 else None for k in range(nst)]
    R = torch.zeros_like(U0)
    for k in range(nst):
        if G[k] is None:
            S.rk_stage(bufs[k], bufs[k + 1], R, a[k % 5], b[k % 5], dt)
        else:
            S.rk_stage_keep(bufs[k], bufs[k + 1], R, a[k % 5], b[k % 5], dt, G[k])
    rng = np.random.default_rng(9)
    w = to_gpu(rng.standard_normal(U0.shape))
    Ub1, Rb1 = w.clone(), torch.zeros_like(w)
    for st in range(2, -1, -1):
        S.rk_step_vjp(bufs[5 * st:5 * st + 5], G[5 * st:5 * st + 5], Ub1, Rb1, dt)
    Ub2, Rb2 = w.clone(), torch.zeros_like(w)
    S.rk_steps_vjp(bufs[:nst], G, Ub2, Rb2, dt)
    torch.cuda.synchronize()
    assert torch.equal(Ub1, Ub2) and torch.equal(Rb1, Rb2)
    assert float(Rb2.abs().max()) == 0.0
    assert float(Rb1.abs().max()) == 0.0 and float(Rb2.abs().max()) == 0.0
