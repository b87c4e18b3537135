"""GPU parity on conforming meshes whose faces meet on any side and in any orientation.

Every element's reference axes are rotated by a seeded proper rotation of the cube, so the
faces of neighbours meet on other sides and in all eight orientation codes (mesh conventions of
include/dgsem.h).  The library's operator and RK stages are compared with the oracle on the
same rotated mesh (bar: 1e-12 per operator evaluation, 1e-10 after RK steps), with its own
result on the unrotated lattice carried node for node (the operator does not depend on the
labelling of the reference axes: 1e-12), and a batched ensemble with a rotated member must
reproduce that member's one-mesh stage bit for bit.  The vector-Jacobian products are built for
structured meshes and must refuse a rotated one.
"""
import numpy as np
import pytest

from paper_1910_02858_amd import inputs
from gpu_common import check_rhs, rel_err, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    from paper_1910_02858_amd import dgsem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def rotated_problem(orc, wl, k, seed=7, perturb=1e-2):
    lgl = orc.basis(wl.N, "lgl")["x"]
    X = inputs.lattice_points(lgl, k, k, k)
    X = inputs.warp_sine(X) if wl.curved else X
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    rot = np.random.default_rng(seed).integers(0, 24, k ** 3)
    Xr, nbr_r, side_r, flip_r, nm = inputs.rotate_elements(X, nbr, side, flip, wl.N, rot)
    M = orc.OracleMesh(Xr, nbr_r, side_r, wl.N, wl.nodes, flip=flip_r)
    U = inputs.initial_state(wl, M.points())
    if perturb:
        U = inputs.random_perturbation(U, seed, perturb)
    return M, (Xr, nbr_r, side_r, flip_r), (X, nbr, side), nm, U


CASES = [
    ("euler_weak_lg3_llf", inputs.workload(1, curved=True), 3),
    ("euler_weak_lgl3_roe", inputs.workload(1, nodes="lgl", riemann="roe", curved=True), 3),
    ("ns_weak_lg4_llf", inputs.workload(2, nodes="lg", form="weak", riemann="llf", N=4), 3),
    ("ns_strong_lgl4_roe", inputs.workload(2, form="strong", volflux="central", N=4), 3),
    ("ns_split_kep_roe_lgl5", inputs.workload(2, N=5), 3),
    ("ns_split_ec_roe_lgl7", inputs.workload(3, curved=True), 3),
    ("ns_split_ec_volflux_roe_lgl3", inputs.workload(3, riemann="volflux_roe", N=3, curved=True), 4),
    ("euler_split_ec_volflux_lgl6", inputs.workload(3, eqn="euler", riemann="volflux", N=6, curved=True), 2),
    ("ns_split_kep_roe_lgl1", inputs.workload(2, N=1), 4),
    ("ns_split_kep_roe_lgl8", inputs.workload(2, N=8), 2),
]


@pytest.mark.parametrize("name,wl,k", CASES, ids=[c[0] for c in CASES])
def test_rhs_parity_rotated(dg, orc, name, wl, k):
    print(f"case {name}", flush=True)
    M, (Xr, nbr, side, flip), _, _, U = rotated_problem(orc, wl, k)
    S = dg.DGSolver.from_workload(wl, Xr, nbr, side, flip=flip)
    ref = M.rhs(orc.Scheme.of(wl), U)
    got = S.rhs(to_gpu(U)).cpu().numpy()
    ne, per = check_rhs(got, ref)
    print(f"normwise {ne:.2e} per-variable {per}")


@pytest.mark.parametrize("name,wl,k", [CASES[4], CASES[5]], ids=[CASES[4][0], CASES[5][0]])
def test_rotation_invariance_gpu(dg, orc, name, wl, k):
    """The library on the rotated mesh against the library on the lattice, carried over."""
    print(f"case {name}", flush=True)
    M, (Xr, nbr_r, side_r, flip_r), (X, nbr, side), nm, Ur = rotated_problem(orc, wl, k)
    inv = np.argsort(nm, axis=1)                       # lattice node -> rotated node
    U = np.take_along_axis(Ur, inv[:, None, :], axis=2)
    Sr = dg.DGSolver.from_workload(wl, Xr, nbr_r, side_r, flip=flip_r)
    S = dg.DGSolver.from_workload(wl, X, nbr, side)
    a = np.take_along_axis(S.rhs(to_gpu(U)).cpu().numpy(), nm[:, None, :], axis=2)
    b = Sr.rhs(to_gpu(Ur)).cpu().numpy()
    err = rel_err(b, a)
    print(f"per-variable {err}")
    assert np.all(err <= 1e-12), err


def test_rk_parity_rotated(dg, orc):
    wl = inputs.workload(2, N=4)
    M, (Xr, nbr, side, flip), _, _, U = rotated_problem(orc, wl, 3, seed=11, perturb=0)
    sc = orc.Scheme.of(wl)
    dt = M.timestep(sc, U, wl.cfl, wl.dfl)
    ref = M.rk(sc, U, 20, dt)
    S = dg.DGSolver.from_workload(wl, Xr, nbr, side, flip=flip)
    got = S.steps(to_gpu(U), 20, dt).cpu().numpy()
    err = rel_err(got, ref)
    print(f"per-variable after 20 steps {err}")
    assert np.all(err <= 1e-10), err


def test_batch_with_rotated_member(dg, orc):
    """A rotated member and a lattice member in one batch: each equals its own stage bitwise."""
    import torch
    wl = inputs.workload(2, N=5)
    _, (Xr, nbr_r, side_r, flip_r), (X, nbr, side), _, Ur = rotated_problem(orc, wl, 3)
    M0 = orc.OracleMesh(X, nbr, side, wl.N, wl.nodes)
    U0 = inputs.random_perturbation(inputs.initial_state(wl, M0.points()), 5, 1e-2)
    sols = [dg.DGSolver.from_workload(wl, Xr, nbr_r, side_r, flip=flip_r),
            dg.DGSolver.from_workload(wl, X, nbr, side)]
    Us = [to_gpu(Ur), to_gpu(U0)]
    a, b, _ = dg.rk_coefficients()
    dts = [S.timestep(U) for S, U in zip(sols, Us)]
    R0 = [torch.full_like(U, 1e-4) for U in Us]
    ref = []
    for S, U, R, dt in zip(sols, Us, R0, dts):
        out, Rr = S.empty(), R.clone()
        S.rk_stage(U, out, Rr, a[1], b[1], dt)
        ref.append((out, Rr))
    B = dg.Batch(sols)
    outs = [S.empty() for S in sols]
    Rs = [R.clone() for R in R0]
    B.rk_stage(Us, outs, Rs, a[1], b[1], dts)
    torch.cuda.synchronize()
    for i, ((ro, rR), o, Rb) in enumerate(zip(ref, outs, Rs)):
        assert torch.equal(o, ro), f"member {i} U_out differs"
        assert torch.equal(Rb, rR), f"member {i} R differs"


def test_vjp_refuses_rotated_mesh(dg, orc):
    wl = inputs.workload(5, K1=2)
    _, (Xr, nbr, side, flip), _, _, U = rotated_problem(orc, wl, 2)
    S = dg.DGSolver.from_workload(wl, Xr, nbr, side, flip=flip)
    Ug = to_gpu(U)
    with pytest.raises(dg.DGError) as ei:
        S.rhs_vjp(Ug, Ug.clone())
    assert ei.value.code == -3
