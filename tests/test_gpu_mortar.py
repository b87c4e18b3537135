"""Non-conforming faces (Sec. 3.2, mortars of types 1, 2, 3) on the GPU against the oracle.

Refined lattices (half of the cells split 2x2x2, 1x2x1 or 1x1x2, so the x-faces between split
and whole cells are mortars of type 3, 1 or 2), curved by a polynomial map, optionally with every
element's reference axes rotated (mortar types, positions and orientation codes all change); the
same arrays go to the library and to the oracle.  One operator evaluation (1e-12), 20 RK steps
(1e-10), free stream on a mesh with exact metric terms, conservation, and the calls that do not
support mortars refuse them.
"""
import math

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


def mortar_problem(orc, wl, ngeo, split, k=2, rot_seed=None, degree=3, perturb=1e-2, seed=5):
    r = orc.basis(ngeo, "lgl")["x"]
    X = inputs.refined_lattice(r, k, split)
    if rot_seed is not None:
        rot = np.random.default_rng(rot_seed).integers(0, 24, X.shape[0])
        gm = np.stack([inputs.rotation_node_map(int(q), ngeo) for q in rot])
        X = np.take_along_axis(X, gm[:, None, :], axis=2)
    nbr, side, flip, mort = inputs.connect_boxes(X, ngeo + 1)
    Xw = inputs.warp_bubble(X, 0.1, degree)
    M = orc.OracleMesh(Xw, nbr, side, wl.N, wl.nodes, flip=flip, ngeo=ngeo, mortar=mort)
    U0 = inputs.initial_state(wl, M.points())
    if perturb:
        U0 = inputs.random_perturbation(U0, seed, perturb)
    return M, (Xw, nbr, side, flip, mort), U0


def mortar_solver(dg, wl, ngeo, mesh):
    Xw, nbr, side, flip, mort = mesh
    return dg.DGSolver.from_workload(wl, Xw, nbr, side, flip=flip, ngeo=ngeo, mortar=mort)


CASES = [
    ("euler_weak_lg3_llf_type3", inputs.workload(1, N=3), 3, (2, 2, 2), None),
    ("ns_split_kep_roe_lgl5_type3_rotated", inputs.workload(2, N=5), 3, (2, 2, 2), 7),
    ("ns_split_ec_volflux_roe_lgl7_type1", inputs.workload(3, riemann="volflux_roe"), 3, (1, 2, 1), None),
    ("ns_weak_lgl4_roe_type2_rotated", inputs.workload(2, form="weak", volflux="central", N=4), 2, (1, 1, 2), 8),
    ("ns_strong_lg4_llf_type1_rotated", inputs.workload(2, nodes="lg", form="strong", volflux="central",
                                                         riemann="llf", N=4), 3, (1, 2, 1), 9),
    ("ns_weak_lg3_roe_type3", inputs.workload(2, nodes="lg", form="weak", volflux="central", N=3), 3, (2, 2, 2),
     None),
    ("euler_split_ec_volflux_lgl6_type2", inputs.workload(3, eqn="euler", riemann="volflux", N=6), 3, (1, 1, 2),
     None),
    ("ns_split_kep_roe_lgl2_type3", inputs.workload(2, N=2), 1, (2, 2, 2), 10),
]


@pytest.mark.parametrize("name,wl,ngeo,split,rot", CASES, ids=[c[0] for c in CASES])
def test_rhs_parity_mortar(dg, orc, name, wl, ngeo, split, rot):
    print(f"case {name}", flush=True)
    M, mesh, U0 = mortar_problem(orc, wl, ngeo, split, rot_seed=rot)
    S = mortar_solver(dg, wl, ngeo, mesh)
    ref = M.rhs(orc.Scheme.of(wl), U0)
    got = S.rhs(to_gpu(U0)).cpu().numpy()
    ne, per = check_rhs(got, ref)
    print(f"normwise {ne:.2e} per-variable {per}")


@pytest.mark.parametrize("split", [(2, 2, 2), (1, 2, 1)])
def test_rk_parity_mortar(dg, orc, split):
    wl = inputs.workload(2, N=4)
    M, mesh, U0 = mortar_problem(orc, wl, 2, split, rot_seed=3, perturb=0)
    sc = orc.Scheme.of(wl)
    dt = M.timestep(sc, U0, wl.cfl, wl.dfl)
    ref = M.rk(sc, U0, 20, dt)
    S = mortar_solver(dg, wl, 2, mesh)
    got = S.steps(to_gpu(U0), 20, dt).cpu().numpy()
    err = rel_err(got, ref)
    print(f"per-variable after 20 steps {err}")
    assert np.all(err <= 1e-10), err


@pytest.mark.parametrize("split", [(2, 2, 2), (1, 2, 1), (1, 1, 2)])
@pytest.mark.parametrize("wl", [inputs.workload(2, N=4), inputs.workload(1, N=4, curved=True)],
                         ids=["ns_split_kep_lgl4", "euler_weak_lg4"])
def test_mortar_freestream_and_conservation_gpu(dg, orc, split, wl):
    """Exact metric terms (geometry of degree 2, N = 4): a uniform flow stays uniform; any state
    conserves mass, momentum and energy to rounding."""
    M, mesh, U0 = mortar_problem(orc, wl, 2, split, rot_seed=4, degree=2)
    S = mortar_solver(dg, wl, 2, mesh)
    Uc = inputs.constant_state(M.K, M.n3)
    Ut = S.rhs(to_gpu(Uc)).cpu().numpy()
    fscale = np.abs(Uc).max() * 2 * (wl.N + 1) ** 2 / (math.pi / 2)
    assert np.abs(Ut).max() < 1e-12 * fscale
    Utg = S.rhs(to_gpu(U0))
    tot = S.integrals(Utg)[:5]
    w = orc.basis(wl.N, wl.nodes)["w"]
    wq = np.einsum("k,j,i->kji", w, w, w).ravel()[None] * M.geometry()["J"]
    scale = np.einsum("eq,evq->v", wq, np.abs(Utg.cpu().numpy()))
    assert np.all(np.abs(tot) < 1e-13 * scale), (tot, scale)


def test_mortar_unsupported_calls(dg, orc):
    import torch
    wl = inputs.workload(2, N=3)
    M, mesh, U0 = mortar_problem(orc, wl, 3, (2, 2, 2))
    S = mortar_solver(dg, wl, 3, mesh)
    U = to_gpu(U0)
    with pytest.raises(dg.DGError) as ei:
        S.rhs_vjp(U, torch.ones_like(U))
    assert ei.value.code == -3
    with pytest.raises(dg.DGError) as ei:
        dg.Batch([S])
    assert ei.value.code == -3
