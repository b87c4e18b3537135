"""The allocation-free entry point dg_integrals_noalloc against dg_integrals.

Two calls in a row on one GPU, the second on a smaller mesh, each compared with the allocating
entry point on the same state (same kernels and summation order: equal bit for bit), and the
size limit of the static scratch refused with DG_ERR_UNSUPPORTED.
"""
import numpy as np
import pytest

from paper_1910_02858_amd import inputs
from gpu_common import problem, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    from paper_1910_02858_amd import dgsem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def test_integrals_noalloc_matches_integrals(dg, orc):
    import torch
    cases = [("ns_tgv_kep_lgl5_k6_curved", inputs.workload(2, K1=6)),
             ("euler_dwave_lg3_k3", inputs.workload(1, K1=3))]
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    for name, wl in cases:  # the second mesh is the smaller one
        print(f"case {name}", flush=True)
        M, xgeo, nbr, side, U0 = problem(orc, wl)
        S = dg.DGSolver.from_workload(wl, xgeo, nbr, side)
        Ug = to_gpu(U0)
        S.integrals_noalloc(Ug, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = S.integrals(Ug)
        assert np.array_equal(got, ref), (got, ref)
        # and both against the oracle's quadrature of the conserved variables, kinetic energy
        # and entropy (the oracle sums in another order: rounding only)
        o = M.integrals(U0)
        np.testing.assert_allclose(got[:7], o, rtol=1e-12, atol=1e-12 * np.abs(o).max())


def test_integrals_noalloc_refuses_meshes_beyond_the_scratch(dg):
    import torch
    k = 52  # 52^3 = 140608 elements > 131072 = 2^20 / 8
    wl = inputs.workload(1, N=1, K1=k, nodes="lgl")
    lgl = np.array([-1.0, 1.0])
    X = inputs.lattice_points(lgl, k, k, k)
    nbr, side, _ = inputs.periodic_lattice(k, k, k)
    S = dg.DGSolver.from_workload(wl, X, nbr, side)
    U = torch.from_numpy(inputs.constant_state(S.K, S.n3)).cuda()
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DGError) as ei:
        S.integrals_noalloc(U, out)
    assert ei.value.code == -3
