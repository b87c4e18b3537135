"""Shared helpers of the GPU parity tests: problem construction and error measures.

Mesh coordinates are sampled at the oracle's LGL nodes and the same arrays are handed to
both sides, so oracle inputs never come from the GPU path.
"""
from __future__ import annotations

import numpy as np

from paper_1910_02858_amd import inputs


def problem(orc, wl, kxyz=None, curved=None, perturb=1e-2, seed=3):
    k = wl.K1
    kx, ky, kz = kxyz if kxyz else (k, k, k)
    cv = wl.curved if curved is None else curved
    lgl = orc.basis(wl.N, "lgl")["x"]
    X = inputs.lattice_points(lgl, kx, ky, kz)
    xgeo = inputs.warp_sine(X) if cv else X
    nbr, side, _ = inputs.periodic_lattice(kx, ky, kz)
    M = orc.OracleMesh(xgeo, nbr, side, wl.N, wl.nodes)
    U0 = inputs.initial_state(wl, M.points())
    if perturb:
        U0 = inputs.random_perturbation(U0, seed, perturb)
    return M, xgeo, nbr, side, U0


def gpu_solver(dg, wl, xgeo, nbr, side):
    return dg.DGSolver.from_workload(wl, xgeo, nbr, side)


def rel_err(g, o):
    """per-variable max-norm relative error max|g-o| / max|o| over all nodes"""
    g = np.asarray(g)
    o = np.asarray(o)
    num = np.abs(g - o).max(axis=(0, 2))
    den = np.abs(o).max(axis=(0, 2))
    return num / np.maximum(den, 1e-300)


def norm_err(g, o):
    """max-norm relative error of the whole vector: max|g-o| / max|o|"""
    g = np.asarray(g)
    o = np.asarray(o)
    return float(np.abs(g - o).max() / max(np.abs(o).max(), 1e-300))


def flux_scale(U, N, h, gamma=1.4):
    """max |F(U)| (N+1)^2 / h: size of the individual terms the operator sums at a node"""
    rho = U[:, 0]
    u = U[:, 1:4] / rho[:, None]
    p = (gamma - 1) * (U[:, 4] - 0.5 * rho * (u ** 2).sum(1))
    F = np.abs(U[:, 4] + p)[:, None] * np.abs(u)
    Fm = np.abs(U[:, 1:4]) * np.abs(u).max(1, keepdims=True) + np.abs(p)[:, None]
    return float(max(F.max(), Fm.max(), 1e-300)) * (N + 1) ** 2 / h


def check_rhs(got, ref, tol=1e-12):
    """Parity bar of one operator evaluation: max-norm relative error <= tol for the whole
    vector and for every conservative variable separately."""
    ne = norm_err(got, ref)
    den = np.abs(ref).max(axis=(0, 2))
    per = np.abs(np.asarray(got) - ref).max(axis=(0, 2)) / np.maximum(den, 1e-300)
    assert ne <= tol, f"normwise {ne:.3e}"
    assert np.all(per <= tol), f"per-variable {per}"
    return ne, per


def to_gpu(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).cuda()


def block_around(e, kxyz, radius=2):
    """global element indices of the (2r+1)^3 periodic block centred on element e"""
    kx, ky, kz = kxyz
    ex, ey, ez = e % kx, (e // kx) % ky, e // (kx * ky)
    r = radius
    idx = []
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                idx.append(((ex + dx) % kx) + kx * (((ey + dy) % ky) + ky * ((ez + dz) % kz)))
    return np.array(idx), (2 * r + 1) ** 3 // 2
