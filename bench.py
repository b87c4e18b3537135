"""Benchmark: DOF updates per second of the DGSEM RK step (Navier-Stokes TGV, N=7, 48^3 elements).

One step = five stages of the 2N-storage Runge-Kutta scheme, each stage = BR1 lifting
kernel + main operator kernel with the RK update fused (split form, entropy-conserving
two-point flux, Roe surface flux), on 56.6 M nodes x 5 variables in FP64 resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--elements 48]

Prints one JSON line.  value = DOF-updates/s = nodes * steps * 5 / wall (DOF counted per
variable, as the paper's performance index does); PID = 1/value seconds per DOF per stage.
The roofline object is for the dominant kernel, timed with HIP events on the library's
stream over extra profiled stages after the timed region; its algorithmic bytes are the
compulsory HBM traffic per node (37 doubles read+write for the main kernel, 22 for the
lifting kernel).  cpu_baseline is the FP64 oracle on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s (PID s/DOF/stage) at N=7 TGV; adjoint/forward cost ratio"
HBM_PEAK_GBS = 8000.0
# split-form operator at N = 7: U 5 + viscous divergence 4 + own face traces of the viscous
# fluxes 3 (24 n^2 values per element, n = 8) + Ja 9 + 1/J 1 + R 5 read, U_new 5 + R 5 written
BYTES_MAIN = 37 * 8
# lifting for the split form: U 5 + Ja 9 + 1/J 1 read, viscous divergence 4 + face traces 3 written
BYTES_LIFT = 22 * 8
# weak-form operator at N = 7 (Navier-Stokes): U 5 + viscous volume term 4 + own face viscous fluxes 3
# (24 n^2 per element) + face normals 2.25 (18 n^2) + Ja 9 + 1/J 1 + R 5 read, U_new 5 + R 5 written
BYTES_WEAK_MAIN = 39.25 * 8
# reverse stage: k_vjp_main reads U 5, the kept viscous fluxes' momentum part 9, Ja 9, 1/J 1,
# Ubar_t 5, Ubar 5 and writes Ubar 5; k_vjp_face reads Ubar 5, Rbar 5 and writes Rbar 5
BYTES_VJP_MAIN = 39 * 8
BYTES_VJP_FACE = 15 * 8


def bytes_fv(n: int) -> float:
    """Algorithmic bytes per subcell of the finite-volume kernel: U 5, R 5, Jbar 1 and the face-mean
    metrics of the three directions (9 (n+1)/n) read, U_new 5 and R 5 written."""
    return 8.0 * (5 + 5 + 1 + 9.0 * (n + 1) / n + 5 + 5)


# HBM traffic of the split kernel from committed counter summaries: FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch) of one rocprofv3 --pmc pass each, scaled by the factors a 1 GiB
# device-to-device copy gives on the same box; valid only while the kernel sources still hash
# to the value recorded with the counters.
COUNTERS = os.path.join(ROOT, "profiles", "k_split_ns_ec_n7_k48_counters.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1910_02858_amd", "csrc", f) for f in ("dg_kernels.hip", "dg_internal.h")]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic():
    """(bytes per launch, source hash matches) from the committed counter summary, or (None, False)."""
    try:
        kv = {}
        with open(COUNTERS) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        fetch = float(kv["FETCH_SIZE_KiB"]) * float(kv["fetch_scale"])
        write = float(kv["WRITE_SIZE_KiB"]) * float(kv["write_scale"])
        return (fetch + write) * 1024.0, kv.get("kernel_source_sha256") == kernel_source_hash()
    except (OSError, KeyError, ValueError):
        return None, False


def _oracle_stages(orc, inputs, wl, k, budget_s):
    """(DOF updates per second, stages, DOF) of the oracle's RK stage for workload wl on k^3 elements."""
    lgl = orc.basis(wl.N, "lgl")["x"]
    X = inputs.lattice_points(lgl, k, k, k)
    if wl.curved:
        X = inputs.warp_sine(X)
    nbr, side, _ = inputs.periodic_lattice(k, k, k)
    M = orc.OracleMesh(X, nbr, side, wl.N, wl.nodes)
    U = inputs.initial_state(wl, M.points())
    R = np.zeros_like(U)
    sc = orc.Scheme.of(wl)
    a, b, _ = orc.rk_coefficients()
    stages = 0
    t0 = time.perf_counter()
    while True:
        U, R = M.rk_stage(sc, U, R, a[stages % 5], b[stages % 5], 1e-4)
        stages += 1
        if time.perf_counter() - t0 > budget_s and stages >= 2:
            break
    wall = time.perf_counter() - t0
    dof = M.K * M.n3
    return dof * stages / wall, stages, dof, wall


def cpu_baseline(wl, budget_s: float = 12.0):
    """Time the oracle's RK stage on a bounded sample of the same workload (16^3 elements, N=7:
    131 k nodes per host thread at 16 threads, where the cost per node no longer depends on the
    size), and the small workloads in full (Euler density wave, the curved 16^3 N=5 TGV, the 12^3
    N=5 adjoint workload's forward stage) for context."""
    from oracle import oracle as orc
    from paper_1910_02858_amd import inputs
    k = 16
    value, stages, dof, wall = _oracle_stages(orc, inputs, wl, k, budget_s)
    configs = {}
    for idx in (1, 2, 5):
        w = inputs.workload(idx)
        v, st, d, _ = _oracle_stages(orc, inputs, w, w.K1, 2.0)
        configs[w.name] = {"value": v, "stages": st, "dof": d}
    return {"value": value, "unit": "DOF-updates/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{stages} RK stages of the same scheme on {k}^3 elements, N={wl.N} ({dof} nodes), FP64",
            "pid_core_s": wall * orc.num_threads() / (dof * stages), "pid_1thread_s": cpu_pid_one_thread(),
            "configs": configs}


_ONE_THREAD = r"""
import sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import oracle as orc
from paper_1910_02858_amd import inputs
wl = inputs.workload(3, K1=4)
lgl = orc.basis(wl.N, "lgl")["x"]
X = inputs.lattice_points(lgl, 4, 4, 4)
nbr, side, _ = inputs.periodic_lattice(4, 4, 4)
M = orc.OracleMesh(X, nbr, side, wl.N, wl.nodes)
U = inputs.initial_state(wl, M.points())
R = np.zeros_like(U)
sc = orc.Scheme.of(wl)
a, b, _ = orc.rk_coefficients()
t0 = time.perf_counter()
for s in range(10):
    U, R = M.rk_stage(sc, U, R, a[s % 5], b[s % 5], 1e-4)
print((time.perf_counter() - t0) / (M.K * M.n3 * 10))
"""


def cpu_pid_one_thread():
    """The oracle's seconds per DOF and stage on one host thread (4^3 elements, N=7, 10 stages),
    in a child process started with OMP_NUM_THREADS=1; None if that fails."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", _ONE_THREAD, os.path.dirname(os.path.abspath(__file__))],
                             env=env, capture_output=True, text=True, timeout=120)
        return float(out.stdout.strip().splitlines()[-1]) if out.returncode == 0 else None
    except (OSError, ValueError, IndexError, subprocess.SubprocessError):
        return None


def adjoint_ratio(dgsem, inputs, torch, repeats: int = 2, general: bool = False, k1=None, steps=None):
    """Wall time of the gradient (checkpoint recomputation + reverse stages) over the wall time
    of the forward rollout that stores the checkpoints: 12^3 curved hexes, N=5, split KEP + Roe +
    BR1, Taylor-Green vortex, 50 RK steps, checkpoint every 10 steps, objective = kinetic energy.
    With ``general`` the mesh is the vortex's symmetry octant with six symmetry planes and
    rotated element axes."""
    wl = inputs.workload(5) if k1 is None else inputs.workload(5, K1=k1)
    if steps is not None:
        wl.steps = steps
    S, U0 = (dgsem.build_solver(wl, rotate_seed=0, symmetry_box=True) if general else dgsem.build_solver(wl))
    dt = S.timestep(U0, wl.cfl, wl.dfl)
    wJ = S.mass_weights()
    best_f, best_b = float("inf"), float("inf")
    for _ in range(repeats + 1):  # the first round warms up
        U = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        UT = dgsem.rollout(S, U, wl.steps, dt, ckpt_every=10)
        ke = dgsem.kinetic_energy(UT, wJ)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (g,) = torch.autograd.grad(ke, U)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        best_f, best_b = min(best_f, t1 - t0), min(best_b, t2 - t1)
    return {"value": best_b / best_f, "forward_ms": best_f * 1e3, "backward_ms": best_b * 1e3,
            "workload": (wl.name.replace("_k12", f"_k{wl.K1}") +
                         ("_octant_symmetry_planes_rotated_elements" if general else "")),
            "dof": S.K * S.n3, "steps": wl.steps, "checkpoint_every": 10}


def ensemble_bench(dgsem, inputs, torch, steps: int = 10, n_members: int = 256):
    """Seeded ensemble of uneven members (K1 ~ U{4..12}, N ~ U{3..7}, amplitude and Mach drawn per
    member; split KEP + Roe + BR1, TGV): DOF updates per second of whole RK steps for
    (a) the batched step replayed as one HIP graph, with one lifting and one operator launch per
    stage for all degrees (fused) and with one pair per degree, (b) the batched stages launched
    eagerly and (c) every member advanced with its own one-mesh launches, all on the same GPU;
    ``batched_graph`` is the launch mode the tuner chose."""
    wls = inputs.ensemble_draw(n_members, 0)
    sols, U0s = [], []
    for wl in wls:
        S, U = dgsem.build_solver(wl)
        sols.append(S)
        U0s.append(U)
    dts = [S.timestep(U, wl.cfl, wl.dfl) for S, U, wl in zip(sols, U0s, wls)]
    dof = sum(S.K * S.n3 for S in sols)
    B = dgsem.Batch(sols)
    tiles = B.tune(U0s, repeats=3)
    cur = [U.clone() for U in U0s]
    nxt = [S.empty() for S in sols]
    Rs = [torch.zeros_like(U) for U in U0s]

    def batched(nsteps, graph):
        nonlocal cur, nxt
        for _ in range(nsteps):
            B.step(cur, nxt, Rs, dts, graph=graph)
            cur, nxt = nxt, cur

    def unbatched(nsteps):
        nonlocal cur, nxt
        a, b, _ = dgsem.rk_coefficients()
        for _ in range(nsteps):
            for s in range(5):
                for S, u, o, R, dt in zip(sols, cur, nxt, Rs, dts):
                    S.rk_stage(u, o, R, a[s], b[s], dt)
                cur, nxt = nxt, cur

    chosen = B.fused
    out = {"members": len(sols), "dof": dof, "steps": steps, "tiles": [list(t) for t in tiles],
           "launch": "fused" if chosen else "per_degree"}

    def fused_graph(k):
        B.fused = True
        batched(k, True)

    def per_degree_graph(k):
        B.fused = False
        batched(k, True)

    for name, fn in (("batched_graph_fused", fused_graph), ("batched_graph_per_degree", per_degree_graph),
                     ("batched_eager", lambda k: batched(k, False)), ("per_member_launches", unbatched)):
        if name == "batched_eager":
            B.fused = chosen
        fn(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = dof * 5 * steps / wall
    B.fused = chosen
    out["batched_graph"] = out["batched_graph_fused" if chosen else "batched_graph_per_degree"]
    if not all(S.check_finite(u) for S, u in zip(sols, cur)):
        raise RuntimeError("non-finite ensemble state")
    out["speedup_vs_per_member"] = out["batched_graph"] / out["per_member_launches"]
    return out


def ec_branch_bench(S, U_smooth, torch, wl, smooth_main_ms: float, stages: int = 5):
    """The EC flux's logarithmic means under real jumps: the headline state with every conservative
    variable multiplied by 1 + 0.1 xi per node (xi ~ N(0,1), seeded), so that most node pairs'
    density and beta ratios take the logarithm branch ((a-b)/(a+b))^2 >= 1e-4 instead of the
    series; the operator kernel's time (HIP events, ``stages`` RK stages) against the smooth TGV's."""
    g = torch.Generator(device="cuda").manual_seed(7)
    U = U_smooth * (1.0 + 0.1 * torch.randn(U_smooth.shape, generator=g, device="cuda", dtype=torch.float64))
    n = wl.N + 1
    rho = U[:, 0].reshape(-1, n, n, n)
    ke = 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2 + U[:, 3] ** 2) / U[:, 0]
    p = 0.4 * (U[:, 4] - ke)  # gamma = 1.4
    beta = (0.5 * U[:, 0] / p).reshape(-1, n, n, n)
    del ke

    def log_frac(a):
        r = (a[..., 1:] - a[..., :-1]) / (a[..., 1:] + a[..., :-1])
        return float(((r * r) >= 1e-4).double().mean())

    fr, fb = log_frac(rho), log_frac(beta)
    del rho, beta, p
    dt = S.timestep(U, wl.cfl, wl.dfl)
    R = torch.zeros_like(U)
    nxt = S.empty()
    from paper_1910_02858_amd import dgsem
    a, b, _ = dgsem.rk_coefficients()
    S.profile(True)
    cur = U
    for s_ in range(stages):
        S.rk_stage(cur, nxt, R, a[s_ % 5], b[s_ % 5], dt)
        cur, nxt = nxt, cur
    prof = S.profile_read()
    S.profile(False)
    if not S.check_finite(cur):
        raise RuntimeError("non-finite state in the EC branch measurement")
    main_ms = prof["main_ms"] / max(prof["main_launches"], 1)
    return {"state": "TGV x (1 + 0.1 xi) per node and variable", "pairs_log_branch_rho": fr,
            "pairs_log_branch_beta": fb, "main_ms": main_ms, "smooth_main_ms": smooth_main_ms,
            "slowdown": main_ms / smooth_main_ms, "stages": stages}


def weak_form_bench(dgsem, inputs, torch, stages: int = 10):
    """The weak and strong forms (k_main: the D-hat or D contraction of the fluxes along every
    line, on LG nodes the face prolongation): the Euler density-wave scheme at N=3 on 96^3 LG
    elements, the Navier-Stokes TGV (central volume flux, Roe, BR1) in weak and strong form at N=7
    on 48^3 on LG and on LGL nodes (strong form on LGL nodes: the split form's reads), all
    56.6 M nodes; per-kernel times (the lifting's includes the LG prolongation), the operator
    kernel priced at 314 B per node (weak form, strong form on LG nodes: face normals and face
    fluxes), 296 B (strong form on LGL nodes) or at its Euler reads and writes (U 5, Ja 9, 1/J 1,
    R 5 read, U_new 5, R 5 written: 240 B)."""
    out = {}
    for name, wl, nbytes in (("euler_dwave_lg3_k96_weak", inputs.workload(1, K1=96), 30 * 8),
                             ("ns_tgv_central_roe_lg7_k48_weak",
                              inputs.workload(3, form="weak", volflux="central", nodes="lg", K1=48), BYTES_WEAK_MAIN),
                             ("ns_tgv_central_roe_lgl7_k48_weak",
                              inputs.workload(3, form="weak", volflux="central", K1=48), BYTES_WEAK_MAIN),
                             ("ns_tgv_central_roe_lgl7_k48_strong",
                              inputs.workload(3, form="strong", volflux="central", K1=48), BYTES_MAIN),
                             ("ns_tgv_central_roe_lg7_k48_strong",
                              inputs.workload(3, form="strong", volflux="central", nodes="lg", K1=48), BYTES_WEAK_MAIN)):
        S, U = dgsem.build_solver(wl)
        dt = S.timestep(U, wl.cfl, wl.dfl)
        a, b, _ = dgsem.rk_coefficients()
        R = torch.zeros_like(U)
        nxt = S.empty()
        cur = U
        for s_ in range(5):  # warm-up
            S.rk_stage(cur, nxt, R, a[s_], b[s_], dt)
            cur, nxt = nxt, cur
        S.profile(True)
        for s_ in range(stages):
            S.rk_stage(cur, nxt, R, a[s_ % 5], b[s_ % 5], dt)
            cur, nxt = nxt, cur
        prof = S.profile_read()
        S.profile(False)
        if not S.check_finite(cur):
            raise RuntimeError("non-finite state in the weak-form measurement")
        dof = S.K * S.n3
        main_ms = prof["main_ms"] / max(prof["main_launches"], 1)
        lift_ms = prof["lift_ms"] / max(prof["lift_launches"], 1) if prof["lift_launches"] else 0.0
        gbs = nbytes * dof / (main_ms * 1e-3) / 1e9
        out[name] = {"dof": dof, "kernels_ms": {"main": main_ms, "lift": lift_ms},
                     "value": dof / ((main_ms + lift_ms) * 1e-3),
                     "roofline": {"bound": "hbm", "kernel": "k_main (" + name.rsplit("_", 1)[1] + " form)", "achieved": gbs,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                  "algorithmic_bytes_per_dof": nbytes}}
        del S, U, R, nxt, cur
        torch.cuda.empty_cache()
    return out


def general_mesh_bench(dgsem, inputs, torch, wl, steps: int, structured_value: float):
    """The same element count and scheme on the vortex's symmetry octant [0, pi]^3 with six
    symmetry planes and every element's reference axes rotated (seeded proper rotations of the
    cube): faces meet on any side and in all eight orientations, and the outer faces are
    boundaries, so the kernels read the face codes.  DOF updates per second of whole RK steps and
    the per-kernel durations."""
    t0 = time.perf_counter()
    S, U = dgsem.build_solver(wl, rotate_seed=0, symmetry_box=True)
    setup_s = time.perf_counter() - t0
    dof = S.K * S.n3
    dt = S.timestep(U, wl.cfl, wl.dfl)
    a, b, _ = dgsem.rk_coefficients()
    R = torch.zeros_like(U)
    cur, nxt = U, S.empty()
    for s in range(5):
        S.rk_stage(cur, nxt, R, a[s], b[s], dt)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s in range(5):
            S.rk_stage(cur, nxt, R, a[s], b[s], dt)
            cur, nxt = nxt, cur
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not S.check_finite(cur):
        raise RuntimeError("non-finite state on the rotated mesh")
    S.profile(True)
    for s in range(5):
        S.rk_stage(cur, nxt, R, a[s], b[s], dt)
        cur, nxt = nxt, cur
    prof = S.profile_read()
    S.profile(False)
    value = dof * 5 * steps / wall
    return {"workload": wl.name + "_octant_symmetry_planes_rotated_elements", "value": value, "unit": "DOF-updates/s", "steps": steps,
            "ms_per_stage": wall * 1e3 / (5 * steps),
            "kernels_ms": {"main": prof["main_ms"] / max(prof["main_launches"], 1),
                           "lift": prof["lift_ms"] / max(prof["lift_launches"], 1)},
            "vs_structured": value / structured_value, "setup_s": setup_s}


def _timed_steps(S, U, torch, dgsem, dt, steps, between=None):
    """Wall time of ``steps`` RK steps after one warm-up step, then per-kernel times of 5 profiled
    stages; ``between(U)`` runs before every step (e.g. the FV switch).  Returns (wall, prof, U)."""
    a, b, _ = dgsem.rk_coefficients()
    R = torch.zeros_like(U)
    cur, nxt = U, S.empty()
    for st in range(steps + 1):
        if st == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        if between is not None:
            between(cur)
        for s_ in range(5):
            S.rk_stage(cur, nxt, R, a[s_], b[s_], dt)
            cur, nxt = nxt, cur
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not S.check_finite(cur):
        raise RuntimeError("non-finite state")
    S.profile(True)
    for s_ in range(5):
        S.rk_stage(cur, nxt, R, a[s_], b[s_], dt)
        cur, nxt = nxt, cur
    prof = S.profile_read()
    S.profile(False)
    return wall, prof, cur


def _per_launch(prof, key):
    n = prof[key + "_launches"]
    return prof[key + "_ms"] / n if n else None


def mortar_bench(dgsem, inputs, torch, steps: int, structured_value: float, k: int = 16):
    """Non-conforming faces (Sec. 3.2): the headline scheme (N=7, split EC + Roe + BR1, TGV) on a
    periodic k^3 lattice whose half x < pi is refined 2x2x2, so the two planes between refined and
    whole cells carry type-3 mortars (4 small sides per big side).  DOF updates per second of
    whole RK steps and the per-kernel times (the mortar flux kernel is the face entry)."""
    wl = inputs.workload(3)
    lgl, _ = dgsem.nodes(wl.N, "lgl")
    t0 = time.perf_counter()
    X = inputs.refined_lattice(lgl, k, (2, 2, 2))
    nbr, side, flip, mort = inputs.connect_boxes(X, wl.N + 1)
    S = dgsem.DGSolver.from_workload(wl, X, nbr, side, flip=flip, mortar=mort)
    setup_s = time.perf_counter() - t0
    del X
    U = torch.from_numpy(inputs.initial_state(wl, S.node_coords())).cuda()
    dt = S.timestep(U, wl.cfl, wl.dfl)
    wall, prof, _ = _timed_steps(S, U, torch, dgsem, dt, steps)
    dof = S.K * S.n3
    value = dof * 5 * steps / wall
    return {"workload": f"ns_tgv_ec_roe_lgl7_k{k}_half_refined_2x2x2", "elements": S.K,
            "mortars": int(((mort >= 1) & (mort <= 3)).sum()), "dof": dof, "value": value, "unit": "DOF-updates/s",
            "steps": steps, "ms_per_stage": wall * 1e3 / (5 * steps),
            "kernels_ms": {"main": _per_launch(prof, "main"), "lift": _per_launch(prof, "lift"),
                           "mortar_flux": _per_launch(prof, "face")},
            "vs_structured": value / structured_value, "setup_s": setup_s}


def fv_bench(dgsem, inputs, torch, steps: int, k: int = 32):
    """Finite-volume subcells (Sec. 4), Euler equations, N=7, split EC volume flux + Roe, on a
    periodic k^3 lattice: the pure DG step; the hybrid step on a periodic shock tube (a dense slab
    2 < x < 4) with the indicator's switch before every step; and every element finite-volume
    (the FV kernel's roofline, algorithmic bytes per subcell from bytes_fv)."""
    import numpy as np
    wl = inputs.workload(3, eqn="euler", K1=k)
    S, _ = dgsem.build_solver(wl)
    x = S.node_coords()
    inside = (x[:, 0] > 2.0) & (x[:, 0] < 4.0)
    rho = np.where(inside, 1.0, 0.3)
    p = np.where(inside, 1.0, 0.2)
    U0 = torch.from_numpy(np.ascontiguousarray(inputs.prim_to_cons(rho, 0 * rho + 0.1, 0 * rho, 0 * rho, p, 1.4))).cuda()
    del x, inside, rho, p
    dt = S.timestep(U0, 0.5, 0.5)
    dof = S.K * S.n3
    out = {"workload": f"euler_shock_tube_ec_roe_lgl7_k{k}", "elements": S.K, "dof": dof, "steps": steps}
    wall, prof, _ = _timed_steps(S, U0.clone(), torch, dgsem, dt, steps)
    out["dg"] = {"value": dof * 5 * steps / wall, "ms_per_stage": wall * 1e3 / (5 * steps)}
    t0 = time.perf_counter()
    S.fv_enable(1, -5.0, -2.5)
    out["fv_setup_s"] = time.perf_counter() - t0
    U = U0.clone()
    wall, prof, U = _timed_steps(S, U, torch, dgsem, dt, steps, between=S.fv_switch)
    fvn = int(S.fv_types().sum())
    out["hybrid"] = {"value": dof * 5 * steps / wall, "ms_per_stage": wall * 1e3 / (5 * steps),
                     "fv_elements": fvn, "fv_fraction": fvn / S.K,
                     "kernels_ms": {"dg": _per_launch(prof, "main"), "faces": _per_launch(prof, "face"),
                                    "fv": _per_launch(prof, "fv")}}
    S.fv_set_types(np.ones(S.K, np.uint8))  # the slab's nodal values read as subcell means
    wall, prof, _ = _timed_steps(S, U0.clone(), torch, dgsem, dt, steps)
    fv_ms = _per_launch(prof, "fv")
    fv_gbs = bytes_fv(wl.N + 1) * dof / (fv_ms * 1e-3) / 1e9
    out["all_fv"] = {"value": dof * 5 * steps / wall, "ms_per_stage": wall * 1e3 / (5 * steps),
                     "kernels_ms": {"dg": _per_launch(prof, "main"), "faces": _per_launch(prof, "face"),
                                    "fv": fv_ms},
                     "roofline": {"bound": "hbm", "kernel": "k_fv_volume", "achieved": fv_gbs, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": fv_gbs / HBM_PEAK_GBS,
                                  "algorithmic_bytes_per_dof": bytes_fv(wl.N + 1)}}
    out["hybrid_vs_dg"] = out["hybrid"]["value"] / out["dg"]["value"]
    return out


def adjoint_roofline(dgsem, inputs, torch, k: int = 32, repeats: int = 3):
    """The reverse sweep at an HBM-resident size: 32^3 curved hexes, N=5, split KEP + Roe + BR1
    (7.1 M nodes, 283 MB per state, beyond the 256 MB last-level cache).  One forward step keeps
    its stage inputs and lifting outputs; its reverse (five k_vjp_main + k_vjp_face pairs and one
    register update) is applied ``repeats`` times (the adjoint of one step applied again: linear,
    no reset needed) and timed with events on the library's stream, beside the same forward
    stages, and priced at BYTES_VJP_MAIN + BYTES_VJP_FACE per node and stage."""
    wl = inputs.workload(5, K1=k)
    S, U0 = dgsem.build_solver(wl)
    dt = S.timestep(U0, wl.cfl, wl.dfl)
    a, b, _ = dgsem.rk_coefficients()
    stage_U = [U0] + [S.empty() for _ in range(4)]
    stage_G = [S.empty_grad() for _ in range(5)]
    R = torch.zeros_like(U0)
    out_U = S.empty()
    st = torch.cuda.current_stream()

    def forward():
        for s_ in range(5):
            S.rk_stage_keep(stage_U[s_], stage_U[s_ + 1] if s_ < 4 else out_U, R, a[s_], b[s_], dt, stage_G[s_])

    forward()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(repeats):
        forward()
    e1.record(st)
    torch.cuda.synchronize()
    fwd_stage_ms = e0.elapsed_time(e1) / (5 * repeats)
    g = torch.Generator(device="cpu").manual_seed(1)
    Ub = torch.randn(U0.shape, generator=g, dtype=torch.float64).cuda()
    Rb = torch.zeros_like(U0)
    S.rk_step_vjp(stage_U, stage_G, Ub, Rb, dt)
    e0.record(st)
    for _ in range(repeats):
        S.rk_step_vjp(stage_U, stage_G, Ub, Rb, dt)
    e1.record(st)
    torch.cuda.synchronize()
    if not bool(torch.isfinite(Ub).all()):
        raise RuntimeError("non-finite adjoint")
    rev_stage_ms = e0.elapsed_time(e1) / (5 * repeats)
    dof = S.K * S.n3
    gbs = (BYTES_VJP_MAIN + BYTES_VJP_FACE) * dof / (rev_stage_ms * 1e-3) / 1e9
    return {"workload": f"ns_tgv_kep_roe_lgl5_k{k}_curved", "dof": dof, "forward_stage_ms": fwd_stage_ms,
            "reverse_stage_ms": rev_stage_ms, "reverse_over_forward_stage": rev_stage_ms / fwd_stage_ms,
            "roofline": {"bound": "hbm", "kernel": "k_vjp_main + k_vjp_face (one reverse stage)", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_dof": BYTES_VJP_MAIN + BYTES_VJP_FACE}}


def order_bench(dgsem, inputs, torch, wl, steps: int, lexicographic_value: float):
    """Element order study on the headline lattice: the elements numbered at random, and the same
    mesh renumbered along the Hilbert curve of its element centroids (dg_mesh_sfc_order).  DOF
    updates per second of whole RK steps and per-kernel durations of each, against the
    lexicographic numbering of the headline run."""
    import numpy as np
    lgl, _ = dgsem.nodes(wl.N, "lgl")
    k = wl.K1
    X = inputs.lattice_points(lgl, k, k, k)
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    rnd = np.random.default_rng(0).permutation(k ** 3)
    out = {}
    for name, order in (("random", rnd), ("hilbert", None)):
        if order is None:
            order = rnd[dgsem.mesh_sfc_order(X[rnd], wl.N)]
        Xo, nbo, sdo, flo = inputs.renumber_elements(X, nbr, side, flip, order)
        S = dgsem.DGSolver.from_workload(wl, Xo, nbo, sdo, flip=flo)
        del Xo
        U = torch.from_numpy(np.ascontiguousarray(inputs.initial_state(wl, S.node_coords()))).cuda()
        dof = S.K * S.n3
        dt = S.timestep(U, wl.cfl, wl.dfl)
        a, b, _ = dgsem.rk_coefficients()
        R = torch.zeros_like(U)
        cur, nxt = U, S.empty()
        for st in range(steps + 1):
            if st == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            for s_ in range(5):
                S.rk_stage(cur, nxt, R, a[s_], b[s_], dt)
                cur, nxt = nxt, cur
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if not S.check_finite(cur):
            raise RuntimeError("non-finite state in the element order study")
        S.profile(True)
        for s_ in range(5):
            S.rk_stage(cur, nxt, R, a[s_], b[s_], dt)
            cur, nxt = nxt, cur
        prof = S.profile_read()
        S.profile(False)
        value = dof * 5 * steps / wall
        out[name] = {"value": value, "ms_per_stage": wall * 1e3 / (5 * steps),
                     "kernels_ms": {"main": prof["main_ms"] / max(prof["main_launches"], 1),
                                    "lift": prof["lift_ms"] / max(prof["lift_launches"], 1)},
                     "vs_lexicographic": value / lexicographic_value}
        del S, U, R, cur, nxt
        torch.cuda.empty_cache()
    out["steps"] = steps
    return out


def progress(msg: str):
    """One line on stderr as each measurement ends (the JSON result line goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# the optional measurements beside the headline, each switched off by --no-<name>
LEGS = ("cpu", "adjoint", "ensemble", "general", "mortar", "fv", "weak", "ec-branch", "adjoint-roofline")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--elements", type=int, default=48, help="elements per direction")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--profile-stages", type=int, default=10)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost measurement")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble measurement")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the measurement on the same mesh with rotated element axes")
    ap.add_argument("--no-mortar", action="store_true", help="skip the non-conforming-mesh measurement")
    ap.add_argument("--no-fv", action="store_true", help="skip the finite-volume subcell measurement")
    ap.add_argument("--no-weak", action="store_true", help="skip the weak-form (LG) operator measurement")
    ap.add_argument("--no-ec-branch", action="store_true",
                    help="skip the EC flux measurement on a state with jumps (logarithm branch)")
    ap.add_argument("--no-adjoint-roofline", action="store_true",
                    help="skip the reverse sweep's roofline at 32^3, N=5")
    ap.add_argument("--order-study", action="store_true",
                    help="also time the lattice with random and with Hilbert-curve element numbering")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the run, copy a 1 GiB device buffer 3 times (reference for HBM counters)")
    ap.add_argument("--only", choices=LEGS + ("none",), default=None,
                    help="run the headline and this one extra measurement only (none: the headline only; "
                         "for profiler runs)")
    args = ap.parse_args()
    if args.only is not None:
        for leg in LEGS:
            if leg != args.only:
                setattr(args, "no_" + leg.replace("-", "_"), True)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the element decomposition across GPUs is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_02858_amd import dgsem, inputs

    wl = inputs.workload(3, K1=args.elements)
    torch.cuda.set_device(0)
    S, U = dgsem.build_solver(wl)
    dof = S.K * S.n3
    dt = S.timestep(U, wl.cfl, wl.dfl)
    a, b, _ = dgsem.rk_coefficients()
    R = torch.zeros_like(U)
    spare = S.empty()

    def run(nsteps, U, spare):
        cur, nxt = U, spare
        for _ in range(nsteps):
            for s in range(5):
                S.rk_stage(cur, nxt, R, a[s], b[s], dt)
                cur, nxt = nxt, cur
        return cur, nxt

    U, spare = run(args.warmup, U, spare)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, spare = run(args.steps, U, spare)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not S.check_finite(U):
        print("non-finite solution after the timed steps", file=sys.stderr)
        sys.exit(1)

    # per-kernel durations (HIP events on the library's stream), extra stages after the timed region
    S.profile(True)
    cur, nxt = U, spare
    for s in range(max(args.profile_stages, 1)):
        S.rk_stage(cur, nxt, R, a[s % 5], b[s % 5], dt)
        cur, nxt = nxt, cur
    prof = S.profile_read()
    S.profile(False)
    main_ms = prof["main_ms"] / max(prof["main_launches"], 1)
    lift_ms = prof["lift_ms"] / max(prof["lift_launches"], 1)
    main_gbs = BYTES_MAIN * dof / (main_ms * 1e-3) / 1e9
    lift_gbs = BYTES_LIFT * dof / (lift_ms * 1e-3) / 1e9

    ec_branch = None
    if not args.no_ec_branch and wl.volflux == "ec":
        ec_branch = ec_branch_bench(S, U, torch, wl, main_ms)
        progress("EC logarithm branch done")
        torch.cuda.empty_cache()

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # bandwidth of a plain device-to-device copy on the same GPU (context for the fractions); not
    # in counter passes, whose only copies are the 1 GiB calibration copies above
    copy_gbs = None
    if not args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst

    stages = args.steps * 5
    value = dof * stages / wall
    progress(f"headline done: {value:.4g} DOF-updates/s")
    tbytes, tvalid = counter_traffic()
    traffic_gbs = tbytes / (main_ms * 1e-3) / 1e9 if (tbytes is not None and tvalid and args.elements == 48) else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name if args.elements == 48 else f"{wl.name}_k{args.elements}",
                   "elements": S.K, "N": wl.N, "nodes": "lgl", "dof": dof, "stages_per_step": 5,
                   "scheme": "navier-stokes split EC volume flux, Roe surface flux, BR1", "ic": "taylor-green Ma=0.1 Re=1600"},
        "pid_s_per_dof_stage": wall / (dof * stages),
        "pid_cu_s": wall * 256 / (dof * stages),  # per compute unit, context beside per-core CPU PIDs
        "ms_per_stage": wall * 1e3 / stages,
        "kernels_ms": {"main": main_ms, "lift": lift_ms},
        "roofline": {"bound": "hbm", "kernel": "k_split (face fluxes + split volume integral + surface integral + RK update)", "achieved": main_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": main_gbs / HBM_PEAK_GBS, "traffic": traffic_gbs,
                     "traffic_bytes_per_launch": tbytes if traffic_gbs is not None else None,
                     "algorithmic_bytes_per_dof": BYTES_MAIN},
        "roofline_lift": {"achieved": lift_gbs, "frac": lift_gbs / HBM_PEAK_GBS,
                          "algorithmic_bytes_per_dof": BYTES_LIFT},
        "stage_hbm_frac": (BYTES_MAIN + BYTES_LIFT) * dof * stages / wall / 1e9 / HBM_PEAK_GBS,
        "copy_gbs": copy_gbs,
        "stage_frac_of_copy": ((BYTES_MAIN + BYTES_LIFT) * dof * stages / wall / 1e9 / copy_gbs
                               if copy_gbs else None),
        "adjoint_forward_ratio": None,
    }
    if ec_branch is not None:
        out["ec_log_branch"] = ec_branch
    if not args.no_adjoint:
        adj = adjoint_ratio(dgsem, inputs, torch)
        progress("adjoint ratio done")
        out["adjoint_forward_ratio"] = adj["value"]
        out["adjoint"] = adj
    if not args.no_ensemble:
        out["ensemble"] = ensemble_bench(dgsem, inputs, torch)
        progress("ensemble done")
    freed = False
    if not args.no_general:
        del S, U, R, spare, cur, nxt
        freed = True
        torch.cuda.empty_cache()
        out["general_mesh"] = general_mesh_bench(dgsem, inputs, torch, wl, 5, value)
        progress("general mesh done")
        if not args.no_adjoint:
            out["general_mesh"]["adjoint"] = adjoint_ratio(dgsem, inputs, torch, repeats=1, general=True)
    if (not args.no_mortar or not args.no_fv or not args.no_weak or not args.no_adjoint_roofline or
            args.order_study) and not freed:
        del S, U, R, spare, cur, nxt
        freed = True
    torch.cuda.empty_cache()
    if not args.no_adjoint_roofline:
        out["adjoint_hbm"] = adjoint_roofline(dgsem, inputs, torch)
        progress("reverse roofline done")
        if not args.no_adjoint:
            # the adjoint/forward rollout ratio at the same size (20 steps, checkpoint every 10)
            out["adjoint_hbm"]["rollout"] = adjoint_ratio(dgsem, inputs, torch, repeats=1, k1=32, steps=20)
        torch.cuda.empty_cache()
    if not args.no_mortar:
        out["mortar"] = mortar_bench(dgsem, inputs, torch, 5, value)
        progress("mortars done")
        torch.cuda.empty_cache()
    if not args.no_fv:
        out["fv"] = fv_bench(dgsem, inputs, torch, 5)
        progress("FV subcells done")
        torch.cuda.empty_cache()
    if not args.no_weak:
        out["weak_form"] = weak_form_bench(dgsem, inputs, torch)
        progress("weak form done")
        torch.cuda.empty_cache()
    if args.order_study:
        out["element_order"] = order_bench(dgsem, inputs, torch, wl, 5, value)
    if not args.no_cpu:
        cb = cpu_baseline(wl)
        progress("CPU baseline done")
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["pid_core_s"] = cb["pid_core_s"]
        out["cpu_baseline"]["pid_1thread_s"] = cb["pid_1thread_s"]
        out["cpu_baseline"]["configs"] = cb["configs"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
