"""CPU-side checks of libdgsem: it loads, exports every symbol include/dgsem.h declares, and
its host setup (nodes, weights, RK table, argument and mesh validation) is right.  No kernel
is launched here; dg_init is only driven into errors it reports before touching the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1910_02858_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dg():
    from paper_1910_02858_amd import dgsem
    if not os.path.exists(dgsem.LIB_PATH):
        from paper_1910_02858_amd import build
        build.build()
    dgsem.lib()
    return dgsem


def test_exports_match_header(dg):
    hdr = open(os.path.join(ROOT, "include", "dgsem.h")).read()
    declared = set(re.findall(r"\b(dg_[a-z_]+)\s*\(", hdr))
    declared = {d for d in declared if d not in ("dg_mesh", "dg_scheme")}
    L = ctypes.CDLL(dg.LIB_PATH)
    missing = [d for d in sorted(declared) if not hasattr(L, d)]
    assert not missing, missing
    assert set(dg.EXPORTS) <= declared


@pytest.mark.parametrize("N", range(1, 9))
@pytest.mark.parametrize("t", ["lg", "lgl"])
def test_nodes_match_oracle(dg, orc, N, t):
    x, w = dg.nodes(N, t)
    b = orc.basis(N, t)
    np.testing.assert_allclose(x, b["x"], atol=4e-16)
    np.testing.assert_allclose(w, b["w"], atol=4e-16)


def test_rk_table_matches_oracle(dg, orc):
    for a, b in zip(dg.rk_coefficients(), orc.rk_coefficients()):
        np.testing.assert_array_equal(a, b)


def test_status_strings(dg):
    L = dg.lib()
    for code in range(0, -7, -1):
        assert L.dg_status_string(code).decode().startswith("DG_")


def _init(dg, xgeo, nbr, side, N, nodes="lgl", form="split", flip=None):
    m = dg._Mesh(xgeo.shape[0], N, xgeo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), side.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                 None if flip is None else flip.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    sc = dg._Scheme(1, dg.FORM[form], 0, 1, 1.4, 1.0, 1e-3, 0.72)
    h = ctypes.c_void_p()
    rc = dg.lib().dg_init(ctypes.byref(m), N, dg.NODES[nodes], ctypes.byref(sc), None, ctypes.byref(h))
    return rc, h


def _mesh(dg, N, k=2):
    lgl, _ = dg.nodes(N, "lgl")
    X = np.ascontiguousarray(inputs.lattice_points(lgl, k, k, k))
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    return X, nbr, side, flip


def test_init_rejects_empty_mesh(dg):
    """No elements: DG_ERR_ARG from dg_init and dg_host_geometry, before any device call."""
    X, nbr, side, _ = _mesh(dg, 3)
    rc, h = _init(dg, X[:0].copy(), nbr[:0].copy(), side[:0].copy(), 3)
    assert rc == -1 and not h.value
    with pytest.raises(dg.DGError) as ei:
        dg.host_geometry(X[:0], nbr[:0], side[:0], 3, "lgl")
    assert ei.value.code == -1


def test_init_rejects_inverted_element(dg):
    X, nbr, side, _ = _mesh(dg, 3)
    X[1, 0] = X[1, 0, ::-1].copy()  # mirror one element in x: J < 0
    rc, h = _init(dg, np.ascontiguousarray(X), nbr, side, 3)
    assert rc == -2 and not h.value


def test_init_rejects_unsupported(dg):
    X, nbr, side, flip = _mesh(dg, 3)
    rc, h = _init(dg, X, nbr, side, 9)            # N beyond the largest supported degree
    assert rc in (-3, -1) and not h.value
    rc, h = _init(dg, X, nbr, side, 3, nodes="lg", form="split")  # split needs LGL
    assert rc == -3
    nb, sd = nbr.copy(), side.copy()
    nb[0, 1], sd[0, 1] = -1, 5                     # a boundary of a kind that does not exist
    rc, h = _init(dg, X, nb, sd, 3)
    assert rc == -3


def test_init_rejects_inconsistent_faces(dg):
    """Sides, orientation codes and coordinates of the two sides of a face must agree."""
    X, nbr, side, flip = _mesh(dg, 3)
    bad = side.copy()
    bad[0, 1] = 3                                  # the neighbour does not name this side back
    rc, h = _init(dg, X, nbr, bad, 3)
    assert rc == -2 and not h.value
    fl = flip.copy()
    fl[0, 0] = 1                                   # neighbour's code is not the inverse
    rc, h = _init(dg, X, nbr, side, 3, flip=fl)
    assert rc == -2
    fl = flip.copy()
    fl[0, 0] = 8                                   # no such orientation
    rc, h = _init(dg, X, nbr, side, 3, flip=fl)
    assert rc == -2
    fl = flip.copy()
    nb, ns = nbr[0, 0], side[0, 0]
    fl[0, 0] = fl[nb, ns] = 3                      # reciprocal codes, but the points do not match
    with pytest.raises(dg.DGError) as ei:
        dg.host_geometry(X, nbr, side, 3, "lgl", flip=fl)
    assert ei.value.code == -2


def _rotated(dg, N, k=3, seed=4, curved=True):
    lgl, _ = dg.nodes(N, "lgl")
    X = inputs.lattice_points(lgl, k, k, k)
    X = inputs.warp_sine(X) if curved else X
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    rot = np.random.default_rng(seed).integers(0, 24, k ** 3)
    return inputs.rotate_elements(X, nbr, side, flip, N, rot)


@pytest.mark.parametrize("N", [2, 5])
@pytest.mark.parametrize("nodes", ["lg", "lgl"])
def test_host_geometry_box_matches_oracle(dg, orc, N, nodes):
    """A curved box whose outer faces are symmetry planes, element axes rotated: tables agree."""
    lgl, _ = dg.nodes(N, "lgl")
    X = inputs.warp_sine(inputs.lattice_points(lgl, 3, 3, 3, box=(np.pi,) * 3))
    nbr, side, flip = inputs.box_lattice(3, 3, 3)
    rot = np.random.default_rng(9).integers(0, 24, 27)
    Xr, nbr, side, flip, _ = inputs.rotate_elements(X, nbr, side, flip, N, rot)
    M = orc.OracleMesh(Xr, nbr, side, N, nodes, flip=flip)
    g = M.geometry()
    h = dg.host_geometry(Xr, nbr, side, N, nodes, flip=flip)
    eps = np.finfo(float).eps
    for key in ("Ja", "J", "fn"):
        assert np.abs(h[key] - g[key]).max() <= 1.0 * eps * np.abs(g[key]).max(), key


@pytest.mark.parametrize("N", [2, 5])
@pytest.mark.parametrize("nodes", ["lg", "lgl"])
def test_host_geometry_rotated_matches_oracle(dg, orc, N, nodes):
    """On a mesh whose faces meet on any side and in any orientation, dg_init's tables
    (including the master normals carried to the slaves) agree with the oracle's."""
    Xr, nbr, side, flip, _ = _rotated(dg, N)
    M = orc.OracleMesh(Xr, nbr, side, N, nodes, flip=flip)
    g = M.geometry()
    h = dg.host_geometry(Xr, nbr, side, N, nodes, flip=flip)
    eps = np.finfo(float).eps
    for key in ("Ja", "J", "fn"):
        assert np.abs(h[key] - g[key]).max() <= 1.0 * eps * np.abs(g[key]).max(), key


def test_init_rejects_broken_connectivity(dg):
    X, nbr, side, _ = _mesh(dg, 3)
    nb = nbr.copy()
    nb[0, 1] = 7  # not reciprocal
    rc, h = _init(dg, X, nb, side, 3)
    assert rc == -2
    nb = nbr.copy()
    nb[0, 1] = 99  # out of range
    rc, h = _init(dg, X, nb, side, 3)
    assert rc == -2
    nb, sd = nbr.copy(), side.copy()
    nb[0, 1], sd[0, 1] = -1, 0  # a symmetry plane whose neighbour still names this side
    rc, h = _init(dg, X, nb, sd, 3)
    assert rc == -2


def test_null_arguments(dg):
    L = dg.lib()
    h = ctypes.c_void_p()
    assert L.dg_init(None, 3, 1, None, None, ctypes.byref(h)) == -1
    assert L.dg_rhs(None, None, None) == -1
    assert L.dg_rk_stage(None, None, None, None, 0.0, 0.0, 0.0) == -1
    assert L.dg_rk_step_vjp(None, None, None, None, None, 0.0) == -1
    assert L.dg_rk_steps_vjp(None, 2, None, None, None, None, 0.0) == -1
    assert L.dg_rk_stage_keep(None, None, None, None, 0.0, 0.0, 0.0, None) == -1
    assert L.dg_set_boundary_state(None, None) == -1
    assert L.dg_set_wall_temperature(None, 1.0) == -1
    assert L.dg_set_outflow_pressure(None, 1.0) == -1
    assert L.dg_nodes(0, 1, None, None) == -1
    b = ctypes.c_void_p()
    assert L.dg_batch_create(None, 0, ctypes.byref(b)) == -1 and not b.value
    assert L.dg_batch_create(None, 1, None) == -1
    assert L.dg_batch_rk_stage(None, None, None, None, None, None, None) == -1
    assert L.dg_batch_step(None, None, None, None, None, 1) == -1
    assert L.dg_batch_tune(None, None, 1) == -1
    assert L.dg_batch_set_tile(None, 3, 1, 1) == -1
    assert L.dg_batch_info(None, None, 0) == -1
    assert L.dg_batch_last_error(None) == b"no batch"
    L.dg_batch_destroy(None)


@pytest.mark.parametrize("N", [3, 5, 7])
@pytest.mark.parametrize("nodes", ["lg", "lgl"])
@pytest.mark.parametrize("curved", [False, True])
def test_host_geometry_matches_oracle(dg, orc, N, nodes, curved):
    """dg_init's tables (extended precision, rounded once) agree with the oracle's to one ulp
    of each table's scale: D, Dhat, metric terms, Jacobian, face normals."""
    k = 3
    lgl = orc.basis(N, "lgl")["x"]
    X = inputs.lattice_points(lgl, k, k, k)
    xg = inputs.warp_sine(X) if curved else X
    nbr, side, _ = inputs.periodic_lattice(k, k, k)
    M = orc.OracleMesh(xg, nbr, side, N, nodes)
    g, b = M.geometry(), orc.basis(N, nodes)
    h = dg.host_geometry(xg, nbr, side, N, nodes)
    eps = np.finfo(float).eps
    for key, ref in (("D", b["D"]), ("Dhat", b["Dhat"]), ("Ja", g["Ja"]), ("J", g["J"]), ("fn", g["fn"])):
        assert np.abs(h[key] - ref).max() <= 1.0 * eps * np.abs(ref).max(), key


def test_rollout_rejects_empty_schedules():
    """Argument checks of the checkpointed rollout run before anything touches the GPU."""
    from paper_1910_02858_amd import dgsem
    with pytest.raises(ValueError):
        dgsem.rollout(None, None, 0, 0.1)
    with pytest.raises(ValueError):
        dgsem.rollout(None, None, 5, 0.1, ckpt_every=0)


@pytest.mark.parametrize("k,curved,seed", [(3, True, None), (3, True, 5), (2, False, 7), (1, False, 3)])
def test_mesh_connect_periodic(dg, k, curved, seed):
    """dg_mesh_connect rebuilds the connectivity of periodic lattices, also with every element's
    axes rotated (any side, any of the eight orientations), from the coordinates alone."""
    N = 3
    lgl, _ = dg.nodes(N, "lgl")
    X = inputs.lattice_points(lgl, k, k, k)
    X = inputs.warp_sine(X) if curved else X
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    if seed is not None:
        rot = np.random.default_rng(seed).integers(0, 24, k ** 3)
        X, nbr, side, flip, _ = inputs.rotate_elements(X, nbr, side, flip, N, rot)
    got = dg.mesh_connect(X, N, period=(2 * np.pi,) * 3)
    for a, b in zip(got, (nbr, side, flip)):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_mesh_connect_box(dg, kind):
    """Without periods the outer faces of a box become boundary sides of the requested kind."""
    N, m = 2, 3
    lgl, _ = dg.nodes(N, "lgl")
    X = inputs.warp_sine(inputs.lattice_points(lgl, m, m, m, box=(np.pi,) * 3))
    nbr, side, flip = inputs.box_lattice(m, m, m, kind=kind)
    rot = np.random.default_rng(kind).integers(0, 24, m ** 3)
    X, nbr, side, flip, _ = inputs.rotate_elements(X, nbr, side, flip, N, rot)
    got = dg.mesh_connect(X, N, bc_kind=kind)
    for a, b in zip(got, (nbr, side, flip)):
        np.testing.assert_array_equal(a, b)
    dg.host_geometry(X, *got[:2], N, "lgl", flip=got[2])  # accepted by dg_init's validation


def test_mesh_connect_arguments(dg):
    X = inputs.lattice_points(np.array([-1.0, 1.0]), 1, 1, 1)
    with pytest.raises(dg.DGError):
        dg.mesh_connect(X, 1, bc_kind=7)
    with pytest.raises(dg.DGError):
        dg.mesh_connect(X, 1, period=(-1.0, 0.0, 0.0))
    with pytest.raises(dg.DGError):
        dg.mesh_connect(np.zeros_like(X), 1)                     # degenerate element
    nbr, side, flip = dg.mesh_connect(X, 1)                      # one element, no periods
    assert np.all(nbr == -1) and np.all(side == 0) and np.all(flip == 0)
    nbr, side, flip = dg.mesh_connect(X, 1, period=(2 * np.pi,) * 3)
    assert np.all(nbr == 0) and np.array_equal(side[0], [1, 0, 3, 2, 5, 4])


def test_sfc_order_is_a_hilbert_curve(dg):
    """On a 2^3-cells-per-direction lattice a Hilbert curve steps from every element to a face
    neighbour; the order does not depend on how the elements were numbered before."""
    k = 8
    lgl, _ = dg.nodes(3, "lgl")
    X = inputs.lattice_points(lgl, k, k, k)
    order = dg.mesh_sfc_order(X, 3)
    assert np.array_equal(np.sort(order), np.arange(k ** 3))
    c = X.mean(axis=2)
    step = np.linalg.norm(np.diff(c[order], axis=0), axis=1) / (2 * np.pi / k)
    np.testing.assert_allclose(step, 1.0, rtol=1e-12)
    shuffle = np.random.default_rng(0).permutation(k ** 3)
    assert np.array_equal(shuffle[dg.mesh_sfc_order(X[shuffle], 3)], order)
    with pytest.raises(dg.DGError):
        dg.mesh_sfc_order(X * np.nan, 3)


def test_renumbered_mesh_connectivity(dg):
    """Renumbering along the curve keeps a valid mesh: the connectivity rebuilt from the
    renumbered coordinates equals the renumbered connectivity, and dg_init's checks pass."""
    N, k = 2, 4
    lgl, _ = dg.nodes(N, "lgl")
    X = inputs.warp_sine(inputs.lattice_points(lgl, k, k, k))
    nbr, side, flip = inputs.periodic_lattice(k, k, k)
    rnd = np.random.default_rng(1).permutation(k ** 3)
    X, nbr, side, flip = inputs.renumber_elements(X, nbr, side, flip, rnd)
    order = dg.mesh_sfc_order(X, N)
    Xs, nbs, sds, fls = inputs.renumber_elements(X, nbr, side, flip, order)
    got = dg.mesh_connect(Xs, N, period=(2 * np.pi,) * 3)
    for a, b in zip(got, (nbs, sds, fls)):
        np.testing.assert_array_equal(a, b)
    dg.host_geometry(Xs, nbs, sds, N, "lgl", flip=fls)


def test_outflow_on_both_node_sets(dg):
    N, m = 2, 2
    lgl, _ = dg.nodes(N, "lgl")
    X = inputs.lattice_points(lgl, m, m, m, box=(np.pi,) * 3)
    nbr, side, flip = inputs.box_lattice(m, m, m, kind=4)
    dg.host_geometry(X, nbr, side, N, "lgl", flip=flip)
    dg.host_geometry(X, nbr, side, N, "lg", flip=flip)


@pytest.mark.parametrize("N,ngeo", [(5, 2), (3, 1), (4, 6), (7, 3)])
@pytest.mark.parametrize("nodes", ["lg", "lgl"])
def test_host_geometry_degree_matches_oracle(dg, orc, N, ngeo, nodes):
    """Geometry of degree N_geo != N (Sec. 2.1): the library's tables, built from the mapping at
    the degree-N_geo LGL nodes, agree with the oracle's to a few ulps of each table's scale."""
    k = 3
    xg = inputs.warp_sine(inputs.lattice_points(orc.basis(ngeo, "lgl")["x"], k, k, k))
    nbr, side, _ = inputs.periodic_lattice(k, k, k)
    M = orc.OracleMesh(xg, nbr, side, N, nodes, ngeo=ngeo)
    g = M.geometry()
    h = dg.host_geometry(xg, nbr, side, N, nodes, ngeo=ngeo)
    eps = np.finfo(float).eps
    for key in ("Ja", "J", "fn"):
        assert np.abs(h[key] - g[key]).max() <= 2.0 * eps * np.abs(g[key]).max(), key
    with pytest.raises(ValueError):
        dg.host_geometry(xg, nbr, side, N, nodes)  # the point count names the degree


def _box_mesh_with_ids(dg, ngeo, m=3, kind=4, seed=2):
    lgl, _ = dg.nodes(ngeo, "lgl")
    X = inputs.lattice_points(lgl, m, m, m, box=(np.pi,) * 3)
    nbr, side, flip = inputs.box_lattice(m, m, m, kind=kind)
    rot = np.random.default_rng(seed).integers(0, 24, m ** 3)
    X, nbr, side, flip, _ = inputs.rotate_elements(X, nbr, side, flip, ngeo, rot)
    ids = inputs.global_node_ids(X)
    return inputs.warp_sine(X), ids, nbr, side, flip


@pytest.mark.parametrize("ngeo", [1, 3])
def test_mesh_file_round_trip(dg, tmp_path, ngeo):
    """Element packages (Sec. 2.1.1): the file read back, whole or as any contiguous range of
    elements, holds exactly what was written."""
    X, ids, nbr, side, flip = _box_mesh_with_ids(dg, ngeo)
    path = str(tmp_path / "box.mesh")
    dg.mesh_file_write(path, X, ids, nbr, side, flip)
    K = X.shape[0]
    n3 = (ngeo + 1) ** 3
    assert os.path.getsize(path) == 64 + K * (32 * n3 + 48)
    got = dg.mesh_file_read(path)
    assert got["ngeo"] == ngeo and got["mortar"] is None
    for a, b in ((got["xgeo"], X), (got["node_id"], ids), (got["nbr"], nbr), (got["side"], side),
                 (got["flip"], flip)):
        assert np.array_equal(a, b)
    for first, count in ((0, 1), (5, 7), (K - 4, 4)):
        part = dg.mesh_file_read(path, first, count)
        assert np.array_equal(part["xgeo"], X[first:first + count])
        assert np.array_equal(part["nbr"], nbr[first:first + count])
        assert np.array_equal(part["node_id"], ids[first:first + count])


def test_mesh_file_with_mortars(dg, orc, tmp_path):
    """A non-conforming mesh keeps its mortar kinds; the mesh read back gives the same geometry."""
    r = orc.basis(2, "lgl")["x"]
    X = inputs.refined_lattice(r, 2, (2, 2, 2))
    nbr, side, flip, mort = inputs.connect_boxes(X, 3)
    Xw = inputs.warp_bubble(X, 0.1, 2)
    path = str(tmp_path / "mortar.mesh")
    dg.mesh_file_write(path, Xw, inputs.global_node_ids(X), nbr, side, flip, mort)
    got = dg.mesh_file_read(path)
    assert np.array_equal(got["mortar"], mort) and np.array_equal(got["flip"], flip)
    a = dg.host_geometry(Xw, nbr, side, 4, "lgl", flip=flip, ngeo=2, mortar=mort)
    b = dg.host_geometry(got["xgeo"], got["nbr"], got["side"], 4, "lgl", flip=got["flip"], ngeo=2,
                         mortar=got["mortar"])
    for key in a:
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("ngeo,kind", [(1, 0), (2, 4), (3, 1)])
def test_mesh_connect_nodes(dg, ngeo, kind):
    """Connectivity from global node indices alone equals the lattice generator's, for elements
    with rotated reference axes (every side and orientation code), no tolerance involved."""
    X, ids, nbr, side, flip = _box_mesh_with_ids(dg, ngeo, kind=kind)
    got = dg.mesh_connect_nodes(ids, ngeo, bc_kind=kind)
    for a, b in zip(got, (nbr, side, flip)):
        np.testing.assert_array_equal(a, b)
    dg.host_geometry(X, *got[:2], 3, "lgl", flip=got[2], ngeo=ngeo)


def test_mesh_file_errors(dg, tmp_path):
    X, ids, nbr, side, flip = _box_mesh_with_ids(dg, 1, m=2)
    path = str(tmp_path / "m.mesh")
    dg.mesh_file_write(path, X, ids, nbr, side, flip)
    with pytest.raises(dg.DGError):
        dg.mesh_file_read(path, 6, 3)                       # beyond the last element
    with pytest.raises(dg.DGError):
        dg.mesh_file_read(str(tmp_path / "missing.mesh"))
    bad = tmp_path / "bad.mesh"
    bad.write_bytes(b"NOTAMESH" + bytes(120))
    with pytest.raises(dg.DGError):
        dg.mesh_file_read(str(bad))
    short = tmp_path / "short.mesh"
    short.write_bytes(open(path, "rb").read()[:200])
    with pytest.raises(dg.DGError):
        dg.mesh_file_read(str(short))
    three = np.concatenate([ids, ids[:1]])                  # a face shared by three sides
    with pytest.raises(dg.DGError) as ei:
        dg.mesh_connect_nodes(three, 1)
    assert ei.value.code == -2
    with pytest.raises(dg.DGError):
        dg.mesh_connect_nodes(ids, 1, bc_kind=9)
