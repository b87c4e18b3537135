"""Python binding of libdgsem (include/dgsem.h): argument marshalling only.

Device memory and streams come from PyTorch; every step of the operator runs in the
library's HIP kernels.  Importing this module does not load the library; the first use
does, and raises if ``libdgsem.so`` has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgsem.so")

DG_OK = 0
STATUS = {0: "DG_OK", -1: "DG_ERR_ARG", -2: "DG_ERR_MESH", -3: "DG_ERR_UNSUPPORTED", -4: "DG_ERR_HIP",
          -5: "DG_ERR_NONFINITE", -6: "DG_ERR_OOM"}
NODES = {"lg": 0, "lgl": 1}
EQN = {"euler": 0, "ns": 1}
FORM = {"weak": 0, "split": 1, "strong": 2}
VF = {"kep": 0, "ec": 1, "central": 2}
RS = {"llf": 0, "roe": 1, "volflux": 2, "volflux_roe": 3}

EXPORTS = [
    "dg_nodes", "dg_rk_coefficients", "dg_init", "dg_set_stream", "dg_set_boundary_state", "dg_set_wall_temperature", "dg_set_outflow_pressure", "dg_mesh_connect", "dg_mesh_sfc_order", "dg_rhs", "dg_rk_stage", "dg_rhs_vjp",
    "dg_rk_stage_vjp", "dg_timestep", "dg_integrals", "dg_check_finite", "dg_node_coords", "dg_info", "dg_destroy",
    "dg_status_string", "dg_last_error", "dg_batch_create", "dg_batch_rk_stage", "dg_batch_destroy", "dg_profile",
    "dg_profile_read", "dg_host_geometry", "dg_mass_weights", "dg_batch_step", "dg_batch_tune", "dg_batch_set_tile",
    "dg_batch_set_fused", "dg_batch_fused",
    "dg_batch_info", "dg_batch_last_error", "dg_rk_stage_keep", "dg_rk_step_vjp", "dg_rk_steps_vjp",
    "dg_integrals_noalloc", "dg_profile_read_ex", "dg_mesh_file_write", "dg_mesh_file_info", "dg_mesh_file_read",
    "dg_mesh_connect_nodes", "dg_fv_enable", "dg_fv_set_types", "dg_fv_types", "dg_fv_indicator", "dg_fv_switch",
]


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("n_elems", ctypes.c_int32), ("n_geo", ctypes.c_int32), ("xgeo", ctypes.POINTER(ctypes.c_double)),
                ("nbr_elem", ctypes.POINTER(ctypes.c_int32)), ("nbr_side", ctypes.POINTER(ctypes.c_int8)),
                ("flip", ctypes.POINTER(ctypes.c_int8)), ("mortar", ctypes.POINTER(ctypes.c_int8))]


class _Scheme(ctypes.Structure):
    _fields_ = [("eqn", ctypes.c_int32), ("form", ctypes.c_int32), ("volflux", ctypes.c_int32),
                ("riemann", ctypes.c_int32), ("gamma", ctypes.c_double), ("R", ctypes.c_double),
                ("mu", ctypes.c_double), ("Pr", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libdgsem.so (raises if it is missing: the GPU path has no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1910_02858_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.dg_nodes.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.dg_rk_coefficients.argtypes = [_D, _D, _D]
        L.dg_init.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Scheme), _VP,
                              ctypes.POINTER(_VP)]
        L.dg_set_stream.argtypes = [_VP, _VP]
        L.dg_set_boundary_state.argtypes = [_VP, ctypes.POINTER(ctypes.c_double)]
        L.dg_set_wall_temperature.argtypes = [_VP, ctypes.c_double]
        L.dg_set_outflow_pressure.argtypes = [_VP, ctypes.c_double]
        L.dg_mesh_sfc_order.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32)]
        L.dg_mesh_connect.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8),
                                      ctypes.POINTER(ctypes.c_int8)]
        L.dg_rhs.argtypes = [_VP, _VP, _VP]
        L.dg_rk_stage.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.dg_rhs_vjp.argtypes = [_VP, _VP, _VP, _VP]
        L.dg_rk_stage_vjp.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.dg_rk_stage_keep.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_double, _VP]
        L.dg_rk_step_vjp.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP, _VP, ctypes.c_double]
        L.dg_rk_steps_vjp.argtypes = [_VP, ctypes.c_int, ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP, _VP,
                                      ctypes.c_double]
        L.dg_timestep.argtypes = [_VP, _VP, ctypes.c_double, ctypes.c_double, _D]
        L.dg_integrals.argtypes = [_VP, _VP, _D]
        L.dg_integrals_noalloc.argtypes = [_VP, _VP, _VP]
        _U8 = ctypes.POINTER(ctypes.c_uint8)
        L.dg_fv_enable.argtypes = [_VP, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.dg_fv_set_types.argtypes = [_VP, _U8]
        L.dg_fv_types.argtypes = [_VP, _U8]
        L.dg_fv_indicator.argtypes = [_VP, _VP, _D]
        L.dg_fv_switch.argtypes = [_VP, _VP]
        L.dg_check_finite.argtypes = [_VP, _VP]
        L.dg_node_coords.argtypes = [_VP, _D]
        L.dg_mass_weights.argtypes = [_VP, _VP]
        L.dg_info.argtypes = [_VP, ctypes.POINTER(ctypes.c_int64)]
        L.dg_destroy.argtypes = [_VP]
        L.dg_destroy.restype = None
        L.dg_status_string.restype = ctypes.c_char_p
        L.dg_status_string.argtypes = [ctypes.c_int]
        L.dg_last_error.restype = ctypes.c_char_p
        L.dg_last_error.argtypes = [_VP]
        L.dg_host_geometry.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_int, ctypes.c_int] + [_D] * 5
        L.dg_profile.argtypes = [_VP, ctypes.c_int]
        L.dg_profile_read.argtypes = [_VP, _D]
        L.dg_profile_read_ex.argtypes = [_VP, _D, ctypes.c_int]
        _I64 = ctypes.POINTER(ctypes.c_int64)
        _I32 = ctypes.POINTER(ctypes.c_int32)
        _I8 = ctypes.POINTER(ctypes.c_int8)
        L.dg_mesh_file_write.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, _D, _I64, _I32, _I8, _I8, _I8]
        L.dg_mesh_file_info.argtypes = [ctypes.c_char_p, _I64]
        L.dg_mesh_file_read.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.c_int, _D, _I64, _I32, _I8, _I8, _I8]
        L.dg_mesh_connect_nodes.argtypes = [ctypes.c_int, ctypes.c_int, _I64, ctypes.c_int, _I32, _I8, _I8]
        L.dg_batch_create.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(_VP)]
        L.dg_batch_rk_stage.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP), _D, _D, _D]
        L.dg_batch_destroy.argtypes = [_VP]
        L.dg_batch_destroy.restype = None
        L.dg_batch_step.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP), _D, ctypes.c_int]
        L.dg_batch_tune.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.c_int]
        L.dg_batch_set_tile.argtypes = [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.dg_batch_set_fused.argtypes = [_VP, ctypes.c_int]
        L.dg_batch_fused.argtypes = [_VP]
        L.dg_batch_info.argtypes = [_VP, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.dg_batch_last_error.restype = ctypes.c_char_p
        L.dg_batch_last_error.argtypes = [_VP]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def nodes(N: int, node_type: str):
    x, w = np.zeros(N + 1), np.zeros(N + 1)
    rc = lib().dg_nodes(N, NODES[node_type], _ptr(x), _ptr(w))
    if rc:
        raise DGError(rc, "dg_nodes")
    return x, w


def rk_coefficients():
    a, b, c = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().dg_rk_coefficients(_ptr(a), _ptr(b), _ptr(c))
    return a, b, c


def mesh_connect(xgeo, N: int, period=None, tol: float = 0.0, bc_kind: int = 0):
    """Connectivity (nbr_elem, nbr_side, flip) of a conforming hex mesh from its element
    coordinates ``xgeo[K][3][(N+1)^3]`` (``dg_mesh_connect``); ``period`` joins the opposite faces
    of a periodic box along the directions with a positive entry."""
    xgeo = np.ascontiguousarray(xgeo, np.float64)
    K = xgeo.shape[0]
    nbr = np.zeros((K, 6), np.int32)
    side = np.zeros((K, 6), np.int8)
    flip = np.zeros((K, 6), np.int8)
    per = None if period is None else np.ascontiguousarray(period, np.float64)
    rc = lib().dg_mesh_connect(K, N, _ptr(xgeo), None if per is None else _ptr(per), tol, bc_kind,
                               nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               side.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                               flip.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    if rc:
        raise DGError(rc, "dg_mesh_connect")
    return nbr, side, flip


def mesh_sfc_order(xgeo, N: int):
    """Element order along the Hilbert curve through the element centroids (``dg_mesh_sfc_order``):
    ``order[i]`` is the element at position ``i``."""
    xgeo = np.ascontiguousarray(xgeo, np.float64)
    order = np.zeros(xgeo.shape[0], np.int32)
    rc = lib().dg_mesh_sfc_order(xgeo.shape[0], N, _ptr(xgeo), order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise DGError(rc, "dg_mesh_sfc_order")
    return order


def _geo_degree(xgeo, N, ngeo):
    ng = N if ngeo is None else int(ngeo)
    if round(xgeo.shape[-1] ** (1.0 / 3.0)) ** 3 != xgeo.shape[-1] or xgeo.shape[-1] != (ng + 1) ** 3:
        raise ValueError("xgeo must hold (ngeo+1)^3 points per element")
    return ng


def _i8(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ct))


def mesh_file_write(path: str, xgeo, node_id, nbr, side, flip=None, mortar=None):
    """Write an element-package mesh file (``dg_mesh_file_write``); ``xgeo[K,3,(ngeo+1)^3]``."""
    xgeo = np.ascontiguousarray(xgeo, np.float64)
    K = xgeo.shape[0]
    ngeo = round(xgeo.shape[-1] ** (1.0 / 3.0)) - 1
    node_id = np.ascontiguousarray(node_id, np.int64)
    nbr, side = np.ascontiguousarray(nbr, np.int32), np.ascontiguousarray(side, np.int8)
    flip = None if flip is None else np.ascontiguousarray(flip, np.int8)
    mortar = None if mortar is None else np.ascontiguousarray(mortar, np.int8)
    rc = lib().dg_mesh_file_write(path.encode(), K, ngeo, _ptr(xgeo), _p(node_id, ctypes.c_int64),
                                  _p(nbr, ctypes.c_int32), _p(side, ctypes.c_int8), _p(flip, ctypes.c_int8),
                                  _p(mortar, ctypes.c_int8))
    if rc:
        raise DGError(rc, "dg_mesh_file_write")


def mesh_file_read(path: str, first: int = 0, count: Optional[int] = None):
    """Elements first .. first+count-1 of an element-package mesh file: a dict with xgeo, node_id,
    nbr, side, flip, mortar (None without mortar kinds), ngeo."""
    info = np.zeros(3, np.int64)
    rc = lib().dg_mesh_file_info(path.encode(), _p(info, ctypes.c_int64))
    if rc:
        raise DGError(rc, "dg_mesh_file_info")
    K, ngeo, flags = int(info[0]), int(info[1]), int(info[2])
    count = K - first if count is None else count
    n3 = (ngeo + 1) ** 3
    xgeo = np.zeros((count, 3, n3))
    node_id = np.zeros((count, n3), np.int64)
    nbr = np.zeros((count, 6), np.int32)
    side, flip, mortar = (np.zeros((count, 6), np.int8) for _ in range(3))
    rc = lib().dg_mesh_file_read(path.encode(), int(first), int(count), _ptr(xgeo), _p(node_id, ctypes.c_int64),
                                 _p(nbr, ctypes.c_int32), _p(side, ctypes.c_int8), _p(flip, ctypes.c_int8),
                                 _p(mortar, ctypes.c_int8))
    if rc:
        raise DGError(rc, "dg_mesh_file_read")
    return dict(xgeo=xgeo, node_id=node_id, nbr=nbr, side=side, flip=flip, mortar=mortar if flags & 1 else None,
                ngeo=ngeo)


def mesh_connect_nodes(node_id, ngeo: int, bc_kind: int = 0):
    """Conforming connectivity (nbr, side, flip) from global node indices (``dg_mesh_connect_nodes``)."""
    node_id = np.ascontiguousarray(node_id, np.int64)
    K = node_id.shape[0]
    nbr = np.zeros((K, 6), np.int32)
    side, flip = np.zeros((K, 6), np.int8), np.zeros((K, 6), np.int8)
    rc = lib().dg_mesh_connect_nodes(K, ngeo, _p(node_id, ctypes.c_int64), bc_kind, _p(nbr, ctypes.c_int32),
                                     _p(side, ctypes.c_int8), _p(flip, ctypes.c_int8))
    if rc:
        raise DGError(rc, "dg_mesh_connect_nodes")
    return nbr, side, flip


def host_geometry(xgeo, nbr, nside, N: int, node_type: str, flip=None, ngeo=None, mortar=None):
    """dg_init's geometry and 1D tables computed on the host only (no device needed).
    ``xgeo[K,3,(ngeo+1)^3]``: the mapping at the LGL nodes of degree ``ngeo`` (default N);
    ``mortar[K,6]``: non-conforming faces in the conventions of ``dg_mesh.mortar``."""
    xgeo = np.ascontiguousarray(xgeo, np.float64)
    nbr = np.ascontiguousarray(nbr, np.int32)
    nside = np.ascontiguousarray(nside, np.int8)
    flip = None if flip is None else np.ascontiguousarray(flip, np.int8)
    mortar = None if mortar is None else np.ascontiguousarray(mortar, np.int8)
    K, n = xgeo.shape[0], N + 1
    ng = _geo_degree(xgeo, N, ngeo)
    m = _Mesh(K, ng, _ptr(xgeo), nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
              nside.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _i8(flip), _i8(mortar))
    Ja, J, fn = np.zeros((K, 9, n ** 3)), np.zeros((K, n ** 3)), np.zeros((K, 6, 3, n * n))
    D, Dh = np.zeros((n, n)), np.zeros((n, n))
    rc = lib().dg_host_geometry(ctypes.byref(m), N, NODES[node_type], _ptr(Ja), _ptr(J), _ptr(fn), _ptr(D), _ptr(Dh))
    if rc:
        raise DGError(rc, "dg_host_geometry")
    return dict(Ja=Ja, J=J, fn=fn, D=D, Dhat=Dh)


def _dptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("solution arrays must be contiguous float64 CUDA tensors")
    return t.data_ptr()


class DGSolver:
    """One mesh + scheme on the GPU (a ``dg_handle``)."""

    def __init__(self, xgeo, nbr, nside, N: int, nodes_: str, eqn="ns", form="split", volflux="kep",
                 riemann="roe", gamma=1.4, R=1.0, mu=0.0, Pr=0.72, flip=None, stream=None, ngeo=None,
                 mortar=None):
        import torch
        self.torch = torch
        xgeo = np.ascontiguousarray(xgeo, np.float64)
        nbr = np.ascontiguousarray(nbr, np.int32)
        nside = np.ascontiguousarray(nside, np.int8)
        K = xgeo.shape[0]
        ng = N if ngeo is None else int(ngeo)
        if xgeo.shape != (K, 3, (ng + 1) ** 3) or nbr.shape != (K, 6) or nside.shape != (K, 6):
            raise ValueError("mesh arrays have inconsistent shapes")
        flip_arr = None if flip is None else np.ascontiguousarray(flip, np.int8)
        mort_arr = None if mortar is None else np.ascontiguousarray(mortar, np.int8)
        m = _Mesh(K, ng, _ptr(xgeo), nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  nside.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _i8(flip_arr), _i8(mort_arr))
        sc = _Scheme(EQN[eqn], FORM[form], VF[volflux], RS[riemann], gamma, R, mu, Pr)
        st = stream if stream is not None else torch.cuda.current_stream()
        h = _VP()
        rc = lib().dg_init(ctypes.byref(m), N, NODES[nodes_], ctypes.byref(sc), _VP(st.cuda_stream), ctypes.byref(h))
        if rc:
            raise DGError(rc, "dg_init")
        self.h = h
        self.K, self.N, self.n3 = K, N, (N + 1) ** 3
        self.shape = (K, 5, self.n3)
        self.eqn, self.form, self.volflux, self.riemann = eqn, form, volflux, riemann
        self.gamma, self.mu = gamma, mu
        self._stream = st.cuda_stream

    @classmethod
    def from_workload(cls, wl, xgeo, nbr, nside, **kw):
        return cls(xgeo, nbr, nside, wl.N, wl.nodes, wl.eqn, wl.form, wl.volflux, wl.riemann, wl.gamma, wl.R, wl.mu,
                   wl.Pr, **kw)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.dg_destroy(h)
            self.h = None

    def _check(self, rc, what):
        if rc:
            msg = lib().dg_last_error(self.h)
            raise DGError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_outflow_pressure(self, p: float):
        """Pressure of the mesh's outflow sides."""
        self._check(lib().dg_set_outflow_pressure(self.h, float(p)), "dg_set_outflow_pressure")

    def set_wall_temperature(self, tw: float):
        """Wall temperature of the mesh's isothermal wall sides."""
        self._check(lib().dg_set_wall_temperature(self.h, float(tw)), "dg_set_wall_temperature")

    def set_boundary_state(self, ub):
        """Outer state (rho, m1, m2, m3, E) of the mesh's given-state boundary sides."""
        ub = np.ascontiguousarray(ub, np.float64)
        if ub.shape != (5,):
            raise ValueError("the boundary state has 5 conservative components")
        self._check(lib().dg_set_boundary_state(self.h, _ptr(ub)), "dg_set_boundary_state")

    def _sync_stream(self):
        st = self.torch.cuda.current_stream().cuda_stream
        if st != self._stream:
            self._check(lib().dg_set_stream(self.h, _VP(st)), "dg_set_stream")
            self._stream = st

    def empty(self):
        return self.torch.empty(self.shape, dtype=self.torch.float64, device="cuda")

    def rhs(self, U, out=None):
        self._sync_stream()
        out = self.empty() if out is None else out
        self._check(lib().dg_rhs(self.h, _VP(_dptr(U)), _VP(_dptr(out))), "dg_rhs")
        return out

    def rk_stage(self, U_in, U_out, R, a, b, dt):
        self._sync_stream()
        self._check(lib().dg_rk_stage(self.h, _VP(_dptr(U_in)), _VP(_dptr(U_out)), _VP(_dptr(R)), float(a), float(b),
                                      float(dt)), "dg_rk_stage")

    def rhs_vjp(self, U, Ut_bar, out=None):
        self._sync_stream()
        out = self.empty() if out is None else out
        self._check(lib().dg_rhs_vjp(self.h, _VP(_dptr(U)), _VP(_dptr(Ut_bar)), _VP(_dptr(out))), "dg_rhs_vjp")
        return out

    def rk_stage_vjp(self, U_in, U_bar, R_bar, a, b, dt):
        self._sync_stream()
        self._check(lib().dg_rk_stage_vjp(self.h, _VP(_dptr(U_in)), _VP(_dptr(U_bar)), _VP(_dptr(R_bar)), float(a),
                                          float(b), float(dt)), "dg_rk_stage_vjp")

    def empty_grad(self):
        """device buffer for the lifted gradients of one state, [K][12][n^3]"""
        return self.torch.empty((self.K, 12, self.n3), dtype=self.torch.float64, device="cuda")

    def rk_stage_keep(self, U_in, U_out, R, a, b, dt, G_out):
        """rk_stage that keeps the lifted gradients of U_in in G_out (Navier-Stokes)."""
        self._sync_stream()
        gp = _VP(_dptr(G_out)) if G_out is not None else _VP()
        self._check(lib().dg_rk_stage_keep(self.h, _VP(_dptr(U_in)), _VP(_dptr(U_out)), _VP(_dptr(R)), a, b, dt,
                                           gp), "dg_rk_stage_keep")

    def rk_step_vjp(self, stage_U, stage_G, U_bar, R_bar, dt):
        """Reverse of one five-stage step given its stage inputs (and kept gradients or None)."""
        self._sync_stream()
        su = (_VP * 5)(*[_dptr(u) for u in stage_U])
        sg = None if stage_G is None else (_VP * 5)(*[(_dptr(g) if g is not None else None) for g in stage_G])
        self._check(lib().dg_rk_step_vjp(self.h, su, sg, _VP(_dptr(U_bar)), _VP(_dptr(R_bar)), dt),
                    "dg_rk_step_vjp")

    def rk_steps_vjp(self, stage_U, stage_G, U_bar, R_bar, dt):
        """Reverse of len(stage_U) // 5 consecutive steps given their stage inputs in forward
        order (and kept lifting outputs, or None entries)."""
        self._sync_stream()
        k = len(stage_U)
        if k == 0 or k % 5:
            raise ValueError("stage_U must hold five stage inputs per step")
        su = (_VP * k)(*[_dptr(u) for u in stage_U])
        sg = None if stage_G is None else (_VP * k)(*[(_dptr(g) if g is not None else None) for g in stage_G])
        self._check(lib().dg_rk_steps_vjp(self.h, k // 5, su, sg, _VP(_dptr(U_bar)), _VP(_dptr(R_bar)), dt),
                    "dg_rk_steps_vjp")

    def timestep(self, U, cfl=0.9, dfl=0.9) -> float:
        self._sync_stream()
        out = ctypes.c_double()
        self._check(lib().dg_timestep(self.h, _VP(_dptr(U)), float(cfl), float(dfl), ctypes.byref(out)), "dg_timestep")
        return out.value

    def integrals(self, U):
        self._sync_stream()
        out = np.zeros(8)
        self._check(lib().dg_integrals(self.h, _VP(_dptr(U)), _ptr(out)), "dg_integrals")
        return out

    def integrals_noalloc(self, U, out):
        """dg_integrals_noalloc: the integrals into the device tensor ``out`` (8 doubles),
        asynchronous on the library stream, scratch in the library's static device buffer."""
        self._sync_stream()
        if out.dtype != self.torch.float64 or out.numel() < 8 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of at least 8 entries")
        self._check(lib().dg_integrals_noalloc(self.h, _VP(_dptr(U)), _VP(_dptr(out))), "dg_integrals_noalloc")

    # ---- hybrid DG / finite-volume subcells (Sec. 4), Euler equations
    def fv_enable(self, limiter: int = 1, lo: float = -4.0, hi: float = -3.0):
        self._check(lib().dg_fv_enable(self.h, int(limiter), float(lo), float(hi)), "dg_fv_enable")

    def fv_set_types(self, types):
        t = np.ascontiguousarray(types, np.uint8)
        self._sync_stream()
        self._check(lib().dg_fv_set_types(self.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "dg_fv_set_types")

    def fv_types(self):
        t = np.zeros(self.K, np.uint8)
        self._sync_stream()
        self._check(lib().dg_fv_types(self.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "dg_fv_types")
        return t

    def fv_indicator(self, U):
        ind = np.zeros(self.K)
        self._sync_stream()
        self._check(lib().dg_fv_indicator(self.h, _VP(_dptr(U)), _ptr(ind)), "dg_fv_indicator")
        return ind

    def fv_switch(self, U):
        """Indicator and switching with hysteresis, in place on the device tensor U."""
        self._sync_stream()
        self._check(lib().dg_fv_switch(self.h, _VP(_dptr(U))), "dg_fv_switch")

    def check_finite(self, U) -> bool:
        self._sync_stream()
        rc = lib().dg_check_finite(self.h, _VP(_dptr(U)))
        if rc == -5:
            return False
        self._check(rc, "dg_check_finite")
        return True

    def profile(self, enable: bool):
        self._check(lib().dg_profile(self.h, int(enable)), "dg_profile")

    def profile_read(self):
        out = np.zeros(8)
        self._check(lib().dg_profile_read_ex(self.h, _ptr(out), 8), "dg_profile_read_ex")
        return {"lift_ms": out[0], "lift_launches": int(out[1]), "main_ms": out[2], "main_launches": int(out[3]),
                "face_ms": out[4], "face_launches": int(out[5]), "fv_ms": out[6], "fv_launches": int(out[7])}

    def mass_weights(self):
        """J w_i w_j w_k per node as a [K, n^3] device tensor."""
        self._sync_stream()
        out = self.torch.empty((self.K, self.n3), dtype=self.torch.float64, device="cuda")
        self._check(lib().dg_mass_weights(self.h, _VP(out.data_ptr())), "dg_mass_weights")
        return out

    def node_coords(self):
        x = np.zeros((self.K, 3, self.n3))
        self._check(lib().dg_node_coords(self.h, _ptr(x)), "dg_node_coords")
        return x

    def steps(self, U, nsteps: int, dt: float, R=None, spare=None):
        """Advance ``nsteps`` full RK steps (5 stages each) with ping-pong buffers; returns the new U."""
        a, b, _ = rk_coefficients()
        R = self.torch.zeros_like(U) if R is None else R
        cur = U
        nxt = self.empty() if spare is None else spare
        for _ in range(nsteps):
            for s in range(5):
                self.rk_stage(cur, nxt, R, a[s], b[s], dt)
                cur, nxt = nxt, cur
        return cur

    def step(self, U, R, dt: float):
        """One RK step from U with register R; U is overwritten with the new state (a buffer of
        the solver's shape is used in between)."""
        out = self.steps(U, 1, dt, R=R)
        if out is not U:
            U.copy_(out)
        return U


class Batch:
    """Several solvers advanced together (``dg_batch``): one lifting and one operator launch per
    degree present and stage, optionally one HIP graph per RK step.  All solvers must use the
    split form on LGL nodes with the same equations, volume flux and Riemann solver."""

    def __init__(self, solvers):
        import torch
        self.torch = torch
        self.solvers = list(solvers)
        n = len(self.solvers)
        self.n = n
        hs = (_VP * n)(*[S.h for S in self.solvers])
        b = _VP()
        rc = lib().dg_batch_create(hs, n, ctypes.byref(b))
        if rc:
            raise DGError(rc, "dg_batch_create")
        self.b = b

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value and _lib is not None:
            _lib.dg_batch_destroy(b)
            self.b = None

    def _check(self, rc, what):
        if rc:
            msg = lib().dg_batch_last_error(self.b)
            raise DGError(rc, f"{what}: {msg.decode() if msg else ''}")

    def _ptrs(self, ts):
        if len(ts) != self.n:
            raise ValueError(f"expected {self.n} tensors, got {len(ts)}")
        for S, t in zip(self.solvers, ts):
            if tuple(t.shape) != S.shape:
                raise ValueError("tensor shape does not match its solver")
        return (_VP * self.n)(*[_dptr(t) for t in ts])

    def _dbl(self, x):
        v = np.ascontiguousarray(np.broadcast_to(np.asarray(x, np.float64), (self.n,)))
        return v, _ptr(v)

    def _sync_stream(self):
        self.solvers[0]._sync_stream()

    def rk_stage(self, U_in, U_out, R, a, b, dt):
        """For every member i: R_i = a_i R_i + dt_i L_i(U_in_i); U_out_i = U_in_i + b_i R_i."""
        self._sync_stream()
        av, ap = self._dbl(a)
        bv, bp = self._dbl(b)
        dv, dp = self._dbl(dt)
        self._check(lib().dg_batch_rk_stage(self.b, self._ptrs(U_in), self._ptrs(U_out), self._ptrs(R), ap, bp, dp),
                    "dg_batch_rk_stage")

    def step(self, U, U_out, R, dt, graph: bool = True):
        """One full RK step of every member: U_out_i = step(U_i); U_i and R_i are working storage."""
        self._sync_stream()
        dv, dp = self._dbl(dt)
        self._check(lib().dg_batch_step(self.b, self._ptrs(U), self._ptrs(U_out), self._ptrs(R), dp, int(graph)),
                    "dg_batch_step")

    def tune(self, U, repeats: int = 3):
        self._sync_stream()
        self._check(lib().dg_batch_tune(self.b, self._ptrs(U), repeats), "dg_batch_tune")
        return self.info()

    def set_tile(self, N: int, epb_lift: int, epb_main: int):
        self._check(lib().dg_batch_set_tile(self.b, N, epb_lift, epb_main), "dg_batch_set_tile")

    @property
    def fused(self) -> bool:
        """One lifting and one operator launch per stage for all degrees (else one pair per degree)."""
        return bool(lib().dg_batch_fused(self.b))

    @fused.setter
    def fused(self, on: bool):
        self._check(lib().dg_batch_set_fused(self.b, int(bool(on))), "dg_batch_set_fused")

    def info(self):
        """[(N, members, elements, elements per workgroup of lifting, of operator)] per degree."""
        buf = (ctypes.c_int * (5 * 8))()
        ng = lib().dg_batch_info(self.b, buf, 5 * 8)
        if ng < 0:
            raise DGError(ng, "dg_batch_info")
        return [tuple(buf[5 * i:5 * i + 5]) for i in range(ng)]


def build_solver(wl, K1: Optional[int] = None, stream=None, curved: Optional[bool] = None,
                 rotate_seed: Optional[int] = None, symmetry_box: bool = False):
    """Mesh, solver and initial state of workload ``wl`` using the library's own LGL nodes.

    With ``rotate_seed`` every element's reference axes are rotated by a seeded proper rotation
    of the cube (same physical mesh; faces meet on other sides and in all orientations).  With
    ``symmetry_box`` the mesh covers [0, pi]^3 (the Taylor-Green vortex's symmetry octant) and its
    six outer faces are symmetry planes instead of periodic."""
    from . import inputs
    import torch
    k = wl.K1 if K1 is None else K1
    cv = wl.curved if curved is None else curved
    lgl, _ = nodes(wl.N, "lgl")
    if symmetry_box:
        X = inputs.lattice_points(lgl, k, k, k, box=(np.pi, np.pi, np.pi))
        nbr, side, flip = inputs.box_lattice(k, k, k)
    else:
        X = inputs.lattice_points(lgl, k, k, k)
        nbr, side, flip = inputs.periodic_lattice(k, k, k)
    xgeo = inputs.warp_sine(X) if cv else X
    if rotate_seed is not None or symmetry_box:
        rot = (np.random.default_rng(rotate_seed).integers(0, 24, k ** 3) if rotate_seed is not None
               else np.zeros(k ** 3, np.int64))
        xgeo, nbr, side, flip, _ = inputs.rotate_elements(xgeo, nbr, side, flip, wl.N, rot)
        del X
        S = DGSolver.from_workload(wl, xgeo, nbr, side, flip=flip, stream=stream)
    else:
        S = DGSolver.from_workload(wl, xgeo, nbr, side, stream=stream)
    U0 = inputs.initial_state(wl, S.node_coords())
    return S, torch.from_numpy(np.ascontiguousarray(U0)).cuda()


# ----------------------------------------------------------------------------- differentiation
def _rollout_forward(S, U0, nsteps, dt, keep_stage_inputs=False):
    """nsteps RK steps from U0 (not modified).  Returns U_T and, if asked, the input of every stage."""
    a, b, _ = rk_coefficients()
    R = S.torch.zeros_like(U0)
    cur = U0.clone()
    nxt = S.empty()
    inputs = []
    for _ in range(nsteps):
        for s in range(5):
            if keep_stage_inputs:
                inputs.append(cur.clone())
            S.rk_stage(cur, nxt, R, a[s], b[s], dt)
            cur, nxt = nxt, cur
    return cur, inputs


def _rollout_backward(S, stage_inputs, Ubar, dt):
    """Reverse of the stages whose inputs are given (in forward order); Ubar is updated in place.
    The RK register's adjoint starts at zero: a_1 = 0 makes R start from zero at every step."""
    a, b, _ = rk_coefficients()
    Rbar = S.torch.zeros_like(Ubar)
    for idx in range(len(stage_inputs) - 1, -1, -1):
        s = idx % 5
        S.rk_stage_vjp(stage_inputs[idx], Ubar, Rbar, a[s], b[s], dt)
    return Ubar


def rollout(S, U0, nsteps: int, dt: float, ckpt_every: int = 10):
    """U(T) after nsteps RK steps as a differentiable function of U0 (torch.autograd).

    The forward pass stores the state at the start of every ckpt_every-step segment and keeps
    the stage inputs and lifting outputs of the last segment; the backward reverses the last
    segment from those and every earlier one after recomputing it from its checkpoint."""
    import torch
    if nsteps < 1 or ckpt_every < 1:
        raise ValueError("nsteps and ckpt_every must be positive")

    class _Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, U):
            a, b, _ = rk_coefficients()
            ns = S.eqn == "ns"
            if not ctx.needs_input_grad[0]:  # nothing to differentiate: a plain rollout
                ctx.ckpts, ctx.tail = [], None
                return S.steps(U.detach().clone(), nsteps, dt)
            nseg = (nsteps + ckpt_every - 1) // ckpt_every
            last = (nseg - 1) * ckpt_every  # first step of the last segment
            ckpts = []
            R = torch.zeros_like(U)
            cur = U.detach().clone()
            nxt = S.empty()
            for step in range(last):
                if step % ckpt_every == 0:
                    ckpts.append(cur.clone())
                for s in range(5):
                    S.rk_stage(cur, nxt, R, a[s], b[s], dt)
                    cur, nxt = nxt, cur
            # the last segment keeps every stage input and lifting output: the backward starts
            # there and need not recompute it
            k = 5 * (nsteps - last)
            bufs = [cur] + [S.empty() for _ in range(k - 1)]
            grads = [S.empty_grad() for _ in range(k)] if ns else [None] * k
            out = S.empty()
            for idx in range(k):
                s = idx % 5
                S.rk_stage_keep(bufs[idx], bufs[idx + 1] if idx + 1 < k else out, R, a[s], b[s], dt, grads[idx])
            ctx.ckpts = ckpts
            ctx.tail = (bufs, grads)
            return out

        @staticmethod
        def backward(ctx, gUT):
            a, b, _ = rk_coefficients()
            Ubar = gUT.detach().contiguous().clone()
            Rbar = torch.zeros_like(Ubar)
            ns = S.eqn == "ns"
            bufs, grads = ctx.tail
            S.rk_steps_vjp(bufs, grads, Ubar, Rbar, dt)
            ctx.tail = None
            del bufs, grads
            nseg = len(ctx.ckpts)  # the segments before the last
            if nseg:
                # buffers of one segment, reused: the input of every stage after the first and
                # the lifting output of every stage but the last
                nst = 5 * ckpt_every
                bufs = [None] + [S.empty() for _ in range(nst - 1)]
                grads = [S.empty_grad() for _ in range(nst - 1)] + [None] if ns else [None] * nst
                R = torch.empty_like(Ubar)
            for seg in range(nseg - 1, -1, -1):
                bufs[0] = ctx.ckpts[seg]
                # recompute up to the input of the segment's last stage (its output is the next
                # checkpoint; the reverse lifts that stage's input itself); the first stage does
                # not read R
                for idx in range(nst - 1):
                    s = idx % 5
                    S.rk_stage_keep(bufs[idx], bufs[idx + 1], R, a[s], b[s], dt, grads[idx])
                S.rk_steps_vjp(bufs, grads, Ubar, Rbar, dt)
            return Ubar

    return _Rollout.apply(U0)


def kinetic_energy(U, wJ):
    """sum over nodes of J w_i w_j w_k |m|^2 / (2 rho), a differentiable torch scalar (wJ from
    DGSolver.mass_weights())."""
    m2 = (U[:, 1:4] ** 2).sum(dim=1)
    return (wJ * 0.5 * m2 / U[:, 0]).sum()
