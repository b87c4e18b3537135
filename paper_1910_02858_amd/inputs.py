"""Seeded, synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds no arithmetic of the discretisation itself: no quadrature
nodes, no derivative matrices, no fluxes.  It only describes *problems*:

* periodic hexahedral lattices and their face connectivity, also with the reference
  axes of elements rotated (faces that meet on other sides and in other orientations),
* analytic maps from the undeformed lattice to a curved mesh,
* closed-form initial states (density wave, Taylor-Green vortex),
* the parameters of the five workloads and the seeded ensemble draw.

Callers pass in the 1D reference nodes at which the map is to be sampled;
each side (oracle, library) brings its own nodes.

Side numbering used everywhere (library and oracle): side ``2*d`` is the
face ``xi_d = -1`` and side ``2*d+1`` the face ``xi_d = +1`` of direction
``d`` in ``(0, 1, 2)``.  Elements are numbered lexicographically,
``e = ex + Kx*(ey + Ky*ez)``.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Optional

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------- mesh
def periodic_lattice(kx: int, ky: int, kz: int):
    """Face connectivity of a fully periodic ``kx*ky*kz`` lattice.

    Returns ``(nbr_elem[K,6] int32, nbr_side[K,6] int8, flip[K,6] int8)``.
    The neighbour across side ``2d`` is the previous element in direction d
    (with wrap-around) and it meets it on its side ``2d+1``; all flips are 0.
    """
    K = kx * ky * kz
    nbr = np.empty((K, 6), np.int32)
    side = np.empty((K, 6), np.int8)
    ez, ey, ex = np.meshgrid(np.arange(kz), np.arange(ky), np.arange(kx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()

    def lin(a, b, c):
        return (a % kx) + kx * ((b % ky) + ky * (c % kz))

    nbr[:, 0] = lin(ex - 1, ey, ez)
    nbr[:, 1] = lin(ex + 1, ey, ez)
    nbr[:, 2] = lin(ex, ey - 1, ez)
    nbr[:, 3] = lin(ex, ey + 1, ez)
    nbr[:, 4] = lin(ex, ey, ez - 1)
    nbr[:, 5] = lin(ex, ey, ez + 1)
    for s in range(6):
        side[:, s] = s ^ 1
    flip = np.zeros((K, 6), np.int8)
    return nbr, side, flip


def box_lattice(kx: int, ky: int, kz: int, kind: int = 0):
    """Face connectivity of a ``kx*ky*kz`` lattice whose six outer faces are boundaries.

    Same numbering as :func:`periodic_lattice`; a side on the outer boundary has neighbour
    ``-1`` and the boundary kind in ``nbr_side`` (0 symmetry plane, 1 given outer state).
    """
    nbr, side, flip = periodic_lattice(kx, ky, kz)
    ez, ey, ex = np.meshgrid(np.arange(kz), np.arange(ky), np.arange(kx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    for s, (c, k, lo) in enumerate([(ex, kx, True), (ex, kx, False), (ey, ky, True), (ey, ky, False),
                                    (ez, kz, True), (ez, kz, False)]):
        at = (c == 0) if lo else (c == k - 1)
        nbr[at, s] = -1
        side[at, s] = kind
    return nbr, side, flip


def face_orientation_map(code: int, a, b, N: int):
    """Neighbour face point matching face point ``(a, b)`` under orientation ``code``.

    Face points of side ``s`` (direction ``d = s // 2``) are indexed by the two tangential
    node indices in increasing direction order.  ``code`` in 0..7: bit 2 swaps ``(a, b)``,
    then bit 0 reverses the first index and bit 1 the second (``x -> N - x``).
    """
    p, q = (b, a) if code & 4 else (a, b)
    return (N - p if code & 1 else p), (N - q if code & 2 else q)


def cube_rotations():
    """The 24 proper rotations of the reference cube ``[-1, 1]^3`` as ``(perm, sign)``:
    new axis ``d`` runs along old axis ``perm[d]``, reversed where ``sign[d] < 0``."""
    out = []
    for perm in itertools.permutations(range(3)):
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        for sg in itertools.product((1, -1), repeat=3):
            if (-1) ** inv * sg[0] * sg[1] * sg[2] == 1:
                out.append((perm, sg))
    return out


def rotation_node_map(r: int, N: int):
    """``old[q']``: the node (index ``i + n*(j + n*k)``) of the unrotated element that the
    rotated element's node ``q'`` is, for rotation ``r`` of :func:`cube_rotations`."""
    perm, sg = cube_rotations()[r]
    n = N + 1
    old = np.empty(n ** 3, np.int64)
    for q in range(n ** 3):
        new = (q % n, (q // n) % n, q // (n * n))
        o = [0, 0, 0]
        for d in range(3):
            o[perm[d]] = new[d] if sg[d] > 0 else N - new[d]
        old[q] = o[0] + n * (o[1] + n * o[2])
    return old


def _rotated_face_table():
    """For rotations ``(re, rn)`` of two face neighbours of a structured lattice and side
    ``s'`` of the rotated element ``e``: the old side of ``e`` behind ``s'`` and the rotated
    neighbour's side and orientation code.  Derived by following every face point (N = 2)."""
    N, n = 2, 3
    rots = cube_rotations()
    old_side = np.empty((24, 6), np.int64)
    tab = np.empty((24, 6, 24, 2), np.int64)
    for re, (pe, se) in enumerate(rots):
        for s2 in range(6):
            d2, p2 = s2 // 2, s2 % 2
            da, db = (1, 2) if d2 == 0 else ((0, 2) if d2 == 1 else (0, 1))
            S = 2 * pe[d2] + (p2 ^ (1 if se[d2] < 0 else 0))
            old_side[re, s2] = S
            for rn, (pn, sn) in enumerate(rots):
                found = None
                for o in range(8):
                    ok, side_n = True, None
                    for a in range(n):
                        for b in range(n):
                            new = [0, 0, 0]
                            new[d2], new[da], new[db] = (N if p2 else 0), a, b
                            old = [0, 0, 0]
                            for d in range(3):
                                old[pe[d]] = new[d] if se[d] > 0 else N - new[d]
                            D = S // 2
                            old[D] = N - old[D]            # the neighbour's node across the face
                            nn = [0, 0, 0]
                            for d in range(3):
                                nn[d] = old[pn[d]] if sn[d] > 0 else N - old[pn[d]]
                            dn = [d for d in range(3) if pn[d] == D][0]
                            sd = 2 * dn + (1 if nn[dn] == N else 0)
                            ta, tb = (1, 2) if dn == 0 else ((0, 2) if dn == 1 else (0, 1))
                            if side_n is None:
                                side_n = sd
                            if sd != side_n or face_orientation_map(o, a, b, N) != (nn[ta], nn[tb]):
                                ok = False
                                break
                        if not ok:
                            break
                    if ok:
                        found = (side_n, o)
                        break
                assert found is not None
                tab[re, s2, rn] = found
    return old_side, tab


_FACE_TABLE = None


def rotate_elements(X, nbr, side, flip, N: int, rot):
    """Relabel the reference axes of every element of a lattice (periodic, or with boundary
    sides as from :func:`box_lattice`, which stay boundary sides of the same kind).

    ``rot[e]`` indexes :func:`cube_rotations`.  The physical mesh is unchanged; each element's
    nodes are renumbered, so neighbouring faces meet on other sides and in other orientations.
    Returns ``(X', nbr', side', flip', node_map)`` with ``X'[e][:, q'] = X[e][:, node_map[e][q']]``
    (a state field is carried over the same way).
    """
    global _FACE_TABLE
    nbr, side, flip = np.asarray(nbr), np.asarray(side), np.asarray(flip)
    K = nbr.shape[0]
    inner = nbr >= 0
    assert np.all((side == np.arange(6)[None, :] ^ 1) | ~inner) and not np.any(flip), "expects a lattice"
    if _FACE_TABLE is None:
        _FACE_TABLE = _rotated_face_table()
    old_side, tab = _FACE_TABLE
    rot = np.asarray(rot, np.int64)
    maps = np.stack([rotation_node_map(r, N) for r in range(24)])
    node_map = maps[rot]
    Xr = np.take_along_axis(np.asarray(X), node_map[:, None, :], axis=2)
    S = old_side[rot]                                   # [K][6] old side behind each new side
    nb = np.take_along_axis(nbr, S, axis=1).astype(np.int32)
    bnd = nb < 0
    t = tab[rot[:, None], np.arange(6)[None, :], rot[np.where(bnd, 0, nb)]]
    side_r = np.where(bnd, np.take_along_axis(side, S, axis=1), t[..., 0]).astype(np.int8)
    flip_r = np.where(bnd, 0, t[..., 1]).astype(np.int8)
    return (np.ascontiguousarray(Xr), nb, side_r, flip_r, node_map)


def renumber_elements(X, nbr, side, flip, order):
    """The same mesh with element ``order[i]`` stored as element ``i`` (connectivity remapped;
    boundary sides, neighbour sides and orientations unchanged).  A state field is carried with
    ``U[order]``."""
    order = np.asarray(order, np.int64)
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size)
    nbr = np.asarray(nbr)[order]
    nbr = np.where(nbr < 0, nbr, inv[np.maximum(nbr, 0)]).astype(np.int32)
    return (np.ascontiguousarray(np.asarray(X)[order]), nbr, np.ascontiguousarray(np.asarray(side)[order]),
            np.ascontiguousarray(np.asarray(flip)[order]))


# ----------------------------------------------------------------------------- non-conforming
# Mortar kinds of a side (Sec. 3.2): 0 conforming; 1, 2, 3 the big side of a non-conforming face
# cut in half along the side's first face direction (1), its second (2), or both (3); 4 + p the
# small side at position p of such a face: p along the cut for types 1 and 2, p = p1 + 2 p2
# (p1 along the first, p2 along the second face direction) for type 3.  Face point (a, b) of a
# side runs along the element's two other directions in increasing order; on a small side the
# orientation code maps it to the point of the big side's sub-face p, whose own (a', b') run
# along the big side's face directions.
MORTAR_SUBFACES = {1: [((-1, 0), (-1, 1)), ((0, 1), (-1, 1))],
                   2: [((-1, 1), (-1, 0)), ((-1, 1), (0, 1))],
                   3: [((-1, 0), (-1, 0)), ((0, 1), (-1, 0)), ((-1, 0), (0, 1)), ((0, 1), (0, 1))]}


def refined_lattice(nodes_1d, k, split=(2, 2, 2), refine=None, box=(TWO_PI, TWO_PI, TWO_PI)):
    """Undeformed node positions ``X[e][3][n^3]`` of a ``k^3`` (or ``kx*ky*kz``) lattice on ``box`` whose cells with
    ``refine(ex, ey, ez)`` true (default: the half ``ex < k/2``) are split into ``split`` children
    per direction (1 or 2 each); the other cells stay whole.  Whole cells come first in
    lexicographic order, then the children of every refined cell (lexicographic, child x fastest).
    Where a refined cell meets a whole one the faces are non-conforming."""
    kx, ky, kz = (k, k, k) if np.isscalar(k) else tuple(k)
    if refine is None:
        def refine(ex, ey, ez):
            return ex < kx // 2
    r = np.asarray(nodes_1d, dtype=np.float64)
    n = r.size
    t = 0.5 * (r + 1.0)
    tk, tj, ti = np.meshgrid(t, t, t, indexing="ij")
    tt = np.stack([ti.ravel(), tj.ravel(), tk.ravel()])  # [3][n^3]
    h = np.array(box, np.float64) / np.array([kx, ky, kz], np.float64)
    whole, fine = [], []
    for ez in range(kz):
        for ey in range(ky):
            for ex in range(kx):
                lo = np.array([ex, ey, ez], np.float64) * h
                if not refine(ex, ey, ez):
                    whole.append((lo, h))
                    continue
                hc = h / np.array(split, np.float64)
                for cz in range(split[2]):
                    for cy in range(split[1]):
                        for cx in range(split[0]):
                            fine.append((lo + np.array([cx, cy, cz]) * hc, hc))
    cells = whole + fine
    X = np.empty((len(cells), 3, n ** 3), np.float64)
    for e, (lo, hh) in enumerate(cells):
        X[e] = lo[:, None] + hh[:, None] * tt
    return X


def warp_bubble(X, amp: float = 0.1, degree: int = 2):
    """Curved map ``x_d = X_d + amp * prod_c b(X_c)`` for every d, with the bubble
    ``b(t) = t(2pi - t)/pi^2`` (degree 2) or ``b(t) = t(2pi - t)(t - pi)/pi^3 * 2.6`` (degree 3).
    It is a polynomial of that degree in each coordinate, so every cell of an affine lattice maps
    to a polynomial element of that degree, children of a refined cell are exact restrictions of
    their parent, and it vanishes on the faces of ``[0, 2pi]^3`` (periodic meshes stay periodic)."""
    X = np.asarray(X)
    if degree == 2:
        b = X * (TWO_PI - X) / math.pi ** 2
    else:
        b = 2.6 * X * (TWO_PI - X) * (X - math.pi) / math.pi ** 3
    s = amp * b[:, 0] * b[:, 1] * b[:, 2]
    return X + s[:, None, :]


def _face_corners(X, n):
    """Corner positions [K][6][4][3] of every side in face-point order (a, b) = (0,0), (N,0),
    (0,N), (N,N), from the element nodes."""
    N = n - 1
    K = X.shape[0]
    out = np.empty((K, 6, 4, 3))
    for s in range(6):
        d, plus = s // 2, s % 2
        for c, (a, b) in enumerate(((0, 0), (N, 0), (0, N), (N, N))):
            idx = [0, 0, 0]
            da, db = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
            idx[d], idx[da], idx[db] = (N if plus else 0), a, b
            q = idx[0] + n * (idx[1] + n * idx[2])
            out[:, s, c, :] = X[:, :, q]
    return out


def _orient(src, dst, tol):
    """Orientation code o (swap the face indices if o & 4, then reverse the first if o & 1 and the
    second if o & 2) that carries the corners src[(a,b)] onto dst[(a',b')], or None."""
    pos = ((0, 0), (1, 0), (0, 1), (1, 1))
    for o in range(8):
        ok = True
        for c, (a, b) in enumerate(pos):
            p, q = (b, a) if o & 4 else (a, b)
            a2 = 1 - p if o & 1 else p
            b2 = 1 - q if o & 2 else q
            if np.abs(src[c] - dst[pos.index((a2, b2))]).max() > tol:
                ok = False
                break
        if ok:
            return o
    return None


def connect_boxes(X, n: int, period=(TWO_PI, TWO_PI, TWO_PI), bc_kind: int = 0):
    """Connectivity of a hexahedral mesh of straight-sided cells (undeformed coordinates, any
    reference-axis orientation) by matching face corners, including non-conforming faces whose
    big side is cut in half in one or both face directions: returns ``(nbr[K,6], side[K,6],
    flip[K,6], mortar[K,6])`` in the conventions of :data:`MORTAR_SUBFACES`.  A big side has
    ``nbr = -1``, ``side = 0``, ``flip = 0``; a small side names the big element and side.  Along
    directions with a positive ``period`` coordinates are compared modulo the period; unmatched
    sides become boundaries of kind ``bc_kind``."""
    X = np.asarray(X, np.float64)
    K = X.shape[0]
    C = _face_corners(X, n)
    ext = np.abs(C.max(axis=2) - C.min(axis=2)).max()
    tol = 1e-9 * max(ext, 1e-300)
    per = np.array([p if p and p > 0 else 0.0 for p in period]) if period is not None else np.zeros(3)

    def wrap(P):
        P = P.copy()
        for d in range(3):
            if per[d] > 0:
                P[..., d] = np.mod(P[..., d] + 0.5 * tol, per[d]) - 0.5 * tol
        return P

    def key(P):
        c = wrap(P).mean(axis=0)
        return tuple(np.round(c / (1e4 * tol)).astype(np.int64))

    def same(A, B):
        # corner sets equal up to the periodic shift
        dA, dB = wrap(A), wrap(B)
        return all(any(np.abs(a - b).max() < 1e3 * tol or
                       all(per[d] > 0 and abs(abs(a[d] - b[d]) - per[d]) < 1e3 * tol or abs(a[d] - b[d]) < 1e3 * tol
                           for d in range(3)) for b in dB) for a in dA)

    faces = {}
    for e in range(K):
        for s in range(6):
            faces.setdefault(key(C[e, s]), []).append((e, s))
    nbr = np.full((K, 6), -1, np.int32)
    side = np.zeros((K, 6), np.int8)
    flip = np.zeros((K, 6), np.int8)
    mortar = np.zeros((K, 6), np.int8)

    def corners_wrapped_to(A, B):
        # shift A by whole periods so that its corners sit next to B's
        A = A.copy()
        for d in range(3):
            if per[d] > 0:
                A[:, d] += per[d] * np.round((B[:, d].mean() - A[:, d].mean()) / per[d])
        return A

    for e in range(K):
        for s in range(6):
            for (e2, s2) in faces[key(C[e, s])]:
                if (e2, s2) == (e, s):
                    continue
                A = corners_wrapped_to(C[e, s], C[e2, s2])
                o = _orient(A, C[e2, s2], 1e3 * tol)
                if o is not None:
                    nbr[e, s], side[e, s], flip[e, s] = e2, s2, o
    # non-conforming faces: sub-faces of unmatched sides
    for e in range(K):
        for s in range(6):
            if nbr[e, s] >= 0:
                continue
            c = C[e, s]  # corners at (eta1, eta2) = (-1,-1), (1,-1), (-1,1), (1,1)

            def at(u, v):
                # bilinear point of the (planar, straight-sided) face at reference (u, v)
                return 0.25 * ((1 - u) * (1 - v) * c[0] + (1 + u) * (1 - v) * c[1] + (1 - u) * (1 + v) * c[2] +
                               (1 + u) * (1 + v) * c[3])

            for typ in (3, 1, 2):
                subs = MORTAR_SUBFACES[typ]
                found = []
                for (u0, u1), (v0, v1) in subs:
                    sub = np.array([at(u0, v0), at(u1, v0), at(u0, v1), at(u1, v1)])
                    hit = None
                    for (e2, s2) in faces.get(key(sub), []):
                        if e2 == e or nbr[e2, s2] >= 0 or mortar[e2, s2]:
                            continue
                        A = corners_wrapped_to(C[e2, s2], sub)
                        o = _orient(A, sub, 1e3 * tol)
                        if o is not None:
                            hit = (e2, s2, o)
                            break
                    if hit is None:
                        break
                    found.append(hit)
                if len(found) == len(subs):
                    mortar[e, s] = typ
                    for p, (e2, s2, o) in enumerate(found):
                        nbr[e2, s2], side[e2, s2], flip[e2, s2] = e, s, o
                        mortar[e2, s2] = 4 + p
                    break
    for e in range(K):
        for s in range(6):
            if nbr[e, s] < 0 and mortar[e, s] == 0:
                side[e, s] = bc_kind
    return nbr, side, flip, mortar


def global_node_ids(X, digits: int = 9):
    """A global index for every element node ``X[K][3][n^3]``: nodes at the same position (rounded
    to ``digits`` decimals) share one index, as in a mesh file's node list."""
    X = np.asarray(X)
    K, _, n3 = X.shape
    keys = np.round(np.transpose(X, (0, 2, 1)).reshape(-1, 3), digits)
    _, ids = np.unique(keys, axis=0, return_inverse=True)
    return ids.reshape(K, n3).astype(np.int64)


def lattice_points(nodes_1d, kx: int, ky: int, kz: int, box=(TWO_PI, TWO_PI, TWO_PI)):
    """Undeformed positions ``X[e][3][n^3]`` of tensor nodes in every lattice cell.

    ``nodes_1d`` are reference coordinates in [-1, 1] (supplied by the caller).
    Node index ``i + n*(j + n*k)`` with i along x.
    """
    r = np.asarray(nodes_1d, dtype=np.float64)
    n = r.size
    K = kx * ky * kz
    hx, hy, hz = box[0] / kx, box[1] / ky, box[2] / kz
    ez, ey, ex = np.meshgrid(np.arange(kz), np.arange(ky), np.arange(kx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    t = 0.5 * (r + 1.0)
    # local tensor coordinates, i fastest
    tk, tj, ti = np.meshgrid(t, t, t, indexing="ij")
    ti, tj, tk = ti.ravel(), tj.ravel(), tk.ravel()
    X = np.empty((K, 3, n ** 3), np.float64)
    X[:, 0, :] = (ex[:, None] + ti[None, :]) * hx
    X[:, 1, :] = (ey[:, None] + tj[None, :]) * hy
    X[:, 2, :] = (ez[:, None] + tk[None, :]) * hz
    return X


def warp_sine(X, amp: float = 0.1):
    """Curved map ``x_d = X_d + amp*sin(X)sin(Y)sin(Z)`` for every d.

    It vanishes on the planes X,Y,Z in {0, 2*pi}, so a periodic [0,2pi]^3
    lattice stays periodic.
    """
    X = np.asarray(X)
    s = amp * np.sin(X[:, 0]) * np.sin(X[:, 1]) * np.sin(X[:, 2])
    return X + s[:, None, :]


# ----------------------------------------------------------------------------- states
def prim_to_cons(rho, u, v, w, p, gamma):
    """Conservative state (rho, rho*u, rho*v, rho*w, E) of an ideal gas."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E], axis=-2)


def density_wave(x, t: float = 0.0, gamma: float = 1.4, amp: float = 0.2):
    """Exact Euler solution rho = 1 + amp*sin(x+y+z-3t), u=(1,1,1), p=1.

    ``x`` has shape ``[K,3,n3]``; returns ``U[K,5,n3]``.
    """
    s = x[:, 0] + x[:, 1] + x[:, 2] - 3.0 * t
    rho = 1.0 + amp * np.sin(s)
    one = np.ones_like(rho)
    return prim_to_cons(rho, one, one, one, one, gamma)


def taylor_green(x, amp: float = 1.0, mach: float = 0.1, gamma: float = 1.4, rho0: float = 1.0):
    """Taylor-Green vortex on [0,2pi]^3 with U0 = amp, rho = rho0.

    u = A sin x cos y cos z, v = -A cos x sin y cos z, w = 0,
    p = p0 + rho0*A^2/16 (cos 2x + cos 2y)(cos 2z + 2), p0 = rho0*A^2/(gamma Ma^2).
    """
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    A = amp
    u = A * np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -A * np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p0 = rho0 * A * A / (gamma * mach * mach)
    p = p0 + rho0 * A * A / 16.0 * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    rho = np.full_like(u, rho0)
    return prim_to_cons(rho, u, v, w, p, gamma)


def isentropic_vortex(x, eps: float = 5.0, gamma: float = 1.4, center=(10.0, 10.0), vel=(1.0, 1.0), t: float = 0.0,
                      period=(20.0, 20.0)):
    """Shu's isentropic vortex in the x-y plane, extruded in z (exact: advected).

    Free stream rho=1, p=1, (u,v)=vel.  Uses the nearest periodic image of
    the advected centre.
    """
    xc = center[0] + vel[0] * t
    yc = center[1] + vel[1] * t
    dx = x[:, 0] - xc
    dy = x[:, 1] - yc
    dx = dx - period[0] * np.round(dx / period[0])
    dy = dy - period[1] * np.round(dy / period[1])
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    du = -eps / (2 * math.pi) * f * dy
    dv = eps / (2 * math.pi) * f * dx
    dT = -(gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi * math.pi) * f * f
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    u = vel[0] + du
    v = vel[1] + dv
    w = np.zeros_like(u)
    return prim_to_cons(rho, u, v, w, p, gamma)


def constant_state(K: int, n3: int, rho=1.2, u=0.3, v=-0.2, w=0.1, p=0.9, gamma=1.4):
    shape = (K, n3)
    return prim_to_cons(np.full(shape, rho), np.full(shape, u), np.full(shape, v), np.full(shape, w),
                        np.full(shape, p), gamma)


def random_perturbation(U, seed: int, rel: float = 1e-2):
    """``U * (1 + rel*xi)`` with xi ~ N(0,1) per entry (seeded).  Keeps rho, p > 0 for small rel."""
    rng = np.random.default_rng(seed)
    return U * (1.0 + rel * rng.standard_normal(U.shape))


def random_directions(U, seed: int, count: int):
    """``count`` directions dU = diag(scale_v) xi, xi ~ N(0,1), scale_v = max|U_v| (seeded)."""
    rng = np.random.default_rng(seed)
    scale = np.abs(U).max(axis=(0, 2))
    out = []
    for _ in range(count):
        xi = rng.standard_normal(U.shape)
        out.append(xi * scale[None, :, None])
    return out


# ----------------------------------------------------------------------------- workloads
@dataclasses.dataclass
class Workload:
    name: str
    eqn: str          # "euler" | "ns"
    form: str         # "weak" | "strong" | "split"
    volflux: str      # "kep" | "ec" | "central"
    riemann: str      # "llf" | "roe" | "volflux" | "volflux_roe"
    nodes: str        # "lg" | "lgl"
    N: int
    K1: int           # elements per direction
    curved: bool
    ic: str           # "density_wave" | "tgv"
    steps: int
    gamma: float = 1.4
    R: float = 1.0
    Re: float = 1600.0
    Pr: float = 0.72
    mach: float = 0.1
    amp: float = 1.0
    cfl: float = 0.9
    dfl: float = 0.9

    @property
    def mu(self) -> float:
        # rho0 = U0 = L = 1 reference scales
        return self.amp / self.Re if self.eqn == "ns" else 0.0

    @property
    def n_elems(self) -> int:
        return self.K1 ** 3

    @property
    def n_dof(self) -> int:
        return self.n_elems * (self.N + 1) ** 3


def workload(idx: int, **over) -> Workload:
    """The five workloads: 1 Euler density wave, 2 NS TGV curved N=5, 3 NS TGV N=7 48^3,
    4 ensemble member template, 5 adjoint case."""
    table = {
        1: Workload("euler_dwave_lg3_k4", "euler", "weak", "central", "llf", "lg", 3, 4, False,
                    "density_wave", 10),
        2: Workload("ns_tgv_kep_roe_lgl5_k16_curved", "ns", "split", "kep", "roe", "lgl", 5, 16, True, "tgv", 100),
        3: Workload("ns_tgv_ec_roe_lgl7_k48", "ns", "split", "ec", "roe", "lgl", 7, 48, False, "tgv", 50),
        4: Workload("ns_tgv_kep_roe_ensemble_member", "ns", "split", "kep", "roe", "lgl", 5, 8, False, "tgv", 100),
        5: Workload("ns_tgv_kep_roe_lgl5_k12_curved_adjoint", "ns", "split", "kep", "roe", "lgl", 5, 12, True,
                    "tgv", 50),
    }
    wl = dataclasses.replace(table[idx])
    for k, v in over.items():
        setattr(wl, k, v)
    return wl


def ensemble_draw(n: int = 256, seed: int = 0):
    """Seeded ensemble: K1 ~ U{4..12}, N ~ U{3..7}, A ~ U[0.5,1.5], Ma ~ U[0.05,0.2] (in that order)."""
    rng = np.random.default_rng(seed)
    K1 = rng.integers(4, 13, size=n)
    N = rng.integers(3, 8, size=n)
    A = rng.uniform(0.5, 1.5, size=n)
    Ma = rng.uniform(0.05, 0.2, size=n)
    out = []
    for i in range(n):
        out.append(Workload(f"ens{i}", "ns", "split", "kep", "roe", "lgl", int(N[i]), int(K1[i]), False, "tgv", 100,
                            amp=float(A[i]), mach=float(Ma[i])))
    return out


def build_problem(wl: Workload, geo_nodes_1d, sol_points=None):
    """Mesh description for ``wl``: geometry sampled at ``geo_nodes_1d`` (degree-N LGL nodes of the
    caller) plus connectivity.  ``sol_points`` (physical solution-node positions, [K,3,n3]) may be
    given to build the initial state there; otherwise the geometry points are used."""
    k = wl.K1
    X = lattice_points(geo_nodes_1d, k, k, k)
    xgeo = warp_sine(X) if wl.curved else X
    nbr, side, flip = periodic_lattice(k, k, k)
    pts = xgeo if sol_points is None else sol_points
    U0 = initial_state(wl, pts)
    return xgeo, nbr, side, flip, U0


def initial_state(wl: Workload, pts):
    if wl.ic == "density_wave":
        return density_wave(pts, 0.0, wl.gamma)
    if wl.ic == "tgv":
        return taylor_green(pts, wl.amp, wl.mach, wl.gamma)
    raise ValueError(wl.ic)
