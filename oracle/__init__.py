"""FP64 CPU oracle of the IFEM coupling step -- test infrastructure only.

Thin ctypes marshalling around ``ifem_oracle.c`` (plain C, double precision,
single threaded).  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the HIP library never imports it and shares none
of its code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ifem_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction beyond explicit fma calls)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_L = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        L.orc_weight.argtypes = [C.c_double]
        L.orc_weight.restype = C.c_double
        L.orc_membrane_W.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_membrane_W.restype = C.c_double
        L.orc_solid_W.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_solid_W.restype = C.c_double
        L.orc_membrane_element.argtypes = [_D, _D, C.c_int, C.c_double, C.c_double, _D]
        L.orc_tet_element.argtypes = [_D, _D, C.c_double, C.c_double, _D]
        L.orc_mls.argtypes = [_D, _I, C.c_double, _D, C.c_int, _L, _D]
        L.orc_forces.argtypes = [C.c_int, _D, _D, C.c_int, _I, _I, _I, _I, C.c_int, _I, C.c_int, _I, _D, _D, _D, _D,
                                 C.c_int, C.c_int, _D, _L]
        L.orc_energy.argtypes = [C.c_int, _D, _D, C.c_int, _I, _I, _I, C.c_int, _I, C.c_int, _I, _D, _D, _D]
        L.orc_reduce.argtypes = [C.c_int, _D, C.c_int, _I, _I, _I, C.c_int, _I, C.c_int, _D]
        L.orc_curvature.argtypes = [_D, C.c_long, C.c_int, C.c_int, _I, C.c_long, C.c_int, C.c_int, _D, _D, _D, _D]
        L.orc_laplacian.argtypes = [_D, C.c_long, C.c_int, C.c_int, _I, C.c_long, C.c_int, C.c_int, _D, _D, _D]
        L.orc_spread.argtypes = [C.c_int, _D, _D, _I, _I, _D, _D, _L, C.c_int64, _D]
        L.orc_interp.argtypes = [C.c_int, _D, _I, _I, _D, _D, _L, C.c_int64, _D, _D]
        L.orc_volume_correct.argtypes = [C.c_int, _D, C.c_int, _I, _I, _I, C.c_int, _I, _D, _D, _D]
        L.orc_advance.argtypes = [C.c_int, _D, _D, C.c_void_p, C.c_double, _D]
        L.orc_interp_cells.argtypes = [C.c_int, _D, _I, _I, _D, _D, _L, C.c_int64, C.c_int, _D, _D]
        L.orc_tet_fluid_element.argtypes = [_D, _D, _D, C.c_void_p, C.c_double, C.c_double, _D]
        L.orc_fluid_forces.argtypes = [C.c_int, _D, _D, _D, C.c_void_p, C.c_int, _I, _I, C.c_int, C.c_double,
                                       C.c_double, _D]
        L.orc_point_triangle.argtypes = [_D, _D, _D, _D, _D]
        L.orc_boundary_faces.argtypes = [C.c_int, _D, C.c_int, _I, _I, C.c_int, C.c_int, _I, _I]
        L.orc_antistick.argtypes = [C.c_int, _D, _D, C.c_int, _I, _I, _I, C.c_int, _I, _I, C.c_int, _I, _D,
                                    C.c_double, _D, _L, _D]
        L.orc_pair_distances.argtypes = [C.c_int, _D, _D, C.c_void_p, C.c_int, _I, _I, C.c_int, _I, _I, C.c_int, _I,
                                         _D, C.c_int, _I, _L, _D]
        L.orc_advance.restype = None
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- element level
def weight(r: float) -> float:
    return lib().orc_weight(float(r))


def membrane_W(law, mu, mu2, I1, I2) -> float:
    return lib().orc_membrane_W(int(law), float(mu), float(mu2), float(I1), float(I2))


def solid_W(mu, lam, I1, I3) -> float:
    return lib().orc_solid_W(float(mu), float(lam), float(I1), float(I3))


def membrane_element(X, x, law, mu, mu2):
    """(3,3) reference and current node rows -> (3,3) nodal forces, status."""
    f = np.zeros((3, 3))
    st = lib().orc_membrane_element(_c(X, np.float64), _c(x, np.float64), int(law), float(mu), float(mu2), f)
    return f, st


def tet_element(X, x, mu, lam):
    f = np.zeros((4, 3))
    st = lib().orc_tet_element(_c(X, np.float64), _c(x, np.float64), float(mu), float(lam), f)
    return f, st


# ---------------------------------------------------------------- scene level
def _scene_args(scene):
    return (_c(scene.node_start, np.int32), _c(scene.tri_start, np.int32), _c(scene.tet_start, np.int32),
            _c(scene.tri, np.int32), scene.n_tris, _c(scene.tet, np.int32), scene.n_tets)


def forces(scene, x=None, elastic=True, bending=True):
    """Internal nodal forces [3][n_nodes] and counts (degenerate/inverted elements, non-finite outputs)."""
    x = scene.x64 if x is None else x
    F = np.zeros((3, scene.n_nodes))
    counts = np.zeros(2, dtype=np.int64)
    ns, ts, qs, tri, ntri, tet, ntet = _scene_args(scene)
    lib().orc_forces(scene.n_nodes, _c(scene.X_ref, np.float64), _c(x, np.float64), scene.n_particles, ns, ts, qs,
                     tri, ntri, tet, ntet, _c(scene.law, np.int32), _c(scene.mu, np.float64), _c(scene.mu2, np.float64),
                     _c(scene.kb, np.float64), _c(scene.c0, np.float64), int(bool(elastic)), int(bool(bending)), F,
                     counts)
    return F, counts


def energy(scene, x=None):
    x = scene.x64 if x is None else x
    E = np.zeros(scene.n_particles)
    ns, ts, qs, tri, ntri, tet, ntet = _scene_args(scene)
    lib().orc_energy(scene.n_nodes, _c(scene.X_ref, np.float64), _c(x, np.float64), scene.n_particles, ts, qs, tri,
                     ntri, tet, ntet, _c(scene.law, np.int32), _c(scene.mu, np.float64), _c(scene.mu2, np.float64), E)
    return E


def reduce(scene, x=None):
    """[n_particles][5] = V, A, centroid."""
    x = scene.x64 if x is None else x
    red = np.zeros((scene.n_particles, 5))
    ns, ts, qs, tri, ntri, tet, ntet = _scene_args(scene)
    lib().orc_reduce(scene.n_nodes, _c(x, np.float64), scene.n_particles, ts, qs, tri, ntri, tet, ntet, red)
    return red


def curvature(scene, p: int, x=None):
    """Per-node (A, kH, kG, normals[3][n]) of membrane particle p."""
    x = _c(scene.x64 if x is None else x, np.float64)
    s, e = int(scene.node_start[p]), int(scene.node_start[p + 1])
    n = e - s
    A, kH, kG, nr = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(3 * n)
    lib().orc_curvature(x, scene.n_nodes, s, e, _c(scene.tri, np.int32), scene.n_tris, int(scene.tri_start[p]),
                        int(scene.tri_start[p + 1]), A, kH, kG, nr)
    return A, kH, kG, nr.reshape(3, n)


def laplacian(scene, p: int, g, A, x=None):
    x = _c(scene.x64 if x is None else x, np.float64)
    s, e = int(scene.node_start[p]), int(scene.node_start[p + 1])
    out = np.zeros(e - s)
    lib().orc_laplacian(x, scene.n_nodes, s, e, _c(scene.tri, np.int32), scene.n_tris, int(scene.tri_start[p]),
                        int(scene.tri_start[p + 1]), _c(A, np.float64), _c(g, np.float64), out)
    return out


def mls(p, box, comp: int):
    """(base[3] int64, phi[27]) of one point on lattice ``comp`` of ``box``."""
    base = np.zeros(3, dtype=np.int64)
    phi = np.zeros(27)
    st = lib().orc_mls(_c(p, np.float64), np.asarray(box.n, dtype=np.int32), float(box.h),
                       np.asarray(box.origin, dtype=np.float64), int(comp), base, phi)
    if st:
        raise RuntimeError("singular MLS moment matrix")
    return base, phi


def _box_args(scene):
    n, h, o, off = scene.box_arrays()
    return _c(n, np.int32), _c(h, np.float64), _c(o, np.float64), _c(off, np.int64)


def _points(scene, x, box_of_point):
    if box_of_point is None:
        box_of_point = scene.box[scene.node_particle()]
    return _c(x, np.float64), _c(box_of_point, np.int32)


def spread(scene, F, x=None, box_of_point=None):
    """[3][total_cells] spread of nodal forces F [3][n_points]."""
    x, bop = _points(scene, scene.x64 if x is None else x, box_of_point)
    n, h, o, off = _box_args(scene)
    grid = np.zeros((3, scene.total_cells))
    lib().orc_spread(x.shape[1], x, _c(F, np.float64), bop, n, h, o, off, scene.total_cells, grid)
    return grid


def interp(scene, grid, x=None, box_of_point=None):
    """[3][n_points] interpolation of a [3][total_cells] grid field."""
    x, bop = _points(scene, scene.x64 if x is None else x, box_of_point)
    n, h, o, off = _box_args(scene)
    v = np.zeros((3, x.shape[1]))
    lib().orc_interp(x.shape[1], x, bop, n, h, o, off, scene.total_cells, _c(grid, np.float64), v)
    return v


def volume_correct(scene, V0=None, x=None):
    """Membrane volume correction of Sec. II.E: (x_out [3][n_nodes], Lambda [n_particles], non-converged count).

    V0 defaults to each particle's volume in the reference configuration."""
    x = scene.x64 if x is None else x
    if V0 is None:
        V0 = reduce(scene, x=scene.X_ref)[:, 0]
    out = np.zeros((3, scene.n_nodes))
    lam = np.zeros(scene.n_particles)
    ns, ts, qs, tri, ntri, tet, ntet = _scene_args(scene)
    bad = lib().orc_volume_correct(scene.n_nodes, _c(x, np.float64), scene.n_particles, ns, ts, tri, ntri,
                                   _c(scene.law, np.int32), _c(V0, np.float64), out, lam)
    return out, lam, bad


def advance(x, v, v_prev, dt):
    """Adams-Bashforth update x + dt (3/2 v - 1/2 v_prev) of [3][n] arrays (forward Euler if v_prev is None)."""
    x = _c(x, np.float64)
    out = np.zeros_like(x)
    vp = None if v_prev is None else _c(v_prev, np.float64)
    lib().orc_advance(x.shape[1], x, _c(v, np.float64), None if vp is None else vp.ctypes.data_as(C.c_void_p),
                      float(dt), out)
    return out


def _opt(a):
    """(keep-alive array, void pointer) of an optional float64 array."""
    if a is None:
        return None, None
    a = _c(a, np.float64)
    return a, a.ctypes.data_as(C.c_void_p)


def interp_cells(scene, grid, x=None, box_of_point=None):
    """[ncomp][n_points] interpolation of cell-centred fields grid [ncomp][total_cells]."""
    x, bop = _points(scene, scene.x64 if x is None else x, box_of_point)
    n, h, o, off = _box_args(scene)
    grid = _c(grid, np.float64)
    out = np.zeros((grid.shape[0], x.shape[1]))
    lib().orc_interp_cells(x.shape[1], x, bop, n, h, o, off, scene.total_cells, grid.shape[0], grid, out)
    return out


def tet_fluid_element(X, x, u, C, eta, G):
    """Fluid-stress forces [4][3] of one tetrahedron; C [4][6] (xx, yy, zz, xy, xz, yz) or None."""
    f = np.zeros((4, 3))
    keep, cp = _opt(None if C is None else np.asarray(C).reshape(24))
    st = lib().orc_tet_fluid_element(_c(X, np.float64), _c(x, np.float64), _c(u, np.float64), cp, float(eta),
                                     float(G), f)
    return f, st


def fluid_forces(scene, u, C=None, eta=1.0, G=1.0, x=None):
    """Fluid-stress nodal forces [3][n_nodes] of every solid and the number of skipped elements."""
    x = scene.x64 if x is None else x
    f = np.zeros((3, scene.n_nodes))
    keep, cp = _opt(C)
    bad = lib().orc_fluid_forces(scene.n_nodes, _c(scene.X_ref, np.float64), _c(x, np.float64), _c(u, np.float64), cp,
                                 scene.n_particles, _c(scene.tet_start, np.int32), _c(scene.tet, np.int32),
                                 scene.n_tets, float(eta), float(G), f)
    return f, bad


def point_triangle(p, a, b, c):
    """(closest point on triangle abc to p, 1 if it is the plane projection)."""
    out = np.zeros(3)
    st = lib().orc_point_triangle(_c(p, np.float64), _c(a, np.float64), _c(b, np.float64), _c(c, np.float64), out)
    return out, st


def boundary_faces(scene):
    """([3][n] outward boundary faces of the solids, [n] owning particle)."""
    cap = 4 * scene.n_tets + 1
    out = np.zeros((3, cap), dtype=np.int32)
    part = np.zeros(cap, dtype=np.int32)
    n = lib().orc_boundary_faces(scene.n_nodes, _c(scene.X_ref, np.float64), scene.n_particles,
                                 _c(scene.tet_start, np.int32), _c(scene.tet, np.int32), scene.n_tets, cap, out, part)
    return out[:, :n].copy(), part[:n].copy()


def _box_lengths(scene):
    return np.array([b.length for b in scene.boxes], dtype=np.float64).reshape(-1, 3)


def antistick(scene, d_min, x=None, with_distance=False):
    """Node-face anti-sticking: (x_out [3][n_nodes], winner face per node or -1, moved count), plus the
    least float64 node-face distance per node (inf where no face can reach) with with_distance."""
    x = scene.x64 if x is None else x
    out = np.zeros((3, scene.n_nodes))
    win = np.zeros(scene.n_nodes, dtype=np.int64)
    dist = np.zeros(scene.n_nodes)
    moved = lib().orc_antistick(scene.n_nodes, _c(scene.X_ref, np.float64), _c(x, np.float64), scene.n_particles,
                                _c(scene.node_start, np.int32), _c(scene.tri_start, np.int32),
                                _c(scene.tri, np.int32), scene.n_tris, _c(scene.tet_start, np.int32),
                                _c(scene.tet, np.int32), scene.n_tets, _c(scene.box, np.int32), _box_lengths(scene),
                                float(d_min), out, win, dist)
    return (out, win, moved, dist) if with_distance else (out, win, moved)


def pair_distances(scene, nodes, faces, x=None, moved=None):
    """Float64 distance from each node to the paired face (face ids as in antistick), the face taken at x
    and the node at `moved` if given (else at x)."""
    x = _c(scene.x64 if x is None else x, np.float64)
    nodes = _c(nodes, np.int32)
    faces = _c(faces, np.int64)
    out = np.zeros(nodes.size)
    mv = None if moved is None else _c(moved, np.float64)
    bad = lib().orc_pair_distances(scene.n_nodes, _c(scene.X_ref, np.float64), x,
                                   None if mv is None else mv.ctypes.data, scene.n_particles,
                                   _c(scene.node_start, np.int32), _c(scene.tri, np.int32), scene.n_tris,
                                   _c(scene.tet_start, np.int32), _c(scene.tet, np.int32), scene.n_tets,
                                   _c(scene.box, np.int32), _box_lengths(scene), nodes.size, nodes, faces, out)
    if bad:
        raise ValueError(f"{bad} face ids out of range")
    return out
