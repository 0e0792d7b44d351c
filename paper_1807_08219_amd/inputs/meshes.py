"""Seeded Lagrangian meshes: geodesic spheres, Evans-Fung red cells, Kuhn-lattice ellipsoids.

Input synthesis only.  Nothing here evaluates a force, a weight or any other
quantity of the coupling step; both the oracle and the HIP library consume
the arrays these functions return.

Conventions
-----------
* Node coordinates are returned as ``(n, 3)`` float64 arrays.
* Triangles are ``(m, 3)`` int32, counter-clockwise seen from outside
  (outward normal by the right-hand rule).
* Tetrahedra are ``(m, 4)`` int32 with positive signed volume
  ``det[x1-x0, x2-x0, x3-x0] > 0``.
"""
from __future__ import annotations

import itertools

import numpy as np

# Icosahedron: 12 vertices on the unit sphere, 20 outward faces.
_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _icosahedron():
    v = np.array(
        [
            [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
            [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
            [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    return v, f


def orient_outward(nodes: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Flip triangles whose normal points towards the mesh centroid (star-shaped meshes)."""
    c = nodes.mean(axis=0)
    a, b, d = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    n = np.cross(b - a, d - a)
    flip = np.einsum("ij,ij->i", n, (a + b + d) / 3.0 - c) < 0
    out = tris.copy()
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def icosphere(nu: int):
    """Frequency-``nu`` geodesic sphere of radius 1 (class-I subdivision of the icosahedron).

    Every icosahedron face is split into ``nu**2`` triangles on a planar
    barycentric lattice whose points are then pushed onto the sphere; shared
    edge and corner points are merged.  Counts: ``10 nu^2 + 2`` nodes and
    ``20 nu^2`` triangles (nu = 8 -> 642 / 1280, nu = 16 -> 2562 / 5120).
    """
    if nu < 1:
        raise ValueError("nu must be >= 1")
    V, F = _icosahedron()
    key_to_id: dict = {}
    pts = []

    def node(key, p):
        idx = key_to_id.get(key)
        if idx is None:
            idx = len(pts)
            key_to_id[key] = idx
            pts.append(p / np.linalg.norm(p))
        return idx

    def edge_key(u, w, k):
        # k steps from u towards w; canonical from the smaller vertex id
        return ("e", u, w, k) if u < w else ("e", w, u, nu - k)

    tris = []
    for fi, (A, B, C) in enumerate(F):
        a, b, c = V[A], V[B], V[C]
        ids = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                p = a + (b - a) * (i / nu) + (c - a) * (j / nu)
                if i == 0 and j == 0:
                    key = ("v", A)
                elif i == nu:
                    key = ("v", B)
                elif j == nu:
                    key = ("v", C)
                elif j == 0:
                    key = edge_key(A, B, i)
                elif i == 0:
                    key = edge_key(A, C, j)
                elif i + j == nu:
                    key = edge_key(B, C, j)
                else:
                    key = ("f", fi, i, j)
                ids[(i, j)] = node(key, p)
        for i in range(nu):
            for j in range(nu - i):
                tris.append((ids[(i, j)], ids[(i + 1, j)], ids[(i, j + 1)]))
                if i + j < nu - 1:
                    tris.append((ids[(i + 1, j)], ids[(i + 1, j + 1)], ids[(i, j + 1)]))
    nodes = np.asarray(pts, dtype=np.float64)
    tris = orient_outward(nodes, np.asarray(tris, dtype=np.int64)).astype(np.int32)
    assert nodes.shape[0] == 10 * nu * nu + 2 and tris.shape[0] == 20 * nu * nu
    return nodes, tris


# Evans & Fung (1972) biconcave profile coefficients (dimensionless).
EF_C0, EF_C2, EF_C4 = 0.2072, 2.0026, -1.1228


def evans_fung(unit_nodes: np.ndarray, R0: float = 3.91) -> np.ndarray:
    """Map unit-sphere nodes to the Evans-Fung red-cell surface of radius ``R0``.

    The profile is z = +-(R0/2) sqrt(1 - rho^2) (C0 + C2 rho^2 + C4 rho^4),
    rho = r / R0.  On the unit sphere sqrt(1 - rho^2) = |z|, so the map
    (x, y, z) -> (R0 x, R0 y, (R0/2) z (C0 + C2 rho^2 + C4 rho^4)) is smooth
    and keeps the triangulation's orientation.
    """
    x, y, z = unit_nodes[:, 0], unit_nodes[:, 1], unit_nodes[:, 2]
    rho2 = x * x + y * y
    out = np.empty_like(unit_nodes)
    out[:, 0] = R0 * x
    out[:, 1] = R0 * y
    out[:, 2] = 0.5 * R0 * z * (EF_C0 + EF_C2 * rho2 + EF_C4 * rho2 * rho2)
    return out


def kuhn_box(nx: int, ny: int, nz: int):
    """Kuhn (Freudenthal) triangulation of [-1, 1]^3 with ``6 nx ny nz`` positive tetrahedra."""
    gx, gy, gz = (np.linspace(-1.0, 1.0, n + 1) for n in (nx, ny, nz))
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def nid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    unit = np.eye(3, dtype=np.int64)
    tets = []
    for i, j, k in itertools.product(range(nx), range(ny), range(nz)):
        base = np.array([i, j, k])
        for perm in itertools.permutations(range(3)):
            p0 = base
            p1 = p0 + unit[perm[0]]
            p2 = p1 + unit[perm[1]]
            p3 = p2 + unit[perm[2]]
            t = [nid(*p0), nid(*p1), nid(*p2), nid(*p3)]
            # odd permutations give a negatively oriented simplex
            sign = np.linalg.det(np.stack([unit[perm[0]], unit[perm[1]], unit[perm[2]]]))
            if sign < 0:
                t[2], t[3] = t[3], t[2]
            tets.append(t)
    return nodes, np.asarray(tets, dtype=np.int32)


def cube_to_ball(p: np.ndarray) -> np.ndarray:
    """Smooth map of [-1, 1]^3 onto the unit ball (faces -> sphere)."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    x2, y2, z2 = x * x, y * y, z * z
    out = np.empty_like(p)
    out[:, 0] = x * np.sqrt(np.maximum(1 - y2 / 2 - z2 / 2 + y2 * z2 / 3, 0.0))
    out[:, 1] = y * np.sqrt(np.maximum(1 - z2 / 2 - x2 / 2 + z2 * x2 / 3, 0.0))
    out[:, 2] = z * np.sqrt(np.maximum(1 - x2 / 2 - y2 / 2 + x2 * y2 / 3, 0.0))
    return out


def signed_tet_volumes(nodes: np.ndarray, tets: np.ndarray) -> np.ndarray:
    a = nodes[tets[:, 0]]
    d = np.stack([nodes[tets[:, 1]] - a, nodes[tets[:, 2]] - a, nodes[tets[:, 3]] - a], axis=2)
    return np.linalg.det(d) / 6.0


def ellipsoid_tets(nx: int, ny: int, nz: int, semi_axes=(1.5, 1.5, 0.375)):
    """Tetrahedral ellipsoid: Kuhn lattice of the cube, mapped to the ball, then scaled."""
    nodes, tets = kuhn_box(nx, ny, nz)
    nodes = cube_to_ball(nodes) * np.asarray(semi_axes, dtype=np.float64)[None, :]
    vol = signed_tet_volumes(nodes, tets)
    if not np.all(vol > 0):
        raise RuntimeError("ellipsoid mesh has non-positive tetrahedra")
    return nodes, tets


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3) from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def rotation_about(axis: np.ndarray, angle: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def triangle_area_ratio(ref: np.ndarray, cur: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Current / reference area of each triangle (input screening only)."""
    def areas(p):
        a = p[tris[:, 0]]
        return 0.5 * np.linalg.norm(np.cross(p[tris[:, 1]] - a, p[tris[:, 2]] - a), axis=1)

    return areas(cur) / areas(ref)
