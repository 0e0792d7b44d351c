"""Seeded synthetic suspensions: particle meshes, placements and periodic boxes.

Input synthesis only (geometry, random draws, array layout); the force,
weight and transfer arithmetic lives in the oracle and in the HIP library,
which both read the arrays assembled here.

Layouts produced (shared by both consumers):

* ``X_ref``, ``x64``: ``[3][n_nodes]`` float64 (reference / current positions).
* ``anchor``: ``[n_particles][3]`` float64, ``x32``: ``[3][n_nodes]`` float32 offsets
  with ``x64 == anchor[p] + float64(x32)`` holding exactly for every node.
* ``tri``: ``[3][n_tris]`` int32, ``tet``: ``[4][n_tets]`` int32, global node ids;
  nodes, triangles and tetrahedra are contiguous per particle
  (``node_start``, ``tri_start``, ``tet_start``, each ``[n_particles + 1]``).
* material per particle: ``law`` (0 neo-Hookean membrane, 1 Skalak membrane,
  2 neo-Hookean tetrahedral solid), ``mu``, ``mu2`` (membrane dilatation
  modulus or solid bulk modulus), ``kb`` (bending modulus), ``c0``
  (spontaneous curvature), ``box`` (index of the periodic box it lives in).
* boxes: ``n = (nx, ny, nz)`` cells, spacing ``h``, ``origin``; the three
  staggered velocity lattices of box ``b`` occupy ``cell_offset[b] ...`` in a
  ``[3][total_cells]`` array, x fastest.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes

LAW_TRI_NEOHOOKE = 0
LAW_TRI_SKALAK = 1
LAW_TET_NEOHOOKE = 2

RBC_R0 = 3.91          # Evans-Fung radius
RBC_R_EFF = 2.82       # equivalent-sphere radius of that shape
RBC_VOLUME = 94.10     # volume enclosed by the Evans-Fung surface at R0 = 3.91
PLT_AXES = (1.5, 1.5, 0.375)
PLT_MU = 1.0 / (0.0421 * RBC_R_EFF)   # platelet / red-cell stiffness from Ca_PLT / Ca_RBC = 0.0421
KAPPA_B = 0.01         # bending parameter k_b / (R_eff^2 mu)
SKALAK_RATIO = 100.0   # mu_D / mu
SOLID_RATIO = 50.0     # lambda_p / mu_p

ANCHOR_QUANTUM = 2.0 ** -10   # anchors are multiples of this (keeps anchor + offset exact)
OFFSET_FLUSH = 2.0 ** -16     # float32 offsets smaller than this are flushed to zero


@dataclass
class Box:
    n: tuple
    h: float
    origin: tuple

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def length(self):
        return tuple(float(k) * self.h for k in self.n)


@dataclass
class Particle:
    X: np.ndarray                  # (n, 3) reference nodes
    x: np.ndarray                  # (n, 3) current nodes
    tri: np.ndarray | None = None  # (m, 3) local ids
    tet: np.ndarray | None = None  # (m, 4) local ids
    law: int = LAW_TRI_NEOHOOKE
    mu: float = 1.0
    mu2: float = 0.0
    kb: float = 0.0
    c0: float = 0.0
    box: int = 0


@dataclass
class Scene:
    name: str
    boxes: list
    node_start: np.ndarray
    tri_start: np.ndarray
    tet_start: np.ndarray
    tri: np.ndarray
    tet: np.ndarray
    law: np.ndarray
    mu: np.ndarray
    mu2: np.ndarray
    kb: np.ndarray
    c0: np.ndarray
    box: np.ndarray
    X_ref: np.ndarray
    x64: np.ndarray
    anchor: np.ndarray
    x32: np.ndarray
    seed: int = 0
    info: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.node_start.shape[0] - 1)

    @property
    def n_nodes(self) -> int:
        return int(self.X_ref.shape[1])

    @property
    def n_tris(self) -> int:
        return int(self.tri.shape[1])

    @property
    def n_tets(self) -> int:
        return int(self.tet.shape[1])

    @property
    def cell_offset(self) -> np.ndarray:
        off = np.zeros(len(self.boxes) + 1, dtype=np.int64)
        off[1:] = np.cumsum([b.cells for b in self.boxes])
        return off

    @property
    def total_cells(self) -> int:
        return int(self.cell_offset[-1])

    def node_particle(self) -> np.ndarray:
        """Owning particle of every node."""
        return np.repeat(np.arange(self.n_particles), np.diff(self.node_start))

    def box_arrays(self):
        """(n [nb][3] int32, h [nb] f64, origin [nb][3] f64, cell_offset [nb] i64)."""
        n = np.array([b.n for b in self.boxes], dtype=np.int32).reshape(-1, 3)
        h = np.array([b.h for b in self.boxes], dtype=np.float64)
        o = np.array([b.origin for b in self.boxes], dtype=np.float64).reshape(-1, 3)
        return n, h, o, self.cell_offset[:-1].copy()


def assemble(name: str, boxes, particles, seed: int = 0, info=None) -> Scene:
    """Concatenate particles into the SoA scene layout and split positions into anchor + offset."""
    node_start = [0]
    tri_start = [0]
    tet_start = [0]
    tris, tets, Xs, xs = [], [], [], []
    for p in particles:
        base = node_start[-1]
        Xs.append(p.X)
        xs.append(p.x)
        t = p.tri if p.tri is not None else np.zeros((0, 3), np.int32)
        q = p.tet if p.tet is not None else np.zeros((0, 4), np.int32)
        tris.append(t.astype(np.int64) + base)
        tets.append(q.astype(np.int64) + base)
        node_start.append(base + p.X.shape[0])
        tri_start.append(tri_start[-1] + t.shape[0])
        tet_start.append(tet_start[-1] + q.shape[0])
    X = np.concatenate(Xs, axis=0) if Xs else np.zeros((0, 3))
    x = np.concatenate(xs, axis=0) if xs else np.zeros((0, 3))
    tri = np.concatenate(tris, axis=0) if tris else np.zeros((0, 3), np.int64)
    tet = np.concatenate(tets, axis=0) if tets else np.zeros((0, 4), np.int64)
    n_p = len(particles)
    anchor = np.zeros((n_p, 3), dtype=np.float64)
    x32 = np.zeros((x.shape[0], 3), dtype=np.float32)
    x64 = np.zeros_like(x)
    for i in range(n_p):
        s, e = node_start[i], node_start[i + 1]
        a = np.round(x[s:e].mean(axis=0) / ANCHOR_QUANTUM) * ANCHOR_QUANTUM
        off = (x[s:e] - a).astype(np.float32)
        off[np.abs(off) < OFFSET_FLUSH] = 0.0
        anchor[i] = a
        x32[s:e] = off
        x64[s:e] = a + off.astype(np.float64)
        if not np.array_equal(x64[s:e] - a, off.astype(np.float64)):
            raise AssertionError("anchor + offset is not exact in float64")
    return Scene(
        name=name,
        boxes=list(boxes),
        node_start=np.asarray(node_start, dtype=np.int32),
        tri_start=np.asarray(tri_start, dtype=np.int32),
        tet_start=np.asarray(tet_start, dtype=np.int32),
        tri=np.ascontiguousarray(tri.T.astype(np.int32)),
        tet=np.ascontiguousarray(tet.T.astype(np.int32)),
        law=np.array([p.law for p in particles], dtype=np.int32),
        mu=np.array([p.mu for p in particles], dtype=np.float64),
        mu2=np.array([p.mu2 for p in particles], dtype=np.float64),
        kb=np.array([p.kb for p in particles], dtype=np.float64),
        c0=np.array([p.c0 for p in particles], dtype=np.float64),
        box=np.array([p.box for p in particles], dtype=np.int32),
        X_ref=np.ascontiguousarray(X.T),
        x64=np.ascontiguousarray(x64.T),
        anchor=anchor,
        x32=np.ascontiguousarray(x32.T),
        seed=seed,
        info=dict(info or {}),
    )


# ---------------------------------------------------------------- particle kinds
_TEMPLATE_CACHE: dict = {}


def _ico(nu):
    key = ("ico", nu)
    if key not in _TEMPLATE_CACHE:
        _TEMPLATE_CACHE[key] = meshes.icosphere(nu)
    return _TEMPLATE_CACHE[key]


def capsule_template(nu: int, radius: float = 1.0):
    nodes, tris = _ico(nu)
    return nodes * radius, tris


def rbc_template(nu: int = 16, R0: float = RBC_R0):
    key = ("rbc", nu, R0)
    if key not in _TEMPLATE_CACHE:
        nodes, tris = _ico(nu)
        _TEMPLATE_CACHE[key] = (meshes.evans_fung(nodes, R0), tris)
    return _TEMPLATE_CACHE[key]


def ellipsoid_template(dims=(5, 5, 5), axes=PLT_AXES):
    key = ("ell", tuple(dims), tuple(axes))
    if key not in _TEMPLATE_CACHE:
        _TEMPLATE_CACHE[key] = meshes.ellipsoid_tets(*dims, semi_axes=axes)
    return _TEMPLATE_CACHE[key]


def shear_about_centroid(X: np.ndarray, Q: np.ndarray, gamma: float) -> np.ndarray:
    """x = c + Q (I + gamma e1 e2^T) Q^T (X - c), c = node mean."""
    c = X.mean(axis=0)
    S = np.eye(3)
    S[0, 1] = gamma
    A = Q @ S @ Q.T
    return c + (X - c) @ A.T


def place(X: np.ndarray, R: np.ndarray, centre) -> np.ndarray:
    """Rigidly rotate about the node mean and move it to ``centre``."""
    c = X.mean(axis=0)
    return (X - c) @ R.T + np.asarray(centre, dtype=np.float64)


# ---------------------------------------------------------------- configurations
def config1(seed: int = 1001) -> Scene:
    """Single neo-Hookean capsule (nu = 8, R = 1) with Gaussian node noise in a 64^3 box, h = 0.125."""
    rng = np.random.default_rng(seed)
    box = Box((64, 64, 64), 0.125, (0.0, 0.0, 0.0))
    X, tris = capsule_template(8, 1.0)
    centre = np.array(box.length) / 2 + rng.uniform(-box.h / 2, box.h / 2, size=3)
    base = X + centre
    x = base + rng.normal(0.0, 0.05, size=X.shape)
    # (area ratio)^2 screens out collapsed triangles: redraw the noise of their nodes
    for _ in range(10000):
        bad = meshes.triangle_area_ratio(X, x, tris) ** 2 < 0.1
        if not bad.any():
            break
        nodes = np.unique(tris[bad].ravel())
        x[nodes] = base[nodes] + rng.normal(0.0, 0.05, size=(nodes.size, 3))
    else:  # pragma: no cover
        raise RuntimeError("config1: no admissible perturbation")
    p = Particle(X=X, x=x, tri=tris, law=LAW_TRI_NEOHOOKE, mu=1.0, mu2=0.0, kb=0.0, c0=0.0)
    return assemble("capsule_642_grid64", [box], [p], seed, {"sigma": 0.05})


def rbc_particle(rng, nu=16, gamma_range=(0.1, 0.3), scale=1.0, kappa_b=KAPPA_B):
    X, tris = rbc_template(nu)
    X = X * scale
    Q = meshes.random_rotation(rng)
    gamma = rng.uniform(*gamma_range)
    x = shear_about_centroid(X, Q, gamma)
    r_eff = RBC_R_EFF * scale
    return Particle(X=X, x=x, tri=tris, law=LAW_TRI_SKALAK, mu=1.0, mu2=SKALAK_RATIO,
                    kb=kappa_b * r_eff * r_eff, c0=0.0), gamma


def config2(seed: int = 1002) -> Scene:
    """Single Skalak red cell (nu = 16 Evans-Fung, R0 = 3.91) with bending, sheared, 128^3 box, h = R0/8."""
    rng = np.random.default_rng(seed)
    h = RBC_R0 / 8
    box = Box((128, 128, 128), h, (0.0, 0.0, 0.0))
    p, gamma = rbc_particle(rng)
    centre = np.array(box.length) / 2 + rng.uniform(-h / 2, h / 2, size=3)
    p.x = p.x - p.x.mean(axis=0) + centre
    return assemble("rbc_2562_grid128", [box], [p], seed, {"gamma": gamma})


def _lattice_slots(L, counts):
    """Centres and sizes of a regular lattice of slots filling a box of lengths L."""
    size = np.array(L) / np.array(counts)
    idx = np.stack(np.meshgrid(*[np.arange(c) for c in counts], indexing="ij"), axis=-1).reshape(-1, 3)
    return (idx + 0.5) * size, size


def _fit_in_slot(rng, x, slot_centre, slot_size):
    """Translate x (already oriented) to a jittered position fully inside its slot."""
    lo, hi = x.min(axis=0), x.max(axis=0)
    ext = hi - lo
    room = slot_size - ext
    if np.any(room < 0):
        return None
    jitter = rng.uniform(-0.5, 0.5, size=3) * room
    return x - (lo + hi) / 2 + slot_centre + jitter


def _dense_suspension(name, seed, n_rbc, n_plt, grid, hct, slot_counts, gamma_rbc, gamma_plt,
                      max_tilt, plt_dims=(5, 5, 5), rbc_nu=16):
    rng = np.random.default_rng(seed)
    h = (n_rbc * RBC_VOLUME / (hct * grid[0] * grid[1] * grid[2])) ** (1.0 / 3.0)
    box = Box(tuple(grid), h, (0.0, 0.0, 0.0))
    centres, size = _lattice_slots(box.length, slot_counts)
    order = rng.permutation(centres.shape[0])
    if order.size < n_rbc + n_plt:
        raise ValueError("not enough slots")
    particles = []
    slot_iter = iter(order)
    kinds = ["rbc"] * n_rbc + ["plt"] * n_plt
    kinds = [kinds[i] for i in rng.permutation(len(kinds))]
    for kind in kinds:
        for attempt in range(50):
            s = next(slot_iter, None) if attempt == 0 else s
            if kind == "rbc":
                X, tris = rbc_template(rbc_nu)
                gamma = rng.uniform(*gamma_rbc)
            else:
                X, tets = ellipsoid_template(plt_dims)
                gamma = rng.uniform(*gamma_plt)
            # in-plane spin is free; the tilt of the cell axis is bounded by slot clearance
            R = meshes.rotation_about([0, 0, 1], rng.uniform(0, 2 * np.pi))
            tilt_axis = np.array([np.cos(t := rng.uniform(0, 2 * np.pi)), np.sin(t), 0.0])
            R = meshes.rotation_about(tilt_axis, rng.uniform(0, max_tilt) * (0.5 ** attempt)) @ R
            S = np.eye(3)
            S[0, 1] = gamma * (0.5 ** attempt)
            xo = (X - X.mean(axis=0)) @ (R @ S).T
            x = _fit_in_slot(rng, xo, centres[s], size)
            if x is not None:
                break
        else:  # pragma: no cover
            raise RuntimeError(f"{name}: particle does not fit its slot")
        if kind == "rbc":
            particles.append(Particle(X=X, x=x, tri=tris, law=LAW_TRI_SKALAK, mu=1.0, mu2=SKALAK_RATIO,
                                      kb=KAPPA_B * RBC_R_EFF ** 2, c0=0.0))
        else:
            particles.append(Particle(X=X, x=x, tet=tets, law=LAW_TET_NEOHOOKE, mu=PLT_MU,
                                      mu2=SOLID_RATIO * PLT_MU, kb=0.0, c0=0.0))
    vol = n_rbc * RBC_VOLUME
    info = {"hct_target": hct, "hct": vol / (np.prod(box.length)), "h": h, "slots": list(slot_counts)}
    return assemble(name, [box], particles, seed, info)


def refined_suspension(seed: int = 1006, n_rbc: int = 130, grid=(256, 128, 128)) -> Scene:
    """Red cells meshed at nu = 32 (10,242 nodes each, above one workgroup's LDS: the global force path)
    at 20% Ht; h = 0.244 = R0 / 16, the mesh spacing of such a cell."""
    return _dense_suspension(f"refined_{n_rbc}rbc_nu32_grid{grid[0]}x{grid[1]}x{grid[2]}", seed, n_rbc, 0, grid,
                             0.20, (7, 3, 9), (0.0, 0.2), (0.0, 0.1), np.deg2rad(4.0), rbc_nu=32)


def config3(seed: int = 1003) -> Scene:
    """500 red cells + 50 platelets at 20% Ht in a 256x128x128 box."""
    return _dense_suspension("blood_500rbc_50plt_grid256x128x128", seed, 500, 50, (256, 128, 128), 0.20,
                             (11, 5, 15), (0.0, 0.2), (0.0, 0.1), np.deg2rad(4.0))


def config5(seed: int = 1005, n_rbc: int = 4000) -> Scene:
    """4000 red cells (10.2M nodes) at 35% Ht in a 512x256x256 box."""
    return _dense_suspension(f"dense_{n_rbc}rbc_grid512x256x256", seed, n_rbc, 0, (512, 256, 256), 0.35,
                             (18, 9, 25), (0.0, 0.2), (0.0, 0.0), np.deg2rad(4.0))


_TET_DIMS = [(4, 4, 6), (5, 5, 5), (5, 5, 6), (6, 6, 6), (6, 6, 8), (7, 7, 7), (7, 7, 8), (8, 8, 8), (8, 8, 10)]


def config4(seed: int = 1004, n_boxes: int = 64) -> Scene:
    """64 independent periodic boxes, 32^3..128^3, 1-20 mixed particles each, h = 1."""
    rng = np.random.default_rng(seed)
    boxes, particles = [], []
    for b in range(n_boxes):
        N = int(rng.choice(np.arange(32, 129, 8)))
        box = Box((N, N, N), 1.0, (0.0, 0.0, 0.0))
        boxes.append(box)
        n_p = int(rng.integers(1, 21))
        r_eq = min((0.10 * box.cells / n_p * 3 / (4 * np.pi)) ** (1 / 3), 6.0)
        if r_eq < 3.0:
            n_p = max(1, int(0.10 * box.cells / (4 / 3 * np.pi * 27.0)))
            r_eq = 3.0
        placed = []  # (centre, bounding radius)
        for _ in range(n_p):
            kind = rng.integers(0, 3)
            if kind == 0:
                nu = int(rng.integers(8, 17))
                X, tris = capsule_template(nu, r_eq)
                x = shear_about_centroid(X, meshes.random_rotation(rng), rng.uniform(0, 0.1))
                p = Particle(X=X, x=x, tri=tris, law=LAW_TRI_NEOHOOKE, mu=1.0, box=b)
            elif kind == 1:
                p, _ = rbc_particle(rng, gamma_range=(0.0, 0.2), scale=r_eq / RBC_R_EFF)
                p.box = b
            else:
                dims = _TET_DIMS[int(rng.integers(0, len(_TET_DIMS)))]
                aspect = rng.uniform(0.5, 1.0)
                a = r_eq / aspect ** (1 / 3)
                X, tets = ellipsoid_template(dims, (a, a, a * aspect))
                x = shear_about_centroid(X, meshes.random_rotation(rng), rng.uniform(0, 0.1))
                p = Particle(X=X, x=x, tet=tets, law=LAW_TET_NEOHOOKE, mu=1.0, mu2=SOLID_RATIO, box=b)
            rb = float(np.max(np.linalg.norm(p.x - p.x.mean(axis=0), axis=1)))
            L = np.array(box.length)
            for _try in range(200):
                c = rng.uniform(rb + 1.0, L - rb - 1.0)
                if all(np.linalg.norm(c - c2) > rb + r2 + 1.0 for c2, r2 in placed):
                    break
            else:
                continue
            placed.append((c, rb))
            p.x = p.x - p.x.mean(axis=0) + c
            particles.append(p)
    return assemble("batched_64boxes", boxes, particles, seed, {})


# ---------------------------------------------------------------- small scenes for tests
def small_capsule(seed=7, nu=3, n=(12, 10, 14), h=0.35, law=LAW_TRI_NEOHOOKE, kb=0.0, c0=0.0,
                  sigma=0.02, gamma=0.15) -> Scene:
    rng = np.random.default_rng(seed)
    box = Box(tuple(n), h, (0.1, -0.2, 0.3))
    X, tris = capsule_template(nu, 1.0)
    x = shear_about_centroid(X, meshes.random_rotation(rng), gamma) + rng.normal(0, sigma, X.shape)
    x = x - x.mean(axis=0) + np.array(box.origin) + np.array(box.length) / 2 + rng.uniform(-h, h, 3)
    mu2 = SKALAK_RATIO if law == LAW_TRI_SKALAK else 0.0
    p = Particle(X=X, x=x, tri=tris, law=law, mu=1.0, mu2=mu2, kb=kb, c0=c0)
    return assemble("small_capsule", [box], [p], seed)


def small_mixed(seed=11) -> Scene:
    """Two boxes (one with a ragged, non-cubic shape) holding a capsule, a red cell and a tet solid."""
    rng = np.random.default_rng(seed)
    b0 = Box((20, 17, 23), 0.5, (0.0, 0.0, 0.0))
    b1 = Box((13, 13, 13), 0.6, (5.0, -3.0, 1.0))
    parts = []
    X, tris = capsule_template(4, 1.5)
    x = shear_about_centroid(X, meshes.random_rotation(rng), 0.2)
    parts.append(Particle(X=X, x=x - x.mean(0) + [3.0, 3.5, 4.0], tri=tris, law=LAW_TRI_NEOHOOKE, mu=1.0, box=0))
    p, _ = rbc_particle(rng, nu=4, gamma_range=(0.1, 0.2), scale=0.6)
    p.x = p.x - p.x.mean(0) + [7.0, 4.5, 7.0]
    p.box = 0
    parts.append(p)
    X, tets = ellipsoid_template((2, 3, 2), (1.2, 1.0, 0.8))
    x = shear_about_centroid(X, meshes.random_rotation(rng), 0.1)
    parts.append(Particle(X=X, x=x - x.mean(0) + [8.9, 0.9, 4.9], tet=tets, law=LAW_TET_NEOHOOKE,
                          mu=2.0, mu2=100.0, box=1))
    return assemble("small_mixed", [b0, b1], parts, seed)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def make_config(i: int, seed: int | None = None) -> Scene:
    fn = CONFIGS[i]
    return fn() if seed is None else fn(seed)


def subset(scene: Scene, particles) -> Scene:
    """A scene holding only the listed particles (same boxes, same positions and anchors)."""
    particles = np.asarray(particles, dtype=np.int64)
    ns, ts, qs = scene.node_start, scene.tri_start, scene.tet_start
    nodes = np.concatenate([np.arange(ns[p], ns[p + 1]) for p in particles])
    tris = np.concatenate([np.arange(ts[p], ts[p + 1]) for p in particles]) if scene.n_tris else np.zeros(0, np.int64)
    tets = np.concatenate([np.arange(qs[p], qs[p + 1]) for p in particles]) if scene.n_tets else np.zeros(0, np.int64)
    remap = np.full(scene.n_nodes, -1, dtype=np.int64)
    remap[nodes] = np.arange(nodes.size)

    def starts(s):
        return np.concatenate([[0], np.cumsum(s[particles + 1] - s[particles])]).astype(np.int32)

    return Scene(
        name=scene.name + "_subset", boxes=scene.boxes, node_start=starts(ns), tri_start=starts(ts),
        tet_start=starts(qs), tri=np.ascontiguousarray(remap[scene.tri[:, tris]].astype(np.int32)),
        tet=np.ascontiguousarray(remap[scene.tet[:, tets]].astype(np.int32)), law=scene.law[particles],
        mu=scene.mu[particles], mu2=scene.mu2[particles], kb=scene.kb[particles], c0=scene.c0[particles],
        box=scene.box[particles], X_ref=np.ascontiguousarray(scene.X_ref[:, nodes]),
        x64=np.ascontiguousarray(scene.x64[:, nodes]), anchor=scene.anchor[particles],
        x32=np.ascontiguousarray(scene.x32[:, nodes]), seed=scene.seed, info=dict(scene.info))


def with_volume_drift(scene: Scene, rel: float = 1e-3, seed: int = 0, roughness: float = 0.0) -> Scene:
    """The scene with every membrane's current nodes scaled about their mean so that its enclosed
    volume drifts by a factor 1 + d, d ~ U(-rel, rel) per membrane (the volume error a time step
    leaves behind), plus optional N(0, roughness^2) noise per coordinate.  Solids are unchanged.
    Anchors stay as they are; offsets and float64 positions are re-split so that
    x64 == anchor + float64(x32) still holds exactly."""
    rng = np.random.default_rng(seed)
    x = scene.x64.T.copy()
    for p in range(scene.n_particles):
        if scene.tri_start[p + 1] == scene.tri_start[p]:
            continue
        s, e = scene.node_start[p], scene.node_start[p + 1]
        c = x[s:e].mean(axis=0)
        d = rng.uniform(-rel, rel)
        x[s:e] = c + (1.0 + d) ** (1.0 / 3.0) * (x[s:e] - c)
        if roughness:
            x[s:e] += roughness * rng.normal(size=(e - s, 3))
    x32 = np.zeros_like(scene.x32.T)
    x64 = np.zeros_like(x)
    for p in range(scene.n_particles):
        s, e = scene.node_start[p], scene.node_start[p + 1]
        a = scene.anchor[p]
        off = (x[s:e] - a).astype(np.float32)
        off[np.abs(off) < OFFSET_FLUSH] = 0.0
        x32[s:e] = off
        x64[s:e] = a + off.astype(np.float64)
    return Scene(**{**scene.__dict__, "name": scene.name + "_drift", "x64": np.ascontiguousarray(x64.T),
                    "x32": np.ascontiguousarray(x32.T)})
