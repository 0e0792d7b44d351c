"""Particle sizes at and beyond the limit of one workgroup's LDS, through the C ABI.

A particle whose nodal force accumulators fit one workgroup's LDS (160 KB: float64 accumulators for
3 components, up to 6741 nodes without bending and 5056 with it, a fourth array holding the
curvature) takes the per-particle force kernel; a larger one takes the global-memory path (element
forces into a scratch slot per corner, a fixed-order gather per node).  Checked against the oracle:
a deformed Kuhn-lattice solid near the bound (17^3 = 4913 nodes, 24,576 tetrahedra) in both
precisions, and, beyond it, one plan holding a nu = 32 red cell (10,242 nodes, Skalak, bending), a
27^3 = 19,683-node solid and a small capsule (the per-particle kernel beside the global path):
forces and reductions, run-to-run bits, the volume correction, the fluid-stress forces, and the
count of inverted elements.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble
from volume_bars import U32, lambda_bars

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F64_TOL = 1e-12
F32_ELASTIC_TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0))


def _big_solid(seed=5):
    rng = np.random.default_rng(seed)
    nodes, tets = meshes.kuhn_box(16, 16, 16)  # 17^3 nodes on [-1, 1]^3
    X = nodes * 2.0  # lattice spacing 0.25
    A = np.eye(3) + 0.05 * rng.normal(size=(3, 3))
    x = X @ A.T + 0.005 * rng.normal(size=X.shape) + 6.0
    return assemble("big_solid", [Box((24, 24, 24), 0.5, (0.0, 0.0, 0.0))],
                    [Particle(X=X, x=x, tet=tets, law=scenes.LAW_TET_NEOHOOKE, mu=1.0, mu2=10.0)])


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_solid_near_the_lds_bound(dtype):
    sc = _big_solid()
    say(f"[gpu] {sc.n_nodes}-node solid ({sc.n_tets} tetrahedra), dtype {dtype}")
    assert sc.n_nodes == 17 ** 3
    Fo, cnt = oracle.forces(sc)
    assert cnt[0] == 0
    plan = ifem.Plan(sc)
    if dtype == ifem.IFEM_F64:
        x, a, dt = cu(sc.x64, torch.float64), None, torch.float64
    else:
        x, a, dt = cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64), torch.float32
    F = torch.empty((3, sc.n_nodes), dtype=dt, device="cuda")
    plan.element_forces(dtype, x, a, F, None)
    torch.cuda.synchronize()
    e = rel(F.cpu().numpy(), Fo)
    say(f"    rel err {e:.3e}")
    assert e <= (F64_TOL if dtype == ifem.IFEM_F64 else F32_ELASTIC_TOL)
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()


def _large_scene(seed=21):
    """A nu = 32 red cell (bending), a 19,683-node tetrahedral solid and a nu = 3 capsule in one box."""
    rng = np.random.default_rng(seed)
    h = scenes.RBC_R0 / 16
    box = Box((176, 112, 112), h, (0.0, 0.0, 0.0))
    rbc, _ = scenes.rbc_particle(rng, nu=32)
    rbc.x = rbc.x - rbc.x.mean(0) + [10.0, 13.5, 13.0]
    nodes, tets = meshes.kuhn_box(26, 26, 26)  # 27^3 nodes on [-1, 1]^3
    X = nodes * 3.0
    A = np.eye(3) + 0.05 * rng.normal(size=(3, 3))
    x = (X - X.mean(0)) @ A.T + 0.01 * rng.normal(size=X.shape) + [27.0, 14.0, 13.5]
    solid = Particle(X=X, x=x, tet=tets, law=scenes.LAW_TET_NEOHOOKE, mu=1.0, mu2=20.0)
    Xc, tris = meshes.icosphere(3)
    cap = Particle(X=Xc, x=Xc * 1.05 + [38.0, 6.0, 6.0], tri=tris, law=scenes.LAW_TRI_NEOHOOKE, mu=1.0)
    return assemble("large_particles", [box], [rbc, solid, cap], seed)


def _nodes_of(sc, p):
    return np.arange(sc.node_start[p], sc.node_start[p + 1])


@pytest.fixture(scope="module")
def large():
    sc = _large_scene()
    assert sc.n_nodes == 10242 + 27 ** 3 + 92
    say(f"[gpu] large-particle plan: {sc.n_nodes} nodes, {sc.n_tris} triangles, {sc.n_tets} tetrahedra")
    plan = ifem.Plan(sc)
    yield sc, plan
    plan.close()


def _pos(sc, dtype):
    if dtype == ifem.IFEM_F64:
        return cu(sc.x64, torch.float64), None, torch.float64
    return cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64), torch.float32


def _forces(plan, sc, dtype, x=None):
    xd, a, dt = _pos(sc, dtype)
    if x is not None:
        xd = x
    F = torch.full((3, sc.n_nodes), float("nan"), dtype=dt, device="cuda")
    red = torch.full((sc.n_particles, 5), float("nan"), dtype=torch.float64, device="cuda")
    plan.element_forces(dtype, xd, a, F, red)
    torch.cuda.synchronize()
    return F.cpu().numpy(), red.cpu().numpy()


# float32 bars per particle: elastic forces as elsewhere; the nu = 32 cell's bending forces carry
# the rounding of edge vectors of length h relative to offsets of size R twice (curvature, then its
# Laplacian), (R / h)^2 = 4 times the nu = 16 cell's, whose bar is 2e-5
F32_BAR = {0: 8e-5, 1: F32_ELASTIC_TOL, 2: F32_ELASTIC_TOL}


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_large_particles_forces_and_reductions(large, dtype):
    sc, plan = large
    say(f"[gpu] large particles: forces dtype {dtype}")
    Fo, cnt = oracle.forces(sc)
    ro = oracle.reduce(sc)
    assert cnt[0] == 0
    F, red = _forces(plan, sc, dtype)
    for p in range(sc.n_particles):
        idx = _nodes_of(sc, p)
        e = rel(F[:, idx], Fo[:, idx])
        bar = F64_TOL if dtype == ifem.IFEM_F64 else F32_BAR[p]
        say(f"    particle {p} ({idx.size} nodes): forces rel err {e:.3e} (bar {bar:.0e})")
        assert e <= bar
    assert rel(red[:, 0], ro[:, 0]) <= 1e-12
    assert rel(red[:, 1], ro[:, 1]) <= 1e-12
    assert rel(red[:, 2:], ro[:, 2:]) <= 1e-12
    assert plan.status() == [0, 0, 0, 0, 0]
    # the global path sums in fixed orders: a second call gives the same bits
    F2, red2 = _forces(plan, sc, dtype)
    assert np.array_equal(F2, F) and np.array_equal(red2, red)


def test_large_particles_count_inverted_elements(large):
    sc, plan = large
    x = sc.x64.copy()
    t = sc.tet_start[1] + 1234  # one tetrahedron of the large solid turned inside out
    ids = sc.tet[:, t]
    face = x[:, ids[1:]].mean(axis=1)
    x[:, ids[0]] = face + 1.5 * (face - x[:, ids[0]])
    Fo, cnt = oracle.forces(sc, x=x)
    assert cnt[0] >= 1
    say(f"[gpu] large solid with {cnt[0]} inverted elements")
    F, _ = _forces(plan, sc, ifem.IFEM_F64, x=cu(x, torch.float64))
    st = plan.status()
    assert st[0] == cnt[0] and st[1] == cnt[1]
    assert rel(F, Fo) <= F64_TOL


def test_large_particles_volume_correction():
    sc = scenes.with_volume_drift(_large_scene(), rel=1e-3, seed=4)
    say("[gpu] large particles: volume correction")
    xo, lo, bad = oracle.volume_correct(sc)
    assert bad == 0
    bars, alpha, xbar = lambda_bars(sc, xo, lo)
    plan = ifem.Plan(sc)
    x = cu(sc.x64, torch.float64)
    xout = torch.empty_like(x)
    lam = torch.full((sc.n_particles,), -7.0, dtype=torch.float64, device="cuda")
    plan.volume_correct(ifem.IFEM_F64, x, xout, lambda_out=lam)
    torch.cuda.synchronize()
    lg, xg = lam.cpu().numpy(), xout.cpu().numpy()
    say(f"    f64: L {lg} oracle {lo}")
    assert np.all(np.abs(lg - lo) <= bars)
    assert np.all(np.abs(xg - xo) <= xbar)
    assert lg[1] == 0.0
    assert np.array_equal(xg[:, _nodes_of(sc, 1)], sc.x64[:, _nodes_of(sc, 1)])
    xin = x.clone()
    plan.volume_correct(ifem.IFEM_F64, xin, xin)
    torch.cuda.synchronize()
    assert np.array_equal(xin.cpu().numpy(), xg)
    x32 = cu(sc.x32, torch.float32)
    o32 = torch.empty_like(x32)
    lam32 = torch.empty_like(lam)
    plan.volume_correct(ifem.IFEM_F32, x32, o32, lambda_out=lam32)
    torch.cuda.synchronize()
    assert np.all(np.abs(lam32.cpu().numpy() - lo) <= bars)
    rel_off = xo - sc.anchor[sc.node_particle()].T
    got = o32.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - rel_off) <= U32 * np.abs(rel_off) + xbar)
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()


def test_large_particles_fluid_forces(large):
    sc, plan = large
    say("[gpu] large particles: fluid-stress forces")
    rng = np.random.default_rng(8)
    v = rng.normal(size=(3, sc.n_nodes))
    C = 1.0 * (np.arange(6) < 3)[:, None] + 0.1 * rng.normal(size=(6, sc.n_nodes))
    eta, G = 1.1, 0.7
    ref, bad = oracle.fluid_forces(sc, v, C, eta=eta, G=G)
    assert bad == 0 and np.abs(ref).max() > 0
    f0 = rng.normal(size=(3, sc.n_nodes))
    f = cu(f0, torch.float64)
    plan.fluid_forces(ifem.IFEM_F64, cu(sc.x64, torch.float64), cu(v, torch.float64), f, C=cu(C, torch.float64),
                      eta=eta, G=G)
    torch.cuda.synchronize()
    got = f.cpu().numpy()
    e = rel(got - f0, ref)
    say(f"    f64 rel err {e:.3e}")
    assert e <= F64_TOL
    for p in (0, 2):
        assert np.array_equal(got[:, _nodes_of(sc, p)], f0[:, _nodes_of(sc, p)])
    v32, C32, f032 = v.astype(np.float32), C.astype(np.float32), f0.astype(np.float32)
    ref32, _ = oracle.fluid_forces(sc, v32.astype(np.float64), C32.astype(np.float64), eta=eta, G=G)
    f = cu(f032, torch.float32)
    plan.fluid_forces(ifem.IFEM_F32, cu(sc.x32, torch.float32), cu(v32, torch.float32), f, C=cu(C32, torch.float32),
                      eta=eta, G=G)
    torch.cuda.synchronize()
    got32 = f.cpu().numpy().astype(np.float64)
    want = f032.astype(np.float64) + ref32
    bar = U32 * (np.abs(f032) + np.abs(ref32)) + 1e-12 * np.abs(ref32).max()
    say(f"    f32 |err| / bar max {(np.abs(got32 - want) / bar).max():.3f}")
    assert np.all(np.abs(got32 - want) <= bar)
    assert plan.status() == [0, 0, 0, 0, 0]


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_large_particles_transfers(large, dtype):
    # the nodes of particles on the global force path are spread and interpolated like any others
    sc, plan = large
    say(f"[gpu] large particles: spread and interpolation, dtype {dtype}")
    from paper_1807_08219_amd.inputs import fields
    rng = np.random.default_rng(12)
    F = rng.normal(size=(3, sc.n_nodes))
    u = fields.scene_velocity(sc).numpy()
    xd, a, dt = _pos(sc, dtype)
    if dtype == ifem.IFEM_F32:
        F = F.astype(np.float32).astype(np.float64)
        u = u.astype(np.float32).astype(np.float64)
    G = torch.empty((3, sc.total_cells), dtype=dt, device="cuda")
    plan.spread(dtype, xd, a, cu(F, dt), G)
    v = torch.empty((3, sc.n_nodes), dtype=dt, device="cuda")
    plan.interp(dtype, xd, a, cu(u, dt), v)
    torch.cuda.synchronize()
    eg = rel(G.cpu().numpy(), oracle.spread(sc, F))
    ev = rel(v.cpu().numpy(), oracle.interp(sc, u))
    say(f"    spread rel err {eg:.3e}, interp rel err {ev:.3e}")
    bar = F64_TOL if dtype == ifem.IFEM_F64 else 1e-6
    assert eg <= bar and ev <= bar
    assert plan.status() == [0, 0, 0, 0, 0]


def test_large_membrane_without_bending():
    # a plan whose only large particle is a neo-Hookean capsule without bending (the global path
    # without its curvature passes), beside a small solid on the per-workgroup kernel
    # sheared and roughened by 0.003 (1/40 of an edge): moving every position by one unit in its last
    # place changes these forces by 5e-13 relative, inside the float64 bar (larger noise, or none,
    # leaves forces that the float64 positions determine less well than 1e-12)
    rng = np.random.default_rng(31)
    X, tris = meshes.icosphere(32)  # 10,242 nodes
    x = scenes.shear_about_centroid(X * 2.0, meshes.random_rotation(rng), 0.1) + 0.003 * rng.normal(size=X.shape)
    x = x + [8.0, 8.0, 8.0]
    Xs, tets = meshes.kuhn_box(4, 4, 4)
    xs = Xs * 1.1 + [15.0, 8.0, 8.0]
    sc = assemble("large_capsule", [Box((40, 32, 32), 0.5, (0.0, 0.0, 0.0))],
                  [Particle(X=X * 2.0, x=x, tri=tris, law=scenes.LAW_TRI_NEOHOOKE, mu=1.0),
                   Particle(X=Xs, x=xs, tet=tets, law=scenes.LAW_TET_NEOHOOKE, mu=1.0, mu2=10.0)], 31)
    say(f"[gpu] large capsule without bending ({sc.node_start[1]} nodes) and a small solid")
    Fo, cnt = oracle.forces(sc)
    ro = oracle.reduce(sc)
    assert cnt[0] == 0
    plan = ifem.Plan(sc)
    for dtype in (ifem.IFEM_F64, ifem.IFEM_F32):
        F, red = _forces(plan, sc, dtype)
        e = rel(F, Fo)
        say(f"    dtype {dtype}: forces rel err {e:.3e}")
        assert e <= (F64_TOL if dtype == ifem.IFEM_F64 else F32_ELASTIC_TOL)
        assert rel(red[:, 0], ro[:, 0]) <= 1e-12 and rel(red[:, 2:], ro[:, 2:]) <= 1e-12
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()
