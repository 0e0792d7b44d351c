"""Particle sizes at the limits of one workgroup's LDS, through the C ABI.

A particle's nodal force accumulators live in one workgroup's LDS (160 KB): float64 accumulators for
3 components fit up to 6826 nodes without bending and 5120 with it (a fourth array for the
curvature).  A deformed Kuhn-lattice solid near that bound (17^3 = 4913 nodes, 24,576 tetrahedra)
is checked against the oracle in both precisions; float32 also stages its positions in LDS,
float64 reads them through the caches at this size.  A membrane above the bound is rejected when the
plan is created, with an error, not a fault.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble

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


def test_membrane_beyond_the_lds_bound_is_rejected():
    X, tris = meshes.icosphere(32)  # 10 * 32^2 + 2 = 10,242 nodes: 4 x 10,242 float64 arrays exceed 160 KB
    sc = assemble("huge_capsule", [Box((40, 40, 40), 0.25, (0.0, 0.0, 0.0))],
                  [Particle(X=X, x=X * 3.0 + 5.0, tri=tris, law=scenes.LAW_TRI_NEOHOOKE, kb=0.01)])
    say(f"[gpu] {sc.n_nodes}-node membrane: plan creation must fail cleanly")
    with pytest.raises(ifem.IfemError):
        ifem.Plan(sc)
    # the library still works afterwards
    sc2 = _big_solid()
    plan = ifem.Plan(sc2)
    F = torch.empty((3, sc2.n_nodes), dtype=torch.float64, device="cuda")
    plan.element_forces(ifem.IFEM_F64, cu(sc2.x64, torch.float64), None, F, None)
    torch.cuda.synchronize()
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()
