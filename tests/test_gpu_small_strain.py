"""Float32 element forces keep their accuracy as the strain shrinks (the compensated metric).

The float32 path forms Delta = g - G from the current edges in float-float, so the invariants
I1 - 2 and J^2 - 1 carry no cancellation error and the relative error of the forces does not
grow like u32 / strain.  Meshes are rotated by a random rigid rotation on top of the small
deformation, so a frame-dependent formulation would also be caught.  Only the float32 path is
checked here: at strain 1e-5 the float64 invariants lose about 11 digits to cancellation on
both sides (the oracle forms I1 - 2 from the current frame), which leaves the float64
comparison ill-conditioned, not wrong.
"""
import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F32_ELASTIC_TOL = 1e-5  # the bar of the float32 elastic forces at any strain


def _scene(law, eps, seed=5):
    rng = np.random.default_rng(seed)
    if law == scenes.LAW_TET_NEOHOOKE:
        X, tets = meshes.ellipsoid_tets(4, 4, 4, (1.5, 1.2, 1.0))
        tris = None
        mu2 = scenes.SOLID_RATIO
    else:
        X, tris = meshes.icosphere(8)
        tets = None
        mu2 = scenes.SKALAK_RATIO if law == scenes.LAW_TRI_SKALAK else 0.0
    E = rng.normal(size=(3, 3))
    E = 0.5 * (E + E.T)
    E /= np.linalg.norm(E)
    Q = meshes.random_rotation(rng)
    c = X.mean(axis=0)
    k = rng.normal(size=3)
    wobble = np.sin((X - c) @ k)[:, None] * rng.normal(size=3)[None, :]
    x = (X - c + eps * ((X - c) @ E.T + 0.3 * wobble)) @ Q.T + [4.0, 4.5, 5.0]
    box = Box((24, 24, 24), 0.4, (0.0, 0.0, 0.0))
    p = Particle(X=X, x=x, tri=tris, tet=tets, law=law, mu=1.0, mu2=mu2)
    return assemble("small_strain", [box], [p], seed)


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-4, 1e-5])
@pytest.mark.parametrize("law", [scenes.LAW_TRI_NEOHOOKE, scenes.LAW_TRI_SKALAK, scenes.LAW_TET_NEOHOOKE])
def test_fp32_forces_at_small_strain(law, eps):
    sc = _scene(law, eps)
    print(f"[gpu] small strain law {law} eps {eps:g}", flush=True)
    Fo, cnt = oracle.forces(sc)
    assert cnt[0] == 0 and cnt[1] == 0
    plan = ifem.Plan(sc)
    x = torch.as_tensor(sc.x32, device="cuda")
    a = torch.as_tensor(sc.anchor, device="cuda")
    F = torch.empty((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    plan.element_forces(ifem.IFEM_F32, x, a, F, None)
    got = F.cpu().numpy().astype(np.float64)
    e = np.linalg.norm(got - Fo) / np.linalg.norm(Fo)
    print(f"    force rel err {e:.3e} (|F| {np.linalg.norm(Fo):.3e})", flush=True)
    assert e <= F32_ELASTIC_TOL
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()
