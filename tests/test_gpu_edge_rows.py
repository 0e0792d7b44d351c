"""Edge cases of the volume correction, the update, the viscoelastic terms and the anti-sticking, through
the C ABI: empty scenes, a particle alone, solids without membranes and membranes without solids.  Each
result is the one the method fixes for that case (nothing to move, nothing to add), compared bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def test_empty_scene_every_row():
    say("[gpu] empty scene: volume, advance, cell interpolation, fluid forces, anti-sticking")
    sc = assemble("empty", [Box((9, 8, 7), 0.5, (0.0, 0.0, 0.0))], [])
    plan = ifem.Plan(sc)
    e = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    plan.volume_correct(ifem.IFEM_F64, e, e)
    plan.advance(ifem.IFEM_F64, e, e, torch.zeros_like(e), v_prev=e, dt=0.1)
    grid = torch.ones((6, sc.total_cells), dtype=torch.float64, device="cuda")
    plan.interp_cells(ifem.IFEM_F64, e, None, grid, torch.zeros((6, 0), dtype=torch.float64, device="cuda"))
    plan.fluid_forces(ifem.IFEM_F64, e, e, torch.zeros_like(e), eta=1.0)
    plan.antistick(ifem.IFEM_F64, e, None, torch.zeros_like(e), 0.5)
    torch.cuda.synchronize()
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()


def _lone_capsule():
    X, tris = meshes.icosphere(3)
    return assemble("lone", [Box((12, 12, 12), 0.5, (0.0, 0.0, 0.0))],
                    [Particle(X=X, x=X * 1.2 + 3.0, tri=tris, law=scenes.LAW_TRI_NEOHOOKE)])


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_a_particle_alone_never_moves_away_from_itself(dtype):
    say(f"[gpu] anti-sticking, one capsule, dtype {dtype}")
    sc = _lone_capsule()
    plan = ifem.Plan(sc)
    faces = torch.full((sc.n_nodes,), 7, dtype=torch.int64, device="cuda")
    if dtype == ifem.IFEM_F64:
        x, anchor = cu(sc.x64, torch.float64), None
    else:
        x, anchor = cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64)
    out = torch.empty_like(x)
    plan.antistick(dtype, x, anchor, out, 0.5, faces)  # d_min well above the mesh spacing: own faces are near
    torch.cuda.synchronize()
    assert torch.equal(out, x)
    assert bool((faces == -1).all())
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()


def _solid_only():
    nodes, tets = meshes.kuhn_box(2, 2, 3)
    return assemble("solid", [Box((10, 10, 10), 0.5, (0.0, 0.0, 0.0))],
                    [Particle(X=nodes, x=nodes * 1.05 + 2.5, tet=tets, law=scenes.LAW_TET_NEOHOOKE, mu=1.0,
                              mu2=4.0)])


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_volume_correction_copies_solids_unchanged(dtype):
    say(f"[gpu] volume correction on a solid only, dtype {dtype}")
    sc = _solid_only()
    plan = ifem.Plan(sc)
    x = cu(sc.x64, torch.float64) if dtype == ifem.IFEM_F64 else cu(sc.x32, torch.float32)
    out = torch.full_like(x, float("nan"))
    lam = torch.full((sc.n_particles,), 9.0, dtype=torch.float64, device="cuda")
    plan.volume_correct(dtype, x, out, lambda_out=lam)
    torch.cuda.synchronize()
    assert torch.equal(out, x)
    assert float(lam.abs().max()) == 0.0
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_fluid_forces_add_nothing_without_solids(dtype):
    say(f"[gpu] fluid-stress forces on a membrane only, dtype {dtype}")
    sc = _lone_capsule()
    plan = ifem.Plan(sc)
    dt = torch.float64 if dtype == ifem.IFEM_F64 else torch.float32
    rng = np.random.default_rng(2)
    x = cu(sc.x64, torch.float64) if dtype == ifem.IFEM_F64 else cu(sc.x32, torch.float32)
    v = cu(rng.normal(size=(3, sc.n_nodes)), dt)
    C = cu(np.tile(np.array([1.1, 0.9, 1.0, 0.05, 0.0, -0.02])[:, None], (1, sc.n_nodes)), dt)
    f0 = cu(rng.normal(size=(3, sc.n_nodes)), dt)
    f = f0.clone()
    plan.fluid_forces(dtype, x, v, f, C=C, eta=0.7, G=3.0)
    torch.cuda.synchronize()
    assert torch.equal(f, f0)
    plan.close()


def test_advance_with_zero_step_and_zero_velocity_is_the_identity():
    say("[gpu] advance: dt = 0, and v = v_prev = 0")
    sc = _lone_capsule()
    plan = ifem.Plan(sc)
    rng = np.random.default_rng(4)
    for dtype, dt in ((ifem.IFEM_F64, torch.float64), (ifem.IFEM_F32, torch.float32)):
        x = cu(sc.x64, torch.float64) if dtype == ifem.IFEM_F64 else cu(sc.x32, torch.float32)
        v = cu(rng.normal(size=(3, sc.n_nodes)), dt)
        out = torch.empty_like(x)
        plan.advance(dtype, x, v, out, v_prev=v, dt=0.0)
        torch.cuda.synchronize()
        assert torch.equal(out, x)
        z = torch.zeros_like(v)
        plan.advance(dtype, x, z, out, v_prev=z, dt=0.37)
        torch.cuda.synchronize()
        assert torch.equal(out, x)
    plan.close()


def test_cell_interpolation_of_a_constant_field_is_that_constant():
    # the linear MLS basis reproduces constants: every node gets the field's value (to rounding)
    say("[gpu] cell interpolation of constant fields")
    sc = _lone_capsule()
    plan = ifem.Plan(sc)
    vals = np.array([1.0, -2.5, 0.125, 3.0, 1e-3, -7.0])
    grid = cu(np.tile(vals[:, None], (1, sc.total_cells)), torch.float64)
    out = torch.empty((6, sc.n_nodes), dtype=torch.float64, device="cuda")
    plan.interp_cells(ifem.IFEM_F64, cu(sc.x64, torch.float64), None, grid, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(np.abs(got - vals[:, None]) <= 1e-13 * np.abs(vals)[:, None])
    plan.close()
