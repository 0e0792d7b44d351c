"""The three step calls captured in a HIP graph replay to the eager result, replay after replay."""
import sys

import numpy as np
import pytest

from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import fields, scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_graph_replays_match_eager():
    print("[gpu] graph capture of the float32 step on the mixed scene", flush=True)
    sc = scenes.small_mixed()
    plan = ifem.Plan(sc)
    x32 = torch.as_tensor(sc.x32, device="cuda")
    anchor = torch.as_tensor(sc.anchor, device="cuda")
    u = fields.scene_velocity(sc).to(torch.float32).cuda()
    F = torch.zeros((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    red = torch.zeros((sc.n_particles, 5), dtype=torch.float64, device="cuda")
    G = torch.zeros((3, sc.total_cells), dtype=torch.float32, device="cuda")
    v = torch.zeros((3, sc.n_nodes), dtype=torch.float32, device="cuda")

    def step(stream=None):
        plan.element_forces(ifem.IFEM_F32, x32, anchor, F, red, stream)
        plan.spread(ifem.IFEM_F32, x32, anchor, F, G, stream)
        plan.interp(ifem.IFEM_F32, x32, anchor, u, v, stream)

    step()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (F, red, G, v)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        step(s)  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            step(s)
    torch.cuda.synchronize()
    for r in range(4):
        for t in (F, red, G, v):
            t.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, ref in zip((F, red, G, v), eager):
            assert torch.equal(got, ref), f"replay {r} differs from the eager step"
    plan.close()


def test_antistick_and_volume_graph_replays_match_eager():
    # the end-of-step calls captured too: their counters and keys are cleared by fill kernels inside
    # the calls, so every replay starts from the same state
    print("[gpu] graph capture of anti-sticking and volume correction", flush=True)
    sc = scenes.small_mixed()
    plan = ifem.Plan(sc)
    x32 = torch.as_tensor(scenes.with_volume_drift(sc, rel=1e-3, seed=2).x32, device="cuda")
    anchor = torch.as_tensor(sc.anchor, device="cuda")
    moved = torch.zeros_like(x32)
    faces = torch.zeros(sc.n_nodes, dtype=torch.int64, device="cuda")
    corrected = torch.zeros_like(x32)
    lam = torch.zeros(sc.n_particles, dtype=torch.float64, device="cuda")
    d_min = sc.boxes[0].h

    def step(stream=None):
        plan.antistick(ifem.IFEM_F32, x32, anchor, moved, d_min, faces, stream)
        plan.volume_correct(ifem.IFEM_F32, moved, corrected, lambda_out=lam, stream=stream)

    step()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (moved, faces, corrected, lam)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        step(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            step(s)
    torch.cuda.synchronize()
    for r in range(4):
        for t in (moved, corrected, lam):
            t.fill_(-1.0)
        faces.fill_(7)
        step()  # eager calls between replays use the same plan workspaces
        torch.cuda.synchronize()
        for t in (moved, corrected, lam):
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, ref in zip((moved, faces, corrected, lam), eager):
            assert torch.equal(got, ref), f"replay {r} differs from the eager calls"
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()
