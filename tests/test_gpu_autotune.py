"""Launch-shape autotuning (ifem_plan_autotune): the tuned plan gives the same results bit for bit as a
plan created with the tuning it chose, and the choice is recorded for later plans of the same sizes (in
the process, and across processes through the IFEM_TUNE_CACHE file)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import fields, scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CANDIDATE_TILES = {(32, 16, 8), (16, 16, 16), (64, 8, 8), (32, 32, 4), (16, 32, 8), (32, 8, 8), (16, 16, 8),
                   (64, 16, 4), (32, 16, 16)}


def say(msg):
    print(msg, flush=True)


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _inputs(sc, dtype):
    tdt = torch.float64 if dtype == ifem.IFEM_F64 else torch.float32
    if dtype == ifem.IFEM_F64:
        x, a = cu(sc.x64, torch.float64), None
    else:
        x, a = cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64)
    F = cu(fields.random_forces(sc, seed=41), tdt)
    u = fields.scene_velocity(sc, device="cuda", dtype=tdt)
    return tdt, x, a, F, u


def _transfers(plan, sc, dtype, x, a, F, u, tdt):
    G = torch.empty((3, sc.total_cells), dtype=tdt, device="cuda")
    v = torch.empty((3, sc.n_nodes), dtype=tdt, device="cuda")
    plan.spread(dtype, x, a, F, G)
    plan.interp(dtype, x, a, u, v)
    torch.cuda.synchronize()
    return G.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("dtype", [ifem.IFEM_F32, ifem.IFEM_F64])
def test_autotuned_plan_equals_a_plan_made_with_its_choice(dtype, tmp_path, monkeypatch):
    cache = tmp_path / "tuning.txt"
    monkeypatch.setenv("IFEM_TUNE_CACHE", str(cache))
    for make in (scenes.small_mixed, scenes.config2):
        sc = make()
        tdt, x, a, F, u = _inputs(sc, dtype)
        plan = ifem.Plan(sc)
        G0 = torch.empty((3, sc.total_cells), dtype=tdt, device="cuda")
        v0 = torch.empty((3, sc.n_nodes), dtype=tdt, device="cuda")
        chosen = plan.autotune(dtype, x, a, F, G0, u, v0)
        say(f"[gpu] autotune {sc.name} dtype {dtype}: {chosen}")
        assert tuple(chosen["tile"]) in CANDIDATE_TILES and chosen["block_points"] in (64, 128, 256)
        assert plan.info()[3:6] == chosen["tile"] and plan.info()[7] == chosen["block_points"]
        G1, v1 = _transfers(plan, sc, dtype, x, a, F, u, tdt)
        ref = ifem.Plan(sc, tuning=chosen)
        G2, v2 = _transfers(ref, sc, dtype, x, a, F, u, tdt)
        assert np.array_equal(G1, G2) and np.array_equal(v1, v2)
        assert plan.status() == [0, 0, 0, 0, 0] and ref.status() == [0, 0, 0, 0, 0]
        # a plan of the same sizes made without a tuning takes the recorded one
        again = ifem.Plan(sc)
        assert again.info()[3:6] == chosen["tile"] and again.info()[7] == chosen["block_points"]
        for p in (plan, ref, again):
            p.close()
        lines = [l.split() for l in cache.read_text().splitlines()]
        assert any(l[0] == "ifem-tuning-v1" and [int(v) for v in l[3:6]] == chosen["tile"] for l in lines)
    # another process reads the file back
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1807_08219_amd import ifem\n"
            "from paper_1807_08219_amd.inputs import scenes\n"
            "import torch; torch.cuda.set_device(0)\n"
            "p = ifem.Plan(scenes.config2()); print('INFO', *p.info()[3:8]); p.close()\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240,
                         env={**os.environ, "IFEM_TUNE_CACHE": str(cache)})
    assert out.returncode == 0, out.stderr[-2000:]
    info = [int(v) for v in next(l for l in out.stdout.splitlines() if l.startswith("INFO")).split()[1:]]
    assert info[:3] == chosen["tile"] and info[4] == chosen["block_points"]
