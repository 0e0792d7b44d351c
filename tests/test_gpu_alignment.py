"""Grids that do not start on a 16-byte boundary, through the C ABI.

The tiled spread writes a tile's cells 16 bytes at a time (empty tiles, the write-out, the merge of the
border rows) only where the grid's first cell and the tile's rows are 16-byte aligned, and one value at
a time otherwise.  A grid that is a view one element into a larger buffer takes the second path
everywhere; its values must equal those of an aligned grid bit for bit (integer tile sums), and the
interpolation from such a grid must equal the interpolation from the aligned one bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import fields, scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
@pytest.mark.parametrize("case", ["rbc_nu16", "small_mixed"])
def test_unaligned_grid_gives_the_aligned_values(case, dtype):
    sc = scenes.make_config(2) if case == "rbc_nu16" else scenes.small_mixed()
    dt = torch.float64 if dtype == ifem.IFEM_F64 else torch.float32
    say(f"[align] {case} dtype {dtype}: {sc.n_nodes} nodes, {sc.total_cells} cells")
    F = fields.random_forces(sc, seed=11)
    if dtype == ifem.IFEM_F64:
        x, a = cu(sc.x64, torch.float64), None
    else:
        x, a = cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64)
    n = 3 * sc.total_cells
    plan = ifem.Plan(sc)
    G = torch.full((3, sc.total_cells), float("nan"), dtype=dt, device="cuda")
    buf = torch.full((n + 1,), float("nan"), dtype=dt, device="cuda")
    Gu = buf[1:].view(3, sc.total_cells)  # one element past a 256-byte aligned allocation
    assert Gu.data_ptr() % 16 != 0
    for call in range(2):  # the plan's first call (second list pass) and a call on its carried lists
        plan.spread(dtype, x, a, cu(F, dt), G)
        plan.spread(dtype, x, a, cu(F, dt), Gu)
        torch.cuda.synchronize()
        assert torch.isnan(buf[:1]).all(), "the element before the grid was written"
        g, gu = G.cpu().numpy(), Gu.cpu().numpy()
        say(f"  call {call}: {int(np.count_nonzero(g))} non-zero values")
        assert np.all(np.isfinite(g))
        assert np.array_equal(g, gu), f"call {call}: the unaligned grid differs"
    assert plan.status() == [0, 0, 0, 0, 0]
    # interpolation: the same velocity field held aligned and one element off
    u = fields.scene_velocity(sc, dtype=torch.float64).to(dt).to("cuda")
    ubuf = torch.empty((n + 1,), dtype=dt, device="cuda")
    uu = ubuf[1:].view(3, sc.total_cells)
    uu.copy_(u)
    v = torch.empty((3, sc.n_nodes), dtype=dt, device="cuda")
    vu = torch.empty_like(v)
    plan.interp(dtype, x, a, u, v)
    plan.interp(dtype, x, a, uu, vu)
    torch.cuda.synchronize()
    assert torch.equal(v, vu)
    assert plan.status() == [0, 0, 0, 0, 0]
