"""The tiled spread's lists carried from call to call, through the C ABI.

A plan lays out each spread call's node lists from the previous call's list lengths; the lists that
outgrow that room (all of them on a plan's first call) are filled by a second pass.  Whatever the
positions did between two calls (nothing, a move of a fraction of a cell, a move of several cells),
the grid must equal the one a fresh plan produces on its first call, bit for bit (the tile sums are
integers: independent of where and in which order a list holds its entries), and match the oracle's
spread (Sec. II.C) to the usual bars.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F64_TOL = 1e-12
F32_TRANSFER_TOL = 1e-6

# absolute translations of every particle, in call order (multiples of 2^-10, so that anchors stay
# exact): the first call, the same positions again, a move of a fraction of a cell, the same again,
# a move of several cells, and back
MOVES = [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.25, -0.125, 0.375), (0.25, -0.125, 0.375),
         (3.0, -2.5, 4.75), (0.0, 0.0, 0.0)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _spread(plan, sc, dtype, shift, F):
    s = np.asarray(shift, dtype=np.float64)
    if dtype == ifem.IFEM_F64:
        x, a, dt = cu(sc.x64 + s[:, None], torch.float64), None, torch.float64
    else:
        x, a, dt = cu(sc.x32, torch.float32), cu(sc.anchor + s[None, :], torch.float64), torch.float32
    G = torch.full((3, sc.total_cells), float("nan"), dtype=dt, device="cuda")
    plan.spread(dtype, x, a, cu(F, dt), G)
    torch.cuda.synchronize()
    return G.cpu().numpy()


# (4, 4, 4): half of the entries sit on a tile's first or last x layer, so the lists together want
# more room than the carried array holds and the lists placed last get none (a non-empty one among
# them is filled by the second pass on every call)
@pytest.mark.parametrize("tile", [None, (8, 8, 8), (4, 4, 4)])
@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
@pytest.mark.parametrize("case", ["rbc_nu16", "small_mixed"])
def test_carried_lists_give_the_first_call_grid(case, dtype, tile):
    sc = scenes.make_config(2) if case == "rbc_nu16" else scenes.small_mixed()
    tuning = None if tile is None else {"tile": list(tile)}
    say(f"[carried] {case} dtype {dtype} tile {tile}: {sc.n_nodes} nodes, {sc.total_cells} cells")
    rng = np.random.default_rng(5)
    F = rng.normal(size=(3, sc.n_nodes))
    if dtype == ifem.IFEM_F32:
        F = F.astype(np.float32).astype(np.float64)
    plan = ifem.Plan(sc, tuning=tuning)
    ref = {}
    for i, shift in enumerate(MOVES):
        got = _spread(plan, sc, dtype, shift, F)
        fresh = _spread(ifem.Plan(sc, tuning=tuning), sc, dtype, shift, F)
        assert np.array_equal(got, fresh, equal_nan=True), f"call {i} (shift {shift}) differs from a fresh plan's"
        if shift not in ref:
            xs = sc.x64 + np.asarray(shift)[:, None] if dtype == ifem.IFEM_F64 else \
                (sc.anchor + np.asarray(shift)[None, :])[sc.node_particle()].T + sc.x32.astype(np.float64)
            ref[shift] = oracle.spread(sc, F, x=xs)
        e = rel(got.astype(np.float64), ref[shift])
        say(f"  call {i} shift {shift}: rel {e:.2e}")
        assert e <= (F64_TOL if dtype == ifem.IFEM_F64 else F32_TRANSFER_TOL)
    assert plan.status()[3] == 0


# the 64-box workload (sparse tiles, lists of every length, boxes of different sizes) in the default
# launch shape: every call equals a fresh plan's first call bit for bit; that call is checked against
# the oracle at full size elsewhere
@pytest.mark.parametrize("dtype", [ifem.IFEM_F64, ifem.IFEM_F32])
def test_carried_lists_batched_boxes(dtype):
    sc = scenes.make_config(4)
    say(f"[carried] {sc.name} dtype {dtype}: {sc.n_nodes} nodes, {sc.total_cells} cells")
    F = np.random.default_rng(6).normal(size=(3, sc.n_nodes))
    if dtype == ifem.IFEM_F32:
        F = F.astype(np.float32).astype(np.float64)
    plan = ifem.Plan(sc)
    for i, shift in enumerate(MOVES[:5]):
        got = _spread(plan, sc, dtype, shift, F)
        fresh = _spread(ifem.Plan(sc), sc, dtype, shift, F)
        say(f"  call {i} shift {shift}: {int(np.count_nonzero(got))} non-zero values")
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, fresh), f"call {i} (shift {shift}) differs from a fresh plan's"
    assert plan.status()[3] == 0
