"""Host-side bounds audit of the kernels that ran, in the float32 Lagrangian loop and the viscoelastic
terms, just before a host crash of an earlier counter run (see the design notes): the conformation
interpolation, the membrane volume correction and the position update.  Their index formulas are
evaluated on the host for every node of the full-size workloads (the 64-box batched one and the dense
4000-cell one) against the sizes of the buffers they address."""
import numpy as np
import pytest

from paper_1807_08219_amd.inputs import scenes

MAX_RING = 12  # a closed triangulated surface of these meshes has valence <= 7


@pytest.fixture(scope="module", params=[4, 5])
def scene(request):
    return scenes.make_config(request.param)


def _nearest_base(sc, stagger):
    """base = floor(t + 1/2), t = (p - origin)/h - s, wrapped into each box (per node, 3 axes)."""
    bop = sc.box[sc.node_particle()]
    base = np.empty((3, sc.n_nodes), dtype=np.int64)
    for b, B in enumerate(sc.boxes):
        sel = bop == b
        t = (sc.x64[:, sel] - np.array(B.origin)[:, None]) / B.h - np.array(stagger)[:, None]
        base[:, sel] = np.floor(t + 0.5).astype(np.int64) % np.array(B.n)[:, None]
    return base, bop


def test_cell_interpolation_indices(scene):
    # k_interp_cells: reads grid[f * total + cell_off + rows[r] + column] for f < ncomp, rows from the
    # wrapped y/z neighbours, columns base-1..base+1 off the seam (one 3-value load) or wrapped at it;
    # writes out[f * N + k]
    sc = scene
    ncomp = 6
    base, bop = _nearest_base(sc, (0.5, 0.5, 0.5))
    n = np.array([B.n for B in sc.boxes])[bop].T  # per node box size
    off = sc.cell_offset[bop]
    seam = (base[0] == 0) | (base[0] == n[0] - 1)
    lo_col = np.where(seam, 0, base[0] - 1)
    hi_col = np.where(seam, n[0] - 1, base[0] + 1)
    assert np.all(lo_col >= 0) and np.all(hi_col < n[0])
    wy = (base[1][None, :] + np.array([-1, 0, 1])[:, None]) % n[1]
    wz = (base[2][None, :] + np.array([-1, 0, 1])[:, None]) % n[2]
    rows_max = wz.max(axis=0) * n[0] * n[1] + wy.max(axis=0) * n[0]
    rows_min = wz.min(axis=0) * n[0] * n[1] + wy.min(axis=0) * n[0]
    assert np.all(rows_min + lo_col >= 0)
    inbox_max = rows_max + hi_col
    assert np.all(inbox_max < n[0] * n[1] * n[2])
    assert np.all(inbox_max < 2 ** 32)  # the kernel forms in-box offsets in 32 bits
    assert np.all((ncomp - 1) * sc.total_cells + off + inbox_max < ncomp * sc.total_cells)
    assert (ncomp - 1) * sc.n_nodes + sc.n_nodes - 1 < ncomp * sc.n_nodes


def test_position_update_indices(scene):
    # k_advance: n = 3 N values, 256 threads x 4 items per block, grid-stride; loads at min(i, n - 1),
    # stores only below n; the grid covers every value
    n = 3 * scene.n_nodes
    per_block = 256 * 4
    blocks = min((n + per_block - 1) // per_block, 1 << 20)
    i0 = np.arange(blocks * 256, dtype=np.int64)
    i0 = (i0 // 256) * per_block + i0 % 256
    covered = np.zeros(n, dtype=bool)
    stride = blocks * per_block
    start = i0
    while start.size:
        for q in range(4):
            i = start + q * 256
            assert np.all(np.minimum(i, n - 1) <= n - 1)
            covered[i[i < n]] = True
        start = start[start + stride < n] + stride
    assert covered.all()


def test_volume_correction_indices(scene):
    # k_volume (membranes): one workgroup per particle; one-ring neighbour ids are particle-local and
    # index both the positions (x + c N + n0) and the LDS alpha arrays [3][cap], cap = the largest
    # particle; the write-out touches n0 + i for i < nn
    sc = scene
    cap = int(np.diff(sc.node_start).max())
    assert 3 * cap * 8 + 1024 <= 160 * 1024  # alpha in LDS
    for p in range(0, sc.n_particles, max(1, sc.n_particles // 200)):
        t0, t1 = sc.tri_start[p], sc.tri_start[p + 1]
        if t1 == t0:
            continue
        n0, nn = sc.node_start[p], sc.node_start[p + 1] - sc.node_start[p]
        local = sc.tri[:, t0:t1] - n0
        assert local.min() >= 0 and local.max() < nn <= cap
        valence = np.bincount(local.ravel(), minlength=nn)
        assert valence.max() <= MAX_RING and valence.min() >= 3
        assert (2 * sc.n_nodes + n0 + nn - 1) < 3 * sc.n_nodes
