"""Pins of the oracle's moving-least-squares transfer (Sec. II.C) against mathematics, not itself."""
import math

import numpy as np
import pytest

import oracle
from paper_1807_08219_amd.inputs import fields
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble


# ---------------------------------------------------------------- the weight W(r)
def test_weight_pieces_join_smoothly():
    # both pieces give 1/6 at r = 1/2, vanish at r = 1 and beyond
    assert oracle.weight(0.5) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert oracle.weight(0.5 + 1e-12) == pytest.approx(1.0 / 6.0, abs=1e-11)
    assert oracle.weight(1.0) == 0.0
    assert oracle.weight(1.3) == 0.0
    assert oracle.weight(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    # slope -1 from both sides at r = 1/2 and second derivative 4 from both sides
    e = 1e-5
    left = (oracle.weight(0.5) - oracle.weight(0.5 - e)) / e
    right = (oracle.weight(0.5 + e) - oracle.weight(0.5)) / e
    assert left == pytest.approx(-1.0, abs=1e-4) and right == pytest.approx(-1.0, abs=1e-4)
    d2l = (oracle.weight(0.5 - 2 * e) - 2 * oracle.weight(0.5 - e) + oracle.weight(0.5)) / e ** 2
    d2r = (oracle.weight(0.5) - 2 * oracle.weight(0.5 + e) + oracle.weight(0.5 + 2 * e)) / e ** 2
    assert d2l == pytest.approx(4.0, rel=1e-3) and d2r == pytest.approx(4.0, rel=1e-3)
    # C^2 at the edge of the support: value, slope and curvature all zero
    assert oracle.weight(1 - 1e-3) == pytest.approx(4 / 3 * 1e-9, rel=1e-9)


def test_weight_matches_printed_outer_piece():
    # the outer piece as printed, 4/3 - 4r + 4r^2 - 4/3 r^3, on (1/2, 1]
    for r in np.linspace(0.51, 1.0, 13):
        printed = 4 / 3 - 4 * r + 4 * r * r - 4 / 3 * r ** 3
        assert oracle.weight(r) == pytest.approx(printed, abs=2e-15)


# ---------------------------------------------------------------- the MLS weights
def _stencil_offsets(p, box, comp, base):
    s = fields.STAGGER[comp]
    out = np.zeros((27, 3))
    i = 0
    for mz in (-1, 0, 1):
        for my in (-1, 0, 1):
            for mx in (-1, 0, 1):
                node = np.array(box.origin) + (base + np.array([mx, my, mz]) + s) * box.h
                out[i] = node - p
                i += 1
    return out


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_mls_partition_of_unity_and_first_moments(comp):
    rng = np.random.default_rng(3 + comp)
    box = Box((16, 12, 20), 0.37, (1.1, -2.3, 0.4))
    for _ in range(200):
        p = np.array(box.origin) + rng.uniform(0, 1, 3) * np.array(box.length)
        base, phi = oracle.mls(p, box, comp)
        X = _stencil_offsets(p, box, comp, base)
        assert phi.sum() == pytest.approx(1.0, abs=1e-13)
        np.testing.assert_allclose(phi @ X, 0.0, atol=1e-13 * box.h)


def test_mls_nearest_node_is_base():
    rng = np.random.default_rng(9)
    box = Box((10, 10, 10), 0.5, (0.0, 0.0, 0.0))
    for comp in range(3):
        s = fields.STAGGER[comp]
        for _ in range(100):
            p = rng.uniform(1, 4, 3)
            base, _ = oracle.mls(p, box, comp)
            # the nearest node of lattice comp, by brute force over a neighbourhood
            cand = np.floor(p / box.h - s) + np.stack(np.meshgrid(*[[-1, 0, 1, 2]] * 3, indexing="ij"), -1).reshape(-1, 3)
            d = np.linalg.norm((cand + s) * box.h - p, axis=1)
            np.testing.assert_array_equal(base, cand[np.argmin(d)])


def test_mls_closed_form_at_a_node():
    # with x_k on a lattice node the first moments vanish by symmetry and
    # phi_J = W_J / sum W: centre, 6 faces, 12 edges, 8 corners at r = 0, 1/sqrt3, sqrt(2/3), 1
    w_face = 4 / 3 * (1 - 1 / math.sqrt(3)) ** 3
    w_edge = 4 / 3 * (1 - math.sqrt(2 / 3)) ** 3
    total = 2 / 3 + 6 * w_face + 12 * w_edge
    box = Box((8, 8, 8), 0.25, (0.0, 0.0, 0.0))
    for comp in range(3):
        s = fields.STAGGER[comp]
        p = (np.array([3, 4, 5]) + s) * box.h
        base, phi = oracle.mls(p, box, comp)
        np.testing.assert_array_equal(base, [3, 4, 5])
        m = np.array([[mx, my, mz] for mz in (-1, 0, 1) for my in (-1, 0, 1) for mx in (-1, 0, 1)])
        nnz = np.abs(m).sum(axis=1)
        expect = np.select([nnz == 0, nnz == 1, nnz == 2, nnz == 3], [2 / 3, w_face, w_edge, 0.0]) / total
        np.testing.assert_allclose(phi, expect, atol=1e-15)
    assert 2 / 3 / total == pytest.approx(0.486786163, abs=1e-9)
    assert w_face / total == pytest.approx(0.073503837, abs=1e-9)
    assert w_edge / total == pytest.approx(0.006015901, abs=1e-9)


def test_mls_equals_weighted_least_squares_in_absolute_coordinates():
    # The definition: Q_k = p(x_k)^T Z with Z minimising sum_J W_J (p(x_J)^T Z - q_J)^2,
    # p(X) = (1, X) in absolute coordinates.  Solve it with an orthogonal (lstsq) solver
    # for each unit data vector q = e_J, near the origin where the absolute basis is
    # well conditioned; phi_J is the resulting Q_k.
    rng = np.random.default_rng(21)
    box = Box((6, 6, 6), 0.3, (-0.9, -0.9, -0.9))
    for comp in range(3):
        for _ in range(20):
            p = rng.uniform(-0.3, 0.3, 3)
            base, phi = oracle.mls(p, box, comp)
            X = _stencil_offsets(p, box, comp, base)
            nodes = X + p
            W = np.array([oracle.weight(np.linalg.norm(d) / (math.sqrt(3) * box.h)) for d in X])
            P = np.hstack([np.ones((27, 1)), nodes])
            sw = np.sqrt(W)[:, None]
            phi_ls = np.zeros(27)
            for J in range(27):
                q = np.zeros(27)
                q[J] = 1.0
                Z, *_ = np.linalg.lstsq(sw * P, sw[:, 0] * q, rcond=None)
                phi_ls[J] = np.concatenate([[1.0], p]) @ Z
            np.testing.assert_allclose(phi, phi_ls, atol=1e-12)


# ---------------------------------------------------------------- spreading and interpolation
def _point_scene(pts, box):
    # a "particle" made of free points: transfers only need positions and the box
    n = pts.shape[0]
    p = Particle(X=pts.copy(), x=pts.copy())
    return assemble("points", [box], [p])


def test_spread_single_point_brute_force_with_periodic_wrap():
    box = Box((7, 9, 8), 0.4, (0.5, 0.0, -1.0))
    # a point next to the upper x face and the lower z face so that the stencil wraps
    p = np.array([[0.5 + 6.9 * 0.4, 1.7, -1.0 + 0.05]])
    sc = _point_scene(p, box)
    F = np.array([[1.5], [-2.0], [0.25]])
    grid = oracle.spread(sc, F, x=p.T.copy())
    expect = np.zeros_like(grid)
    for d in range(3):
        base, phi = oracle.mls(p[0], box, d)
        i = 0
        for mz in (-1, 0, 1):
            for my in (-1, 0, 1):
                for mx in (-1, 0, 1):
                    ii, jj, kk = (base + [mx, my, mz]) % np.array(box.n)
                    expect[d, (kk * box.n[1] + jj) * box.n[0] + ii] += phi[i] * F[d, 0]
                    i += 1
    np.testing.assert_allclose(grid, expect, atol=1e-15)
    np.testing.assert_allclose(grid.sum(axis=1), F[:, 0], rtol=1e-14)


def test_spread_preserves_total_force_and_is_adjoint_to_interp():
    rng = np.random.default_rng(4)
    box = Box((11, 13, 9), 0.3, (0.2, 0.1, -0.4))
    pts = np.array(box.origin) + rng.uniform(0, 1, (300, 3)) * np.array(box.length)
    sc = _point_scene(pts, box)
    x = pts.T.copy()
    F = rng.normal(size=(3, 300))
    u = rng.normal(size=(3, box.cells))
    G = oracle.spread(sc, F, x=x)
    v = oracle.interp(sc, u, x=x)
    np.testing.assert_allclose(G.sum(axis=1), F.sum(axis=1), rtol=1e-13, atol=1e-12)
    for d in range(3):
        lhs = G[d] @ u[d]
        rhs = F[d] @ v[d]
        assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-12)


def test_interp_reproduces_constant_and_linear_fields():
    rng = np.random.default_rng(8)
    box = Box((12, 12, 12), 0.25, (0.0, 0.0, 0.0))
    # keep points away from the periodic seam so the linear field is continuous on every stencil
    pts = 0.75 + rng.uniform(0, 1.5, (100, 3))
    sc = _point_scene(pts, box)
    a, b = 0.7, np.array([[0.3, -1.1, 2.0], [1.4, 0.2, -0.5], [-0.6, 0.9, 0.1]])
    grid = np.zeros((3, box.cells))
    for d in range(3):
        lp = fields.lattice_positions(box, d).reshape(-1, 3)
        grid[d] = a + lp @ b[d]
    v = oracle.interp(sc, grid, x=pts.T.copy())
    np.testing.assert_allclose(v, a + b @ pts.T, atol=1e-13)
    const = np.full((3, box.cells), -3.25)
    v = oracle.interp(sc, const, x=pts.T.copy())
    np.testing.assert_allclose(v, -3.25, atol=1e-14)
