"""Pins of the oracle's node-face anti-sticking (Sec. III.B) and its geometric parts.

  * closest point on a triangle: never farther than any of 20,000 sampled points of the triangle,
    and no more than the sampling's resolution nearer; exact plane, edge and vertex cases;
  * boundary faces of a tetrahedral mesh: the count of a Kuhn box's surface triangles, and a closed,
    outward surface (its enclosed volume by numpy determinants equals the tetrahedra's);
  * two spheres closer than d_min: only nodes within d_min of the other sphere move, each to
    d_min from its winning face, after which no node is closer than d_min (convex obstacles);
    own faces never count; a particle moved by a whole box period gives the same result;
  * a membrane near a solid cube is pushed along the cube's face normal to d_min.
"""
import numpy as np
import pytest

import oracle
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble


def _tri_sample_min(p, a, b, c, n=200):
    u, v = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n))
    m = u + v <= 1
    pts = a + u[m, None] * (b - a) + v[m, None] * (c - a)
    return np.linalg.norm(pts - p, axis=1).min()


@pytest.mark.parametrize("seed", range(30))
def test_point_triangle_against_sampling(seed):
    rng = np.random.default_rng(seed)
    a, b, c = rng.normal(size=(3, 3))
    p = rng.normal(size=3) * rng.choice([0.3, 1.0, 3.0])
    q, _ = oracle.point_triangle(p, a, b, c)
    d = np.linalg.norm(q - p)
    ds = _tri_sample_min(p, a, b, c)
    h = max(np.linalg.norm(b - a), np.linalg.norm(c - a)) / 199 * 1.5
    assert d <= ds + 1e-12
    assert d >= ds - h
    # q lies on the triangle: non-negative barycentric coordinates summing to 1
    M = np.stack([b - a, c - a], axis=1)
    uv = np.linalg.lstsq(M, q - a, rcond=None)[0]
    assert uv.min() >= -1e-9 and uv.sum() <= 1 + 1e-9
    assert np.linalg.norm(M @ uv + a - q) <= 1e-9


def test_point_triangle_exact_regions():
    a, b, c = np.array([0.0, 0, 0]), np.array([2.0, 0, 0]), np.array([0.0, 2, 0])
    q, st = oracle.point_triangle(np.array([0.5, 0.5, 3.0]), a, b, c)
    assert st == 1 and np.allclose(q, [0.5, 0.5, 0.0], atol=1e-15)
    q, st = oracle.point_triangle(np.array([-1.0, -2.0, 0.5]), a, b, c)
    assert st == 0 and np.allclose(q, a, atol=1e-15)
    q, _ = oracle.point_triangle(np.array([1.0, -1.0, 0.0]), a, b, c)
    assert np.allclose(q, [1.0, 0.0, 0.0], atol=1e-15)
    q, _ = oracle.point_triangle(np.array([2.0, 2.0, 1.0]), a, b, c)
    assert np.allclose(q, [1.0, 1.0, 0.0], atol=1e-15)


def _volume(x, faces):
    p = x.T[faces.T]
    return np.linalg.det(p).sum() / 6.0


def test_boundary_faces_of_a_kuhn_box():
    nodes, tets = meshes.kuhn_box(2, 3, 4)
    sc = assemble("k", [Box((8, 8, 8), 1.0, (0, 0, 0))],
                  [Particle(X=nodes, x=nodes + 3.0, tet=tets, law=scenes.LAW_TET_NEOHOOKE)])
    faces, part = oracle.boundary_faces(sc)
    assert faces.shape[1] == 2 * 2 * (2 * 3 + 3 * 4 + 2 * 4)
    assert np.all(part == 0)
    assert _volume(sc.X_ref, faces) == pytest.approx(8.0, rel=1e-13)
    assert _volume(sc.x64, faces) == pytest.approx(8.0, rel=1e-12)  # translation keeps it closed
    # every edge of a closed oriented surface appears once in each direction
    e = np.concatenate([faces[[0, 1]].T, faces[[1, 2]].T, faces[[2, 0]].T])
    fw = {tuple(r) for r in e}
    assert len(fw) == e.shape[0] and all((j, i) in fw for i, j in fw)


def _two_spheres(gap, shift=(0.0, 0.0, 0.0), nu=6):
    X, tris = meshes.icosphere(nu)
    box = Box((20, 16, 16), 0.5, (0.0, 0.0, 0.0))
    c1 = np.array([4.0, 4.0, 4.0])
    c2 = c1 + [2.0 + gap, 0.3, -0.2]
    parts = [Particle(X=X, x=X + c1, tri=tris), Particle(X=X, x=X + c2 + np.array(shift), tri=tris)]
    return assemble("two", [box], parts)


def test_two_spheres_are_pushed_apart_to_d_min():
    d_min = 0.5
    sc = _two_spheres(0.2)
    out, win, moved = oracle.antistick(sc, d_min)
    assert moved > 0
    still = win < 0
    assert np.array_equal(out[:, still], sc.x64[:, still])
    faces = sc.tri
    part = sc.node_particle()
    # each moved node sits at d_min from its winning face, computed with numpy's own sampling
    for k in np.where(~still)[0][:40]:
        f = faces[:, win[k]]
        a, b, c = sc.x64[:, f[0]], sc.x64[:, f[1]], sc.x64[:, f[2]]
        ds = _tri_sample_min(out[:, k], a, b, c, n=120)
        assert ds == pytest.approx(d_min, abs=d_min * 2e-2)
        assert part[k] != (0 if win[k] < sc.tri_start[1] else 1)
    # afterwards nothing is closer than d_min (convex obstacles); a second pass moves nothing
    sc2 = scenes.Scene(**{**sc.__dict__, "x64": out})
    out2, win2, moved2 = oracle.antistick(sc2, d_min * (1 - 1e-9))
    assert moved2 == 0 and np.array_equal(out2, out)


def test_own_faces_never_count_and_far_pairs_do_not_move():
    X, tris = meshes.icosphere(4)
    sc = assemble("one", [Box((20, 16, 16), 0.5, (0, 0, 0))], [Particle(X=X, x=X * 0.3 + 4.0, tri=tris)])
    out, win, moved = oracle.antistick(sc, 1.0)  # every node is within d_min of its own faces
    assert moved == 0 and np.array_equal(out, sc.x64)
    sc = _two_spheres(1.5)
    out, win, moved = oracle.antistick(sc, 0.5)
    assert moved == 0


def test_periodic_image_gives_the_same_result():
    d_min = 0.5
    a = _two_spheres(0.1)
    b = _two_spheres(0.1, shift=(-10.0, 8.0, 0.0))  # the second sphere one period away in x and y
    oa, wa, ma = oracle.antistick(a, d_min)
    ob, wb, mb = oracle.antistick(b, d_min)
    assert ma == mb > 0 and np.array_equal(wa, wb)
    shift = np.zeros_like(oa)
    shift[:, a.node_start[1]:] = np.array([-10.0, 8.0, 0.0])[:, None]
    np.testing.assert_allclose(ob, oa + shift, rtol=0, atol=1e-12)


def test_membrane_near_a_solid_is_pushed_along_the_face_normal():
    nodes, tets = meshes.kuhn_box(2, 2, 2)  # the cube [-1, 1]^3
    Xs, tris = meshes.icosphere(3)
    c = np.array([5.0 + 1.0 + 0.3 + 0.25, 5.0, 5.0])  # sphere of radius 0.25, 0.3 from the face x = 1
    parts = [Particle(X=nodes, x=nodes + 5.0, tet=tets, law=scenes.LAW_TET_NEOHOOKE),
             Particle(X=Xs, x=0.25 * Xs + c, tri=tris)]
    sc = assemble("cube", [Box((16, 16, 16), 0.75, (0, 0, 0))], parts)
    d_min = 0.5
    out, win, moved = oracle.antistick(sc, d_min)
    m = np.where(win >= 0)[0]
    assert moved == m.size > 0
    owner = sc.node_particle()[m]
    assert np.all(win[m][owner == 1] >= sc.n_tris) and np.all(win[m][owner == 0] < sc.n_tris)
    # the cube's node at the centre of its x = 1 face moves away from the sphere, in -x
    c0 = m[owner == 0]
    assert c0.size == 1 and np.allclose(sc.x64[:, c0[0]], [6.0, 5.0, 5.0])
    assert out[0, c0[0]] < 6.0 and np.allclose(out[1:, c0[0]], [5.0, 5.0], atol=1e-12)
    # sphere nodes that face the cube's x = 1 face (closest point inside that face) end at x = 6 + d_min
    m = m[owner == 1]
    inner = m[(np.abs(sc.x64[1, m] - 5.0) < 0.9) & (np.abs(sc.x64[2, m] - 5.0) < 0.9)]
    assert inner.size > 0
    np.testing.assert_allclose(out[0, inner], 6.0 + d_min, rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[1:, inner], sc.x64[1:, inner], rtol=0, atol=1e-12)


def test_faces_half_a_box_away_are_not_torn_by_the_periodic_image():
    # the second sphere's centre half a box length away in x: per-corner wrapping would split faces
    # that straddle the half-box distance into two images and fake a near face; nothing is near
    d_min = 0.5
    sc = _two_spheres(3.0)  # centres 5.0 apart in x in a box 10 long
    assert np.isclose(sc.x64[0, sc.node_start[1]:].mean() - sc.x64[0, :sc.node_start[1]].mean(), 5.0, atol=0.05)
    out, win, moved = oracle.antistick(sc, d_min)
    assert moved == 0 and np.array_equal(out, sc.x64)
