"""Pins of the oracle's membrane volume correction (Sec. II.E, conservation of volume for membranes).

The correction moves node I by Lambda alpha_I, alpha_I = -(1/2) dV/dx_I, with Lambda the root of
the cubic V(x + Lambda alpha) = V0 of smallest magnitude.  The pins use only numpy's determinant
for the enclosed volume, so they do not retype the oracle's face sums:
  * V(x_out) = V0 to rounding;
  * alpha is -1/2 of the volume gradient, by finite differences (V is linear in each coordinate
    of one node, so a central difference is exact up to rounding);
  * Lambda is the smallest real root of the cubic V(x + L alpha) - V0, whose coefficients are
    fitted from four evaluations of V along alpha;
  * a regular icosahedron, rotated and moved, is scaled back about its centre: closed form;
  * no drift leaves the nodes in place up to rounding, solids are left alone.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble

SK, TET = scenes.LAW_TRI_SKALAK, scenes.LAW_TET_NEOHOOKE


def np_volume(x, tris):
    """Enclosed volume: sum of signed tetrahedra (origin, face) by numpy determinants; x [3][n]."""
    p = x.T[tris]  # [m][3 nodes][3]
    return np.linalg.det(p).sum() / 6.0


def _scene(X, x, tris, law=SK):
    return assemble("v", [Box((8, 8, 8), 1.0, (0, 0, 0))], [Particle(X=X, x=x, tri=tris, law=law, mu=1.0, mu2=1.0)])


def _drifted(nu=4, rel=2e-3, seed=3):
    """Red-cell mesh, rotated, moved and roughened, then swollen so that its volume drifts by about rel."""
    rng = np.random.default_rng(seed)
    X, tris = scenes.rbc_template(nu)
    Q = meshes.random_rotation(rng)
    x = X @ Q.T + [3.0, -2.0, 5.0]
    x = x + 0.02 * rng.normal(size=x.shape)
    c = x.mean(axis=0)
    x = c + (1.0 + rel / 3) * (x - c)
    return _scene(X, x, tris), tris


def test_corrected_volume_equals_target():
    sc, tris = _drifted()
    V0 = np_volume(sc.X_ref, tris)
    assert abs(np_volume(sc.x64, tris) / V0 - 1) > 1e-3
    out, lam, bad = oracle.volume_correct(sc)
    assert bad == 0
    assert np_volume(out, tris) == pytest.approx(V0, rel=1e-13)
    # an explicit target other than the reference volume
    out, lam, bad = oracle.volume_correct(sc, V0=np.array([0.97 * V0]))
    assert np_volume(out, tris) == pytest.approx(0.97 * V0, rel=1e-13)


def test_displacement_is_minus_half_the_volume_gradient():
    sc, tris = _drifted(nu=3)
    out, lam, _ = oracle.volume_correct(sc)
    alpha = (out - sc.x64) / lam[0]
    h = 1e-3
    grad = np.zeros_like(sc.x64)
    for d in range(3):
        for k in range(sc.n_nodes):
            xp, xm = sc.x64.copy(), sc.x64.copy()
            xp[d, k] += h
            xm[d, k] -= h
            grad[d, k] = (np_volume(xp, tris) - np_volume(xm, tris)) / (2 * h)
    np.testing.assert_allclose(alpha, -0.5 * grad, rtol=0, atol=1e-9 * np.abs(grad).max())


@pytest.mark.parametrize("rel", [1e-4, 2e-3, -5e-3, 0.05])
def test_lambda_is_the_smallest_real_root_of_the_cubic(rel):
    sc, tris = _drifted(nu=4, rel=rel)
    V0 = np_volume(sc.X_ref, tris)
    out, lam, bad = oracle.volume_correct(sc)
    assert bad == 0
    alpha = (out - sc.x64) / lam[0] if lam[0] != 0 else None
    # the cubic V(x + L alpha) - V0, from four exact evaluations along alpha
    s = abs(lam[0]) * 4 + 1e-3
    Ls = np.array([-2 * s, -s, s, 2 * s])
    vals = np.array([np_volume(sc.x64 + L * alpha, tris) - V0 for L in Ls])
    coef = np.linalg.solve(np.vander(Ls, 4), vals)  # [A, B, C, D]
    roots = np.roots(coef)
    real = roots[np.abs(roots.imag) <= 1e-12 * np.abs(roots).max()].real
    smallest = real[np.argmin(np.abs(real))]
    assert lam[0] == pytest.approx(smallest, rel=1e-9)
    assert np.all(np.abs(real) >= abs(lam[0]) * (1 - 1e-9))


def test_regular_icosahedron_closed_form():
    # a regular icosahedron of circumradius r has volume (5/12)(3 + sqrt 5) a^3 with edge
    # a = 4 r / sqrt(10 + 2 sqrt 5); by symmetry dV/dx_I = 3 V (x_I - c) / (12 r^2), so the
    # correction is a scaling about the centre c by s = (V0 / V)^(1/3), Lambda = 8 r^2 (1 - s) / V
    rng = np.random.default_rng(9)
    X, tris = meshes.icosphere(1)
    Q = meshes.random_rotation(rng)
    c = np.array([1.5, -4.0, 2.25])
    r0, r = 2.0, 1.7
    Xr = r0 * X @ Q.T + c
    x = r * X @ Q.T + c
    sc = _scene(Xr, x, tris)  # the scene's current positions are float32-rounded: pass the exact ones
    vol = lambda R: 5.0 / 12.0 * (3 + math.sqrt(5)) * (4 * R / math.sqrt(10 + 2 * math.sqrt(5))) ** 3
    out, lam, bad = oracle.volume_correct(sc, V0=np.array([vol(r0)]), x=np.ascontiguousarray(x.T))
    assert bad == 0
    V, V0 = vol(r), vol(r0)
    s = (V0 / V) ** (1 / 3)
    assert lam[0] == pytest.approx(8 * r * r * (1 - s) / V, rel=1e-13)
    np.testing.assert_allclose(out, Xr.T, rtol=0, atol=1e-13)


def test_no_drift_and_solids_untouched():
    sc, tris = _drifted()
    V = np_volume(sc.x64, tris)
    out, lam, _ = oracle.volume_correct(sc, V0=np.array([V]))
    # the target differs from the oracle's own face sum by rounding only: a rounding-sized move
    np.testing.assert_allclose(out, sc.x64, rtol=0, atol=1e-14 * np.abs(sc.x64).max())
    mixed = scenes.small_mixed()
    out, lam, bad = oracle.volume_correct(mixed)
    assert bad == 0
    npart = mixed.node_particle()
    for p in range(mixed.n_particles):
        sel = npart == p
        if mixed.law[p] == TET:
            assert lam[p] == 0.0 and np.array_equal(out[:, sel], mixed.x64[:, sel])
        else:
            t = mixed.tri[:, mixed.tri_start[p]:mixed.tri_start[p + 1]].T
            assert np_volume(out, t) == pytest.approx(np_volume(mixed.X_ref, t), rel=1e-13)


def test_correction_is_the_shortest_along_any_direction():
    # the cost function of Sec. II.E: among displacements mu w that restore V0 along random
    # directions w, none is shorter than Lambda alpha (to second order in the drift)
    sc, tris = _drifted(nu=4, rel=2e-3)
    V0 = np_volume(sc.X_ref, tris)
    out, lam, _ = oracle.volume_correct(sc)
    best = np.linalg.norm(out - sc.x64)
    rng = np.random.default_rng(17)
    alpha = (out - sc.x64) / lam[0]
    for trial in range(20):
        w = rng.normal(size=sc.x64.shape) + (3.0 if trial % 2 else 0.0) * alpha / np.abs(alpha).max()
        # V(x + mu w) - V0 is a cubic in mu: fit it from four evaluations, take the smallest root
        s = 1e-2 / np.abs(w).max()
        Ms = np.array([-2 * s, -s, s, 2 * s])
        vals = np.array([np_volume(sc.x64 + m * w, tris) - V0 for m in Ms])
        roots = np.roots(np.linalg.solve(np.vander(Ms, 4), vals))
        real = roots[np.abs(roots.imag) <= 1e-9 * np.abs(roots).max()].real
        mu = real[np.argmin(np.abs(real))]
        assert np.linalg.norm(mu * w) >= best * (1 - 1e-3)
