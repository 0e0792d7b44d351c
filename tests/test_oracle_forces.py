"""Pins of the oracle's element forces (Sec. II.A-B) against closed forms, energy gradients and invariances."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble

NH, SK, TET = scenes.LAW_TRI_NEOHOOKE, scenes.LAW_TRI_SKALAK, scenes.LAW_TET_NEOHOOKE


# ---------------------------------------------------------------- membrane: closed forms
def _dW_dlambda_membrane(law, mu, mu2, l1, l2):
    """d W / d lambda_1 of the two membrane laws in principal stretches, differentiated by hand."""
    if law == NH:  # W = mu/2 (l1^2 + l2^2 + 1/(l1^2 l2^2) - 3)
        return mu * (l1 - 1.0 / (l1 ** 3 * l2 ** 2))
    a = l1 * l1 + l2 * l2 - 2.0  # Skalak, I1 - 2
    b = l1 * l1 * l2 * l2 - 1.0  # I2 - 1
    return mu * l1 * (a + 1.0 - l2 * l2) + 0.5 * mu2 * b * l1 * l2 * l2


@pytest.mark.parametrize("law,mu2", [(NH, 0.0), (SK, 100.0), (SK, 3.0)])
@pytest.mark.parametrize("l1,l2", [(1.2, 0.9), (0.8, 1.1), (1.0, 1.0), (1.5, 1.5)])
def test_membrane_principal_stretch_closed_form(law, mu2, l1, l2):
    # right triangle (0,0), (1,0), (0,1) stretched by diag(l1, l2): P^ = diag(dW/dl1, dW/dl2),
    # grad N1 = (1,0), grad N2 = (0,1), A0 = 1/2 -> f1 = -(1/2) dW/dl1 e_x, f2 = -(1/2) dW/dl2 e_y
    mu = 1.7
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    x = X * np.array([l1, l2, 1.0])
    f, stt = oracle.membrane_element(X, x, law, mu, mu2)
    assert stt == 0
    g1 = _dW_dlambda_membrane(law, mu, mu2, l1, l2)
    g2 = _dW_dlambda_membrane(law, mu, mu2, l2, l1)
    expect = np.array([[0.5 * g1, 0.5 * g2, 0], [-0.5 * g1, 0, 0], [0, -0.5 * g2, 0]])
    np.testing.assert_allclose(f, expect, atol=1e-13)


@pytest.mark.parametrize("law,mu2", [(NH, 0.0), (SK, 100.0)])
def test_membrane_uniform_dilation_virtual_work(law, mu2):
    # scaling a whole closed mesh by lam makes every element equibiaxial:
    # E(lam) = A0_tot W(lam, lam) and sum_k F_k . X_k = -dE/dlam
    X, tris = meshes.icosphere(6)
    X = X * 1.3
    lam, mu = 1.07, 0.8
    sc = assemble("s", [Box((4, 4, 4), 1.0, (0, 0, 0))], [Particle(X=X, x=lam * X, tri=tris, law=law, mu=mu, mu2=mu2)])
    F, cnt = oracle.forces(sc, x=(lam * X).T.copy(), bending=False)
    a = X[tris[:, 0]]
    A0 = 0.5 * np.linalg.norm(np.cross(X[tris[:, 1]] - a, X[tris[:, 2]] - a), axis=1).sum()
    if law == NH:
        dW = 0.5 * mu * (4 * lam - 4 * lam ** -5)
    else:
        I1b, I2b = 2 * lam ** 2 - 2, lam ** 4 - 1
        dW = 0.5 * mu * (I1b * 4 * lam + 4 * lam - 4 * lam ** 3) + mu2 / 4 * I2b * 4 * lam ** 3
    assert np.sum(F * X.T) == pytest.approx(-A0 * dW, rel=1e-12)


def _rand_tri(rng):
    X = rng.normal(size=(3, 3))
    x = X + 0.2 * rng.normal(size=(3, 3))
    return X, x


@pytest.mark.parametrize("law,mu2", [(NH, 0.0), (SK, 100.0)])
def test_membrane_force_is_minus_energy_gradient(law, mu2):
    rng = np.random.default_rng(5)
    for _ in range(20):
        X, x = _rand_tri(rng)
        f, stt = oracle.membrane_element(X, x, law, 1.3, mu2)
        assert stt == 0
        h = 1e-6
        g = np.zeros((3, 3))
        sc = assemble("s", [Box((4, 4, 4), 1.0, (0, 0, 0))],
                      [Particle(X=X, x=x, tri=np.array([[0, 1, 2]], np.int32), law=law, mu=1.3, mu2=mu2)])
        for k in range(3):
            for i in range(3):
                xp, xm = x.copy(), x.copy()
                xp[k, i] += h
                xm[k, i] -= h
                g[k, i] = (oracle.energy(sc, xp.T.copy())[0] - oracle.energy(sc, xm.T.copy())[0]) / (2 * h)
        np.testing.assert_allclose(f, -g, atol=1e-7 * max(1.0, np.abs(f).max()))


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 2 ** 31 - 1), law=st.sampled_from([NH, SK]))
def test_membrane_balance_and_rigid_invariance(seed, law):
    rng = np.random.default_rng(seed)
    X, x = _rand_tri(rng)
    f, stt = oracle.membrane_element(X, x, law, 1.0, 100.0 if law == SK else 0.0)
    if stt:
        return
    scale = np.abs(f).max() + 1e-300
    np.testing.assert_allclose(f.sum(axis=0), 0.0, atol=1e-13 * scale)
    torque = np.cross(x, f).sum(axis=0)
    np.testing.assert_allclose(torque, 0.0, atol=1e-12 * scale * np.abs(x).max())
    Q = meshes.random_rotation(rng)
    c = rng.normal(size=3) * 10
    f2, _ = oracle.membrane_element(X, x @ Q.T + c, law, 1.0, 100.0 if law == SK else 0.0)
    np.testing.assert_allclose(f2, f @ Q.T, atol=1e-12 * scale)
    # zero force in the reference configuration, moved rigidly
    mu2 = 100.0 if law == SK else 0.0
    f3, _ = oracle.membrane_element(X, X @ Q.T + c, law, 1.0, mu2)
    # rounding of positions ~|c| enters I2 - 1, amplified by mu_D
    np.testing.assert_allclose(f3, 0.0, atol=1e-14 * (1 + mu2) * (1 + np.abs(c).max()))


def test_membrane_collapsed_triangle_is_flagged():
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    x = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0]])
    f, stt = oracle.membrane_element(X, x, NH, 1.0, 0.0)
    assert stt == 1 and not f.any()


# ---------------------------------------------------------------- tetrahedra
def _dW_dlambda_solid(mu, lam, l):
    # W = lam/4 (J^2 - 1) - (lam/2 + mu) ln J + mu/2 (sum l^2 - 3), J = l1 l2 l3
    J = l[0] * l[1] * l[2]
    return np.array([0.5 * lam * (J * J - 1) / li + mu * (li - 1 / li) for li in l])


@pytest.mark.parametrize("l", [(1.1, 0.9, 1.05), (0.95, 0.95, 0.95), (1.3, 1.0, 0.8), (1, 1, 1)])
def test_tet_principal_stretch_closed_form(l):
    mu, lam = 2.0, 50.0 * 2.0
    X = np.vstack([np.zeros(3), np.eye(3)])
    x = X * np.array(l)
    f, stt = oracle.tet_element(X, x, mu, lam)
    assert stt == 0
    P = _dW_dlambda_solid(mu, lam, l)
    expect = np.vstack([P / 6.0, -np.diag(P) / 6.0])
    np.testing.assert_allclose(f, expect, atol=1e-12 * max(1, np.abs(P).max()))


def test_tet_uniform_dilation_virtual_work():
    nodes, tets = meshes.ellipsoid_tets(3, 3, 3, (1.0, 0.8, 0.6))
    lam, mu, lp = 1.04, 1.5, 75.0
    sc = assemble("t", [Box((4, 4, 4), 1.0, (0, 0, 0))],
                  [Particle(X=nodes, x=lam * nodes, tet=tets, law=TET, mu=mu, mu2=lp)])
    F, _ = oracle.forces(sc, x=(lam * nodes).T.copy())
    V0 = meshes.signed_tet_volumes(nodes, tets).sum()
    J = lam ** 3
    dW = lp / 4 * 6 * lam ** 5 - (lp / 2 + mu) * 3 / lam + mu / 2 * 6 * lam  # d/dlam of W(I1 = 3 lam^2, I3 = lam^6)
    assert np.sum(F * nodes.T) == pytest.approx(-V0 * dW, rel=1e-12)
    assert J > 1


def test_tet_force_is_minus_energy_gradient_and_balanced():
    rng = np.random.default_rng(12)
    for _ in range(20):
        X = np.vstack([np.zeros(3), np.eye(3)]) + 0.1 * rng.normal(size=(4, 3))
        x = X + 0.1 * rng.normal(size=(4, 3))
        mu, lam = 1.0, 50.0
        f, stt = oracle.tet_element(X, x, mu, lam)
        assert stt == 0
        sc = assemble("t", [Box((4, 4, 4), 1.0, (0, 0, 0))],
                      [Particle(X=X, x=x, tet=np.array([[0, 1, 2, 3]], np.int32), law=TET, mu=mu, mu2=lam)])
        h = 1e-6
        g = np.zeros((4, 3))
        for k in range(4):
            for i in range(3):
                xp, xm = x.copy(), x.copy()
                xp[k, i] += h
                xm[k, i] -= h
                g[k, i] = (oracle.energy(sc, xp.T.copy())[0] - oracle.energy(sc, xm.T.copy())[0]) / (2 * h)
        sc_ = np.abs(f).max()
        np.testing.assert_allclose(f, -g, atol=2e-7 * max(1, sc_))
        np.testing.assert_allclose(f.sum(0), 0, atol=1e-13 * sc_)
        np.testing.assert_allclose(np.cross(x, f).sum(0), 0, atol=1e-12 * sc_)
        Q = meshes.random_rotation(rng)
        f2, _ = oracle.tet_element(X, x @ Q.T + 5.0, mu, lam)
        np.testing.assert_allclose(f2, f @ Q.T, atol=1e-12 * sc_)


def test_inverted_tet_is_flagged():
    X = np.vstack([np.zeros(3), np.eye(3)])
    x = X.copy()
    x[3, 2] = -0.5
    f, stt = oracle.tet_element(X, x, 1.0, 50.0)
    assert stt == 1 and not f.any()


def test_zero_force_in_reference_configuration_whole_scenes():
    sc = scenes.small_mixed()
    Q = meshes.random_rotation(np.random.default_rng(1))
    x = (sc.X_ref.T @ Q.T + np.array([3.0, -2.0, 7.0])).T.copy()
    F, cnt = oracle.forces(sc, x=x, bending=False)
    assert cnt[0] == 0
    assert np.abs(F).max() < 1e-15 * (1 + sc.mu2.max()) * 10  # rounding amplified by the stiff moduli


# ---------------------------------------------------------------- bending
def _sphere_scene(nu, R=1.0, kb=1.0, c0=0.0):
    X, tris = meshes.icosphere(nu)
    sc = assemble("sph", [Box((4, 4, 4), 1.0, (0, 0, 0))],
                  [Particle(X=X * R, x=X * R, tri=tris, law=NH, mu=1.0, kb=kb, c0=c0)])
    sc.x64 = (X * R).T.copy()  # exact sphere, not the float32-offset split of the assembler
    return sc


@pytest.mark.parametrize("nu", [1, 4, 9])
def test_gauss_bonnet_and_area_partition(nu):
    sc = _sphere_scene(nu, R=1.7)
    A, kH, kG, nr = oracle.curvature(sc, 0)
    assert np.sum(kG * A) == pytest.approx(4 * math.pi, rel=1e-12)
    X = sc.x64.T
    t = sc.tri.T
    area = 0.5 * np.linalg.norm(np.cross(X[t[:, 1]] - X[t[:, 0]], X[t[:, 2]] - X[t[:, 0]]), axis=1).sum()
    assert A.sum() == pytest.approx(area, rel=1e-12)
    # outward unit normals
    np.testing.assert_allclose(np.linalg.norm(nr, axis=0), 1.0, atol=1e-14)
    assert np.all(np.einsum("ij,ij->j", nr, sc.x64) > 0)


def test_gauss_bonnet_on_red_cell():
    sc = scenes.config2()
    A, kH, kG, _ = oracle.curvature(sc, 0)
    assert np.sum(kG * A) == pytest.approx(4 * math.pi, rel=1e-12)


def test_icosahedron_closed_form_curvatures():
    # every vertex of the unit icosahedron: five equilateral faces, all angles 60 deg
    sc = _sphere_scene(1)
    A, kH, kG, nr = oracle.curvature(sc, 0)
    a = math.sqrt(2 - 2 / math.sqrt(5))  # edge length for circumradius 1
    Ak = 5 * (math.sqrt(3) / 4 * a * a) / 3  # Voronoi share of a non-obtuse equilateral face is 1/3
    np.testing.assert_allclose(A, Ak, rtol=1e-13)
    np.testing.assert_allclose(kG, (2 * math.pi - 5 * math.pi / 3) / Ak, rtol=1e-12)
    # K = (1/2A) sum_j 2 cot60 (x_k - x_j); neighbours sit at cos(angle) = 1/sqrt5 from x_k
    Kmag = (1 / (2 * Ak)) * (2 / math.sqrt(3)) * 5 * (1 - 1 / math.sqrt(5))
    np.testing.assert_allclose(kH, 0.5 * Kmag, rtol=1e-12)


def test_laplacian_of_height_on_sphere_converges():
    # z is an l = 1 spherical harmonic: Lap_s z = -2 z / R^2 on a sphere of radius R
    errs = []
    for nu in (8, 16):
        sc = _sphere_scene(nu, R=2.0)
        A, *_ = oracle.curvature(sc, 0)
        z = sc.x64[2]
        lap = oracle.laplacian(sc, 0, z, A)
        errs.append(np.abs(lap + 2 * z / 4.0).max())
    assert errs[1] < errs[0] / 3 and errs[1] < 5e-3


def test_sphere_bending_with_spontaneous_curvature():
    # E = 2 pi kb (2 + c0 R)^2 on a sphere -> sum_k F_k . n_k -> -dE/dR = -4 pi kb c0 (2 + c0 R)
    kb, c0, R = 0.7, 0.8, 1.5
    target = -4 * math.pi * kb * c0 * (2 + c0 * R)
    rel = []
    for nu in (8, 16):
        sc = _sphere_scene(nu, R=R, kb=kb, c0=c0)
        F, _ = oracle.forces(sc, elastic=False)
        n = sc.x64 / np.linalg.norm(sc.x64, axis=0)
        rel.append(abs(np.sum(F * n) - target) / abs(target))
    assert rel[0] < 0.02 and rel[1] < rel[0] / 3


def test_sphere_without_spontaneous_curvature_has_vanishing_bending_force():
    mags = []
    for nu in (8, 16):
        sc = _sphere_scene(nu, kb=1.0, c0=0.0)
        F, _ = oracle.forces(sc, elastic=False)
        A, *_ = oracle.curvature(sc, 0)
        mags.append(np.abs(F / A).max())  # force per area
    assert mags[1] < mags[0] / 2


def test_bending_restores_a_flattened_sphere():
    # a sphere squashed along z: bending pushes the flattened poles back out (F_z . z > 0 there)
    X, tris = meshes.icosphere(12)
    x = X * np.array([1.0, 1.0, 0.8])
    sc = assemble("s", [Box((4, 4, 4), 1.0, (0, 0, 0))], [Particle(X=X, x=x, tri=tris, law=NH, kb=1.0)])
    F, _ = oracle.forces(sc, x=x.T.copy(), elastic=False)
    poles = np.abs(x[:, 2]) > 0.78
    assert np.all(F[2, poles] * x[poles, 2] > 0)


def _spheroid_curvatures(a, c, th):
    """Mean and Gaussian curvature of the spheroid (a sin th cos ph, a sin th sin ph, c cos th) with
    outward normals (positive on a sphere), and the squared speed E = |dX/dth|^2 of its meridian."""
    E = a * a * np.cos(th) ** 2 + c * c * np.sin(th) ** 2
    k_meridian = a * c / E ** 1.5
    k_parallel = c / (a * np.sqrt(E))
    return 0.5 * (k_meridian + k_parallel), k_meridian * k_parallel, E


def _spheroid_energy(a, c, kb, c0, n=40001):
    """Helfrich energy 2 kb int (kH - kH0)^2 dA of the spheroid (kH0 = -c0/2), Simpson's rule in th."""
    th = np.linspace(0.0, math.pi, n)
    H, _, E = _spheroid_curvatures(a, c, th)
    f = (H + 0.5 * c0) ** 2 * a * np.sin(th) * np.sqrt(E)
    w = np.ones(n)
    w[1:-1:2], w[2:-1:2] = 4.0, 2.0
    return 2.0 * kb * 2.0 * math.pi * np.sum(w * f) * (th[1] - th[0]) / 3.0


@pytest.mark.parametrize("a,c,c0", [(1.0, 0.6, 0.0), (1.0, 1.5, 0.0), (1.0, 0.6, 0.8), (1.2, 1.0, -0.5)])
def test_spheroid_bending_virtual_work(a, c, c0):
    # The bending force is the restoring force of the Helfrich energy, so its virtual work along the
    # deformation that changes a spheroid's polar semi-axis c (velocity z/c e_z) or its equatorial
    # semi-axis a (velocity (x, y, 0)/a) converges to minus the derivative of the closed-form energy.
    # On spheroids the Laplacian term does not vanish: it carries most of this work (about 95 % of the
    # c-derivative of the oblate case), so a wrong factor or sign on it fails the pin, and the
    # curvature product term with kH0 != 0 is checked beside it.  Second order: the error falls by
    # about 4 per mesh refinement.
    kb, d = 0.7, 1e-5
    dE = {"c": (_spheroid_energy(a, c + d, kb, c0) - _spheroid_energy(a, c - d, kb, c0)) / (2 * d),
          "a": (_spheroid_energy(a + d, c, kb, c0) - _spheroid_energy(a - d, c, kb, c0)) / (2 * d)}
    rel = {"a": [], "c": []}
    for nu in (8, 16, 32):
        X, tris = meshes.icosphere(nu)
        x = X * np.array([a, a, c])
        sc = assemble("s", [Box((4, 4, 4), 1.0, (0, 0, 0))],
                      [Particle(X=x, x=x, tri=tris, law=NH, kb=kb, c0=c0)])
        F, _ = oracle.forces(sc, x=x.T.copy(), elastic=False)
        work_c = np.sum(F[2] * x[:, 2] / c)
        work_a = np.sum(F[0] * x[:, 0] / a + F[1] * x[:, 1] / a)
        rel["c"].append(abs(work_c + dE["c"]) / abs(dE["c"]))
        rel["a"].append(abs(work_a + dE["a"]) / abs(dE["a"]))
    for k in ("a", "c"):
        r = rel[k]
        assert r[0] < 0.05 and r[2] < 0.004, (k, r)
        assert r[1] < r[0] / 3.5 and r[2] < r[1] / 3.5, (k, r)


def test_bending_rigid_motion_invariance():
    sc = scenes.small_capsule(law=SK, kb=0.3, c0=0.2, nu=4)
    F, _ = oracle.forces(sc, elastic=False)
    Q = meshes.random_rotation(np.random.default_rng(2))
    x2 = (sc.x64.T @ Q.T + 4.0).T.copy()
    F2, _ = oracle.forces(sc, x=x2, elastic=False)
    np.testing.assert_allclose(F2, Q @ F, atol=1e-11 * np.abs(F).max())


# ---------------------------------------------------------------- reductions
def _cube_surface():
    v = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=float)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return v, meshes.orient_outward(v, np.array(t)).astype(np.int32)


def test_reductions_unit_cube_exact():
    v, t = _cube_surface()
    sc = assemble("c", [Box((4, 4, 4), 1.0, (0, 0, 0))], [Particle(X=v, x=v + 2.5, tri=t)])
    red = oracle.reduce(sc)[0]
    np.testing.assert_allclose(red, [1.0, 6.0, 3.0, 3.0, 3.0], atol=1e-14)
    nodes, tets = meshes.kuhn_box(3, 2, 4)
    sc = assemble("k", [Box((4, 4, 4), 1.0, (0, 0, 0))], [Particle(X=nodes, x=nodes + 1.0, tet=tets, law=TET)])
    red = oracle.reduce(sc)[0]
    np.testing.assert_allclose(red, [8.0, 0.0, 1.0, 1.0, 1.0], atol=1e-13)


def test_reductions_scaling_and_translation():
    sc = scenes.config2()
    red = oracle.reduce(sc)[0]
    lam, c = 1.3, np.array([-7.0, 2.0, 11.0])
    m = sc.x64.mean(axis=1, keepdims=True)
    x2 = (lam * (sc.x64 - m) + m + c[:, None]).copy()
    red2 = oracle.reduce(sc, x=x2)[0]
    assert red2[0] == pytest.approx(lam ** 3 * red[0], rel=1e-11)
    assert red2[1] == pytest.approx(lam ** 2 * red[1], rel=1e-12)
    np.testing.assert_allclose(red2[2:], lam * (red[2:] - m[:, 0]) + m[:, 0] + c, rtol=0, atol=1e-9)


def test_red_cell_volume_matches_effective_radius():
    # the paper's red-cell effective radius 2.82 um (Sec. IV.A, migration of a single RBC)
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rbc_effective_radius.json")))
    vols = []
    for nu in (8, 16, 32):
        X, tris = scenes.rbc_template(nu)
        sc = assemble("r", [Box((4, 4, 4), 1.0, (0, 0, 0))], [Particle(X=X, x=X, tri=tris, law=SK)])
        vols.append(oracle.reduce(sc)[0][0])
    r_eq = [(3 * V / (4 * math.pi)) ** (1 / 3) for V in vols]
    assert abs(r_eq[-1] - g["r_eff"]) < g["tolerance"]
    assert abs(vols[2] - vols[1]) < abs(vols[1] - vols[0]) / 2
