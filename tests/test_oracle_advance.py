"""Pins of the oracle's Adams-Bashforth position update (Sec. III.A, last step of the algorithm).

x^{n+1} = x^n + dt (3/2 v^n - 1/2 v^{n-1}), forward Euler when there is no previous velocity.
  * a rigid translation is advected exactly (dyadic data: every sum is exact);
  * on solid-body rotation, integrated with the analytic velocity at the current nodes, the error
    at a fixed time falls 4x when dt halves (second order), where forward Euler falls 2x;
  * a constant grid velocity interpolated by the MLS kernel (which reproduces constant fields) and
    fed to the update translates a whole scene to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_1807_08219_amd.inputs import scenes


def test_rigid_translation_is_exact():
    rng = np.random.default_rng(4)
    x = rng.integers(-4096, 4096, size=(3, 500)) * 2.0 ** -10
    v = np.array([0.75, -1.25, 0.5])[:, None] * np.ones((3, 500))
    dt = 2.0 ** -4
    cur = oracle.advance(x, v, None, dt)
    for n in range(2, 40):
        cur = oracle.advance(cur, v, v, dt)
        assert np.array_equal(cur, x + n * dt * v)


def _rotate_to(T, steps, ab2=True):
    """Integrate dx/dt = w x (x - c) to time T; return the max error against the exact rotation."""
    rng = np.random.default_rng(1)
    x0 = rng.normal(size=(3, 64))
    c = np.array([0.3, -0.2, 0.1])[:, None]
    w = np.array([0.2, 0.5, 1.0])
    vel = lambda x: np.cross(w, (x - c).T).T
    dt = T / steps
    x, vp = x0.copy(), None
    for _ in range(steps):
        v = vel(x)
        x = oracle.advance(x, v, vp if ab2 else None, dt)
        vp = v
    # exact solution: rotation about w by |w| T (Rodrigues)
    a = np.linalg.norm(w) * T
    k = w / np.linalg.norm(w)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + np.sin(a) * K + (1 - np.cos(a)) * K @ K
    return np.abs(x - (c + R @ (x0 - c))).max()


@pytest.mark.parametrize("steps", [100, 200])
def test_second_order_in_dt(steps):
    e1, e2 = _rotate_to(2.0, steps), _rotate_to(2.0, 2 * steps)
    assert 3.6 < e1 / e2 < 4.4
    f1, f2 = _rotate_to(2.0, steps, ab2=False), _rotate_to(2.0, 2 * steps, ab2=False)
    assert 1.8 < f1 / f2 < 2.2  # the pin tells first order from second


def test_constant_grid_velocity_translates_a_scene():
    sc = scenes.small_mixed()
    u_const = np.array([0.3, -0.7, 0.45])
    grid = np.repeat(u_const[:, None], sc.total_cells, axis=1)
    x, vp = sc.x64.copy(), None
    dt = 0.05
    for _ in range(10):
        v = oracle.interp(sc, grid, x=x)
        x = oracle.advance(x, v, vp, dt)
        vp = v
    np.testing.assert_allclose(x, sc.x64 + 10 * dt * u_const[:, None], rtol=0, atol=1e-12)
