"""The extended-precision element forces (tests/extended_elements.py) against the oracle.

Both evaluate the element forces of slightly compressible neo-Hookean tetrahedra (Sec. II.B) and of
neo-Hookean and Skalak membranes (Sec. II.A, elastic part), one in 80-bit and one in 64-bit
arithmetic.  On every solid tried the oracle stays within a tenth of the
forces' own conditioning (the change a one-ulp move of the positions produces) of the 80-bit result,
and to 2e-14 on a well-conditioned one; on a near-incompressible platelet under a small isochoric shear
(lambda / mu = 50, flattened reference tetrahedra) it is more than 1e-12 off, which bounds what any
float64 evaluation of those forces can reach.
"""
import numpy as np
import pytest

import extended_elements
import oracle
from paper_1807_08219_amd.inputs import scenes


def _platelet(gamma=0.01, ratio=scenes.SOLID_RATIO, dims=(5, 5, 5), seed=3):
    """One platelet-shaped solid (flattened ellipsoid of tetrahedra) under a simple shear gamma, with
    lambda / mu = ratio."""
    rng = np.random.default_rng(seed)
    X, tets = scenes.ellipsoid_template(dims)
    S = np.eye(3)
    S[0, 1] = gamma  # simple shear: isochoric, J = 1 up to rounding
    R = scenes.meshes.random_rotation(rng)
    x = (X - X.mean(axis=0)) @ (R @ S).T + np.array([4.0, 4.0, 4.0])
    box = scenes.Box((16, 16, 16), 0.5, (0.0, 0.0, 0.0))
    p = scenes.Particle(X=X, x=x, tet=tets, law=scenes.LAW_TET_NEOHOOKE, mu=scenes.PLT_MU,
                        mu2=ratio * scenes.PLT_MU)
    return scenes.assemble("platelet", [box], [p], seed)


def _one_ulp_change(sc, Fo, seed=0):
    """Relative change of the oracle's forces when every position coordinate moves by at most one unit
    in its last place: the forces' own conditioning."""
    rng = np.random.default_rng(seed)
    x = sc.x64 + np.spacing(np.abs(sc.x64)) * rng.integers(-1, 2, sc.x64.shape)
    Fp, _ = oracle.forces(scenes.Scene(**{**sc.__dict__, "x64": x}))
    return np.linalg.norm(Fp - Fo) / np.linalg.norm(Fo)


@pytest.mark.parametrize("ratio,gamma", [(1.0, 0.6), (1.0, 0.05), (50.0, 0.3), (50.0, 0.01)])
def test_oracle_is_within_a_tenth_of_its_conditioning_of_the_80_bit_forces(ratio, gamma):
    # the same formula evaluated in 80 and in 64 bits: the float64 result stays within a small part
    # of what a one-ulp move of the inputs changes (measured: a fiftieth), while a slip in the
    # formula (a dropped or scaled term) would be off by the order of the strain
    sc = _platelet(gamma=gamma, ratio=ratio)
    Fo, _ = oracle.forces(sc)
    e = extended_elements.rel_ld(Fo, extended_elements.particle_forces(sc, 0))
    one = _one_ulp_change(sc, Fo)
    assert e <= 0.1 * one, (e, one)
    if (ratio, gamma) == (1.0, 0.6):
        assert e <= 2e-14, e


def test_near_incompressible_platelet_cannot_meet_1e_12_in_float64():
    # lambda / mu = 50 and a shear of 0.01: the oracle itself is off the 80-bit forces by more than
    # 1e-12 relative, so no float64 evaluation can be held to 1e-12 there
    sc = _platelet(gamma=0.01, ratio=50.0)
    Fo, _ = oracle.forces(sc)
    e = extended_elements.rel_ld(Fo, extended_elements.particle_forces(sc, 0))
    assert e > 1e-12, e


@pytest.mark.parametrize("cfg", [1, 2])
def test_oracle_membranes_are_within_a_tenth_of_their_conditioning_of_the_80_bit_forces(cfg):
    # the noisy neo-Hookean capsule and the sheared Skalak red cell, elastic forces only
    sc = scenes.make_config(cfg)
    sc = scenes.Scene(**{**sc.__dict__, "kb": np.zeros_like(sc.kb)})
    Fo, _ = oracle.forces(sc)
    e = extended_elements.rel_ld(Fo, extended_elements.particle_membrane_forces(sc, 0))
    one = _one_ulp_change(sc, Fo)
    assert e <= 0.1 * one, (e, one)
