"""Element-by-element float32 bounds: every grid value, interpolated velocity and nodal force of
the float32 path is within C u32 of the magnitude that could produce it.

  spread  |G_J - G_J^o| <= C u32 sum_k |phi_Jk| |F_k|   (+ the fixed-point quantum)
  interp  |v_k - v_k^o| <= C u32 sum_J |phi_Jk| |u_J|
  forces  |F_k - F_k^o| <= C u32 sum_e |f_e,k|          (elastic only: each element's share)

with u32 = 2^-24; the oracle runs on the float32-rounded inputs, so only the arithmetic of the
float32 path is measured.  The magnitudes come from the oracle's own stencil weights and element
forces.  C is 256 for the transfers: a weight phi_m = W_m (c0 + c.xi_m) near the edge of the
support loses digits to the cancellation in c0 + c.xi_m (measured worst cases 56-61).  C is 512
for the forces: the neo-Hookean stress of a strongly distorted triangle (J^2 down to 0.1 in the
perturbed config 1 capsule) amplifies rounding by about 1 / J^2 (measured worst case 168).  A
wrong value, as opposed to a rounded one, is off by order one and fails both bars by far; a
normwise bar can hide a few such values among many right ones, these cannot.
"""
import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import fields, scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
C_TRANSFER = 256.0
C_FORCES = 512.0

SCENES = {
    "mixed_two_boxes": scenes.small_mixed,
    "config1_capsule_642": scenes.config1,
    "config2_rbc_2562": scenes.config2,
}


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def abs_stencil_sums(sc, F=None, u=None):
    """sum_k |phi||F_k| per grid value (F given) or sum_J |phi||u_J| per node (u given)."""
    bop = sc.box[sc.node_particle()]
    off = sc.cell_offset
    out = np.zeros((3, sc.total_cells)) if F is not None else np.zeros((3, sc.n_nodes))
    for k in range(sc.n_nodes):
        box = sc.boxes[bop[k]]
        n = np.array(box.n)
        for d in range(3):
            base, phi = oracle.mls(sc.x64[:, k], box, d)
            m = np.arange(27)
            ix = (base[0] + m % 3 - 1) % n[0]
            iy = (base[1] + (m // 3) % 3 - 1) % n[1]
            iz = (base[2] + m // 9 - 1) % n[2]
            cells = off[bop[k]] + (iz * n[1] + iy) * n[0] + ix
            if F is not None:
                np.add.at(out[d], cells, np.abs(phi) * abs(F[d, k]))
            else:
                out[d, k] = np.sum(np.abs(phi) * np.abs(u[d, cells]))
    return out


@pytest.mark.parametrize("name", list(SCENES))
def test_spread_and_interp_elementwise(name):
    sc = SCENES[name]()
    print(f"[gpu] elementwise float32 transfers {name}", flush=True)
    plan = ifem.Plan(sc)
    x, a = cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64)
    F = fields.random_forces(sc, seed=21).astype(np.float32).astype(np.float64)
    G = torch.empty((3, sc.total_cells), dtype=torch.float32, device="cuda")
    plan.spread(ifem.IFEM_F32, x, a, cu(F, torch.float32), G)
    got = G.cpu().numpy().astype(np.float64)
    ref = oracle.spread(sc, F)
    mag = abs_stencil_sums(sc, F=F)
    quantum = 1e-12 * np.abs(F).max()
    ratio = np.abs(got - ref) / (U32 * mag + quantum)
    print(f"    spread: max |err| / (u32 sum|phi||F|) = {ratio.max():.2f}", flush=True)
    assert ratio.max() <= C_TRANSFER

    u = fields.scene_velocity(sc).numpy().astype(np.float32).astype(np.float64)
    v = torch.empty((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    plan.interp(ifem.IFEM_F32, x, a, cu(u, torch.float32), v)
    got = v.cpu().numpy().astype(np.float64)
    ref = oracle.interp(sc, u)
    mag = abs_stencil_sums(sc, u=u)
    ratio = np.abs(got - ref) / (U32 * mag + 1e-300)
    print(f"    interp: max |err| / (u32 sum|phi||u|) = {ratio.max():.2f}", flush=True)
    assert ratio.max() <= C_TRANSFER
    plan.close()


@pytest.mark.parametrize("name", ["config1_capsule_642", "capsule_nh", "solid_and_capsule"])
def test_elastic_forces_elementwise(name):
    if name == "config1_capsule_642":
        sc = scenes.config1()
    elif name == "capsule_nh":
        sc = scenes.small_capsule(law=scenes.LAW_TRI_NEOHOOKE)
    else:
        sc = scenes.small_mixed()
        sc.kb = np.zeros_like(sc.kb)  # elastic forces only: bending is bounded separately
    print(f"[gpu] elementwise float32 forces {name}", flush=True)
    plan = ifem.Plan(sc)
    F = torch.empty((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    plan.element_forces(ifem.IFEM_F32, cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64), F, None)
    got = F.cpu().numpy().astype(np.float64)
    ref, cnt = oracle.forces(sc)
    assert cnt[0] == 0
    # sum over elements of |element force on the node|, from the oracle's element routines
    mag = np.zeros((3, sc.n_nodes))
    X, x = sc.X_ref.T, sc.x64.T
    for p in range(sc.n_particles):
        for e in range(sc.tri_start[p], sc.tri_start[p + 1]):
            ids = sc.tri[:, e]
            f, _ = oracle.membrane_element(X[ids], x[ids], sc.law[p], sc.mu[p], sc.mu2[p])
            mag[:, ids] += np.abs(f).T
        for e in range(sc.tet_start[p], sc.tet_start[p + 1]):
            ids = sc.tet[:, e]
            f, _ = oracle.tet_element(X[ids], x[ids], sc.mu[p], sc.mu2[p])
            mag[:, ids] += np.abs(f).T
    ratio = np.abs(got - ref) / (U32 * mag + 1e-300)
    print(f"    forces: max |err| / (u32 sum|f_e|) = {ratio.max():.2f}", flush=True)
    assert ratio.max() <= C_FORCES
    plan.close()


@pytest.mark.parametrize("shift", [0, 32])
def test_spread_scale_sees_every_lane(shift):
    # The fixed-point scale of a list comes from the largest force of each wavefront of 64 consecutive
    # nodes that feeds it.  One node per wavefront carries a force 10^6 times the others, at a lane
    # that moves from wavefront to wavefront (7 w + shift mod 64); a scale that missed that lane would
    # overflow the 64-bit sums of its cells and miss the bound below by orders of magnitude.
    sc = scenes.config2()
    print(f"[gpu] spread scale, one large force per wavefront (lane shift {shift})", flush=True)
    rng = np.random.default_rng(5 + shift)
    F = 1e-3 * rng.normal(size=(3, sc.n_nodes))
    waves = np.arange((sc.n_nodes + 63) // 64)
    big = np.minimum(waves * 64 + (7 * waves + shift) % 64, sc.n_nodes - 1)
    F[:, big] = 1e3 * rng.choice([-1.0, 1.0], size=(3, big.size))
    F = F.astype(np.float32).astype(np.float64)
    plan = ifem.Plan(sc)
    x, a = cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64)
    G = torch.empty((3, sc.total_cells), dtype=torch.float32, device="cuda")
    plan.spread(ifem.IFEM_F32, x, a, cu(F, torch.float32), G)
    got = G.cpu().numpy().astype(np.float64)
    ref = oracle.spread(sc, F)
    mag = abs_stencil_sums(sc, F=F)
    ratio = np.abs(got - ref) / (U32 * mag + 1e-12 * np.abs(F).max())
    print(f"    max |err| / (u32 sum|phi||F|) = {ratio.max():.2f}", flush=True)
    assert ratio.max() <= C_TRANSFER
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()
