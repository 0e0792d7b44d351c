"""GPU node-face anti-sticking (Sec. III.B) against the oracle's brute-force search.

Both sides decide in the same precision (the closest face by float32 distance, then face id; a move
when that distance is below float32 d_min), from float64 distances; the winning face per node is
compared exactly, moved positions to float64 rounding (1e-12 of the positions), float32 offsets to
one rounding.  Full-size workloads are checked on sampled particles together with every particle
whose box can reach them.
"""
import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import meshes, scenes
from paper_1807_08219_amd.inputs.scenes import Box, Particle, assemble

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _spheres(gap, shift=(0.0, 0.0, 0.0), nu=6, noise=0.0, seed=0):
    rng = np.random.default_rng(seed)
    X, tris = meshes.icosphere(nu)
    box = Box((20, 16, 16), 0.5, (0.0, 0.0, 0.0))
    c1 = np.array([4.0, 4.0, 4.0])
    c2 = c1 + [2.0 + gap, 0.3, -0.2]
    x1 = X + c1 + noise * rng.normal(size=X.shape)
    x2 = X + c2 + np.array(shift) + noise * rng.normal(size=X.shape)
    return assemble("two_spheres", [box], [Particle(X=X, x=x1, tri=tris), Particle(X=X, x=x2, tri=tris)], seed)


def _sphere_and_cube():
    nodes, tets = meshes.kuhn_box(3, 3, 3)
    Xs, tris = meshes.icosphere(4)
    parts = [Particle(X=nodes, x=nodes + 5.0, tet=tets, law=scenes.LAW_TET_NEOHOOKE),
             Particle(X=Xs, x=0.6 * Xs + [6.0 + 0.2 + 0.6, 5.3, 4.6], tri=tris)]
    return assemble("cube_sphere", [Box((16, 16, 16), 0.75, (0, 0, 0))], parts)


def _squeezed_mixed():
    """The two-box mixed scene with every particle moved towards the first one."""
    sc = scenes.small_mixed()
    x = sc.x64.copy()
    part = sc.node_particle()
    c0 = x[:, part == 0].mean(axis=1)
    for p in range(1, sc.n_particles):
        if sc.box[p] != sc.box[0]:
            continue
        sel = part == p
        c = x[:, sel].mean(axis=1)
        x[:, sel] -= 0.35 * (c - c0)[:, None]
    X = sc.X_ref.T
    parts = []
    for p in range(sc.n_particles):
        s, e = sc.node_start[p], sc.node_start[p + 1]
        tri = sc.tri[:, sc.tri_start[p]:sc.tri_start[p + 1]].T - s if sc.tri_start[p + 1] > sc.tri_start[p] else None
        tet = sc.tet[:, sc.tet_start[p]:sc.tet_start[p + 1]].T - s if sc.tet_start[p + 1] > sc.tet_start[p] else None
        parts.append(Particle(X=X[s:e], x=x[:, s:e].T, tri=tri, tet=tet, law=int(sc.law[p]), mu=float(sc.mu[p]),
                              mu2=float(sc.mu2[p]), kb=float(sc.kb[p]), c0=float(sc.c0[p]), box=int(sc.box[p])))
    return assemble("squeezed_mixed", sc.boxes, parts, sc.seed)


CASES = {
    "spheres_gap_0.2": (lambda: _spheres(0.2), 0.5),
    "spheres_rough_overlap": (lambda: _spheres(-0.1, noise=0.02, seed=3), 0.5),
    "spheres_across_the_seam": (lambda: _spheres(0.15, shift=(-10.0, 8.0, 0.0)), 0.5),
    "sphere_and_solid_cube": (_sphere_and_cube, 0.75),
    "squeezed_mixed": (_squeezed_mixed, None),
    # d_min equal to the contact-cell width (1.0 here): grown boxes reach four cells per axis, so
    # faces take the slow list as well as the work list
    "spheres_d_min_at_cell_width": (lambda: _spheres(0.3, noise=0.01, seed=5), 1.0),
}


def _check(sc, d_min, plan, out, faces, ref_x, ref_w, dtype):
    got_w = faces.cpu().numpy()
    assert np.array_equal(got_w, ref_w)
    if dtype == ifem.IFEM_F64:
        got = out.cpu().numpy()
        assert np.all(np.abs(got - ref_x) <= 1e-12 * (1.0 + np.abs(ref_x)))
    else:
        off = ref_x - sc.anchor[sc.node_particle()].T
        got = out.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - off) <= U32 * np.abs(off) + 1e-12 * (1.0 + np.abs(ref_x)))


@pytest.mark.parametrize("name", list(CASES))
def test_antistick_matches_oracle(name):
    make, d_min = CASES[name]
    sc = make()
    d_min = d_min if d_min is not None else sc.boxes[0].h
    ref_x, ref_w, moved = oracle.antistick(sc, d_min)
    say(f"[gpu] anti-sticking {name}: {sc.n_nodes} nodes, d_min {d_min}, oracle moved {moved}")
    assert moved > 0
    plan = ifem.Plan(sc)
    faces = torch.empty(sc.n_nodes, dtype=torch.int64, device="cuda")
    out = torch.empty((3, sc.n_nodes), dtype=torch.float64, device="cuda")
    plan.antistick(ifem.IFEM_F64, cu(sc.x64, torch.float64), None, out, d_min, faces)
    torch.cuda.synchronize()
    _check(sc, d_min, plan, out, faces, ref_x, ref_w, ifem.IFEM_F64)
    first = out.cpu().numpy()
    plan.antistick(ifem.IFEM_F64, cu(sc.x64, torch.float64), None, out, d_min, faces)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), first)  # run to run
    out32 = torch.empty((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    plan.antistick(ifem.IFEM_F32, cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64), out32, d_min, faces)
    torch.cuda.synchronize()
    _check(sc, d_min, plan, out32, faces, ref_x, ref_w, ifem.IFEM_F32)
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()


def test_argument_errors():
    sc = _spheres(0.2)
    plan = ifem.Plan(sc)
    x = cu(sc.x64, torch.float64)
    out = torch.empty_like(x)
    for bad in (0.0, -1.0, float("nan"), 100.0):
        with pytest.raises(ifem.IfemError):
            plan.antistick(ifem.IFEM_F64, x, None, out, bad)
    with pytest.raises(ifem.IfemError):  # in place would let nodes see each other's moves
        plan.antistick(ifem.IFEM_F64, x, None, x, 0.5)
    plan.close()


def _boxes(sc):
    """Per-particle bounding boxes (lo, hi) [n_p][3] of the current positions."""
    starts = sc.node_start[:-1]
    return np.minimum.reduceat(sc.x64, starts, axis=1).T, np.maximum.reduceat(sc.x64, starts, axis=1).T


def _neighbours(sc, p, reach, lohi):
    """Particles of p's box whose bounding boxes, grown by reach, meet p's (periodic)."""
    lo, hi = lohi
    L = np.array(sc.boxes[sc.box[p]].length)
    out = [p]
    for q in range(sc.n_particles):
        if q == p or sc.box[q] != sc.box[p]:
            continue
        d = 0.5 * (lo[q] + hi[q]) - 0.5 * (lo[p] + hi[p])
        d -= L * np.round(d / L)
        if np.all(np.abs(d) <= 0.5 * (hi[q] - lo[q]) + 0.5 * (hi[p] - lo[p]) + reach):
            out.append(q)
    return out


@pytest.mark.parametrize("cfg", [3, 5])
def test_fullsize_sampled(cfg):
    sc = scenes.make_config(cfg)
    d_min = sc.boxes[0].h
    plan = ifem.Plan(sc)
    faces = torch.empty(sc.n_nodes, dtype=torch.int64, device="cuda")
    out = torch.empty((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    say(f"[gpu] anti-sticking config {cfg}: {sc.n_nodes} nodes, d_min {d_min}")
    plan.antistick(ifem.IFEM_F32, cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64), out, d_min, faces)
    torch.cuda.synchronize()
    w = faces.cpu().numpy()
    got = out.cpu().numpy().astype(np.float64)
    part = sc.node_particle()
    # float64 positions are anchor + offset exactly, so the float64 pass picks the same faces and moves
    # every node to the float32 result up to that result's rounding
    faces64 = torch.empty_like(faces)
    out64 = torch.empty((3, sc.n_nodes), dtype=torch.float64, device="cuda")
    plan.antistick(ifem.IFEM_F64, cu(sc.x64, torch.float64), None, out64, d_min, faces64)
    torch.cuda.synchronize()
    assert np.array_equal(faces64.cpu().numpy(), w)
    abs32 = got + sc.anchor[part].T
    o64 = out64.cpu().numpy()
    assert np.all(np.abs(o64 - abs32) <= U32 * np.abs(got) + 1e-12 * (1 + np.abs(o64)))
    moved_parts = np.unique(part[w >= 0])
    say(f"    moved nodes {(w >= 0).sum()} in {moved_parts.size} particles")
    rng = np.random.default_rng(cfg)
    picks = list(rng.choice(moved_parts, size=min(3, moved_parts.size), replace=False)) if moved_parts.size else []
    picks += list(rng.choice(sc.n_particles, size=2, replace=False))
    lohi = _boxes(sc)
    for p in picks:
        group = _neighbours(sc, p, 3 * d_min, lohi)
        sub = scenes.subset(sc, group)
        ref_x, ref_w, _ = oracle.antistick(sub, d_min)
        nodes = np.arange(sc.node_start[p], sc.node_start[p + 1])
        mine = np.arange(sub.node_start[0], sub.node_start[1])
        # face ids of the subset map back through the triangle offsets of the chosen particles
        fmap = np.concatenate([np.arange(sc.tri_start[q], sc.tri_start[q + 1]) for q in group]).astype(np.int64)
        rw = ref_w[mine]
        mapped = np.where(rw >= 0, fmap[np.clip(rw, 0, max(fmap.size - 1, 0))] if fmap.size else -1, -1)
        if sc.n_tets == 0 or np.all(rw < sub.n_tris):
            assert np.array_equal(w[nodes], mapped), f"particle {p}"
        off = ref_x[:, mine] - sc.anchor[p][:, None]
        assert np.all(np.abs(got[:, nodes] - off) <= U32 * np.abs(off) + 1e-12 * (1 + np.abs(ref_x[:, mine])))
    plan.close()
