"""GPU node-face anti-sticking (Sec. III.B) against the oracle's brute-force search.

Both sides take the closest face as the one of least float64 distance (ties to the lower face id) and
move a node when that distance is below d_min.  They evaluate the closest point by different routines,
so where two faces lie at the same distance up to rounding (faces sharing the closest edge or vertex)
either may win, and a node within rounding of d_min may move on one side only.  The check is therefore
one of validity, with the rounding bound EPS of a float64 distance between points of magnitude |x|:
  * a node moved by one side only is within EPS of d_min (by the oracle's distance);
  * the face the GPU chose is, by the oracle's own distance, within EPS of the least distance;
  * the moved node is d_min from that face (the oracle measures it), to EPS in float64 and to the
    offset's rounding in float32;
  * where both sides chose the same face the moved positions agree to 1e-12 of the positions, float32
    offsets to one rounding; unmoved nodes are copied exactly;
  * where the oracle's closest face is unique (no other face of another particle within EPS of the
    least distance) and the least distance is not within EPS of d_min, the GPU chose that face.
Full-size workloads are checked on sampled particles together with every particle whose box can reach
them.
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
U64 = 2.0 ** -53


def eps_of(x):
    """Rounding bound of a float64 node-face distance among points of magnitude up to max|x|."""
    return 256 * U64 * (1.0 + np.abs(x).max())


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


def _validate(sc, d_min, got_w, got_abs, ref_x, ref_w, ref_d, nodes, off_scale, tag):
    """Validity of the GPU's anti-sticking on `nodes` of scene sc (face ids of sc): see the module
    docstring.  got_abs [3][n] absolute moved positions; off_scale [n] the magnitude of each node's
    stored value (0 in float64, |offset| in float32) for the float32 rounding of the result."""
    eps = eps_of(sc.x64)
    gw, rw = got_w[nodes], ref_w[nodes]
    mg, mo = gw >= 0, rw >= 0
    one = mg != mo
    assert np.all(np.abs(ref_d[nodes][one] - d_min) <= eps), f"{tag}: a node moved on one side only, far from d_min"
    k = nodes[mg]
    if k.size:
        dg = oracle.pair_distances(sc, k, gw[mg])
        assert np.all(dg <= ref_d[k] + eps), f"{tag}: the GPU's face is not the closest"
        assert np.all(dg < d_min + eps), f"{tag}: moved although the face is not within d_min"
        dm = oracle.pair_distances(sc, k, gw[mg], moved=got_abs)
        tol = eps + 4 * U32 * off_scale[k]
        assert np.all(np.abs(dm - d_min) <= tol), f"{tag}: moved node not at d_min from its face"
    same = nodes[mg & mo & (gw == rw)]
    assert np.all(np.abs(got_abs[:, same] - ref_x[:, same])
                  <= 1e-12 * (1.0 + np.abs(ref_x[:, same])) + U32 * off_scale[same]), f"{tag}: moved positions"
    stay = nodes[~mg]
    assert np.all(np.abs(got_abs[:, stay] - sc.x64[:, stay]) <= U32 * off_scale[stay]), f"{tag}: unmoved nodes"
    # unique winners must agree
    cand = nodes[mo & (np.abs(ref_d[nodes] - d_min) > eps)]
    uniq = cand[_n_near_faces(sc, cand, ref_d[cand] + eps) == 1]
    assert np.array_equal(got_w[uniq], ref_w[uniq]), f"{tag}: a unique closest face was not chosen"
    differ = int(np.count_nonzero(mg & mo & (gw != rw)) + np.count_nonzero(one))
    return differ


def _n_near_faces(sc, nodes, bound):
    """Per node: how many faces of other particles lie within bound[i] of it (oracle distances)."""
    if nodes.size == 0:
        return np.zeros(0, dtype=np.int64)
    part = sc.node_particle()
    fpart = part[sc.tri[0]] if sc.n_tris else np.zeros(0, np.int32)
    if sc.n_tets:
        _, bp = oracle.boundary_faces(sc)
        fpart = np.concatenate([fpart, bp])
    nf = fpart.size
    out = np.zeros(nodes.size, dtype=np.int64)
    for i, k in enumerate(nodes):
        faces = np.nonzero(fpart != part[k])[0].astype(np.int64)
        d = oracle.pair_distances(sc, np.full(faces.size, k, dtype=np.int32), faces)
        out[i] = np.count_nonzero(d <= bound[i])
    return out


def _check(sc, d_min, out, faces, ref, dtype):
    ref_x, ref_w, _, ref_d = ref
    got_w = faces.cpu().numpy()
    part = sc.node_particle()
    nodes = np.arange(sc.n_nodes)
    if dtype == ifem.IFEM_F64:
        got_abs = out.cpu().numpy()
        off_scale = np.zeros(sc.n_nodes)
    else:
        got = out.cpu().numpy().astype(np.float64)
        got_abs = got + sc.anchor[part].T
        off_scale = np.abs(got).max(axis=0)
    return _validate(sc, d_min, got_w, got_abs, ref_x, ref_w, ref_d, nodes, off_scale, "scene")


@pytest.mark.parametrize("name", list(CASES))
def test_antistick_matches_oracle(name):
    make, d_min = CASES[name]
    sc = make()
    d_min = d_min if d_min is not None else sc.boxes[0].h
    ref = oracle.antistick(sc, d_min, with_distance=True)
    moved = ref[2]
    say(f"[gpu] anti-sticking {name}: {sc.n_nodes} nodes, d_min {d_min}, oracle moved {moved}")
    assert moved > 0
    plan = ifem.Plan(sc)
    faces = torch.empty(sc.n_nodes, dtype=torch.int64, device="cuda")
    out = torch.empty((3, sc.n_nodes), dtype=torch.float64, device="cuda")
    plan.antistick(ifem.IFEM_F64, cu(sc.x64, torch.float64), None, out, d_min, faces)
    torch.cuda.synchronize()
    differ = _check(sc, d_min, out, faces, ref, ifem.IFEM_F64)
    say(f"    winners that differ from the oracle's (rounding ties): {differ}")
    first, first_w = out.cpu().numpy(), faces.cpu().numpy()
    plan.antistick(ifem.IFEM_F64, cu(sc.x64, torch.float64), None, out, d_min, faces)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), first)  # run to run
    assert np.array_equal(faces.cpu().numpy(), first_w)
    out32 = torch.empty((3, sc.n_nodes), dtype=torch.float32, device="cuda")
    plan.antistick(ifem.IFEM_F32, cu(sc.x32, torch.float32), cu(sc.anchor, torch.float64), out32, d_min, faces)
    torch.cuda.synchronize()
    # float32 offsets from float64 anchors give the same float64 positions: the same decisions
    assert np.array_equal(faces.cpu().numpy(), first_w)
    _check(sc, d_min, out32, faces, ref, ifem.IFEM_F32)
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
    bf_full = _bface_keys(sc) if sc.n_tets else {}
    for p in picks:
        group = _neighbours(sc, p, 3 * d_min, lohi)
        sub = scenes.subset(sc, group)
        ref_x, ref_w, _, ref_d = oracle.antistick(sub, d_min, with_distance=True)
        nodes = np.arange(sc.node_start[p], sc.node_start[p + 1])
        mine = np.arange(sub.node_start[0], sub.node_start[1])
        # the GPU's face ids (full scene) in the subset's numbering
        sub_w = np.full(sub.n_nodes, -1, dtype=np.int64)
        sub_w[mine] = _to_subset_faces(sc, sub, group, w[nodes], bf_full)
        got_abs = np.zeros((3, sub.n_nodes))
        got_abs[:, mine] = got[:, nodes] + sc.anchor[p][:, None]
        off_scale = np.zeros(sub.n_nodes)
        off_scale[mine] = np.abs(got[:, nodes]).max(axis=0)
        _validate(sub, d_min, sub_w, got_abs, ref_x, ref_w, ref_d, mine, off_scale, f"particle {p}")
    plan.close()


def _bface_keys(sc):
    """Boundary face id of the full scene by its sorted node triple."""
    bf, _ = oracle.boundary_faces(sc)
    return {tuple(sorted(bf[:, j])): sc.n_tris + j for j in range(bf.shape[1])}


def _to_subset_faces(sc, sub, group, faces, bf_full):
    """Face ids of the full scene -> ids of the subset made of particles `group` (in that order)."""
    tri_map, node_map = {}, {}
    t_off, n_off = 0, 0
    for q in group:
        for t in range(sc.tri_start[q], sc.tri_start[q + 1]):
            tri_map[t] = t_off + t - sc.tri_start[q]
        t_off += sc.tri_start[q + 1] - sc.tri_start[q]
        for k in range(sc.node_start[q], sc.node_start[q + 1]):
            node_map[k] = n_off + k - sc.node_start[q]
        n_off += sc.node_start[q + 1] - sc.node_start[q]
    inv_bf = {v: key for key, v in bf_full.items()}
    sub_bf = _bface_keys(sub) if sub.n_tets else {}
    out = np.full(faces.size, -1, dtype=np.int64)
    for i, f in enumerate(faces):
        if f < 0:
            continue
        if f < sc.n_tris:
            out[i] = tri_map[int(f)]
        else:
            key = tuple(sorted(node_map[v] for v in inv_bf[int(f)]))
            out[i] = sub_bf[key]
    return out
