"""The C-ABI library loads, exports every declared entry point and rejects bad arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ifem.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ifem_status|const char\*|int32_t)\s+(ifem_[a-z_]+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = ifem.lib()
    decl = _declared()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(ifem.EXPORTED) == decl
    assert L.ifem_version() == 10400


def _declarations():
    """name -> list of parameter declarations, from include/ifem.h."""
    text = open(os.path.join(ROOT, "include", "ifem.h")).read()
    out = {}
    for m in re.finditer(r"^\s*(?:ifem_status|const char\*|int32_t)\s+(ifem_[a-z_]+)\s*\(([^)]*)\)", text, re.M):
        params = [q.strip() for q in m.group(2).replace("\n", " ").split(",") if q.strip()]
        out[m.group(1)] = [] if params == ["void"] else params
    return out


def test_binding_declares_every_argument_type():
    # ctypes passes an undeclared Python int as a 32-bit C int: a device pointer would be cut to its
    # low half, so every entry point with parameters must declare them, pointers as pointers
    L = ifem.lib()
    for name, params in _declarations().items():
        if not params:
            continue
        at = getattr(L, name).argtypes
        assert at is not None, name
        assert len(at) == len(params), name
        for decl, t in zip(params, at):
            # ifem_plan is a pointer to an opaque struct; an array parameter is a pointer
            if "*" in decl or "[" in decl or decl.startswith("ifem_plan "):
                assert t is C.c_void_p or issubclass(t, C._Pointer), (name, decl)
            elif decl.startswith("double"):
                assert t is C.c_double, (name, decl)
            else:
                assert t in (C.c_int32, C.c_int64), (name, decl)


def _desc(sc):
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.c_void_p) if a.size else None

    d = ifem.ifem_mesh_desc()
    d.n_particles, d.n_nodes, d.n_tris, d.n_tets = sc.n_particles, sc.n_nodes, sc.n_tris, sc.n_tets
    d.tri, d.tet = arr(sc.tri, np.int32), arr(sc.tet, np.int32)
    d.node_start, d.tri_start, d.tet_start = (arr(sc.node_start, np.int32), arr(sc.tri_start, np.int32),
                                              arr(sc.tet_start, np.int32))
    d.law, d.box = arr(sc.law, np.int32), arr(sc.box, np.int32)
    d.mu, d.mu2, d.kb, d.c0 = (arr(sc.mu, np.float64), arr(sc.mu2, np.float64), arr(sc.kb, np.float64),
                               arr(sc.c0, np.float64))
    d.X_ref = arr(sc.X_ref, np.float64)
    boxes = (ifem.ifem_box * len(sc.boxes))()
    for i, b in enumerate(sc.boxes):
        boxes[i].n[:] = list(b.n)
        boxes[i].h = b.h
        boxes[i].origin[:] = list(b.origin)
    return d, boxes, keep


def _create(d, boxes, nb=None, tuning=None):
    h = C.c_void_p()
    code = ifem.lib().ifem_plan_create(C.byref(d), boxes, len(boxes) if nb is None else nb, tuning, None, C.byref(h))
    return code, ifem.last_error()


@pytest.fixture
def mixed():
    return scenes.small_mixed()


def test_null_arguments_are_rejected():
    L = ifem.lib()
    h = C.c_void_p()
    assert L.ifem_plan_create(None, None, 0, None, None, C.byref(h)) == ifem.IFEM_ERR_INVALID_ARG
    assert "NULL" in ifem.last_error()
    assert L.ifem_plan_destroy(None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_element_forces(None, 0, None, None, None, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_spread(None, 1, None, None, None, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_interp(None, 1, None, None, None, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_volume_correct(None, 1, None, None, None, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_advance(None, 1, None, None, None, 1.0, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_interp_cells(None, 1, None, None, None, 6, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_fluid_forces(None, 1, None, None, None, 1.0, 0.0, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_antistick(None, 1, None, None, 1.0, None, None, None) == ifem.IFEM_ERR_INVALID_ARG
    assert L.ifem_plan_set(None, 1, 0) == ifem.IFEM_ERR_INVALID_ARG
    out = (C.c_int64 * 5)()
    assert L.ifem_plan_status(None, None, out, 0) == ifem.IFEM_ERR_INVALID_ARG


def test_bad_box_and_counts_are_rejected(mixed):
    d, boxes, keep = _desc(mixed)
    code, msg = _create(d, boxes, nb=0)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "box" in msg
    boxes[1].n[2] = 2
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "n < 3" in msg
    boxes[1].n[2] = 13
    boxes[0].h = -1.0
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "spacing" in msg


def test_inconsistent_mesh_is_rejected(mixed):
    sc = mixed
    ns = sc.node_start.copy()
    ns[-1] += 1
    sc2 = scenes.Scene(**{**sc.__dict__, "node_start": ns})
    d, boxes, keep = _desc(sc2)
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "totals" in msg
    law = sc.law.copy()
    law[2] = scenes.LAW_TRI_SKALAK  # a tetrahedral particle with a membrane law
    d, boxes, keep = _desc(scenes.Scene(**{**sc.__dict__, "law": law}))
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "membrane law with tetrahedra" in msg
    tri = sc.tri.copy()
    tri[0, 0] = sc.node_start[1]  # a triangle of particle 0 pointing into particle 1
    d, boxes, keep = _desc(scenes.Scene(**{**sc.__dict__, "tri": tri}))
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "another particle" in msg
    bx = sc.box.copy()
    bx[0] = 7
    d, boxes, keep = _desc(scenes.Scene(**{**sc.__dict__, "box": bx}))
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_INVALID_ARG and "box index" in msg


def test_open_bending_surface_is_unsupported():
    # a bending membrane with one triangle removed has an open one-ring
    sc = scenes.small_capsule(kb=0.1, nu=2)
    keep_t = np.arange(sc.n_tris) != 5
    tri = np.ascontiguousarray(sc.tri[:, keep_t])
    ts = np.array([0, tri.shape[1]], dtype=np.int32)
    sc2 = scenes.Scene(**{**sc.__dict__, "tri": tri, "tri_start": ts})
    d, boxes, keep = _desc(sc2)
    code, msg = _create(d, boxes)
    assert code == ifem.IFEM_ERR_UNSUPPORTED and ("one-ring" in msg or "closed" in msg)


def test_bad_tuning_is_rejected(mixed):
    d, boxes, keep = _desc(mixed)
    t = ifem.ifem_tuning()
    t.tile[:] = [2, 16, 16]
    t.block_forces, t.block_points = 256, 256
    code, msg = _create(d, boxes, tuning=C.byref(t))
    assert code == ifem.IFEM_ERR_INVALID_ARG and "tile" in msg
    t.tile[:] = [16, 16, 16]
    t.block_forces = 100
    code, msg = _create(d, boxes, tuning=C.byref(t))
    assert code == ifem.IFEM_ERR_INVALID_ARG and "block_forces" in msg


def test_binding_checks_element_types_and_counts():
    # the kernels trust the element type and size of every device array; the binding checks both
    # against the plan before the call (a stand-in plan: the checks run before anything is launched)
    torch = pytest.importorskip("torch")
    plan = ifem.Plan.__new__(ifem.Plan)
    plan.handle, plan.n_nodes, plan.n_particles, plan.total_cells = None, 10, 2, 64
    f64, f32 = torch.float64, torch.float32
    x64, x32 = torch.zeros((3, 10), dtype=f64), torch.zeros((3, 10), dtype=f32)
    g64 = torch.zeros((3, 64), dtype=f64)
    cases = [
        (lambda: plan.spread(ifem.IFEM_F64, x32, None, x64, g64), "x: expected torch.float64"),
        (lambda: plan.spread(ifem.IFEM_F32, x32, torch.zeros((2, 3), dtype=f64), x32, g64), "grid: expected torch.float32"),
        (lambda: plan.spread(ifem.IFEM_F64, x64, None, x64, torch.zeros((3, 63), dtype=f64)), "grid: expected 192"),
        (lambda: plan.interp(ifem.IFEM_F64, x64, None, g64, torch.zeros((3, 9), dtype=f64)), "v_out: expected 30"),
        (lambda: plan.element_forces(ifem.IFEM_F32, x32, torch.zeros((2, 2), dtype=f64), x32), "anchor: expected 6"),
        (lambda: plan.element_forces(ifem.IFEM_F64, x64, None, x64, torch.zeros((2, 5), dtype=f32)),
         "red_out: expected torch.float64"),
        (lambda: plan.volume_correct(ifem.IFEM_F64, x64, x64, lambda_out=torch.zeros(3, dtype=f64)),
         "lambda_out: expected 2"),
        (lambda: plan.advance(ifem.IFEM_F32, x32, x64, x32), "v: expected torch.float32"),
        (lambda: plan.interp_cells(ifem.IFEM_F64, x64, None, torch.zeros((6, 64), dtype=f64),
                                   torch.zeros((3, 10), dtype=f64)), "out: expected 60"),
        (lambda: plan.fluid_forces(ifem.IFEM_F64, x64, x64, x64, C=torch.zeros((6, 9), dtype=f64)), "C: expected 60"),
        (lambda: plan.antistick(ifem.IFEM_F64, x64, None, x64, 0.5, torch.zeros(10, dtype=torch.int32)),
         "face_out: expected torch.int64"),
    ]
    for call, msg in cases:
        with pytest.raises(ValueError, match=msg):
            call()
    # well-typed host tensors pass these checks and stop at the device check
    with pytest.raises(ValueError, match="device tensor"):
        plan.spread(ifem.IFEM_F64, x64, None, x64, g64)
