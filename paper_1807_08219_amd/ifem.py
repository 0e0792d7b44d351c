"""Python binding of the C ABI in include/ifem.h (argument marshalling only).

Every step of the coupling path runs in the HIP kernels of ``libifem.so``;
this module only converts torch tensors to device pointers, torch streams to
``hipStream_t`` and return codes to exceptions.  It raises if the library is
missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libifem.so")

IFEM_OK = 0
IFEM_ERR_INVALID_ARG = -1
IFEM_ERR_UNSUPPORTED = -2
IFEM_ERR_DEVICE = -3
IFEM_ERR_DEGENERATE = -4
IFEM_ERR_NOMEM = -5
IFEM_F32 = 0
IFEM_F64 = 1
IFEM_SPREAD_TILED = 0
IFEM_SPREAD_ATOMIC = 1
IFEM_OPT_SPREAD_MODE = 1
IFEM_OPT_KERNEL_TIMING = 2
KERNEL_SLOTS = {0: "k_forces", 1: "k_bin_count", 2: "k_scan", 3: "k_bin_fill", 4: "k_spread_home",
                5: "k_spread_atomic", 6: "k_interp", 7: "k_fill", 8: "k_spread_merge", 9: "k_volume",
                10: "k_advance", 11: "k_interp_cells", 12: "k_fluid", 13: "k_contact"}

EXPORTED = [
    "ifem_plan_create", "ifem_plan_destroy", "ifem_plan_set", "ifem_plan_info", "ifem_element_forces",
    "ifem_plan_autotune", "ifem_spread", "ifem_spread_noalloc", "ifem_interp", "ifem_volume_correct", "ifem_advance", "ifem_interp_cells", "ifem_fluid_forces",
    "ifem_antistick", "ifem_plan_status", "ifem_plan_kernel_times", "ifem_last_error", "ifem_version",
]


class IfemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ifem error {code}: {msg}")
        self.code = code


class ifem_mesh_desc(C.Structure):
    _fields_ = [
        ("n_particles", C.c_int32), ("n_nodes", C.c_int32), ("n_tris", C.c_int32), ("n_tets", C.c_int32),
        ("tri", C.c_void_p), ("tet", C.c_void_p), ("node_start", C.c_void_p), ("tri_start", C.c_void_p),
        ("tet_start", C.c_void_p), ("law", C.c_void_p), ("mu", C.c_void_p), ("mu2", C.c_void_p),
        ("kb", C.c_void_p), ("c0", C.c_void_p), ("box", C.c_void_p), ("X_ref", C.c_void_p),
    ]


class ifem_box(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("origin", C.c_double * 3)]


class ifem_tuning(C.Structure):
    _fields_ = [("tile", C.c_int32 * 3), ("block_forces", C.c_int32), ("block_points", C.c_int32)]


_lib = None


def lib():
    """Load libifem.so (built in-tree by ``python -m paper_1807_08219_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first (python -m paper_1807_08219_amd.build)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.ifem_plan_create.argtypes = [C.POINTER(ifem_mesh_desc), C.POINTER(ifem_box), C.c_int32,
                                       C.POINTER(ifem_tuning), P, C.POINTER(P)]
        L.ifem_plan_destroy.argtypes = [P]
        L.ifem_plan_set.argtypes = [P, C.c_int32, C.c_int64]
        L.ifem_plan_info.argtypes = [P, C.POINTER(C.c_int64)]
        L.ifem_element_forces.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.ifem_spread.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.ifem_spread_noalloc.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.ifem_plan_autotune.argtypes = [P, C.c_int32, P, P, P, P, P, P, P, C.POINTER(ifem_tuning)]
        L.ifem_interp.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.ifem_volume_correct.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.ifem_advance.argtypes = [P, C.c_int32, P, P, P, C.c_double, P, P]
        L.ifem_interp_cells.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P]
        L.ifem_fluid_forces.argtypes = [P, C.c_int32, P, P, P, C.c_double, C.c_double, P, P]
        L.ifem_antistick.argtypes = [P, C.c_int32, P, P, C.c_double, P, P, P]
        L.ifem_plan_status.argtypes = [P, P, C.POINTER(C.c_int64), C.c_int32]
        L.ifem_plan_kernel_times.argtypes = [P, P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
        L.ifem_last_error.restype = C.c_char_p
        L.ifem_version.restype = C.c_int32
        for name in EXPORTED:
            if name not in ("ifem_last_error", "ifem_version"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def last_error() -> str:
    return lib().ifem_last_error().decode()


def _check(code):
    if code != IFEM_OK:
        raise IfemError(code, last_error())


def _ptr(t):
    """Device pointer of a CUDA tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _torch_dtype(dtype):
    """The element type of positions, forces, grids and velocities for an IFEM_* precision flag, or None
    for a flag the library does not know (the C ABI then rejects the call)."""
    import torch

    return {IFEM_F32: torch.float32, IFEM_F64: torch.float64}.get(int(dtype))


def _check_arg(t, name, dt, numel):
    """Check `t`'s element type and count against what the call reads or writes (the kernels trust
    both: a mismatch would access memory outside the tensor).  dt None skips the type check (an unknown
    precision flag, left to the C ABI)."""
    if t is None:
        return
    if dt is not None and t.dtype != dt:
        raise ValueError(f"{name}: expected {dt}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")


def _stream(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Plan:
    """A plan for one set of Lagrangian meshes and periodic boxes (ifem_plan_create)."""

    def __init__(self, scene, tuning=None, stream=None):
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a.ctypes.data_as(C.c_void_p) if a.size else None

        d = ifem_mesh_desc()
        d.n_particles, d.n_nodes, d.n_tris, d.n_tets = scene.n_particles, scene.n_nodes, scene.n_tris, scene.n_tets
        d.tri = arr(scene.tri, np.int32)
        d.tet = arr(scene.tet, np.int32)
        d.node_start = arr(scene.node_start, np.int32)
        d.tri_start = arr(scene.tri_start, np.int32)
        d.tet_start = arr(scene.tet_start, np.int32)
        d.law = arr(scene.law, np.int32)
        d.mu = arr(scene.mu, np.float64)
        d.mu2 = arr(scene.mu2, np.float64)
        d.kb = arr(scene.kb, np.float64)
        d.c0 = arr(scene.c0, np.float64)
        d.box = arr(scene.box, np.int32)
        d.X_ref = arr(scene.X_ref, np.float64)
        boxes = (ifem_box * len(scene.boxes))()
        for i, b in enumerate(scene.boxes):
            boxes[i].n[:] = [int(v) for v in b.n]
            boxes[i].h = float(b.h)
            boxes[i].origin[:] = [float(v) for v in b.origin]
        tp = None
        if tuning is not None:
            t = ifem_tuning()
            t.tile[:] = list(tuning.get("tile", (32, 16, 8)))
            t.block_forces = int(tuning.get("block_forces", 512))
            t.block_points = int(tuning.get("block_points", 256))
            tp = C.byref(t)
        h = C.c_void_p()
        _check(lib().ifem_plan_create(C.byref(d), boxes, len(scene.boxes), tp, _stream(stream), C.byref(h)))
        self.handle = h
        self.n_nodes = scene.n_nodes
        self.n_particles = scene.n_particles
        self.total_cells = scene.total_cells
        self._keep = []

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().ifem_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, option, value):
        _check(lib().ifem_plan_set(self.handle, int(option), int(value)))

    def info(self):
        out = (C.c_int64 * 10)()
        _check(lib().ifem_plan_info(self.handle, out))
        return list(out)

    def status(self, reset=True, stream=None):
        out = (C.c_int64 * 5)()
        _check(lib().ifem_plan_status(self.handle, _stream(stream), out, int(bool(reset))))
        return list(out)

    def kernel_times(self, reset=True, stream=None):
        """{kernel name: (total ms, launches)} recorded since the last reset (needs IFEM_OPT_KERNEL_TIMING)."""
        ms = (C.c_double * 16)()
        n = (C.c_int64 * 16)()
        _check(lib().ifem_plan_kernel_times(self.handle, _stream(stream), ms, n, int(bool(reset))))
        out = {KERNEL_SLOTS[i]: (ms[i], n[i]) for i in KERNEL_SLOTS if n[i]}
        if n[15]:
            out["dropped"] = (0.0, n[15])
        return out

    # --- argument checks: element types and counts from the plan (the C ABI checks pointers, aliasing
    # and values; it cannot see the size of a device allocation).  Every argument is checked before
    # any pointer is taken.  Kinds: "node" [ncomp][n_nodes] and "cell" [ncomp][total_cells] in the
    # call's precision, "particle" [n_particles][ncomp] float64, "face" [n_nodes] int64.
    def _pointers(self, dtype, *args):
        import torch

        for t, name, kind, ncomp in args:
            if kind == "node":
                _check_arg(t, name, _torch_dtype(dtype), ncomp * self.n_nodes)
            elif kind == "cell":
                _check_arg(t, name, _torch_dtype(dtype), ncomp * self.total_cells)
            elif kind == "particle":
                _check_arg(t, name, torch.float64, ncomp * self.n_particles)
            else:
                _check_arg(t, name, torch.int64, self.n_nodes)
        return [_ptr(a[0]) for a in args]

    # --- the three steps (device tensors in, device tensors out)
    def element_forces(self, dtype, x, anchor, f_out, red_out=None, stream=None):
        p = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3), (f_out, "f_out", "node", 3),
                           (red_out, "red_out", "particle", 5))
        _check(lib().ifem_element_forces(self.handle, dtype, *p, _stream(stream)))

    def spread(self, dtype, x, anchor, F, grid, stream=None):
        p = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3), (F, "F", "node", 3),
                           (grid, "grid", "cell", 3))
        _check(lib().ifem_spread(self.handle, dtype, *p, _stream(stream)))

    def autotune(self, dtype, x, anchor, F, grid, grid_u, v_out, stream=None):
        """Time the candidate launch shapes on these inputs, keep the fastest (ifem_plan_autotune) and
        return it as {"tile", "block_forces", "block_points"}."""
        p = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3), (F, "F", "node", 3),
                           (grid, "grid", "cell", 3), (grid_u, "grid_u", "cell", 3), (v_out, "v_out", "node", 3))
        t = ifem_tuning()
        _check(lib().ifem_plan_autotune(self.handle, dtype, *p, _stream(stream), C.byref(t)))
        return {"tile": [int(v) for v in t.tile], "block_forces": int(t.block_forces), "block_points": int(t.block_points)}

    def spread_noalloc(self, dtype, x, anchor, F, grid, stream=None):
        """ifem_spread (tiled) with its workspace in the library's static device array (allocates nothing)."""
        p = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3), (F, "F", "node", 3),
                           (grid, "grid", "cell", 3))
        _check(lib().ifem_spread_noalloc(self.handle, dtype, *p, _stream(stream)))

    def interp(self, dtype, x, anchor, grid_u, v_out, stream=None):
        p = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3),
                           (grid_u, "grid_u", "cell", 3), (v_out, "v_out", "node", 3))
        _check(lib().ifem_interp(self.handle, dtype, *p, _stream(stream)))

    def volume_correct(self, dtype, x, x_out, V0=None, lambda_out=None, stream=None):
        """Membrane volume correction; x_out may be x itself (in place)."""
        px, pv0, pxo, plam = self._pointers(dtype, (x, "x", "node", 3), (V0, "V0", "particle", 1),
                                            (x_out, "x_out", "node", 3), (lambda_out, "lambda_out", "particle", 1))
        _check(lib().ifem_volume_correct(self.handle, dtype, px, pv0, pxo, plam, _stream(stream)))

    def advance(self, dtype, x, v, x_out, v_prev=None, dt=1.0, stream=None):
        """Adams-Bashforth update x_out = x + dt (3/2 v - 1/2 v_prev) (forward Euler without v_prev)."""
        px, pv, pvp, pxo = self._pointers(dtype, (x, "x", "node", 3), (v, "v", "node", 3),
                                          (v_prev, "v_prev", "node", 3), (x_out, "x_out", "node", 3))
        _check(lib().ifem_advance(self.handle, dtype, px, pv, pvp, float(dt), pxo, _stream(stream)))

    def interp_cells(self, dtype, x, anchor, grid, out, stream=None):
        """Cell-centred fields grid [ncomp][total_cells] to the nodes, out [ncomp][n_nodes]."""
        ncomp = int(grid.shape[0]) if grid.dim() == 2 else 0
        if ncomp < 1:
            raise ValueError("grid: expected [ncomp][total_cells]")
        px, pa, pg, po = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3),
                                        (grid, "grid", "cell", ncomp), (out, "out", "node", ncomp))
        _check(lib().ifem_interp_cells(self.handle, dtype, px, pa, pg, ncomp, po, _stream(stream)))

    def fluid_forces(self, dtype, x, v, f_inout, C=None, eta=1.0, G=0.0, stream=None):
        """Add the Newtonian and polymer fluid-stress forces of every solid to f_inout."""
        px, pv, pc, pf = self._pointers(dtype, (x, "x", "node", 3), (v, "v", "node", 3), (C, "C", "node", 6),
                                        (f_inout, "f_inout", "node", 3))
        _check(lib().ifem_fluid_forces(self.handle, dtype, px, pv, pc, float(eta), float(G), pf, _stream(stream)))

    def antistick(self, dtype, x, anchor, x_out, d_min, face_out=None, stream=None):
        """Node-face anti-sticking: nodes closer than d_min to another particle's face move to d_min."""
        px, pa, pxo, pf = self._pointers(dtype, (x, "x", "node", 3), (anchor, "anchor", "particle", 3),
                                         (x_out, "x_out", "node", 3), (face_out, "face_out", "face", 1))
        _check(lib().ifem_antistick(self.handle, dtype, px, pa, float(d_min), pxo, pf, _stream(stream)))
