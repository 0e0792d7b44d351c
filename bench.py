"""Coupling-step throughput on one MI355X: Lagrangian nodes/s and % of HBM roofline.

One step = ifem_element_forces (elastic + bending + float64 reductions) +
ifem_spread + ifem_interp on the dense red-cell suspension (4000 Evans-Fung
cells, 2562 nodes each, 35% Ht, 512x256x256 staggered grid), inputs resident
in HBM.  Float32 path (compensated invariants, deterministic tiled spread),
with the plain float64 path (global atomic spread) timed on the same inputs,
and the FP64 CPU oracle timed on a bounded sample of the same workload.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lagrangian nodes/s per coupling step (FP32 vs FP64) + % HBM roofline"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Per-unit algorithmic figures (float32 path; float64 doubles the node and grid terms):
#   node 12 B per 3-vector access, cell 12 B per 3-component access,
#   triangle 44 B (12 B indices + 24 B float64 metric + 8 B area),
#   tetrahedron 96 B (16 B indices + 72 B inverse reference edge matrix + 8 B volume; the scope
#   table's 72 B counts a 48 B metric, which squares the condition number of flat tetrahedra), bending one-rings
#   +12 B per triangle (3 neighbour ids per triangle of a closed surface) and +4 B per node;
#   MLS weights + one transfer: 753 flops per (node, component)
#   [27 stencil nodes x 14 (distance, spline, moments) + 9 x 20 (moment sums)
#    + 60 (4x4 solve) + 27 x 5 (weight and multiply-add)].
MLS_FLOPS = 27 * 14 + 9 * 20 + 60 + 27 * 5
VALU_PEAK_TFLOPS = 157.3  # MI355X float32 vector peak (packed issue); 256 CU x 2.4 GHz x 256 flop/cycle
VALU_NONPACKED_TFLOPS = 78.6  # the same without packed float32 issue, which this build does not use
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X float64 vector peak


def algorithmic(sc, fp64: bool):
    """Algorithmic bytes and flops of each kernel of one step."""
    vec = 24 if fp64 else 12
    cells = sc.total_cells
    bend = sc.kb != 0
    tris_bend = int(np.diff(sc.tri_start)[bend].sum())
    nodes_bend = int(np.diff(sc.node_start)[bend].sum())
    transfer_flops = 3 * sc.n_nodes * MLS_FLOPS
    return {
        "k_forces": (sc.n_nodes * 2 * vec + sc.n_tris * 44 + sc.n_tets * 96 + tris_bend * 12 + nodes_bend * 4, None),
        "k_spread_home": (sc.n_nodes * 2 * vec + cells * vec, transfer_flops),
        "k_spread_atomic": (sc.n_nodes * 2 * vec + cells * vec, transfer_flops),
        "k_interp": (sc.n_nodes * 2 * vec + cells * vec, transfer_flops),
        "k_bin_count": (sc.n_nodes * vec, None),
        "k_bin_fill": (sc.n_nodes * vec + 3 * sc.n_nodes * 4, None),
    }


def volume_algorithmic(sc, fp64: bool):
    """Algorithmic bytes and float64 flops of one membrane volume correction (Sec. II.E).

    Bytes: positions read and written once (2 x 12 B per node in float32, 2 x 24 B in float64) and
    the connectivity once (12 B per triangle: its three corners, which are also the one-ring
    entries of the three nodes).  Flops, as the kernel evaluates the face sums node by node over
    one-rings (3 entries per triangle): per ring entry an edge vector (3), a cross product (9) and
    its sum (3) for alpha, a cross product of alpha values (9) and its sum (3) for beta: 27; per
    node alpha's scaling (3), |alpha|^2 and x.alpha (15), alpha.beta and x.beta (12) and the
    update x + L alpha (6): 36."""
    vec = 24 if fp64 else 12
    mem = sc.tri_start[1:] != sc.tri_start[:-1]
    nodes = int(np.diff(sc.node_start)[mem].sum())
    return sc.n_nodes * 2 * vec + sc.n_tris * 12, sc.n_tris * 3 * 27 + nodes * 36


def step_bytes(sc, fp64: bool):
    a = algorithmic(sc, fp64)
    return a["k_forces"][0] + a["k_spread_home"][0] + a["k_interp"][0]


def step_bytes_table(sc, fp64: bool):
    """The step's bytes by the per-unit table of the hot-path scope (node 72 B over the three calls, triangle
    44 B, tetrahedron 72 B, bending +24 B per triangle and +48 B per bending node, grid 12 + 12 B per cell;
    float64 doubles the node and grid terms).  The library keeps the bending intermediates in LDS and
    reads one-rings instead, so step_bytes counts 12 B per triangle and 4 B per node there."""
    vec = 2 if fp64 else 1
    bend = sc.kb != 0
    tris_bend = int(np.diff(sc.tri_start)[bend].sum())
    nodes_bend = int(np.diff(sc.node_start)[bend].sum())
    return (sc.n_nodes * 72 * vec + sc.n_tris * 44 + sc.n_tets * 72 + tris_bend * 24 + nodes_bend * 48 +
            sc.total_cells * 24 * vec)


# the sources the spread's accumulation kernel is built from: its counters go stale when one changes
TRAFFIC_SOURCES = ("ifem_transfer.hip", "ifem_device.hpp", "ifem_internal.hpp")


def source_digest():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1807_08219_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, tile):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if it is current
    (same kernel sources, same spread tile)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        block = text.split("```json")[1].split("```")[0]
        rec = json.loads(block)
    except (IndexError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None  # the kernel changed since the counters were taken
    if rec.get("spread_tile") != [int(v) for v in tile]:
        return None  # taken with another tile shape
    return rec.get("hbm_bytes_per_launch")


def _oracle_chunk_work(sc, u64, ids):
    """The oracle on the particles `ids` of sc: forces + bending + reductions, spread onto the full grid,
    interpolation; returns the nodes done."""
    import oracle
    from paper_1807_08219_amd.inputs import scenes

    sub = scenes.subset(sc, ids)
    F, _ = oracle.forces(sub)
    oracle.reduce(sub)
    oracle.spread(sub, F)
    oracle.interp(sub, u64)
    return sub.n_nodes


_POOL_STATE = {}


def _pool_worker(args):
    """One worker of the all-cores leg: chunks `chunks` of the shared scene until the budget is spent."""
    chunks, budget_s = args
    sc, u64 = _POOL_STATE["sc"], _POOL_STATE["u64"]
    t0 = time.perf_counter()
    done = 0
    for ids in chunks:
        if time.perf_counter() - t0 >= budget_s:
            break
        done += _oracle_chunk_work(sc, u64, ids)
    return done, time.perf_counter() - t0


def cpu_leg(config: int, budget_s: float, workers: int):
    """Both oracle baselines on the host (run in a child process, before or without any GPU use): the
    oracle single-threaded until ~budget_s of work, then `workers` processes, each the same oracle
    single-threaded on its own particles, for ~budget_s of wall time."""
    import multiprocessing as mp

    import oracle
    from paper_1807_08219_amd.inputs import fields, scenes

    oracle.build(force=False)
    sc = scenes.make_config(config)
    u64 = fields.scene_velocity(sc, dtype=__import__("torch").float64,
                                shear_rate=1.0 if config == 3 else 0.0).numpy()
    chunk = 25
    order = [np.arange(i, min(i + chunk, sc.n_particles)) for i in range(0, sc.n_particles, chunk)]
    done, t_total, n_chunks = 0, 0.0, 0
    while t_total < budget_s and n_chunks < len(order):
        t0 = time.perf_counter()
        done += _oracle_chunk_work(sc, u64, order[n_chunks])
        t_total += time.perf_counter() - t0
        n_chunks += 1
    single = {"value": done / t_total, "unit": "nodes/s", "cores": 1, "kind": "oracle",
              "sample": f"{sum(len(c) for c in order[:n_chunks])} of {sc.n_particles} particles ({done} nodes): "
                        f"forces+bending+reductions, spread onto the full grid, interpolation; {t_total:.1f} s "
                        f"single-threaded FP64"}
    # all cores: the chunks dealt round robin to the workers, each worker running the same oracle
    _POOL_STATE.update(sc=sc, u64=u64)
    per = [order[w::workers] for w in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_pool_worker, [(c, budget_s) for c in per])
    wall = time.perf_counter() - t0
    nodes = sum(r[0] for r in res)
    multi = {"value": nodes / wall, "unit": "nodes/s", "cores": workers, "kind": "oracle",
             "sample": f"{nodes} nodes in {wall:.1f} s wall: {workers} processes, each the single-threaded FP64 "
                       f"oracle on its own chunks of {chunk} particles (forces+bending+reductions, spread onto "
                       f"the full grid, interpolation) for ~{budget_s:.0f} s"}
    return {"single": single, "all_cores": multi, "host_cpu": host_cpu(), "host_threads": os.cpu_count()}


def cpu_baselines_in_child(config: int, budget_s: float):
    """Run cpu_leg in a child process (the oracle never runs in the GPU process) and return its JSON."""
    import subprocess

    workers = max(1, min(16, os.cpu_count() or 1))
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", "--config", str(config),
                          "--cpu-budget", str(budget_s), "--cpu-workers", str(workers)],
                         capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(f"cpu leg failed: {out.stderr[-2000:]}")
    return json.loads(out.stdout.strip().splitlines()[-1])


def host_cpu():
    """Model name of the host processor (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def bench_volume(plan, sc, steps, dev, stream):
    """Membrane volume correction (Sec. II.E) of positions whose volumes drifted by up to 0.1 %:
    float32 offsets and float64 positions, kernel time from the library's event timer."""
    import torch

    from paper_1807_08219_amd import ifem
    from paper_1807_08219_amd.inputs import scenes

    dr = scenes.with_volume_drift(sc, rel=1e-3, seed=5)
    res = {"workload": f"{sc.name}, membrane volumes drifted by U(-0.1 %, 0.1 %)"}
    for dt, key, xin in ((ifem.IFEM_F32, "f32", dr.x32), (ifem.IFEM_F64, "f64", dr.x64)):
        x = torch.as_tensor(xin, device=dev)
        xo = torch.empty_like(x)
        lam = torch.empty(sc.n_particles, dtype=torch.float64, device=dev)
        for _ in range(3):
            plan.volume_correct(dt, x, xo, lambda_out=lam)
        torch.cuda.synchronize()
        plan.set(ifem.IFEM_OPT_KERNEL_TIMING, steps + 8)
        plan.kernel_times(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.volume_correct(dt, x, xo, lambda_out=lam)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        kt = plan.kernel_times(reset=True)
        plan.set(ifem.IFEM_OPT_KERNEL_TIMING, 0)
        ms = kt["k_volume"][0] / kt["k_volume"][1]
        nbytes, flops = volume_algorithmic(sc, key == "f64")
        gbs, tfs = nbytes / (ms * 1e-3) / 1e9, flops / (ms * 1e-3) / 1e12
        res[key] = {"ms": round(ms, 4), "wall_ms": round(wall, 4), "value": round(sc.n_nodes / (ms * 1e-3), 1),
                    "unit": "nodes/s",
                    "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes),
                                 "fp64_tflops": round(tfs, 3), "fp64_frac": round(tfs / FP64_PEAK_TFLOPS, 4)},
                    "multiplier_range": [float(lam.min()), float(lam.max())]}
        log(f"volume correction {key}: {ms:.4f} ms ({gbs:.0f} GB/s algorithmic, {tfs:.2f} fp64 TFLOP/s)")
        del x, xo
    res["device_status"] = plan.status()
    return res


def bench_loop(plan, sc, steps, dev, anchor, u32):
    """The Lagrangian loop in float32: forces, spread, interpolation of the steady synthetic velocity,
    Adams-Bashforth update and volume correction, two steps captured as one HIP graph."""
    import torch

    from paper_1807_08219_amd import ifem

    x = torch.as_tensor(sc.x32, device=dev).clone()
    F = torch.empty_like(x)
    G = torch.empty((3, sc.total_cells), dtype=torch.float32, device=dev)
    vA, vB = torch.empty_like(x), torch.empty_like(x)
    dt = 0.05 * min(b.h for b in sc.boxes) / max(float(u32.abs().max()), 1e-30)  # 1/20 cell per step at most

    def step(v_new, v_old, stream=None):
        plan.element_forces(ifem.IFEM_F32, x, anchor, F, None, stream)
        plan.spread(ifem.IFEM_F32, x, anchor, F, G, stream)
        plan.interp(ifem.IFEM_F32, x, anchor, u32, v_new, stream)
        plan.advance(ifem.IFEM_F32, x, v_new, x, v_prev=v_old, dt=dt, stream=stream)
        plan.volume_correct(ifem.IFEM_F32, x, x, stream=stream)

    step(vA, None)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        step(vB, vA, side)
        step(vA, vB, side)
        with torch.cuda.graph(graph, stream=side):
            step(vB, vA, side)
            step(vA, vB, side)
    torch.cuda.current_stream().wait_stream(side)
    graph.replay()
    torch.cuda.synchronize()
    pairs = max(1, steps // 2)
    t0 = time.perf_counter()
    for _ in range(pairs):
        graph.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (2 * pairs)
    del graph
    # the update kernel alone (eager, event timer): float32 positions, two velocities
    plan.set(ifem.IFEM_OPT_KERNEL_TIMING, steps + 8)
    plan.kernel_times(reset=True)
    for _ in range(steps):
        plan.advance(ifem.IFEM_F32, x, vA, F, v_prev=vB, dt=dt)
    kt = plan.kernel_times(reset=True)
    plan.set(ifem.IFEM_OPT_KERNEL_TIMING, 0)
    ms_adv = kt["k_advance"][0] / kt["k_advance"][1]
    nbytes = 4 * 12 * sc.n_nodes
    gbs = nbytes / (ms_adv * 1e-3) / 1e9
    log(f"Lagrangian loop (graph, float32): {ms:.3f} ms/step; advance kernel {ms_adv:.4f} ms ({gbs:.0f} GB/s)")
    st = plan.status()
    return {"ms_per_step": round(ms, 4), "value": round(sc.n_nodes / (ms * 1e-3), 1), "unit": "nodes/s",
            "steps": 2 * pairs, "dt": dt,
            "step": "forces + spread + interp + Adams-Bashforth update + volume correction (float32, one graph)",
            "advance": {"ms": round(ms_adv, 4), "roofline": {"bound": "hbm", "achieved": round(gbs, 2),
                                                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                            "frac": round(gbs / HBM_PEAK_GBS, 4),
                                                            "algorithmic_bytes": nbytes}},
            "device_status": st}


def _kernel_ms(plan, slot, fn, steps):
    from paper_1807_08219_amd import ifem

    fn()
    plan.set(ifem.IFEM_OPT_KERNEL_TIMING, steps + 8)
    plan.kernel_times(reset=True)
    for _ in range(steps):
        fn()
    kt = plan.kernel_times(reset=True)
    plan.set(ifem.IFEM_OPT_KERNEL_TIMING, 0)
    return kt[slot][0] / kt[slot][1]


def bench_viscoelastic(plan, sc, steps, dev, x32, anchor):
    """Conformation interpolation (six cell-centred fields to every node) on the main workload, and
    the fluid-stress forces of the solids of the 64-box workload (config 4), float32."""
    import torch

    from paper_1807_08219_amd import ifem
    from paper_1807_08219_amd.inputs import fields, scenes

    res = {}
    Cg = fields.conformation_field(sc, dtype=torch.float32).to(dev)
    Cn = torch.empty((6, sc.n_nodes), dtype=torch.float32, device=dev)
    ms = _kernel_ms(plan, "k_interp_cells", lambda: plan.interp_cells(ifem.IFEM_F32, x32, anchor, Cg, Cn), steps)
    nbytes = sc.n_nodes * (12 + 24) + sc.total_cells * 24
    flops = sc.n_nodes * (27 * 14 + 9 * 20 + 60 + 27 * 4 + 6 * 27 * 2)
    gbs, tfs = nbytes / (ms * 1e-3) / 1e9, flops / (ms * 1e-3) / 1e12
    log(f"conformation interpolation: {ms:.4f} ms ({gbs:.0f} GB/s algorithmic, {tfs:.1f} TFLOP/s)")
    res["interp_cells"] = {
        "workload": f"{sc.name}, 6 conformation components at the cell centres", "ms": round(ms, 4),
        "value": round(sc.n_nodes / (ms * 1e-3), 1), "unit": "nodes/s",
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes),
                     "tflops": round(tfs, 2), "alu_frac_nonpacked": round(tfs / VALU_NONPACKED_TFLOPS, 4)}}
    del Cg, Cn
    s4 = scenes.make_config(4)
    p4 = ifem.Plan(s4)
    x4, a4 = torch.as_tensor(s4.x32, device=dev), torch.as_tensor(s4.anchor, device=dev)
    C4 = torch.empty((6, s4.n_nodes), dtype=torch.float32, device=dev)
    p4.interp_cells(ifem.IFEM_F32, x4, a4, fields.conformation_field(s4, dtype=torch.float32).to(dev), C4)
    v4 = torch.randn((3, s4.n_nodes), dtype=torch.float32, device=dev)
    f4 = torch.zeros((3, s4.n_nodes), dtype=torch.float32, device=dev)
    ms = _kernel_ms(p4, "k_fluid", lambda: p4.fluid_forces(ifem.IFEM_F32, x4, v4, f4, C=C4, eta=1.0, G=0.5), steps)
    solid = s4.law == scenes.LAW_TET_NEOHOOKE
    sn = int(np.diff(s4.node_start)[solid].sum())
    nbytes = s4.n_tets * 16 + sn * (12 + 12 + 24 + 24)
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"fluid-stress forces: {ms:.4f} ms for {s4.n_tets} tets ({gbs:.0f} GB/s algorithmic)")
    res["fluid_forces"] = {
        "workload": f"{s4.name}: {int(solid.sum())} solids, {s4.n_tets} tetrahedra, {sn} nodes", "ms": round(ms, 4),
        "value": round(s4.n_tets / (ms * 1e-3), 1), "unit": "tets/s",
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes)}}
    res["device_status"] = p4.status()
    p4.close()
    return res


def bench_antistick(plan, sc, steps, dev, x32, anchor):
    """Node-face anti-sticking (Sec. III.B) on the main workload with d_min = h, float32 offsets."""
    import torch

    from paper_1807_08219_amd import ifem

    d_min = min(b.h for b in sc.boxes)
    out = torch.empty_like(x32)
    faces = torch.empty(sc.n_nodes, dtype=torch.int64, device=dev)
    ms = _kernel_ms(plan, "k_contact", lambda: plan.antistick(ifem.IFEM_F32, x32, anchor, out, d_min, faces), steps)
    moved = int((faces >= 0).sum())
    nf = sc.n_tris + 4 * sc.n_tets  # upper bound on the solids' boundary faces
    nbytes = sc.n_nodes * (12 + 12) + nf * 12
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"anti-sticking: {ms:.4f} ms, {moved} nodes moved ({gbs:.0f} GB/s algorithmic)")
    return {"workload": f"{sc.name}, d_min = h", "ms": round(ms, 4), "value": round(sc.n_nodes / (ms * 1e-3), 1),
            "unit": "nodes/s", "moved_nodes": moved,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes)},
            "device_status": plan.status()}


def _cells_near(sc, rng, n):
    """n sampled (component, cell) grid values -- each on a lattice cell next to a random node -- and every
    node that can reach them (nodes hashed by the cell holding them, gathered from the 6^3 cells around
    each sampled cell, a superset of the contributors)."""
    off = sc.cell_offset
    bop = sc.box[sc.node_particle()]
    keys = np.empty(sc.n_nodes, dtype=np.int64)
    for b, B in enumerate(sc.boxes):
        sel = bop == b
        u = np.floor((sc.x64[:, sel].T - np.array(B.origin)) / B.h).astype(np.int64) % np.array(B.n)
        keys[sel] = off[b] + (u[:, 2] * B.n[1] + u[:, 1]) * B.n[0] + u[:, 0]
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    idx, near = [], []
    for _ in range(n):
        k = int(rng.integers(0, sc.n_nodes))
        b = int(bop[k])
        B = sc.boxes[b]
        ijk = (np.floor((sc.x64[:, k] - np.array(B.origin)) / B.h).astype(np.int64) + rng.integers(-1, 2, 3)) % np.array(B.n)
        idx.append((int(rng.integers(0, 3)), off[b] + (ijk[2] * B.n[1] + ijk[1]) * B.n[0] + ijk[0]))
        for dz in range(-3, 3):
            for dy in range(-3, 3):
                for dx in range(-3, 3):
                    c = (ijk + np.array([dx, dy, dz])) % np.array(B.n)
                    key = off[b] + (c[2] * B.n[1] + c[1]) * B.n[0] + c[0]
                    lo, hi = np.searchsorted(skeys, key), np.searchsorted(skeys, key, side="right")
                    if hi > lo:
                        near.append(order[lo:hi])
    return idx, np.unique(np.concatenate(near)), bop


# the bars the parity tests hold each result to (u32 = 2^-24); the float32 element-wise constants are
# the measured worst cases with a margin: a weight near the edge of the stencil's support loses digits
# to the cancellation in c0 + c.xi (56-61 u32 measured), a strongly distorted neo-Hookean triangle
# amplifies rounding by about 1/J^2 (168 u32 measured)
BARS_F64 = "1e-12 normwise per result; grid values element by element within 1e-12 sum|phi||F| (+ the fixed-point quantum)"
BARS_F32 = ("forces 1e-5 normwise (2e-5 with bending), element by element 512 u32 sum|f_e|; reductions 1e-12 "
            "(float64); grid 1e-6 normwise, element by element 256 u32 sum|phi||F| (+ the fixed-point quantum); "
            "velocities 1e-6 normwise, element by element 256 u32 sum|phi||u|")


def sampled_errors(sc, F, red, G, v, u, seed=0):
    """Error of one step's results against the FP64 oracle, per result, on samples: the forces and the
    float64 reductions of 6 whole particles, 40 grid values of the spread of the step's own forces (every
    node that reaches them), the velocities of 2000 nodes.  Normwise relative errors over each sample;
    the oracle sees the positions the library sees (x64 = anchor + float64(x32))."""
    import oracle
    from paper_1807_08219_amd.inputs import scenes

    def rel(a, b):
        nb = np.linalg.norm(b)
        return float(np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0))

    rng = np.random.default_rng(seed)
    parts = np.unique(np.linspace(0, sc.n_particles - 1, 6).astype(int))
    sub = scenes.subset(sc, parts)
    Fo, _ = oracle.forces(sub)
    nodes = np.concatenate([np.arange(sc.node_start[p], sc.node_start[p + 1]) for p in parts])
    ro = oracle.reduce(sub)
    mem = ro[:, 1] != 0
    F64 = F.astype(np.float64)
    idx, near, bop = _cells_near(sc, rng, 40)
    Go = oracle.spread(sc, F64[:, near], x=sc.x64[:, near], box_of_point=bop[near])
    samp = rng.choice(sc.n_nodes, size=min(2000, sc.n_nodes), replace=False)
    vo = oracle.interp(sc, u.astype(np.float64), x=sc.x64[:, samp], box_of_point=bop[samp])
    return {"forces": rel(F[:, nodes], Fo), "volume": rel(red[parts, 0], ro[:, 0]),
            "area": rel(red[parts, 1][mem], ro[mem, 1]) if mem.any() else None,
            "centroid": rel(red[parts, 2:], ro[:, 2:]),
            "spread": rel(np.array([G[d, i] for d, i in idx]), np.array([Go[d, i] for d, i in idx])),
            "interp": rel(v[:, samp], vo),
            "sample": f"forces and reductions of particles {parts.tolist()} ({nodes.size} nodes), 40 grid values "
                      f"({near.size} contributing nodes), velocities of {samp.size} nodes",
            "bars": BARS_F64 if F.dtype == np.float64 else BARS_F32}


def autotune(plan, sc, dev, x32, anchor, u32):
    """ifem_plan_autotune on the workload's own float32 inputs (the forces of its positions); returns the
    chosen launch shape and the time the tuning took."""
    import torch

    from paper_1807_08219_amd import ifem

    F = torch.empty((3, sc.n_nodes), dtype=torch.float32, device=dev)
    plan.element_forces(ifem.IFEM_F32, x32, anchor, F, None)
    G = torch.empty((3, sc.total_cells), dtype=torch.float32, device=dev)
    v = torch.empty((3, sc.n_nodes), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    chosen = plan.autotune(ifem.IFEM_F32, x32, anchor, F, G, u32, v)
    chosen["tuning_s"] = round(time.perf_counter() - t0, 2)
    del F, G, v
    return chosen


def bench_workload(config, steps, warmup, dev):
    """One step on another workload (float32 as one captured graph, float64 eager with the tiled spread):
    nodes/s and the step's HBM fraction."""
    import torch

    from paper_1807_08219_amd import ifem
    from paper_1807_08219_amd.inputs import fields, scenes

    sc = scenes.refined_suspension() if config == "refined" else scenes.make_config(config)
    plan = ifem.Plan(sc)
    u64 = fields.scene_velocity(sc, dtype=torch.float64, shear_rate=1.0 if config == 3 else 0.0).to(dev)
    u32 = u64.to(torch.float32)
    x32, anchor = torch.as_tensor(sc.x32, device=dev), torch.as_tensor(sc.anchor, device=dev)
    tuning = autotune(plan, sc, dev, x32, anchor, u32)
    red = torch.empty((sc.n_particles, 5), dtype=torch.float64, device=dev)
    out = {"workload": sc.name, "nodes": sc.n_nodes, "particles": sc.n_particles, "cells": sc.total_cells,
           "tuning": tuning}
    x64 = torch.as_tensor(sc.x64, device=dev)
    for key, dt, x, a, u, tdt in (("f32", ifem.IFEM_F32, x32, anchor, u32, torch.float32),
                                  ("f64", ifem.IFEM_F64, x64, None, u64, torch.float64)):
        F = torch.empty((3, sc.n_nodes), dtype=tdt, device=dev)
        G = torch.empty((3, sc.total_cells), dtype=tdt, device=dev)
        v = torch.empty((3, sc.n_nodes), dtype=tdt, device=dev)

        def step():
            plan.element_forces(dt, x, a, F, red)
            plan.spread(dt, x, a, F, G)
            plan.interp(dt, x, a, u, v)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if key == "f32":
            graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                step()
            torch.cuda.current_stream().wait_stream(side)
            with torch.cuda.graph(graph):
                step()
            graph.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                graph.replay()
            torch.cuda.synchronize()
            del graph
        else:
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        nbytes = step_bytes(sc, key == "f64")
        out[key] = {"ms_per_step": round(ms, 4), "value": round(sc.n_nodes / (ms * 1e-3), 1), "unit": "nodes/s",
                    "timing": "graph replay" if key == "f32" else "eager",
                    "step_hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "step_hbm_frac_table": round(step_bytes_table(sc, key == "f64") / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[key]["errors_vs_oracle"] = sampled_errors(sc, F.cpu().numpy(), red.cpu().numpy(), G.cpu().numpy(),
                                                      v.cpu().numpy(), u.cpu().numpy())
        log(f"{sc.name} {key}: {ms:.3f} ms/step, {out[key]['value']:.3g} nodes/s, "
            f"errors {({k: v for k, v in out[key]['errors_vs_oracle'].items() if k not in ('sample', 'bars')})}")
        del F, G, v
    out["speedup_f32_vs_f64"] = round(out["f64"]["ms_per_step"] / out["f32"]["ms_per_step"], 3)
    out["device_status"] = plan.status()
    plan.close()
    return out


def bench_batched(steps, warmup, dev):
    """The FP32 coupling step on the batched workload (64 independent boxes of uneven size and mixed
    particles): eager launches and one captured graph, with its share of the HBM roofline."""
    import torch

    from paper_1807_08219_amd import ifem
    from paper_1807_08219_amd.inputs import fields, scenes

    sc = scenes.make_config(4)
    plan = ifem.Plan(sc)
    u32 = fields.scene_velocity(sc, dtype=torch.float32).to(dev)
    x32 = torch.as_tensor(sc.x32, device=dev)
    anchor = torch.as_tensor(sc.anchor, device=dev)
    tuning = autotune(plan, sc, dev, x32, anchor, u32)
    log(f"batched workload tuning {tuning}")
    F = torch.empty((3, sc.n_nodes), dtype=torch.float32, device=dev)
    red = torch.empty((sc.n_particles, 5), dtype=torch.float64, device=dev)
    G = torch.empty((3, sc.total_cells), dtype=torch.float32, device=dev)
    v = torch.empty((3, sc.n_nodes), dtype=torch.float32, device=dev)

    def step():
        plan.element_forces(ifem.IFEM_F32, x32, anchor, F, red)
        plan.spread(ifem.IFEM_F32, x32, anchor, F, G)
        plan.interp(ifem.IFEM_F32, x32, anchor, u32, v)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    nbytes = step_bytes(sc, False)
    log(f"batched workload ({sc.n_nodes} nodes, {sc.total_cells} cells in {len(sc.boxes)} boxes): {ms:.3f} ms/step, "
        f"graph {ms_graph:.3f} ms/step, {nbytes / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS:.3f} of HBM roofline")
    out = {"workload": sc.name, "nodes": sc.n_nodes, "cells": sc.total_cells, "boxes": len(sc.boxes),
           "ms_per_step": round(ms, 4), "value": round(sc.n_nodes / (ms * 1e-3), 1), "unit": "nodes/s",
           "graph_ms_per_step": round(ms_graph, 4), "graph_value": round(sc.n_nodes / (ms_graph * 1e-3), 1),
           "tuning": tuning, "algorithmic_bytes": int(nbytes),
           "graph_step_hbm_frac_table": round(step_bytes_table(sc, False) / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "step_hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "graph_step_hbm_frac": round(nbytes / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "device_status": plan.status()}
    del graph
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # after an idle moment the device takes about 8 steps to reach its steady clock (the first replays of
    # the dense step run 2.2-2.5 ms, then 1.99 ms): by default 10 untimed steps and 100 timed ones
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-visco", action="store_true")
    ap.add_argument("--no-contact", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the FP32 step on the 64-box batched workload")
    ap.add_argument("--tile", type=str, default=None, help="spread tile, e.g. 32,16,8 (powers of two)")
    ap.add_argument("--block-forces", type=int, default=None, help="threads per particle workgroup")
    ap.add_argument("--block-points", type=int, default=None, help="threads per workgroup of the point kernels")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="bytes of a plain device copy made before the steps (scale for HBM counters)")
    ap.add_argument("--no-autotune", action="store_true", help="time the default launch shape (or --tile)")
    ap.add_argument("--no-config3", action="store_true", help="skip the line of the blood suspension (config 3)")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the line of the suspension of nu = 32 red cells (the global-memory force path)")
    ap.add_argument("--no-errors", action="store_true", help="skip the sampled errors against the oracle")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)  # the child running the oracle
    ap.add_argument("--cpu-workers", type=int, default=16, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_leg:
        print(json.dumps(cpu_leg(args.config, args.cpu_budget, args.cpu_workers)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (multi-GPU sharding is a design "
                                   "note, not implemented)"}), flush=True)
        sys.exit(2)

    import torch

    from paper_1807_08219_amd import ifem
    from paper_1807_08219_amd.inputs import fields, scenes

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    sc = scenes.make_config(args.config)
    log(f"scene {sc.name}: {sc.n_particles} particles, {sc.n_nodes} nodes, {sc.n_tris} tris, {sc.n_tets} tets, "
        f"{sc.total_cells} cells ({time.time() - t0:.1f} s)")
    t0 = time.time()
    tuning = None
    if args.tile is not None or args.block_forces is not None or args.block_points is not None:
        tuning = {"tile": [int(v) for v in args.tile.split(",")] if args.tile else [32, 16, 8],
                  "block_forces": args.block_forces or 512, "block_points": args.block_points or 256}
    plan = ifem.Plan(sc, tuning=tuning)
    log(f"plan created ({time.time() - t0:.1f} s), info {plan.info()}")
    u64 = fields.scene_velocity(sc, dtype=torch.float64, shear_rate=1.0 if args.config == 3 else 0.0).to(dev)
    u32 = u64.to(torch.float32)
    x32 = torch.as_tensor(sc.x32, device=dev)
    anchor = torch.as_tensor(sc.anchor, device=dev)
    chosen = None
    if tuning is None and not args.no_autotune:
        chosen = autotune(plan, sc, dev, x32, anchor, u32)
        log(f"autotuned launch shape {chosen}")
    F32 = torch.empty((3, sc.n_nodes), dtype=torch.float32, device=dev)
    red = torch.empty((sc.n_particles, 5), dtype=torch.float64, device=dev)
    G32 = torch.empty((3, sc.total_cells), dtype=torch.float32, device=dev)
    v32 = torch.empty((3, sc.n_nodes), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step32():
        plan.element_forces(ifem.IFEM_F32, x32, anchor, F32, red)
        plan.spread(ifem.IFEM_F32, x32, anchor, F32, G32)
        plan.interp(ifem.IFEM_F32, x32, anchor, u32, v32)

    def timed(step, n, phases):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(n):
            e = ev[i]
            e[0].record(stream)
            phases[0]()
            e[1].record(stream)
            phases[1]()
            e[2].record(stream)
            phases[2]()
            e[3].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        per = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in ev])  # ms
        return wall, per

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"calibration copy of {args.copy_calibration} bytes done")
    plan.set(ifem.IFEM_OPT_SPREAD_MODE, ifem.IFEM_SPREAD_TILED)
    for _ in range(args.warmup):
        step32()
    torch.cuda.synchronize()
    log(f"fp32 warmup done; status {plan.status()}")
    ph32 = [lambda: plan.element_forces(ifem.IFEM_F32, x32, anchor, F32, red),
            lambda: plan.spread(ifem.IFEM_F32, x32, anchor, F32, G32),
            lambda: plan.interp(ifem.IFEM_F32, x32, anchor, u32, v32)]
    plan.set(ifem.IFEM_OPT_KERNEL_TIMING, 8 * args.steps + 64)
    plan.kernel_times(reset=True)
    wall, per = timed(step32, args.steps, ph32)
    ktimes = plan.kernel_times(reset=True)
    plan.set(ifem.IFEM_OPT_KERNEL_TIMING, 0)
    ms_step = wall * 1e3 / args.steps
    ms_phase = per.mean(axis=0)
    log(f"fp32: {ms_step:.3f} ms/step (wall), phases forces/spread/interp {ms_phase.round(4).tolist()} ms")
    kavg = {k: (t / n, n / args.steps) for k, (t, n) in ktimes.items() if k != "dropped"}
    log("fp32 kernels (avg ms, launches/step): " + ", ".join(f"{k} {v[0]:.4f} x{v[1]:.0f}" for k, v in kavg.items()))
    nodes_per_s = sc.n_nodes / (ms_step * 1e-3)
    alg = algorithmic(sc, fp64=False)
    # dominant kernel among those with an algorithmic figure (the merge and the scans have none)
    dom = max((k for k in kavg if k in alg), key=lambda k: kavg[k][0] * kavg[k][1])
    t_dom = kavg[dom][0] * 1e-3
    bytes_dom, flops_dom = alg.get(dom, (None, None))
    gbs = bytes_dom / t_dom / 1e9 if bytes_dom else None
    tfs = flops_dom / t_dom / 1e12 if flops_dom else None
    hbm_frac = gbs / HBM_PEAK_GBS if gbs else 0.0
    # the metric is a share of HBM bandwidth: the headline is the dominant kernel's HBM fraction; its
    # vector-ALU fraction (against the non-packed float32 rate this build runs at) is beside it
    roofline = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    roofline.update({
        "traffic": measured_traffic(dom, sc.name, plan.info()[3:6]), "kernel": dom, "kernel_ms": round(kavg[dom][0], 4),
        "algorithmic_bytes": int(bytes_dom) if bytes_dom else None,
        "algorithmic_flops": int(flops_dom) if flops_dom else None,
        "alu_tflops": round(tfs, 3) if tfs else None,
        "alu_frac_nonpacked": round(tfs / VALU_NONPACKED_TFLOPS, 4) if tfs else None,
        "alu_peak_nonpacked": VALU_NONPACKED_TFLOPS,
        "step_hbm_frac": round(step_bytes(sc, False) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels_ms": {k: round(v[0], 4) for k, v in kavg.items()},
    })
    out = {"metric": METRIC, "value": round(nodes_per_s, 1), "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": sc.name, "nodes": sc.n_nodes, "particles": sc.n_particles, "tris": sc.n_tris,
                      "tets": sc.n_tets, "cells": sc.total_cells, "grid": list(sc.boxes[0].n),
                      "precision": "f32 compensated invariants, f64 reductions, deterministic tiled spread",
                      "spread_tile": plan.info()[3:6], "block_forces": plan.info()[6],
                      "block_points": plan.info()[7], "autotuned": chosen is not None},
           "roofline": roofline}
    if chosen is not None:
        out["autotune"] = chosen
    st = plan.status()
    out["device_status"] = st

    # the same step captured once as a HIP graph and replayed (no host launch work per step), right
    # after the eager steps, so that no host-side work idles the device in between
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step32()
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(graph):
        step32()
    for _ in range(max(args.warmup, 1)):
        graph.replay()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t_start) * 1e3 / args.steps
    # per-replay durations (events on the replay stream) for the median
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        graph.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    med_graph = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
    log(f"fp32 graph replay: {ms_graph:.3f} ms/step (median of {args.steps} replays {med_graph:.3f} ms)")
    # the headline: the coupling step as one replayed graph, K replays between two synchronisations
    out["eager"] = {"ms_per_step": out["ms_per_step"], "value": out["value"], "steps": args.steps}
    out["ms_per_step"] = round(ms_graph, 4)
    out["value"] = round(sc.n_nodes / (ms_graph * 1e-3), 1)
    out["graph_replay"] = {"ms_per_step": round(ms_graph, 4), "median_ms": round(med_graph, 4),
                           "value": round(sc.n_nodes / (ms_graph * 1e-3), 1), "steps": args.steps}
    out["roofline"]["step_hbm_frac"] = round(step_bytes(sc, False) / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    out["roofline"]["step_hbm_frac_table"] = round(step_bytes_table(sc, False) / (ms_graph * 1e-3) / 1e9 /
                                                   HBM_PEAK_GBS, 4)
    del graph
    # the replays wrote the same results as the eager steps (same inputs): compared with the oracle now
    if not args.no_errors:
        out["errors_vs_oracle"] = {"f32": sampled_errors(sc, F32.cpu().numpy(), red.cpu().numpy(), G32.cpu().numpy(),
                                                         v32.cpu().numpy(), u32.cpu().numpy())}
        log(f"fp32 errors vs oracle {out['errors_vs_oracle']['f32']}")

    if not args.no_volume:
        out["volume_correct"] = bench_volume(plan, sc, args.steps, dev, stream)
    if not args.no_loop:
        out["lagrangian_loop"] = bench_loop(plan, sc, args.steps, dev, anchor, u32)
    if not args.no_visco:
        out["viscoelastic"] = bench_viscoelastic(plan, sc, args.steps, dev, x32, anchor)
    if not args.no_contact:
        out["antistick"] = bench_antistick(plan, sc, args.steps, dev, x32, anchor)
    if not args.no_batched and args.config != 4:
        out["batched"] = bench_batched(args.steps, args.warmup, dev)
    if not args.no_config3 and args.config != 3:
        out.setdefault("workloads", {})["blood_500rbc_50plt"] = bench_workload(3, args.steps, args.warmup, dev)
    if not args.no_refined:
        # red cells meshed at nu = 32: every particle takes the global-memory force path
        out.setdefault("workloads", {})["refined_130rbc_nu32"] = bench_workload("refined", args.steps, args.warmup,
                                                                                 dev)

    if not args.no_fp64:
        x64 = torch.as_tensor(sc.x64, device=dev)
        F64 = torch.empty((3, sc.n_nodes), dtype=torch.float64, device=dev)
        G64 = torch.empty((3, sc.total_cells), dtype=torch.float64, device=dev)
        v64 = torch.empty((3, sc.n_nodes), dtype=torch.float64, device=dev)
        ph64 = [lambda: plan.element_forces(ifem.IFEM_F64, x64, None, F64, red),
                lambda: plan.spread(ifem.IFEM_F64, x64, None, F64, G64),
                lambda: plan.interp(ifem.IFEM_F64, x64, None, u64, v64)]
        for mode, key, label in ((ifem.IFEM_SPREAD_TILED, "fp64", "tiled fixed-point spread"),
                                 (ifem.IFEM_SPREAD_ATOMIC, "fp64_plain", "global atomics")):
            plan.set(ifem.IFEM_OPT_SPREAD_MODE, mode)
            for f in ph64:
                f()
            torch.cuda.synchronize()
            wall64, per64 = timed(None, args.fp64_steps, ph64)
            ms64 = wall64 * 1e3 / args.fp64_steps
            log(f"{key} ({label}): {ms64:.3f} ms/step, phases {per64.mean(axis=0).round(4).tolist()} ms")
            out[key] = {"value": round(sc.n_nodes / (ms64 * 1e-3), 1), "unit": "nodes/s", "ms_per_step": round(ms64, 4),
                        "steps": args.fp64_steps, "phases_ms": per64.mean(axis=0).round(4).tolist(), "spread": label}
            out["speedup_fp32_vs_" + key] = round(ms64 / ms_step, 3)
        plan.set(ifem.IFEM_OPT_SPREAD_MODE, ifem.IFEM_SPREAD_TILED)
        if not args.no_errors:  # one more step with the tiled spread, the one the errors describe
            for f in ph64:
                f()
            torch.cuda.synchronize()
            out.setdefault("errors_vs_oracle", {})["f64"] = sampled_errors(
                sc, F64.cpu().numpy(), red.cpu().numpy(), G64.cpu().numpy(), v64.cpu().numpy(), u64.cpu().numpy())
            log(f"fp64 errors vs oracle {out['errors_vs_oracle']['f64']}")
        del F64, G64, v64, x64

    plan.close()
    if not args.no_cpu_baseline:
        log("cpu baselines (oracle, in a child process) ...")
        cb = cpu_baselines_in_child(args.config, args.cpu_budget)
        out["cpu_baseline"] = {**cb["all_cores"], "host_cpu": cb["host_cpu"], "host_threads": cb["host_threads"]}
        out["cpu_baseline_single_thread"] = cb["single"]
        log(f"cpu baselines: {cb['single']['value']:.1f} nodes/s single-threaded, "
            f"{cb['all_cores']['value']:.1f} nodes/s on {cb['all_cores']['cores']} processes")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
