"""GPU Lagrangian update (Sec. III.A, last step) and a multi-step Lagrangian loop in a HIP graph.

The update is float64 in the order written without fused multiply-add, so the float64 path equals
the oracle bit for bit; float32 offsets are rounded once (bar: u32 of the result, plus the
float64 rounding of the absolute position the oracle forms).  The loop (forces, spread,
interpolation of a steady synthetic velocity, Adams-Bashforth update, volume correction) is run
eagerly and as graph replays, which must agree bitwise, and against the oracle's loop, to the
volume correction's bars carried through the steps.
"""
import numpy as np
import pytest

import oracle
from paper_1807_08219_amd import ifem
from paper_1807_08219_amd.inputs import fields, scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def cu(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("name", ["mixed_two_boxes", "config2_rbc_2562"])
def test_advance_matches_oracle(name):
    sc = scenes.small_mixed() if name == "mixed_two_boxes" else scenes.config2()
    print(f"[gpu] advance {name}", flush=True)
    rng = np.random.default_rng(3)
    v = rng.normal(size=(3, sc.n_nodes))
    vp = rng.normal(size=(3, sc.n_nodes))
    dt = 0.0137
    plan = ifem.Plan(sc)
    x = cu(sc.x64, torch.float64)
    out = torch.empty_like(x)
    for prev in (vp, None):
        plan.advance(ifem.IFEM_F64, x, cu(v, torch.float64), out, v_prev=None if prev is None else cu(prev, torch.float64),
                     dt=dt)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.advance(sc.x64, v, prev, dt))
    # in place
    xin = x.clone()
    plan.advance(ifem.IFEM_F64, xin, cu(v, torch.float64), xin, v_prev=cu(vp, torch.float64), dt=dt)
    torch.cuda.synchronize()
    assert np.array_equal(xin.cpu().numpy(), oracle.advance(sc.x64, v, vp, dt))

    # float32 offsets and velocities
    v32, vp32 = v.astype(np.float32), vp.astype(np.float32)
    x32 = cu(sc.x32, torch.float32)
    o32 = torch.empty_like(x32)
    plan.advance(ifem.IFEM_F32, x32, cu(v32, torch.float32), o32, v_prev=cu(vp32, torch.float32), dt=dt)
    torch.cuda.synchronize()
    ref = oracle.advance(sc.x64, v32.astype(np.float64), vp32.astype(np.float64), dt)
    a = sc.anchor[sc.node_particle()].T
    got = o32.cpu().numpy().astype(np.float64)
    bar = U32 * np.abs(ref - a) + 4 * U64 * np.abs(ref)
    assert np.all(np.abs(got - (ref - a)) <= bar)

    with pytest.raises(ifem.IfemError):  # a velocity written over
        plan.advance(ifem.IFEM_F64, x, out, out, dt=dt)
    with pytest.raises(ifem.IfemError):
        plan.advance(ifem.IFEM_F64, x, cu(v, torch.float64), out, dt=float("nan"))
    plan.close()


def _oracle_loop(sc, u, steps, dt):
    """Oracle loop: interpolate, update (Euler first), correct volumes; returns positions and the last grid."""
    x, vp, G = sc.x64.copy(), None, None
    for _ in range(steps):
        Fo, _ = oracle.forces(sc, x=x)
        G = oracle.spread(sc, Fo, x=x)
        v = oracle.interp(sc, u, x=x)
        x = oracle.advance(x, v, vp, dt)
        x, _, bad = oracle.volume_correct(sc, x=x)
        assert bad == 0
        vp = v
    return x, G


def test_lagrangian_loop_in_a_graph():
    sc = scenes.small_mixed()
    u = fields.scene_velocity(sc).numpy()
    dt = 0.02
    plan = ifem.Plan(sc)
    x = cu(sc.x64, torch.float64)
    ud = cu(u, torch.float64)
    F = torch.empty_like(x)
    G = torch.empty((3, sc.total_cells), dtype=torch.float64, device="cuda")
    vA, vB = torch.empty_like(x), torch.empty_like(x)

    def step(v_new, v_old, stream=None):
        plan.element_forces(ifem.IFEM_F64, x, None, F, None, stream)
        plan.spread(ifem.IFEM_F64, x, None, F, G, stream)
        plan.interp(ifem.IFEM_F64, x, None, ud, v_new, stream)
        plan.advance(ifem.IFEM_F64, x, v_new, x, v_prev=v_old, dt=dt, stream=stream)
        plan.volume_correct(ifem.IFEM_F64, x, x, stream=stream)

    print("[gpu] Lagrangian loop: eager", flush=True)
    step(vA, None)  # forward Euler start
    for _ in range(3):
        step(vB, vA)
        step(vA, vB)
    torch.cuda.synchronize()
    x_eager, G_eager = x.cpu().numpy(), G.cpu().numpy()

    print("[gpu] Lagrangian loop: graph", flush=True)
    x.copy_(cu(sc.x64, torch.float64))
    step(vA, None)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    x_keep = x.clone()
    with torch.cuda.stream(s):
        step(vB, vA, s)  # warm-up on the capture stream, then restore the state
        step(vA, vB, s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            step(vB, vA, s)
            step(vA, vB, s)
    torch.cuda.synchronize()
    # the warm-up and the capture moved x (capture does not run, warm-up did): restart from after step 0
    x.copy_(cu(sc.x64, torch.float64))
    step(vA, None)
    torch.cuda.synchronize()
    assert torch.equal(x, x_keep)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), x_eager)
    assert np.array_equal(G.cpu().numpy(), G_eager)

    print("[gpu] Lagrangian loop: oracle", flush=True)
    xo, Go = _oracle_loop(sc, u, 7, dt)
    e = np.linalg.norm(x_eager - xo) / np.linalg.norm(xo)
    print(f"    positions rel err {e:.3e} after 7 steps (moved {np.abs(xo - sc.x64).max():.3f})", flush=True)
    assert e <= 1e-12
    assert np.linalg.norm(G_eager - Go) / np.linalg.norm(Go) <= 1e-10
    assert plan.status() == [0, 0, 0, 0, 0]
    plan.close()
