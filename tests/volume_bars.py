"""Error bars of the GPU volume correction against the oracle (Sec. II.E), shared by the tests.

Tolerances.  The kernel works in a particle-local frame; the oracle in absolute coordinates,
where the face sums cancel: a triple product y1.(y2 x y3) of positions of size |y| carries a
rounding error of a few u64 |y1| |y2 x y3| however small the result.  So the oracle's
volume error is bounded by u64 M_V, M_V = sum over faces and corners |y_k| |y_k1 x y_k2| / 18
(taken for the current and the reference positions), and the multiplier L ~ -D / C inherits
M_V / |C|; the relative error of C itself is bounded by u64 M_C / |C| with
M_C = sum |a_k| |y_k1 x y_k2| / 6.  The bars are 32 times those bounds plus 1e-12 |L|:
  |L_gpu - L_orc| <= 1e-12 |L| + 32 u64 (M_V(x) + M_V(X)) / |C| + 32 u64 |L| M_C / |C|,
  |x_gpu - x_orc| <= 4 u64 |x| + |alpha| (bar on L) + 8 u64 |L| M_a   (float64 positions),
  |x_gpu - x_orc| <= u32 |x - anchor| + the float64 bar                (float32 offsets),
where M_a = sum over the faces at the node of |y_j| |y_k| / 12 bounds the oracle's rounding of
alpha itself (the cross products of absolute positions).
"""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def lambda_bars(sc, x_orc, lam_orc):
    """Per-particle bar on L, per-node bar on x (see the module docstring) and alpha [3][n]."""
    alpha = np.zeros_like(sc.x64)
    bars = np.zeros(sc.n_particles)
    m_a = np.zeros(sc.n_nodes)
    for p in range(sc.n_particles):
        t0, t1 = sc.tri_start[p], sc.tri_start[p + 1]
        if t1 == t0:
            continue
        s, e = sc.node_start[p], sc.node_start[p + 1]
        if lam_orc[p] != 0:
            alpha[:, s:e] = (x_orc[:, s:e] - sc.x64[:, s:e]) / lam_orc[p]
        tri = sc.tri[:, t0:t1].T

        def m_v(y):
            q = y.T[tri]  # [m][3][3]
            return sum(np.sum(np.linalg.norm(q[:, k], axis=1) *
                              np.linalg.norm(np.cross(q[:, (k + 1) % 3], q[:, (k + 2) % 3]), axis=1))
                       for k in range(3)) / 18.0

        q = sc.x64.T[tri]
        for k in range(3):
            np.add.at(m_a, tri[:, k], np.linalg.norm(q[:, (k + 1) % 3], axis=1) *
                      np.linalg.norm(q[:, (k + 2) % 3], axis=1) / 12.0)
        a = alpha.T[tri]
        cr = [np.cross(q[:, (k + 1) % 3], q[:, (k + 2) % 3]) for k in range(3)]
        C = sum(np.sum(a[:, k] * cr[k]) for k in range(3)) / 6.0
        m_c = sum(np.sum(np.linalg.norm(a[:, k], axis=1) * np.linalg.norm(cr[k], axis=1)) for k in range(3)) / 6.0
        bars[p] = 1e-12 * abs(lam_orc[p]) + 32 * U64 * (m_v(sc.x64) + m_v(sc.X_ref)) / abs(C) + \
            32 * U64 * abs(lam_orc[p]) * m_c / abs(C)
    npart = sc.node_particle()
    xbar = 4 * U64 * np.abs(sc.x64) + np.abs(alpha) * bars[npart] + 8 * U64 * np.abs(lam_orc[npart]) * m_a
    return bars, alpha, xbar
