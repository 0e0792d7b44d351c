"""Element forces (Sec. II.A and II.B) in x87 extended precision.

Test infrastructure only: the same element forces as the oracle's float64 ones, evaluated with
numpy's 80-bit longdouble (64-bit significand), so that for a particle whose float64 forces are
ill-conditioned (near-incompressible solids with flattened reference tetrahedra, membranes with thin
reference triangles) both float64 evaluations, the library's and the oracle's, can be measured
against a reference that is about 2^11 times more precise.

Tetrahedra (slightly compressible neo-Hookean solid):
Per element, with D0 the reference edges from node 0 (columns) and g_a the rows of D0^-1 (the shape
function gradients of nodes 1..3; node 0 takes minus their sum): F = sum_a (x_a - x_0) (x) g_a,
J = det F, C^-1 = F^-1 F^-T, S = lam/2 (J^2 - 1) C^-1 + mu (I - C^-1), P = F S and
f_k = -V0 P g_k with V0 = det D0 / 6.
"""
import numpy as np

LD = np.longdouble


def _det(m):
    return (m[..., 0, 0] * (m[..., 1, 1] * m[..., 2, 2] - m[..., 1, 2] * m[..., 2, 1])
            - m[..., 0, 1] * (m[..., 1, 0] * m[..., 2, 2] - m[..., 1, 2] * m[..., 2, 0])
            + m[..., 0, 2] * (m[..., 1, 0] * m[..., 2, 1] - m[..., 1, 1] * m[..., 2, 0]))


def _inv(m):
    """Inverse of a stack of 3 x 3 matrices by cofactors (numpy's linalg has no longdouble), and det."""
    d = _det(m)
    r = np.empty_like(m)
    r[..., 0, 0] = m[..., 1, 1] * m[..., 2, 2] - m[..., 1, 2] * m[..., 2, 1]
    r[..., 0, 1] = m[..., 0, 2] * m[..., 2, 1] - m[..., 0, 1] * m[..., 2, 2]
    r[..., 0, 2] = m[..., 0, 1] * m[..., 1, 2] - m[..., 0, 2] * m[..., 1, 1]
    r[..., 1, 0] = m[..., 1, 2] * m[..., 2, 0] - m[..., 1, 0] * m[..., 2, 2]
    r[..., 1, 1] = m[..., 0, 0] * m[..., 2, 2] - m[..., 0, 2] * m[..., 2, 0]
    r[..., 1, 2] = m[..., 0, 2] * m[..., 1, 0] - m[..., 0, 0] * m[..., 1, 2]
    r[..., 2, 0] = m[..., 1, 0] * m[..., 2, 1] - m[..., 1, 1] * m[..., 2, 0]
    r[..., 2, 1] = m[..., 0, 1] * m[..., 2, 0] - m[..., 0, 0] * m[..., 2, 1]
    r[..., 2, 2] = m[..., 0, 0] * m[..., 1, 1] - m[..., 0, 1] * m[..., 1, 0]
    return r / d[..., None, None], d


def tet_forces(X, x, tets, mu, lam):
    """[n][3] longdouble nodal forces of the tetrahedra tets [m][4] (local node ids) of one solid with
    reference positions X [n][3] and current positions x [n][3] (float64, widened exactly)."""
    X = np.asarray(X, dtype=np.float64).astype(LD)
    x = np.asarray(x, dtype=np.float64).astype(LD)
    t = np.asarray(tets, dtype=np.int64)
    D0 = np.transpose(X[t[:, 1:]] - X[t[:, :1]], (0, 2, 1))  # [m][i][a] = X_a+1,i - X_0,i
    Di, det0 = _inv(D0)
    g = np.empty((len(t), 4, 3), dtype=LD)
    g[:, 1:, :] = Di  # rows of D0^-1
    g[:, 0, :] = -(g[:, 1, :] + g[:, 2, :] + g[:, 3, :])
    V0 = det0 / LD(6)
    d = x[t[:, 1:]] - x[t[:, :1]]  # [m][a][i] current edges
    F = np.einsum("mai,maj->mij", d, g[:, 1:, :])
    Fi, J = _inv(F)
    Cinv = np.einsum("mkl,mjl->mkj", Fi, Fi)
    eye = np.eye(3, dtype=LD)
    S = (LD(0.5) * LD(lam) * (J * J - LD(1)))[:, None, None] * Cinv + LD(mu) * (eye - Cinv)
    P = np.einsum("mik,mkj->mij", F, S)
    fe = -V0[:, None, None] * np.einsum("mij,mkj->mki", P, g)  # [m][k][i]
    out = np.zeros((len(X), 3), dtype=LD)
    np.add.at(out, t.reshape(-1), fe.reshape(-1, 3))
    return out


def particle_forces(sc, p):
    """[3][n_p] longdouble nodal forces of solid particle p of a scene (its tetrahedra only)."""
    n0, n1 = int(sc.node_start[p]), int(sc.node_start[p + 1])
    t0, t1 = int(sc.tet_start[p]), int(sc.tet_start[p + 1])
    tets = sc.tet[:, t0:t1].T - n0
    f = tet_forces(sc.X_ref[:, n0:n1].T, sc.x64[:, n0:n1].T, tets, float(sc.mu[p]), float(sc.mu2[p]))
    return f.T


def rel_ld(a, ref):
    """Normwise relative difference of a float64 (or longdouble) array from a longdouble reference, in
    longdouble."""
    d = np.asarray(a).astype(LD) - ref
    return float(np.sqrt((d * d).sum()) / np.sqrt((ref * ref).sum()))


def _normalize(v):
    return v / np.sqrt((v * v).sum(axis=-1, keepdims=True))


def tri_forces(X, x, tris, law, mu, mu2):
    """[n][3] longdouble nodal forces of the triangles tris [m][3] of one membrane (elastic part only).

    Per element, in the tangent frame of each configuration (e1 along edge 0 -> 1, e2 = n x e1):
    the reference edges' frame coordinates D0 (columns), whose inverse's rows are the shape
    gradients of nodes 1 and 2 (node 0: minus their sum); the surface deformation gradient
    F^ = sum_k (e_l . (x_k - x_0)) g_k; C^ = F^T F^, I1 = tr C^, I2 = det C^;
    S^ = 2 (W1 I + I2 C^-1 W2) with W1, W2 the derivatives of the neo-Hookean or Skalak energy;
    P^ = F^ S^ and f_k = -A0 sum_l (P^ g_k)_l e_l with A0 = det D0 / 2."""
    X = np.asarray(X, dtype=np.float64).astype(LD)
    x = np.asarray(x, dtype=np.float64).astype(LD)
    t = np.asarray(tris, dtype=np.int64)

    def frame(P):
        a = P[t[:, 1]] - P[t[:, 0]]
        b = P[t[:, 2]] - P[t[:, 0]]
        n = np.cross(a, b)
        e1 = _normalize(a)
        e2 = np.cross(_normalize(n), e1)
        return a, b, e1, e2

    a0, b0, E1, E2 = frame(X)
    D00 = (a0 * E1).sum(-1)
    D01 = (b0 * E1).sum(-1)
    D10 = (a0 * E2).sum(-1)
    D11 = (b0 * E2).sum(-1)
    det = D00 * D11 - D01 * D10
    g = np.empty((len(t), 3, 2), dtype=LD)
    g[:, 1, 0], g[:, 1, 1] = D11 / det, -D01 / det
    g[:, 2, 0], g[:, 2, 1] = -D10 / det, D00 / det
    g[:, 0, :] = -(g[:, 1, :] + g[:, 2, :])
    A0 = det / LD(2)
    a, b, e1, e2 = frame(x)
    e = np.stack([e1, e2], axis=1)  # [m][l][3]
    d = np.stack([a, b], axis=1)  # [m][k-1][3]
    proj = np.einsum("mkc,mlc->mlk", d, e)  # [m][l][k-1]: e_l . (x_k - x_0)
    Fh = np.einsum("mlk,mkj->mlj", proj, g[:, 1:, :])
    C = np.einsum("mli,mlj->mij", Fh, Fh)
    I1 = C[:, 0, 0] + C[:, 1, 1]
    I2 = C[:, 0, 0] * C[:, 1, 1] - C[:, 0, 1] * C[:, 1, 0]
    mu, mu2 = LD(mu), LD(mu2)
    if law == 0:  # neo-Hookean membrane
        W1 = np.full_like(I1, LD(0.5) * mu)
        W2 = -LD(0.5) * mu / (I2 * I2)
    else:  # Skalak
        W1 = LD(0.5) * mu * ((I1 - LD(2)) + LD(1))
        W2 = -LD(0.5) * mu + LD(0.25) * mu2 * (I2 - LD(1))
    Ci = np.empty_like(C)
    Ci[:, 0, 0], Ci[:, 0, 1] = C[:, 1, 1] / I2, -C[:, 0, 1] / I2
    Ci[:, 1, 0], Ci[:, 1, 1] = -C[:, 1, 0] / I2, C[:, 0, 0] / I2
    eye = np.eye(2, dtype=LD)
    S = LD(2) * (W1[:, None, None] * eye + (I2 * W2)[:, None, None] * Ci)
    P = np.einsum("mik,mkj->mij", Fh, S)
    c = np.einsum("mlj,mkj->mkl", P, g)  # [m][k][l]
    fe = -A0[:, None, None] * np.einsum("mkl,mlc->mkc", c, e)
    out = np.zeros((len(X), 3), dtype=LD)
    np.add.at(out, t.reshape(-1), fe.reshape(-1, 3))
    return out


def particle_membrane_forces(sc, p):
    """[3][n_p] longdouble elastic nodal forces of membrane particle p of a scene (no bending)."""
    n0, n1 = int(sc.node_start[p]), int(sc.node_start[p + 1])
    t0, t1 = int(sc.tri_start[p]), int(sc.tri_start[p + 1])
    tris = sc.tri[:, t0:t1].T - n0
    f = tri_forces(sc.X_ref[:, n0:n1].T, sc.x64[:, n0:n1].T, tris, int(sc.law[p]), float(sc.mu[p]),
                   float(sc.mu2[p]))
    return f.T
