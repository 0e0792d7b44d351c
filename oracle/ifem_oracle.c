/*
 * FP64 CPU oracle for the IFEM coupling step of Saadat, Guido, Iaccarino &
 * Shaqfeh, "Immersed-finite-element method for deformable particle
 * suspensions in viscous and viscoelastic media" (arXiv 1807.08219).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  It shares no code,
 * header, table or helper with the library, and the library never calls it.
 *
 * Everything is plain double precision, single threaded, in the order the
 * paper states it:
 *   - membrane element forces in a per-element tangent frame
 *       (Sec. II.B, eq. FEM_Membrane and the surface deformation gradient),
 *     with the constitutive laws of Sec. II.A (tension relation, neo-Hookean
 *     and Skalak energies);
 *   - tetrahedral element forces (Sec. II.B, eq. FEM with the discrete
 *     deformation gradient and the first Piola-Kirchhoff stress of the
 *     slightly compressible neo-Hookean solid);
 *   - Helfrich bending nodal force (Sec. II.B, bending force equation) with
 *     the discrete curvature operators of Meyer, Desbrun, Schroeder & Barr
 *     (2003) for the quantities the paper names (Voronoi area, mean and
 *     Gaussian curvature, surface Laplacian);
 *   - linear moving-least-squares weights, interpolation and spreading
 *     (Sec. II.C, Interpolation Scheme);
 *   - per-particle volume (Sec. II.E volume formula), area and centroid;
 *   - the membrane volume correction (Sec. II.E, conservation of volume for
 *     membranes: the Lagrange-multiplier displacement and its cubic);
 *   - the second-order Adams-Bashforth update of the positions (Sec. III.A);
 *   - the interpolation of the conformation tensor to the nodes and the
 *     fluid-stress (Newtonian and polymer) forces on solids (Sec. II.B,
 *     Sec. III.A steps 1 and 4);
 *   - node-face anti-sticking (Sec. III.B).
 *
 * Readings of the paper where it is silent or garbled are marked READING.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_LAW_TRI_NEOHOOKE 0
#define ORC_LAW_TRI_SKALAK 1
#define ORC_LAW_TET_NEOHOOKE 2

/* ------------------------------------------------------------ small linear algebra */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void sub3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[0] - b[0];
  c[1] = a[1] - b[1];
  c[2] = a[2] - b[2];
}
static double det3(const double m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}
/* inverse by cofactors; returns the determinant */
static double inv3(const double m[3][3], double r[3][3]) {
  double d = det3(m);
  r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / d;
  r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / d;
  r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / d;
  r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / d;
  r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / d;
  r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / d;
  r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / d;
  r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / d;
  r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / d;
  return d;
}
static void pos(const double* x, long stride, int k, double out[3]) {
  out[0] = x[k];
  out[1] = x[stride + k];
  out[2] = x[2 * stride + k];
}

/* ------------------------------------------------------------ constitutive laws (Sec. II.A) */
/* Membrane energy density per reference area as a function of I1 = tr C^, I2 = det C^. */
double orc_membrane_W(int law, double mu, double mu2, double I1, double I2) {
  if (law == ORC_LAW_TRI_NEOHOOKE) return 0.5 * mu * (I1 + 1.0 / I2 - 3.0); /* neo-Hookean membrane */
  /* Skalak law with the shifted invariants I1 - 2 and I2 - 1 */
  double a = I1 - 2.0, b = I2 - 1.0;
  return 0.5 * mu * (0.5 * a * a + a - b) + mu2 / 8.0 * b * b;
}
/* dW/dI1 and dW/dI2 of the two membrane laws. */
static void membrane_dW(int law, double mu, double mu2, double I1, double I2, double* W1, double* W2) {
  if (law == ORC_LAW_TRI_NEOHOOKE) {
    *W1 = 0.5 * mu;
    *W2 = -0.5 * mu / (I2 * I2);
  } else {
    *W1 = 0.5 * mu * ((I1 - 2.0) + 1.0);
    *W2 = -0.5 * mu + 0.25 * mu2 * (I2 - 1.0);
  }
}
/* Slightly compressible neo-Hookean solid, I3 = J^2.  READING: the logarithmic
 * term is ln(I3^(1/2)) = ln J, the only reading consistent with the discrete
 * stress the paper gives for tetrahedra. */
double orc_solid_W(double mu, double lam, double I1, double I3) {
  return 0.25 * lam * (I3 - 1.0) - (0.5 * lam + mu) * log(sqrt(I3)) + 0.5 * mu * (I1 - 3.0);
}

/* ------------------------------------------------------------ membrane element (Sec. II.B) */
/* Local orthonormal tangent frame of a triangle: e1 along edge 0->1, e2 = n x e1. */
static int tri_frame(const double p0[3], const double p1[3], const double p2[3], double e1[3], double e2[3]) {
  double a[3], b[3], n[3];
  sub3(p1, p0, a);
  sub3(p2, p0, b);
  cross3(a, b, n);
  double la = norm3(a), ln = norm3(n);
  if (!(la > 0.0) || !(ln > 0.0)) return 1;
  for (int i = 0; i < 3; ++i) {
    e1[i] = a[i] / la;
    n[i] /= ln;
  }
  cross3(n, e1, e2);
  return 0;
}

/* Reference data of a linear triangle: gradients of the three shape functions
 * in the reference tangent coordinates and the reference area. */
static int tri_reference(const double X[3][3], double gradN[3][2], double* A0) {
  double E1[3], E2[3], d1[3], d2[3];
  if (tri_frame(X[0], X[1], X[2], E1, E2)) return 1;
  sub3(X[1], X[0], d1);
  sub3(X[2], X[0], d2);
  /* columns of D0 are the two reference edges in the local frame */
  double D0[2][2] = {{dot3(d1, E1), dot3(d2, E1)}, {dot3(d1, E2), dot3(d2, E2)}};
  double det = D0[0][0] * D0[1][1] - D0[0][1] * D0[1][0];
  if (!(det > 0.0)) return 1;
  /* barycentric (s, t) = D0^-1 (xi - xi0): grad N1 and grad N2 are the rows of D0^-1 */
  double inv[2][2] = {{D0[1][1] / det, -D0[0][1] / det}, {-D0[1][0] / det, D0[0][0] / det}};
  gradN[1][0] = inv[0][0];
  gradN[1][1] = inv[0][1];
  gradN[2][0] = inv[1][0];
  gradN[2][1] = inv[1][1];
  gradN[0][0] = -gradN[1][0] - gradN[2][0];
  gradN[0][1] = -gradN[1][1] - gradN[2][1];
  *A0 = 0.5 * det;
  return 0;
}

/* Surface deformation gradient F^_ij = sum_k (x_k . e_i) dN^_k/dxi_j in the
 * current tangent frame.  The sum over k of the shape-function gradients is
 * zero, so positions are taken relative to node 0 (same value, no loss of
 * digits far from the origin). */
static void tri_defgrad(const double x[3][3], const double gradN[3][2], const double e[2][3], double Fh[2][2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double s = 0.0;
      for (int k = 1; k < 3; ++k) {
        double d[3];
        sub3(x[k], x[0], d);
        s += dot3(d, e[i]) * gradN[k][j];
      }
      Fh[i][j] = s;
    }
}

/* Membrane element: nodal forces f[k][i] = -A0 sum_{l,j} P^_lj dN^_k/dxi_j e_l,i.
 * Returns 0, or 1 when the element is degenerate (I2 <= 0) and contributes 0. */
int orc_membrane_element(const double X[3][3], const double x[3][3], int law, double mu, double mu2,
                         double f[3][3]) {
  memset(f, 0, 9 * sizeof(double));
  double gradN[3][2], A0, e[2][3];
  if (tri_reference(X, gradN, &A0)) return 1;
  if (tri_frame(x[0], x[1], x[2], e[0], e[1])) return 1;
  double Fh[2][2];
  tri_defgrad(x, gradN, (const double(*)[3])e, Fh);
  double C[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) C[i][j] = Fh[0][i] * Fh[0][j] + Fh[1][i] * Fh[1][j];
  double I1 = C[0][0] + C[1][1];
  double I2 = C[0][0] * C[1][1] - C[0][1] * C[1][0];
  if (!(I2 > 0.0)) return 1;
  double W1, W2;
  membrane_dW(law, mu, mu2, I1, I2, &W1, &W2);
  /* S^ = 2 (dW/dI1 I + J^2 C^-1 dW/dI2) with J^2 = I2 */
  double Ci[2][2] = {{C[1][1] / I2, -C[0][1] / I2}, {-C[1][0] / I2, C[0][0] / I2}};
  double S[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) S[i][j] = 2.0 * ((i == j ? W1 : 0.0) + I2 * Ci[i][j] * W2);
  double P[2][2]; /* P^ = F^ S^ */
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) P[i][j] = Fh[i][0] * S[0][j] + Fh[i][1] * S[1][j];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 2; ++l) {
      double c = 0.0;
      for (int j = 0; j < 2; ++j) c += P[l][j] * gradN[k][j];
      for (int i = 0; i < 3; ++i) f[k][i] -= A0 * c * e[l][i];
    }
  return 0;
}

double orc_membrane_element_energy(const double X[3][3], const double x[3][3], int law, double mu, double mu2) {
  double gradN[3][2], A0, e[2][3];
  if (tri_reference(X, gradN, &A0)) return NAN;
  if (tri_frame(x[0], x[1], x[2], e[0], e[1])) return NAN;
  double Fh[2][2];
  tri_defgrad(x, gradN, (const double(*)[3])e, Fh);
  double C[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) C[i][j] = Fh[0][i] * Fh[0][j] + Fh[1][i] * Fh[1][j];
  return A0 * orc_membrane_W(law, mu, mu2, C[0][0] + C[1][1], C[0][0] * C[1][1] - C[0][1] * C[1][0]);
}

/* ------------------------------------------------------------ tetrahedral element (Sec. II.B) */
/* Shape-function gradients of a linear tetrahedron: rows of D0^-1 for nodes
 * 1..3, minus their sum for node 0.  Returns the reference volume. */
static double tet_reference(const double X[4][3], double gradN[4][3]) {
  double D0[3][3], Di[3][3];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) D0[i][a] = X[a + 1][i] - X[0][i];
  double det = inv3(D0, Di);
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) gradN[a + 1][j] = Di[a][j];
  for (int j = 0; j < 3; ++j) gradN[0][j] = -(gradN[1][j] + gradN[2][j] + gradN[3][j]);
  return det / 6.0;
}

/* F_ij = sum_k x_i,k dN_k/dX_j, with positions relative to node 0 (the gradients sum to zero). */
static void tet_defgrad(const double x[4][3], const double gradN[4][3], double F[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 1; k < 4; ++k) s += (x[k][i] - x[0][i]) * gradN[k][j];
      F[i][j] = s;
    }
}

/* Tet element: f[k][i] = -V0 P_ij dN_k/dX_j with
 * P = F S,  S = lam/2 (J^2 - 1) F^-1 F^-T + mu (I - F^-1 F^-T).
 * Returns 1 (and zero forces) for a degenerate reference or J <= 0. */
int orc_tet_element(const double X[4][3], const double x[4][3], double mu, double lam, double f[4][3]) {
  memset(f, 0, 12 * sizeof(double));
  double gradN[4][3];
  double V0 = tet_reference(X, gradN);
  if (!(V0 > 0.0)) return 1;
  double F[3][3], Fi[3][3];
  tet_defgrad(x, gradN, F);
  double J = inv3(F, Fi);
  if (!(J > 0.0)) return 1;
  double Cinv[3][3]; /* F^-1 F^-T */
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) Cinv[k][j] = Fi[k][0] * Fi[j][0] + Fi[k][1] * Fi[j][1] + Fi[k][2] * Fi[j][2];
  double S[3][3];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) S[k][j] = 0.5 * lam * (J * J - 1.0) * Cinv[k][j] + mu * ((k == j) - Cinv[k][j]);
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i][j] = F[i][0] * S[0][j] + F[i][1] * S[1][j] + F[i][2] * S[2][j];
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 3; ++i) f[k][i] = -V0 * (P[i][0] * gradN[k][0] + P[i][1] * gradN[k][1] + P[i][2] * gradN[k][2]);
  return 0;
}

double orc_tet_element_energy(const double X[4][3], const double x[4][3], double mu, double lam) {
  double gradN[4][3];
  double V0 = tet_reference(X, gradN);
  double F[3][3];
  tet_defgrad(x, gradN, F);
  double J = det3(F);
  double I1 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I1 += F[i][j] * F[i][j];
  return V0 * orc_solid_W(mu, lam, I1, J * J);
}

/* ------------------------------------------------------------ bending (Sec. II.B) */
/* Discrete differential-geometry quantities per node of one closed triangulated
 * surface (Meyer et al. 2003):
 *   A[k]   mixed Voronoi area,
 *   K[k]   sum_j (cot a_kj + cot b_kj)(x_k - x_j)   (not yet divided by 2 A_k),
 *   th[k]  sum of the triangle angles at k,
 *   N[k]   sum of the face area vectors around k.
 * READING: the paper names Sinha & Graham's operators without stating them;
 * these are the published operators behind that choice. */
static void tri_angles_cot(const double p[3][3], double theta[3], double cotv[3]) {
  for (int v = 0; v < 3; ++v) {
    double u[3], w[3], c[3];
    sub3(p[(v + 1) % 3], p[v], u);
    sub3(p[(v + 2) % 3], p[v], w);
    cross3(u, w, c);
    double s = norm3(c), d = dot3(u, w);
    theta[v] = atan2(s, d);
    cotv[v] = d / s;
  }
}

int orc_curvature(const double* x, long stride, int node_begin, int node_end, const int* tri, long tri_stride,
                  int tri_begin, int tri_end, double* A, double* kH, double* kG, double* nrm /*[3][n_local]*/) {
  int n = node_end - node_begin;
  double* K = (double*)calloc((size_t)3 * n, sizeof(double));
  double* th = (double*)calloc((size_t)n, sizeof(double));
  for (int i = 0; i < n; ++i) A[i] = 0.0;
  for (int i = 0; i < 3 * n; ++i) nrm[i] = 0.0;
  for (int t = tri_begin; t < tri_end; ++t) {
    int id[3] = {tri[t] - node_begin, tri[tri_stride + t] - node_begin, tri[2 * tri_stride + t] - node_begin};
    double p[3][3], theta[3], cotv[3];
    for (int v = 0; v < 3; ++v) pos(x, stride, id[v] + node_begin, p[v]);
    tri_angles_cot(p, theta, cotv);
    double e1[3], e2[3], fa[3];
    sub3(p[1], p[0], e1);
    sub3(p[2], p[0], e2);
    cross3(e1, e2, fa);
    double area = 0.5 * norm3(fa);
    int obtuse = -1;
    for (int v = 0; v < 3; ++v)
      if (theta[v] > M_PI / 2) obtuse = v;
    for (int v = 0; v < 3; ++v) {
      int a = (v + 1) % 3, b = (v + 2) % 3; /* edge (v,a) is opposite b, edge (v,b) opposite a */
      double dva[3], dvb[3];
      sub3(p[v], p[a], dva);
      sub3(p[v], p[b], dvb);
      for (int i = 0; i < 3; ++i) K[3 * id[v] + i] += cotv[b] * dva[i] + cotv[a] * dvb[i];
      th[id[v]] += theta[v];
      for (int i = 0; i < 3; ++i) nrm[i * n + id[v]] += 0.5 * fa[i];
      if (obtuse < 0)
        A[id[v]] += 0.125 * (dot3(dvb, dvb) * cotv[a] + dot3(dva, dva) * cotv[b]);
      else
        A[id[v]] += (obtuse == v) ? 0.5 * area : 0.25 * area;
    }
  }
  for (int k = 0; k < n; ++k) {
    double nv[3] = {nrm[k], nrm[n + k], nrm[2 * n + k]};
    double ln = norm3(nv);
    for (int i = 0; i < 3; ++i) nrm[i * n + k] = nv[i] / ln;
    double Kk[3] = {K[3 * k] / (2.0 * A[k]), K[3 * k + 1] / (2.0 * A[k]), K[3 * k + 2] / (2.0 * A[k])};
    kH[k] = 0.5 * (Kk[0] * nrm[k] + Kk[1] * nrm[n + k] + Kk[2] * nrm[2 * n + k]);
    kG[k] = (2.0 * M_PI - th[k]) / A[k];
  }
  free(K);
  free(th);
  return 0;
}

/* Cotangent surface Laplacian (1/2A_k) sum_j (cot a + cot b)(g_j - g_k) of a nodal field g. */
int orc_laplacian(const double* x, long stride, int node_begin, int node_end, const int* tri, long tri_stride,
                  int tri_begin, int tri_end, const double* A, const double* g, double* out) {
  int n = node_end - node_begin;
  for (int i = 0; i < n; ++i) out[i] = 0.0;
  for (int t = tri_begin; t < tri_end; ++t) {
    int id[3] = {tri[t] - node_begin, tri[tri_stride + t] - node_begin, tri[2 * tri_stride + t] - node_begin};
    double p[3][3], theta[3], cotv[3];
    for (int v = 0; v < 3; ++v) pos(x, stride, id[v] + node_begin, p[v]);
    tri_angles_cot(p, theta, cotv);
    for (int v = 0; v < 3; ++v) {
      int a = (v + 1) % 3, b = (v + 2) % 3;
      out[id[v]] += cotv[b] * (g[id[a]] - g[id[v]]) + cotv[a] * (g[id[b]] - g[id[v]]);
    }
  }
  for (int k = 0; k < n; ++k) out[k] /= 2.0 * A[k];
  return 0;
}

/* Helfrich bending force of one membrane particle, added to F:
 * F_k = 2 kb [ Lap(kH - kH0) + 2 (kH - kH0)(kH^2 - kG + kH0 kH) ] n_k A_k,
 * READING: kH0 = -c0/2 so that the energy density kb/2 (2 kH + c0)^2 equals
 * 2 kb (kH - kH0)^2; kH = +1/R on a sphere with outward normals. */
int orc_bending(const double* x, long stride, int node_begin, int node_end, const int* tri, long tri_stride,
                int tri_begin, int tri_end, double kb, double c0, double* F /*[3][stride], accumulated*/) {
  int n = node_end - node_begin;
  double* A = (double*)malloc(sizeof(double) * n);
  double* kH = (double*)malloc(sizeof(double) * n);
  double* kG = (double*)malloc(sizeof(double) * n);
  double* nr = (double*)malloc(sizeof(double) * 3 * n);
  double* g = (double*)malloc(sizeof(double) * n);
  double* lap = (double*)malloc(sizeof(double) * n);
  double kH0 = -0.5 * c0;
  orc_curvature(x, stride, node_begin, node_end, tri, tri_stride, tri_begin, tri_end, A, kH, kG, nr);
  for (int k = 0; k < n; ++k) g[k] = kH[k] - kH0;
  orc_laplacian(x, stride, node_begin, node_end, tri, tri_stride, tri_begin, tri_end, A, g, lap);
  for (int k = 0; k < n; ++k) {
    double s = 2.0 * kb * (lap[k] + 2.0 * g[k] * (kH[k] * kH[k] - kG[k] + kH0 * kH[k])) * A[k];
    for (int i = 0; i < 3; ++i) F[i * stride + node_begin + k] += s * nr[i * n + k];
  }
  free(A);
  free(kH);
  free(kG);
  free(nr);
  free(g);
  free(lap);
  return 0;
}

/* ------------------------------------------------------------ all particle forces */
/* Internal nodal forces of every particle (elastic always, bending when kb != 0
 * and do_bending != 0), overwriting F [3][n_nodes].
 * counts[0] += elements that were degenerate or inverted (contribute 0),
 * counts[1] += non-finite nodal force components. */
int orc_forces(int n_nodes, const double* X, const double* x, int n_particles, const int* node_start,
               const int* tri_start, const int* tet_start, const int* tri, int n_tri, const int* tet, int n_tet,
               const int* law, const double* mu, const double* mu2, const double* kb, const double* c0,
               int do_elastic, int do_bending, double* F, long long* counts) {
  memset(F, 0, sizeof(double) * 3 * (size_t)n_nodes);
  for (int p = 0; p < n_particles; ++p) {
    if (do_elastic) {
      for (int t = tri_start[p]; t < tri_start[p + 1]; ++t) {
        double Xe[3][3], xe[3][3], f[3][3];
        int id[3] = {tri[t], tri[n_tri + t], tri[2 * n_tri + t]};
        for (int v = 0; v < 3; ++v) {
          pos(X, n_nodes, id[v], Xe[v]);
          pos(x, n_nodes, id[v], xe[v]);
        }
        if (orc_membrane_element(Xe, xe, law[p], mu[p], mu2[p], f)) counts[0]++;
        for (int v = 0; v < 3; ++v)
          for (int i = 0; i < 3; ++i) F[i * (size_t)n_nodes + id[v]] += f[v][i];
      }
      for (int t = tet_start[p]; t < tet_start[p + 1]; ++t) {
        double Xe[4][3], xe[4][3], f[4][3];
        int id[4] = {tet[t], tet[n_tet + t], tet[2 * n_tet + t], tet[3 * n_tet + t]};
        for (int v = 0; v < 4; ++v) {
          pos(X, n_nodes, id[v], Xe[v]);
          pos(x, n_nodes, id[v], xe[v]);
        }
        if (orc_tet_element(Xe, xe, mu[p], mu2[p], f)) counts[0]++;
        for (int v = 0; v < 4; ++v)
          for (int i = 0; i < 3; ++i) F[i * (size_t)n_nodes + id[v]] += f[v][i];
      }
    }
    if (do_bending && kb[p] != 0.0 && tri_start[p + 1] > tri_start[p])
      orc_bending(x, n_nodes, node_start[p], node_start[p + 1], tri, n_tri, tri_start[p], tri_start[p + 1], kb[p],
                  c0[p], F);
  }
  for (size_t i = 0; i < 3 * (size_t)n_nodes; ++i)
    if (!isfinite(F[i])) counts[1]++;
  return 0;
}

/* Total elastic energy of each particle (membrane or solid), for gradient checks. */
int orc_energy(int n_nodes, const double* X, const double* x, int n_particles, const int* tri_start,
               const int* tet_start, const int* tri, int n_tri, const int* tet, int n_tet, const int* law,
               const double* mu, const double* mu2, double* E) {
  for (int p = 0; p < n_particles; ++p) {
    double s = 0.0;
    for (int t = tri_start[p]; t < tri_start[p + 1]; ++t) {
      double Xe[3][3], xe[3][3];
      int id[3] = {tri[t], tri[n_tri + t], tri[2 * n_tri + t]};
      for (int v = 0; v < 3; ++v) {
        pos(X, n_nodes, id[v], Xe[v]);
        pos(x, n_nodes, id[v], xe[v]);
      }
      s += orc_membrane_element_energy(Xe, xe, law[p], mu[p], mu2[p]);
    }
    for (int t = tet_start[p]; t < tet_start[p + 1]; ++t) {
      double Xe[4][3], xe[4][3];
      int id[4] = {tet[t], tet[n_tet + t], tet[2 * n_tet + t], tet[3 * n_tet + t]};
      for (int v = 0; v < 4; ++v) {
        pos(X, n_nodes, id[v], Xe[v]);
        pos(x, n_nodes, id[v], xe[v]);
      }
      s += orc_tet_element_energy(Xe, xe, mu[p], mu2[p]);
    }
    E[p] = s;
  }
  return 0;
}

/* ------------------------------------------------------------ per-particle reductions */
/* red[p] = {V, A, cx, cy, cz}.  Membranes: V by the three-term face sum
 * (Sec. II.E volume formula), A = sum of triangle areas, c = volume centroid
 * from the cone of every face to the coordinate origin.  Solids: V = sum of
 * tetrahedron volumes, c = volume-weighted tetrahedron centroids, A = 0. */
int orc_reduce(int n_nodes, const double* x, int n_particles, const int* tri_start, const int* tet_start,
               const int* tri, int n_tri, const int* tet, int n_tet, double* red) {
  for (int p = 0; p < n_particles; ++p) {
    double V = 0.0, A = 0.0, m[3] = {0, 0, 0};
    for (int t = tri_start[p]; t < tri_start[p + 1]; ++t) {
      double a[3], b[3], c[3], bc[3], ca[3], ab[3];
      pos(x, n_nodes, tri[t], a);
      pos(x, n_nodes, tri[n_tri + t], b);
      pos(x, n_nodes, tri[2 * n_tri + t], c);
      cross3(b, c, bc);
      cross3(c, a, ca);
      cross3(a, b, ab);
      double three = dot3(a, bc) + dot3(b, ca) + dot3(c, ab);
      V += three / 18.0;
      double cone = three / 18.0; /* volume of the tetrahedron (0, a, b, c) */
      for (int i = 0; i < 3; ++i) m[i] += cone * (a[i] + b[i] + c[i]) / 4.0;
      double u[3], w[3], n[3];
      sub3(b, a, u);
      sub3(c, a, w);
      cross3(u, w, n);
      A += 0.5 * norm3(n);
    }
    for (int t = tet_start[p]; t < tet_start[p + 1]; ++t) {
      double q[4][3], D[3][3];
      for (int v = 0; v < 4; ++v) pos(x, n_nodes, tet[v * n_tet + t], q[v]);
      for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) D[i][a] = q[a + 1][i] - q[0][i];
      double vol = det3(D) / 6.0;
      V += vol;
      for (int i = 0; i < 3; ++i) m[i] += vol * (q[0][i] + q[1][i] + q[2][i] + q[3][i]) / 4.0;
    }
    red[5 * p + 0] = V;
    red[5 * p + 1] = A;
    for (int i = 0; i < 3; ++i) red[5 * p + 2 + i] = m[i] / V;
  }
  return 0;
}

/* ------------------------------------------------------------ MLS transfer (Sec. II.C) */
/* Cubic-spline weight.  READING: the inner piece is printed as 2/3 - 4r + 4r^3,
 * which is negative at r = 1/2 and discontinuous with the outer piece; the
 * cubic B-spline 2/3 - 4r^2 + 4r^3 joins it with equal value, slope and
 * curvature.  The outer piece 4/3 - 4r + 4r^2 - 4/3 r^3 is (4/3)(1 - r)^3. */
double orc_weight(double r) {
  if (r > 1.0) return 0.0;
  if (r <= 0.5) return 2.0 / 3.0 - 4.0 * r * r + 4.0 * r * r * r;
  double s = 1.0 - r;
  return 4.0 / 3.0 * s * s * s;
}

/* Solve the 4x4 system A z = b by Gaussian elimination with partial pivoting. */
static int solve4(double A[4][4], double b[4], double z[4]) {
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (A[piv][c] == 0.0) return 1;
    if (piv != c) {
      for (int j = 0; j < 4; ++j) {
        double t = A[c][j];
        A[c][j] = A[piv][j];
        A[piv][j] = t;
      }
      double t = b[c];
      b[c] = b[piv];
      b[piv] = t;
    }
    for (int r = c + 1; r < 4; ++r) {
      double m = A[r][c] / A[c][c];
      for (int j = c; j < 4; ++j) A[r][j] -= m * A[c][j];
      b[r] -= m * b[c];
    }
  }
  for (int r = 3; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < 4; ++j) s -= A[r][j] * z[j];
    z[r] = s / A[r][r];
  }
  return 0;
}

/* Lattice offsets in cells: rows 0..2 the MAC lattices of the three velocity
 * components, row 3 the cell centres, where the six components of the
 * conformation tensor live.  READING: the paper's grid is collocated; on this
 * staggered grid the conformation, a cell quantity like the pressure, sits at
 * the cell centres. */
static const double ORC_STAGGER[4][3] = {{0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}, {0.5, 0.5, 0.5}};

/* MLS weights of one Lagrangian point p on lattice `comp` of a periodic box
 * (n cells per axis, spacing h, lattice nodes at origin + (i + s) h with s the
 * lattice's offset: velocity component comp = 0..2, cell centres comp = 3).
 *
 * Stencil: the lattice node nearest to p and the 26 nodes sharing a cell
 * with it.  READING (nearest-node rule, bit-specified so that every
 * implementation selects the same stencil): q = p - origin,
 * t = fma(q, 1/h, -s), base = floor(t + 1/2) per axis.
 *
 * Weights: minimise sum_J W_J (p(X_J)^T Z - q_J)^2 with linear basis
 * p(X) = (1, X) and W_J = W(|X_J| / rho); phi = p(x_k)^T A^-1 B.
 * READING: the support rho is the largest distance from a node to its 26
 * neighbours, sqrt(3) h.  READING: the basis is written about x_k itself
 * (X_J = x_J - x_k); the moving-least-squares weights do not change under a
 * shift of the basis origin, and p(x_k) becomes (1, 0, 0, 0).
 *
 * Output: base[3] (unwrapped lattice index of the nearest node) and phi[27],
 * ordered m = (mx, my, mz) in {-1,0,1}^3 with mx fastest. */
int orc_mls(const double p[3], const int n[3], double h, const double origin[3], int comp, int64_t base[3],
            double phi[27]) {
  (void)n;
  double inv_h = 1.0 / h, t[3];
  for (int a = 0; a < 3; ++a) {
    double q = p[a] - origin[a];
    t[a] = fma(q, inv_h, -ORC_STAGGER[comp][a]);
    base[a] = (int64_t)floor(t[a] + 0.5);
  }
  double rho = sqrt(3.0) * h;
  double A[4][4] = {{0}}, B[27][4], Wv[27];
  for (int mz = -1; mz <= 1; ++mz)
    for (int my = -1; my <= 1; ++my)
      for (int mx = -1; mx <= 1; ++mx) {
        int idx = (mz + 1) * 9 + (my + 1) * 3 + (mx + 1);
        int64_t m[3] = {mx, my, mz};
        double XJ[3];
        for (int a = 0; a < 3; ++a) {
          double xJ = origin[a] + ((double)(base[a] + m[a]) + ORC_STAGGER[comp][a]) * h;
          XJ[a] = xJ - p[a];
        }
        double W = orc_weight(norm3(XJ) / rho);
        double pv[4] = {1.0, XJ[0], XJ[1], XJ[2]};
        Wv[idx] = W;
        for (int i = 0; i < 4; ++i) {
          B[idx][i] = W * pv[i];
          for (int j = 0; j < 4; ++j) A[i][j] += W * pv[i] * pv[j];
        }
      }
  double rhs[4] = {1.0, 0.0, 0.0, 0.0}, z[4];
  if (solve4(A, rhs, z)) return 1;
  for (int J = 0; J < 27; ++J) phi[J] = z[0] * B[J][0] + z[1] * B[J][1] + z[2] * B[J][2] + z[3] * B[J][3];
  (void)Wv;
  return 0;
}

static int64_t wrap(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

/* Spreading F_J = sum_k phi_J(x_J - x_k) F_k on every component lattice
 * (Sec. II.C spreading operator; step 2 of the algorithm).  Overwrites grid
 * [3][total_cells].  READING: the result is the nodal force itself (its sum
 * over the grid equals the Lagrangian total); dividing by h^3 for a density
 * is left to the caller. */
int orc_spread(int n_points, const double* x, const double* F, const int* box_of_point, const int* bn,
               const double* bh, const double* borig, const int64_t* cell_off, int64_t total_cells, double* grid) {
  memset(grid, 0, sizeof(double) * 3 * (size_t)total_cells);
  int bad = 0;
  for (int k = 0; k < n_points; ++k) {
    int b = box_of_point[k];
    const int* n = bn + 3 * b;
    double p[3] = {x[k], x[n_points + k], x[2 * (size_t)n_points + k]};
    for (int d = 0; d < 3; ++d) {
      int64_t base[3];
      double phi[27];
      if (orc_mls(p, n, bh[b], borig + 3 * b, d, base, phi)) {
        bad++;
        continue;
      }
      for (int mz = -1; mz <= 1; ++mz)
        for (int my = -1; my <= 1; ++my)
          for (int mx = -1; mx <= 1; ++mx) {
            int64_t i = wrap(base[0] + mx, n[0]), j = wrap(base[1] + my, n[1]), kk = wrap(base[2] + mz, n[2]);
            int64_t cell = cell_off[b] + (kk * n[1] + j) * n[0] + i;
            grid[d * (size_t)total_cells + cell] += phi[(mz + 1) * 9 + (my + 1) * 3 + (mx + 1)] * F[d * (size_t)n_points + k];
          }
    }
  }
  return bad;
}

/* Interpolation v_k = sum_J phi_J(x_J - x_k) v_J per component (Sec. II.C;
 * step 4 of the algorithm).  Overwrites v [3][n_points]. */
int orc_interp(int n_points, const double* x, const int* box_of_point, const int* bn, const double* bh,
               const double* borig, const int64_t* cell_off, int64_t total_cells, const double* grid, double* v) {
  int bad = 0;
  for (int k = 0; k < n_points; ++k) {
    int b = box_of_point[k];
    const int* n = bn + 3 * b;
    double p[3] = {x[k], x[n_points + k], x[2 * (size_t)n_points + k]};
    for (int d = 0; d < 3; ++d) {
      int64_t base[3];
      double phi[27], s = 0.0;
      if (orc_mls(p, n, bh[b], borig + 3 * b, d, base, phi)) {
        bad++;
        v[d * (size_t)n_points + k] = NAN;
        continue;
      }
      for (int mz = -1; mz <= 1; ++mz)
        for (int my = -1; my <= 1; ++my)
          for (int mx = -1; mx <= 1; ++mx) {
            int64_t i = wrap(base[0] + mx, n[0]), j = wrap(base[1] + my, n[1]), kk = wrap(base[2] + mz, n[2]);
            int64_t cell = cell_off[b] + (kk * n[1] + j) * n[0] + i;
            s += phi[(mz + 1) * 9 + (my + 1) * 3 + (mx + 1)] * grid[d * (size_t)total_cells + cell];
          }
      v[d * (size_t)n_points + k] = s;
    }
  }
  return bad;
}

/* ------------------------------------------------------------ membrane volume conservation (Sec. II.E) */
/* For every membrane particle: the node displacements dx_I = L v_I with
 * v_I = alpha_I = -(1/12) sum over the faces at I of the cross product of the
 * face's other two nodes taken in the face's cyclic order (I1 -> x_I2 x x_I3,
 * I2 -> x_I3 x x_I1, I3 -> x_I1 x x_I2), and L a root of
 * A L^3 + B L^2 + C L + D = 0 with the printed coefficients:
 *   A = 1/18 sum [v1.(v2 x v3) + v2.(v3 x v1) + v3.(v1 x v2)],
 *   B = 1/6  sum [x1.(v2 x v3) + x2.(v3 x v1) + x3.(v1 x v2)],
 *   C = 1/6  sum [v1.(x2 x x3) + v2.(x3 x x1) + v3.(x1 x x2)],
 *   D = V(x) - V0, V by the three-term face formula,
 * so that V(x + L v) = V0 exactly.  READING: the paper does not say which
 * root; the one of smallest magnitude is the smallest correction, i.e. the
 * minimiser of the cost function.  It is found by Newton's iteration from
 * L = 0, which converges to it in the method's regime (|D| small against
 * C^2 / |B|: relative volume drifts of 1e-4 per step); the tests compare it
 * with all three roots.  Solids (tetrahedral particles) are copied unchanged
 * and get L = 0.  x, x_out [3][n_nodes]; V0, lam [n_particles].  Returns the
 * number of membrane particles whose iteration did not converge. */
int orc_volume_correct(int n_nodes, const double* x, int n_particles, const int* node_start, const int* tri_start,
                       const int* tri, int n_tri, const int* law, const double* V0, double* x_out, double* lam) {
  memcpy(x_out, x, sizeof(double) * 3 * (size_t)n_nodes);
  int bad = 0;
  for (int p = 0; p < n_particles; ++p) {
    lam[p] = 0.0;
    if (law[p] == ORC_LAW_TET_NEOHOOKE || tri_start[p + 1] == tri_start[p]) continue;
    const int n0 = node_start[p], nn = node_start[p + 1] - n0;
    double* v = calloc(3 * (size_t)nn, sizeof(double));
    for (int t = tri_start[p]; t < tri_start[p + 1]; ++t) {
      const int id[3] = {tri[t], tri[n_tri + t], tri[2 * n_tri + t]};
      double q[3][3];
      for (int k = 0; k < 3; ++k) pos(x, n_nodes, id[k], q[k]);
      for (int k = 0; k < 3; ++k) {
        double c[3];
        cross3(q[(k + 1) % 3], q[(k + 2) % 3], c);
        for (int i = 0; i < 3; ++i) v[3 * (id[k] - n0) + i] -= c[i] / 12.0;
      }
    }
    double A = 0.0, B = 0.0, C = 0.0, V = 0.0;
    for (int t = tri_start[p]; t < tri_start[p + 1]; ++t) {
      const int id[3] = {tri[t], tri[n_tri + t], tri[2 * n_tri + t]};
      double q[3][3], w[3][3];
      for (int k = 0; k < 3; ++k) {
        pos(x, n_nodes, id[k], q[k]);
        for (int i = 0; i < 3; ++i) w[k][i] = v[3 * (id[k] - n0) + i];
      }
      for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        double c[3];
        cross3(w[k1], w[k2], c);
        A += dot3(w[k], c) / 18.0;
        B += dot3(q[k], c) / 6.0;
        cross3(q[k1], q[k2], c);
        C += dot3(w[k], c) / 6.0;
        V += dot3(q[k], c) / 18.0;
      }
    }
    const double D = V - V0[p];
    double L = 0.0;
    int it = 0, done = 0;
    for (; it < 100 && !done; ++it) {
      const double f = ((A * L + B) * L + C) * L + D;
      const double df = (3.0 * A * L + 2.0 * B) * L + C;
      const double step = f / df;
      L -= step;
      done = fabs(step) <= 1e-15 * fabs(L) || f == 0.0;
    }
    if (!done || !isfinite(L)) bad++;
    lam[p] = L;
    for (int k = 0; k < nn; ++k)
      for (int i = 0; i < 3; ++i) x_out[(size_t)i * n_nodes + n0 + k] = x[(size_t)i * n_nodes + n0 + k] + L * v[3 * k + i];
    free(v);
  }
  return bad;
}

/* ------------------------------------------------------------ Lagrangian update (Sec. III.A, last step) */
/* Second-order Adams-Bashforth update of the node positions with the
 * interpolated velocities of this step and the previous one:
 *   x^{n+1} = x^n + dt (3/2 v^n - 1/2 v^{n-1}).
 * READING: the paper does not say how the first step starts; with no previous
 * velocity (v_prev NULL) it is the forward Euler step x^n + dt v^n.  All arrays
 * [3][n_nodes]. */
void orc_advance(int n_nodes, const double* x, const double* v, const double* v_prev, double dt, double* x_out) {
  for (long i = 0; i < 3L * n_nodes; ++i) {
    const double rate = v_prev ? 1.5 * v[i] - 0.5 * v_prev[i] : v[i];
    x_out[i] = x[i] + dt * rate;
  }
}

/* ------------------------------------------------------------ conformation interpolation (Sec. III.A step 4) */
/* C_k = sum_J phi_J(x_J - x_k) C_J for each of ncomp cell-centred fields
 * (the six components of the symmetric conformation tensor, in the order
 * xx, yy, zz, xy, xz, yz), with the MLS weights of the cell-centre lattice.
 * grid [ncomp][total_cells], out [ncomp][n_points]. */
int orc_interp_cells(int n_points, const double* x, const int* box_of_point, const int* bn, const double* bh,
                     const double* borig, const int64_t* cell_off, int64_t total_cells, int ncomp,
                     const double* grid, double* out) {
  int bad = 0;
  for (int k = 0; k < n_points; ++k) {
    int b = box_of_point[k];
    const int* n = bn + 3 * b;
    double p[3] = {x[k], x[n_points + k], x[2 * (size_t)n_points + k]};
    int64_t base[3];
    double phi[27];
    const int singular = orc_mls(p, n, bh[b], borig + 3 * b, 3, base, phi);
    bad += singular;
    for (int c = 0; c < ncomp; ++c) {
      double s = 0.0;
      for (int mz = -1; mz <= 1; ++mz)
        for (int my = -1; my <= 1; ++my)
          for (int mx = -1; mx <= 1; ++mx) {
            int64_t i = wrap(base[0] + mx, n[0]), j = wrap(base[1] + my, n[1]), kk = wrap(base[2] + mz, n[2]);
            int64_t cell = cell_off[b] + (kk * n[1] + j) * n[0] + i;
            s += phi[(mz + 1) * 9 + (my + 1) * 3 + (mx + 1)] * grid[c * (size_t)total_cells + cell];
          }
      out[c * (size_t)n_points + k] = singular ? NAN : s;
    }
  }
  return bad;
}

/* ------------------------------------------------------------ fluid-stress forces on solids (Sec. II.B) */
/* The fluid part of eq. FEM for one tetrahedron, split into its Newtonian and
 * polymer parts:
 *   L      = sum_k u_k (x) grad N_k F^-1               (velocity gradient),
 *   P^fN   = eta J (L + L^T) F^-T,
 *   P^fP   = J G (1/4 sum_k (C_k - I)) F^-T,
 *   f_k    = +V0 (P^fN + P^fP) grad N_k,
 * the sign of the fluid stress in F_k = -V0 (P^s - P^f) grad N_k.  eta is the
 * Newtonian viscosity and G the polymer modulus eta_p / lambda (written
 * eta (1 - beta) / lambda in the paper, with eta the total viscosity there).
 * C [4][6] per node xx, yy, zz, xy, xz, yz, or NULL for a Newtonian fluid.
 * Returns 1 (and zero forces) for a degenerate reference or J <= 0. */
int orc_tet_fluid_element(const double X[4][3], const double x[4][3], const double u[4][3], const double* C,
                          double eta, double G, double f[4][3]) {
  memset(f, 0, 12 * sizeof(double));
  double gradN[4][3];
  const double V0 = tet_reference(X, gradN);
  if (!(V0 > 0.0)) return 1;
  double F[3][3], Fi[3][3];
  tet_defgrad(x, gradN, F);
  const double J = inv3(F, Fi);
  if (!(J > 0.0)) return 1;
  double L[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 3; ++l) s += u[k][i] * gradN[k][l] * Fi[l][j];
      L[i][j] = s;
    }
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += (L[i][k] + L[k][i]) * Fi[j][k]; /* (L + L^T) F^-T */
      P[i][j] = eta * J * s;
    }
  if (C) {
    static const int sym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    double Cb[3][3];
    for (int i = 0; i < 3; ++i)
      for (int l = 0; l < 3; ++l) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += (C[6 * k + sym[i][l]] - (i == l)) / 4.0;
        Cb[i][l] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += Cb[i][l] * Fi[j][l];
        P[i][j] += J * G * s;
      }
  }
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 3; ++i) f[k][i] = V0 * (P[i][0] * gradN[k][0] + P[i][1] * gradN[k][1] + P[i][2] * gradN[k][2]);
  return 0;
}

/* Fluid-stress nodal forces of every solid (sum of the element forces over its
 * tetrahedra); membranes get none.  u [3][n_nodes], C [6][n_nodes] or NULL,
 * f [3][n_nodes] overwritten.  Returns the number of skipped elements. */
int orc_fluid_forces(int n_nodes, const double* X, const double* x, const double* u, const double* C, int n_particles,
                     const int* tet_start, const int* tet, int n_tet, double eta, double G, double* f) {
  memset(f, 0, sizeof(double) * 3 * (size_t)n_nodes);
  int bad = 0;
  for (int p = 0; p < n_particles; ++p)
    for (int t = tet_start[p]; t < tet_start[p + 1]; ++t) {
      int id[4];
      double Xe[4][3], xe[4][3], ue[4][3], Ce[24], fe[4][3];
      for (int v = 0; v < 4; ++v) {
        id[v] = tet[v * n_tet + t];
        pos(X, n_nodes, id[v], Xe[v]);
        pos(x, n_nodes, id[v], xe[v]);
        pos(u, n_nodes, id[v], ue[v]);
        if (C)
          for (int c = 0; c < 6; ++c) Ce[6 * v + c] = C[c * (size_t)n_nodes + id[v]];
      }
      bad += orc_tet_fluid_element(Xe, xe, ue, C ? Ce : NULL, eta, G, fe);
      for (int v = 0; v < 4; ++v)
        for (int i = 0; i < 3; ++i) f[i * (size_t)n_nodes + id[v]] += fe[v][i];
    }
  return bad;
}

/* ------------------------------------------------------------ node-face anti-sticking (Sec. III.B) */
/* Closest point on the segment [a, b] to p. */
static void seg_closest(const double p[3], const double a[3], const double b[3], double out[3]) {
  double ab[3], ap[3];
  sub3(b, a, ab);
  sub3(p, a, ap);
  const double L2 = dot3(ab, ab);
  double t = L2 > 0.0 ? dot3(ap, ab) / L2 : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  for (int i = 0; i < 3; ++i) out[i] = a[i] + t * ab[i];
}

/* Closest point on triangle (a, b, c) to p: the projection of p on the
 * triangle's plane when it lies inside the triangle (on the inner side of all
 * three edges), otherwise the nearest of the closest points of the three edges
 * (first of ab, bc, ca on ties).  Returns 1 if the closest point is the plane
 * projection. */
int orc_point_triangle(const double p[3], const double a[3], const double b[3], const double c[3], double out[3]) {
  double ab[3], ac[3], n[3], ap[3];
  sub3(b, a, ab);
  sub3(c, a, ac);
  cross3(ab, ac, n);
  sub3(p, a, ap);
  const double n2 = dot3(n, n);
  if (n2 > 0.0) {
    const double s = dot3(ap, n) / n2;
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = p[i] - s * n[i];
    const double* v[3] = {a, b, c};
    int inside = 1;
    for (int e = 0; e < 3; ++e) {
      double ed[3], vq[3], cr[3];
      sub3(v[(e + 1) % 3], v[e], ed);
      sub3(q, v[e], vq);
      cross3(ed, vq, cr);
      if (dot3(cr, n) < 0.0) inside = 0;
    }
    if (inside) {
      for (int i = 0; i < 3; ++i) out[i] = q[i];
      return 1;
    }
  }
  const double* v[3] = {a, b, c};
  double best = INFINITY;
  for (int e = 0; e < 3; ++e) {
    double q[3], d[3];
    seg_closest(p, v[e], v[(e + 1) % 3], q);
    sub3(q, p, d);
    const double dd = dot3(d, d);
    if (dd < best) {
      best = dd;
      for (int i = 0; i < 3; ++i) out[i] = q[i];
    }
  }
  return 0;
}

static int cmp_face_key(const void* pa, const void* pb) {
  const int64_t* a = (const int64_t*)pa;
  const int64_t* b = (const int64_t*)pb;
  return a[0] < b[0] ? -1 : (a[0] > b[0] ? 1 : (a[1] < b[1] ? -1 : (a[1] > b[1])));
}

/* Boundary faces of the tetrahedral meshes of the solids: the faces that
 * belong to one tetrahedron only, oriented outward (away from the
 * tetrahedron's fourth node, in the reference configuration X), listed in the
 * order of (tetrahedron, face opposite node j = 0..3).  READING: the paper's
 * node-face check needs a surface for every particle; a solid's surface is its
 * mesh boundary.  out [3][cap] node ids, part [cap] owning particle; returns
 * the number of faces (at most cap) or -1 if cap is too small. */
int orc_boundary_faces(int n_nodes, const double* X, int n_particles, const int* tet_start, const int* tet, int n_tet,
                       int cap, int* out, int* part) {
  int nf = 0;
  for (int p = 0; p < n_particles; ++p) {
    const int t0 = tet_start[p], nt = tet_start[p + 1] - t0;
    if (nt == 0) continue;
    int64_t* keys = malloc(sizeof(int64_t) * 2 * 4 * (size_t)nt); /* (sorted-triple key, 4 t + j) */
    for (int t = 0; t < nt; ++t)
      for (int j = 0; j < 4; ++j) {
        int v[3], m = 0;
        for (int q = 0; q < 4; ++q)
          if (q != j) v[m++] = tet[q * n_tet + t0 + t];
        for (int a = 0; a < 2; ++a) /* sort the triple */
          for (int b = 0; b < 2 - a; ++b)
            if (v[b] > v[b + 1]) {
              const int s = v[b];
              v[b] = v[b + 1];
              v[b + 1] = s;
            }
        keys[2 * (4 * t + j)] = ((int64_t)v[0] << 42) | ((int64_t)v[1] << 21) | (int64_t)v[2];
        keys[2 * (4 * t + j) + 1] = 4 * t + j;
      }
    qsort(keys, 4 * (size_t)nt, 2 * sizeof(int64_t), cmp_face_key);
    char* boundary = calloc(4 * (size_t)nt, 1);
    for (int i = 0; i < 4 * nt;) {
      int e = i;
      while (e < 4 * nt && keys[2 * e] == keys[2 * i]) ++e;
      if (e - i == 1) boundary[keys[2 * i + 1]] = 1;
      i = e;
    }
    for (int t = 0; t < nt; ++t)
      for (int j = 0; j < 4; ++j) {
        if (!boundary[4 * t + j]) continue;
        if (nf >= cap) {
          free(keys);
          free(boundary);
          return -1;
        }
        int v[3], m = 0;
        for (int q = 0; q < 4; ++q)
          if (q != j) v[m++] = tet[q * n_tet + t0 + t];
        double a[3], b[3], c[3], o[3], ab[3], ac[3], n[3], ao[3];
        pos(X, n_nodes, v[0], a);
        pos(X, n_nodes, v[1], b);
        pos(X, n_nodes, v[2], c);
        pos(X, n_nodes, tet[j * n_tet + t0 + t], o);
        sub3(b, a, ab);
        sub3(c, a, ac);
        cross3(ab, ac, n);
        sub3(o, a, ao);
        if (dot3(n, ao) > 0.0) { /* the normal points at the fourth node: flip */
          const int s = v[1];
          v[1] = v[2];
          v[2] = s;
        }
        for (int i = 0; i < 3; ++i) out[i * cap + nf] = v[i];
        part[nf++] = p;
      }
    free(keys);
    free(boundary);
  }
  return nf;
}

/* Node-face anti-sticking (Sec. III.B, resolving numerical sticking): every
 * node closer than d_min to a face of another particle of its box is moved
 * away from the closest point of that face until it is d_min from it.
 * Faces: the membrane triangles (ids 0 .. n_tri-1) and the boundary faces of
 * the solids (ids n_tri + k, in the order orc_boundary_faces lists them).
 * Distances use the periodic image of each face nearest to the node (the
 * image of its first corner, applied to the whole face).  READINGS: the closest
 * face is the one of least float64 distance, ties to the lower face id (the
 * paper's minimum distance; exact ties occur where faces share the closest
 * edge or vertex); a node moves when that distance is below d_min; the move is along
 * (x - c)/|x - c| from the closest point c (the face normal when x lies on the
 * face), to c + d_min (x - c)/|x - c|; all nodes are tested against the
 * positions before the pass (none sees another's move).  The paper's particle
 * bounding-box check is a culling step: particles whose box, grown by 2 d_min
 * and taken periodically, cannot reach the node are skipped, which changes no
 * result.  x, x_out [3][n_nodes]; box_len [n_boxes][3] box lengths;
 * winner [n_nodes]: the face that moved the node, or -1; dist [n_nodes] (or
 * NULL): the least distance to a face of another particle whose bounding box
 * can reach the node, INFINITY where none can.  Returns the number of moved
 * nodes. */
int orc_antistick(int n_nodes, const double* X, const double* x, int n_particles, const int* node_start,
                  const int* tri_start, const int* tri, int n_tri, const int* tet_start, const int* tet, int n_tet,
                  const int* box_of_particle, const double* box_len, double d_min, double* x_out, int64_t* winner,
                  double* dist) {
  memcpy(x_out, x, sizeof(double) * 3 * (size_t)n_nodes);
  const int cap = 4 * n_tet + 1;
  int* bf = malloc(sizeof(int) * 3 * (size_t)cap);
  int* bp = malloc(sizeof(int) * (size_t)cap);
  const int nb = orc_boundary_faces(n_nodes, X, n_particles, tet_start, tet, n_tet, cap, bf, bp);
  double* lo = malloc(sizeof(double) * 3 * (size_t)n_particles);
  double* hi = malloc(sizeof(double) * 3 * (size_t)n_particles);
  for (int p = 0; p < n_particles; ++p)
    for (int i = 0; i < 3; ++i) {
      lo[3 * p + i] = INFINITY;
      hi[3 * p + i] = -INFINITY;
      for (int k = node_start[p]; k < node_start[p + 1]; ++k) {
        const double v = x[(size_t)i * n_nodes + k];
        lo[3 * p + i] = fmin(lo[3 * p + i], v);
        hi[3 * p + i] = fmax(hi[3 * p + i], v);
      }
    }
  int moved = 0;
  for (int P = 0; P < n_particles; ++P) {
    const int b = box_of_particle[P];
    const double* Lb = box_len + 3 * b;
    for (int k = node_start[P]; k < node_start[P + 1]; ++k) {
      double xk[3];
      pos(x, n_nodes, k, xk);
      double best = INFINITY;
      int64_t bestf = -1;
      double bestc[3] = {0, 0, 0}, bestn[3] = {0, 0, 0};
      for (int Q = 0; Q < n_particles; ++Q) {
        if (Q == P || box_of_particle[Q] != b) continue;
        int near = 1; /* periodic box test, grown by 2 d_min */
        for (int i = 0; i < 3; ++i) {
          const double c = 0.5 * (lo[3 * Q + i] + hi[3 * Q + i]), r = 0.5 * (hi[3 * Q + i] - lo[3 * Q + i]) + 2.0 * d_min;
          double d = xk[i] - c;
          d -= Lb[i] * nearbyint(d / Lb[i]);
          if (fabs(d) > r) near = 0;
        }
        if (!near) continue;
        const int nfq = tri_start[Q + 1] - tri_start[Q];
        for (int s = 0; s < nfq + nb; ++s) {
          int v[3];
          int64_t fid;
          if (s < nfq) {
            const int t = tri_start[Q] + s;
            for (int i = 0; i < 3; ++i) v[i] = tri[i * n_tri + t];
            fid = t;
          } else {
            const int j = s - nfq;
            if (bp[j] != Q) continue;
            for (int i = 0; i < 3; ++i) v[i] = bf[i * cap + j];
            fid = (int64_t)n_tri + j;
          }
          /* corners relative to the node in the periodic image of the face nearest to the node,
           * chosen by its first corner and applied to all three (a face is one piece) */
          double r[3][3];
          for (int i = 0; i < 3; ++i) {
            const double d0 = x[(size_t)i * n_nodes + v[0]] - xk[i];
            const double shift = Lb[i] * nearbyint(d0 / Lb[i]);
            for (int m = 0; m < 3; ++m) r[m][i] = x[(size_t)i * n_nodes + v[m]] - xk[i] - shift;
          }
          const double zero[3] = {0.0, 0.0, 0.0};
          double c[3];
          orc_point_triangle(zero, r[0], r[1], r[2], c);
          const double dc = norm3(c);
          if (dc < best || (dc == best && fid < bestf)) {
            best = dc;
            bestf = fid;
            double e1[3], e2[3];
            sub3(r[1], r[0], e1);
            sub3(r[2], r[0], e2);
            cross3(e1, e2, bestn);
            for (int i = 0; i < 3; ++i) bestc[i] = c[i];
          }
        }
      }
      if (winner) winner[k] = -1;
      if (dist) dist[k] = best;
      if (bestf < 0 || !(best < d_min)) continue;
      const double dc = norm3(bestc);
      double dir[3];
      if (dc > 0.0) {
        for (int i = 0; i < 3; ++i) dir[i] = -bestc[i] / dc; /* from the closest point to the node */
      } else {
        const double nn = norm3(bestn);
        for (int i = 0; i < 3; ++i) dir[i] = bestn[i] / nn;
      }
      for (int i = 0; i < 3; ++i) x_out[(size_t)i * n_nodes + k] = xk[i] + bestc[i] + d_min * dir[i];
      if (winner) winner[k] = bestf;
      moved++;
    }
  }
  free(bf);
  free(bp);
  free(lo);
  free(hi);
  return moved;
}

/* Distance from node node[i] to face face[i] (ids as in orc_antistick), in the
 * periodic image of the face nearest to the node (chosen by its first corner),
 * for i < n_pairs; out[i] = the distance.  With moved != NULL the node's
 * position is taken from moved [3][n_nodes] instead of x (to measure where a
 * move put it; the face stays at x). */
int orc_pair_distances(int n_nodes, const double* X, const double* x, const double* moved, int n_particles,
                       const int* node_start, const int* tri, int n_tri, const int* tet_start, const int* tet,
                       int n_tet, const int* box_of_particle, const double* box_len, int n_pairs, const int* node,
                       const int64_t* face, double* out) {
  const int cap = 4 * n_tet + 1;
  int* bf = malloc(sizeof(int) * 3 * (size_t)cap);
  int* bp = malloc(sizeof(int) * (size_t)cap);
  const int nb = orc_boundary_faces(n_nodes, X, n_particles, tet_start, tet, n_tet, cap, bf, bp);
  int bad = 0;
  for (int i = 0; i < n_pairs; ++i) {
    const int k = node[i];
    const int64_t f = face[i];
    int v[3];
    if (f >= 0 && f < n_tri) {
      for (int m = 0; m < 3; ++m) v[m] = tri[m * n_tri + f];
    } else if (f >= n_tri && f < (int64_t)n_tri + nb) {
      for (int m = 0; m < 3; ++m) v[m] = bf[m * cap + (f - n_tri)];
    } else {
      out[i] = NAN;
      ++bad;
      continue;
    }
    int P = 0;
    while (P + 1 < n_particles && node_start[P + 1] <= k) ++P;
    const double* Lb = box_len + 3 * box_of_particle[P];
    double xk[3];
    pos(moved ? moved : x, n_nodes, k, xk);
    double r[3][3];
    for (int j = 0; j < 3; ++j) {
      const double d0 = x[(size_t)j * n_nodes + v[0]] - xk[j];
      const double shift = Lb[j] * nearbyint(d0 / Lb[j]);
      for (int m = 0; m < 3; ++m) r[m][j] = x[(size_t)j * n_nodes + v[m]] - xk[j] - shift;
    }
    const double zero[3] = {0.0, 0.0, 0.0};
    double c[3];
    orc_point_triangle(zero, r[0], r[1], r[2], c);
    out[i] = norm3(c);
  }
  free(bf);
  free(bp);
  return bad;
}
