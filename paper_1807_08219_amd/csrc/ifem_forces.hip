// Element forces of the IFEM coupling step on gfx950.
//
//  k_ref_tri / k_ref_tet  reference data of every element (float64 setup):
//                         triangles the metric G = D0^T D0 of the reference
//                         edge matrix D0 and the area A0 = sqrt(det G)/2,
//                         tetrahedra D0^-1 and the volume V0 = det D0 / 6.
//  k_forces<T>            one workgroup per particle: elastic element forces,
//                         Helfrich bending, float64 volume/area/centroid, and a
//                         single coalesced write of the nodal forces.
//  k_large_*<T>           the same for particles larger than a workgroup's
//                         LDS: element forces into a scratch slot per corner,
//                         curvature and Laplacian passes per node, a fixed-order
//                         gather per node (see the section below).
//
// Membrane forces use the covariant form of the paper's constitutive laws.
// With current edges D = [d1 d2], g = D^T D, Delta = g - G and M = G^-1 Delta,
// the second Piola-Kirchhoff stress in edge coordinates is (Sec. II.A tension
// relation)  S = 2 (W1 I + W2 adj(I + M)) G^-1,
//     Skalak:       S G = mu M + (mu_D / 2) I2b ((1 + tr M) I - M)
//     neo-Hookean:  S G = mu ((tr M + 2 det M + I2b^2) I + M) / (1 + I2b)^2
//     with I1 - 2 = tr M and I2b = I2 - 1 = tr M + det M,
// and the nodal forces are [f1 f2] = -A0 D S, f0 = -(f1 + f2) (eq.
// FEM_Membrane with linear shape functions).  These equal the paper's
// frame-based expressions exactly; the per-element tangent frame drops out
// because the laws depend on the invariants only.  In float32 the metric
// difference Delta is formed error-free (float-float), so the small strain
// invariants carry no cancellation error.  Tetrahedra (Sec. II.B, eq. FEM)
// use the deformation gradient F = D D0^-1 directly (tet_element below).
#include "ifem_device.hpp"
#include "ifem_internal.hpp"

namespace ifem {

// ------------------------------------------------------------------ setup: reference metrics
// Inverse of a 3 x 3 matrix by cofactors; returns the determinant.
__device__ __forceinline__ double inverse3(const double m[3][3], double r[3][3]) {
  const double d = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                   m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
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

__global__ void k_ref_tri(int n_tris, int n_nodes, const int32_t* __restrict__ src, const int32_t* __restrict__ tri,
                          const double* __restrict__ X, double* __restrict__ ref, unsigned long long* status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_tris) return;
  const int e = src[s];
  const int i0 = tri[e], i1 = tri[n_tris + e], i2 = tri[2 * n_tris + e];
  double d1[3], d2[3];
  for (int a = 0; a < 3; ++a) {
    d1[a] = X[a * n_nodes + i1] - X[a * n_nodes + i0];
    d2[a] = X[a * n_nodes + i2] - X[a * n_nodes + i0];
  }
  const double G11 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
  const double G12 = d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2];
  const double G22 = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
  const double det = G11 * G22 - G12 * G12;
  ref[s] = G11;
  ref[n_tris + s] = G12;
  ref[2 * n_tris + s] = G22;
  ref[3 * n_tris + s] = det > 0.0 ? 0.5 * sqrt(det) : 0.0;
  if (!(det > 1e-300) || !(det >= 1e-24 * G11 * G22)) atomicAdd(status + 3, 1ull);
}

__global__ void k_ref_tet(int n_tets, int n_nodes, const int32_t* __restrict__ src, const int32_t* __restrict__ tet,
                          const double* __restrict__ X, double* __restrict__ ref, unsigned long long* status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_tets) return;
  const int e = src[s];
  int id[4];
  for (int v = 0; v < 4; ++v) id[v] = tet[v * n_tets + e];
  // reference edge matrix D0 (column a = X_{a+1} - X_0) and its inverse, whose row a is the
  // gradient of node a+1's shape function; the inverse's condition number is that of D0, where a
  // metric (D0^T D0) would square it
  double D0[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) D0[c][a] = X[c * n_nodes + id[a + 1]] - X[c * n_nodes + id[0]];
  double Di[3][3];
  const double det = inverse3(D0, Di);
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) ref[(3 * a + j) * n_tets + s] = Di[a][j];
  ref[9 * n_tets + s] = det / 6.0;
  if (!(det > 0.0)) atomicAdd(status + 3, 1ull);
}

// ------------------------------------------------------------------ metric difference
// Delta = g - G for the edges (e1, e2, e3) that start at node 0.  Float64:
// plain products.  Float32: edges split exactly into (hi, lo) and the Gram
// entries accumulated in float-float, so Delta carries no cancellation error.
__device__ __forceinline__ void metric_delta(const float xs[][3], int ne, float (*dh)[3], float (*dl)[3],
                                             const double* Gref, float* Delta) {
  for (int a = 0; a < ne; ++a)
    for (int c = 0; c < 3; ++c) two_diff(xs[a + 1][c], xs[0][c], dh[a][c], dl[a][c]);
  int k = 0;
  for (int a = 0; a < ne; ++a)
    for (int b = a; b < ne; ++b, ++k) {
      float s, e;
      dot3_ff(dh[a], dl[a], dh[b], dl[b], s, e);
      Delta[k] = diff_ff(s, e, Gref[k]);
    }
}

__device__ __forceinline__ void metric_delta(const double xs[][3], int ne, double (*dh)[3], double (*)[3],
                                             const double* Gref, double* Delta) {
  for (int a = 0; a < ne; ++a)
    for (int c = 0; c < 3; ++c) dh[a][c] = xs[a + 1][c] - xs[0][c];
  int k = 0;
  for (int a = 0; a < ne; ++a)
    for (int b = a; b < ne; ++b, ++k)
      Delta[k] = (dh[a][0] * dh[b][0] + dh[a][1] * dh[b][1] + dh[a][2] * dh[b][2]) - Gref[k];
}

// ------------------------------------------------------------------ membrane element
// Returns false (and zero forces) when the current triangle is collapsed (I2 <= 0).
template <typename T>
__device__ __forceinline__ bool tri_element(const T xs[3][3], const double G[3], double A0, int law, T mu, T mu2,
                                            T f[3][3]) {
  T dh[2][3], dl[2][3], D[3];
  metric_delta(xs, 2, dh, dl, G, D);  // D = {D11, D12, D22}
  // inverse reference metric in float64, then rounded to the working precision
  const double inv_detG = 1.0 / (G[0] * G[2] - G[1] * G[1]);
  const T Gi11 = (T)(G[2] * inv_detG), Gi12 = (T)(-G[1] * inv_detG), Gi22 = (T)(G[0] * inv_detG);
  const T M11 = Gi11 * D[0] + Gi12 * D[1], M12 = Gi11 * D[1] + Gi12 * D[2];
  const T M21 = Gi12 * D[0] + Gi22 * D[1], M22 = Gi12 * D[1] + Gi22 * D[2];
  const T trM = M11 + M22, detM = M11 * M22 - M12 * M21;
  const T I2b = trM + detM;  // J^2 - 1
  // J^2 = |e1 x e2|^2 / |E1 x E2|^2: a current triangle with coincident or collinear edges has J^2 = 0
  // exactly, which 1 + (tr M + det M) only approximates; test the cross product itself as well
  const T cx = dh[0][1] * dh[1][2] - dh[0][2] * dh[1][1];
  const T cy = dh[0][2] * dh[1][0] - dh[0][0] * dh[1][2];
  const T cz = dh[0][0] * dh[1][1] - dh[0][1] * dh[1][0];
  bool ok = (T(1) + I2b) > T(0) && (cx != T(0) || cy != T(0) || cz != T(0));
  T SG11, SG12, SG21, SG22;
  if (law == 1) {  // Skalak
    const T k = T(0.5) * mu2 * I2b;
    SG11 = mu * M11 + k * (T(1) + trM - M11);
    SG12 = mu * M12 - k * M12;
    SG21 = mu * M21 - k * M21;
    SG22 = mu * M22 + k * (T(1) + trM - M22);
  } else {  // neo-Hookean membrane
    const T J2 = T(1) + I2b;
    const T s = mu * frcp(J2 * J2);
    const T diag = trM + T(2) * detM + I2b * I2b;
    SG11 = s * (diag + M11);
    SG12 = s * M12;
    SG21 = s * M21;
    SG22 = s * (diag + M22);
  }
  const T S11 = SG11 * Gi11 + SG12 * Gi12, S12 = SG11 * Gi12 + SG12 * Gi22;
  const T S21 = SG21 * Gi11 + SG22 * Gi12, S22 = SG21 * Gi12 + SG22 * Gi22;
  const T a0 = (T)A0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T f1 = ok ? -a0 * (dh[0][c] * S11 + dh[1][c] * S21) : T(0);
    const T f2 = ok ? -a0 * (dh[0][c] * S12 + dh[1][c] * S22) : T(0);
    f[1][c] = f1;
    f[2][c] = f2;
    f[0][c] = -(f1 + f2);
  }
  return ok;
}

// ------------------------------------------------------------------ tetrahedral element
// Slightly compressible neo-Hookean tetrahedron (Sec. II.B) in the deformation-gradient form:
// F = sum_a e_a (x) g_a with the current edges e_a = x_{a+1} - x_0 and the rows g_a of the inverse
// reference edge matrix, J = det F, C^-1 = F^-1 F^-T, S = lam/2 (J^2 - 1) C^-1 + mu (I - C^-1),
// P = F S and f_k = -V0 P g_k (g_0 = -(g_1 + g_2 + g_3)).  All of it in float64 from exact edges
// (float32 offsets split into (hi, lo) pairs): near-incompressible solids turn any rounding of the
// volumetric strain into a stress error lambda / mu times larger, and flat reference tetrahedra are
// ill-conditioned, so the element works with the edge matrices themselves, never with their metrics
// (which square the condition number).  Returns false (and zero forces) for an inverted element.
template <typename T>
__device__ __forceinline__ bool tet_element(const T xs[4][3], const double Di[9], double V0, T mu_t, T lam_t,
                                            T f[4][3]) {
  double e[3][3];  // e[a] = x_{a+1} - x_0, exactly in the float32 path
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      if (sizeof(T) == 4) {
        float hi, lo;
        two_diff((float)xs[a + 1][c], (float)xs[0][c], hi, lo);
        e[a][c] = (double)hi + (double)lo;
      } else {
        e[a][c] = (double)xs[a + 1][c] - (double)xs[0][c];
      }
    }
  const double mu = (double)mu_t, lam = (double)lam_t;
  double F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i][j] = e[0][i] * Di[j] + e[1][i] * Di[3 + j] + e[2][i] * Di[6 + j];
  double Fi[3][3];
  const double J = inverse3(F, Fi);
  const bool ok = J > 0.0;
  double Ci[3][3];  // F^-1 F^-T
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) Ci[k][j] = Fi[k][0] * Fi[j][0] + Fi[k][1] * Fi[j][1] + Fi[k][2] * Fi[j][2];
  const double kv = 0.5 * lam * (J * J - 1.0);
  double S[3][3];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) S[k][j] = kv * Ci[k][j] + mu * ((k == j ? 1.0 : 0.0) - Ci[k][j]);
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i][j] = F[i][0] * S[0][j] + F[i][1] * S[1][j] + F[i][2] * S[2][j];
  double g[4][3];
  for (int j = 0; j < 3; ++j) {
    g[1][j] = Di[j];
    g[2][j] = Di[3 + j];
    g[3][j] = Di[6 + j];
    g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
  }
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 3; ++i)
      f[k][i] = ok ? (T)(-V0 * (P[i][0] * g[k][0] + P[i][1] * g[k][1] + P[i][2] * g[k][2])) : T(0);
  return ok;
}

// ------------------------------------------------------------------ bending, per node
// One-ring of node k: neighbours j_1..j_v (local ids) with triangles
// (k, j_i, j_{i+1}) counter-clockwise.  Per triangle: the cotangents of the
// angles at j_i and j_{i+1}, the angle at k, the mixed-area share, the face
// area vector (Meyer et al. 2003 operators).
template <typename T>
struct RingGeom {
  T A;         // mixed area
  T K[3];      // sum (cot a + cot b)(x_k - x_j)
  T N[3];      // sum of face area vectors
  T zr, zi;    // product of (u.w + i |u x w|) over the fan: its argument is sum(theta) - 2 pi
};

template <typename T>
__device__ __forceinline__ T atan2_t(T y, T x);
template <>
__device__ __forceinline__ float atan2_t<float>(float y, float x) {
  return atan2f(y, x);
}
template <>
__device__ __forceinline__ double atan2_t<double>(double y, double x) {
  return atan2(y, x);
}

// |v| and 1 / |v| from |v|^2: one reciprocal square root in float32, refined
// square root and reciprocal in float64.
__device__ __forceinline__ void norm_and_inverse(float n2, float& n, float& inv) {
  inv = __builtin_amdgcn_rsqf(n2);
  n = n2 * inv;
}
__device__ __forceinline__ void norm_and_inverse(double n2, double& n, double& inv) {
  n = fsqrt(n2);
  inv = frcp(n);
}

// One-ring quantities of node k for the curvature pass: mixed area, the
// cotangent sum K, the area-vector sum N and the angle product z.
template <typename T>
__device__ __forceinline__ void ring_geometry(int k, const int32_t* __restrict__ ring, int rb, int re, const T* xx,
                                              const T* xy, const T* xz, RingGeom<T>& R) {
  const T xk[3] = {xx[k], xy[k], xz[k]};
  R.A = 0;
  R.zr = 1;
  R.zi = 0;
  for (int c = 0; c < 3; ++c) R.K[c] = R.N[c] = 0;
  int ja = ring[re - 1];
  T u[3] = {xx[ja] - xk[0], xy[ja] - xk[1], xz[ja] - xk[2]};
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int r = rb; r < re; ++r) {
    const int jb = ring[r];
    // triangle (k, ja, jb): wedge from the previous neighbour to this one
    const T w[3] = {xx[jb] - xk[0], xy[jb] - xk[1], xz[jb] - xk[2]};
    const T cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    T s, inv;  // twice the area and its reciprocal
    norm_and_inverse(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2], s, inv);
    const T uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
    const T ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    // with e = w - u (edge ja -> jb): u.e = uw - uu, w.e = ww - uw
    const T ue = uw - uu, we = ww - uw;
    const T cot_a = -ue * inv;  // angle at ja, opposite edge (k, jb)
    const T cot_b = we * inv;   // angle at jb, opposite edge (k, ja)
    for (int c = 0; c < 3; ++c) {
      R.K[c] -= cot_b * u[c] + cot_a * w[c];
      R.N[c] += T(0.5) * cr[c];
    }
    // the angle at k enters through the argument of a running complex product: uw + i s has the
    // argument of the angle, and so has (uw + i s) / s = cot + i, whose modulus 1 / sin stays small
    const T cot_k = uw * inv;
    const T zr = R.zr * cot_k - R.zi;
    R.zi = R.zr + R.zi * cot_k;
    R.zr = zr;
    const bool obt_k = uw < T(0), obt_a = ue > T(0), obt_b = we < T(0);
    if (!(obt_k || obt_a || obt_b))
      R.A += T(0.125) * (uu * cot_b + ww * cot_a);
    else
      R.A += obt_k ? T(0.25) * s : T(0.125) * s;
    ja = jb;
    for (int c = 0; c < 3; ++c) u[c] = w[c];
    uu = ww;
  }
}

// One-ring quantities of node k for the Laplacian pass: the area-vector sum N
// (the same operations as ring_geometry, so the same normal) and the
// cotangent sum of g_j - g_k.
template <typename T>
__device__ __forceinline__ void ring_laplacian(int k, const int32_t* __restrict__ ring, int rb, int re, const T* xx,
                                               const T* xy, const T* xz, const T* g, T N[3], T& lap) {
  const T xk[3] = {xx[k], xy[k], xz[k]};
  const T gk = g[k];
  N[0] = N[1] = N[2] = 0;
  lap = 0;
  int ja = ring[re - 1];
  T u[3] = {xx[ja] - xk[0], xy[ja] - xk[1], xz[ja] - xk[2]};
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  T ga = g[ja];
  for (int r = rb; r < re; ++r) {
    const int jb = ring[r];
    const T w[3] = {xx[jb] - xk[0], xy[jb] - xk[1], xz[jb] - xk[2]};
    const T cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    T s, inv;
    norm_and_inverse(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2], s, inv);
    const T uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
    const T ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const T cot_a = -(uw - uu) * inv;
    const T cot_b = (ww - uw) * inv;
    for (int c = 0; c < 3; ++c) N[c] += T(0.5) * cr[c];
    const T gb = g[jb];
    lap += cot_b * (ga - gk) + cot_a * (gb - gk);
    ga = gb;
    for (int c = 0; c < 3; ++c) u[c] = w[c];
    uu = ww;
  }
}

// Mean curvature kH = K.n / (4 A), and (with_gauss) the Gaussian curvature
// kG = (2 pi - sum theta) / A = -arg(prod z) / A; the argument is the angle
// deficit itself when it lies in (-pi, pi), with no cancellation against 2 pi.
template <typename T>
__device__ __forceinline__ void ring_curvature(const RingGeom<T>& R, bool with_gauss, T& kH, T& kG, T n[3]) {
  const T iln = frcp(fsqrt(R.N[0] * R.N[0] + R.N[1] * R.N[1] + R.N[2] * R.N[2]));
  for (int c = 0; c < 3; ++c) n[c] = R.N[c] * iln;
  const T iA = frcp(R.A);
  kH = T(0.25) * (R.K[0] * n[0] + R.K[1] * n[1] + R.K[2] * n[2]) * iA;
  kG = with_gauss ? -atan2_t<T>(R.zi, R.zr) * iA : T(0);
}

// ------------------------------------------------------------------ the per-particle force kernel
template <typename T>
__device__ __forceinline__ void load_pos(const T* __restrict__ x, int64_t N, int i, T out[3]) {
  out[0] = x[i];
  out[1] = x[N + i];
  out[2] = x[2 * N + i];
}

// POS_LDS: the particle's positions are staged in LDS once (coalesced) and
// every element and one-ring read hits LDS; otherwise they are read through
// the caches (particles too large for the staging copy).
template <typename T, bool POS_LDS>
__global__ void __launch_bounds__(512) k_forces(const ForceArgs a, const T* __restrict__ x,
                                                 const double* __restrict__ anchor, T* __restrict__ fout,
                                                 double* __restrict__ red) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_lds[5 * 16];
  __shared__ unsigned int bad_elems, bad_out;
  const int p = a.lds_part ? a.lds_part[blockIdx.x] : (int)blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n0 = a.node_start[p];
  const int nn = a.node_start[p + 1] - n0;
  const int64_t N = a.n_nodes;
  T* acc = reinterpret_cast<T*>(smem_raw);  // [3][cap]
  T* kh = acc + 3 * a.cap;                  // [cap] (bending only)
  for (int i = tid; i < nn; i += nt) {
    acc[i] = 0;
    acc[a.cap + i] = 0;
    acc[2 * a.cap + i] = 0;
  }
  if (tid == 0) bad_elems = bad_out = 0;
  __syncthreads();

  const T* xx = x + n0;
  const T* xy = x + N + n0;
  const T* xz = x + 2 * N + n0;
  if (POS_LDS) {
    T* px = kh + (a.has_bending ? a.cap : 0);  // [3][cap] after the curvature array
    for (int i = tid; i < nn; i += nt) {
      px[i] = xx[i];
      px[a.cap + i] = xy[i];
      px[2 * a.cap + i] = xz[i];
    }
    __syncthreads();
    xx = px;
    xy = px + a.cap;
    xz = px + 2 * a.cap;
  }
  const int law = a.law[p];
  const T mu = (T)a.mu[p], mu2 = (T)a.mu2[p];
  // local origin for the float64 reductions: float32 offsets are already
  // particle-relative; float64 absolute positions are taken relative to node 0
  double o[3] = {0.0, 0.0, 0.0};
  if (sizeof(T) == 8) {
    o[0] = (double)xx[0];
    o[1] = (double)xy[0];
    o[2] = (double)xz[0];
  }
  double r[5] = {0, 0, 0, 0, 0};  // V, A, V*cx, V*cy, V*cz (local frame)
  unsigned int my_bad = 0;

  // --- membrane elements, colour by colour (no two triangles of a colour share a node)
  for (int c = a.pcol_tri[p]; c < a.pcol_tri[p + 1]; ++c) {
    const int e1 = a.colb_tri[c + 1];
    for (int s = a.colb_tri[c] + tid; s < e1; s += nt) {
      const int i0 = a.tri_local[s], i1 = a.tri_local[a.n_tris + s], i2 = a.tri_local[2 * a.n_tris + s];
      T xs[3][3];
      xs[0][0] = xx[i0]; xs[0][1] = xy[i0]; xs[0][2] = xz[i0];
      xs[1][0] = xx[i1]; xs[1][1] = xy[i1]; xs[1][2] = xz[i1];
      xs[2][0] = xx[i2]; xs[2][1] = xy[i2]; xs[2][2] = xz[i2];
      const double G[3] = {a.tri_ref[s], a.tri_ref[a.n_tris + s], a.tri_ref[2 * a.n_tris + s]};
      const double A0 = a.tri_ref[3 * a.n_tris + s];
      T f[3][3];
      if (!tri_element<T>(xs, G, A0, law, mu, mu2, f)) ++my_bad;
      const int ids[3] = {i0, i1, i2};
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        acc[ids[v]] += f[v][0];
        acc[a.cap + ids[v]] += f[v][1];
        acc[2 * a.cap + ids[v]] += f[v][2];
      }
      if (red) {
        // cone volume q0.(q1 x q2) = q0.(u x w) with the edges u, w of the area vector
        double q[3][3];
        for (int v = 0; v < 3; ++v)
          for (int cc = 0; cc < 3; ++cc) q[v][cc] = (double)xs[v][cc] - o[cc];
        double u[3], w[3];
        for (int cc = 0; cc < 3; ++cc) {
          u[cc] = q[1][cc] - q[0][cc];
          w[cc] = q[2][cc] - q[0][cc];
        }
        const double nx = u[1] * w[2] - u[2] * w[1], ny = u[2] * w[0] - u[0] * w[2], nz = u[0] * w[1] - u[1] * w[0];
        const double cone = (q[0][0] * nx + q[0][1] * ny + q[0][2] * nz) * (1.0 / 6.0);
        r[0] += cone;
        for (int cc = 0; cc < 3; ++cc) r[2 + cc] += cone * (q[0][cc] + q[1][cc] + q[2][cc]) * 0.25;
        const double n2 = nx * nx + ny * ny + nz * nz;
        r[1] += 0.5 * fsqrt(n2);
      }
    }
    __syncthreads();
  }
  // --- tetrahedral elements
  for (int c = a.pcol_tet[p]; c < a.pcol_tet[p + 1]; ++c) {
    const int e1 = a.colb_tet[c + 1];
    for (int s = a.colb_tet[c] + tid; s < e1; s += nt) {
      int ids[4];
      T xs[4][3];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ids[v] = a.tet_local[v * a.n_tets + s];
        xs[v][0] = xx[ids[v]];
        xs[v][1] = xy[ids[v]];
        xs[v][2] = xz[ids[v]];
      }
      double Di[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Di[k] = a.tet_ref[k * a.n_tets + s];
      const double V0 = a.tet_ref[9 * a.n_tets + s];
      T f[4][3];
      if (!tet_element<T>(xs, Di, V0, mu, mu2, f)) ++my_bad;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[ids[v]] += f[v][0];
        acc[a.cap + ids[v]] += f[v][1];
        acc[2 * a.cap + ids[v]] += f[v][2];
      }
      if (red) {
        double q[4][3];
        for (int v = 0; v < 4; ++v)
          for (int cc = 0; cc < 3; ++cc) q[v][cc] = (double)xs[v][cc] - o[cc];
        double d[3][3];
        for (int v = 0; v < 3; ++v)
          for (int cc = 0; cc < 3; ++cc) d[v][cc] = q[v + 1][cc] - q[0][cc];
        const double vol = (d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                            d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                            d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0])) / 6.0;
        r[0] += vol;
        for (int cc = 0; cc < 3; ++cc) r[2 + cc] += vol * (q[0][cc] + q[1][cc] + q[2][cc] + q[3][cc]) * 0.25;
      }
    }
    __syncthreads();
  }
  // --- Helfrich bending: F = 2 kb [Lap(kH - kH0) + 2 (kH - kH0)(kH^2 - kG + kH0 kH)] n A.  The
  // curvature pass adds the second term; with Lap f = (1 / 2A) sum (cot a + cot b)(f_j - f_k), the
  // first is kb n sum (cot a + cot b)(g_j - g_k), g = kH - kH0, added by the Laplacian pass.
  const double kbp = a.kb[p];
  if (kbp != 0.0 && a.ring_start != nullptr) {
    const int* rs = a.ring_start + n0;
    const T kH0 = (T)(-0.5 * a.c0[p]);
    const T kb = (T)kbp;
    for (int k = tid; k < nn; k += nt) {
      if (rs[k + 1] - rs[k] < 3) {  // node without a closed fan: no curvature
        kh[k] = 0;
        continue;
      }
      RingGeom<T> R;
      ring_geometry<T>(k, a.ring, rs[k], rs[k + 1], xx, xy, xz, R);
      T kH, kG, nv[3];
      ring_curvature(R, true, kH, kG, nv);
      const T gk = kH - kH0;
      kh[k] = gk;
      const T s2 = T(4) * kb * gk * (kH * kH - kG + kH0 * kH) * R.A;
      acc[k] += s2 * nv[0];
      acc[a.cap + k] += s2 * nv[1];
      acc[2 * a.cap + k] += s2 * nv[2];
    }
    __syncthreads();
    for (int k = tid; k < nn; k += nt) {
      if (rs[k + 1] - rs[k] < 3) continue;
      T N[3], lap;
      ring_laplacian<T>(k, a.ring, rs[k], rs[k + 1], xx, xy, xz, kh, N, lap);
      const T s1 = kb * lap * frcp(fsqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]));
      acc[k] += s1 * N[0];
      acc[a.cap + k] += s1 * N[1];
      acc[2 * a.cap + k] += s1 * N[2];
    }
    __syncthreads();
  }
  // --- write the nodal forces once
  unsigned int nonfinite = 0;
  for (int i = tid; i < nn; i += nt) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T v = acc[c * a.cap + i];
      if (!isfinite(v)) ++nonfinite;
      fout[c * N + n0 + i] = v;
    }
  }
  if (my_bad) atomicAdd(&bad_elems, my_bad);
  if (nonfinite) atomicAdd(&bad_out, nonfinite);
  // --- float64 per-particle reductions
  if (red) {
    block_sum<5>(r, red_lds);
    if (tid == 0) {
      const double V = r[0];
      double base[3] = {o[0], o[1], o[2]};
      if (anchor) {
        base[0] += anchor[3 * p];
        base[1] += anchor[3 * p + 1];
        base[2] += anchor[3 * p + 2];
      }
      red[5 * p + 0] = V;
      red[5 * p + 1] = r[1];
      for (int c = 0; c < 3; ++c) red[5 * p + 2 + c] = base[c] + r[2 + c] / V;
    }
  } else {
    __syncthreads();
  }
  if (tid == 0) {
    if (bad_elems) atomicAdd(a.status + 0, (unsigned long long)bad_elems);
    if (bad_out) atomicAdd(a.status + 1, (unsigned long long)bad_out);
  }
}

// ------------------------------------------------------------------ particles larger than a workgroup's LDS
// A particle whose forces (and curvature) do not fit one workgroup's LDS takes
// this path instead of k_forces: the same element and one-ring routines, with
// every intermediate in global memory and no element colouring:
//  k_large_elems<T>  one thread per element: its nodal forces into a scratch
//                    slot (no accumulation), its volume/area/centroid terms;
//  k_large_curv<T>   one thread per node of a bending membrane: curvature, the
//                    curvature term of the Helfrich force, kH - kH0;
//  k_large_lap<T>    one thread per such node: the Laplacian term (needs every
//                    node's kH - kH0: a launch of its own);
//  k_large_gather<T> one thread per node: its element shares in a fixed order
//                    (a node -> element-slot list built at plan creation) plus
//                    the bending terms, written once;
//  k_large_partial,  the element terms of the float64 reductions summed in a
//  k_large_reduce    fixed order: 16 shares per particle, then the shares.
// Sums run in fixed orders, so the forces are reproducible run to run.

// One corner's force in the element scratch: x, y, z and a pad, 16-byte aligned (one float4 or two
// double2 accesses).
__device__ __forceinline__ void store_corner(float* p, const float f[3]) {
  *reinterpret_cast<float4*>(p) = make_float4(f[0], f[1], f[2], 0.0f);
}
__device__ __forceinline__ void store_corner(double* p, const double f[3]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(f[0], f[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(f[2], 0.0);
}
__device__ __forceinline__ void load_corner(const float* p, float f[3]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  f[0] = q.x;
  f[1] = q.y;
  f[2] = q.z;
}
__device__ __forceinline__ void load_corner(const double* p, double f[3]) {
  const double2 q0 = reinterpret_cast<const double2*>(p)[0], q1 = reinterpret_cast<const double2*>(p)[1];
  f[0] = q0.x;
  f[1] = q0.y;
  f[2] = q1.x;
}

template <typename T>
__device__ __forceinline__ void large_pos(const T* __restrict__ x, int64_t N, int k, T out[3]) {
  out[0] = x[k];
  out[1] = x[N + k];
  out[2] = x[2 * N + k];
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_elems(const ForceArgs a, const LargeArgs L, const T* __restrict__ x,
                                                      double* __restrict__ red_terms) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t N = a.n_nodes;
  bool bad = false;
  if (e < L.n_tri + L.n_tet) {
    const bool tri = e < L.n_tri;
    const int s = tri ? L.tri_slot[e] : L.tet_slot[e - L.n_tri];
    const int p = tri ? L.tri_part[e] : L.tet_part[e - L.n_tri];
    const int n0 = a.node_start[p];
    const T mu = (T)a.mu[p], mu2 = (T)a.mu2[p];
    // float64 positions are taken relative to the particle's node 0 for the reductions, as in k_forces
    double o[3] = {0.0, 0.0, 0.0};
    if (sizeof(T) == 8) {
      o[0] = (double)x[n0];
      o[1] = (double)x[N + n0];
      o[2] = (double)x[2 * N + n0];
    }
    double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (tri) {
      int ids[3];
      T xs[3][3];
      for (int v = 0; v < 3; ++v) {
        ids[v] = a.tri_local[v * a.n_tris + s];
        large_pos(x, N, n0 + ids[v], xs[v]);
      }
      const double G[3] = {a.tri_ref[s], a.tri_ref[a.n_tris + s], a.tri_ref[2 * a.n_tris + s]};
      T f[3][3];
      bad = !tri_element<T>(xs, G, a.tri_ref[3 * a.n_tris + s], a.law[p], mu, mu2, f);
      for (int v = 0; v < 3; ++v) store_corner(reinterpret_cast<T*>(L.ef_tri) + ((int64_t)v * L.n_tri + e) * 4, f[v]);
      double q[3][3];
      for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) q[v][c] = (double)xs[v][c] - o[c];
      double u[3], w[3];
      for (int c = 0; c < 3; ++c) {
        u[c] = q[1][c] - q[0][c];
        w[c] = q[2][c] - q[0][c];
      }
      const double nx = u[1] * w[2] - u[2] * w[1], ny = u[2] * w[0] - u[0] * w[2], nz = u[0] * w[1] - u[1] * w[0];
      const double cone = (q[0][0] * nx + q[0][1] * ny + q[0][2] * nz) * (1.0 / 6.0);
      r[0] = cone;
      r[1] = 0.5 * fsqrt(nx * nx + ny * ny + nz * nz);
      for (int c = 0; c < 3; ++c) r[2 + c] = cone * (q[0][c] + q[1][c] + q[2][c]) * 0.25;
    } else {
      const int et = e - L.n_tri;
      T xs[4][3];
      for (int v = 0; v < 4; ++v) large_pos(x, N, n0 + a.tet_local[v * a.n_tets + s], xs[v]);
      double Di[9];
      for (int k = 0; k < 9; ++k) Di[k] = a.tet_ref[k * a.n_tets + s];
      T f[4][3];
      bad = !tet_element<T>(xs, Di, a.tet_ref[9 * a.n_tets + s], mu, mu2, f);
      for (int v = 0; v < 4; ++v) store_corner(reinterpret_cast<T*>(L.ef_tet) + ((int64_t)v * L.n_tet + et) * 4, f[v]);
      double q[4][3];
      for (int v = 0; v < 4; ++v)
        for (int c = 0; c < 3; ++c) q[v][c] = (double)xs[v][c] - o[c];
      double d[3][3];
      for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) d[v][c] = q[v + 1][c] - q[0][c];
      const double vol = (d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                          d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                          d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0])) / 6.0;
      r[0] = vol;
      for (int c = 0; c < 3; ++c) r[2 + c] = vol * (q[0][c] + q[1][c] + q[2][c] + q[3][c]) * 0.25;
    }
    if (red_terms)
      for (int k = 0; k < 5; ++k) red_terms[k * (int64_t)(L.n_tri + L.n_tet) + e] = r[k];
  }
  const unsigned long long m = __ballot(bad);
  if (m && lane == __ffsll((long long)m) - 1) atomicAdd(a.status + 0, (unsigned long long)__popcll(m));
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_curv(const ForceArgs a, const LargeArgs L, const T* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_node) return;
  const int p = L.node_part[i];
  if (a.kb[p] == 0.0 || a.ring_start == nullptr) return;
  const int n0 = a.node_start[p], lb = L.node_base[i];  // lb: the compact index of the particle's node 0
  const int k = i - lb;
  const int64_t N = a.n_nodes;
  T* kh = reinterpret_cast<T*>(L.kh);
  T* fb = reinterpret_cast<T*>(L.fb);
  const int* rs = a.ring_start + n0;
  if (rs[k + 1] - rs[k] < 3) {  // node without a closed fan: no curvature, no bending force
    kh[i] = 0;
    for (int c = 0; c < 3; ++c) fb[c * (int64_t)L.n_node + i] = 0;
    return;
  }
  const T kH0 = (T)(-0.5 * a.c0[p]);
  const T kb = (T)a.kb[p];
  RingGeom<T> R;
  ring_geometry<T>(k, a.ring, rs[k], rs[k + 1], x + n0, x + N + n0, x + 2 * N + n0, R);
  T kH, kG, nv[3];
  ring_curvature(R, true, kH, kG, nv);
  const T gk = kH - kH0;
  kh[i] = gk;
  const T s2 = T(4) * kb * gk * (kH * kH - kG + kH0 * kH) * R.A;
  for (int c = 0; c < 3; ++c) fb[c * (int64_t)L.n_node + i] = s2 * nv[c];
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_lap(const ForceArgs a, const LargeArgs L, const T* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_node) return;
  const int p = L.node_part[i];
  if (a.kb[p] == 0.0 || a.ring_start == nullptr) return;
  const int n0 = a.node_start[p], lb = L.node_base[i];
  const int k = i - lb;
  const int64_t N = a.n_nodes;
  const int* rs = a.ring_start + n0;
  if (rs[k + 1] - rs[k] < 3) return;
  T* fb = reinterpret_cast<T*>(L.fb);
  T Nv[3], lap;
  ring_laplacian<T>(k, a.ring, rs[k], rs[k + 1], x + n0, x + N + n0, x + 2 * N + n0,
                    reinterpret_cast<const T*>(L.kh) + lb, Nv, lap);
  const T s1 = (T)a.kb[p] * lap * frcp(fsqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]));
  for (int c = 0; c < 3; ++c) fb[c * (int64_t)L.n_node + i] += s1 * Nv[c];
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_gather(const ForceArgs a, const LargeArgs L, T* __restrict__ fout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  unsigned int nonfinite = 0;
  if (i < L.n_node) {
    const int p = L.node_part[i];
    const int k = a.node_start[p] + (i - L.node_base[i]);
    const T* ef_tri = reinterpret_cast<const T*>(L.ef_tri);
    const T* ef_tet = reinterpret_cast<const T*>(L.ef_tet);
    T f[3] = {T(0), T(0), T(0)};
    for (int j = L.gather_start[i]; j < L.gather_start[i + 1]; ++j) {
      const int g = L.gather[j];  // element e and corner v: e * 4 + v, tetrahedra after the triangles
      const int e = g >> 2, v = g & 3;
      T fc[3];
      load_corner(e < L.n_tri ? ef_tri + ((int64_t)v * L.n_tri + e) * 4 : ef_tet + ((int64_t)v * L.n_tet + (e - L.n_tri)) * 4,
                  fc);
      for (int c = 0; c < 3; ++c) f[c] += fc[c];
    }
    if (a.kb[p] != 0.0 && a.ring_start != nullptr) {
      const T* fb = reinterpret_cast<const T*>(L.fb);
      for (int c = 0; c < 3; ++c) f[c] += fb[c * (int64_t)L.n_node + i];
    }
    for (int c = 0; c < 3; ++c) {
      if (!isfinite(f[c])) ++nonfinite;
      fout[c * (int64_t)a.n_nodes + k] = f[c];
    }
  }
  const unsigned long long m = __ballot(nonfinite != 0);
  // every lane's count, summed over the wavefront
  unsigned int total = nonfinite;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) total += __shfl_xor(total, off, kWave);
  if (m && lane == 0) atomicAdd(a.status + 1, (unsigned long long)total);
}

// The reductions of the large particles in two fixed-order stages: kRedParts workgroups per particle
// each sum one contiguous share of its elements' terms (strided over the threads, then the block sum),
// then one thread per particle adds the shares in order and writes volume, area and centroid.
constexpr int kRedParts = 16;

__global__ void __launch_bounds__(256) k_large_partial(const LargeArgs L, const double* __restrict__ red_terms) {
  __shared__ double red_lds[5 * 16];
  const int lp = blockIdx.x / kRedParts, j = blockIdx.x % kRedParts;
  const int ne = L.n_tri + L.n_tet;
  double r[5] = {0, 0, 0, 0, 0};
  // the particle's triangles, then its tetrahedra, as one index range split into kRedParts shares
  const int t0 = L.tri_begin[lp], nt = L.tri_begin[lp + 1] - t0;
  const int q0 = L.tet_begin[lp], nq = L.tet_begin[lp + 1] - q0;
  const int n = nt + nq;
  const int lo = (int)((int64_t)n * j / kRedParts), hi = (int)((int64_t)n * (j + 1) / kRedParts);
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int64_t col = i < nt ? t0 + i : L.n_tri + q0 + (i - nt);
    for (int k = 0; k < 5; ++k) r[k] += red_terms[k * (int64_t)ne + col];
  }
  block_sum<5>(r, red_lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) L.red_part[(lp * kRedParts + j) * 5 + k] = r[k];
}

__global__ void __launch_bounds__(64) k_large_reduce(const ForceArgs a, const LargeArgs L,
                                                     const double* __restrict__ origin_x, int64_t N, int fp64,
                                                     const double* __restrict__ anchor, double* __restrict__ red) {
  const int lp = blockIdx.x * blockDim.x + threadIdx.x;
  if (lp >= L.n_part) return;
  const int p = L.part[lp];
  double r[5] = {0, 0, 0, 0, 0};
  for (int j = 0; j < kRedParts; ++j)
    for (int k = 0; k < 5; ++k) r[k] += L.red_part[(lp * kRedParts + j) * 5 + k];
  const int n0 = a.node_start[p];
  double base[3] = {0.0, 0.0, 0.0};
  if (fp64)
    for (int c = 0; c < 3; ++c) base[c] = origin_x[c * N + n0];
  if (anchor)
    for (int c = 0; c < 3; ++c) base[c] += anchor[3 * p + c];
  const double V = r[0];
  red[5 * p + 0] = V;
  red[5 * p + 1] = r[1];
  for (int c = 0; c < 3; ++c) red[5 * p + 2 + c] = base[c] + r[2 + c] / V;
}

template <typename T>
static hipError_t launch_large_t(const PlanDev& P, const T* x, const double* anchor, T* f, double* red,
                                 hipStream_t st) {
  const LargeArgs& L = P.large;
  const int B = 256;
  const int ne = L.n_tri + L.n_tet;
  if (ne > 0)
    hipLaunchKernelGGL(k_large_elems<T>, dim3((ne + B - 1) / B), dim3(B), 0, st, P.fargs, L, x,
                       red ? L.red_terms : (double*)nullptr);
  if (L.n_node > 0) {
    if (L.any_bending) {
      hipLaunchKernelGGL(k_large_curv<T>, dim3((L.n_node + B - 1) / B), dim3(B), 0, st, P.fargs, L, x);
      hipLaunchKernelGGL(k_large_lap<T>, dim3((L.n_node + B - 1) / B), dim3(B), 0, st, P.fargs, L, x);
    }
    hipLaunchKernelGGL(k_large_gather<T>, dim3((L.n_node + B - 1) / B), dim3(B), 0, st, P.fargs, L, f);
  }
  if (red) {
    hipLaunchKernelGGL(k_large_partial, dim3(L.n_part * kRedParts), dim3(B), 0, st, L, L.red_terms);
    hipLaunchKernelGGL(k_large_reduce, dim3((L.n_part + 63) / 64), dim3(64), 0, st, P.fargs, L,
                       sizeof(T) == 8 ? (const double*)x : (const double*)nullptr, (int64_t)P.n_nodes,
                       sizeof(T) == 8 ? 1 : 0, anchor, red);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_ref_setup(const PlanDev& P, const double* X, hipStream_t st) {
  const int B = 256;
  if (P.n_tris)
    hipLaunchKernelGGL(k_ref_tri, dim3((P.n_tris + B - 1) / B), dim3(B), 0, st, P.n_tris, P.n_nodes, P.tri_src,
                       P.tri_global, X, P.tri_ref, P.status);
  if (P.n_tets)
    hipLaunchKernelGGL(k_ref_tet, dim3((P.n_tets + B - 1) / B), dim3(B), 0, st, P.n_tets, P.n_nodes, P.tet_src,
                       P.tet_global, X, P.tet_ref, P.status);
  return hipGetLastError();
}

template <typename T>
static size_t force_lds(const PlanDev& P, bool pos_lds) {
  return (size_t)(3 + (P.has_bending ? 1 : 0) + (pos_lds ? 3 : 0)) * P.cap * sizeof(T);
}

// Stage positions in LDS when the particle's forces, curvature and positions fit.
template <typename T>
static bool use_pos_lds(const PlanDev& P) {
  return force_lds<T>(P, true) <= 160 * 1024 - 2048;
}

hipError_t prepare_force_kernels(const PlanDev& P) {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_forces<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)force_lds<float>(P, false));
  if (e == hipSuccess && use_pos_lds<float>(P))
    e = hipFuncSetAttribute((const void*)k_forces<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)force_lds<float>(P, true));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_forces<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)force_lds<double>(P, false));
  if (e == hipSuccess && use_pos_lds<double>(P))
    e = hipFuncSetAttribute((const void*)k_forces<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)force_lds<double>(P, true));
  return e;
}

size_t force_lds_bytes(const PlanDev& P, int dtype) {
  return dtype == 0 ? force_lds<float>(P, use_pos_lds<float>(P)) : force_lds<double>(P, use_pos_lds<double>(P));
}

size_t force_lds_per_node(bool has_bending) { return (size_t)(3 + (has_bending ? 1 : 0)) * sizeof(double); }

hipError_t launch_forces(const PlanDev& P, int dtype, const void* x, const double* anchor, void* f, double* red,
                         int block, hipStream_t st) {
  if (P.n_particles == 0) return hipSuccess;
  P.timer->begin(K_FORCES, st);
  if (P.large.n_part > 0) {
    const hipError_t e = dtype == 0 ? launch_large_t<float>(P, (const float*)x, anchor, (float*)f, red, st)
                                    : launch_large_t<double>(P, (const double*)x, anchor, (double*)f, red, st);
    if (e != hipSuccess || P.n_lds_part == 0) {
      P.timer->end(st);
      return e;
    }
  }
  const dim3 g(P.n_lds_part), b(block);
  if (dtype == 0) {
    if (use_pos_lds<float>(P))
      hipLaunchKernelGGL((k_forces<float, true>), g, b, force_lds<float>(P, true), st, P.fargs, (const float*)x,
                         anchor, (float*)f, red);
    else
      hipLaunchKernelGGL((k_forces<float, false>), g, b, force_lds<float>(P, false), st, P.fargs, (const float*)x,
                         anchor, (float*)f, red);
  } else {
    if (use_pos_lds<double>(P))
      hipLaunchKernelGGL((k_forces<double, true>), g, b, force_lds<double>(P, true), st, P.fargs, (const double*)x,
                         anchor, (double*)f, red);
    else
      hipLaunchKernelGGL((k_forces<double, false>), g, b, force_lds<double>(P, false), st, P.fargs,
                         (const double*)x, anchor, (double*)f, red);
  }
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
