// Viscoelastic coupling terms (Sec. II.B, Sec. III.A steps 1 and 4):
//
//  k_interp_cells<T>  interpolation of cell-centred fields (the six
//                     components of the conformation tensor) to the nodes:
//                     the MLS weights of the cell-centre lattice once per
//                     node, then one 27-value gather per field;
//  k_fluid<T>         the fluid-stress part of eq. FEM for solids, added to
//                     the nodal forces.
//
// Fluid forces.  The paper writes the Newtonian and polymer stresses as first
// Piola-Kirchhoff tensors on the reference element,
//   P^fN = eta J (L + L^T) F^-T,  P^fP = J G (C_avg - I) F^-T,
//   L = sum_k u_k (x) grad_X N_k F^-1,  f_k = +V0 (P^fN + P^fP) grad_X N_k.
// Since J V0 = V (the current volume) and F^-T grad_X N_k = grad_x N_k, the
// same forces are f_k = V sigma grad_x N_k with the Cauchy stress
// sigma = eta (L + L^T) + G (C_avg - I) and L = sum_k u_k (x) grad_x N_k: only
// the current element is needed.  With the current edges d_1..d_3 from node 0,
// V grad_x N_1 = (d_2 x d_3) / 6 (cyclically) and grad_x N_0 = -sum, so the
// forces need no division, and L one reciprocal of det[d_1 d_2 d_3] = 6 V.
// All of it is float64 (float32 offsets and velocities are widened exactly).
#include <algorithm>

#include "ifem_internal.hpp"

namespace ifem {

template <typename T>
struct alignas(sizeof(T)) Row3c {
  T v[3];
};

template <typename T>
__global__ void __launch_bounds__(256) k_interp_cells(const TransferArgs a, const T* __restrict__ x,
                                                      const double* __restrict__ anchor, const T* __restrict__ grid,
                                                      int ncomp, T* __restrict__ out) {
  const int k = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= a.n_nodes) return;
  const int p = a.node_particle[k];
  const BoxDev B = box_of(a, p);
  double pos[3];
  const int64_t N = a.n_nodes;
  if (sizeof(T) == 4) {
    pos[0] = anchor[3 * p] + (double)x[k];
    pos[1] = anchor[3 * p + 1] + (double)x[N + k];
    pos[2] = anchor[3 * p + 2] + (double)x[2 * N + k];
  } else {
    pos[0] = (double)x[k];
    pos[1] = (double)x[N + k];
    pos[2] = (double)x[2 * N + k];
  }
  int32_t base[3];
  double tau64[3];
  nearest_node(B, 3, pos, base, tau64);  // lattice 3: the cell centres
  const T tau[3] = {(T)tau64[0], (T)tau64[1], (T)tau64[2]};
  T W[27], c[4];
  const bool ok = mls_weights<T>(tau, W, c);
  T phi[27];
  mls_phi<T>(W, c, phi);
  const bool seam = base[0] == 0 || base[0] == B.n[0] - 1;
  const int32_t x0 = seam ? 0 : base[0] - 1;
  int32_t ix[3], rows[9];
#pragma unroll
  for (int m = 0; m < 3; ++m) ix[m] = wrap1(base[0] + m - 1, B.n[0]);
  const int32_t nxy = B.n[0] * B.n[1];
#pragma unroll
  for (int mz = 0; mz < 3; ++mz)
#pragma unroll
    for (int my = 0; my < 3; ++my)
      rows[mz * 3 + my] = wrap1(base[2] + mz - 1, B.n[2]) * nxy + wrap1(base[1] + my - 1, B.n[1]) * B.n[0];
#pragma unroll 1
  for (int f = 0; f < ncomp; ++f) {
    const T* g = grid + f * a.total_cells + B.cell_off;  // cells of one box fit 32-bit offsets
    T s = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const T* row = g + (uint32_t)rows[r];
      T u[3];
      if (!seam) {
        const Row3c<T> r3 = *reinterpret_cast<const Row3c<T>*>(row + x0);
        u[0] = r3.v[0];
        u[1] = r3.v[1];
        u[2] = r3.v[2];
      } else {
        u[0] = row[ix[0]];
        u[1] = row[ix[1]];
        u[2] = row[ix[2]];
      }
#pragma unroll
      for (int mx = 0; mx < 3; ++mx) s += phi[r * 3 + mx] * u[mx];
    }
    out[f * N + k] = s;
  }
  if (!ok) atomicAdd(a.status + 2, 1ull);
}

// Forces of one tetrahedron's viscous and polymeric stress on its four corners
// (q: corner positions in a local frame, u: corner velocities, C: the
// conformation [6][N] of the particle's nodes or null, ids: the corners' indices
// into it).  False for an inverted or flat element, which gets no force.
template <typename T>
__device__ __forceinline__ bool fluid_tet(const double q[4][3], const double u[4][3], const T* __restrict__ Cp,
                                          int64_t N, const int ids[4], double eta, double G, double fk[4][3]) {
  double d[3][3], du[3][3];  // current edges and velocity differences from node 0
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d[k][c] = q[k + 1][c] - q[0][c];
      du[k][c] = u[k + 1][c] - u[0][c];
    }
  double g[3][3];  // V grad_x N_k for k = 1..3: (d_k+1 x d_k+2) / 6
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double* b = d[(k + 1) % 3];
    const double* e = d[(k + 2) % 3];
    g[k][0] = (b[1] * e[2] - b[2] * e[1]) * (1.0 / 6.0);
    g[k][1] = (b[2] * e[0] - b[0] * e[2]) * (1.0 / 6.0);
    g[k][2] = (b[0] * e[1] - b[1] * e[0]) * (1.0 / 6.0);
  }
  const double V = d[0][0] * g[0][0] + d[0][1] * g[0][1] + d[0][2] * g[0][2];  // det / 6
  if (!(V > 0.0)) return false;
  const double iv = 1.0 / V;
  double L[3][3];  // sum_k du_k (x) grad_x N_k
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) L[i][j] = (du[0][i] * g[0][j] + du[1][i] * g[1][j] + du[2][i] * g[2][j]) * iv;
  double sg[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) sg[i][j] = eta * (L[i][j] + L[j][i]);
  if (Cp) {
    constexpr int sym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        double cs = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) cs += (double)Cp[sym[i][j] * N + ids[k]];
        const double pj = G * (cs * 0.25 - (i == j ? 1.0 : 0.0));
        sg[i][j] += pj;
        if (j != i) sg[j][i] += pj;
      }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    fk[0][i] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fk[k + 1][i] = sg[i][0] * g[k][0] + sg[i][1] * g[k][1] + sg[i][2] * g[k][2];
      fk[0][i] -= fk[k + 1][i];
    }
  }
  return true;
}

// One workgroup per particle that fits its LDS (larger ones: the global path below); particles without tetrahedra return at once.
// Element forces are accumulated in LDS (float64) colour by colour, then
// added to f once per node.
template <typename T>
__global__ void __launch_bounds__(512) k_fluid(const ForceArgs a, const T* __restrict__ x, const T* __restrict__ v,
                                               const T* __restrict__ C, double eta, double G, T* __restrict__ f) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int p = a.lds_part ? a.lds_part[blockIdx.x] : (int)blockIdx.x;
  if (a.pcol_tet[p] == a.pcol_tet[p + 1]) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n0 = a.node_start[p];
  const int nn = a.node_start[p + 1] - n0;
  const int64_t N = a.n_nodes;
  double* acc = reinterpret_cast<double*>(smem_raw);  // [3][cap]
  for (int i = tid; i < nn; i += nt) {
    acc[i] = 0.0;
    acc[a.cap_solid + i] = 0.0;
    acc[2 * a.cap_solid + i] = 0.0;
  }
  __syncthreads();
  const T* xx = x + n0;
  const T* vx = v + n0;
  const T* Cp = C ? C + n0 : nullptr;
  double o[3] = {0.0, 0.0, 0.0};
  if (sizeof(T) == 8) {
    o[0] = (double)xx[0];
    o[1] = (double)xx[N];
    o[2] = (double)xx[2 * N];
  }
  for (int col = a.pcol_tet[p]; col < a.pcol_tet[p + 1]; ++col) {
    const int e1 = a.colb_tet[col + 1];
    for (int s = a.colb_tet[col] + tid; s < e1; s += nt) {
      int ids[4];
      double q[4][3], u[4][3];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ids[k] = a.tet_local[k * a.n_tets + s];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          q[k][c] = (double)xx[c * N + ids[k]] - o[c];
          u[k][c] = (double)vx[c * N + ids[k]];
        }
      }
      double fk[4][3];
      if (!fluid_tet(q, u, Cp, N, ids, eta, G, fk)) continue;  // inverted or flat: no force (counted by the elastic pass)
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c * a.cap_solid + ids[k]] += fk[k][c];
    }
    __syncthreads();
  }
  for (int i = tid; i < nn; i += nt)
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c * N + n0 + i] = (T)((double)f[c * N + n0 + i] + acc[c * a.cap_solid + i]);
}

// Solids too large for one workgroup's LDS: each tetrahedron's corner forces
// into the element scratch (float64), then one thread per node adds its
// tetrahedra's shares in element order (deterministic) to f.
template <typename T>
__global__ void __launch_bounds__(256) k_large_fluid_elems(const ForceArgs a, const LargeArgs L,
                                                            const T* __restrict__ x, const T* __restrict__ v,
                                                            const T* __restrict__ C, double eta, double G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n_tet) return;
  const int s = L.tet_slot[t], p = L.tet_part[t];
  const int n0 = a.node_start[p];
  const int64_t N = a.n_nodes;
  double o[3] = {0.0, 0.0, 0.0};
  if (sizeof(T) == 8)
    for (int c = 0; c < 3; ++c) o[c] = (double)x[c * N + n0];
  int ids[4];
  double q[4][3], u[4][3];
  for (int k = 0; k < 4; ++k) {
    ids[k] = a.tet_local[k * a.n_tets + s];
    for (int c = 0; c < 3; ++c) {
      q[k][c] = (double)x[c * N + n0 + ids[k]] - o[c];
      u[k][c] = (double)v[c * N + n0 + ids[k]];
    }
  }
  double fk[4][3];
  if (!fluid_tet(q, u, C ? C + n0 : (const T*)nullptr, N, ids, eta, G, fk))
    for (int k = 0; k < 4; ++k) fk[k][0] = fk[k][1] = fk[k][2] = 0.0;
  double* ef = reinterpret_cast<double*>(L.ef_tet);  // [4 corners][n_tet][4]
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 3; ++c) ef[((int64_t)k * L.n_tet + t) * 4 + c] = fk[k][c];
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_fluid_gather(const ForceArgs a, const LargeArgs L, T* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_node) return;
  const int p = L.node_part[i];
  if (a.pcol_tet[p] == a.pcol_tet[p + 1]) return;
  const int k = a.node_start[p] + (i - L.node_base[i]);
  const double* ef = reinterpret_cast<const double*>(L.ef_tet);
  double s[3] = {0.0, 0.0, 0.0};
  for (int j = L.gather_start[i]; j < L.gather_start[i + 1]; ++j) {
    const int g = L.gather[j];  // element e and corner v: e * 4 + v, tetrahedra after the triangles
    const int e = (g >> 2) - L.n_tri, v = g & 3;
    if (e < 0) continue;
    for (int c = 0; c < 3; ++c) s[c] += ef[((int64_t)v * L.n_tet + e) * 4 + c];
  }
  const int64_t N = a.n_nodes;
  for (int c = 0; c < 3; ++c) f[c * N + k] = (T)((double)f[c * N + k] + s[c]);
}

// ------------------------------------------------------------------ host launchers
static size_t fluid_lds(const PlanDev& P) { return (size_t)3 * std::max(P.fargs.cap_solid, 1) * sizeof(double); }

hipError_t prepare_fluid_kernels(const PlanDev& P) {
  const int lds = (int)fluid_lds(P);
  hipError_t e = hipFuncSetAttribute((const void*)k_fluid<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fluid<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  return e;
}

hipError_t launch_interp_cells(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* grid,
                               int ncomp, void* out, hipStream_t st) {
  if (P.n_nodes == 0) return hipSuccess;
  P.timer->begin(K_INTERP_CELLS, st);
  const int block = 256;
  const dim3 g((unsigned)((P.n_nodes + block - 1) / block));
  if (dtype == 0)
    hipLaunchKernelGGL(k_interp_cells<float>, g, dim3(block), 0, st, P.targs, (const float*)x, anchor,
                       (const float*)grid, ncomp, (float*)out);
  else
    hipLaunchKernelGGL(k_interp_cells<double>, g, dim3(block), 0, st, P.targs, (const double*)x, anchor,
                       (const double*)grid, ncomp, (double*)out);
  P.timer->end(st);
  return hipGetLastError();
}

hipError_t launch_fluid(const PlanDev& P, int dtype, const void* x, const void* v, const void* C, double eta, double G,
                        void* f, hipStream_t st) {
  if (P.n_tets == 0) return hipSuccess;
  P.timer->begin(K_FLUID, st);
  const size_t lds = fluid_lds(P);
  if (P.n_lds_part > 0) {
    if (dtype == 0)
      hipLaunchKernelGGL(k_fluid<float>, dim3(P.n_lds_part), dim3(256), lds, st, P.fargs, (const float*)x,
                         (const float*)v, (const float*)C, eta, G, (float*)f);
    else
      hipLaunchKernelGGL(k_fluid<double>, dim3(P.n_lds_part), dim3(256), lds, st, P.fargs, (const double*)x,
                         (const double*)v, (const double*)C, eta, G, (double*)f);
  }
  const LargeArgs& L = P.large;
  if (L.n_tet > 0) {
    const int B = 256;
    const dim3 ge((L.n_tet + B - 1) / B), gn((L.n_node + B - 1) / B);
    if (dtype == 0) {
      hipLaunchKernelGGL(k_large_fluid_elems<float>, ge, dim3(B), 0, st, P.fargs, L, (const float*)x,
                         (const float*)v, (const float*)C, eta, G);
      hipLaunchKernelGGL(k_large_fluid_gather<float>, gn, dim3(B), 0, st, P.fargs, L, (float*)f);
    } else {
      hipLaunchKernelGGL(k_large_fluid_elems<double>, ge, dim3(B), 0, st, P.fargs, L, (const double*)x,
                         (const double*)v, (const double*)C, eta, G);
      hipLaunchKernelGGL(k_large_fluid_gather<double>, gn, dim3(B), 0, st, P.fargs, L, (double*)f);
    }
  }
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
