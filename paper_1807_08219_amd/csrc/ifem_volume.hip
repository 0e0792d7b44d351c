// Membrane volume conservation (Sec. II.E): the displacement that restores each
// membrane's enclosed volume with the least sum of squared nodal moves.
//
// The cost function of Sec. II.E (squared displacements plus a Lagrange
// multiplier times the volume error) is stationary at dx_I = L alpha_I, where
// alpha_I is -1/2 of the gradient of the enclosed volume with respect to node
// I: -1/12 times the sum, over the faces at I, of the cross product of the
// face's other two nodes in the face's cyclic order.  The volume after the move
// is the cubic A L^3 + B L^2 + C L + D of the section, whose coefficients are
// sums over faces f = (1, 2, 3) of triple products:
//   A = 1/18 sum_f [a1.(a2 x a3) + a2.(a3 x a1) + a3.(a1 x a2)],
//   B = 1/6  sum_f [x1.(a2 x a3) + x2.(a3 x a1) + x3.(a1 x a2)],
//   C = 1/6  sum_f [a1.(x2 x x3) + a2.(x3 x x1) + a3.(x1 x x2)],
//   D = V(x) - V0,  V = 1/18 sum_f [x1.(x2 x x3) + x2.(x3 x x1) + x3.(x1 x x2)].
// L is the root of smallest magnitude, reached by Newton's iteration from 0.
//
// Node-centric evaluation.  Every term above pairs one corner I of a face with
// the cross product of the face's other two corners, which in the ordered
// one-ring j_1..j_v of I (faces (I, j_m, j_m+1)) are consecutive neighbours.
// Gathering the terms by corner turns the face sums into node sums of one-ring
// sums, with no scatter:
//   alpha_I = -1/12 sum_m (x_jm - x_I) x (x_jm+1 - x_I)   (the x_I terms of a
//             closed fan cancel, so edge vectors give it without cancellation),
//   beta_I  = sum_m a_jm x a_jm+1,
//   A = 1/18 sum_I alpha_I . beta_I,   B = 1/6 sum_I x_I . beta_I,
//   C = 1/6 sum_I alpha_I . (-12 alpha_I) = -2 sum_I |alpha_I|^2,
//   V = 1/18 sum_I x_I . (-12 alpha_I) = -2/3 sum_I x_I . alpha_I.
//
// All arithmetic is float64.  Volume, alpha and the coefficients are unchanged
// by a translation of the closed surface, so positions enter in a
// particle-local frame: the float32 offsets themselves (already
// particle-relative), or the float64 positions minus the particle's first node.
#include <algorithm>

#include "ifem_internal.hpp"

namespace ifem {

// One-ring neighbours gathered per batch of loads: the typical degree of a
// closed triangulation (its mean tends to 6).
constexpr int kRingChunk = 6;

// s += u x w with every product rounded on its own (no fused multiply-add), so
// that u x u is exactly zero: a ring's last chunk is padded by repeating its
// last neighbour, whose term must vanish.
__device__ __forceinline__ void cross_acc(const double u[3], const double w[3], double& sx, double& sy, double& sz) {
#pragma clang fp contract(off)
  sx += u[1] * w[2] - u[2] * w[1];
  sy += u[2] * w[0] - u[0] * w[2];
  sz += u[0] * w[1] - u[1] * w[0];
}

// The multiplier L from the four node sums r (alpha.beta, x.beta, |alpha|^2,
// x.alpha): the cubic's coefficients, then Newton's iteration from 0.  A run
// that does not converge to a finite root is counted in status[4].
__device__ inline double volume_multiplier(const double r[4], double target, unsigned long long* status) {
  const double A = r[0] * (1.0 / 18.0), B = r[1] * (1.0 / 6.0), C = -2.0 * r[2];
  const double D = r[3] * (-2.0 / 3.0) - target;
  double L = 0.0;
  bool done = false;
  for (int it = 0; it < 100 && !done; ++it) {
    const double f = ((A * L + B) * L + C) * L + D;
    const double df = (3.0 * A * L + 2.0 * B) * L + C;
    const double step = f / df;
    L -= step;
    done = fabs(step) <= 1e-15 * fabs(L) || f == 0.0;
  }
  if (!done || !isfinite(L)) atomicAdd(status + 4, 1ull);
  return L;
}

// One workgroup per particle: alpha of every node in LDS (float64), two node
// passes, a block reduction, the cubic solved by one thread, the write-out.
// Positions and one-rings are gathered from global memory (the caches): the
// float64 alpha of a red cell already takes 61 KB of LDS, and staging the
// positions and rings beside it would leave room for one workgroup per compute
// unit instead of two, which measured slower.  Each node's offsets and position
// are requested one iteration ahead.  x and x_out may be the same array: each
// thread rewrites only the nodes whose positions it reads in the write-out,
// after the workgroup's last other read.
template <typename T>
__global__ void __launch_bounds__(512) k_volume(const ForceArgs a, const T* x, const double* __restrict__ V0,
                                                 const double* __restrict__ vref, T* x_out,
                                                 double* __restrict__ lam_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_lds[4 * 16];
  __shared__ double lam_s;
  const int p = a.lds_part ? a.lds_part[blockIdx.x] : (int)blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n0 = a.node_start[p];
  const int nn = a.node_start[p + 1] - n0;
  const int64_t N = a.n_nodes;
  if (a.colb_tri[a.pcol_tri[p]] == a.colb_tri[a.pcol_tri[p + 1]]) {  // solids (no faces) keep their nodes
    if (x_out != x)
      for (int i = tid; i < nn; i += nt)
        for (int c = 0; c < 3; ++c) x_out[c * N + n0 + i] = x[c * N + n0 + i];
    if (lam_out && tid == 0) lam_out[p] = 0.0;
    return;
  }
  double* al = reinterpret_cast<double*>(smem_raw);  // [3][cap] alpha
  const T* xx = x + n0;
  const T* xy = x + N + n0;
  const T* xz = x + 2 * N + n0;
  const int32_t* rs = a.ring_start + n0;
  const int32_t* __restrict__ ring = a.ring;
  double o[3] = {0.0, 0.0, 0.0};
  if (sizeof(T) == 8) {
    o[0] = (double)xx[0];
    o[1] = (double)xy[0];
    o[2] = (double)xz[0];
  }
  double r[4] = {0.0, 0.0, 0.0, 0.0};  // sum alpha.beta, sum x.beta, sum |alpha|^2, sum x.alpha

  // --- alpha from the one-ring edge vectors.  Neighbours are taken a chunk at a
  // time: their ids, then their positions, are all requested before any is used,
  // so the loads of one chunk are in flight together.  Ids past the ring's end
  // repeat its last entry, whose edge vector equals the running u: the term
  // u x u is exactly zero and u stays (no branch, which would sink each load
  // into its own guarded block).
  int k = tid;
  int rb_n = 0, re_n = 0;
  T xk_n[3] = {T(0), T(0), T(0)};
  if (k < nn) {
    rb_n = rs[k];
    re_n = rs[k + 1];
    xk_n[0] = xx[k];
    xk_n[1] = xy[k];
    xk_n[2] = xz[k];
  }
  for (; k < nn; k += nt) {
    const int rb = rb_n, re = re_n;
    const double xk[3] = {(double)xk_n[0], (double)xk_n[1], (double)xk_n[2]};
    const int kn = min(k + nt, nn - 1);  // the next node's offsets and position, requested now
    rb_n = rs[kn];
    re_n = rs[kn + 1];
    xk_n[0] = xx[kn];
    xk_n[1] = xy[kn];
    xk_n[2] = xz[kn];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (re > rb) {
      int j = ring[re - 1];
      double u[3] = {(double)xx[j] - xk[0], (double)xy[j] - xk[1], (double)xz[j] - xk[2]};
      for (int m0 = rb; m0 < re; m0 += kRingChunk) {
        int js[kRingChunk];
#pragma unroll
        for (int q = 0; q < kRingChunk; ++q) js[q] = ring[min(m0 + q, re - 1)];
        T wx[kRingChunk], wy[kRingChunk], wz[kRingChunk];
#pragma unroll
        for (int q = 0; q < kRingChunk; ++q) {
          wx[q] = xx[js[q]];
          wy[q] = xy[js[q]];
          wz[q] = xz[js[q]];
        }
#pragma unroll
        for (int q = 0; q < kRingChunk; ++q) {
          const double w[3] = {(double)wx[q] - xk[0], (double)wy[q] - xk[1], (double)wz[q] - xk[2]};
          cross_acc(u, w, sx, sy, sz);
          u[0] = w[0];
          u[1] = w[1];
          u[2] = w[2];
        }
      }
    }
    const double ax = sx * (-1.0 / 12.0), ay = sy * (-1.0 / 12.0), az = sz * (-1.0 / 12.0);
    al[k] = ax;
    al[a.cap_mem + k] = ay;
    al[2 * a.cap_mem + k] = az;
    r[2] += ax * ax + ay * ay + az * az;
    r[3] += (xk[0] - o[0]) * ax + (xk[1] - o[1]) * ay + (xk[2] - o[2]) * az;
  }
  __syncthreads();
  // --- beta from the neighbours' alpha (the same chunked gathers and padding, from LDS)
  k = tid;
  if (k < nn) {
    rb_n = rs[k];
    re_n = rs[k + 1];
    xk_n[0] = xx[k];
    xk_n[1] = xy[k];
    xk_n[2] = xz[k];
  }
  for (; k < nn; k += nt) {
    const int rb = rb_n, re = re_n;
    const double xk[3] = {(double)xk_n[0] - o[0], (double)xk_n[1] - o[1], (double)xk_n[2] - o[2]};
    const int kn = min(k + nt, nn - 1);
    rb_n = rs[kn];
    re_n = rs[kn + 1];
    xk_n[0] = xx[kn];
    xk_n[1] = xy[kn];
    xk_n[2] = xz[kn];
    if (re == rb) continue;
    double bx = 0.0, by = 0.0, bz = 0.0;
    int j = ring[re - 1];
    double u[3] = {al[j], al[a.cap_mem + j], al[2 * a.cap_mem + j]};
    for (int m0 = rb; m0 < re; m0 += kRingChunk) {
      int js[kRingChunk];
#pragma unroll
      for (int q = 0; q < kRingChunk; ++q) js[q] = ring[min(m0 + q, re - 1)];
      double w[kRingChunk][3];
#pragma unroll
      for (int q = 0; q < kRingChunk; ++q) {
        w[q][0] = al[js[q]];
        w[q][1] = al[a.cap_mem + js[q]];
        w[q][2] = al[2 * a.cap_mem + js[q]];
      }
#pragma unroll
      for (int q = 0; q < kRingChunk; ++q) {
        cross_acc(u, w[q], bx, by, bz);
        u[0] = w[q][0];
        u[1] = w[q][1];
        u[2] = w[q][2];
      }
    }
    r[0] += al[k] * bx + al[a.cap_mem + k] * by + al[2 * a.cap_mem + k] * bz;
    r[1] += xk[0] * bx + xk[1] * by + xk[2] * bz;
  }
  block_sum<4>(r, red_lds);
  if (tid == 0) {
    const double L = volume_multiplier(r, V0 ? V0[p] : vref[p], a.status);
    lam_s = L;
    if (lam_out) lam_out[p] = L;
  }
  __syncthreads();
  const double L = lam_s;
  // two nodes per iteration, both read before either is written (x_out may be x)
  for (int i = tid; i < nn; i += 2 * nt) {
    const int i2 = min(i + nt, nn - 1);
    const T p1[3] = {xx[i], xy[i], xz[i]};
    const T p2[3] = {xx[i2], xy[i2], xz[i2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) x_out[c * N + n0 + i] = (T)((double)p1[c] + L * al[c * a.cap_mem + i]);
    if (i + nt < nn)
#pragma unroll
      for (int c = 0; c < 3; ++c) x_out[c * N + n0 + i2] = (T)((double)p2[c] + L * al[c * a.cap_mem + i2]);
  }
}

// ------------------------------------------------------------------ membranes larger than a workgroup's LDS
// The same sums with alpha in global memory (float64), one thread per node and
// a launch per dependency: alpha (needs positions), beta (needs every
// neighbour's alpha), the multiplier (one workgroup per particle sums the node
// terms in a fixed order), the move.  Solids among the large particles keep
// their nodes.  x and x_out may be the same array: the move reads only the
// node it writes, after every other read has finished.
template <typename T>
__global__ void __launch_bounds__(256) k_large_vol_alpha(const ForceArgs a, const LargeArgs L, const T* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_node) return;
  const int p = L.node_part[i];
  if (a.pcol_tri[p] == a.pcol_tri[p + 1]) return;
  const int n0 = a.node_start[p], k = i - L.node_base[i];
  const int64_t N = a.n_nodes;
  const T* xx = x + n0;
  const T* xy = x + N + n0;
  const T* xz = x + 2 * N + n0;
  double o[3] = {0.0, 0.0, 0.0};
  if (sizeof(T) == 8) {
    o[0] = (double)xx[0];
    o[1] = (double)xy[0];
    o[2] = (double)xz[0];
  }
  const int32_t* rs = a.ring_start + n0;
  const int rb = rs[k], re = rs[k + 1];
  const double xk[3] = {(double)xx[k], (double)xy[k], (double)xz[k]};
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (re > rb) {
    int j = a.ring[re - 1];
    double u[3] = {(double)xx[j] - xk[0], (double)xy[j] - xk[1], (double)xz[j] - xk[2]};
    for (int m = rb; m < re; ++m) {
      j = a.ring[m];
      const double w[3] = {(double)xx[j] - xk[0], (double)xy[j] - xk[1], (double)xz[j] - xk[2]};
      cross_acc(u, w, sx, sy, sz);
      u[0] = w[0];
      u[1] = w[1];
      u[2] = w[2];
    }
  }
  const double ax = sx * (-1.0 / 12.0), ay = sy * (-1.0 / 12.0), az = sz * (-1.0 / 12.0);
  double* al = reinterpret_cast<double*>(L.fb);
  const int64_t M = L.n_node;
  al[i] = ax;
  al[M + i] = ay;
  al[2 * M + i] = az;
  L.vol_terms[2 * M + i] = ax * ax + ay * ay + az * az;
  L.vol_terms[3 * M + i] = (xk[0] - o[0]) * ax + (xk[1] - o[1]) * ay + (xk[2] - o[2]) * az;
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_vol_beta(const ForceArgs a, const LargeArgs L, const T* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_node) return;
  const int p = L.node_part[i];
  if (a.pcol_tri[p] == a.pcol_tri[p + 1]) return;
  const int n0 = a.node_start[p], lb = L.node_base[i], k = i - lb;
  const int64_t N = a.n_nodes, M = L.n_node;
  double o[3] = {0.0, 0.0, 0.0};
  if (sizeof(T) == 8)
    for (int c = 0; c < 3; ++c) o[c] = (double)x[c * N + n0];
  const double xk[3] = {(double)x[n0 + k] - o[0], (double)x[N + n0 + k] - o[1], (double)x[2 * N + n0 + k] - o[2]};
  const double* al = reinterpret_cast<const double*>(L.fb) + lb;  // the particle's alpha
  const int32_t* rs = a.ring_start + n0;
  const int rb = rs[k], re = rs[k + 1];
  double bx = 0.0, by = 0.0, bz = 0.0;
  if (re > rb) {
    int j = a.ring[re - 1];
    double u[3] = {al[j], al[M + j], al[2 * M + j]};
    for (int m = rb; m < re; ++m) {
      j = a.ring[m];
      const double w[3] = {al[j], al[M + j], al[2 * M + j]};
      cross_acc(u, w, bx, by, bz);
      u[0] = w[0];
      u[1] = w[1];
      u[2] = w[2];
    }
  }
  L.vol_terms[i] = al[k] * bx + al[M + k] * by + al[2 * M + k] * bz;
  L.vol_terms[M + i] = xk[0] * bx + xk[1] * by + xk[2] * bz;
}

// One workgroup per large particle: the node terms summed (thread-strided in
// node order, then the fixed block sum), the multiplier into lam[lp].
__global__ void __launch_bounds__(256) k_large_vol_solve(const ForceArgs a, const LargeArgs L,
                                                          const double* __restrict__ V0,
                                                          const double* __restrict__ vref, double* __restrict__ lam,
                                                          double* __restrict__ lam_out) {
  __shared__ double red_lds[4 * 16];
  const int lp = blockIdx.x, p = L.part[lp];
  const int n0 = a.node_start[p], nn = a.node_start[p + 1] - n0;
  if (a.pcol_tri[p] == a.pcol_tri[p + 1]) {
    if (threadIdx.x == 0) {
      lam[lp] = 0.0;
      if (lam_out) lam_out[p] = 0.0;
    }
    return;
  }
  const int lb = L.part_base[lp];  // the particle's nodes are contiguous in the compact numbering
  const int64_t M = L.n_node;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nn; k += blockDim.x)
    for (int c = 0; c < 4; ++c) r[c] += L.vol_terms[c * M + lb + k];
  block_sum<4>(r, red_lds);
  if (threadIdx.x == 0) {
    const double Lm = volume_multiplier(r, V0 ? V0[p] : vref[p], a.status);
    lam[lp] = Lm;
    if (lam_out) lam_out[p] = Lm;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_large_vol_apply(const ForceArgs a, const LargeArgs L, const T* x,
                                                          const double* __restrict__ lam, T* x_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_node) return;
  const int p = L.node_part[i];
  const int k = a.node_start[p] + (i - L.node_base[i]);
  const int64_t N = a.n_nodes, M = L.n_node;
  if (a.pcol_tri[p] == a.pcol_tri[p + 1]) {
    if (x_out != x)
      for (int c = 0; c < 3; ++c) x_out[c * N + k] = x[c * N + k];
    return;
  }
  const double Lm = lam[L.node_lp[i]];
  const double* al = reinterpret_cast<const double*>(L.fb);
  for (int c = 0; c < 3; ++c) x_out[c * N + k] = (T)((double)x[c * N + k] + Lm * al[c * M + i]);
}

// Reference volume of every membrane (float64 reference positions X [3][n_nodes]).
__global__ void __launch_bounds__(256) k_ref_volume(const ForceArgs a, const double* __restrict__ X,
                                                    double* __restrict__ vref) {
  __shared__ double red_lds[16];
  const int p = blockIdx.x;
  const int n0 = a.node_start[p];
  const int64_t N = a.n_nodes;
  const double o[3] = {X[n0], X[N + n0], X[2 * N + n0]};
  double r[1] = {0.0};
  for (int t = a.colb_tri[a.pcol_tri[p]] + threadIdx.x; t < a.colb_tri[a.pcol_tri[p + 1]]; t += blockDim.x) {
    double q[3][3];
    for (int v = 0; v < 3; ++v) {
      const int k = n0 + a.tri_local[v * a.n_tris + t];
      for (int c = 0; c < 3; ++c) q[v][c] = X[c * N + k] - o[c];
    }
    const double cx = q[1][1] * q[2][2] - q[1][2] * q[2][1], cy = q[1][2] * q[2][0] - q[1][0] * q[2][2],
                 cz = q[1][0] * q[2][1] - q[1][1] * q[2][0];
    r[0] += (q[0][0] * cx + q[0][1] * cy + q[0][2] * cz) * (1.0 / 6.0);
  }
  block_sum<1>(r, red_lds);
  if (threadIdx.x == 0) vref[p] = r[0];
}

// ------------------------------------------------------------------ host launchers
static size_t volume_lds(const PlanDev& P) { return (size_t)3 * std::max(P.fargs.cap_mem, 1) * sizeof(double); }

// Threads per workgroup: 512, or fewer for small particles.  Two 512-thread
// workgroups (16 waves) share a compute unit; 576 threads, which would save
// the sixth pass of a 2562-node red cell, measured slower.
static int volume_block(const PlanDev& P) { return std::max(64, std::min(512, (P.fargs.cap_mem + 63) / 64 * 64)); }

hipError_t prepare_volume_kernels(const PlanDev& P) {
  hipError_t e = hipFuncSetAttribute((const void*)k_volume<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)volume_lds(P));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_volume<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)volume_lds(P));
  return e;
}

hipError_t launch_ref_volume(const PlanDev& P, const double* X, double* vref, hipStream_t st) {
  if (P.n_particles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_volume, dim3(P.n_particles), dim3(256), 0, st, P.fargs, X, vref);
  return hipGetLastError();
}

hipError_t launch_volume(const PlanDev& P, int dtype, const void* x, const double* V0, void* x_out, double* lam,
                         hipStream_t st) {
  if (P.n_particles == 0) return hipSuccess;
  P.timer->begin(K_VOLUME, st);
  const LargeArgs& L = P.large;
  const int B = 256;
  const dim3 gn((L.n_node + B - 1) / B);
  // the large membranes read x before the per-particle kernel may rewrite it in place (x_out == x)
  if (L.n_part > 0) {
    if (dtype == 0) {
      hipLaunchKernelGGL(k_large_vol_alpha<float>, gn, dim3(B), 0, st, P.fargs, L, (const float*)x);
      hipLaunchKernelGGL(k_large_vol_beta<float>, gn, dim3(B), 0, st, P.fargs, L, (const float*)x);
    } else {
      hipLaunchKernelGGL(k_large_vol_alpha<double>, gn, dim3(B), 0, st, P.fargs, L, (const double*)x);
      hipLaunchKernelGGL(k_large_vol_beta<double>, gn, dim3(B), 0, st, P.fargs, L, (const double*)x);
    }
    hipLaunchKernelGGL(k_large_vol_solve, dim3(L.n_part), dim3(B), 0, st, P.fargs, L, V0, P.vref, L.lam, lam);
    if (dtype == 0)
      hipLaunchKernelGGL(k_large_vol_apply<float>, gn, dim3(B), 0, st, P.fargs, L, (const float*)x, L.lam,
                         (float*)x_out);
    else
      hipLaunchKernelGGL(k_large_vol_apply<double>, gn, dim3(B), 0, st, P.fargs, L, (const double*)x, L.lam,
                         (double*)x_out);
  }
  if (P.n_lds_part > 0) {
    const dim3 g(P.n_lds_part), b(volume_block(P));
    if (dtype == 0)
      hipLaunchKernelGGL(k_volume<float>, g, b, volume_lds(P), st, P.fargs, (const float*)x, V0, P.vref,
                         (float*)x_out, lam);
    else
      hipLaunchKernelGGL(k_volume<double>, g, b, volume_lds(P), st, P.fargs, (const double*)x, V0, P.vref,
                         (double*)x_out, lam);
  }
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
