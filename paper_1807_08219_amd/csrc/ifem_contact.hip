// Node-face anti-sticking (Sec. III.B): every node closer than d_min to a face
// of another particle of its box moves away from the closest point of that
// face until it is d_min from it.  The paper finds candidate pairs with a
// bounding-box check and searches them densely; here one uniform grid of
// coarse cells per box (4 lattice cells wide) replaces both: nodes are binned
// by cell, and every face visits the cells its bounding box, grown by d_min,
// covers.  A face within d_min of a node always visits the node's cell, so the
// search is exact; a cell whose nodes all belong to the face's own particle is
// skipped whole.
//
//  k_ac_count<T>  per node: its cell; one atomic per distinct cell and wavefront;
//  (k_scan)       cell offsets;
//  k_ac_fill<T>   per node: writes the node id into its cell's list;
//  k_ac_owner     per cell: the particle owning all its nodes, -2 if mixed, -1 empty;
//  k_ac_faces<T>  per face: for the nodes of other particles in the cells it
//                 reaches, the distance to the face (float64, the face's
//                 periodic image nearest to the node); below d_min, an atomic minimum of the key
//                 (float32 distance, face id) per node;
//  k_ac_push<T>   per node: the move from its winning face, or a copy.
//
// The key orders faces by float32 distance, then face id, so the choice is
// deterministic; positions are float64 throughout.
#include "ifem_internal.hpp"

namespace ifem {

constexpr unsigned long long kNoFace = ~0ull;

// Closest point to the origin on triangle (a, b, c): the Voronoi-region tests
// of Ericson (Real-Time Collision Detection, 2005, Sec. 5.1.5), vertex regions,
// then edge regions, then the face.  A triangle of zero area that reaches the
// face case falls back to the nearest of its edges.  No fused multiply-add, so
// the search and the move compute the same point bit for bit.
__device__ __forceinline__ void seg_closest0(const double a[3], const double b[3], double out[3]) {
#pragma clang fp contract(off)
  const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
  double t = L2 > 0.0 ? -(a[0] * ab[0] + a[1] * ab[1] + a[2] * ab[2]) / L2 : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  for (int i = 0; i < 3; ++i) out[i] = a[i] + t * ab[i];
}

__device__ __forceinline__ void closest_on_triangle0(const double a[3], const double b[3], const double c[3],
                                                     double out[3]) {
#pragma clang fp contract(off)
  const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double d1 = -(ab[0] * a[0] + ab[1] * a[1] + ab[2] * a[2]);
  const double d2 = -(ac[0] * a[0] + ac[1] * a[1] + ac[2] * a[2]);
  if (d1 <= 0.0 && d2 <= 0.0) {
    for (int i = 0; i < 3; ++i) out[i] = a[i];
    return;
  }
  const double d3 = -(ab[0] * b[0] + ab[1] * b[1] + ab[2] * b[2]);
  const double d4 = -(ac[0] * b[0] + ac[1] * b[1] + ac[2] * b[2]);
  if (d3 >= 0.0 && d4 <= d3) {
    for (int i = 0; i < 3; ++i) out[i] = b[i];
    return;
  }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    const double t = d1 / (d1 - d3);
    for (int i = 0; i < 3; ++i) out[i] = a[i] + t * ab[i];
    return;
  }
  const double d5 = -(ab[0] * c[0] + ab[1] * c[1] + ab[2] * c[2]);
  const double d6 = -(ac[0] * c[0] + ac[1] * c[1] + ac[2] * c[2]);
  if (d6 >= 0.0 && d5 <= d6) {
    for (int i = 0; i < 3; ++i) out[i] = c[i];
    return;
  }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    const double t = d2 / (d2 - d6);
    for (int i = 0; i < 3; ++i) out[i] = a[i] + t * ac[i];
    return;
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
    const double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) out[i] = b[i] + t * (c[i] - b[i]);
    return;
  }
  const double den = va + vb + vc;
  if (!(den > 0.0)) {  // zero area: the nearest edge
    double q[3][3], best = 1e308;
    seg_closest0(a, b, q[0]);
    seg_closest0(b, c, q[1]);
    seg_closest0(c, a, q[2]);
    for (int e = 0; e < 3; ++e) {
      const double dd = q[e][0] * q[e][0] + q[e][1] * q[e][1] + q[e][2] * q[e][2];
      if (dd < best) {
        best = dd;
        for (int i = 0; i < 3; ++i) out[i] = q[e][i];
      }
    }
    return;
  }
  const double v = vb / den, w = vc / den;
  for (int i = 0; i < 3; ++i) out[i] = a[i] + ab[i] * v + ac[i] * w;
}

template <typename T>
__device__ __forceinline__ void abs_position(const ContactArgs& a, const T* __restrict__ x,
                                             const double* __restrict__ anchor, int k, int p, double out[3]) {
  const int64_t N = a.n_nodes;
#pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = (sizeof(T) == 4 ? anchor[3 * p + i] : 0.0) + (double)x[i * N + k];
}

// Corners of a face relative to point xk, in the periodic image of the face
// nearest to xk: the image of the first corner, applied to all three (a face
// is one piece; wrapping each corner on its own could tear a face that sits
// half a box away).
__device__ __forceinline__ void face_image(const double pv[3][3], const double xk[3], const ContactBoxDev& C,
                                           double r[3][3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double shift = C.len[j] * rint((pv[0][j] - xk[j]) * C.inv_len[j]);
#pragma unroll
    for (int m = 0; m < 3; ++m) r[m][j] = pv[m][j] - xk[j] - shift;
  }
}

// |c|, summed in the order x, y, z without fused multiply-add.
__device__ __forceinline__ double norm_nc(const double c[3]) {
#pragma clang fp contract(off)
  return sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
}

__device__ __forceinline__ int cell_of(const ContactBoxDev& C, const double p[3]) {
  int idx[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int c = (int)floor((p[i] - C.origin[i]) * C.inv_cs[i]);
    c %= C.nc[i];
    idx[i] = c < 0 ? c + C.nc[i] : c;
  }
  return C.base + (idx[2] * C.nc[1] + idx[1]) * C.nc[0] + idx[0];
}

template <typename T>
__global__ void __launch_bounds__(256) k_ac_count(const ContactArgs a, const T* __restrict__ x,
                                                  const double* __restrict__ anchor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1;
  if (k < a.n_nodes) {
    const int p = a.node_particle[k];
    double pos[3];
    abs_position(a, x, anchor, k, p, pos);
    key = cell_of(a.boxes[a.particle_box[p]], pos);
  }
  int leader, rank, size;
  wave_groups(key, leader, rank, size);
  if (size > 0) atomicAdd(a.count + key, size);
}

template <typename T>
__global__ void __launch_bounds__(256) k_ac_fill(const ContactArgs a, const T* __restrict__ x,
                                                 const double* __restrict__ anchor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1;
  if (k < a.n_nodes) {
    const int p = a.node_particle[k];
    double pos[3];
    abs_position(a, x, anchor, k, p, pos);
    key = cell_of(a.boxes[a.particle_box[p]], pos);
  }
  int leader, rank, size;
  wave_groups(key, leader, rank, size);
  const int base = size > 0 ? atomicAdd(a.cursor + key, size) : 0;
  const int slot = __shfl(base, leader, kWave) + rank;
  if (key >= 0 && slot < a.n_nodes) a.list[slot] = k;
}

__global__ void __launch_bounds__(256) k_ac_owner(const ContactArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_cells) return;
  const int n = a.count[c], o = a.off[c];
  int owner = -1;
  for (int i = 0; i < n; ++i) {
    const int k = a.list[o + i];
    if ((unsigned)k >= (unsigned)a.n_nodes) continue;
    const int p = a.node_particle[k];
    owner = (owner == -1 || owner == p) ? p : -2;
  }
  a.owner[c] = owner;
}

// The corners of contact face f (global node ids) and its particle.
__device__ __forceinline__ void face_nodes(const ContactArgs& a, int f, int v[3]) {
  if (f < a.n_tris) {
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = a.tri[i * (int64_t)a.n_tris + f];
  } else {
    const int j = f - a.n_tris;
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = a.bface[i * (int64_t)a.n_bfaces + j];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ac_faces(const ContactArgs a, const T* __restrict__ x,
                                                  const double* __restrict__ anchor, double d_min,
                                                  unsigned long long* __restrict__ keys) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= a.n_tris + a.n_bfaces) return;
  int v[3];
  face_nodes(a, f, v);
  const int q = a.node_particle[v[0]];
  const int b = a.particle_box[q];
  const ContactBoxDev C = a.boxes[b];
  double pv[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) abs_position(a, x, anchor, v[m], q, pv[m]);
  int lo[3], cnt[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double mn = fmin(pv[0][i], fmin(pv[1][i], pv[2][i]));
    const double mx = fmax(pv[0][i], fmax(pv[1][i], pv[2][i]));
    // a face that is not finite or spans half a box belongs to a broken mesh: skipped
    if (!(mx - mn <= 0.5 * C.len[i])) return;
    lo[i] = (int)floor((mn - d_min - C.origin[i]) * C.inv_cs[i]);
    const int hi = (int)floor((mx + d_min - C.origin[i]) * C.inv_cs[i]);
    cnt[i] = min(hi - lo[i] + 1, C.nc[i]);  // a range wider than the box visits each cell once
  }
  const float dmin32 = (float)d_min;
  for (int iz = 0; iz < cnt[2]; ++iz)
    for (int iy = 0; iy < cnt[1]; ++iy)
      for (int ix = 0; ix < cnt[0]; ++ix) {
        int c[3] = {lo[0] + ix, lo[1] + iy, lo[2] + iz};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          c[i] %= C.nc[i];
          c[i] = c[i] < 0 ? c[i] + C.nc[i] : c[i];
        }
        const int cell = C.base + (c[2] * C.nc[1] + c[1]) * C.nc[0] + c[0];
        const int owner = a.owner[cell];
        if (owner == -1 || owner == q) continue;
        const int o = a.off[cell], n = a.count[cell];
        for (int i = 0; i < n; ++i) {
          const int k = a.list[o + i];
          if ((unsigned)k >= (unsigned)a.n_nodes) continue;
          const int p = a.node_particle[k];
          if (p == q) continue;
          double xk[3];
          abs_position(a, x, anchor, k, p, xk);
          double r[3][3];
          face_image(pv, xk, C, r);
          double cp[3];
          closest_on_triangle0(r[0], r[1], r[2], cp);
          const float dist = (float)norm_nc(cp);
          if (dist < dmin32)
            atomicMin(keys + k, ((unsigned long long)__float_as_uint(dist) << 32) | (unsigned)f);
        }
      }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ac_push(const ContactArgs a, const T* __restrict__ x,
                                                 const double* __restrict__ anchor, double d_min,
                                                 const unsigned long long* __restrict__ keys, T* __restrict__ x_out,
                                                 int64_t* __restrict__ face_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_nodes) return;
  const int64_t N = a.n_nodes;
  const unsigned long long key = keys[k];
  if (key == kNoFace) {
#pragma unroll
    for (int i = 0; i < 3; ++i) x_out[i * N + k] = x[i * N + k];
    if (face_out) face_out[k] = -1;
    return;
  }
  const int f = (int)(key & 0xffffffffull);
  const int p = a.node_particle[k];
  double xk[3];
  abs_position(a, x, anchor, k, p, xk);
  int v[3];
  face_nodes(a, f, v);
  const int q = a.node_particle[v[0]];
  const ContactBoxDev C = a.boxes[a.particle_box[q]];
  double pv[3][3], r[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) abs_position(a, x, anchor, v[m], q, pv[m]);
  face_image(pv, xk, C, r);
  double cp[3];
  closest_on_triangle0(r[0], r[1], r[2], cp);
  const double dc = norm_nc(cp);
  double dir[3];
  if (dc > 0.0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) dir[i] = -cp[i] / dc;  // from the closest point to the node
  } else {  // on the face: its normal
    const double e1[3] = {r[1][0] - r[0][0], r[1][1] - r[0][1], r[1][2] - r[0][2]};
    const double e2[3] = {r[2][0] - r[0][0], r[2][1] - r[0][1], r[2][2] - r[0][2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) dir[i] = n[i] / nn;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double moved = xk[i] + cp[i] + d_min * dir[i];
    x_out[i * N + k] = (T)(sizeof(T) == 4 ? moved - anchor[3 * p + i] : moved);
  }
  if (face_out) face_out[k] = f;
}

// ------------------------------------------------------------------ host launcher
hipError_t launch_antistick(const PlanDev& P, int dtype, const void* x, const double* anchor, double d_min,
                            void* x_out, int64_t* face_out, hipStream_t st) {
  if (P.n_nodes == 0) return hipSuccess;
  const ContactArgs& a = P.cargs;
  const int B = 256;
  const dim3 gn((unsigned)((P.n_nodes + B - 1) / B)), gc((unsigned)((a.n_cells + B - 1) / B));
  const int nf = a.n_tris + a.n_bfaces;
  hipError_t e;
  P.timer->begin(K_FILL, st);
  e = launch_fill_i32(a.count, a.n_cells, 0, st);
  if (e == hipSuccess) e = launch_fill_u64(a.keys, a.n_nodes, kNoFace, st);
  P.timer->end(st);
  if (e != hipSuccess) return e;
  P.timer->begin(K_CONTACT, st);
  if (dtype == 0)
    hipLaunchKernelGGL(k_ac_count<float>, gn, dim3(B), 0, st, a, (const float*)x, anchor);
  else
    hipLaunchKernelGGL(k_ac_count<double>, gn, dim3(B), 0, st, a, (const double*)x, anchor);
  e = launch_scan(a.n_cells, a.count, a.off, a.cursor, (int64_t)a.n_nodes, P.status, st);
  if (e != hipSuccess) return e;
  if (dtype == 0)
    hipLaunchKernelGGL(k_ac_fill<float>, gn, dim3(B), 0, st, a, (const float*)x, anchor);
  else
    hipLaunchKernelGGL(k_ac_fill<double>, gn, dim3(B), 0, st, a, (const double*)x, anchor);
  hipLaunchKernelGGL(k_ac_owner, gc, dim3(B), 0, st, a);
  if (nf > 0) {
    const dim3 gf((unsigned)((nf + B - 1) / B));
    if (dtype == 0)
      hipLaunchKernelGGL(k_ac_faces<float>, gf, dim3(B), 0, st, a, (const float*)x, anchor, d_min, a.keys);
    else
      hipLaunchKernelGGL(k_ac_faces<double>, gf, dim3(B), 0, st, a, (const double*)x, anchor, d_min, a.keys);
  }
  if (dtype == 0)
    hipLaunchKernelGGL(k_ac_push<float>, gn, dim3(B), 0, st, a, (const float*)x, anchor, d_min, a.keys,
                       (float*)x_out, face_out);
  else
    hipLaunchKernelGGL(k_ac_push<double>, gn, dim3(B), 0, st, a, (const double*)x, anchor, d_min, a.keys,
                       (double*)x_out, face_out);
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
