// Node-face anti-sticking (Sec. III.B): every node closer than d_min to a face
// of another particle of its box moves away from the closest point of that
// face until it is d_min from it.  The paper finds candidate pairs with a
// bounding-box check and searches them densely; here one uniform grid of
// coarse cells per box (2 lattice cells wide) replaces both: nodes are binned
// by cell, and every face visits the cells its bounding box, grown by d_min,
// covers.  A face within d_min of a node always visits the node's cell, so the
// search is exact; a cell whose nodes all belong to the face's own particle is
// skipped whole.
//
//  k_ac_count<T>  per node: its cell; one atomic per distinct cell and wavefront;
//                 the node's least distance and face cleared;
//  k_cscan        cell offsets (any disjoint placement: one pass, a running
//                 total per workgroup chunk), owners cleared;
//  k_ac_fill<T>   per node: a record {position, node, particle} in its cell's list,
//                 and the cell's owner: the particle of all its nodes, -2 if
//                 mixed, -1 empty (a compare-and-swap per wavefront group);
//  k_ac_near      per cell: the least and greatest owner over the 3^3 cells around
//                 it, so that a face whose whole neighbourhood holds only its own
//                 particle is dropped at once;
//  k_ac_faces<T>  per face: the cells it reaches that hold nodes of other
//                 particles, appended as (face, cell) work items to one of
//                 kWorkSegs segments (one counter per segment); a face reaching
//                 more than 27 cells, or a full segment, goes to the slow list;
//  k_ac_pairs<T>  per work item: the face against the cell's records, the distance
//                 (float64, the face's periodic image nearest to the node);
//                 below d_min, an atomic minimum of the distance's float64 bits
//                 per node, and the item joins the hit list;
//  k_ac_slow<T>   per slow face: the same over every cell its grown box covers
//                 (a hit marks the slow-list entry);
//  k_ac_hits<T>   second pass over the hit list (and k_ac_slow over the marked
//                 slow faces): a pair whose distance equals its node's minimum
//                 bit for bit takes an atomic minimum of the face id;
//  k_ac_push<T>   per node: the move from its winning face, or a copy.
//
// The closest face is the one of least float64 distance, ties (faces sharing
// the closest edge or vertex) to the lower face id, so the choice is exact and
// deterministic: the second pass recomputes each marked pair's distance with
// the same code, without fused multiply-add, so it reproduces the first pass's
// bits.  Positions are float64 throughout.
#include "ifem_internal.hpp"

namespace ifem {

constexpr unsigned long long kNoFace = ~0ull;
constexpr int32_t kNoFaceId = 0x7fffffff;
constexpr unsigned kHitBit = 0x80000000u;  // marks a work item or slow face that found a pair below d_min
constexpr int kWorkSegs = 256;  // segments of the (face, cell) work list, one counter each

struct alignas(4) Row3c {  // three consecutive cells' owners
  int32_t v[3];
};

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

// The stored coordinates of node k, requested before its particle (and so its anchor) is known.
template <typename T>
__device__ __forceinline__ void load_coords(const ContactArgs& a, const T* __restrict__ x, int k, T out[3]) {
  const int64_t N = a.n_nodes;
#pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = x[i * N + k];
}

// Absolute float64 position from stored coordinates and the particle's anchor (float32 offsets).
template <typename T>
__device__ __forceinline__ void abs_from(const double* __restrict__ anchor, int p, const T xv[3], double out[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = (sizeof(T) == 4 ? anchor[3 * p + i] : 0.0) + (double)xv[i];
}

// Corners of a face relative to point xk, in the periodic image of the face
// nearest to xk: the image of the first corner, applied to all three (a face
// is one piece; wrapping each corner on its own could tear a face that sits
// half a box away).
__device__ __forceinline__ void face_image(const double pv[3][3], const double xk[3], const ContactBoxDev& C,
                                           double r[3][3]) {
#pragma clang fp contract(off)
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
    a.keys[k] = kNoFace;  // the node's least distance and face so far: none
    a.keyf[k] = kNoFaceId;
    T xv[3];
    load_coords(a, x, k, xv);
    const int p = a.node_particle[k];
    double pos[3];
    abs_from(anchor, p, xv, pos);
    key = cell_of(cbox_of(a, p), pos);
  }
  int leader, rank, size;
  wave_groups(key, leader, rank, size);
  if (size > 0) atomicAdd(a.count + key, size);
}

template <typename T>
__global__ void __launch_bounds__(256) k_ac_fill(const ContactArgs a, const T* __restrict__ x,
                                                 const double* __restrict__ anchor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1, p = 0;
  double pos[3] = {0.0, 0.0, 0.0};
  if (k < a.n_nodes) {
    T xv[3];
    load_coords(a, x, k, xv);
    p = a.node_particle[k];
    abs_from(anchor, p, xv, pos);
    key = cell_of(cbox_of(a, p), pos);
  }
  int leader, rank, size;
  wave_groups(key, leader, rank, size);
  const int base = size > 0 ? atomicAdd(a.cursor + key, size) : 0;
  // the cell's owner (cleared to -1 by the placement pass): the group leader claims the cell for its
  // particle; a cell claimed for another particle, or a member of another particle than its leader's,
  // marks the cell mixed (-2), whatever the order of the atomics
  const int pl = __shfl(p, leader, kWave);
  if (size > 0) {
    const int old = atomicCAS(a.owner + key, -1, pl);
    if (old != -1 && old != pl) atomicExch(a.owner + key, -2);
  }
  if (key >= 0 && p != pl) atomicExch(a.owner + key, -2);
  const int slot = __shfl(base, leader, kWave) + rank;
  if (key >= 0 && slot < a.n_nodes) {
    ContactNode r;
    r.x = pos[0];
    r.y = pos[1];
    r.z = pos[2];
    r.k = k;
    r.p = p;
    a.rec[slot] = r;
  }
}

// Neighbourhood test: every cell gets the least and the greatest owner over the
// (2 kNear + 1)^3 cells around it (periodic), empty cells neutral and mixed
// cells forcing lo < hi, so that lo < hi says that those cells hold nodes of
// more than one particle; a face whose grown box stays inside that
// neighbourhood of its first corner's cell, and finds lo == hi there, has no
// other particle's node to test and is skipped.
constexpr int kNear = 1;  // a face with d_min <= h reaches at most one contact cell past its first corner
constexpr int kOwnerEmptyLo = 0x7fffffff, kOwnerEmptyHi = -0x7fffffff;

// The whole neighbourhood at once: every cell reads the owners of the 3^3 cells around it (the
// window of kNear = 1, periodic; on an axis shorter than the window a cell may come twice:
// harmless) and keeps the least and the greatest.  One pass over the owners instead of an
// initialisation and one pass per axis.
static_assert(kNear == 1, "the neighbourhood pass reads a 3^3 window");
__device__ __forceinline__ int near_lo_of(int o) { return o == -1 ? kOwnerEmptyLo : (o == -2 ? -1 : o); }
__device__ __forceinline__ int near_hi_of(int o) { return o == -1 ? kOwnerEmptyHi : (o == -2 ? kOwnerEmptyLo : o); }

__global__ void __launch_bounds__(256) k_ac_near(const ContactArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_cells) return;
  // the box holding cell c: boxes are few and ordered by base
  int b = 0;
  while (b + 1 < a.n_boxes && a.boxes[b + 1].base <= c) ++b;
  const ContactBoxDev& C = a.boxes[b];
  const int r = c - C.base;
  const int n0 = C.nc[0], n1 = C.nc[1], n2 = C.nc[2];
  const int ix = r % n0, iy = (r / n0) % n1, iz = r / (n0 * n1);
  const int xs[3] = {ix == 0 ? n0 - 1 : ix - 1, ix, ix == n0 - 1 ? 0 : ix + 1};
  const int ys[3] = {(iy == 0 ? n1 - 1 : iy - 1) * n0, iy * n0, (iy == n1 - 1 ? 0 : iy + 1) * n0};
  const int zs[3] = {(iz == 0 ? n2 - 1 : iz - 1) * n0 * n1, iz * n0 * n1, (iz == n2 - 1 ? 0 : iz + 1) * n0 * n1};
  int o[27];  // all 27 owners requested before any is used
#pragma unroll
  for (int j = 0; j < 27; ++j) o[j] = a.owner[C.base + zs[j / 9] + ys[(j / 3) % 3] + xs[j % 3]];
  int l = kOwnerEmptyLo, h = kOwnerEmptyHi;
#pragma unroll
  for (int j = 0; j < 27; ++j) {
    l = min(l, near_lo_of(o[j]));
    h = max(h, near_hi_of(o[j]));
  }
  a.near_lo[c] = l;
  a.near_hi[c] = h;
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

// c wrapped into [0, n).
__device__ __forceinline__ int wrap_cell(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

// Cell index of the (periodically wrapped) cell coordinates (cx, cy, cz) of box C.
__device__ __forceinline__ int contact_cell(const ContactBoxDev& C, int cx, int cy, int cz) {
  int c[3] = {cx, cy, cz};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c[i] %= C.nc[i];
    c[i] = c[i] < 0 ? c[i] + C.nc[i] : c[i];
  }
  return C.base + (c[2] * C.nc[1] + c[1]) * C.nc[0] + c[0];
}

// Face f of particle q against the nodes of other particles among the n records
// of one cell starting at recs, loaded four at a time.  First pass (second == false): every pair below
// d_min lowers its node's least distance; returns whether there was one.
// Second pass: a pair at exactly its node's least distance lowers the node's
// face id.
__device__ __forceinline__ bool face_records(const ContactArgs& a, int f, int q, const ContactBoxDev& C,
                                             const double pv[3][3], const double blo[3], const double bhi[3],
                                             double d_min, bool second, const ContactNode* __restrict__ recs,
                                             int n) {
  bool hit = false;
  for (int i0 = 0; i0 < n; i0 += 4) {
    ContactNode r4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r4[u] = recs[min(i0 + u, n - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u >= n || r4[u].p == q || (unsigned)r4[u].k >= (unsigned)a.n_nodes) continue;
      const double xk[3] = {r4[u].x, r4[u].y, r4[u].z};
      // the node's image nearest to the face's first corner, tested against the grown box
      bool inside = true;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double d = xk[j] - pv[0][j];
        const double dn = d - C.len[j] * rint(d * C.inv_len[j]);
        inside = inside && dn >= blo[j] && dn <= bhi[j];
      }
      if (!inside) continue;
      double r[3][3];
      face_image(pv, xk, C, r);
      double cp[3];
      closest_on_triangle0(r[0], r[1], r[2], cp);
      const double dist = norm_nc(cp);
      if (!(dist < d_min)) continue;
      // non-negative doubles order like their bit patterns
      const unsigned long long bits = (unsigned long long)__double_as_longlong(dist);
      if (!second) {
        atomicMin(a.keys + r4[u].k, bits);
        hit = true;
      } else if (bits == a.keys[r4[u].k]) {
        atomicMin(a.keyf + r4[u].k, f);
      }
    }
  }
  return hit;
}

// The same against all records of one cell.
__device__ __forceinline__ bool face_cell_nodes(const ContactArgs& a, int f, int q, const ContactBoxDev& C,
                                                const double pv[3][3], const double blo[3], const double bhi[3],
                                                double d_min, bool second, int cell) {
  return face_records(a, f, q, C, pv, blo, bhi, d_min, second, a.rec + a.off[cell], a.count[cell]);
}

// Face f: its particle q, box C, corners pv, the cell range its box grown by d_min
// covers (lo, cnt per axis) and that box relative to the first corner (blo, bhi,
// grown a hair more, so that no pair whose rounded distance could still fall
// below d_min is dropped).  False for a face that is not finite or spans half a
// box: it belongs to a broken mesh and is skipped.
template <typename T>
__device__ __forceinline__ bool face_setup(const ContactArgs& a, const T* __restrict__ x,
                                           const double* __restrict__ anchor, int f, double d_min, int& q,
                                           ContactBoxDev& C, double pv[3][3], int lo[3], int cnt[3], double blo[3],
                                           double bhi[3]) {
  int v[3];
  face_nodes(a, f, v);
  T xv[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) load_coords(a, x, v[m], xv[m]);
  q = a.node_particle[v[0]];
  C = cbox_of(a, q);
#pragma unroll
  for (int m = 0; m < 3; ++m) abs_from(anchor, q, xv[m], pv[m]);
  bool ok = true;
  const double g = d_min * (1.0 + 1e-6);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double mn = fmin(pv[0][i], fmin(pv[1][i], pv[2][i]));
    const double mx = fmax(pv[0][i], fmax(pv[1][i], pv[2][i]));
    ok = ok && (mx - mn <= 0.5 * C.len[i]);
    lo[i] = ok ? (int)floor((mn - d_min - C.origin[i]) * C.inv_cs[i]) : 0;
    const int hi = ok ? (int)floor((mx + d_min - C.origin[i]) * C.inv_cs[i]) : -1;
    cnt[i] = min(hi - lo[i] + 1, C.nc[i]);  // a range wider than the box visits each cell once
    blo[i] = fmin(0.0, fmin(pv[1][i] - pv[0][i], pv[2][i] - pv[0][i])) - g;
    bhi[i] = fmax(0.0, fmax(pv[1][i] - pv[0][i], pv[2][i] - pv[0][i])) + g;
  }
  return ok;
}

// Phase 1, one thread per face: the cells of its grown box that hold nodes of
// other particles (at most 3 x 3 x 3 for a face no wider than a cell less
// 2 d_min, their owners requested together) become (face, cell) work items,
// appended with one atomic per wavefront.  A face whose box covers more cells,
// or whose items do not all fit the list, goes to the list of faces searched
// whole (which holds every face at most once, so it cannot overflow).
template <typename T>
__global__ void __launch_bounds__(256) k_ac_faces(const ContactArgs a, const T* __restrict__ x,
                                                  const double* __restrict__ anchor, double d_min,
                                                  unsigned long long* __restrict__ keys) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int q = -1, lo[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
  ContactBoxDev C;
  double pv[3][3], blo[3], bhi[3];
  bool ok = f < a.n_tris + a.n_bfaces;
  if (ok) ok = face_setup(a, x, anchor, f, d_min, q, C, pv, lo, cnt, blo, bhi);
  int ncell = ok ? cnt[0] * cnt[1] * cnt[2] : 0;
  unsigned visit = 0;
  int cx[3], cy[3], cz[3];  // wrapped cell coordinates of the first three cells per axis
  if (ok) {  // one particle alone around the first corner, and the grown box inside that neighbourhood: nothing to test
    const int c0[3] = {(int)floor((pv[0][0] - C.origin[0]) * C.inv_cs[0]),
                       (int)floor((pv[0][1] - C.origin[1]) * C.inv_cs[1]),
                       (int)floor((pv[0][2] - C.origin[2]) * C.inv_cs[2])};
    bool inside = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) inside = inside && lo[i] >= c0[i] - kNear && lo[i] + cnt[i] - 1 <= c0[i] + kNear;
    if (inside) {
      const int cell0 = contact_cell(C, c0[0], c0[1], c0[2]);
      if (a.near_lo[cell0] >= a.near_hi[cell0]) ok = false;
    }
  }
  if (!ok) ncell = 0;
  if (ok && ncell <= 27) {
    const int w0 = wrap_cell(lo[0], C.nc[0]), w1 = wrap_cell(lo[1], C.nc[1]), w2 = wrap_cell(lo[2], C.nc[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {  // one step past the end wraps to the start: cnt <= nc per axis
      cx[i] = w0 + i >= C.nc[0] ? w0 + i - C.nc[0] : w0 + i;
      cy[i] = (w1 + i >= C.nc[1] ? w1 + i - C.nc[1] : w1 + i) * C.nc[0];
      cz[i] = (w2 + i >= C.nc[2] ? w2 + i - C.nc[2] : w2 + i) * C.nc[0] * C.nc[1];
    }
    // owners by rows of three cells along x: one 12-byte load per row unless the row wraps
    int own[27];
    const bool row = w0 + 2 < C.nc[0];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int iy = r % 3, iz = r / 3;
      const bool use = iy < cnt[1] && iz < cnt[2];
      const int rb = C.base + cz[iz] + cy[iy];
      if (use && row) {
        const Row3c i3 = *reinterpret_cast<const Row3c*>(a.owner + rb + w0);
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) own[3 * r + ix] = ix < cnt[0] ? i3.v[ix] : -1;
      } else {
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) own[3 * r + ix] = use && ix < cnt[0] ? a.owner[rb + cx[ix]] : -1;
      }
    }
#pragma unroll
    for (int j = 0; j < 27; ++j) visit |= (own[j] != -1 && own[j] != q ? 1u : 0u) << j;
  }
  // wavefront prefix of the items, one atomic for the wavefront's run
  const int mine = __popc(visit);
  int incl = mine;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += u;
  }
  const int total = __shfl(incl, kWave - 1, kWave);
  // the list is cut into kWorkSegs segments with a counter each, so that the wavefronts' atomics
  // spread over many addresses instead of queueing on one
  const int seg = (int)((blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) % kWorkSegs);
  int base = 0;
  if (lane == 0 && total > 0) base = atomicAdd(a.work_count + seg, total);
  base = __shfl(base, 0, kWave) + incl - mine;
  const int seg_cap = a.work_cap / kWorkSegs;
  if ((ok && ncell > 27) || (mine > 0 && base + mine > seg_cap)) {
    for (int i = base; i < min(base + mine, seg_cap); ++i) a.work[seg * seg_cap + i] = make_uint2(~0u, 0u);  // reserved, unused
    a.slow[atomicAdd(a.slow_count, 1)] = f;
    return;
  }
  uint2* w = a.work + (size_t)seg * seg_cap;
  while (visit) {
    const int j = __builtin_ctz(visit);
    visit &= visit - 1;
    w[base++] = make_uint2((unsigned)f, (unsigned)(C.base + cz[j / 9] + cy[(j / 3) % 3] + cx[j % 3]));
  }
}

// Faces searched whole: every cell of the grown box, one by one.
template <typename T>
__global__ void __launch_bounds__(256) k_ac_slow(const ContactArgs a, const T* __restrict__ x,
                                                 const double* __restrict__ anchor, double d_min, int second) {
  const int n = min(*a.slow_count, a.n_tris + a.n_bfaces);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const unsigned s = (unsigned)a.slow[i];
    if (second && !(s & kHitBit)) continue;
    const int f = (int)(s & ~kHitBit);
    if (f >= a.n_tris + a.n_bfaces) continue;
    int q, lo[3], cnt[3];
    ContactBoxDev C;
    double pv[3][3], blo[3], bhi[3];
    if (!face_setup(a, x, anchor, f, d_min, q, C, pv, lo, cnt, blo, bhi)) continue;
    bool hit = false;
    for (int iz = 0; iz < cnt[2]; ++iz)
      for (int iy = 0; iy < cnt[1]; ++iy)
        for (int ix = 0; ix < cnt[0]; ++ix) {
          const int cell = contact_cell(C, lo[0] + ix, lo[1] + iy, lo[2] + iz);
          const int owner = a.owner[cell];
          if (owner != -1 && owner != q) hit |= face_cell_nodes(a, f, q, C, pv, blo, bhi, d_min, second != 0, cell);
        }
    if (!second && hit) a.slow[i] = (int32_t)(s | kHitBit);
  }
}

// Phase 2, one thread per (face, cell) work item (grid-stride over the items
// phase 1 listed): the face against the cell's nodes of other particles.
// First pass: every work item; an item that found a pair below d_min is appended to the hit list
// (one atomic per wavefront), which the second pass walks.
template <typename T>
__global__ void __launch_bounds__(256) k_ac_pairs(const ContactArgs a, const T* __restrict__ x,
                                                  const double* __restrict__ anchor, double d_min) {
  // blocks are dealt to the segments round robin (the grid is a multiple of kWorkSegs)
  const int seg_cap = a.work_cap / kWorkSegs;
  const int seg = (int)(blockIdx.x % kWorkSegs), per_seg = (int)(gridDim.x / kWorkSegs);
  const int n = min(a.work_count[seg], seg_cap);
  const int lane = threadIdx.x & (kWave - 1);
  const uint2* __restrict__ list = a.work + (size_t)seg * seg_cap;
  const int stride = per_seg * (int)blockDim.x;
  int i = (int)(blockIdx.x / kWorkSegs) * blockDim.x + threadIdx.x;
  // each thread's next work item is requested one item ahead, and an item's record range before its
  // face set-up, so that these loads overlap the work of the chain in front of them
  uint2 w_next = i < n ? list[i] : make_uint2(~0u, 0u);
  for (; i < n; i += stride) {
    const uint2 w = w_next;
    if (i + stride < n) w_next = list[i + stride];
    bool hit = false;
    if (w.x < (unsigned)(a.n_tris + a.n_bfaces)) {  // not a reserved slot
      const int o = a.off[w.y], nrec = a.count[w.y];
      int q, lo[3], cnt[3];
      ContactBoxDev C;
      double pv[3][3], blo[3], bhi[3];
      face_setup(a, x, anchor, (int)w.x, d_min, q, C, pv, lo, cnt, blo, bhi);
      hit = face_records(a, (int)w.x, q, C, pv, blo, bhi, d_min, false, a.rec + o, nrec);
    }
    // the lanes still in the loop append their hits together
    const unsigned long long m = __ballot(hit);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(a.hit_count, (int)__popcll(m));
      base = __shfl(base, leader, kWave);
      if (hit) a.hits[base + (int)__popcll(m & ((1ull << lane) - 1ull))] = seg * seg_cap + i;
    }
  }
}

// Second pass: the listed items again, each pair at exactly its node's least distance lowering the
// node's face id.
template <typename T>
__global__ void __launch_bounds__(256) k_ac_hits(const ContactArgs a, const T* __restrict__ x,
                                                 const double* __restrict__ anchor, double d_min) {
  const int n = min(*a.hit_count, a.work_cap);
  const int stride = gridDim.x * blockDim.x;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int slot_next = i < n ? a.hits[i] : -1;  // the next listed item, requested one item ahead
  for (; i < n; i += stride) {
    const uint2 w = a.work[slot_next];
    slot_next = i + stride < n ? a.hits[i + stride] : -1;
    if (w.x >= (unsigned)(a.n_tris + a.n_bfaces)) continue;
    const int o = a.off[w.y], nrec = a.count[w.y];
    int q, lo[3], cnt[3];
    ContactBoxDev C;
    double pv[3][3], blo[3], bhi[3];
    face_setup(a, x, anchor, (int)w.x, d_min, q, C, pv, lo, cnt, blo, bhi);
    face_records(a, (int)w.x, q, C, pv, blo, bhi, d_min, true, a.rec + o, nrec);
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
  const int f = a.keyf[k];
  if (key == kNoFace || (unsigned)f >= (unsigned)(a.n_tris + a.n_bfaces)) {
    // a distance without a face id: the second pass did not reproduce it (positions written during the call)
    if (key != kNoFace) atomicAdd(a.status + 3, 1ull);
#pragma unroll
    for (int i = 0; i < 3; ++i) x_out[i * N + k] = x[i * N + k];
    if (face_out) face_out[k] = -1;
    return;
  }
  const int p = a.node_particle[k];
  double xk[3];
  abs_position(a, x, anchor, k, p, xk);
  int v[3];
  face_nodes(a, f, v);
  const int q = a.node_particle[v[0]];
  const ContactBoxDev C = cbox_of(a, q);
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

// ------------------------------------------------------------------ cell offsets
// Any disjoint placement of the cells' record ranges works, so the cells are cut
// into chunks of kScanItems, one per workgroup: a workgroup sums its counts
// (thread t takes the counts t, t + kScanBlock, ... of the chunk: coalesced
// loads; kScanPer consecutive cells per thread made the loads strided and the
// pass twice as slow), scans the thread totals, reserves its chunk's total with
// one atomic on a running total, and each thread lays its cells out one after
// another from there.  No workgroup waits for another.
constexpr int kScanBlock = 256, kScanPer = 16, kScanItems = kScanBlock * kScanPer;

__global__ void __launch_bounds__(kScanBlock) k_cscan(int32_t n, const int32_t* __restrict__ cnt,
                                                      int32_t* __restrict__ running, int32_t* __restrict__ off,
                                                      int32_t* __restrict__ cursor, int32_t* __restrict__ owner) {
  __shared__ int32_t wsum[kScanBlock / kWave];
  __shared__ int32_t chunk_base;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int64_t i0 = (int64_t)blockIdx.x * kScanItems + tid;
  int32_t c[kScanPer], s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = i0 + (int64_t)j * kScanBlock;
    c[j] = i < n ? cnt[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) s += c[j];
  int32_t incl = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t u = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += u;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  int32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / kWave; ++w) {
    if (w < wave) before += wsum[w];
    total += wsum[w];
  }
  if (tid == 0) chunk_base = atomicAdd(running, total);
  __syncthreads();
  int32_t run = chunk_base + before + incl - s;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = i0 + (int64_t)j * kScanBlock;
    if (i < n) {
      off[i] = run;
      cursor[i] = run;
      owner[i] = -1;  // no node yet (the fill pass claims the cell)
      run += c[j];
    }
  }
}

int32_t contact_scan_blocks(int32_t n_cells) { return (n_cells + kScanItems - 1) / kScanItems; }

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
  // segment, slow-face and hit counters, and the running total of the cell placement
  if (e == hipSuccess) e = launch_fill_i32(a.work_count, kWorkSegs + 3, 0, st);
  P.timer->end(st);
  if (e != hipSuccess) return e;
  P.timer->begin(K_CONTACT, st);
  if (dtype == 0)
    hipLaunchKernelGGL(k_ac_count<float>, gn, dim3(B), 0, st, a, (const float*)x, anchor);
  else
    hipLaunchKernelGGL(k_ac_count<double>, gn, dim3(B), 0, st, a, (const double*)x, anchor);
  hipLaunchKernelGGL(k_cscan, dim3((unsigned)contact_scan_blocks(a.n_cells)), dim3(kScanBlock), 0, st, a.n_cells,
                     a.count, a.place, a.off, a.cursor, a.owner);
  if (dtype == 0)
    hipLaunchKernelGGL(k_ac_fill<float>, gn, dim3(B), 0, st, a, (const float*)x, anchor);
  else
    hipLaunchKernelGGL(k_ac_fill<double>, gn, dim3(B), 0, st, a, (const double*)x, anchor);
  hipLaunchKernelGGL(k_ac_near, gc, dim3(B), 0, st, a);
  if (nf > 0) {
    const dim3 gf((unsigned)((nf + B - 1) / B));
    if (dtype == 0)
      hipLaunchKernelGGL(k_ac_faces<float>, gf, dim3(B), 0, st, a, (const float*)x, anchor, d_min, a.keys);
    else
      hipLaunchKernelGGL(k_ac_faces<double>, gf, dim3(B), 0, st, a, (const double*)x, anchor, d_min, a.keys);
    const dim3 gp(16 * kWorkSegs);
    // least distance, then least face id at that distance
    if (dtype == 0) {
      hipLaunchKernelGGL(k_ac_pairs<float>, gp, dim3(B), 0, st, a, (const float*)x, anchor, d_min);
      hipLaunchKernelGGL(k_ac_slow<float>, gp, dim3(B), 0, st, a, (const float*)x, anchor, d_min, 0);
      hipLaunchKernelGGL(k_ac_hits<float>, dim3(1024), dim3(B), 0, st, a, (const float*)x, anchor, d_min);
      hipLaunchKernelGGL(k_ac_slow<float>, gp, dim3(B), 0, st, a, (const float*)x, anchor, d_min, 1);
    } else {
      hipLaunchKernelGGL(k_ac_pairs<double>, gp, dim3(B), 0, st, a, (const double*)x, anchor, d_min);
      hipLaunchKernelGGL(k_ac_slow<double>, gp, dim3(B), 0, st, a, (const double*)x, anchor, d_min, 0);
      hipLaunchKernelGGL(k_ac_hits<double>, dim3(1024), dim3(B), 0, st, a, (const double*)x, anchor, d_min);
      hipLaunchKernelGGL(k_ac_slow<double>, gp, dim3(B), 0, st, a, (const double*)x, anchor, d_min, 1);
    }
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
