// Host side of the C ABI declared in include/ifem.h: plan construction,
// argument validation and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ifem.h"
#include "ifem_internal.hpp"

using namespace ifem;

namespace {

thread_local std::string g_last_error;

ifem_status fail(ifem_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

ifem_status ok() {
  g_last_error.clear();
  return IFEM_OK;
}

constexpr int kMaxColours = 128;
constexpr size_t kLdsLimit = 160 * 1024;

struct DeviceBuffers {
  std::vector<void*> ptrs;
  template <typename T>
  hipError_t alloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct ifem_plan_s {
  PlanDev P{};
  KernelTimer timer;
  DeviceBuffers mem;
  DeviceBuffers spread_mem;          // the tile-dependent spread workspace (rebuilt by ifem_plan_autotune)
  std::vector<ifem::BoxDev> boxes;   // box geometry on the host (tile fields set by build_spread)
  uint64_t shape_hash = 0;           // hash of the plan's sizes: the key of the tuning cache
  ifem_tuning tune{};
  int spread_mode = IFEM_SPREAD_TILED;
  int64_t workspace_bytes = 0;
  int32_t open_surface = -1;  // first membrane whose faces do not close, or -1
  double contact_cell = 0.0;  // smallest contact-cell width over the boxes
  double min_box_len = 0.0;   // smallest box length over the axes and boxes
};

// ------------------------------------------------------------------ host-side mesh preprocessing
namespace {

// Greedy colouring of the elements of one particle so that no two elements of
// a colour share a node; returns the colour of each element (or -1 on overflow).
template <int NV>
int colour_elements(const int32_t* conn, int n_all, int e0, int e1, int node0, int nn, std::vector<int>& colour) {
  std::vector<uint64_t> used((size_t)nn * 2, 0ull);
  int ncol = 0;
  for (int e = e0; e < e1; ++e) {
    uint64_t m0 = 0, m1 = 0;
    for (int v = 0; v < NV; ++v) {
      const int l = conn[v * n_all + e] - node0;
      m0 |= used[2 * l];
      m1 |= used[2 * l + 1];
    }
    int c;
    if (~m0)
      c = __builtin_ctzll(~m0);
    else if (~m1)
      c = 64 + __builtin_ctzll(~m1);
    else
      return -1;
    colour[e - e0] = c;
    ncol = std::max(ncol, c + 1);
    for (int v = 0; v < NV; ++v) {
      const int l = conn[v * n_all + e] - node0;
      if (c < 64)
        used[2 * l] |= 1ull << c;
      else
        used[2 * l + 1] |= 1ull << (c - 64);
    }
  }
  return ncol;
}

// Colouring for workgroup rounds: every colour holds at most B elements, no
// two of which share a node, so the force kernel runs one colour per round of
// B threads.  Each colour is filled greedily from the uncoloured elements taken
// by decreasing number of uncoloured elements they conflict with (ties by
// element order): the hard-to-place elements go first and the last colours
// still fill up (a 5120-triangle red cell takes 10 colours of 512, where the
// plain greedy colouring needs 16 rounds).  Returns the colour count, or -1
// beyond kMaxColours.
template <int NV>
int colour_rounds(const int32_t* conn, int n_all, int e0, int e1, int node0, int nn, int B, std::vector<int>& colour) {
  const int n = e1 - e0;
  std::vector<int> ioff(nn + 1, 0), inc((size_t)n * NV);
  for (int e = 0; e < n; ++e)
    for (int v = 0; v < NV; ++v) ioff[conn[v * n_all + e0 + e] - node0 + 1]++;
  for (int i = 0; i < nn; ++i) ioff[i + 1] += ioff[i];
  std::vector<int> cur(ioff.begin(), ioff.end() - 1);
  for (int e = 0; e < n; ++e)
    for (int v = 0; v < NV; ++v) inc[cur[conn[v * n_all + e0 + e] - node0]++] = e;
  std::vector<int> noff(n + 1, 0), nbr, mark(n, -1);
  nbr.reserve((size_t)n * 4 * NV);
  for (int e = 0; e < n; ++e) {
    for (int v = 0; v < NV; ++v) {
      const int l = conn[v * n_all + e0 + e] - node0;
      for (int i = ioff[l]; i < ioff[l + 1]; ++i) {
        const int f = inc[i];
        if (f != e && mark[f] != e) {
          mark[f] = e;
          nbr.push_back(f);
        }
      }
    }
    noff[e + 1] = (int)nbr.size();
  }
  std::vector<int> deg(n), order, stamp(nn, -1);
  for (int e = 0; e < n; ++e) deg[e] = noff[e + 1] - noff[e];
  std::vector<char> done(n, 0);
  int ncol = 0, left = n;
  while (left > 0) {
    if (ncol >= kMaxColours) return -1;
    order.clear();
    for (int e = 0; e < n; ++e)
      if (!done[e]) order.push_back(e);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return deg[a] != deg[b] ? deg[a] > deg[b] : a < b; });
    int taken = 0;
    for (int e : order) {
      if (taken >= B) break;
      bool free = true;
      for (int v = 0; v < NV && free; ++v) free = stamp[conn[v * n_all + e0 + e] - node0] != ncol;
      if (!free) continue;
      for (int v = 0; v < NV; ++v) stamp[conn[v * n_all + e0 + e] - node0] = ncol;
      colour[e] = ncol;
      done[e] = 1;
      ++taken;
    }
    for (int e : order)
      if (done[e] && colour[e] == ncol)
        for (int i = noff[e]; i < noff[e + 1]; ++i) --deg[nbr[i]];
    left -= taken;
    ++ncol;
  }
  return ncol;
}

// Rounds of B threads a colouring takes: sum over colours of ceil(size / B).
int colouring_rounds(const std::vector<int>& colour, int nc, int B) {
  std::vector<int> size(nc, 0);
  for (int c : colour) size[c]++;
  int r = 0;
  for (int c = 0; c < nc; ++c) r += (size[c] + B - 1) / B;
  return r;
}

// Sort the elements of every particle by colour.  Outputs the slot -> element
// map, the particle-local connectivity in slot order, per-particle colour
// offsets and per-colour slot offsets.  Of the plain greedy colouring and the
// round colouring for workgroups of B threads, the one with fewer rounds is
// kept; particles with the same local connectivity (all red cells of a
// suspension) share one computation.
template <int NV>
ifem_status build_coloured(const int32_t* conn, int n_all, int n_p, const int32_t* estart, const int32_t* nstart,
                           int B, std::vector<int32_t>& src, std::vector<int32_t>& local, std::vector<int32_t>& pcol,
                           std::vector<int32_t>& colb) {
  src.resize(n_all);
  local.resize((size_t)NV * n_all);
  pcol.assign(n_p + 1, 0);
  colb.clear();
  std::vector<int> colour, greedy;
  // topology hash -> particles already coloured with it (their colourings kept below)
  std::unordered_multimap<uint64_t, int> seen;
  std::vector<std::vector<int>> kept(n_p);
  std::vector<int> kept_nc(n_p, 0);
  for (int p = 0; p < n_p; ++p) {
    const int e0 = estart[p], e1 = estart[p + 1], node0 = nstart[p], nn = nstart[p + 1] - nstart[p];
    pcol[p] = (int32_t)colb.size();
    if (e1 == e0) continue;
    uint64_t hsh = 1469598103934665603ull ^ (uint64_t)nn;
    for (int e = e0; e < e1; ++e)
      for (int v = 0; v < NV; ++v) hsh = (hsh ^ (uint64_t)(conn[v * n_all + e] - node0 + 1)) * 1099511628211ull;
    int nc = -1;
    const auto range = seen.equal_range(hsh);
    for (auto it = range.first; it != range.second && nc < 0; ++it) {
      const int q = it->second, f0 = estart[q], m0 = nstart[q];
      if (estart[q + 1] - f0 != e1 - e0 || nstart[q + 1] - m0 != nn) continue;
      bool same = true;
      for (int e = 0; e < e1 - e0 && same; ++e)
        for (int v = 0; v < NV && same; ++v) same = conn[v * n_all + f0 + e] - m0 == conn[v * n_all + e0 + e] - node0;
      if (same) {
        colour = kept[q];
        nc = kept_nc[q];
      }
    }
    if (nc < 0) {
      greedy.assign(e1 - e0, 0);
      const int ng = colour_elements<NV>(conn, n_all, e0, e1, node0, nn, greedy);
      colour.assign(e1 - e0, 0);
      const int nr = colour_rounds<NV>(conn, n_all, e0, e1, node0, nn, B, colour);
      if (ng < 0 && nr < 0)
        return fail(IFEM_ERR_UNSUPPORTED, "particle %d needs more than %d element colours", p, kMaxColours);
      if (nr < 0 || (ng >= 0 && colouring_rounds(greedy, ng, B) < colouring_rounds(colour, nr, B))) {
        colour.swap(greedy);
        nc = ng;
      } else {
        nc = nr;
      }
      seen.emplace(hsh, p);
      kept[p] = colour;
      kept_nc[p] = nc;
    }
    std::vector<int> count(nc + 1, 0);
    for (int c : colour) count[c + 1]++;
    for (int c = 0; c < nc; ++c) count[c + 1] += count[c];
    for (int c = 0; c < nc; ++c) colb.push_back(e0 + count[c]);
    std::vector<int> cur(count.begin(), count.end() - 1);
    for (int e = e0; e < e1; ++e) {
      const int s = e0 + cur[colour[e - e0]]++;
      src[s] = e;
      for (int v = 0; v < NV; ++v) local[(size_t)v * n_all + s] = conn[v * n_all + e] - node0;
    }
  }
  pcol[n_p] = (int32_t)colb.size();
  colb.push_back(n_all);
  return IFEM_OK;
}

// Ordered one-ring of every node of the selected particles (bending, and the
// volume correction): neighbours j_1..j_v with (k, j_i, j_{i+1})
// counter-clockwise triangles of the mesh.  On failure *bad_node is the node
// whose fan is open, non-manifold or pinched.
ifem_status build_rings(const ifem_mesh_desc& m, const std::vector<char>& bend, std::vector<int32_t>& rstart,
                        std::vector<int32_t>& ring, int* bad_node) {
  const int nN = m.n_nodes, nT = m.n_tris;
  std::vector<int32_t> wcount(nN + 1, 0);
  for (int p = 0; p < m.n_particles; ++p) {
    if (!bend[p]) continue;
    for (int t = m.tri_start[p]; t < m.tri_start[p + 1]; ++t)
      for (int v = 0; v < 3; ++v) wcount[m.tri[v * nT + t] + 1]++;
  }
  for (int i = 0; i < nN; ++i) wcount[i + 1] += wcount[i];
  std::vector<int32_t> wa(wcount[nN]), wb(wcount[nN]);
  std::vector<int32_t> cur(wcount.begin(), wcount.end() - 1);
  for (int p = 0; p < m.n_particles; ++p) {
    if (!bend[p]) continue;
    for (int t = m.tri_start[p]; t < m.tri_start[p + 1]; ++t) {
      const int id[3] = {m.tri[t], m.tri[nT + t], m.tri[2 * nT + t]};
      for (int v = 0; v < 3; ++v) {
        const int k = id[v], s = cur[k]++;
        wa[s] = id[(v + 1) % 3];
        wb[s] = id[(v + 2) % 3];
      }
    }
  }
  rstart.assign(nN + 1, 0);
  ring.clear();
  ring.reserve(wcount[nN]);
  std::vector<int> node_p(nN, -1);
  for (int p = 0; p < m.n_particles; ++p)
    for (int k = m.node_start[p]; k < m.node_start[p + 1]; ++k) node_p[k] = p;
  for (int k = 0; k < nN; ++k) {
    rstart[k] = (int32_t)ring.size();
    const int b = wcount[k], e = wcount[k + 1], v = e - b;
    if (v == 0) continue;
    const int node0 = m.node_start[node_p[k]];
    *bad_node = k;
    if (v < 3) return fail(IFEM_ERR_UNSUPPORTED, "node %d has %d incident triangles; bending needs a closed surface", k, v);
    int j = wa[b];
    for (int step = 0; step < v; ++step) {
      ring.push_back(j - node0);
      int nxt = -1, hits = 0;
      for (int s = b; s < e; ++s)
        if (wa[s] == j) {
          nxt = wb[s];
          ++hits;
        }
      if (hits != 1) return fail(IFEM_ERR_UNSUPPORTED, "non-manifold or open one-ring at node %d", k);
      j = nxt;
      if (j == wa[b] && step + 1 < v)
        return fail(IFEM_ERR_UNSUPPORTED, "node %d joins two fans of triangles (pinched surface)", k);
    }
    if (j != wa[b]) return fail(IFEM_ERR_UNSUPPORTED, "one-ring of node %d does not close", k);
  }
  rstart[nN] = (int32_t)ring.size();
  return IFEM_OK;
}

ifem_status validate_mesh(const ifem_mesh_desc* m, const ifem_box* boxes, int n_boxes) {
  if (!m) return fail(IFEM_ERR_INVALID_ARG, "mesh is NULL");
  if (m->n_particles < 0 || m->n_nodes < 0 || m->n_tris < 0 || m->n_tets < 0)
    return fail(IFEM_ERR_INVALID_ARG, "negative count");
  if (n_boxes <= 0 || !boxes) return fail(IFEM_ERR_INVALID_ARG, "at least one box is required");
  if (m->n_particles > 0 &&
      (!m->node_start || !m->tri_start || !m->tet_start || !m->law || !m->mu || !m->mu2 || !m->kb || !m->c0 ||
       !m->box))
    return fail(IFEM_ERR_INVALID_ARG, "NULL per-particle array");
  if ((m->n_tris > 0 && !m->tri) || (m->n_tets > 0 && !m->tet) || (m->n_nodes > 0 && !m->X_ref))
    return fail(IFEM_ERR_INVALID_ARG, "NULL connectivity or reference positions");
  for (int b = 0; b < n_boxes; ++b) {
    const ifem_box& B = boxes[b];
    if (B.n[0] < 3 || B.n[1] < 3 || B.n[2] < 3) return fail(IFEM_ERR_INVALID_ARG, "box %d: n < 3 on some axis", b);
    if (!(B.h > 0.0) || !std::isfinite(B.h)) return fail(IFEM_ERR_INVALID_ARG, "box %d: bad spacing", b);
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(B.origin[a])) return fail(IFEM_ERR_INVALID_ARG, "box %d: bad origin", b);
    if ((int64_t)B.n[0] * B.n[1] * B.n[2] > (int64_t)1 << 31)
      return fail(IFEM_ERR_UNSUPPORTED, "box %d: more than 2^31 cells", b);
  }
  if (m->n_particles == 0) return IFEM_OK;
  if (m->node_start[0] != 0 || m->tri_start[0] != 0 || m->tet_start[0] != 0)
    return fail(IFEM_ERR_INVALID_ARG, "start arrays must begin at 0");
  const int P = m->n_particles;
  if (m->node_start[P] != m->n_nodes || m->tri_start[P] != m->n_tris || m->tet_start[P] != m->n_tets)
    return fail(IFEM_ERR_INVALID_ARG, "start arrays must end at the totals");
  for (int p = 0; p < P; ++p) {
    if (m->node_start[p + 1] <= m->node_start[p] || m->tri_start[p + 1] < m->tri_start[p] ||
        m->tet_start[p + 1] < m->tet_start[p])
      return fail(IFEM_ERR_INVALID_ARG, "particle %d: non-increasing start arrays or no nodes", p);
    const int law = m->law[p];
    const bool tri = m->tri_start[p + 1] > m->tri_start[p], tet = m->tet_start[p + 1] > m->tet_start[p];
    if (law == IFEM_LAW_TET_NEOHOOKE) {
      if (tri) return fail(IFEM_ERR_INVALID_ARG, "particle %d: solid law with triangles", p);
    } else if (law == IFEM_LAW_TRI_NEOHOOKE || law == IFEM_LAW_TRI_SKALAK) {
      if (tet) return fail(IFEM_ERR_INVALID_ARG, "particle %d: membrane law with tetrahedra", p);
    } else {
      return fail(IFEM_ERR_INVALID_ARG, "particle %d: unknown law %d", p, law);
    }
    if (m->box[p] < 0 || m->box[p] >= n_boxes) return fail(IFEM_ERR_INVALID_ARG, "particle %d: bad box index", p);
    if (!std::isfinite(m->mu[p]) || !std::isfinite(m->mu2[p]) || !std::isfinite(m->kb[p]) || !std::isfinite(m->c0[p]))
      return fail(IFEM_ERR_INVALID_ARG, "particle %d: non-finite material parameter", p);
    const int n0 = m->node_start[p], n1 = m->node_start[p + 1];
    for (int t = m->tri_start[p]; t < m->tri_start[p + 1]; ++t)
      for (int v = 0; v < 3; ++v) {
        const int i = m->tri[v * m->n_tris + t];
        if (i < n0 || i >= n1) return fail(IFEM_ERR_INVALID_ARG, "triangle %d refers to a node of another particle", t);
      }
    for (int t = m->tet_start[p]; t < m->tet_start[p + 1]; ++t)
      for (int v = 0; v < 4; ++v) {
        const int i = m->tet[v * m->n_tets + t];
        if (i < n0 || i >= n1) return fail(IFEM_ERR_INVALID_ARG, "tetrahedron %d refers to a node of another particle", t);
      }
  }
  for (int64_t i = 0; i < 3 * (int64_t)m->n_nodes; ++i)
    if (!std::isfinite(m->X_ref[i])) return fail(IFEM_ERR_INVALID_ARG, "non-finite reference position");
  return IFEM_OK;
}

template <typename T>
hipError_t upload(DeviceBuffers& mem, T** dst, const T* src, size_t n, hipStream_t st) {
  hipError_t e = mem.alloc(dst, n);
  if (e != hipSuccess || n == 0) return e;
  return hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, st);
}

#define HIP_TRY(call)                                                                               \
  do {                                                                                              \
    hipError_t _e = (call);                                                                         \
    if (_e != hipSuccess) {                                                                         \
      plan->mem.release();                                                                          \
      plan->spread_mem.release();                                                                   \
      delete plan;                                                                                  \
      return fail(_e == hipErrorOutOfMemory ? IFEM_ERR_NOMEM : IFEM_ERR_DEVICE, "%s: %s", #call,    \
                  hipGetErrorString(_e));                                                           \
    }                                                                                               \
  } while (0)

}  // namespace

namespace {

// Boundary faces of the solids' tetrahedral meshes: the faces of one
// tetrahedron only, listed by (tetrahedron, face opposite local node j =
// 0..3), corners in the tetrahedron's order without node j, turned (second and
// third corner swapped) so that the normal points away from node j in the
// reference configuration.  out [3][n] global node ids.
void boundary_faces(const ifem_mesh_desc& m, std::vector<int32_t>& out) {
  out.clear();
  struct Key {
    int32_t v[3];
    int32_t slot;
  };
  std::vector<Key> keys;
  std::vector<char> single;
  std::vector<int32_t> f0, f1, f2;
  for (int p = 0; p < m.n_particles; ++p) {
    const int t0 = m.tet_start[p], nt = m.tet_start[p + 1] - t0;
    if (nt == 0) continue;
    keys.resize((size_t)4 * nt);
    for (int t = 0; t < nt; ++t)
      for (int j = 0; j < 4; ++j) {
        Key& k = keys[(size_t)4 * t + j];
        int c = 0;
        for (int q = 0; q < 4; ++q)
          if (q != j) k.v[c++] = m.tet[q * m.n_tets + t0 + t];
        std::sort(k.v, k.v + 3);
        k.slot = 4 * t + j;
      }
    std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
      return std::lexicographical_compare(a.v, a.v + 3, b.v, b.v + 3);
    });
    single.assign((size_t)4 * nt, 0);
    for (size_t i = 0; i < keys.size();) {
      size_t e = i + 1;
      while (e < keys.size() && std::equal(keys[e].v, keys[e].v + 3, keys[i].v)) ++e;
      if (e - i == 1) single[keys[i].slot] = 1;
      i = e;
    }
    for (int t = 0; t < nt; ++t)
      for (int j = 0; j < 4; ++j) {
        if (!single[(size_t)4 * t + j]) continue;
        int v[3], c = 0;
        for (int q = 0; q < 4; ++q)
          if (q != j) v[c++] = m.tet[q * m.n_tets + t0 + t];
        const int o = m.tet[j * m.n_tets + t0 + t];
        double e1[3], e2[3], eo[3];
        for (int a = 0; a < 3; ++a) {
          const double x0 = m.X_ref[(size_t)a * m.n_nodes + v[0]];
          e1[a] = m.X_ref[(size_t)a * m.n_nodes + v[1]] - x0;
          e2[a] = m.X_ref[(size_t)a * m.n_nodes + v[2]] - x0;
          eo[a] = m.X_ref[(size_t)a * m.n_nodes + o] - x0;
        }
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        if (n[0] * eo[0] + n[1] * eo[1] + n[2] * eo[2] > 0.0) std::swap(v[1], v[2]);
        f0.push_back(v[0]);
        f1.push_back(v[1]);
        f2.push_back(v[2]);
      }
  }
  out.insert(out.end(), f0.begin(), f0.end());
  out.insert(out.end(), f1.begin(), f1.end());
  out.insert(out.end(), f2.begin(), f2.end());
}

// First particle whose triangles do not form a closed, consistently oriented
// surface (every directed edge once and its reverse once), or -1.  The
// enclosed volume, and so the volume correction, is defined only for those.
int first_open_surface(const ifem_mesh_desc& m) {
  std::vector<int32_t> start, fill, nb;
  for (int p = 0; p < m.n_particles; ++p) {
    const int t0 = m.tri_start[p], t1 = m.tri_start[p + 1];
    if (t1 == t0) continue;
    const int n0 = m.node_start[p], nn = m.node_start[p + 1] - n0;
    start.assign((size_t)nn + 1, 0);
    for (int t = t0; t < t1; ++t)
      for (int v = 0; v < 3; ++v) ++start[m.tri[v * m.n_tris + t] - n0 + 1];
    for (int i = 0; i < nn; ++i) start[i + 1] += start[i];
    fill.assign(start.begin(), start.end() - 1);
    nb.resize(start[nn]);
    for (int t = t0; t < t1; ++t)
      for (int v = 0; v < 3; ++v) nb[fill[m.tri[v * m.n_tris + t] - n0]++] = m.tri[((v + 1) % 3) * m.n_tris + t] - n0;
    for (int a = 0; a < nn; ++a)
      for (int i = start[a]; i < start[a + 1]; ++i) {
        const int b = nb[i];
        for (int j = start[a]; j < i; ++j)
          if (nb[j] == b) return p;  // the directed edge a -> b twice
        bool rev = false;
        for (int j = start[b]; j < start[b + 1] && !rev; ++j) rev = nb[j] == a;
        if (!rev) return p;  // a boundary edge or an orientation flip
      }
  }
  return -1;
}

}  // namespace

// ------------------------------------------------------------------ launch-shape tuning
namespace {

// FNV-1a hash of the sizes that decide which launch shape is fastest: the counts of particles, nodes,
// elements and bending membranes and every box's lattice.  The key of the tuning cache.
uint64_t shape_hash(const ifem_mesh_desc& m, const ifem_box* boxes, int32_t n_boxes) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)m.n_particles);
  mix((uint64_t)m.n_nodes);
  mix((uint64_t)m.n_tris);
  mix((uint64_t)m.n_tets);
  mix((uint64_t)n_boxes);
  uint64_t bending = 0;
  for (int p = 0; p < m.n_particles; ++p) bending += (m.kb && m.kb[p] != 0.0) ? 1 : 0;
  mix(bending);
  for (int b = 0; b < n_boxes; ++b)
    for (int a = 0; a < 3; ++a) mix((uint64_t)boxes[b].n[a]);
  return h;
}

// The current device as "<arch>_<compute units>_<name>" (spaces replaced), or "unknown".
std::string device_key() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string k = std::string(prop.gcnArchName) + "_" + std::to_string(prop.multiProcessorCount) + "_" + prop.name;
  for (char& c : k)
    if (c == ' ' || c == '\t' || c == '\n') c = '_';
  return k;
}

// Tuning cache: (device, shape hash) -> launch shape, filled by ifem_plan_autotune and read by
// ifem_plan_create when it is given no tuning.  Kept for the process; with IFEM_TUNE_CACHE naming a
// file, also read from it on first use and appended to on every store, one line per entry:
// "ifem-tuning-v1 <device> <hash hex> <tile x y z> <block_forces> <block_points>" (later lines win).
struct TuneEntry {
  std::string dev;
  uint64_t hash;
  ifem_tuning t;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
bool g_tune_loaded = false;

const char* tune_file() {
  const char* f = getenv("IFEM_TUNE_CACHE");
  return f && *f ? f : nullptr;
}

void tune_upsert_locked(const std::string& dev, uint64_t hash, const ifem_tuning& t) {
  for (TuneEntry& e : g_tune)
    if (e.dev == dev && e.hash == hash) {
      e.t = t;
      return;
    }
  g_tune.push_back({dev, hash, t});
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* f = tune_file();
  if (!f) return;
  std::ifstream in(f);
  std::string tag, dev;
  unsigned long long hash;
  ifem_tuning t;
  while (in >> tag >> dev >> std::hex >> hash >> std::dec >> t.tile[0] >> t.tile[1] >> t.tile[2] >> t.block_forces >>
         t.block_points)
    if (tag == "ifem-tuning-v1") tune_upsert_locked(dev, (uint64_t)hash, t);
}

bool tuning_cache_find(const std::string& dev, uint64_t hash, ifem_tuning* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load_locked();
  for (const TuneEntry& e : g_tune)
    if (e.dev == dev && e.hash == hash) {
      *out = e.t;
      return true;
    }
  return false;
}

void tuning_cache_store(const std::string& dev, uint64_t hash, const ifem_tuning& t) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load_locked();
  tune_upsert_locked(dev, hash, t);
  if (const char* f = tune_file()) {
    std::ofstream out(f, std::ios::app);
    out << "ifem-tuning-v1 " << dev << " " << std::hex << (unsigned long long)hash << std::dec << " " << t.tile[0]
        << " " << t.tile[1] << " " << t.tile[2] << " " << t.block_forces << " " << t.block_points << "\n";
  }
}

bool tile_fits_lds(const int32_t tile[3]) {
  for (int a = 0; a < 3; ++a)
    if (tile[a] < 4 || tile[a] > 64 || (tile[a] & (tile[a] - 1))) return false;
  return (int64_t)(tile[0] + 5) * (tile[1] + 2) * (tile[2] + 2) * 12 + 1024 <= (int64_t)kLdsLimit;
}

// The tile-dependent part of a plan: tiles per box, the tile -> box map, the spread lists, counts,
// offsets, cursors, flags, force bounds and halo rows, in a buffer set of their own, so that
// ifem_plan_autotune can rebuild them for another tile shape.  On failure the old workspace stays.
ifem_status build_spread(ifem_plan plan, const int32_t tile[3], hipStream_t st) {
  PlanDev& P = plan->P;
  std::vector<BoxDev> hb = plan->boxes;
  std::vector<int32_t> tile_box;
  int lists_per_entry = 2;
  for (size_t b = 0; b < hb.size(); ++b) {
    BoxDev& B = hb[b];
    int64_t nt = 1;
    for (int a = 0; a < 3; ++a) {
      B.ntile[a] = (B.n[a] + tile[a] - 1) / tile[a];
      nt *= B.ntile[a];
    }
    B.tile_base = (int32_t)tile_box.size();
    if ((int64_t)tile_box.size() + nt > (1 << 28)) return fail(IFEM_ERR_UNSUPPORTED, "too many tiles");
    tile_box.insert(tile_box.end(), (size_t)nt, (int32_t)b);
    // a (node, component) sits in its home list and at most one x-neighbour's, or both neighbours'
    // when a box ends in a one-cell-wide tile between two others
    if (B.n[0] % tile[0] == 1 && B.ntile[0] >= 3) lists_per_entry = 3;
  }
  const int n_tiles = (int)tile_box.size();
  const int64_t list_cap = (int64_t)3 * lists_per_entry * P.n_nodes;
  // lists carried between calls: room for the usual entries, half as many again, and a few per list
  const int64_t bk_cap = list_cap + (int64_t)kBucketSlack * 3 * n_tiles;
  if (bk_cap >= ((int64_t)1 << 31)) return fail(IFEM_ERR_UNSUPPORTED, "too many nodes for the spread lists");
  const int region_cells = (tile[0] + 5) * (tile[1] + 2) * (tile[2] + 2);
  const int halo_cells = tile[0] * (2 * (tile[1] + tile[2]) + 4);
  DeviceBuffers mem;
  BoxDev* d_boxes = nullptr;
  int32_t *d_tile_box = nullptr, *d_cnt = nullptr, *d_off = nullptr, *d_cur = nullptr, *d_list = nullptr,
          *d_flag = nullptr, *d_bk_list = nullptr, *d_bk_state = nullptr, *d_place = nullptr;
  int2* d_bk_lay = nullptr;
  uint32_t* d_fmax = nullptr;
  double* d_halo = nullptr;  // sized for float64
  hipError_t e = upload(mem, &d_boxes, hb.data(), hb.size(), st);
  if (e == hipSuccess) e = upload(mem, &d_tile_box, tile_box.data(), tile_box.size(), st);
  if (e == hipSuccess) e = mem.alloc(&d_cnt, (size_t)3 * n_tiles);
  if (e == hipSuccess) e = mem.alloc(&d_off, (size_t)3 * n_tiles);
  if (e == hipSuccess) e = mem.alloc(&d_place, 2);
  if (e == hipSuccess) e = mem.alloc(&d_cur, (size_t)3 * n_tiles);
  if (e == hipSuccess) e = mem.alloc(&d_list, (size_t)std::max<int64_t>(list_cap, 1));
  if (e == hipSuccess) e = mem.alloc(&d_flag, (size_t)3 * n_tiles);
  if (e == hipSuccess) e = mem.alloc(&d_fmax, (size_t)3 * n_tiles);
  if (e == hipSuccess) e = mem.alloc(&d_halo, (size_t)3 * n_tiles * halo_cells);
  // lists carried from one call's counts to the next call's layout: both layouts start without room,
  // so that the first call fills every list in the second pass
  if (e == hipSuccess) e = mem.alloc(&d_bk_list, (size_t)bk_cap);
  if (e == hipSuccess) e = mem.alloc(&d_bk_lay, (size_t)2 * 3 * n_tiles);
  if (e == hipSuccess) e = mem.alloc(&d_bk_state, 2);
  if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t*>(d_bk_lay), (int64_t)4 * 3 * n_tiles, 0, st);
  if (e == hipSuccess) e = launch_fill_i32(d_bk_state, 2, 0, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the uploads read host vectors of this frame
  if (e != hipSuccess) {
    mem.release();
    return fail(e == hipErrorOutOfMemory ? IFEM_ERR_NOMEM : IFEM_ERR_DEVICE, "spread workspace: %s",
                hipGetErrorString(e));
  }
  (void)hipDeviceSynchronize();  // no queued call may still use the old workspace
  plan->spread_mem.release();
  plan->spread_mem = std::move(mem);
  TransferArgs& ta = P.targs;
  ta.boxes = d_boxes;
  ta.tile_box = d_tile_box;
  ta.tile_count = d_cnt;
  ta.tile_off = d_off;
  ta.place = d_place;
  ta.tile_cursor = d_cur;
  ta.bin_list = d_list;
  ta.tile_flag = d_flag;
  ta.tile_fmax = d_fmax;
  ta.halo = d_halo;
  ta.bk_list = d_bk_list;
  ta.bk_lay = d_bk_lay;
  ta.bk_state = d_bk_state;
  ta.bk_cap = bk_cap;
  ta.region_cells = region_cells;
  ta.halo_cells = halo_cells;
  ta.list_cap = list_cap;
  ta.n_tiles = n_tiles;
  for (int a = 0; a < 3; ++a) {
    ta.tile[a] = tile[a];
    ta.tile_shift[a] = __builtin_ctz(tile[a]);
    plan->tune.tile[a] = tile[a];
  }
  plan->workspace_bytes =
      (int64_t)(27 * (int64_t)n_tiles + 4 + list_cap + bk_cap) * 4 + (int64_t)3 * n_tiles * halo_cells * 8;
  e = prepare_transfer_kernels(P);
  if (e != hipSuccess) return fail(IFEM_ERR_DEVICE, "spread kernel attributes: %s", hipGetErrorString(e));
  return IFEM_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

int32_t ifem_version(void) { return 10400; }

const char* ifem_last_error(void) { return g_last_error.c_str(); }

ifem_status ifem_plan_create(const ifem_mesh_desc* mesh, const ifem_box* boxes, int32_t n_boxes,
                             const ifem_tuning* tuning, void* stream, ifem_plan* out) {
  if (!out) return fail(IFEM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ifem_status s = validate_mesh(mesh, boxes, n_boxes);
  if (s != IFEM_OK) return s;
  const ifem_mesh_desc& m = *mesh;
  hipStream_t st = (hipStream_t)stream;

  // default launch shape, the fastest measured on dense suspensions and on sparse boxes of mixed
  // particles alike: 32 x 16 x 8 tiles
  ifem_tuning tn{{32, 16, 8}, 512, 256};
  if (tuning) {
    tn = *tuning;
  } else {
    ifem_tuning cached;
    if (tuning_cache_find(device_key(), shape_hash(m, boxes, n_boxes), &cached)) tn = cached;
  }
  for (int a = 0; a < 3; ++a)
    if (tn.tile[a] < 4 || tn.tile[a] > 64 || (tn.tile[a] & (tn.tile[a] - 1)))
      return fail(IFEM_ERR_INVALID_ARG, "tile sizes must be powers of two in [4, 64]");
  // spread region: the tile plus a one-cell halo along y and z and rows padded by two cells on each
  // side (odd pitch), 12 bytes per cell in float64 (a 64-bit word and a 32-bit remainder word)
  if ((int64_t)(tn.tile[0] + 5) * (tn.tile[1] + 2) * (tn.tile[2] + 2) * 12 + 1024 > (int64_t)kLdsLimit)
    return fail(IFEM_ERR_INVALID_ARG, "tile too large for LDS: (tile_x + 5)(tile_y + 2)(tile_z + 2) must be <= 13568");
  if (tn.block_forces < 64 || tn.block_forces > 512 || (tn.block_forces & (tn.block_forces - 1)))
    return fail(IFEM_ERR_INVALID_ARG, "block_forces must be a power of two in [64, 512]");
  if (tn.block_points != 64 && tn.block_points != 128 && tn.block_points != 256)
    return fail(IFEM_ERR_INVALID_ARG, "block_points must be 64, 128 or 256");

  // --- host preprocessing
  std::vector<int32_t> tri_src, tri_local, tri_pcol, tri_colb, tet_src, tet_local, tet_pcol, tet_colb;
  s = build_coloured<3>(m.tri, m.n_tris, m.n_particles, m.tri_start, m.node_start, tn.block_forces, tri_src,
                        tri_local, tri_pcol, tri_colb);
  if (s != IFEM_OK) return s;
  s = build_coloured<4>(m.tet, m.n_tets, m.n_particles, m.tet_start, m.node_start, tn.block_forces, tet_src,
                        tet_local, tet_pcol, tet_colb);
  if (s != IFEM_OK) return s;
  std::vector<char> bend(m.n_particles, 0);
  bool any_bend = false;
  for (int p = 0; p < m.n_particles; ++p) {
    bend[p] = (m.kb[p] != 0.0 && m.law[p] != IFEM_LAW_TET_NEOHOOKE && m.tri_start[p + 1] > m.tri_start[p]) ? 1 : 0;
    any_bend = any_bend || bend[p];
  }
  // A particle whose nodal forces (and curvature) fit one workgroup's LDS takes the per-particle
  // force kernel; a larger one the global-memory path.  cap: the largest of the former.
  int cap = 1, cap_mem = 0, cap_solid = 0;
  std::vector<int32_t> lds_part, large_part;
  for (int p = 0; p < m.n_particles; ++p) {
    const int nn = m.node_start[p + 1] - m.node_start[p];
    if ((size_t)nn * force_lds_per_node(any_bend) + 2048 <= kLdsLimit) {
      lds_part.push_back(p);
      cap = std::max(cap, nn);
      if (m.tri_start[p + 1] > m.tri_start[p]) cap_mem = std::max(cap_mem, nn);
      if (m.tet_start[p + 1] > m.tet_start[p]) cap_solid = std::max(cap_solid, nn);
    } else {
      large_part.push_back(p);
    }
  }
  // one-rings for bending, and for every membrane when all are closed (the volume correction)
  int open_surface = first_open_surface(m);
  std::vector<char> ringset(bend);
  bool any_ring = any_bend;
  if (open_surface < 0)
    for (int p = 0; p < m.n_particles; ++p)
      if (m.tri_start[p + 1] > m.tri_start[p]) ringset[p] = 1, any_ring = true;
  std::vector<int32_t> rstart, ring;
  if (any_ring) {
    int bad_node = -1;
    s = build_rings(m, ringset, rstart, ring, &bad_node);
    if (s != IFEM_OK) {
      int pb = 0;
      while (m.node_start[pb + 1] <= bad_node) ++pb;
      if (bend[pb]) return s;  // a bending surface must close
      open_surface = pb;       // only the volume correction is out of reach
      any_ring = any_bend;
      rstart.clear();
      ring.clear();
      if (any_bend) {
        s = build_rings(m, bend, rstart, ring, &bad_node);
        if (s != IFEM_OK) return s;
      }
    }
  }
  // the global-memory path's lists: its elements (slot order, particle by particle), and per node
  // the element corners it gathers, in element order
  std::vector<int32_t> lg_tri_begin(1, 0), lg_tet_begin(1, 0), lg_tri_slot, lg_tri_part, lg_tet_slot, lg_tet_part;
  std::vector<int32_t> lg_node_part, lg_node_base, lg_node_lp, lg_part_base(1, 0), lg_gstart, lg_gather;
  int lg_bend = 0;
  if (!large_part.empty()) {
    for (int p : large_part) {
      for (int s2 = m.tri_start[p]; s2 < m.tri_start[p + 1]; ++s2) lg_tri_slot.push_back(s2), lg_tri_part.push_back(p);
      for (int s2 = m.tet_start[p]; s2 < m.tet_start[p + 1]; ++s2) lg_tet_slot.push_back(s2), lg_tet_part.push_back(p);
      lg_tri_begin.push_back((int32_t)lg_tri_slot.size());
      lg_tet_begin.push_back((int32_t)lg_tet_slot.size());
      const int base = (int)lg_node_part.size(), lp = (int)lg_part_base.size() - 1;
      for (int k = m.node_start[p]; k < m.node_start[p + 1]; ++k)
        lg_node_part.push_back(p), lg_node_base.push_back(base), lg_node_lp.push_back(lp);
      lg_part_base.push_back((int32_t)lg_node_part.size());
      lg_bend |= bend[p];
    }
    const int64_t n_el = (int64_t)lg_tri_slot.size() + (int64_t)lg_tet_slot.size();
    if (n_el * 4 >= ((int64_t)1 << 31) || lg_node_part.size() >= ((size_t)1 << 31))
      return fail(IFEM_ERR_UNSUPPORTED, "too many elements in particles larger than a workgroup's LDS");
    const int n_ln = (int)lg_node_part.size(), n_lt = (int)lg_tri_slot.size();
    // compact index of particle p's node k: node_base + (k - node_start[p]); per element its corners
    std::vector<int32_t> first_of(m.n_particles, -1);
    for (int i = 0; i < n_ln; ++i)
      if (first_of[lg_node_part[i]] < 0) first_of[lg_node_part[i]] = i;
    auto corner = [&](int e, int v) -> int {
      if (e < n_lt) return first_of[lg_tri_part[e]] + tri_local[(size_t)v * m.n_tris + lg_tri_slot[e]];
      const int t = e - n_lt;
      return first_of[lg_tet_part[t]] + tet_local[(size_t)v * m.n_tets + lg_tet_slot[t]];
    };
    lg_gstart.assign(n_ln + 1, 0);
    for (int e = 0; e < (int)n_el; ++e)
      for (int v = 0; v < (e < n_lt ? 3 : 4); ++v) lg_gstart[corner(e, v) + 1]++;
    for (int i = 0; i < n_ln; ++i) lg_gstart[i + 1] += lg_gstart[i];
    lg_gather.resize(lg_gstart[n_ln]);
    std::vector<int32_t> cur(lg_gstart.begin(), lg_gstart.end() - 1);
    for (int e = 0; e < (int)n_el; ++e)
      for (int v = 0; v < (e < n_lt ? 3 : 4); ++v) lg_gather[cur[corner(e, v)]++] = e * 4 + v;
  }
  std::vector<int32_t> node_particle(m.n_nodes);
  for (int p = 0; p < m.n_particles; ++p)
    for (int k = m.node_start[p]; k < m.node_start[p + 1]; ++k) node_particle[k] = p;
  std::vector<int32_t> bfaces;
  boundary_faces(m, bfaces);
  const int n_bfaces = (int)(bfaces.size() / 3);
  if ((int64_t)m.n_tris + n_bfaces >= ((int64_t)1 << 31)) return fail(IFEM_ERR_UNSUPPORTED, "too many faces");
  std::vector<BoxDev> hb(n_boxes);
  int64_t total_cells = 0;
  for (int b = 0; b < n_boxes; ++b) {
    BoxDev& B = hb[b];
    memset(&B, 0, sizeof B);
    for (int a = 0; a < 3; ++a) {
      B.n[a] = boxes[b].n[a];
      B.origin[a] = boxes[b].origin[a];
    }
    for (int a = 0; a < 3; ++a) B.inv_n[a] = 1.0 / (double)B.n[a];
    B.h = boxes[b].h;
    B.inv_h = 1.0 / boxes[b].h;
    B.cell_off = total_cells;
    total_cells += (int64_t)B.n[0] * B.n[1] * B.n[2];
  }
  {
    int64_t tiles = 0;
    for (int b = 0; b < n_boxes; ++b) {
      int64_t nt = 1;
      for (int a = 0; a < 3; ++a) nt *= (boxes[b].n[a] + tn.tile[a] - 1) / tn.tile[a];
      tiles += nt;
    }
    if (tiles > (1 << 28)) return fail(IFEM_ERR_UNSUPPORTED, "too many tiles");
  }

  // contact cells: about 2 lattice cells wide, an exact tiling of every periodic box
  std::vector<ContactBoxDev> cb(n_boxes);
  int64_t n_ccells = 0;
  double contact_cell = 1e308, min_box_len = 1e308;
  for (int b = 0; b < n_boxes; ++b) {
    ContactBoxDev& C = cb[b];
    memset(&C, 0, sizeof C);
    C.base = (int32_t)n_ccells;
    int64_t nb = 1;
    for (int a = 0; a < 3; ++a) {
      C.nc[a] = std::max(1, boxes[b].n[a] / 2);
      C.origin[a] = boxes[b].origin[a];
      C.len[a] = boxes[b].n[a] * boxes[b].h;
      C.inv_len[a] = 1.0 / C.len[a];
      C.inv_cs[a] = C.nc[a] / C.len[a];
      contact_cell = std::min(contact_cell, C.len[a] / C.nc[a]);
      min_box_len = std::min(min_box_len, C.len[a]);
      nb *= C.nc[a];
    }
    n_ccells += nb;
    if (n_ccells >= ((int64_t)1 << 30)) return fail(IFEM_ERR_UNSUPPORTED, "too many contact cells");
  }

  // --- device upload
  ifem_plan plan = new ifem_plan_s();
  plan->contact_cell = contact_cell;
  plan->min_box_len = min_box_len;
  plan->tune = tn;
  plan->open_surface = open_surface;
  plan->boxes = hb;
  plan->shape_hash = shape_hash(m, boxes, n_boxes);
  PlanDev& P = plan->P;
  P.timer = &plan->timer;
  P.n_particles = m.n_particles;
  P.n_nodes = m.n_nodes;
  P.n_tris = m.n_tris;
  P.n_tets = m.n_tets;
  P.n_boxes = n_boxes;
  P.total_cells = total_cells;
  P.cap = cap;
  P.has_bending = any_bend ? 1 : 0;
  P.n_lds_part = (int32_t)lds_part.size();
  DeviceBuffers& mem = plan->mem;
  int32_t *d_ns, *d_law, *d_box, *d_tri_src, *d_tri_glob, *d_tri_local, *d_tri_pcol, *d_tri_colb;
  int32_t *d_tet_src, *d_tet_glob, *d_tet_local, *d_tet_pcol, *d_tet_colb, *d_rstart = nullptr, *d_ring = nullptr;
  int32_t* d_np;
  double *d_mu, *d_mu2, *d_kb, *d_c0, *d_tri_ref, *d_tet_ref, *d_X, *d_vref;
  unsigned long long* d_status;
  const int np = m.n_particles;
  HIP_TRY(upload(mem, &d_ns, m.node_start, np + 1, st));
  HIP_TRY(upload(mem, &d_law, m.law, np, st));
  HIP_TRY(upload(mem, &d_box, m.box, np, st));
  HIP_TRY(upload(mem, &d_mu, m.mu, np, st));
  HIP_TRY(upload(mem, &d_mu2, m.mu2, np, st));
  std::vector<double> kb_eff(np);  // bending only where a closed one-ring exists
  for (int p = 0; p < np; ++p) kb_eff[p] = bend[p] ? m.kb[p] : 0.0;
  HIP_TRY(upload(mem, &d_kb, kb_eff.data(), np, st));
  HIP_TRY(upload(mem, &d_c0, m.c0, np, st));
  HIP_TRY(upload(mem, &d_tri_src, tri_src.data(), tri_src.size(), st));
  HIP_TRY(upload(mem, &d_tri_glob, m.tri, (size_t)3 * m.n_tris, st));
  HIP_TRY(upload(mem, &d_tri_local, tri_local.data(), tri_local.size(), st));
  HIP_TRY(upload(mem, &d_tri_pcol, tri_pcol.data(), tri_pcol.size(), st));
  HIP_TRY(upload(mem, &d_tri_colb, tri_colb.data(), tri_colb.size(), st));
  HIP_TRY(upload(mem, &d_tet_src, tet_src.data(), tet_src.size(), st));
  HIP_TRY(upload(mem, &d_tet_glob, m.tet, (size_t)4 * m.n_tets, st));
  HIP_TRY(upload(mem, &d_tet_local, tet_local.data(), tet_local.size(), st));
  HIP_TRY(upload(mem, &d_tet_pcol, tet_pcol.data(), tet_pcol.size(), st));
  HIP_TRY(upload(mem, &d_tet_colb, tet_colb.data(), tet_colb.size(), st));
  int32_t* d_lds_part = nullptr;
  if (!large_part.empty() && !lds_part.empty()) HIP_TRY(upload(mem, &d_lds_part, lds_part.data(), lds_part.size(), st));
  if (!large_part.empty()) {
    LargeArgs& L = P.large;
    L.n_part = (int32_t)large_part.size();
    L.n_tri = (int32_t)lg_tri_slot.size();
    L.n_tet = (int32_t)lg_tet_slot.size();
    L.n_node = (int32_t)lg_node_part.size();
    L.any_bending = lg_bend;
    int32_t *d1, *d2, *d3, *d4, *d5, *d6, *d7, *d8, *d9, *d10 = nullptr, *d11 = nullptr, *d12, *d13;
    HIP_TRY(upload(mem, &d12, lg_node_lp.data(), lg_node_lp.size(), st));
    HIP_TRY(upload(mem, &d13, lg_part_base.data(), lg_part_base.size(), st));
    L.node_lp = d12;
    L.part_base = d13;
    HIP_TRY(upload(mem, &d1, large_part.data(), large_part.size(), st));
    HIP_TRY(upload(mem, &d2, lg_tri_begin.data(), lg_tri_begin.size(), st));
    HIP_TRY(upload(mem, &d3, lg_tet_begin.data(), lg_tet_begin.size(), st));
    HIP_TRY(upload(mem, &d8, lg_node_part.data(), lg_node_part.size(), st));
    HIP_TRY(upload(mem, &d9, lg_node_base.data(), lg_node_base.size(), st));
    HIP_TRY(upload(mem, &d10, lg_gstart.data(), lg_gstart.size(), st));
    if (!lg_gather.empty()) HIP_TRY(upload(mem, &d11, lg_gather.data(), lg_gather.size(), st));
    d4 = d5 = d6 = d7 = nullptr;
    if (L.n_tri) {
      HIP_TRY(upload(mem, &d4, lg_tri_slot.data(), lg_tri_slot.size(), st));
      HIP_TRY(upload(mem, &d5, lg_tri_part.data(), lg_tri_part.size(), st));
    }
    if (L.n_tet) {
      HIP_TRY(upload(mem, &d6, lg_tet_slot.data(), lg_tet_slot.size(), st));
      HIP_TRY(upload(mem, &d7, lg_tet_part.data(), lg_tet_part.size(), st));
    }
    L.part = d1;
    L.tri_begin = d2;
    L.tet_begin = d3;
    L.tri_slot = d4;
    L.tri_part = d5;
    L.tet_slot = d6;
    L.tet_part = d7;
    L.node_part = d8;
    L.node_base = d9;
    L.gather_start = d10;
    L.gather = d11;
    double *ef_tri, *ef_tet, *kh, *fb, *rt;
    HIP_TRY(mem.alloc(&ef_tri, (size_t)12 * std::max(L.n_tri, 1)));
    HIP_TRY(mem.alloc(&ef_tet, (size_t)16 * std::max(L.n_tet, 1)));
    HIP_TRY(mem.alloc(&kh, (size_t)std::max(L.n_node, 1)));
    HIP_TRY(mem.alloc(&fb, (size_t)3 * std::max(L.n_node, 1)));
    HIP_TRY(mem.alloc(&rt, (size_t)5 * std::max(L.n_tri + L.n_tet, 1)));
    HIP_TRY(mem.alloc(&L.vol_terms, (size_t)4 * std::max(L.n_node, 1)));
    HIP_TRY(mem.alloc(&L.lam, (size_t)L.n_part));
    HIP_TRY(mem.alloc(&L.red_part, (size_t)L.n_part * 16 * 5));
    L.ef_tri = ef_tri;
    L.ef_tet = ef_tet;
    L.kh = kh;
    L.fb = fb;
    L.red_terms = rt;
  }
  if (any_ring) {
    HIP_TRY(upload(mem, &d_rstart, rstart.data(), rstart.size(), st));
    HIP_TRY(upload(mem, &d_ring, ring.data(), ring.size(), st));
  }
  HIP_TRY(upload(mem, &d_np, node_particle.data(), node_particle.size(), st));
  HIP_TRY(upload(mem, &d_X, m.X_ref, (size_t)3 * m.n_nodes, st));
  HIP_TRY(mem.alloc(&d_tri_ref, (size_t)4 * m.n_tris));
  HIP_TRY(mem.alloc(&d_tet_ref, (size_t)10 * m.n_tets));
  HIP_TRY(mem.alloc(&d_status, 5));
  HIP_TRY(mem.alloc(&d_vref, (size_t)np));
  ContactBoxDev* d_cboxes;
  int32_t *d_bface, *d_ccount, *d_coff, *d_ccur, *d_cown;
  ContactNode* d_crec;
  unsigned long long* d_ckeys;
  HIP_TRY(upload(mem, &d_cboxes, cb.data(), cb.size(), st));
  HIP_TRY(upload(mem, &d_bface, bfaces.data(), bfaces.size(), st));
  HIP_TRY(mem.alloc(&d_ccount, (size_t)n_ccells));
  HIP_TRY(mem.alloc(&d_coff, (size_t)n_ccells));
  HIP_TRY(mem.alloc(&d_ccur, (size_t)n_ccells));
  HIP_TRY(mem.alloc(&d_cown, (size_t)n_ccells));
  int32_t *d_nlo, *d_nhi;
  HIP_TRY(mem.alloc(&d_nlo, (size_t)n_ccells));
  HIP_TRY(mem.alloc(&d_nhi, (size_t)n_ccells));
  HIP_TRY(mem.alloc(&d_crec, (size_t)m.n_nodes));
  HIP_TRY(mem.alloc(&d_ckeys, (size_t)m.n_nodes));
  int32_t* d_ckeyf;
  HIP_TRY(mem.alloc(&d_ckeyf, (size_t)m.n_nodes));
  // (face, cell) work of the contact search, in 256 equal segments: two items per face on average
  // fit; a face whose items do not fit its segment is searched whole from the slow list
  const int32_t work_cap = (int32_t)std::min<int64_t>(std::max<int64_t>(2 * ((int64_t)m.n_tris + n_bfaces), 1 << 16),
                                                      (int64_t)1 << 30);
  uint2* d_cwork;
  int32_t* d_cwcount;
  int32_t* d_cslow;
  HIP_TRY(mem.alloc(&d_cwork, (size_t)work_cap));
  HIP_TRY(mem.alloc(&d_cwcount, 256 + 3));
  int32_t* d_chits;
  HIP_TRY(mem.alloc(&d_chits, (size_t)work_cap));
  HIP_TRY(mem.alloc(&d_cslow, (size_t)m.n_tris + n_bfaces));

  P.tri_src = d_tri_src;
  P.tri_global = d_tri_glob;
  P.tri_ref = d_tri_ref;
  P.tet_src = d_tet_src;
  P.tet_global = d_tet_glob;
  P.tet_ref = d_tet_ref;
  P.status = d_status;
  P.vref = d_vref;
  ForceArgs& fa = P.fargs;
  fa.node_start = d_ns;
  fa.law = d_law;
  fa.mu = d_mu;
  fa.mu2 = d_mu2;
  fa.kb = d_kb;
  fa.c0 = d_c0;
  fa.pcol_tri = d_tri_pcol;
  fa.colb_tri = d_tri_colb;
  fa.tri_local = d_tri_local;
  fa.tri_ref = d_tri_ref;
  fa.pcol_tet = d_tet_pcol;
  fa.colb_tet = d_tet_colb;
  fa.tet_local = d_tet_local;
  fa.tet_ref = d_tet_ref;
  fa.ring_start = d_rstart;
  fa.ring = d_ring;
  fa.status = d_status;
  fa.n_nodes = m.n_nodes;
  fa.n_tris = m.n_tris;
  fa.n_tets = m.n_tets;
  fa.cap = cap;
  fa.cap_mem = cap_mem;
  fa.cap_solid = cap_solid;
  fa.lds_part = d_lds_part;
  fa.has_bending = any_bend ? 1 : 0;
  TransferArgs& ta = P.targs;
  ta.node_particle = d_np;
  ta.particle_box = d_box;
  ta.status = d_status;
  ta.total_cells = total_cells;
  ta.n_nodes = m.n_nodes;
  ta.n_boxes = n_boxes;
  {
    const ifem_status bs = build_spread(plan, tn.tile, st);
    if (bs != IFEM_OK) {
      plan->mem.release();
      plan->spread_mem.release();
      delete plan;
      return bs;
    }
  }
  ContactArgs& ca = P.cargs;
  ca.node_particle = d_np;
  ca.particle_box = d_box;
  ca.boxes = d_cboxes;
  ca.tri = d_tri_glob;
  ca.bface = d_bface;
  ca.count = d_ccount;
  ca.off = d_coff;
  ca.cursor = d_ccur;
  ca.owner = d_cown;
  ca.near_lo = d_nlo;
  ca.near_hi = d_nhi;
  ca.n_boxes = n_boxes;
  ca.rec = d_crec;
  ca.keys = d_ckeys;
  ca.keyf = d_ckeyf;
  ca.work = d_cwork;
  ca.work_count = d_cwcount;
  ca.slow_count = d_cwcount + 256;
  ca.hit_count = d_cwcount + 257;
  ca.place = d_cwcount + 258;
  ca.hits = d_chits;
  ca.slow = d_cslow;
  ca.status = d_status;
  ca.work_cap = work_cap;
  ca.n_nodes = m.n_nodes;
  ca.n_tris = m.n_tris;
  ca.n_bfaces = n_bfaces;
  ca.n_cells = (int32_t)n_ccells;

  // --- reference metrics on the device (float64), degeneracy check
  HIP_TRY(launch_fill_u64(d_status, 5, st));
  HIP_TRY(launch_ref_setup(P, d_X, st));
  HIP_TRY(launch_ref_volume(P, d_X, d_vref, st));
  unsigned long long hs[5];
  HIP_TRY(hipMemcpyAsync(hs, d_status, sizeof hs, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hs[3] != 0) {
    plan->mem.release();
    plan->spread_mem.release();
    delete plan;
    return fail(IFEM_ERR_DEGENERATE, "%llu reference elements have non-positive area or volume", hs[3]);
  }
  HIP_TRY(launch_fill_u64(d_status, 5, st));
  HIP_TRY(prepare_force_kernels(P));
  HIP_TRY(prepare_volume_kernels(P));
  HIP_TRY(prepare_fluid_kernels(P));
  HIP_TRY(hipStreamSynchronize(st));
  *out = plan;
  return ok();
}

static void release_timer(KernelTimer& t) {
  for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  t.ev.clear();
  t.slot.clear();
  t.used = t.dropped = 0;
  t.enabled = false;
}

ifem_status ifem_plan_destroy(ifem_plan plan) {
  if (!plan) return fail(IFEM_ERR_INVALID_ARG, "plan is NULL");
  (void)hipDeviceSynchronize();
  release_timer(plan->timer);
  plan->mem.release();
  plan->spread_mem.release();
  delete plan;
  return ok();
}

ifem_status ifem_plan_set(ifem_plan plan, int32_t option, int64_t value) {
  if (!plan) return fail(IFEM_ERR_INVALID_ARG, "plan is NULL");
  if (option == IFEM_OPT_SPREAD_MODE) {
    if (value != IFEM_SPREAD_TILED && value != IFEM_SPREAD_ATOMIC)
      return fail(IFEM_ERR_INVALID_ARG, "unknown spread mode %lld", (long long)value);
    plan->spread_mode = (int)value;
    return ok();
  }
  if (option == IFEM_OPT_KERNEL_TIMING) {
    if (value < 0 || value > (1 << 20)) return fail(IFEM_ERR_INVALID_ARG, "kernel timing capacity out of range");
    (void)hipDeviceSynchronize();
    release_timer(plan->timer);
    if (value > 0) {
      KernelTimer& t = plan->timer;
      t.ev.resize(2 * (size_t)value);
      t.slot.assign((size_t)value, 0);
      for (auto& e : t.ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
          release_timer(t);
          return fail(IFEM_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(r));
        }
      }
      t.enabled = true;
    }
    return ok();
  }
  return fail(IFEM_ERR_INVALID_ARG, "unknown option %d", option);
}

ifem_status ifem_plan_info(ifem_plan plan, int64_t info[10]) {
  if (!plan || !info) return fail(IFEM_ERR_INVALID_ARG, "NULL argument");
  info[0] = plan->P.total_cells;
  info[1] = plan->P.n_nodes;
  info[2] = plan->P.n_particles;
  for (int a = 0; a < 3; ++a) info[3 + a] = plan->tune.tile[a];
  info[6] = plan->tune.block_forces;
  info[7] = plan->tune.block_points;
  info[8] = plan->workspace_bytes;
  info[9] = plan->spread_mode;
  return ok();
}

}  // extern "C"

// Workspace of the allocation-free spread (ifem_spread_noalloc): a file-scope device array, one copy
// per GPU the library runs on, held until the process ends.  Host code never passes `scratch` itself
// (on the host it is a stand-in, not a device address): static_scratch() looks up each device's
// address once, with that device current, and the kernels receive that pointer.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr size_t kStaticAlign = 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call per device).
ifem_status static_scratch(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(IFEM_ERR_DEVICE, "no current device for the static scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(IFEM_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return IFEM_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

ifem_status check_common(ifem_plan plan, int32_t dtype, const void* x, const double* anchor) {
  if (!plan) return fail(IFEM_ERR_INVALID_ARG, "plan is NULL");
  if (dtype != IFEM_F32 && dtype != IFEM_F64) return fail(IFEM_ERR_INVALID_ARG, "unknown dtype %d", dtype);
  if (plan->P.n_nodes > 0 && !x) return fail(IFEM_ERR_INVALID_ARG, "x is NULL");
  if (dtype == IFEM_F32 && plan->P.n_particles > 0 && !anchor)
    return fail(IFEM_ERR_INVALID_ARG, "float32 positions need per-particle anchors");
  if (dtype == IFEM_F64 && anchor) return fail(IFEM_ERR_INVALID_ARG, "float64 positions are absolute: anchor must be NULL");
  return IFEM_OK;
}

ifem_status launched(hipError_t e) {
  if (e != hipSuccess) return fail(IFEM_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ok();
}

}  // namespace

extern "C" {

ifem_status ifem_element_forces(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, void* f_out,
                                double* red_out, void* stream) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  const PlanDev& P = plan->P;
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es, rb = (size_t)5 * P.n_particles * 8;
  if (P.n_nodes > 0 && !f_out) return fail(IFEM_ERR_INVALID_ARG, "f_out is NULL");
  if (overlaps(f_out, nb, x, nb) || overlaps(red_out, rb, x, nb) || overlaps(red_out, rb, f_out, nb) ||
      overlaps(f_out, nb, anchor, (size_t)3 * P.n_particles * 8))
    return fail(IFEM_ERR_INVALID_ARG, "outputs alias inputs");
  return launched(launch_forces(P, dtype, x, anchor, f_out, red_out, plan->tune.block_forces, (hipStream_t)stream));
}

ifem_status ifem_spread(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* F, void* grid,
                        void* stream) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  const PlanDev& P = plan->P;
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es, gb = (size_t)3 * P.total_cells * es;
  if (!grid || (P.n_nodes > 0 && !F)) return fail(IFEM_ERR_INVALID_ARG, "F or grid is NULL");
  if (overlaps(grid, gb, x, nb) || overlaps(grid, gb, F, nb) || overlaps(grid, gb, anchor, (size_t)3 * P.n_particles * 8))
    return fail(IFEM_ERR_INVALID_ARG, "grid aliases an input");
  hipStream_t st = (hipStream_t)stream;
  if (plan->spread_mode == IFEM_SPREAD_ATOMIC)
    return launched(launch_spread_atomic(P, dtype, x, anchor, F, grid, plan->tune.block_points, st));
  return launched(launch_spread_tiled(P, P.targs, dtype, x, anchor, F, grid, st));
}

ifem_status ifem_spread_noalloc(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* F,
                                void* grid, void* stream) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  const PlanDev& P = plan->P;
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es, gb = (size_t)3 * P.total_cells * es;
  if (!grid || (P.n_nodes > 0 && !F)) return fail(IFEM_ERR_INVALID_ARG, "F or grid is NULL");
  if (overlaps(grid, gb, x, nb) || overlaps(grid, gb, F, nb) || overlaps(grid, gb, anchor, (size_t)3 * P.n_particles * 8))
    return fail(IFEM_ERR_INVALID_ARG, "grid aliases an input");
  // the plan's spread workspace, laid out in the device's static array instead
  const TransferArgs& t = P.targs;
  const int64_t nl = 3 * (int64_t)t.n_tiles;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + kStaticAlign - 1) / kStaticAlign * kStaticAlign;
    return at;
  };
  const size_t o_cnt = take((size_t)nl * 4), o_off = take((size_t)nl * 4), o_cur = take((size_t)nl * 4),
               o_place = take(2 * 4),
               o_flag = take((size_t)nl * 4), o_fmax = take((size_t)nl * 4),
               o_list = take((size_t)std::max<int64_t>(t.list_cap, 1) * 4),
               o_halo = take((size_t)nl * t.halo_cells * es);
  if (off > kStaticScratchBytes)
    return fail(IFEM_ERR_UNSUPPORTED, "the spread workspace of this plan (%zu bytes in this precision) exceeds the "
                                      "static scratch of %zu bytes", off, kStaticScratchBytes);
  unsigned char* base = nullptr;
  s = static_scratch(&base);
  if (s != IFEM_OK) return s;
  TransferArgs a = t;
  a.tile_count = reinterpret_cast<int32_t*>(base + o_cnt);
  a.tile_off = reinterpret_cast<int32_t*>(base + o_off);
  a.place = reinterpret_cast<int32_t*>(base + o_place);
  a.tile_cursor = reinterpret_cast<int32_t*>(base + o_cur);
  a.tile_flag = reinterpret_cast<int32_t*>(base + o_flag);
  a.tile_fmax = reinterpret_cast<uint32_t*>(base + o_fmax);
  a.bin_list = reinterpret_cast<int32_t*>(base + o_list);
  a.halo = base + o_halo;
  a.bk_list = nullptr;  // no lists carried between calls: every call fills its lists in the second pass
  a.bk_lay = nullptr;
  a.bk_state = nullptr;
  return launched(launch_spread_tiled(P, a, dtype, x, anchor, F, grid, (hipStream_t)stream));
}

ifem_status ifem_interp(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* grid_u,
                        void* v_out, void* stream) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  const PlanDev& P = plan->P;
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es, gb = (size_t)3 * P.total_cells * es;
  if (!grid_u || (P.n_nodes > 0 && !v_out)) return fail(IFEM_ERR_INVALID_ARG, "grid_u or v_out is NULL");
  if (overlaps(v_out, nb, x, nb) || overlaps(v_out, nb, grid_u, gb) ||
      overlaps(v_out, nb, anchor, (size_t)3 * P.n_particles * 8))
    return fail(IFEM_ERR_INVALID_ARG, "v_out aliases an input");
  return launched(launch_interp(P, dtype, x, anchor, grid_u, v_out, plan->tune.block_points, (hipStream_t)stream));
}

ifem_status ifem_volume_correct(ifem_plan plan, int32_t dtype, const void* x, const double* V0, void* x_out,
                                double* lambda_out, void* stream) {
  if (!plan) return fail(IFEM_ERR_INVALID_ARG, "plan is NULL");
  if (dtype != IFEM_F32 && dtype != IFEM_F64) return fail(IFEM_ERR_INVALID_ARG, "unknown dtype %d", dtype);
  const PlanDev& P = plan->P;
  if (P.n_nodes > 0 && (!x || !x_out)) return fail(IFEM_ERR_INVALID_ARG, "x or x_out is NULL");
  if (plan->open_surface >= 0)
    return fail(IFEM_ERR_UNSUPPORTED, "particle %d: the volume correction needs a closed, consistently oriented surface",
                plan->open_surface);
  const size_t nb = (size_t)3 * P.n_nodes * (dtype == IFEM_F32 ? 4 : 8), pb = (size_t)P.n_particles * 8;
  if ((x_out != x && overlaps(x_out, nb, x, nb)) || overlaps(x_out, nb, V0, pb) || overlaps(lambda_out, pb, x, nb) ||
      overlaps(lambda_out, pb, x_out, nb) || overlaps(lambda_out, pb, V0, pb))
    return fail(IFEM_ERR_INVALID_ARG, "outputs alias inputs (only x_out == x is allowed)");
  return launched(launch_volume(P, dtype, x, V0, x_out, lambda_out, (hipStream_t)stream));
}

ifem_status ifem_advance(ifem_plan plan, int32_t dtype, const void* x, const void* v, const void* v_prev, double dt,
                         void* x_out, void* stream) {
  if (!plan) return fail(IFEM_ERR_INVALID_ARG, "plan is NULL");
  if (dtype != IFEM_F32 && dtype != IFEM_F64) return fail(IFEM_ERR_INVALID_ARG, "unknown dtype %d", dtype);
  const PlanDev& P = plan->P;
  if (P.n_nodes > 0 && (!x || !v || !x_out)) return fail(IFEM_ERR_INVALID_ARG, "x, v or x_out is NULL");
  if (!std::isfinite(dt)) return fail(IFEM_ERR_INVALID_ARG, "dt is not finite");
  const size_t nb = (size_t)3 * P.n_nodes * (dtype == IFEM_F32 ? 4 : 8);
  if ((x_out != x && overlaps(x_out, nb, x, nb)) || overlaps(x_out, nb, v, nb) || overlaps(x_out, nb, v_prev, nb))
    return fail(IFEM_ERR_INVALID_ARG, "x_out aliases an input (only x_out == x is allowed)");
  return launched(launch_advance(P, dtype, x, v, v_prev, dt, x_out, (hipStream_t)stream));
}

ifem_status ifem_interp_cells(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* grid,
                              int32_t ncomp, void* out, void* stream) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  const PlanDev& P = plan->P;
  if (ncomp < 1 || ncomp > 64) return fail(IFEM_ERR_INVALID_ARG, "ncomp must be in [1, 64]");
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es;
  const size_t ob = (size_t)ncomp * P.n_nodes * es, gb = (size_t)ncomp * P.total_cells * es;
  if (!grid || (P.n_nodes > 0 && !out)) return fail(IFEM_ERR_INVALID_ARG, "grid or out is NULL");
  if (overlaps(out, ob, x, nb) || overlaps(out, ob, grid, gb) || overlaps(out, ob, anchor, (size_t)3 * P.n_particles * 8))
    return fail(IFEM_ERR_INVALID_ARG, "out aliases an input");
  return launched(launch_interp_cells(P, dtype, x, anchor, grid, ncomp, out, (hipStream_t)stream));
}

ifem_status ifem_fluid_forces(ifem_plan plan, int32_t dtype, const void* x, const void* v, const void* C, double eta,
                              double G, void* f_inout, void* stream) {
  if (!plan) return fail(IFEM_ERR_INVALID_ARG, "plan is NULL");
  if (dtype != IFEM_F32 && dtype != IFEM_F64) return fail(IFEM_ERR_INVALID_ARG, "unknown dtype %d", dtype);
  const PlanDev& P = plan->P;
  if (P.n_nodes > 0 && (!x || !v || !f_inout)) return fail(IFEM_ERR_INVALID_ARG, "x, v or f_inout is NULL");
  if (!std::isfinite(eta) || !std::isfinite(G)) return fail(IFEM_ERR_INVALID_ARG, "eta and G must be finite");
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es, cb = (size_t)6 * P.n_nodes * es;
  if (overlaps(f_inout, nb, x, nb) || overlaps(f_inout, nb, v, nb) || overlaps(f_inout, nb, C, cb))
    return fail(IFEM_ERR_INVALID_ARG, "f_inout aliases an input");
  return launched(launch_fluid(P, dtype, x, v, C, eta, G, f_inout, (hipStream_t)stream));
}

ifem_status ifem_antistick(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, double d_min,
                           void* x_out, int64_t* face_out, void* stream) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  const PlanDev& P = plan->P;
  if (P.n_nodes > 0 && !x_out) return fail(IFEM_ERR_INVALID_ARG, "x_out is NULL");
  if (!(d_min > 0.0) || !(d_min <= plan->contact_cell) || !(d_min <= 0.25 * plan->min_box_len))
    return fail(IFEM_ERR_INVALID_ARG, "d_min must be positive, at most the contact-cell width %g and a quarter box",
                plan->contact_cell);
  const size_t nb = (size_t)3 * P.n_nodes * (dtype == IFEM_F32 ? 4 : 8), fb = (size_t)P.n_nodes * 8;
  const size_t ab = (size_t)3 * P.n_particles * 8;
  if (overlaps(x_out, nb, x, nb) || overlaps(x_out, nb, anchor, ab) || overlaps(face_out, fb, x, nb) ||
      overlaps(face_out, fb, x_out, nb) || overlaps(face_out, fb, anchor, ab))
    return fail(IFEM_ERR_INVALID_ARG, "outputs alias inputs (every node reads the positions before the pass)");
  return launched(launch_antistick(P, dtype, x, anchor, d_min, x_out, face_out, (hipStream_t)stream));
}

ifem_status ifem_plan_kernel_times(ifem_plan plan, void* stream, double total_ms[16], int64_t launches[16],
                                   int32_t reset) {
  if (!plan || !total_ms || !launches) return fail(IFEM_ERR_INVALID_ARG, "NULL argument");
  KernelTimer& t = plan->timer;
  for (int i = 0; i < 16; ++i) {
    total_ms[i] = 0.0;
    launches[i] = 0;
  }
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess && t.used) e = hipEventSynchronize(t.ev[2 * t.used - 1]);
  if (e != hipSuccess) return fail(IFEM_ERR_DEVICE, "timer synchronisation failed: %s", hipGetErrorString(e));
  for (size_t i = 0; i < t.used; ++i) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]);
    if (e != hipSuccess) return fail(IFEM_ERR_DEVICE, "hipEventElapsedTime: %s", hipGetErrorString(e));
    total_ms[t.slot[i]] += ms;
    launches[t.slot[i]] += 1;
  }
  launches[15] = (int64_t)t.dropped;
  if (reset) t.used = t.dropped = 0;
  return ok();
}

ifem_status ifem_plan_status(ifem_plan plan, void* stream, int64_t counts[5], int32_t reset) {
  if (!plan || !counts) return fail(IFEM_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long hs[5];
  hipError_t e = hipMemcpyAsync(hs, plan->P.status, sizeof hs, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(IFEM_ERR_DEVICE, "status read failed: %s", hipGetErrorString(e));
  for (int i = 0; i < 5; ++i) counts[i] = (int64_t)hs[i];
  if (reset) {
    e = launch_fill_u64(plan->P.status, 5, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(IFEM_ERR_DEVICE, "status reset failed: %s", hipGetErrorString(e));
  }
  return ok();
}

}  // extern "C"

extern "C" {

ifem_status ifem_plan_autotune(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* F,
                               void* grid, const void* grid_u, void* v_out, void* stream, ifem_tuning* chosen) {
  ifem_status s = check_common(plan, dtype, x, anchor);
  if (s != IFEM_OK) return s;
  PlanDev& P = plan->P;
  const size_t es = dtype == IFEM_F32 ? 4 : 8, nb = (size_t)3 * P.n_nodes * es, gb = (size_t)3 * P.total_cells * es;
  if (!grid || !grid_u || (P.n_nodes > 0 && (!F || !v_out)))
    return fail(IFEM_ERR_INVALID_ARG, "F, grid, grid_u or v_out is NULL");
  if (overlaps(grid, gb, x, nb) || overlaps(grid, gb, F, nb) || overlaps(grid, gb, grid_u, gb) ||
      overlaps(v_out, nb, x, nb) || overlaps(v_out, nb, grid_u, gb) || overlaps(v_out, nb, F, nb) ||
      overlaps(v_out, nb, grid, gb))
    return fail(IFEM_ERR_INVALID_ARG, "outputs alias inputs or each other");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return fail(IFEM_ERR_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(IFEM_ERR_DEVICE, "hipEventCreate failed");
  }
  // median of kReps timed calls after two untimed ones, each call after an untimed `between` (the
  // other transfer, which streams its own grid through the caches as a coupling step does, so that no
  // candidate is timed on data still cached from its previous call); +inf if a launch fails
  constexpr int kReps = 5;
  auto timed = [&](auto&& call, auto&& between) -> float {
    for (int i = 0; i < 2; ++i)
      if (call() != hipSuccess) return INFINITY;
    float t[kReps];
    for (int i = 0; i < kReps; ++i) {
      if (between() != hipSuccess) return INFINITY;
      (void)hipEventRecord(ev[0], st);
      if (call() != hipSuccess) return INFINITY;
      (void)hipEventRecord(ev[1], st);
      if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&t[i], ev[0], ev[1]) != hipSuccess)
        return INFINITY;
    }
    std::sort(t, t + kReps);
    return t[kReps / 2];
  };
  // spread tiles: the shapes measured competitive on dense and on sparse workloads
  static const int32_t kTiles[][3] = {{32, 16, 8}, {16, 16, 16}, {64, 8, 8}, {32, 32, 4}, {16, 32, 8},
                                      {32, 8, 8},  {16, 16, 8},  {64, 16, 4}, {32, 16, 16}};
  const ifem_tuning before = plan->tune;
  // bring the clocks up first (a freshly started device times its first candidates slow), then time the
  // candidates in order and again in reverse order and keep each one's better median, so that a drift
  // during the tuning favours no candidate
  for (int i = 0; i < 30; ++i)
    if (launch_spread_tiled(P, P.targs, dtype, x, anchor, F, grid, st) != hipSuccess ||
        launch_interp(P, dtype, x, anchor, grid_u, v_out, before.block_points, st) != hipSuccess)
      break;
  constexpr int kNTiles = (int)(sizeof kTiles / sizeof kTiles[0]);
  float tile_ms[kNTiles];
  for (int i = 0; i < kNTiles; ++i) tile_ms[i] = INFINITY;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < kNTiles; ++j) {
      const int i = pass == 0 ? j : kNTiles - 1 - j;
      if (!tile_fits_lds(kTiles[i])) continue;
      if (build_spread(plan, kTiles[i], st) != IFEM_OK) continue;  // e.g. no memory for this shape's workspace
      const float ms = timed([&] { return launch_spread_tiled(P, P.targs, dtype, x, anchor, F, grid, st); }, [&] {
        return launch_interp(P, dtype, x, anchor, grid_u, v_out, before.block_points, st);
      });
      tile_ms[i] = std::min(tile_ms[i], ms);
    }
  int32_t best[3] = {before.tile[0], before.tile[1], before.tile[2]};
  float best_ms = INFINITY;
  for (int i = 0; i < kNTiles; ++i)
    if (tile_ms[i] < best_ms) {
      best_ms = tile_ms[i];
      for (int a = 0; a < 3; ++a) best[a] = kTiles[i][a];
    }
  if (best[0] != P.targs.tile[0] || best[1] != P.targs.tile[1] || best[2] != P.targs.tile[2]) {
    s = build_spread(plan, best, st);
    if (s != IFEM_OK) {
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
      return s;
    }
  }
  // threads per workgroup of the point kernels, timed on the interpolation
  static const int kBlocks[] = {64, 128, 256};
  float bp_ms[3] = {INFINITY, INFINITY, INFINITY};
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < 3; ++j) {
      const int i = pass == 0 ? j : 2 - j;
      const float ms = timed([&] { return launch_interp(P, dtype, x, anchor, grid_u, v_out, kBlocks[i], st); },
                             [&] { return launch_spread_tiled(P, P.targs, dtype, x, anchor, F, grid, st); });
      bp_ms[i] = std::min(bp_ms[i], ms);
    }
  int best_bp = before.block_points;
  float best_bp_ms = INFINITY;
  for (int i = 0; i < 3; ++i)
    if (bp_ms[i] < best_bp_ms) {
      best_bp_ms = bp_ms[i];
      best_bp = kBlocks[i];
    }
  plan->tune.block_points = best_bp;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  tuning_cache_store(device_key(), plan->shape_hash, plan->tune);
  if (chosen) *chosen = plan->tune;
  return ok();
}

}  // extern "C"
