// Lagrangian <-> Eulerian transfer of the IFEM coupling step on gfx950
// (Sec. II.C: linear MLS weights on the 27-node stencil around the nearest
// lattice node; interpolation v_k = sum_J phi_J v_J, spreading
// F_J = sum_k phi_J F_k).
//
//  k_interp<T>          one thread per node, three components, gathers 27
//                       lattice values per component.
//  k_spread_atomic<T>   the plain baseline: one global atomic add per
//                       (node, component, stencil node).
//  tiled spread         deterministic and free of global float atomics:
//    k_bin_count<T>     per (node, component): counts the node in the list
//                       of the tile holding its nearest lattice node and
//                       writes it into that list as laid out from the
//                       previous call's counts, when it fits there;
//    k_scan             list offsets from the counts, and the layout for
//                       the next call;
//    k_bin_fill<T>      writes the nodes of the lists that outgrew their
//                       layout into lists laid out from this call's counts
//                       (returns at once when none did);
//    k_spread_home<T>   one workgroup per (component, tile): accumulates all
//                       contributions of the tile's list in an LDS region
//                       (tile + one-cell halo) as 64-bit fixed-point
//                       integers (exact, order-independent sums; float64
//                       uses a two-word split); writes the interior to the
//                       grid and the halo shell to scratch;
//    k_spread_merge<T>  adds the neighbours' halo values to each tile's
//                       border cells in a fixed order.
#include <cfloat>
#include <algorithm>
#include <climits>

#include "ifem_device.hpp"
#include "ifem_internal.hpp"

namespace ifem {

// Absolute float64 position of a node of particle p from its stored coordinates xv (float32 offsets
// from the particle's anchor, or float64 positions).
template <typename T>
__device__ __forceinline__ void position_of(const T xv[3], const double* __restrict__ anchor, int p, double out[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = sizeof(T) == 4 ? anchor[3 * p + c] + (double)xv[c] : (double)xv[c];
}

template <typename T>
__device__ __forceinline__ void node_position(const TransferArgs& a, const T* __restrict__ x,
                                              const double* __restrict__ anchor, int k, int p, double out[3]) {
  const int64_t N = a.n_nodes;
  const T xv[3] = {x[k], x[N + k], x[2 * N + k]};
  position_of(xv, anchor, p, out);
}

// ------------------------------------------------------------------ fills (graph-safe, no memset nodes)
template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The list counts and bound codes of the spread, cleared together with the placement's running totals
// (graph-safe: no memset node); the layout the previous call's scan prepared becomes this call's, and
// its overflow flag is cleared.
__global__ void k_zero_counters(int32_t* __restrict__ count, uint32_t* __restrict__ code, int n,
                                int32_t* __restrict__ place, int32_t* __restrict__ bk_state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    count[i] = 0;
    code[i] = 0u;
  }
  if (i == 0) {
    place[0] = 0;
    place[1] = 0;
  }
  if (i == 0 && bk_state) {
    bk_state[0] ^= 1;
    bk_state[1] = 0;
  }
}

template <typename T>
static hipError_t fill(T* p, int64_t n, T v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int B = 256;
  int64_t g = (n + B - 1) / B;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)g), dim3(B), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st) { return fill(p, n, 0ull, st); }
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
  return fill(p, n, v, st);
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) { return fill(p, n, v, st); }

// ------------------------------------------------------------------ interpolation
// Three consecutive lattice values of one x-row, in one 12- or 24-byte load
// when the row does not cross the periodic seam.
template <typename T>
struct alignas(sizeof(T)) Row3 {
  T v[3];
};

template <typename T>
__global__ void __launch_bounds__(256) k_interp(const TransferArgs a, const T* __restrict__ x,
                                                const double* __restrict__ anchor, const T* __restrict__ grid,
                                                T* __restrict__ v) {
  const int k = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= a.n_nodes) return;
  const int64_t N = a.n_nodes;
  const T xv[3] = {x[k], x[N + k], x[2 * N + k]};  // requested before the particle's box is known
  const int p = a.node_particle[k];
  const BoxDev B = box_of(a, p);
  double pos[3];
  position_of(xv, anchor, p, pos);
  unsigned int bad = 0;
  // unrolled: the three components' loads and arithmetic interleave
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int32_t base[3];
    double tau64[3];
    nearest_node(B, d, pos, base, tau64);
    const T tau[3] = {(T)tau64[0], (T)tau64[1], (T)tau64[2]};
    T W[27], c[4];
    if (!mls_weights<T>(tau, W, c)) ++bad;
    const T* g = grid + d * a.total_cells + B.cell_off;  // cells of one box fit 32-bit offsets
    const int32_t nxy = B.n[0] * B.n[1];
    int32_t ro[9];  // in-box offsets of the stencil's rows, first column
#pragma unroll
    for (int mz = 0; mz < 3; ++mz)
#pragma unroll
      for (int my = 0; my < 3; ++my)
        ro[mz * 3 + my] = wrap1(base[2] + mz - 1, B.n[2]) * nxy + wrap1(base[1] + my - 1, B.n[1]) * B.n[0];
    T u[27];
    if (__builtin_expect(base[0] != 0 && base[0] != B.n[0] - 1, 1)) {  // one 12- or 24-byte load per row
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const Row3<T> r3 = *reinterpret_cast<const Row3<T>*>(g + (uint32_t)(ro[r] + base[0] - 1));
        u[3 * r] = r3.v[0];
        u[3 * r + 1] = r3.v[1];
        u[3 * r + 2] = r3.v[2];
      }
    } else {  // the stencil crosses the periodic seam along x
      const int32_t ix0 = wrap1(base[0] - 1, B.n[0]), ix2 = wrap1(base[0] + 1, B.n[0]);
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        u[3 * r] = g[(uint32_t)(ro[r] + ix0)];
        u[3 * r + 1] = g[(uint32_t)(ro[r] + base[0])];
        u[3 * r + 2] = g[(uint32_t)(ro[r] + ix2)];
      }
    }
    T s = 0;
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const T vz = mz == 0 ? c[0] - c[3] : (mz == 1 ? c[0] : c[0] + c[3]);
#pragma unroll
      for (int my = 0; my < 3; ++my) {
        const T* uu = u + (mz * 3 + my) * 3;
        const T vyz = my == 0 ? vz - c[2] : (my == 1 ? vz : vz + c[2]);
        const T* w = W + (mz * 3 + my) * 3;
        s += w[0] * (vyz - c[1]) * uu[0];
        s += w[1] * vyz * uu[1];
        s += w[2] * (vyz + c[1]) * uu[2];
      }
    }
    v[d * (int64_t)a.n_nodes + k] = s;
  }
  if (bad) atomicAdd(a.status + 2, (unsigned long long)bad);
}

// ------------------------------------------------------------------ plain atomic spread
template <typename T>
__global__ void __launch_bounds__(256) k_spread_atomic(const TransferArgs a, const T* __restrict__ x,
                                                       const double* __restrict__ anchor, const T* __restrict__ F,
                                                       T* __restrict__ grid) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_nodes) return;
  const int p = a.node_particle[k];
  const BoxDev B = box_of(a, p);
  double pos[3];
  node_position(a, x, anchor, k, p, pos);
  unsigned int bad = 0;
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    int32_t base[3];
    double tau64[3];
    nearest_node(B, d, pos, base, tau64);
    const T tau[3] = {(T)tau64[0], (T)tau64[1], (T)tau64[2]};
    T W[27], c[4];
    if (!mls_weights<T>(tau, W, c)) ++bad;
    const T f = F[d * (int64_t)a.n_nodes + k];
    T* g = grid + d * a.total_cells + B.cell_off;
    T phi[27];
    mls_phi<T>(W, c, phi);
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const int64_t zo = (int64_t)wrap1(base[2] + mz - 1, B.n[2]) * B.n[1] * B.n[0];
#pragma unroll
      for (int my = 0; my < 3; ++my) {
        const int64_t yo = zo + (int64_t)wrap1(base[1] + my - 1, B.n[1]) * B.n[0];
#pragma unroll
        for (int mx = 0; mx < 3; ++mx)
          atomicAdd(g + yo + wrap1(base[0] + mx - 1, B.n[0]), phi[(mz * 3 + my) * 3 + mx] * f);
      }
    }
  }
  if (bad) atomicAdd(a.status + 2, (unsigned long long)bad);
}

// ------------------------------------------------------------------ tiled spread: binning
// A (node, component) belongs to the list of the tile holding its nearest
// lattice node and, when that node lies on the tile's first or last x layer,
// also to the list of the x-neighbour tile that its stencil reaches into.
// Each tile thus sees every contribution that lands inside its x range (no
// halo along x) and keeps a one-cell halo along y and z only, whose rows are
// contiguous in memory.  The atomics on the list counters are aggregated per
// wavefront (one per distinct list among 64 consecutive nodes, which lie close
// together on one surface).
//
// Lists change little from one call to the next (positions move by a fraction
// of a cell per step), so each call lays out the next call's lists from its own
// counts with some room to grow (bk_want).  The count pass takes a node's slot
// in a list from the atomic that counts it and writes the node there when the
// list's room allows; only the lists that outgrow their room (none, in the
// steady state; all of them on a plan's first call) are filled again by a
// second pass over the nodes, into lists laid out from this call's counts.
// The tile sums do not depend on where or in which order a list holds its
// entries (integer sums), so the result is the same either way.
constexpr int kListsPerEntry = 3;
// Room of a list of cnt entries in the next call's layout.  32-bit: the rooms of all lists add up to
// at most 1.5 list_cap + kBucketSlack per list, less than 1.5 times the carried array (< 2^31), so
// below 2^32.
__host__ __device__ __forceinline__ uint32_t bk_want(int32_t cnt) {
  return (uint32_t)cnt + (uint32_t)(cnt >> 1) + kBucketSlack;
}

// This call's layout of the carried lists: per list its first slot in bk_list and its room.
__device__ __forceinline__ const int2* bk_layout(const TransferArgs& a) {
  return a.bk_lay + (int64_t)a.bk_state[0] * (3 * a.n_tiles);
}

// Lists of a node for one component: keys[0] the home tile, keys[1] and
// keys[2] the left and right x-neighbours when reached (else -1; a tile that
// equals an earlier key is not repeated).  The count and fill passes both call
// this on the same inputs, so they agree bit for bit.
__device__ __forceinline__ void node_lists(const TransferArgs& a, const BoxDev& B, int d, const int32_t base[3],
                                           int keys[kListsPerEntry]) {
  const int tx = base[0] >> a.tile_shift[0], ty = base[1] >> a.tile_shift[1], tz = base[2] >> a.tile_shift[2];
  const int row = d * a.n_tiles + B.tile_base + (tz * B.ntile[1] + ty) * B.ntile[0];
  const int c0x = tx << a.tile_shift[0];
  const int exx = min(a.tile[0], B.n[0] - c0x);
  int left = -1, right = -1;
  if (base[0] == c0x) {
    const int t = tx == 0 ? B.ntile[0] - 1 : tx - 1;
    if (t != tx) left = t;
  }
  if (base[0] == c0x + exx - 1) {
    const int t = tx == B.ntile[0] - 1 ? 0 : tx + 1;
    if (t != tx && t != left) right = t;
  }
  keys[0] = row + tx;
  keys[1] = left >= 0 ? row + left : -1;
  keys[2] = right >= 0 ? row + right : -1;
}

// The lists of one node, all components: keys[d * kListsPerEntry + j].
template <typename T>
__device__ __forceinline__ void all_lists(const TransferArgs& a, const T* __restrict__ x,
                                          const double* __restrict__ anchor, int k, int keys[3 * kListsPerEntry]) {
#pragma unroll
  for (int i = 0; i < 3 * kListsPerEntry; ++i) keys[i] = -1;
  if (k < a.n_nodes) {
    const int64_t N = a.n_nodes;
    const T xv[3] = {x[k], x[N + k], x[2 * N + k]};  // requested before the particle's box is known
    const int p = a.node_particle[k];
    const BoxDev B = box_of(a, p);
    double pos[3];
    position_of(xv, anchor, p, pos);
    int32_t b0[3], bh[3];
    nearest_bases(B, pos, b0, bh);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int32_t base[3] = {d == 0 ? b0[0] : bh[0], d == 1 ? b0[1] : bh[1], d == 2 ? b0[2] : bh[2]};
      node_lists(a, B, d, base, keys + d * kListsPerEntry);
    }
  }
}

// Bound code of a force value for the fixed-point scale: 0 for 0, e + 1100 for
// a finite |f| < 2^e (e from frexp: -1073..1024 in float64, so the code is
// positive), all ones for a non-finite value.  Codes order like the bounds,
// so a list's bound is the atomic maximum of its codes.
constexpr int kBoundBias = 1100;
constexpr uint32_t kBoundPoison = 0xffffffffu;
template <typename T>
__device__ __forceinline__ uint32_t bound_code(T f) {
  const double v = fabs((double)f);
  if (!(v <= DBL_MAX)) return kBoundPoison;
  if (v == 0.0) return 0u;
  int e;
  frexp(v, &e);
  return (uint32_t)(e + kBoundBias);
}

// Count pass: one thread per node; every (node, component) counts once in
// each of its lists, one atomic per distinct list per wavefront.  The same
// atomics raise each list's bound code (bound_code) to the wavefront's largest
// of that component; the bound sets the list's fixed-point scale.  With the
// carried layout, the count a group's atomic returns places its members in the
// list; a member past the list's room raises the overflow flag instead.
template <typename T>
__global__ void __launch_bounds__(256) k_bin_count(const TransferArgs a, const T* __restrict__ x,
                                                   const double* __restrict__ anchor, const T* __restrict__ F) {
  constexpr int NK = 3 * kListsPerEntry;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int2* lay = a.bk_list ? bk_layout(a) : nullptr;  // read early: its latency hides under the keys'
  int key[NK];
  all_lists(a, x, anchor, k, key);
  T fv[3];  // the three loads in flight together (bound_code(0) = 0 past the last node)
#pragma unroll
  for (int d = 0; d < 3; ++d) fv[d] = k < a.n_nodes ? F[d * (int64_t)a.n_nodes + k] : T(0);
  uint32_t fm[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) fm[d] = wave_max_u32(bound_code(fv[d]));
  if (!a.bk_list) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      int leader, rank, size;
      wave_groups(key[i], leader, rank, size);
      if (size > 0) {
        atomicAdd(a.tile_count + key[i], size);
        atomicMax(a.tile_fmax + key[i], fm[i / kListsPerEntry]);
      }
    }
    return;
  }
  // the layout loads and all atomics of the wavefront in flight before any result is used
  int2 lk[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) lk[i] = lay[max(key[i], 0)];
  int leader[NK], rank[NK], size[NK], base[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) wave_groups(key[i], leader[i], rank[i], size[i]);
#pragma unroll
  for (int i = 0; i < NK; ++i)
    if (size[i] > 0) atomicMax(a.tile_fmax + key[i], fm[i / kListsPerEntry]);
#pragma unroll
  for (int i = 0; i < NK; ++i) base[i] = size[i] > 0 ? atomicAdd(a.tile_count + key[i], size[i]) : 0;
  // every destination before the first store, so that no store waits on another
  int dst[NK];
  bool over = false;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const int slot = __shfl(base[i], leader[i], kWave) + rank[i];
    const bool fits = slot < lk[i].y;
    dst[i] = key[i] >= 0 && fits ? lk[i].x + slot : -1;
    over = over || (key[i] >= 0 && !fits);
  }
#pragma unroll
  for (int i = 0; i < NK; ++i)
    if (dst[i] >= 0) a.bk_list[dst[i]] = k;
  const unsigned long long ob = __ballot(over);  // one flag store per wavefront
  if (ob && (threadIdx.x & (kWave - 1)) == __ffsll((long long)ob) - 1) a.bk_state[1] = 1;
}

// Fill pass: the same keys; each group's leader takes a run of slots from the
// list's cursor (initialised to the list's offset by the scan) and the group
// members write the node id into it.  All atomics of a wavefront are issued
// before any result is used.  With the carried layout only the lists that
// outgrew their room are filled here, and only when some did.
template <typename T>
__global__ void __launch_bounds__(256) k_bin_fill(const TransferArgs a, const T* __restrict__ x,
                                                  const double* __restrict__ anchor) {
  constexpr int NK = 3 * kListsPerEntry;
  if (a.bk_list && !a.bk_state[1]) return;  // every list fitted (uniform)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int key[NK], leader[NK], rank[NK], size[NK], base[NK];
  all_lists(a, x, anchor, k, key);
  if (a.bk_list) {  // only the lists that outgrew their room
    const int2* lay = bk_layout(a);
    int room[NK], cnt[NK];
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      room[i] = key[i] >= 0 ? lay[key[i]].y : 0;
      cnt[i] = key[i] >= 0 ? a.tile_count[key[i]] : 0;
    }
#pragma unroll
    for (int i = 0; i < NK; ++i)
      if (cnt[i] <= room[i]) key[i] = -1;
  }
#pragma unroll
  for (int i = 0; i < NK; ++i) wave_groups(key[i], leader[i], rank[i], size[i]);
#pragma unroll
  for (int i = 0; i < NK; ++i) base[i] = size[i] > 0 ? atomicAdd(a.tile_cursor + key[i], size[i]) : 0;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const int slot = __shfl(base[i], leader[i], kWave) + rank[i];
    if (key[i] >= 0 && slot < a.list_cap) a.bin_list[slot] = k;
  }
}

// List placement: any disjoint placement of the lists works, so the lists are
// cut into chunks of kScanThreads * kScanPer, one per workgroup; a workgroup
// sums its counts (thread t takes the counts t, t + 256, ... of the chunk:
// coalesced loads), scans the thread totals and reserves its chunk's total
// with one atomic on a running total, and each thread lays its lists out one
// after another from there.  No workgroup waits for another.  Every cursor
// starts at its list's offset; a total above the list capacity is flagged.
// With the carried layout the same pass lays out the next call's lists, each
// with room bk_want(count), from a second running total; lists past the end of
// bk_list get no room (their nodes take the fill pass).
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;  // lists per thread

__device__ __forceinline__ int2 bk_place(uint32_t at, uint32_t want, int64_t cap) {
  const int64_t b = min((int64_t)at, cap), e = min((int64_t)at + want, cap);
  return make_int2((int32_t)b, (int32_t)(e - b));
}

__global__ void __launch_bounds__(kScanThreads) k_scan(const TransferArgs a, int32_t n) {
  __shared__ int32_t wsum[kScanThreads / kWave];
  __shared__ uint32_t wsum2[kScanThreads / kWave];
  __shared__ int32_t chunk_base;
  __shared__ uint32_t chunk_base2;
  const int32_t* __restrict__ cnt = a.tile_count;
  int2* __restrict__ next = a.bk_list ? a.bk_lay + (int64_t)(a.bk_state[0] ^ 1) * n : nullptr;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int i0 = blockIdx.x * (kScanThreads * kScanPer) + tid;
  int32_t c[kScanPer];
  int32_t s = 0;
  uint32_t s2 = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int i = i0 + u * kScanThreads;
    c[u] = i < n ? cnt[i] : 0;
  }
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    s += c[u];
    s2 += i0 + u * kScanThreads < n ? bk_want(c[u]) : 0u;
  }
  // inclusive scans of the thread totals: within each wavefront, then across the wavefront totals
  int32_t incl = s;
  uint32_t incl2 = s2;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t v = __shfl_up(incl, o, kWave);
    const uint32_t v2 = __shfl_up(incl2, o, kWave);
    if (lane >= o) {
      incl += v;
      incl2 += v2;
    }
  }
  if (lane == kWave - 1) {
    wsum[wave] = incl;
    wsum2[wave] = incl2;
  }
  __syncthreads();
  int32_t before = 0, total = 0;
  uint32_t before2 = 0, total2 = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    if (w < wave) {
      before += wsum[w];
      before2 += wsum2[w];
    }
    total += wsum[w];
    total2 += wsum2[w];
  }
  if (tid == 0) {
    const int32_t b0 = atomicAdd(a.place, total);
    chunk_base = b0;
    chunk_base2 = atomicAdd(reinterpret_cast<uint32_t*>(a.place + 1), total2);
    if ((int64_t)b0 + total > a.list_cap) atomicAdd(a.status + 3, 1ull);
  }
  __syncthreads();
  int32_t run = chunk_base + before + incl - s;
  uint32_t run2 = chunk_base2 + before2 + incl2 - s2;
  const int64_t bcap = a.bk_cap;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int i = i0 + u * kScanThreads;
    if (i < n) {
      a.tile_off[i] = run;
      a.tile_cursor[i] = run;
      if (next) next[i] = bk_place(run2, bk_want(c[u]), bcap);
      run += c[u];
      run2 += bk_want(c[u]);
    }
  }
}

// Four consecutive values to / from a 16-byte aligned address.
__device__ __forceinline__ void store4(float* p, const float v[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(double* p, const double v[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}
__device__ __forceinline__ void load4(const float* p, float v[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ __forceinline__ void load4(const double* p, double v[4]) {
  const double2 q0 = reinterpret_cast<const double2*>(p)[0], q1 = reinterpret_cast<const double2*>(p)[1];
  v[0] = q0.x;
  v[1] = q0.y;
  v[2] = q1.x;
  v[3] = q1.y;
}

// ------------------------------------------------------------------ tiled spread: accumulation
template <typename T>
struct FixedAcc;
template <>
struct FixedAcc<float> {
  static constexpr int kWords = 1;
};
template <>
struct FixedAcc<double> {
  static constexpr int kWords = 2;
};

constexpr int kTileThreads = 512;  // threads of a spread-tile workgroup (8 wavefronts)

// Tile accumulation: workgroup (tile, component) takes the nodes of its list
// and accumulates every contribution that lands inside the tile's x range
// into an LDS region covering the tile plus a one-cell halo along y and z
// (64-bit fixed point: exact, order-independent sums).  The region interior
// is written straight to the grid, the y/z halo rows to scratch for the merge;
// a tile with an empty list only writes zeros to its interior.
template <typename T>
__device__ __forceinline__ void spread_item(const TransferArgs& a, const T* __restrict__ x,
                                            const double* __restrict__ anchor, const T* __restrict__ F,
                                            T* __restrict__ grid, int w, unsigned char* smem_raw, int& bad_entry) {
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem_raw);
  constexpr int NW = FixedAcc<T>::kWords;
  const int tile = w / 3, d = w - 3 * tile;  // the 3 components of a tile are adjacent items
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int nwaves = nt / kWave;
  const int L = d * a.n_tiles + tile;
  const BoxDev B = a.boxes[a.tile_box[tile]];
  const int tl = tile - B.tile_base;
  const int tx = tl % B.ntile[0], ty = (tl / B.ntile[0]) % B.ntile[1], tz = tl / (B.ntile[0] * B.ntile[1]);
  const int c0[3] = {tx * a.tile[0], ty * a.tile[1], tz * a.tile[2]};
  int ex[3];
  for (int i = 0; i < 3; ++i) ex[i] = min(a.tile[i], B.n[i] - c0[i]);
  // region rows hold two pad cells, the ex_x cells of the tile and two more pad cells, so that the
  // three stencil columns of every entry (home or x-neighbour) are consecutive cells of a row; the
  // pads take the shares of columns outside the tile (an x-neighbour holds the node in its list too)
  // and are never written out, except where one tile spans the box along x: there columns -1 and
  // ex_x are the tile's own last and first columns, and the write-out adds them in (integer sums, so
  // the result does not depend on where a share was held).  An odd pitch of 64-bit words spreads the rows and planes of the
  // stencil over the LDS banks.
  const int rx = (ex[0] + 4) | 1, ry = ex[1] + 2, rz = ex[2] + 2, nreg = rx * ry * rz;
  const int cnt = a.tile_count[L];
  T* g = grid + d * a.total_cells + B.cell_off;
  T* halo = reinterpret_cast<T*>(a.halo) + (int64_t)L * a.halo_cells;
  const int64_t NN = a.n_nodes;
  const T* Fd = F + d * NN;
  if (cnt == 0) {  // nothing lands in this tile (uniform over the workgroup): zeros, no halo, no LDS
    const int rows = ex[1] * ex[2];
    constexpr int VW = 16 / (int)sizeof(T);  // values per 16-byte store
    if (ex[0] % VW == 0 && B.n[0] % VW == 0 && (reinterpret_cast<uintptr_t>(g) & 15) == 0) {
      // 16-byte stores: every row of the tile starts on a 16-byte boundary
      const int per_row = ex[0] / VW;
      for (int v = tid; v < rows * per_row; v += nt) {
        const int row = v / per_row, iz = row / ex[1], iy = row - iz * ex[1];
        const int ix = (v - row * per_row) * VW;
        T* cell = g + (uint32_t)(((c0[2] + iz) * B.n[1] + (c0[1] + iy)) * B.n[0] + c0[0] + ix);
        *reinterpret_cast<uint4*>(cell) = make_uint4(0u, 0u, 0u, 0u);
      }
    } else {
      const int lrow = lane >> a.tile_shift[0], ix = lane & (a.tile[0] - 1);
      const int rpw = kWave >> a.tile_shift[0];
      if (ix < ex[0])
        for (int row = wave * rpw + lrow; row < rows; row += nwaves * rpw) {
          const int iz = row / ex[1], iy = row - iz * ex[1];
          g[(uint32_t)(((c0[2] + iz) * B.n[1] + (c0[1] + iy)) * B.n[0] + c0[0] + ix)] = T(0);
        }
    }
    if (tid == 0) a.tile_flag[L] = 0;
    return;  // no barrier follows
  }

  // the carried layout holds the list when it fitted its room, else the fill pass's layout does
  const int32_t* list = a.bin_list + a.tile_off[L];
  if (a.bk_list) {
    const int2 lk = bk_layout(a)[L];
    if (cnt <= lk.y) list = a.bk_list + lk.x;
  }
  // fixed-point scale from the bound code of the list (raised by the count pass) and its length; a
  // non-finite force cannot be held in fixed point and poisons (NaN) the tile's whole region instead,
  // as does an entry whose MLS system has no solution (a non-finite position)
  const uint32_t code = a.tile_fmax[L];
  bool poison = code == kBoundPoison;
  // float64 keeps a 32-bit remainder word per cell after the 64-bit words (12 bytes per cell)
  unsigned int* lo = reinterpret_cast<unsigned int*>(acc + nreg);
  unsigned int* acc32 = reinterpret_cast<unsigned int*>(acc);
  {
    const int nw32 = (NW == 2 ? 3 : 2) * nreg;  // 32-bit words of the region, cleared 16 bytes at a time
    uint4* acc128 = reinterpret_cast<uint4*>(smem_raw);
    for (int i = tid; i < (nw32 >> 2); i += nt) acc128[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int i = (nw32 & ~3) + tid; i < nw32; i += nt) acc32[i] = 0u;
  }
  if (tid == 0) bad_entry = 0;
  __syncthreads();
  // every entry goes through the loop when the forces are finite, also when they are all zero, so
  // that an entry with a non-finite position is found
  const bool active = !poison;
  const bool nonzero = code > 0u && !poison;
  int sc = 0, sl = 0;
  if (active) {
    // |F| < 2^em; one contribution is at most 4 max|F| (sum of |phi| <= 4) < 2^(em + 2), a cell sum
    // at most cnt < 2^lc times that: keep every contribution below 2^50 and every sum below 2^62
    const int em = nonzero ? (int)code - kBoundBias : 0;
    const int lc = 32 - __builtin_clz((unsigned)cnt);  // 2^(lc - 1) <= cnt < 2^lc
    sc = min(48 - em, 60 - em - lc);
    // float64 remainder scale: |remainder| <= 1/2 unit, at most cnt of them per cell, so every
    // cell's sum stays below 2^29 in its 32-bit word
    sl = 30 - lc;
    const double lscale = ldexp(1.0, sl);
    // entry order: qi -> (qi * stride) mod cnt with a prime stride that does not divide cnt (a
    // permutation), so that the lanes of a wavefront take nodes far apart in the list, i.e. far apart
    // on the surface, and rarely add to the same LDS cell in one instruction
    int stride = 1;
    if (cnt % 97) stride = 97;
    else if (cnt % 89) stride = 89;
    else if (cnt % 83) stride = 83;
    const int step = (int)(((int64_t)nt * stride) % cnt);
    int e = (int)(((int64_t)tid * stride) % cnt);
    for (int qi = tid; qi < cnt; qi += nt) {
      const int k = list[e];
      e += step;
      if (e >= cnt) e -= cnt;
      double pos[3], tau64[3];
      int32_t base[3];
      node_position(a, x, anchor, k, a.node_particle[k], pos);
      nearest_node(B, d, pos, base, tau64);
      // the nearest node's x relative to the tile, taken periodically: -1 (left neighbour's last
      // layer) .. ex_x (right neighbour's first layer)
      int dx = base[0] - c0[0];
      dx = dx < -1 ? dx + B.n[0] : (dx > ex[0] ? dx - B.n[0] : dx);
      if ((unsigned)(base[1] - c0[1]) >= (unsigned)ex[1] || (unsigned)(base[2] - c0[2]) >= (unsigned)ex[2] ||
          dx < -1 || dx > ex[0]) {
        atomicAdd(a.status + 3, 1ull);  // positions changed since binning: the node is skipped, not misplaced
        continue;
      }
      const T tau[3] = {(T)tau64[0], (T)tau64[1], (T)tau64[2]};
      T W[27], cf[4];
      if (!mls_weights<T>(tau, W, cf)) {  // no weights: the tile cannot hold this node's share
        atomicAdd(a.status + 2, 1ull);
        bad_entry = 1;
        continue;
      }
      const double fs = ldexp((double)Fd[k], sc);  // exact: |F| 2^sc < 2^48
      T phi[27];
      mls_phi<T>(W, cf, phi);
      // first cell of stencil row (my, mz) = 0: the region starts one cell before the tile in y and z
      // and two pad cells before it in x, so column x - 1 of the stencil sits at dx + 1
      const int r0 = ((base[2] - c0[2]) * ry + (base[1] - c0[1])) * rx + dx + 1;
#pragma unroll
      for (int mz = 0; mz < 3; ++mz) {
#pragma unroll
        for (int my = 0; my < 3; ++my) {
          unsigned long long* cell = acc + r0 + (mz * ry + my) * rx;
#pragma unroll
          for (int mx = 0; mx < 3; ++mx) {
            const double q = (double)phi[(mz * 3 + my) * 3 + mx] * fs;
            const double t = q + kRoundMagic;  // q rounded to an integer, held in the low mantissa bits
            const long long qh = __double_as_longlong(t) - __double_as_longlong(kRoundMagic);
            atomicAdd(cell + mx, (unsigned long long)qh);
            if (NW == 2) {  // t - magic is that integer as a double, exactly (no integer conversion)
              const long long ql = round_to_i64((q - (t - kRoundMagic)) * lscale);
              atomicAdd(lo + (cell - acc) + mx, (unsigned int)(int)ql);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  if (bad_entry) poison = true;  // uniform: read after the barrier
  // interior -> grid (final unless a neighbour's halo adds to it), y/z halo rows -> scratch (rows of
  // tile_x values).  Region row -> (iy, iz): (row + 1/2) / ry is at least 1/(2 ry) away from an
  // integer, far above the rounding of this small quotient, so the truncation is exact.
  const int nrows = ry * rz;
  const float inv_ry = frcp((float)ry);
  const bool halo_on = nonzero || poison;
  const bool wrap_x = B.ntile[0] == 1;
  const bool sums = nonzero && !poison;
  const T fillv = poison ? (T)__builtin_nan("") : T(0);
  const int pitch = a.tile[0];
  // the value of region cell r, column ixc of the tile (the pad columns wrap onto a tile that spans the
  // box along x; integer sums, so the result does not depend on where a share was held)
  auto cell_value = [&](int r, int ixc) -> T {
    if (!sums) return fillv;
    long long wi = (long long)acc[r];
    int li = NW == 2 ? (int)lo[r] : 0;
    if (wrap_x) {
      if (ixc == 0) {
        wi += (long long)acc[r + ex[0]];
        if (NW == 2) li += (int)lo[r + ex[0]];
      }
      if (ixc == ex[0] - 1) {
        wi += (long long)acc[r - ex[0]];
        if (NW == 2) li += (int)lo[r - ex[0]];
      }
    }
    double w = (double)wi;
    if (NW == 2) w += (double)li * ldexp(1.0, -sl);
    return (T)ldexp(w, -sc);
  };
  if ((ex[0] & 3) == 0 && a.tile_shift[0] >= 2) {
    // four consecutive cells per lane: one row decode per four values, 16-byte stores where aligned
    // (halo rows always are: their pitch and every halo block are multiples of four values)
    const int sh = a.tile_shift[0] - 2;
    const int lrow = lane >> sh, ix = (lane & ((1 << sh) - 1)) * 4;
    const int rpw = kWave >> sh;  // region rows per wavefront pass
    const bool g_vec = (reinterpret_cast<uintptr_t>(g) & 15) == 0 && (B.n[0] & 3) == 0;
    for (int row0 = wave * rpw; row0 < nrows; row0 += nwaves * rpw) {
      const int row = row0 + lrow;
      if (row >= nrows || ix >= ex[0]) continue;
      const int iz = (int)(((float)row + 0.5f) * inv_ry);
      const int iy = row - iz * ry;
      const int r = row * rx + ix + 2;
      T v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = cell_value(r + j, ix + j);
      if ((unsigned)(iy - 1) < (unsigned)ex[1] && (unsigned)(iz - 1) < (unsigned)ex[2]) {
        T* dst = g + (uint32_t)(((c0[2] + iz - 1) * B.n[1] + (c0[1] + iy - 1)) * B.n[0] + c0[0] + ix);
        if (g_vec)
          store4(dst, v);
        else
#pragma unroll
          for (int j = 0; j < 4; ++j) dst[j] = v[j];
      } else if (halo_on) {
        store4(halo + halo_row(iy, iz, ry, rz) * pitch + ix, v);
      }
    }
  } else {
    // one cell per lane: a wavefront takes 64 / tile_x region rows at a time
    const int lrow = lane >> a.tile_shift[0], ix = lane & (a.tile[0] - 1);
    const int rpw = kWave >> a.tile_shift[0];  // tiles are at most 64 cells wide
    for (int row0 = wave * rpw; row0 < nrows; row0 += nwaves * rpw) {
      const int row = row0 + lrow;
      if (row >= nrows || ix >= ex[0]) continue;
      const int iz = (int)(((float)row + 0.5f) * inv_ry);
      const int iy = row - iz * ry;
      const T v = cell_value(row * rx + ix + 2, ix);
      if ((unsigned)(iy - 1) < (unsigned)ex[1] && (unsigned)(iz - 1) < (unsigned)ex[2])
        g[(uint32_t)(((c0[2] + iz - 1) * B.n[1] + (c0[1] + iy - 1)) * B.n[0] + c0[0] + ix)] = v;
      else if (halo_on)
        halo[halo_row(iy, iz, ry, rz) * pitch + ix] = v;
    }
  }
  if (tid == 0) a.tile_flag[L] = halo_on ? 1 : 0;
}

// One workgroup per item (tile, component), the items of neighbouring tiles on one XCD.  Float64: at
// least four wavefronts per SIMD (at most 128 registers), so that two workgroups share a compute unit
// as their LDS regions allow (float32 needs no hint: 80 registers).
template <typename T>
__global__ void __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 1)))
k_spread_home(const TransferArgs a, const T* __restrict__ x,
                                                              const double* __restrict__ anchor,
                                                              const T* __restrict__ F, T* __restrict__ grid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int bad_entry;
  spread_item<T>(a, x, anchor, F, grid, xcd_remap(blockIdx.x, gridDim.x), smem_raw, bad_entry);
}

// Merge: every tile adds, to its y/z border rows, the halo rows that its 8
// neighbours in the y-z plane (periodic; possibly itself) accumulated for
// them, in a fixed order.  Tiles that are neighbours in y or z share their x
// range, so every row is a contiguous run of ex_x cells on both sides.
// One wavefront per (tile, component): most workgroups of a sparse grid only read their neighbours'
// flags, and small workgroups keep more of them in flight.
constexpr int kMergeThreads = 64;

template <typename T>
__global__ void __launch_bounds__(kMergeThreads) k_spread_merge(const TransferArgs a, T* __restrict__ grid) {
  __shared__ int nbL[9];
  __shared__ int nbflag[9];
  __shared__ int nbe[9][2];  // neighbour extents along y and z
  __shared__ int any;
  const int w = xcd_remap(blockIdx.x, gridDim.x), tile = w / 3, d = w - 3 * tile, tid = threadIdx.x;
  const BoxDev B = a.boxes[a.tile_box[tile]];
  const int tl = tile - B.tile_base;
  const int t[3] = {tl % B.ntile[0], (tl / B.ntile[0]) % B.ntile[1], tl / (B.ntile[0] * B.ntile[1])};
  if (tid == 0) any = 0;
  __syncthreads();
  if (tid < 9) {
    const int o[2] = {tid % 3 - 1, tid / 3 - 1};  // (oy, oz)
    int nb[2];
    for (int ax = 0; ax < 2; ++ax) {
      nb[ax] = t[ax + 1] + o[ax];
      if (nb[ax] < 0) nb[ax] += B.ntile[ax + 1];
      if (nb[ax] >= B.ntile[ax + 1]) nb[ax] -= B.ntile[ax + 1];
      nbe[tid][ax] = min(a.tile[ax + 1], B.n[ax + 1] - nb[ax] * a.tile[ax + 1]);
    }
    const int Ln = d * a.n_tiles + B.tile_base + (nb[1] * B.ntile[1] + nb[0]) * B.ntile[0] + t[0];
    nbL[tid] = Ln;
    const int f = tid == 4 ? 0 : a.tile_flag[Ln];  // 4 = the tile itself, already in the grid
    nbflag[tid] = f;
    if (f) atomicOr(&any, 1);
  }
  __syncthreads();
  if (!any) return;
  const int c0[3] = {t[0] * a.tile[0], t[1] * a.tile[1], t[2] * a.tile[2]};
  const int exx = min(a.tile[0], B.n[0] - c0[0]);
  const int ey = nbe[4][0], ez = nbe[4][1];
  T* g = grid + d * a.total_cells + B.cell_off;
  const T* halo = reinterpret_cast<const T*>(a.halo);
  // border rows: the z faces (all y), then the y faces without the z-face rows
  const int zf = ez > 1 ? 2 : 1, yf = ey > 1 ? 2 : 1, inz = max(ez - 2, 0);
  const int nzr = zf * ey, nrows = nzr + yf * inz;
  // lanes cover rows of the power-of-two tile width, VW consecutive cells each (four, with 16-byte
  // accesses, where the tile's extent and the grid rows allow; halo rows always do); lanes past the
  // tile's extent idle
  const bool vec = (exx & 3) == 0 && a.tile_shift[0] >= 2 && (B.n[0] & 3) == 0 &&
                   (reinterpret_cast<uintptr_t>(g) & 15) == 0;
  const int vsh = vec ? 2 : 0;
  const int sh = a.tile_shift[0] - vsh;  // lanes per row: tile_x >> vsh
  const int rpp = (1 << sh) >= (int)blockDim.x ? 1 : (int)blockDim.x >> sh;  // rows per workgroup pass
  const int ix = (tid & ((1 << sh) - 1)) << vsh, lrow = tid >> sh;
  if (ix >= exx || lrow >= rpp) return;  // no barrier follows
  for (int row = lrow; row < nrows; row += rpp) {
    int iy, iz;
    if (row < nzr) {
      const int f = row >= ey ? 1 : 0;
      iy = row - f * ey;
      iz = f ? ez - 1 : 0;
    } else {
      const int b = row - nzr, f = b >= inz ? 1 : 0;
      iz = 1 + b - f * inz;
      iy = f ? ey - 1 : 0;
    }
    const uint32_t cell = (uint32_t)(((c0[2] + iz) * B.n[1] + (c0[1] + iy)) * B.n[0] + c0[0] + ix);
    T v[4];
    if (vec)
      load4(g + cell, v);
    else
      v[0] = g[cell];
    for (int oz = -1; oz <= 1; ++oz) {
      if ((oz == -1 && iz != 0) || (oz == 1 && iz != ez - 1)) continue;
      for (int oy = -1; oy <= 1; ++oy) {
        if ((oy == -1 && iy != 0) || (oy == 1 && iy != ey - 1)) continue;
        const int nbi = (oz + 1) * 3 + (oy + 1);
        if (!nbflag[nbi]) continue;
        // region coordinates of this cell in the neighbour: -1 -> its last+1, +1 -> 0, 0 -> i + 1; a
        // shell row of the neighbour's region
        const int ry = oy == -1 ? nbe[nbi][0] + 1 : (oy == 1 ? 0 : iy + 1);
        const int rz = oz == -1 ? nbe[nbi][1] + 1 : (oz == 1 ? 0 : iz + 1);
        const int hr = halo_row(ry, rz, nbe[nbi][0] + 2, nbe[nbi][1] + 2);
        const T* hp = halo + (int64_t)nbL[nbi] * a.halo_cells + hr * a.tile[0] + ix;
        if (vec) {
          T h4[4];
          load4(hp, h4);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] += h4[j];
        } else {
          v[0] += hp[0];
        }
      }
    }
    if (vec)
      store4(g + cell, v);
    else
      g[cell] = v[0];
  }
}

// ------------------------------------------------------------------ host launchers
size_t spread_tile_lds_bytes(const PlanDev& P, int dtype) {
  return (size_t)P.targs.region_cells * (dtype == 0 ? 8 : 12);
}

hipError_t prepare_transfer_kernels(const PlanDev& P) {
  hipError_t e = hipFuncSetAttribute((const void*)k_spread_home<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)spread_tile_lds_bytes(P, 0));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_spread_home<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)spread_tile_lds_bytes(P, 1));
}

static inline dim3 node_grid(int n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

hipError_t launch_interp(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* grid, void* v,
                         int block, hipStream_t st) {
  if (P.n_nodes == 0) return hipSuccess;
  P.timer->begin(K_INTERP, st);
  if (dtype == 0)
    hipLaunchKernelGGL(k_interp<float>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs, (const float*)x,
                       anchor, (const float*)grid, (float*)v);
  else
    hipLaunchKernelGGL(k_interp<double>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs, (const double*)x,
                       anchor, (const double*)grid, (double*)v);
  P.timer->end(st);
  return hipGetLastError();
}

hipError_t launch_spread_atomic(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* F,
                                void* grid, int block, hipStream_t st) {
  hipError_t e;
  P.timer->begin(K_FILL, st);
  if (dtype == 0)
    e = fill((float*)grid, 3 * P.total_cells, 0.0f, st);
  else
    e = fill((double*)grid, 3 * P.total_cells, 0.0, st);
  P.timer->end(st);
  if (e != hipSuccess || P.n_nodes == 0) return e;
  P.timer->begin(K_SPREAD_ATOMIC, st);
  if (dtype == 0)
    hipLaunchKernelGGL(k_spread_atomic<float>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs,
                       (const float*)x, anchor, (const float*)F, (float*)grid);
  else
    hipLaunchKernelGGL(k_spread_atomic<double>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs,
                       (const double*)x, anchor, (const double*)F, (double*)grid);
  P.timer->end(st);
  return hipGetLastError();
}

hipError_t launch_spread_tiled(const PlanDev& P, const TransferArgs& a, int dtype, const void* x, const double* anchor,
                               const void* F, void* grid, hipStream_t st) {
  const int nl = 3 * a.n_tiles;
  P.timer->begin(K_FILL, st);
  if (nl > 0)
    hipLaunchKernelGGL(k_zero_counters, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, a.tile_count,
                       a.tile_fmax, nl, a.place, a.bk_list ? a.bk_state : nullptr);
  P.timer->end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 ng = node_grid(a.n_nodes, 256), nb(256);
  if (a.n_nodes) {
    P.timer->begin(K_BIN_COUNT, st);
    if (dtype == 0)
      hipLaunchKernelGGL(k_bin_count<float>, ng, nb, 0, st, a, (const float*)x, anchor, (const float*)F);
    else
      hipLaunchKernelGGL(k_bin_count<double>, ng, nb, 0, st, a, (const double*)x, anchor, (const double*)F);
    P.timer->end(st);
  }
  P.timer->begin(K_SCAN, st);
  if (nl > 0)
    hipLaunchKernelGGL(k_scan, dim3((unsigned)((nl + kScanThreads * kScanPer - 1) / (kScanThreads * kScanPer))),
                       dim3(kScanThreads), 0, st, a, nl);
  P.timer->end(st);
  if (a.n_nodes) {
    P.timer->begin(K_BIN_FILL, st);
    if (dtype == 0)
      hipLaunchKernelGGL(k_bin_fill<float>, ng, nb, 0, st, a, (const float*)x, anchor);
    else
      hipLaunchKernelGGL(k_bin_fill<double>, ng, nb, 0, st, a, (const double*)x, anchor);
    P.timer->end(st);
  }
  const dim3 g((unsigned)(3 * a.n_tiles));  // (tile, component) pairs, components fastest
  P.timer->begin(K_SPREAD_HOME, st);
  if (dtype == 0)
    hipLaunchKernelGGL(k_spread_home<float>, g, dim3(kTileThreads), spread_tile_lds_bytes(P, 0), st, a,
                       (const float*)x, anchor, (const float*)F, (float*)grid);
  else
    hipLaunchKernelGGL(k_spread_home<double>, g, dim3(kTileThreads), spread_tile_lds_bytes(P, 1), st, a,
                       (const double*)x, anchor, (const double*)F, (double*)grid);
  P.timer->end(st);
  P.timer->begin(K_SPREAD_MERGE, st);
  if (dtype == 0)
    hipLaunchKernelGGL(k_spread_merge<float>, g, dim3(kMergeThreads), 0, st, a, (float*)grid);
  else
    hipLaunchKernelGGL(k_spread_merge<double>, g, dim3(kMergeThreads), 0, st, a, (double*)grid);
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
