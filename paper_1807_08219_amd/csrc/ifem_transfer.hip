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
//                       of the tile holding its nearest lattice node;
//    k_scan             exclusive scan of the counts (single workgroup);
//    k_bin_fill<T>      writes every node into its lists;
//    k_spread_home<T>   one workgroup per (component, tile): accumulates all
//                       contributions of the tile's list in an LDS region
//                       (tile + one-cell halo) as 64-bit fixed-point
//                       integers (exact, order-independent sums; float64
//                       uses a two-word split); writes the interior to the
//                       grid and the halo shell to scratch;
//    k_spread_merge<T>  adds the neighbours' halo values to each tile's
//                       border cells in a fixed order.
#include <cfloat>
#include <climits>

#include "ifem_device.hpp"
#include "ifem_internal.hpp"

namespace ifem {

template <typename T>
__device__ __forceinline__ void node_position(const TransferArgs& a, const T* __restrict__ x,
                                              const double* __restrict__ anchor, int k, int p, double out[3]) {
  const int64_t N = a.n_nodes;
  if (sizeof(T) == 4) {
    out[0] = anchor[3 * p] + (double)x[k];
    out[1] = anchor[3 * p + 1] + (double)x[N + k];
    out[2] = anchor[3 * p + 2] + (double)x[2 * N + k];
  } else {
    out[0] = (double)x[k];
    out[1] = (double)x[N + k];
    out[2] = (double)x[2 * N + k];
  }
}

// ------------------------------------------------------------------ fills (graph-safe, no memset nodes)
template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
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
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_nodes) return;
  const int p = a.node_particle[k];
  const BoxDev B = a.boxes[a.particle_box[p]];
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
    const T* g = grid + d * a.total_cells + B.cell_off;  // cells of one box fit 32-bit offsets
    const bool seam = base[0] == 0 || base[0] == B.n[0] - 1;
    const int32_t x0 = seam ? 0 : base[0] - 1;
    int32_t ix[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) ix[m] = wrap1(base[0] + m - 1, B.n[0]);
    const int32_t nxy = B.n[0] * B.n[1];
    T s = 0;
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const int32_t zo = wrap1(base[2] + mz - 1, B.n[2]) * nxy;
      const T cz = c[0] + c[3] * (T(mz - 1) - tau[2]);
#pragma unroll
      for (int my = 0; my < 3; ++my) {
        const T* row = g + (uint32_t)(zo + wrap1(base[1] + my - 1, B.n[1]) * B.n[0]);
        T u[3];
        if (!seam) {
          const Row3<T> r3 = *reinterpret_cast<const Row3<T>*>(row + x0);
          u[0] = r3.v[0];
          u[1] = r3.v[1];
          u[2] = r3.v[2];
        } else {
          u[0] = row[ix[0]];
          u[1] = row[ix[1]];
          u[2] = row[ix[2]];
        }
        const T cyz = cz + c[2] * (T(my - 1) - tau[1]);
#pragma unroll
        for (int mx = 0; mx < 3; ++mx) {
          const T phi = W[(mz * 3 + my) * 3 + mx] * (cyz + c[1] * (T(mx - 1) - tau[0]));
          s += phi * u[mx];
        }
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
  const BoxDev B = a.boxes[a.particle_box[p]];
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
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const int64_t zo = (int64_t)wrap1(base[2] + mz - 1, B.n[2]) * B.n[1] * B.n[0];
      const T cz = c[0] + c[3] * (T(mz - 1) - tau[2]);
#pragma unroll
      for (int my = 0; my < 3; ++my) {
        const int64_t yo = zo + (int64_t)wrap1(base[1] + my - 1, B.n[1]) * B.n[0];
        const T cyz = cz + c[2] * (T(my - 1) - tau[1]);
#pragma unroll
        for (int mx = 0; mx < 3; ++mx) {
          const T phi = W[(mz * 3 + my) * 3 + mx] * (cyz + c[1] * (T(mx - 1) - tau[0]));
          atomicAdd(g + yo + wrap1(base[0] + mx - 1, B.n[0]), phi * f);
        }
      }
    }
  }
  if (bad) atomicAdd(a.status + 2, (unsigned long long)bad);
}

// ------------------------------------------------------------------ tiled spread: binning
// Every (node, component) belongs to exactly one list: the tile holding its
// nearest lattice node.  Count, scan and fill build the lists; the atomics
// on the list counters are aggregated per wavefront (one per distinct list
// among 64 consecutive nodes, which lie close together on one surface).
// Home list of a node for one component: the (component, tile) that holds
// its nearest lattice node.  The count and fill passes both call this, on the
// same inputs, so they agree bit for bit.
__device__ __forceinline__ int home_list(const TransferArgs& a, const BoxDev& B, int d, const double pos[3]) {
  int32_t base[3];
  double tau[3];
  nearest_node(B, d, pos, base, tau);
  const int tx = base[0] >> a.tile_shift[0], ty = base[1] >> a.tile_shift[1], tz = base[2] >> a.tile_shift[2];
  return d * a.n_tiles + B.tile_base + (tz * B.ntile[1] + ty) * B.ntile[0] + tx;
}

// Adds one entry per active lane (key >= 0) to counter[key] with one atomic
// per distinct key in the wavefront; returns each lane's slot (the counter's
// old value plus the lane's rank among the lanes with its key).  Every lane
// of the wavefront must call it.
__device__ __forceinline__ int wave_append(int32_t* __restrict__ counter, int key) {
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long todo = __ballot(key >= 0);
  int slot = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int kl = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long m = __ballot(key == kl) & todo;
    int b = 0;
    if (lane == leader) b = atomicAdd(counter + kl, (int)__popcll(m));
    b = __builtin_amdgcn_readlane(b, leader);
    if (key == kl) slot = b + (int)__popcll(m & ((1ull << lane) - 1ull));
    todo &= ~m;
  }
  return slot;
}

// Count pass: one thread per node; every (node, component) counts once in
// its home list.
template <typename T>
__global__ void __launch_bounds__(256) k_bin_count(const TransferArgs a, const T* __restrict__ x,
                                                   const double* __restrict__ anchor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int key[3] = {-1, -1, -1};
  if (k < a.n_nodes) {
    const int p = a.node_particle[k];
    const BoxDev& B = a.boxes[a.particle_box[p]];
    double pos[3];
    node_position(a, x, anchor, k, p, pos);
#pragma unroll
    for (int d = 0; d < 3; ++d) key[d] = home_list(a, B, d, pos);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) (void)wave_append(a.tile_count, key[d]);
}

// Fill pass: the same keys; each (node, component) takes a slot of its home
// list from the cursor (initialised to the list's offset by the scan).
template <typename T>
__global__ void __launch_bounds__(256) k_bin_fill(const TransferArgs a, const T* __restrict__ x,
                                                  const double* __restrict__ anchor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int key[3] = {-1, -1, -1};
  if (k < a.n_nodes) {
    const int p = a.node_particle[k];
    const BoxDev& B = a.boxes[a.particle_box[p]];
    double pos[3];
    node_position(a, x, anchor, k, p, pos);
#pragma unroll
    for (int d = 0; d < 3; ++d) key[d] = home_list(a, B, d, pos);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int slot = wave_append(a.tile_cursor, key[d]);
    if (key[d] >= 0 && slot < a.list_cap) a.bin_list[slot] = k;
  }
}

// Exclusive scan of tile_count into tile_off (n + 1 entries) with one
// workgroup; starts every cursor at its list's offset; flags a total above
// the list capacity (which holds exactly one entry per node and component).
__global__ void __launch_bounds__(1024) k_scan(int32_t n, const int32_t* __restrict__ cnt, int32_t* __restrict__ off,
                                               int32_t* __restrict__ cursor, int64_t cap,
                                               unsigned long long* status) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int chunk = (n + nt - 1) / nt;
  const int b = tid * chunk, e = min(n, b + chunk);
  int32_t s = 0;
  for (int i = b; i < e; ++i) s += cnt[i];
  part[tid] = s;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {  // Hillis-Steele inclusive scan of the per-thread sums
    const int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - s;
  for (int i = b; i < e; ++i) {
    off[i] = run;
    cursor[i] = run;
    run += cnt[i];
  }
  if (tid == nt - 1) {
    off[n] = part[nt - 1];
    if ((int64_t)part[nt - 1] > cap) atomicAdd(status + 3, 1ull);
  }
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

// Home-tile accumulation: workgroup (tile, component) takes the nodes of its
// list (nearest lattice node in the tile) and accumulates all 27 of their
// contributions into an LDS region covering the tile plus a one-cell halo
// (64-bit fixed point: exact, order-independent sums).  The region interior
// is written straight to the grid, the halo shell to scratch for the merge.
template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_spread_home(const TransferArgs a, const T* __restrict__ x,
                                                              const double* __restrict__ anchor,
                                                              const T* __restrict__ F, T* __restrict__ grid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double wm[16];
  __shared__ int wb[16];
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem_raw);
  constexpr int NW = FixedAcc<T>::kWords;
  const int tile = blockIdx.x, d = blockIdx.y;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int nwaves = nt / kWave;
  const int L = d * a.n_tiles + tile;
  const BoxDev B = a.boxes[a.tile_box[tile]];
  const int tl = tile - B.tile_base;
  const int tx = tl % B.ntile[0], ty = (tl / B.ntile[0]) % B.ntile[1], tz = tl / (B.ntile[0] * B.ntile[1]);
  const int c0[3] = {tx * a.tile[0], ty * a.tile[1], tz * a.tile[2]};
  int ex[3];
  for (int i = 0; i < 3; ++i) ex[i] = min(a.tile[i], B.n[i] - c0[i]);
  const int rx = ex[0] + 2, ry = ex[1] + 2, rz = ex[2] + 2, nreg = rx * ry * rz;
  const int32_t* list = a.bin_list + a.tile_off[L];
  const int cnt = a.tile_count[L];
  T* g = grid + d * a.total_cells + B.cell_off;
  T* halo = reinterpret_cast<T*>(a.halo) + (int64_t)L * a.region_cells;
  const int64_t NN = a.n_nodes;
  const T* Fd = F + d * NN;

  // fixed-point scale from the largest |F| of the list and its length; a non-finite force
  // cannot be held in fixed point and poisons (NaN) the tile's whole region instead
  double m = 0.0;
  bool bad = false;
  for (int e = tid; e < cnt; e += nt) {
    const double v = fabs((double)Fd[list[e]]);
    bad |= !(v <= DBL_MAX);
    m = fmax(m, v);
  }
  m = wave_max(m);
  const bool wbad = __ballot(bad) != 0ull;
  if (lane == 0) {
    wm[wave] = m;
    wb[wave] = wbad ? 1 : 0;
  }
  for (int i = tid; i < NW * nreg; i += nt) acc[i] = 0ull;
  __syncthreads();
  m = 0.0;
  bool poison = false;
  for (int w = 0; w < nwaves; ++w) {
    m = fmax(m, wm[w]);
    poison |= wb[w] != 0;
  }
  const bool active = cnt > 0 && m > 0.0 && !poison;
  int sc = 0;
  if (active) {
    // one contribution is at most 4 max|F| (sum of |phi| <= 4), a cell sum at most cnt times that:
    // keep every contribution below 2^50 and every sum below 2^62
    int e1, e2;
    frexp(4.0 * m, &e1);
    frexp(4.0 * (double)cnt * m, &e2);
    sc = min(50 - e1, 62 - e2);
    const double scale = ldexp(1.0, sc);
    for (int e = tid; e < cnt; e += nt) {
      const int k = list[e];
      double pos[3], tau64[3];
      int32_t base[3];
      node_position(a, x, anchor, k, a.node_particle[k], pos);
      nearest_node(B, d, pos, base, tau64);
      if ((unsigned)(base[0] - c0[0]) >= (unsigned)ex[0] || (unsigned)(base[1] - c0[1]) >= (unsigned)ex[1] ||
          (unsigned)(base[2] - c0[2]) >= (unsigned)ex[2]) {
        atomicAdd(a.status + 3, 1ull);  // positions changed since binning: the node is skipped, not misplaced
        continue;
      }
      const T tau[3] = {(T)tau64[0], (T)tau64[1], (T)tau64[2]};
      T W[27], cf[4];
      mls_weights<T>(tau, W, cf);
      const double fs = (double)Fd[k] * scale;
      // region cell of stencil node m: local base + m (the region starts one cell before the tile)
      const int r0 = ((base[2] - c0[2]) * ry + (base[1] - c0[1])) * rx + (base[0] - c0[0]);
#pragma unroll
      for (int mz = 0; mz < 3; ++mz) {
        const T vz = cf[0] + cf[3] * (T(mz - 1) - tau[2]);
#pragma unroll
        for (int my = 0; my < 3; ++my) {
          const T vyz = vz + cf[2] * (T(my - 1) - tau[1]);
          const int row = r0 + (mz * ry + my) * rx;
#pragma unroll
          for (int mx = 0; mx < 3; ++mx) {
            const T phi = W[(mz * 3 + my) * 3 + mx] * (vyz + cf[1] * (T(mx - 1) - tau[0]));
            const double q = (double)phi * fs;
            const long long qh = round_to_i64(q);
            atomicAdd(acc + row + mx, (unsigned long long)qh);
            if (NW == 2) {
              const long long ql = round_to_i64((q - (double)qh) * 0x1p40);
              atomicAdd(acc + nreg + row + mx, (unsigned long long)ql);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // interior -> grid (final unless a neighbour's halo adds to it), halo shell -> scratch.  Region
  // index r -> (ix, iy, iz) by float reciprocals: (r + 1/2) / d is at least 1/(2d) away from an
  // integer, far above the rounding of these small quotients, so the truncation is exact.
  const double inv = ldexp(1.0, -sc);
  const float inv_rxy = frcp((float)(rx * ry)), inv_rx = frcp((float)rx);
  for (int r = tid; r < nreg; r += nt) {
    const int iz = (int)(((float)r + 0.5f) * inv_rxy);
    const int rr = r - iz * rx * ry;
    const int iy = (int)(((float)rr + 0.5f) * inv_rx);
    const int ix = rr - iy * rx;
    T v = poison ? (T)__builtin_nan("") : T(0);
    if (active) {
      double w = (double)(long long)acc[r];
      if (NW == 2) w += (double)(long long)acc[nreg + r] * 0x1p-40;
      v = (T)(w * inv);
    }
    if (ix >= 1 && ix <= ex[0] && iy >= 1 && iy <= ex[1] && iz >= 1 && iz <= ex[2])
      g[(uint32_t)(((c0[2] + iz - 1) * B.n[1] + (c0[1] + iy - 1)) * B.n[0] + c0[0] + ix - 1)] = v;
    else if (active || poison)
      halo[r] = v;
  }
  if (tid == 0) a.tile_flag[L] = (active || poison) ? 1 : 0;
}

// Merge: every tile adds, to its border cells, the halo values that its 26
// neighbours (periodic; possibly itself) accumulated for them, in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_spread_merge(const TransferArgs a, T* __restrict__ grid) {
  __shared__ int nbL[27];
  __shared__ int nbflag[27];
  __shared__ int nbex[27][3];
  __shared__ int any;
  const int tile = blockIdx.x, d = blockIdx.y, tid = threadIdx.x;
  const BoxDev B = a.boxes[a.tile_box[tile]];
  const int tl = tile - B.tile_base;
  const int t[3] = {tl % B.ntile[0], (tl / B.ntile[0]) % B.ntile[1], tl / (B.ntile[0] * B.ntile[1])};
  if (tid == 0) any = 0;
  __syncthreads();
  if (tid < 27) {
    const int o[3] = {tid % 3 - 1, (tid / 3) % 3 - 1, tid / 9 - 1};
    int nb[3];
    for (int ax = 0; ax < 3; ++ax) {
      nb[ax] = t[ax] + o[ax];
      if (nb[ax] < 0) nb[ax] += B.ntile[ax];
      if (nb[ax] >= B.ntile[ax]) nb[ax] -= B.ntile[ax];
      nbex[tid][ax] = min(a.tile[ax], B.n[ax] - nb[ax] * a.tile[ax]);
    }
    const int Ln = d * a.n_tiles + B.tile_base + (nb[2] * B.ntile[1] + nb[1]) * B.ntile[0] + nb[0];
    nbL[tid] = Ln;
    const int f = tid == 13 ? 0 : a.tile_flag[Ln];  // 13 = the tile itself, already in the grid
    nbflag[tid] = f;
    if (f) atomicOr(&any, 1);
  }
  __syncthreads();
  if (!any) return;
  const int c0[3] = {t[0] * a.tile[0], t[1] * a.tile[1], t[2] * a.tile[2]};
  const int ex[3] = {nbex[13][0], nbex[13][1], nbex[13][2]};
  T* g = grid + d * a.total_cells + B.cell_off;
  const T* halo = reinterpret_cast<const T*>(a.halo);
  // border cells only: the two z faces, then the two y faces without z-face cells, then the two x
  // faces without y/z-face cells (each border cell exactly once, rows along x stay coalesced)
  const int inz = max(ex[2] - 2, 0), iny = max(ex[1] - 2, 0);
  const int zf = ex[2] > 1 ? 2 : 1, yf = ex[1] > 1 ? 2 : 1, xf = ex[0] > 1 ? 2 : 1;
  const int nzc = zf * ex[0] * ex[1], nyc = yf * ex[0] * inz, nxc = xf * iny * inz;
  const int total = nzc + nyc + nxc;
  for (int bi = tid; bi < total; bi += blockDim.x) {
    int i[3];
    if (bi < nzc) {
      const int f = bi / (ex[0] * ex[1]), r = bi - f * ex[0] * ex[1];
      i[0] = r % ex[0];
      i[1] = r / ex[0];
      i[2] = f ? ex[2] - 1 : 0;
    } else if (bi < nzc + nyc) {
      const int b = bi - nzc, f = b / (ex[0] * inz), r = b - f * ex[0] * inz;
      i[0] = r % ex[0];
      i[1] = f ? ex[1] - 1 : 0;
      i[2] = 1 + r / ex[0];
    } else {
      const int b = bi - nzc - nyc, f = b / (iny * inz), r = b - f * iny * inz;
      i[0] = f ? ex[0] - 1 : 0;
      i[1] = 1 + r % iny;
      i[2] = 1 + r / iny;
    }
    const uint32_t cell = (uint32_t)(((c0[2] + i[2]) * B.n[1] + (c0[1] + i[1])) * B.n[0] + c0[0] + i[0]);
    T v = g[cell];
    for (int oz = -1; oz <= 1; ++oz) {
      if ((oz == -1 && i[2] != 0) || (oz == 1 && i[2] != ex[2] - 1)) continue;
      for (int oy = -1; oy <= 1; ++oy) {
        if ((oy == -1 && i[1] != 0) || (oy == 1 && i[1] != ex[1] - 1)) continue;
        for (int ox = -1; ox <= 1; ++ox) {
          if ((ox == -1 && i[0] != 0) || (ox == 1 && i[0] != ex[0] - 1)) continue;
          const int nbi = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
          if (!nbflag[nbi]) continue;
          // region coordinates of this cell in the neighbour: -1 -> its last+1, +1 -> 0, 0 -> i + 1
          const int r[3] = {ox == -1 ? nbex[nbi][0] + 1 : (ox == 1 ? 0 : i[0] + 1),
                            oy == -1 ? nbex[nbi][1] + 1 : (oy == 1 ? 0 : i[1] + 1),
                            oz == -1 ? nbex[nbi][2] + 1 : (oz == 1 ? 0 : i[2] + 1)};
          const int rxn = nbex[nbi][0] + 2, ryn = nbex[nbi][1] + 2;
          v += halo[(int64_t)nbL[nbi] * a.region_cells + (r[2] * ryn + r[1]) * rxn + r[0]];
        }
      }
    }
    g[cell] = v;
  }
}

// ------------------------------------------------------------------ host launchers
size_t spread_tile_lds_bytes(const PlanDev& P, int dtype) {
  return (size_t)P.targs.region_cells * 8 * (dtype == 0 ? 1 : 2);
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

hipError_t launch_spread_tiled(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* F,
                               void* grid, int block, hipStream_t st) {
  (void)block;
  const TransferArgs& a = P.targs;
  const int nl = 3 * a.n_tiles;
  P.timer->begin(K_FILL, st);
  hipError_t e = fill(a.tile_count, (int64_t)nl, 0, st);
  P.timer->end(st);
  if (e != hipSuccess) return e;
  const dim3 ng = node_grid(a.n_nodes, 256), nb(256);
  if (a.n_nodes) {
    P.timer->begin(K_BIN_COUNT, st);
    if (dtype == 0)
      hipLaunchKernelGGL(k_bin_count<float>, ng, nb, 0, st, a, (const float*)x, anchor);
    else
      hipLaunchKernelGGL(k_bin_count<double>, ng, nb, 0, st, a, (const double*)x, anchor);
    P.timer->end(st);
  }
  P.timer->begin(K_SCAN, st);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, nl, a.tile_count, a.tile_off, a.tile_cursor, a.list_cap,
                     a.status);
  P.timer->end(st);
  if (a.n_nodes) {
    P.timer->begin(K_BIN_FILL, st);
    if (dtype == 0)
      hipLaunchKernelGGL(k_bin_fill<float>, ng, nb, 0, st, a, (const float*)x, anchor);
    else
      hipLaunchKernelGGL(k_bin_fill<double>, ng, nb, 0, st, a, (const double*)x, anchor);
    P.timer->end(st);
  }
  const dim3 g((unsigned)a.n_tiles, 3);
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
    hipLaunchKernelGGL(k_spread_merge<float>, g, dim3(256), 0, st, a, (float*)grid);
  else
    hipLaunchKernelGGL(k_spread_merge<double>, g, dim3(256), 0, st, a, (double*)grid);
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
