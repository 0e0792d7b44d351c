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
//    k_bin_count        counts, per (component, lattice tile), the nodes whose
//                       stencil touches the tile;
//    k_scan             exclusive scan of the counts (single workgroup);
//    k_bin_fill         writes the node lists;
//    k_spread_tile<T>   one workgroup per (component, tile): accumulates the
//                       contributions of its node list in LDS as 64-bit
//                       fixed-point integers (exact, order-independent sums;
//                       float64 uses a two-word split), then writes every
//                       lattice value of the tile exactly once.
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
    const T* g = grid + d * a.total_cells + B.cell_off;
    int32_t ix[3], iy[3], iz[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      ix[m] = wrap1(base[0] + m - 1, B.n[0]);
      iy[m] = wrap1(base[1] + m - 1, B.n[1]) * B.n[0];
      iz[m] = wrap1(base[2] + m - 1, B.n[2]);
    }
    T s = 0;
#pragma unroll
    for (int mz = 0; mz < 3; ++mz) {
      const int64_t zo = (int64_t)iz[mz] * B.n[1] * B.n[0];
      const T cz = c[0] + c[3] * (T(mz - 1) - tau[2]);
#pragma unroll
      for (int my = 0; my < 3; ++my) {
        const T cyz = cz + c[2] * (T(my - 1) - tau[1]);
#pragma unroll
        for (int mx = 0; mx < 3; ++mx) {
          const T phi = W[(mz * 3 + my) * 3 + mx] * (cyz + c[1] * (T(mx - 1) - tau[0]));
          s += phi * g[zo + iy[my] + ix[mx]];
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
// Distinct tiles (per axis) holding the cells base-1, base, base+1 (wrapped).
__device__ __forceinline__ int axis_tiles(int32_t base, int32_t n, int32_t T, int32_t out[3]) {
  const int32_t t0 = wrap1(base - 1, n) / T, t1 = base / T, t2 = wrap1(base + 1, n) / T;
  int c = 0;
  out[c++] = t0;
  if (t1 != t0) out[c++] = t1;
  if (t2 != t0 && t2 != t1) out[c++] = t2;
  return c;
}

template <typename T, bool FILL>
__global__ void __launch_bounds__(256) k_bin(const TransferArgs a, const T* __restrict__ x,
                                             const double* __restrict__ anchor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_nodes) return;
  const int p = a.node_particle[k];
  const BoxDev B = a.boxes[a.particle_box[p]];
  double pos[3];
  node_position(a, x, anchor, k, p, pos);
  for (int d = 0; d < 3; ++d) {
    int32_t base[3];
    double tau[3];
    nearest_node(B, d, pos, base, tau);
    int32_t tx[3], ty[3], tz[3];
    const int nx = axis_tiles(base[0], B.n[0], a.tile[0], tx);
    const int ny = axis_tiles(base[1], B.n[1], a.tile[1], ty);
    const int nz = axis_tiles(base[2], B.n[2], a.tile[2], tz);
    for (int iz = 0; iz < nz; ++iz)
      for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
          const int tile = B.tile_base + (tz[iz] * B.ntile[1] + ty[iy]) * B.ntile[0] + tx[ix];
          const int L = d * a.n_tiles + tile;
          if (FILL) {
            const int slot = atomicAdd(a.tile_cursor + L, 1);
            a.tile_list[a.tile_off[L] + slot] = k;
          } else {
            atomicAdd(a.tile_count + L, 1);
          }
        }
  }
}

// Exclusive scan of tile_count into tile_off (n + 1 entries) with one workgroup; zeroes the cursors.
__global__ void __launch_bounds__(1024) k_scan(int32_t n, const int32_t* __restrict__ cnt, int32_t* __restrict__ off,
                                               int32_t* __restrict__ cursor) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int chunk = (n + nt - 1) / nt;
  const int b = tid * chunk, e = min(n, b + chunk);
  int32_t s = 0;
  for (int i = b; i < e; ++i) s += cnt[i];
  part[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the per-thread sums
  for (int o = 1; o < nt; o <<= 1) {
    const int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - s;
  for (int i = b; i < e; ++i) {
    off[i] = run;
    run += cnt[i];
    cursor[i] = 0;
  }
  if (tid == nt - 1) off[n] = part[nt - 1];
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

template <typename T>
__global__ void __launch_bounds__(256) k_spread_tile(const TransferArgs a, const T* __restrict__ x,
                                                     const double* __restrict__ anchor, const T* __restrict__ F,
                                                     T* __restrict__ grid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double wmax[16];
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem_raw);
  constexpr int NW = FixedAcc<T>::kWords;
  const int tile = blockIdx.x, d = blockIdx.y;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int L = d * a.n_tiles + tile;
  const BoxDev B = a.boxes[a.tile_box[tile]];
  const int tl = tile - B.tile_base;
  const int tx = tl % B.ntile[0], ty = (tl / B.ntile[0]) % B.ntile[1], tz = tl / (B.ntile[0] * B.ntile[1]);
  const int c0[3] = {tx * a.tile[0], ty * a.tile[1], tz * a.tile[2]};
  int ex[3];
  for (int i = 0; i < 3; ++i) ex[i] = min(a.tile[i], B.n[i] - c0[i]);
  const int ncell = ex[0] * ex[1] * ex[2];
  const int cnt = a.tile_count[L], off = a.tile_off[L];
  T* g = grid + d * a.total_cells + B.cell_off;
  const int64_t NN = a.n_nodes;

  // largest |F| over the list fixes the fixed-point scale (order independent)
  double m = 0.0;
  for (int i = tid; i < cnt; i += nt) m = fmax(m, fabs((double)F[d * NN + a.tile_list[off + i]]));
  m = wave_max(m);
  const int lane = tid & (kWave - 1), wave = tid / kWave, nw = (nt + kWave - 1) / kWave;
  if (lane == 0) wmax[wave] = m;
  for (int i = tid; i < NW * ncell; i += nt) acc[i] = 0ull;
  __syncthreads();
  m = 0.0;
  for (int w = 0; w < nw; ++w) m = fmax(m, wmax[w]);
  if (cnt > 0 && m > 0.0 && isfinite(m)) {
    // |sum| <= cnt * sum_m |phi_m| * max|F| <= 4 cnt max|F| <= 2^e  ->  scale 2^(62 - e)
    int e;
    frexp(4.0 * (double)cnt * m, &e);
    const double scale = ldexp(1.0, 62 - e);
    for (int i = tid; i < cnt; i += nt) {
      const int k = a.tile_list[off + i];
      const int p = a.node_particle[k];
      double pos[3];
      node_position(a, x, anchor, k, p, pos);
      int32_t base[3];
      double tau64[3];
      nearest_node(B, d, pos, base, tau64);
      const T tau[3] = {(T)tau64[0], (T)tau64[1], (T)tau64[2]};
      T W[27], c[4];
      mls_weights<T>(tau, W, c);
      const T f = F[d * NN + k];
#pragma unroll
      for (int mz = 0; mz < 3; ++mz) {
        const int cz = wrap1(base[2] + mz - 1, B.n[2]) - c0[2];
        if (cz < 0 || cz >= ex[2]) continue;
        const T vz = c[0] + c[3] * (T(mz - 1) - tau[2]);
#pragma unroll
        for (int my = 0; my < 3; ++my) {
          const int cy = wrap1(base[1] + my - 1, B.n[1]) - c0[1];
          if (cy < 0 || cy >= ex[1]) continue;
          const T vyz = vz + c[2] * (T(my - 1) - tau[1]);
#pragma unroll
          for (int mx = 0; mx < 3; ++mx) {
            const int cx = wrap1(base[0] + mx - 1, B.n[0]) - c0[0];
            if (cx < 0 || cx >= ex[0]) continue;
            const T phi = W[(mz * 3 + my) * 3 + mx] * (vyz + c[1] * (T(mx - 1) - tau[0]));
            const double q = (double)(phi * f) * scale;
            const int li = (cz * ex[1] + cy) * ex[0] + cx;
            const double qh = rint(q);
            atomicAdd(acc + li, (unsigned long long)(long long)qh);
            if (NW == 2) {
              const double ql = rint((q - qh) * 0x1p40);
              atomicAdd(acc + ncell + li, (unsigned long long)(long long)ql);
            }
          }
        }
      }
    }
    __syncthreads();
    const double inv = 1.0 / scale;
    for (int li = tid; li < ncell; li += nt) {
      const int cx = li % ex[0], cy = (li / ex[0]) % ex[1], cz = li / (ex[0] * ex[1]);
      double v = (double)(long long)acc[li];
      if (NW == 2) v += (double)(long long)acc[ncell + li] * 0x1p-40;
      g[((int64_t)(c0[2] + cz) * B.n[1] + (c0[1] + cy)) * B.n[0] + c0[0] + cx] = (T)(v * inv);
    }
  } else {
    for (int li = tid; li < ncell; li += nt) {
      const int cx = li % ex[0], cy = (li / ex[0]) % ex[1], cz = li / (ex[0] * ex[1]);
      g[((int64_t)(c0[2] + cz) * B.n[1] + (c0[1] + cy)) * B.n[0] + c0[0] + cx] = (T)0;
    }
  }
}

// ------------------------------------------------------------------ host launchers
size_t spread_tile_lds_bytes(const PlanDev& P, int dtype) {
  const size_t cells = (size_t)P.targs.tile[0] * P.targs.tile[1] * P.targs.tile[2];
  return cells * 8 * (dtype == 0 ? 1 : 2);
}

hipError_t prepare_transfer_kernels(const PlanDev& P) {
  hipError_t e = hipFuncSetAttribute((const void*)k_spread_tile<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)spread_tile_lds_bytes(P, 0));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_spread_tile<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)spread_tile_lds_bytes(P, 1));
}

static inline dim3 node_grid(int n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

hipError_t launch_interp(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* grid, void* v,
                         int block, hipStream_t st) {
  if (P.n_nodes == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_interp<float>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs, (const float*)x,
                       anchor, (const float*)grid, (float*)v);
  else
    hipLaunchKernelGGL(k_interp<double>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs, (const double*)x,
                       anchor, (const double*)grid, (double*)v);
  return hipGetLastError();
}

hipError_t launch_spread_atomic(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* F,
                                void* grid, int block, hipStream_t st) {
  hipError_t e;
  if (dtype == 0)
    e = fill((float*)grid, 3 * P.total_cells, 0.0f, st);
  else
    e = fill((double*)grid, 3 * P.total_cells, 0.0, st);
  if (e != hipSuccess || P.n_nodes == 0) return e;
  if (dtype == 0)
    hipLaunchKernelGGL(k_spread_atomic<float>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs,
                       (const float*)x, anchor, (const float*)F, (float*)grid);
  else
    hipLaunchKernelGGL(k_spread_atomic<double>, node_grid(P.n_nodes, block), dim3(block), 0, st, P.targs,
                       (const double*)x, anchor, (const double*)F, (double*)grid);
  return hipGetLastError();
}

hipError_t launch_spread_tiled(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* F,
                               void* grid, int block, hipStream_t st) {
  const TransferArgs& a = P.targs;
  const int nl = 3 * a.n_tiles;
  hipError_t e = fill(a.tile_count, (int64_t)nl, 0, st);
  if (e != hipSuccess) return e;
  if (P.n_nodes) {
    if (dtype == 0)
      hipLaunchKernelGGL((k_bin<float, false>), node_grid(P.n_nodes, block), dim3(block), 0, st, a, (const float*)x,
                         anchor);
    else
      hipLaunchKernelGGL((k_bin<double, false>), node_grid(P.n_nodes, block), dim3(block), 0, st, a,
                         (const double*)x, anchor);
  }
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, nl, a.tile_count, a.tile_off, a.tile_cursor);
  if (P.n_nodes) {
    if (dtype == 0)
      hipLaunchKernelGGL((k_bin<float, true>), node_grid(P.n_nodes, block), dim3(block), 0, st, a, (const float*)x,
                         anchor);
    else
      hipLaunchKernelGGL((k_bin<double, true>), node_grid(P.n_nodes, block), dim3(block), 0, st, a,
                         (const double*)x, anchor);
  }
  const dim3 g((unsigned)a.n_tiles, 3);
  if (dtype == 0)
    hipLaunchKernelGGL(k_spread_tile<float>, g, dim3(256), spread_tile_lds_bytes(P, 0), st, a, (const float*)x,
                       anchor, (const float*)F, (float*)grid);
  else
    hipLaunchKernelGGL(k_spread_tile<double>, g, dim3(256), spread_tile_lds_bytes(P, 1), st, a, (const double*)x,
                       anchor, (const double*)F, (double*)grid);
  return hipGetLastError();
}

}  // namespace ifem
