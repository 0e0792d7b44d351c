// Lagrangian update (Sec. III.A, last step): second-order Adams-Bashforth,
//   x^{n+1} = x^n + dt (3/2 v^n - 1/2 v^{n-1}),
// or the forward Euler step x^n + dt v^n when there is no previous velocity.
// Float64 arithmetic in the order written (no fused multiply-add), so the
// float64 path reproduces the formula's plain evaluation bit for bit; float32
// offsets and velocities are widened exactly and the result rounded once.
#include <algorithm>

#include "ifem_internal.hpp"

namespace ifem {

constexpr int kAdvanceBlock = 256;
constexpr int kAdvanceItems = 4;  // independent elements per thread and pass

template <typename T, bool AB2>
__device__ __forceinline__ T advance_one(T x, T v, T vp, double dt) {
#pragma clang fp contract(off)
  const double rate = AB2 ? 1.5 * (double)v - 0.5 * (double)vp : (double)v;
  return (T)((double)x + dt * rate);
}

// n = 3 n_nodes values (the [3][n_nodes] arrays are one flat range).  x_out
// may be x: every element is read before it is written, by the same thread.
template <typename T, bool AB2>
__global__ void __launch_bounds__(kAdvanceBlock) k_advance(int64_t n, const T* x, const T* __restrict__ v,
                                                           const T* __restrict__ vp, double dt, T* x_out) {
  const int64_t stride = (int64_t)gridDim.x * kAdvanceBlock * kAdvanceItems;
  for (int64_t i0 = (int64_t)blockIdx.x * kAdvanceBlock * kAdvanceItems + threadIdx.x; i0 < n; i0 += stride) {
    T xs[kAdvanceItems], vs[kAdvanceItems], ps[kAdvanceItems];
#pragma unroll
    for (int q = 0; q < kAdvanceItems; ++q) {
      const int64_t i = min(i0 + (int64_t)q * kAdvanceBlock, n - 1);
      xs[q] = x[i];
      vs[q] = v[i];
      ps[q] = AB2 ? vp[i] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kAdvanceItems; ++q) {
      const int64_t i = i0 + (int64_t)q * kAdvanceBlock;
      if (i < n) x_out[i] = advance_one<T, AB2>(xs[q], vs[q], ps[q], dt);
    }
  }
}

template <typename T>
static void launch_advance_t(int64_t n, const void* x, const void* v, const void* vp, double dt, void* x_out,
                             hipStream_t st) {
  const int64_t per_block = (int64_t)kAdvanceBlock * kAdvanceItems;
  const int blocks = (int)std::min<int64_t>((n + per_block - 1) / per_block, 1 << 20);
  if (vp)
    hipLaunchKernelGGL((k_advance<T, true>), dim3(blocks), dim3(kAdvanceBlock), 0, st, n, (const T*)x, (const T*)v,
                       (const T*)vp, dt, (T*)x_out);
  else
    hipLaunchKernelGGL((k_advance<T, false>), dim3(blocks), dim3(kAdvanceBlock), 0, st, n, (const T*)x,
                       (const T*)v, (const T*)nullptr, dt, (T*)x_out);
}

hipError_t launch_advance(const PlanDev& P, int dtype, const void* x, const void* v, const void* v_prev, double dt,
                          void* x_out, hipStream_t st) {
  const int64_t n = (int64_t)3 * P.n_nodes;
  if (n == 0) return hipSuccess;
  P.timer->begin(K_ADVANCE, st);
  if (dtype == 0)
    launch_advance_t<float>(n, x, v, v_prev, dt, x_out, st);
  else
    launch_advance_t<double>(n, x, v, v_prev, dt, x_out, st);
  P.timer->end(st);
  return hipGetLastError();
}

}  // namespace ifem
