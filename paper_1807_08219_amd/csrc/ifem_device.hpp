// Device-side building blocks shared by the force and transfer kernels.
//
// Compiled for gfx950 only.  Float-float helpers follow the error-free
// transformations of Knuth (TwoSum) and Dekker/Ogita-Rump-Oishi (TwoProduct
// with a fused multiply-add).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ifem {

constexpr int kWave = 64;

// ------------------------------------------------------------------ error-free transformations
// Every operation below must round on its own: with the default fp-contract
// the compiler would fuse the sum s + a*b of an inlined caller into one FMA,
// which breaks TwoSum's error term and leaves g - G with plain float error.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_diff(float a, float b, float& s, float& e) { two_sum(a, -b, s, e); }
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

// a.b of two 3-vectors given as (hi, lo) float pairs, returned as an
// unevaluated float-float sum (s, e) accurate to ~u^2 |a||b|.
__device__ __forceinline__ void dot3_ff(const float ah[3], const float al[3], const float bh[3], const float bl[3],
                                        float& s, float& e) {
#pragma clang fp contract(off)
  float p, ep, t, et;
  two_prod(ah[0], bh[0], s, e);
  two_prod(ah[1], bh[1], p, ep);
  two_sum(s, p, t, et);
  s = t;
  e += ep + et;
  two_prod(ah[2], bh[2], p, ep);
  two_sum(s, p, t, et);
  s = t;
  e += ep + et;
  // first-order terms of the low parts
  e += ah[0] * bl[0] + ah[1] * bl[1] + ah[2] * bl[2];
  e += al[0] * bh[0] + al[1] * bh[1] + al[2] * bh[2];
}

// (g_s + g_e) - G for a float64 reference value G: exact leading difference
// (Sterbenz) plus the low parts.
__device__ __forceinline__ float diff_ff(float gs, float ge, double G) {
#pragma clang fp contract(off)
  float Gh = (float)G;
  float Gl = (float)(G - (double)Gh);
  return (gs - Gh) + (ge - Gl);
}

// ------------------------------------------------------------------ reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, kWave));
  return v;
}

// Block-wide deterministic sum of NV doubles (shuffle tree per wave, then waves in order).
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double* lds /*[NV][16]*/) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0)
    for (int i = 0; i < NV; ++i) lds[i * 16 + wave] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[i * 16 + w];
      v[i] = s;
    }
  __syncthreads();
}

// Groups the active lanes (key >= 0) of a wavefront by key: every lane gets
// the lane of its group's leader and its rank in the group; the leader also
// gets the group size (0 elsewhere).  Ballots and lane reads only, no memory
// traffic, so the atomics that follow can all be in flight at once.  Every
// lane of the wavefront must call it.
__device__ __forceinline__ void wave_groups(int key, int& leader, int& rank, int& size) {
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long todo = __ballot(key >= 0);
  leader = lane;
  rank = 0;
  size = 0;
  while (todo) {
    const int l = __ffsll((long long)todo) - 1;
    const int kl = __builtin_amdgcn_readlane(key, l);
    const unsigned long long m = __ballot(key == kl) & todo;
    if (key == kl) {
      leader = l;
      rank = (int)__popcll(m & ((1ull << lane) - 1ull));
    }
    if (lane == l) size = (int)__popcll(m);
    todo &= ~m;
  }
}

// Largest of a value over the 64 lanes of a wavefront, returned to every lane:
// data-parallel-primitive moves instead of LDS permutes.  Within each row of
// 16 lanes: the quad swaps, then shifts by 4 and 8 (lanes shifted in from
// outside the row read 0, the identity of the maximum), which leave lane 15 of
// the row with the row's largest; then row 1 and 3 take lane 15 of the row
// before them and rows 2 and 3 take lane 31, which leaves lane 63 with the
// wavefront's largest, read back as a uniform value.  All lanes must be active.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));  // row_shr 4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));  // row_shr 8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast 15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast 31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// ------------------------------------------------------------------ fast elementary functions
// float32: the hardware square root and reciprocal (about 1 ulp); float64:
// the correctly rounded operations.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// float64 square root: the hardware estimate (relative error about 2^-29)
// refined by one Newton step to about 2^-56; exactly 0 at 0.
__device__ __forceinline__ double fsqrt(double x) {
  const double y = __builtin_amdgcn_sqrt(x);
  const double r = __builtin_amdgcn_rcp(y);
  const double s = __builtin_fma(0.5 * __builtin_fma(-y, y, x), r, y);
  return x > 0.0 ? s : y;
}
// float64 reciprocal: the hardware estimate refined by two Newton steps
// (e = 1 - x r, r += r e; each step squares the relative error).
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// ------------------------------------------------------------------ launch order
// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  xcd_remap turns the hardware workgroup id into a logical
// one such that every XCD runs one contiguous range of logical workgroups, so
// neighbouring work (nodes of one particle, the components of one tile) shares
// an L2.  It is a bijection on [0, n) for any n.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n / kXcds, r = n % kXcds, xcd = bid % kXcds;
  return xcd * q + (xcd < r ? xcd : r) + bid / kXcds;
}

// ------------------------------------------------------------------ MLS weights
// Linear moving-least-squares weights on one 27-node stencil, in lattice
// units (h = 1).  tau = t - base is the point's offset from its nearest node
// (each component in [-1/2, 1/2]); stencil node m in {-1,0,1}^3 sits at
// xi_m = m - tau from the point.  W_m = W(|xi_m| / sqrt 3) with the cubic
// spline W(r) = 2/3 - 4 r^2 + 4 r^3 (r <= 1/2), 4/3 (1 - r)^3 (1/2 < r <= 1).
//
// The weighted least-squares fit uses the linear basis p = (1, m) in the
// stencil's integer offsets: an affine change of the linear basis leaves phi
// unchanged, and in this basis every moment of the weights is a sum or a
// difference of weights (m_i, m_i m_j in {-1, 0, 1}), no products.  With
// A = sum_m W_m p_m p_m^T and the point at p = (1, tau), A c = (1, tau) gives
// phi_m = W_m (c0 + c1 m_x + c2 m_y + c3 m_z).
// phi does not change when every W_m is scaled by one factor (c scales by its
// inverse), so the weights are taken as 3/4 W: with R = |xi| and
// s0 = 1 - R / sqrt 3 the inner piece is 1/2 - R^2 s0 and the outer one s0^3,
// clamped at 0 past the support.  The two pieces agree to second order at
// R^2 = 3/4 (their difference is a positive multiple of (R - sqrt(3)/2)^3),
// so the right piece is always the smaller one.
// Output: the scaled W[27] (m_x fastest), c[4]; returns false if A is singular
// (or tau not finite).
template <typename T>
__device__ __forceinline__ bool mls_weights(const T tau[3], T W[27], T c[4]) {
  const T kInvSqrt3 = T(0.57735026918962576451);
  T qx[3], qy[3], qz[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T ax = T(i - 1) - tau[0], ay = T(i - 1) - tau[1], az = T(i - 1) - tau[2];
    qx[i] = ax * ax;
    qy[i] = ay * ay;
    qz[i] = az * az;
  }
  // plane sums (per m_z): sum w, sum w m_x, sum w m_x^2, sum w m_y, sum w m_y^2, sum w m_x m_y
  T PS[3], PD[3], PE[3], PY[3], PYY[3], PXY[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T RS[3], RD[3], RE[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T qyz = qy[j] + qz[k];
      T w[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        // |tau| <= 1/2 bounds q by the number of off-centre offsets: the centre node always takes the
        // inner piece (q <= 3/4), a corner the outer one (q >= 3/4), and only nodes with two or three
        // off-centre offsets can leave the support (q > 3); compile-time facts after unrolling
        const int noff = (i != 1) + (j != 1) + (k != 1);
        const T q = qx[i] + qyz;
        const T s0 = T(1) - fsqrt(q) * kInvSqrt3;
        const T inner = T(0.5) - q * s0;
        const T sc = noff >= 2 ? fmax(s0, T(0)) : s0;
        const T outer = (sc * sc) * sc;
        w[i] = noff == 0 ? inner : (noff == 3 ? outer : fmin(inner, outer));
        W[(k * 3 + j) * 3 + i] = w[i];
      }
      RE[j] = w[0] + w[2];
      RS[j] = RE[j] + w[1];
      RD[j] = w[2] - w[0];
    }
    PS[k] = RS[0] + RS[1] + RS[2];
    PD[k] = RD[0] + RD[1] + RD[2];
    PE[k] = RE[0] + RE[1] + RE[2];
    PY[k] = RS[2] - RS[0];
    PYY[k] = RS[0] + RS[2];
    PXY[k] = RD[2] - RD[0];
  }
  const T S0 = PS[0] + PS[1] + PS[2];
  const T Sx = PD[0] + PD[1] + PD[2], Sy = PY[0] + PY[1] + PY[2], Sz = PS[2] - PS[0];
  const T Sxx = PE[0] + PE[1] + PE[2], Syy = PYY[0] + PYY[1] + PYY[2], Szz = PS[0] + PS[2];
  const T Sxy = PXY[0] + PXY[1] + PXY[2], Sxz = PD[2] - PD[0], Syz = PY[2] - PY[0];
  // Schur complement on the 3x3 second-moment block Q with s = (Sx, Sy, Sz):
  // y = Q^-1 s, z = Q^-1 tau, c0 = (1 - s.z) / (S0 - s.y), (c1, c2, c3) = z - c0 y.
  const T a00 = Syy * Szz - Syz * Syz;
  const T a01 = Sxz * Syz - Sxy * Szz;
  const T a02 = Sxy * Syz - Sxz * Syy;
  const T a11 = Sxx * Szz - Sxz * Sxz;
  const T a12 = Sxy * Sxz - Sxx * Syz;
  const T a22 = Sxx * Syy - Sxy * Sxy;
  const T detQ = Sxx * a00 + Sxy * a01 + Sxz * a02;
  const T inv = frcp(detQ);
  const T y0 = (a00 * Sx + a01 * Sy + a02 * Sz) * inv;
  const T y1 = (a01 * Sx + a11 * Sy + a12 * Sz) * inv;
  const T y2 = (a02 * Sx + a12 * Sy + a22 * Sz) * inv;
  const T z0 = (a00 * tau[0] + a01 * tau[1] + a02 * tau[2]) * inv;
  const T z1 = (a01 * tau[0] + a11 * tau[1] + a12 * tau[2]) * inv;
  const T z2 = (a02 * tau[0] + a12 * tau[1] + a22 * tau[2]) * inv;
  const T schur = S0 - (Sx * y0 + Sy * y1 + Sz * y2);
  const bool ok = detQ > T(0) && schur > T(0);
  const T c0 = ok ? (T(1) - (Sx * z0 + Sy * z1 + Sz * z2)) * frcp(schur) : T(0);
  c[0] = c0;
  c[1] = ok ? z0 - c0 * y0 : T(0);
  c[2] = ok ? z1 - c0 * y1 : T(0);
  c[3] = ok ? z2 - c0 * y2 : T(0);
  return ok;
}

// phi_m = W_m (c0 + c1 m_x + c2 m_y + c3 m_z) for the 27 stencil nodes (m_x fastest).
template <typename T>
__device__ __forceinline__ void mls_phi(const T W[27], const T c[4], T phi[27]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T vz = k == 0 ? c[0] - c[3] : (k == 1 ? c[0] : c[0] + c[3]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T vyz = j == 0 ? vz - c[2] : (j == 1 ? vz : vz + c[2]);
      phi[(k * 3 + j) * 3 + 0] = W[(k * 3 + j) * 3 + 0] * (vyz - c[1]);
      phi[(k * 3 + j) * 3 + 1] = W[(k * 3 + j) * 3 + 1] * vyz;
      phi[(k * 3 + j) * 3 + 2] = W[(k * 3 + j) * 3 + 2] * (vyz + c[1]);
    }
  }
}

// Round a float64 value (|v| < 2^51) to the nearest integer (ties to even)
// and return it as int64, with one add and one integer subtract: adding
// 1.5 * 2^52 places the integer in the low mantissa bits.
constexpr double kRoundMagic = 6755399441055744.0;  // 1.5 * 2^52
__device__ __forceinline__ long long round_to_i64(double v) {
  return __double_as_longlong(v + kRoundMagic) - __double_as_longlong(kRoundMagic);
}

// ------------------------------------------------------------------ lattices
// Geometry of one periodic box on the device.
struct BoxDev {
  int32_t n[3];
  int32_t ntile[3];   // tiles per axis
  double h, inv_h;
  double origin[3];
  double inv_n[3];    // 1 / n per axis (wrapping)
  int64_t cell_off;   // first cell of this box in every component array
  int32_t tile_base;  // first tile of this box
  int32_t pad;
};

__device__ __forceinline__ double stagger(int comp, int axis) { return comp == axis ? 0.0 : 0.5; }

// Lattice coordinate t = fma(p - origin, 1/h, -s) and its nearest node
// f = floor(t + 1/2) (float64, bit-specified; the same rule everywhere).
__device__ __forceinline__ double lattice_coord(const BoxDev& B, int comp, int a, double p, double& f) {
  const double t = __builtin_fma(p - B.origin[a], B.inv_h, -stagger(comp, a));
  f = floor(t + 0.5);
  return t;
}

// Wrap an integral float64 index into [0, n) (exact for |f| < 2^52; a
// non-finite or huge coordinate maps to 0, so every index stays in range).
__device__ __forceinline__ int32_t wrap_index(const BoxDev& B, int a, double f) {
  if (!(fabs(f) < 4503599627370496.0)) f = 0.0;
  const double qn = floor(f * B.inv_n[a]);
  int32_t w = (int32_t)(f - qn * (double)B.n[a]);
  if (w >= B.n[a]) w -= B.n[a];
  if (w < 0) w += B.n[a];
  return w;
}

// Bit-specified nearest-node rule: t = fma(p - origin, 1/h, -s), base = floor(t + 1/2).
// Returns the wrapped base index per axis and tau = t - base (exact in float64).
__device__ __forceinline__ void nearest_node(const BoxDev& B, int comp, const double p[3], int32_t base[3],
                                             double tau[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f;
    const double t = lattice_coord(B, comp, a, p[a], f);
    tau[a] = t - f;
    base[a] = wrap_index(B, a, f);
  }
}

// The wrapped nearest nodes of one position for all three staggered components at once: per axis
// the lattice coordinates with stagger 0 (the component along that axis) and 1/2 (the other two),
// each by the rule of lattice_coord, so the bases equal those of nearest_node bit for bit.
// Component d's base along axis a is (a == d ? b0[a] : bh[a]).
__device__ __forceinline__ void nearest_bases(const BoxDev& B, const double p[3], int32_t b0[3], int32_t bh[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double dp = p[a] - B.origin[a];
    b0[a] = wrap_index(B, a, floor(__builtin_fma(dp, B.inv_h, -0.0) + 0.5));
    bh[a] = wrap_index(B, a, floor(__builtin_fma(dp, B.inv_h, -0.5) + 0.5));
  }
}

__device__ __forceinline__ int32_t wrap1(int32_t i, int32_t n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

}  // namespace ifem
