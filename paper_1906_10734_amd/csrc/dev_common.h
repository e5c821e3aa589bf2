// Device helpers shared by the HIP kernels: gridlet node geometry, 1-D Lagrange and Legendre
// bases, Morton keys, wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpm {

constexpr int kMaxLevels = 11;  // levels 0..10 (30-bit Morton keys)

// Gridlet node i of a gridlet of N_g points per axis widened by EXT nodes on each side (EXT = 1:
// the extended target gridlet, Sec. 2.5), in cell units centred on the cell:
// (i - EXT + 1/2)/N_g - 1/2 for i = 0 .. N_g + 2 EXT - 1.
template <int NG, int EXT = 0>
constexpr double node_xi(int i) { return (2.0 * (i - EXT) + 1.0 - NG) / (2.0 * NG); }

// 1 / prod_{m != i} (xi_i - xi_m): denominators of the Lagrange basis on those nodes.
template <int NG, int EXT = 0>
constexpr double lagrange_inv_den(int i) {
  double d = 1.0;
  for (int m = 0; m < NG + 2 * EXT; ++m)
    if (m != i) d *= (node_xi<NG, EXT>(i) - node_xi<NG, EXT>(m));
  return 1.0 / d;
}

// l_i(u) = prod_{m != i} (u - xi_m)/(xi_i - xi_m) for all i, via prefix and suffix products.
template <int NG, int EXT = 0, typename T>
__device__ __forceinline__ void lagrange_basis(T u, T (&l)[NG + 2 * EXT]) {
  constexpr int NP = NG + 2 * EXT;
  T pre[NP], suf[NP];
  pre[0] = T(1);
#pragma unroll
  for (int m = 1; m < NP; ++m) pre[m] = pre[m - 1] * (u - T(node_xi<NG, EXT>(m - 1)));
  suf[NP - 1] = T(1);
#pragma unroll
  for (int m = NP - 2; m >= 0; --m) suf[m] = suf[m + 1] * (u - T(node_xi<NG, EXT>(m + 1)));
#pragma unroll
  for (int i = 0; i < NP; ++i) l[i] = pre[i] * suf[i] * T(lagrange_inv_den<NG, EXT>(i));
}

// l_i(u) and l_i'(u), by carrying (value, derivative) through the product.
template <int NG, int EXT = 0, typename T>
__device__ __forceinline__ void lagrange_basis_d(T u, T (&l)[NG + 2 * EXT],
                                                 T (&dl)[NG + 2 * EXT]) {
  constexpr int NP = NG + 2 * EXT;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    T v = T(1), d = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      if (m == i) continue;
      const T f = u - T(node_xi<NG, EXT>(m));
      d = d * f + v;
      v = v * f;
    }
    l[i] = v * T(lagrange_inv_den<NG, EXT>(i));
    dl[i] = d * T(lagrange_inv_den<NG, EXT>(i));
  }
}

// Legendre polynomials P_0..P_{NG-1} at t (three-term recurrence).
template <int NG, typename T>
__device__ __forceinline__ void legendre(T t, T (&p)[NG]) {
  p[0] = T(1);
  if (NG > 1) p[1] = t;
#pragma unroll
  for (int k = 1; k + 1 < NG; ++k)
    p[k + 1] = (T(2 * k + 1) * t * p[k] - T(k) * p[k - 1]) * T(1.0 / (k + 1));
}

__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z, int bits) {
  uint32_t k = 0;
  for (int b = 0; b < bits; ++b) {
    k |= ((x >> b) & 1u) << (3 * b);
    k |= ((y >> b) & 1u) << (3 * b + 1);
    k |= ((z >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

__device__ __forceinline__ int coord_x(int c) { return c & 1023; }
__device__ __forceinline__ int coord_y(int c) { return (c >> 10) & 1023; }
__device__ __forceinline__ int coord_z(int c) { return (c >> 20) & 1023; }
__device__ __forceinline__ int pack_coord(int x, int y, int z) { return x | (y << 10) | (z << 20); }

// [first index with keys >= v0, first index with keys >= v1) within [lo, hi), v0 <= v1: the two
// bisections run in lockstep, so the loads of a step do not wait on each other
__device__ __forceinline__ void key_range_u32(const uint32_t* keys, int lo, int hi, uint32_t v0,
                                              uint32_t v1, int& b, int& e) {
  int l0 = lo, h0 = hi, l1 = lo, h1 = hi;
  while (l0 < h0 || l1 < h1) {
    const int m0 = (l0 + h0) >> 1, m1 = (l1 + h1) >> 1;
    const uint32_t k0 = l0 < h0 ? keys[m0] : 0u;
    const uint32_t k1 = l1 < h1 ? keys[m1] : 0u;
    if (l0 < h0) {
      if (k0 < v0) l0 = m0 + 1;
      else h0 = m0;
    }
    if (l1 < h1) {
      if (k1 < v1) l1 = m1 + 1;
      else h1 = m1;
    }
  }
  b = l0;
  e = l1;
}

// level of a global cell id from the per-level offsets (levels are contiguous in id space)
__device__ __forceinline__ int level_of(int gid, const int* off, int nlevels) {
  int l = 0;
  while (l + 1 < nlevels && gid >= off[l + 1]) ++l;
  return l;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Neumaier two-term accumulate: (s, c) += x
template <typename T>
__device__ __forceinline__ void neumaier_add(T& s, T& c, T x) {
  const T t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// Float-float arithmetic (a value as an unevaluated sum hi + lo of two floats, about 48 bits),
// from error-free transformations: Knuth's two-sum and the FMA two-product.
struct ff32 {
  float hi, lo;
};

__device__ __forceinline__ ff32 ff_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ ff32 ff_two_prod(float a, float b) {
  const float p = a * b;
  return {p, fmaf(a, b, -p)};
}

// renormalised sum of two float-float values
__device__ __forceinline__ ff32 ff_add(ff32 a, ff32 b) {
  const ff32 s = ff_two_sum(a.hi, b.hi);
  const float e = s.lo + (a.lo + b.lo);
  const float hi = s.hi + e;
  return {hi, e - (hi - s.hi)};
}

__device__ __forceinline__ ff32 ff_neg(ff32 a) { return {-a.hi, -a.lo}; }

// a float times a float-float value
__device__ __forceinline__ ff32 ff_mul(float a, ff32 b) {
  ff32 p = ff_two_prod(a, b.hi);
  p.lo = fmaf(a, b.lo, p.lo);
  const float hi = p.hi + p.lo;
  return {hi, p.lo - (hi - p.hi)};
}

// a float-float value divided by a positive integer d (< 2^24)
__device__ __forceinline__ ff32 ff_div(ff32 a, int d) {
  const float fd = float(d), inv = 1.0f / fd;
  const float q = a.hi * inv;
  const ff32 r = ff_add(a, ff_neg(ff_two_prod(q, fd)));  // a - q d
  const float q2 = r.hi * inv;
  const float hi = q + q2;
  return {hi, q2 - (hi - q)};
}

}  // namespace hpm
