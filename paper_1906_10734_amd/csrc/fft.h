// In-register complex FFTs of compile-time length for the source-to-target step.
//
// Each thread transforms one line held entirely in registers. The transform is a recursive
// mixed-radix decimation-in-time Cooley-Tukey split (radix 4, 2 and 3, so lengths 8*N_g for
// N_g in {2, 3, 4, 6, 8} are covered); every index and twiddle is a template constant, so after
// inlining the line is straight-line code on VGPRs with twiddles as immediates.
//
// Convention: SIGN = -1 is the forward transform X_k = sum_j x_j exp(-2 pi i jk/N), SIGN = +1
// the unnormalised inverse.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "twiddle.h"

namespace hpm {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by SIGN * i
template <int SIGN, typename T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> a) {
  if constexpr (SIGN > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int fft_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : n;
}

// z <- DFT_R(z) with kernel exp(SIGN 2 pi i / R)
template <int R, int SIGN, typename T>
__device__ __forceinline__ void butterfly(cplx<T> (&z)[R]) {
  if constexpr (R == 2) {
    const cplx<T> a = z[0], b = z[1];
    z[0] = cadd(a, b);
    z[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const cplx<T> s02 = cadd(z[0], z[2]), d02 = csub(z[0], z[2]);
    const cplx<T> s13 = cadd(z[1], z[3]), d13 = cmul_i<SIGN>(csub(z[1], z[3]));
    z[0] = cadd(s02, s13);
    z[1] = cadd(d02, d13);
    z[2] = csub(s02, s13);
    z[3] = csub(d02, d13);
  } else if constexpr (R == 3) {
    constexpr T half = T(0.5);
    constexpr T s3 = T(0.86602540378443864676372317075293618);  // sqrt(3)/2
    const cplx<T> t1 = cadd(z[1], z[2]);
    const cplx<T> t2 = cscale(cmul_i<SIGN>(csub(z[1], z[2])), s3);
    const cplx<T> m = csub(z[0], cscale(t1, half));
    z[0] = cadd(z[0], t1);
    z[1] = cadd(m, t2);
    z[2] = csub(m, t2);
  } else {
    static_assert(R == 2 || R == 3 || R == 4, "unsupported radix");
  }
}

// Twiddle exp(SIGN 2 pi i E / N) applied to a; E = 0 is skipped at compile time.
template <int E, int N, int SIGN, typename T>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> a) {
  if constexpr (E % N == 0) {
    return a;
  } else {
    constexpr double c = cis_cos(E, N);
    constexpr double s = SIGN * cis_sin(E, N);
    return cmul(a, cplx<T>{T(c), T(s)});
  }
}

// out[0..N) = DFT_N of in[OFF + STR * t], t = 0..N-1.
template <int N, int SIGN, typename T>
struct Fft {
  template <int OFF, int STR, int NIN>
  static __device__ __forceinline__ void run(const cplx<T> (&in)[NIN], cplx<T> (&out)[N]) {
    if constexpr (N == 1) {
      out[0] = in[OFF];
    } else {
      constexpr int R = fft_radix(N);
      constexpr int S = N / R;
      cplx<T> sub[R][S];
      static_for<0, R>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        Fft<S, SIGN, T>::template run<OFF + a * STR, STR * R, NIN>(in, sub[a]);
      });
      static_for<0, S>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        cplx<T> z[R];
        static_for<0, R>([&](auto ac) {
          constexpr int a = decltype(ac)::value;
          z[a] = twiddle<a * k, N, SIGN>(sub[a][k]);
        });
        butterfly<R, SIGN>(z);
        static_for<0, R>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          out[k + q * S] = z[q];
        });
      });
    }
  }
};

template <int N, int SIGN, typename T>
__device__ __forceinline__ void fft(const cplx<T> (&in)[N], cplx<T> (&out)[N]) {
  Fft<N, SIGN, T>::template run<0, 1, N>(in, out);
}

}  // namespace hpm
