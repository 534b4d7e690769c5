// In-register small DFTs for the gfx950 kernels.
//
// dft<R, r, INV>(v) replaces v[0..R) by its R-point DFT (natural order in and
// out), y_m = sum_s v_s w_R^{+-s m}, w_R = exp(-2 pi i / R) (Sec. "1D problem";
// INV uses conj(w), the conjugate F_R of Alg. alg:butterfly-related-kernel).
// R = r^g is computed through g levels of radix-r butterflies with the
// constant inner twiddles w_R^{s2 m1} of the Cooley-Tukey split
// R = r x (R/r); every index is a compile-time constant after unrolling, so
// the arrays live in VGPRs and the final reordering is a register renaming.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "omega_const.h"

namespace pafc {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// a * (-i) and a * (+i)
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }
template <typename T>
__device__ __forceinline__ cx<T> mul_pi(cx<T> a) { return {-a.im, a.re}; }

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// base-r reversal of g digits
template <int r, int g>
constexpr int digrev(int m) {
  int p = 0;
  for (int k = 0; k < g; ++k) {
    p = p * r + m % r;
    m /= r;
  }
  return p;
}

// compile-time loop
template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// v * w_N^E (INV: v * conj(w_N^E)) with exact handling of the points where
// w is +-1, +-i or (+-1 +-i)/sqrt(2).
template <int N, int E, bool INV, typename T>
__device__ __forceinline__ cx<T> mulw(cx<T> v) {
  constexpr int e0 = ((E % N) + N) % N;
  constexpr int e = INV ? (N - e0) % N : e0;  // conj(w^e) = w^{-e}
  if constexpr (e == 0) {
    return v;
  } else if constexpr (2 * e == N) {
    return {-v.re, -v.im};
  } else if constexpr (4 * e == N) {
    return mul_mi(v);  // w^{N/4} = -i
  } else if constexpr (4 * e == 3 * N) {
    return mul_pi(v);  // w^{3N/4} = +i
  } else if constexpr ((8 * e) % N == 0) {
    // (+-1 +-i)/sqrt(2): two multiplies
    constexpr double c = Omega<N>::re[e];
    constexpr double s = Omega<N>::im[e];
    const T h = (T)(c < 0 ? -c : c);  // 1/sqrt(2)
    // v * (c + i s) with |c| = |s| = h
    T a = (c > 0 ? v.re : -v.re), b = (s > 0 ? v.im : -v.im);
    T p = (s > 0 ? v.re : -v.re), q = (c > 0 ? v.im : -v.im);
    return {h * (a - b), h * (p + q)};
  } else {
    constexpr double c = Omega<N>::re[e];
    constexpr double s = Omega<N>::im[e];
    return cmul(v, cx<T>{(T)c, (T)s});
  }
}

// ---------------------------------------------------------------- base DFTs

template <int r, bool INV, typename T>
struct Base;

template <bool INV, typename T>
struct Base<2, INV, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename T>
struct Base<3, INV, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    // y1,2 = a - (b+c)/2 -+ i (sqrt(3)/2)(b - c)   (forward; INV swaps)
    const T h = (T)0.8660254037844386;  // sqrt(3)/2
    cx<T> a = v[0], b = v[1], c = v[2];
    cx<T> s = cadd(b, c), d = csub(b, c);
    v[0] = cadd(a, s);
    cx<T> t = {a.re - (T)0.5 * s.re, a.im - (T)0.5 * s.im};
    cx<T> u = {h * d.re, h * d.im};
    cx<T> mu = INV ? mul_pi(u) : mul_mi(u);
    v[1] = cadd(t, mu);
    v[2] = csub(t, mu);
  }
};

template <bool INV, typename T>
struct Base<4, INV, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
    cx<T> t1 = cadd(a, c), t2 = csub(a, c), t3 = cadd(b, d), t4 = csub(b, d);
    cx<T> r4 = INV ? mul_pi(t4) : mul_mi(t4);
    v[0] = cadd(t1, t3);
    v[2] = csub(t1, t3);
    v[1] = cadd(t2, r4);
    v[3] = csub(t2, r4);
  }
};

template <bool INV, typename T>
struct Base<5, INV, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    const T c1 = (T)Omega<5>::re[1], c2 = (T)Omega<5>::re[2];
    const T s1 = (T)-Omega<5>::im[1], s2 = (T)-Omega<5>::im[2];  // sin 72, sin 144
    cx<T> x0 = v[0];
    cx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    cx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    v[0] = cadd(x0, cadd(t1, t2));
    cx<T> a1 = {x0.re + c1 * t1.re + c2 * t2.re, x0.im + c1 * t1.im + c2 * t2.im};
    cx<T> a2 = {x0.re + c2 * t1.re + c1 * t2.re, x0.im + c2 * t1.im + c1 * t2.im};
    cx<T> b1 = {s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im};
    cx<T> b2 = {s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im};
    cx<T> m1 = INV ? mul_pi(b1) : mul_mi(b1);
    cx<T> m2 = INV ? mul_pi(b2) : mul_mi(b2);
    v[1] = cadd(a1, m1);
    v[4] = csub(a1, m1);
    v[2] = cadd(a2, m2);
    v[3] = csub(a2, m2);
  }
};

// -------------------------------------------------------- composite DFT_R

template <int R, int r, bool INV, typename T>
struct Dft {
  static constexpr int M = R / r;
  __device__ __forceinline__ static void run(cx<T>* v) {
    // s = s1*M + s2, m = m1 + r*m2
    static_for<M>([&](auto s2c) {
      constexpr int s2 = decltype(s2c)::value;
      cx<T> t[r];
      static_for<r>([&](auto s1c) { t[s1c.value] = v[s1c.value * M + s2]; });
      Base<r, INV, T>::run(t);
      static_for<r>([&](auto m1c) {
        constexpr int m1 = decltype(m1c)::value;
        v[m1 * M + s2] = mulw<R, s2 * m1, INV>(t[m1]);
      });
    });
    static_for<r>([&](auto m1c) {
      constexpr int m1 = decltype(m1c)::value;
      Dft<M, r, INV, T>::run(v + m1 * M);
    });
    // frequency m1 + r*m2 sits at m1*M + m2: rename into natural order
    cx<T> o[R];
    static_for<r>([&](auto m1c) {
      static_for<M>([&](auto m2c) { o[m1c.value + r * m2c.value] = v[m1c.value * M + m2c.value]; });
    });
    static_for<R>([&](auto k) { v[k.value] = o[k.value]; });
  }
};

template <int r, bool INV, typename T>
struct Dft<r, r, INV, T> {
  __device__ __forceinline__ static void run(cx<T>* v) { Base<r, INV, T>::run(v); }
};

// radix-8 groups use the 2 x 4 split internally
template <bool INV, typename T>
struct Base<8, INV, T> {
  __device__ __forceinline__ static void run(cx<T>* v) { Dft<8, 2, INV, T>::run(v); }
};

}  // namespace pafc
