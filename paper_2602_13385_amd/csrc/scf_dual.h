// Forward-mode dual numbers for the adjoint kernels.
//
// The reverse-mode step needs two directional derivatives of the hot-path
// quantities along per-particle cotangent directions mu_i:
//   - the Hessian-vector product of psi_SCF, i.e. the derivative of the
//     acceleration a(x_i + eps mu_i) at eps = 0, and
//   - gamma_t = sum_i mu_i . grad b_t(x_i), the derivative of the basis sums
//     of Eq. (sumanlm) along the same directions.
// Evaluating the forward kernels' arithmetic on Dual<T> = v + eps d gives
// both exactly (to rounding), with no hand-derived second derivatives of the
// Gegenbauer and Legendre recurrences.  EpsAcc<T> accumulates only the eps
// part of a product of duals (the coefficient sums of the gamma pass).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

namespace scf {

using ::fma;

template <typename T>
struct Dual {
  T v, d;
  Dual() = default;
  __host__ __device__ constexpr Dual(T a, T b) : v(a), d(b) {}
  template <typename U, typename = typename std::enable_if<std::is_arithmetic<U>::value>::type>
  __host__ __device__ constexpr Dual(U a) : v(T(a)), d(T(0)) {}
};

template <typename T>
struct EpsAcc {
  T d;
  EpsAcc() = default;
  template <typename U, typename = typename std::enable_if<std::is_arithmetic<U>::value>::type>
  __host__ __device__ constexpr EpsAcc(U a) : d(T(a)) {}
};

// scalar type of the tables a kernel reads, and accumulator type of its sums
template <typename R>
struct RealTraits {
  using scalar = R;
  using acc = R;
  static constexpr bool dual = false;
};
template <typename T>
struct RealTraits<Dual<T>> {
  using scalar = T;
  using acc = EpsAcc<T>;
  static constexpr bool dual = true;
};
template <typename R>
using scalar_t = typename RealTraits<R>::scalar;
template <typename R>
using acc_t = typename RealTraits<R>::acc;

template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return {a.v * b.v, fma(a.v, b.d, a.d * b.v)};
}
template <typename T>
__device__ __forceinline__ Dual<T> operator*(T a, Dual<T> b) { return {a * b.v, a * b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, T b) { return {a.v * b, a.d * b}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
  const T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <typename T>
__device__ __forceinline__ Dual<T>& operator*=(Dual<T>& a, Dual<T> b) { return a = a * b; }
template <typename T>
__device__ __forceinline__ Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { return a = a + b; }
template <typename T>
__device__ __forceinline__ bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <typename T>
__device__ __forceinline__ bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <typename T>
__device__ __forceinline__ bool operator==(Dual<T> a, Dual<T> b) { return a.v == b.v; }

template <typename T>
__device__ __forceinline__ Dual<T> fma(Dual<T> a, Dual<T> b, Dual<T> c) {
  return {fma(a.v, b.v, c.v), fma(a.v, b.d, fma(a.d, b.v, c.d))};
}
template <typename T>
__device__ __forceinline__ Dual<T> fma(T a, Dual<T> b, Dual<T> c) {
  return {fma(a, b.v, c.v), fma(a, b.d, c.d)};
}
template <typename T>
__device__ __forceinline__ Dual<T> fma(Dual<T> a, T b, Dual<T> c) {
  return {fma(a.v, b, c.v), fma(a.d, b, c.d)};
}
// eps part of a * b added to c
template <typename T>
__device__ __forceinline__ EpsAcc<T> fma(Dual<T> a, Dual<T> b, EpsAcc<T> c) {
  EpsAcc<T> r;
  r.d = fma(a.v, b.d, fma(a.d, b.v, c.d));
  return r;
}
template <typename T>
__device__ __forceinline__ EpsAcc<T>& operator+=(EpsAcc<T>& a, EpsAcc<T> b) {
  a.d += b.d;
  return a;
}

}  // namespace scf
