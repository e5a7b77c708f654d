// Forward-mode dual numbers carrying N directional derivatives.
//
// Used on the device for exact Jacobians: the metric derivatives of the
// geometry kernel (N = 2: d/dx1, d/dx2), the 4x4 Jacobian of the PMHD
// implicit residual (N = 4: d/du_g, d/du~^i), and the local Jacobians of the
// adjoint step.  Every operator propagates the chain rule; sqrt/exp/sin/cos
// use their analytic derivatives.
#pragma once
#include <hip/hip_runtime.h>

#define GR_HD __host__ __device__ __forceinline__

template <int N>
struct Dual {
  double v;
  double d[N];
  GR_HD Dual() : v(0.0) {
#pragma unroll
    for (int i = 0; i < N; i++) d[i] = 0.0;
  }
  GR_HD Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; i++) d[i] = 0.0;
  }
  GR_HD static Dual var(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

template <int N>
GR_HD Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
GR_HD Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
GR_HD Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = -a.d[i];
  return r;
}
template <int N>
GR_HD Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
GR_HD Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  const double inv = 1.0 / b.v;
  r.v = a.v * inv;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
  return r;
}
template <int N> GR_HD Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> GR_HD Dual<N> operator+(double b, const Dual<N>& a) { Dual<N> r = a; r.v += b; return r; }
template <int N> GR_HD Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> GR_HD Dual<N> operator-(double b, const Dual<N>& a) { return Dual<N>(b) - a; }
template <int N>
GR_HD Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r;
  r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> GR_HD Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> GR_HD Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> GR_HD Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

template <int N>
GR_HD Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r;
  r.v = ::sqrt(a.v);
  const double h = 0.5 / r.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * h;
  return r;
}
template <int N>
GR_HD Dual<N> log(const Dual<N>& a) {
  Dual<N> r;
  r.v = ::log(a.v);
  const double h = 1.0 / a.v;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * h;
  return r;
}
template <int N>
GR_HD Dual<N> exp(const Dual<N>& a) {
  Dual<N> r;
  r.v = ::exp(a.v);
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * r.v;
  return r;
}
template <int N>
GR_HD Dual<N> sin(const Dual<N>& a) {
  Dual<N> r;
  r.v = ::sin(a.v);
  const double c = ::cos(a.v);
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * c;
  return r;
}
template <int N>
GR_HD Dual<N> cos(const Dual<N>& a) {
  Dual<N> r;
  r.v = ::cos(a.v);
  const double s = -::sin(a.v);
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = a.d[i] * s;
  return r;
}

// Piecewise functions take the derivative of the branch the value selects
// (ties: the first argument), as the adjoint of a step differentiates the
// branch the forward step took.
template <int N>
GR_HD Dual<N> fabs(const Dual<N>& a) {
  return (a.v < 0.0) ? -a : a;
}
template <int N>
GR_HD Dual<N> fmax(const Dual<N>& a, const Dual<N>& b) {
  return (a.v >= b.v || b.v != b.v) ? a : b;
}
template <int N>
GR_HD Dual<N> fmin(const Dual<N>& a, const Dual<N>& b) {
  return (a.v <= b.v || b.v != b.v) ? a : b;
}
// One operand constant: the same selection, the constant's derivative zero.
template <int N>
GR_HD Dual<N> fmax(const Dual<N>& a, double b) {
  return (a.v >= b || b != b) ? a : Dual<N>(b);
}
template <int N>
GR_HD Dual<N> fmax(double a, const Dual<N>& b) {
  return (a >= b.v || b.v != b.v) ? Dual<N>(a) : b;
}
template <int N>
GR_HD Dual<N> fmin(const Dual<N>& a, double b) {
  return (a.v <= b || b != b) ? a : Dual<N>(b);
}
template <int N>
GR_HD Dual<N> fmin(double a, const Dual<N>& b) {
  return (a <= b.v || b.v != b.v) ? Dual<N>(a) : b;
}
// |a| with the sign of b
template <int N>
GR_HD Dual<N> copysign(const Dual<N>& a, const Dual<N>& b) {
  return (__builtin_signbit(a.v) != __builtin_signbit(b.v)) ? -a : a;
}
template <int N> GR_HD bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N> GR_HD bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N> GR_HD bool operator<=(const Dual<N>& a, const Dual<N>& b) { return a.v <= b.v; }
template <int N> GR_HD bool operator>=(const Dual<N>& a, const Dual<N>& b) { return a.v >= b.v; }

// value accessor usable for both double and Dual
GR_HD double val(double x) { return x; }
GR_HD float val(float x) { return x; }
template <int N> GR_HD double val(const Dual<N>& x) { return x.v; }
