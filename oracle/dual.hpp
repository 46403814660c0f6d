// Forward-mode dual numbers for the FP64 oracle.
//
// TEST INFRASTRUCTURE ONLY: the oracle exists to check the HIP path; no
// product code may link or call it.
//
// Dual<P> carries a value and P directional derivatives.  The oracle seeds
// one direction per simulation parameter and per window start-state
// component, which yields the gradients the paper obtains by automatic
// differentiation (Sec. III-A) by an independent method (forward mode)
// from the HIP path's hand-written reverse mode.
#pragma once
#include <cmath>

template <int P>
struct Dual {
  double v;
  double d[P];
  Dual() : v(0.0) {
    for (int i = 0; i < P; ++i) d[i] = 0.0;
  }
  Dual(double x) : v(x) {  // NOLINT: implicit promotion of constants
    for (int i = 0; i < P; ++i) d[i] = 0.0;
  }
};

inline double val(double x) { return x; }
template <int P>
inline double val(const Dual<P>& x) { return x.v; }

template <int P>
inline Dual<P> operator+(const Dual<P>& a, const Dual<P>& b) {
  Dual<P> r;
  r.v = a.v + b.v;
  for (int i = 0; i < P; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int P>
inline Dual<P> operator-(const Dual<P>& a, const Dual<P>& b) {
  Dual<P> r;
  r.v = a.v - b.v;
  for (int i = 0; i < P; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int P>
inline Dual<P> operator-(const Dual<P>& a) {
  Dual<P> r;
  r.v = -a.v;
  for (int i = 0; i < P; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int P>
inline Dual<P> operator*(const Dual<P>& a, const Dual<P>& b) {
  Dual<P> r;
  r.v = a.v * b.v;
  for (int i = 0; i < P; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int P>
inline Dual<P> operator/(const Dual<P>& a, const Dual<P>& b) {
  Dual<P> r;
  r.v = a.v / b.v;
  for (int i = 0; i < P; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
// mixed double/dual forms
template <int P> inline Dual<P> operator+(double a, const Dual<P>& b) { return Dual<P>(a) + b; }
template <int P> inline Dual<P> operator+(const Dual<P>& a, double b) { return a + Dual<P>(b); }
template <int P> inline Dual<P> operator-(double a, const Dual<P>& b) { return Dual<P>(a) - b; }
template <int P> inline Dual<P> operator-(const Dual<P>& a, double b) { return a - Dual<P>(b); }
template <int P> inline Dual<P> operator*(double a, const Dual<P>& b) {
  Dual<P> r;
  r.v = a * b.v;
  for (int i = 0; i < P; ++i) r.d[i] = a * b.d[i];
  return r;
}
template <int P> inline Dual<P> operator*(const Dual<P>& a, double b) { return b * a; }
template <int P> inline Dual<P> operator/(const Dual<P>& a, double b) { return a / Dual<P>(b); }
template <int P> inline Dual<P> operator/(double a, const Dual<P>& b) { return Dual<P>(a) / b; }

template <int P> inline Dual<P>& operator+=(Dual<P>& a, const Dual<P>& b) { a = a + b; return a; }
template <int P> inline Dual<P>& operator-=(Dual<P>& a, const Dual<P>& b) { a = a - b; return a; }
template <int P> inline Dual<P>& operator*=(Dual<P>& a, const Dual<P>& b) { a = a * b; return a; }
template <int P> inline Dual<P>& operator+=(Dual<P>& a, double b) { a.v += b; return a; }

template <int P>
inline Dual<P> sin(const Dual<P>& a) {
  Dual<P> r;
  r.v = std::sin(a.v);
  const double c = std::cos(a.v);
  for (int i = 0; i < P; ++i) r.d[i] = c * a.d[i];
  return r;
}
template <int P>
inline Dual<P> cos(const Dual<P>& a) {
  Dual<P> r;
  r.v = std::cos(a.v);
  const double s = -std::sin(a.v);
  for (int i = 0; i < P; ++i) r.d[i] = s * a.d[i];
  return r;
}
template <int P>
inline Dual<P> sqrt(const Dual<P>& a) {
  Dual<P> r;
  r.v = std::sqrt(a.v);
  for (int i = 0; i < P; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r;
}
template <int P>
inline Dual<P> exp(const Dual<P>& a) {
  Dual<P> r;
  r.v = std::exp(a.v);
  for (int i = 0; i < P; ++i) r.d[i] = r.v * a.d[i];
  return r;
}
template <int P>
inline Dual<P> log(const Dual<P>& a) {
  Dual<P> r;
  r.v = std::log(a.v);
  for (int i = 0; i < P; ++i) r.d[i] = a.d[i] / a.v;
  return r;
}
