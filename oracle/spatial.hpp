// 6D spatial vector algebra (Featherstone, "Rigid Body Dynamics
// Algorithms"), written out plainly with full 6x6 matrices for the FP64
// oracle.  The paper computes forward dynamics with the Articulated Body
// Algorithm (App. B-A, eq. "dynamics"); this file supplies the algebra the
// oracle's ABA, CRBA and RNEA are written in.
//
// TEST INFRASTRUCTURE ONLY (see oracle.cpp header).
//
// Conventions: a spatial motion vector is [angular; linear] with the linear
// part the velocity of the body-fixed point at the frame origin; a force
// vector is [moment about origin; force].  An Xform maps motion vectors from
// parent coordinates to child coordinates: E rotates parent coordinates into
// child coordinates and r is the child origin expressed in parent
// coordinates.
#pragma once
#include <cmath>

template <class S> struct V3 { S x[3]; };
template <class S> struct M3 { S a[3][3]; };
template <class S> struct SV { S a[6]; };
template <class S> struct M6 { S a[6][6]; };
template <class S> struct Xform { M3<S> E; V3<S> r; };

template <class S> inline V3<S> v3(S a, S b, S c) { V3<S> v; v.x[0] = a; v.x[1] = b; v.x[2] = c; return v; }
template <class S> inline V3<S> v3zero() { return v3<S>(S(0.0), S(0.0), S(0.0)); }
template <class S> inline V3<S> add(const V3<S>& a, const V3<S>& b) { return v3<S>(a.x[0] + b.x[0], a.x[1] + b.x[1], a.x[2] + b.x[2]); }
template <class S> inline V3<S> sub(const V3<S>& a, const V3<S>& b) { return v3<S>(a.x[0] - b.x[0], a.x[1] - b.x[1], a.x[2] - b.x[2]); }
template <class S> inline V3<S> scale(const V3<S>& a, S s) { return v3<S>(a.x[0] * s, a.x[1] * s, a.x[2] * s); }
template <class S> inline V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.x[1] * b.x[2] - a.x[2] * b.x[1], a.x[2] * b.x[0] - a.x[0] * b.x[2], a.x[0] * b.x[1] - a.x[1] * b.x[0]);
}
template <class S> inline S dot(const V3<S>& a, const V3<S>& b) { return a.x[0] * b.x[0] + a.x[1] * b.x[1] + a.x[2] * b.x[2]; }

template <class S> inline M3<S> m3ident() {
  M3<S> m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = S(i == j ? 1.0 : 0.0);
  return m;
}
template <class S> inline M3<S> m3mul(const M3<S>& A, const M3<S>& B) {
  M3<S> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S s(0.0);
      for (int k = 0; k < 3; ++k) s = s + A.a[i][k] * B.a[k][j];
      C.a[i][j] = s;
    }
  return C;
}
template <class S> inline M3<S> m3T(const M3<S>& A) {
  M3<S> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[j][i];
  return C;
}
template <class S> inline V3<S> m3v(const M3<S>& A, const V3<S>& v) {
  V3<S> r;
  for (int i = 0; i < 3; ++i) r.x[i] = A.a[i][0] * v.x[0] + A.a[i][1] * v.x[1] + A.a[i][2] * v.x[2];
  return r;
}
// skew(c) * v == cross(c, v)
template <class S> inline M3<S> skew(const V3<S>& c) {
  M3<S> m;
  m.a[0][0] = S(0.0);  m.a[0][1] = -c.x[2]; m.a[0][2] = c.x[1];
  m.a[1][0] = c.x[2];  m.a[1][1] = S(0.0);  m.a[1][2] = -c.x[0];
  m.a[2][0] = -c.x[1]; m.a[2][1] = c.x[0];  m.a[2][2] = S(0.0);
  return m;
}

// Active rotation by angle q about unit axis n (Rodrigues).  The coordinate
// transform from the parent frame into a frame rotated this way is its
// transpose.
template <class S> inline M3<S> rodrigues(const double n[3], const S& q) {
  using std::cos; using std::sin;
  const S c = cos(q), s = sin(q);
  const S t = S(1.0) - c;
  M3<S> R;
  R.a[0][0] = c + t * (n[0] * n[0]);
  R.a[0][1] = t * (n[0] * n[1]) - s * n[2];
  R.a[0][2] = t * (n[0] * n[2]) + s * n[1];
  R.a[1][0] = t * (n[1] * n[0]) + s * n[2];
  R.a[1][1] = c + t * (n[1] * n[1]);
  R.a[1][2] = t * (n[1] * n[2]) - s * n[0];
  R.a[2][0] = t * (n[2] * n[0]) - s * n[1];
  R.a[2][1] = t * (n[2] * n[1]) + s * n[0];
  R.a[2][2] = c + t * (n[2] * n[2]);
  return R;
}

template <class S> inline SV<S> svzero() { SV<S> v; for (int i = 0; i < 6; ++i) v.a[i] = S(0.0); return v; }
template <class S> inline SV<S> svadd(const SV<S>& a, const SV<S>& b) { SV<S> r; for (int i = 0; i < 6; ++i) r.a[i] = a.a[i] + b.a[i]; return r; }
template <class S> inline SV<S> svsub(const SV<S>& a, const SV<S>& b) { SV<S> r; for (int i = 0; i < 6; ++i) r.a[i] = a.a[i] - b.a[i]; return r; }
template <class S> inline SV<S> svscale(const SV<S>& a, const S& s) { SV<S> r; for (int i = 0; i < 6; ++i) r.a[i] = a.a[i] * s; return r; }
template <class S> inline S svdot(const SV<S>& a, const SV<S>& b) { S s(0.0); for (int i = 0; i < 6; ++i) s = s + a.a[i] * b.a[i]; return s; }
template <class S> inline V3<S> ang(const SV<S>& v) { return v3<S>(v.a[0], v.a[1], v.a[2]); }
template <class S> inline V3<S> lin(const SV<S>& v) { return v3<S>(v.a[3], v.a[4], v.a[5]); }
template <class S> inline SV<S> sv(const V3<S>& w, const V3<S>& l) {
  SV<S> r;
  for (int i = 0; i < 3; ++i) { r.a[i] = w.x[i]; r.a[3 + i] = l.x[i]; }
  return r;
}

template <class S> inline M6<S> m6zero() { M6<S> m; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) m.a[i][j] = S(0.0); return m; }
template <class S> inline M6<S> m6add(const M6<S>& A, const M6<S>& B) { M6<S> C; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C.a[i][j] = A.a[i][j] + B.a[i][j]; return C; }
template <class S> inline M6<S> m6sub(const M6<S>& A, const M6<S>& B) { M6<S> C; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C.a[i][j] = A.a[i][j] - B.a[i][j]; return C; }
template <class S> inline M6<S> m6mul(const M6<S>& A, const M6<S>& B) {
  M6<S> C;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      S s(0.0);
      for (int k = 0; k < 6; ++k) s = s + A.a[i][k] * B.a[k][j];
      C.a[i][j] = s;
    }
  return C;
}
template <class S> inline M6<S> m6T(const M6<S>& A) { M6<S> C; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C.a[i][j] = A.a[j][i]; return C; }
template <class S> inline SV<S> m6v(const M6<S>& A, const SV<S>& v) {
  SV<S> r;
  for (int i = 0; i < 6; ++i) {
    S s(0.0);
    for (int k = 0; k < 6; ++k) s = s + A.a[i][k] * v.a[k];
    r.a[i] = s;
  }
  return r;
}
template <class S> inline M6<S> outer(const SV<S>& a, const SV<S>& b) { M6<S> C; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C.a[i][j] = a.a[i] * b.a[j]; return C; }

// Plucker motion transform as a 6x6 matrix: [[E, 0], [-E skew(r), E]].
template <class S> inline M6<S> xmat(const Xform<S>& X) {
  M6<S> m = m6zero<S>();
  const M3<S> Er = m3mul(X.E, skew(X.r));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      m.a[i][j] = X.E.a[i][j];
      m.a[3 + i][3 + j] = X.E.a[i][j];
      m.a[3 + i][j] = -Er.a[i][j];
    }
  return m;
}
// Composition: first X1 (a -> b), then X2 (b -> c).
template <class S> inline Xform<S> xcompose(const Xform<S>& X2, const Xform<S>& X1) {
  Xform<S> X;
  X.E = m3mul(X2.E, X1.E);
  X.r = add(X1.r, m3v(m3T(X1.E), X2.r));
  return X;
}

// Spatial cross products: crm(v) m and crf(v) f.
template <class S> inline SV<S> crm(const SV<S>& v, const SV<S>& m) {
  const V3<S> w = ang(v), vo = lin(v), mw = ang(m), mv = lin(m);
  return sv(cross(w, mw), add(cross(w, mv), cross(vo, mw)));
}
template <class S> inline SV<S> crf(const SV<S>& v, const SV<S>& f) {
  const V3<S> w = ang(v), vo = lin(v), fn = ang(f), ff = lin(f);
  return sv(add(cross(w, fn), cross(vo, ff)), cross(w, ff));
}

// Rigid-body spatial inertia about the frame origin from mass m, centre of
// mass c and rotational inertia Ic about the centre of mass:
// [[Ic + m skew(c) skew(c)^T, m skew(c)], [m skew(c)^T, m 1]].
template <class S> inline M6<S> rbi(const S& m, const V3<S>& c, const M3<S>& Ic) {
  M6<S> I = m6zero<S>();
  const M3<S> C = skew(c);
  const M3<S> CCt = m3mul(C, m3T(C));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      I.a[i][j] = Ic.a[i][j] + m * CCt.a[i][j];
      I.a[i][3 + j] = m * C.a[i][j];
      I.a[3 + i][j] = m * C.a[j][i];
      I.a[3 + i][3 + j] = (i == j) ? m : S(0.0);
    }
  return I;
}
