// Spatial algebra, forward dynamics and the reverse step of the 7-joint arm
// with its box (App. B-A: the Articulated Body Algorithm and the
// semi-implicit Euler step; Sec. IV-C: the Panda arm carrying a box).
//
// Bodies 0..6 are the arm links: joint i turns about its local z axis after
// the modified-DH placement Rot_x(alpha_i) Trans_x(a_i) Trans_z(d_i).  Body
// 7 is the box on a hinge about the flange x axis, or the massless ring of
// a universal joint about that axis; body 8 is the box turning about the
// ring's y axis.  Joint i's frame is reached from its parent's by four
// elementary operations: a shift a_i along the parent's x, a rotation
// alpha_i about x, a shift d_i along the new z, the joint rotation q_i about
// the joint axis (bodies 7 and 8: no alpha and no a; body 8 no d either).
// Every transform below applies them one by one, so no 3x3 rotation matrix
// is ever formed: a rotation about a coordinate axis mixes two components
// (4 multiplies, 2 adds per 3-vector), a shift along an axis touches two.
//
// Articulated inertias are symmetric 6x6 matrices in blocks [[A, B], [B^T,
// C]] (A, C symmetric 3x3, B general).  Their congruence into the parent
// frame, X^T I X, is likewise done as two rotations about axes (R M R^T
// for the symmetric blocks in 23 flops, 36 for B) and two shifts along axes
// (A - B R - (B R)^T - R C R, B + R C with R = [r]x and r along one axis).
// For a table with the Panda arm's structure (ArmDh below) its right-angle
// twists become signed swaps and its zero offsets vanish at compile time.
//
// Reverse step.  With F(q, qd, qdd, theta) = ID(q, qd, qdd; theta) -
// tau(q, qd, t) = 0 defining qdd, the vector-Jacobian product of forward
// dynamics with seed qdd_bar is -(dF/dx)^T lambda, lambda = H^{-1} qdd_bar.
// lambda comes from an ABA solve that reuses the forward pass's U and D;
// dF/dx^T lambda is the reverse of recursive Newton-Euler inverse dynamics.
// Both adjoint channels of a window (observation and constraint) go
// through one call: the primal terms they share (body forces, transformed
// accelerations and velocities) are formed once.  The parents' velocities
// and accelerations seen through the joint transform are read off the
// child's own (X v_{i-1} = v_i - S qd_i, X a_{i-1} = a_i - v_i x S qd_i -
// S qdd_i), and the outward force adjoints are walked back inward through
// the inverse transforms, so the reverse sweep holds one body's terms at a
// time.
//
// Generic over the scalar type R: float on the device, double in host
// checks, a counting scalar for the algorithmic FLOPs.  No HIP headers.
#pragma once

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "sincos.h"

#define PDS_ALWAYS_INLINE inline __attribute__((always_inline))

namespace pds {

// How the box hangs from the flange: on a hinge about the flange x axis
// (8 bodies; theta = the in-plane positions of two point masses in the
// box; observes the hinge angle), or on a universal joint, a massless ring
// about the flange x axis and then the box about the ring's y axis (9
// bodies; theta = the box's inertia about its centre of mass (xx, yy, zz,
// xy, xz, yz), its centre of mass and the viscous friction of both axes;
// observes the box frame: its origin and the points 1 m along its x, y, z
// axes in world coordinates, 12 numbers), or on the universal joint with
// the box's inertia and the joints' friction known and theta the in-plane
// positions of two point masses on the box floor (observes the box frame).
enum ArmBox { kHinge = 0, kUJoint = 1, kUJointWeights = 2 };

// Kinematic structure of the arm's modified-DH table.  Generic: every twist
// is applied with its cosine and sine and every offset with its value.  The
// Panda arm's structure (the arm of Sec. IV-C): twists of 0, -90, 90, 90,
// -90, 90 and 90 degrees, and the offsets a_0, a_1, a_2, a_5 (along x) and
// d_1, d_3, d_5, d_6 (along z) zero; a right-angle twist is then a signed
// swap of two axes and a zero offset drops out, both at compile time, while
// every value in the table stays a run-time input.  The set-up picks the
// structure from the table itself.
enum ArmDh { kDhGeneric = 0, kDhPanda = 1 };
constexpr int kPandaTwist[7] = {0, -1, 1, 1, -1, 1, 1};  // twist / (pi/2)
constexpr bool kPandaA[7] = {false, false, false, true, true, false, true};
constexpr bool kPandaD[7] = {true, false, true, false, true, false, false};
template <int BOX>
struct ArmShape {
  static constexpr int NB = BOX == kHinge ? 8 : 9;    // bodies = joints
  static constexpr int DS = 2 * NB;                  // state (q, qd)
  static constexpr int M = BOX == kUJoint ? 11 : 4;  // parameters
  static constexpr int DX = BOX == kHinge ? 1 : 12;  // observed numbers per step
  static constexpr int BOXB = BOX == kHinge ? 7 : 8;  // the box's body
  static constexpr bool PM = BOX != kUJoint;         // point masses in the box (theta)
};
constexpr int kArmMaxBodies = 9;

// Per-job constants derived once per call from the caller's raw model
// description (see pds.h for the raw layout).  Each body's constants sit in
// one 128-byte record, so the kernels fetch a body's constants with a few
// wide scalar loads instead of one load per array.
struct ArmBody {
  float ca, sa;  // cos, sin of the DH twist alpha (arm joints)
  float ra, rd;  // DH shifts: a along the parent's x, d along the twisted z
  float m;       // link mass (hinge: body 7 the box alone; joint: body 8 the box)
  float c[3];    // centre of mass
  float Ic[6];   // inertia about the centre of mass: xx, xy, xz, yy, yz, zz
  float Ar[6];   // angular block of the body's spatial inertia, Ic + m (|c|^2 1 - c c^T)
  float kp, kd, qc, amp, om, ph;  // PD gains and the sinusoidal target (arm joints)
  float Id[3];   // the diagonal of Ic (xx, yy, zz), contiguous
  float pad[3];
};
static_assert(sizeof(ArmBody) == 128, "one 128-byte record per body");
struct ArmConst {
  ArmBody b[kArmMaxBodies];
  float g[3];
  float bh;                 // hinge damping (universal joint with weights: first axis)
  float b8;                 // universal joint with weights: damping of the second axis
  float pm_m, pm_z;         // point masses: mass each, height in the box frame
  int32_t dh;               // ArmDh of the table
};

// Target of arm joint i's PD controller at `time`: the sinusoid q_d =
// qc + amp sin(om t + ph) and its rate qd_d = amp om cos(om t + ph).  One
// function for every caller, so a table of targets holds exactly the values
// a direct evaluation gives.
template <class R>
__host__ __device__ PDS_ALWAYS_INLINE void pd_target(R qc, R amp, R om, R ph, R time, R* qdes, R* qddes);

// The 14 targets of one time step, precomputed (q_d of the 7 arm joints,
// then their qd_d): the kernels pass this instead of the time, so each
// forward-dynamics evaluation reads its targets instead of evaluating 7
// sinusoids.  P is a pointer type (the constant address space on the
// device, so the wave-uniform reads are scalar loads).
template <class P>
struct TargetRow {
  P p;
};
constexpr int kArmTargets = 14;  // floats per time step of the target table

// Raw model description -> derived constants.  The caller's consts array:
// gravity[3]; per arm joint 7 x (a, alpha, d, m, cx, cy, cz, Ixx, Iyy, Izz,
// kp, kd, qc, amp, omega, phase); then for the hinge flange_d, hinge
// damping, box m, box c[3], box I[3] (diagonal), point-mass m, point-mass
// z; for the universal joint flange_d, box m; for the universal joint with
// weights flange_d, box m, box c[3], box I (xx, yy, zz, xy, xz, yz), the
// damping of both axes, point-mass m, point-mass z.
__host__ __device__ inline void arm_setup(const float* raw, ArmConst* K, int mount) {
  for (int d = 0; d < 3; ++d) K->g[d] = raw[d];
  for (int i = 0; i < 7; ++i) {
    const float* j = raw + 3 + 16 * i;
    float s, c;
    sincosf(j[1], &s, &c);
    K->b[i].ca = c;
    K->b[i].sa = s;
    K->b[i].ra = j[0];
    K->b[i].rd = j[2];
    K->b[i].m = j[3];
    K->b[i].c[0] = j[4]; K->b[i].c[1] = j[5]; K->b[i].c[2] = j[6];
    K->b[i].Ic[0] = j[7]; K->b[i].Ic[1] = 0.f; K->b[i].Ic[2] = 0.f;
    K->b[i].Ic[3] = j[8]; K->b[i].Ic[4] = 0.f; K->b[i].Ic[5] = j[9];
    K->b[i].kp = j[10]; K->b[i].kd = j[11]; K->b[i].qc = j[12];
    K->b[i].amp = j[13]; K->b[i].om = j[14]; K->b[i].ph = j[15];
  }
  // the Panda structure: each twist within float rounding of its right
  // angle, the offsets it has as zeros exactly zero
  K->dh = kDhPanda;
  for (int i = 0; i < 7; ++i) {
    const float* j = raw + 3 + 16 * i;
    const float tw = 1.5707963267948966f * (float)kPandaTwist[i];
    if (!(fabsf(j[1] - tw) <= 2e-7f) || (!kPandaA[i] && j[0] != 0.f) || (!kPandaD[i] && j[2] != 0.f))
      K->dh = kDhGeneric;
  }
  const float* h = raw + 3 + 16 * 7;
  for (int b = 7; b < kArmMaxBodies; ++b) {
    K->b[b].ca = 1.f;
    K->b[b].sa = 0.f;
    K->b[b].ra = K->b[b].rd = 0.f;
    for (int d = 0; d < 3; ++d) K->b[b].c[d] = 0.f;
    for (int e = 0; e < 6; ++e) K->b[b].Ic[e] = 0.f;
    K->b[b].m = 0.f;
  }
  K->b[7].rd = h[0];
  K->bh = K->b8 = K->pm_m = K->pm_z = 0.f;
  if (mount == kUJoint) {
    K->b[8].m = h[1];  // the box; its centre of mass and inertia come from theta
  } else if (mount == kUJointWeights) {
    K->b[8].m = h[1];
    K->b[8].c[0] = h[2]; K->b[8].c[1] = h[3]; K->b[8].c[2] = h[4];
    K->b[8].Ic[0] = h[5]; K->b[8].Ic[1] = h[8]; K->b[8].Ic[2] = h[9];
    K->b[8].Ic[3] = h[6]; K->b[8].Ic[4] = h[10]; K->b[8].Ic[5] = h[7];
    K->bh = h[11];
    K->b8 = h[12];
    K->pm_m = h[13];
    K->pm_z = h[14];
  } else {
    K->bh = h[1];
    K->b[7].m = h[2];
    K->b[7].c[0] = h[3]; K->b[7].c[1] = h[4]; K->b[7].c[2] = h[5];
    K->b[7].Ic[0] = h[6]; K->b[7].Ic[1] = 0.f; K->b[7].Ic[2] = 0.f;
    K->b[7].Ic[3] = h[7]; K->b[7].Ic[4] = 0.f; K->b[7].Ic[5] = h[8];
    K->pm_m = h[9];
    K->pm_z = h[10];
  }
  for (int b = 0; b < kArmMaxBodies; ++b) {
    K->b[b].Id[0] = K->b[b].Ic[0];
    K->b[b].Id[1] = K->b[b].Ic[3];
    K->b[b].Id[2] = K->b[b].Ic[5];
    const float m = K->b[b].m, cx = K->b[b].c[0], cy = K->b[b].c[1], cz = K->b[b].c[2];
    const float cc = cx * cx + cy * cy + cz * cz;
    K->b[b].Ar[0] = K->b[b].Ic[0] + m * (cc - cx * cx);
    K->b[b].Ar[1] = K->b[b].Ic[1] - m * cx * cy;
    K->b[b].Ar[2] = K->b[b].Ic[2] - m * cx * cz;
    K->b[b].Ar[3] = K->b[b].Ic[3] + m * (cc - cy * cy);
    K->b[b].Ar[4] = K->b[b].Ic[4] - m * cy * cz;
    K->b[b].Ar[5] = K->b[b].Ic[5] + m * (cc - cz * cz);
  }
}

__host__ __device__ inline void sincos_r(float x, float* sn, float* cs) { sincos_fast(x, sn, cs); }
inline void sincos_r(double x, double* sn, double* cs) {
  *sn = std::sin(x);
  *cs = std::cos(x);
}

template <class R>
__host__ __device__ PDS_ALWAYS_INLINE void pd_target(R qc, R amp, R om, R ph, R time, R* qdes, R* qddes) {
  R sn, cs;
  sincos_r(om * time + ph, &sn, &cs);
  *qdes = qc + amp * sn;
  *qddes = amp * om * cs;
}

// Calls f(std::integral_constant<int, I>) for I = B .. E-1 (up) or E-1 .. B
// (down), so that each body's code is specialised at compile time.
template <int B, int E, class F>
__host__ __device__ PDS_ALWAYS_INLINE void for_bodies_up(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    for_bodies_up<B + 1, E>(f);
  }
}
template <int B, int E, class F>
__host__ __device__ PDS_ALWAYS_INLINE void for_bodies_down(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>{});
    for_bodies_down<B, E - 1>(f);
  }
}

// KC is the type the model constants are read through: on the device the
// constant address space, so that their wave-uniform loads become scalar
// loads into SGPRs instead of vector registers.
template <class R, int BOX, class KC = ArmConst, int DH = kDhGeneric>
struct ArmMath {
  static constexpr int NB = ArmShape<BOX>::NB;
  static constexpr int M = ArmShape<BOX>::M;
  static constexpr int BOXB = ArmShape<BOX>::BOXB;
  static constexpr bool PM = ArmShape<BOX>::PM;

  struct V3 {
    R x, y, z;
  };
  __host__ __device__ static inline V3 v3(R a, R b, R c) { return V3{a, b, c}; }
  __host__ __device__ static inline V3 zero3() { return V3{R(0.f), R(0.f), R(0.f)}; }
  __host__ __device__ friend inline V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
  __host__ __device__ friend inline V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
  __host__ __device__ friend inline V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
  __host__ __device__ friend inline V3 operator*(R s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
  __host__ __device__ static inline V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
  }
  __host__ __device__ static inline R dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
  template <int K>
  __host__ __device__ static inline R comp(V3 v) {
    if constexpr (K == 0) return v.x; else if constexpr (K == 1) return v.y; else return v.z;
  }
  template <int K>
  __host__ __device__ static inline V3 along(R s) {  // s e_K
    if constexpr (K == 0) return v3(s, R(0.f), R(0.f));
    else if constexpr (K == 1) return v3(R(0.f), s, R(0.f));
    else return v3(R(0.f), R(0.f), s);
  }
  template <int K>
  __host__ __device__ static inline void add_along(V3& v, R s) {  // v += s e_K
    if constexpr (K == 0) v.x = v.x + s; else if constexpr (K == 1) v.y = v.y + s; else v.z = v.z + s;
  }
  // v x (s e_K)
  template <int K>
  __host__ __device__ static inline V3 xe(V3 v, R s) {
    if constexpr (K == 0) return v3(R(0.f), s * v.z, -(s * v.y));
    else if constexpr (K == 1) return v3(-(s * v.z), R(0.f), s * v.x);
    else return v3(s * v.y, -(s * v.x), R(0.f));
  }

  // Products with e_K x . without the component that vanishes: x . (e_K x
  // y), v += s (e_K x m), and a += v x (s e_K).
  template <int K>
  __host__ __device__ static inline R dot_ex(V3 x, V3 y) {
    if constexpr (K == 0) return x.z * y.y - x.y * y.z;
    else if constexpr (K == 1) return x.x * y.z - x.z * y.x;
    else return x.y * y.x - x.x * y.y;
  }
  template <int K>
  __host__ __device__ static inline void add_ex(V3& v, R s, V3 m) {
    if constexpr (K == 0) { v.y = v.y - s * m.z; v.z = v.z + s * m.y; }
    else if constexpr (K == 1) { v.x = v.x + s * m.z; v.z = v.z - s * m.x; }
    else { v.x = v.x - s * m.y; v.y = v.y + s * m.x; }
  }
  template <int K>
  __host__ __device__ static inline void add_xe(V3& a, V3 v, R s) {
    if constexpr (K == 0) { a.y = a.y + s * v.z; a.z = a.z - s * v.y; }
    else if constexpr (K == 1) { a.x = a.x - s * v.z; a.z = a.z + s * v.x; }
    else { a.x = a.x + s * v.y; a.y = a.y - s * v.x; }
  }

  // Rotation by an angle (c = cos, s = sin) about coordinate axis K applied
  // to a vector, and its transpose.  The pair (P, Q) it mixes: x -> (y, z),
  // y -> (z, x), z -> (x, y); P' = c P - s Q, Q' = s P + c Q.
  template <int K>
  __host__ __device__ static inline V3 rot(R c, R s, V3 p) {
    if constexpr (K == 0) return v3(p.x, c * p.y - s * p.z, s * p.y + c * p.z);
    else if constexpr (K == 1) return v3(c * p.x + s * p.z, p.y, c * p.z - s * p.x);
    else return v3(c * p.x - s * p.y, s * p.x + c * p.y, p.z);
  }
  template <int K>
  __host__ __device__ static inline V3 rotT(R c, R s, V3 p) {
    if constexpr (K == 0) return v3(p.x, c * p.y + s * p.z, c * p.z - s * p.y);
    else if constexpr (K == 1) return v3(c * p.x - s * p.z, p.y, s * p.x + c * p.z);
    else return v3(c * p.x + s * p.y, c * p.y - s * p.x, p.z);
  }

  // Spatial vectors: motion (w; v), force (n; f).
  struct SV {
    V3 a, l;
  };
  __host__ __device__ static inline SV sv(V3 a, V3 l) { return SV{a, l}; }
  __host__ __device__ static inline SV zero6() { return SV{zero3(), zero3()}; }
  __host__ __device__ friend inline SV operator+(SV p, SV q) { return sv(p.a + q.a, p.l + q.l); }
  __host__ __device__ friend inline SV operator-(SV p, SV q) { return sv(p.a - q.a, p.l - q.l); }
  __host__ __device__ friend inline SV operator-(SV p) { return sv(-p.a, -p.l); }
  __host__ __device__ friend inline SV operator*(R s, SV p) { return sv(s * p.a, s * p.l); }
  __host__ __device__ static inline R sdot(SV p, SV q) { return dot(p.a, q.a) + dot(p.l, q.l); }
  // v x m  and  v x* f
  __host__ __device__ static inline SV crm(SV v, SV m) { return sv(cross(v.a, m.a), cross(v.a, m.l) + cross(v.l, m.a)); }
  __host__ __device__ static inline SV crf(SV v, SV f) { return sv(cross(v.a, f.a) + cross(v.l, f.l), cross(v.a, f.l)); }
  // with S = (e_K; 0): v x (s S)
  template <int K>
  __host__ __device__ static inline SV crmS(SV v, R s) { return sv(xe<K>(v.a, s), xe<K>(v.l, s)); }
  // x . (S x* y) (S x* is S x on motion and force vectors alike) and
  // m += v x (s S), skipping the vanishing terms
  template <int K>
  __host__ __device__ static inline R sdot_crS(SV x, SV y) { return dot_ex<K>(x.a, y.a) + dot_ex<K>(x.l, y.l); }
  template <int K>
  __host__ __device__ static inline void add_crmS(SV& m, SV v, R s) {
    add_xe<K>(m.a, v.a, s);
    add_xe<K>(m.l, v.l, s);
  }

  // Joint axis of body I: arm joints about z, the hinge (or ring) about x,
  // the universal joint's box about y.
  template <int I>
  __host__ __device__ static constexpr int axis() { return I == 7 ? 0 : (I == 8 ? 1 : 2); }
  // The universal joint's ring carries no mass: its inertia terms vanish.
  template <int I>
  __host__ __device__ static constexpr bool massless() { return BOX != kHinge && I == 7; }

  // The table's structure at body I (ArmDh): the twist about x in right
  // angles (0, +-1; 2: a general twist, its cosine and sine from the
  // table), and whether the offsets a (along x) and d (along z) enter.
  // Bodies 7 and 8 have no twist and no a; body 7 has the flange offset d.
  template <int I>
  __host__ __device__ static constexpr int twist() {
    if constexpr (I >= 7) return 0;
    else if constexpr (DH == kDhPanda) return kPandaTwist[I];
    else return 2;
  }
  template <int I>
  __host__ __device__ static constexpr bool has_a() {
    if constexpr (I >= 7) return false;
    else if constexpr (DH == kDhPanda) return kPandaA[I];
    else return true;
  }
  template <int I>
  __host__ __device__ static constexpr bool has_d() {
    if constexpr (I >= 8) return false;
    else if constexpr (I == 7 || DH != kDhPanda) return true;
    else return kPandaD[I];
  }
  // Body I's twist rotation about x applied to a vector (rot), and its
  // transpose; a right angle with sign t gives y' = -t z, z' = t y (rot).
  template <int I>
  __host__ __device__ static inline V3 twist_rot(const KC& K, V3 p) {
    constexpr int t = twist<I>();
    if constexpr (t == 2) return rot<0>(R(K.b[I].ca), R(K.b[I].sa), p);
    else if constexpr (t == 0) return p;
    else if constexpr (t == 1) return v3(p.x, -p.z, p.y);
    else return v3(p.x, p.z, -p.y);
  }
  template <int I>
  __host__ __device__ static inline V3 twist_rotT(const KC& K, V3 p) {
    constexpr int t = twist<I>();
    if constexpr (t == 2) return rotT<0>(R(K.b[I].ca), R(K.b[I].sa), p);
    else if constexpr (t == 0) return p;
    else if constexpr (t == 1) return v3(p.x, p.z, -p.y);
    else return v3(p.x, -p.z, p.y);
  }

  // Plucker transform parent -> body I, motion vectors: shift by a along
  // x, rotate by alpha about x, shift by d along z, rotate by q about the
  // joint axis (each a change of coordinates: v - r x w, then R^T).
  template <int I>
  __host__ __device__ static inline SV xm(const KC& K, R cq, R sq, SV m) {
    V3 w = m.a, v = m.l;
    if constexpr (has_a<I>()) {
      const R a = K.b[I].ra;
      v = v3(v.x, v.y + a * w.z, v.z - a * w.y);
    }
    if constexpr (I < 7) {
      w = twist_rotT<I>(K, w);
      v = twist_rotT<I>(K, v);
    }
    if constexpr (has_d<I>()) {
      const R d = K.b[I].rd;
      v = v3(v.x + d * w.y, v.y - d * w.x, v.z);
    }
    return sv(rotT<axis<I>()>(cq, sq, w), rotT<axis<I>()>(cq, sq, v));
  }
  // Transpose of xm: force vectors body I -> parent (n + r x f).  It also
  // carries motion-space adjoints back to the parent.
  template <int I>
  __host__ __device__ static inline SV xtf(const KC& K, R cq, R sq, SV f) {
    V3 n = rot<axis<I>()>(cq, sq, f.a), g = rot<axis<I>()>(cq, sq, f.l);
    if constexpr (has_d<I>()) {
      const R d = K.b[I].rd;
      n = v3(n.x - d * g.y, n.y + d * g.x, n.z);
    }
    if constexpr (I < 7) {
      n = twist_rot<I>(K, n);
      g = twist_rot<I>(K, g);
    }
    if constexpr (has_a<I>()) {
      const R a = K.b[I].ra;
      n = v3(n.x, n.y - a * g.z, n.z + a * g.y);
    }
    return sv(n, g);
  }
  // Inverse of xm: motion vectors body I -> parent.
  template <int I>
  __host__ __device__ static inline SV minv(const KC& K, R cq, R sq, SV m) {
    V3 w = rot<axis<I>()>(cq, sq, m.a), v = rot<axis<I>()>(cq, sq, m.l);
    if constexpr (has_d<I>()) {
      const R d = K.b[I].rd;
      v = v3(v.x - d * w.y, v.y + d * w.x, v.z);
    }
    if constexpr (I < 7) {
      w = twist_rot<I>(K, w);
      v = twist_rot<I>(K, v);
    }
    if constexpr (has_a<I>()) {
      const R a = K.b[I].ra;
      v = v3(v.x, v.y - a * w.z, v.z + a * w.y);
    }
    return sv(w, v);
  }

  // Symmetric 3x3 (xx, xy, xz, yy, yz, zz) and general 3x3 (row-major).
  struct Sym3 {
    R e[6];
  };
  struct M3 {
    R e[9];
  };
  // index of entry (i, j) of a symmetric 3x3, a compile-time constant
  template <int i, int j>
  static constexpr int si = i > j ? (j == 0 ? i : (j == 1 ? 2 + i : 5)) : (i == 0 ? j : (i == 1 ? 2 + j : 5));
  // R M R^T for the rotation about axis K (pair P, Q; T unchanged).
  template <int K>
  __host__ __device__ static inline void rot_sym(R c, R s, Sym3& Mx) {
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1), T = K;
    const R mpp = Mx.e[si<P, P>], mqq = Mx.e[si<Q, Q>], mpq = Mx.e[si<P, Q>];
    const R mpt = Mx.e[si<P, T>], mqt = Mx.e[si<Q, T>];
    const R cc = c * c, ss = s * s, cs = c * s;
    const R two_cs_pq = (cs + cs) * mpq;
    Mx.e[si<P, P>] = cc * mpp - two_cs_pq + ss * mqq;
    Mx.e[si<Q, Q>] = ss * mpp + two_cs_pq + cc * mqq;
    Mx.e[si<P, Q>] = cs * (mpp - mqq) + (cc - ss) * mpq;
    Mx.e[si<P, T>] = c * mpt - s * mqt;
    Mx.e[si<Q, T>] = s * mpt + c * mqt;
  }
  template <int K>
  __host__ __device__ static inline void rot_gen(R c, R s, M3& B) {
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1);
  #pragma unroll
    for (int j = 0; j < 3; ++j) {  // rows
      const R bp = B.e[3 * P + j], bq = B.e[3 * Q + j];
      B.e[3 * P + j] = c * bp - s * bq;
      B.e[3 * Q + j] = s * bp + c * bq;
    }
  #pragma unroll
    for (int i = 0; i < 3; ++i) {  // columns
      const R bp = B.e[3 * i + P], bq = B.e[3 * i + Q];
      B.e[3 * i + P] = c * bp - s * bq;
      B.e[3 * i + Q] = s * bp + c * bq;
    }
  }

  // The same when row and column K vanish (the angular blocks of an
  // articulated inertia after its joint's update): P, Q entries only.
  template <int K>
  __host__ __device__ static inline void rot_sym_null(R c, R s, Sym3& Mx) {
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1);
    const R mpp = Mx.e[si<P, P>], mqq = Mx.e[si<Q, Q>], mpq = Mx.e[si<P, Q>];
    const R cc = c * c, ss = s * s, cs = c * s;
    const R two_cs_pq = (cs + cs) * mpq;
    Mx.e[si<P, P>] = cc * mpp - two_cs_pq + ss * mqq;
    Mx.e[si<Q, Q>] = ss * mpp + two_cs_pq + cc * mqq;
    Mx.e[si<P, Q>] = cs * (mpp - mqq) + (cc - ss) * mpq;
  }
  template <int K>
  __host__ __device__ static inline void rot_gen_null(R c, R s, M3& B) {  // row K of B zero
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1);
  #pragma unroll
    for (int j = 0; j < 3; ++j) {  // rows
      const R bp = B.e[3 * P + j], bq = B.e[3 * Q + j];
      B.e[3 * P + j] = c * bp - s * bq;
      B.e[3 * Q + j] = s * bp + c * bq;
    }
  #pragma unroll
    for (int i = 0; i < 3; ++i) {  // columns of rows P and Q
      if (i == K) continue;
      const R bp = B.e[3 * i + P], bq = B.e[3 * i + Q];
      B.e[3 * i + P] = c * bp - s * bq;
      B.e[3 * i + Q] = s * bp + c * bq;
    }
  }

  // The same for a right angle with sign S (c = 0, s = S): entries swap
  // and change sign, no arithmetic.
  template <int S>
  __host__ __device__ static inline R sgn(R x) {
    if constexpr (S > 0) return x; else return -x;
  }
  template <int K, int S>
  __host__ __device__ static inline void rot_sym_r(Sym3& Mx) {
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1), T = K;
    const R mpp = Mx.e[si<P, P>], mqq = Mx.e[si<Q, Q>], mpq = Mx.e[si<P, Q>];
    const R mpt = Mx.e[si<P, T>], mqt = Mx.e[si<Q, T>];
    Mx.e[si<P, P>] = mqq;
    Mx.e[si<Q, Q>] = mpp;
    Mx.e[si<P, Q>] = -mpq;
    Mx.e[si<P, T>] = sgn<-S>(mqt);
    Mx.e[si<Q, T>] = sgn<S>(mpt);
  }
  template <int K, int S>
  __host__ __device__ static inline void rot_gen_r(M3& B) {
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1);
  #pragma unroll
    for (int j = 0; j < 3; ++j) {  // rows
      const R bp = B.e[3 * P + j], bq = B.e[3 * Q + j];
      B.e[3 * P + j] = sgn<-S>(bq);
      B.e[3 * Q + j] = sgn<S>(bp);
    }
  #pragma unroll
    for (int i = 0; i < 3; ++i) {  // columns
      const R bp = B.e[3 * i + P], bq = B.e[3 * i + Q];
      B.e[3 * i + P] = sgn<-S>(bq);
      B.e[3 * i + Q] = sgn<S>(bp);
    }
  }

  // Symmetric 6x6 [[A, B], [B^T, C]].
  struct Sym6 {
    Sym3 A;
    M3 B;
    Sym3 C;
  };
  __host__ __device__ static inline SV sym6_mul(const Sym6& I, SV x) {
    const R* A = I.A.e;
    const R* B = I.B.e;
    const R* C = I.C.e;
    const V3 w = x.a, v = x.l;
    const V3 top = v3(A[0] * w.x + A[1] * w.y + A[2] * w.z + B[0] * v.x + B[1] * v.y + B[2] * v.z,
                      A[1] * w.x + A[3] * w.y + A[4] * w.z + B[3] * v.x + B[4] * v.y + B[5] * v.z,
                      A[2] * w.x + A[4] * w.y + A[5] * w.z + B[6] * v.x + B[7] * v.y + B[8] * v.z);
    const V3 bot = v3(B[0] * w.x + B[3] * w.y + B[6] * w.z + C[0] * v.x + C[1] * v.y + C[2] * v.z,
                      B[1] * w.x + B[4] * w.y + B[7] * w.z + C[1] * v.x + C[3] * v.y + C[4] * v.z,
                      B[2] * w.x + B[5] * w.y + B[8] * w.z + C[2] * v.x + C[4] * v.y + C[5] * v.z);
    return sv(top, bot);
  }
  // sym6_mul for an articulated inertia whose angular row and column K
  // vanish (A's row K, B's row K) times a vector whose K components vanish.
  template <int K>
  __host__ __device__ static inline SV sym6_mul_null(const Sym6& I, SV x) {
    constexpr int P = K == 0 ? 1 : (K == 1 ? 2 : 0), Q = K == 0 ? 2 : (K == 1 ? 0 : 1);
    const R* A = I.A.e;
    const R* B = I.B.e;
    const R* C = I.C.e;
    const R a[3] = {x.a.x, x.a.y, x.a.z}, l[3] = {x.l.x, x.l.y, x.l.z};
    R top[3], bot[3];
    top[K] = R(0.f);
    top[P] = A[si<P, P>] * a[P] + A[si<P, Q>] * a[Q] + B[3 * P + P] * l[P] + B[3 * P + Q] * l[Q];
    top[Q] = A[si<P, Q>] * a[P] + A[si<Q, Q>] * a[Q] + B[3 * Q + P] * l[P] + B[3 * Q + Q] * l[Q];
    bot[0] = B[3 * P + 0] * a[P] + B[3 * Q + 0] * a[Q] + C[si<0, P>] * l[P] + C[si<0, Q>] * l[Q];
    bot[1] = B[3 * P + 1] * a[P] + B[3 * Q + 1] * a[Q] + C[si<1, P>] * l[P] + C[si<1, Q>] * l[Q];
    bot[2] = B[3 * P + 2] * a[P] + B[3 * Q + 2] * a[Q] + C[si<2, P>] * l[P] + C[si<2, Q>] * l[Q];
    return sv(v3(top[0], top[1], top[2]), v3(bot[0], bot[1], bot[2]));
  }
  // X^T I X for a shift of the frame by d along z (r = d e_z, R = [r]x):
  // A - B R - (B R)^T - R C R and B + R C (C unchanged).
  // (NULLZ: A's row z and B's row z vanish and stay zero.)
  template <bool NULLZ = false>
  __host__ __device__ static inline void shift_z(Sym6& I, R d) {
    R* A = I.A.e;
    R* B = I.B.e;
    const R* C = I.C.e;
    const R dd = d * d;
    const R b00 = B[0], b01 = B[1], b10 = B[3], b11 = B[4];
    A[0] = A[0] - (d + d) * b01 + dd * C[3];
    A[1] = A[1] + d * (b00 - b11) - dd * C[1];
    A[3] = A[3] + (d + d) * b10 + dd * C[0];
    if constexpr (!NULLZ) {
      const R b20 = B[6], b21 = B[7];
      A[2] = A[2] - d * b21;
      A[4] = A[4] + d * b20;
    }
    // B += R C: row 0 -= d C[1, :], row 1 += d C[0, :]
    B[0] = b00 - d * C[1];
    B[1] = b01 - d * C[3];
    B[2] = B[2] - d * C[4];
    B[3] = b10 + d * C[0];
    B[4] = b11 + d * C[1];
    B[5] = B[5] + d * C[2];
  }
  // The same for a shift by a along x (r = a e_x).
  __host__ __device__ static inline void shift_x(Sym6& I, R a) {
    R* A = I.A.e;
    R* B = I.B.e;
    const R* C = I.C.e;
    const R aa = a * a;
    const R b01 = B[1], b02 = B[2], b11 = B[4], b12 = B[5], b21 = B[7], b22 = B[8];
    A[1] = A[1] - a * b02;
    A[2] = A[2] + a * b01;
    A[3] = A[3] - (a + a) * b12 + aa * C[5];
    A[4] = A[4] + a * (b11 - b22) - aa * C[4];
    A[5] = A[5] + (a + a) * b21 + aa * C[3];
    // B += R C: row 1 -= a C[2, :], row 2 += a C[1, :]
    B[3] = B[3] - a * C[2];
    B[4] = b11 - a * C[4];
    B[5] = b12 - a * C[5];
    B[6] = B[6] + a * C[1];
    B[7] = b21 + a * C[3];
    B[8] = b22 + a * C[4];
  }
  // Articulated inertia of body I seen from its parent, X^T Ia X, for Ia
  // after the joint's update (its angular row and column along the joint
  // axis zero).
  template <int I>
  __host__ __device__ static inline void congruence(const KC& K, R cq, R sq, Sym6& Ia) {
    constexpr int k = axis<I>();
    rot_sym_null<k>(cq, sq, Ia.A);
    rot_gen_null<k>(cq, sq, Ia.B);
    rot_sym<k>(cq, sq, Ia.C);
    if constexpr (has_d<I>()) shift_z<k == 2>(Ia, R(K.b[I].rd));
    constexpr int t = twist<I>();
    if constexpr (t == 2) {
      const R ca = K.b[I].ca, sa = K.b[I].sa;
      rot_sym<0>(ca, sa, Ia.A);
      rot_gen<0>(ca, sa, Ia.B);
      rot_sym<0>(ca, sa, Ia.C);
    } else if constexpr (t != 0) {
      rot_sym_r<0, t>(Ia.A);
      rot_gen_r<0, t>(Ia.B);
      rot_sym_r<0, t>(Ia.C);
    }
    if constexpr (has_a<I>()) shift_x(Ia, R(K.b[I].ra));
  }

  // Rigid-body inertia applied to a motion vector, from (m, c, Ic):
  // I [w; v] = [Ic w + c x p; p] with p = m (v - c x w).
  // (DIAG: Ic is diagonal and holds its xx, yy, zz only.)
  template <bool DIAG = false, class T>
  __host__ __device__ static inline SV rbi_mul(R m, V3 c, const T* Ic, SV x) {
    const V3 p = m * (x.l - cross(c, x.a));
    V3 Iw;
    if constexpr (DIAG)
      Iw = v3(R(Ic[0]) * x.a.x, R(Ic[1]) * x.a.y, R(Ic[2]) * x.a.z);
    else
      Iw = v3(Ic[0] * x.a.x + Ic[1] * x.a.y + Ic[2] * x.a.z, Ic[1] * x.a.x + Ic[3] * x.a.y + Ic[4] * x.a.z,
              Ic[2] * x.a.x + Ic[4] * x.a.y + Ic[5] * x.a.z);
    return sv(Iw + cross(c, p), p);
  }
  // Point mass m at c: I [w; v] = [c x p; p], p = m (v - c x w).
  __host__ __device__ static inline SV pm_mul(R m, V3 c, SV x) {
    const V3 p = m * (x.l - cross(c, x.a));
    return sv(cross(c, p), p);
  }
  // Adds a point mass m at c to a spatial inertia: A += m (|c|^2 1 - c c^T),
  // B += m [c]x, C += m 1.
  __host__ __device__ static inline void add_pm(Sym6& I, R m, V3 c) {
    const R mx = m * c.x, my = m * c.y, mz = m * c.z;
    I.A.e[0] = I.A.e[0] + my * c.y + mz * c.z;
    I.A.e[1] = I.A.e[1] - mx * c.y;
    I.A.e[2] = I.A.e[2] - mx * c.z;
    I.A.e[3] = I.A.e[3] + mx * c.x + mz * c.z;
    I.A.e[4] = I.A.e[4] - my * c.z;
    I.A.e[5] = I.A.e[5] + mx * c.x + my * c.y;
    I.B.e[1] = I.B.e[1] - mz; I.B.e[2] = I.B.e[2] + my;
    I.B.e[3] = I.B.e[3] + mz; I.B.e[5] = I.B.e[5] - mx;
    I.B.e[6] = I.B.e[6] - my; I.B.e[7] = I.B.e[7] + mx;
    I.C.e[0] = I.C.e[0] + m; I.C.e[3] = I.C.e[3] + m; I.C.e[5] = I.C.e[5] + m;
  }

  // The box's centre of mass and inertia about it from theta (universal
  // joint): Ic in the order xx, xy, xz, yy, yz, zz.
  __host__ __device__ static inline void box_from_theta(const R* th, V3* c, R* Ic) {
    *c = v3(th[6], th[7], th[8]);
    Ic[0] = th[0]; Ic[1] = th[3]; Ic[2] = th[4];
    Ic[3] = th[1]; Ic[4] = th[5]; Ic[5] = th[2];
  }

  // Spatial inertia of body I (rigid part plus the point masses in theta).
  template <int I>
  __host__ __device__ static inline Sym6 body_inertia(const KC& K, const R* th) {
    Sym6 S;
    R m = R(K.b[I].m);
    V3 c;
    if constexpr (BOX == kUJoint && I == 8) {
      R Ic[6];
      box_from_theta(th, &c, Ic);
      const R mx = m * c.x, my = m * c.y, mz = m * c.z;
      S.A.e[0] = Ic[0] + my * c.y + mz * c.z;
      S.A.e[1] = Ic[1] - mx * c.y;
      S.A.e[2] = Ic[2] - mx * c.z;
      S.A.e[3] = Ic[3] + mx * c.x + mz * c.z;
      S.A.e[4] = Ic[4] - my * c.z;
      S.A.e[5] = Ic[5] + mx * c.x + my * c.y;
    } else if constexpr (std::is_same<R, double>::value) {
      // FP64 host checks: the same block formed in FP64 (the precomputed
      // one is rounded to float), so the forward dynamics and the inertia
      // the reverse step applies agree to FP64 rounding
      c = v3(K.b[I].c[0], K.b[I].c[1], K.b[I].c[2]);
      const R mx = m * c.x, my = m * c.y, mz = m * c.z;
      S.A.e[0] = R(K.b[I].Ic[0]) + my * c.y + mz * c.z;
      S.A.e[1] = R(K.b[I].Ic[1]) - mx * c.y;
      S.A.e[2] = R(K.b[I].Ic[2]) - mx * c.z;
      S.A.e[3] = R(K.b[I].Ic[3]) + mx * c.x + mz * c.z;
      S.A.e[4] = R(K.b[I].Ic[4]) - my * c.z;
      S.A.e[5] = R(K.b[I].Ic[5]) + mx * c.x + my * c.y;
    } else {
      c = v3(K.b[I].c[0], K.b[I].c[1], K.b[I].c[2]);
  #pragma unroll
      for (int e = 0; e < 6; ++e) S.A.e[e] = R(K.b[I].Ar[e]);
    }
    const R mx = m * c.x, my = m * c.y, mz = m * c.z;
    S.B.e[0] = R(0.f); S.B.e[1] = -mz; S.B.e[2] = my;
    S.B.e[3] = mz; S.B.e[4] = R(0.f); S.B.e[5] = -mx;
    S.B.e[6] = -my; S.B.e[7] = mx; S.B.e[8] = R(0.f);
    S.C.e[0] = m; S.C.e[1] = R(0.f); S.C.e[2] = R(0.f); S.C.e[3] = m; S.C.e[4] = R(0.f); S.C.e[5] = m;
    if constexpr (PM && I == BOXB) {
      const R pm = R(K.pm_m), z = R(K.pm_z);
      add_pm(S, pm, v3(th[0], th[1], z));
      add_pm(S, pm, v3(th[2], th[3], z));
    }
    return S;
  }
  // I_body x, with the same terms as body_inertia.
  template <int I>
  __host__ __device__ static inline SV body_mul(const KC& K, const R* th, SV x) {
    SV r;
    if constexpr (BOX == kUJoint && I == 8) {
      V3 c;
      R Ic[6];
      box_from_theta(th, &c, Ic);
      r = rbi_mul(R(K.b[I].m), c, Ic, x);
    } else {
      // the arm links' and the hinged box's inertias about their centres
      // of mass are diagonal by the constants' layout
      constexpr bool diag = I < 7 || (BOX == kHinge && I == 7);
      if constexpr (diag)
        r = rbi_mul<true>(R(K.b[I].m), v3(K.b[I].c[0], K.b[I].c[1], K.b[I].c[2]), K.b[I].Id, x);
      else
        r = rbi_mul(R(K.b[I].m), v3(K.b[I].c[0], K.b[I].c[1], K.b[I].c[2]), K.b[I].Ic, x);
    }
    if constexpr (PM && I == BOXB) {
      const R pm = R(K.pm_m), z = R(K.pm_z);
      r = r + pm_mul(pm, v3(th[0], th[1], z), x) + pm_mul(pm, v3(th[2], th[3], z), x);
    }
    return r;
  }

  // Joint torque at time `time` (PD on the arm, viscous damping on the
  // passive axes).
  // (`time` is the time itself, or the time step's row of precomputed
  // targets.)
  template <int I>
  __host__ __device__ static PDS_ALWAYS_INLINE void targets(const KC& K, R time, R* qdes, R* qddes) {
    pd_target(R(K.b[I].qc), R(K.b[I].amp), R(K.b[I].om), R(K.b[I].ph), time, qdes, qddes);
  }
  template <int I, class P>
  __host__ __device__ static PDS_ALWAYS_INLINE void targets(const KC&, TargetRow<P> row, R* qdes, R* qddes) {
    *qdes = R(row.p[I]);
    *qddes = R(row.p[7 + I]);
  }
  template <int I, class TM>
  __host__ __device__ static inline R joint_tau(const KC& K, const R* th, TM time, R q, R qd) {
    if constexpr (I >= 7) {
      if constexpr (BOX == kUJoint) return -(th[I + 2] * qd);
      else if constexpr (BOX == kUJointWeights && I == 8) return -(R(K.b8) * qd);
      else return -(R(K.bh) * qd);
    } else {
      R qdes, qddes;
      targets<I>(K, time, &qdes, &qddes);
      return R(K.b[I].kp) * (qdes - q) + R(K.b[I].kd) * (qddes - qd);
    }
  }

  // Intermediates of one forward-dynamics evaluation kept for the reverse.
  // (The reverse step recovers the other bodies' velocities and
  // accelerations from the last body's through the inverse transforms.)
  struct Tape {
    R cs[NB], sn[NB];
    SV v_last;  // velocity of the last body
    SV a_last;  // acceleration of the last body (incl. S qdd)
    SV U[NB];   // IA S
    R invD[NB];
    R qdd[NB];
  };

  // Compiler-level memory barrier: the model constants are re-read (scalar
  // loads, cached) inside every body's code instead of being hoisted out of
  // the step loops into vector registers.
  __host__ __device__ static PDS_ALWAYS_INLINE void keep_consts_in_memory() {
  #if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" ::: "memory");
  #endif
  }

  // Articulated Body Algorithm (three passes over the chain).
  template <class TM>
  __host__ __device__ static PDS_ALWAYS_INLINE void aba(const KC& K, const R* th, const R* q, const R* qd, TM time,
                                                      Tape& T) {
    R u[NB];
    SV vb[NB];  // body velocities
    for_bodies_up<0, NB>([&](auto Ic) {
      constexpr int i = decltype(Ic)::value;
      keep_consts_in_memory();
      sincos_r(q[i], &T.sn[i], &T.cs[i]);
      if constexpr (i == 0) {
        vb[0] = sv(along<axis<0>()>(qd[0]), zero3());
      } else {
        vb[i] = xm<i>(K, T.cs[i], T.sn[i], vb[i - 1]);
        add_along<axis<i>()>(vb[i].a, qd[i]);
      }
    });
    Sym6 IAc;   // child's articulated inertia seen from this body
    SV pAc;     // and its bias force
    for_bodies_down<0, NB>([&](auto Ic) {
      constexpr int i = decltype(Ic)::value;
      constexpr int k = axis<i>();
      keep_consts_in_memory();
      Sym6 IA;
      SV pA;
      if constexpr (massless<i>()) {
        IA = IAc;
        pA = pAc;
      } else {
        IA = body_inertia<i>(K, th);
        const SV h = body_mul<i>(K, th, vb[i]);
        pA = crf(vb[i], h);
        if constexpr (i < NB - 1) {
          // a body's own B has a zero diagonal and its C is m times the
          // identity (body_inertia): those entries take the child's alone
  #pragma unroll
          for (int e = 0; e < 6; ++e) {
            IA.A.e[e] = IA.A.e[e] + IAc.A.e[e];
            IA.C.e[e] = (e == 1 || e == 2 || e == 4) ? IAc.C.e[e] : IA.C.e[e] + IAc.C.e[e];
          }
  #pragma unroll
          for (int e = 0; e < 9; ++e) IA.B.e[e] = (e % 4 == 0) ? IAc.B.e[e] : IA.B.e[e] + IAc.B.e[e];
          pA = pA + pAc;
        }
      }
      const SV U = sv(v3(IA.A.e[si<0, k>], IA.A.e[si<1, k>], IA.A.e[si<2, k>]),
                      v3(IA.B.e[3 * k], IA.B.e[3 * k + 1], IA.B.e[3 * k + 2]));
      const R invD = recip(comp<k>(U.a));
      u[i] = joint_tau<i, TM>(K, th, time, q[i], qd[i]) - comp<k>(pA.a);
      T.U[i] = U;
      T.invD[i] = invD;
      if constexpr (i > 0) {
        // Ia = IA - U U^T / D.  Its angular row and column k vanish (Ia S =
        // U - U D / D = 0): they are set to zero instead of computed, and
        // the products below skip them.
        constexpr int P = k == 0 ? 1 : (k == 1 ? 2 : 0), Q = k == 0 ? 2 : (k == 1 ? 0 : 1);
        constexpr int lo = P < Q ? P : Q, hi = P < Q ? Q : P;
        const V3 wa = invD * U.a, wl = invD * U.l;
        const R wa3[3] = {wa.x, wa.y, wa.z}, ua3[3] = {U.a.x, U.a.y, U.a.z};
        const R wl3[3] = {wl.x, wl.y, wl.z}, ul3[3] = {U.l.x, U.l.y, U.l.z};
        Sym6& Ia = IA;
        Ia.A.e[si<P, P>] = Ia.A.e[si<P, P>] - wa3[P] * ua3[P];
        Ia.A.e[si<Q, Q>] = Ia.A.e[si<Q, Q>] - wa3[Q] * ua3[Q];
        Ia.A.e[si<lo, hi>] = Ia.A.e[si<lo, hi>] - wa3[lo] * ua3[hi];
        Ia.A.e[si<k, k>] = Ia.A.e[si<P, k>] = Ia.A.e[si<Q, k>] = R(0.f);
  #pragma unroll
        for (int r = 0; r < 3; ++r)
  #pragma unroll
          for (int c = r; c < 3; ++c) {
            const int e = r == 0 ? c : (r == 1 ? 2 + c : 5);
            Ia.C.e[e] = Ia.C.e[e] - wl3[r] * ul3[c];
          }
  #pragma unroll
        for (int r = 0; r < 3; ++r)
  #pragma unroll
          for (int c = 0; c < 3; ++c)
            Ia.B.e[3 * r + c] = r == k ? R(0.f) : Ia.B.e[3 * r + c] - wa3[r] * ul3[c];
        const SV ci = crmS<k>(vb[i], qd[i]);
        const SV pa = pA + sym6_mul_null<k>(Ia, ci) + (u[i] * invD) * U;
        congruence<i>(K, T.cs[i], T.sn[i], Ia);
        IAc = Ia;
        pAc = xtf<i>(K, T.cs[i], T.sn[i], pa);
      }
    });
    SV ap = sv(zero3(), v3(-R(K.g[0]), -R(K.g[1]), -R(K.g[2])));
    for_bodies_up<0, NB>([&](auto Ic) {
      constexpr int i = decltype(Ic)::value;
      constexpr int k = axis<i>();
      keep_consts_in_memory();
      SV a1 = xm<i>(K, T.cs[i], T.sn[i], ap);
      if constexpr (i > 0) add_crmS<k>(a1, vb[i], qd[i]);
      const R qdd = (u[i] - sdot(T.U[i], a1)) * T.invD[i];
      T.qdd[i] = qdd;
      add_along<k>(a1.a, qdd);
      ap = a1;
    });
    T.v_last = vb[NB - 1];
    T.a_last = ap;
  }

  template <class TM>
  __host__ __device__ static PDS_ALWAYS_INLINE void step(const KC& K, const R* th, TM time, R dt, R* q, R* qd) {
    Tape T;
    aba(K, th, q, qd, time, T);
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      qd[i] = qd[i] + dt * T.qdd[i];
      q[i] = q[i] + dt * qd[i];
    }
  }

  // Reverse of one Euler step for both adjoint channels.  (qb[c], qdb[c])
  // enter as channel c's adjoints of the step's outputs and leave as its
  // adjoints of the step's inputs; thb[c] accumulates d/d theta.
  __host__ __device__ static PDS_ALWAYS_INLINE void step_rev(const KC& K, const R* th, const R* qd, const Tape& T,
                                                           R dt, R (&qb)[2][NB], R (&qdb)[2][NB], R (&thb)[2][M]) {
    // Euler: q' = q + dt qd', qd' = qd + dt qdd.  lam first holds qdd_bar.
    R lam[2][NB], us[2][NB];
  #pragma unroll
    for (int c = 0; c < 2; ++c)
  #pragma unroll
      for (int i = 0; i < NB; ++i) {
        qdb[c][i] = qdb[c][i] + dt * qb[c][i];
        lam[c][i] = dt * qdb[c][i];
      }
    // lambda = H^{-1} qdd_bar: ABA with zero velocity and gravity, the
    // child's bias-force contribution carried inward.
    {
      SV pAc[2];
      for_bodies_down<0, NB>([&](auto Ic) {
        constexpr int i = decltype(Ic)::value;
        constexpr int k = axis<i>();
        keep_consts_in_memory();
  #pragma unroll
        for (int c = 0; c < 2; ++c) {
          if constexpr (i < NB - 1) us[c][i] = lam[c][i] - comp<k>(pAc[c].a);
          else us[c][i] = lam[c][i];
          if constexpr (i > 0) {
            SV t = (us[c][i] * T.invD[i]) * T.U[i];
            if constexpr (i < NB - 1) t = t + pAc[c];
            pAc[c] = xtf<i>(K, T.cs[i], T.sn[i], t);
          }
        }
      });
    }
    {
      SV ap[2];
      for_bodies_up<0, NB>([&](auto Ic) {
        constexpr int i = decltype(Ic)::value;
        constexpr int k = axis<i>();
        keep_consts_in_memory();
  #pragma unroll
        for (int c = 0; c < 2; ++c) {
          if constexpr (i == 0) {
            lam[c][0] = us[c][0] * T.invD[0];
            ap[c] = sv(along<k>(lam[c][0]), zero3());
          } else {
            SV a1 = xm<i>(K, T.cs[i], T.sn[i], ap[c]);
            lam[c][i] = (us[c][i] - sdot(T.U[i], a1)) * T.invD[i];
            add_along<k>(a1.a, lam[c][i]);
            ap[c] = a1;
          }
        }
      });
    }
    // x_bar += -lambda^T dF/dx, F = ID - tau.  The tau part: d tau / d q =
    // -kp, d tau / d qd = -kd (arm), -b (passive axes); for the joint's
    // friction coefficients d tau / d b = -qd.
  #pragma unroll
    for (int c = 0; c < 2; ++c) {
  #pragma unroll
      for (int i = 0; i < 7; ++i) {
        qb[c][i] = qb[c][i] - R(K.b[i].kp) * lam[c][i];
        qdb[c][i] = qdb[c][i] - R(K.b[i].kd) * lam[c][i];
      }
      if constexpr (BOX == kHinge) {
        qdb[c][7] = qdb[c][7] - R(K.bh) * lam[c][7];
      } else if constexpr (BOX == kUJointWeights) {
        qdb[c][7] = qdb[c][7] - R(K.bh) * lam[c][7];
        qdb[c][8] = qdb[c][8] - R(K.b8) * lam[c][8];
      } else {
  #pragma unroll
        for (int i = 7; i < NB; ++i) {
          qdb[c][i] = qdb[c][i] - th[i + 2] * lam[c][i];
          thb[c][i + 2] = thb[c][i + 2] - lam[c][i] * qd[i];
        }
      }
    }
    // ID part: reverse of RNEA with output seed mu = -lambda.  Total-force
    // adjoints outward, ftb_i = S_i mu_i + X_i ftb_{i-1}; only the last is
    // kept, the others are recovered inward through X_i^{-1}.
    SV ftb[2];
    for_bodies_up<0, NB>([&](auto Ic) {
      constexpr int i = decltype(Ic)::value;
      constexpr int k = axis<i>();
      keep_consts_in_memory();
  #pragma unroll
      for (int c = 0; c < 2; ++c) {
        if constexpr (i == 0) {
          ftb[c] = sv(along<k>(-lam[c][0]), zero3());
        } else {
          ftb[c] = xm<i>(K, T.cs[i], T.sn[i], ftb[c]);
          add_along<k>(ftb[c].a, -lam[c][i]);
        }
      }
    });
    // Inward: total forces ft_i = f_i + X_{i+1}^T ft_{i+1} (shared), the q
    // dependence of X_i^T ft_i, and the reverse of the outward pass
    // (velocities, accelerations) with body-force adjoints ftb_i.
    SV ftc;          // X_{i+1}^T ft_{i+1}
    SV abar[2], vbar[2];
    SV v = T.v_last, a = T.a_last;  // body i's velocity and acceleration
    for_bodies_down<0, NB>([&](auto Ic) {
      constexpr int i = decltype(Ic)::value;
      constexpr int k = axis<i>();
      keep_consts_in_memory();
      SV ft, h;
      if constexpr (massless<i>()) {
        ft = ftc;
      } else {
        h = body_mul<i>(K, th, v);
        ft = body_mul<i>(K, th, a) + crf(v, h);
        if constexpr (i < NB - 1) ft = ft + ftc;
      }
      // X_i a_{i-1} and X_i v_{i-1}, read off this body's own terms
      SV ya = a;
      add_crmS<k>(ya, v, -qd[i]);
      add_along<k>(ya.a, -T.qdd[i]);
      SV yv = v;
      add_along<k>(yv.a, -qd[i]);
  #pragma unroll
      for (int c = 0; c < 2; ++c) {
        const SV fb = ftb[c];
        SV vxfb;
        if constexpr (!massless<i>()) vxfb = crm(v, fb);
        if constexpr (BOX == kUJoint && i == 8) {
          // theta: fb . f = g(a, fb) + g(v, -v x fb) with g(x, y) = y . I x,
          // I x = [Ic x_w + c x p; p], p = m (x_l - c x x_w).  d g / d Ic is
          // the symmetric outer product of y_n and x_w; d g / d c as for the
          // hinge's point masses.
          V3 cm;
          R Icb[6];
          box_from_theta(th, &cm, Icb);
          const R mb = R(K.b[i].m);
  #pragma unroll
          for (int term = 0; term < 2; ++term) {
            const SV x = term == 0 ? a : v;
            const SV y = term == 0 ? fb : -vxfb;
            thb[c][0] = thb[c][0] + y.a.x * x.a.x;
            thb[c][1] = thb[c][1] + y.a.y * x.a.y;
            thb[c][2] = thb[c][2] + y.a.z * x.a.z;
            thb[c][3] = thb[c][3] + y.a.x * x.a.y + y.a.y * x.a.x;
            thb[c][4] = thb[c][4] + y.a.x * x.a.z + y.a.z * x.a.x;
            thb[c][5] = thb[c][5] + y.a.y * x.a.z + y.a.z * x.a.y;
            const V3 p = mb * (x.l - cross(cm, x.a));
            const V3 z = cross(y.a, cm) + y.l;
            const V3 gc = cross(p, y.a) - mb * cross(x.a, z);
            thb[c][6] = thb[c][6] + gc.x;
            thb[c][7] = thb[c][7] + gc.y;
            thb[c][8] = thb[c][8] + gc.z;
          }
        }
        if constexpr (PM && i == BOXB) {
          // theta: the point-mass positions (x, y) in f = I(c) a + v x* I(c) v.
          // With g(c; x, y) = y . I(c) x = y_n . (c x p) + y_f . p and
          // p = m (x_l - c x x_w):  dg/dc = p x y_n - m x_w x (y_n x c + y_f).
          // fb . f = g(c; a, fb) + g(c; v, -v x fb)  (fb . (v x* h) = -(v x fb) . h).
          const R mm = R(K.pm_m), z0 = R(K.pm_z);
  #pragma unroll
          for (int w = 0; w < 2; ++w) {
            const V3 cp = v3(th[2 * w], th[2 * w + 1], z0);
            V3 gsum = zero3();
  #pragma unroll
            for (int term = 0; term < 2; ++term) {
              const SV x = term == 0 ? a : v;
              const SV y = term == 0 ? fb : -vxfb;
              const V3 p = mm * (x.l - cross(cp, x.a));
              const V3 z = cross(y.a, cp) + y.l;
              gsum = gsum + cross(p, y.a) - mm * cross(x.a, z);
            }
            thb[c][2 * w] = thb[c][2 * w] + gsum.x;
            thb[c][2 * w + 1] = thb[c][2 * w + 1] + gsum.y;
          }
        }
        // X_i ftb_{i-1} = ftb_i - S_i mu_i; d/dq_i of ftb_{i-1} . X_i^T ft_i
        // = (X_i ftb_{i-1}) . (S x* ft_i)
        SV xf = fb;
        add_along<k>(xf.a, lam[c][i]);
        if constexpr (i > 0) qb[c][i] = qb[c][i] + sdot_crS<k>(xf, ft);
        // f = I a + v x* (I v):  a_bar += I fb;  v_bar += -fb x* h - I (v x fb)
        if constexpr (!massless<i>()) {
          const SV Ifb = body_mul<i>(K, th, fb);
          const SV dv = crf(fb, h) + body_mul<i>(K, th, vxfb);
          if constexpr (i < NB - 1) {
            abar[c] = abar[c] + Ifb;
            vbar[c] = vbar[c] - dv;
          } else {
            abar[c] = Ifb;
            vbar[c] = -dv;
          }
        }
        // a_i = X_i a_{i-1} + v_i x (S qd_i) + S qdd_i (qdd held fixed)
        add_ex<k>(vbar[c].a, qd[i], abar[c].a);
        add_ex<k>(vbar[c].l, qd[i], abar[c].l);
        qdb[c][i] = qdb[c][i] - comp<k>(crf(v, abar[c]).a) + comp<k>(vbar[c].a);
        // d/dq (abar . X a_prev) = -abar . (S x X a_prev), likewise for v
        qb[c][i] = qb[c][i] - sdot_crS<k>(abar[c], ya);
        if constexpr (i > 0) {
          qb[c][i] = qb[c][i] - sdot_crS<k>(vbar[c], yv);
          abar[c] = xtf<i>(K, T.cs[i], T.sn[i], abar[c]);
          vbar[c] = xtf<i>(K, T.cs[i], T.sn[i], vbar[c]);
          ftb[c] = minv<i>(K, T.cs[i], T.sn[i], xf);
        }
      }
      if constexpr (i > 0) {
        ftc = xtf<i>(K, T.cs[i], T.sn[i], ft);
        // the parent's velocity and acceleration: X_i^{-1} of X_i v_{i-1}, X_i a_{i-1}
        v = minv<i>(K, T.cs[i], T.sn[i], yv);
        a = minv<i>(K, T.cs[i], T.sn[i], ya);
      }
    });
  }

  // World pose of every joint along the chain for the box-frame
  // observation: calls f(body, world axis of its joint, joint origin) and
  // returns the last body's origin o and rotation Rw (columns = its axes).
  // R_i = R_{i-1} Rot_x(alpha) Rot_axis(q), o_i = o_{i-1} + R_{i-1} r_i.
  template <class F>
  __host__ __device__ static PDS_ALWAYS_INLINE void chain_pose(const KC& K, const R* cs, const R* sn, V3* o_out,
                                                            V3 (&Rw)[3], F&& f) {
    Rw[0] = v3(R(1.f), R(0.f), R(0.f));  // columns
    Rw[1] = v3(R(0.f), R(1.f), R(0.f));
    Rw[2] = v3(R(0.f), R(0.f), R(1.f));
    V3 o = zero3();
    for_bodies_up<0, NB>([&](auto Ic) {
      constexpr int i = decltype(Ic)::value;
      constexpr int k = axis<i>();
      keep_consts_in_memory();
      if constexpr (has_a<i>()) o = o + R(K.b[i].ra) * Rw[0];
      constexpr int t = twist<i>();
      const V3 y = Rw[1], z = Rw[2];
      if constexpr (t == 2) {
        const R ca = K.b[i].ca, sa = K.b[i].sa;
        Rw[1] = ca * y + sa * z;
        Rw[2] = ca * z - sa * y;
      } else if constexpr (t == 1) {  // ca = 0, sa = 1
        Rw[1] = z;
        Rw[2] = -y;
      } else if constexpr (t == -1) {
        Rw[1] = -z;
        Rw[2] = y;
      }
      if constexpr (has_d<i>()) o = o + R(K.b[i].rd) * Rw[2];
      constexpr int P = k == 0 ? 1 : (k == 1 ? 2 : 0), Q = k == 0 ? 2 : (k == 1 ? 0 : 1);
      const V3 p = Rw[P], qv = Rw[Q];
      Rw[P] = cs[i] * p + sn[i] * qv;
      Rw[Q] = cs[i] * qv - sn[i] * p;
      f(Ic, Rw[k], o);
    });
    *o_out = o;
  }

  // The box frame (universal joint): its origin and the points 1 m along its
  // x, y, z axes (12 numbers).
  __host__ __device__ static PDS_ALWAYS_INLINE void box_frame(const KC& K, const R* q, R* x) {
    R cs[NB], sn[NB];
  #pragma unroll
    for (int i = 0; i < NB; ++i) sincos_r(q[i], &sn[i], &cs[i]);
    V3 o, Rw[3];
    chain_pose(K, cs, sn, &o, Rw, [](auto, V3, V3) {});
    x[0] = o.x; x[1] = o.y; x[2] = o.z;
  #pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[3 + 3 * a] = o.x + Rw[a].x;
      x[4 + 3 * a] = o.y + Rw[a].y;
      x[5 + 3 * a] = o.z + Rw[a].z;
    }
  }

  // Observation term of one state (universal joint): returns
  // sum_c ((obs_c - x_c) w_c)^2 and, with ADJ, adds d/dq of -1/2 of it to
  // qb.  Every observed point p sits on the box, so dp/dq_j = z_j x
  // (p - o_j) with z_j and o_j joint j's world axis and origin; with rt_p =
  // w^2 (obs - p) summed as A = sum p x rt_p and B = sum rt_p, the adjoint of
  // q_j is z_j . (A - o_j x B).
    template <bool ADJ, class OP>
  __host__ __device__ static PDS_ALWAYS_INLINE R box_obs(const KC& K, const R* q, OP obs, const float* w,
                                                       R* qb) {
    R cs[NB], sn[NB];
  #pragma unroll
    for (int i = 0; i < NB; ++i) sincos_r(q[i], &sn[i], &cs[i]);
    V3 o, Rw[3];
    chain_pose(K, cs, sn, &o, Rw, [](auto, V3, V3) {});
    R ss = R(0.f);
    V3 A = zero3(), Bs = zero3();
  #pragma unroll
    for (int pnt = 0; pnt < 4; ++pnt) {
      const V3 p = pnt == 0 ? o : o + Rw[pnt - 1];
      const int c0 = 3 * pnt;
      const R r0 = (R(obs[c0]) - p.x) * R(w[c0]), r1 = (R(obs[c0 + 1]) - p.y) * R(w[c0 + 1]),
              r2 = (R(obs[c0 + 2]) - p.z) * R(w[c0 + 2]);
      ss = ss + r0 * r0 + r1 * r1 + r2 * r2;
      const V3 rt = v3(r0 * R(w[c0]), r1 * R(w[c0 + 1]), r2 * R(w[c0 + 2]));
      A = A + cross(p, rt);
      Bs = Bs + rt;
    }
    if constexpr (ADJ) {
      V3 o2, Rw2[3];
      chain_pose(K, cs, sn, &o2, Rw2, [&](auto Ic, V3 z, V3 oj) {
        constexpr int i = decltype(Ic)::value;
        qb[i] = qb[i] + dot(z, A - cross(oj, Bs));
      });
    }
    return ss;
  }
};

}  // namespace pds
