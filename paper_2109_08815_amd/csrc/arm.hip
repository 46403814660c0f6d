// Window rollouts and their reverse-mode adjoint for the 7-joint arm that
// carries a box on a passive hinge (8 bodies, 6D spatial algebra).
//
// Model.  Bodies 0..6 are the arm links, joint i revolute about its local z
// axis after the fixed modified-DH placement (Rot_x(alpha), Trans_x(a),
// Trans_z(d)); body 7 is the box on a hinge about the flange x axis, offset
// by flange_d along the flange z axis.  Arm joints are PD-controlled
// towards a sinusoid q_d(t) = qc + A sin(omega t + phase); the hinge has
// viscous damping.  theta = (x_a, y_a, x_b, y_b), the in-plane positions of
// two equal point masses in the box frame.  The observation is the hinge
// angle.
//
// Forward dynamics: the Articulated Body Algorithm (App. B-A) in body
// coordinates; articulated inertias are symmetric 6x6 matrices kept as
// three 3x3 blocks [[A, B], [B^T, C]] (A, C symmetric).  A step is the
// semi-implicit Euler update of eq. dynamics.
//
// Reverse step.  With F(q, qd, qdd, theta) = ID(q, qd, qdd; theta) -
// tau(q, qd, t) = 0 defining qdd, the vector-Jacobian product of forward
// dynamics with seed qdd_bar is x_bar = -(dF/dx)^T lambda with
// lambda = H^{-1} qdd_bar.  lambda comes from an ABA solve (zero velocity,
// no gravity) that reuses the articulated-body terms U, D of the forward
// pass; dF/dx^T lambda is the reverse of the recursive Newton-Euler
// inverse dynamics.  No articulated inertia is ever differentiated.
//
// Work layout as for planar chains: one lane per window unit, the window's
// checkpoints and the segment being reversed in LDS [slot][component][lane].
#include <cmath>
#include <vector>

#include "common.h"
#include "sincos.h"
#include "flop_count.h"

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
// description (see pds.h for the raw layout).
struct ArmConst {
  float g[3];
  float E[kArmMaxBodies][9];   // tree rotation: parent coordinates -> joint frame (row-major)
  float r[kArmMaxBodies][3];   // tree translation (joint origin in parent coordinates)
  float m[kArmMaxBodies];      // link mass (hinge: body 7 the box alone; joint: body 8 the box)
  float c[kArmMaxBodies][3];   // centre of mass
  float Ic[kArmMaxBodies][6];  // inertia about the COM: xx, xy, xz, yy, yz, zz
  float kp[7], kd[7], qc[7], amp[7], om[7], ph[7];
  float bh;                 // hinge damping (universal joint with weights: first axis)
  float b8;                 // universal joint with weights: damping of the second axis
  float pm_m, pm_z;         // point masses: mass each, height in the box frame
};

namespace {

__host__ __device__ inline void sincos_r(float x, float* sn, float* cs) { sincos_fast(x, sn, cs); }

// The spatial algebra, forward dynamics and reverse step, generic over the
// scalar type R: float on the device; a counting scalar on the host gives
// the algorithmic FLOPs of one step.
template <class R, int BOX>
struct ArmMath {
  static constexpr int NB = ArmShape<BOX>::NB;
  static constexpr int BOXB = ArmShape<BOX>::BOXB;
  static constexpr bool PM = ArmShape<BOX>::PM;
  struct V3 {
    R x, y, z;
  };
  __host__ __device__ static inline V3 v3(R a, R b, R c) { return V3{a, b, c}; }
  __host__ __device__ friend inline V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
  __host__ __device__ friend inline V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
  __host__ __device__ friend inline V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
  __host__ __device__ friend inline V3 operator*(R s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
  __host__ __device__ static inline V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
  }
  __host__ __device__ static inline R dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

  // Rotation E (row-major 3x3) applied to v and its transpose.
  __host__ __device__ static inline V3 mulE(const R* E, V3 v) {
    return v3(E[0] * v.x + E[1] * v.y + E[2] * v.z, E[3] * v.x + E[4] * v.y + E[5] * v.z,
              E[6] * v.x + E[7] * v.y + E[8] * v.z);
  }
  __host__ __device__ static inline V3 mulEt(const R* E, V3 v) {
    return v3(E[0] * v.x + E[3] * v.y + E[6] * v.z, E[1] * v.x + E[4] * v.y + E[7] * v.z,
              E[2] * v.x + E[5] * v.y + E[8] * v.z);
  }

  // Spatial vectors: motion (w; v), force (n; f).
  struct SV {
    V3 a, l;
  };
  __host__ __device__ static inline SV sv(V3 a, V3 l) { return SV{a, l}; }
  __host__ __device__ friend inline SV operator+(SV p, SV q) { return sv(p.a + q.a, p.l + q.l); }
  __host__ __device__ friend inline SV operator-(SV p, SV q) { return sv(p.a - q.a, p.l - q.l); }
  __host__ __device__ friend inline SV operator*(R s, SV p) { return sv(s * p.a, s * p.l); }
  __host__ __device__ static inline R sdot(SV p, SV q) { return dot(p.a, q.a) + dot(p.l, q.l); }
  // v x m  and  v x* f
  __host__ __device__ static inline SV crm(SV v, SV m) { return sv(cross(v.a, m.a), cross(v.a, m.l) + cross(v.l, m.a)); }
  __host__ __device__ static inline SV crf(SV v, SV f) { return sv(cross(v.a, f.a) + cross(v.l, f.l), cross(v.a, f.l)); }

  // Plucker transform parent -> body: (E, r).  Motion: X m; force: X^T f.
  __host__ __device__ static inline SV xm(const R* E, V3 r, SV m) { return sv(mulE(E, m.a), mulE(E, m.l - cross(r, m.a))); }
  __host__ __device__ static inline SV xtf(const R* E, V3 r, SV f) {
    const V3 fl = mulEt(E, f.l);
    return sv(mulEt(E, f.a) + cross(r, fl), fl);
  }
  // Transpose of xm (maps a motion-space adjoint back to the parent): X^T y
  __host__ __device__ static inline SV xtm(const R* E, V3 r, SV y) { return xtf(E, r, y); }
  // Transpose of xtf (maps a force adjoint to the body): X y
  __host__ __device__ static inline SV xf(const R* E, V3 r, SV y) { return xm(E, r, y); }

  // Joint axis: bodies 0..6 about z, body 7 about x, body 8 about y.
  __host__ __device__ static inline int axis_of(int i) { return i == 7 ? 0 : (i == 8 ? 1 : 2); }
  __host__ __device__ static inline R comp(V3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }
  __host__ __device__ static inline V3 unit(int k) { return v3(k == 0 ? 1.f : 0.f, k == 1 ? 1.f : 0.f, k == 2 ? 1.f : 0.f); }

  // Body rotation: joint rotation (about the axis, by q) after the tree rotation.
  __host__ __device__ static inline void body_E(const ArmConst& K, int i, R cs, R sn, R* E) {
    const float* T = K.E[i];
    if (axis_of(i) == 2) {  // Rz(q)^T T
  #pragma unroll
      for (int k = 0; k < 3; ++k) {
        E[k] = cs * T[k] + sn * T[3 + k];
        E[3 + k] = -sn * T[k] + cs * T[3 + k];
        E[6 + k] = T[6 + k];
      }
    } else if (axis_of(i) == 0) {  // Rx(q)^T T
  #pragma unroll
      for (int k = 0; k < 3; ++k) {
        E[k] = T[k];
        E[3 + k] = cs * T[3 + k] + sn * T[6 + k];
        E[6 + k] = -sn * T[3 + k] + cs * T[6 + k];
      }
    } else {  // Ry(q)^T T
  #pragma unroll
      for (int k = 0; k < 3; ++k) {
        E[k] = cs * T[k] - sn * T[6 + k];
        E[3 + k] = T[3 + k];
        E[6 + k] = sn * T[k] + cs * T[6 + k];
      }
    }
  }

  // Rigid-body inertia applied to a motion vector, from (m, c, Ic):
  // I [w; v] = [Ic w + c x p; p] with p = m (v - c x w).
  template <class T>
  __host__ __device__ static inline SV rbi_mul(float m, V3 c, const T* Ic, SV x) {
    const V3 p = m * (x.l - cross(c, x.a));
    const V3 Iw = v3(Ic[0] * x.a.x + Ic[1] * x.a.y + Ic[2] * x.a.z, Ic[1] * x.a.x + Ic[3] * x.a.y + Ic[4] * x.a.z,
                     Ic[2] * x.a.x + Ic[4] * x.a.y + Ic[5] * x.a.z);
    return sv(Iw + cross(c, p), p);
  }
  // Point mass m at c: I [w; v] = [c x p; p], p = m (v - c x w).
  __host__ __device__ static inline SV pm_mul(float m, V3 c, SV x) {
    const V3 p = m * (x.l - cross(c, x.a));
    return sv(cross(c, p), p);
  }

  // Symmetric 6x6 as blocks A (sym 3: xx,xy,xz,yy,yz,zz), B (3x3 row-major), C (sym 3).
  struct Sym6 {
    R A[6], B[9], C[6];
  };
  __host__ __device__ static inline R s3(const R* S, int i, int j) {
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? S[b] : (a == 1 ? S[2 + b] : S[5]);
  }

  // Adds the rigid inertia of (m, c, Ic) to I: [[Ic + m cx cx^T, m cx], [m cx^T, m 1]].
  template <class T>
  __host__ __device__ static inline void add_rbi(Sym6& I, float m, V3 c, const T* Ic) {
    // cx cx^T = |c|^2 1 - c c^T
    const R cc = dot(c, c);
    I.A[0] += Ic[0] + m * (cc - c.x * c.x);
    I.A[1] += Ic[1] - m * c.x * c.y;
    I.A[2] += Ic[2] - m * c.x * c.z;
    I.A[3] += Ic[3] + m * (cc - c.y * c.y);
    I.A[4] += Ic[4] - m * c.y * c.z;
    I.A[5] += Ic[5] + m * (cc - c.z * c.z);
    // m skew(c)
    I.B[1] += -m * c.z; I.B[2] += m * c.y;
    I.B[3] += m * c.z;  I.B[5] += -m * c.x;
    I.B[6] += -m * c.y; I.B[7] += m * c.x;
    I.C[0] += m; I.C[3] += m; I.C[5] += m;
  }

  __host__ __device__ static inline SV sym6_mul(const Sym6& I, SV x) {
    const V3 w = x.a, v = x.l;
    const V3 Aw = v3(I.A[0] * w.x + I.A[1] * w.y + I.A[2] * w.z, I.A[1] * w.x + I.A[3] * w.y + I.A[4] * w.z,
                     I.A[2] * w.x + I.A[4] * w.y + I.A[5] * w.z);
    const V3 Bv = mulE(I.B, v);
    const V3 Btw = mulEt(I.B, w);
    const V3 Cv = v3(I.C[0] * v.x + I.C[1] * v.y + I.C[2] * v.z, I.C[1] * v.x + I.C[3] * v.y + I.C[4] * v.z,
                     I.C[2] * v.x + I.C[4] * v.y + I.C[5] * v.z);
    return sv(Aw + Bv, Btw + Cv);
  }

  // IA_parent += X^T Ia X for X = (E, r), R = skew(r):
  // with A' = E^T A E, B' = E^T B E, C' = E^T C E:
  // TL = A' - B' R + R B'^T - R C' R, TR = B' + R C', BR = C'.
  __host__ __device__ static __forceinline__ void add_xtix(Sym6& P, const Sym6& I, const R* E, V3 r) {
    R A[9], B[9], C[9];
  #pragma unroll
    for (int i = 0; i < 3; ++i)
  #pragma unroll
      for (int j = 0; j < 3; ++j) {
        R sa = 0.f, sb = 0.f, sc = 0.f;
  #pragma unroll
        for (int k = 0; k < 3; ++k)
  #pragma unroll
          for (int l = 0; l < 3; ++l) {
            const R e = E[3 * k + i] * E[3 * l + j];
            sa += e * s3(I.A, k, l);
            sb += e * I.B[3 * k + l];
            sc += e * s3(I.C, k, l);
          }
        A[3 * i + j] = sa;
        B[3 * i + j] = sb;
        C[3 * i + j] = sc;
      }
    // skew(r) rows
    const R Rs[9] = {0.f, -r.z, r.y, r.z, 0.f, -r.x, -r.y, r.x, 0.f};
    R BR[9], RC[9], RCR[9];
  #pragma unroll
    for (int i = 0; i < 3; ++i)
  #pragma unroll
      for (int j = 0; j < 3; ++j) {
        R s1 = 0.f, s2 = 0.f;
  #pragma unroll
        for (int k = 0; k < 3; ++k) {
          s1 += B[3 * i + k] * Rs[3 * k + j];
          s2 += Rs[3 * i + k] * C[3 * k + j];
        }
        BR[3 * i + j] = s1;
        RC[3 * i + j] = s2;
      }
  #pragma unroll
    for (int i = 0; i < 3; ++i)
  #pragma unroll
      for (int j = 0; j < 3; ++j) {
        R s = 0.f;
  #pragma unroll
        for (int k = 0; k < 3; ++k) s += RC[3 * i + k] * Rs[3 * k + j];
        RCR[3 * i + j] = s;
      }
    // TL(i,j) = A - BR - BR^T - RCR   (R B'^T = -(B' R)^T)
    const int si[6] = {0, 0, 0, 1, 1, 2}, sj[6] = {0, 1, 2, 1, 2, 2};
  #pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int i = si[e], j = sj[e];
      P.A[e] += A[3 * i + j] - BR[3 * i + j] - BR[3 * j + i] - RCR[3 * i + j];
      P.C[e] += C[3 * i + j];
    }
  #pragma unroll
    for (int e = 0; e < 9; ++e) P.B[e] += B[e] + RC[e];
  }

  // The box's centre of mass and inertia about it from theta (universal
  // joint): Ic in the order xx, xy, xz, yy, yz, zz.
  __host__ __device__ static inline void box_from_theta(const R* th, V3* c, R* Ic) {
    *c = v3(th[6], th[7], th[8]);
    Ic[0] = th[0]; Ic[1] = th[3]; Ic[2] = th[4];
    Ic[3] = th[1]; Ic[4] = th[5]; Ic[5] = th[2];
  }

  // Joint torque at time `time` (PD on the arm, viscous damping on the
  // passive axes).
  __host__ __device__ static inline R arm_tau(const ArmConst& K, const R* th, int i, R time, R q, R qd) {
    if (BOX == kHinge && i == 7) return -K.bh * qd;
    if (BOX == kUJoint && i >= 7) return -th[i + 2] * qd;
    if (BOX == kUJointWeights && i == 7) return -K.bh * qd;
    if (BOX == kUJointWeights && i == 8) return -K.b8 * qd;
    R sn, cs;
    sincos_r(K.om[i] * time + K.ph[i], &sn, &cs);
    const R qdes = K.qc[i] + K.amp[i] * sn;
    const R qddes = K.amp[i] * K.om[i] * cs;
    return K.kp[i] * (qdes - q) + K.kd[i] * (qddes - qd);
  }

  // Intermediates of one forward-dynamics evaluation kept for the reverse.
  struct ArmTape {
    R cs[NB], sn[NB];
    SV v[NB];   // body velocities
    SV a[NB];   // body accelerations (incl. S qdd)
    SV U[NB];   // IA S
    R invD[NB];
    R qdd[NB];
  };

  // Compiler-level memory barrier: the model constants are re-read (scalar
  // loads, cached) inside every step instead of being hoisted out of the step
  // loops into vector registers.
  __host__ __device__ static __forceinline__ void keep_consts_in_memory() {
  #if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" ::: "memory");
  #endif
  }

  // Articulated Body Algorithm (three passes over the chain).  The inward
  // pass carries only the child's contribution to the articulated inertia and
  // bias force; each body's rigid inertia is rebuilt on the fly.
  __host__ __device__ static __forceinline__ void arm_aba(const ArmConst& K, const R* th, const R* q, const R* qd,
                                          R time, ArmTape& T) {
    R u[NB];
    const V3 ca = v3(th[0], th[1], K.pm_z), cb = PM ? v3(th[2], th[3], K.pm_z) : v3(0.f, 0.f, 0.f);
    const float z0[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      sincos_r(q[i], &T.sn[i], &T.cs[i]);
      R E[9];
      body_E(K, i, T.cs[i], T.sn[i], E);
      const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
      const SV vj = sv(qd[i] * unit(axis_of(i)), v3(0.f, 0.f, 0.f));
      T.v[i] = (i == 0 ? sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f)) : xm(E, r, T.v[i - 1])) + vj;
    }
    Sym6 IAc;  // child's contribution X^T Ia X
    SV pAc = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
  #pragma unroll
    for (int e = 0; e < 6; ++e) { IAc.A[e] = 0.f; IAc.C[e] = 0.f; }
  #pragma unroll
    for (int e = 0; e < 9; ++e) IAc.B[e] = 0.f;
  #pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      keep_consts_in_memory();
      const int k = axis_of(i);
      Sym6 IA = IAc;
      SV h;
      if (BOX == kUJoint && i == 8) {
        V3 cm;
        R Icb[6];
        box_from_theta(th, &cm, Icb);
        add_rbi(IA, K.m[i], cm, Icb);
        h = rbi_mul(K.m[i], cm, Icb, T.v[i]);
      } else {
        const V3 cm = v3(K.c[i][0], K.c[i][1], K.c[i][2]);
        add_rbi(IA, K.m[i], cm, K.Ic[i]);
        h = rbi_mul(K.m[i], cm, K.Ic[i], T.v[i]);
      }
      if (PM && i == BOXB) {
        add_rbi(IA, K.pm_m, ca, z0);
        add_rbi(IA, K.pm_m, cb, z0);
        h = h + pm_mul(K.pm_m, ca, T.v[i]) + pm_mul(K.pm_m, cb, T.v[i]);
      }
      const SV pA = crf(T.v[i], h) + pAc;
      const SV U = sv(v3(s3(IA.A, 0, k), s3(IA.A, 1, k), s3(IA.A, 2, k)),
                      v3(IA.B[3 * k], IA.B[3 * k + 1], IA.B[3 * k + 2]));
      const R invD = recip(comp(U.a, k));
      u[i] = arm_tau(K, th, i, time, q[i], qd[i]) - comp(pA.a, k);
      T.U[i] = U;
      T.invD[i] = invD;
      if (i > 0) {
        Sym6 Ia = IA;
        const R Uw[3] = {U.a.x, U.a.y, U.a.z}, Uv[3] = {U.l.x, U.l.y, U.l.z};
        const int si[6] = {0, 0, 0, 1, 1, 2}, sj[6] = {0, 1, 2, 1, 2, 2};
  #pragma unroll
        for (int e = 0; e < 6; ++e) {
          Ia.A[e] -= Uw[si[e]] * Uw[sj[e]] * invD;
          Ia.C[e] -= Uv[si[e]] * Uv[sj[e]] * invD;
        }
  #pragma unroll
        for (int a2 = 0; a2 < 3; ++a2)
  #pragma unroll
          for (int b2 = 0; b2 < 3; ++b2) Ia.B[3 * a2 + b2] -= Uw[a2] * Uv[b2] * invD;
        const SV ci = crm(T.v[i], sv(qd[i] * unit(k), v3(0.f, 0.f, 0.f)));
        const SV pa = pA + sym6_mul(Ia, ci) + (u[i] * invD) * U;
        R E[9];
        body_E(K, i, T.cs[i], T.sn[i], E);
        const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
  #pragma unroll
        for (int e = 0; e < 6; ++e) { IAc.A[e] = 0.f; IAc.C[e] = 0.f; }
  #pragma unroll
        for (int e = 0; e < 9; ++e) IAc.B[e] = 0.f;
        add_xtix(IAc, Ia, E, r);
        pAc = xtf(E, r, pa);
      }
    }
    SV ap = sv(v3(0.f, 0.f, 0.f), v3(-K.g[0], -K.g[1], -K.g[2]));
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      R E[9];
      body_E(K, i, T.cs[i], T.sn[i], E);
      const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
      const SV ci = crm(T.v[i], sv(qd[i] * unit(axis_of(i)), v3(0.f, 0.f, 0.f)));
      const SV a1 = xm(E, r, ap) + ci;
      const R qdd = (u[i] - sdot(T.U[i], a1)) * T.invD[i];
      T.qdd[i] = qdd;
      T.a[i] = a1 + sv(qdd * unit(axis_of(i)), v3(0.f, 0.f, 0.f));
      ap = T.a[i];
    }
  }

  __host__ __device__ static __forceinline__ void arm_step(const ArmConst& K, const R* th, R time, R dt, R* q,
                                           R* qd) {
    keep_consts_in_memory();
    ArmTape T;
    arm_aba(K, th, q, qd, time, T);
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      qd[i] = qd[i] + dt * T.qdd[i];
      q[i] = q[i] + dt * qd[i];
    }
  }

  // Reverse of one Euler step.  (qb, qdb) enter as adjoints of the step's
  // outputs and leave as adjoints of its inputs; thb accumulates d/d theta.
  __host__ __device__ static __forceinline__ void arm_step_rev(const ArmConst& K, const R* th, const R* q, const R* qd,
                                               const ArmTape& T, R dt, R* qb, R* qdb, R* thb) {
    keep_consts_in_memory();
    // Euler: q' = q + dt qd', qd' = qd + dt qdd
    R qddb[NB];
    #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      qdb[i] += dt * qb[i];
      qddb[i] = dt * qdb[i];
    }
    // lambda = H^{-1} qddb: ABA with zero velocity and gravity (the child's
    // bias-force contribution is carried inward).
    R lam[NB], us[NB];
    {
      SV pAc = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
  #pragma unroll
      for (int i = NB - 1; i >= 0; --i) {
        keep_consts_in_memory();
        const int k = axis_of(i);
        us[i] = qddb[i] - comp(pAc.a, k);
        if (i > 0) {
          R E[9];
          body_E(K, i, T.cs[i], T.sn[i], E);
          const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
          pAc = xtf(E, r, pAc + (us[i] * T.invD[i]) * T.U[i]);
        }
      }
    }
    {
      SV ap = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
  #pragma unroll
      for (int i = 0; i < NB; ++i) {
        keep_consts_in_memory();
        R E[9];
        body_E(K, i, T.cs[i], T.sn[i], E);
        const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
        const SV a1 = xm(E, r, ap);
        lam[i] = (us[i] - sdot(T.U[i], a1)) * T.invD[i];
        ap = a1 + sv(lam[i] * unit(axis_of(i)), v3(0.f, 0.f, 0.f));
      }
    }
    // x_bar += -lambda^T dF/dx, F = ID - tau.  The tau part:
    // d tau / d q = -kp, d tau / d qd = -kd (arm), -b (passive axes), and
    // for the joint's friction coefficients d tau / d b = -qd.
    #pragma unroll
    for (int i = 0; i < 7; ++i) {
      keep_consts_in_memory();
      qb[i] += -K.kp[i] * lam[i];
      qdb[i] += -K.kd[i] * lam[i];
    }
    if constexpr (BOX == kHinge) {
      qdb[7] += -K.bh * lam[7];
    } else if constexpr (BOX == kUJointWeights) {
      qdb[7] += -K.bh * lam[7];
      qdb[8] += -K.b8 * lam[8];
    } else {
  #pragma unroll
      for (int i = 7; i < NB; ++i) {
        qdb[i] += -th[i + 2] * lam[i];
        thb[i + 2] += -lam[i] * qd[i];
      }
    }
    // ID part: reverse of RNEA with output seed mu = -lambda.  Total-force
    // adjoints first (outward; they do not depend on the forces):
    // ftb_i = S_i mu_i + X_i ftb_{i-1}.
    const V3 ca = v3(th[0], th[1], K.pm_z), cb = PM ? v3(th[2], th[3], K.pm_z) : v3(0.f, 0.f, 0.f);
    SV ftb[NB];
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      SV b = sv((-lam[i]) * unit(axis_of(i)), v3(0.f, 0.f, 0.f));
      if (i > 0) {
        R E[9];
        body_E(K, i, T.cs[i], T.sn[i], E);
        const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
        b = b + xf(E, r, ftb[i - 1]);
      }
      ftb[i] = b;
    }
    // Inward: total forces ft_i = f_i + X_{i+1}^T ft_{i+1} (carried), the
    // q dependence of X_i^T ft_i, and the reverse of the outward pass
    // (velocities, accelerations) with body-force adjoints ftb_i.
    SV ftc = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));  // X_{i+1}^T ft_{i+1}
    SV abar = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
    SV vbar = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
  #pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      keep_consts_in_memory();
      const SV fb = ftb[i];
      const SV v = T.v[i], a = T.a[i];
      const V3 ax = unit(axis_of(i));
      const SV sax = sv(ax, v3(0.f, 0.f, 0.f));
      // body force and total force
      const SV vxfb = crm(v, fb);
      SV Ia, h, Ifb, Ivxfb;
      if (BOX == kUJoint && i == 8) {
        V3 cm;
        R Icb[6];
        box_from_theta(th, &cm, Icb);
        Ia = rbi_mul(K.m[i], cm, Icb, a);
        h = rbi_mul(K.m[i], cm, Icb, v);
        Ifb = rbi_mul(K.m[i], cm, Icb, fb);
        Ivxfb = rbi_mul(K.m[i], cm, Icb, vxfb);
        // theta: fb . f = g(a, fb) + g(v, -v x fb) with g(x, y) = y . I x,
        // I x = [Ic x_w + c x p; p], p = m (x_l - c x x_w).  d g / d Ic is
        // the symmetric outer product of y_n and x_w; d g / d c as for the
        // hinge's point masses.
  #pragma unroll
        for (int term = 0; term < 2; ++term) {
          const SV x = term == 0 ? a : v;
          const SV y = term == 0 ? fb : sv(-vxfb.a, -vxfb.l);
          thb[0] += y.a.x * x.a.x;
          thb[1] += y.a.y * x.a.y;
          thb[2] += y.a.z * x.a.z;
          thb[3] += y.a.x * x.a.y + y.a.y * x.a.x;
          thb[4] += y.a.x * x.a.z + y.a.z * x.a.x;
          thb[5] += y.a.y * x.a.z + y.a.z * x.a.y;
          const V3 p = K.m[i] * (x.l - cross(cm, x.a));
          const V3 z = cross(y.a, cm) + y.l;
          const V3 gc = cross(p, y.a) - K.m[i] * cross(x.a, z);
          thb[6] += gc.x;
          thb[7] += gc.y;
          thb[8] += gc.z;
        }
      } else {
        const V3 cm = v3(K.c[i][0], K.c[i][1], K.c[i][2]);
        Ia = rbi_mul(K.m[i], cm, K.Ic[i], a);
        h = rbi_mul(K.m[i], cm, K.Ic[i], v);
        Ifb = rbi_mul(K.m[i], cm, K.Ic[i], fb);
        Ivxfb = rbi_mul(K.m[i], cm, K.Ic[i], vxfb);
      }
      if (PM && i == BOXB) {
        Ia = Ia + pm_mul(K.pm_m, ca, a) + pm_mul(K.pm_m, cb, a);
        h = h + pm_mul(K.pm_m, ca, v) + pm_mul(K.pm_m, cb, v);
        Ifb = Ifb + pm_mul(K.pm_m, ca, fb) + pm_mul(K.pm_m, cb, fb);
        Ivxfb = Ivxfb + pm_mul(K.pm_m, ca, vxfb) + pm_mul(K.pm_m, cb, vxfb);
        // theta: the point-mass positions (x, y) in f = I(c) a + v x* I(c) v.
        // With g(c; x, y) = y . I(c) x = y_n . (c x p) + y_f . p and
        // p = m (x_l - c x x_w):  dg/dc = p x y_n - m x_w x (y_n x c + y_f).
        // fb . f = g(c; a, fb) + g(c; v, -v x fb)  (fb . (v x* h) = -(v x fb) . h).
  #pragma unroll
        for (int w = 0; w < 2; ++w) {
          const V3 cp = w == 0 ? ca : cb;
          const float mm = K.pm_m;
          V3 gsum = v3(0.f, 0.f, 0.f);
  #pragma unroll
          for (int term = 0; term < 2; ++term) {
            const SV x = term == 0 ? a : v;
            const SV y = term == 0 ? fb : sv(-vxfb.a, -vxfb.l);
            const V3 p = mm * (x.l - cross(cp, x.a));
            const V3 z = cross(y.a, cp) + y.l;
            gsum = gsum + cross(p, y.a) - mm * cross(x.a, z);
          }
          thb[2 * w] += gsum.x;
          thb[2 * w + 1] += gsum.y;
        }
      }
      const SV ft = Ia + crf(v, h) + ftc;
      R E[9];
      body_E(K, i, T.cs[i], T.sn[i], E);
      const V3 r = v3(K.r[i][0], K.r[i][1], K.r[i][2]);
      if (i > 0) {
        // d/dq_i of ftb_{i-1} . X_i^T ft_i = (X_i ftb_{i-1}) . (S x* ft_i)
        qb[i] += sdot(xf(E, r, ftb[i - 1]), crf(sax, ft));
        ftc = xtf(E, r, ft);
      }
      // f = I a + v x* (I v):  a_bar += I fb;  v_bar += -crf(fb) h - I (v x fb)
      abar = abar + Ifb;
      vbar = vbar - crf(fb, h) - Ivxfb;
      // a_i = X_i a_{i-1} + v_i x (S qd_i) + S qdd_i (qdd held fixed)
      const SV sq = sv(qd[i] * ax, v3(0.f, 0.f, 0.f));
      vbar = vbar + crf(sq, abar);
      qdb[i] += -comp(crf(v, abar).a, axis_of(i));
      // v_i = X_i v_{i-1} + S qd_i
      qdb[i] += comp(vbar.a, axis_of(i));
      if (i > 0) {
        const SV ya = xm(E, r, T.a[i - 1]), yv = xm(E, r, T.v[i - 1]);
        // d/dq (abar . X a_prev) = -abar . (S x y)
        qb[i] += -sdot(abar, crm(sax, ya)) - sdot(vbar, crm(sax, yv));
        abar = xtm(E, r, abar);
        vbar = xtm(E, r, vbar);
      } else {
        // body 0: its parent is the fixed base (gravity as base acceleration)
        const SV ya = xm(E, r, sv(v3(0.f, 0.f, 0.f), v3(-K.g[0], -K.g[1], -K.g[2])));
        qb[0] += -sdot(abar, crm(sax, ya));
      }
    }
  }

  // Forward kinematics of the last body's frame (universal joint: the box):
  // body-to-world rotation R_i = R_{i-1} E_i^T and origin o_i = o_{i-1} +
  // R_{i-1} r_i.  Writes its origin and the points 1 m along its x, y, z
  // axes (12 numbers).
  __host__ __device__ static __forceinline__ void box_frame(const ArmConst& K, const R* q, R* x) {
    R Rw[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    V3 o = v3(0.f, 0.f, 0.f);
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      R sn, cs;
      sincos_r(q[i], &sn, &cs);
      R E[9];
      body_E(K, i, cs, sn, E);
      o = o + mulE(Rw, v3(K.r[i][0], K.r[i][1], K.r[i][2]));
      R Rn[9];
  #pragma unroll
      for (int a = 0; a < 3; ++a)
  #pragma unroll
        for (int b = 0; b < 3; ++b) Rn[3 * a + b] = Rw[3 * a] * E[3 * b] + Rw[3 * a + 1] * E[3 * b + 1] + Rw[3 * a + 2] * E[3 * b + 2];
  #pragma unroll
      for (int e = 0; e < 9; ++e) Rw[e] = Rn[e];
    }
    x[0] = o.x; x[1] = o.y; x[2] = o.z;
  #pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[3 + 3 * a] = o.x + Rw[a];
      x[4 + 3 * a] = o.y + Rw[3 + a];
      x[5 + 3 * a] = o.z + Rw[6 + a];
    }
  }

  // Observation term of one state (universal joint): returns
  // sum_c ((obs_c - x_c) w_c)^2 and adds d/dq of -1/2 of it to qb.  Every
  // observed point p sits on the box, so dp/dq_j = z_j x (p - o_j) with z_j
  // and o_j joint j's world axis and origin; with rt_p = w^2 (obs - p)
  // summed as A = sum p x rt_p and B = sum rt_p, the adjoint of q_j is
  // z_j . (A - o_j x B).
  __host__ __device__ static __forceinline__ R box_obs(const ArmConst& K, const R* q, const float* obs, const float* w,
                                                       R* qb) {
    R x[12];
    box_frame(K, q, x);
    R ss = 0.f;
    V3 A = v3(0.f, 0.f, 0.f), B = v3(0.f, 0.f, 0.f);
  #pragma unroll
    for (int pnt = 0; pnt < 4; ++pnt) {
      const int c0 = 3 * pnt;
      const R r0 = (obs[c0] - x[c0]) * w[c0], r1 = (obs[c0 + 1] - x[c0 + 1]) * w[c0 + 1],
              r2 = (obs[c0 + 2] - x[c0 + 2]) * w[c0 + 2];
      ss += r0 * r0 + r1 * r1 + r2 * r2;
      const V3 rt = v3(r0 * w[c0], r1 * w[c0 + 1], r2 * w[c0 + 2]);
      A = A + cross(v3(x[c0], x[c0 + 1], x[c0 + 2]), rt);
      B = B + rt;
    }
    R Rw[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    V3 o = v3(0.f, 0.f, 0.f);
  #pragma unroll
    for (int i = 0; i < NB; ++i) {
      keep_consts_in_memory();
      R sn, cs;
      sincos_r(q[i], &sn, &cs);
      R E[9];
      body_E(K, i, cs, sn, E);
      o = o + mulE(Rw, v3(K.r[i][0], K.r[i][1], K.r[i][2]));
      R Rn[9];
  #pragma unroll
      for (int a = 0; a < 3; ++a)
  #pragma unroll
        for (int b = 0; b < 3; ++b) Rn[3 * a + b] = Rw[3 * a] * E[3 * b] + Rw[3 * a + 1] * E[3 * b + 1] + Rw[3 * a + 2] * E[3 * b + 2];
  #pragma unroll
      for (int e = 0; e < 9; ++e) Rw[e] = Rn[e];
      const int k = axis_of(i);
      const V3 z = v3(Rw[k], Rw[3 + k], Rw[6 + k]);
      qb[i] += dot(z, A - cross(o, B));
    }
    return ss;
  }
};

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
    const float a = j[0], al = j[1], d = j[2];
    float sa, ca;
    sincosf(al, &sa, &ca);
    const float E[9] = {1.f, 0.f, 0.f, 0.f, ca, sa, 0.f, -sa, ca};  // Rot_x(alpha)^T
    for (int e = 0; e < 9; ++e) K->E[i][e] = E[e];
    K->r[i][0] = a;
    K->r[i][1] = -d * sa;
    K->r[i][2] = d * ca;
    K->m[i] = j[3];
    K->c[i][0] = j[4]; K->c[i][1] = j[5]; K->c[i][2] = j[6];
    K->Ic[i][0] = j[7]; K->Ic[i][1] = 0.f; K->Ic[i][2] = 0.f;
    K->Ic[i][3] = j[8]; K->Ic[i][4] = 0.f; K->Ic[i][5] = j[9];
    K->kp[i] = j[10]; K->kd[i] = j[11]; K->qc[i] = j[12];
    K->amp[i] = j[13]; K->om[i] = j[14]; K->ph[i] = j[15];
  }
  const float* h = raw + 3 + 16 * 7;
  for (int b = 7; b < kArmMaxBodies; ++b) {
    for (int e = 0; e < 9; ++e) K->E[b][e] = (e % 4 == 0) ? 1.f : 0.f;
    for (int d = 0; d < 3; ++d) K->r[b][d] = K->c[b][d] = 0.f;
    for (int e = 0; e < 6; ++e) K->Ic[b][e] = 0.f;
    K->m[b] = 0.f;
  }
  K->r[7][2] = h[0];
  K->bh = K->b8 = K->pm_m = K->pm_z = 0.f;
  if (mount == kUJoint) {
    K->m[8] = h[1];  // the box; its centre of mass and inertia come from theta
    return;
  }
  if (mount == kUJointWeights) {
    K->m[8] = h[1];
    K->c[8][0] = h[2]; K->c[8][1] = h[3]; K->c[8][2] = h[4];
    K->Ic[8][0] = h[5]; K->Ic[8][1] = h[8]; K->Ic[8][2] = h[9];
    K->Ic[8][3] = h[6]; K->Ic[8][4] = h[10]; K->Ic[8][5] = h[7];
    K->bh = h[11];
    K->b8 = h[12];
    K->pm_m = h[13];
    K->pm_z = h[14];
    return;
  }
  K->bh = h[1];
  K->m[7] = h[2];
  K->c[7][0] = h[3]; K->c[7][1] = h[4]; K->c[7][2] = h[5];
  K->Ic[7][0] = h[6]; K->Ic[7][1] = 0.f; K->Ic[7][2] = 0.f;
  K->Ic[7][3] = h[7]; K->Ic[7][4] = 0.f; K->Ic[7][5] = h[8];
  K->pm_m = h[9];
  K->pm_z = h[10];
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__device__ inline const ArmConst* arm_const_of(char* ws, uint64_t off) {
  return reinterpret_cast<const ArmConst*>(ws + off);
}

__global__ void arm_setup_kernel(JobMap map, const pds_job* __restrict__ jobs, char* __restrict__ ws) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  if (threadIdx.x == 0)
    arm_setup(J.consts, reinterpret_cast<ArmConst*>(ws + map.ws_off[e]),
              J.model == PDS_MODEL_ARM_UJOINT ? kUJoint : (J.model == PDS_MODEL_ARM_UJOINT_WEIGHTS ? kUJointWeights : kHinge));
}

struct AUnit {
  int i, k, j;
};
__device__ inline AUnit aunit_of(const pds_job& J, int u) {
  AUnit r;
  r.i = u % J.N;
  const int kj = u / J.N;
  r.k = kj / J.n_s;
  r.j = kj % J.n_s;
  return r;
}
template <int DS>
__device__ inline const float* astart_ptr(const pds_job& J, const AUnit& w) {
  if (w.j == 0) return J.s0 + (size_t)w.k * DS;
  return J.S + (((size_t)w.i * J.K + w.k) * (J.n_s - 1) + (w.j - 1)) * DS;
}

// Observation term of the state after a step: -1/2 sum ((obs - x) w)^2
// without the constant; with qb non-null, its q-adjoint is added there.
template <int BOX>
__device__ __forceinline__ float arm_obs_term(const ArmConst& K, const float* q, const float* obs_row,
                                              const float* w, float* qb) {
  if (BOX == kHinge) {
    const float r = (obs_row[0] - q[7]) * w[0];
    if (qb) qb[7] += r * w[0];
    return r * r;
  }
  float tmp[ArmShape<BOX>::NB];
  float* acc = qb;
  if (!qb) {
    for (int i = 0; i < ArmShape<BOX>::NB; ++i) tmp[i] = 0.f;
    acc = tmp;
  }
  return ArmMath<float, BOX>::box_obs(K, q, obs_row, w, acc);
}

template <int BOX>
__device__ inline double arm_obs_log_norm(const pds_job& J) {
  double c = 0.0;
  for (int d = 0; d < ArmShape<BOX>::DX; ++d) c += log((double)J.w_x[d]) - 0.91893853320467274178;
  return c;
}

template <int BOX>
__global__ void __launch_bounds__(kWave) arm_forward_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                            char* ws, int with_ll) {
  using AM = ArmMath<float, BOX>;
  constexpr int NB = ArmShape<BOX>::NB, DS = ArmShape<BOX>::DS, M = ArmShape<BOX>::M, DX = ArmShape<BOX>::DX;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const ArmConst& K = *arm_const_of(ws, map.ws_off[e]);
  const int U = J.N * J.K * J.n_s;
  const int u = (blockIdx.x - map.begin[e]) * kWave + threadIdx.x;
  if (u >= U) return;
  const AUnit w = aunit_of(J, u);
  float th[M];
  for (int m = 0; m < M; ++m) th[m] = J.theta[(size_t)w.i * M + m];
  const float* st = astart_ptr<DS>(J, w);
  float q[NB], qd[NB];
  for (int d = 0; d < NB; ++d) { q[d] = st[d]; qd[d] = st[NB + d]; }
  const float dt = J.dt;
  const int t0 = w.j * J.h;
  const float* obs = J.obs + ((size_t)w.k * J.T + t0) * DX;
  float* traj = J.traj ? J.traj + (((size_t)w.i * J.K + w.k) * J.T + t0) * DS : nullptr;
  float wx[DX];
  for (int d = 0; d < DX; ++d) wx[d] = J.w_x[d];
  double ll = 0.0;
  for (int s = 0; s < J.h; ++s) {
    AM::arm_step(K, th, (float)(t0 + s) * dt, dt, q, qd);
    if (with_ll) ll -= 0.5 * (double)arm_obs_term<BOX>(K, q, obs + (size_t)s * DX, wx, nullptr);
    if (traj)
      for (int d = 0; d < NB; ++d) { traj[s * DS + d] = q[d]; traj[s * DS + NB + d] = qd[d]; }
  }
  const size_t iu = ((size_t)w.i * J.K + w.k) * J.n_s + w.j;
  float* es = J.end_states + iu * DS;
  bool bad = false;
  for (int d = 0; d < NB; ++d) {
    es[d] = q[d];
    es[NB + d] = qd[d];
    bad |= !isfinite(q[d]) || !isfinite(qd[d]);
  }
  if (with_ll) {
    ll += (double)J.h * arm_obs_log_norm<BOX>(J);
    if (w.j + 1 < J.n_s) {
      const float* sn = J.S + (((size_t)w.i * J.K + w.k) * (J.n_s - 1) + w.j) * DS;
      double g = 0.0;
      for (int d = 0; d < NB; ++d) {
        const float e0 = (sn[d] - q[d]) * J.u[d];
        const float e1 = (sn[NB + d] - qd[d]) * J.u[NB + d];
        g += (double)e0 * e0 + (double)e1 * e1;
      }
      g /= (double)J.sigma_def * J.sigma_def;
      J.gdef[((size_t)w.i * J.K + w.k) * (J.n_s - 1) + w.j] = g;
      if (J.lik == PDS_LIK_DEFECT) ll += -0.5 * g + defect_log_norm(J);
    }
    J.ll_win[iu] = ll;
    bad |= !isfinite(ll);
  }
  if (bad && J.flags) atomicOr(&J.flags[w.i], 1);
}


// Adjoint kernel: one lane per unit, both adjoint channels.  The forward
// pass stores every state of the window in the job's workspace (layout
// [wave][step][component][lane], so each access is one coalesced row); the
// reverse sweep reads them back and recomputes only the step's own ABA
// intermediates.  No LDS: occupancy is set by registers alone.
template <int BOX>
__global__ void __launch_bounds__(kWave) arm_adjoint_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                            char* ws) {
  using AM = ArmMath<float, BOX>;
  constexpr int NB = ArmShape<BOX>::NB, DS = ArmShape<BOX>::DS, M = ArmShape<BOX>::M, DX = ArmShape<BOX>::DX;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const ArmConst& K = *arm_const_of(ws, map.ws_off[e]);
  const int U = J.N * J.K * J.n_s;
  const int lane = threadIdx.x;
  const int u = (blockIdx.x - map.begin[e]) * kWave + lane;
  if (u >= U) return;
  const WsLayout L = ws_layout(J);
  char* base = ws + map.ws_off[e];
  double* gth_obs = reinterpret_cast<double*>(base + L.gth_obs);
  double* gth_con = reinterpret_cast<double*>(base + L.gth_con);
  float* gs_obs = reinterpret_cast<float*>(base + L.gs_obs);
  float* gs_con = reinterpret_cast<float*>(base + L.gs_con);
  const AUnit w = aunit_of(J, u);
  float th[M];
  for (int m = 0; m < M; ++m) th[m] = J.theta[(size_t)w.i * M + m];
  const float* st = astart_ptr<DS>(J, w);
  float q[NB], qd[NB];
  for (int d = 0; d < NB; ++d) { q[d] = st[d]; qd[d] = st[NB + d]; }
  const float dt = J.dt;
  const int h = J.h;
  const int t0 = w.j * h;
  const float* obs = J.obs + ((size_t)w.k * J.T + t0) * DX;
  float wx[DX];
  for (int d = 0; d < DX; ++d) wx[d] = J.w_x[d];
  float* states = reinterpret_cast<float*>(base + L.arm_states) + (size_t)(u / kWave) * (h + 1) * DS * kWave;
  auto slot = [&](int s, int d) -> float& { return states[((size_t)s * DS + d) * kWave + lane]; };

  double ll = 0.0;
  for (int s = 0; s < h; ++s) {
    for (int d = 0; d < NB; ++d) { slot(s, d) = q[d]; slot(s, NB + d) = qd[d]; }
    AM::arm_step(K, th, (float)(t0 + s) * dt, dt, q, qd);
    ll -= 0.5 * (double)arm_obs_term<BOX>(K, q, obs + (size_t)s * DX, wx, nullptr);
  }
  for (int d = 0; d < NB; ++d) { slot(h, d) = q[d]; slot(h, NB + d) = qd[d]; }
  ll += (double)h * arm_obs_log_norm<BOX>(J);
  const size_t iu = ((size_t)w.i * J.K + w.k) * J.n_s + w.j;
  float* es = J.end_states + iu * DS;
  bool bad = false;
  for (int d = 0; d < NB; ++d) {
    es[d] = q[d];
    es[NB + d] = qd[d];
    bad |= !isfinite(q[d]) || !isfinite(qd[d]);
  }

  float qb_o[NB], qdb_o[NB], qb_c[NB], qdb_c[NB];
  for (int d = 0; d < NB; ++d) { qb_o[d] = qdb_o[d] = qb_c[d] = qdb_c[d] = 0.f; }
  if (w.j + 1 < J.n_s) {
    const size_t id = ((size_t)w.i * J.K + w.k) * (J.n_s - 1) + w.j;
    const float* sn = J.S + id * DS;
    float e0[NB], e1[NB];
    double g = 0.0;
    for (int d = 0; d < NB; ++d) {
      e0[d] = (sn[d] - q[d]) * J.u[d];
      e1[d] = (sn[NB + d] - qd[d]) * J.u[NB + d];
      g += (double)e0[d] * e0[d] + (double)e1[d] * e1[d];
    }
    const double inv_s2 = 1.0 / ((double)J.sigma_def * J.sigma_def);
    g *= inv_s2;
    J.gdef[id] = g;
    const bool in_lik = J.lik == PDS_LIK_DEFECT;
    if (in_lik) ll += -0.5 * g + defect_log_norm(J);
    const double seed =
        J.seed_gdef ? J.seed_gdef[id] : (in_lik ? 0.0 : (double)J.lam_def[id] + (double)J.c * g);
    // d g / d s_end = -2 e u / sigma^2; in the likelihood, d(-g/2) / d s_end = e u / sigma^2
    const float sc = (float)(-2.0 * seed * inv_s2);
    const float so = in_lik ? (float)inv_s2 : 0.f;
    for (int d = 0; d < NB; ++d) {
      qb_o[d] = so * e0[d] * J.u[d];
      qdb_o[d] = so * e1[d] * J.u[NB + d];
      qb_c[d] = sc * e0[d] * J.u[d];
      qdb_c[d] = sc * e1[d] * J.u[NB + d];
    }
  }
  bad |= !isfinite(ll);
  J.ll_win[iu] = ll;
  double gm_o[M], gm_c[M];
  for (int m = 0; m < M; ++m) gm_o[m] = gm_c[m] = 0.0;
  for (int s = h - 1; s >= 0; --s) {
    {
      float qn[NB];
      for (int d = 0; d < NB; ++d) qn[d] = slot(s + 1, d);
      arm_obs_term<BOX>(K, qn, obs + (size_t)s * DX, wx, qb_o);
    }
    float qs[NB], qds[NB];
    for (int d = 0; d < NB; ++d) { qs[d] = slot(s, d); qds[d] = slot(s, NB + d); }
    typename AM::ArmTape T;
    const float time = (float)(t0 + s) * dt;
    AM::keep_consts_in_memory();
    AM::arm_aba(K, th, qs, qds, time, T);
    float tb[M];
    for (int m = 0; m < M; ++m) tb[m] = 0.f;
    AM::arm_step_rev(K, th, qs, qds, T, dt, qb_o, qdb_o, tb);
    for (int m = 0; m < M; ++m) gm_o[m] += (double)tb[m];
    for (int m = 0; m < M; ++m) tb[m] = 0.f;
    AM::arm_step_rev(K, th, qs, qds, T, dt, qb_c, qdb_c, tb);
    for (int m = 0; m < M; ++m) gm_c[m] += (double)tb[m];
  }
  for (int m = 0; m < M; ++m) {
    gth_obs[iu * M + m] = gm_o[m];
    gth_con[iu * M + m] = gm_c[m];
    bad |= !isfinite(gm_o[m]) || !isfinite(gm_c[m]);
  }
  for (int d = 0; d < NB; ++d) {
    gs_obs[iu * DS + d] = qb_o[d];
    gs_obs[iu * DS + NB + d] = qdb_o[d];
    gs_con[iu * DS + d] = qb_c[d];
    gs_con[iu * DS + NB + d] = qdb_c[d];
  }
  if (bad && J.flags) atomicOr(&J.flags[w.i], 2);
}

}  // namespace

static_assert(sizeof(ArmConst) <= kArmConstBytes, "ArmConst must fit its workspace region");

hipError_t launch_arm_setup(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(arm_setup_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_arm_forward(const JobMap& map, int mount, const pds_job* d_jobs, char* ws, int grid,
                              bool with_ll, hipStream_t s) {
  const int ll = with_ll ? 1 : 0;
  if (mount == kUJoint)
    hipLaunchKernelGGL(arm_forward_kernel<kUJoint>, dim3(grid), dim3(kWave), 0, s, map, d_jobs, ws, ll);
  else if (mount == kUJointWeights)
    hipLaunchKernelGGL(arm_forward_kernel<kUJointWeights>, dim3(grid), dim3(kWave), 0, s, map, d_jobs, ws, ll);
  else
    hipLaunchKernelGGL(arm_forward_kernel<kHinge>, dim3(grid), dim3(kWave), 0, s, map, d_jobs, ws, ll);
  return hipGetLastError();
}

hipError_t launch_arm_adjoint(const JobMap& map, int mount, const pds_job* d_jobs, char* ws, int grid,
                              hipStream_t s) {
  if (mount == kUJoint)
    hipLaunchKernelGGL(arm_adjoint_kernel<kUJoint>, dim3(grid), dim3(kWave), 0, s, map, d_jobs, ws);
  else if (mount == kUJointWeights)
    hipLaunchKernelGGL(arm_adjoint_kernel<kUJointWeights>, dim3(grid), dim3(kWave), 0, s, map, d_jobs, ws);
  else
    hipLaunchKernelGGL(arm_adjoint_kernel<kHinge>, dim3(grid), dim3(kWave), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

// Algorithmic FLOPs of one arm time step: the forward step (ABA + Euler +
// the observation residuals and their FP64 accumulation) and the reverse
// step of one adjoint channel (with its observation seed and the FP64
// accumulation of the parameter adjoints), from the same step functions
// the kernels run, instantiated with the counting scalar.
template <int BOX>
static void count_arm(double* fwd, double* rev, double* transc) {
  using CM = ArmMath<Counted, BOX>;
  constexpr int NB = ArmShape<BOX>::NB, M = ArmShape<BOX>::M;
  ArmConst K;
  std::vector<float> raw(130, 0.5f);  // the longest consts layout
  raw[0] = 0.f;
  raw[1] = 0.f;
  raw[2] = -9.81f;
  arm_setup(raw.data(), &K, BOX);
  Counted th[11];
  for (int m = 0; m < 11; ++m) th[m] = Counted(0.01f * (m + 1));
  Counted q[NB], qd[NB], qb[NB], qdb[NB], thb[M];
  for (int i = 0; i < NB; ++i) {
    q[i] = Counted(0.1f * i);
    qd[i] = Counted(0.05f);
    qb[i] = Counted(1.f);
    qdb[i] = Counted(1.f);
  }
  const float obs[12] = {0.1f, 0.2f, 0.3f, 1.f, 0.2f, 0.3f, 0.1f, 1.f, 0.3f, 0.1f, 0.2f, 1.f};
  const float w[12] = {100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f};
  g_tally = FlopTally();
  typename CM::ArmTape T;
  CM::arm_aba(K, th, q, qd, Counted(0.5f), T);
  for (int i = 0; i < NB; ++i) {
    qd[i] = qd[i] + Counted(0.004f) * T.qdd[i];
    q[i] = q[i] + Counted(0.004f) * qd[i];
  }
  if (BOX != kHinge) {
    Counted x[12];
    CM::box_frame(K, q, x);  // the kinematics of the observation, sin/cos included
  }
  // + the residuals (x - obs) w, their squares and the FP64 accumulation
  *fwd = g_tally.flops + (BOX != kHinge ? 12 * 4 + 2 : 4.0);
  *transc = g_tally.transc;
  g_tally = FlopTally();
  CM::arm_step_rev(K, th, q, qd, T, Counted(0.004f), qb, qdb, thb);
  const double rev_step = g_tally.flops;
  double obs_rev = 2.0;  // hinge: the observation seed r w
  if (BOX != kHinge) {
    g_tally = FlopTally();
    Counted qb2[NB];
    for (int i = 0; i < NB; ++i) qb2[i] = Counted(0.f);
    CM::box_obs(K, q, obs, w, qb2);
    obs_rev = g_tally.flops;
  }
  *rev = rev_step + obs_rev + M;  // + the FP64 accumulation of the M parameter adjoints
}

void count_arm_flops(int mount, double* fwd, double* rev, double* transc) {
  if (mount == kUJoint)
    count_arm<kUJoint>(fwd, rev, transc);
  else if (mount == kUJointWeights)
    count_arm<kUJointWeights>(fwd, rev, transc);
  else
    count_arm<kHinge>(fwd, rev, transc);
}

}  // namespace pds
