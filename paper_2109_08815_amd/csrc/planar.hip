// Window rollouts and their reverse-mode adjoint for planar chains
// (revolute joints about z, point masses on massless links).
//
// Forward dynamics is the Articulated Body Algorithm (App. B-A) written in
// planar spatial vectors: a motion vector is (w, vx, vy), a force vector
// (n, fx, fy), and an articulated inertia is a symmetric 3x3 stored as its
// six unique entries [00, 01, 02, 11, 12, 22].  Each step is the
// semi-implicit Euler update of App. B-A eq. dynamics.  Body i's frame sits
// on joint i and turns with q_i; its parent-to-body transform rotates by q_i
// after translating by L_i = l_{i-1} along the parent's -y axis (L_0 = 0).
//
// One lane owns one window unit (particle i, trajectory k, window j): the
// whole window runs in registers, and only window start states are read
// from memory.  The adjoint kernel keeps the state at the start of every
// segment of B steps (checkpoints) and the states of the segment being
// reversed in LDS, laid out [slot][component][lane] so lanes hit distinct
// banks; each reverse step recomputes its ABA intermediates from the stored
// state (recompute inside the window, nothing but start states in HBM).
//
// The reverse of one ABA evaluation is written by hand statement by
// statement (reverse order of passes 3, 2, 1).  Two adjoint channels share
// the primal recompute: the observation channel, seeded at every step with
// d l / d x = r * w (unit trajectory weight), and the constraint channel,
// seeded at the window end with seed_gdef * d g_def / d s_end.  Per-window
// sums over steps are accumulated in FP64.
#include <cmath>

#include "common.h"
#include "sincos.h"
#include "flop_count.h"

namespace pds {
namespace {

__host__ __device__ inline void sincos_r(float x, float* sn, float* cs) { sincos_fast(x, sn, cs); }
// FP64 versions for host-side checks of the step functions.
__host__ __device__ inline void sincos_r(double x, double* sn, double* cs) {
  *sn = sin(x);
  *cs = cos(x);
}

// A load through a global-memory pointer.  The job's arrays reach the
// kernels as generic pointers, whose loads also count against the LDS wait
// counter; typed as global they count only against the vector-memory one,
// in order, so a load issued a step ahead is not waited for by the next LDS
// access or by older loads.
__device__ __forceinline__ float ldg(const float* p) {
  return *(const __attribute__((address_space(1))) float*)p;
}

// Link parameters.  Point-mass chain (PDS_MODEL_PLANAR): mass m_i at the
// tip of a massless rod of length l_i, joint i+1 at that tip.  Rigid chain
// (PDS_MODEL_PLANAR_RIGID, RIGID = true): link i has mass m_i, rotational
// inertia I_i about its centre of mass at (cx_i, cy_i) in the link frame,
// joint friction b_i, and joint i sits at (0, -L_i) in the frame of link
// i-1 (L_0 unused); the point-mass chain is the rigid one with c = (0, -l),
// I = 0 and L_i = l_{i-1}.
template <int NB, class R = float>
struct Planar {
  R m[NB], l[NB], b[NB];
  R I[NB], cx[NB], cy[NB], L[NB];  // rigid chain only
  R gx, gy;
};

// theta layout.  Point masses: (m_1..m_n, l_1..l_n).  Rigid chain: link 1
// (m, I, cx, cy, b), then per further link (L, m, I, cx, cy, b): 6 n - 1.
template <int NB, bool RIGID>
struct PlanarParams {
  static constexpr int M = RIGID ? 6 * NB - 1 : 2 * NB;
  __host__ __device__ static constexpr int base(int i) { return i == 0 ? 0 : 5 + 6 * (i - 1); }
  __host__ __device__ static constexpr int L(int i) { return base(i); }  // i >= 1
  __host__ __device__ static constexpr int m(int i) { return RIGID ? base(i) + (i > 0) : i; }
  __host__ __device__ static constexpr int l(int i) { return NB + i; }  // point masses
  __host__ __device__ static constexpr int I(int i) { return base(i) + (i > 0) + 1; }
  __host__ __device__ static constexpr int cx(int i) { return base(i) + (i > 0) + 2; }
  __host__ __device__ static constexpr int cy(int i) { return base(i) + (i > 0) + 3; }
  __host__ __device__ static constexpr int b(int i) { return base(i) + (i > 0) + 4; }
};

// Offset of joint i (i >= 1) along the parent's -y axis.
template <int NB, bool RIGID, class R>
__host__ __device__ __forceinline__ R joint_offset(const Planar<NB, R>& P, int i) {
  if constexpr (RIGID) return P.L[i];
  else return P.l[i - 1];
}

// Intermediates of one ABA evaluation needed by its reverse.
template <int NB, class R = float>
struct Tape {
  R cs[NB], sn[NB];
  R v[NB][3];
  R IA[NB][6];  // final articulated inertia
  R pA[NB][3];  // final bias force
  R invD[NB], u[NB];
  R ap[NB][3];  // X a_parent + c
  R qdd[NB];
};

// Two point-mass links in closed form.  The forward dynamics of the chain
// are unique, so for n_dof = 2 they can be written out in joint
// coordinates instead of running the ABA passes: with phi_1 = q_1,
// phi_2 = q_1 + q_2, a = (m_1 + m_2) l_1^2, b = m_2 l_2^2,
// c = m_2 l_1 l_2 cos q_2 and s~ = m_2 l_1 l_2 sin q_2 the joint-space
// inertia is H = [[a + b + 2c, b + c], [b + c, b]], and H qdd = r with
//   r_1 = -b_1 qd_1 + s~ (2 qd_1 qd_2 + qd_2^2) + (m_1 + m_2) l_1 e_1 + m_2 l_2 e_2
//   r_2 = -b_2 qd_2 - s~ qd_1^2 + m_2 l_2 e_2,
// e_i = g . (cos phi_i, sin phi_i) (Coriolis and centripetal terms,
// gravity, joint damping).  A quarter of the ABA's arithmetic.  The tape
// keeps sin/cos of q_1, q_2, qdd and 1 / det H.
template <class R>
__host__ __device__ __forceinline__ void dp2_forward(const Planar<2, R>& P, const R* q, const R* qd, Tape<2, R>& T) {
  sincos_r(q[0], &T.sn[0], &T.cs[0]);
  sincos_r(q[1], &T.sn[1], &T.cs[1]);
  const R s1 = T.sn[0], c1 = T.cs[0], s2 = T.sn[1], c2 = T.cs[1];
  const R s12 = s1 * c2 + c1 * s2, c12 = c1 * c2 - s1 * s2;
  const R m1 = P.m[0], m2 = P.m[1], l1 = P.l[0], l2 = P.l[1];
  const R k = m2 * l1 * l2;
  const R cc = k * c2, st = k * s2;
  const R a = (m1 + m2) * l1 * l1, bb = m2 * l2 * l2;
  const R H11 = a + bb + 2.f * cc, H12 = bb + cc, H22 = bb;
  const R e1 = P.gx * c1 + P.gy * s1, e2 = P.gx * c12 + P.gy * s12;
  const R g2 = m2 * l2 * e2;
  const R r1 = -P.b[0] * qd[0] + st * (2.f * qd[0] * qd[1] + qd[1] * qd[1]) + (m1 + m2) * l1 * e1 + g2;
  const R r2 = -P.b[1] * qd[1] - st * qd[0] * qd[0] + g2;
  const R idet = recip(H11 * H22 - H12 * H12);
  T.invD[0] = idet;
  T.qdd[0] = (H22 * r1 - H12 * r2) * idet;
  T.qdd[1] = (H11 * r2 - H12 * r1) * idet;
}

// Reverse of dp2_forward: qdd = H^{-1} r, so with lambda = H^{-1} qddb
// (H is symmetric) every input x gets lambda . (dr/dx - (dH/dx) qdd).
template <class R>
__host__ __device__ __forceinline__ void dp2_reverse(const Planar<2, R>& P, const R* qd, const Tape<2, R>& T,
                                                     const R* qddb, R* qb, R* qdb, R* thb) {
  const R s1 = T.sn[0], c1 = T.cs[0], s2 = T.sn[1], c2 = T.cs[1];
  const R s12 = s1 * c2 + c1 * s2, c12 = c1 * c2 - s1 * s2;
  const R m1 = P.m[0], m2 = P.m[1], l1 = P.l[0], l2 = P.l[1];
  const R k = m2 * l1 * l2;
  const R cc = k * c2, st = k * s2;
  const R bb = m2 * l2 * l2;
  const R H11 = (m1 + m2) * l1 * l1 + bb + 2.f * cc, H12 = bb + cc, H22 = bb;
  const R idet = T.invD[0];
  const R lam1 = (H22 * qddb[0] - H12 * qddb[1]) * idet;
  const R lam2 = (H11 * qddb[1] - H12 * qddb[0]) * idet;
  const R x1 = T.qdd[0], x2 = T.qdd[1];
  // lambda^T (dH/dx) qdd = mu11 dH11 + mu12 dH12 + mu22 dH22
  const R mu11 = lam1 * x1, mu12 = lam1 * x2 + lam2 * x1, mu22 = lam2 * x2;
  const R e1 = P.gx * c1 + P.gy * s1, e2 = P.gx * c12 + P.gy * s12;
  const R f1 = P.gy * c1 - P.gx * s1, f2 = P.gy * c12 - P.gx * s12;  // d e_i / d phi_i
  const R w1 = qd[0], w2 = qd[1];
  const R cor = 2.f * w1 * w2 + w2 * w2;  // r_1's factor of s~
  const R lsum = lam1 + lam2;
  // joint angles
  qb[0] += lam1 * (m1 + m2) * l1 * f1 + lsum * m2 * l2 * f2;
  qb[1] += lam1 * cc * cor - lam2 * cc * w1 * w1 + lsum * m2 * l2 * f2 + st * (2.f * mu11 + mu12);
  // joint velocities
  qdb[0] += lam1 * (-P.b[0] + 2.f * st * w2) - lam2 * 2.f * st * w1;
  qdb[1] += lam1 * 2.f * st * (w1 + w2) - lam2 * P.b[1];
  // theta = (m_1, m_2, l_1, l_2)
  const R hl = l1 * l2;
  thb[0] += lam1 * l1 * e1 - mu11 * l1 * l1;
  thb[1] += lam1 * (hl * s2 * cor + l1 * e1 + l2 * e2) + lam2 * (l2 * e2 - hl * s2 * w1 * w1) -
            (mu11 * (l1 * l1 + l2 * l2 + 2.f * hl * c2) + mu12 * (l2 * l2 + hl * c2) + mu22 * l2 * l2);
  thb[2] += lam1 * (m2 * l2 * s2 * cor + (m1 + m2) * e1) - lam2 * m2 * l2 * s2 * w1 * w1 -
            (mu11 * (2.f * (m1 + m2) * l1 + 2.f * m2 * l2 * c2) + mu12 * m2 * l2 * c2);
  thb[3] += lam1 * (m2 * l1 * s2 * cor + m2 * e2) + lam2 * (m2 * e2 - m2 * l1 * s2 * w1 * w1) -
            (mu11 * (2.f * m2 * l2 + 2.f * m2 * l1 * c2) + mu12 * (2.f * m2 * l2 + m2 * l1 * c2) + mu22 * 2.f * m2 * l2);
}

// Articulated Body Algorithm, planar form.  Fills the tape; qdd in T.qdd.
template <int NB, class R = float, bool RIGID = false>
__host__ __device__ __forceinline__ void aba(const Planar<NB, R>& P, const R* q, const R* qd, Tape<NB, R>& T) {
  if constexpr (NB == 2 && !RIGID) {
    dp2_forward<R>(P, q, qd, T);
  } else {
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    sincos_r(q[i], &T.sn[i], &T.cs[i]);
    R v0, v1, v2;
    if (i == 0) {
      v0 = qd[0]; v1 = 0.f; v2 = 0.f;
    } else {
      const R L = joint_offset<NB, RIGID>(P, i);
      const R w = T.v[i - 1][0];
      const R tx = T.v[i - 1][1] + w * L, ty = T.v[i - 1][2];
      v0 = w + qd[i];
      v1 = T.cs[i] * tx + T.sn[i] * ty;
      v2 = -T.sn[i] * tx + T.cs[i] * ty;
    }
    T.v[i][0] = v0; T.v[i][1] = v1; T.v[i][2] = v2;
    const R m = P.m[i];
    R h1, h2;  // linear momentum of the link, m (v + w x c)
    if constexpr (RIGID) {
      const R cx = P.cx[i], cy = P.cy[i];
      h1 = m * (v1 - cy * v0);
      h2 = m * (v2 + cx * v0);
      T.IA[i][0] = P.I[i] + m * (cx * cx + cy * cy); T.IA[i][1] = -m * cy; T.IA[i][2] = m * cx;
      T.IA[i][3] = m;                                T.IA[i][4] = 0.f;     T.IA[i][5] = m;
    } else {
      const R l = P.l[i];
      h1 = m * (l * v0 + v1);
      h2 = m * v2;
      T.IA[i][0] = m * l * l; T.IA[i][1] = m * l; T.IA[i][2] = 0.f;
      T.IA[i][3] = m;         T.IA[i][4] = 0.f;   T.IA[i][5] = m;
    }
    T.pA[i][0] = v1 * h2 - v2 * h1;
    T.pA[i][1] = -v0 * h2;
    T.pA[i][2] = v0 * h1;
  }
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    const R invD = recip(T.IA[i][0]);
    const R U1 = T.IA[i][1], U2 = T.IA[i][2];
    const R u = -P.b[i] * qd[i] - T.pA[i][0];
    T.invD[i] = invD;
    T.u[i] = u;
    if (i > 0) {
      const R c1 = T.v[i][2] * qd[i], c2 = -T.v[i][1] * qd[i];
      const R a = T.IA[i][3] - U1 * U1 * invD;
      const R bb = T.IA[i][4] - U1 * U2 * invD;
      const R d = T.IA[i][5] - U2 * U2 * invD;
      const R k = u * invD;
      const R pa0 = T.pA[i][0] + u;
      const R pa1 = T.pA[i][1] + a * c1 + bb * c2 + U1 * k;
      const R pa2 = T.pA[i][2] + bb * c1 + d * c2 + U2 * k;
      const R cs = T.cs[i], sn = T.sn[i], L = joint_offset<NB, RIGID>(P, i);
      const R A00 = a * cs * cs - 2.f * bb * cs * sn + d * sn * sn;
      const R A01 = (a - d) * cs * sn + bb * (cs * cs - sn * sn);
      const R A11 = a * sn * sn + 2.f * bb * cs * sn + d * cs * cs;
      T.IA[i - 1][0] += L * L * A00;
      T.IA[i - 1][1] += L * A00;
      T.IA[i - 1][2] += L * A01;
      T.IA[i - 1][3] += A00;
      T.IA[i - 1][4] += A01;
      T.IA[i - 1][5] += A11;
      const R f1 = cs * pa1 - sn * pa2, f2 = sn * pa1 + cs * pa2;
      T.pA[i - 1][0] += pa0 + L * f1;
      T.pA[i - 1][1] += f1;
      T.pA[i - 1][2] += f2;
    }
  }
  R a0 = 0.f, a1 = -P.gx, a2 = -P.gy;  // base acceleration = -gravity
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const R L = (i == 0) ? R(0.f) : joint_offset<NB, RIGID>(P, i);
    const R tx = a1 + a0 * L, ty = a2;
    const R c1 = T.v[i][2] * qd[i], c2 = -T.v[i][1] * qd[i];
    const R ap0 = a0;
    const R ap1 = T.cs[i] * tx + T.sn[i] * ty + c1;
    const R ap2 = -T.sn[i] * tx + T.cs[i] * ty + c2;
    T.ap[i][0] = ap0; T.ap[i][1] = ap1; T.ap[i][2] = ap2;
    const R qdd = (T.u[i] - (T.IA[i][0] * ap0 + T.IA[i][1] * ap1 + T.IA[i][2] * ap2)) * T.invD[i];
    T.qdd[i] = qdd;
    a0 = ap0 + qdd; a1 = ap1; a2 = ap2;
  }
  }
}

// Reverse of aba(): given qddb = d L / d qdd, accumulates d L / d q, d L / d qd
// and d L / d theta into thb (layout of PlanarParams).
template <int NB, class R = float, bool RIGID = false>
__host__ __device__ __forceinline__ void aba_rev(const Planar<NB, R>& P, const R* qd, const Tape<NB, R>& T,
                                        const R* qddb_in, R* qb, R* qdb, R* thb) {
  if constexpr (NB == 2 && !RIGID) {
    dp2_reverse<R>(P, qd, T, qddb_in, qb, qdb, thb);
  } else {
  using PP = PlanarParams<NB, RIGID>;
  R csb[NB], snb[NB], Lb[NB], taub[NB];
  R IAb[NB][6], pAb[NB][3], vb[NB][3], cb1[NB], cb2[NB];
  R ub[NB], Db[NB], U1b[NB], U2b[NB], invDb[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    csb[i] = snb[i] = Lb[i] = taub[i] = 0.f;
    cb1[i] = cb2[i] = 0.f;
    ub[i] = Db[i] = U1b[i] = U2b[i] = invDb[i] = 0.f;
#pragma unroll
    for (int e = 0; e < 6; ++e) IAb[i][e] = 0.f;
#pragma unroll
    for (int e = 0; e < 3; ++e) { pAb[i][e] = 0.f; vb[i][e] = 0.f; }
  }
  // ---- pass 3 (outward accelerations), reversed ----
  R ab0 = 0.f, ab1 = 0.f, ab2 = 0.f;
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    R qddb = qddb_in[i] + ab0;  // a_i = a'_i + S qdd_i
    R apb0 = ab0, apb1 = ab1, apb2 = ab2;
    const R D = T.IA[i][0], U1 = T.IA[i][1], U2 = T.IA[i][2], invD = T.invD[i];
    const R ap0 = T.ap[i][0], ap1 = T.ap[i][1], ap2 = T.ap[i][2];
    const R g = qddb * invD;
    ub[i] += g;
    Db[i] -= g * ap0;
    U1b[i] -= g * ap1;
    U2b[i] -= g * ap2;
    apb0 -= g * D;
    apb1 -= g * U1;
    apb2 -= g * U2;
    invDb[i] += qddb * (T.u[i] - (D * ap0 + U1 * ap1 + U2 * ap2));
    cb1[i] += apb1;
    cb2[i] += apb2;
    R x0, x1, x2, L;
    if (i == 0) {
      x0 = 0.f; x1 = -P.gx; x2 = -P.gy; L = 0.f;
    } else {
      x0 = T.ap[i - 1][0] + T.qdd[i - 1]; x1 = T.ap[i - 1][1]; x2 = T.ap[i - 1][2];
      L = joint_offset<NB, RIGID>(P, i);
    }
    const R cs = T.cs[i], sn = T.sn[i];
    const R tx = x1 + x0 * L, ty = x2;
    const R txb = cs * apb1 - sn * apb2, tyb = sn * apb1 + cs * apb2;
    csb[i] += apb1 * tx + apb2 * ty;
    snb[i] += apb1 * ty - apb2 * tx;
    if (i > 0) Lb[i] += x0 * txb;
    ab0 = apb0 + L * txb;
    ab1 = txb;
    ab2 = tyb;
  }
  // ---- pass 2 (inward articulated inertias), reversed ----
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const R U1 = T.IA[i][1], U2 = T.IA[i][2], invD = T.invD[i], u = T.u[i];
    if (i > 0) {
      const int p = i - 1;
      const R c1 = T.v[i][2] * qd[i], c2 = -T.v[i][1] * qd[i];
      const R a = T.IA[i][3] - U1 * U1 * invD;
      const R bb = T.IA[i][4] - U1 * U2 * invD;
      const R d = T.IA[i][5] - U2 * U2 * invD;
      const R k = u * invD;
      const R pa1 = T.pA[i][1] + a * c1 + bb * c2 + U1 * k;
      const R pa2 = T.pA[i][2] + bb * c1 + d * c2 + U2 * k;
      const R cs = T.cs[i], sn = T.sn[i], L = joint_offset<NB, RIGID>(P, i);
      const R A00 = a * cs * cs - 2.f * bb * cs * sn + d * sn * sn;
      const R A01 = (a - d) * cs * sn + bb * (cs * cs - sn * sn);
      const R f1 = cs * pa1 - sn * pa2;
      // parent updates
      const R A00b = L * L * IAb[p][0] + L * IAb[p][1] + IAb[p][3];
      const R A01b = L * IAb[p][2] + IAb[p][4];
      const R A11b = IAb[p][5];
      Lb[i] += 2.f * L * A00 * IAb[p][0] + A00 * IAb[p][1] + A01 * IAb[p][2];
      const R f1b = L * pAb[p][0] + pAb[p][1], f2b = pAb[p][2];
      Lb[i] += f1 * pAb[p][0];
      const R pab0 = pAb[p][0];
      const R pab1 = cs * f1b + sn * f2b;
      const R pab2 = -sn * f1b + cs * f2b;
      csb[i] += pa1 * f1b + pa2 * f2b;
      snb[i] += -pa2 * f1b + pa1 * f2b;
      // rotated inertia A' -> (a, bb, d, cs, sn)
      const R cc = cs * cs, ss = sn * sn, cn = cs * sn;
      R abar = cc * A00b + cn * A01b + ss * A11b;
      R bbar = -2.f * cn * A00b + (cc - ss) * A01b + 2.f * cn * A11b;
      R dbar = ss * A00b - cn * A01b + cc * A11b;
      csb[i] += (2.f * a * cs - 2.f * bb * sn) * A00b + ((a - d) * sn + 2.f * bb * cs) * A01b +
                (2.f * bb * sn + 2.f * d * cs) * A11b;
      snb[i] += (-2.f * bb * cs + 2.f * d * sn) * A00b + ((a - d) * cs - 2.f * bb * sn) * A01b +
                (2.f * a * sn + 2.f * bb * cs) * A11b;
      // pa = pA + Ia c + U u / D
      R kb = 0.f;
      pAb[i][0] += pab0;
      ub[i] += pab0;
      pAb[i][1] += pab1;
      abar += pab1 * c1;
      bbar += pab1 * c2;
      cb1[i] += a * pab1;
      cb2[i] += bb * pab1;
      U1b[i] += pab1 * k;
      kb += U1 * pab1;
      pAb[i][2] += pab2;
      bbar += pab2 * c1;
      dbar += pab2 * c2;
      cb1[i] += bb * pab2;
      cb2[i] += d * pab2;
      U2b[i] += pab2 * k;
      kb += U2 * pab2;
      ub[i] += kb * invD;
      invDb[i] += kb * u;
      // Ia = IA - U U^T / D (rows/columns 0 vanish identically)
      IAb[i][3] += abar;
      U1b[i] -= 2.f * U1 * invD * abar;
      invDb[i] -= U1 * U1 * abar;
      IAb[i][4] += bbar;
      U1b[i] -= U2 * invD * bbar;
      U2b[i] -= U1 * invD * bbar;
      invDb[i] -= U1 * U2 * bbar;
      IAb[i][5] += dbar;
      U2b[i] -= 2.f * U2 * invD * dbar;
      invDb[i] -= U2 * U2 * dbar;
    }
    // u = tau - pA0
    taub[i] += ub[i];
    pAb[i][0] -= ub[i];
    // invD = 1 / D, D = IA00, U = (IA00, IA01, IA02)
    Db[i] -= invD * invD * invDb[i];
    IAb[i][0] += Db[i];
    IAb[i][1] += U1b[i];
    IAb[i][2] += U2b[i];
    const R m = P.m[i];
    if constexpr (RIGID) {
      // rigid inertia [I + m |c|^2, -m cy, m cx, m, 0, m]
      const R cx = P.cx[i], cy = P.cy[i];
      thb[PP::m(i)] += (cx * cx + cy * cy) * IAb[i][0] - cy * IAb[i][1] + cx * IAb[i][2] + IAb[i][3] + IAb[i][5];
      thb[PP::I(i)] += IAb[i][0];
      thb[PP::cx(i)] += 2.f * m * cx * IAb[i][0] + m * IAb[i][2];
      thb[PP::cy(i)] += 2.f * m * cy * IAb[i][0] - m * IAb[i][1];
    } else {
      // rigid inertia of a point mass at (0, -l): m [l^2, l, 0, 1, 0, 1]
      const R l = P.l[i];
      thb[PP::m(i)] += l * l * IAb[i][0] + l * IAb[i][1] + IAb[i][3] + IAb[i][5];
      thb[PP::l(i)] += 2.f * m * l * IAb[i][0] + m * IAb[i][1];
    }
  }
  // ---- pass 1 (outward velocities and bias forces), reversed ----
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    const R v0 = T.v[i][0], v1 = T.v[i][1], v2 = T.v[i][2];
    const R m = P.m[i];
    R h1, h2;
    if constexpr (RIGID) {
      h1 = m * (v1 - P.cy[i] * v0);
      h2 = m * (v2 + P.cx[i] * v0);
    } else {
      h1 = m * (P.l[i] * v0 + v1);
      h2 = m * v2;
    }
    R vb0 = vb[i][0], vb1 = vb[i][1], vb2 = vb[i][2];
    const R pb0 = pAb[i][0], pb1 = pAb[i][1], pb2 = pAb[i][2];
    vb1 += pb0 * h2;
    R h2b = pb0 * v1;
    vb2 -= pb0 * h1;
    R h1b = -pb0 * v2;
    vb0 -= pb1 * h2;
    h2b -= pb1 * v0;
    vb0 += pb2 * h1;
    h1b += pb2 * v0;
    if constexpr (RIGID) {
      const R cx = P.cx[i], cy = P.cy[i];
      vb0 += -m * cy * h1b + m * cx * h2b;
      vb1 += m * h1b;
      vb2 += m * h2b;
      thb[PP::m(i)] += (v1 - cy * v0) * h1b + (v2 + cx * v0) * h2b;
      thb[PP::cy(i)] += -m * v0 * h1b;
      thb[PP::cx(i)] += m * v0 * h2b;
    } else {
      const R l = P.l[i];
      vb0 += m * l * h1b;
      vb1 += m * h1b;
      thb[PP::m(i)] += (l * v0 + v1) * h1b + v2 * h2b;
      thb[PP::l(i)] += m * v0 * h1b;
      vb2 += m * h2b;
    }
    // c = (0, v2 qd, -v1 qd)
    vb2 += cb1[i] * qd[i];
    qdb[i] += cb1[i] * v2;
    vb1 -= cb2[i] * qd[i];
    qdb[i] -= cb2[i] * v1;
    // v_i = X_i v_{i-1} + (qd_i, 0, 0)
    qdb[i] += vb0;
    if (i > 0) {
      const R x0 = T.v[i - 1][0], x1 = T.v[i - 1][1], x2 = T.v[i - 1][2];
      const R L = joint_offset<NB, RIGID>(P, i), cs = T.cs[i], sn = T.sn[i];
      const R tx = x1 + x0 * L, ty = x2;
      const R txb = cs * vb1 - sn * vb2, tyb = sn * vb1 + cs * vb2;
      csb[i] += vb1 * tx + vb2 * ty;
      snb[i] += vb1 * ty - vb2 * tx;
      vb[i - 1][0] += vb0 + L * txb;
      vb[i - 1][1] += txb;
      vb[i - 1][2] += tyb;
      Lb[i] += x0 * txb;
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    qb[i] += -T.sn[i] * csb[i] + T.cs[i] * snb[i];
    qdb[i] += -P.b[i] * taub[i];
    if constexpr (RIGID) {
      thb[PP::b(i)] += -qd[i] * taub[i];  // tau_i = -b_i qd_i
      if (i > 0) thb[PP::L(i)] += Lb[i];
    } else {
      if (i > 0) thb[PP::l(i - 1)] += Lb[i];
    }
  }
  }
}

// Semi-implicit Euler: qd' = qd + dt qdd, q' = q + dt qd'.
template <int NB, class R = float>
__host__ __device__ __forceinline__ void euler(R dt, const Tape<NB, R>& T, R* q, R* qd) {
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    qd[i] = qd[i] + dt * T.qdd[i];
    q[i] = q[i] + dt * qd[i];
  }
}

template <int NB, class R = float, bool RIGID = false>
__host__ __device__ __forceinline__ void step(const Planar<NB, R>& P, R dt, R* q, R* qd) {
  Tape<NB, R> T;
  aba<NB, R, RIGID>(P, q, qd, T);
  euler<NB, R>(dt, T, q, qd);
}

// Reverse of one Euler step given the tape at its input state.  On entry
// (qb, qdb) are the adjoints of the step's outputs; on exit of its inputs.
template <int NB, class R = float, bool RIGID = false>
__host__ __device__ __forceinline__ void step_rev(const Planar<NB, R>& P, R dt, const R* qd, const Tape<NB, R>& T,
                                         R* qb, R* qdb, R* thb) {
  R qddb[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    qdb[i] = qdb[i] + dt * qb[i];
    qddb[i] = dt * qdb[i];
  }
  aba_rev<NB, R, RIGID>(P, qd, T, qddb, qb, qdb, thb);
}

template <int NB, bool RIGID>
__device__ __forceinline__ void load_model(const pds_job& J, const float* th, Planar<NB>& P) {
  using PP = PlanarParams<NB, RIGID>;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    P.m[i] = th[PP::m(i)];
    if constexpr (RIGID) {
      P.I[i] = th[PP::I(i)];
      P.cx[i] = th[PP::cx(i)];
      P.cy[i] = th[PP::cy(i)];
      P.b[i] = th[PP::b(i)];
      P.L[i] = i > 0 ? th[PP::L(i)] : 0.f;
    } else {
      P.l[i] = th[PP::l(i)];
      P.b[i] = J.consts[2 + i];
    }
  }
  P.gx = J.consts[0];
  P.gy = J.consts[1];
}

struct Unit {
  int i, k, j;
};

__device__ inline Unit unit_of(const pds_job& J, int u) {
  Unit r;
  r.i = u % J.N;
  const int kj = u / J.N;
  r.k = kj / J.n_s;
  r.j = kj % J.n_s;
  return r;
}

__device__ inline const float* start_ptr(const pds_job& J, const Unit& w, int ds) {
  if (w.j == 0) return J.s0 + (size_t)w.k * ds;
  return J.S + (((size_t)w.i * J.K + w.k) * (J.n_s - 1) + (w.j - 1)) * ds;
}

__device__ inline double log_norm_const(const pds_job& J) {
  // sum_d log(w_d / sqrt(2 pi)) per observed step
  double c = 0.0;
  for (int d = 0; d < J.d_x; ++d) c += log((double)J.w_x[d]) - 0.91893853320467274178;
  return c;
}

template <int NB, bool RIGID>
__global__ void __launch_bounds__(kWave) planar_forward_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                               int with_ll) {
  constexpr int MP = PlanarParams<NB, RIGID>::M;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int U = J.N * J.K * J.n_s;
  const int u = (blockIdx.x - map.begin[e]) * kWave + threadIdx.x;
  if (u >= U) return;
  constexpr int DS = 2 * NB;
  const Unit w = unit_of(J, u);
  Planar<NB> P;
  float th[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) th[m] = J.theta[(size_t)w.i * J.M + m];
  load_model<NB, RIGID>(J, th, P);
  const float* st = start_ptr(J, w, DS);
  float q[NB], qd[NB];
#pragma unroll
  for (int d = 0; d < NB; ++d) { q[d] = ldg(st + d); qd[d] = ldg(st + NB + d); }
  const float dt = J.dt;
  const int t0 = w.j * J.h;
  const float* obs = J.obs + ((size_t)w.k * J.T + t0) * J.d_x;
  float* traj = J.traj ? J.traj + (((size_t)w.i * J.K + w.k) * J.T + t0) * DS : nullptr;
  // d_x = NB observes q; d_x = 2 NB the whole state (q, qd)
  const bool obs_v = J.d_x == DS;
  const int DX = obs_v ? DS : NB;
  float* tobs = J.traj_obs ? J.traj_obs + (((size_t)w.i * J.K + w.k) * J.T + t0) * DX : nullptr;
  float wx[DS];
#pragma unroll
  for (int d = 0; d < DS; ++d) wx[d] = (d < NB || obs_v) ? J.w_x[d] : 0.f;
  constexpr bool kAhead = NB <= 2;
  // Short chains (kAhead) read observation rows one step ahead, so each
  // load's latency hides behind a step of arithmetic instead of stalling the
  // wave; longer chains have enough arithmetic per step to hide a load made
  // at its use, and the extra live registers would cost them more.
  // load_row is unconditional and in bounds (no branch the compiler must
  // merge): when only q is observed the velocity half reads a value of the
  // same row, which is never used.
  auto load_row = [&](int s, float* o) {
    const float* row = obs + (size_t)s * DX;
#pragma unroll
    for (int d = 0; d < NB; ++d) o[d] = ldg(row + d);
#pragma unroll
    for (int d = 0; d < NB; ++d) o[NB + d] = ldg(row + min(NB + d, DX - 1));
  };
  float ob[DS] = {};
  auto obs_at = [&](int s, int d) -> float { return kAhead ? ob[d] : obs[s * DX + d]; };
  if (kAhead && with_ll && J.h > 0) load_row(0, ob);
  double ll = 0.0;
  for (int s = 0; s < J.h; ++s) {
    step<NB, float, RIGID>(P, dt, q, qd);
    if (with_ll) {
      float acc = 0.f;
#pragma unroll
      for (int d = 0; d < NB; ++d) {
        const float r = (obs_at(s, d) - q[d]) * wx[d];
        acc += r * r;
      }
      if (obs_v) {
#pragma unroll
        for (int d = 0; d < NB; ++d) {
          const float r = (obs_at(s, NB + d) - qd[d]) * wx[NB + d];
          acc += r * r;
        }
      }
      ll -= 0.5 * (double)acc;
      if (kAhead) load_row(min(s + 1, J.h - 1), ob);  // in flight during the next step
    }
    if (traj) {
#pragma unroll
      for (int d = 0; d < NB; ++d) { traj[s * DS + d] = q[d]; traj[s * DS + NB + d] = qd[d]; }
    }
    if (tobs) {
#pragma unroll
      for (int d = 0; d < NB; ++d) tobs[s * DX + d] = q[d];
      if (obs_v) {
#pragma unroll
        for (int d = 0; d < NB; ++d) tobs[s * DX + NB + d] = qd[d];
      }
    }
  }
  const size_t iu = ((size_t)w.i * J.K + w.k) * J.n_s + w.j;
  float* es = J.end_states + iu * DS;
#pragma unroll
  for (int d = 0; d < NB; ++d) { es[d] = q[d]; es[NB + d] = qd[d]; }
  bool bad = false, bad_ll = false;
#pragma unroll
  for (int d = 0; d < NB; ++d) bad |= !isfinite(q[d]) || !isfinite(qd[d]);
  if (with_ll) {
    ll += (double)J.h * log_norm_const(J);
    if (w.j + 1 < J.n_s) {
      const float* sn = J.S + (((size_t)w.i * J.K + w.k) * (J.n_s - 1) + w.j) * DS;
      double g = 0.0;
#pragma unroll
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
    bad_ll = !isfinite(ll);
  }
  const int fl = (bad ? PDS_FLAG_STATE : 0) | (bad_ll ? PDS_FLAG_GRAD : 0);
  if (fl && J.flags) atomicOr(&J.flags[w.i], fl);
}

// Segment length of the adjoint's checkpointing: about sqrt(h).
__host__ __device__ inline int seg_len_of(int h) {
  int B = 1;
  while (B * B < h) ++B;
  return B;
}

// Adjoint kernel.  SPLIT = false: a lane owns a unit and carries both
// adjoint channels.  SPLIT = true (problems too small to fill the GPU): a
// wave owns 32 units, lanes l and l + 32 share a unit, run the same primal
// sweeps and each carries one channel (selected by data, so the two halves
// execute the same instructions).  full = 1 keeps every state of the window
// in LDS (no recomputation), full = 0 keeps checkpoints every B ~ sqrt(h)
// steps and recomputes one segment at a time.  TAPE (two point-mass links,
// SPLIT, full = 1): the forward sweep also keeps each step's dynamics tape
// (sin/cos of both angles, qdd, 1 / det H) in LDS after the states, one
// copy per unit, and the reverse sweep reads it instead of evaluating the
// dynamics again (the reverse then uses exactly the forward sweep's values;
// a re-evaluation, compiled in another context, may round differently).
template <int NB, bool SPLIT, bool RIGID, bool TAPE = false>
__global__ void __launch_bounds__(kWave) planar_adjoint_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                               char* __restrict__ ws, int full) {
  static_assert(!TAPE || (NB == 2 && SPLIT && !RIGID), "the tape holds the closed-form two-link dynamics");
  constexpr int MP = PlanarParams<NB, RIGID>::M;
  extern __shared__ float lds[];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int U = J.N * J.K * J.n_s;
  const int lane = threadIdx.x;
  constexpr int UPW = SPLIT ? kWave / 2 : kWave;  // units per wave
  const int u = (blockIdx.x - map.begin[e]) * UPW + (SPLIT ? (lane & (UPW - 1)) : lane);
  // channel of this lane: 0 observation, 1 constraint (SPLIT only)
  const int ch = SPLIT ? (lane >= UPW) : 0;
  if (u >= U) return;
  constexpr int DS = 2 * NB;
  const WsLayout L = ws_layout(J);
  char* base = ws + map.ws_off[e];
  double* gth_obs = reinterpret_cast<double*>(base + L.gth_obs);
  double* gth_con = reinterpret_cast<double*>(base + L.gth_con);
  float* gs_obs = reinterpret_cast<float*>(base + L.gs_obs);
  float* gs_con = reinterpret_cast<float*>(base + L.gs_con);

  const Unit w = unit_of(J, u);
  Planar<NB> P;
  float th[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) th[m] = J.theta[(size_t)w.i * J.M + m];
  load_model<NB, RIGID>(J, th, P);
  const float* st = start_ptr(J, w, DS);
  float q[NB], qd[NB];
#pragma unroll
  for (int d = 0; d < NB; ++d) { q[d] = ldg(st + d); qd[d] = ldg(st + NB + d); }
  const float dt = J.dt;
  const int h = J.h;
  const int B = full ? h : seg_len_of(h);
  const int nseg = (h + B - 1) / B;
  // full: slots 0..h hold states 0..h.  Otherwise slots [0, nseg) hold
  // checkpoints and [nseg, nseg + B + 1) the segment being reversed.
  const int segbase = full ? 0 : nseg;
  const int t0 = w.j * h;
  const float* obs = J.obs + ((size_t)w.k * J.T + t0) * J.d_x;
  const bool obs_v = J.d_x == DS;  // observes (q, qd), else q
  const int DX = obs_v ? DS : NB;
  float wx[DS];
#pragma unroll
  for (int d = 0; d < DS; ++d) wx[d] = (d < NB || obs_v) ? J.w_x[d] : 0.f;
  auto slot = [&](int s, int d) -> float& { return lds[((size_t)s * DS + d) * kWave + lane]; };
  // Tape of step s, [step][entry][unit of the wave]: both lanes of a unit
  // write the same values to the same word, so each lane reads back what it
  // wrote itself.
  constexpr int kTapeW = 7;
  float* const tape = lds + (size_t)(h + 1) * DS * kWave;
  const int ul = lane & (UPW - 1);
  auto tp = [&](int s, int t) -> float& { return tape[((size_t)s * kTapeW + t) * UPW + ul]; };

  constexpr bool kAhead = NB <= 2;
  // Short chains (kAhead) read observation rows one step ahead in both
  // sweeps, so each load's latency hides behind a step of arithmetic; longer
  // chains load at the use (enough arithmetic per step to hide it, fewer
  // live registers).  load_row is unconditional and in bounds (no branch the
  // compiler must merge): when only q is observed the velocity half reads a
  // value of the same row, which is never used.
  auto load_row = [&](int s, float* o) {
    const float* row = obs + (size_t)s * DX;
#pragma unroll
    for (int d = 0; d < NB; ++d) o[d] = ldg(row + d);
#pragma unroll
    for (int d = 0; d < NB; ++d) o[NB + d] = ldg(row + min(NB + d, DX - 1));
  };
  float ob[DS] = {};
  auto obs_at = [&](int s, int d) -> float { return kAhead ? ob[d] : obs[s * DX + d]; };

  // ---- forward sweep: log-likelihood, end state, stored states ----
  // Short chains store state 0 first: its slot is the start state in both
  // storage modes, and storing it here completes the start-state loads
  // before the loop, so the loop never waits on them.
  if (kAhead) {
#pragma unroll
    for (int d = 0; d < NB; ++d) { slot(0, d) = q[d]; slot(0, NB + d) = qd[d]; }
    load_row(0, ob);
  }
  double ll = 0.0;
  for (int s = 0; s < h; ++s) {
    if ((!kAhead || s > 0) && (full || s % B == 0)) {
      const int sl = full ? s : s / B;
#pragma unroll
      for (int d = 0; d < NB; ++d) { slot(sl, d) = q[d]; slot(sl, NB + d) = qd[d]; }
    }
    if constexpr (TAPE) {
      Tape<NB> T;
      aba<NB, float, RIGID>(P, q, qd, T);
      tp(s, 0) = T.sn[0]; tp(s, 1) = T.sn[1];
      tp(s, 2) = T.cs[0]; tp(s, 3) = T.cs[1];
      tp(s, 4) = T.qdd[0]; tp(s, 5) = T.qdd[1];
      tp(s, 6) = T.invD[0];
      euler<NB>(dt, T, q, qd);
    } else {
      step<NB, float, RIGID>(P, dt, q, qd);
    }
    float acc = 0.f;
#pragma unroll
    for (int d = 0; d < NB; ++d) {
      const float r = (obs_at(s, d) - q[d]) * wx[d];
      acc += r * r;
    }
    if (obs_v) {
#pragma unroll
      for (int d = 0; d < NB; ++d) {
        const float r = (obs_at(s, NB + d) - qd[d]) * wx[NB + d];
        acc += r * r;
      }
    }
    ll -= 0.5 * (double)acc;
    if (kAhead) load_row(min(s + 1, h - 1), ob);  // in flight during the next step
  }
  if (full) {
#pragma unroll
    for (int d = 0; d < NB; ++d) { slot(h, d) = q[d]; slot(h, NB + d) = qd[d]; }
  }
  ll += (double)h * log_norm_const(J);
  const size_t iu = ((size_t)w.i * J.K + w.k) * J.n_s + w.j;
  bool bad = false, bad_g = false;  // non-finite state; likelihood or gradient
#pragma unroll
  for (int d = 0; d < NB; ++d) bad |= !isfinite(q[d]) || !isfinite(qd[d]);
  if (ch == 0) {
    float* es = J.end_states + iu * DS;
#pragma unroll
    for (int d = 0; d < NB; ++d) { es[d] = q[d]; es[NB + d] = qd[d]; }
  }

  // ---- seeds ----
  // channel variables: a (obs), c (con); with SPLIT a lane carries only
  // its own channel in (qb_a, qdb_a) and the observation seed is scaled by
  // obs_on (1 for the observation lane, 0 for the constraint lane).
  float qb_a[NB], qdb_a[NB], qb_c[NB], qdb_c[NB];
#pragma unroll
  for (int d = 0; d < NB; ++d) { qb_a[d] = qdb_a[d] = qb_c[d] = qdb_c[d] = 0.f; }
  const float obs_on = (SPLIT && ch == 1) ? 0.f : 1.f;
  if (w.j + 1 < J.n_s) {
    const size_t id = ((size_t)w.i * J.K + w.k) * (J.n_s - 1) + w.j;
    const float* sn = J.S + id * DS;
    float e0[NB], e1[NB];
    double g = 0.0;
#pragma unroll
    for (int d = 0; d < NB; ++d) {
      e0[d] = (sn[d] - q[d]) * J.u[d];
      e1[d] = (sn[NB + d] - qd[d]) * J.u[NB + d];
      g += (double)e0[d] * e0[d] + (double)e1[d] * e1[d];
    }
    const double inv_s2 = 1.0 / ((double)J.sigma_def * J.sigma_def);
    g *= inv_s2;
    if (ch == 0) J.gdef[id] = g;
    const bool in_lik = J.lik == PDS_LIK_DEFECT;
    if (in_lik) ll += -0.5 * g + defect_log_norm(J);
    const double seed = con_seed(J, id, g, in_lik);
    // d g / d s_end = -2 e u / sigma^2; in the likelihood, d(-g/2) / d s_end = e u / sigma^2
    const float sc = (float)(-2.0 * seed * inv_s2);
    const float so = in_lik ? (float)inv_s2 : 0.f;
    if (SPLIT) {
      const float con_on = 1.f - obs_on;
      const float sa = obs_on * so + con_on * sc;
#pragma unroll
      for (int d = 0; d < NB; ++d) {
        qb_a[d] = sa * e0[d] * J.u[d];
        qdb_a[d] = sa * e1[d] * J.u[NB + d];
      }
    } else {
#pragma unroll
      for (int d = 0; d < NB; ++d) {
        qb_a[d] = so * e0[d] * J.u[d];
        qdb_a[d] = so * e1[d] * J.u[NB + d];
        qb_c[d] = sc * e0[d] * J.u[d];
        qdb_c[d] = sc * e1[d] * J.u[NB + d];
      }
    }
  }
  bad_g |= !isfinite(ll);
  if (ch == 0) J.ll_win[iu] = ll;

  // ---- reverse sweep over segments (steps h-1 .. 0 in one descending order) ----
  if (kAhead) load_row(h - 1, ob);
  double gm_a[MP], gm_c[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) { gm_a[m] = 0.0; gm_c[m] = 0.0; }
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int a = sg * B;
    const int bnd = min(h, a + B);
    if (!full) {
#pragma unroll
      for (int d = 0; d < NB; ++d) { q[d] = slot(sg, d); qd[d] = slot(sg, NB + d); }
#pragma unroll
      for (int d = 0; d < NB; ++d) { slot(segbase, d) = q[d]; slot(segbase, NB + d) = qd[d]; }
      for (int s = a; s < bnd; ++s) {
        step<NB, float, RIGID>(P, dt, q, qd);
#pragma unroll
        for (int d = 0; d < NB; ++d) {
          slot(segbase + s - a + 1, d) = q[d];
          slot(segbase + s - a + 1, NB + d) = qd[d];
        }
      }
    }
    for (int s = bnd - 1; s >= a; --s) {
      // observation seed at the step's output state s+1
#pragma unroll
      for (int d = 0; d < NB; ++d) {
        const float x = slot(segbase + s - a + 1, d);
        const float r = (obs_at(s, d) - x) * wx[d];
        qb_a[d] += obs_on * (r * wx[d]);
      }
      if (obs_v) {
#pragma unroll
        for (int d = 0; d < NB; ++d) {
          const float x = slot(segbase + s - a + 1, NB + d);
          const float r = (obs_at(s, NB + d) - x) * wx[NB + d];
          qdb_a[d] += obs_on * (r * wx[NB + d]);
        }
      }
      if (kAhead) load_row(max(s - 1, 0), ob);  // in flight during this step's reverse
      float qs[NB], qds[NB];
#pragma unroll
      for (int d = 0; d < NB; ++d) { qs[d] = slot(segbase + s - a, d); qds[d] = slot(segbase + s - a, NB + d); }
      Tape<NB> T;
      if constexpr (TAPE) {
        T.sn[0] = tp(s, 0); T.sn[1] = tp(s, 1);
        T.cs[0] = tp(s, 2); T.cs[1] = tp(s, 3);
        T.qdd[0] = tp(s, 4); T.qdd[1] = tp(s, 5);
        T.invD[0] = tp(s, 6);
      } else {
        aba<NB, float, RIGID>(P, qs, qds, T);
      }
      float thb[MP];
#pragma unroll
      for (int m = 0; m < MP; ++m) thb[m] = 0.f;
      step_rev<NB, float, RIGID>(P, dt, qds, T, qb_a, qdb_a, thb);
#pragma unroll
      for (int m = 0; m < MP; ++m) gm_a[m] += (double)thb[m];
      if (!SPLIT) {
#pragma unroll
        for (int m = 0; m < MP; ++m) thb[m] = 0.f;
        step_rev<NB, float, RIGID>(P, dt, qds, T, qb_c, qdb_c, thb);
#pragma unroll
        for (int m = 0; m < MP; ++m) gm_c[m] += (double)thb[m];
      }
    }
  }
  // ---- per-unit outputs ----
  if (SPLIT) {
    double* gth = ch == 0 ? gth_obs : gth_con;
    float* gs = ch == 0 ? gs_obs : gs_con;
#pragma unroll
    for (int m = 0; m < MP; ++m) bad_g |= !isfinite(gm_a[m]);
    store_row<MP>(gth + iu * MP, gm_a);
    float row[DS];
#pragma unroll
    for (int d = 0; d < NB; ++d) { row[d] = qb_a[d]; row[NB + d] = qdb_a[d]; }
    store_row<DS>(gs + iu * DS, row);
  } else {
#pragma unroll
    for (int m = 0; m < MP; ++m) bad_g |= !isfinite(gm_a[m]) || !isfinite(gm_c[m]);
    store_row<MP>(gth_obs + iu * MP, gm_a);
    store_row<MP>(gth_con + iu * MP, gm_c);
    float ra[DS], rc[DS];
#pragma unroll
    for (int d = 0; d < NB; ++d) {
      ra[d] = qb_a[d];
      ra[NB + d] = qdb_a[d];
      rc[d] = qb_c[d];
      rc[NB + d] = qdb_c[d];
    }
    store_row<DS>(gs_obs + iu * DS, ra);
    store_row<DS>(gs_con + iu * DS, rc);
  }
  const int fl = (bad ? PDS_FLAG_STATE : 0) | (bad_g ? PDS_FLAG_GRAD : 0);
  if (fl && J.flags) atomicOr(&J.flags[w.i], fl);
}

}  // namespace

template <int NB, bool RIGID>
static hipError_t fwd_nb(const JobMap& map, const pds_job* d_jobs, int grid, bool with_ll, hipStream_t s) {
  hipLaunchKernelGGL((planar_forward_kernel<NB, RIGID>), dim3(grid), dim3(kWave), 0, s, map, d_jobs,
                     with_ll ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_planar_forward(const JobMap& map, int nb, bool rigid, const pds_job* d_jobs, int grid,
                                 bool with_ll, hipStream_t s) {
  if (rigid) {
    switch (nb) {
      case 1: return fwd_nb<1, true>(map, d_jobs, grid, with_ll, s);
      case 2: return fwd_nb<2, true>(map, d_jobs, grid, with_ll, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nb) {
    case 1: return fwd_nb<1, false>(map, d_jobs, grid, with_ll, s);
    case 2: return fwd_nb<2, false>(map, d_jobs, grid, with_ll, s);
    case 3: return fwd_nb<3, false>(map, d_jobs, grid, with_ll, s);
    case 4: return fwd_nb<4, false>(map, d_jobs, grid, with_ll, s);
    case 5: return fwd_nb<5, false>(map, d_jobs, grid, with_ll, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NB, bool RIGID>
static hipError_t adj_nb(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, size_t lds, bool split,
                         bool full, bool tape, hipStream_t s) {
  if constexpr (NB == 2 && !RIGID) {
    if (tape) {
      if (!split || !full) return hipErrorInvalidValue;
      hipLaunchKernelGGL((planar_adjoint_kernel<2, true, false, true>), dim3(grid), dim3(kWave), lds, s, map, d_jobs,
                         ws, 1);
      return hipGetLastError();
    }
  } else {
    if (tape) return hipErrorInvalidValue;
  }
  if (split)
    hipLaunchKernelGGL((planar_adjoint_kernel<NB, true, RIGID>), dim3(grid), dim3(kWave), lds, s, map, d_jobs, ws,
                       full ? 1 : 0);
  else
    hipLaunchKernelGGL((planar_adjoint_kernel<NB, false, RIGID>), dim3(grid), dim3(kWave), lds, s, map, d_jobs,
                       ws, full ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_planar_adjoint(const JobMap& map, int nb, bool rigid, const pds_job* d_jobs, char* ws, int grid,
                                 bool split, bool full, bool tape, size_t lds_bytes, hipStream_t s) {
  if (rigid) {
    switch (nb) {
      case 1: return adj_nb<1, true>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
      case 2: return adj_nb<2, true>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nb) {
    case 1: return adj_nb<1, false>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
    case 2: return adj_nb<2, false>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
    case 3: return adj_nb<3, false>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
    case 4: return adj_nb<4, false>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
    case 5: return adj_nb<5, false>(map, d_jobs, ws, grid, lds_bytes, split, full, tape, s);
    default: return hipErrorInvalidValue;
  }
}

size_t planar_tape_bytes(int h) { return (size_t)h * 7 * (kWave / 2) * sizeof(float); }

int planar_seg_len(int h) { return seg_len_of(h); }

// ---------------------------------------------------------------------------
// Algorithmic FLOP count of one step and of one reverse step, obtained by
// running the same templated step functions on the host with a counting
// scalar (add, sub, mul, div each 1; negation 0; sin/cos tallied apart).
// ---------------------------------------------------------------------------
namespace {
template <int NB, bool RIGID>
void count_planar(double* fwd, double* rev, double* transc) {
  constexpr int MP = PlanarParams<NB, RIGID>::M;
  Planar<NB, Counted> P;
  Counted q[NB], qd[NB], qb[NB], qdb[NB], thb[MP];
  for (int i = 0; i < NB; ++i) {
    P.m[i] = Counted(1.0f); P.l[i] = Counted(1.0f); P.b[i] = Counted(0.05f);
    P.I[i] = Counted(0.01f); P.cx[i] = Counted(0.02f); P.cy[i] = Counted(-0.1f); P.L[i] = Counted(0.2f);
    q[i] = Counted(0.3f); qd[i] = Counted(0.1f); qb[i] = Counted(1.f); qdb[i] = Counted(1.f);
  }
  P.gx = Counted(0.f); P.gy = Counted(-9.81f);
  g_tally = FlopTally();
  Tape<NB, Counted> T;
  aba<NB, Counted, RIGID>(P, q, qd, T);
  for (int i = 0; i < NB; ++i) {  // Euler update
    qd[i] = qd[i] + Counted(0.01f) * T.qdd[i];
    q[i] = q[i] + Counted(0.01f) * qd[i];
  }
  // observation residual r = (x - q) w; acc += r r; one FP64 accumulate
  *fwd = g_tally.flops + 4.0 * NB + 1.0;
  *transc = g_tally.transc;
  g_tally = FlopTally();
  step_rev<NB, Counted, RIGID>(P, Counted(0.01f), qd, T, qb, qdb, thb);
  // observation seed r w per component; FP64 accumulation of the M parameter adjoints
  *rev = g_tally.flops + 4.0 * NB + (double)MP;
}
}  // namespace

extern "C" int pds_algorithmic_flops(int32_t model, int32_t n_dof, double* fwd_step, double* rev_step,
                                     double* transcendental) {
  if (!fwd_step || !rev_step || !transcendental) return PDS_EINVAL;
  if (model == PDS_MODEL_ARM || model == PDS_MODEL_ARM_UJOINT || model == PDS_MODEL_ARM_UJOINT_WEIGHTS) {
    count_arm_flops(pds::arm_mount(model), fwd_step, rev_step, transcendental);
    return PDS_OK;
  }
  if (model == PDS_MODEL_PLANAR_RIGID) {
    switch (n_dof) {
      case 1: count_planar<1, true>(fwd_step, rev_step, transcendental); break;
      case 2: count_planar<2, true>(fwd_step, rev_step, transcendental); break;
      default: return PDS_EUNSUPPORTED;
    }
    return PDS_OK;
  }
  if (model != PDS_MODEL_PLANAR) return PDS_EINVAL;
  switch (n_dof) {
    case 1: count_planar<1, false>(fwd_step, rev_step, transcendental); break;
    case 2: count_planar<2, false>(fwd_step, rev_step, transcendental); break;
    case 3: count_planar<3, false>(fwd_step, rev_step, transcendental); break;
    case 4: count_planar<4, false>(fwd_step, rev_step, transcendental); break;
    case 5: count_planar<5, false>(fwd_step, rev_step, transcendental); break;
    default: return PDS_EUNSUPPORTED;
  }
  return PDS_OK;
}

}  // namespace pds
