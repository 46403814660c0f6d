// FP64 CPU oracle for one iteration of Constrained SVGD (CSVGD) over
// simulation parameters, after Heiden et al., "Probabilistic Inference of
// Simulation Parameters via Parallel Differentiable Simulation".
//
// TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
// the test suite, the smoke check and the CPU-baseline leg of the benchmark
// may load it.  It shares no code, header, table or constant generator with
// the GPU library, and nothing in the GPU library calls it.
//
// It is deliberately plain and slow: 6D spatial algebra with full 6x6
// matrices for every model (planar ones included), forward-mode dual numbers
// for every gradient, and a full sort for the kernel-bandwidth median.
//
// What each part follows (section / equation / algorithm of the paper):
//   * aba()          Articulated Body Algorithm, App. B-A (forward dynamics).
//   * crba_rnea()    Composite-rigid-body + recursive Newton-Euler, used only
//                    to cross-check aba() (textbook identity H qdd = tau - C).
//   * step()         semi-implicit Euler, App. B-A eq. "dynamics".
//   * window()       one multiple-shooting window, Sec. III-C: rollout from
//                    the window start state and the Gaussian observation
//                    likelihood of eq. "combinedlikelihood".
//   * defects        eq. "likelihood-defect" and g_def of Sec. III-E.
//   * combination    eq. "traj_likelihood" (sum / GMM, in log space) and
//                    App. A-B eq. "traj_likelihood_prod".
//   * gradients      MDMM flow of Sec. III-E applied to eq. "mdmm-loss";
//                    assembled per Algorithm 1.
//   * bandwidth/phi  eq. "svgd_update" with the RBF kernel and the median
//                    heuristic (Sec. III-A).
//   * mdmm_step      Algorithm 1 update lines, with Adam or plain SGD.
//
// Readings taken where the paper is silent or garbled: window
// j starts at step j*h and compares states j*h+1 .. (j+1)*h with the
// observations of the same steps; each trajectory has its own shooting
// states; g_def = ||(S - s_end) * u||^2 / sigma_def^2 >= 0; the SUM
// combination includes -log K; Gaussian constants are included in reported
// log-likelihoods; the bandwidth is med^2 / log N over the N(N-1)/2
// distinct scaled pair distances.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "dual.hpp"
#include "spatial.hpp"

extern "C" {

// Model description.  kind: 1 planar chain of point masses on massless rods
// (joints about z, q = 0 hangs along -y), 2 seven-joint arm (modified DH)
// carrying a box on a passive hinge about the flange x axis, 3 linear toy
// (one prismatic unit mass, no gravity, force theta0 + theta1 * time),
// 4 planar chain of rigid links (joints about z) parameterised as the
// physical double pendulum of Sec. IV-B: per link mass, rotational inertia
// about the centre of mass, centre of mass (x, y) in the link frame and
// joint friction, and the offset of every further joint along -y of its
// parent (the link length), 5 the seven-joint arm of kind 2 carrying the box
// on a passive universal joint (Sec. IV-C and its appendix, phase I): a
// massless ring turning about the flange x axis, then the box about the
// ring's y axis; theta = the box's inertia about its centre of mass (xx,
// yy, zz, xy, xz, yz), its centre of mass and the viscous friction of the
// two joint axes; the observation is the box frame (origin and the points
// 1 m along its x, y, z axes, in world coordinates), 6 the same mount
// with the box's inertia and the joints' friction known and theta the
// in-plane positions of two point masses on the box floor (phase II).
typedef struct {
  int32_t kind;
  int32_t n_dof;
  int32_t M;
  int32_t d_x;
  int32_t obs_index[16];
  double gravity[3];
  double damping[8];
  double dh_a[7], dh_alpha[7], dh_d[7];
  double link_m[7], link_c[7][3], link_I[7][3];
  double kp[7], kd[7], qc[7], amp[7], omega[7], phase[7];
  double flange_d;
  double box_m, box_c[3], box_I[3];
  double pm_m, pm_z;
  double box_Ioff[3];  // kind 6: the box's products of inertia xy, xz, yz
  double ujoint_b[2];  // kind 6: viscous friction of the two joint axes
} OrcModel;

typedef struct {
  int32_t N, K, T, n_s, h, combine;  // combine: 0 sum (GMM), 1 product
  int32_t lik;  // 0: defects as MDMM constraints; 1: defect densities inside p_ms
  double dt, sigma_def, c;
  const double* w_x;      // [d_x]   observation weights (1 / sigma_obs)
  const double* u;        // [d_s]   defect state scales
  const double* s0;       // [K, d_s]
  const double* obs;      // [K, T, d_x]; row t-1 observes state t
  const double* theta;    // [N, M]
  const double* S;        // [N, K, n_s-1, d_s]; S[.., j-1, :] starts window j
  const double* lam_def;  // [N, K, n_s-1]
} OrcProblem;

}  // extern "C"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxB = 10;  // bodies of the longest chain (the U-joint arm has 9)

template <class S>
struct Chain {
  int n;
  Xform<S> Xtree[kMaxB];
  int jtype[kMaxB];  // 0 revolute, 1 prismatic
  double axis[kMaxB][3];
  M6<S> I[kMaxB];
};

template <class S>
M3<S> diag3(const S& a, const S& b, const S& c) {
  M3<S> m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = S(0.0);
  m.a[0][0] = a; m.a[1][1] = b; m.a[2][2] = c;
  return m;
}

// Parameter slots of the rigid planar chain (kind 4): link 0 holds (m, I,
// cx, cy, b); every further link i holds (L, m, I, cx, cy, b), L being the
// distance from joint i-1 to joint i.
inline int rigid_base(int i) { return i == 0 ? 0 : 5 + 6 * (i - 1); }
inline int rigid_slot(int i, int f) { return rigid_base(i) + (i > 0 ? 1 : 0) + f; }  // f: 0 m, 1 I, 2 cx, 3 cy, 4 b

// Builds the articulated chain for parameters theta.  Planar chain: theta =
// (m_1..m_n, l_1..l_n).  Rigid planar chain: see rigid_slot().  Arm: theta = (x_a, y_a, x_b, y_b), the in-plane
// positions of the two point masses in the hinge frame.  Toy: theta drives
// the force only.
template <class S>
Chain<S> build_chain(const OrcModel& md, const S* th) {
  Chain<S> ch;
  ch.n = md.n_dof;
  if (md.kind == 1) {
    const int n = md.n_dof;
    for (int i = 0; i < n; ++i) {
      ch.Xtree[i].E = m3ident<S>();
      ch.Xtree[i].r = (i == 0) ? v3zero<S>() : v3<S>(S(0.0), -th[n + i - 1], S(0.0));
      ch.jtype[i] = 0;
      ch.axis[i][0] = 0.0; ch.axis[i][1] = 0.0; ch.axis[i][2] = 1.0;
      ch.I[i] = rbi<S>(th[i], v3<S>(S(0.0), -th[n + i], S(0.0)), diag3<S>(S(0.0), S(0.0), S(0.0)));
    }
  } else if (md.kind == 4) {
    for (int i = 0; i < md.n_dof; ++i) {
      ch.Xtree[i].E = m3ident<S>();
      ch.Xtree[i].r = (i == 0) ? v3zero<S>() : v3<S>(S(0.0), -th[rigid_base(i)], S(0.0));
      ch.jtype[i] = 0;
      ch.axis[i][0] = 0.0; ch.axis[i][1] = 0.0; ch.axis[i][2] = 1.0;
      // Only the inertia about the joint axis acts in planar motion; the
      // other two principal moments are set equal to it.
      const S Iz = th[rigid_slot(i, 1)];
      ch.I[i] = rbi<S>(th[rigid_slot(i, 0)], v3<S>(th[rigid_slot(i, 2)], th[rigid_slot(i, 3)], S(0.0)),
                       diag3<S>(Iz, Iz, Iz));
    }
  } else if (md.kind == 2 || md.kind == 5 || md.kind == 6) {
    for (int i = 0; i < 7; ++i) {
      const double ca = std::cos(md.dh_alpha[i]), sa = std::sin(md.dh_alpha[i]);
      // Rot_x(alpha) as an active rotation; the coordinate transform is its transpose.
      M3<S> Rx;
      Rx.a[0][0] = S(1.0); Rx.a[0][1] = S(0.0); Rx.a[0][2] = S(0.0);
      Rx.a[1][0] = S(0.0); Rx.a[1][1] = S(ca);  Rx.a[1][2] = S(-sa);
      Rx.a[2][0] = S(0.0); Rx.a[2][1] = S(sa);  Rx.a[2][2] = S(ca);
      ch.Xtree[i].E = m3T(Rx);
      ch.Xtree[i].r = v3<S>(S(md.dh_a[i]), S(-md.dh_d[i] * sa), S(md.dh_d[i] * ca));
      ch.jtype[i] = 0;
      ch.axis[i][0] = 0.0; ch.axis[i][1] = 0.0; ch.axis[i][2] = 1.0;
      ch.I[i] = rbi<S>(S(md.link_m[i]), v3<S>(S(md.link_c[i][0]), S(md.link_c[i][1]), S(md.link_c[i][2])),
                       diag3<S>(S(md.link_I[i][0]), S(md.link_I[i][1]), S(md.link_I[i][2])));
    }
    ch.Xtree[7].E = m3ident<S>();
    ch.Xtree[7].r = v3<S>(S(0.0), S(0.0), S(md.flange_d));
    ch.jtype[7] = 0;
    ch.axis[7][0] = 1.0; ch.axis[7][1] = 0.0; ch.axis[7][2] = 0.0;
    const M3<S> zero3 = diag3<S>(S(0.0), S(0.0), S(0.0));
    if (md.kind == 5 || md.kind == 6) {
      // massless ring, then the box about the ring's y axis at the same point
      ch.I[7] = rbi<S>(S(0.0), v3zero<S>(), zero3);
      ch.Xtree[8].E = m3ident<S>();
      ch.Xtree[8].r = v3zero<S>();
      ch.jtype[8] = 0;
      ch.axis[8][0] = 0.0; ch.axis[8][1] = 1.0; ch.axis[8][2] = 0.0;
      M3<S> Ic;
      if (md.kind == 6) {
        Ic.a[0][0] = S(md.box_I[0]); Ic.a[1][1] = S(md.box_I[1]); Ic.a[2][2] = S(md.box_I[2]);
        Ic.a[0][1] = Ic.a[1][0] = S(md.box_Ioff[0]);
        Ic.a[0][2] = Ic.a[2][0] = S(md.box_Ioff[1]);
        Ic.a[1][2] = Ic.a[2][1] = S(md.box_Ioff[2]);
        const M6<S> Ib = rbi<S>(S(md.box_m), v3<S>(S(md.box_c[0]), S(md.box_c[1]), S(md.box_c[2])), Ic);
        const M6<S> Ia = rbi<S>(S(md.pm_m), v3<S>(th[0], th[1], S(md.pm_z)), zero3);
        const M6<S> Ibb = rbi<S>(S(md.pm_m), v3<S>(th[2], th[3], S(md.pm_z)), zero3);
        ch.I[8] = m6add(m6add(Ib, Ia), Ibb);
        return ch;
      }
      Ic.a[0][0] = th[0]; Ic.a[1][1] = th[1]; Ic.a[2][2] = th[2];
      Ic.a[0][1] = Ic.a[1][0] = th[3];
      Ic.a[0][2] = Ic.a[2][0] = th[4];
      Ic.a[1][2] = Ic.a[2][1] = th[5];
      ch.I[8] = rbi<S>(S(md.box_m), v3<S>(th[6], th[7], th[8]), Ic);
      return ch;
    }
    M6<S> Ib = rbi<S>(S(md.box_m), v3<S>(S(md.box_c[0]), S(md.box_c[1]), S(md.box_c[2])),
                      diag3<S>(S(md.box_I[0]), S(md.box_I[1]), S(md.box_I[2])));
    M6<S> Ia = rbi<S>(S(md.pm_m), v3<S>(th[0], th[1], S(md.pm_z)), zero3);
    M6<S> Ibb = rbi<S>(S(md.pm_m), v3<S>(th[2], th[3], S(md.pm_z)), zero3);
    ch.I[7] = m6add(m6add(Ib, Ia), Ibb);
  } else {
    ch.Xtree[0].E = m3ident<S>();
    ch.Xtree[0].r = v3zero<S>();
    ch.jtype[0] = 1;
    ch.axis[0][0] = 1.0; ch.axis[0][1] = 0.0; ch.axis[0][2] = 0.0;
    ch.I[0] = rbi<S>(S(1.0), v3zero<S>(), diag3<S>(S(0.0), S(0.0), S(0.0)));
  }
  return ch;
}

// Joint torques as explicit functions of time (App. B-A: controls enter
// f_step through t).
template <class S>
void joint_torque(const OrcModel& md, const S* th, double time, const S* q, const S* qd, S* tau) {
  if (md.kind == 1) {
    for (int i = 0; i < md.n_dof; ++i) tau[i] = -(md.damping[i] * qd[i]);
  } else if (md.kind == 4) {
    for (int i = 0; i < md.n_dof; ++i) tau[i] = -(th[rigid_slot(i, 4)] * qd[i]);
  } else if (md.kind == 2 || md.kind == 5 || md.kind == 6) {
    for (int i = 0; i < 7; ++i) {
      const double ph = md.omega[i] * time + md.phase[i];
      const double qdes = md.qc[i] + md.amp[i] * std::sin(ph);
      const double qddes = md.amp[i] * md.omega[i] * std::cos(ph);
      tau[i] = md.kp[i] * (qdes - q[i]) + md.kd[i] * (qddes - qd[i]);
    }
    if (md.kind == 2) {
      tau[7] = -(md.damping[7] * qd[7]);
    } else if (md.kind == 6) {
      tau[7] = -(md.ujoint_b[0] * qd[7]);
      tau[8] = -(md.ujoint_b[1] * qd[8]);
    } else {
      tau[7] = -(th[9] * qd[7]);
      tau[8] = -(th[10] * qd[8]);
    }
  } else {
    tau[0] = th[0];
    if (md.M >= 2) tau[0] = tau[0] + th[1] * time;
  }
}

template <class S>
SV<S> motion_subspace(const Chain<S>& ch, int i) {
  SV<S> s = svzero<S>();
  const int off = (ch.jtype[i] == 0) ? 0 : 3;
  for (int d = 0; d < 3; ++d) s.a[off + d] = S(ch.axis[i][d]);
  return s;
}

template <class S>
Xform<S> joint_xform(const Chain<S>& ch, int i, const S& q) {
  Xform<S> XJ;
  if (ch.jtype[i] == 0) {
    XJ.E = m3T(rodrigues<S>(ch.axis[i], q));
    XJ.r = v3zero<S>();
  } else {
    XJ.E = m3ident<S>();
    XJ.r = v3<S>(q * ch.axis[i][0], q * ch.axis[i][1], q * ch.axis[i][2]);
  }
  return XJ;
}

// U U^T / D for the articulated-inertia update.
template <class S>
M6<S> m6v_outer_div(const SV<S>& Uv, const S& D) {
  M6<S> m;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) m.a[i][j] = Uv.a[i] * Uv.a[j] / D;
  return m;
}

// Articulated Body Algorithm: three passes over the chain (outward
// velocities and bias terms, inward articulated inertias, outward
// accelerations).  Gravity enters as a fictitious base acceleration.
template <class S>
void aba(const Chain<S>& ch, const double g[3], const S* q, const S* qd, const S* tau, S* qdd) {
  const int n = ch.n;
  Xform<S> X[kMaxB];
  SV<S> Sj[kMaxB], v[kMaxB], c[kMaxB], pA[kMaxB], U[kMaxB], a[kMaxB];
  M6<S> IA[kMaxB];
  S D[kMaxB], uu[kMaxB];
  for (int i = 0; i < n; ++i) {
    X[i] = xcompose(joint_xform(ch, i, q[i]), ch.Xtree[i]);
    Sj[i] = motion_subspace(ch, i);
    const SV<S> vJ = svscale(Sj[i], qd[i]);
    const SV<S> vp = (i == 0) ? svzero<S>() : v[i - 1];
    v[i] = svadd(m6v(xmat(X[i]), vp), vJ);
    c[i] = crm(v[i], vJ);
    IA[i] = ch.I[i];
    pA[i] = crf(v[i], m6v(ch.I[i], v[i]));
  }
  for (int i = n - 1; i >= 0; --i) {
    U[i] = m6v(IA[i], Sj[i]);
    D[i] = svdot(Sj[i], U[i]);
    uu[i] = tau[i] - svdot(Sj[i], pA[i]);
    if (i > 0) {
      const M6<S> Ia = m6sub(IA[i], m6v_outer_div(U[i], D[i]));
      const SV<S> pa = svadd(svadd(pA[i], m6v(Ia, c[i])), svscale(U[i], uu[i] / D[i]));
      const M6<S> Xm = xmat(X[i]);
      IA[i - 1] = m6add(IA[i - 1], m6mul(m6T(Xm), m6mul(Ia, Xm)));
      pA[i - 1] = svadd(pA[i - 1], m6v(m6T(Xm), pa));
    }
  }
  SV<S> a0 = svzero<S>();
  for (int d = 0; d < 3; ++d) a0.a[3 + d] = S(-g[d]);
  for (int i = 0; i < n; ++i) {
    const SV<S> ap = (i == 0) ? a0 : a[i - 1];
    const SV<S> a1 = svadd(m6v(xmat(X[i]), ap), c[i]);
    qdd[i] = (uu[i] - svdot(U[i], a1)) / D[i];
    a[i] = svadd(a1, svscale(Sj[i], qdd[i]));
  }
}


// Composite-rigid-body algorithm (joint-space inertia H) and recursive
// Newton-Euler with zero acceleration (bias C, gravity included).  Used only
// as an independent cross-check of aba(): qdd = H^{-1} (tau - C).
void crba_rnea(const Chain<double>& ch, const double g[3], const double* q, const double* qd,
               double* H, double* C) {
  const int n = ch.n;
  Xform<double> X[kMaxB];
  SV<double> Sj[kMaxB], v[kMaxB], a[kMaxB], f[kMaxB];
  SV<double> a0 = svzero<double>();
  for (int d = 0; d < 3; ++d) a0.a[3 + d] = -g[d];
  for (int i = 0; i < n; ++i) {
    X[i] = xcompose(joint_xform(ch, i, q[i]), ch.Xtree[i]);
    Sj[i] = motion_subspace(ch, i);
    const SV<double> vJ = svscale(Sj[i], qd[i]);
    const SV<double> vp = (i == 0) ? svzero<double>() : v[i - 1];
    const SV<double> ap = (i == 0) ? a0 : a[i - 1];
    v[i] = svadd(m6v(xmat(X[i]), vp), vJ);
    a[i] = svadd(m6v(xmat(X[i]), ap), crm(v[i], vJ));
    f[i] = svadd(m6v(ch.I[i], a[i]), crf(v[i], m6v(ch.I[i], v[i])));
  }
  for (int i = n - 1; i >= 0; --i) {
    C[i] = svdot(Sj[i], f[i]);
    if (i > 0) f[i - 1] = svadd(f[i - 1], m6v(m6T(xmat(X[i])), f[i]));
  }
  M6<double> IC[kMaxB];
  for (int i = 0; i < n; ++i) IC[i] = ch.I[i];
  for (int i = n - 1; i >= 0; --i)
    if (i > 0) IC[i - 1] = m6add(IC[i - 1], m6mul(m6T(xmat(X[i])), m6mul(IC[i], xmat(X[i]))));
  for (int i = 0; i < n; ++i) {
    SV<double> F = m6v(IC[i], Sj[i]);
    H[i * n + i] = svdot(Sj[i], F);
    int j = i;
    while (j > 0) {
      F = m6v(m6T(xmat(X[j])), F);
      j = j - 1;
      H[i * n + j] = svdot(Sj[j], F);
      H[j * n + i] = H[i * n + j];
    }
  }
}

// One semi-implicit Euler step (App. B-A eq. "dynamics"): the acceleration
// from ABA at (q_t, qd_t, tau(t)) updates the velocity first, and the new
// velocity updates the position.
template <class S>
void step(const OrcModel& md, const Chain<S>& ch, const S* th, double time, double dt, S* q, S* qd) {
  S tau[kMaxB], qdd[kMaxB];
  joint_torque<S>(md, th, time, q, qd, tau);
  aba<S>(ch, md.gravity, q, qd, tau, qdd);
  for (int i = 0; i < md.n_dof; ++i) qd[i] = qd[i] + dt * qdd[i];
  for (int i = 0; i < md.n_dof; ++i) q[i] = q[i] + dt * qd[i];
}

// World-frame points of the last body's frame: its origin, then the points
// 1 m along its x, y and z axes (12 numbers).  Each transform X = (E, r)
// holds the rotation from parent to body coordinates and the body origin in
// parent coordinates, so the body-to-world rotation is R_parent E^T and the
// origin o_parent + R_parent r.
template <class S>
void frame_points(const Chain<S>& ch, const S* q, S* x) {
  M3<S> R = m3ident<S>();
  V3<S> o = v3zero<S>();
  for (int i = 0; i < ch.n; ++i) {
    const Xform<S> X = xcompose(joint_xform(ch, i, q[i]), ch.Xtree[i]);
    o = add(o, m3v(R, X.r));
    R = m3mul(R, m3T(X.E));
  }
  for (int d = 0; d < 3; ++d) {
    x[d] = o.x[d];
    for (int a = 0; a < 3; ++a) x[3 + 3 * a + d] = o.x[d] + R.a[d][a];
  }
}

// The observed quantities of a state: the box-frame points for kind 5,
// otherwise the state components listed in obs_index.
template <class S>
void observe(const OrcModel& md, const Chain<S>& ch, const S* q, const S* qd, S* x) {
  if (md.kind == 5 || md.kind == 6) {
    frame_points<S>(ch, q, x);
    return;
  }
  for (int d = 0; d < md.d_x; ++d) {
    const int si = md.obs_index[d];
    x[d] = (si < md.n_dof) ? q[si] : qd[si - md.n_dof];
  }
}

// One multiple-shooting window (Sec. III-C): start at state `start` at step
// j*h, take h steps, and accumulate the Gaussian log-likelihood
// (eq. "combinedlikelihood") of the observations of steps j*h+1..(j+1)*h.
// Returns the end state; optionally writes the h visited states.
template <class S>
S window(const OrcModel& md, const OrcProblem& pr, const S* th, const S* start, int k, int j,
         S* end_state, double* traj /* [h, d_s] or null */) {
  const int n = md.n_dof, ds = 2 * n;
  const Chain<S> ch = build_chain<S>(md, th);
  S q[kMaxB], qd[kMaxB];
  for (int i = 0; i < n; ++i) { q[i] = start[i]; qd[i] = start[n + i]; }
  const double log_sqrt_2pi = 0.5 * std::log(2.0 * kPi);
  S ll(0.0);
  for (int s = 0; s < pr.h; ++s) {
    const int t = j * pr.h + s;  // index of the state the step starts from
    step<S>(md, ch, th, t * pr.dt, pr.dt, q, qd);
    const double* x_real = pr.obs + ((size_t)k * pr.T + t) * md.d_x;  // observes state t+1
    S xs[16];
    observe<S>(md, ch, q, qd, xs);
    for (int d = 0; d < md.d_x; ++d) {
      const S r = (x_real[d] - xs[d]) * pr.w_x[d];
      ll = ll - 0.5 * (r * r) - (log_sqrt_2pi - std::log(pr.w_x[d]));
    }
    if (traj)
      for (int i = 0; i < n; ++i) {
        traj[s * ds + i] = val(q[i]);
        traj[s * ds + n + i] = val(qd[i]);
      }
  }
  for (int i = 0; i < n; ++i) { end_state[i] = q[i]; end_state[n + i] = qd[i]; }
  return ll;
}

const double* start_state(const OrcProblem& pr, int ds, int i, int k, int j) {
  if (j == 0) return pr.s0 + (size_t)k * ds;
  return pr.S + (((size_t)i * pr.K + k) * (pr.n_s - 1) + (j - 1)) * ds;
}

// Defect constraint of Sec. III-E: g_def = ||(S_{j+1} - s_end) * u||^2 / sigma_def^2.
double defect(const OrcProblem& pr, int ds, const double* S_next, const double* s_end) {
  double g = 0.0;
  for (int d = 0; d < ds; ++d) {
    const double e = (S_next[d] - s_end[d]) * pr.u[d];
    g += e * e;
  }
  return g / (pr.sigma_def * pr.sigma_def);
}

// Log density of defect g (eq. "likelihood-defect"): the shooting state
// S ~ N(s_end, sigma_def^2 / u_d^2) per state dimension, i.e.
// -g / 2 + sum_d log(u_d / (sigma_def sqrt(2 pi))).
double defect_log_density(const OrcProblem& pr, int ds, double g) {
  double lp = -0.5 * g;
  for (int d = 0; d < ds; ++d) lp += std::log(pr.u[d] / (pr.sigma_def * std::sqrt(2.0 * kPi)));
  return lp;
}

// Combination over trajectories: eq. "traj_likelihood" (equally weighted
// mixture, evaluated in log space with the 1/K weight) or App. A-B
// eq. "traj_likelihood_prod".  Returns log p and writes the weights
// w_k = d log p / d l_k.
double combine(const OrcProblem& pr, const double* l_k, double* w) {
  const int K = pr.K;
  if (pr.combine == 1) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) { s += l_k[k]; w[k] = 1.0; }
    return s;
  }
  double mx = l_k[0];
  for (int k = 1; k < K; ++k) mx = std::max(mx, l_k[k]);
  double z = 0.0;
  for (int k = 0; k < K; ++k) z += std::exp(l_k[k] - mx);
  for (int k = 0; k < K; ++k) w[k] = std::exp(l_k[k] - mx) / z;
  return mx + std::log(z) - std::log((double)K);
}

template <int P>
void window_grad(const OrcModel& md, const OrcProblem& pr, const double* th, const double* start,
                 int k, int j, double* ll, double* dl_dth, double* dl_ds, double* send,
                 double* dsend_dth /* [d_s][M] */, double* dsend_ds /* [d_s][d_s] */) {
  const int M = md.M, ds = 2 * md.n_dof;
  Dual<P> thd[16], sd[2 * kMaxB], ed[2 * kMaxB];
  for (int m = 0; m < M; ++m) { thd[m] = Dual<P>(th[m]); thd[m].d[m] = 1.0; }
  for (int d = 0; d < ds; ++d) { sd[d] = Dual<P>(start[d]); sd[d].d[M + d] = 1.0; }
  const Dual<P> l = window<Dual<P>>(md, pr, thd, sd, k, j, ed, nullptr);
  *ll = l.v;
  for (int m = 0; m < M; ++m) dl_dth[m] = l.d[m];
  for (int d = 0; d < ds; ++d) dl_ds[d] = l.d[M + d];
  for (int d = 0; d < ds; ++d) {
    send[d] = ed[d].v;
    for (int m = 0; m < M; ++m) dsend_dth[d * M + m] = ed[d].d[m];
    for (int e = 0; e < ds; ++e) dsend_ds[d * ds + e] = ed[d].d[M + e];
  }
}

}  // namespace

extern "C" {

int orc_version(void) { return 1; }

// Threads the OpenMP loops use.
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Sets the thread count of later OpenMP loops (timing on one core).
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Joint torques at time `time` (for tests of the controllers).
void orc_tau(const OrcModel* md, const double* th, double time, const double* q, const double* qd, double* tau) {
  joint_torque<double>(*md, th, time, q, qd, tau);
}

void orc_aba(const OrcModel* md, const double* th, const double* q, const double* qd, const double* tau,
             double* qdd) {
  const Chain<double> ch = build_chain<double>(*md, th);
  aba<double>(ch, md->gravity, q, qd, tau, qdd);
}

void orc_crba_rnea(const OrcModel* md, const double* th, const double* q, const double* qd, double* H,
                   double* C) {
  const Chain<double> ch = build_chain<double>(*md, th);
  crba_rnea(ch, md->gravity, q, qd, H, C);
}

// Single-shooting rollout of n_steps from state s0 at step index t0:
// f_sim of Sec. II, writing states t0+1 .. t0+n_steps.
// Observed quantities (d_x numbers) of the states (q, qd) under parameters th.
void orc_observe(const OrcModel* md, const double* th, const double* q, const double* qd, double* x) {
  const Chain<double> ch = build_chain<double>(*md, th);
  observe<double>(*md, ch, q, qd, x);
}

void orc_rollout(const OrcModel* md, const double* th, const double* s0, int t0, int n_steps, double dt,
                 double* traj) {
  const int n = md->n_dof, ds = 2 * n;
  const Chain<double> ch = build_chain<double>(*md, th);
  double q[kMaxB], qd[kMaxB];
  for (int i = 0; i < n; ++i) { q[i] = s0[i]; qd[i] = s0[n + i]; }
  for (int s = 0; s < n_steps; ++s) {
    step<double>(*md, ch, th, (t0 + s) * dt, dt, q, qd);
    for (int i = 0; i < n; ++i) { traj[s * ds + i] = q[i]; traj[s * ds + n + i] = qd[i]; }
  }
}

// Forward pass for selected particles: per-window end states, visited
// states (optional), window log-likelihoods, defects, and the combined
// log-likelihood with its trajectory weights.
void orc_forward(const OrcModel* md, const OrcProblem* pr, int n_sel, const int* sel, double* traj,
                 double* end_states, double* ll_win, double* gdef, double* logp, double* wk) {
  const int ds = 2 * md->n_dof, K = pr->K, ns = pr->n_s, M = md->M;
  const int units = n_sel * K * ns;
#pragma omp parallel for schedule(dynamic, 4)
  for (int u = 0; u < units; ++u) {
    const int s = u / (K * ns), k = (u / ns) % K, j = u % ns;
    const int i = sel[s];
    const double* th = pr->theta + (size_t)i * M;
    double* tr = traj ? traj + (((size_t)s * K + k) * pr->T + (size_t)j * pr->h) * ds : nullptr;
    ll_win[u] = window<double>(*md, *pr, th, start_state(*pr, ds, i, k, j), k, j, end_states + (size_t)u * ds, tr);
  }
  for (int s = 0; s < n_sel; ++s) {
    const int i = sel[s];
    std::vector<double> lk(K);
    for (int k = 0; k < K; ++k) {
      for (int j = 0; j + 1 < ns; ++j) {
        const size_t u = ((size_t)s * K + k) * ns + j;
        const double g = defect(*pr, ds, start_state(*pr, ds, i, k, j + 1), end_states + u * ds);
        gdef[((size_t)s * K + k) * (ns - 1) + j] = g;
        // eq. "ms_likelihood": the defect density is a factor of p_ms
        if (pr->lik == 1) ll_win[u] += defect_log_density(*pr, ds, g);
      }
      double acc = 0.0;
      for (int j = 0; j < ns; ++j) acc += ll_win[((size_t)s * K + k) * ns + j];
      lk[k] = acc;
    }
    logp[s] = combine(*pr, lk.data(), wk + (size_t)s * K);
  }
}

// Gradients for selected particles by forward-mode dual numbers, assembled
// into the MDMM flow of Sec. III-E / Algorithm 1:
//   g_obs[i]  = d log p_obs / d theta                (enters phi)
//   g_con[i]  = sum_{k,j} (lam_def + c g_def) d g_def / d theta
//   S_dot     = w_ik d l_ikj / d S_j - d Phi / d S_j  (Phi = lam g + c/2 g^2)
// With lik = 1 the defect densities are factors of p_ms (eq. "ms_likelihood"):
// l_ikj gains log p_def of window j's defect, g_obs and S_dot carry its
// derivatives with the trajectory weights, and g_con is zero.
// Also returns the forward quantities of orc_forward.  Returns 0, or -1 if
// M + d_s exceeds the compiled dual width.
int orc_gradient(const OrcModel* md, const OrcProblem* pr, int n_sel, const int* sel, double* end_states,
                 double* ll_win, double* gdef, double* logp, double* wk, double* g_obs, double* g_con,
                 double* S_dot, double* dl_dth_unit /* [n_sel,K,n_s,M] or null */,
                 double* dcon_dth_unit /* [n_sel,K,n_s,M] or null */) {
  const int ds = 2 * md->n_dof, K = pr->K, ns = pr->n_s, M = md->M;
  const int P = M + ds;
  if (P > 32 || M > 16 || ds > 2 * kMaxB) return -1;
  const int units = n_sel * K * ns;
  std::vector<double> dl_dth((size_t)units * M), dl_ds((size_t)units * ds);
  std::vector<double> dse_dth((size_t)units * ds * M), dse_ds((size_t)units * ds * ds);
#pragma omp parallel for schedule(dynamic, 2)
  for (int u = 0; u < units; ++u) {
    const int s = u / (K * ns), k = (u / ns) % K, j = u % ns;
    const int i = sel[s];
    const double* th = pr->theta + (size_t)i * M;
    const double* st = start_state(*pr, ds, i, k, j);
    double* a0 = &dl_dth[(size_t)u * M];
    double* a1 = &dl_ds[(size_t)u * ds];
    double* a2 = end_states + (size_t)u * ds;
    double* a3 = &dse_dth[(size_t)u * ds * M];
    double* a4 = &dse_ds[(size_t)u * ds * ds];
    if (P <= 4) window_grad<4>(*md, *pr, th, st, k, j, &ll_win[u], a0, a1, a2, a3, a4);
    else if (P <= 8) window_grad<8>(*md, *pr, th, st, k, j, &ll_win[u], a0, a1, a2, a3, a4);
    else if (P <= 20) window_grad<20>(*md, *pr, th, st, k, j, &ll_win[u], a0, a1, a2, a3, a4);
    else window_grad<32>(*md, *pr, th, st, k, j, &ll_win[u], a0, a1, a2, a3, a4);
  }
  if (dcon_dth_unit)
    for (size_t t = 0; t < (size_t)units * M; ++t) dcon_dth_unit[t] = 0.0;
  const double inv_s2 = 1.0 / (pr->sigma_def * pr->sigma_def);
  const bool in_lik = pr->lik == 1;
  for (int s = 0; s < n_sel; ++s) {
    const int i = sel[s];
    // defects first: with the densities inside p_ms (eq. "ms_likelihood")
    // their log densities join the window terms, and d log p_def / d s_end
    // = -(1/2) d g / d s_end joins the window's theta gradient through
    // d s_end / d theta
    for (int k = 0; k < K; ++k)
      for (int j = 0; j + 1 < ns; ++j) {
        const size_t u = ((size_t)s * K + k) * ns + j;
        const double* Snext = start_state(*pr, ds, i, k, j + 1);
        const double* se = end_states + u * ds;
        const double g = defect(*pr, ds, Snext, se);
        gdef[((size_t)s * K + k) * (ns - 1) + j] = g;
        if (!in_lik) continue;
        ll_win[u] += defect_log_density(*pr, ds, g);
        for (int m = 0; m < M; ++m) {
          double acc = 0.0;
          for (int d = 0; d < ds; ++d) {
            const double e = (Snext[d] - se[d]) * pr->u[d];
            acc += (e * pr->u[d] * inv_s2) * dse_dth[(u * ds + d) * M + m];  // -(1/2) d g / d s_end = e u / sigma^2
          }
          dl_dth[u * M + m] += acc;
        }
        for (int c = 0; c < ds; ++c) {
          double acc = 0.0;
          for (int d = 0; d < ds; ++d) {
            const double e = (Snext[d] - se[d]) * pr->u[d];
            acc += (e * pr->u[d] * inv_s2) * dse_ds[(u * ds + d) * ds + c];
          }
          dl_ds[u * ds + c] += acc;
        }
      }
    std::vector<double> lk(K);
    for (int k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int j = 0; j < ns; ++j) acc += ll_win[((size_t)s * K + k) * ns + j];
      lk[k] = acc;
    }
    double* w = wk + (size_t)s * K;
    logp[s] = combine(*pr, lk.data(), w);
    for (int m = 0; m < M; ++m) { g_obs[(size_t)s * M + m] = 0.0; g_con[(size_t)s * M + m] = 0.0; }
    for (int k = 0; k < K; ++k) {
      for (int j = 0; j < ns; ++j) {
        const size_t u = ((size_t)s * K + k) * ns + j;
        for (int m = 0; m < M; ++m) g_obs[(size_t)s * M + m] += w[k] * dl_dth[u * M + m];
      }
      for (int j = 1; j < ns; ++j) {
        double* sd = S_dot + (((size_t)s * K + k) * (ns - 1) + (j - 1)) * ds;
        const size_t u = ((size_t)s * K + k) * ns + j;
        for (int d = 0; d < ds; ++d) sd[d] = w[k] * dl_ds[u * ds + d];
      }
      for (int j = 0; j + 1 < ns; ++j) {
        const size_t u = ((size_t)s * K + k) * ns + j;
        const double* Snext = start_state(*pr, ds, i, k, j + 1);
        const double* se = end_states + u * ds;
        double* sn = S_dot + (((size_t)s * K + k) * (ns - 1) + j) * ds;
        if (in_lik) {
          // direct dependence of the defect density on its target S_{j+1}:
          // d log p_def / d S_next = -e u / sigma^2, weighted like the window
          for (int d = 0; d < ds; ++d) {
            const double e = (Snext[d] - se[d]) * pr->u[d];
            sn[d] += w[k] * (-e * pr->u[d] * inv_s2);
          }
          continue;
        }
        const double g = gdef[((size_t)s * K + k) * (ns - 1) + j];
        const double lam = pr->lam_def[((size_t)i * K + k) * (ns - 1) + j];
        const double mult = lam + pr->c * g;  // d Phi / d g
        // d g / d s_end = -2 e u / sigma^2 with e = (S_next - s_end) u
        double dg_dse[2 * kMaxB];
        for (int d = 0; d < ds; ++d) {
          const double e = (Snext[d] - se[d]) * pr->u[d];
          dg_dse[d] = -2.0 * e * pr->u[d] * inv_s2;
        }
        for (int m = 0; m < M; ++m) {
          double acc = 0.0;
          for (int d = 0; d < ds; ++d) acc += dg_dse[d] * dse_dth[(u * ds + d) * M + m];
          g_con[(size_t)s * M + m] += mult * acc;
          if (dcon_dth_unit) dcon_dth_unit[u * M + m] = mult * acc;
        }
        // window j's start state is a variable only for j >= 1
        if (j >= 1) {
          double* sd = S_dot + (((size_t)s * K + k) * (ns - 1) + (j - 1)) * ds;
          for (int e = 0; e < ds; ++e) {
            double acc = 0.0;
            for (int d = 0; d < ds; ++d) acc += dg_dse[d] * dse_ds[(u * ds + d) * ds + e];
            sd[e] -= mult * acc;
          }
        }
        // direct dependence of defect j on its target S_{j+1}: d g / d S_next = +2 e u / sigma^2
        for (int d = 0; d < ds; ++d) sn[d] -= mult * (-dg_dse[d]);
      }
    }
  }
  if (dl_dth_unit) std::memcpy(dl_dth_unit, dl_dth.data(), sizeof(double) * units * M);
  return 0;
}

// Median-heuristic bandwidth (Sec. III-A): distances between the N(N-1)/2
// distinct pairs, each coordinate difference scaled by 1/rho_m, sorted in
// full; the
// median (mean of the two middle values for an even count) gives
// h = med^2 / log N.  N = 1 or a vanishing median gives h = 1.
double orc_bandwidth(int N, int M, const double* theta, const double* rho, const int* live, double* med_out) {
  std::vector<double> d2;
  d2.reserve((size_t)N * (N - 1) / 2);
  int n_live = 0;
  for (int i = 0; i < N; ++i) n_live += (!live || live[i]) ? 1 : 0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {
      if (live && !(live[i] && live[j])) continue;
      double s = 0.0;
      for (int m = 0; m < M; ++m) {
        const double z = (theta[(size_t)i * M + m] - theta[(size_t)j * M + m]) * (1.0 / rho[m]);
        s += z * z;
      }
      d2.push_back(s);
    }
  double med = 0.0;
  if (!d2.empty()) {
    std::sort(d2.begin(), d2.end());
    const size_t P = d2.size();
    med = 0.5 * (std::sqrt(d2[(P - 1) / 2]) + std::sqrt(d2[P / 2]));
  }
  if (med_out) *med_out = med;
  if (n_live <= 1 || med * med < 1e-300) return 1.0;
  return med * med / std::log((double)n_live);
}

// SVGD direction of eq. "svgd_update" with k(a, b) = exp(-||(a - b)/rho||^2 / h):
// phi_i = (1/N) sum_j [ k(theta_j, theta_i) grad_j + grad_{theta_j} k(theta_j, theta_i) ].
// With `live` (NULL = every particle) the ensemble is the live particles
// alone: the sum runs over live j, N is their number, and a particle that
// is not live gets phi = 0.
void orc_phi(int N, int M, const double* theta, const double* grad, const double* rho, double h, const int* live,
             int n_sel, const int* sel, double* phi) {
  int n_live = 0;
  for (int j = 0; j < N; ++j) n_live += (!live || live[j]) ? 1 : 0;
  for (int s = 0; s < n_sel; ++s) {
    const int i = sel[s];
    for (int m = 0; m < M; ++m) phi[(size_t)s * M + m] = 0.0;
    if (live && !live[i]) continue;
    for (int j = 0; j < N; ++j) {
      if (live && !live[j]) continue;
      double d2 = 0.0;
      for (int m = 0; m < M; ++m) {
        const double z = (theta[(size_t)j * M + m] - theta[(size_t)i * M + m]) / rho[m];
        d2 += z * z;
      }
      const double kij = std::exp(-d2 / h);
      for (int m = 0; m < M; ++m) {
        const double dk = kij * (2.0 / h) * (theta[(size_t)i * M + m] - theta[(size_t)j * M + m]) / (rho[m] * rho[m]);
        phi[(size_t)s * M + m] += kij * grad[(size_t)j * M + m] + dk;
      }
    }
    for (int m = 0; m < M; ++m) phi[(size_t)s * M + m] /= (double)n_live;
  }
}

// One MDMM update (Sec. III-E, Algorithm 1), simultaneous for all variables:
//   g_lim = clamp(theta, lo, hi) - theta, d g_lim / d theta = -1 outside [lo, hi]
//   theta_dot = phi - (lam_lim + c g_lim) d g_lim/d theta - g_con
//   lam_lim_dot = g_lim, lam_def_dot = g_def, S_dot as given.
// optimizer 0: x += lr * x_dot.  optimizer 1: Adam on (theta, S) with -x_dot
// as the gradient (beta1 0.9, beta2 0.999, eps 1e-8), iteration `it` >= 1.
// Lagrange multipliers always take plain ascent steps of size eps_lam.
// Particles with frozen[i] != 0 (frozen may be NULL) keep every variable.
void orc_mdmm_step(int N, int M, int K, int n_s, int d_s, double c, const double* lo, const double* hi,
                   const double* phi, const double* g_con, const double* S_dot, const double* gdef,
                   const double* lr_theta, const double* lr_S, double eps_lam, int optimizer, int it,
                   double* theta, double* S, double* lam_lim, double* lam_def, double* adam_m, double* adam_v,
                   const int* frozen) {
  const int nS = K * (n_s - 1) * d_s;
  const int stride = M + nS;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int i = 0; i < N; ++i) {
    if (frozen && frozen[i]) continue;
    for (int m = 0; m < M; ++m) {
      const size_t im = (size_t)i * M + m;
      const double x = theta[im];
      const double cl = std::min(std::max(x, lo[m]), hi[m]);
      const double g = cl - x;
      const double dgdx = (x < lo[m] || x > hi[m]) ? -1.0 : 0.0;
      const double xdot = phi[im] - (lam_lim[im] + c * g) * dgdx - g_con[im];
      if (optimizer == 0) {
        theta[im] = x + lr_theta[m] * xdot;
      } else {
        const size_t a = (size_t)i * stride + m;
        const double gr = -xdot;
        adam_m[a] = b1 * adam_m[a] + (1.0 - b1) * gr;
        adam_v[a] = b2 * adam_v[a] + (1.0 - b2) * gr * gr;
        const double mh = adam_m[a] / (1.0 - std::pow(b1, it));
        const double vh = adam_v[a] / (1.0 - std::pow(b2, it));
        theta[im] = x - lr_theta[m] * mh / (std::sqrt(vh) + eps);
      }
      lam_lim[im] += eps_lam * g;
    }
    for (int e = 0; e < nS; ++e) {
      const size_t ie = (size_t)i * nS + e;
      const int d = e % d_s;
      const double xdot = S_dot[ie];
      if (optimizer == 0) {
        S[ie] += lr_S[d] * xdot;
      } else {
        const size_t a = (size_t)i * stride + M + e;
        const double gr = -xdot;
        adam_m[a] = b1 * adam_m[a] + (1.0 - b1) * gr;
        adam_v[a] = b2 * adam_v[a] + (1.0 - b2) * gr * gr;
        const double mh = adam_m[a] / (1.0 - std::pow(b1, it));
        const double vh = adam_v[a] / (1.0 - std::pow(b2, it));
        S[ie] -= lr_S[d] * mh / (std::sqrt(vh) + eps);
      }
    }
    for (int e = 0; e < K * (n_s - 1); ++e) {
      const size_t ie = (size_t)i * K * (n_s - 1) + e;
      lam_def[ie] += eps_lam * gdef[ie];
    }
  }
}

}  // extern "C"
