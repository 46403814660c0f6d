// Host check of the arm's step functions in FP64 (built with g++ and run by
// tests/test_arm_step_host.py), compiled for the kinematic structure the
// set-up finds in the table (Panda or generic; printed first).  Reads a
// model (mount, raw constants) and
// states from stdin; prints, per state, the joint accelerations of the
// library's Articulated Body Algorithm and (universal-joint mounts) the
// observed box-frame points, for comparison with the oracle; then checks
// the reverse step of both adjoint channels and the box-frame observation
// adjoint against central differences of the same functions and prints the
// worst relative errors.
#include <cstdio>
#include <random>
#include <vector>

#include "arm_math.h"

using namespace pds;

template <int BOX, int DH>
int run(const std::vector<float>& raw) {
  using AM = ArmMath<double, BOX, ArmConst, DH>;
  constexpr int NB = ArmShape<BOX>::NB, M = ArmShape<BOX>::M;
  ArmConst K;
  arm_setup(raw.data(), &K, BOX);
  int n = 0;
  if (scanf("%d", &n) != 1) return 2;
  std::vector<double> th_all;
  std::vector<double> q_all, qd_all, t_all;
  for (int c = 0; c < n; ++c) {
    double th[M], q[NB], qd[NB], t;
    for (int m = 0; m < M; ++m) if (scanf("%lf", &th[m]) != 1) return 2;
    for (int i = 0; i < NB; ++i) if (scanf("%lf", &q[i]) != 1) return 2;
    for (int i = 0; i < NB; ++i) if (scanf("%lf", &qd[i]) != 1) return 2;
    if (scanf("%lf", &t) != 1) return 2;
    typename AM::Tape T;
    AM::aba(K, th, q, qd, t, T);
    printf("qdd");
    for (int i = 0; i < NB; ++i) printf(" %.17g", T.qdd[i]);
    printf("\n");
    if (BOX != kHinge) {
      double x[12];
      AM::box_frame(K, q, x);
      printf("frame");
      for (int d = 0; d < 12; ++d) printf(" %.17g", x[d]);
      printf("\n");
    }
    th_all.insert(th_all.end(), th, th + M);
    q_all.insert(q_all.end(), q, q + NB);
    qd_all.insert(qd_all.end(), qd, qd + NB);
    t_all.push_back(t);
  }
  // reverse step of both channels against central differences of the step
  std::mt19937 g(5);
  std::normal_distribution<double> N01(0.0, 1.0);
  double worst_rev = 0.0, worst_obs = 0.0;
  const double dt = 1.0 / 240.0;
  for (int c = 0; c < n; ++c) {
    const double* th = &th_all[c * M];
    const double* q0 = &q_all[c * NB];
    const double* qd0 = &qd_all[c * NB];
    const double t = t_all[c];
    double qb[2][NB], qdb[2][NB], thb[2][M], sq[2][NB], sqd[2][NB];
    for (int ch = 0; ch < 2; ++ch) {
      for (int i = 0; i < NB; ++i) { sq[ch][i] = qb[ch][i] = N01(g); sqd[ch][i] = qdb[ch][i] = N01(g); }
      for (int m = 0; m < M; ++m) thb[ch][m] = 0.0;
    }
    typename AM::Tape T;
    AM::aba(K, th, q0, qd0, t, T);
    AM::step_rev(K, th, qd0, T, dt, qb, qdb, thb);
    for (int dir = 0; dir < 4; ++dir) {
      double dq[NB], dqd[NB], dth[M];
      for (int i = 0; i < NB; ++i) { dq[i] = N01(g); dqd[i] = N01(g); }
      for (int m = 0; m < M; ++m) dth[m] = N01(g) * 0.01;
      auto F = [&](double e, int ch) {
        double q[NB], qd[NB], tt[M];
        for (int i = 0; i < NB; ++i) { q[i] = q0[i] + e * dq[i]; qd[i] = qd0[i] + e * dqd[i]; }
        for (int m = 0; m < M; ++m) tt[m] = th[m] + e * dth[m];
        AM::step(K, tt, t, dt, q, qd);
        double s = 0.0;
        for (int i = 0; i < NB; ++i) s += sq[ch][i] * q[i] + sqd[ch][i] * qd[i];
        return s;
      };
      for (int ch = 0; ch < 2; ++ch) {
        const double e = 1e-6;
        const double fd = (F(e, ch) - F(-e, ch)) / (2 * e);
        double an = 0.0, scale = 0.0;
        for (int i = 0; i < NB; ++i) {
          an += qb[ch][i] * dq[i] + qdb[ch][i] * dqd[i];
          scale += std::fabs(qb[ch][i] * dq[i]) + std::fabs(qdb[ch][i] * dqd[i]);
        }
        for (int m = 0; m < M; ++m) { an += thb[ch][m] * dth[m]; scale += std::fabs(thb[ch][m] * dth[m]); }
        worst_rev = std::max(worst_rev, std::fabs(an - fd) / (scale + 1e-30));
      }
    }
    if (BOX != kHinge) {
      float obs[12], w[12];
      double x[12];
      AM::box_frame(K, q0, x);
      for (int d = 0; d < 12; ++d) { obs[d] = (float)(x[d] + 0.01 * N01(g)); w[d] = 100.0f; }
      double qbo[NB];
      for (int i = 0; i < NB; ++i) qbo[i] = 0.0;
      AM::template box_obs<true>(K, q0, obs, w, qbo);
      for (int i = 0; i < NB; ++i) {
        double qp[NB], qm[NB];
        for (int j = 0; j < NB; ++j) qp[j] = qm[j] = q0[j];
        const double e = 1e-6;
        qp[i] += e;
        qm[i] -= e;
        const double fd = -0.5 * (AM::template box_obs<false>(K, qp, obs, w, nullptr) - AM::template box_obs<false>(K, qm, obs, w, nullptr)) / (2 * e);
        worst_obs = std::max(worst_obs, std::fabs(qbo[i] - fd) / (1.0 + std::fabs(fd)));
      }
    }
  }
  printf("reverse %.3e\nobs_adjoint %.3e\n", worst_rev, worst_obs);
  return 0;
}

int main() {
  int mount = 0, nraw = 0;
  if (scanf("%d %d", &mount, &nraw) != 2) return 2;
  std::vector<float> raw(nraw);
  for (int i = 0; i < nraw; ++i) {
    double v;
    if (scanf("%lf", &v) != 1) return 2;
    raw[i] = (float)v;
  }
  // the structure the kernels would run for this table
  ArmConst K;
  arm_setup(raw.data(), &K, mount);
  printf("structure %d\n", K.dh);
  if (K.dh == kDhPanda) {
    if (mount == kUJoint) return run<kUJoint, kDhPanda>(raw);
    if (mount == kUJointWeights) return run<kUJointWeights, kDhPanda>(raw);
    return run<kHinge, kDhPanda>(raw);
  }
  if (mount == kUJoint) return run<kUJoint, kDhGeneric>(raw);
  if (mount == kUJointWeights) return run<kUJointWeights, kDhGeneric>(raw);
  return run<kHinge, kDhGeneric>(raw);
}
