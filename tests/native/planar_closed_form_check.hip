// Host check of the planar step functions in FP64: the two-link closed form
// against the generic ABA (run through the equivalent rigid-link
// parameters) and its reverse against central differences.  Built and run
// by tests/test_planar_closed_form.py.
#include "planar.hip"

namespace pds {
void count_arm_flops(int, double*, double*, double*) {}  // not needed here
}
#include <cstdio>
#include <random>
using namespace pds;
int main() {
  std::mt19937 g(1);
  std::uniform_real_distribution<double> U(-2, 2), Um(0.5, 2), Ul(0.5, 1.5);
  double worst_q = 0, worst_g = 0;
  for (int t = 0; t < 200; ++t) {
    Planar<2, double> P{};
    P.m[0] = Um(g); P.m[1] = Um(g); P.l[0] = Ul(g); P.l[1] = Ul(g);
    P.b[0] = 0.1 * Ul(g); P.b[1] = 0.1 * Ul(g); P.gx = 0.3 * U(g); P.gy = -9.81;
    double q[2] = {U(g), U(g)}, qd[2] = {U(g), U(g)};
    Tape<2, double> T;
    aba<2, double, false>(P, q, qd, T);
    // generic ABA through the rigid parameterisation: c = (0, -l), I = 0, L_1 = l_0
    Planar<2, double> Rg = P;
    for (int i = 0; i < 2; ++i) { Rg.I[i] = 0; Rg.cx[i] = 0; Rg.cy[i] = -P.l[i]; }
    Rg.L[0] = 0; Rg.L[1] = P.l[0];
    Tape<2, double> T2;
    aba<2, double, true>(Rg, q, qd, T2);
    for (int i = 0; i < 2; ++i) worst_q = std::max(worst_q, std::fabs(T.qdd[i] - T2.qdd[i]) / (1 + std::fabs(T2.qdd[i])));
    // reverse vs central differences of lambda . qdd
    double sb[2] = {U(g), U(g)};
    double qb[2] = {0, 0}, qdb[2] = {0, 0}, thb[4] = {0, 0, 0, 0};
    aba_rev<2, double, false>(P, qd, T, sb, qb, qdb, thb);
    auto F = [&](Planar<2, double> PP, double* qq, double* qqd) {
      Tape<2, double> TT; aba<2, double, false>(PP, qq, qqd, TT); return sb[0] * TT.qdd[0] + sb[1] * TT.qdd[1]; };
    const double e = 1e-6;
    double fd[8];
    for (int v = 0; v < 8; ++v) {
      Planar<2, double> Pp = P, Pm = P; double qp[2] = {q[0], q[1]}, qm[2] = {q[0], q[1]}, qdp[2] = {qd[0], qd[1]}, qdm[2] = {qd[0], qd[1]};
      if (v < 2) { qp[v] += e; qm[v] -= e; }
      else if (v < 4) { qdp[v - 2] += e; qdm[v - 2] -= e; }
      else if (v < 6) { Pp.m[v - 4] += e; Pm.m[v - 4] -= e; }
      else { Pp.l[v - 6] += e; Pm.l[v - 6] -= e; }
      fd[v] = (F(Pp, qp, qdp) - F(Pm, qm, qdm)) / (2 * e);
    }
    const double an[8] = {qb[0], qb[1], qdb[0], qdb[1], thb[0], thb[1], thb[2], thb[3]};
    for (int v = 0; v < 8; ++v) worst_g = std::max(worst_g, std::fabs(an[v] - fd[v]) / (1 + std::fabs(fd[v])));
  }
  printf("closed form vs generic ABA: worst rel %.3e\nreverse vs central differences: worst rel %.3e\n", worst_q, worst_g);
  return (worst_q < 1e-12 && worst_g < 1e-6) ? 0 : 1;
}
