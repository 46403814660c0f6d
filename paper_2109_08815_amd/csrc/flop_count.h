// Host-only counting scalar: running a templated step function with it
// tallies the arithmetic the step performs (add, sub, mul, div each 1,
// negation 0; sin and cos tallied apart), which is how the algorithmic FLOP
// counts per time step are obtained.
#pragma once
#include <cmath>

namespace pds {

struct FlopTally {
  double flops = 0, transc = 0;
};
inline FlopTally g_tally;

struct Counted {
  float v;
  Counted() : v(0.f) {}
  Counted(float x) : v(x) {}  // NOLINT: implicit from literals, like float
};
inline Counted operator+(Counted a, Counted b) { g_tally.flops += 1; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { g_tally.flops += 1; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { g_tally.flops += 1; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { g_tally.flops += 1; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline Counted operator+(float a, Counted b) { return Counted(a) + b; }
inline Counted operator-(float a, Counted b) { return Counted(a) - b; }
inline Counted operator*(float a, Counted b) { return Counted(a) * b; }
inline Counted operator/(float a, Counted b) { return Counted(a) / b; }
inline Counted operator+(Counted a, float b) { return a + Counted(b); }
inline Counted operator-(Counted a, float b) { return a - Counted(b); }
inline Counted operator*(Counted a, float b) { return a * Counted(b); }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline Counted recip(Counted x) { return 1.0f / x; }
inline void sincos_r(Counted x, Counted* sn, Counted* cs) {
  g_tally.transc += 2;
  float s, c;
  sincosf(x.v, &s, &c);
  *sn = Counted(s);
  *cs = Counted(c);
}

// Arm model: forward step, reverse step of one adjoint channel, sin/cos
// per step (implemented in arm.hip).
void count_arm_flops(int mount, double* fwd, double* rev, double* transc);

}  // namespace pds
