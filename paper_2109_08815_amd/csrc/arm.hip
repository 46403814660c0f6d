// Window rollouts and their reverse-mode adjoint for the 7-joint arm with
// its box (Sec. IV-C; the spatial algebra, forward dynamics and reverse
// step are in arm_math.h).
//
// Work layout: one lane per window unit (particle i, trajectory k, window
// j), lanes of a wave sharing (k, j).  The adjoint keeps only the window's
// start state in device memory (the shooting state S_{i,k,j}, or s0_k) and
// recomputes everything inside the window (Sec. III-C windows, App. B-A
// chain rule): the forward sweep leaves level-1 checkpoints every B1 steps
// in LDS; the reverse sweep goes through the segments backwards, refills
// level-2 checkpoints every B2 steps of the segment from its level-1
// checkpoint, and reverses each block of B2 steps from its checkpoint: a
// block of two steps by one roll forward that keeps the first step's
// dynamics tape in registers while the second is reversed, a longer block
// by rolling forward to each step being reversed.  (B1, B2) is chosen per job so
// that the checkpoints fit the LDS every wave of the job can have while all
// of them are resident, at the least number of forward-dynamics
// evaluations.  Checkpoints are [slot][component][lane] floats: each lane
// owns a bank, so the accesses are conflict-free.  Each kernel holds two
// compiled variants of the window code, for the Panda arm's kinematic
// structure and for any other table (ArmDh); the set-up kernel derives
// which one a job's table has, and each block branches on it once.
#include <cmath>
#include <vector>

#include "arm_math.h"
#include "common.h"
#include "flop_count.h"

namespace pds {

namespace {

// The derived constants as the kernels read them: through the constant
// address space (written by arm_setup_kernel earlier in the stream, read
// only afterwards), so their uniform loads are scalar.
using KConst = const __attribute__((address_space(4))) ArmConst;
template <int BOX, int DH>
using AMd = ArmMath<float, BOX, KConst, DH>;

__device__ inline KConst& arm_const_of(char* ws, uint64_t off) {
  return *(KConst*)(ws + off);
}

// Block 0 of a job derives the constants: the raw constants are first
// staged in LDS by the whole block (one coalesced load), so the single
// thread that derives the table reads them from LDS instead of waiting on
// one global round trip after another.  The job's other blocks fill the
// table of PD targets, one (time step, joint) entry per thread, with the
// target function every direct evaluation uses.
constexpr int kSetupThreads = kArmSetupThreads;
__global__ void __launch_bounds__(kSetupThreads) arm_setup_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                  char* __restrict__ ws) {
  constexpr int kRawMax = 130;  // raw floats of the largest arm model
  __shared__ float raw[kRawMax];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int b = blockIdx.x - map.begin[e];
  char* base = ws + map.ws_off[e];
  if (b == 0) {
    const int mount =
        J.model == PDS_MODEL_ARM_UJOINT ? kUJoint : (J.model == PDS_MODEL_ARM_UJOINT_WEIGHTS ? kUJointWeights : kHinge);
    const int n = mount == kUJoint ? 117 : (mount == kUJointWeights ? 130 : 126);
    for (int t = threadIdx.x; t < n; t += blockDim.x) raw[t] = J.consts[t];
    __syncthreads();
    if (threadIdx.x == 0) arm_setup(raw, reinterpret_cast<ArmConst*>(base), mount);
    return;
  }
  const int x = (b - 1) * kSetupThreads + threadIdx.x;  // entry (time step, joint)
  if (x >= J.T * 7) return;
  const int t = x / 7, i = x % 7;
  const float* jr = J.consts + 3 + 16 * i;  // joint i: ..., qc, amp, omega, phase at 12 .. 15
  float qdes, qddes;
  pd_target(jr[12], jr[13], jr[14], jr[15], (float)t * J.dt, &qdes, &qddes);
  float* tab = reinterpret_cast<float*>(base + kArmConstBytes) + (size_t)t * kArmTargets;
  tab[i] = qdes;
  tab[7 + i] = qddes;
}

// Window unit of a lane.  A job's blocks (one wave each) come in groups of
// ceil(N / 64) per (trajectory k, window j), so every lane of a wave shares
// (k, j) and the time of each step: the observation row and the PD targets
// of a step are wave-uniform loads.  Lanes past the last particle (i >= N)
// have no unit.
struct AUnit {
  int i, k, j;
};
__device__ inline AUnit aunit_of(const pds_job& J, int block, int lane) {
  const int wpg = (J.N + kWave - 1) / kWave;  // waves per (k, j)
  const int g = block / wpg;
  AUnit r;
  r.i = (block - g * wpg) * kWave + lane;
  r.k = g / J.n_s;
  r.j = g - r.k * J.n_s;
  return r;
}

// Row of the PD-target table at time step n, read through the constant
// address space (its wave-uniform reads are scalar loads).
using CFloat = const __attribute__((address_space(4))) float*;
using TRow = TargetRow<CFloat>;
__device__ inline TRow target_row(char* ws, uint64_t off, int n) {
  return TRow{(CFloat)(ws + off + kArmConstBytes) + (size_t)n * kArmTargets};
}
template <int DS>
__device__ inline const float* astart_ptr(const pds_job& J, const AUnit& w) {
  if (w.j == 0) return J.s0 + (size_t)w.k * DS;
  return J.S + (((size_t)w.i * J.K + w.k) * (J.n_s - 1) + (w.j - 1)) * DS;
}

// Observation term of the state after a step: sum ((obs - x) w)^2 without
// the constant; with ADJ, the q-adjoint of -1/2 of it is added to qb.
template <int BOX, int DH, bool ADJ>
__device__ __forceinline__ float arm_obs_term(KConst& K, const float* q, const float* obs_row, const float* w,
                                              float* qb) {
  if constexpr (BOX == kHinge) {
    const float r = (obs_row[0] - q[7]) * w[0];
    if constexpr (ADJ) qb[7] += r * w[0];
    return r * r;
  } else {
    return AMd<BOX, DH>::template box_obs<ADJ>(K, q, obs_row, w, qb);
  }
}

template <int BOX>
__device__ inline double arm_obs_log_norm(const pds_job& J) {
  double c = 0.0;
  for (int d = 0; d < ArmShape<BOX>::DX; ++d) c += log((double)J.w_x[d]) - 0.91893853320467274178;
  return c;
}

template <int BOX, int DH>
__device__ __forceinline__ void arm_forward_body(const JobMap& map, const pds_job* __restrict__ jobs, char* ws,
                                                 int with_ll) {
  using AM = AMd<BOX, DH>;
  constexpr int NB = ArmShape<BOX>::NB, DS = ArmShape<BOX>::DS, M = ArmShape<BOX>::M, DX = ArmShape<BOX>::DX;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  KConst& K = arm_const_of(ws, map.ws_off[e]);
  const AUnit w = aunit_of(J, blockIdx.x - map.begin[e], threadIdx.x);
  if (w.i >= J.N) return;
  float th[M];
  for (int m = 0; m < M; ++m) th[m] = J.theta[(size_t)w.i * M + m];
  const float* st = astart_ptr<DS>(J, w);
  float q[NB], qd[NB];
  for (int d = 0; d < NB; ++d) { q[d] = st[d]; qd[d] = st[NB + d]; }
  const float dt = J.dt;
  const int t0 = w.j * J.h;
  const float* obs = J.obs + ((size_t)w.k * J.T + t0) * DX;
  float* traj = J.traj ? J.traj + (((size_t)w.i * J.K + w.k) * J.T + t0) * DS : nullptr;
  float* tobs = J.traj_obs ? J.traj_obs + (((size_t)w.i * J.K + w.k) * J.T + t0) * DX : nullptr;
  float wx[DX];
  for (int d = 0; d < DX; ++d) wx[d] = J.w_x[d];
  double ll = 0.0;
  for (int s = 0; s < J.h; ++s) {
    AM::step(K, th, target_row(ws, map.ws_off[e], t0 + s), dt, q, qd);
    if (with_ll) ll -= 0.5 * (double)arm_obs_term<BOX, DH, false>(K, q, obs + (size_t)s * DX, wx, nullptr);
    if (traj)
      for (int d = 0; d < NB; ++d) { traj[s * DS + d] = q[d]; traj[s * DS + NB + d] = qd[d]; }
    if (tobs) {
      if constexpr (BOX == kHinge) {
        tobs[s] = q[7];
      } else {
        float x[DX];
        AM::box_frame(K, q, x);
        for (int d = 0; d < DX; ++d) tobs[(size_t)s * DX + d] = x[d];
      }
    }
  }
  const size_t iu = ((size_t)w.i * J.K + w.k) * J.n_s + w.j;
  float* es = J.end_states + iu * DS;
  bool bad = false, bad_ll = false;
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
    bad_ll = !isfinite(ll);
  }
  const int fl = (bad ? PDS_FLAG_STATE : 0) | (bad_ll ? PDS_FLAG_GRAD : 0);
  if (fl && J.flags) atomicOr(&J.flags[w.i], fl);
}

// One kernel per mount; the table's structure (set by the set-up kernel,
// read as a scalar) selects the compiled variant, uniformly per block.
template <int BOX>
__global__ void __launch_bounds__(kWave) arm_forward_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                            char* ws, int with_ll) {
  if (arm_const_of(ws, map.ws_off[map_entry(map, blockIdx.x)]).dh == kDhPanda)
    arm_forward_body<BOX, kDhPanda>(map, jobs, ws, with_ll);
  else
    arm_forward_body<BOX, kDhGeneric>(map, jobs, ws, with_ll);
}

// Adjoint kernel: one lane per unit, both adjoint channels in one reverse
// sweep; only the window start state comes from device memory (see the
// file comment for the checkpoints).  map.aux[e] = B1 | B2 << 16.
template <int BOX, int DH>
__device__ __forceinline__ void arm_adjoint_body(const JobMap& map, const pds_job* __restrict__ jobs, char* ws) {
  using AM = AMd<BOX, DH>;
  constexpr int NB = ArmShape<BOX>::NB, DS = ArmShape<BOX>::DS, M = ArmShape<BOX>::M, DX = ArmShape<BOX>::DX;
  extern __shared__ float ck[];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  KConst& K = arm_const_of(ws, map.ws_off[e]);
  const int lane = threadIdx.x;
  const AUnit w = aunit_of(J, blockIdx.x - map.begin[e], lane);
  if (w.i >= J.N) return;
  const WsLayout L = ws_layout(J);
  char* base = ws + map.ws_off[e];
  double* gth_obs = reinterpret_cast<double*>(base + L.gth_obs);
  double* gth_con = reinterpret_cast<double*>(base + L.gth_con);
  float* gs_obs = reinterpret_cast<float*>(base + L.gs_obs);
  float* gs_con = reinterpret_cast<float*>(base + L.gs_con);
  const int h = J.h;
  const int B1 = map.aux[e] & 0xffff, B2 = map.aux[e] >> 16;
  const int nseg = (h + B1 - 1) / B1, n1 = nseg - 1, last0 = n1 * B1;
  float* my = ck + lane;
  auto put = [&](int slot, const float* q, const float* qd) {
    float* p = my + (size_t)slot * DS * kWave;
  #pragma unroll
    for (int d = 0; d < NB; ++d) { p[d * kWave] = q[d]; p[(NB + d) * kWave] = qd[d]; }
  };
  auto get = [&](int slot, float* q, float* qd) {
    const float* p = my + (size_t)slot * DS * kWave;
  #pragma unroll
    for (int d = 0; d < NB; ++d) { q[d] = p[d * kWave]; qd[d] = p[(NB + d) * kWave]; }
  };
  float th[M];
  for (int m = 0; m < M; ++m) th[m] = J.theta[(size_t)w.i * M + m];
  const float* st = astart_ptr<DS>(J, w);
  auto get_start = [&](float* q, float* qd) {
  #pragma unroll
    for (int d = 0; d < NB; ++d) { q[d] = st[d]; qd[d] = st[NB + d]; }
  };
  const float dt = J.dt;
  const int t0 = w.j * h;
  const float* obs = J.obs + ((size_t)w.k * J.T + t0) * DX;
  float wx[DX];
  for (int d = 0; d < DX; ++d) wx[d] = J.w_x[d];

  // forward sweep: log-likelihood, end state, checkpoints
  float q[NB], qd[NB];
  get_start(q, qd);
  double ll = 0.0;
  {
    int next1 = B1, slot1 = 0;            // level-1 checkpoints at c B1, c = 1 .. nseg-1
    int next2 = last0 + B2, slot2 = n1;   // level-2 checkpoints of the last segment
    for (int s = 0; s < h; ++s) {
      if (s == next1 && s <= last0) {
        put(slot1++, q, qd);
        next1 += B1;
      } else if (s == next2) {
        put(slot2++, q, qd);
        next2 += B2;
      }
      AM::step(K, th, target_row(ws, map.ws_off[e], t0 + s), dt, q, qd);
      ll -= 0.5 * (double)arm_obs_term<BOX, DH, false>(K, q, obs + (size_t)s * DX, wx, nullptr);
    }
  }
  ll += (double)h * arm_obs_log_norm<BOX>(J);
  const size_t iu = ((size_t)w.i * J.K + w.k) * J.n_s + w.j;
  float* es = J.end_states + iu * DS;
  bool bad = false, bad_g = false;  // non-finite state; likelihood or gradient
  for (int d = 0; d < NB; ++d) {
    es[d] = q[d];
    es[NB + d] = qd[d];
    bad |= !isfinite(q[d]) || !isfinite(qd[d]);
  }

  // adjoint seeds at the window end: channel 0 the observation channel,
  // channel 1 the constraint channel
  float qb[2][NB], qdb[2][NB];
  for (int c = 0; c < 2; ++c)
    for (int d = 0; d < NB; ++d) qb[c][d] = qdb[c][d] = 0.f;
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
    const double seed = con_seed(J, id, g, in_lik);
    // d g / d s_end = -2 e u / sigma^2; in the likelihood, d(-g/2) / d s_end = e u / sigma^2
    const float sc = (float)(-2.0 * seed * inv_s2);
    const float so = in_lik ? (float)inv_s2 : 0.f;
    for (int d = 0; d < NB; ++d) {
      qb[0][d] = so * e0[d] * J.u[d];
      qdb[0][d] = so * e1[d] * J.u[NB + d];
      qb[1][d] = sc * e0[d] * J.u[d];
      qdb[1][d] = sc * e1[d] * J.u[NB + d];
    }
  }
  bad_g |= !isfinite(ll);
  J.ll_win[iu] = ll;

  // reverse sweep over the segments, each from its checkpoints
  double gm[2][M];
  for (int c = 0; c < 2; ++c)
    for (int m = 0; m < M; ++m) gm[c][m] = 0.0;
  float qn[NB];  // q of the state after the step being reversed
  for (int d = 0; d < NB; ++d) qn[d] = q[d];
  for (int c = nseg - 1; c >= 0; --c) {
    const int s0 = c * B1, len = min(B1, h - s0), nblk = (len + B2 - 1) / B2;
    if (c < nseg - 1) {  // refill the segment's level-2 checkpoints
      if (c == 0) get_start(q, qd); else get(c - 1, q, qd);
      int s = s0;
      for (int b = 1; b < nblk; ++b) {
        for (int r = 0; r < B2; ++r, ++s) AM::step(K, th, target_row(ws, map.ws_off[e], t0 + s), dt, q, qd);
        put(n1 + b - 1, q, qd);
      }
    }
    for (int b = nblk - 1; b >= 0; --b) {
      const int x0 = s0 + b * B2, nb = min(B2, s0 + len - x0);
      auto load_block = [&]() {
        if (b > 0) get(n1 + b - 1, q, qd);
        else if (c > 0) get(c - 1, q, qd);
        else get_start(q, qd);
      };
      // reverse of step t from its state (q, qd) and dynamics tape T
      auto reverse_step = [&](int t, const typename AM::Tape& T) {
        arm_obs_term<BOX, DH, true>(K, qn, obs + (size_t)t * DX, wx, qb[0]);
        float tb[2][M];
        for (int ch = 0; ch < 2; ++ch)
          for (int m = 0; m < M; ++m) tb[ch][m] = 0.f;
        AM::step_rev(K, th, qd, T, dt, qb, qdb, tb);
        for (int ch = 0; ch < 2; ++ch)
          for (int m = 0; m < M; ++m) gm[ch][m] += (double)tb[ch][m];
        for (int d = 0; d < NB; ++d) qn[d] = q[d];
      };
      if (B2 == 2 && nb == 2) {
        // a pair: one roll forward gives both steps' tapes; the first is
        // kept in registers while the second step is reversed
        load_block();
        typename AM::Tape T0, Tc;
        float q0[NB], qd0[NB];
  #pragma unroll 1
        for (int r = 0; r < 2; ++r) {
          AM::keep_consts_in_memory();
          AM::aba(K, th, q, qd, target_row(ws, map.ws_off[e], t0 + x0 + r), Tc);
          if (r == 0) {
            T0 = Tc;
            for (int d = 0; d < NB; ++d) {
              q0[d] = q[d];
              qd0[d] = qd[d];
              qd[d] = qd[d] + dt * Tc.qdd[d];
              q[d] = q[d] + dt * qd[d];
            }
          }
        }
  #pragma unroll 1
        for (int r = 0; r < 2; ++r) {
          reverse_step(x0 + 1 - r, Tc);
          if (r == 0) {
            Tc = T0;
            for (int d = 0; d < NB; ++d) {
              q[d] = q0[d];
              qd[d] = qd0[d];
            }
          }
        }
      } else {
        // any other block: each step's state by rolling forward from the
        // block's checkpoint
        for (int t = x0 + nb - 1; t >= x0; --t) {
          load_block();
          for (int s = x0; s < t; ++s) AM::step(K, th, target_row(ws, map.ws_off[e], t0 + s), dt, q, qd);
          typename AM::Tape T;
          AM::keep_consts_in_memory();
          AM::aba(K, th, q, qd, target_row(ws, map.ws_off[e], t0 + t), T);
          reverse_step(t, T);
        }
      }
    }
  }
  for (int m = 0; m < M; ++m) {
    gth_obs[iu * M + m] = gm[0][m];
    gth_con[iu * M + m] = gm[1][m];
    bad_g |= !isfinite(gm[0][m]) || !isfinite(gm[1][m]);
  }
  for (int d = 0; d < NB; ++d) {
    gs_obs[iu * DS + d] = qb[0][d];
    gs_obs[iu * DS + NB + d] = qdb[0][d];
    gs_con[iu * DS + d] = qb[1][d];
    gs_con[iu * DS + NB + d] = qdb[1][d];
  }
  const int fl = (bad ? PDS_FLAG_STATE : 0) | (bad_g ? PDS_FLAG_GRAD : 0);
  if (fl && J.flags) atomicOr(&J.flags[w.i], fl);
}

template <int BOX>
__global__ void __launch_bounds__(kWave) arm_adjoint_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                            char* ws) {
  if (arm_const_of(ws, map.ws_off[map_entry(map, blockIdx.x)]).dh == kDhPanda)
    arm_adjoint_body<BOX, kDhPanda>(map, jobs, ws);
  else
    arm_adjoint_body<BOX, kDhGeneric>(map, jobs, ws);
}

}  // namespace

static_assert(sizeof(ArmConst) <= kArmConstBytes, "ArmConst must fit its workspace region");
static_assert(kArmTargets == kArmTargetFloats, "one PD-target row per time step");

// Checkpoint plan of an arm job's adjoint: the level-1 stride B1 and the
// level-2 stride B2 that need the fewest forward-dynamics evaluations per
// window with at most `slots` checkpoints (level 1: nseg - 1; level 2:
// ceil(B1 / B2) - 1).  Evaluations: h for the forward sweep, the refill of
// every segment but the last (its level-2 checkpoints are left by the
// forward sweep), and in the reverse sweep one per step for blocks of up to
// two steps, L (L + 1) / 2 for a block of L > 2 steps.  Returns false when
// no plan fits.
bool arm_ck_plan(int h, int slots, int* B1_out, int* B2_out, long* evals_out) {
  // reverse-sweep evaluations of a segment of len steps in blocks of B2:
  // one per step for blocks of one or two steps (a pair reuses the tape of
  // its roll forward), L (L + 1) / 2 for a longer block of L steps
  auto rev = [](long len, long B2) {
    if (B2 <= 2) return len;
    const long r = len % B2;
    return (len / B2) * B2 * (B2 + 1) / 2 + r * (r + 1) / 2;
  };
  long best = -1;
  int bb1 = 0, bb2 = 0;
  for (int B2 = 1; B2 <= 64 && B2 <= h; ++B2) {
    for (int B1 = B2; B1 <= h; ++B1) {
      const int nseg = (h + B1 - 1) / B1;
      const int n2 = (B1 + B2 - 1) / B2 - 1;
      if ((nseg - 1) + n2 > slots) continue;
      const long last = h - (long)(nseg - 1) * B1;
      // forward sweep, refill of every full segment but the last, reverse sweep
      const long ev = h + (long)(nseg - 1) * ((long)n2 * B2 + rev(B1, B2)) + rev(last, B2);
      if (best < 0 || ev < best) {
        best = ev;
        bb1 = B1;
        bb2 = B2;
      }
    }
  }
  if (best < 0) return false;
  *B1_out = bb1;
  *B2_out = bb2;
  if (evals_out) *evals_out = best;
  return true;
}

hipError_t launch_arm_setup(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(arm_setup_kernel, dim3(grid), dim3(kSetupThreads), 0, s, map, d_jobs, ws);
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
                              size_t lds_bytes, hipStream_t s) {
  if (mount == kUJoint)
    hipLaunchKernelGGL(arm_adjoint_kernel<kUJoint>, dim3(grid), dim3(kWave), lds_bytes, s, map, d_jobs, ws);
  else if (mount == kUJointWeights)
    hipLaunchKernelGGL(arm_adjoint_kernel<kUJointWeights>, dim3(grid), dim3(kWave), lds_bytes, s, map, d_jobs, ws);
  else
    hipLaunchKernelGGL(arm_adjoint_kernel<kHinge>, dim3(grid), dim3(kWave), lds_bytes, s, map, d_jobs, ws);
  return hipGetLastError();
}

// Algorithmic FLOPs of one arm time step: the forward step (ABA + Euler +
// the observation residuals and their FP64 accumulation) and the reverse
// step of one adjoint channel -- half of the reverse step of both channels,
// which share its primal terms, with the observation seed and the FP64
// accumulation of the parameter adjoints -- from the same step functions
// the kernels run, instantiated with the counting scalar.
template <int BOX, int DH>
static void count_arm(const ArmConst& K, double* fwd, double* rev, double* transc) {
  using CM = ArmMath<Counted, BOX, ArmConst, DH>;
  constexpr int NB = ArmShape<BOX>::NB, M = ArmShape<BOX>::M;
  Counted th[11];
  for (int m = 0; m < 11; ++m) th[m] = Counted(0.01f * (m + 1));
  Counted q[NB], qd[NB], qb[2][NB], qdb[2][NB], thb[2][M];
  for (int i = 0; i < NB; ++i) {
    q[i] = Counted(0.1f * i);
    qd[i] = Counted(0.05f);
    qb[0][i] = qb[1][i] = Counted(1.f);
    qdb[0][i] = qdb[1][i] = Counted(1.f);
  }
  for (int m = 0; m < M; ++m) thb[0][m] = thb[1][m] = Counted(0.f);
  const float obs[12] = {0.1f, 0.2f, 0.3f, 1.f, 0.2f, 0.3f, 0.1f, 1.f, 0.3f, 0.1f, 0.2f, 1.f};
  const float w[12] = {100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f, 100.f};
  g_tally = FlopTally();
  typename CM::Tape T;
  CM::aba(K, th, q, qd, Counted(0.5f), T);
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
  CM::step_rev(K, th, qd, T, Counted(0.004f), qb, qdb, thb);
  const double rev_both = g_tally.flops;
  double obs_rev = 2.0;  // hinge: the observation seed r w
  if (BOX != kHinge) {
    g_tally = FlopTally();
    Counted qb2[NB];
    for (int i = 0; i < NB; ++i) qb2[i] = Counted(0.f);
    CM::template box_obs<true>(K, q, obs, w, qb2);
    obs_rev = g_tally.flops;
  }
  // per channel: half the shared reverse, its own FP64 accumulation of the
  // M parameter adjoints; the observation seed enters one channel
  *rev = 0.5 * (rev_both + obs_rev) + M;
}

template <int BOX>
static void count_arm_dh(const ArmConst& K, double* fwd, double* rev, double* transc) {
  if (K.dh == kDhPanda)
    count_arm<BOX, kDhPanda>(K, fwd, rev, transc);
  else
    count_arm<BOX, kDhGeneric>(K, fwd, rev, transc);
}

// raw: the job's raw constants (host memory), or NULL for a generic table;
// returns the table's kinematic structure (ArmDh), whose step it counted.
static int count_arm_table(int mount, const float* raw, double* fwd, double* rev, double* transc) {
  std::vector<float> dflt(130, 0.5f);  // the longest consts layout; a generic table
  dflt[0] = 0.f;
  dflt[1] = 0.f;
  dflt[2] = -9.81f;
  ArmConst K;
  arm_setup(raw ? raw : dflt.data(), &K, mount);
  if (mount == kUJoint)
    count_arm_dh<kUJoint>(K, fwd, rev, transc);
  else if (mount == kUJointWeights)
    count_arm_dh<kUJointWeights>(K, fwd, rev, transc);
  else
    count_arm_dh<kHinge>(K, fwd, rev, transc);
  return K.dh;
}

void count_arm_flops(int mount, double* fwd, double* rev, double* transc) {
  count_arm_table(mount, nullptr, fwd, rev, transc);
}

}  // namespace pds

extern "C" int pds_arm_algorithmic_flops(int32_t model, const float* consts, double* fwd_step, double* rev_step,
                                         double* transcendental, int32_t* panda) {
  if (!consts || !fwd_step || !rev_step || !transcendental) return PDS_EINVAL;
  if (model != PDS_MODEL_ARM && model != PDS_MODEL_ARM_UJOINT && model != PDS_MODEL_ARM_UJOINT_WEIGHTS)
    return PDS_EINVAL;
  const int dh = pds::count_arm_table(pds::arm_mount(model), consts, fwd_step, rev_step, transcendental);
  if (panda) *panda = dh == pds::kDhPanda ? 1 : 0;
  return PDS_OK;
}
