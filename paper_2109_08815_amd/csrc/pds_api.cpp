// Host side of the C ABI declared in pds.h: argument validation, per-launch
// job maps, workspace carving and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace pds {
int planar_seg_len(int h);
size_t planar_tape_bytes(int h);
}

namespace {

thread_local std::string g_err;
// Offset, in sample positions, of the sampled median bracket (tests only).
int g_median_rank_shift = 0;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

using pds::JobMap;
using pds::WsLayout;

// Timing ring of event pairs around window-kernel launches.  One pair
// brackets `reps` back-to-back launches of the same kernels (they rewrite
// the same outputs from the same inputs), so the dispatch latency an event
// pair adds is paid once per pair, not once per launch.
constexpr int kRing = 4096;
constexpr int kMaxReps = 64;
struct Timing {
  bool on = false;
  int n = 0;
  int reps = 1;
  std::vector<hipEvent_t> ev;
  std::vector<int> reps_of;
};
Timing g_timing;

// Returns how many times the caller launches its timed kernels: reps while
// timing is on and the ring has room, else 1.
int timing_begin(hipStream_t s, int* slot) {
  *slot = -1;
  if (!g_timing.on || g_timing.n >= kRing) return 1;
  *slot = g_timing.n++;
  g_timing.reps_of[*slot] = g_timing.reps;
  (void)hipEventRecord(g_timing.ev[2 * *slot], s);
  return g_timing.reps;
}
void timing_end(hipStream_t s, int slot) {
  if (slot >= 0) (void)hipEventRecord(g_timing.ev[2 * slot + 1], s);
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Which pointers a call reads or writes (bit set).
enum : unsigned {
  NEED_FWD = 1u,       // theta, S, s0, consts, end_states
  NEED_LL = 2u,        // obs, w_x, u, ll_win, gdef, logp, wk
  NEED_ADJ = 4u,       // lam_def, g_obs, g_con, S_dot
  NEED_PHI = 8u,       // rho, g_obs, phi, bandwidth
  NEED_BW = 32u,       // rho, theta, bandwidth
  NEED_STEP = 16u,     // lo, hi, lr_*, lam_lim, lam_def, adam, phi, g_con, S_dot, gdef
};

int validate_job(const pds_job& J, int idx, unsigned need) {
#define REQ(ptr, al)                                                                          \
  do {                                                                                        \
    if (!(J.ptr)) return fail(PDS_EINVAL, "job %d: " #ptr " is NULL", idx);                   \
    if (!aligned(J.ptr, al)) return fail(PDS_EINVAL, "job %d: " #ptr " is misaligned", idx);  \
  } while (0)
  if (J.model == PDS_MODEL_ARM) {
    if (J.n_dof != 8 || J.M != 4 || J.d_x != 1)
      return fail(PDS_EINVAL, "job %d: the arm model has n_dof = 8, M = 4, d_x = 1", idx);
  } else if (J.model == PDS_MODEL_ARM_UJOINT) {
    if (J.n_dof != 9 || J.M != 11 || J.d_x != 12)
      return fail(PDS_EINVAL, "job %d: the universal-joint arm model has n_dof = 9, M = 11, d_x = 12", idx);
  } else if (J.model == PDS_MODEL_ARM_UJOINT_WEIGHTS) {
    if (J.n_dof != 9 || J.M != 4 || J.d_x != 12)
      return fail(PDS_EINVAL, "job %d: the universal-joint arm with weights has n_dof = 9, M = 4, d_x = 12", idx);
  } else if (J.model == PDS_MODEL_PLANAR) {
    if (J.n_dof < 1 || J.n_dof > 5)
      return fail(PDS_EUNSUPPORTED, "job %d: planar n_dof %d outside 1..5", idx, J.n_dof);
    if (J.M != 2 * J.n_dof) return fail(PDS_EINVAL, "job %d: planar model needs M = 2 n_dof (got M=%d)", idx, J.M);
    if (J.d_x != J.n_dof && J.d_x != 2 * J.n_dof)
      return fail(PDS_EINVAL, "job %d: planar models observe q (d_x = n_dof) or (q, qd) (d_x = 2 n_dof)", idx);
  } else if (J.model == PDS_MODEL_PLANAR_RIGID) {
    if (J.n_dof < 1 || J.n_dof > 2)
      return fail(PDS_EUNSUPPORTED, "job %d: rigid planar n_dof %d outside 1..2", idx, J.n_dof);
    if (J.M != 6 * J.n_dof - 1)
      return fail(PDS_EINVAL, "job %d: rigid planar model needs M = 6 n_dof - 1 (got M=%d)", idx, J.M);
    if (J.d_x != J.n_dof && J.d_x != 2 * J.n_dof)
      return fail(PDS_EINVAL, "job %d: planar models observe q (d_x = n_dof) or (q, qd) (d_x = 2 n_dof)", idx);
  } else {
    return fail(PDS_EINVAL, "job %d: unknown model %d", idx, J.model);
  }
  if (J.N < 1 || J.K < 1 || J.n_s < 1 || J.h < 1 || J.T != J.n_s * J.h)
    return fail(PDS_EINVAL, "job %d: need N, K, n_s, h >= 1 and T = n_s h (N=%d K=%d T=%d n_s=%d h=%d)", idx, J.N,
                J.K, J.T, J.n_s, J.h);
  const double units = (double)J.N * J.K * J.n_s;
  // shooting states and multipliers share one flat index in the step kernel
  if (units > 2.0e9 || (double)J.N * J.K * (J.n_s) * (2 * J.n_dof + 1) > 2.0e9)
    return fail(PDS_EUNSUPPORTED, "job %d: problem too large for 32-bit indexing", idx);
  if (J.N > PDS_MAX_N) return fail(PDS_EUNSUPPORTED, "job %d: N=%d above %d particles", idx, J.N, PDS_MAX_N);
  if (!(J.dt > 0.f) || !std::isfinite(J.dt)) return fail(PDS_EINVAL, "job %d: dt must be > 0", idx);
  if (!(J.sigma_def > 0.f)) return fail(PDS_EINVAL, "job %d: sigma_def must be > 0", idx);
  if (!(J.c >= 0.f)) return fail(PDS_EINVAL, "job %d: c must be >= 0", idx);
  if (J.combine != PDS_COMBINE_SUM && J.combine != PDS_COMBINE_PROD)
    return fail(PDS_EINVAL, "job %d: unknown combine %d", idx, J.combine);
  if (J.lik != PDS_LIK_MDMM && J.lik != PDS_LIK_DEFECT)
    return fail(PDS_EINVAL, "job %d: unknown likelihood mode %d", idx, J.lik);
  if (J.limits != PDS_LIMITS_SOFT && J.limits != PDS_LIMITS_PROJECT)
    return fail(PDS_EINVAL, "job %d: unknown limits mode %d", idx, J.limits);
  if (need & (NEED_FWD | NEED_LL | NEED_ADJ)) {
    REQ(consts, 4); REQ(theta, 4); REQ(s0, 4); REQ(end_states, 4);
    if (J.n_s > 1) REQ(S, 4);
    if (J.traj && !aligned(J.traj, 4)) return fail(PDS_EINVAL, "job %d: traj is misaligned", idx);
    if (J.traj_obs && !aligned(J.traj_obs, 4)) return fail(PDS_EINVAL, "job %d: traj_obs is misaligned", idx);
  }
  if (need & (NEED_LL | NEED_ADJ)) {
    REQ(obs, 4); REQ(w_x, 4); REQ(u, 4); REQ(ll_win, 8); REQ(logp, 8); REQ(wk, 8);
    if (J.n_s > 1) REQ(gdef, 8);
  }
  if (need & NEED_ADJ) {
    REQ(g_obs, 8); REQ(g_con, 8);
    if (J.seed_gdef && J.cot_gdef) return fail(PDS_EINVAL, "job %d: seed_gdef and cot_gdef are exclusive", idx);
    if (J.seed_gdef && !aligned(J.seed_gdef, 8)) return fail(PDS_EINVAL, "job %d: seed_gdef is misaligned", idx);
    if (J.cot_gdef && !aligned(J.cot_gdef, 8)) return fail(PDS_EINVAL, "job %d: cot_gdef is misaligned", idx);
    if (J.seed_logp && !aligned(J.seed_logp, 8)) return fail(PDS_EINVAL, "job %d: seed_logp is misaligned", idx);
    if (J.g_theta && !aligned(J.g_theta, 8)) return fail(PDS_EINVAL, "job %d: g_theta is misaligned", idx);
    if (J.n_s > 1) { REQ(S_dot, 4); if (!J.seed_gdef && !J.cot_gdef) REQ(lam_def, 4); }
  }
  if (need & NEED_PHI) {
    REQ(rho, 4); REQ(g_obs, 8); REQ(phi, 4); REQ(bandwidth, 8); REQ(theta, 4);
    if (J.n_masked && !aligned(J.n_masked, 4)) return fail(PDS_EINVAL, "job %d: n_masked is misaligned", idx);
  }
  if (need & NEED_BW) { REQ(rho, 4); REQ(bandwidth, 8); REQ(theta, 4); }
  if (need & NEED_STEP) {
    REQ(theta, 4); REQ(lo, 4); REQ(hi, 4); REQ(lr_theta, 4); REQ(lam_lim, 4); REQ(phi, 4); REQ(g_con, 8);
    REQ(adam_m, 4); REQ(adam_v, 4);
    if (J.n_s > 1) { REQ(S, 4); REQ(S_dot, 4); REQ(lam_def, 4); REQ(gdef, 8); REQ(lr_S, 4); }
    if (J.iter_dev && !aligned(J.iter_dev, 8)) return fail(PDS_EINVAL, "job %d: iter_dev is misaligned", idx);
  }
#undef REQ
  return PDS_OK;
}

int validate_batch(const pds_job* h_jobs, const pds_job* d_jobs, int n_jobs, unsigned need) {
  g_err.clear();
  if (!h_jobs || !d_jobs) return fail(PDS_EINVAL, "h_jobs and d_jobs must be non-NULL");
  if (n_jobs < 1 || n_jobs > PDS_MAX_JOBS) return fail(PDS_EINVAL, "n_jobs %d outside 1..%d", n_jobs, PDS_MAX_JOBS);
  if (!aligned(d_jobs, 8)) return fail(PDS_EINVAL, "d_jobs is misaligned");
  for (int j = 0; j < n_jobs; ++j) {
    const int rc = validate_job(h_jobs[j], j, need);
    if (rc) return rc;
  }
  return PDS_OK;
}

bool is_arm(const pds_job& J) {
  return J.model == PDS_MODEL_ARM || J.model == PDS_MODEL_ARM_UJOINT || J.model == PDS_MODEL_ARM_UJOINT_WEIGHTS;
}

size_t job_ws(const pds_job& J, int which) {
  const WsLayout L = pds::ws_layout(J);
  switch (which) {
    case PDS_CALL_FORWARD:
    case PDS_CALL_LOGLIK: return is_arm(J) ? pds::align256(pds::arm_model_bytes(J)) : 0;
    case PDS_CALL_STEP: return 0;
    default: return L.total;
  }
}

// Workspace offsets of every job for a call (0-sized calls give all zeros).
std::vector<uint64_t> ws_offsets(const pds_job* h_jobs, int n, int which, size_t* total) {
  std::vector<uint64_t> off(n);
  size_t o = 0;
  for (int j = 0; j < n; ++j) {
    off[j] = o;
    o = pds::align256(o + job_ws(h_jobs[j], which));
  }
  *total = o;
  return off;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return PDS_OK;
  if (!ws) return fail(PDS_EWORKSPACE, "workspace of %zu bytes required, got NULL", need);
  if (!aligned(ws, 256)) return fail(PDS_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(PDS_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return PDS_OK;
}

// Builds a map over the jobs selected by `pick`, with `blocks(job)` blocks each.
template <class Pick, class Blocks>
JobMap make_map(const pds_job* h_jobs, int n, const std::vector<uint64_t>& off, Pick pick, Blocks blocks,
                int* grid) {
  JobMap m;
  std::memset(&m, 0, sizeof m);
  int b = 0;
  for (int j = 0; j < n; ++j) {
    if (!pick(h_jobs[j])) continue;
    const int nb = blocks(h_jobs[j]);
    if (nb <= 0) continue;
    m.job[m.n] = j;
    m.begin[m.n] = b;
    m.ws_off[m.n] = off[j];
    ++m.n;
    b += nb;
  }
  m.begin[m.n] = b;
  *grid = b;
  return m;
}

int launch_rc(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(PDS_ELAUNCH, "%s: %s", what, hipGetErrorString(e));
  return PDS_OK;
}

int div_up(long a, long b) { return (int)((a + b - 1) / b); }

// Blocks (one wave each) of an arm window kernel: ceil(N / 64) per
// (trajectory, window), so that a wave's lanes share their time steps.
int arm_blocks(const pds_job& J) { return J.K * J.n_s * div_up(J.N, pds::kWave); }

int arm_setup_all(const pds_job* h_jobs, const pds_job* d_jobs, int n, const std::vector<uint64_t>& off, char* w,
                  hipStream_t s) {
  int grid = 0;
  JobMap m = make_map(
      h_jobs, n, off, [](const pds_job& J) { return is_arm(J); },
      [](const pds_job& J) { return 1 + div_up((long)J.T * 7, pds::kArmSetupThreads); }, &grid);
  if (m.n == 0) return PDS_OK;
  return launch_rc(pds::launch_arm_setup(m, d_jobs, w, grid, s), "arm_setup");
}

int rollout_calls(const pds_job* h_jobs, const pds_job* d_jobs, int n, bool with_ll, void* ws, size_t ws_bytes,
                  hipStream_t s) {
  size_t need = 0;
  std::vector<uint64_t> off = ws_offsets(h_jobs, n, with_ll ? PDS_CALL_LOGLIK : PDS_CALL_FORWARD, &need);
  int rc = check_ws(ws, ws_bytes, need);
  if (rc) return rc;
  char* w = static_cast<char*>(ws);
  rc = arm_setup_all(h_jobs, d_jobs, n, off, w, s);
  if (rc) return rc;
  int slot = -1;
  const int reps = with_ll ? timing_begin(s, &slot) : 1;
  for (int r = 0; r < reps; ++r) {
  for (int model : {PDS_MODEL_ARM, PDS_MODEL_ARM_UJOINT, PDS_MODEL_ARM_UJOINT_WEIGHTS}) {
    int grid = 0;
    JobMap m = make_map(
        h_jobs, n, off, [&](const pds_job& J) { return J.model == model; }, arm_blocks, &grid);
    if (m.n > 0) {
      rc = launch_rc(pds::launch_arm_forward(m, pds::arm_mount(model), d_jobs, w, grid, with_ll, s), "arm_forward");
      if (rc) return rc;
    }
  }
  for (int model : {PDS_MODEL_PLANAR, PDS_MODEL_PLANAR_RIGID})
    for (int nb = 1; nb <= 5; ++nb) {
      int grid = 0;
      JobMap m = make_map(
          h_jobs, n, off, [&](const pds_job& J) { return J.model == model && J.n_dof == nb; },
          [](const pds_job& J) { return div_up((long)J.N * J.K * J.n_s, pds::kWave); }, &grid);
      if (m.n == 0) continue;
      rc = launch_rc(pds::launch_planar_forward(m, nb, model == PDS_MODEL_PLANAR_RIGID, d_jobs, grid, with_ll, s),
                     "planar_forward");
      if (rc) return rc;
    }
  }
  timing_end(s, slot);
  return PDS_OK;
}

// Adjoint launch shape of one job, from its own size.  Planar: with fewer
// waves than SIMDs the two adjoint channels go to two lanes per unit
// (split); whole windows stay in LDS (full) when every wave of the job can
// be resident at once, else sqrt(h) checkpoints.  (The arm adjoint's shape
// is arm_plan's.)
struct AdjShape {
  bool split, full, tape;
  size_t lds;  // dynamic LDS bytes per block
};

// Blocks of `lds` bytes that fit on the chip at once (256 CUs, 160 KiB
// each), 0 when one does not fit a CU.
long resident_blocks(size_t lds) { return lds <= 160 * 1024 ? 256L * (long)((160 * 1024) / lds) : 0L; }

AdjShape planar_shape(const pds_job& J) {
  const long units = (long)J.N * J.K * J.n_s;
  const int ds = 2 * J.n_dof;
  const long kSimds = 256 * 4;
  const size_t full_lds = (size_t)(J.h + 1) * ds * pds::kWave * sizeof(float);
  AdjShape a;
  a.split = div_up(units, pds::kWave) < kSimds;
  const long waves = a.split ? div_up(units, pds::kWave / 2) : div_up(units, pds::kWave);
  a.full = waves <= resident_blocks(full_lds);
  // The closed-form double pendulum keeps its dynamics tape beside the
  // window when every wave of the job still fits on the chip at once.
  const size_t tape_lds = full_lds + pds::planar_tape_bytes(J.h);
  a.tape = a.split && a.full && J.model == PDS_MODEL_PLANAR && J.n_dof == 2 && waves <= resident_blocks(tape_lds);
  const int B = a.full ? J.h : pds::planar_seg_len(J.h);
  const int nseg = div_up(J.h, B);
  a.lds = a.tape ? tape_lds : a.full ? full_lds : (size_t)(nseg + B + 1) * ds * pds::kWave * sizeof(float);
  return a;
}

// Arm adjoint launch shape of one job, from its own size: the checkpoint
// strides (packed B1 | B2 << 16) and the block's dynamic LDS.  The LDS
// budget per wave is what lets every wave of the job be resident at once
// (256 CUs of 160 KiB, at most kArmWavesPerCu waves per CU, the kernel's
// register-limited occupancy); the plan needs the fewest forward-dynamics
// evaluations within it.  False if no plan fits one wave per CU.
constexpr long kArmWavesPerCu = 4;
struct ArmShapePlan {
  int32_t aux;
  size_t lds;
};
bool arm_plan(const pds_job& J, ArmShapePlan* out) {
  const long waves = arm_blocks(J);
  const long per_cu = std::min(std::max(div_up(waves, 256), 1), (int)kArmWavesPerCu);
  const size_t slot_bytes = (size_t)2 * J.n_dof * pds::kWave * sizeof(float);
  const int slots = (int)((160 * 1024 / per_cu) / slot_bytes);
  int B1 = 0, B2 = 0;
  if (!pds::arm_ck_plan(J.h, slots, &B1, &B2, nullptr)) return false;
  const int nseg = (J.h + B1 - 1) / B1, n2 = (B1 + B2 - 1) / B2 - 1;
  out->aux = B1 | (B2 << 16);
  out->lds = std::max<size_t>((size_t)(nseg - 1 + n2) * slot_bytes, 4);
  return true;
}

int assemble_logp(const pds_job* h_jobs, const pds_job* d_jobs, int n, hipStream_t s) {
  std::vector<uint64_t> off(n, 0);
  int grid = 0;
  JobMap m = make_map(
      h_jobs, n, off, [](const pds_job&) { return true; }, [](const pds_job& J) { return div_up(J.N, 64); },
      &grid);
  return launch_rc(pds::launch_assemble(m, d_jobs, nullptr, grid, false, s), "assemble_logp");
}

// Shared prologue of the phi-family calls: validation, workspace offsets.
int phi_prologue(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, unsigned need, void* ws,
                 size_t ws_bytes, std::vector<uint64_t>* off, int* mmax) {
  int rc = validate_batch(h_jobs, d_jobs, n_jobs, need);
  if (rc) return rc;
  size_t total = 0;
  *off = ws_offsets(h_jobs, n_jobs, PDS_CALL_PHI, &total);
  rc = check_ws(ws, ws_bytes, total);
  if (rc) return rc;
  *mmax = 1;
  for (int j = 0; j < n_jobs; ++j) *mmax = h_jobs[j].M > *mmax ? h_jobs[j].M : *mmax;
  return PDS_OK;
}

// Waves the window kernels of sim_batch_adjoint launch for a batch (one
// wave per arm block; planar blocks of 32 or 64 units).
long adjoint_waves(const pds_job* h_jobs, int n) {
  long w = 0;
  for (int j = 0; j < n; ++j) {
    const pds_job& J = h_jobs[j];
    if (is_arm(J)) {
      w += arm_blocks(J);
    } else {
      const long units = (long)J.N * J.K * J.n_s;
      w += div_up(units, planar_shape(J).split ? pds::kWave / 2 : pds::kWave);
    }
  }
  return w;
}

// concurrent: the bandwidth runs beside the batch's sim_batch_adjoint
// (svgd_bandwidth).  Larger jobs then take the narrow chain of one-wave
// blocks when the window kernels leave SIMDs free (their blocks of 256 or
// 1024 threads would wait for the window kernels' end) and run long enough
// to hide it: the chain takes 0.3 to 0.6 ms, an arm window kernel about
// 25 us per step of its windows, so the batch must hold an arm job with
// windows of at least kNarrowMinSteps steps.  The result is the same exact
// median either way.
constexpr int kNarrowMinSteps = 32;
int bandwidth_calls(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, const std::vector<uint64_t>& off,
                    int mmax, char* w, hipStream_t s, bool concurrent) {
  int rc = PDS_OK;
  auto all = [](const pds_job&) { return true; };
  auto npairs = [](const pds_job& J) { return (long)J.N * (J.N - 1) / 2; };
  // bandwidth: keys (or a sample of them), one selecting block per job,
  // then the count and final kernels for jobs above kSmallPairs pairs
  bool long_windows = false;
  for (int j = 0; j < n_jobs; ++j) long_windows |= is_arm(h_jobs[j]) && h_jobs[j].h >= kNarrowMinSteps;
  const bool narrow = concurrent && long_windows && adjoint_waves(h_jobs, n_jobs) <= 1024 - 4;
  auto large = [&](const pds_job& J) { return npairs(J) > pds::kSmallPairs; };
  auto lean = [&](const pds_job& J) { return narrow && large(J); };
  auto wide = [&](const pds_job& J) { return !lean(J); };
  auto wide_large = [&](const pds_job& J) { return large(J) && !lean(J); };
  auto tiles = [](const pds_job& J) {
    const long nb = div_up(J.N, pds::kCountTile);
    return nb * (nb + 1) / 2;
  };
  pds::MedianMaps mm;
  mm.keys = make_map(
      h_jobs, n_jobs, off, wide,
      [&](const pds_job& J) { return div_up(large(J) ? pds::kSampleKeys : npairs(J), 256); }, &mm.grid_keys);
  mm.select = make_map(h_jobs, n_jobs, off, wide, [](const pds_job&) { return 1; }, &mm.grid_select);
  mm.count = make_map(h_jobs, n_jobs, off, wide_large, tiles, &mm.grid_count);
  mm.large = make_map(h_jobs, n_jobs, off, wide_large, [](const pds_job&) { return 1; }, &mm.grid_large);
  mm.lean_keys = make_map(
      h_jobs, n_jobs, off, lean, [](const pds_job&) { return div_up(pds::kSampleKeys, pds::kWave); },
      &mm.grid_lean_keys);
  mm.lean_count = make_map(h_jobs, n_jobs, off, lean, tiles, &mm.grid_lean_count);
  mm.lean_final = make_map(h_jobs, n_jobs, off, lean, [](const pds_job&) { return 1; }, &mm.grid_lean_final);
  rc = launch_rc(pds::launch_median(mm, d_jobs, w, mmax, g_median_rank_shift, s), "median");
  if (rc) return rc;
  return PDS_OK;
}

int phi_calls(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, const std::vector<uint64_t>& off,
              char* w, hipStream_t s) {
  int rc = PDS_OK;
  // one launch per parameter-count class and per phi scheme (chosen from
  // the job's own N), so a job's code path does not depend on the batch
  for (int cls = 0; cls < 4; ++cls) {
    const int lo_m = 1 + 4 * cls, hi_m = cls == 3 ? PDS_MAX_M : 4 + 4 * cls;
    auto in_cls = [&](const pds_job& J) { return J.M >= lo_m && J.M <= hi_m; };
    int grid = 0;
    for (int ti : {pds::kPhiTISmall, pds::kPhiTILarge}) {
      JobMap mf = make_map(
          h_jobs, n_jobs, off,
          [&](const pds_job& J) { return in_cls(J) && J.N <= pds::kPhiFusedMaxN && pds::phi_ti(J.N) == ti; },
          [&](const pds_job& J) { return div_up(J.N, ti); }, &grid);
      if (mf.n > 0) {
        rc = launch_rc(pds::launch_phi(mf, d_jobs, grid, hi_m, ti, s), "phi");
        if (rc) return rc;
      }
    }
    JobMap mp = make_map(
        h_jobs, n_jobs, off, [&](const pds_job& J) { return in_cls(J) && J.N > pds::kPhiFusedMaxN; },
        [](const pds_job& J) { return div_up(J.N, 64) * div_up(J.N, pds::kPhiChunk); }, &grid);
    if (mp.n > 0) {
      rc = launch_rc(pds::launch_phi_partial(mp, d_jobs, w, grid, hi_m, s), "phi_partial");
      if (rc) return rc;
    }
  }
  int rgrid = 0;
  JobMap mr = make_map(
      h_jobs, n_jobs, off, [](const pds_job& J) { return J.N > pds::kPhiFusedMaxN; },
      [](const pds_job& J) { return div_up((long)J.N * J.M, 256); }, &rgrid);
  if (mr.n > 0) return launch_rc(pds::launch_phi_reduce(mr, d_jobs, w, rgrid, s), "phi_reduce");
  return PDS_OK;
}

}  // namespace

extern "C" {

int32_t pds_version(void) { return 100; }

int pds_timing_enable(int32_t enable) {
  g_err.clear();
  if (enable < 0 || enable > kMaxReps)
    return fail(PDS_EINVAL, "pds_timing_enable: %d launches per timed call (0 .. %d)", enable, kMaxReps);
  if (g_timing.ev.empty() && enable) {
    g_timing.ev.resize(2 * kRing);
    for (auto& e : g_timing.ev) {
      if (hipEventCreate(&e) != hipSuccess) {
        g_timing.ev.clear();
        return fail(PDS_ELAUNCH, "hipEventCreate failed");
      }
    }
  }
  g_timing.reps_of.assign(kRing, 1);
  g_timing.on = enable != 0;
  g_timing.reps = enable > 0 ? enable : 1;
  g_timing.n = 0;
  return PDS_OK;
}

int pds_timing_read(float* ms, int32_t max_n) {
  if (!ms || max_n < 0) return fail(PDS_EINVAL, "pds_timing_read: bad arguments");
  const int n = g_timing.n < max_n ? g_timing.n : max_n;
  for (int i = 0; i < n; ++i) {
    if (hipEventSynchronize(g_timing.ev[2 * i + 1]) != hipSuccess) return fail(PDS_ELAUNCH, "event sync failed");
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]) != hipSuccess)
      return fail(PDS_ELAUNCH, "hipEventElapsedTime failed");
    ms[i] = t / (float)g_timing.reps_of[i];
  }
  return n;
}

const char* pds_last_error(void) { return g_err.c_str(); }

size_t pds_workspace_size(const pds_job* h_jobs, int32_t n_jobs, int32_t which) {
  g_err.clear();
  if (!h_jobs || n_jobs < 1 || n_jobs > PDS_MAX_JOBS) {
    fail(PDS_EINVAL, "pds_workspace_size: bad job array");
    return 0;
  }
  if (which < 0 || which > PDS_CALL_ALL) {
    fail(PDS_EINVAL, "pds_workspace_size: bad call selector %d", which);
    return 0;
  }
  size_t best = 0;
  for (int w = 0; w < PDS_CALL_ALL; ++w) {
    if (which != PDS_CALL_ALL && w != which) continue;
    size_t t = 0;
    ws_offsets(h_jobs, n_jobs, w, &t);
    if (t > best) best = t;
  }
  return best;
}

size_t pds_job_footprint(const pds_job* h_job) {
  g_err.clear();
  if (!h_job) {
    fail(PDS_EINVAL, "pds_job_footprint: NULL job");
    return 0;
  }
  const pds_job& J = *h_job;
  if (validate_job(J, 0, 0)) return 0;
  const size_t N = J.N, K = J.K, T = J.T, ns = J.n_s, M = J.M, ds = 2 * (size_t)J.n_dof, dx = J.d_x;
  const size_t nsm = ns - 1, nsm1 = nsm > 0 ? nsm : 1;
  size_t f32 = J.model == PDS_MODEL_ARM ? 126
               : J.model == PDS_MODEL_ARM_UJOINT ? 117
               : J.model == PDS_MODEL_ARM_UJOINT_WEIGHTS ? 130
                                                    : 2 + (size_t)J.n_dof;  // consts
  f32 += 3 * M + dx + ds + M + ds + K * ds + K * T * dx;              // lo hi rho w_x u lr_theta lr_S s0 obs
  f32 += N * M + N * K * nsm * ds + N * M + N * K * nsm;               // theta S lam_lim lam_def
  f32 += 2 * N * (M + K * nsm * ds);                                   // adam_m adam_v
  f32 += N * K * ns * ds + N * K * nsm1 * ds + N * M;                  // end_states S_dot phi
  size_t f64 = N * K * ns + N * K * nsm1 + N + N * K + 2 * N * M + 1;  // ll_win gdef logp wk g_obs g_con bandwidth
  const size_t i32 = N + 3;                                            // flags iter_dev n_masked
  if (J.traj) f32 += N * K * T * ds;
  if (J.traj_obs) f32 += N * K * T * dx;
  if (J.g_theta) f64 += N * M;
  if (J.seed_logp) f64 += N;
  if (J.seed_gdef) f64 += N * K * nsm;
  if (J.cot_gdef) f64 += N * K * nsm;
  return 4 * f32 + 8 * f64 + 4 * i32 + job_ws(J, PDS_CALL_ALL);
}

int sim_batch_forward(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = validate_batch(h_jobs, d_jobs, n_jobs, NEED_FWD);
  if (rc) return rc;
  return rollout_calls(h_jobs, d_jobs, n_jobs, false, ws, ws_bytes, (hipStream_t)stream);
}

int loglik_multishoot(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = validate_batch(h_jobs, d_jobs, n_jobs, NEED_FWD | NEED_LL);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = rollout_calls(h_jobs, d_jobs, n_jobs, true, ws, ws_bytes, s);
  if (rc) return rc;
  return assemble_logp(h_jobs, d_jobs, n_jobs, s);
}

int sim_batch_adjoint(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                      void* stream) {
  int rc = validate_batch(h_jobs, d_jobs, n_jobs, NEED_FWD | NEED_LL | NEED_ADJ);
  if (rc) return rc;
  size_t need = 0;
  std::vector<uint64_t> off = ws_offsets(h_jobs, n_jobs, PDS_CALL_ADJOINT, &need);
  rc = check_ws(ws, ws_bytes, need);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  // every launch shape is checked before anything is queued
  std::vector<ArmShapePlan> arm_shape(n_jobs);
  for (int j = 0; j < n_jobs; ++j) {
    const pds_job& J = h_jobs[j];
    if (is_arm(J)) {
      if (!arm_plan(J, &arm_shape[j]))
        return fail(PDS_EUNSUPPORTED, "job %d: windows of %d steps need more checkpoints than LDS holds", j, J.h);
    } else if (planar_shape(J).lds > 160 * 1024) {
      return fail(PDS_EUNSUPPORTED, "job %d: window of %d steps needs %zu bytes of LDS", j, J.h, planar_shape(J).lds);
    }
  }
  rc = arm_setup_all(h_jobs, d_jobs, n_jobs, off, w, s);
  if (rc) return rc;
  int slot = -1;
  const int reps = timing_begin(s, &slot);
  // Launch shapes are chosen per job from its own size, never from the
  // batch, so a job runs the same code path alone and in any mix; jobs
  // sharing a shape share a launch.
  for (int r = 0; r < reps; ++r) {
  for (int model : {PDS_MODEL_ARM, PDS_MODEL_ARM_UJOINT, PDS_MODEL_ARM_UJOINT_WEIGHTS}) {
    std::vector<size_t> done;
    for (int j = 0; j < n_jobs; ++j) {
      if (h_jobs[j].model != model) continue;
      const size_t lds = arm_shape[j].lds;
      if (std::find(done.begin(), done.end(), lds) != done.end()) continue;
      done.push_back(lds);
      int grid = 0;
      JobMap m = make_map(
          h_jobs, n_jobs, off, [&](const pds_job& J) { return J.model == model && arm_shape[&J - h_jobs].lds == lds; },
          arm_blocks, &grid);
      for (int e = 0; e < m.n; ++e) m.aux[e] = arm_shape[m.job[e]].aux;
      rc = launch_rc(pds::launch_arm_adjoint(m, pds::arm_mount(model), d_jobs, w, grid, lds, s), "arm_adjoint");
      if (rc) return rc;
    }
  }
  for (int model : {PDS_MODEL_PLANAR, PDS_MODEL_PLANAR_RIGID})
  for (int nb = 1; nb <= 5; ++nb) {
    for (int mode = 0; mode < 8; ++mode) {
      const bool split = (mode & 1) != 0, full = (mode & 2) != 0, tape = (mode & 4) != 0;
      auto pick = [&](const pds_job& J) {
        if (J.model != model || J.n_dof != nb) return false;
        const AdjShape a = planar_shape(J);
        return a.split == split && a.full == full && a.tape == tape;
      };
      int grid = 0;
      size_t lds = 0;
      JobMap m = make_map(
          h_jobs, n_jobs, off, pick,
          [&](const pds_job& J) {
            const size_t b = planar_shape(J).lds;
            if (b > lds) lds = b;
            return div_up((long)J.N * J.K * J.n_s, split ? pds::kWave / 2 : pds::kWave);
          },
          &grid);
      if (m.n == 0) continue;
      rc = launch_rc(pds::launch_planar_adjoint(m, nb, model == PDS_MODEL_PLANAR_RIGID, d_jobs, w, grid, split, full,
                                                tape, lds, s),
                     "planar_adjoint");
      if (rc) return rc;
    }
  }
  }
  timing_end(s, slot);
  int grid = 0;
  JobMap mg = make_map(
      h_jobs, n_jobs, off, [](const pds_job&) { return true; },
      [](const pds_job& J) { return J.N; }, &grid);
  rc = launch_rc(pds::launch_assemble_grad(mg, d_jobs, w, grid, s), "assemble_grad");
  if (rc) return rc;
  JobMap ms = make_map(
      h_jobs, n_jobs, off,
      [](const pds_job& J) { return J.n_s > 1 && (long)J.K * (J.n_s - 1) * 2 * J.n_dof > pds::kSdotInline; },
      [](const pds_job& J) { return div_up((long)J.N * J.K * (J.n_s - 1) * 2 * J.n_dof, 256); }, &grid);
  if (ms.n > 0) {
    rc = launch_rc(pds::launch_assemble_sdot(ms, d_jobs, w, grid, s), "assemble_sdot");
    if (rc) return rc;
  }
  return PDS_OK;
}

int pds_test_adjoint_shape(const pds_job* h_job, size_t* lds_bytes) {
  g_err.clear();
  if (!h_job || !lds_bytes) return fail(PDS_EINVAL, "pds_test_adjoint_shape: null argument");
  const pds_job& J = *h_job;
  if (J.model != PDS_MODEL_PLANAR && J.model != PDS_MODEL_PLANAR_RIGID)
    return fail(PDS_EINVAL, "pds_test_adjoint_shape: not a planar model (%d)", J.model);
  if (J.N < 1 || J.K < 1 || J.n_s < 1 || J.h < 1 || J.n_dof < 1)
    return fail(PDS_EINVAL, "pds_test_adjoint_shape: sizes must be positive");
  const AdjShape a = planar_shape(J);
  *lds_bytes = a.lds;
  return (a.split ? 1 : 0) | (a.full ? 2 : 0) | (a.tape ? 4 : 0);
}

int pds_test_median_shift(int32_t ranks) {
  if (ranks < -1000000 || ranks > 1000000) return fail(PDS_EINVAL, "rank shift %d out of range", ranks);
  g_median_rank_shift = ranks;
  return PDS_OK;
}

int svgd_phi(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
             void* stream) {
  std::vector<uint64_t> off;
  int mmax = 1;
  int rc = phi_prologue(h_jobs, d_jobs, n_jobs, NEED_PHI, ws, ws_bytes, &off, &mmax);
  if (rc) return rc;
  rc = bandwidth_calls(h_jobs, d_jobs, n_jobs, off, mmax, static_cast<char*>(ws), (hipStream_t)stream, false);
  if (rc) return rc;
  return phi_calls(h_jobs, d_jobs, n_jobs, off, static_cast<char*>(ws), (hipStream_t)stream);
}

int svgd_phi_noalloc(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* stream) {
  int rc = validate_batch(h_jobs, d_jobs, n_jobs, NEED_PHI);
  if (rc) return rc;
  size_t total = 0;
  std::vector<uint64_t> off = ws_offsets(h_jobs, n_jobs, PDS_CALL_PHI, &total);
  if (total > PDS_NOALLOC_SCRATCH_BYTES)
    return fail(PDS_EWORKSPACE, "svgd_phi_noalloc: the batch needs %zu bytes of workspace, above the %llu the "
                "fixed array holds (use svgd_phi with a workspace)", total,
                (unsigned long long)PDS_NOALLOC_SCRATCH_BYTES);
  hipStream_t s = (hipStream_t)stream;
  int device = 0;
  hipError_t e = s ? hipStreamGetDevice(s, &device) : hipGetDevice(&device);
  if (e != hipSuccess) return fail(PDS_ELAUNCH, "svgd_phi_noalloc: device of the stream: %s", hipGetErrorString(e));
  void* ws = nullptr;
  e = pds::noalloc_scratch(device, &ws);
  if (e != hipSuccess) return fail(PDS_ELAUNCH, "svgd_phi_noalloc: workspace array: %s", hipGetErrorString(e));
  int mmax = 1;
  for (int j = 0; j < n_jobs; ++j) mmax = h_jobs[j].M > mmax ? h_jobs[j].M : mmax;
  char* w = static_cast<char*>(ws);
  rc = bandwidth_calls(h_jobs, d_jobs, n_jobs, off, mmax, w, s, false);
  if (rc) return rc;
  return phi_calls(h_jobs, d_jobs, n_jobs, off, w, s);
}

int svgd_bandwidth(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                   void* stream) {
  std::vector<uint64_t> off;
  int mmax = 1;
  int rc = phi_prologue(h_jobs, d_jobs, n_jobs, NEED_BW, ws, ws_bytes, &off, &mmax);
  if (rc) return rc;
  return bandwidth_calls(h_jobs, d_jobs, n_jobs, off, mmax, static_cast<char*>(ws), (hipStream_t)stream, true);
}

int svgd_phi_at_bandwidth(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                          void* stream) {
  std::vector<uint64_t> off;
  int mmax = 1;
  int rc = phi_prologue(h_jobs, d_jobs, n_jobs, NEED_PHI, ws, ws_bytes, &off, &mmax);
  if (rc) return rc;
  return phi_calls(h_jobs, d_jobs, n_jobs, off, static_cast<char*>(ws), (hipStream_t)stream);
}

int svgd_step(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, int32_t optimizer, int32_t iter,
              void* stream) {
  int rc = validate_batch(h_jobs, d_jobs, n_jobs, NEED_STEP);
  if (rc) return rc;
  if (optimizer != PDS_OPT_SGD && optimizer != PDS_OPT_ADAM) return fail(PDS_EINVAL, "unknown optimizer %d", optimizer);
  for (int j = 0; j < n_jobs; ++j)
    if (optimizer == PDS_OPT_ADAM && iter < 1 && !h_jobs[j].iter_dev)
      return fail(PDS_EINVAL, "Adam needs iter >= 1 or a device iteration counter");
  std::vector<uint64_t> off(n_jobs, 0);
  auto blocks = [](const pds_job& J) {
    const long ds = 2 * J.n_dof;
    const long n = (long)J.N * J.M + (long)J.N * J.K * (J.n_s - 1) * ds + (long)J.N * J.K * (J.n_s - 1);
    return std::min(div_up(n, pds::kStepThreads), pds::kStepCountBlocks);
  };
  int grid = 0;
  JobMap m = make_map(h_jobs, n_jobs, off, [](const pds_job&) { return true; }, blocks, &grid);
  return launch_rc(pds::launch_step(m, d_jobs, grid, optimizer, iter, (hipStream_t)stream), "step");
}

size_t pds_traj_metrics_workspace(int32_t n, int32_t m, int32_t d) {
  g_err.clear();
  if (n < 2 || m < 2 || d < 1 || (long)n + m > PDS_METRICS_MAX_ROWS) {
    fail(PDS_EINVAL, "pds_traj_metrics_workspace: need n, m >= 2, d >= 1, n + m <= %d", PDS_METRICS_MAX_ROWS);
    return 0;
  }
  return pds::metrics_plan(n, m, d).bytes;
}

int pds_traj_metrics(const float* P, int32_t n, const float* Q, int32_t m, int32_t d, const float* w, int32_t k,
                     int32_t l, double sigma, double* out, double* rows, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!P || !Q || !out || !ws) return fail(PDS_EINVAL, "pds_traj_metrics: P, Q, out and ws must be non-NULL");
  if (!aligned(P, 4) || !aligned(Q, 4) || (w && !aligned(w, 4)) || !aligned(out, 8) || (rows && !aligned(rows, 8)) ||
      !aligned(ws, 256))
    return fail(PDS_EINVAL, "pds_traj_metrics: misaligned buffer (floats 4, doubles 8, workspace 256 bytes)");
  if (k < 1 || l < 1 || k > PDS_METRICS_MAX_K || l > PDS_METRICS_MAX_K)
    return fail(PDS_EUNSUPPORTED, "pds_traj_metrics: k = %d, l = %d outside 1..%d", k, l, PDS_METRICS_MAX_K);
  const int need = std::max(std::max(k, l + 1), 2);
  if (n < need || m < need)
    return fail(PDS_EINVAL, "pds_traj_metrics: each set needs at least %d rows (n = %d, m = %d)", need, n, m);
  if (d < 1) return fail(PDS_EINVAL, "pds_traj_metrics: d = %d", d);
  if ((long)n + m > PDS_METRICS_MAX_ROWS)
    return fail(PDS_EUNSUPPORTED, "pds_traj_metrics: n + m = %ld above %d", (long)n + m, PDS_METRICS_MAX_ROWS);
  if (!std::isfinite(sigma)) return fail(PDS_EINVAL, "pds_traj_metrics: sigma must be finite (<= 0: median)");
  const pds::MetricsPlan plan = pds::metrics_plan(n, m, d);
  if (ws_bytes < plan.bytes)
    return fail(PDS_EINVAL, "pds_traj_metrics: workspace of %zu bytes, %zu needed", ws_bytes, plan.bytes);
  hipStream_t s = (hipStream_t)stream;
  char* w8 = static_cast<char*>(ws);
  int slot;
  const int reps = timing_begin(s, &slot);
  int rc = PDS_OK;
  for (int r = 0; r < reps && rc == PDS_OK; ++r)
    rc = launch_rc(pds::launch_metric_dist(plan, P, Q, n, m, d, w, w8, s), "metric_dist");
  timing_end(s, slot);
  if (rc != PDS_OK) return rc;
  return launch_rc(pds::launch_metric_rest(plan, n, m, d, k, l, sigma, out, rows, w8, s), "metric_rest");
}

}  // extern "C"
