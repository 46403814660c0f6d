// Internal declarations shared by the HIP translation units of libpds.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pds.h"

namespace pds {

constexpr int kWave = 64;

// Block ranges of the jobs in one launch: job j owns blocks
// [begin[j], begin[j+1]).  Passed by value as a kernel argument.
struct JobMap {
  int32_t n;
  int32_t job[PDS_MAX_JOBS];        // index into d_jobs
  int32_t begin[PDS_MAX_JOBS + 1];  // first block of each entry
  uint64_t ws_off[PDS_MAX_JOBS];    // byte offset of the job's workspace region
  int32_t aux[PDS_MAX_JOBS];        // per-entry launch parameter (arm adjoint: checkpoint strides)
};

// Entry of the block's job (scalar loop: every lane agrees).
__device__ inline int map_entry(const JobMap& m, int block) {
  int e = 0;
  while (e + 1 < m.n && block >= m.begin[e + 1]) ++e;
  return e;
}

// Per-unit adjoint rows: N consecutive values from registers to memory with
// 16-byte (double) or 8-byte (float) vector stores.  p must be aligned to
// that width and N even; odd-length double rows (rows of odd length start at
// any 8-byte boundary) are stored element by element.
template <int N>
__device__ inline void store_row(double* p, const double* v) {
  if constexpr (N % 2 == 0) {
#pragma unroll
    for (int c = 0; c < N / 2; ++c) reinterpret_cast<double2*>(p)[c] = make_double2(v[2 * c], v[2 * c + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < N; ++c) p[c] = v[c];
  }
}
template <int N>
__device__ inline void store_row(float* p, const float* v) {
  static_assert(N % 2 == 0, "even rows only");
#pragma unroll
  for (int c = 0; c < N / 2; ++c) reinterpret_cast<float2*>(p)[c] = make_float2(v[2 * c], v[2 * c + 1]);
}

// Normalising constant of the defect density of eq. likelihood-defect,
// N(S | s_end, sigma_def^2 / u^2): sum_d log(u_d / (sigma_def sqrt(2 pi))),
// so log p_def = -g_def / 2 + defect_log_norm (PDS_LIK_DEFECT).
__device__ inline double defect_log_norm(const pds_job& J) {
  const int ds = 2 * J.n_dof;
  double c = 0.0;
  for (int d = 0; d < ds; ++d) c += log((double)J.u[d]) - log((double)J.sigma_def) - 0.91893853320467274178;
  return c;
}

// Seed of the constraint channel for defect `id` with value g: the caller's
// seed_gdef, or minus its cotangent cot_gdef (a vector-Jacobian product), or
// the MDMM multiplier term lam_def + c g (Sec. III-E); 0 when the defects
// are densities inside p_ms and nothing was given.
__device__ inline double con_seed(const pds_job& J, size_t id, double g, bool in_lik) {
  if (J.seed_gdef) return J.seed_gdef[id];
  if (J.cot_gdef) return -J.cot_gdef[id];
  return in_lik ? 0.0 : (double)J.lam_def[id] + (double)J.c * g;
}

constexpr size_t kArmConstBytes = 2048;  // derived arm model constants per job
constexpr int kArmTargetFloats = 14;     // PD targets per time step (q_d, qd_d of 7 joints)
// Workspace of an arm job's model: the derived constants, then the table of
// PD targets of every time step of its trajectories.
__host__ __device__ inline size_t arm_model_bytes(const pds_job& J) {
  return kArmConstBytes + (size_t)J.T * kArmTargetFloats * sizeof(float);
}

// Bandwidth median (see svgd.hip).  Up to kSmallPairs pairs one block
// selects exactly; above, a sampled bracket plus a counting pass.
constexpr int kSmallPairs = 32768;
constexpr int kSampleKeys = 32768;
constexpr int kMedThreads = 1024;
constexpr int kDirectMax = 512;      // keys a selection finishes on by direct counting
constexpr int kSelLdsCap = 8192;     // keys the select kernel's tie path stages in LDS
// The select kernel is held to the registers of this many waves per SIMD
// (and to a small LDS footprint) so that its block fits on a compute unit
// beside an adjoint block and runs concurrently with it.
constexpr int kSelWavesPerSimd = 5;
constexpr int kSelBins = 2048;       // bins per selection level (2^11)
constexpr int kMaxLevels = 8;        // selection levels never exceed 6
constexpr int kCountTile = 64;       // pairs per count block: 64 x 64
constexpr int kLastCap = 4096;       // candidates the final kernel holds in LDS

struct MedianState {
  uint64_t a, b;    // bracket keys from the sample
  uint64_t packed;  // (keys inside [a, b] << 32) | keys below a, over all count blocks
};

// Workspace layout of one job (byte offsets from the job's region start).
// The arm model's derived constants come first, so forward-only calls can
// use a region of just that size.
struct WsLayout {
  size_t arm;                               // derived arm constants (arm jobs)
  size_t gth_obs, gth_con, gs_obs, gs_con;  // adjoint per-unit gradients: [iu][m], [iu][d] with
                                            // iu = (i K + k) n_s + j (one particle's units adjacent)
  size_t med;                               // median selection state
  size_t khi, klo;                          // median key words (all pairs, or a sample's high words)
  size_t cand;                              // median candidates: 64-bit keys of larger jobs, or the
                                            // low-word lists of small jobs (one slot per pair)
  size_t phi_part;                          // phi partial sums (jobs above kPhiFusedMaxN particles)
  size_t phi_live;                          // live particles of each phi chunk (same jobs)
  size_t total;
};

constexpr int kPhiChunk = 32;    // particles j per LDS chunk in phi
constexpr int kPhiThreads = 1024;  // threads per block of the one-kernel phi
// particles i per block of the one-kernel phi: kPhiTISmall up to
// kPhiTIMaxN particles, kPhiTILarge above
constexpr int kPhiTISmall = 16;
constexpr int kPhiTILarge = 8;
constexpr int kPhiTIMaxN = 128;
inline int phi_ti(int N) { return N <= kPhiTIMaxN ? kPhiTISmall : kPhiTILarge; }
constexpr int kPhiRows = 512;       // particle rows per LDS chunk of the one-kernel phi
constexpr int kPhiFusedMaxN = 4096;  // larger jobs use partial sums and a reduction

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline WsLayout ws_layout(const pds_job& J) {
  WsLayout L;
  const size_t U = (size_t)J.N * J.K * J.n_s;
  const int ds = 2 * J.n_dof;
  size_t o = 0;
  const bool arm = J.model == PDS_MODEL_ARM || J.model == PDS_MODEL_ARM_UJOINT || J.model == PDS_MODEL_ARM_UJOINT_WEIGHTS;
  L.arm = o;     o = align256(o + (arm ? arm_model_bytes(J) : 0));
  L.gth_obs = o; o = align256(o + U * J.M * sizeof(double));
  L.gth_con = o; o = align256(o + U * J.M * sizeof(double));
  L.gs_obs = o;  o = align256(o + U * ds * sizeof(float));
  L.gs_con = o;  o = align256(o + U * ds * sizeof(float));
  L.med = o;     o = align256(o + sizeof(MedianState));
  const size_t P = (size_t)J.N * (J.N - 1) / 2;
  const bool large = P > (size_t)kSmallPairs;
  L.khi = o;     o = align256(o + (large ? (size_t)kSampleKeys : P) * sizeof(uint32_t));
  L.klo = o;     o = align256(o + (large ? 0 : P) * sizeof(uint32_t));
  L.cand = o;    o = align256(o + P * (large ? sizeof(uint64_t) : sizeof(uint32_t)));
  const size_t chunks = J.N > kPhiFusedMaxN ? ((size_t)J.N + kPhiChunk - 1) / kPhiChunk : 0;
  L.phi_part = o; o = align256(o + chunks * (size_t)J.N * J.M * sizeof(float));
  L.phi_live = o; o = align256(o + chunks * sizeof(uint32_t));
  L.total = o;
  return L;
}

// Launchers implemented in the .hip files.  Each returns a hipError_t.
hipError_t launch_planar_forward(const JobMap& map, int nb, bool rigid, const pds_job* d_jobs, int grid,
                                 bool with_ll, hipStream_t s);
hipError_t launch_planar_adjoint(const JobMap& map, int nb, bool rigid, const pds_job* d_jobs, char* ws, int grid,
                                 bool split, bool full, bool tape, size_t lds_bytes, hipStream_t s);
hipError_t launch_assemble(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, bool with_grad,
                           hipStream_t s);
hipError_t launch_assemble_grad(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_assemble_sdot(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
// Particles with at most this many shooting-state components get S_dot from
// their assembly block (two per thread); larger ones from a
// one-thread-per-component kernel.
constexpr int kSdotInline = 512;
struct MedianMaps {
  JobMap keys, select, count, large;
  int grid_keys, grid_select, grid_count, grid_large;
  // the narrow chain of larger jobs whose bandwidth runs beside a window
  // kernel that leaves SIMDs free (one-wave blocks; svgd.hip)
  JobMap lean_keys, lean_count, lean_final;
  int grid_lean_keys = 0, grid_lean_count = 0, grid_lean_final = 0;
};
hipError_t launch_median(const MedianMaps& mm, const pds_job* d_jobs, char* ws, int mmax, int rank_shift,
                         hipStream_t s);
// A step launch gives each job at most this many blocks (each thread
// taking every (blocks x threads)-th element), so that the blocks can
// advance the device iteration counter themselves by a completion count.
constexpr int kStepCountBlocks = 256;
constexpr int kStepThreads = 1024;  // threads per step-kernel block
// Device address of the fixed workspace array of svgd_phi_noalloc on
// `device` (looked up once per device).
hipError_t noalloc_scratch(int device, void** out);
// Arm box mounts (the kernels' template argument): 0 hinge, 1 universal
// joint with the box's parameters in theta, 2 universal joint with two
// point masses in theta.
inline int arm_mount(int model) {
  return model == PDS_MODEL_ARM_UJOINT ? 1 : (model == PDS_MODEL_ARM_UJOINT_WEIGHTS ? 2 : 0);
}
constexpr int kArmSetupThreads = 256;  // threads per block of the arm set-up kernel
hipError_t launch_arm_setup(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_arm_forward(const JobMap& map, int mount, const pds_job* d_jobs, char* ws, int grid, bool with_ll,
                              hipStream_t s);
hipError_t launch_arm_adjoint(const JobMap& map, int mount, const pds_job* d_jobs, char* ws, int grid,
                              size_t lds_bytes, hipStream_t s);
// Checkpoint strides of the arm adjoint for windows of h steps with at most
// `slots` checkpoint states in LDS (false if none fits); *evals gets the
// forward-dynamics evaluations per window.
bool arm_ck_plan(int h, int slots, int* B1, int* B2, long* evals);
hipError_t launch_phi(const JobMap& map, const pds_job* d_jobs, int grid, int mmax, int ti, hipStream_t s);
hipError_t launch_phi_partial(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int mmax,
                              hipStream_t s);
hipError_t launch_phi_reduce(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_step(const JobMap& map, const pds_job* d_jobs, int grid, int optimizer, int iter,
                       hipStream_t s);

// Posterior-consistency metrics (metrics.hip): launch shape and workspace
// layout for n + m rows of d floats.
struct MetricsPlan {
  int R = 0;       // pooled rows n + m
  int tiles = 0;   // 64 x 64 pair tiles on and above the diagonal
  int splits = 1;  // blocks that share one tile's coordinate range
  size_t off_dist = 0, off_part = 0, off_rows = 0, off_sel = 0, bytes = 0;
};
MetricsPlan metrics_plan(int n, int m, int d);
hipError_t launch_metric_dist(const MetricsPlan& p, const float* P, const float* Q, int n, int m, int d,
                              const float* w, char* ws, hipStream_t s);
hipError_t launch_metric_rest(const MetricsPlan& p, int n, int m, int d, int k, int l, double sigma, double* out,
                              double* rows_out, char* ws, hipStream_t s);

}  // namespace pds
