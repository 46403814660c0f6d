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
};

// Entry of the block's job (scalar loop: every lane agrees).
__device__ inline int map_entry(const JobMap& m, int block) {
  int e = 0;
  while (e + 1 < m.n && block >= m.begin[e + 1]) ++e;
  return e;
}

constexpr size_t kArmConstBytes = 2048;  // derived arm model constants per job

// Workspace layout of one job (byte offsets from the job's region start).
// The arm model's derived constants come first, so forward-only calls can
// use a region of just that size.
struct WsLayout {
  size_t arm;                               // derived arm constants (arm jobs)
  size_t gth_obs, gth_con, gs_obs, gs_con;  // adjoint per-unit gradients
  size_t hist;                              // median radix histograms + state
  size_t cand;                              // median candidate keys
  size_t keys;                              // materialised pair keys (small problems)
  size_t phi_part;                          // phi partial sums
  size_t total;
};

constexpr int kPhiChunk = 32;    // particles j per phi partial
constexpr int kRadixPasses = 8;  // 8-bit digits of a 64-bit key
constexpr int kRadixJT = 16;     // particles j per radix-pass block (64 i per block)

// Selection state of the bandwidth median, carried between radix passes.
constexpr int kCandCap = 8192;   // keys the compaction pass may collect
// Up to this many pairs the median is one materialising kernel plus one
// single-block selection; above it, multi-block radix passes.
constexpr int kSmallPairs = 1 << 19;

struct RadixState {
  uint64_t pre[2];   // key prefix fixed so far, for both middle ranks
  uint64_t rem[2];   // rank among keys sharing that prefix
  uint32_t count[kRadixPasses];  // blocks finished per pass
  uint32_t done;        // selection finished
  uint32_t compact_at;  // 1 + pass that collects candidates, 0 = none yet
  uint32_t ncand;       // candidates collected
  uint32_t pad[kRadixPasses - 3];
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline WsLayout ws_layout(const pds_job& J) {
  WsLayout L;
  const size_t U = (size_t)J.N * J.K * J.n_s;
  const int ds = 2 * J.n_dof;
  size_t o = 0;
  L.arm = o;     o = align256(o + (J.model == PDS_MODEL_ARM ? kArmConstBytes : 0));
  L.gth_obs = o; o = align256(o + U * J.M * sizeof(double));
  L.gth_con = o; o = align256(o + U * J.M * sizeof(double));
  L.gs_obs = o;  o = align256(o + U * ds * sizeof(float));
  L.gs_con = o;  o = align256(o + U * ds * sizeof(float));
  L.hist = o;    o = align256(o + (size_t)kRadixPasses * 2 * 256 * sizeof(uint32_t) + sizeof(RadixState));
  L.cand = o;    o = align256(o + (size_t)kCandCap * sizeof(uint64_t));
  const size_t P = (size_t)J.N * (J.N - 1) / 2;
  L.keys = o;    o = align256(o + (P <= (size_t)kSmallPairs ? P : 0) * sizeof(uint64_t));
  const size_t chunks = ((size_t)J.N + kPhiChunk - 1) / kPhiChunk;
  L.phi_part = o; o = align256(o + chunks * (size_t)J.N * J.M * sizeof(float));
  L.total = o;
  return L;
}

// Launchers implemented in the .hip files.  Each returns a hipError_t.
hipError_t launch_planar_forward(const JobMap& map, int nb, const pds_job* d_jobs, int grid, bool with_ll,
                                 hipStream_t s);
hipError_t launch_planar_adjoint(const JobMap& map, int nb, const pds_job* d_jobs, char* ws, int grid, bool split,
                                 bool full, size_t lds_bytes, hipStream_t s);
hipError_t launch_assemble(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, bool with_grad,
                           hipStream_t s);
hipError_t launch_assemble_grad(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_assemble_sdot(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_median_small(const JobMap& map_keys, int grid_keys, const JobMap& map_sel, int grid_sel,
                               const pds_job* d_jobs, char* ws, int mmax, hipStream_t s);
hipError_t launch_iter_bump(const JobMap& map, const pds_job* d_jobs, int grid, hipStream_t s);
hipError_t launch_arm_setup(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_arm_forward(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, bool with_ll,
                              hipStream_t s);
hipError_t launch_arm_adjoint(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, bool full,
                              size_t lds_bytes, hipStream_t s);
int arm_seg_len_host(int h);
hipError_t launch_hist_clear(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_radix_pass(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int pass, int mmax,
                             hipStream_t s);
hipError_t launch_phi_partial(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int mmax,
                              hipStream_t s);
hipError_t launch_phi_reduce(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_step(const JobMap& map, const pds_job* d_jobs, int grid, int optimizer, int iter,
                       hipStream_t s);

}  // namespace pds
