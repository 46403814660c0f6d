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

// Workspace layout of one job (byte offsets from the job's region start).
struct WsLayout {
  size_t gth_obs, gth_con, gs_obs, gs_con;  // adjoint per-unit gradients
  size_t hist;                              // median radix histograms
  size_t phi_part;                          // phi partial sums
  size_t total;
};

constexpr int kPhiChunk = 32;    // particles j per phi partial
constexpr int kRadixPasses = 8;  // 8-bit digits of a 64-bit key
constexpr int kRadixJT = 16;     // particles j per radix-pass block (64 i per block)

// Selection state of the bandwidth median, carried between radix passes.
struct RadixState {
  uint64_t pre[2];   // key prefix fixed so far, for both middle ranks
  uint64_t rem[2];   // rank among keys sharing that prefix
  uint32_t count[kRadixPasses];  // blocks finished per pass
  uint32_t pad[kRadixPasses];
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline WsLayout ws_layout(const pds_job& J) {
  WsLayout L;
  const size_t U = (size_t)J.N * J.K * J.n_s;
  const int ds = 2 * J.n_dof;
  size_t o = 0;
  L.gth_obs = o; o = align256(o + U * J.M * sizeof(double));
  L.gth_con = o; o = align256(o + U * J.M * sizeof(double));
  L.gs_obs = o;  o = align256(o + U * ds * sizeof(float));
  L.gs_con = o;  o = align256(o + U * ds * sizeof(float));
  L.hist = o;    o = align256(o + (size_t)kRadixPasses * 2 * 256 * sizeof(uint32_t) + sizeof(RadixState));
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
hipError_t launch_hist_clear(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_radix_pass(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int pass,
                             hipStream_t s);
hipError_t launch_phi_partial(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_phi_reduce(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s);
hipError_t launch_iter_bump(const JobMap& map, const pds_job* d_jobs, int grid, hipStream_t s);
hipError_t launch_step(const JobMap& map, const pds_job* d_jobs, int grid, int optimizer, int iter,
                       hipStream_t s);

}  // namespace pds
