// Per-particle reductions after the window kernels, all in FP64 and in a
// fixed order (deterministic, independent of the batch a job runs in).
//
//   logp / wk   combination over trajectories (eq. traj_likelihood, in log
//               space with the 1/K weight, or the product of App. A-B):
//               l_k = sum_j l_kj; SUM: log p = logsumexp_k l_k - log K,
//               w_k = softmax_k l_k; PROD: log p = sum_k l_k, w_k = 1.
//   g_obs       seed_logp * sum_k w_k sum_j d l_kj / d theta.
//   g_con       sum_{k,j} seed_gdef_kj d g_def_kj / d theta.
//   S_dot       for shooting state S_kj (j >= 1): seed_logp w_k d l_kj / d S_kj
//               - seed_gdef_kj d g_def_kj / d S_kj - seed_gdef_k(j-1) d g_def_k(j-1) / d S_kj,
//               the last term the direct dependence of the previous window's
//               defect on its target (Sec. III-E, Algorithm 1).
#include <cmath>

#include "common.h"

namespace pds {
namespace {

// sum_{j < n} p[j * stride], added in order j = 0, 1, ...; the loads are
// issued eight at a time (clamped in-bounds indices) so they overlap.
__device__ inline double sum_in_order(const double* p, size_t stride, int n) {
  double a = 0.0;
  constexpr int B = 8;
  for (int j0 = 0; j0 < n; j0 += B) {
    double v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = p[(size_t)(j0 + b < n ? j0 + b : n - 1) * stride];
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (j0 + b < n) a += v[b];
  }
  return a;
}

// Combination over trajectories for particle i; writes logp and wk.
__device__ inline void combine_particle(const pds_job& J, int i) {
  const int K = J.K, ns = J.n_s;
  const double* lw = J.ll_win + (size_t)i * K * ns;
  double mx = -INFINITY, lp = 0.0;
  for (int k = 0; k < K; ++k) {
    const double a = sum_in_order(lw + k * ns, 1, ns);
    J.wk[(size_t)i * K + k] = a;  // holds l_k until the weights are known
    mx = fmax(mx, a);
    lp += a;
  }
  if (J.combine == PDS_COMBINE_PROD) {
    for (int k = 0; k < K; ++k) J.wk[(size_t)i * K + k] = 1.0;
  } else {
    double z = 0.0;
    for (int k = 0; k < K; ++k) z += exp(J.wk[(size_t)i * K + k] - mx);
    for (int k = 0; k < K; ++k) J.wk[(size_t)i * K + k] = exp(J.wk[(size_t)i * K + k] - mx) / z;
    lp = mx + log(z) - log((double)K);
  }
  J.logp[i] = lp;
  if (!isfinite(lp) && J.flags) atomicOr(&J.flags[i], 2);
}

// Forward-only path: one thread per particle.
__global__ void __launch_bounds__(64) assemble_logp_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int i = (blockIdx.x - map.begin[e]) * 64 + threadIdx.x;
  if (i >= J.N) return;
  combine_particle(J, i);
}

// S_dot of shooting-state component r = ((k (n_s-1) + j-1) d_s + d) of
// particle i (window j >= 1 starts from it).
__device__ inline void sdot_element(const pds_job& J, int i, int r, size_t U, const float* gso, const float* gsc) {
  const int ds = 2 * J.n_dof;
  const int nS = J.K * (J.n_s - 1) * ds;
  const int d = r % ds;
  const int kj = r / ds;
  const int k = kj / (J.n_s - 1);
  const int j = kj % (J.n_s - 1) + 1;  // window started by this shooting state
  const size_t u = ((size_t)k * J.n_s + j) * J.N + i;
  const double seed = J.seed_logp ? J.seed_logp[i] : 1.0;
  double v = seed * J.wk[(size_t)i * J.K + k] * (double)gso[(size_t)d * U + u] - (double)gsc[(size_t)d * U + u];
  // defect of window j-1, whose target is this shooting state
  const size_t id = ((size_t)i * J.K + k) * (J.n_s - 1) + (j - 1);
  const double g = J.gdef[id];
  const double sg = J.seed_gdef ? J.seed_gdef[id] : (double)J.lam_def[id] + (double)J.c * g;
  const float s_next = J.S[id * ds + d];
  const float s_end = J.end_states[(((size_t)i * J.K + k) * J.n_s + (j - 1)) * ds + d];
  const double ud = J.u[d];
  const double err = (double)(s_next - s_end) * ud;
  v -= sg * 2.0 * err * ud / ((double)J.sigma_def * J.sigma_def);
  J.S_dot[(size_t)i * nS + r] = (float)v;
  if (!isfinite(v) && J.flags) atomicOr(&J.flags[i], 2);
}

// Adjoint path: one 64-lane block per particle.  Lane 0 combines the
// window log-likelihoods over trajectories; lanes then sum the per-window
// parameter gradients of one (parameter, trajectory) pair each (per-unit
// terms laid out [m][u], u = (k n_s + j) N + i); lane m weights and sums
// over trajectories; finally the lanes write the particle's S_dot.  Every
// sum runs in a fixed order.
constexpr int kMaxKM = 256;  // (parameter, trajectory) pairs held in LDS per pass

__global__ void __launch_bounds__(64) assemble_grad_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                           char* __restrict__ ws) {
  __shared__ double sa[kMaxKM], sc[kMaxKM];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int i = blockIdx.x - map.begin[e];
  if (i >= J.N) return;
  const int K = J.K, ns = J.n_s, M = J.M;
  const int t = threadIdx.x;
  if (t == 0) combine_particle(J, i);
  __syncthreads();
  const WsLayout L = ws_layout(J);
  const char* base = ws + map.ws_off[e];
  const size_t U = (size_t)J.N * K * ns;
  const double* go = reinterpret_cast<const double*>(base + L.gth_obs);
  const double* gc = reinterpret_cast<const double*>(base + L.gth_con);
  const double seed = J.seed_logp ? J.seed_logp[i] : 1.0;
  // parameters in groups so that (parameter, trajectory) pairs fit in LDS
  const int mg = K >= kMaxKM ? 1 : kMaxKM / K;
  for (int m0 = 0; m0 < M; m0 += mg) {
    const int m1 = min(M, m0 + mg);
    const int npair = (m1 - m0) * K;
    for (int p = t; p < npair; p += 64) {
      const int m = m0 + p / K, k = p % K;
      const size_t u0 = (size_t)k * ns * J.N + i;  // unit of window 0; window j adds j N
      sa[p] = sum_in_order(go + (size_t)m * U + u0, J.N, ns);
      sc[p] = sum_in_order(gc + (size_t)m * U + u0, J.N, ns);
    }
    __syncthreads();
    for (int m = m0 + t; m < m1; m += 64) {
      double so = 0.0, scon = 0.0;
      for (int k = 0; k < K; ++k) {
        const int p = (m - m0) * K + k;
        so += J.wk[(size_t)i * K + k] * sa[p];
        scon += sc[p];
      }
      J.g_obs[(size_t)i * M + m] = seed * so;
      J.g_con[(size_t)i * M + m] = scon;
    }
    __syncthreads();
  }
  const int nS = K * (ns - 1) * 2 * J.n_dof;
  if (ns > 1 && nS <= kSdotInline) {  // else assemble_sdot_kernel, one thread per component
    const float* gso = reinterpret_cast<const float*>(base + L.gs_obs);
    const float* gsc = reinterpret_cast<const float*>(base + L.gs_con);
    for (int r = t; r < nS; r += 64) sdot_element(J, i, r, U, gso, gsc);
  }
}

// S_dot with one thread per shooting-state component, for particles with
// more than kSdotInline components.
__global__ void __launch_bounds__(256) assemble_sdot_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                            char* __restrict__ ws) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int nS = J.K * (J.n_s - 1) * 2 * J.n_dof;
  const int t = (blockIdx.x - map.begin[e]) * 256 + threadIdx.x;
  if (t >= J.N * nS) return;
  const WsLayout L = ws_layout(J);
  const char* base = ws + map.ws_off[e];
  const size_t U = (size_t)J.N * J.K * J.n_s;
  sdot_element(J, t / nS, t % nS, U, reinterpret_cast<const float*>(base + L.gs_obs),
               reinterpret_cast<const float*>(base + L.gs_con));
}

}  // namespace

hipError_t launch_assemble(const JobMap& map, const pds_job* d_jobs, char* /*ws*/, int grid, bool /*with_grad*/,
                           hipStream_t s) {
  hipLaunchKernelGGL(assemble_logp_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs);
  return hipGetLastError();
}

hipError_t launch_assemble_sdot(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(assemble_sdot_kernel, dim3(grid), dim3(256), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_assemble_grad(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(assemble_grad_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}


}  // namespace pds
