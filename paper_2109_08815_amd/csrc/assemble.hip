// Per-particle reductions after the window kernels, all in FP64 and in a
// fixed order (deterministic, independent of the batch a job runs in).
//
//   logp / wk   combination over trajectories (eq. traj_likelihood, in log
//               space with the 1/K weight, or the product of App. A-B):
//               l_k = sum_j l_kj; SUM: log p = logsumexp_k l_k - log K,
//               w_k = softmax_k l_k; PROD: log p = sum_k l_k, w_k = 1.
//   g_obs       seed_logp * sum_k w_k sum_j d l_kj / d theta.
//   g_con       sum_{k,j} seed_gdef_kj d g_def_kj / d theta.
//   g_theta     g_obs - g_con (optional), the theta counterpart of S_dot.
//   S_dot       for shooting state S_kj (j >= 1): seed_logp w_k d l_kj / d S_kj
//               - seed_gdef_kj d g_def_kj / d S_kj - seed_gdef_k(j-1) d g_def_k(j-1) / d S_kj,
//               the last term the direct dependence of the previous window's
//               defect on its target (Sec. III-E, Algorithm 1).
#include <cmath>

#include "common.h"

namespace pds {
namespace {

// sum_{j < n} p[j * stride], added in order j = 0, 1, ...; the loads are
// issued B at a time (clamped in-bounds indices) so they overlap.
template <int B = 8>
__device__ inline double sum_in_order(const double* p, size_t stride, int n) {
  double a = 0.0;
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
  if (!isfinite(lp) && J.flags) atomicOr(&J.flags[i], PDS_FLAG_GRAD);
}

// Forward-only path: one thread per particle.
__global__ void __launch_bounds__(64) assemble_logp_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int i = (blockIdx.x - map.begin[e]) * 64 + threadIdx.x;
  if (i >= J.N) return;
  combine_particle(J, i);
}

// Per-unit adjoint outputs are laid out with the unit index in particle
// order, iu = (i K + k) n_s + j: parameter terms as [iu][m], shooting-state
// terms as [iu][d].  One particle's terms are therefore contiguous.

// S_dot of shooting-state component r = ((k (n_s-1) + j-1) d_s + d) of
// particle i (window j >= 1 starts from it), split into the parts known
// before the trajectory weights: S_dot = seed w_k a - b - c (with
// PDS_LIK_DEFECT, a includes the defect's direct term).
struct SdotPart {
  double a, b, c;
  int k;
};

__device__ inline SdotPart sdot_part(const pds_job& J, int i, int r, const float* gso, const float* gsc) {
  const int ds = 2 * J.n_dof;
  const int d = r % ds;
  const int kj = r / ds;
  const int k = kj / (J.n_s - 1);
  const int j = kj % (J.n_s - 1) + 1;  // window started by this shooting state
  const size_t iu = ((size_t)i * J.K + k) * J.n_s + j;
  SdotPart p;
  p.k = k;
  p.a = (double)gso[iu * ds + d];
  p.b = (double)gsc[iu * ds + d];
  // defect of window j-1, whose target is this shooting state
  const size_t id = ((size_t)i * J.K + k) * (J.n_s - 1) + (j - 1);
  const double g = J.gdef[id];
  const bool in_lik = J.lik == PDS_LIK_DEFECT;
  const double sg = con_seed(J, id, g, in_lik);
  const float s_next = J.S[id * ds + d];
  const float s_end = J.end_states[(iu - 1) * ds + d];
  const double ud = J.u[d];
  const double err = (double)(s_next - s_end) * ud;
  p.c = sg * 2.0 * err * ud / ((double)J.sigma_def * J.sigma_def);
  // in the likelihood the defect's log density depends on its target
  // directly: d(-g/2) / d S = -e u / sigma^2, weighted like the window terms
  if (in_lik) p.a -= err * ud / ((double)J.sigma_def * J.sigma_def);
  return p;
}

__device__ inline void sdot_finish(const pds_job& J, int i, int r, const SdotPart& p, double seed, double w) {
  const int nS = J.K * (J.n_s - 1) * 2 * J.n_dof;
  double v = seed * w * p.a - p.b;
  v -= p.c;
  J.S_dot[(size_t)i * nS + r] = (float)v;
  if (!isfinite(v) && J.flags) atomicOr(&J.flags[i], PDS_FLAG_GRAD);
}

// Wave sum over the 64 lanes by a fixed xor tree (every lane gets the sum).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Trajectory combination for particle i from l_k in LDS (K <= kAsmCap),
// by the block's first wave: lane t handles k = t, t + 64, ... (in order),
// lanes meet by fixed shuffle trees.  Weights to w (LDS) and wk, log p to
// logp.
__device__ inline void combine_wave(const pds_job& J, int i, const double* l, double* w) {
  const int K = J.K, lane = threadIdx.x;
  double mx = -INFINITY, ls = 0.0;
  for (int k = lane; k < K; k += kWave) {
    mx = fmax(mx, l[k]);
    ls += l[k];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  double lp;
  if (J.combine == PDS_COMBINE_PROD || K == 1) {
    // (one trajectory: the mixture's weight is 1 and its log-sum-exp the
    // trajectory's sum, exactly, so both combinations coincide)
    for (int k = lane; k < K; k += kWave) w[k] = 1.0;
    lp = wave_sum(ls);
  } else {
    double z = 0.0;
    for (int k = lane; k < K; k += kWave) {
      const double ek = exp(l[k] - mx);
      w[k] = ek;
      z += ek;
    }
    z = wave_sum(z);
    for (int k = lane; k < K; k += kWave) w[k] /= z;
    lp = mx + log(z) - log((double)K);
  }
  for (int k = lane; k < K; k += kWave) J.wk[(size_t)i * K + k] = w[k];
  if (lane == 0) {
    J.logp[i] = lp;
    if (!isfinite(lp) && J.flags) atomicOr(&J.flags[i], PDS_FLAG_GRAD);
  }
}

// Trajectory combination for particle i from l_k already held in wk.
__device__ inline void combine_sums(const pds_job& J, int i) {
  const int K = J.K;
  double* wk = J.wk + (size_t)i * K;
  double mx = -INFINITY, lp = 0.0;
  for (int k = 0; k < K; ++k) {
    mx = fmax(mx, wk[k]);
    lp += wk[k];
  }
  if (J.combine == PDS_COMBINE_PROD) {
    for (int k = 0; k < K; ++k) wk[k] = 1.0;
  } else {
    double z = 0.0;
    for (int k = 0; k < K; ++k) z += exp(wk[k] - mx);
    for (int k = 0; k < K; ++k) wk[k] = exp(wk[k] - mx) / z;
    lp = mx + log(z) - log((double)K);
  }
  J.logp[i] = lp;
  if (!isfinite(lp) && J.flags) atomicOr(&J.flags[i], PDS_FLAG_GRAD);
}

// Adjoint path: one block per particle.  Every global load of the particle
// is issued up front, spread over the block's threads: the trajectory sums
// l_k = sum_j l_kj, the (parameter, trajectory) window sums of both
// channels (contiguous rows of n_s terms) and the particle's S_dot inputs.
// Thread 0 then combines over trajectories; threads m weight and sum the
// parameter rows over k; S_dot takes its trajectory weight last.  Every
// sum runs in a fixed order.
constexpr int kAsmThreads = 256;
constexpr int kAsmCap = 512;  // (parameter, trajectory) sums per channel held in LDS per pass

__global__ void __launch_bounds__(kAsmThreads) assemble_grad_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                    char* __restrict__ ws) {
  __shared__ double sa[kAsmCap], sc[kAsmCap], sw[kAsmCap], sl[kAsmCap];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int i = blockIdx.x - map.begin[e];
  if (i >= J.N) return;
  const int K = J.K, ns = J.n_s, M = J.M;
  const int t = threadIdx.x;
  const WsLayout L = ws_layout(J);
  const char* base = ws + map.ws_off[e];
  const size_t pu = (size_t)i * K * ns;  // first unit of particle i
  const double* go = reinterpret_cast<const double*>(base + L.gth_obs);
  const double* gc = reinterpret_cast<const double*>(base + L.gth_con);
  const double seed = J.seed_logp ? J.seed_logp[i] : 1.0;
  const int nS = K * (ns - 1) * 2 * J.n_dof;
  const bool inl = ns > 1 && nS <= kSdotInline;  // else assemble_sdot_kernel
  SdotPart sp[2];
  if (inl) {
    const float* gso = reinterpret_cast<const float*>(base + L.gs_obs);
    const float* gsc = reinterpret_cast<const float*>(base + L.gs_con);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = t + q * kAsmThreads;
      if (r < nS) sp[q] = sdot_part(J, i, r, gso, gsc);
    }
  }
  const int kc = K < kAsmCap ? K : kAsmCap;  // trajectories per chunk
  const int mg = kAsmCap / kc;               // parameters per pass
  // up to kAsmCap trajectories: l_k and the weights stay in LDS (one chunk)
  const bool in_lds = K <= kAsmCap;
  bool first = true;
  for (int m0 = 0; m0 < M; m0 += mg) {
    const int m1 = min(M, m0 + mg);
    double so = 0.0, scon = 0.0;  // thread t < m1 - m0 owns parameter m0 + t
    for (int k0 = 0; k0 < K; k0 += kc) {
      const int nk = min(K, k0 + kc) - k0;
      const int np = (m1 - m0) * nk;
      const int lead = first ? K : 0;  // the first pass also sums the window log-likelihoods
      for (int r = t; r < lead + 2 * np; r += kAsmThreads) {
        if (r < lead) {
          const double l = sum_in_order<16>(J.ll_win + pu + (size_t)r * ns, 1, ns);
          if (in_lds) sl[r] = l;
          else J.wk[(size_t)i * K + r] = l;  // l_k for now
        } else {
          // row p = (k - k0) (m1 - m0) + (m - m0): neighbouring threads read
          // neighbouring parameters of one unit
          const bool con = r - lead >= np;
          const int p = con ? r - lead - np : r - lead;
          const int m = m0 + p % (m1 - m0), k = k0 + p / (m1 - m0);
          const double v = sum_in_order<16>((con ? gc : go) + (pu + (size_t)k * ns) * M + m, M, ns);
          if (con) sc[p] = v; else sa[p] = v;
        }
      }
      __syncthreads();
      if (first) {
        if (in_lds) {
          if (t < kWave) combine_wave(J, i, sl, sw);
        } else if (t == 0) {
          combine_sums(J, i);
        }
        first = false;
        __syncthreads();
      }
      if (!in_lds) {
        for (int k = t; k < nk; k += kAsmThreads) sw[k] = J.wk[(size_t)i * K + k0 + k];
        __syncthreads();
      }
      if (t < m1 - m0) {
        for (int k = 0; k < nk; ++k) {
          so += sw[k] * sa[k * (m1 - m0) + t];
          scon += sc[k * (m1 - m0) + t];
        }
      }
      __syncthreads();
    }
    if (t < m1 - m0) {
      const double gob = seed * so;
      J.g_obs[(size_t)i * M + m0 + t] = gob;
      J.g_con[(size_t)i * M + m0 + t] = scon;
      if (J.g_theta) J.g_theta[(size_t)i * M + m0 + t] = gob - scon;
      if (!(isfinite(gob) && isfinite(scon)) && J.flags) atomicOr(&J.flags[i], PDS_FLAG_GRAD);
    }
  }
  if (inl) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = t + q * kAsmThreads;
      if (r < nS) sdot_finish(J, i, r, sp[q], seed, in_lds ? sw[sp[q].k] : J.wk[(size_t)i * K + sp[q].k]);
    }
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
  const int i = t / nS, r = t % nS;
  const SdotPart p = sdot_part(J, i, r, reinterpret_cast<const float*>(base + L.gs_obs),
                               reinterpret_cast<const float*>(base + L.gs_con));
  const double seed = J.seed_logp ? J.seed_logp[i] : 1.0;
  sdot_finish(J, i, r, p, seed, J.wk[(size_t)i * J.K + p.k]);
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
  hipLaunchKernelGGL(assemble_grad_kernel, dim3(grid), dim3(kAsmThreads), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}


}  // namespace pds
