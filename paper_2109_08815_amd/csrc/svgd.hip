// SVGD direction (eq. svgd_update) with the median-heuristic RBF kernel
// (Sec. III-A) and the MDMM parameter update (Sec. III-E, Algorithm 1).
//
// Bandwidth.  h = med^2 / log N with med the exact median of the N (N-1)/2
// pair distances ||(theta_i - theta_j) / rho||, computed in FP64 from the
// FP32 particles.  A non-negative IEEE double orders like its bit pattern
// read as uint64, so the median is found by an exact most-significant-digit
// radix select over the 64-bit patterns of the squared distances: eight
// passes of 8 bits, each a per-block LDS histogram (wave-aggregated
// increments) of the keys that still match the prefix fixed by earlier
// passes, summed into a global histogram with integer atomics
// (order-independent, hence deterministic).  The last block of a pass to
// finish fixes that pass's digit, so the next pass only reads the carried
// prefix.  Every pass recomputes the distances instead of storing the
// N^2/2 keys.  Both middle order statistics ((P-1)/2 and P/2 of P pairs) are
// selected at once.
//
// phi.  Blocks of 64 particles i against chunks of 128 particles j staged
// in LDS; FP32 partial sums per chunk, reduced in chunk order.
#include <cmath>

#include "common.h"

namespace pds {
namespace {

constexpr int kPairBlock = 64;  // particles i per block

__device__ inline uint32_t* hist_of(const pds_job& J, char* ws, uint64_t off) {
  const WsLayout L = ws_layout(J);
  return reinterpret_cast<uint32_t*>(ws + off + L.hist);
}

__device__ inline RadixState* state_of(uint32_t* hist) {
  return reinterpret_cast<RadixState*>(hist + kRadixPasses * 2 * 256);
}

__global__ void __launch_bounds__(256) hist_clear_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                         char* __restrict__ ws) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  uint32_t* hist = hist_of(J, ws, map.ws_off[e]);
  const int n = kRadixPasses * 2 * 256 + (int)(sizeof(RadixState) / sizeof(uint32_t));
  for (int t = threadIdx.x; t < n; t += 256) hist[t] = 0u;
}

// Squared scaled distance in FP64, summed in parameter order.
__device__ inline double pair_d2(const float* ti, const float* tj, const double* inv_rho, int M) {
  double s = 0.0;
  for (int m = 0; m < M; ++m) {
    const double z = ((double)ti[m] - (double)tj[m]) * inv_rho[m];
    s = __dadd_rn(s, __dmul_rn(z, z));
  }
  return s;
}

// Adds one count per valid lane to lh[bin]; the most common bin of the wave
// (the first valid lane's) is added once with the wave's tally.
__device__ inline void wave_hist_add(uint32_t* lh, bool valid, int bin) {
  const unsigned long long m = __ballot(valid);
  if (m == 0ull) return;
  const int leader = __ffsll((long long)m) - 1;
  const int lbin = __shfl(bin, leader);
  const bool same = valid && bin == lbin;
  const unsigned long long sm = __ballot(same);
  if ((int)(threadIdx.x & 63) == leader) atomicAdd(&lh[lbin], (uint32_t)__popcll(sm));
  if (valid && !same) atomicAdd(&lh[bin], 1u);
}

// One radix pass.  Block (ib, jc) covers particles i in [64 ib, 64 ib + 64)
// against j in [16 jc, 16 jc + 16), pairs with i < j only.  The last block
// of the job to finish fixes the pass's digit for both middle ranks (and,
// after the last pass, computes the bandwidth).
__global__ void __launch_bounds__(kPairBlock) radix_pass_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                char* __restrict__ ws, int pass) {
  __shared__ uint32_t lh[2][256];
  __shared__ float tj_s[kRadixJT * PDS_MAX_M];
  __shared__ int last_s;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int N = J.N, M = J.M;
  const int nib = (N + kPairBlock - 1) / kPairBlock;
  const int local = blockIdx.x - map.begin[e];
  const int nblocks = map.begin[e + 1] - map.begin[e];
  const int ib = local % nib, jc = local / nib;
  uint32_t* hist = hist_of(J, ws, map.ws_off[e]);
  RadixState* st = state_of(hist);
  const uint64_t P = (uint64_t)N * (N - 1) / 2;
  uint64_t p0 = 0, p1 = 0;
  if (pass > 0) {
    p0 = st->pre[0];
    p1 = st->pre[1];
  }
  for (int t = threadIdx.x; t < 512; t += kPairBlock) lh[t >> 8][t & 255] = 0u;
  const int j0 = jc * kRadixJT;
  const int nj = max(0, min(kRadixJT, N - j0));
  for (int t = threadIdx.x; t < nj * M; t += kPairBlock) tj_s[t] = J.theta[(size_t)j0 * M + t];
  __syncthreads();
  const int i = ib * kPairBlock + threadIdx.x;
  const bool row = i < N;
  if (nj > 0 && j0 + nj - 1 > ib * kPairBlock) {  // block touches the upper triangle
    double inv_rho[PDS_MAX_M];
    float ti[PDS_MAX_M];
    for (int m = 0; m < M; ++m) {
      inv_rho[m] = 1.0 / (double)J.rho[m];
      ti[m] = row ? J.theta[(size_t)i * M + m] : 0.f;
    }
    const int shift = 56 - 8 * pass;
    for (int jj = 0; jj < nj; ++jj) {
      const int j = j0 + jj;
      const bool valid = row && j > i;
      const double d2 = pair_d2(ti, &tj_s[jj * M], inv_rho, M);
      const uint64_t key = (uint64_t)__double_as_longlong(d2);
      const int bin = (int)((key >> shift) & 255u);
      const bool m0 = valid && (pass == 0 || (key >> (64 - 8 * pass)) == (p0 >> (64 - 8 * pass)));
      const bool m1 = valid && (pass == 0 || (key >> (64 - 8 * pass)) == (p1 >> (64 - 8 * pass)));
      wave_hist_add(lh[0], m0, bin);
      wave_hist_add(lh[1], m1, bin);
    }
  }
  __syncthreads();
  uint32_t* gh = hist + pass * 2 * 256;
  for (int t = threadIdx.x; t < 512; t += kPairBlock) {
    const uint32_t c = lh[t >> 8][t & 255];
    if (c) atomicAdd(&gh[t], c);
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last_s = (atomicAdd(&st->count[pass], 1u) == (uint32_t)(nblocks - 1));
  __syncthreads();
  if (!last_s) return;
  __threadfence();
  // ---- last block: fix this pass's digit ----
  for (int t = threadIdx.x; t < 512; t += kPairBlock)
    lh[t >> 8][t & 255] = __hip_atomic_load(&gh[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (threadIdx.x < 2) {
    const int tg = threadIdx.x;
    uint64_t pre = pass > 0 ? st->pre[tg] : 0ull;
    uint64_t r = pass > 0 ? st->rem[tg] : (P == 0 ? 0ull : (tg == 0 ? (P - 1) / 2 : P / 2));
    int b = 0;
    for (; b < 255; ++b) {
      const uint64_t c = lh[tg][b];
      if (r < c) break;
      r -= c;
    }
    pre |= (uint64_t)b << (56 - 8 * pass);
    st->pre[tg] = pre;
    st->rem[tg] = r;
  }
  if (pass == kRadixPasses - 1) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double h = 1.0;
      if (P > 0) {
        const double a = __longlong_as_double((long long)st->pre[0]);
        const double c = __longlong_as_double((long long)st->pre[1]);
        const double med = 0.5 * (sqrt(a) + sqrt(c));
        const double lg = log((double)N);
        if (med * med >= 1e-300 && lg > 0.0) h = med * med / lg;
      }
      J.bandwidth[0] = h;
    }
  }
}

// Writes h = 1 for jobs with a single particle (no pairs, no radix passes).
__global__ void bandwidth_single_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  if (threadIdx.x == 0) J.bandwidth[0] = 1.0;
}

// Partial phi of particles i (one per lane) over one chunk of j.
__global__ void __launch_bounds__(kPairBlock) phi_partial_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                 char* __restrict__ ws) {
  __shared__ float tj_s[kPhiChunk * PDS_MAX_M];
  __shared__ float gj_s[kPhiChunk * PDS_MAX_M];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int N = J.N, M = J.M;
  const int nib = (N + kPairBlock - 1) / kPairBlock;
  const int local = blockIdx.x - map.begin[e];
  const int ib = local % nib, jc = local / nib;
  const int j0 = jc * kPhiChunk;
  const int nj = min(kPhiChunk, N - j0);
  for (int t = threadIdx.x; t < nj * M; t += kPairBlock) {
    tj_s[t] = J.theta[(size_t)j0 * M + t];
    gj_s[t] = (float)J.g_obs[(size_t)j0 * M + t];
  }
  __syncthreads();
  const int i = ib * kPairBlock + threadIdx.x;
  if (i >= N) return;
  const float h = (float)J.bandwidth[0];
  const float inv_h = 1.0f / h;
  float ti[PDS_MAX_M], ir[PDS_MAX_M], ir2[PDS_MAX_M], acc[PDS_MAX_M];
  for (int m = 0; m < M; ++m) {
    ti[m] = J.theta[(size_t)i * M + m];
    ir[m] = 1.0f / J.rho[m];
    ir2[m] = ir[m] * ir[m];
    acc[m] = 0.f;
  }
  for (int jj = 0; jj < nj; ++jj) {
    float d2 = 0.f;
    for (int m = 0; m < M; ++m) {
      const float z = (ti[m] - tj_s[jj * M + m]) * ir[m];
      d2 += z * z;
    }
    const float k = expf(-d2 * inv_h);
    const float k2h = 2.0f * k * inv_h;
    for (int m = 0; m < M; ++m) acc[m] += k * gj_s[jj * M + m] + k2h * (ti[m] - tj_s[jj * M + m]) * ir2[m];
  }
  const WsLayout L = ws_layout(J);
  float* part = reinterpret_cast<float*>(ws + map.ws_off[e] + L.phi_part);
  for (int m = 0; m < M; ++m) part[((size_t)jc * N + i) * M + m] = acc[m];
}

__global__ void __launch_bounds__(256) phi_reduce_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                         char* __restrict__ ws) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int t = (blockIdx.x - map.begin[e]) * 256 + threadIdx.x;
  if (t >= J.N * J.M) return;
  const int chunks = (J.N + kPhiChunk - 1) / kPhiChunk;
  const WsLayout L = ws_layout(J);
  const float* part = reinterpret_cast<const float*>(ws + map.ws_off[e] + L.phi_part);
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += part[(size_t)c * J.N * J.M + t];
  J.phi[t] = s / (float)J.N;
}

// MDMM + optimizer update.  Flat index over theta (N M), S (N K (n_s-1) d_s)
// and lam_def (N K (n_s-1)).
__global__ void __launch_bounds__(256) step_kernel(JobMap map, const pds_job* __restrict__ jobs, int optimizer,
                                                   int iter) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int ds = 2 * J.n_dof;
  const int nSp = J.K * (J.n_s - 1) * ds;  // shooting floats per particle
  const int nLp = J.K * (J.n_s - 1);
  const int nT = J.N * J.M, nS = J.N * nSp, nL = J.N * nLp;
  const int t = (blockIdx.x - map.begin[e]) * 256 + threadIdx.x;
  const int stride = J.M + nSp;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int it = J.iter_dev ? *J.iter_dev + 1 : iter;
  const float bc1 = 1.0f - powf(b1, (float)it), bc2 = 1.0f - powf(b2, (float)it);
  if (t < nT) {
    const int i = t / J.M, m = t % J.M;
    const float x = J.theta[t];
    const float lo = J.lo[m], hi = J.hi[m];
    const float g = fminf(fmaxf(x, lo), hi) - x;
    const float dg = (x < lo || x > hi) ? -1.0f : 0.0f;
    const float xdot = J.phi[t] - (J.lam_lim[t] + J.c * g) * dg - (float)J.g_con[t];
    float xn;
    if (optimizer == PDS_OPT_SGD) {
      xn = x + J.lr_theta[m] * xdot;
    } else {
      const size_t a = (size_t)i * stride + m;
      const float gr = -xdot;
      const float mm = b1 * J.adam_m[a] + (1.0f - b1) * gr;
      const float vv = b2 * J.adam_v[a] + (1.0f - b2) * gr * gr;
      J.adam_m[a] = mm;
      J.adam_v[a] = vv;
      xn = x - J.lr_theta[m] * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    }
    J.theta[t] = xn;
    J.lam_lim[t] += J.eps_lam * g;
    if ((xn < lo || xn > hi) && J.flags) atomicOr(&J.flags[i], 4);
  } else if (t < nT + nS) {
    const int r = t - nT;
    const int i = r / nSp, q = r % nSp;
    const int d = q % ds;
    const float xdot = J.S_dot[r];
    if (optimizer == PDS_OPT_SGD) {
      J.S[r] += J.lr_S[d] * xdot;
    } else {
      const size_t a = (size_t)i * stride + J.M + q;
      const float gr = -xdot;
      const float mm = b1 * J.adam_m[a] + (1.0f - b1) * gr;
      const float vv = b2 * J.adam_v[a] + (1.0f - b2) * gr * gr;
      J.adam_m[a] = mm;
      J.adam_v[a] = vv;
      J.S[r] -= J.lr_S[d] * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    }
  } else if (t < nT + nS + nL) {
    const int r = t - nT - nS;
    J.lam_def[r] += J.eps_lam * (float)J.gdef[r];
  }
}

// Advances the device iteration counters after a step.
__global__ void iter_bump_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  if (threadIdx.x == 0 && J.iter_dev) *J.iter_dev += 1;
}

}  // namespace

hipError_t launch_iter_bump(const JobMap& map, const pds_job* d_jobs, int grid, hipStream_t s) {
  hipLaunchKernelGGL(iter_bump_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs);
  return hipGetLastError();
}

hipError_t launch_hist_clear(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(hist_clear_kernel, dim3(grid), dim3(256), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_radix_pass(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int pass,
                             hipStream_t s) {
  if (pass >= kRadixPasses) {
    hipLaunchKernelGGL(bandwidth_single_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs);
  } else {
    hipLaunchKernelGGL(radix_pass_kernel, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws, pass);
  }
  return hipGetLastError();
}

hipError_t launch_phi_partial(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(phi_partial_kernel, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_phi_reduce(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(phi_reduce_kernel, dim3(grid), dim3(256), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_step(const JobMap& map, const pds_job* d_jobs, int grid, int optimizer, int iter,
                       hipStream_t s) {
  hipLaunchKernelGGL(step_kernel, dim3(grid), dim3(256), 0, s, map, d_jobs, optimizer, iter);
  return hipGetLastError();
}

}  // namespace pds
