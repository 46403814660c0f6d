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

// Squared scaled distance in FP64, summed in parameter order.  MM is a
// compile-time bound on M so per-lane arrays stay in registers.
template <int MM>
__device__ inline double pair_d2(const float* ti, const float* tj, const double* inv_rho, int M) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    if (m < M) {
      const double z = ((double)ti[m] - (double)tj[m]) * inv_rho[m];
      s = __dadd_rn(s, __dmul_rn(z, z));
    }
  }
  return s;
}

// Inclusive scan over the 64 lanes of a wave (fixed order of additions).
__device__ inline uint32_t wave_scan(uint32_t v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o);
    if ((int)(threadIdx.x & 63) >= o) v += t;
  }
  return v;
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

// Exact selection among the collected candidate keys, by the remaining
// radix digits (from `pass` on), in one 64-lane block.
__device__ void finish_from_candidates(const uint64_t* cand, uint32_t n, int pass, uint64_t pre[2],
                                       uint64_t rem[2], uint32_t (*lh)[256]) {
  for (int q = pass; q < kRadixPasses; ++q) {
    for (int t = threadIdx.x; t < 512; t += 64) lh[t >> 8][t & 255] = 0u;
    __syncthreads();
    const int shift = 56 - 8 * q;
    for (uint32_t c = threadIdx.x; c < n; c += 64) {
      const uint64_t key = cand[c];
      const int bin = (int)((key >> shift) & 255u);
      const bool m0 = q == 0 || (key >> (64 - 8 * q)) == (pre[0] >> (64 - 8 * q));
      const bool m1 = q == 0 || (key >> (64 - 8 * q)) == (pre[1] >> (64 - 8 * q));
      if (m0) atomicAdd(&lh[0][bin], 1u);
      if (m1) atomicAdd(&lh[1][bin], 1u);
    }
    __syncthreads();
    for (int tg = 0; tg < 2; ++tg) {
      const int l = threadIdx.x;
      const uint32_t c0 = lh[tg][4 * l], c1 = lh[tg][4 * l + 1], c2 = lh[tg][4 * l + 2], c3 = lh[tg][4 * l + 3];
      const uint32_t incl = wave_scan(c0 + c1 + c2 + c3);
      const uint32_t excl = incl - (c0 + c1 + c2 + c3);
      const uint64_t r = rem[tg];
      const bool own = (uint64_t)excl <= r && r < (uint64_t)incl;
      const unsigned long long bal = __ballot(own);
      const int owner = bal ? __ffsll((long long)bal) - 1 : 63;
      int b = 4 * l;
      uint64_t rr = r - excl;
      if (rr >= c0) { rr -= c0; ++b;
        if (rr >= c1) { rr -= c1; ++b;
          if (rr >= c2) { rr -= c2; ++b; } } }
      const int bo = __shfl(b, owner);
      const uint64_t ro = __shfl((long long)rr, owner);
      pre[tg] |= (uint64_t)bo << shift;
      rem[tg] = ro;
    }
    __syncthreads();
  }
}

__device__ inline void write_bandwidth(const pds_job& J, uint64_t k0, uint64_t k1) {
  const uint64_t P = (uint64_t)J.N * (J.N - 1) / 2;
  double h = 1.0;
  if (P > 0) {
    const double a = __longlong_as_double((long long)k0);
    const double c = __longlong_as_double((long long)k1);
    const double med = 0.5 * (sqrt(a) + sqrt(c));
    const double lg = log((double)J.N);
    if (med * med >= 1e-300 && lg > 0.0) h = med * med / lg;
  }
  J.bandwidth[0] = h;
}

// One radix pass.  Block (ib, jc) covers particles i in [64 ib, 64 ib + 64)
// against j in [16 jc, 16 jc + 16), pairs with i < j only.  The last block
// of the job to finish fixes the pass's digit for both middle ranks.  Once
// both ranks lie among at most kCandCap keys, the next pass instead collects
// those keys and its last block finishes the selection from them; the
// passes after that return at once.
template <int MM>
__global__ void __launch_bounds__(kPairBlock) radix_pass_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                char* __restrict__ ws, int pass) {
  __shared__ uint32_t lh[2][256];
  __shared__ float tj_s[kRadixJT * PDS_MAX_M];
  __shared__ int last_s;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  uint32_t* hist = hist_of(J, ws, map.ws_off[e]);
  RadixState* st = state_of(hist);
  if (st->done) return;
  const int N = J.N, M = J.M;
  const int nib = (N + kPairBlock - 1) / kPairBlock;
  const int local = blockIdx.x - map.begin[e];
  const int nblocks = map.begin[e + 1] - map.begin[e];
  const int ib = local % nib, jc = local / nib;
  const WsLayout L = ws_layout(J);
  uint64_t* cand = reinterpret_cast<uint64_t*>(ws + map.ws_off[e] + L.cand);
  const bool compact = st->compact_at == (uint32_t)(pass + 1);
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
  const int lane = threadIdx.x & 63;
  if (nj > 0 && j0 + nj - 1 > ib * kPairBlock) {  // block touches the upper triangle
    double inv_rho[MM];
    float ti[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      inv_rho[m] = m < M ? 1.0 / (double)J.rho[m] : 0.0;
      ti[m] = (row && m < M) ? J.theta[(size_t)i * M + m] : 0.f;
    }
    const int shift = 56 - 8 * pass;
    for (int jj = 0; jj < nj; ++jj) {
      const int j = j0 + jj;
      const bool valid = row && j > i;
      const double d2 = pair_d2<MM>(ti, &tj_s[jj * M], inv_rho, M);
      const uint64_t key = (uint64_t)__double_as_longlong(d2);
      const int bin = (int)((key >> shift) & 255u);
      const bool m0 = valid && (pass == 0 || (key >> (64 - 8 * pass)) == (p0 >> (64 - 8 * pass)));
      const bool m1 = valid && (pass == 0 || (key >> (64 - 8 * pass)) == (p1 >> (64 - 8 * pass)));
      if (compact) {
        const bool want = m0 || m1;
        const unsigned long long bm = __ballot(want);
        if (bm) {
          const int leader = __ffsll((long long)bm) - 1;
          uint32_t base = 0;
          if (lane == leader) base = atomicAdd(&st->ncand, (uint32_t)__popcll(bm));
          base = __shfl(base, leader);
          const uint32_t off = (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
          if (want && base + off < (uint32_t)kCandCap) cand[base + off] = key;
        }
      } else {
        wave_hist_add(lh[0], m0, bin);
        wave_hist_add(lh[1], m1, bin);
      }
    }
  }
  __syncthreads();
  uint32_t* gh = hist + pass * 2 * 256;
  if (!compact) {
    for (int t = threadIdx.x; t < 512; t += kPairBlock) {
      const uint32_t c = lh[t >> 8][t & 255];
      if (c) atomicAdd(&gh[t], c);
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last_s = (atomicAdd(&st->count[pass], 1u) == (uint32_t)(nblocks - 1));
  __syncthreads();
  if (!last_s) return;
  __threadfence();
  // ---- last block ----
  uint64_t pre[2], rem[2];
  for (int tg = 0; tg < 2; ++tg) {
    pre[tg] = pass > 0 ? st->pre[tg] : 0ull;
    rem[tg] = pass > 0 ? st->rem[tg] : (P == 0 ? 0ull : (tg == 0 ? (P - 1) / 2 : P / 2));
  }
  if (compact) {
    const uint32_t n = min(__hip_atomic_load(&st->ncand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                           (uint32_t)kCandCap);
    finish_from_candidates(cand, n, pass, pre, rem, lh);
    if (threadIdx.x == 0) {
      write_bandwidth(J, pre[0], pre[1]);
      st->done = 1u;
    }
    return;
  }
  for (int t = threadIdx.x; t < 512; t += kPairBlock)
    lh[t >> 8][t & 255] = __hip_atomic_load(&gh[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  // Each lane owns 4 consecutive bins; a wave scan locates the bin holding
  // the wanted rank.
  uint32_t chosen[2];
  for (int tg = 0; tg < 2; ++tg) {
    const int l = threadIdx.x;
    const uint32_t c0 = lh[tg][4 * l], c1 = lh[tg][4 * l + 1], c2 = lh[tg][4 * l + 2], c3 = lh[tg][4 * l + 3];
    const uint32_t incl = wave_scan(c0 + c1 + c2 + c3);
    const uint32_t excl = incl - (c0 + c1 + c2 + c3);
    const uint64_t r = rem[tg];
    const bool own = (uint64_t)excl <= r && r < (uint64_t)incl;
    const unsigned long long bal = __ballot(own);
    const int owner = bal ? __ffsll((long long)bal) - 1 : 63;
    int b = 4 * l;
    uint64_t rr = r - excl;
    if (rr >= c0) { rr -= c0; ++b;
      if (rr >= c1) { rr -= c1; ++b;
        if (rr >= c2) { rr -= c2; ++b; } } }
    const int bo = __shfl(b, owner);
    const uint64_t ro = __shfl((long long)rr, owner);
    pre[tg] |= (uint64_t)bo << (56 - 8 * pass);
    rem[tg] = ro;
    chosen[tg] = lh[tg][bo];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->pre[0] = pre[0];
    st->rem[0] = rem[0];
    st->pre[1] = pre[1];
    st->rem[1] = rem[1];
    if (pass == kRadixPasses - 1) {
      write_bandwidth(J, pre[0], pre[1]);
      st->done = 1u;
    } else if ((uint64_t)chosen[0] + chosen[1] <= (uint64_t)kCandCap) {
      st->compact_at = (uint32_t)(pass + 2);
    }
  }
}

// ---------------------------------------------------------------------------
// Median for up to kSmallPairs pairs: one kernel writes every pair's key,
// one 1024-lane block per job selects both middle keys exactly.
// ---------------------------------------------------------------------------

// Row i of pair p in the row-major enumeration of pairs (i < j).
__device__ inline void pair_of(uint64_t p, int N, int* pi, int* pj) {
  const double b = 2.0 * N - 1.0;
  int i = (int)floor((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
  auto off = [N](long long r) -> unsigned long long { return (unsigned long long)(r * N - r * (r + 1) / 2); };
  if (i < 0) i = 0;
  if (i > N - 2) i = N - 2;
  while (i > 0 && off(i) > p) --i;
  while (i < N - 2 && off(i + 1) <= p) ++i;
  *pi = i;
  *pj = (int)(p - off(i)) + i + 1;
}

template <int MM>
__global__ void __launch_bounds__(256) median_keys_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                          char* __restrict__ ws) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int N = J.N, M = J.M;
  const uint64_t P = (uint64_t)N * (N - 1) / 2;
  const uint64_t p = (uint64_t)(blockIdx.x - map.begin[e]) * 256 + threadIdx.x;
  if (p >= P) return;
  int i, j;
  pair_of(p, N, &i, &j);
  double inv_rho[MM];
  float ti[MM], tj[MM];
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    inv_rho[m] = m < M ? 1.0 / (double)J.rho[m] : 0.0;
    ti[m] = m < M ? J.theta[(size_t)i * M + m] : 0.f;
    tj[m] = m < M ? J.theta[(size_t)j * M + m] : 0.f;
  }
  const WsLayout L = ws_layout(J);
  uint64_t* keys = reinterpret_cast<uint64_t*>(ws + map.ws_off[e] + L.keys);
  keys[p] = (uint64_t)__double_as_longlong(pair_d2<MM>(ti, tj, inv_rho, M));
}

constexpr int kSelThreads = 1024;

// Radix digit `q` of both targets from a 2 x 256 LDS histogram; wave 0
// scans.  Updates pre/rem in LDS.  Returns after a block barrier.
__device__ inline void select_digit(uint32_t (*lh)[256], int q, uint64_t* pre, uint64_t* rem, uint32_t* chosen) {
  if (threadIdx.x < 64) {
    for (int tg = 0; tg < 2; ++tg) {
      const int l = threadIdx.x;
      const uint32_t c0 = lh[tg][4 * l], c1 = lh[tg][4 * l + 1], c2 = lh[tg][4 * l + 2], c3 = lh[tg][4 * l + 3];
      const uint32_t incl = wave_scan(c0 + c1 + c2 + c3);
      const uint32_t excl = incl - (c0 + c1 + c2 + c3);
      const uint64_t r = rem[tg];
      const bool own = (uint64_t)excl <= r && r < (uint64_t)incl;
      const unsigned long long bal = __ballot(own);
      const int owner = bal ? __ffsll((long long)bal) - 1 : 63;
      int b = 4 * l;
      uint64_t rr = r - excl;
      if (rr >= c0) { rr -= c0; ++b;
        if (rr >= c1) { rr -= c1; ++b;
          if (rr >= c2) { rr -= c2; ++b; } } }
      const int bo = __shfl(b, owner);
      const uint64_t ro = __shfl((long long)rr, owner);
      if (threadIdx.x == 0) {
        pre[tg] |= (uint64_t)bo << (56 - 8 * q);
        rem[tg] = ro;
        chosen[tg] = lh[tg][bo];
      }
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kSelThreads) median_select_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                    char* __restrict__ ws) {
  __shared__ uint32_t lh[2][256];
  __shared__ uint64_t cand[kCandCap];
  __shared__ uint64_t pre[2], rem[2];
  __shared__ uint32_t chosen[2], ncand;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const uint64_t P = (uint64_t)J.N * (J.N - 1) / 2;
  const WsLayout L = ws_layout(J);
  const uint64_t* keys = reinterpret_cast<const uint64_t*>(ws + map.ws_off[e] + L.keys);
  if (threadIdx.x == 0) {
    pre[0] = pre[1] = 0ull;
    rem[0] = (P - 1) / 2;
    rem[1] = P / 2;
    ncand = 0u;
  }
  bool in_lds = false;
  uint32_t n = 0;
  for (int q = 0; q < kRadixPasses; ++q) {
    for (int t = threadIdx.x; t < 512; t += kSelThreads) lh[t >> 8][t & 255] = 0u;
    __syncthreads();
    const int shift = 56 - 8 * q;
    const uint64_t p0 = pre[0], p1 = pre[1];
    const uint64_t lim = in_lds ? (uint64_t)n : P;
    for (uint64_t c = threadIdx.x; c < lim + ((kSelThreads - lim % kSelThreads) % kSelThreads); c += kSelThreads) {
      const bool ok = c < lim;
      const uint64_t key = ok ? (in_lds ? cand[c] : keys[c]) : 0ull;
      const int bin = (int)((key >> shift) & 255u);
      const bool m0 = ok && (q == 0 || (key >> (64 - 8 * q)) == (p0 >> (64 - 8 * q)));
      const bool m1 = ok && (q == 0 || (key >> (64 - 8 * q)) == (p1 >> (64 - 8 * q)));
      wave_hist_add(lh[0], m0, bin);
      wave_hist_add(lh[1], m1, bin);
    }
    __syncthreads();
    select_digit(lh, q, pre, rem, chosen);
    // compact the surviving keys into LDS once they fit
    if (!in_lds && q + 1 < kRadixPasses && (uint64_t)chosen[0] + chosen[1] <= (uint64_t)kCandCap) {
      const int qs = 8 * (q + 1);
      const uint64_t a0 = pre[0], a1 = pre[1];
      for (uint64_t c = threadIdx.x; c < P; c += kSelThreads) {
        const uint64_t key = keys[c];
        if ((key >> (64 - qs)) == (a0 >> (64 - qs)) || (key >> (64 - qs)) == (a1 >> (64 - qs))) {
          const uint32_t slot = atomicAdd(&ncand, 1u);
          cand[slot] = key;
        }
      }
      __syncthreads();
      n = ncand;
      in_lds = true;
    }
  }
  if (threadIdx.x == 0) write_bandwidth(J, pre[0], pre[1]);
}

hipError_t median_small_impl(const JobMap& mk, int gk, const JobMap& ms, int gs, const pds_job* d_jobs, char* ws,
                             int mmax, hipStream_t s) {
  if (mmax <= 4)
    hipLaunchKernelGGL(median_keys_kernel<4>, dim3(gk), dim3(256), 0, s, mk, d_jobs, ws);
  else if (mmax <= 8)
    hipLaunchKernelGGL(median_keys_kernel<8>, dim3(gk), dim3(256), 0, s, mk, d_jobs, ws);
  else
    hipLaunchKernelGGL(median_keys_kernel<PDS_MAX_M>, dim3(gk), dim3(256), 0, s, mk, d_jobs, ws);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(median_select_kernel, dim3(gs), dim3(kSelThreads), 0, s, ms, d_jobs, ws);
  return hipGetLastError();
}

// Writes h = 1 for jobs with a single particle (no pairs, no radix passes).
__global__ void bandwidth_single_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  if (threadIdx.x == 0) J.bandwidth[0] = 1.0;
}

// Partial phi of particles i (one per lane) over one chunk of j.
template <int MM>
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
  float ti[MM], ir[MM], ir2[MM], acc[MM];
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    ti[m] = m < M ? J.theta[(size_t)i * M + m] : 0.f;
    ir[m] = m < M ? 1.0f / J.rho[m] : 0.f;
    ir2[m] = ir[m] * ir[m];
    acc[m] = 0.f;
  }
  for (int jj = 0; jj < nj; ++jj) {
    float d2 = 0.f;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      if (m < M) {
        const float z = (ti[m] - tj_s[jj * M + m]) * ir[m];
        d2 += z * z;
      }
    }
    const float k = expf(-d2 * inv_h);
    const float k2h = 2.0f * k * inv_h;
#pragma unroll
    for (int m = 0; m < MM; ++m)
      if (m < M) acc[m] += k * gj_s[jj * M + m] + k2h * (ti[m] - tj_s[jj * M + m]) * ir2[m];
  }
  const WsLayout L = ws_layout(J);
  float* part = reinterpret_cast<float*>(ws + map.ws_off[e] + L.phi_part);
#pragma unroll
  for (int m = 0; m < MM; ++m)
    if (m < M) part[((size_t)jc * N + i) * M + m] = acc[m];
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
  const int it = J.iter_dev ? J.iter_dev[0] + 1 : iter;
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

// Advances the device iteration counter after the step kernel (a separate
// launch: the step's blocks all read the counter, and a cross-block
// completion count would cost more than this kernel).
__global__ void iter_bump_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  if (threadIdx.x == 0 && J.iter_dev) J.iter_dev[0] += 1;
}

}  // namespace

hipError_t launch_median_small(const JobMap& map_keys, int grid_keys, const JobMap& map_sel, int grid_sel,
                               const pds_job* d_jobs, char* ws, int mmax, hipStream_t s) {
  return median_small_impl(map_keys, grid_keys, map_sel, grid_sel, d_jobs, ws, mmax, s);
}

hipError_t launch_iter_bump(const JobMap& map, const pds_job* d_jobs, int grid, hipStream_t s) {
  hipLaunchKernelGGL(iter_bump_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs);
  return hipGetLastError();
}

hipError_t launch_hist_clear(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(hist_clear_kernel, dim3(grid), dim3(256), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_radix_pass(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int pass, int mmax,
                             hipStream_t s) {
  if (pass >= kRadixPasses) {
    hipLaunchKernelGGL(bandwidth_single_kernel, dim3(grid), dim3(64), 0, s, map, d_jobs);
  } else if (mmax <= 4) {
    hipLaunchKernelGGL(radix_pass_kernel<4>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws, pass);
  } else if (mmax <= 8) {
    hipLaunchKernelGGL(radix_pass_kernel<8>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws, pass);
  } else {
    hipLaunchKernelGGL(radix_pass_kernel<PDS_MAX_M>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws, pass);
  }
  return hipGetLastError();
}

hipError_t launch_phi_partial(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int mmax,
                              hipStream_t s) {
  if (mmax <= 4)
    hipLaunchKernelGGL(phi_partial_kernel<4>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  else if (mmax <= 8)
    hipLaunchKernelGGL(phi_partial_kernel<8>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  else
    hipLaunchKernelGGL(phi_partial_kernel<PDS_MAX_M>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
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
