// Posterior-consistency metrics between two sets of trajectories: the
// k-nearest-neighbour KL estimate (App. A-D eq. knn-kl, after Wang et al.)
// in both directions and the squared maximum mean discrepancy of Sec. III-F
// (unbiased estimate, Gaussian kernel with the median-heuristic bandwidth).
//
// Rows of the pooled set Z = P u Q (n + m rows of d floats) are compared
// pairwise.  Pipeline on one stream:
//   metric_dist_kernel      squared distances of every pair, 64 x 64 pair
//                           tiles; small sets split the d range over blocks
//                           (metric_dist_reduce_kernel adds the parts in a
//                           fixed order)
//   metric_sel_*            exact median of the n+m choose 2 squared
//                           distances: radix select on the FP64 bit
//                           patterns, 8 bits per pass, both middle ranks at
//                           once, each pass deriving its digit prefix from
//                           the previous pass's histogram
//   metric_rows_kernel      one wave per row: k-th / l-th nearest squared
//                           distance in the other / own set, and the
//                           kernel sums over both sets
//   metric_final_kernel     fixed-order sums into the four outputs
//
// Distances are direct differences, squared and summed in FP32 over 32
// coordinates and in FP64 across those chunks.  Expanding into norms and a
// Gram matrix (the form a matrix core would take) cancels catastrophically
// for close pairs, and close pairs are exactly the nearest-neighbour
// distances whose logarithms the estimate adds up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"

namespace pds {
namespace {

constexpr int kMT = 64;       // pair-tile edge
constexpr int kMC = 32;       // coordinates per LDS chunk
constexpr int kMS = kMT + 4;  // LDS row stride (floats), keeps float4 rows aligned
constexpr int kKMax = PDS_METRICS_MAX_K;

__device__ inline const float* zrow(const float* P, const float* Q, int n, int d, int r) {
  return r < n ? P + (size_t)r * d : Q + (size_t)(r - n) * d;
}

// Squared distances of the pairs of one 64 x 64 tile (ti <= tj), over the
// chunk range [c_begin, c_end) of split `blockIdx.y`.  With one split the
// tile is written to both triangles of `dist`; with several, the upper
// triangle (i <= j) of split s goes to part + s R R.  Weights scale each
// coordinate's difference (not the coordinates), so a close pair keeps
// the relative accuracy of its difference.
template <bool HAS_W>
__global__ void __launch_bounds__(256) metric_dist_kernel(const float* __restrict__ P, const float* __restrict__ Q,
                                                          int n, int m, int d, const float* __restrict__ w,
                                                          double* __restrict__ dist, double* __restrict__ part,
                                                          int splits) {
  const int R = n + m;
  const int T = (R + kMT - 1) / kMT;
  int b = blockIdx.x, ti = 0;
  while (b >= T - ti) {
    b -= T - ti;
    ++ti;
  }
  const int tj = ti + b;
  const int chunks = (d + kMC - 1) / kMC;
  const int s = blockIdx.y;
  const int cb = (int)((long long)chunks * s / splits), ce = (int)((long long)chunks * (s + 1) / splits);
  __shared__ __align__(16) float As[kMC][kMS];
  __shared__ __align__(16) float Bs[kMC][kMS];
  __shared__ float Ws[kMC];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = ti * kMT, j0 = tj * kMT;
  // This thread stages coordinate lc of rows lr + 8 q (q = 0..7) of both
  // row blocks; row pointers are fixed for the whole coordinate range.
  constexpr int kRowsPerThread = kMT * kMC / 256;
  const int lc = threadIdx.x % kMC, lr = threadIdx.x / kMC;
  const float* pa[kRowsPerThread];
  const float* pb[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int ra = i0 + lr + 8 * q, rb = j0 + lr + 8 * q;
    pa[q] = ra < R ? zrow(P, Q, n, d, ra) + lc : nullptr;
    pb[q] = rb < R ? zrow(P, Q, n, d, rb) + lc : nullptr;
  }
  float na[kRowsPerThread], nb[kRowsPerThread];
  float nw = 0.f;
  auto fetch = [&](int ch) {
    const int col = ch * kMC;
    const bool in = col + lc < d;
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
      na[q] = (in && pa[q]) ? pa[q][col] : 0.f;
      nb[q] = (in && pb[q]) ? pb[q][col] : 0.f;
    }
    if (HAS_W) nw = in ? w[col + lc] : 0.f;
  };
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
  if (cb < ce) fetch(cb);
  for (int ch = cb; ch < ce; ++ch) {
    __syncthreads();  // the previous chunk is consumed
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
      As[lc][lr + 8 * q] = na[q];
      Bs[lc][lr + 8 * q] = nb[q];
    }
    if (HAS_W && lr == 0) Ws[lc] = nw;
    __syncthreads();
    if (ch + 1 < ce) fetch(ch + 1);  // in flight while this chunk is computed
    float sacc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) sacc[r][q] = 0.f;
#pragma unroll 8
    for (int c = 0; c < kMC; ++c) {
      const float4 a4 = *reinterpret_cast<const float4*>(&As[c][ty * 4]);
      const float4 b4 = *reinterpret_cast<const float4*>(&Bs[c][tx * 4]);
      const float av[4] = {a4.x, a4.y, a4.z, a4.w};
      const float bv[4] = {b4.x, b4.y, b4.z, b4.w};
      const float wc = HAS_W ? Ws[c] : 1.f;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float df = HAS_W ? (av[r] - bv[q]) * wc : av[r] - bv[q];
          sacc[r][q] = fmaf(df, df, sacc[r][q]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] += (double)sacc[r][q];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + q;
      if (i >= R || j >= R) continue;
      if (splits == 1) {
        dist[(size_t)i * R + j] = acc[r][q];
        dist[(size_t)j * R + i] = acc[r][q];
      } else if (i <= j) {
        part[(size_t)s * R * R + (size_t)i * R + j] = acc[r][q];
      }
    }
}

// Adds the split parts of each pair in split order and fills both triangles.
__global__ void __launch_bounds__(256) metric_dist_reduce_kernel(const double* __restrict__ part, int R, int splits,
                                                                 double* __restrict__ dist) {
  const size_t RR = (size_t)R * R;
  for (size_t f = (size_t)blockIdx.x * 256 + threadIdx.x; f < RR; f += (size_t)gridDim.x * 256) {
    const int i = (int)(f / R), j = (int)(f % R);
    if (j < i) continue;
    double v = 0.0;
    if (j > i)
      for (int s = 0; s < splits; ++s) v += part[(size_t)s * RR + f];
    dist[f] = v;
    dist[(size_t)j * R + i] = v;
  }
}

// ---- exact median of the squared distances over pairs i < j ----
// Non-negative doubles order like their bit patterns read as unsigned
// integers, so a most-significant-digit radix select on the bits is exact.
// Pass p (p = 0..7) histograms digit p (bits 56 - 8p and up) of the keys
// that match prefix[p] on the digits above; each of its blocks first
// derives prefix[p] and rank[p] from pass p-1's histogram, so no separate
// digit kernel runs between passes.  Both middle ranks travel together.
constexpr int kSelPasses = 8;

struct SelState {
  unsigned long long prefix[kSelPasses + 1][2];
  unsigned long long rank[kSelPasses + 1][2];
  unsigned int hist[kSelPasses][2][256];
  double sigma;
};

__global__ void __launch_bounds__(256) metric_sel_init_kernel(SelState* st, int R) {
  const unsigned long long C = (unsigned long long)R * (R - 1) / 2;
  if (threadIdx.x == 0) {
    st->prefix[0][0] = st->prefix[0][1] = 0ULL;
    st->rank[0][0] = (C % 2) ? (C - 1) / 2 : C / 2 - 1;
    st->rank[0][1] = (C % 2) ? (C - 1) / 2 : C / 2;
  }
  for (int p = 0; p < kSelPasses; ++p) {
    st->hist[p][0][threadIdx.x] = 0u;
    st->hist[p][1][threadIdx.x] = 0u;
  }
}

// Block-wide: digit of pass p-1 for both targets from its histogram, giving
// (prefix, rank) for pass p in pre[] / rk[] (LDS).  256 threads.
__device__ inline void sel_advance(const SelState* st, int p, unsigned long long* pre, unsigned long long* rk,
                                   unsigned int (*scan)[256]) {
  const int t = threadIdx.x;
  const int shift_prev = 56 - 8 * (p - 1);
  for (int g = 0; g < 2; ++g) scan[g][t] = st->hist[p - 1][g][t];
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {  // inclusive scan (Hillis-Steele)
    unsigned int v0 = 0u, v1 = 0u;
    if (t >= o) {
      v0 = scan[0][t - o];
      v1 = scan[1][t - o];
    }
    __syncthreads();
    scan[0][t] += v0;
    scan[1][t] += v1;
    __syncthreads();
  }
  for (int g = 0; g < 2; ++g) {
    const unsigned long long incl = scan[g][t];
    const unsigned long long excl = t ? scan[g][t - 1] : 0ULL;
    const unsigned long long r = st->rank[p - 1][g];
    if (r >= excl && r < incl) {
      pre[g] = st->prefix[p - 1][g] | ((unsigned long long)t << shift_prev);
      rk[g] = r - excl;
    }
  }
  __syncthreads();
}

// Pass p: histogram of digit p over the keys matching prefix[p] above it.
// Blocks walk rows i of the upper triangle (pairs j > i).
__global__ void __launch_bounds__(256) metric_sel_hist_kernel(const double* __restrict__ dist, int R, SelState* st,
                                                              int p) {
  __shared__ unsigned int h[2][256];
  __shared__ unsigned int scan[2][256];
  __shared__ unsigned long long pre[2], rk[2];
  if (p == 0) {
    if (threadIdx.x < 2) {
      pre[threadIdx.x] = st->prefix[0][threadIdx.x];
      rk[threadIdx.x] = st->rank[0][threadIdx.x];
    }
  } else {
    sel_advance(st, p, pre, rk, scan);
  }
  h[0][threadIdx.x] = 0u;
  h[1][threadIdx.x] = 0u;
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 2) {
    st->prefix[p][threadIdx.x] = pre[threadIdx.x];
    st->rank[p][threadIdx.x] = rk[threadIdx.x];
  }
  const int shift = 56 - 8 * p;
  const unsigned long long hi_mask = (p == 0) ? 0ULL : (~0ULL << (shift + 8));
  const unsigned long long p0 = pre[0] & hi_mask, p1 = pre[1] & hi_mask;
  for (int i = blockIdx.x; i < R - 1; i += gridDim.x) {
    const double* row = dist + (size_t)i * R;
    for (int j = i + 1 + threadIdx.x; j < R; j += 256) {
      const unsigned long long key = (unsigned long long)__double_as_longlong(row[j]);
      const unsigned int dg = (unsigned int)(key >> shift) & 255u;
      if ((key & hi_mask) == p0) atomicAdd(&h[0][dg], 1u);
      if ((key & hi_mask) == p1) atomicAdd(&h[1][dg], 1u);
    }
  }
  __syncthreads();
  for (int g = 0; g < 2; ++g)
    if (h[g][threadIdx.x]) atomicAdd(&st->hist[p][g][threadIdx.x], h[g][threadIdx.x]);
}

// Last digit, then sigma = median distance (mean of the two middle
// distances for an even pair count), 1 when that median is 0.
__global__ void __launch_bounds__(256) metric_sel_final_kernel(SelState* st, int R) {
  __shared__ unsigned int scan[2][256];
  __shared__ unsigned long long pre[2], rk[2];
  sel_advance(st, kSelPasses, pre, rk, scan);
  if (threadIdx.x == 0) {
    st->prefix[kSelPasses][0] = pre[0];
    st->prefix[kSelPasses][1] = pre[1];
    const unsigned long long C = (unsigned long long)R * (R - 1) / 2;
    const double a = sqrt(__longlong_as_double((long long)pre[0]));
    const double b = sqrt(__longlong_as_double((long long)pre[1]));
    double sg = (C % 2) ? a : 0.5 * (a + b);
    if (sg * sg < 1e-300) sg = 1.0;
    st->sigma = sg;
  }
}

// The caller's sigma.
__global__ void metric_sigma_given_kernel(SelState* st, double given) {
  if (threadIdx.x == 0) st->sigma = given;
}

__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// Keeps t[0..K) as the K smallest values seen, ascending (entries at and
// beyond K stay +inf).
__device__ inline void top_insert(double (&t)[kKMax], double v, int K) {
  if (!(v < t[K - 1])) return;
#pragma unroll
  for (int q = 0; q < kKMax; ++q)
    if (q == K - 1) t[q] = v;
#pragma unroll
  for (int q = kKMax - 1; q >= 1; --q) {
    if (q < K) {
      const double a = t[q - 1], b = t[q];
      t[q - 1] = fmin(a, b);
      t[q] = fmax(a, b);
    }
  }
}

// K-th smallest value over the wave's per-lane sorted lists.
__device__ inline double wave_kth(const double (&t)[kKMax], int K, int lane) {
  int pos = 0;
  double mn = INFINITY;
  for (int it = 0; it < K; ++it) {
    double v = INFINITY;
#pragma unroll
    for (int q = 0; q < kKMax; ++q)
      if (q == pos) v = t[q];
    mn = wave_min(v);
    const unsigned long long hit = __ballot(v == mn);
    if (lane == __ffsll((long long)hit) - 1) ++pos;
  }
  return mn;
}

// One wave per pooled row r: the k-th nearest squared distance in the other
// set and the l-th in the own set without r, and the Gaussian-kernel sums
// over both sets.  rows[r] = (d/2 (log nu_k^2 - log rho_l^2), own sum,
// other sum).
__global__ void __launch_bounds__(256) metric_rows_kernel(const double* __restrict__ dist, int n, int m, int d,
                                                          int k, int l, const SelState* __restrict__ st,
                                                          double* __restrict__ rows) {
  const int R = n + m;
  const int r = blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (r >= R) return;
  const int own0 = r < n ? 0 : n, own1 = r < n ? n : R;
  const double sg = st->sigma;
  const double g = 1.0 / (2.0 * sg * sg);
  double to[kKMax], tx[kKMax];
#pragma unroll
  for (int q = 0; q < kKMax; ++q) to[q] = tx[q] = INFINITY;
  double so = 0.0, sx = 0.0;
  const double* row = dist + (size_t)r * R;
  for (int j = lane; j < R; j += kWave) {
    if (j == r) continue;
    const double d2 = row[j];
    const double kv = exp(-d2 * g);
    if (j >= own0 && j < own1) {
      so += kv;
      top_insert(to, d2, l);
    } else {
      sx += kv;
      top_insert(tx, d2, k);
    }
  }
  so = wave_sum(so);
  sx = wave_sum(sx);
  const double nu2 = wave_kth(tx, k, lane);
  const double rho2 = wave_kth(to, l, lane);
  if (lane == 0) {
    rows[(size_t)r * 3 + 0] = 0.5 * (double)d * (log(nu2) - log(rho2));
    rows[(size_t)r * 3 + 1] = so;
    rows[(size_t)r * 3 + 2] = sx;
  }
}

// Fixed-order sums of the row terms into (KL(P||Q), KL(Q||P), MMD^2, sigma).
__global__ void __launch_bounds__(256) metric_final_kernel(const double* __restrict__ rows, int n, int m, int k,
                                                           int l, const SelState* __restrict__ st,
                                                           double* __restrict__ out) {
  __shared__ double red[5][256];
  const int R = n + m;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // S_P, S_Q, own P, own Q, cross from P
  const int per = (R + 255) / 256;
  const int r0 = threadIdx.x * per, r1 = min(R, r0 + per);
  for (int r = r0; r < r1; ++r) {
    const double* x = rows + (size_t)r * 3;
    if (r < n) {
      v[0] += x[0];
      v[2] += x[1];
      v[4] += x[2];
    } else {
      v[1] += x[0];
      v[3] += x[1];
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
#pragma unroll
      for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // psi(l) - psi(k) = H_{l-1} - H_{k-1}
    double dpsi = 0.0;
    for (int j = 1; j < l; ++j) dpsi += 1.0 / j;
    for (int j = 1; j < k; ++j) dpsi -= 1.0 / j;
    const double dn = n, dm = m;
    out[0] = red[0][0] / dn + dpsi + log(dm / (dn - 1.0));
    out[1] = red[1][0] / dm + dpsi + log(dn / (dm - 1.0));
    out[2] = red[2][0] / (dn * (dn - 1.0)) + red[3][0] / (dm * (dm - 1.0)) - 2.0 * red[4][0] / (dn * dm);
    out[3] = st->sigma;
  }
}

}  // namespace

MetricsPlan metrics_plan(int n, int m, int d) {
  MetricsPlan p;
  p.R = n + m;
  const int T = (p.R + kMT - 1) / kMT;
  p.tiles = T * (T + 1) / 2;
  const int chunks = (d + kMC - 1) / kMC;
  int s = (1024 + p.tiles - 1) / p.tiles;
  if (s > chunks) s = chunks;
  if (s > 8) s = 8;
  p.splits = s < 1 ? 1 : s;
  const size_t RR = (size_t)p.R * p.R;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  p.off_dist = take(RR * sizeof(double));
  p.off_part = p.splits > 1 ? take((size_t)p.splits * RR * sizeof(double)) : 0;
  p.off_rows = take((size_t)p.R * 3 * sizeof(double));
  p.off_sel = take(sizeof(SelState));
  p.bytes = off;
  return p;
}

hipError_t launch_metric_dist(const MetricsPlan& p, const float* P, const float* Q, int n, int m, int d,
                              const float* w, char* ws, hipStream_t s) {
  double* dist = reinterpret_cast<double*>(ws + p.off_dist);
  double* part = p.splits > 1 ? reinterpret_cast<double*>(ws + p.off_part) : nullptr;
  if (w)
    hipLaunchKernelGGL(metric_dist_kernel<true>, dim3(p.tiles, p.splits), dim3(256), 0, s, P, Q, n, m, d, w, dist,
                       part, p.splits);
  else
    hipLaunchKernelGGL(metric_dist_kernel<false>, dim3(p.tiles, p.splits), dim3(256), 0, s, P, Q, n, m, d, w, dist,
                       part, p.splits);
  if (p.splits > 1) {
    const size_t RR = (size_t)p.R * p.R;
    const int grid = (int)std::min<size_t>((RR + 255) / 256, 4096);
    hipLaunchKernelGGL(metric_dist_reduce_kernel, dim3(grid), dim3(256), 0, s, part, p.R, p.splits, dist);
  }
  return hipGetLastError();
}

hipError_t launch_metric_rest(const MetricsPlan& p, int n, int m, int d, int k, int l, double sigma, double* out,
                              double* rows_out, char* ws, hipStream_t s) {
  const double* dist = reinterpret_cast<const double*>(ws + p.off_dist);
  double* rows = rows_out ? rows_out : reinterpret_cast<double*>(ws + p.off_rows);
  SelState* st = reinterpret_cast<SelState*>(ws + p.off_sel);
  const int R = p.R;
  if (!(sigma > 0.0)) {
    const int grid = std::min(R - 1, 512);
    hipLaunchKernelGGL(metric_sel_init_kernel, dim3(1), dim3(256), 0, s, st, R);
    for (int p = 0; p < kSelPasses; ++p)
      hipLaunchKernelGGL(metric_sel_hist_kernel, dim3(grid), dim3(256), 0, s, dist, R, st, p);
    hipLaunchKernelGGL(metric_sel_final_kernel, dim3(1), dim3(256), 0, s, st, R);
  } else {
    hipLaunchKernelGGL(metric_sigma_given_kernel, dim3(1), dim3(64), 0, s, st, sigma);
  }
  hipLaunchKernelGGL(metric_rows_kernel, dim3((R + 3) / 4), dim3(256), 0, s, dist, n, m, d, k, l, st, rows);
  hipLaunchKernelGGL(metric_final_kernel, dim3(1), dim3(256), 0, s, rows, n, m, k, l, st, out);
  return hipGetLastError();
}

}  // namespace pds
