// SVGD direction (eq. svgd_update) with the median-heuristic RBF kernel
// (Sec. III-A) and the MDMM parameter update (Sec. III-E, Algorithm 1).
//
// Bandwidth.  h = med^2 / log N with med the exact median of the N (N-1)/2
// pair distances ||(theta_i - theta_j) / rho||, computed in FP64 from the
// FP32 particles.  A non-negative IEEE double orders like its bit pattern
// read as uint64, so selection works on the 64-bit patterns ("keys") of
// the squared distances, and both middle order statistics ((P-1)/2 and P/2
// of P pairs) are found together.  Kernels:
//  * keys: up to kSmallPairs pairs, every pair's key (high and low words);
//    above, the high words of a fixed pseudo-random sample of kSampleKeys
//    pairs.
//  * select: one block per job, the high words in registers.  A histogram
//    of 2^11 bins over [min, max] narrows both middle ranks; the keys of
//    the two bins are then ranked by direct counting (further levels when
//    the bins hold more than kDirectMax keys).  Small jobs get the exact
//    median; larger ones a bracket [a, b] on the sample's order statistics
//    widened by four binomial standard deviations.
//  * count (larger jobs): every pair once, 64 x 64 pairs per block; keys
//    below a are counted and keys inside [a, b] appended to a candidate
//    array, both with one atomic add per block.
//  * final (larger jobs): one block selects exactly among the candidates,
//    or, if the bracket missed a middle rank, among all keys of the side
//    that holds it.
// Counts are integers, so the result does not depend on the order in which
// blocks finish.
//
// Failed particles.  Particles with flag bit 3 are out of the median's
// ensemble: a pair with such an endpoint gets the key kMaskedKey, above
// every key of a non-negative double, so the ensemble's keys keep their
// ranks from the bottom, and the targets are the middle ranks of the
// ensemble's P' = N' (N' - 1) / 2 pairs.  Count kernels skip such pairs.
// phi leaves out particles with flag bit 0, 1 or 3: each chunk of rows is
// compacted to its live particles before the sums, and the sums are
// divided by their number.
//
// phi.  Up to kPhiFusedMaxN particles: one block per 16 particles i (4
// above 128 particles) with every particle's row in LDS and 1024 / 16 (or
// 1024 / 4) slices of the j range.  Larger jobs: blocks of 64 particles i against
// chunks of 32 particles j (enough blocks to fill the chip), then a
// reduction over chunks.  Both accumulate in FP32 in a fixed order.
#include <cmath>

#include <mutex>

#include "common.h"

namespace pds {
namespace {

constexpr int kPairBlock = 64;  // particles i per block

__device__ inline MedianState* med_state(const pds_job& J, char* ws, uint64_t off) {
  const WsLayout L = ws_layout(J);
  return reinterpret_cast<MedianState*>(ws + off + L.med);
}

// Flag bits that take a particle out of phi and freeze it in the step.
constexpr int kOutOfEnsemble = PDS_FLAG_STATE | PDS_FLAG_GRAD | PDS_FLAG_FROZEN;
// Key of a pair with a frozen endpoint (its sign bit set: above every key).
constexpr uint64_t kMaskedKey = ~0ull;

// Whether particle i is out of the median's ensemble (flag bit 3).  An
// atomic load: a concurrent adjoint may OR bits 0 and 1 into the same
// word; bit 3 changes only in the step kernel.
__device__ inline bool frozen_particle(const pds_job& J, int i) {
  return J.flags && (__hip_atomic_load(J.flags + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & PDS_FLAG_FROZEN);
}

// Whether particle i takes part in phi (no flag bit 0, 1 or 3).
__device__ inline bool in_phi(const pds_job& J, int i) { return !J.flags || (J.flags[i] & kOutOfEnsemble) == 0; }

// Size N' of the median's ensemble, counted by a block of NT threads into
// *s (every thread returns it).  Contains two block barriers.
template <int NT>
__device__ inline uint32_t ensemble_size(const pds_job& J, uint32_t* s) {
  uint32_t c = 0;
  for (int i = threadIdx.x; i < J.N; i += NT) c += frozen_particle(J, i) ? 0u : 1u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (threadIdx.x == 0) *s = 0u;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) atomicAdd(s, c);
  __syncthreads();
  return *s;
}

// Squared scaled distance in FP64, summed in parameter order.  MM is a
// compile-time bound on M; the rows and inv_rho are zero beyond M, so the
// padded terms add +0 to a non-negative sum and the loop needs no
// per-parameter branch (a branch per term would serialise the LDS reads).
// Every kernel that forms keys calls this with the smaller particle index
// first, so a pair's key is the same bit pattern wherever it is computed.
template <int MM>
__device__ inline double pair_d2(const float* ti, const float* tj, const double* inv_rho, int M) {
  (void)M;
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    const double z = ((double)ti[m] - (double)tj[m]) * inv_rho[m];
    s = __dadd_rn(s, __dmul_rn(z, z));
  }
  return s;
}

__device__ inline uint64_t key_of(double d2) { return (uint64_t)__double_as_longlong(d2); }

// Loads v[0..M) into out[0..MM), zero beyond M.  Every load is issued
// unconditionally at an in-bounds index (clamped to M - 1) and the padding
// is a select, so the loads need no branches and one wait.
template <int MM>
__device__ inline void load_padded(const float* v, int M, float* out) {
  float t[MM];
#pragma unroll
  for (int m = 0; m < MM; ++m) t[m] = v[m < M ? m : M - 1];
#pragma unroll
  for (int m = 0; m < MM; ++m) out[m] = m < M ? t[m] : 0.f;
}

// 1 / rho in FP64, zero beyond M.
template <int MM>
__device__ inline void load_inv_rho(const pds_job& J, double* inv_rho) {
  float r[MM];
  load_padded<MM>(J.rho, J.M, r);
#pragma unroll
  for (int m = 0; m < MM; ++m) inv_rho[m] = m < J.M ? 1.0 / (double)r[m] : 0.0;
}

template <int MM>
__device__ inline void load_row(const pds_job& J, int i, float* t) {
  load_padded<MM>(J.theta + (size_t)i * J.M, J.M, t);
}

template <int MM>
__device__ inline uint64_t pair_key(const pds_job& J, int i, int j, const double* inv_rho) {
  float ti[MM], tj[MM];
  load_row<MM>(J, i, ti);
  load_row<MM>(J, j, tj);
  return key_of(pair_d2<MM>(ti, tj, inv_rho, J.M));
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

__device__ inline int bit_len(uint32_t x) { return x ? 32 - __clz((int)x) : 0; }
__device__ inline int bit_len(uint64_t x) { return x ? 64 - __clzll((long long)x) : 0; }

// ---------------------------------------------------------------------------
// Block-wide exact selection of two ranks among unsigned keys (32- or
// 64-bit).  A target is a key interval [lo, hi] known to hold the wanted
// key and that key's rank among the current keys inside the interval.
// ---------------------------------------------------------------------------

template <class KT>
struct SelTarget {
  KT lo, hi;
  uint32_t t;
};

template <class KT>
struct SelShared {
  SelTarget<KT> tg[2];
  uint32_t cnt[2];  // keys inside each target's interval after a level
  uint32_t hist[2][kSelBins];
  uint32_t wsum[16];
  KT red[2][16];
};

// Exclusive prefix of v over the block's threads and the block total.
template <int NT, class SS>
__device__ inline uint32_t block_scan(uint32_t v, SS& S, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_scan(v);
  if (lane == 63) S.wsum[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const uint32_t s = S.wsum[k];
    base += k < w ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

template <int NT, class KT>
__device__ inline void block_minmax(KT mn, KT mx, SelShared<KT>& S, KT* out_min, KT* out_max) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const KT a = (KT)__shfl_xor((unsigned long long)mn, o);
    const KT b = (KT)__shfl_xor((unsigned long long)mx, o);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    S.red[0][w] = mn;
    S.red[1][w] = mx;
  }
  __syncthreads();
  mn = S.red[0][0];
  mx = S.red[1][0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) {
    mn = S.red[0][k] < mn ? S.red[0][k] : mn;
    mx = S.red[1][k] > mx ? S.red[1][k] : mx;
  }
  __syncthreads();
  *out_min = mn;
  *out_max = mx;
}

// Bins of one level: (key - lo) >> sh, with sh the smallest shift that puts
// [lo, hi] into kSelBins = 2^11 bins.
template <class KT>
__device__ inline int sel_shift(KT span) {
  const int bits = bit_len(span);
  return bits > 11 ? bits - 11 : 0;
}

// Both targets count into hist[0] while their intervals coincide.
template <class KT>
__device__ inline bool sel_shared(const SelTarget<KT>* t, const bool* live) {
  return live[0] && live[1] && t[0].lo == t[1].lo && t[0].hi == t[1].hi;
}

template <int NT, class KT>
__device__ void sel_histogram(const KT* src, uint32_t n, SelShared<KT>& S, const SelTarget<KT>* t, const bool* live,
                              const int* sh) {
  for (int i = threadIdx.x; i < 2 * kSelBins; i += NT) (&S.hist[0][0])[i] = 0u;
  __syncthreads();
  const bool share = sel_shared(t, live);
  const bool use1 = live[1] && !share;
  constexpr int U = 16;  // loads in flight per thread
  for (uint32_t c0 = 0; c0 < n; c0 += NT * U) {
    KT key[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {  // in-bounds index for every lane: no branch per load
      const uint32_t c = c0 + u * NT + threadIdx.x;
      key[u] = src[c < n ? c : n - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = c0 + u * NT + threadIdx.x < n;
      if (ok && live[0] && key[u] >= t[0].lo && key[u] <= t[0].hi)
        atomicAdd(&S.hist[0][(uint32_t)((key[u] - t[0].lo) >> sh[0])], 1u);
      if (ok && use1 && key[u] >= t[1].lo && key[u] <= t[1].hi)
        atomicAdd(&S.hist[1][(uint32_t)((key[u] - t[1].lo) >> sh[1])], 1u);
    }
  }
  __syncthreads();
}

// Narrows target k to the bin holding its rank: the thread whose bins
// contain the rank rewrites the target.
template <int NT, class KT>
__device__ void sel_narrow(SelShared<KT>& S, int k, int hk, const SelTarget<KT> t, int sh) {
  constexpr int BPT = kSelBins / NT;
  const int b0 = threadIdx.x * BPT;
  uint32_t c[BPT];
  uint32_t local = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    c[q] = S.hist[hk][b0 + q];
    local += c[q];
  }
  uint32_t total;
  const uint32_t base = block_scan<NT>(local, S, &total);
  if (base <= t.t && t.t < base + local) {
    uint32_t r = t.t - base;
    int b = -1;
    uint32_t cb = 0;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      if (b < 0) {
        if (r < c[q]) {
          b = b0 + q;
          cb = c[q];
        } else {
          r -= c[q];
        }
      }
    }
    const KT span = t.hi - t.lo;
    S.tg[k].lo = t.lo + ((KT)b << sh);
    S.tg[k].hi = (KT)b == (KT)(span >> sh) ? t.hi : (KT)(t.lo + (((KT)b + 1) << sh) - 1);
    S.tg[k].t = r;
    S.cnt[k] = cb;
  }
  __syncthreads();
}

// Copies the keys inside either live target's interval from src to dst
// (LDS, at most cap keys), in block-scan order.  Returns their number.
template <int NT, class KT>
__device__ uint32_t sel_compact(const KT* src, uint32_t n, KT* dst, uint32_t cap, SelShared<KT>& S) {
  const SelTarget<KT> t0 = S.tg[0], t1 = S.tg[1];
  const bool l0 = t0.lo != t0.hi, l1 = t1.lo != t1.hi;
  constexpr int U = 16;  // loads in flight per thread
  uint32_t base = 0;
  for (uint32_t c0 = 0; c0 < n; c0 += NT * U) {
    KT key[U];
    bool keep[U];
    uint32_t cnt = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t c = c0 + u * NT + threadIdx.x;
      key[u] = src[c < n ? c : n - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t c = c0 + u * NT + threadIdx.x;
      keep[u] = c < n && ((l0 && key[u] >= t0.lo && key[u] <= t0.hi) || (l1 && key[u] >= t1.lo && key[u] <= t1.hi));
      cnt += keep[u] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t o = base + block_scan<NT>(cnt, S, &total);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (keep[u]) {
        if (o < cap) dst[o] = key[u];
        ++o;
      }
    base += total;
  }
  __syncthreads();
  return base < cap ? base : cap;
}

// Direct finish for n <= NT keys in LDS: the thread holding a key inside
// a live target's interval counts the keys of that interval below it
// (equal keys ordered by position); the one whose count is the target's
// rank holds the answer.  Ends with a barrier.
template <int NT, class KT, class SS>
__device__ void sel_count_finish(const KT* src, uint32_t n, SS& S) {
  const SelTarget<KT> t0 = S.tg[0], t1 = S.tg[1];
  const bool l0 = t0.lo != t0.hi, l1 = t1.lo != t1.hi;
  __syncthreads();
  const uint32_t c = threadIdx.x;
  const KT x = n > 0 ? src[c < n ? c : n - 1] : (KT)0;
  const bool in0 = c < n && l0 && x >= t0.lo && x <= t0.hi;
  const bool in1 = c < n && l1 && x >= t1.lo && x <= t1.hi;
  uint32_t r0 = 0, r1 = 0;
  constexpr int U = 8;  // keys read per batch (one wait per batch)
  // only threads holding a key count (waves past n skip the loop)
  for (uint32_t q0 = 0; c < n && q0 < n; q0 += U) {
    KT y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) y[u] = src[q0 + u < n ? q0 + u : n - 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t q = q0 + u;
      const bool before = q < n && (y[u] < x || (y[u] == x && q < c));
      r0 += (before && y[u] >= t0.lo && y[u] <= t0.hi) ? 1u : 0u;
      r1 += (before && y[u] >= t1.lo && y[u] <= t1.hi) ? 1u : 0u;
    }
  }
  if (in0 && r0 == t0.t) S.tg[0] = SelTarget<KT>{x, x, 0u};
  if (in1 && r1 == t1.t) S.tg[1] = SelTarget<KT>{x, x, 0u};
  __syncthreads();
}

// Direct finish with g = min(64, NT / 2^ceil(log2 n)) consecutive threads
// per key, each counting over its share of the n keys; the shares are
// summed across the g lanes.  Same ranks and result as sel_count_finish.
template <int NT, class KT, class SS>
__device__ void sel_count_finish_split(const KT* src, uint32_t n, SS& S) {
  __syncthreads();
  const SelTarget<KT> t0 = S.tg[0], t1 = S.tg[1];
  const bool l0 = t0.lo != t0.hi, l1 = t1.lo != t1.hi;
  uint32_t np2 = 1;
  while (np2 < n) np2 <<= 1;
  const uint32_t g = NT / np2 < 64 ? NT / np2 : 64;  // n <= NT, so g >= 1
  const uint32_t c = threadIdx.x / g, part = threadIdx.x % g;
  const uint32_t per = (n + g - 1) / g;
  const uint32_t q0 = part * per, q1 = q0 + per < n ? q0 + per : n;
  const KT x = n > 0 ? src[c < n ? c : n - 1] : (KT)0;
  uint32_t r0 = 0, r1 = 0;
  constexpr int U = 8;
  for (uint32_t qb = q0; c < n && qb < q1; qb += U) {
    KT y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) y[u] = src[qb + u < q1 ? qb + u : q1 - 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t q = qb + u;
      const bool before = q < q1 && (y[u] < x || (y[u] == x && q < c));
      r0 += (before && y[u] >= t0.lo && y[u] <= t0.hi) ? 1u : 0u;
      r1 += (before && y[u] >= t1.lo && y[u] <= t1.hi) ? 1u : 0u;
    }
  }
  for (uint32_t o = 1; o < g; o <<= 1) {
    r0 += __shfl_xor(r0, (int)o);
    r1 += __shfl_xor(r1, (int)o);
  }
  if (part == 0 && c < n) {
    if (l0 && x >= t0.lo && x <= t0.hi && r0 == t0.t) S.tg[0] = SelTarget<KT>{x, x, 0u};
    if (l1 && x >= t1.lo && x <= t1.hi && r1 == t1.t) S.tg[1] = SelTarget<KT>{x, x, 0u};
  }
  __syncthreads();
}

// Two targets alone (the state of a direct finish).
template <class KT>
struct SelPair {
  SelTarget<KT> tg[2];
};

// Exact keys of both targets among the n keys src[0..n).  Each level
// histograms the keys inside a live target's interval into 2^11 bins and
// keeps the bin holding the rank, so an interval of b-bit span shrinks to
// one below 2^(b-11): 32-bit keys need at most 3 levels, 64-bit keys 6.
// Keys held in global memory move to `lds` as soon as the keys inside the
// live intervals fit there; at most NT keys in LDS are finished by direct
// counting.  On return S.tg[k].lo is the key; S.tg[k].t is its rank among
// the keys equal to it only when the levels resolved it.
template <int NT, class KT>
__device__ void select_keys(const KT* src, uint32_t n, bool src_global, KT* lds, uint32_t lds_cap,
                            SelShared<KT>& S, KT out[2], bool count_finish = true) {
  for (int level = 0; level < kMaxLevels; ++level) {
    SelTarget<KT> t[2] = {S.tg[0], S.tg[1]};
    bool live[2];
    int sh[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      live[k] = t[k].lo != t[k].hi;
      sh[k] = sel_shift<KT>(t[k].hi - t[k].lo);
    }
    if (!live[0] && !live[1]) break;
    if (count_finish && !src_global && n <= (uint32_t)NT) {
      sel_count_finish<NT>(src, n, S);
      break;
    }
    const bool share = sel_shared(t, live);
    sel_histogram<NT>(src, n, S, t, live, sh);
    if (live[0]) sel_narrow<NT>(S, 0, 0, t[0], sh[0]);
    if (live[1]) sel_narrow<NT>(S, 1, share ? 0 : 1, t[1], sh[1]);
    if (src_global) {
      uint64_t need = 0;
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (S.tg[k].lo != S.tg[k].hi) need += S.cnt[k];
      if (need == 0) break;
      if (need <= lds_cap) {
        n = sel_compact<NT>(src, n, lds, lds_cap, S);
        src = lds;
        src_global = false;
      }
    }
  }
  out[0] = S.tg[0].lo;
  out[1] = S.tg[1].lo;
}

// h = med^2 / log N' from the two middle keys of an ensemble of nb
// particles (h = 1 when it has no pair).
__device__ inline void write_bandwidth(const pds_job& J, uint64_t k0, uint64_t k1, uint32_t nb) {
  double h = 1.0;
  if (nb > 1) {
    const double a = __longlong_as_double((long long)k0);
    const double c = __longlong_as_double((long long)k1);
    const double med = 0.5 * (sqrt(a) + sqrt(c));
    const double lg = log((double)nb);
    if (med * med >= 1e-300 && lg > 0.0) h = med * med / lg;
  }
  J.bandwidth[0] = h;
}

// Row i and column j of pair p in the row-major enumeration of pairs i < j.
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

// Tile (bi, bj), bi <= bj, of tile t in the row-major enumeration of the
// upper triangle (diagonal included) of an nb x nb tile grid.
__device__ inline void tile_of(int t, int nb, int* pbi, int* pbj) {
  const double b = 2.0 * nb + 1.0;
  int r = (int)floor((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  auto off = [nb](long long q) -> long long { return q * nb - q * (q - 1) / 2; };
  if (r < 0) r = 0;
  if (r > nb - 1) r = nb - 1;
  while (r > 0 && off(r) > t) --r;
  while (r < nb - 1 && off(r + 1) <= t) ++r;
  *pbi = r;
  *pbj = (int)(t - off(r)) + r;
}

// Sample position k: a fixed 64-bit mix of k scaled onto [0, P).
__device__ inline uint64_t sample_pair(uint64_t k, uint64_t P) {
  uint64_t z = k * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return __umul64hi(z, P);
}

// Keys kernel, one pair per thread (256-thread blocks, or one-wave blocks
// for the narrow median below).  Jobs with at most kSmallPairs pairs:
// every pair's key, split into high and low 32-bit words.  Larger jobs:
// the high words of a fixed pseudo-random sample of kSampleKeys keys; their
// first block also clears the count kernel's counter.
template <int MM>
__global__ void __launch_bounds__(256) median_keys_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                          char* __restrict__ ws) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const uint64_t P = (uint64_t)J.N * (J.N - 1) / 2;
  const bool small = P <= (uint64_t)kSmallPairs;
  const uint32_t k = (uint32_t)(blockIdx.x - map.begin[e]) * blockDim.x + threadIdx.x;
  const WsLayout L = ws_layout(J);
  char* base = ws + map.ws_off[e];
  if (!small && k == 0) med_state(J, ws, map.ws_off[e])->packed = 0ull;
  if (small && k >= P) return;
  double inv_rho[MM];
  load_inv_rho<MM>(J, inv_rho);
  int i, j;
  pair_of(small ? (uint64_t)k : sample_pair(k, P), J.N, &i, &j);
  const uint64_t key =
      (frozen_particle(J, i) || frozen_particle(J, j)) ? kMaskedKey : pair_key<MM>(J, i, j, inv_rho);
  reinterpret_cast<uint32_t*>(base + L.khi)[k] = (uint32_t)(key >> 32);
  if (small) reinterpret_cast<uint32_t*>(base + L.klo)[k] = (uint32_t)key;
}

// More than kDirectMax keys in the middle bins of the first level (heavy
// ties): further levels over the high words in global memory (moved to the
// LDS buffer lbuf once the live keys fit), then, for small jobs, over the
// low words of the keys whose high word is a selected one, compacted into
// the job's list region.  Out of line, so its registers stay out of the
// common path.
template <int NT>
__device__ __attribute__((noinline)) void select_rest(const pds_job& J, char* ws, uint64_t ws_off, uint32_t* lbuf,
                                                      SelShared<uint32_t>& S, const uint32_t* khi,
                                                      const uint32_t* klo, uint32_t* lists, uint32_t n, bool small,
                                                      bool a_open, bool b_open, uint32_t nb) {
  uint32_t hsel[2];
  select_keys<NT>(khi, n, true, lbuf, (uint32_t)kSelLdsCap, S, hsel, false);
  if (!small) {
    if (threadIdx.x == 0) {
      MedianState* st = med_state(J, ws, ws_off);
      st->a = a_open ? 0ull : (uint64_t)hsel[0] << 32;
      st->b = b_open ? ~0ull : (((uint64_t)hsel[1] << 32) | 0xffffffffull);
    }
    return;
  }
  const uint32_t rk0 = S.tg[0].t, rk1 = S.tg[1].t;
  const bool same = hsel[0] == hsel[1];
  // Low words of the keys whose high word is a selected one: list A for
  // hsel[0], then list B for hsel[1] when it differs.
  uint32_t cA = 0u, cB = 0u;
  for (uint32_t c = threadIdx.x; c < n; c += NT) {
    const uint32_t h = khi[c];
    cA += h == hsel[0] ? 1u : 0u;
    cB += (!same && h == hsel[1]) ? 1u : 0u;
  }
  uint32_t nA, nB;
  uint32_t oA = block_scan<NT>(cA, S, &nA);
  uint32_t oB = nA + block_scan<NT>(cB, S, &nB);
  for (uint32_t c = threadIdx.x; c < n; c += NT) {
    const uint32_t h = khi[c];
    if (h == hsel[0]) lists[oA++] = klo[c];
    else if (!same && h == hsel[1]) lists[oB++] = klo[c];
  }
  if (threadIdx.x == 0) {
    S.tg[0] = SelTarget<uint32_t>{0u, ~0u, rk0};
    S.tg[1] = same ? SelTarget<uint32_t>{0u, ~0u, rk1} : SelTarget<uint32_t>{0u, 0u, 0u};
  }
  __syncthreads();  // the lists are complete and visible to the block
  uint32_t lsel[2], tmp[2];
  select_keys<NT>(lists, nA, true, lbuf, (uint32_t)kSelLdsCap, S, lsel);
  if (!same) {
    __syncthreads();
    if (threadIdx.x == 0) {
      S.tg[0] = SelTarget<uint32_t>{0u, 0u, 0u};
      S.tg[1] = SelTarget<uint32_t>{0u, ~0u, rk1};
    }
    __syncthreads();
    select_keys<NT>(lists + nA, nB, true, lbuf, (uint32_t)kSelLdsCap, S, tmp);
    lsel[1] = tmp[1];
  }
  if (threadIdx.x == 0)
    write_bandwidth(J, ((uint64_t)hsel[0] << 32) | lsel[0], ((uint64_t)hsel[1] << 32) | lsel[1], nb);
}

// Select kernel, one block per job.  Loads the high words written by the
// keys kernel into registers and selects two ranks among them: the middle
// ranks of the ensemble's pairs for small jobs, which then finish on the
// low words of the keys sharing the selected high words; for larger jobs
// the sample's order statistics at the middle ranks' sample positions
// widened by four binomial standard deviations, stored as the bracket
// [a, b] (whole high words) for the count kernel.  Masked keys (high word
// kNoKey) take part in no range or count.
__global__ void __launch_bounds__(kMedThreads, kSelWavesPerSimd) median_select_kernel(
    JobMap map, const pds_job* __restrict__ jobs, char* __restrict__ ws, int rank_shift) {
  __shared__ uint32_t lbuf[kSelLdsCap];  // used by select_rest only
  __shared__ SelShared<uint32_t> S;
  __shared__ uint64_t cand[kDirectMax];
  __shared__ uint32_t cidx[kDirectMax];
  __shared__ SelPair<uint64_t> P64;
  __shared__ uint32_t s_lo, s_hi, s_cnt, s_nb, s_nv;
  constexpr int NT = kMedThreads;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const uint64_t P = (uint64_t)J.N * (J.N - 1) / 2;
  if (P == 0) {
    if (threadIdx.x == 0) write_bandwidth(J, 0ull, 0ull, 1u);
    return;
  }
  const bool small = P <= (uint64_t)kSmallPairs;
  const uint32_t n = small ? (uint32_t)P : (uint32_t)kSampleKeys;
  const WsLayout L = ws_layout(J);
  char* base = ws + map.ws_off[e];
  const uint32_t* khi = reinterpret_cast<const uint32_t*>(base + L.khi);
  const uint32_t* klo = reinterpret_cast<const uint32_t*>(base + L.klo);
  // Every key's high word in registers: thread element k = 4 v + c is key
  // 4 (v NT + thread) + c, loaded 16 bytes at a time, all loads in flight
  // together (the last vector may extend past n into the region's 256-byte
  // padding).  Elements past n hold kNoKey, above every key's high word
  // (the sign bit is clear), so each later test is a compare on the value
  // itself, made where it is used.
  constexpr int V = kSmallPairs / (4 * NT);
  constexpr uint32_t kNoKey = 0xffffffffu;
  static_assert(kSampleKeys <= kSmallPairs, "register layout holds the sample");
  static_assert(kSelBins == 2 * NT, "two histogram bins per thread");
  uint32_t hv[4 * V];
  const uint32_t n4 = (n + 3) / 4;
  uint4 q[V];
  {
    const uint4* k4 = reinterpret_cast<const uint4*>(khi);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint32_t idx = v * NT + threadIdx.x;
      q[v] = k4[idx < n4 ? idx : n4 - 1];
    }
  }
  auto key_at = [&](int k) { return 4u * ((k >> 2) * NT + threadIdx.x) + (k & 3); };
  // while the loads are in flight: the ensemble's particles, and clear the
  // histogram and the block's min / max / key counts
  uint32_t nbl = 0u;
  for (int i = threadIdx.x; i < J.N; i += NT) nbl += frozen_particle(J, i) ? 0u : 1u;
  for (int b = threadIdx.x; b < kSelBins; b += NT) S.hist[0][b] = 0u;
  if (threadIdx.x == 0) {
    s_lo = kNoKey;
    s_hi = 0u;
    s_cnt = 0u;
    s_nb = 0u;
    s_nv = 0u;
  }
  __syncthreads();
  uint32_t mn = kNoKey, mx = 0u, nvl = 0u;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t w4[4] = {q[v].x, q[v].y, q[v].z, q[v].w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t h = key_at(4 * v + c) < n ? w4[c] : kNoKey;
      hv[4 * v + c] = h;
      mn = h < mn ? h : mn;
      mx = (h != kNoKey && h > mx) ? h : mx;
      nvl += h != kNoKey ? 1u : 0u;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t a = (uint32_t)__shfl_xor((int)mn, o), b = (uint32_t)__shfl_xor((int)mx, o);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    nvl += (uint32_t)__shfl_xor((int)nvl, o);
    nbl += (uint32_t)__shfl_xor((int)nbl, o);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s_lo, mn);
    atomicMax(&s_hi, mx);
    atomicAdd(&s_nv, nvl);
    atomicAdd(&s_nb, nbl);
  }
  __syncthreads();
  const uint32_t lo = s_lo, hi = s_hi;
  const uint32_t nb = s_nb, nv = s_nv;  // ensemble particles, unmasked keys in registers
  const uint64_t Pe = (uint64_t)nb * (nb - 1) / 2;
  if (Pe == 0 || nv == 0) {
    // no pair in the ensemble (h = 1), or none in the sample: then the
    // bracket is every key and the count kernel collects the ensemble's
    if (threadIdx.x == 0) {
      if (small || Pe == 0) {
        write_bandwidth(J, 0ull, 0ull, nb);
      } else {
        MedianState* st = med_state(J, ws, map.ws_off[e]);
        st->a = 0ull;
        st->b = ~0ull;
      }
    }
    return;
  }
  uint32_t t0, t1;
  bool a_open = false, b_open = false;
  if (small) {
    t0 = (uint32_t)((Pe - 1) / 2);
    t1 = (uint32_t)(Pe / 2);
  } else {
    // sample positions of the ensemble's middle ranks: masked keys sort
    // above them, so the first nv sample positions hold the ensemble's keys
    const double d = 2.0 * sqrt((double)n) + 2.0;
    const double c0 = (double)n * (double)((Pe - 1) / 2) / (double)P - d + rank_shift;
    const double c1 = (double)n * (double)(Pe / 2 + 1) / (double)P + d + rank_shift;
    a_open = c0 < 0.0 || c0 > (double)(nv - 1);
    b_open = c1 > (double)(nv - 1);
    t0 = a_open ? 0u : (uint32_t)floor(c0);
    t1 = b_open ? nv - 1 : (uint32_t)fmax(ceil(c1), 0.0);
  }
  // First level over the keys' own range [lo, hi]: one histogram for both
  // targets and one block scan over it narrows both.
  if (lo != hi) {
    const uint32_t span = hi - lo;
    const int sh = sel_shift<uint32_t>(span);
#pragma unroll
    for (int k = 0; k < 4 * V; ++k) {
      const uint32_t d = hv[k] - lo;
      if (d <= span) atomicAdd(&S.hist[0][d >> sh], 1u);
    }
    __syncthreads();
    const int b0 = 2 * threadIdx.x;
    const uint32_t c0 = S.hist[0][b0], c1 = S.hist[0][b0 + 1];
    const uint32_t local = c0 + c1;
    const uint32_t inc = wave_scan(local);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) S.wsum[w] = inc;
    __syncthreads();
    uint32_t below = inc - local;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) below += k < w ? S.wsum[k] : 0u;
    const uint32_t tt[2] = {t0, t1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (below <= tt[k] && tt[k] < below + local) {
        const bool first = tt[k] - below < c0;
        const uint32_t b = first ? b0 : b0 + 1;
        S.tg[k].lo = lo + (b << sh);
        S.tg[k].hi = b == (span >> sh) ? hi : lo + ((b + 1) << sh) - 1;
        S.tg[k].t = first ? tt[k] - below : tt[k] - below - c0;
        S.cnt[k] = first ? c0 : c1;
      }
    }
  } else if (threadIdx.x == 0) {
    S.tg[0] = SelTarget<uint32_t>{lo, hi, t0};
    S.tg[1] = SelTarget<uint32_t>{lo, hi, t1};
  }
  __syncthreads();
  const SelTarget<uint32_t> g0 = S.tg[0], g1 = S.tg[1];
  const bool same_bin = g0.lo == g1.lo && g0.hi == g1.hi;
  const uint32_t need = lo == hi ? nv : (same_bin ? S.cnt[0] : S.cnt[0] + S.cnt[1]);
  if (need <= (uint32_t)kDirectMax) {
    // Direct finish: the indices of the keys in the two bins go to cidx
    // (order immaterial: the ranking below orders by value, then by
    // position), their full 64-bit keys are fetched with one pair of loads
    // per thread, and the two ranks are found by counting.
    uint32_t mask = 0u;
#pragma unroll
    for (int k = 0; k < 4 * V; ++k) {
      const uint32_t h = hv[k];
      const bool in = h - g0.lo <= g0.hi - g0.lo || h - g1.lo <= g1.hi - g1.lo;  // kNoKey is in neither
      mask |= (in ? 1u : 0u) << k;
    }
    if (mask) {
      uint32_t o = atomicAdd(&s_cnt, (uint32_t)__popc(mask));
#pragma unroll
      for (int k = 0; k < 4 * V; ++k)
        if ((mask >> k) & 1u) cidx[o++] = key_at(k);
    }
    if (threadIdx.x == 0) {
      P64.tg[0] = SelTarget<uint64_t>{(uint64_t)g0.lo << 32, ((uint64_t)g0.hi << 32) | 0xffffffffull, g0.t};
      P64.tg[1] = SelTarget<uint64_t>{(uint64_t)g1.lo << 32, ((uint64_t)g1.hi << 32) | 0xffffffffull, g1.t};
    }
    __syncthreads();
    const uint32_t total = s_cnt;
    if (threadIdx.x < total) {
      const uint32_t k = cidx[threadIdx.x];
      cand[threadIdx.x] = ((uint64_t)khi[k] << 32) | (small ? (uint64_t)klo[k] : 0ull);
    }
    sel_count_finish_split<NT>(cand, total, P64);
    if (threadIdx.x == 0) {
      const uint64_t k0 = P64.tg[0].lo, k1 = P64.tg[1].lo;
      if (small) {
        write_bandwidth(J, k0, k1, nb);
      } else {
        MedianState* st = med_state(J, ws, map.ws_off[e]);
        st->a = a_open ? 0ull : (k0 >> 32) << 32;
        st->b = b_open ? ~0ull : ((k1 >> 32) << 32) | 0xffffffffull;
      }
    }
    return;
  }
  select_rest<NT>(J, ws, map.ws_off[e], lbuf, S, khi, klo, reinterpret_cast<uint32_t*>(base + L.cand), n, small,
                  a_open, b_open, nb);
}

// Keys of every ensemble pair inside [lo, hi] into cand (block-scan
// order); one block, used only when the sampled bracket missed a middle
// rank.
template <int MM, int NT>
__device__ uint32_t collect_pairs(const pds_job& J, const double* inv_rho, uint64_t lo, uint64_t hi, uint64_t* cand,
                                  SelShared<uint64_t>& S) {
  const uint32_t P = (uint32_t)((uint64_t)J.N * (J.N - 1) / 2);
  constexpr int U = 4;
  uint32_t base = 0;
  for (uint32_t c0 = 0; c0 < P; c0 += NT * U) {
    uint64_t key[U];
    bool keep[U];
    uint32_t cnt = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t p = c0 + u * NT + threadIdx.x;
      keep[u] = false;
      key[u] = 0ull;
      if (p < P) {
        int i, j;
        pair_of(p, J.N, &i, &j);
        if (!frozen_particle(J, i) && !frozen_particle(J, j)) {
          key[u] = pair_key<MM>(J, i, j, inv_rho);
          keep[u] = key[u] >= lo && key[u] <= hi;
        }
      }
      cnt += keep[u] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t o = base + block_scan<NT>(cnt, S, &total);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (keep[u]) cand[o++] = key[u];
    base += total;
  }
  return base;
}

// Count kernel over all pairs of the larger jobs, 64 x 64 pairs per block.
// Each block adds its number of ensemble keys below a and inside [a, b] to
// one packed 64-bit counter and appends the latter to the job's candidate
// array at the offset the addition returned.
template <int MM>
__global__ void __launch_bounds__(kMedThreads) median_count_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                   char* __restrict__ ws) {
  __shared__ uint64_t lbuf[kCountTile * kCountTile];
  __shared__ uint32_t wsum[16];
  __shared__ float ti_s[kCountTile * MM], tj_s[kCountTile * MM];
  __shared__ bool fi_s[kCountTile], fj_s[kCountTile];  // frozen particles of the two tiles
  __shared__ uint32_t less_s;
  __shared__ uint32_t base_s;
  constexpr int NT = kMedThreads;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  MedianState* st = med_state(J, ws, map.ws_off[e]);
  const int N = J.N, M = J.M;
  const int nb = (N + kCountTile - 1) / kCountTile;
  int bi, bj;
  tile_of(blockIdx.x - map.begin[e], nb, &bi, &bj);
  const uint64_t a = st->a, b = st->b;
  const int ri = bi * kCountTile, rj = bj * kCountTile;
  const int ni = min(kCountTile, N - ri), nj = min(kCountTile, N - rj);
  // tiles of theta rows, zero-padded to MM parameters
  for (int t = threadIdx.x; t < kCountTile * MM; t += NT) {
    const int r = t / MM, m = t % MM;
    ti_s[t] = (r < ni && m < M) ? J.theta[(size_t)(ri + r) * M + m] : 0.f;
    tj_s[t] = (r < nj && m < M) ? J.theta[(size_t)(rj + r) * M + m] : 0.f;
  }
  if (threadIdx.x < kCountTile) fi_s[threadIdx.x] = threadIdx.x < ni && frozen_particle(J, ri + threadIdx.x);
  else if (threadIdx.x < 2 * kCountTile) {
    const int r = threadIdx.x - kCountTile;
    fj_s[r] = r < nj && frozen_particle(J, rj + r);
  }
  if (threadIdx.x == 0) less_s = 0u;
  __syncthreads();
  double inv_rho[MM];
  load_inv_rho<MM>(J, inv_rho);
  const int row = threadIdx.x & (kCountTile - 1);
  const int cg = threadIdx.x / kCountTile;  // 16 groups of 4 columns
  const int i = ri + row;
  uint64_t key[4];
  bool keep[4];
  uint32_t nless = 0, nkeep = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int jl = cg * 4 + q;
    const bool valid = row < ni && jl < nj && i < rj + jl && !fi_s[row] && !fj_s[jl];
    key[q] = valid ? key_of(pair_d2<MM>(&ti_s[row * MM], &tj_s[jl * MM], inv_rho, M)) : 0ull;
    nless += (valid && key[q] < a) ? 1u : 0u;
    keep[q] = valid && key[q] >= a && key[q] <= b;
    nkeep += keep[q] ? 1u : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nless += __shfl_xor(nless, o);
  if ((threadIdx.x & 63) == 0 && nless) atomicAdd(&less_s, nless);
  // block scan of nkeep (its barriers also publish less_s)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_scan(nkeep);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t o = inc - nkeep, total = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    o += k < w ? wsum[k] : 0u;
    total += wsum[k];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (keep[q]) lbuf[o++] = key[q];
  if (threadIdx.x == 0 && (total | less_s)) {
    const uint64_t old = atomicAdd((unsigned long long*)&st->packed,
                                   (unsigned long long)(((uint64_t)total << 32) | (uint64_t)less_s));
    base_s = (uint32_t)(old >> 32);
  }
  __syncthreads();
  const WsLayout L = ws_layout(J);
  uint64_t* cand = reinterpret_cast<uint64_t*>(ws + map.ws_off[e] + L.cand);
  for (uint32_t c = threadIdx.x; c < total; c += NT) cand[base_s + c] = lbuf[c];
}

// ---------------------------------------------------------------------------
// Narrow median for larger jobs whose bandwidth runs concurrently with a
// window kernel that leaves whole SIMDs free for its whole duration (the
// 2048-particle arm job has 960 waves for 1024 SIMDs, one wave per SIMD,
// LDS nearly full).  Blocks of the kernels above (256 or 1024 threads)
// cannot be placed beside such a kernel and would wait for its end; these
// run one wave per block with at most 40 KiB of LDS, so they fit the free
// SIMDs and finish inside the window kernel's time, slowly but off the
// critical path.  The results are the same keys: the bracket is the same
// pair of sample order statistics, the candidates the same keys (in
// another order), the selection exact.
// ---------------------------------------------------------------------------
constexpr int kLeanThreads = 64;
constexpr int kLeanCap = 4096;     // 32-bit sample keys the bracket kernel holds in LDS
constexpr int kLeanLastCap = 2048;  // 64-bit candidates the narrow final holds in LDS

// Bracket of a larger job from its sample (as the select kernel computes
// it): the sample's order statistics at the middle ranks' sample positions
// widened by four binomial standard deviations, as whole high words.
__global__ void __launch_bounds__(kLeanThreads) median_bracket_lean_kernel(JobMap map,
                                                                           const pds_job* __restrict__ jobs,
                                                                           char* __restrict__ ws, int rank_shift) {
  constexpr int NT = kLeanThreads;
  constexpr uint32_t kNoKey = 0xffffffffu;
  __shared__ uint32_t lbuf[kLeanCap];
  __shared__ SelShared<uint32_t> S;
  __shared__ uint32_t s_nb;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const uint64_t P = (uint64_t)J.N * (J.N - 1) / 2;
  const uint32_t n = (uint32_t)kSampleKeys;
  const WsLayout L = ws_layout(J);
  const uint32_t* khi = reinterpret_cast<const uint32_t*>(ws + map.ws_off[e] + L.khi);
  MedianState* st = med_state(J, ws, map.ws_off[e]);
  const uint32_t nb = ensemble_size<NT>(J, &s_nb);
  const uint64_t Pe = (uint64_t)nb * (nb - 1) / 2;
  // unmasked sample keys and their range
  uint32_t nvl = 0u, mn = kNoKey, mx = 0u;
  for (uint32_t c = threadIdx.x; c < n; c += NT) {
    const uint32_t h = khi[c];
    if (h != kNoKey) {
      ++nvl;
      mn = h < mn ? h : mn;
      mx = h > mx ? h : mx;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    nvl += (uint32_t)__shfl_xor((int)nvl, o);
    const uint32_t a = (uint32_t)__shfl_xor((int)mn, o), b = (uint32_t)__shfl_xor((int)mx, o);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  const uint32_t nv = nvl;
  if (Pe == 0 || nv == 0) {
    if (threadIdx.x == 0) {
      st->a = 0ull;
      st->b = ~0ull;
    }
    return;
  }
  const double d = 2.0 * sqrt((double)n) + 2.0;
  const double c0 = (double)n * (double)((Pe - 1) / 2) / (double)P - d + rank_shift;
  const double c1 = (double)n * (double)(Pe / 2 + 1) / (double)P + d + rank_shift;
  const bool a_open = c0 < 0.0 || c0 > (double)(nv - 1);
  const bool b_open = c1 > (double)(nv - 1);
  const uint32_t t0 = a_open ? 0u : (uint32_t)floor(c0);
  const uint32_t t1 = b_open ? nv - 1 : (uint32_t)fmax(ceil(c1), 0.0);
  if (threadIdx.x == 0) {
    S.tg[0] = SelTarget<uint32_t>{mn, mx, t0};
    S.tg[1] = SelTarget<uint32_t>{mn, mx, t1};
  }
  __syncthreads();
  uint32_t hsel[2];
  select_keys<NT>(khi, n, true, lbuf, (uint32_t)kLeanCap, S, hsel);
  if (threadIdx.x == 0) {
    st->a = a_open ? 0ull : (uint64_t)hsel[0] << 32;
    st->b = b_open ? ~0ull : (((uint64_t)hsel[1] << 32) | 0xffffffffull);
  }
}

// Count kernel of the narrow median: one wave per 64 x 64 tile, four
// columns per lane at a time; the keys below a are counted and those inside
// [a, b] appended to the candidate array, one atomic per group of columns.
template <int MM>
__global__ void __launch_bounds__(kLeanThreads) median_count_lean_kernel(JobMap map,
                                                                         const pds_job* __restrict__ jobs,
                                                                         char* __restrict__ ws) {
  __shared__ float ti_s[kCountTile * MM], tj_s[kCountTile * MM];
  __shared__ bool fi_s[kCountTile], fj_s[kCountTile];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  MedianState* st = med_state(J, ws, map.ws_off[e]);
  const int N = J.N, M = J.M;
  const int nb = (N + kCountTile - 1) / kCountTile;
  int bi, bj;
  tile_of(blockIdx.x - map.begin[e], nb, &bi, &bj);
  const uint64_t a = st->a, b = st->b;
  const int ri = bi * kCountTile, rj = bj * kCountTile;
  const int ni = min(kCountTile, N - ri), nj = min(kCountTile, N - rj);
  for (int t = threadIdx.x; t < kCountTile * MM; t += kLeanThreads) {
    const int r = t / MM, m = t % MM;
    ti_s[t] = (r < ni && m < M) ? J.theta[(size_t)(ri + r) * M + m] : 0.f;
    tj_s[t] = (r < nj && m < M) ? J.theta[(size_t)(rj + r) * M + m] : 0.f;
  }
  const int row = threadIdx.x;
  fi_s[row] = row < ni && frozen_particle(J, ri + row);
  fj_s[row] = row < nj && frozen_particle(J, rj + row);
  __syncthreads();
  double inv_rho[MM];
  load_inv_rho<MM>(J, inv_rho);
  const int i = ri + row;
  const WsLayout L = ws_layout(J);
  uint64_t* cand = reinterpret_cast<uint64_t*>(ws + map.ws_off[e] + L.cand);
  uint32_t nless = 0;
  for (int cg = 0; cg < kCountTile / 4; ++cg) {
    uint64_t key[4];
    bool keep[4];
    uint32_t nkeep = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jl = cg * 4 + q;
      const bool valid = row < ni && jl < nj && i < rj + jl && !fi_s[row] && !fj_s[jl];
      key[q] = valid ? key_of(pair_d2<MM>(&ti_s[row * MM], &tj_s[jl * MM], inv_rho, M)) : 0ull;
      nless += (valid && key[q] < a) ? 1u : 0u;
      keep[q] = valid && key[q] >= a && key[q] <= b;
      nkeep += keep[q] ? 1u : 0u;
    }
    const uint32_t inc = wave_scan(nkeep);
    const uint32_t total = (uint32_t)__shfl((int)inc, 63);
    if (total == 0) continue;
    uint32_t base = 0;
    if (threadIdx.x == 63)
      base = (uint32_t)(atomicAdd((unsigned long long*)&st->packed, (unsigned long long)total << 32) >> 32);
    base = (uint32_t)__shfl((int)base, 63);
    uint32_t o = base + inc - nkeep;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (keep[q]) cand[o++] = key[q];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nless += __shfl_xor(nless, o);
  if (threadIdx.x == 0 && nless) atomicAdd((unsigned long long*)&st->packed, (unsigned long long)nless);
}

// Final kernel, one block per larger job: both middle keys of the
// ensemble's pairs exactly among the candidates or, if the bracket missed a
// middle rank, among the keys of the interval that holds both (recomputed
// from theta).
template <int MM, int NT = kMedThreads, int CAP = kLastCap>
__global__ void __launch_bounds__(NT) median_final_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                          char* __restrict__ ws) {
  __shared__ uint64_t lbuf[CAP];
  __shared__ SelShared<uint64_t> S;
  __shared__ uint32_t s_nb;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const MedianState* st = med_state(J, ws, map.ws_off[e]);
  const uint32_t nb = ensemble_size<NT>(J, &s_nb);
  const uint32_t P = (uint32_t)((uint64_t)nb * (nb - 1) / 2);  // the ensemble's pairs
  if (P == 0) {
    if (threadIdx.x == 0) write_bandwidth(J, 0ull, 0ull, nb);
    return;
  }
  const WsLayout L = ws_layout(J);
  uint64_t* cand = reinterpret_cast<uint64_t*>(ws + map.ws_off[e] + L.cand);
  const uint64_t a = st->a, b = st->b, packed = st->packed;
  const uint32_t cl = (uint32_t)(packed & 0xffffffffull), nc = (uint32_t)(packed >> 32);
  const uint32_t r0 = (P - 1) / 2, r1 = P / 2;
  uint32_t n = nc, off = cl;
  uint64_t lo = a, hi = b;
  if (!(cl <= r0 && (uint64_t)r1 < (uint64_t)cl + nc)) {
    double inv_rho[MM];
    load_inv_rho<MM>(J, inv_rho);
    lo = r0 < cl ? 0ull : a;
    hi = (uint64_t)r1 >= (uint64_t)cl + nc ? ~0ull : b;
    off = r0 < cl ? 0u : cl;
    n = collect_pairs<MM, NT>(J, inv_rho, lo, hi, cand, S);
  }
  if (threadIdx.x == 0) {
    S.tg[0] = SelTarget<uint64_t>{lo, hi, r0 - off};
    S.tg[1] = SelTarget<uint64_t>{lo, hi, r1 - off};
  }
  __syncthreads();
  uint64_t out[2];
  select_keys<NT>((const uint64_t*)cand, n, true, lbuf, (uint32_t)CAP, S, out);
  if (threadIdx.x == 0) write_bandwidth(J, out[0], out[1], nb);
}

// Larger jobs: partial phi of particles i (one per lane) over one chunk
// of j (many blocks), then a reduction over the chunks in chunk order.  The
// chunk's live rows sit in LDS in particle order with stride MM, zero
// beyond M, so the parameter loops run unconditionally (padded terms
// contribute 0); the blocks of the first i range store each chunk's number
// of live rows for the reduction.
template <int MM>
__global__ void __launch_bounds__(kPairBlock) phi_partial_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                                 char* __restrict__ ws) {
  __shared__ float tj_s[kPhiChunk * MM];
  __shared__ float gj_s[kPhiChunk * MM];
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int N = J.N, M = J.M;
  const int nib = (N + kPairBlock - 1) / kPairBlock;
  const int local = blockIdx.x - map.begin[e];
  const int ib = local % nib, jc = local / nib;
  const int j0 = jc * kPhiChunk;
  const int nj = min(kPhiChunk, N - j0);
  static_assert(kPhiChunk <= kPairBlock && kPairBlock == kWave, "one wave compacts the chunk");
  const bool lv = (int)threadIdx.x < nj && in_phi(J, j0 + threadIdx.x);
  const uint64_t bal = __ballot(lv);
  const int nl = __popcll(bal);
  if (lv) {
    const int pos = __popcll(bal & ((1ull << threadIdx.x) - 1ull));
    const size_t src = (size_t)(j0 + threadIdx.x) * M;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      tj_s[pos * MM + m] = m < M ? J.theta[src + m] : 0.f;
      gj_s[pos * MM + m] = m < M ? (float)J.g_obs[src + m] : 0.f;
    }
  }
  __syncthreads();
  const WsLayout L = ws_layout(J);
  if (ib == 0 && threadIdx.x == 0) reinterpret_cast<uint32_t*>(ws + map.ws_off[e] + L.phi_live)[jc] = (uint32_t)nl;
  const int i = ib * kPairBlock + threadIdx.x;
  if (i >= N) return;
  const float h = (float)J.bandwidth[0];
  const float inv_h = 1.0f / h;
  float ti[MM], rh[MM], ir[MM], ir2[MM], acc[MM];
  load_padded<MM>(J.theta + (size_t)i * M, M, ti);
  load_padded<MM>(J.rho, M, rh);
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    ir[m] = m < M ? 1.0f / rh[m] : 0.f;
    ir2[m] = ir[m] * ir[m];
    acc[m] = 0.f;
  }
  for (int jj = 0; jj < nl; ++jj) {
    float d2 = 0.f;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      const float z = (ti[m] - tj_s[jj * MM + m]) * ir[m];
      d2 += z * z;
    }
    const float k = expf(-d2 * inv_h);
    const float k2h = 2.0f * k * inv_h;
#pragma unroll
    for (int m = 0; m < MM; ++m) acc[m] += k * gj_s[jj * MM + m] + k2h * (ti[m] - tj_s[jj * MM + m]) * ir2[m];
  }
  float* part = reinterpret_cast<float*>(ws + map.ws_off[e] + L.phi_part);
#pragma unroll
  for (int m = 0; m < MM; ++m)
    if (m < M) part[((size_t)jc * N + i) * M + m] = acc[m];
}

// phi_i = (sum of the partials) / N' with N' the live rows of all chunks;
// 0 for particles out of the ensemble.
__global__ void __launch_bounds__(256) phi_reduce_kernel(JobMap map, const pds_job* __restrict__ jobs,
                                                         char* __restrict__ ws) {
  __shared__ uint32_t s_live;
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int t = (blockIdx.x - map.begin[e]) * 256 + threadIdx.x;
  const int chunks = (J.N + kPhiChunk - 1) / kPhiChunk;
  const WsLayout L = ws_layout(J);
  {
    const uint32_t* lc = reinterpret_cast<const uint32_t*>(ws + map.ws_off[e] + L.phi_live);
    uint32_t c = 0;
    for (int q = threadIdx.x; q < chunks; q += 256) c += lc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (threadIdx.x == 0) s_live = 0u;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_live, c);
    __syncthreads();
  }
  const uint32_t n_live = s_live;
  if (J.n_masked && blockIdx.x == map.begin[e] && threadIdx.x == 0) *J.n_masked = J.N - (int)n_live;
  if (t >= J.N * J.M) return;
  const float* part = reinterpret_cast<const float*>(ws + map.ws_off[e] + L.phi_part);
  const size_t stride = (size_t)J.N * J.M;
  float s = 0.f;
  constexpr int B = 8;  // partials loaded per batch, added in chunk order
  for (int c0 = 0; c0 < chunks; c0 += B) {
    float v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = part[(size_t)(c0 + b < chunks ? c0 + b : chunks - 1) * stride + t];
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (c0 + b < chunks) s += v[b];
  }
  J.phi[t] = in_phi(J, t / J.M) ? s / (float)n_live : 0.f;
}

// Jobs up to kPhiFusedMaxN particles: phi for TI particles i per block
// (16 up to 128 particles, 8 above: more blocks, each with less work).  The
// block stages the live particles' rows and driving terms in LDS, from
// kPhiRows particles at a time, compacted in particle order (rows padded
// with zeros to MM parameters, so the parameter loops run without
// branches); thread (il, js) accumulates particle i0 + il over staged rows
// js, js + 1024 / TI, ... in that order; the slices of a wave that share
// il are added by a fixed shuffle tree, then the 16 waves' sums in wave
// order.  Every sum has a fixed order that depends on N and the flags
// alone.
template <int MM, int TI>
__global__ void __launch_bounds__(kPhiThreads) phi_kernel(JobMap map, const pds_job* __restrict__ jobs) {
  constexpr int kPhiTI = TI;
  static_assert(kPhiRows % (kPhiThreads / kPhiTI) == 0, "chunks keep each slice's j order");
  static_assert(kWave % kPhiTI == 0, "a wave holds whole groups of slices");
  __shared__ float tj_s[kPhiRows * MM];
  __shared__ float gj_s[kPhiRows * MM];
  __shared__ float red[kPhiThreads / kWave][kPhiTI * MM];
  __shared__ uint32_t wlive[kPhiThreads / kWave];
  static_assert(kPhiRows <= kPhiThreads, "one thread per row of a chunk");
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int N = J.N, M = J.M;
  const int il = threadIdx.x % kPhiTI, js = threadIdx.x / kPhiTI;
  const int w = threadIdx.x / kWave;
  const int i = (blockIdx.x - map.begin[e]) * kPhiTI + il;
  constexpr int kSlices = kPhiThreads / kPhiTI;  // j stride
  const float h = (float)J.bandwidth[0];
  const float inv_h = 1.0f / h;
  float ti[MM], rh[MM], ir[MM], ir2[MM], acc[MM];
  load_padded<MM>(J.theta + (size_t)min(i, N - 1) * M, M, ti);
  load_padded<MM>(J.rho, M, rh);
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    ir[m] = m < M ? 1.0f / rh[m] : 0.f;
    ir2[m] = ir[m] * ir[m];
    acc[m] = 0.f;
  }
  const int lane = threadIdx.x % kWave;
  uint32_t n_live = 0;  // live particles of the chunks so far (the same in every thread)
  for (int j0 = 0; j0 < N; j0 += kPhiRows) {
    const int nr = min(kPhiRows, N - j0);
    if (j0 > 0) __syncthreads();  // the previous chunk is consumed
    // thread r < nr owns row j0 + r; live rows go to their rank among the
    // chunk's live rows
    const bool lv = (int)threadIdx.x < nr && in_phi(J, j0 + threadIdx.x);
    const uint64_t bal = __ballot(lv);
    if (lane == 0) wlive[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = 0, nl = 0;
#pragma unroll
    for (int v = 0; v < kPhiThreads / kWave; ++v) {
      before += v < w ? wlive[v] : 0u;
      nl += wlive[v];
    }
    if (lv) {
      const uint32_t pos = before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
      const size_t src = (size_t)(j0 + threadIdx.x) * M;
#pragma unroll
      for (int m = 0; m < MM; ++m) {
        tj_s[pos * MM + m] = m < M ? J.theta[src + m] : 0.f;
        gj_s[pos * MM + m] = m < M ? (float)J.g_obs[src + m] : 0.f;
      }
    }
    __syncthreads();
    n_live += nl;
    for (int jl = js; jl < (int)nl; jl += kSlices) {
      float d2 = 0.f;
#pragma unroll
      for (int m = 0; m < MM; ++m) {
        const float z = (ti[m] - tj_s[jl * MM + m]) * ir[m];
        d2 += z * z;
      }
      const float k = expf(-d2 * inv_h);
      const float k2h = 2.0f * k * inv_h;
#pragma unroll
      for (int m = 0; m < MM; ++m) acc[m] += k * gj_s[jl * MM + m] + k2h * (ti[m] - tj_s[jl * MM + m]) * ir2[m];
    }
  }
  // lanes il, il + TI, il + 2 TI, ... of a wave hold the same particle
#pragma unroll
  for (int o = kPhiTI; o < kWave; o <<= 1) {
#pragma unroll
    for (int m = 0; m < MM; ++m) acc[m] += __shfl_xor(acc[m], o);
  }
  if ((threadIdx.x % kWave) < kPhiTI) {
#pragma unroll
    for (int m = 0; m < MM; ++m) red[w][il * MM + m] = acc[m];
  }
  __syncthreads();
  if (threadIdx.x < kPhiTI * MM) {
    const int r = threadIdx.x / MM, m = threadIdx.x % MM;
    const int ir_ = (blockIdx.x - map.begin[e]) * kPhiTI + r;
    float s = 0.f;
#pragma unroll
    for (int v = 0; v < kPhiThreads / kWave; ++v) s += red[v][r * MM + m];
    if (ir_ < N && m < M) J.phi[(size_t)ir_ * M + m] = in_phi(J, ir_) ? s / (float)n_live : 0.f;
  }
  if (J.n_masked && blockIdx.x == map.begin[e] && threadIdx.x == 0) *J.n_masked = N - (int)n_live;
}

// MDMM + optimizer update.  Flat index over theta (N M), S (N K (n_s-1) d_s)
// and lam_def (N K (n_s-1)).  Particles out of the ensemble keep every
// variable; the thread of their first parameter sets flag bit 3.  (That
// bit is set only where bit 0 or 1 already is, so every thread of the
// particle takes the same branch whether or not it sees it.)
__global__ void __launch_bounds__(kStepThreads) step_kernel(JobMap map, const pds_job* __restrict__ jobs, int optimizer,
                                                   int iter) {
  const int e = map_entry(map, blockIdx.x);
  const pds_job& J = jobs[map.job[e]];
  const int ds = 2 * J.n_dof;
  const int nSp = J.K * (J.n_s - 1) * ds;  // shooting floats per particle
  const int nLp = J.K * (J.n_s - 1);
  const int nT = J.N * J.M, nS = J.N * nSp, nL = J.N * nLp;
  const int nb = map.begin[e + 1] - map.begin[e];
  const int stride = J.M + nSp;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  // Adam bias corrections 1 - b^it per thread, b^it = 2^(it log2 b): no
  // block-wide wait before the element loads
  const int it = J.iter_dev ? J.iter_dev[0] + 1 : iter;
  const float bc1 = 1.0f - exp2f((float)it * log2f(b1)), bc2 = 1.0f - exp2f((float)it * log2f(b2));
  // the job's elements, grid-stride over its (at most kStepCountBlocks) blocks
  for (int t = (blockIdx.x - map.begin[e]) * kStepThreads + threadIdx.x; t < nT + nS + nL; t += nb * kStepThreads) {
  if (t < nT && !in_phi(J, t / J.M)) {
    const int i = t / J.M;
    if (t % J.M == 0 && !(J.flags[i] & PDS_FLAG_FROZEN)) atomicOr(&J.flags[i], PDS_FLAG_FROZEN);
  } else if (t < nT) {
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
    if (J.limits == PDS_LIMITS_PROJECT) xn = fminf(fmaxf(xn, lo), hi);
    J.theta[t] = xn;
    J.lam_lim[t] += J.eps_lam * g;
    if ((xn < lo || xn > hi) && J.flags) atomicOr(&J.flags[i], PDS_FLAG_LIMIT);
  } else if (t < nT + nS && in_phi(J, (t - nT) / nSp)) {
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
  } else if (t >= nT + nS && t < nT + nS + nL && J.lik != PDS_LIK_DEFECT && in_phi(J, (t - nT - nS) / nLp)) {
    const int r = t - nT - nS;
    J.lam_def[r] += J.eps_lam * (float)J.gdef[r];
  }
  }
  if (J.iter_dev) {
    // Advance the device counter once every block of the job is past its
    // use of it: each thread's stores above depend on the value it read,
    // so after the barrier every read of this block has returned.  Blocks
    // count themselves in iter_dev[1] with device-scope atomics; the last
    // one bumps the counter and leaves the count at zero for the next call.
    // (Same-address atomics serialise: hence at most kStepCountBlocks
    // blocks per job, each taking several elements.)
    __syncthreads();
    if (threadIdx.x == 0) {
      if (atomicAdd(&J.iter_dev[1], 1) == nb - 1) {
        atomicExch(&J.iter_dev[1], 0);
        atomicAdd(&J.iter_dev[0], 1);
      }
    }
  }
}

}  // namespace

#define PDS_MEDIAN_LAUNCH(kernel, grid, threads, map, ...)                                                  \
  do {                                                                                                      \
    if (mmax <= 4)                                                                                          \
      hipLaunchKernelGGL(kernel<4>, dim3(grid), dim3(threads), 0, s, map, d_jobs, ws, ##__VA_ARGS__);         \
    else if (mmax <= 8)                                                                                     \
      hipLaunchKernelGGL(kernel<8>, dim3(grid), dim3(threads), 0, s, map, d_jobs, ws, ##__VA_ARGS__);         \
    else                                                                                                    \
      hipLaunchKernelGGL(kernel<PDS_MAX_M>, dim3(grid), dim3(threads), 0, s, map, d_jobs, ws, ##__VA_ARGS__); \
  } while (0)

hipError_t launch_median(const MedianMaps& mm, const pds_job* d_jobs, char* ws, int mmax, int rank_shift,
                         hipStream_t s) {
  hipError_t err = hipSuccess;
  if (mm.keys.n > 0) {
    PDS_MEDIAN_LAUNCH(median_keys_kernel, mm.grid_keys, 256, mm.keys);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (mm.select.n > 0) {
    hipLaunchKernelGGL(median_select_kernel, dim3(mm.grid_select), dim3(kMedThreads), 0, s, mm.select, d_jobs, ws,
                       rank_shift);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (mm.large.n > 0) {
    PDS_MEDIAN_LAUNCH(median_count_kernel, mm.grid_count, kMedThreads, mm.count);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    PDS_MEDIAN_LAUNCH(median_final_kernel, mm.grid_large, kMedThreads, mm.large);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (mm.lean_final.n > 0) {  // the narrow chain (see median_bracket_lean_kernel)
    PDS_MEDIAN_LAUNCH(median_keys_kernel, mm.grid_lean_keys, kLeanThreads, mm.lean_keys);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(median_bracket_lean_kernel, dim3(mm.grid_lean_final), dim3(kLeanThreads), 0, s,
                       mm.lean_final, d_jobs, ws, rank_shift);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    PDS_MEDIAN_LAUNCH(median_count_lean_kernel, mm.grid_lean_count, kLeanThreads, mm.lean_count);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (mmax <= 4)
      hipLaunchKernelGGL((median_final_kernel<4, kLeanThreads, kLeanLastCap>), dim3(mm.grid_lean_final),
                         dim3(kLeanThreads), 0, s, mm.lean_final, d_jobs, ws);
    else if (mmax <= 8)
      hipLaunchKernelGGL((median_final_kernel<8, kLeanThreads, kLeanLastCap>), dim3(mm.grid_lean_final),
                         dim3(kLeanThreads), 0, s, mm.lean_final, d_jobs, ws);
    else
      hipLaunchKernelGGL((median_final_kernel<PDS_MAX_M, kLeanThreads, kLeanLastCap>), dim3(mm.grid_lean_final),
                         dim3(kLeanThreads), 0, s, mm.lean_final, d_jobs, ws);
    err = hipGetLastError();
  }
  return err;
}

// Workspace of svgd_phi_noalloc: one fixed array per device, held until the
// process ends.  Host code never passes the array's name to a kernel (in
// host code it is a stand-in, not a device address): noalloc_scratch looks
// up this device's address once, with the device current, and every launch
// gets that address.
static __device__ __align__(256) unsigned char scratch[PDS_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(int device, void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptr[device] = p;
  }
  *out = ptr[device];
  return hipSuccess;
}

hipError_t launch_phi_partial(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, int mmax,
                              hipStream_t s) {
  if (mmax <= 4)
    hipLaunchKernelGGL(phi_partial_kernel<4>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  else if (mmax <= 8)
    hipLaunchKernelGGL(phi_partial_kernel<8>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  else if (mmax <= 12)
    hipLaunchKernelGGL(phi_partial_kernel<12>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  else
    hipLaunchKernelGGL(phi_partial_kernel<PDS_MAX_M>, dim3(grid), dim3(kPairBlock), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

hipError_t launch_phi_reduce(const JobMap& map, const pds_job* d_jobs, char* ws, int grid, hipStream_t s) {
  hipLaunchKernelGGL(phi_reduce_kernel, dim3(grid), dim3(256), 0, s, map, d_jobs, ws);
  return hipGetLastError();
}

template <int TI>
static void launch_phi_ti(const JobMap& map, const pds_job* d_jobs, int grid, int mmax, hipStream_t s) {
  const dim3 blk(kPhiThreads);
  if (mmax <= 4)
    hipLaunchKernelGGL((phi_kernel<4, TI>), dim3(grid), blk, 0, s, map, d_jobs);
  else if (mmax <= 8)
    hipLaunchKernelGGL((phi_kernel<8, TI>), dim3(grid), blk, 0, s, map, d_jobs);
  else if (mmax <= 12)
    hipLaunchKernelGGL((phi_kernel<12, TI>), dim3(grid), blk, 0, s, map, d_jobs);
  else
    hipLaunchKernelGGL((phi_kernel<PDS_MAX_M, TI>), dim3(grid), blk, 0, s, map, d_jobs);
}

hipError_t launch_phi(const JobMap& map, const pds_job* d_jobs, int grid, int mmax, int ti, hipStream_t s) {
  if (ti == kPhiTISmall)
    launch_phi_ti<kPhiTISmall>(map, d_jobs, grid, mmax, s);
  else
    launch_phi_ti<kPhiTILarge>(map, d_jobs, grid, mmax, s);
  return hipGetLastError();
}

hipError_t launch_step(const JobMap& map, const pds_job* d_jobs, int grid, int optimizer, int iter,
                       hipStream_t s) {
  hipLaunchKernelGGL(step_kernel, dim3(grid), dim3(kStepThreads), 0, s, map, d_jobs, optimizer, iter);
  return hipGetLastError();
}

}  // namespace pds
