// Device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// The radix sort is the binning sort of the rasterizer: (tile, depth) keys
// are ordered by stable passes over 8-bit (or narrower) digits, least
// significant first.  Each pass = per-workgroup digit histograms (LDS
// atomics), one exclusive scan of the digit-major histogram table, and a
// scatter in which every key's rank among equal digits of its workgroup comes
// from wavefront ballots (a match mask per digit) plus per-wave counts in LDS,
// so equal keys keep their input order.
#include "internal.h"

namespace dcgs {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of the block's thread values; returns the block total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *excl) {
  __shared__ uint32_t wsum[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / kWave; ++k) {
    uint32_t s = wsum[k];
    if (k < w) off += s;
    tot += s;
  }
  *excl = off + inc - v;
  __syncthreads();
  return tot;
}

// Element count of a launch: the host value, or (when the launch was made
// for a capacity) the device counter clamped to that capacity.
__device__ inline int64_t count_of(const int64_t *n_dev, int64_t n) {
  return n_dev ? min(*n_dev, n) : n;
}

__device__ inline uint32_t load_item(const uint32_t *in, const uint32_t *gather,
                                     int64_t i, int64_t n) {
  if (i >= n) return 0;
  return gather ? in[gather[i]] : in[i];
}

__global__ void __launch_bounds__(kScanThreads)
    k_scan_reduce(const uint32_t *__restrict__ in,
                  const uint32_t *__restrict__ gather, const int64_t *__restrict__ n_dev,
                  int64_t n, uint32_t *__restrict__ part) {
  n = count_of(n_dev, n);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    s += load_item(in, gather, base + k * kScanThreads + threadIdx.x, n);
  uint32_t excl;
  uint32_t tot = block_exclusive_scan(s, &excl);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of the per-block totals, one workgroup.
__global__ void __launch_bounds__(kScanThreads)
    k_scan_top(uint32_t *__restrict__ part, int64_t nb) {
  __shared__ uint32_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t r = 0; r < nb; r += kScanThreads) {
    int64_t i = r + threadIdx.x;
    uint32_t v = i < nb ? part[i] : 0;
    uint32_t excl;
    uint32_t tot = block_exclusive_scan(v, &excl);
    uint32_t c = carry_s;
    if (i < nb) part[i] = c + excl;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = c + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) part[nb] = carry_s;
}

__global__ void __launch_bounds__(kScanThreads)
    k_scan_down(const uint32_t *__restrict__ in,
                const uint32_t *__restrict__ gather, const int64_t *__restrict__ n_dev,
                int64_t n, const uint32_t *__restrict__ part, uint32_t *__restrict__ out) {
  __shared__ uint32_t tile[kScanTile + kScanTile / 32];
  n = count_of(n_dev, n);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  auto pad = [](int i) { return i + (i >> 5); };
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int li = k * kScanThreads + threadIdx.x;
    tile[pad(li)] = load_item(in, gather, base + li, n);
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = tile[pad(threadIdx.x * kScanItems + k)];
    s += v[k];
  }
  uint32_t excl;
  block_exclusive_scan(s, &excl);
  uint32_t run = part[blockIdx.x] + excl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    tile[pad(threadIdx.x * kScanItems + k)] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int li = k * kScanThreads + threadIdx.x;
    if (base + li < n) out[base + li] = tile[pad(li)];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[gridDim.x];
}

// ---------------------------------------------------------------- radix --
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 keys per block
constexpr int kSortWaves = kSortThreads / kWave;

template <typename K>
__device__ inline uint32_t digit_of(K key, int shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

// Digits of up to 8 bits take 256-bin tables, of 9 bits 512 (a 17- or
// 18-bit key then sorts in two passes instead of three).
template <typename K, int kBins>
__global__ void __launch_bounds__(kSortThreads)
    k_rs_hist(const K *__restrict__ keys, const int64_t *__restrict__ n_dev, int64_t n,
              int shift, int width, uint32_t *__restrict__ hist, int64_t nb) {
  __shared__ uint32_t h[kBins];
  n = count_of(n_dev, n);
  const uint32_t bins = 1u << width, mask = bins - 1;
  for (int t = threadIdx.x; t < kBins; t += kSortThreads) h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  // all of the thread's keys in flight at once, then the counts
  K key[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    key[r] = i < n ? keys[i] : K(0);
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r)
    if (base + r * kSortThreads + threadIdx.x < n) atomicAdd(&h[digit_of(key[r], shift, mask)], 1u);
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < bins; d += kSortThreads)
    hist[(int64_t)d * nb + blockIdx.x] = h[d];
}

// Scatter of one pass.  The workgroup first ranks its 4096 keys stably by
// digit into LDS (so its keys sit there grouped by digit, in input order
// within a digit), then writes each digit's run to its global offset:
// consecutive threads write consecutive addresses of one run.
// Ranking: wavefront w owns the contiguous keys [1024 w, 1024 w + 1024) and
// walks them 64 at a time in order; a key's rank among equal digits of its
// step comes from ballots (a match mask per digit), and a per-wavefront
// running count per digit (LDS, touched by that wavefront only) places it
// after the equal digits of the wavefront's earlier steps.  One scan of the
// per-wavefront counts, digit-major, then gives every key its slot: the
// workgroup synchronises a fixed number of times, not once per step.
template <typename K, bool kVals, int kBins>
__global__ void __launch_bounds__(kSortThreads)
    k_rs_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                 K *__restrict__ kout, uint32_t *__restrict__ vout,
                 const int64_t *__restrict__ n_dev, int64_t n, int shift, int width,
                 const uint32_t *__restrict__ hist, const uint32_t *__restrict__ offs,
                 int64_t nb) {
  constexpr int kPerWave = kSortTile / kSortWaves;  // 1024 keys
  constexpr int kSteps = kPerWave / kWave;           // 16
  __shared__ K sk[kSortTile];
  __shared__ uint32_t sv[kVals ? kSortTile : 1];
  static_assert(kBins % kSortThreads == 0, "whole digits per thread");
  constexpr int kPer = kBins / kSortThreads;  // digits per thread in the slot scan
  __shared__ uint32_t gofs[kBins];  // global offset of the block's run of digit d
  __shared__ uint32_t lofs[kBins];  // start of digit d's run in sk
  __shared__ uint32_t wcnt[kSortWaves][kBins];  // per wavefront: count, then slot base
  n = count_of(n_dev, n);
  const uint32_t bins = 1u << width, mask = bins - 1;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) return;  // uniform across the block
  const int cnt = (int)min<int64_t>(kSortTile, n - base);
  for (int t = threadIdx.x; t < kSortWaves * kBins; t += kSortThreads) (&wcnt[0][0])[t] = 0;
  for (int d = threadIdx.x; d < kBins; d += kSortThreads)
    gofs[d] = (uint32_t)d < bins ? offs[(int64_t)d * nb + blockIdx.x] : 0u;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  K key[kSteps];
  uint32_t val[kVals ? kSteps : 1];
  uint32_t pos[kSteps];
#pragma unroll
  for (int r = 0; r < kSteps; ++r) {
    const int li = w * kPerWave + r * kWave + lane;
    const bool valid = li < cnt;
    key[r] = valid ? kin[base + li] : K(0);
    if (kVals) val[r] = valid ? vin[base + li] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSteps; ++r) {
    const int li = w * kPerWave + r * kWave + lane;
    const bool valid = li < cnt;
    const uint32_t d = digit_of(key[r], shift, mask);
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < width; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    // the running count is read by every lane before the step's leader
    // adds to it (in-order LDS access within the wavefront)
    const uint32_t before = valid ? wcnt[w][d] : 0u;
    pos[r] = before + (uint32_t)__popcll(peers & lt);
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {  // slot bases: exclusive scan over (digit, wavefront), digit-major;
     // thread t takes digits kPer t .. kPer t + kPer - 1
    uint32_t c[kPer][kSortWaves], tot[kPer], all = 0;
#pragma unroll
    for (int p = 0; p < kPer; ++p) {
      const uint32_t d = threadIdx.x * kPer + p;
      tot[p] = 0;
#pragma unroll
      for (int k = 0; k < kSortWaves; ++k) {
        c[p][k] = d < bins ? wcnt[k][d] : 0u;
        tot[p] += c[p][k];
      }
      all += tot[p];
    }
    uint32_t excl;
    block_exclusive_scan(all, &excl);
#pragma unroll
    for (int p = 0; p < kPer; ++p) {
      const uint32_t d = threadIdx.x * kPer + p;
      if (d < bins) {
        lofs[d] = excl;
        uint32_t run = excl;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
          wcnt[k][d] = run;
          run += c[p][k];
        }
      }
      excl += tot[p];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSteps; ++r) {
    const int li = w * kPerWave + r * kWave + lane;
    if (li < cnt) {
      const uint32_t q = wcnt[w][digit_of(key[r], shift, mask)] + pos[r];
      sk[q] = key[r];
      if (kVals) sv[q] = val[r];
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < cnt; p += kSortThreads) {
    const K k = sk[p];
    const uint32_t d = digit_of(k, shift, mask);
    const uint32_t o = gofs[d] + (uint32_t)p - lofs[d];
    kout[o] = k;
    if (kVals) vout[o] = sv[p];
  }
}

template <typename T>
__global__ void k_copy_n(const T *__restrict__ a, const int64_t *__restrict__ n_dev, int64_t n,
                         T *__restrict__ b) {
  n = count_of(n_dev, n);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <typename T>
void copy_n(const T *a, const int64_t *n_dev, int64_t n, T *b, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy_n<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n_dev,
                     n, b);
  DCGS_LAUNCH_CHECK();
}

size_t radix_scratch_bins(int64_t n, int64_t bins) {
  const int64_t tab = bins * ((n + kSortTile - 1) / kSortTile);
  return 2 * (size_t)(tab + 1) + scan_part_size(tab) + 16;
}

template <typename K, bool kVals>
void radix_pass(const K *kin, const uint32_t *vin, K *kout, uint32_t *vout,
                const int64_t *n_dev, int64_t n, int shift, int width,
                DevBuf<uint32_t> &hist, hipStream_t st) {
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  const int64_t bins = int64_t(1) << width;
  const int64_t tab = bins * nb;
  // histogram table, then its scan (part area after table + 1)
  uint32_t *h = hist.need(radix_scratch_bins(n, bins));
  uint32_t *scanned = h + tab + 1;
  uint32_t *part = scanned + tab + 1;
  DCGS_CHECK(width >= 1 && width <= 9, DCGS_E_INVALID, "radix pass: 1..9-bit digits");
  if (width <= 8)
    hipLaunchKernelGGL((k_rs_hist<K, 256>), dim3((unsigned)nb), dim3(kSortThreads), 0, st, kin,
                       n_dev, n, shift, width, h, nb);
  else
    hipLaunchKernelGGL((k_rs_hist<K, 512>), dim3((unsigned)nb), dim3(kSortThreads), 0, st, kin,
                       n_dev, n, shift, width, h, nb);
  DCGS_LAUNCH_CHECK();
  scan_u32(h, nullptr, scanned, tab, part, st);
  if (width <= 8)
    hipLaunchKernelGGL((k_rs_scatter<K, kVals, 256>), dim3((unsigned)nb), dim3(kSortThreads), 0,
                       st, kin, vin, kout, vout, n_dev, n, shift, width, h, scanned, nb);
  else
    hipLaunchKernelGGL((k_rs_scatter<K, kVals, 512>), dim3((unsigned)nb), dim3(kSortThreads), 0,
                       st, kin, vin, kout, vout, n_dev, n, shift, width, h, scanned, nb);
  DCGS_LAUNCH_CHECK();
}

}  // namespace

size_t scan_part_size(int64_t n) {
  return (size_t)((n + kScanTile - 1) / kScanTile) + 2;
}

size_t radix_scratch(int64_t n) { return radix_scratch_bins(n, 512); }

void scan_u32(const uint32_t *in, const uint32_t *gather, uint32_t *out,
              int64_t n, uint32_t *part, hipStream_t st, const int64_t *n_dev) {
  // one block at least, so that out[count] is always written
  const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0,
                     st, in, gather, n_dev, n, part);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, part, nb);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0,
                     st, in, gather, n_dev, n, part, out);
  DCGS_LAUNCH_CHECK();
}

void sort_u32_pairs(uint32_t *keys, uint32_t *vals, uint32_t *ktmp,
                    uint32_t *vtmp, int64_t n, int bits, DevBuf<uint32_t> &hist,
                    hipStream_t st, const int64_t *n_dev) {
  if (n == 0) return;
  int passes, width;
  digit_plan(bits, &passes, &width);
  uint32_t *ka = keys, *va = vals, *kb = ktmp, *vb = vtmp;
  for (int p = 0; p < passes; ++p) {
    int shift = p * width;
    int w = (shift + width > bits) ? bits - shift : width;
    radix_pass<uint32_t, true>(ka, va, kb, vb, n_dev, n, shift, w, hist, st);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    copy_n(ka, n_dev, n, keys, st);
    copy_n(va, n_dev, n, vals, st);
  }
}

void sort_u64_bits(uint64_t *a, uint64_t *tmp, int64_t n, int lo, int bits,
                   DevBuf<uint32_t> &hist, hipStream_t st, const int64_t *n_dev) {
  if (n == 0) return;
  int passes, width;
  digit_plan(bits, &passes, &width);
  uint64_t *x = a, *y = tmp;
  for (int p = 0; p < passes; ++p) {
    int shift = p * width;
    int w = (shift + width > bits) ? bits - shift : width;
    radix_pass<uint64_t, false>(x, nullptr, y, nullptr, n_dev, n, lo + shift, w, hist, st);
    std::swap(x, y);
  }
  if (x != a) copy_n(x, n_dev, n, a, st);
}

}  // namespace dcgs
