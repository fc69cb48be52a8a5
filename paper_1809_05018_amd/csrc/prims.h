// Device-wide data-parallel primitives shared by the neighbourhood builder
// and the image path: exclusive scans and a stable LSD radix sort.  Every
// primitive takes its scratch from the caller and may read its item count
// from device memory (a count pointer, with the grid sized for an upper
// bound), so a chain of them needs no host round trip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmrf_prims {
namespace {  // each translation unit gets its own copies of the kernels

constexpr int kBT = 256;  // threads per block

__device__ __forceinline__ int32_t shfl_up(int32_t v, int d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ int64_t shfl_up(int64_t v, int d) {
  const uint32_t lo = (uint32_t)__shfl_up((int32_t)(uint32_t)v, d, 64);
  const uint32_t hi = (uint32_t)__shfl_up((int32_t)(uint32_t)((uint64_t)v >> 32), d, 64);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t shfl_down64(int64_t v, int d) {
  const uint32_t lo = (uint32_t)__shfl_down((int32_t)(uint32_t)v, d, 64);
  const uint32_t hi = (uint32_t)__shfl_down((int32_t)(uint32_t)((uint64_t)v >> 32), d, 64);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Exclusive prefix sum over the block (blockDim a multiple of 64, at most
// 1024); lds holds one value per wave.  Returns the thread's prefix and sets
// *total.  Ends with a barrier, so lds may be reused at once.
template <class T>
__device__ T block_excl_scan(T v, T *lds, T *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const T u = shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const T x = lds[i];
    if (i < w) off += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// The item count: *dn when given (never above the bound n), else n.
__device__ __forceinline__ int64_t item_count(int64_t n, const int64_t *dn) {
  if (!dn) return n;
  const int64_t c = *dn;
  return c < n ? c : n;
}

// ------------------------------------------------------------------- scans
constexpr int kScanPer = 8;
constexpr int kScanTile = kBT * kScanPer;

inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

template <class T>
__global__ void __launch_bounds__(kBT) k_scan_reduce(const T *in, int64_t nb, const int64_t *dn, T *sums) {
  __shared__ T lds[kBT / 64];
  const int64_t n = item_count(nb, dn);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t k = base + i * kBT + threadIdx.x;
    if (k < n) s += in[k];
  }
  T tot;
  block_excl_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive prefix of the tile sums in place; the grand total goes
// to out[n] (n the item count).
template <class T>
__global__ void __launch_bounds__(kBT) k_scan_sums(T *sums, int64_t ntb, int64_t nb, const int64_t *dn, T *out) {
  __shared__ T lds[kBT / 64];
  const int64_t n = item_count(nb, dn);
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  T carry = 0;
  for (int64_t b = 0; b < nt; b += kBT) {
    const int64_t k = b + threadIdx.x;
    const T v = k < nt ? sums[k] : T(0);
    T tot;
    const T ex = block_excl_scan(v, lds, &tot);
    if (k < nt) sums[k] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
  (void)ntb;
}

// Each thread takes kScanPer consecutive items (in and out may alias).
template <class T>
__global__ void __launch_bounds__(kBT) k_scan_down(const T *in, T *out, int64_t nb, const int64_t *dn, const T *sums) {
  __shared__ T lds[kBT / 64];
  const int64_t n = item_count(nb, dn);
  if ((int64_t)blockIdx.x * kScanTile >= n) return;  // uniform per block
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  T v[kScanPer];
  T s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = base + i < n ? in[base + i] : T(0);
    s += v[i];
  }
  T tot;
  T ex = block_excl_scan(s, lds, &tot) + sums[blockIdx.x];
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

// Scratch of a scan over at most n items, in T.
inline int64_t scan_scratch(int64_t n) { return scan_tiles(n) + 1; }

// out[0..c] = exclusive prefix sums of in[0..c), out[c] = the total, where c
// = *dn if dn is given (at most n) else n; in may be out.  sums: scan_scratch(n)
// entries.  Enqueued on s; the caller checks hipGetLastError.
template <class T>
void scan(hipStream_t s, const T *in, T *out, int64_t n, const int64_t *dn, T *sums) {
  const int64_t nt = scan_tiles(n);
  if (nt) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_reduce<T>), dim3(nt), dim3(kBT), 0, s, in, n, dn, sums);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_sums<T>), dim3(1), dim3(kBT), 0, s, sums, nt, n, dn, out);
  if (nt) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_down<T>), dim3(nt), dim3(kBT), 0, s, in, out, n, dn, sums);
}

// ------------------------------------------------------------- radix sort
// Stable LSD sort of keys (uint32_t or uint64_t), with or without int32
// values, 8 bits per pass.  Within a tile of 4096 items, items are ranked
// round by round (256 per round, in index order); equal digits inside a wave
// are found with eight ballots.
constexpr int kSortPer = 16;
constexpr int kSortTile = kBT * kSortPer;

inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

template <class K>
__global__ void __launch_bounds__(kBT) k_sort_hist(const K *keys, int64_t nb, const int64_t *dn, int shift,
                                                   int32_t *hist, int64_t ntiles) {
  __shared__ int32_t cnt[256];
  const int64_t n = item_count(nb, dn);
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortPer; ++r) {
    const int64_t k = base + r * kBT + threadIdx.x;
    if (k < n) atomicAdd(&cnt[(int)((keys[k] >> shift) & 255u)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

template <class K, bool VALS>
__global__ void __launch_bounds__(kBT) k_sort_scatter(const K *kin, const int32_t *vin, K *kout, int32_t *vout,
                                                      int64_t nb, const int64_t *dn, int shift, const int32_t *offs,
                                                      int64_t ntiles) {
  __shared__ int32_t base[256];
  __shared__ int32_t wc[kBT / 64][256];
  const int64_t n = item_count(nb, dn);
  if ((int64_t)blockIdx.x * kSortTile >= n) return;  // uniform per block
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  base[t] = offs[(int64_t)t * ntiles + blockIdx.x];
  for (int i = 0; i < kBT / 64; ++i) wc[i][t] = 0;
  __syncthreads();
  const uint64_t below = (uint64_t(1) << lane) - 1;
  for (int r = 0; r < kSortPer; ++r) {
    const int64_t k = (int64_t)blockIdx.x * kSortTile + r * kBT + t;
    const bool ok = k < n;
    const K key = ok ? kin[k] : K(0);
    int32_t val = 0;
    if (VALS && ok) val = vin[k];
    const int d = (int)((key >> shift) & 255u);
    uint64_t m = __ballot(ok);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const int rank = __popcll(m & below);
    if (ok && rank == 0) wc[w][d] = __popcll(m);
    __syncthreads();
    if (ok) {
      int32_t pos = base[d] + rank;
      for (int i = 0; i < w; ++i) pos += wc[i][d];
      kout[pos] = key;
      if (VALS) vout[pos] = val;
    }
    __syncthreads();
    int32_t add = 0;
    for (int i = 0; i < kBT / 64; ++i) {
      add += wc[i][t];
      wc[i][t] = 0;
    }
    base[t] += add;
    __syncthreads();
  }
}

// Scratch of a sort of at most n items: histogram (int32) entries.
inline int64_t sort_hist_entries(int64_t n) { return 256 * sort_tiles(n) + 1; }

// Stable sort by the low `bits` bits of the keys; c = *dn (at most n) or n
// items.  Ping-pongs between (keys, vals) and (k2, v2); returns whether the
// result ended in (k2, v2) (an odd number of passes).  hist:
// sort_hist_entries(n) int32; hsums: scan_scratch(256 * sort_tiles(n)) int32.
template <class K, bool VALS>
bool sort_pairs(hipStream_t s, K *keys, int32_t *vals, K *k2, int32_t *v2, int64_t n, const int64_t *dn, int bits,
                int32_t *hist, int32_t *hsums) {
  const int64_t nt = sort_tiles(n);
  if (nt == 0) return false;
  K *ka = keys, *kb = k2;
  int32_t *va = vals, *vb = v2;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_sort_hist<K>), dim3(nt), dim3(kBT), 0, s, ka, n, dn, shift, hist, nt);
    scan<int32_t>(s, hist, hist, 256 * nt, nullptr, hsums);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_sort_scatter<K, VALS>), dim3(nt), dim3(kBT), 0, s, ka, va, kb, vb, n, dn,
                       shift, hist, nt);
    K *tk = ka;
    ka = kb;
    kb = tk;
    int32_t *tv = va;
    va = vb;
    vb = tv;
  }
  return passes & 1;
}

// ------------------------------------------- radix sort on a fixed grid
// The same stable sort for an item count known only on the device: a fixed
// grid of G blocks, block b taking the contiguous items [b * chunk, (b + 1) *
// chunk) with chunk = ceil(count / G), so the histogram holds 256 x G entries
// whatever the bound.
constexpr int kFixedBlocks = 1024;
static_assert(kFixedBlocks == 4 * kBT, "a histogram row is scanned by one block, four entries a thread");

__device__ __forceinline__ void fixed_range(int64_t nb, const int64_t *dn, int64_t &lo, int64_t &hi) {
  const int64_t n = item_count(nb, dn);
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  lo = (int64_t)blockIdx.x * chunk;
  hi = lo + chunk < n ? lo + chunk : n;
}

template <class K>
__global__ void __launch_bounds__(kBT) k_fsort_hist(const K *keys, int64_t nb, const int64_t *dn, int shift,
                                                    int32_t *hist) {
  __shared__ int32_t cnt[256];
  int64_t lo, hi;
  fixed_range(nb, dn, lo, hi);
  cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t k = lo + threadIdx.x; k < hi; k += kBT) atomicAdd(&cnt[(int)((keys[k] >> shift) & 255u)], 1);
  __syncthreads();
  hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Row d of the histogram (the G blocks' counts of digit d) to its exclusive
// prefix sums, the row total to tot[d]; one block per digit, thread t holding
// entries 4 t .. 4 t + 3.
__global__ void __launch_bounds__(kBT) k_fsort_rows(int32_t *hist, int32_t *tot) {
  __shared__ int32_t lds[kBT / 64];
  int4 *row = reinterpret_cast<int4 *>(hist + (int64_t)blockIdx.x * kFixedBlocks);
  const int4 v = row[threadIdx.x];
  int32_t total;
  const int32_t ex = block_excl_scan(v.x + v.y + v.z + v.w, lds, &total);
  row[threadIdx.x] = make_int4(ex, ex + v.x, ex + v.x + v.y, ex + v.x + v.y + v.z);
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

template <class K, bool VALS>
__global__ void __launch_bounds__(kBT) k_fsort_scatter(const K *kin, const int32_t *vin, K *kout, int32_t *vout,
                                                       int64_t nb, const int64_t *dn, int shift,
                                                       const int32_t *offs, const int32_t *tot) {
  __shared__ int32_t base[256];
  __shared__ int32_t wc[kBT / 64][256];
  int64_t lo, hi;
  fixed_range(nb, dn, lo, hi);
  if (lo >= hi) return;  // uniform per block
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  {
    // digit t starts after every item of a smaller digit and after digit t's
    // items of the blocks before this one
    int32_t all;
    const int32_t below_digit = block_excl_scan(tot[t], &wc[0][0], &all);
    base[t] = below_digit + offs[(int64_t)t * gridDim.x + blockIdx.x];
  }
  for (int i = 0; i < kBT / 64; ++i) wc[i][t] = 0;
  __syncthreads();
  const uint64_t below = (uint64_t(1) << lane) - 1;
  for (int64_t r0 = lo; r0 < hi; r0 += kBT) {
    const int64_t k = r0 + t;
    const bool ok = k < hi;
    const K key = ok ? kin[k] : K(0);
    int32_t val = 0;
    if (VALS && ok) val = vin[k];
    const int d = (int)((key >> shift) & 255u);
    uint64_t m = __ballot(ok);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const int rank = __popcll(m & below);
    if (ok && rank == 0) wc[w][d] = __popcll(m);
    __syncthreads();
    if (ok) {
      int32_t pos = base[d] + rank;
      for (int i = 0; i < w; ++i) pos += wc[i][d];
      kout[pos] = key;
      if (VALS) vout[pos] = val;
    }
    __syncthreads();
    int32_t add = 0;
    for (int i = 0; i < kBT / 64; ++i) {
      add += wc[i][t];
      wc[i][t] = 0;
    }
    base[t] += add;
    __syncthreads();
  }
}

// In-place exclusive scan of a small array (n <= CH * 4096) by one block of
// 1024 threads, the total to a[n]: thread t holds items 4 t .. 4 t + 3 of
// every chunk of 4096 (all requested before the first is used), the chunks
// are scanned in order.
template <class T, int CH>
__global__ void __launch_bounds__(1024) k_scan_one_block(T *a, int64_t n) {
  __shared__ T lds[16];
  T v[CH][4];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = (int64_t)c * 4096 + 4 * threadIdx.x + q;
      v[c][q] = i < n ? a[i] : T(0);
    }
  T carry = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    T tot;
    T ex = block_excl_scan(v[c][0] + v[c][1] + v[c][2] + v[c][3], lds, &tot) + carry;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = (int64_t)c * 4096 + 4 * threadIdx.x + q;
      if (i < n) a[i] = ex;
      ex += v[c][q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) a[n] = carry;
}

// Scratch of the fixed-grid sort: the histogram (int32 entries).
constexpr int64_t kFixedHist = 256 * (int64_t)kFixedBlocks + 256;

// As sort_pairs, for counts in device memory: any bound, constant scratch
// (hist: kFixedHist entries).
template <class K, bool VALS>
bool sort_pairs_fixed(hipStream_t s, K *keys, int32_t *vals, K *k2, int32_t *v2, int64_t n, const int64_t *dn,
                      int bits, int32_t *hist) {
  if (n <= 0) return false;
  K *ka = keys, *kb = k2;
  int32_t *va = vals, *vb = v2;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    int32_t *tot = hist + 256 * (int64_t)kFixedBlocks;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fsort_hist<K>), dim3(kFixedBlocks), dim3(kBT), 0, s, ka, n, dn, shift, hist);
    hipLaunchKernelGGL(k_fsort_rows, dim3(256), dim3(kBT), 0, s, hist, tot);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fsort_scatter<K, VALS>), dim3(kFixedBlocks), dim3(kBT), 0, s, ka, va, kb, vb,
                       n, dn, shift, (const int32_t *)hist, (const int32_t *)tot);
    K *tk = ka;
    ka = kb;
    kb = tk;
    int32_t *tv = va;
    va = vb;
    vb = tv;
  }
  return passes & 1;
}

// ------------------------------------------- unique of sorted keys, fixed grid
// The first of each run of equal keys among the c = *dn sorted keys, kept in
// order: block b counts the run starts of its contiguous chunk, one block
// scans the G counts, block b writes its run starts at its offset; the number
// of unique keys goes to *m.
template <class K>
__device__ __forceinline__ bool run_start(const K *k, int64_t i) { return i == 0 || k[i] != k[i - 1]; }

template <class K>
__global__ void __launch_bounds__(kBT) k_funique_count(const K *k, int64_t nb, const int64_t *dn, int64_t *cnt) {
  __shared__ int64_t lds[kBT / 64];
  int64_t lo, hi;
  fixed_range(nb, dn, lo, hi);
  int64_t c = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) c += run_start(k, i);
  int64_t tot;
  block_excl_scan(c, lds, &tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

template <class K>
__global__ void __launch_bounds__(kBT) k_funique_write(const K *k, int64_t nb, const int64_t *dn,
                                                       const int64_t *off, K *out, long long *m) {
  __shared__ int64_t lds[kBT / 64];
  int64_t lo, hi;
  fixed_range(nb, dn, lo, hi);
  if (blockIdx.x == 0 && threadIdx.x == 0) *m = off[gridDim.x];
  int64_t base = off[blockIdx.x];
  for (int64_t r0 = lo; r0 < hi; r0 += kBT) {  // rounds in index order
    const int64_t i = r0 + threadIdx.x;
    const int64_t f = i < hi && run_start(k, i);
    int64_t tot;
    const int64_t o = block_excl_scan(f, lds, &tot);
    if (f) out[base + o] = k[i];
    base += tot;
  }
}

// scratch: kFixedBlocks + 1 int64
template <class K>
void unique_fixed(hipStream_t s, const K *k, int64_t n, const int64_t *dn, K *out, long long *m, int64_t *cnt) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_funique_count<K>), dim3(kFixedBlocks), dim3(kBT), 0, s, k, n, dn, cnt);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_one_block<int64_t, 1>), dim3(1), dim3(1024), 0, s, cnt,
                     (int64_t)kFixedBlocks);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_funique_write<K>), dim3(kFixedBlocks), dim3(kBT), 0, s, k, n, dn,
                     (const int64_t *)cnt, out, m);
}

}  // namespace
}  // namespace pmrf_prims
