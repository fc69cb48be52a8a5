// Image in, segmentation out: the region adjacency graph and region means of
// an oversegmented image (the graph the EM loop consumes), labels painted back
// onto the pixels, and the confusion counts behind the paper's verification
// metrics (Sec. 4.2.1).
//
// The graph: regions u != v are adjacent when some pixel of u and some pixel
// of v are horizontal or vertical neighbours (4-connectivity); the CSR is
// symmetric with every row ascending.  The mean of a region is the sum of its
// pixel values over its pixel count, in FP64 (sums are exact integers).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <string>

#include "pmrf_internal.h"

using pmrf::clear_error;
using pmrf::fail;

#define IMG_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(PMRF_EDEVICE, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr int kImgThreads = 256;
constexpr int kWavePixels = 64 * 16;  // consecutive pixels per wave in the boundary passes

int64_t boundary_waves(int64_t npix) { return std::max<int64_t>(1, (npix + kWavePixels - 1) / kWavePixels); }

// Keys pack a pair of region ids as (first << B) | second with B the bit width
// of n - 1 (at least 1), so the sorts look at 2B bits only.
int id_bits(int64_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// Workspace of pmrf_image_graph, in 256-byte aligned pieces.
struct ImgPlan {
  int64_t pairs = 0;                   // upper bound on boundary pixel pairs
  size_t keys_a = 0, keys_b = 0;       // uint64[2 * pairs] each
  size_t sums = 0, counts = 0;         // int64[n] each
  size_t scalars = 0;                  // int64[4]: pair count, unique count, bad ids, spare
  size_t wcount = 0, woff = 0;         // uint32[boundary waves] each: pairs per wave, their offsets
  size_t temp = 0, temp_bytes = 0;     // hipCUB scratch
  size_t total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

ImgPlan plan_image(int64_t width, int64_t height, int64_t depth, int64_t n) {
  ImgPlan p;
  const int64_t w1 = std::max<int64_t>(0, width - 1), h1 = std::max<int64_t>(0, height - 1),
                d1 = std::max<int64_t>(0, depth - 1);
  p.pairs = std::max<int64_t>(1, depth * height * w1 + depth * h1 * width + d1 * height * width);
  const int64_t keys = 2 * p.pairs;  // both directions of every unique pair fit as well
  size_t off = 0;
  p.keys_a = off;
  off = align256(off + (size_t)keys * 8);
  p.keys_b = off;
  off = align256(off + (size_t)keys * 8);
  p.sums = off;
  off = align256(off + (size_t)std::max<int64_t>(1, n) * 8);
  p.counts = off;
  off = align256(off + (size_t)std::max<int64_t>(1, n) * 8);
  p.scalars = off;
  off = align256(off + 4 * 8);
  const int64_t waves = boundary_waves(width * height * depth);
  p.wcount = off;
  off = align256(off + (size_t)waves * 4);
  p.woff = off;
  off = align256(off + (size_t)waves * 4);
  size_t sort_bytes = 0, uniq_bytes = 0, scan_bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                         (int)waves);
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)keys);
  (void)hipcub::DeviceSelect::Unique(nullptr, uniq_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                               (int64_t *)nullptr, (int)keys);
  p.temp = off;
  p.temp_bytes = std::max<size_t>(256, std::max(scan_bytes, std::max(sort_bytes, uniq_bytes)));
  off = align256(off + p.temp_bytes);
  p.total = off;
  return p;
}

// Boundary pairs: pixel (r, c) against its right and lower neighbour; a pair
// of different regions becomes the key (min << B) | max.  Two passes over
// the same pixels: wave w takes pixels [w * kWavePixels, (w + 1) *
// kWavePixels), 64 at a time; the first pass counts its pairs, an exclusive
// scan turns the counts into offsets, the second pass writes the keys there in
// pixel order (right, then lower, then next-slice pairs within each 64
// pixels), ranks from ballots.  A volume (depth > 1) adds the neighbour in the
// next slice (6-connectivity).  Ids outside [0, n) are counted by the first
// pass.
struct PixelPairs {
  bool right, down, back, bad;
  uint64_t kr, kd, kb;
};

__device__ __forceinline__ PixelPairs pixel_pairs(const int32_t *__restrict__ reg, int64_t p, int64_t npix,
                                                  int32_t width, int32_t height, int32_t n, int B) {
  PixelPairs q{false, false, false, false, 0, 0, 0};
  if (p < npix) {
    const int64_t plane = (int64_t)width * height;
    const int64_t z = p / plane, rem = p - z * plane;
    const int32_t r = (int32_t)(rem / width), c = (int32_t)(rem - (int64_t)r * width);
    const int32_t u = reg[p];
    q.bad = u < 0 || u >= n;
    if (c + 1 < width) {
      const int32_t v = reg[p + 1];
      q.bad |= v < 0 || v >= n;
      q.right = u != v;
      q.kr = ((uint64_t)(uint32_t)min(u, v) << B) | (uint32_t)max(u, v);
    }
    if (r + 1 < height) {
      const int32_t v = reg[p + width];
      q.bad |= v < 0 || v >= n;
      q.down = u != v;
      q.kd = ((uint64_t)(uint32_t)min(u, v) << B) | (uint32_t)max(u, v);
    }
    if (p + plane < npix) {
      const int32_t v = reg[p + plane];
      q.bad |= v < 0 || v >= n;
      q.back = u != v;
      q.kb = ((uint64_t)(uint32_t)min(u, v) << B) | (uint32_t)max(u, v);
    }
  }
  return q;
}

__global__ __launch_bounds__(kImgThreads) void k_boundary_count(const int32_t *__restrict__ reg, int32_t width,
                                                                 int32_t height, int32_t depth, int32_t n, int B,
                                                                 int64_t waves, uint32_t *__restrict__ wcount,
                                                                 unsigned long long *__restrict__ scal) {
  const int64_t npix = (int64_t)width * height * depth;
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (kImgThreads / 64) + (threadIdx.x >> 6);
  if (w >= waves) return;
  uint32_t cnt = 0, bad = 0;
  for (int i = 0; i < kWavePixels / 64; ++i) {
    const PixelPairs q = pixel_pairs(reg, w * kWavePixels + i * 64 + lane, npix, width, height, n, B);
    cnt += (uint32_t)(__popcll(__ballot(q.right)) + __popcll(__ballot(q.down)) + __popcll(__ballot(q.back)));
    bad += (uint32_t)__popcll(__ballot(q.bad));
  }
  if (lane == 0) {
    wcount[w] = cnt;
    if (bad) atomicAdd(&scal[2], (unsigned long long)bad);
  }
}

__global__ __launch_bounds__(kImgThreads) void k_boundary_emit(const int32_t *__restrict__ reg, int32_t width,
                                                                int32_t height, int32_t depth, int32_t n, int B,
                                                                int64_t waves, const uint32_t *__restrict__ woff,
                                                                uint64_t *__restrict__ keys) {
  const int64_t npix = (int64_t)width * height * depth;
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (kImgThreads / 64) + (threadIdx.x >> 6);
  if (w >= waves) return;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t base = woff[w];
  for (int i = 0; i < kWavePixels / 64; ++i) {
    const PixelPairs q = pixel_pairs(reg, w * kWavePixels + i * 64 + lane, npix, width, height, n, B);
    const uint64_t br = __ballot(q.right), bd = __ballot(q.down), bk = __ballot(q.back);
    if (q.right) keys[base + __popcll(br & below)] = q.kr;
    if (q.down) keys[base + __popcll(br) + __popcll(bd & below)] = q.kd;
    if (q.back) keys[base + __popcll(br) + __popcll(bd) + __popcll(bk & below)] = q.kb;
    base += __popcll(br) + __popcll(bd) + __popcll(bk);
  }
}

// Total pair count from the last wave's offset and count.
__global__ void k_pair_total(const uint32_t *__restrict__ wcount, const uint32_t *__restrict__ woff, int64_t waves,
                             unsigned long long *__restrict__ scal) {
  if (threadIdx.x == 0 && blockIdx.x == 0) scal[0] = (unsigned long long)woff[waves - 1] + wcount[waves - 1];
}

// Directed edges: unique pair i = (a, b) gives (a, b) and (b, a).
__global__ __launch_bounds__(kImgThreads) void k_expand(const uint64_t *__restrict__ uniq, int64_t m, int B,
                                                         uint64_t *__restrict__ out) {
  const uint64_t low = ((uint64_t)1 << B) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = uniq[i];
    out[2 * i] = k;
    out[2 * i + 1] = ((k & low) << B) | (k >> B);
  }
}

// CSR from the sorted directed edges: row_ptr[r] = first edge whose row is
// >= r (binary search), col_idx = the low B bits in order.
__global__ __launch_bounds__(kImgThreads) void k_csr(const uint64_t *__restrict__ e, int64_t nnz, int32_t n, int B,
                                                      int32_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t low = ((uint64_t)1 << B) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride)
    col_idx[i] = (int32_t)(uint32_t)(e[i] & low);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += stride) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)(e[mid] >> B) < r) lo = mid + 1;
      else hi = mid;
    }
    row_ptr[r] = (int32_t)lo;
  }
}

__global__ __launch_bounds__(kImgThreads) void k_zero64(long long *__restrict__ a, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// Pixel sums and counts per region, one block per tile of kTileRows x
// kTileCols pixels; thread t walks kTileCols / 16 consecutive pixels of one
// tile row (16 threads per row) and adds each run of equal ids once.  When
// the valid ids of the tile span fewer than kTileTable values (neighbouring
// regions have neighbouring ids in the usual oversegmentations) the runs are
// added in an LDS table indexed by id - (smallest id) and each non-empty entry
// goes to memory with one atomic; otherwise every run does.  Integer sums, so
// the totals do not depend on the order.  Ids outside [0, n) are skipped
// (k_boundary_count has counted them).
constexpr int kTileRows = kImgThreads / 16, kTileCols = 128, kTileTable = 2048;
constexpr int kTileSeg = kTileCols / 16;  // pixels per thread

__global__ __launch_bounds__(kImgThreads) void k_region_sums(const int32_t *__restrict__ reg,
                                                              const uint8_t *__restrict__ pix, int32_t width,
                                                              int32_t height, int32_t n,
                                                              unsigned long long *__restrict__ sums,
                                                              unsigned long long *__restrict__ counts) {
  __shared__ unsigned long long tsum[kTileTable];
  __shared__ unsigned int tcnt[kTileTable];
  __shared__ int id_lo, id_hi;
  const int64_t tiles_x = (width + kTileCols - 1) / kTileCols;
  const int64_t r = (int64_t)(blockIdx.x / tiles_x) * kTileRows + threadIdx.x / 16;
  const int32_t c0 = (int32_t)(blockIdx.x % tiles_x) * kTileCols + (threadIdx.x % 16) * kTileSeg;
  const int32_t c1 = (r < height) ? min(width, c0 + kTileSeg) : c0;  // empty past the last row
  const int64_t row = r * width;
  if (threadIdx.x == 0) {
    id_lo = 0x7fffffff;
    id_hi = -1;
  }
  __syncthreads();
  int lo = 0x7fffffff, hi = -1;
  for (int32_t c = c0; c < c1; ++c) {
    const int32_t u = reg[row + c];
    if (u >= 0 && u < n) {
      lo = min(lo, u);
      hi = max(hi, u);
    }
  }
  if (hi >= 0) {
    atomicMin(&id_lo, lo);
    atomicMax(&id_hi, hi);
  }
  __syncthreads();
  const int base = id_lo;
  const bool table = id_hi >= 0 && id_hi - base < kTileTable;  // the same for every thread
  if (table) {
    for (int i = threadIdx.x; i < kTileTable; i += blockDim.x) {
      tsum[i] = 0;
      tcnt[i] = 0;
    }
  }
  __syncthreads();
  int32_t cur = -1;
  unsigned long long sm = 0;
  unsigned int k = 0;
  auto flush = [&]() {
    if (k && cur >= 0 && cur < n) {
      if (table) {
        atomicAdd(&tsum[cur - base], sm);
        atomicAdd(&tcnt[cur - base], k);
      } else {
        atomicAdd(&sums[cur], sm);
        atomicAdd(&counts[cur], (unsigned long long)k);
      }
    }
  };
  for (int32_t c = c0; c < c1; ++c) {
    const int32_t u = reg[row + c];
    if (u != cur) {
      flush();
      cur = u;
      sm = 0;
      k = 0;
    }
    sm += pix[row + c];
    k += 1;
  }
  flush();
  if (table) {
    __syncthreads();
    for (int i = threadIdx.x; i <= id_hi - base; i += blockDim.x)
      if (tcnt[i]) {
        atomicAdd(&sums[base + i], tsum[i]);
        atomicAdd(&counts[base + i], (unsigned long long)tcnt[i]);
      }
  }
}

__global__ __launch_bounds__(kImgThreads) void k_means(const unsigned long long *__restrict__ sums,
                                                        const unsigned long long *__restrict__ counts, int32_t n,
                                                        double *__restrict__ means) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    means[r] = counts[r] ? (double)sums[r] / (double)counts[r] : 0.0;
}

__global__ __launch_bounds__(kImgThreads) void k_paint(const int32_t *__restrict__ reg,
                                                        const int32_t *__restrict__ labels, int64_t npix, int32_t n,
                                                        uint8_t *__restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = reg[p];
    const int32_t l = (u >= 0 && u < n) ? labels[u] : -1;
    out[p] = (l >= 0 && l < 255) ? (uint8_t)l : (uint8_t)255;
  }
}

// Confusion counts: counts[a * k + b] = #pixels with a[p] = a, b[p] = b (both
// below k <= 16).  A block histogram in LDS, then one integer atomic per bin.
__global__ __launch_bounds__(kImgThreads) void k_confusion(const uint8_t *__restrict__ a,
                                                            const uint8_t *__restrict__ b, int64_t npix, int32_t k,
                                                            unsigned long long *__restrict__ counts) {
  __shared__ unsigned int hist[16 * 16];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    const int x = a[p], y = b[p];
    if (x < k && y < k) atomicAdd(&hist[x * k + y], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k * k; i += blockDim.x)
    if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

int grid_for(int64_t work, int per_cu = 8) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int64_t need = (work + kImgThreads - 1) / kImgThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * per_cu));
}

}  // namespace

namespace {

pmrf_status workspace_bytes(int32_t width, int32_t height, int32_t depth, int32_t n, int64_t *bytes) {
  clear_error();
  if (!bytes) return fail(PMRF_EINVAL, "NULL argument");
  if (width < 0 || height < 0 || depth < 0 || n < 0) return fail(PMRF_EINVAL, "negative size");
  if ((int64_t)width * height * depth > (int64_t)1 << 28) return fail(PMRF_EUNSUPPORTED, "more than 2^28 pixels");
  *bytes = (int64_t)plan_image(width, height, depth, n).total;
  return PMRF_OK;
}

// The region graph and means of a depth x height x width volume (an image is
// the volume of depth 1).
pmrf_status region_graph(const int32_t *d_regions, const uint8_t *d_pixels, int32_t width, int32_t height,
                         int32_t depth, int32_t n, int32_t *d_row_ptr, int32_t *d_col_idx, int64_t col_capacity,
                         double *d_means, int64_t *nnz, void *d_ws, int64_t ws_bytes, void *hip_stream) {
  clear_error();
  if (!nnz || !d_row_ptr || (n > 0 && !d_means)) return fail(PMRF_EINVAL, "NULL argument");
  if (width < 0 || height < 0 || depth < 0 || n < 0 || col_capacity < 0) return fail(PMRF_EINVAL, "negative size");
  if ((int64_t)width * height * depth > (int64_t)1 << 28) return fail(PMRF_EUNSUPPORTED, "more than 2^28 pixels");
  const int64_t npix = (int64_t)width * height * depth;
  if (npix > (int64_t)1 << 28) return fail(PMRF_EUNSUPPORTED, "more than 2^28 pixels");
  if (npix > 0 && (!d_regions || !d_pixels)) return fail(PMRF_EINVAL, "NULL image");
  if (npix > 0 && n == 0) return fail(PMRF_EINVAL, "pixels but no regions");
  const ImgPlan plan = plan_image(width, height, depth, n);
  if (!d_ws || ws_bytes < (int64_t)plan.total)
    return fail(PMRF_ENOMEM, "workspace smaller than pmrf_image_graph_workspace_bytes");
  hipStream_t s = (hipStream_t)hip_stream;
  char *ws = (char *)d_ws;
  uint64_t *ka = (uint64_t *)(ws + plan.keys_a), *kb = (uint64_t *)(ws + plan.keys_b);
  unsigned long long *sums = (unsigned long long *)(ws + plan.sums), *counts = (unsigned long long *)(ws + plan.counts);
  unsigned long long *scal = (unsigned long long *)(ws + plan.scalars);
  void *temp = ws + plan.temp;

  hipLaunchKernelGGL(k_zero64, dim3(grid_for(2 * std::max(1, n) + 4)), dim3(kImgThreads), 0, s, (long long *)sums,
                     (int64_t)(plan.counts - plan.sums) / 8 + std::max<int64_t>(1, n));
  IMG_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_zero64, dim3(1), dim3(kImgThreads), 0, s, (long long *)scal, (int64_t)4);
  IMG_TRY(hipGetLastError());
  const int64_t waves = boundary_waves(npix);
  const int B = id_bits(n);
  uint32_t *wcount = (uint32_t *)(ws + plan.wcount), *woff = (uint32_t *)(ws + plan.woff);
  if (npix > 0) {
    const int blocks = (int)((waves + kImgThreads / 64 - 1) / (kImgThreads / 64));
    hipLaunchKernelGGL(k_boundary_count, dim3(blocks), dim3(kImgThreads), 0, s, d_regions, width, height, depth, n,
                       B, waves, wcount, scal);
    IMG_TRY(hipGetLastError());
    size_t tb = plan.temp_bytes;
    IMG_TRY(hipcub::DeviceScan::ExclusiveSum(temp, tb, (const uint32_t *)wcount, woff, (int)waves, s));
    hipLaunchKernelGGL(k_pair_total, dim3(1), dim3(64), 0, s, (const uint32_t *)wcount, (const uint32_t *)woff,
                       waves, scal);
    IMG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_boundary_emit, dim3(blocks), dim3(kImgThreads), 0, s, d_regions, width, height, depth, n,
                       B, waves, (const uint32_t *)woff, ka);
    IMG_TRY(hipGetLastError());
  }
  unsigned long long host_scal[4] = {0, 0, 0, 0};
  IMG_TRY(hipMemcpyAsync(host_scal, scal, sizeof(host_scal), hipMemcpyDeviceToHost, s));
  IMG_TRY(hipStreamSynchronize(s));
  if (host_scal[2]) return fail(PMRF_EINVAL, "region id outside [0, n)");
  const int64_t pairs = (int64_t)host_scal[0];
  int64_t m = 0;  // unique undirected pairs
  if (pairs > 0) {
    size_t tb = plan.temp_bytes;
    IMG_TRY(hipcub::DeviceRadixSort::SortKeys(temp, tb, (const uint64_t *)ka, kb, (int)pairs, 0, 2 * B, s));
    tb = plan.temp_bytes;
    IMG_TRY(hipcub::DeviceSelect::Unique(temp, tb, (const uint64_t *)kb, ka, (int64_t *)(scal + 1), (int)pairs, s));
    IMG_TRY(hipMemcpyAsync(host_scal, scal, sizeof(host_scal), hipMemcpyDeviceToHost, s));
    IMG_TRY(hipStreamSynchronize(s));
    m = (int64_t)host_scal[1];
  }
  const int64_t edges = 2 * m;
  if (edges > col_capacity) {
    *nnz = edges;
    return fail(PMRF_ENOMEM, "col_idx capacity below the number of adjacency entries (returned in *nnz)");
  }
  if (edges > 0 && !d_col_idx) return fail(PMRF_EINVAL, "NULL col_idx");
  if (m > 0) {
    hipLaunchKernelGGL(k_expand, dim3(grid_for(m)), dim3(kImgThreads), 0, s, (const uint64_t *)ka, m, B, kb);
    IMG_TRY(hipGetLastError());
    size_t tb = plan.temp_bytes;
    IMG_TRY(hipcub::DeviceRadixSort::SortKeys(temp, tb, (const uint64_t *)kb, ka, (int)edges, 0, 2 * B, s));
  }
  hipLaunchKernelGGL(k_csr, dim3(grid_for(std::max<int64_t>(edges, (int64_t)n + 1))), dim3(kImgThreads), 0, s,
                     (const uint64_t *)ka, edges, n, B, d_row_ptr, d_col_idx);
  IMG_TRY(hipGetLastError());
  if (npix > 0) {
    const int64_t rows = (int64_t)height * depth;  // the sums walk rows; slices follow one another
    const int64_t tiles = (rows + kTileRows - 1) / kTileRows * (((int64_t)width + kTileCols - 1) / kTileCols);
    hipLaunchKernelGGL(k_region_sums, dim3((unsigned)tiles), dim3(kImgThreads), 0, s, d_regions, d_pixels, width,
                       (int32_t)rows, n, sums, counts);
    IMG_TRY(hipGetLastError());
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_means, dim3(grid_for(n)), dim3(kImgThreads), 0, s, (const unsigned long long *)sums,
                       (const unsigned long long *)counts, n, d_means);
    IMG_TRY(hipGetLastError());
  }
  *nnz = edges;
  return PMRF_OK;
}

}  // namespace

extern "C" pmrf_status pmrf_image_graph_workspace_bytes(int32_t width, int32_t height, int32_t n, int64_t *bytes) {
  return workspace_bytes(width, height, 1, n, bytes);
}

extern "C" pmrf_status pmrf_image_graph(const int32_t *d_regions, const uint8_t *d_pixels, int32_t width,
                                        int32_t height, int32_t n, int32_t *d_row_ptr, int32_t *d_col_idx,
                                        int64_t col_capacity, double *d_means, int64_t *nnz, void *d_ws,
                                        int64_t ws_bytes, void *hip_stream) {
  return region_graph(d_regions, d_pixels, width, height, 1, n, d_row_ptr, d_col_idx, col_capacity, d_means, nnz,
                      d_ws, ws_bytes, hip_stream);
}

extern "C" pmrf_status pmrf_volume_graph_workspace_bytes(int32_t width, int32_t height, int32_t depth, int32_t n,
                                                         int64_t *bytes) {
  return workspace_bytes(width, height, depth, n, bytes);
}

extern "C" pmrf_status pmrf_volume_graph(const int32_t *d_regions, const uint8_t *d_voxels, int32_t width,
                                         int32_t height, int32_t depth, int32_t n, int32_t *d_row_ptr,
                                         int32_t *d_col_idx, int64_t col_capacity, double *d_means, int64_t *nnz,
                                         void *d_ws, int64_t ws_bytes, void *hip_stream) {
  return region_graph(d_regions, d_voxels, width, height, depth, n, d_row_ptr, d_col_idx, col_capacity, d_means,
                      nnz, d_ws, ws_bytes, hip_stream);
}

extern "C" pmrf_status pmrf_labels_to_pixels(const int32_t *d_regions, const int32_t *d_labels, int64_t npixels,
                                             int32_t n, uint8_t *d_out, void *hip_stream) {
  clear_error();
  if (npixels < 0 || n < 0) return fail(PMRF_EINVAL, "negative size");
  if (npixels == 0) return PMRF_OK;
  if (!d_regions || !d_out || (n > 0 && !d_labels)) return fail(PMRF_EINVAL, "NULL argument");
  hipLaunchKernelGGL(k_paint, dim3(grid_for(npixels)), dim3(kImgThreads), 0, (hipStream_t)hip_stream, d_regions,
                     d_labels, npixels, n, d_out);
  IMG_TRY(hipGetLastError());
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_confusion(const uint8_t *d_a, const uint8_t *d_b, int64_t npixels, int32_t k,
                                      int64_t *d_counts, void *hip_stream) {
  clear_error();
  if (npixels < 0 || k < 1 || k > 16) return fail(PMRF_EINVAL, "need npixels >= 0 and 1 <= k <= 16");
  if (!d_counts || (npixels > 0 && (!d_a || !d_b))) return fail(PMRF_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_zero64, dim3(1), dim3(kImgThreads), 0, s, (long long *)d_counts, (int64_t)k * k);
  IMG_TRY(hipGetLastError());
  if (npixels > 0) {
    hipLaunchKernelGGL(k_confusion, dim3(grid_for(npixels, 4)), dim3(kImgThreads), 0, s, d_a, d_b, npixels, k,
                       (unsigned long long *)d_counts);
    IMG_TRY(hipGetLastError());
  }
  return PMRF_OK;
}
