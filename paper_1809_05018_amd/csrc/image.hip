// Image in, segmentation out: the region adjacency graph and region means of
// an oversegmented image (the graph the EM loop consumes), labels painted back
// onto the pixels, and the confusion counts behind the paper's verification
// metrics (Sec. 4.1.2).
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
constexpr int kRunPixels = 16;  // pixels of one row per thread in the region sums

// Workspace of pmrf_image_graph, in 256-byte aligned pieces.
struct ImgPlan {
  int64_t pairs = 0;                   // upper bound on boundary pixel pairs
  size_t keys_a = 0, keys_b = 0;       // uint64[2 * pairs] each
  size_t sums = 0, counts = 0;         // int64[n] each
  size_t scalars = 0;                  // int64[4]: pair count, unique count, bad ids, spare
  size_t temp = 0, temp_bytes = 0;     // hipCUB scratch
  size_t total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

ImgPlan plan_image(int64_t width, int64_t height, int64_t n) {
  ImgPlan p;
  p.pairs = std::max<int64_t>(1, height * std::max<int64_t>(0, width - 1) + std::max<int64_t>(0, height - 1) * width);
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
  size_t sort_bytes = 0, uniq_bytes = 0;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)keys);
  (void)hipcub::DeviceSelect::Unique(nullptr, uniq_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                               (int64_t *)nullptr, (int)keys);
  p.temp = off;
  p.temp_bytes = std::max<size_t>(256, std::max(sort_bytes, uniq_bytes));
  off = align256(off + p.temp_bytes);
  p.total = off;
  return p;
}

// Boundary pairs: pixel (r, c) against its right and lower neighbours; a pair
// of different regions becomes the key (min << 32) | max.  Slots are taken
// with one atomic per wave (ballot + rank), so the list is complete but in no
// particular order (it is sorted next).  Ids outside [0, n) are counted.
__global__ __launch_bounds__(kImgThreads) void k_boundary(const int32_t *__restrict__ reg, int32_t width,
                                                           int32_t height, int32_t n, uint64_t *__restrict__ keys,
                                                           unsigned long long *__restrict__ scal) {
  const int64_t npix = (int64_t)width * height;
  const int lane = threadIdx.x & 63;
  for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x; p0 < npix; p0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = p0 + threadIdx.x;
    bool right = false, down = false, bad = false;
    uint64_t kr = 0, kd = 0;
    if (p < npix) {
      const int32_t r = (int32_t)(p / width), c = (int32_t)(p - (int64_t)r * width);
      const int32_t u = reg[p];
      bad = u < 0 || u >= n;
      if (c + 1 < width) {
        const int32_t v = reg[p + 1];
        bad |= v < 0 || v >= n;
        right = u != v;
        kr = ((uint64_t)(uint32_t)min(u, v) << 32) | (uint32_t)max(u, v);
      }
      if (r + 1 < height) {
        const int32_t v = reg[p + width];
        bad |= v < 0 || v >= n;
        down = u != v;
        kd = ((uint64_t)(uint32_t)min(u, v) << 32) | (uint32_t)max(u, v);
      }
    }
    const uint64_t br = __ballot(right), bd = __ballot(down), bb = __ballot(bad);
    const int cnt = __popcll(br) + __popcll(bd);
    unsigned long long base = 0;
    if (lane == 0) {
      if (cnt) base = atomicAdd(&scal[0], (unsigned long long)cnt);
      if (bb) atomicAdd(&scal[2], (unsigned long long)__popcll(bb));
    }
    base = __shfl(base, 0);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int rank_r = __popcll(br & below);
    const int rank_d = __popcll(br) + __popcll(bd & below);
    if (right) keys[base + rank_r] = kr;
    if (down) keys[base + rank_d] = kd;
  }
}

// Directed edges: unique pair i = (a, b) gives (a, b) and (b, a).
__global__ __launch_bounds__(kImgThreads) void k_expand(const uint64_t *__restrict__ uniq, int64_t m,
                                                         uint64_t *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = uniq[i];
    out[2 * i] = k;
    out[2 * i + 1] = (k << 32) | (k >> 32);
  }
}

// CSR from the sorted directed edges: row_ptr[r] = first edge whose row is
// >= r (binary search), col_idx = the low halves in order.
__global__ __launch_bounds__(kImgThreads) void k_csr(const uint64_t *__restrict__ e, int64_t nnz, int32_t n,
                                                      int32_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride)
    col_idx[i] = (int32_t)(uint32_t)(e[i] & 0xffffffffull);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += stride) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)(e[mid] >> 32) < r) lo = mid + 1;
      else hi = mid;
    }
    row_ptr[r] = (int32_t)lo;
  }
}

__global__ __launch_bounds__(kImgThreads) void k_zero64(long long *__restrict__ a, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// Pixel sums and counts per region: a thread walks kRunPixels pixels of one
// row and adds each run of equal ids with one integer atomic (integer sums,
// so the totals do not depend on the order of the atomics).  Ids outside
// [0, n) are skipped (k_boundary has counted them).
__global__ __launch_bounds__(kImgThreads) void k_region_sums(const int32_t *__restrict__ reg,
                                                              const uint8_t *__restrict__ pix, int32_t width,
                                                              int32_t height, int32_t n,
                                                              unsigned long long *__restrict__ sums,
                                                              unsigned long long *__restrict__ counts) {
  const int64_t runs_per_row = (width + kRunPixels - 1) / kRunPixels;
  const int64_t runs = runs_per_row * height;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < runs; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / runs_per_row;
    const int32_t c0 = (int32_t)(t - r * runs_per_row) * kRunPixels;
    const int32_t c1 = min(width, c0 + kRunPixels);
    const int64_t row = r * width;
    int32_t cur = -1;
    unsigned long long s = 0, k = 0;
    for (int32_t c = c0; c < c1; ++c) {
      const int32_t u = reg[row + c];
      if (u != cur) {
        if (k && cur >= 0 && cur < n) {
          atomicAdd(&sums[cur], s);
          atomicAdd(&counts[cur], k);
        }
        cur = u;
        s = 0;
        k = 0;
      }
      s += pix[row + c];
      k += 1;
    }
    if (k && cur >= 0 && cur < n) {
      atomicAdd(&sums[cur], s);
      atomicAdd(&counts[cur], k);
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

extern "C" pmrf_status pmrf_image_graph_workspace_bytes(int32_t width, int32_t height, int32_t n, int64_t *bytes) {
  clear_error();
  if (!bytes) return fail(PMRF_EINVAL, "NULL argument");
  if (width < 0 || height < 0 || n < 0) return fail(PMRF_EINVAL, "negative size");
  if ((int64_t)width * height > (int64_t)1 << 28) return fail(PMRF_EUNSUPPORTED, "more than 2^28 pixels");
  *bytes = (int64_t)plan_image(width, height, n).total;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_image_graph(const int32_t *d_regions, const uint8_t *d_pixels, int32_t width,
                                        int32_t height, int32_t n, int32_t *d_row_ptr, int32_t *d_col_idx,
                                        int64_t col_capacity, double *d_means, int64_t *nnz, void *d_ws,
                                        int64_t ws_bytes, void *hip_stream) {
  clear_error();
  if (!nnz || !d_row_ptr || (n > 0 && !d_means)) return fail(PMRF_EINVAL, "NULL argument");
  if (width < 0 || height < 0 || n < 0 || col_capacity < 0) return fail(PMRF_EINVAL, "negative size");
  const int64_t npix = (int64_t)width * height;
  if (npix > (int64_t)1 << 28) return fail(PMRF_EUNSUPPORTED, "more than 2^28 pixels");
  if (npix > 0 && (!d_regions || !d_pixels)) return fail(PMRF_EINVAL, "NULL image");
  if (npix > 0 && n == 0) return fail(PMRF_EINVAL, "pixels but no regions");
  const ImgPlan plan = plan_image(width, height, n);
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
  if (npix > 0) {
    hipLaunchKernelGGL(k_boundary, dim3(grid_for(npix)), dim3(kImgThreads), 0, s, d_regions, width, height, n, ka,
                       scal);
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
    IMG_TRY(hipcub::DeviceRadixSort::SortKeys(temp, tb, (const uint64_t *)ka, kb, (int)pairs, 0, 64, s));
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
    hipLaunchKernelGGL(k_expand, dim3(grid_for(m)), dim3(kImgThreads), 0, s, (const uint64_t *)ka, m, kb);
    IMG_TRY(hipGetLastError());
    size_t tb = plan.temp_bytes;
    IMG_TRY(hipcub::DeviceRadixSort::SortKeys(temp, tb, (const uint64_t *)kb, ka, (int)edges, 0, 64, s));
  }
  hipLaunchKernelGGL(k_csr, dim3(grid_for(std::max<int64_t>(edges, (int64_t)n + 1))), dim3(kImgThreads), 0, s,
                     (const uint64_t *)ka, edges, n, d_row_ptr, d_col_idx);
  IMG_TRY(hipGetLastError());
  if (npix > 0) {
    const int64_t runs = (int64_t)height * ((width + kRunPixels - 1) / kRunPixels);
    hipLaunchKernelGGL(k_region_sums, dim3(grid_for(runs)), dim3(kImgThreads), 0, s, d_regions, d_pixels, width,
                       height, n, sums, counts);
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
