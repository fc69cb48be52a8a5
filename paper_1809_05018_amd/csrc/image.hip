// Image in, segmentation out: the region adjacency graph and region means of
// an oversegmented image (the graph the EM loop consumes), labels painted back
// onto the pixels, and the confusion counts behind the paper's verification
// metrics (Sec. 4.2.1).
//
// The graph: regions u != v are adjacent when some pixel of u and some pixel
// of v are horizontal or vertical neighbours (4-connectivity; a volume adds
// the neighbour in the next slice); the CSR is symmetric with every row
// ascending.  The mean of a region is the sum of its pixel values over its
// pixel count, in FP64 (sums are exact integers).
//
// The graph is built without a host round trip until the end:
//   1. one block per tile of 16 x 128 pixels collects the tile's boundary pairs
//      (min << B | max) in an LDS hash set, so each pair leaves the tile once;
//   2. the tiles' pairs are packed into one list (scan of the tile counts),
//      sorted (LSD radix on 2B bits) and made unique (run starts counted per
//      block of a fixed grid, the counts scanned by one block);
//   3. every unique pair (u, v), u < v, adds to u's forward and v's backward
//      count; row r of the CSR holds its backward neighbours (all below r)
//      then its forward ones (all above r), so the forward part comes straight
//      from the sorted list and only each row's short backward part is sorted.
// One wait brings back the pair count and the bad-id count; only then are
// the caller's outputs written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <string>

#include "pmrf_internal.h"
#include "prims.h"

using pmrf::clear_error;
using pmrf::fail;

#define IMG_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(PMRF_EDEVICE, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

using pmrf_prims::block_excl_scan;

constexpr int kImgThreads = 256;
constexpr int kTileRows = kImgThreads / 16, kTileCols = 128;  // a block's tile
constexpr int kTileSeg = kTileCols / 16;                       // pixels per thread
constexpr int kTilePairs = 3 * kTileRows * kTileCols;          // boundary pairs a tile can hold
// LDS hash set of a tile's pairs: 8 KB, so eight blocks fit a CU and the 2,048
// tiles of a 2048 x 2048 image run in one round (a tile of an oversegmentation
// with ~40-pixel regions holds ~150 distinct pairs; 4096 entries: 26.4 us,
// 1024: 16.9 us on that image).  Pairs that find no slot go out as they are.
constexpr int kTileSet = 1024;
constexpr uint64_t kEmpty = ~0ull;

// Keys pack a pair of region ids as (first << B) | second with B the bit width
// of n - 1 (at least 1), so the sorts look at 2B bits only.
int id_bits(int64_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace of pmrf_image_graph / pmrf_volume_graph, in 256-byte aligned
// pieces; P bounds the boundary pairs, so every list below has room for all.
struct ImgPlan {
  int64_t rows = 0, tiles = 0, P = 0;
  size_t tile_keys = 0;      // uint64[tiles * kTilePairs]: each tile's unique pairs
  size_t tile_off = 0;       // int64[tiles + 1]
  size_t tile_set = 0;       // int32[tiles]: pairs of a tile held in its set part
  size_t keys_a = 0, keys_b = 0;  // uint64[P] each: the pair list and its sort partner
  size_t hist = 0;           // int32: radix histogram
  size_t s64 = 0, s32 = 0;   // scan scratch, int64 and int32
  size_t zero_lo = 0;        // [zero_lo, zero_hi) cleared at the start:
  size_t fdeg = 0, bdeg = 0, cur = 0;  //   int32[n] each: forward run ends, backward counts, fill cursors
  size_t sums = 0, counts = 0;         //   uint64[n] each
  size_t scal = 0;                     //   int64[8]: bad ids, unique pairs
  size_t zero_hi = 0;
  size_t fstart = 0;         // int32[n]: first list index of each row's forward pairs
  size_t rp = 0;             // int32[n + 1]
  size_t col = 0;            // int32[2 P]
  size_t total = 0;
};

ImgPlan plan_image(int64_t width, int64_t height, int64_t depth, int64_t n) {
  namespace pp = pmrf_prims;
  ImgPlan p;
  const int64_t w1 = std::max<int64_t>(0, width - 1), h1 = std::max<int64_t>(0, height - 1),
                d1 = std::max<int64_t>(0, depth - 1);
  p.P = std::max<int64_t>(1, depth * height * w1 + depth * h1 * width + d1 * height * width);
  p.rows = height * depth;
  p.tiles = (p.rows + kTileRows - 1) / kTileRows * ((width + kTileCols - 1) / kTileCols);
  const int64_t n1 = std::max<int64_t>(1, n);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + std::max<size_t>(bytes, 8));
    return at;
  };
  p.tile_keys = take((size_t)std::max<int64_t>(1, p.tiles) * kTilePairs * 8);
  p.tile_off = take((size_t)(p.tiles + 1) * 8);
  p.tile_set = take((size_t)std::max<int64_t>(1, p.tiles) * 4);
  p.keys_a = take((size_t)p.P * 8);
  p.keys_b = take((size_t)p.P * 8);
  p.hist = take((size_t)pp::kFixedHist * 4);
  p.s64 = take((size_t)std::max<int64_t>(pp::scan_scratch(p.tiles), pp::kFixedBlocks + 1) * 8);
  p.s32 = take((size_t)pp::scan_scratch(n1) * 4);
  p.zero_lo = off;
  p.fdeg = take((size_t)n1 * 4);
  p.bdeg = take((size_t)n1 * 4);
  p.cur = take((size_t)n1 * 4);
  p.sums = take((size_t)n1 * 8);
  p.counts = take((size_t)n1 * 8);
  p.scal = take(8 * 8);
  p.zero_hi = off;
  p.fstart = take((size_t)n1 * 4);
  p.rp = take((size_t)(n1 + 1) * 4);
  p.col = take((size_t)p.P * 2 * 4);
  p.total = off;
  return p;
}

__global__ __launch_bounds__(kImgThreads) void k_zero(unsigned long long *__restrict__ a, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// One tile of kTileRows x kTileCols pixels (rows of all slices one after the
// other): thread t takes kTileSeg consecutive pixels of one row (vector loads
// where the row allows).  Each pixel pairs with its right neighbour, the one
// below in the same slice and the one at the same place in the next slice; a
// pair of different valid ids goes into the LDS set once (a thread skips a
// pair equal to the last one it added in the same direction), an invalid id
// is counted (scal[0]).  A pair that finds no free slot within kSetProbes
// probes is written out as it is (the global unique pass removes repeats).
// The tile's pairs end up in its part of tkeys, their number in tcount[tile].
constexpr int kSetProbes = 64;

__device__ __forceinline__ uint32_t set_slot(uint64_t key) {
  return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 52) & (kTileSet - 1);
}

// ids of pixels [p, p + kTileSeg) of one row, cnt of them valid (-1 past cnt)
__device__ __forceinline__ void load_ids(const int32_t *__restrict__ reg, int64_t p, int cnt, int32_t *id) {
  if (cnt == kTileSeg && ((uintptr_t)(reg + p) & 15) == 0) {
    const int4 a = *reinterpret_cast<const int4 *>(reg + p), b = *reinterpret_cast<const int4 *>(reg + p + 4);
    id[0] = a.x, id[1] = a.y, id[2] = a.z, id[3] = a.w, id[4] = b.x, id[5] = b.y, id[6] = b.z, id[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < kTileSeg; ++i) id[i] = i < cnt ? reg[p + i] : -1;
  }
}

__global__ __launch_bounds__(kImgThreads) void k_tile_pairs(const int32_t *__restrict__ reg, int32_t width,
                                                             int32_t height, int32_t depth, int32_t n, int B,
                                                             uint64_t *__restrict__ tkeys, int64_t *__restrict__ tcount,
                                                             int32_t *__restrict__ tset, long long *__restrict__ scal) {
  __shared__ uint64_t set[kTileSet];
  __shared__ int64_t lds[kImgThreads / 64];
  __shared__ int bad_block, nover;
  for (int i = threadIdx.x; i < kTileSet; i += blockDim.x) set[i] = kEmpty;
  if (threadIdx.x == 0) bad_block = nover = 0;
  __syncthreads();
  const int64_t plane = (int64_t)width * height, npix = plane * depth;
  const int64_t rows = (int64_t)height * depth;
  const int64_t tiles_x = (width + kTileCols - 1) / kTileCols;
  const int64_t R = (int64_t)(blockIdx.x / tiles_x) * kTileRows + threadIdx.x / 16;
  const int32_t c0 = (int32_t)(blockIdx.x % tiles_x) * kTileCols + (threadIdx.x % 16) * kTileSeg;
  const int cnt = R < rows ? max(0, min(kTileSeg, width - c0)) : 0;
  const int32_t r = (int32_t)(R % height);
  const int64_t p0 = R * width + c0;
  uint64_t *out = tkeys + (size_t)blockIdx.x * kTilePairs;
  int bad = 0;
  uint64_t last[3] = {kEmpty, kEmpty, kEmpty};
  auto add = [&](int dir, int32_t u, int32_t v) {
    if (u == v) return;
    if (u < 0 || u >= n || v < 0 || v >= n) {
      bad = 1;
      return;
    }
    const uint64_t key = ((uint64_t)(uint32_t)min(u, v) << B) | (uint32_t)max(u, v);
    if (key == last[dir]) return;
    last[dir] = key;
    uint32_t h = set_slot(key);
    for (int probe = 0; probe < kSetProbes; ++probe) {
      const uint64_t prev = atomicCAS((unsigned long long *)&set[h], (unsigned long long)kEmpty,
                                      (unsigned long long)key);
      if (prev == kEmpty || prev == key) return;
      h = (h + 1) & (kTileSet - 1);
    }
    out[kTilePairs - 1 - atomicAdd(&nover, 1)] = key;  // no room: out as it is, from the far end
  };
  if (cnt > 0) {
    int32_t id[kTileSeg], nb[kTileSeg];
    load_ids(reg, p0, cnt, id);
#pragma unroll
    for (int i = 0; i < kTileSeg; ++i)
      if (i < cnt && (id[i] < 0 || id[i] >= n)) bad = 1;
    // right neighbours: the next pixel of the run, then the one past it
#pragma unroll
    for (int i = 0; i + 1 < kTileSeg; ++i)
      if (i + 1 < cnt) add(0, id[i], id[i + 1]);
    if (c0 + cnt < width) add(0, id[cnt - 1], reg[p0 + cnt]);
    if (r + 1 < height) {
      load_ids(reg, p0 + width, cnt, nb);
#pragma unroll
      for (int i = 0; i < kTileSeg; ++i)
        if (i < cnt) add(1, id[i], nb[i]);
    }
    if (p0 + plane < npix) {
      load_ids(reg, p0 + plane, cnt, nb);
#pragma unroll
      for (int i = 0; i < kTileSeg; ++i)
        if (i < cnt) add(2, id[i], nb[i]);
    }
  }
  if (bad) bad_block = 1;
  __syncthreads();
  // the set's entries (slot order) go to the front of the tile's part; the
  // pairs that found no slot sit at its far end (every entry comes from its
  // own pair, so the two parts never meet)
  constexpr int kPer = kTileSet / kImgThreads;
  int64_t mine = 0;
  for (int i = 0; i < kPer; ++i) mine += set[threadIdx.x * kPer + i] != kEmpty;
  int64_t total;
  int64_t o = block_excl_scan(mine, lds, &total);
  for (int i = 0; i < kPer; ++i) {
    const uint64_t k = set[threadIdx.x * kPer + i];
    if (k != kEmpty) out[o++] = k;
  }
  if (threadIdx.x == 0) {
    tcount[blockIdx.x] = total + nover;
    tset[blockIdx.x] = (int32_t)total;
    if (bad_block) atomicAdd((unsigned long long *)&scal[0], 1ull);
  }
}

// Tile t's pairs to the list at its offset: the set part, then the far end.
__global__ __launch_bounds__(kImgThreads) void k_pack(const uint64_t *__restrict__ tkeys,
                                                       const int64_t *__restrict__ toff,
                                                       const int32_t *__restrict__ tset, uint64_t *__restrict__ out) {
  const int64_t b = toff[blockIdx.x], cnt = toff[blockIdx.x + 1] - b, set_n = tset[blockIdx.x];
  const uint64_t *src = tkeys + (size_t)blockIdx.x * kTilePairs;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
    out[b + i] = i < set_n ? src[i] : src[kTilePairs - (cnt - set_n) + (i - set_n)];
}

// Forward / backward counts of the unique pairs (u, v), u < v, and the list
// index where each row's forward pairs start.
// The unique pairs are sorted, so row a's forward neighbours are one run of
// the list: its first element writes fstart[a], its last fend[a] = index + 1
// (fend is zeroed beforehand, so 0 marks a row without forward neighbours);
// only the backward counts need atomics.
__global__ __launch_bounds__(kImgThreads) void k_degrees(const uint64_t *__restrict__ u, int64_t P,
                                                          const long long *__restrict__ m, int B,
                                                          int32_t *__restrict__ fend, int32_t *__restrict__ bdeg,
                                                          int32_t *__restrict__ fstart) {
  const int64_t c = min((int64_t)*m, P);
  const uint64_t low = ((uint64_t)1 << B) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = u[i];
    const int32_t a = (int32_t)(k >> B), b = (int32_t)(k & low);
    atomicAdd(&bdeg[b], 1);
    if (i == 0 || (int32_t)(u[i - 1] >> B) != a) fstart[a] = (int32_t)i;
    if (i + 1 == c || (int32_t)(u[i + 1] >> B) != a) fend[a] = (int32_t)(i + 1);
  }
}

__global__ __launch_bounds__(kImgThreads) void k_row_sizes(const int32_t *__restrict__ fend,
                                                            const int32_t *__restrict__ fstart,
                                                            const int32_t *__restrict__ bdeg, int32_t n,
                                                            int32_t *__restrict__ rp) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    rp[v] = (fend[v] ? fend[v] - fstart[v] : 0) + bdeg[v];
}

// Row a: its backward neighbours (below a) first, then its forward ones in
// list order (ascending); a backward entry takes the next free place of its
// row's backward part.
__global__ __launch_bounds__(kImgThreads) void k_fill(const uint64_t *__restrict__ u, int64_t P,
                                                       const long long *__restrict__ m, int B,
                                                       const int32_t *__restrict__ rp, const int32_t *__restrict__ bdeg,
                                                       const int32_t *__restrict__ fstart, int32_t *__restrict__ cur,
                                                       int32_t *__restrict__ col) {
  const int64_t c = min((int64_t)*m, P);
  const uint64_t low = ((uint64_t)1 << B) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = u[i];
    const int32_t a = (int32_t)(k >> B), b = (int32_t)(k & low);
    col[rp[a] + bdeg[a] + ((int32_t)i - fstart[a])] = b;
    col[rp[b] + atomicAdd(&cur[b], 1)] = a;
  }
}

// Each row's backward part in ascending order (insertion sort; a region has
// few neighbours below it).
__global__ __launch_bounds__(kImgThreads) void k_sort_back(const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ bdeg, int32_t n,
                                                            int32_t *__restrict__ col) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t *a = col + rp[v];
    const int32_t d = bdeg[v];
    for (int32_t i = 1; i < d; ++i) {
      const int32_t x = a[i];
      int32_t j = i - 1;
      while (j >= 0 && a[j] > x) {
        a[j + 1] = a[j];
        --j;
      }
      a[j + 1] = x;
    }
  }
}

// Pixel sums and counts per region, one block per tile of kTileRows x
// kTileCols pixels; thread t holds kTileSeg consecutive pixels of one tile row
// (one vector load of ids and one of pixels where the row allows) and adds
// each run of equal ids once.  When the valid ids of the tile span fewer than
// kTileTable values (neighbouring regions have neighbouring ids in the usual
// oversegmentations) the runs are added in an LDS table indexed by id -
// (smallest id), count and sum packed in one 64-bit word (a tile has at most
// kTileRows * kTileCols pixels, so both fit in 32 bits: one LDS atomic per
// run), and each non-empty entry goes to memory with one atomic per array;
// otherwise every run does.  A block's LDS (16 KB) leaves room for eight
// blocks per compute unit.  Integer sums, so the totals do not depend on the
// order.  Ids outside [0, n) are skipped (the pair pass counts them).
constexpr int kTileTable = 2048;

__global__ __launch_bounds__(kImgThreads) void k_region_sums(const int32_t *__restrict__ reg,
                                                              const uint8_t *__restrict__ pix, int32_t width,
                                                              int32_t rows, int32_t n,
                                                              unsigned long long *__restrict__ sums,
                                                              unsigned long long *__restrict__ counts) {
  static_assert((uint64_t)kTileRows * kTileCols * 255 < (1ull << 32), "a tile's sum fits in 32 bits");
  __shared__ unsigned long long tab[kTileTable];  // (count << 32) | sum
  __shared__ int id_lo, id_hi;
  const int64_t tiles_x = (width + kTileCols - 1) / kTileCols;
  const int64_t R = (int64_t)(blockIdx.x / tiles_x) * kTileRows + threadIdx.x / 16;
  const int32_t c0 = (int32_t)(blockIdx.x % tiles_x) * kTileCols + (threadIdx.x % 16) * kTileSeg;
  const int32_t cnt = R < rows ? max(0, min(kTileSeg, width - c0)) : 0;
  const int64_t p0 = R * width + c0;
  if (threadIdx.x == 0) {
    id_lo = INT_MAX;
    id_hi = -1;
  }
  int32_t id[kTileSeg];
  uint32_t px[kTileSeg];
  if (cnt == kTileSeg && ((uintptr_t)(reg + p0) & 15) == 0 && ((uintptr_t)(pix + p0) & 7) == 0) {
    const int4 a = *reinterpret_cast<const int4 *>(reg + p0), b = *reinterpret_cast<const int4 *>(reg + p0 + 4);
    const uint2 q = *reinterpret_cast<const uint2 *>(pix + p0);
    id[0] = a.x, id[1] = a.y, id[2] = a.z, id[3] = a.w, id[4] = b.x, id[5] = b.y, id[6] = b.z, id[7] = b.w;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      px[i] = (q.x >> (8 * i)) & 255u;
      px[4 + i] = (q.y >> (8 * i)) & 255u;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kTileSeg; ++i) {
      id[i] = i < cnt ? reg[p0 + i] : -1;
      px[i] = i < cnt ? pix[p0 + i] : 0u;
    }
  }
  int lo = INT_MAX, hi = -1;
#pragma unroll
  for (int i = 0; i < kTileSeg; ++i)
    if (id[i] >= 0 && id[i] < n) {
      lo = min(lo, id[i]);
      hi = max(hi, id[i]);
    }
  for (int d = 32; d > 0; d >>= 1) {
    lo = min(lo, __shfl_down(lo, d, 64));
    hi = max(hi, __shfl_down(hi, d, 64));
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && hi >= 0) {
    atomicMin(&id_lo, lo);
    atomicMax(&id_hi, hi);
  }
  __syncthreads();
  const int base = id_lo, span = id_hi - base + 1;
  const bool table = id_hi >= 0 && span <= kTileTable;  // the same for every thread
  if (table) {
    for (int i = threadIdx.x; i < span; i += blockDim.x) tab[i] = 0;
  }
  __syncthreads();
  int32_t cur = -1;
  unsigned long long sm = 0;
  unsigned int k = 0;
  auto flush = [&]() {
    if (k && cur >= 0 && cur < n) {
      if (table) {
        atomicAdd(&tab[cur - base], ((unsigned long long)k << 32) | sm);
      } else {
        atomicAdd(&sums[cur], sm);
        atomicAdd(&counts[cur], (unsigned long long)k);
      }
    }
  };
#pragma unroll
  for (int i = 0; i < kTileSeg; ++i) {
    if (i < cnt) {
      if (id[i] != cur) {
        flush();
        cur = id[i];
        sm = 0;
        k = 0;
      }
      sm += px[i];
      k += 1;
    }
  }
  flush();
  if (table) {
    __syncthreads();
    for (int i = threadIdx.x; i < span; i += blockDim.x) {
      const unsigned long long e = tab[i];
      if (e) {
        atomicAdd(&sums[base + i], e & 0xffffffffull);
        atomicAdd(&counts[base + i], e >> 32);
      }
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
// below k <= 16).  Each thread takes kConfPer consecutive pixels per round
// (16-byte loads of each image where the address allows); a block has
// kConfThreads threads and there are at most as many blocks as compute units.
// Every block ends with its atomics on the same k * k addresses, which
// serialise, so fewer, larger blocks pay less for them.  Three ways to
// count, by k:
//  * k = 2 (two-phase segmentations, the verification metrics): four bytes at
//    a time; a byte pair counts when both bytes are 0 or 1, and the four bins
//    follow from population counts of a & b, a & ~b and ~a & b over those
//    bytes;
//  * k * k <= 16: 16-bit per-lane counters, four to a 64-bit word (bin j in
//    word j / 4);
//  * otherwise: an LDS atomic per pixel.
// Lane counts are summed over the wave (only the k * k bins in use), each wave
// adds its sums to the block's LDS histogram, and each block adds that to
// memory with one integer atomic per non-empty bin.
constexpr int kConfPer = 32;  // on 2048 x 2048: 16 pixels 7.3 us, 32 pixels 5.8 us, 64 pixels 6.2 us
constexpr int kConfThreads = 1024;

__device__ __forceinline__ void conf_load(const uint8_t *__restrict__ x, int64_t p, int cnt, uint32_t *w) {
  if (cnt == kConfPer && ((uintptr_t)(x + p) & 15) == 0) {
#pragma unroll
    for (int q = 0; q < kConfPer / 16; ++q) {
      const uint4 v = *reinterpret_cast<const uint4 *>(x + p + 16 * q);
      w[4 * q] = v.x, w[4 * q + 1] = v.y, w[4 * q + 2] = v.z, w[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kConfPer / 4; ++q) {
      uint32_t word = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = 4 * q + i;
        word |= (uint32_t)(j < cnt ? x[p + j] : (uint8_t)255) << (8 * i);  // 255 is never counted
      }
      w[q] = word;
    }
  }
}

__device__ __forceinline__ unsigned int conf_wave_sum(unsigned int v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__global__ __launch_bounds__(kConfThreads) void k_confusion(const uint8_t *__restrict__ a,
                                                             const uint8_t *__restrict__ b, int64_t npix, int32_t k,
                                                             unsigned long long *__restrict__ counts) {
  __shared__ unsigned int hist[16 * 16];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int kk = k * k;
  const int lane = threadIdx.x & 63;
  const int mode = k == 2 ? 0 : kk <= 16 ? 1 : 2;  // the same for every thread
  unsigned int n11 = 0, n10 = 0, n01 = 0, nv = 0;  // k = 2
  uint64_t acc[4] = {0, 0, 0, 0};                  // k * k <= 16: bin j in bits 16 (j % 4) .. of acc[j / 4]
  // sums the 16-bit lane fields of acc into the histogram (a field holds at
  // most kConfPer per round, and this runs at least every kConfFlush rounds)
  auto flush = [&]() {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j < kk) {
        const unsigned int v = conf_wave_sum((unsigned int)((acc[j >> 2] >> (16 * (j & 3))) & 0xffffu));
        if (lane == 0 && v) atomicAdd(&hist[j], v);
      }
    acc[0] = acc[1] = acc[2] = acc[3] = 0;
  };
  constexpr int kConfFlush = 0xffff / kConfPer;
  int rounds = 0;
  // the loop runs per wave (every lane of a wave takes the same rounds, as the
  // cross-lane sums need)
  for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63)) * kConfPer; q < npix;
       q += (int64_t)gridDim.x * blockDim.x * kConfPer) {
    const int64_t p0 = q + (int64_t)lane * kConfPer;
    const int cnt = (int)max((int64_t)0, min((int64_t)kConfPer, npix - p0));
    uint32_t wa[kConfPer / 4], wb[kConfPer / 4];
    conf_load(a, p0, cnt, wa);
    conf_load(b, p0, cnt, wb);
    if (mode == 0) {
#pragma unroll
      for (int i = 0; i < kConfPer / 4; ++i) {
        // bit 7 of a byte of `bad` is set when either byte of the pair is >= 2
        const uint32_t hi = (wa[i] | wb[i]) & 0xFEFEFEFEu;
        const uint32_t bad = ((hi & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | hi;
        const uint32_t ok = (~bad >> 7) & 0x01010101u;
        n11 += __popc(wa[i] & wb[i] & ok);
        n10 += __popc(wa[i] & ~wb[i] & ok);
        n01 += __popc(~wa[i] & wb[i] & ok);
        nv += __popc(ok);
      }
    } else if (mode == 1) {
#pragma unroll
      for (int i = 0; i < kConfPer; ++i) {
        const int x = (wa[i / 4] >> (8 * (i % 4))) & 255, y = (wb[i / 4] >> (8 * (i % 4))) & 255;
        const int code = x * k + y;
        const uint64_t inc = (x < k && y < k) ? 1ull << (16 * (code & 3)) : 0ull;
        const int word = code >> 2;
        acc[0] += word == 0 ? inc : 0ull;
        acc[1] += word == 1 ? inc : 0ull;
        acc[2] += word == 2 ? inc : 0ull;
        acc[3] += word == 3 ? inc : 0ull;
      }
      if (++rounds == kConfFlush) {
        flush();
        rounds = 0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kConfPer; ++i) {
        const int x = (wa[i / 4] >> (8 * (i % 4))) & 255, y = (wb[i / 4] >> (8 * (i % 4))) & 255;
        if (x < k && y < k) atomicAdd(&hist[x * k + y], 1u);
      }
    }
  }
  if (mode == 0) {
    // bins (0,0), (0,1), (1,0), (1,1)
    const unsigned int s11 = conf_wave_sum(n11), s10 = conf_wave_sum(n10), s01 = conf_wave_sum(n01),
                       sv = conf_wave_sum(nv);
    if (lane == 0 && sv) {
      atomicAdd(&hist[0], sv - s11 - s10 - s01);
      atomicAdd(&hist[1], s01);
      atomicAdd(&hist[2], s10);
      atomicAdd(&hist[3], s11);
    }
  } else if (mode == 1) {
    flush();
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kk; i += blockDim.x)
    if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return cus;
}

int grid_for(int64_t work, int per_cu = 8) {
  const int64_t need = (work + kImgThreads - 1) / kImgThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cu_count() * per_cu));
}

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
  namespace pp = pmrf_prims;
  clear_error();
  if (!nnz || !d_row_ptr || (n > 0 && !d_means)) return fail(PMRF_EINVAL, "NULL argument");
  if (width < 0 || height < 0 || depth < 0 || n < 0 || col_capacity < 0) return fail(PMRF_EINVAL, "negative size");
  const int64_t npix = (int64_t)width * height * depth;
  if (npix > (int64_t)1 << 28) return fail(PMRF_EUNSUPPORTED, "more than 2^28 pixels");
  if (npix > 0 && (!d_regions || !d_pixels)) return fail(PMRF_EINVAL, "NULL image");
  if (npix > 0 && n == 0) return fail(PMRF_EINVAL, "pixels but no regions");
  const ImgPlan plan = plan_image(width, height, depth, n);
  if (!d_ws || ws_bytes < (int64_t)plan.total)
    return fail(PMRF_ENOMEM, "workspace smaller than pmrf_image_graph_workspace_bytes");
  hipStream_t s = (hipStream_t)hip_stream;
  char *ws = (char *)d_ws;
  uint64_t *tkeys = (uint64_t *)(ws + plan.tile_keys), *ka = (uint64_t *)(ws + plan.keys_a),
           *kb = (uint64_t *)(ws + plan.keys_b);
  int64_t *toff = (int64_t *)(ws + plan.tile_off), *s64 = (int64_t *)(ws + plan.s64);
  int32_t *tset = (int32_t *)(ws + plan.tile_set);
  int32_t *hist = (int32_t *)(ws + plan.hist), *s32 = (int32_t *)(ws + plan.s32);
  int32_t *fdeg = (int32_t *)(ws + plan.fdeg), *bdeg = (int32_t *)(ws + plan.bdeg), *cur = (int32_t *)(ws + plan.cur);
  int32_t *fstart = (int32_t *)(ws + plan.fstart), *rp = (int32_t *)(ws + plan.rp), *col = (int32_t *)(ws + plan.col);
  unsigned long long *sums = (unsigned long long *)(ws + plan.sums), *counts = (unsigned long long *)(ws + plan.counts);
  long long *scal = (long long *)(ws + plan.scal);
  const int B = id_bits(n);
  const int64_t zero_words = (int64_t)(plan.zero_hi - plan.zero_lo) / 8;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(zero_words)), dim3(kImgThreads), 0, s,
                     (unsigned long long *)(ws + plan.zero_lo), zero_words);
  IMG_TRY(hipGetLastError());
  const uint64_t *uniq = ka;  // the unique pairs (u < v), ascending
  if (npix > 0) {
    // 1. each tile's unique pairs, 2. one list, sorted and unique
    hipLaunchKernelGGL(k_tile_pairs, dim3((unsigned)plan.tiles), dim3(kImgThreads), 0, s,
                       d_regions, width, height, depth, n, B, tkeys, toff, tset, scal);
    pp::scan<int64_t>(s, toff, toff, plan.tiles, nullptr, s64);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)plan.tiles), dim3(kImgThreads), 0, s, (const uint64_t *)tkeys,
                       (const int64_t *)toff, (const int32_t *)tset, ka);
    IMG_TRY(hipGetLastError());
    const int64_t *dlist = toff + plan.tiles;  // pairs in the list
    const bool in_b = pp::sort_pairs_fixed<uint64_t, false>(s, ka, nullptr, kb, nullptr, plan.P, dlist, 2 * B, hist);
    const uint64_t *sorted = in_b ? kb : ka;
    uint64_t *u = in_b ? ka : kb;
    pp::unique_fixed<uint64_t>(s, sorted, plan.P, dlist, u, scal + 1, s64);
    IMG_TRY(hipGetLastError());
    uniq = u;
    // 3. rows: backward part, then forward part
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(plan.P)), dim3(kImgThreads), 0, s, uniq, plan.P,
                       (const long long *)(scal + 1), B, fdeg, bdeg, fstart);
    IMG_TRY(hipGetLastError());
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_row_sizes, dim3(grid_for(n)), dim3(kImgThreads), 0, s, (const int32_t *)fdeg,
                       (const int32_t *)fstart, (const int32_t *)bdeg, n, rp);
    IMG_TRY(hipGetLastError());
  }
  pp::scan<int32_t>(s, rp, rp, n, nullptr, s32);
  if (npix > 0) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(plan.P)), dim3(kImgThreads), 0, s, uniq, plan.P,
                       (const long long *)(scal + 1), B, (const int32_t *)rp, (const int32_t *)bdeg,
                       (const int32_t *)fstart, cur, col);
    IMG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sort_back, dim3(grid_for(n)), dim3(kImgThreads), 0, s, (const int32_t *)rp,
                       (const int32_t *)bdeg, n, col);
    IMG_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_region_sums, dim3((unsigned)plan.tiles), dim3(kImgThreads), 0, s, d_regions, d_pixels,
                       width, (int32_t)plan.rows, n, sums, counts);
    IMG_TRY(hipGetLastError());
  }
  // the one wait: bad ids and the unique pair count
  long long host_scal[2] = {0, 0};
  IMG_TRY(hipMemcpyAsync(host_scal, scal, sizeof(host_scal), hipMemcpyDeviceToHost, s));
  IMG_TRY(hipStreamSynchronize(s));
  if (host_scal[0]) return fail(PMRF_EINVAL, "region id outside [0, n)");
  const int64_t edges = 2 * (int64_t)host_scal[1];
  if (edges > col_capacity) {
    *nnz = edges;
    return fail(PMRF_ENOMEM, "col_idx capacity below the number of adjacency entries (returned in *nnz)");
  }
  if (edges > 0 && !d_col_idx) return fail(PMRF_EINVAL, "NULL col_idx");
  IMG_TRY(hipMemcpyAsync(d_row_ptr, rp, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, s));
  if (edges > 0) IMG_TRY(hipMemcpyAsync(d_col_idx, col, (size_t)edges * 4, hipMemcpyDeviceToDevice, s));
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
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kImgThreads), 0, s, (unsigned long long *)d_counts, (int64_t)k * k);
  IMG_TRY(hipGetLastError());
  if (npixels > 0) {
    // at most one block per compute unit: every block ends with one
    // device-scope atomic per bin, all on the same k * k addresses
    const int64_t per_block = (int64_t)kConfThreads * kConfPer;
    const int blocks = (int)std::min<int64_t>((npixels + per_block - 1) / per_block, cu_count());
    hipLaunchKernelGGL(k_confusion, dim3(blocks), dim3(kConfThreads), 0, s, d_a, d_b, npixels, k,
                       (unsigned long long *)d_counts);
    IMG_TRY(hipGetLastError());
  }
  return PMRF_OK;
}
