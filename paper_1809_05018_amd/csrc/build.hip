// Neighbourhood construction on the device (Alg. 2: enumerate the maximal
// cliques, then construct the k-neighbourhoods; Sec. 3.2.1 and the steps of
// Sec. 3.2.2 "Construction of Neighborhoods"), ending in the same packed
// device layout as the host builder, written straight into device memory.
//
// The steps, all data parallel with a count / scan / write shape:
//   1. CSR checks (one thread per vertex).
//   2. Maximal cliques level by level.  The k-cliques of a level are kept as
//      ascending member lists in lexicographic order.  One thread per clique
//      walks the row of its member of least degree (every common neighbour is
//      in that row): a common neighbour above the last member extends the
//      clique to a (k+1)-clique; no common neighbour at all makes it maximal.
//      Extensions are written in parent order, candidates ascending, so every
//      level stays in lexicographic order and every clique appears once.
//   3. Canonical order of the maximal cliques over all levels: a clique's rank
//      is the number of maximal cliques lexicographically below it, found by
//      a binary search in every level (no maximal clique is a prefix of
//      another, so a comparison ends inside the shorter one).
//   4. Neighbourhoods (Find / Count / Get Neighbors, then Remove Duplicate
//      Neighbors): each member contributes itself and its row; the candidates
//      of one neighbourhood are sorted and made unique in LDS by one block.
//      A radius k > 1 repeats the step from the previous neighbourhood.
//   5. Owners, the processing order (neighbourhoods of at most 64 members
//      first), per-vertex occurrence lists (a stable radix sort by vertex of
//      the elements in canonical order), packets (next-fit packing of small
//      neighbourhoods into 64 lanes, as a scan over the packing state
//      machine), adjacency words, slot layout, chunk headers and superchunk
//      vertex ranges.
// Every result is a function of the graph alone (no atomics decide an order),
// so the layout is byte for byte the host builder's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pmrf_internal.h"
#include "prims.h"

using namespace pmrf;

namespace {

constexpr int kBT = 256;             // threads per block of the builder's kernels
constexpr int kCandCap = 8192;       // candidate entries of one neighbourhood sorted in LDS (32 KB)
constexpr int kFitBlock = 1024;      // neighbourhoods per block of the packing scan
constexpr int kFitStates = kWave + 1;  // packing state: 0 = no open packet, else its fill
constexpr int64_t kMaxLevelInts = int64_t(1) << 30;  // members of one clique level

struct BuildError {
  pmrf_status code;
  std::string msg;
};

#define BTRY(expr)                                                                                   \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      throw BuildError{e_ == hipErrorOutOfMemory ? PMRF_ENOMEM : PMRF_EDEVICE,                       \
                       std::string("HIP: ") + hipGetErrorString(e_)};                                \
  } while (0)

// Temporaries of a build come from a memory pool of the library's own, one per
// device, stream-ordered on the build's stream (hipMallocFromPoolAsync /
// hipFreeAsync): no device-wide synchronisation when a temporary is freed,
// and freed blocks are reused by the next build.  The pool keeps up to
// kPoolKeep bytes between builds.  The arrays handed over to the result are
// plain hipMalloc allocations (freed with the result).
constexpr uint64_t kPoolKeep = uint64_t(1) << 30;
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;

hipMemPool_t build_pool() {
  int dev = 0;
  BTRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pools.find(dev);
  if (it != g_pools.end()) return it->second;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  BTRY(hipMemPoolCreate(&pool, &props));
  uint64_t keep = kPoolKeep;
  BTRY(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  g_pools[dev] = pool;
  return pool;
}

// the stream and pool of the build running on this thread (set by BuildScope)
thread_local hipStream_t t_build_stream = nullptr;
thread_local hipMemPool_t t_build_pool = nullptr;

struct BuildScope {
  BuildScope(hipStream_t s) {
    t_build_pool = build_pool();
    t_build_stream = s;
  }
  ~BuildScope() {
    t_build_pool = nullptr;
    t_build_stream = nullptr;
  }
};

enum BufKind { kTemp = 0, kKeep = 1 };

// Device array owned by the builder (released when it goes out of scope:
// kTemp, from the build's pool) or handed over to the result (kKeep).
template <class T>
struct Buf {
  T *p = nullptr;
  int64_t n = 0;
  bool pooled = false;
  hipStream_t s = nullptr;
  Buf() = default;
  explicit Buf(int64_t count, BufKind kind = kTemp) { alloc(count, kind); }
  void alloc(int64_t count, BufKind kind = kTemp) {
    release();
    n = count;
    const size_t bytes = (size_t)std::max<int64_t>(1, count) * sizeof(T);
    if (kind == kTemp && t_build_pool) {
      s = t_build_stream;
      BTRY(hipMallocFromPoolAsync(reinterpret_cast<void **>(&p), bytes, t_build_pool, s));
      pooled = true;
    } else {
      BTRY(hipMalloc(&p, bytes));
      pooled = false;
    }
  }
  void release() {
    if (p) (void)(pooled ? hipFreeAsync(p, s) : hipFree(p));
    p = nullptr;
    n = 0;
    pooled = false;
  }
  T *take() {
    if (pooled) throw BuildError{PMRF_EDEVICE, "internal: a pooled temporary cannot be handed over"};
    T *q = p;
    p = nullptr;
    n = 0;
    return q;
  }
  ~Buf() { release(); }
  Buf(const Buf &) = delete;
  Buf &operator=(const Buf &) = delete;
  Buf(Buf &&o) noexcept : p(o.p), n(o.n), pooled(o.pooled), s(o.s) { o.p = nullptr, o.n = 0, o.pooled = false; }
  Buf &operator=(Buf &&o) noexcept {
    release();
    p = o.p, n = o.n, pooled = o.pooled, s = o.s;
    o.p = nullptr, o.n = 0, o.pooled = false;
    return *this;
  }
};

int64_t blocks_for(int64_t items, int64_t per_block, int64_t cap = 1 << 20) {
  return std::max<int64_t>(1, std::min<int64_t>(cap, (items + per_block - 1) / per_block));
}

using pmrf_prims::block_excl_scan;
using pmrf_prims::shfl_down64;

__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

// ---------------------------------------------------------- small kernels
__global__ void k_iota(int32_t *a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (int32_t)i;
}

template <class T>
__global__ void k_fill(T *a, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// max over h of ptr[h + 1] - ptr[h], into *out (start at 0)
template <class P>
__global__ void k_max_len(const P *ptr, int64_t H, int64_t *out) {
  int64_t m = 0;
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x)
    m = max(m, (int64_t)(ptr[h + 1] - ptr[h]));
  for (int d = 32; d > 0; d >>= 1) m = max(m, shfl_down64(m, d));
  if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long *)out, (unsigned long long)m);
}

__device__ __forceinline__ bool has_edge(const int32_t *rp, const int32_t *ci, int32_t a, int32_t b) {
  int32_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    const int32_t x = ci[mid];
    if (x < b) lo = mid + 1;
    else if (x > b) hi = mid;
    else return true;
  }
  return false;
}

// position of v in the ascending list a[0..len), -1 if absent
__device__ __forceinline__ int32_t find_sorted(const int32_t *a, int32_t len, int32_t v) {
  int32_t lo = 0, hi = len;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    const int32_t x = a[mid];
    if (x < v) lo = mid + 1;
    else if (x > v) hi = mid;
    else return mid;
  }
  return -1;
}

// ------------------------------------------------------------- CSR checks
// bad[0]: a decreasing row_ptr step (smallest vertex)
__global__ void k_check_rows(const int32_t *rp, int32_t n, int32_t *bad) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (rp[v + 1] < rp[v]) atomicMin(&bad[0], (int32_t)v);
}

// bad[1..4]: id out of range, self loop, row not strictly ascending, missing
// reverse edge (smallest vertex of each kind); rows must already be checked
__global__ void k_check_cols(const int32_t *rp, const int32_t *ci, int32_t n, int32_t *bad) {
  for (int64_t vv = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; vv < n; vv += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)vv;
    for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t u = ci[k];
      if (u < 0 || u >= n) atomicMin(&bad[1], v);
      else if (u == v) atomicMin(&bad[2], v);
      else if (k > rp[v] && ci[k - 1] >= u) atomicMin(&bad[3], v);
      else if (!has_edge(rp, ci, u, v)) atomicMin(&bad[4], v);
    }
  }
}

// --------------------------------------------------------- clique levels
// Cliques of one level: k members each, ascending, the list lexicographic.
// WRITE = false: ext[i] = extensions of clique i (common neighbours above its
// last member), maximal[i] = 1 when it has no common neighbour at all.
// WRITE = true: the extensions, at (k + 1) * (ext_off[i] + j).
template <bool WRITE>
__global__ void k_extend(const int32_t *C, int64_t count, int k, const int32_t *rp, const int32_t *ci, int64_t *ext,
                         int32_t *maximal, const int64_t *ext_off, int32_t *next) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t *c = C + (int64_t)k * i;
    int m = 0;
    int32_t md = INT_MAX;
    for (int j = 0; j < k; ++j) {
      const int32_t d = rp[c[j] + 1] - rp[c[j]];
      if (d < md) md = d, m = j;
    }
    const int32_t last = c[k - 1], cm = c[m];
    int32_t cnt = 0;
    bool any = false;
    int32_t *out = WRITE ? next + (int64_t)(k + 1) * ext_off[i] : nullptr;
    for (int32_t e = rp[cm]; e < rp[cm + 1]; ++e) {
      const int32_t w = ci[e];
      bool common = true;  // a member w fails its own test: no self loops
      for (int j = 0; j < k && common; ++j)
        if (j != m) common = has_edge(rp, ci, c[j], w);
      if (!common) continue;
      any = true;
      if (w > last) {
        if (WRITE) {
          for (int j = 0; j < k; ++j) out[j] = c[j];
          out[k] = w;
          out += k + 1;
        }
        ++cnt;
      }
    }
    if (!WRITE) {
      ext[i] = cnt;
      maximal[i] = any ? 0 : 1;
    }
  }
}

// the maximal cliques of a level, kept in order (pos: prefix sums of the
// maximal flags, so clique i is maximal when pos[i + 1] > pos[i])
__global__ void k_keep_maximal(const int32_t *C, int64_t count, int k, const int32_t *pos, int32_t *out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    if (pos[i + 1] > pos[i])
      for (int j = 0; j < k; ++j) out[(int64_t)k * pos[i] + j] = C[(int64_t)k * i + j];
}

struct Level {
  const int32_t *c;  // maximal cliques of k members, lexicographic
  int64_t count;
  int32_t k, pad;
};

__device__ int lex_cmp(const int32_t *a, int ka, const int32_t *b, int kb) {
  const int m = min(ka, kb);
  for (int i = 0; i < m; ++i)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return ka < kb ? -1 : ka > kb ? 1 : 0;
}

// rank of each maximal clique of level `self` among all maximal cliques; the
// clique's size goes to size[rank] and its rank to each member's first[v]
__global__ void k_rank(const Level *lv, int nlev, int self, int32_t *rank, int32_t *size, int32_t *first) {
  const Level me = lv[self];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < me.count; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t *c = me.c + (int64_t)me.k * i;
    int64_t r = i;
    for (int j = 0; j < nlev; ++j) {
      if (j == self) continue;
      const Level o = lv[j];
      int64_t lo = 0, hi = o.count;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (lex_cmp(o.c + (int64_t)o.k * mid, o.k, c, me.k) < 0) lo = mid + 1;
        else hi = mid;
      }
      r += lo;
    }
    rank[i] = (int32_t)r;
    size[r] = me.k;
    for (int j = 0; j < me.k; ++j) atomicMin(&first[c[j]], (int32_t)r);
  }
}

__global__ void k_place_cliques(const int32_t *C, int64_t count, int k, const int32_t *rank, const int32_t *cptr,
                                int32_t *cvid) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    for (int j = 0; j < k; ++j) cvid[cptr[rank[i]] + j] = C[(int64_t)k * i + j];
}

// ---------------------------------------------------------- neighbourhoods
// candidates contributed by each element: the member and its row
__global__ void k_cand_count(const int32_t *vid, int64_t E, const int32_t *rp, int64_t *cnt) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = vid[e];
    cnt[e] = 1 + rp[u + 1] - rp[u];
  }
}

__global__ void k_cand_write(const int32_t *vid, int64_t E, const int32_t *rp, const int32_t *ci, const int64_t *off,
                             int32_t *cand) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = vid[e];
    int32_t *o = cand + off[e];
    *o++ = u;
    for (int32_t q = rp[u]; q < rp[u + 1]; ++q) *o++ = ci[q];
  }
}

// candidate range of neighbourhood h: the offsets of its first element
__global__ void k_hood_cand_ptr(const int32_t *sptr, int64_t H, const int64_t *off, int64_t *cptr) {
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h <= H; h += (int64_t)gridDim.x * blockDim.x)
    cptr[h] = off[sptr[h]];
}

// One block per neighbourhood: sort its candidates in LDS (bitonic network
// over P = a power of two >= every candidate count), keep the first of each
// run of equal ids, write them back to the front of its range; usize[h] = kept.
__global__ void __launch_bounds__(kBT) k_sort_unique(int32_t *cand, const int64_t *cptr, int64_t H, int32_t P,
                                                     int32_t *usize) {
  extern __shared__ int32_t s[];
  __shared__ int32_t lds[kBT / 64];
  const int t = threadIdx.x, bd = blockDim.x;
  for (int64_t h = blockIdx.x; h < H; h += gridDim.x) {
    const int64_t b = cptr[h];
    const int32_t cnt = (int32_t)(cptr[h + 1] - b);
    // this neighbourhood's network: the power of two at or above its count
    // (P, the largest, sizes the LDS)
    int32_t Ph = 2;
    while (Ph < cnt) Ph <<= 1;
    const int per = (Ph + bd - 1) / bd;
    for (int i = t; i < Ph; i += bd) s[i] = i < cnt ? cand[b + i] : INT_MAX;
    __syncthreads();
    for (int kk = 2; kk <= Ph; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = t; i < (Ph >> 1); i += bd) {
          const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1)), hi = lo + j;
          const int32_t x = s[lo], y = s[hi];
          if ((x > y) == ((lo & kk) == 0)) s[lo] = y, s[hi] = x;
        }
        __syncthreads();
      }
    int32_t keep = 0;
    for (int q = 0; q < per; ++q) {
      const int p = t * per + q;
      keep += p < cnt && (p == 0 || s[p] != s[p - 1]);
    }
    int32_t total;
    int32_t o = block_excl_scan(keep, lds, &total);
    for (int q = 0; q < per; ++q) {
      const int p = t * per + q;
      if (p < cnt && (p == 0 || s[p] != s[p - 1])) cand[b + o++] = s[p];
    }
    if (t == 0) usize[h] = total;
    __syncthreads();
  }
}

// one wave per segment: dst[dptr[h] ..] = src[sptr[h] ..], len[h] entries
template <class SP>
__global__ void k_copy_segs(const int32_t *src, const SP *sptr, const int32_t *dptr, const int32_t *len, int64_t H,
                            int32_t *dst) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t h = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); h < H; h += nw) {
    const int64_t s0 = sptr[h];
    const int32_t d0 = dptr[h], l = len[h];
    for (int32_t i = lane; i < l; i += 64) dst[d0 + i] = src[s0 + i];
  }
}

// owner[v]: v's element in the first clique holding it
__global__ void k_owner(const int32_t *first, int32_t n, const int32_t *hptr, const int32_t *hvid, int32_t *owner) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t h = first[v];
    owner[v] = hptr[h] + find_sorted(hvid + hptr[h], hptr[h + 1] - hptr[h], (int32_t)v);
  }
}

// ------------------------------------------------------- processing order
__global__ void k_small_flag(const int32_t *hptr, int64_t H, int32_t *flag) {
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x)
    flag[h] = hptr[h + 1] - hptr[h] <= kWave;
}

// neighbourhoods of at most 64 members first, each group in canonical order
__global__ void k_perm(const int32_t *hptr, int64_t H, const int32_t *spos, int32_t *perm, int32_t *inv,
                       int32_t *psize) {
  const int32_t ns = spos[H];
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = hptr[h + 1] - hptr[h];
    const int32_t p = s <= kWave ? spos[h] : ns + (int32_t)h - spos[h];
    perm[p] = (int32_t)h;
    inv[h] = p;
    psize[p] = s;
  }
}

// one wave per neighbourhood (processing order): members into the device
// array, each processing element's neighbourhood, and for each canonical
// element its processing index (the values of the occurrence sort)
__global__ void k_place_proc(const int32_t *perm, int64_t H, const int32_t *hptr, const int32_t *hvid,
                             const int32_t *pptr, int32_t *dev_vid, int32_t *pe_hood, int32_t *canon_pe) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t hp = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); hp < H; hp += nw) {
    const int32_t h = perm[hp], c0 = hptr[h], s = hptr[h + 1] - c0, p0 = pptr[hp];
    for (int32_t j = lane; j < s; j += 64) {
      dev_vid[p0 + j] = hvid[c0 + j];
      pe_hood[p0 + j] = (int32_t)hp;
      canon_pe[c0 + j] = p0 + j;
    }
  }
}

// ptr[v] = the first index of v in the sorted ids (the insertion point where
// v is absent), ptr[n] = M: each run start writes the entries of the ids after
// the previous element's up to its own, the last element those past its id.
__global__ void k_run_starts(const uint32_t *keys, int64_t M, int32_t n, int32_t *ptr) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cur = keys[e], prev = e ? (int64_t)keys[e - 1] : -1;
    for (int64_t v = prev + 1; v <= cur; ++v) ptr[v] = (int32_t)e;
    if (e == M - 1)
      for (int64_t v = cur + 1; v <= n; ++v) ptr[v] = (int32_t)M;
  }
}

// bit e of lastbits: element e holds its vertex's last occurrence
__global__ void k_lastbits(const int32_t *occ_ptr, const int32_t *occ, int32_t n, unsigned long long *bits) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (occ_ptr[v + 1] > occ_ptr[v]) {
      const int32_t e = occ[occ_ptr[v + 1] - 1];
      atomicOr(&bits[e >> 6], 1ull << (e & 63));
    }
}

// ------------------------------------------------------------- packing
// Next-fit packing of the processing order: a neighbourhood of at most 64
// members joins the open packet when it fits in the 64 lanes, else opens a
// new one; a LARGE one takes a packet of its own and closes the open one.
// The state is the open packet's fill (0: none), so each block of kFitBlock
// neighbourhoods is summarised by its effect on every entry state.
__device__ __forceinline__ void fit_step(int32_t s, int32_t &fill, int32_t &opened) {
  if (s <= kWave) {
    if (fill == 0 || fill + s > kWave) ++opened, fill = 0;
    fill += s;
  } else {
    ++opened;
    fill = 0;
  }
}

__global__ void __launch_bounds__(128) k_fit_table(const int32_t *psize, int64_t H, int32_t *table) {
  __shared__ int32_t sz[kFitBlock];
  const int64_t b0 = (int64_t)blockIdx.x * kFitBlock;
  const int cnt = (int)imin64(kFitBlock, H - b0);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) sz[i] = psize[b0 + i];
  __syncthreads();
  if (threadIdx.x < kFitStates) {
    int32_t fill = threadIdx.x, opened = 0;
    for (int i = 0; i < cnt; ++i) fit_step(sz[i], fill, opened);
    table[((int64_t)blockIdx.x * kFitStates + threadIdx.x) * 2] = fill;
    table[((int64_t)blockIdx.x * kFitStates + threadIdx.x) * 2 + 1] = opened;
  }
}

// one thread: entry state and first new packet of every block; the packet
// count goes to *ntiles
__global__ void k_fit_chain(const int32_t *table, int64_t nb, int32_t *entry, int64_t *ntiles) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t st = 0;
  int64_t tiles = 0;
  for (int64_t b = 0; b < nb; ++b) {
    entry[2 * b] = st;
    entry[2 * b + 1] = (int32_t)tiles;
    const int32_t *e = table + (b * kFitStates + st) * 2;
    st = e[0];
    tiles += e[1];
  }
  *ntiles = tiles;
}

__global__ void __launch_bounds__(64) k_fit_assign(const int32_t *psize, int64_t H, const int32_t *entry,
                                                   int32_t *tile_of, int32_t *pos_of) {
  __shared__ int32_t sz[kFitBlock];
  const int64_t b0 = (int64_t)blockIdx.x * kFitBlock;
  const int cnt = (int)imin64(kFitBlock, H - b0);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) sz[i] = psize[b0 + i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  int32_t fill = entry[2 * blockIdx.x], cur = entry[2 * blockIdx.x + 1] - 1;
  for (int i = 0; i < cnt; ++i) {
    int32_t opened = 0;
    const int32_t s = sz[i];
    fit_step(s, fill, opened);
    cur += opened;
    tile_of[b0 + i] = cur;
    pos_of[b0 + i] = s <= kWave ? fill - s : 0;
  }
}

__device__ __forceinline__ int32_t words_of(int32_t s) { return s <= 32 ? 1 : (s + 31) / 32; }

// a packet holding a neighbourhood above 32 members is MID
__global__ void k_tile_mid(const int32_t *psize, int64_t H, const int32_t *tile_of, int32_t *t_mid, int32_t *mid) {
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = psize[h];
    if (s > 32 && s <= kWave) {
      t_mid[tile_of[h]] = 1;
      *mid = 1;
    }
  }
}

// adjacency words per element of each neighbourhood (its packet's: two in a
// MID packet, one in a SMALL one; a LARGE neighbourhood's own) and the
// neighbourhood's share of the mask array
__global__ void k_mask_words(const int32_t *psize, int64_t H, const int32_t *tile_of, const int32_t *t_mid,
                             int64_t *mw, int32_t *hw) {
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = psize[h];
    const int32_t w = s > kWave ? words_of(s) : t_mid[tile_of[h]] ? 2 : 1;
    hw[h] = w;
    mw[h] = (int64_t)s * w;
  }
}

// packet fields set by its first neighbourhood; lanes and start bits gathered
__global__ void k_tile_hoods(const int32_t *psize, int64_t H, const int32_t *tile_of, const int32_t *pos_of,
                             const int32_t *pptr, const int64_t *moff, const int32_t *hw, TileDesc *tiles,
                             unsigned long long *t_start, int32_t *t_nelem) {
  for (int64_t hp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; hp < H; hp += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = psize[hp], T = tile_of[hp], pos = pos_of[hp];
    if (pos == 0) {
      TileDesc &t = tiles[T];
      t.elem_start = pptr[hp];
      t.hood_start = (int32_t)hp;
      t.mask_start = (int32_t)moff[hp];
      t.kind = s > kWave ? kLarge : hw[hp] == 2 ? kMid : kSmall;
      t.words = (uint8_t)hw[hp];
    }
    atomicOr(&t_start[T], 1ull << pos);
    atomicMax(&t_nelem[T], pos + s);
  }
}

__global__ void k_tile_finish(int64_t ntiles, const unsigned long long *t_start, const int32_t *t_nelem,
                              TileDesc *tiles) {
  for (int64_t T = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; T < ntiles; T += (int64_t)gridDim.x * blockDim.x) {
    tiles[T].start_mask = t_start[T];
    tiles[T].nelem = (int16_t)t_nelem[T];
  }
}

// adjacency words of every element (processing order): bit p of the element's
// words marks member p as a neighbour, its own bit marks the owner element
__global__ void k_masks(int64_t M, const int32_t *pe_hood, const int32_t *pptr, const int32_t *perm,
                        const int32_t *hptr, const int32_t *dev_vid, const int32_t *owner, const int32_t *rp,
                        const int32_t *ci, const int64_t *moff, const int32_t *hw, uint32_t *mask,
                        unsigned long long *A) {
  unsigned long long a = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t hp = pe_hood[e], p0 = pptr[hp], s = pptr[hp + 1] - p0, j = (int32_t)e - p0;
    const int32_t nw = hw[hp];
    const int32_t v = dev_vid[e];
    const int32_t *mem = dev_vid + p0;
    uint32_t *w = mask + moff[hp] + (int64_t)j * nw;
    const bool own = owner[v] == hptr[perm[hp]] + j;
    const int32_t q0 = rp[v], q1 = rp[v + 1];
    if (nw <= 2) {
      // at most 64 members: both words in registers, written once; the graph
      // neighbours' ids requested eight at a time
      uint64_t bits = own ? 1ull << j : 0ull;
      for (int32_t qb = q0; qb < q1; qb += 8) {
        int32_t nb[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) nb[i] = qb + i < q1 ? ci[qb + i] : -1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int32_t p = nb[i] >= 0 ? find_sorted(mem, s, nb[i]) : -1;
          if (p >= 0) {
            bits |= 1ull << p;
            ++a;
          }
        }
      }
      w[0] = (uint32_t)bits;
      if (nw == 2) w[1] = (uint32_t)(bits >> 32);
    } else {
      for (int q = 0; q < nw; ++q) w[q] = 0u;
      for (int32_t q = q0; q < q1; ++q) {
        const int32_t p = find_sorted(mem, s, ci[q]);
        if (p >= 0) {
          w[p >> 5] |= 1u << (p & 31);
          ++a;
        }
      }
      if (own) w[j >> 5] |= 1u << (j & 31);
    }
  }
  for (int d = 32; d > 0; d >>= 1) a += (unsigned long long)shfl_down64((int64_t)a, d);
  if ((threadIdx.x & 63) == 0 && a) atomicAdd(A, a);
}

// slot layout of the packets before the first LARGE one
__global__ void k_slots(int64_t Ms, const int32_t *pe_hood, const int32_t *pptr, const int32_t *tile_of,
                        const int32_t *pos_of, const int32_t *dev_vid, const int64_t *moff, const int32_t *hw,
                        const uint32_t *mask, int32_t *svid, uint32_t *smask, uint32_t *smask_hi) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Ms; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t hp = pe_hood[e], p0 = pptr[hp], j = (int32_t)e - p0;
    const int32_t nw = hw[hp];
    const int64_t slot = (int64_t)tile_of[hp] * kWave + pos_of[hp] + j;
    const uint32_t *w = mask + moff[hp] + (int64_t)j * nw;
    svid[slot] = (int32_t)((uint32_t)dev_vid[e] | ((uint32_t)j << kSlotJShift));
    smask[slot] = w[0];
    if (nw == 2) smask_hi[slot] = w[1];
  }
}

__global__ void k_chunks(const TileDesc *tiles, int64_t ntiles, int64_t nchunks, int32_t H, ChunkHdr *chdr) {
  for (int64_t ck = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ck < nchunks; ck += (int64_t)gridDim.x * blockDim.x) {
    ChunkHdr c{};
    const int64_t tb = ck * kChunkTiles, te = imin64(ntiles, tb + kChunkTiles);
    c.elem_start = tiles[tb].elem_start;
    c.hood_start = tiles[tb].hood_start;
    c.hood_end = te < ntiles ? tiles[te].hood_start : H;
    for (int64_t ti = tb; ti < te; ++ti) {
      const TileDesc t = tiles[ti];
      const int i = (int)(ti - tb);
      if (t.kind == kLarge) c.flags |= kHdrLarge;
      if (t.kind == kMid) c.flags |= 1 << (kHdrMidShift + i);
      c.elem_off[i] = (uint16_t)imin64(t.elem_start - c.elem_start, 0xffff);
    }
    chdr[ck] = c;
  }
}

// member vertex range of each superchunk's slots (empty: 0, 0)
__global__ void __launch_bounds__(kBT) k_srange(const int32_t *svid, int64_t slots, int64_t per_super, int32_t *srange) {
  __shared__ int32_t lo_s[kBT / 64], hi_s[kBT / 64];
  const int64_t s0 = blockIdx.x * per_super, s1 = imin64(slots, s0 + per_super);
  int32_t lo = INT_MAX, hi = INT_MIN;
  for (int64_t k = s0 + threadIdx.x; k < s1; k += blockDim.x) {
    const uint32_t w = (uint32_t)svid[k];
    if (w == kSlotEmpty) continue;
    const int32_t v = (int32_t)(w & kSlotVidMask);
    lo = min(lo, v);
    hi = max(hi, v + 1);
  }
  for (int d = 32; d > 0; d >>= 1) {
    lo = min(lo, __shfl_down(lo, d, 64));
    hi = max(hi, __shfl_down(hi, d, 64));
  }
  if ((threadIdx.x & 63) == 0) lo_s[threadIdx.x >> 6] = lo, hi_s[threadIdx.x >> 6] = hi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBT / 64; ++i) lo = min(lo, lo_s[i]), hi = max(hi, hi_s[i]);
    lo = min(lo, lo_s[0]);
    hi = max(hi, hi_s[0]);
    if (lo > hi) lo = hi = 0;
    srange[2 * blockIdx.x] = lo;
    srange[2 * blockIdx.x + 1] = hi;
  }
}

// ----------------------------------------------------------- host driver
struct Builder {
  hipStream_t s;
  Buf<int64_t> scal{4};  // small results read back by the host

  explicit Builder(hipStream_t st) : s(st) {}

  void check() { BTRY(hipGetLastError()); }
  void sync() { BTRY(hipStreamSynchronize(s)); }

  template <class T>
  T read(const T *d) {
    T v;
    BTRY(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
    sync();
    return v;
  }
  template <class T>
  void zero(T *p, int64_t n) {
    if (n > 0) BTRY(hipMemsetAsync(p, 0, (size_t)n * sizeof(T), s));
  }
  template <class T>
  void copy(T *dst, const T *src, int64_t n) {
    if (n > 0) BTRY(hipMemcpyAsync(dst, src, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s));
  }

  // out[0..n] = exclusive prefix sums of in[0..n), out[n] = the total (in may
  // be out)
  template <class T>
  void scan(const T *in, T *out, int64_t n) {
    Buf<T> sums(pmrf_prims::scan_scratch(n));
    pmrf_prims::scan<T>(s, in, out, n, nullptr, sums.p);
    check();
    sync();  // sums is released on return
  }

  template <class P>
  int64_t max_len(const P *ptr, int64_t H) {
    zero(scal.p, 1);
    k_max_len<P><<<blocks_for(H, kBT, 4096), kBT, 0, s>>>(ptr, H, scal.p);
    check();
    return read(scal.p);
  }

  // stable sort of (keys, vals) by the low `bits` bits of the keys, in place
  void sort_pairs(uint32_t *keys, int32_t *vals, int64_t n, int bits) {
    if (n <= 1) return;
    Buf<uint32_t> k2(n);
    Buf<int32_t> v2(n), hist(pmrf_prims::sort_hist_entries(n)),
        hsums(pmrf_prims::scan_scratch(256 * pmrf_prims::sort_tiles(n)));
    const bool other = pmrf_prims::sort_pairs<uint32_t, true>(s, keys, vals, k2.p, v2.p, n, nullptr, bits, hist.p,
                                                                hsums.p);
    check();
    if (other) {
      copy(keys, k2.p, n);
      copy(vals, v2.p, n);
    }
    sync();
  }
};

int id_bits(int64_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

int64_t waves_grid(int64_t items) { return blocks_for(items, kBT / 64); }

void build_on_device(int32_t n, const int32_t *rp, const int32_t *ci, int32_t k, hipStream_t st, pmrf_hoods *hd) {
  BuildScope scope(st);
  Builder B(st);
  const int64_t G = blocks_for(std::max<int32_t>(n, 1), kBT);

  // ---- 1. the CSR
  int32_t ends[2] = {0, 0};
  BTRY(hipMemcpyAsync(&ends[0], rp, 4, hipMemcpyDeviceToHost, st));
  BTRY(hipMemcpyAsync(&ends[1], rp + n, 4, hipMemcpyDeviceToHost, st));
  B.sync();
  if (ends[0] != 0) throw BuildError{PMRF_EINVAL, "row_ptr[0] must be 0"};
  {
    Buf<int32_t> bad(5);
    k_fill<int32_t><<<1, 64, 0, st>>>(bad.p, 5, INT_MAX);
    k_check_rows<<<G, kBT, 0, st>>>(rp, n, bad.p);
    B.check();
    const int32_t r = B.read(bad.p);
    if (r != INT_MAX) throw BuildError{PMRF_EINVAL, "row_ptr must be non-decreasing (row " + std::to_string(r) + ")"};
    if (ends[1] > 0 && !ci) throw BuildError{PMRF_EINVAL, "col_idx is NULL"};
    k_check_cols<<<G, kBT, 0, st>>>(rp, ci, n, bad.p);
    B.check();
    int32_t b[5];
    BTRY(hipMemcpyAsync(b, bad.p, sizeof b, hipMemcpyDeviceToHost, st));
    B.sync();
    const int32_t first_bad = std::min({b[1], b[2], b[3]});
    if (first_bad != INT_MAX) {
      const char *what = first_bad == b[1]   ? "col_idx out of range in row "
                         : first_bad == b[2] ? "self loop at vertex "
                                             : "a row is not strictly ascending: row ";
      throw BuildError{PMRF_EINVAL, what + std::to_string(first_bad)};
    }
    if (b[4] != INT_MAX)
      throw BuildError{PMRF_EINVAL, "an edge of vertex " + std::to_string(b[4]) + " is missing its reverse"};
  }
  hd->n = n;
  hd->k = k;

  // ---- 2. maximal cliques, level by level (level 1: every vertex)
  std::vector<Buf<int32_t>> mc;
  std::vector<Level> levels;
  {
    Buf<int32_t> C(n);
    if (n) k_iota<<<G, kBT, 0, st>>>(C.p, n);
    int64_t count = n;
    for (int kk = 1; count > 0; ++kk) {
      const int64_t g = blocks_for(count, kBT);
      Buf<int64_t> ext(count + 1);
      Buf<int32_t> pos(count + 1);
      k_extend<false><<<g, kBT, 0, st>>>(C.p, count, kk, rp, ci, ext.p, pos.p, nullptr, nullptr);
      B.check();
      B.scan(ext.p, ext.p, count);
      B.scan(pos.p, pos.p, count);
      const int64_t next = B.read(ext.p + count);
      const int32_t nmax = B.read(pos.p + count);
      if (nmax) {
        Buf<int32_t> out((int64_t)kk * nmax);
        k_keep_maximal<<<g, kBT, 0, st>>>(C.p, count, kk, pos.p, out.p);
        B.check();
        levels.push_back(Level{out.p, nmax, kk, 0});
        mc.push_back(std::move(out));
      }
      if (next == 0) break;
      if ((kk + 1) * next > kMaxLevelInts)
        throw BuildError{PMRF_EUNSUPPORTED, "the graph has more than " + std::to_string(next) + " cliques of " +
                                                std::to_string(kk + 1) + " vertices: beyond the device builder"};
      Buf<int32_t> N((kk + 1) * next);
      k_extend<true><<<g, kBT, 0, st>>>(C.p, count, kk, rp, ci, nullptr, nullptr, ext.p, N.p);
      B.check();
      B.sync();
      C = std::move(N);
      count = next;
    }
  }
  int64_t H = 0;
  for (const Level &l : levels) H += l.count;
  if (H >= (int64_t(1) << 30)) throw BuildError{PMRF_EUNSUPPORTED, "more than 2^30 maximal cliques"};

  // ---- 3. canonical order
  Buf<int32_t> cptr(H + 1, kKeep), first(n);
  {
    Buf<Level> dlev((int64_t)levels.size());
    if (!levels.empty())
      BTRY(hipMemcpyAsync(dlev.p, levels.data(), levels.size() * sizeof(Level), hipMemcpyHostToDevice, st));
    if (n) k_fill<int32_t><<<G, kBT, 0, st>>>(first.p, n, INT_MAX);
    std::vector<Buf<int32_t>> ranks;
    for (size_t li = 0; li < levels.size(); ++li) {
      ranks.emplace_back(levels[li].count);
      k_rank<<<blocks_for(levels[li].count, kBT), kBT, 0, st>>>(dlev.p, (int)levels.size(), (int)li, ranks.back().p,
                                                                 cptr.p, first.p);
      B.check();
    }
    B.scan(cptr.p, cptr.p, H);
    const int64_t ctotal = B.read(cptr.p + H);
    Buf<int32_t> cvid(ctotal, kKeep);
    for (size_t li = 0; li < levels.size(); ++li)
      k_place_cliques<<<blocks_for(levels[li].count, kBT), kBT, 0, st>>>(levels[li].c, levels[li].count, levels[li].k,
                                                                          ranks[li].p, cptr.p, cvid.p);
    B.check();
    B.sync();
    hd->dev_clique_total = ctotal;
    hd->dev_clique_vid = cvid.take();
  }
  mc.clear();
  levels.clear();

  // ---- 4. neighbourhoods: the clique, then k times its members' rows
  Buf<int32_t> hptr, hvid;
  int64_t M = hd->dev_clique_total, max_hood = 0;
  {
    const int32_t *sp = cptr.p, *sv = static_cast<const int32_t *>(hd->dev_clique_vid);
    for (int32_t round = 0; round < k; ++round) {
      const int64_t E = M;
      Buf<int64_t> off(E + 1);
      k_cand_count<<<blocks_for(E, kBT), kBT, 0, st>>>(sv, E, rp, off.p);
      B.check();
      B.scan(off.p, off.p, E);
      const int64_t ctotal = B.read(off.p + E);
      if (ctotal >= INT32_MAX) throw BuildError{PMRF_EUNSUPPORTED, "neighbourhood candidates beyond 2^31"};
      Buf<int32_t> cand(ctotal);
      k_cand_write<<<blocks_for(E, kBT), kBT, 0, st>>>(sv, E, rp, ci, off.p, cand.p);
      Buf<int64_t> hcp(H + 1);
      k_hood_cand_ptr<<<blocks_for(H + 1, kBT), kBT, 0, st>>>(sp, H, off.p, hcp.p);
      B.check();
      const int64_t mx = B.max_len(hcp.p, H);
      if (mx > kCandCap)
        throw BuildError{PMRF_EUNSUPPORTED, "a neighbourhood gathers " + std::to_string(mx) +
                                                " candidate members, above the device builder's " +
                                                std::to_string(kCandCap)};
      int32_t P = 64;
      while (P < mx) P <<= 1;
      const int bd = std::min(256, std::max(64, P / 2));
      Buf<int32_t> usize(H + 1), nptr(H + 1, kKeep);
      if (H) {
        k_sort_unique<<<std::min<int64_t>(H, 1 << 16), bd, (size_t)P * 4, st>>>(cand.p, hcp.p, H, P, usize.p);
        B.check();
      }
      B.scan(usize.p, nptr.p, H);
      max_hood = B.max_len(nptr.p, H);
      M = B.read(nptr.p + H);
      if (max_hood > kMaxHood)
        throw BuildError{PMRF_EUNSUPPORTED, "a neighbourhood has " + std::to_string(max_hood) + " members (limit 1024)"};
      if (M >= (int64_t(1) << 31) / 2)
        throw BuildError{PMRF_EUNSUPPORTED, "more than 2^30 neighbourhood elements in one graph"};
      Buf<int32_t> nvid(M, kKeep);
      k_copy_segs<int64_t><<<waves_grid(H), kBT, 0, st>>>(cand.p, hcp.p, nptr.p, usize.p, H, nvid.p);
      B.check();
      B.sync();
      hptr = std::move(nptr);
      hvid = std::move(nvid);
      sp = hptr.p;
      sv = hvid.p;
    }
  }
  hd->H = H;
  hd->M = M;
  hd->max_hood = (int32_t)max_hood;
  Buf<int32_t> owner(n, kKeep);
  if (n) k_owner<<<G, kBT, 0, st>>>(first.p, n, hptr.p, hvid.p, owner.p);
  B.check();
  first.release();

  // ---- 5. processing order
  Buf<int32_t> spos(H + 1), perm(H), inv(H), psize(H + 1), pptr(H + 1);
  k_small_flag<<<blocks_for(H, kBT), kBT, 0, st>>>(hptr.p, H, spos.p);
  B.check();
  B.scan(spos.p, spos.p, H);
  const int32_t ns = B.read(spos.p + H);
  k_perm<<<blocks_for(H, kBT), kBT, 0, st>>>(hptr.p, H, spos.p, perm.p, inv.p, psize.p);
  B.check();
  B.scan(psize.p, pptr.p, H);

  // ---- 6. packets
  const int64_t nb = (H + kFitBlock - 1) / kFitBlock;
  Buf<int32_t> tile_of(H), pos_of(H);
  int64_t ntiles = 0;
  if (nb) {
    Buf<int32_t> table(nb * kFitStates * 2), entry(2 * nb);
    k_fit_table<<<nb, 128, 0, st>>>(psize.p, H, table.p);
    k_fit_chain<<<1, 64, 0, st>>>(table.p, nb, entry.p, B.scal.p);
    k_fit_assign<<<nb, 64, 0, st>>>(psize.p, H, entry.p, tile_of.p, pos_of.p);
    B.check();
    ntiles = B.read(B.scal.p);
  }
  Buf<int64_t> moff(H + 1);
  Buf<int32_t> midf(1), t_mid(std::max<int64_t>(1, ntiles)), hw(H);
  B.zero(midf.p, 1);
  B.zero(t_mid.p, std::max<int64_t>(1, ntiles));
  k_tile_mid<<<blocks_for(H, kBT), kBT, 0, st>>>(psize.p, H, tile_of.p, t_mid.p, midf.p);
  k_mask_words<<<blocks_for(H, kBT), kBT, 0, st>>>(psize.p, H, tile_of.p, t_mid.p, moff.p, hw.p);
  B.check();
  B.scan(moff.p, moff.p, H);
  const int64_t mask_words = B.read(moff.p + H);
  const bool any_mid = B.read(midf.p) != 0;
  if (mask_words >= INT32_MAX) throw BuildError{PMRF_EUNSUPPORTED, "more than 2^31 adjacency words"};
  const int64_t slot_tiles = ns < H ? B.read(tile_of.p + ns) : ntiles;

  // ---- 7. the layout, written in place
  const int64_t nchunks = (ntiles + kChunkTiles - 1) / kChunkTiles;
  const int64_t chunks_alloc = std::max<int64_t>(1, nchunks);
  const int64_t slots = chunks_alloc * kChunkTiles * kWave;
  const int64_t sc = superchunk_chunks_of(nchunks);
  const int64_t nsuper = std::max<int64_t>(1, (nchunks + sc - 1) / sc);
  LayoutSizes z{};
  z.ntiles = ntiles;
  z.H = H;
  z.M = M;
  z.mask_words = mask_words;
  z.nchdr = chunks_alloc;
  z.slots = slots;
  z.slots_hi = any_mid ? slots : 0;
  z.nsrange = 2 * nsuper;
  z.nlastbits = M / 64 + 2;
  z.nocc_ptr = (int64_t)n + 1;
  z.nocc = std::max<int64_t>(1, M);
  const DeviceLayout L = layout_of(z);
  Buf<char> lay(L.total, kKeep);
  B.zero(lay.p, L.total);
  char *base = lay.p;
  TileDesc *tiles = reinterpret_cast<TileDesc *>(base + L.tiles_off);
  int32_t *dptr = reinterpret_cast<int32_t *>(base + L.hptr_off);
  int32_t *dvid = reinterpret_cast<int32_t *>(base + L.vid_off);
  uint32_t *mask = reinterpret_cast<uint32_t *>(base + L.mask_off);
  ChunkHdr *chdr = reinterpret_cast<ChunkHdr *>(base + L.chdr_off);
  int32_t *svid = reinterpret_cast<int32_t *>(base + L.svid_off);
  uint32_t *smask = reinterpret_cast<uint32_t *>(base + L.smask_off);
  uint32_t *smask_hi = reinterpret_cast<uint32_t *>(base + L.smaskhi_off);
  int32_t *dperm = reinterpret_cast<int32_t *>(base + L.perm_off);
  int32_t *srange = reinterpret_cast<int32_t *>(base + L.srange_off);
  unsigned long long *lastbits = reinterpret_cast<unsigned long long *>(base + L.lastbits_off);
  int32_t *occ_ptr = reinterpret_cast<int32_t *>(base + L.occptr_off);
  int32_t *occ = reinterpret_cast<int32_t *>(base + L.occ_off);
  B.copy(dptr, pptr.p, H + 1);
  B.copy(dperm, perm.p, H);

  Buf<int32_t> pe_hood(M), canon_pe(M);
  k_place_proc<<<waves_grid(H), kBT, 0, st>>>(perm.p, H, hptr.p, hvid.p, pptr.p, dvid, pe_hood.p, canon_pe.p);
  B.check();
  // occurrence lists: elements in canonical order, stably sorted by vertex
  {
    Buf<uint32_t> keys(M);
    B.copy(keys.p, reinterpret_cast<const uint32_t *>(hvid.p), M);
    B.sort_pairs(keys.p, canon_pe.p, M, id_bits(n));
    B.copy(occ, canon_pe.p, M);
    // (an empty graph keeps the zeroed pointers)
    if (M) k_run_starts<<<blocks_for(M, kBT), kBT, 0, st>>>(keys.p, M, n, occ_ptr);
    B.check();
    if (n) k_lastbits<<<G, kBT, 0, st>>>(occ_ptr, occ, n, lastbits);
    B.check();
  }
  // packets
  if (ntiles) {
    Buf<unsigned long long> t_start(ntiles);
    Buf<int32_t> t_nelem(ntiles);
    B.zero(t_start.p, ntiles);
    B.zero(t_nelem.p, ntiles);
    k_tile_hoods<<<blocks_for(H, kBT), kBT, 0, st>>>(psize.p, H, tile_of.p, pos_of.p, pptr.p, moff.p, hw.p, tiles,
                                                     t_start.p, t_nelem.p);
    k_tile_finish<<<blocks_for(ntiles, kBT), kBT, 0, st>>>(ntiles, t_start.p, t_nelem.p, tiles);
    B.check();
    B.sync();
  }
  // adjacency words and the in-neighbourhood adjacency count
  B.zero(B.scal.p, 1);
  k_masks<<<blocks_for(M, kBT), kBT, 0, st>>>(M, pe_hood.p, pptr.p, perm.p, hptr.p, dvid, owner.p, rp, ci, moff.p, hw.p,
                                             mask, reinterpret_cast<unsigned long long *>(B.scal.p));
  B.check();
  hd->A = B.read(B.scal.p);
  // slot layout, chunk headers, superchunk ranges
  k_fill<int32_t><<<blocks_for(slots, kBT), kBT, 0, st>>>(svid, slots, (int32_t)kSlotEmpty);
  const int64_t Ms = ns < H ? B.read(pptr.p + ns) : M;
  k_slots<<<blocks_for(Ms, kBT), kBT, 0, st>>>(Ms, pe_hood.p, pptr.p, tile_of.p, pos_of.p, dvid, moff.p, hw.p, mask,
                                              svid, smask, smask_hi);
  if (nchunks) k_chunks<<<blocks_for(nchunks, kBT), kBT, 0, st>>>(tiles, ntiles, nchunks, (int32_t)H, chdr);
  k_srange<<<nsuper, kBT, 0, st>>>(svid, slots, sc * kChunkTiles * kWave, srange);
  B.check();
  B.sync();

  hd->ntiles = ntiles;
  hd->slot_tiles = slot_tiles;
  hd->layout = L;
  hd->dev_layout = lay.take();
  hd->dev_clique_ptr = cptr.take();
  hd->dev_hood_ptr = hptr.take();
  hd->dev_hood_vid = hvid.take();
  hd->dev_owner = owner.take();
}

}  // namespace

extern "C" pmrf_status pmrf_build_neighborhoods_device(int32_t n, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                                                       int32_t k, void *hip_stream, pmrf_hoods **out) {
  clear_error();
  if (!out) return fail(PMRF_EINVAL, "out is NULL");
  if (k < 1) return fail(PMRF_EINVAL, "k must be >= 1");
  if (k > kMaxHoodRadius) return fail(PMRF_EUNSUPPORTED, "k above " + std::to_string(kMaxHoodRadius) + " is not supported");
  if (n < 0) return fail(PMRF_EINVAL, "n must be >= 0");
  if (!d_row_ptr) return fail(PMRF_EINVAL, "row_ptr is NULL");
  if (n > kMaxSlotVertices)
    return fail(PMRF_EUNSUPPORTED, "more than " + std::to_string(kMaxSlotVertices) + " vertices in one graph");
  pmrf_hoods *hd = nullptr;
  try {
    hd = new pmrf_hoods();
    hd->on_device = true;
    if (hipGetDevice(&hd->device) != hipSuccess) throw BuildError{PMRF_EDEVICE, "no current HIP device"};
    build_on_device(n, d_row_ptr, d_col_idx, k, static_cast<hipStream_t>(hip_stream), hd);
  } catch (const BuildError &e) {
    delete hd;
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    delete hd;
    return fail(PMRF_ENOMEM, "host allocation failed while building neighbourhoods");
  }
  *out = hd;
  return PMRF_OK;
}
