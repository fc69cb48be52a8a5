// EM optimisation of DPP-PMRF on gfx950 (Alg. 2, EM loop; Sec. 3.2.2 "EM
// Parameter Estimation").
//
// k_iter works through chunks of 10 consecutive work packets (a packet is up to
// 64 elements of whole neighbourhoods).  For every packet, one lane per element
// (neighbourhood h, member v) does, for every label l:
//   - gather y_v and the current labels of the packet (label bit planes from
//     __ballot, so every lane sees its neighbourhood's labels without LDS);
//   - count in-neighbourhood neighbours per label with popcounts of its
//     adjacency bit mask against the planes (the Potts term);
//   - form the Gaussian energy and keep the minimum, the lowest arg-minimum and
//     the gap to the runner-up (the paper's SortByKey + ReduceByKey<Min>, in
//     registers: no replicated arrays exist);
//   - the owner element of each vertex writes the vertex's new label (the
//     paper's Scatter, without write conflicts) and adds y - mu to its lane's
//     per-label statistics of the parameter update;
//   - the minimum goes to LDS.
// After up to 10 packets, one lane per neighbourhood sums its members' minima in
// member order (the paper's ReduceByKey<Add>), checks the neighbourhood's
// convergence window and adds the sum to its lane's energy total.  At the end
// of a chunk the wave's lane statistics pass through LDS eight values at a
// time and are summed in a fixed order (eight lanes in order, then DPP moves)
// into the chunk's row, and the block adds its 16 rows in order into one
// record per superchunk.
// There is no cross-block communication and no memory fence inside a launch.
//
// The parameter update folds the superchunk records of an iteration in one
// fixed order (fold_stage1 / fold_stage2) and turns the totals into the next
// parameters (mean, standard deviation) and the per-iteration results.  For a
// single graph every block of iteration t's launch folds the records of t - 1
// itself (so one launch per EM iteration); otherwise k_fold (one block per
// graph) does it between the iteration launches.  Both fold in the same order,
// so the results are the same bits.
//
// Chunks and their order are fixed by the graph alone, so the results do not
// depend on the launch shape or on how graphs are batched.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pmrf_internal.h"

using namespace pmrf;

namespace {

// Pointers read from descriptors carry no address space; casting them to the
// global space keeps loads and stores off the flat path (whose waits would
// also stall LDS traffic).
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> gbl(T *p) {
  return (gptr<T>)p;
}

// ------------------------------------------------------------ device records
// statistics record: 3L + 4 doubles, stored word-major (word w of record r at
// rec[w * nrec + r]):
//   per label l: [3l] count, [3l+1] sum of (y - c_l), [3l+2] sum of (y - c_l)^2
//                (c_l = the mean used in this iteration)
//   [3L] total energy, [3L+1] near ties, [3L+2] neighbourhoods not converged,
//   [3L+3] labels out of range.
// Counts are integers below 2^53, so their double sums are exact in any order;
// every word of every record is combined with the same double addition.
__host__ __device__ constexpr int rec_words(int L) { return 3 * L + 4; }
constexpr int kRecMax = 3 * kMaxLabels + 4;

// Chunks per superchunk (one statistics record): superchunk_chunks_of keeps a
// graph at or below kFoldLanes records where it can (one record per virtual
// thread of the fold, so a single graph's fold fits the iteration launch); a
// function of the graph alone, so part of the result's definition.
constexpr int kGroupTiles = kChunkTiles;  // packets per neighbourhood-sum group (LDS buffer of 64 minima each)
// Register budgets of the two-label iteration kernels, as resident waves per
// SIMD: one graph (a single round of waves; the lower budget keeps every value
// in registers) and a batch (many rounds; one more wave hides more latency at
// the cost of one spilled value outside the packet loop).
#ifndef PMRF_ITER_WAVES_PER_EU
#define PMRF_ITER_WAVES_PER_EU 4
#endif
#ifndef PMRF_BATCH_WAVES_PER_EU
#define PMRF_BATCH_WAVES_PER_EU 5
#endif
constexpr int kVertPerBlock = 1024;

// Parameters of one label, with the two values each energy uses
// (w = 1 / (2 sigma^2), lg = ln sigma).
struct LabelTheta {
  double mu, sigma, w, lg;
};

// Per vertex, in the workspace: its intensity and its label in the two label
// buffers (iteration t reads x[t & 1] and writes x[(t + 1) & 1]), so that one
// 16-byte gather brings both values an element needs (one cache line per
// vertex instead of one per array).
struct VertexRec {
  double y;
  int32_t x[2];
};
static_assert(sizeof(VertexRec) == 16, "VertexRec layout");
typedef int32_t v4i __attribute__((ext_vector_type(4)));

struct GraphState {
  LabelTheta th[2][kMaxLabels];  // parameters of iteration t in th[t & 1]
  int32_t done;                // 1: no further iterations (early exit or error)
  int32_t status;
  int32_t iters;
  int32_t map_conv, em_conv;
  // stop[t & 1]: the run stops before iteration t (the fused launch of
  // iteration t + 1 reads it while that of t writes the other slot, so no
  // launch reads a flag that one of its own blocks writes)
  int32_t stop[2];
  int32_t pad;
  int64_t ties_total;
};

struct GraphDev {
  const TileDesc *tiles;
  const int32_t *vid;
  const uint32_t *mask;
  const ChunkHdr *chdr;  // slot layout
  const int32_t *svid;
  const uint32_t *smask, *smask_hi;
  const int32_t *hood_ptr;  // element offset of each neighbourhood, H+1 entries
  const double *y;
  int32_t *x0;    // caller labels: read at the start, written at the end
  VertexRec *vr;  // workspace: intensities and both label buffers
  double *ring;  // (W+1) x H neighbourhood sums
  double *thist;
  GraphState *st;
  double *rec;  // statistics records (chunks, or vertex blocks)
  const double *in_mu, *in_sigma;
  double *out_mu, *out_sigma, *out_S, *out_trace;
  int64_t *out_stats, *out_ctr;
  int64_t M;
  int64_t rec_stride;  // words of one record buffer (records of iteration t at rec + (t & 1) * rec_stride)
  int32_t n, H, ntiles, nchunks, nsuper, L, P, W, max_iters, early_exit, init_from_labels;
  int32_t sc;        // chunks per superchunk (record)
  int32_t bc;        // chunks per slot-kernel block (a multiple of sc)
  int32_t nslot;     // superchunks on the slot path: [0, nslot); the rest take the packet path
  int32_t slot_end;  // first chunk past the slot kernel's superchunks
  double beta, tol, sigma_min, tie_eps;
  int32_t block0, nblocks;    // slot-kernel blocks of this graph: chunks [bc b, bc (b + 1)) of [0, slot_end)
  int32_t pblock0, pnblocks;  // packet-kernel blocks: superchunks [nslot, nsuper), one each
  int32_t vblock0, vnblocks;  // blocks of this graph in a vertex-parallel launch
  const int32_t *perm;        // processing index -> canonical neighbourhood
  const int32_t *srange;      // member vertex range of superchunk s: [srange[2 s], srange[2 s + 1])
  int32_t rule;               // scatter rule (PMRF_SCATTER_*)
  int32_t nrec;               // statistics records per iteration: superchunks, then (rule MIN) vertex blocks
  const uint64_t *lastbits;   // rule LAST: element holds its vertex's last occurrence
  const int32_t *occ_ptr, *occ;  // rule MIN: each vertex's elements in canonical order
  double *em, *eg;            // rule MIN: per element (processing order) minimum energy and gap
  int32_t *ea;                //           and arg-minimum label
};

constexpr int kDescPerPack = 12;
struct DescPack {
  GraphDev d[kDescPerPack];
  int32_t first, count;
};

// Order the wave's own LDS writes before its LDS reads (a single wave executes
// its LDS instructions in order; this also stops the compiler moving them).
// The calling thread's wave within its block.  The value is the same on every
// lane, which the compiler cannot see from threadIdx.x alone; reading it from
// the first lane keeps it (and all chunk bookkeeping derived from it) in
// scalar registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Sums across the 64 lanes in one fixed order, with DPP lane moves (no trip
// through the LDS crossbar): pairs, quads, half rows and rows combine inside
// each row of 16 (every lane of a row ends with the row's sum; a + b and b + a
// round alike), then row 0 joins row 1 and row 2 joins row 3 (row_bcast15),
// then rows 0+1 join rows 2+3 (row_bcast31).  Lane 63 holds
// ((r3 + r2) + (r1 + r0)), which readlane hands to every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_i64(long long x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffff), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWS, 0xf, false);
  return ((long long)hi << 32) | (unsigned)lo;
}
constexpr int kDppSwap1 = 0xb1;           // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4e;           // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;     // row_half_mirror
constexpr int kDppMirror = 0x140;         // row_mirror
constexpr int kDppBcast15 = 0x142;        // row_bcast:15
constexpr int kDppBcast31 = 0x143;        // row_bcast:31
__device__ __forceinline__ double wave_sum(double v) {
  v = v + dpp_f64<kDppSwap1, 0xf>(v);
  v = v + dpp_f64<kDppSwap2, 0xf>(v);
  v = v + dpp_f64<kDppHalfMirror, 0xf>(v);
  v = v + dpp_f64<kDppMirror, 0xf>(v);
  v = v + dpp_f64<kDppBcast15, 0xa>(v);  // rows 1 and 3 (others add 0)
  v = v + dpp_f64<kDppBcast31, 0xc>(v);  // rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ long long wave_sum(long long v) {
  v = v + dpp_i64<kDppSwap1, 0xf>(v);
  v = v + dpp_i64<kDppSwap2, 0xf>(v);
  v = v + dpp_i64<kDppHalfMirror, 0xf>(v);
  v = v + dpp_i64<kDppMirror, 0xf>(v);
  v = v + dpp_i64<kDppBcast15, 0xa>(v);
  v = v + dpp_i64<kDppBcast31, 0xc>(v);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), 63);
  return ((long long)hi << 32) | (unsigned)lo;
}

template <int LMAX>
struct LaneStats {
  int cnt[LMAX];
  double s1[LMAX], s2[LMAX];
  double T;
  int ties, nonconv, err;
  __device__ void clear() {
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
      cnt[l] = 0;
      s1[l] = 0.0;
      s2[l] = 0.0;
    }
    T = 0.0;
    ties = nonconv = err = 0;
  }
  // owner element with label a and d = y - mu_a
  __device__ __forceinline__ void add_owner(int a, double d) {
    const double d2 = d * d;
#pragma unroll
    for (int l = 0; l < LMAX; ++l)
      if (a == l) {
        cnt[l] += 1;
        s1[l] = s1[l] + d;
        s2[l] = s2[l] + d2;
      }
  }
  // wave-reduce and store one record (lane 0 writes word w at rec[w * stride]);
  // Ptr is a global or LDS pointer
  template <typename Ptr>
  __device__ void store(Ptr rec, size_t stride, int L, int lane) {
#pragma unroll
    for (int l = 0; l < LMAX; ++l)
      if (l < L) {
        long long c = wave_sum((long long)cnt[l]);
        double a = wave_sum(s1[l]);
        double b = wave_sum(s2[l]);
        if (lane == 0) {
          rec[(3 * l) * stride] = (double)c;
          rec[(3 * l + 1) * stride] = a;
          rec[(3 * l + 2) * stride] = b;
        }
      }
    double t = wave_sum(T);
    long long ti = wave_sum((long long)ties), nc = wave_sum((long long)nonconv);
    const int e = __popcll(__ballot(err != 0));
    if (lane == 0) {
      rec[(3 * L) * stride] = t;
      rec[(3 * L + 1) * stride] = (double)ti;
      rec[(3 * L + 2) * stride] = (double)nc;
      rec[(3 * L + 3) * stride] = (double)e;
    }
  }
};

// Totals of a graph's statistics records in a fixed order that depends on the
// record count alone (not on the block size):
//   stage 1: virtual thread v (0 .. 255) adds records v, v + 256, v + 512, ...
//            in that order, one partial sum per word;
//   stage 2: for word w, lane k (0 .. 15) of a row of 16 lanes adds the
//            partials of virtual threads 16 k .. 16 k + 15 in order, and the
//            16 lanes combine with pair, quad, half-row and row moves (every
//            lane of the row ends with the same value: a + b and b + a round
//            alike).
// A block of nw waves plays virtual wave q (virtual threads 64 q .. 64 q + 63)
// with its wave q mod nw.  The partials pass through LDS transposed (slot of
// virtual thread v: 16 (v mod 16) + v / 16), so stage 2 reads consecutive
// addresses across a row.
constexpr int kFoldLanes = kMaxRecordsPerPass;  // virtual threads of stage 1 (256)
constexpr int kFoldThreads = 256;  // block size of the fold kernels
constexpr int kFoldGroup = 16;     // words folded per pass (LDS: 16 x 256 doubles)

__device__ __forceinline__ int fold_slot(int w, int v) { return w * kFoldLanes + (v & 15) * 16 + (v >> 4); }

// Stage 1 for words [w0, w0 + nwords) (nwords <= kFoldGroup) of records laid
// out word-major (word w of record r at rec[w * R + r]); partials to scr.
__device__ __forceinline__ void fold_stage1(gptr<const double> rec, int R, int w0, int nwords, double *scr, int nw,
                                            int wave, int lane) {
  constexpr int WG = 8;  // loads requested together
  for (int q = wave; q < kFoldLanes / 64; q += nw) {
    const int v = q * 64 + lane;
    for (int wg = 0; wg < nwords; wg += WG) {
      double acc[WG];
#pragma unroll
      for (int j = 0; j < WG; ++j) acc[j] = 0.0;
      for (int r = v; r < R; r += kFoldLanes) {
        double x[WG];
#pragma unroll
        for (int j = 0; j < WG; ++j) x[j] = wg + j < nwords ? rec[(size_t)(w0 + wg + j) * R + r] : 0.0;
#pragma unroll
        for (int j = 0; j < WG; ++j) acc[j] = acc[j] + x[j];
      }
#pragma unroll
      for (int j = 0; j < WG; ++j)
        if (wg + j < nwords) scr[fold_slot(wg + j, v)] = acc[j];
    }
  }
}

// Stage 2 for nwords words whose partials are in scr; totals to tot[0 .. nwords).
__device__ __forceinline__ void fold_stage2(const double *scr, int nwords, double *tot, int nw, int wave, int lane) {
  for (int i0 = wave * 64; i0 < 16 * nwords; i0 += nw * 64) {
    const int i = i0 + lane, w = i >> 4, k = i & 15;
    double s = 0.0;
    if (w < nwords) {
      const double *p = scr + w * kFoldLanes + k;
      double r[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) r[j] = p[j * 16];
#pragma unroll
      for (int j = 0; j < 16; ++j) s = s + r[j];
    }
    s = s + dpp_f64<kDppSwap1, 0xf>(s);
    s = s + dpp_f64<kDppSwap2, 0xf>(s);
    s = s + dpp_f64<kDppHalfMirror, 0xf>(s);
    s = s + dpp_f64<kDppMirror, 0xf>(s);
    if (k == 0 && w < nwords) tot[w] = s;
  }
}

// Both stages over all words, by every thread of the block; on return tot[]
// is visible to the whole block.  scr: kFoldGroup * kFoldLanes doubles of LDS.
__device__ __forceinline__ void fold_all(gptr<const double> rec, int R, int words, double *scr, double *tot, int nw,
                                         int wave, int lane) {
  for (int w0 = 0; w0 < words; w0 += kFoldGroup) {
    const int nwords = min(kFoldGroup, words - w0);
    fold_stage1(rec, R, w0, nwords, scr, nw, wave, lane);
    __syncthreads();
    fold_stage2(scr, nwords, tot + w0, nw, wave, lane);
    __syncthreads();
  }
}

__device__ __forceinline__ void set_label_theta(LabelTheta *s, int l, double mu, double sigma) {
  s[l].mu = mu;
  s[l].sigma = sigma;
  s[l].w = 1.0 / (2.0 * sigma * sigma);
  s[l].lg = log(sigma);
}

// Parameters for the next iteration from the per-label sums ("Update
// Parameters"): mu = c + D1, sigma^2 = D2 - D1^2 with D1 = sum(y - c)/n,
// D2 = sum((y - c)^2)/n, c = the mean used this iteration (pass 0 of the
// starting update uses c = 0 and keeps sigma).  A label with no vertex keeps
// its parameters.  One label: (mu, sigma, w, lg) hold its parameters of this
// iteration on entry and the next ones on return.
__device__ __forceinline__ void next_label_theta(double nd, double s1, double s2, double sigma_min, bool mean_only,
                                                 double &mu, double &sigma, double &w, double &lg) {
  if (!(nd > 0.0)) return;
  const double d1 = s1 / nd;
  double m, sg;
  if (mean_only) {
    m = d1;
    sg = sigma;
  } else {
    const double d2 = s2 / nd;
    const double var = d2 - d1 * d1;
    const double r = sqrt(var > 0.0 ? var : 0.0);
    m = mu + d1;
    sg = r < sigma_min ? sigma_min : r;
  }
  mu = m;
  sigma = sg;
  w = 1.0 / (2.0 * sg * sg);
  lg = log(sg);
}

// All labels, by one thread (s: parameters of this iteration on entry, the
// next ones on return).
__device__ __forceinline__ void update_theta(LabelTheta *s, const double *tot, int L, double sigma_min,
                                             bool mean_only) {
  for (int l = 0; l < L; ++l) {
    double mu = s[l].mu, sg = s[l].sigma, w = s[l].w, lg = s[l].lg;
    next_label_theta(tot[3 * l], tot[3 * l + 1], tot[3 * l + 2], sigma_min, mean_only, mu, sg, w, lg);
    s[l].mu = mu;
    s[l].sigma = sg;
    s[l].w = w;
    s[l].lg = lg;
  }
}

// Graph owning a block: the last graph whose first block is <= block.
enum GridKind { kGridSlot = 0, kGridVertex = 1, kGridPacket = 2 };
__device__ __forceinline__ int find_graph(const GraphDev *graphs, int B, int block, int grid) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    int first = grid == kGridVertex ? graphs[mid].vblock0 : grid == kGridPacket ? graphs[mid].pblock0 : graphs[mid].block0;
    if (first <= block) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Workgroups are dealt to the chip's XCDs round-robin (workgroup i on XCD
// i % kXcds), and each XCD has its own L2.  The block that workgroup i plays is
// chosen so that each XCD takes one contiguous run of blocks: neighbouring
// superchunks gather mostly the same vertices, which then stay in one L2
// instead of being fetched by every XCD.  A bijection on [0, grid), so any
// device (or a different dealing order) still gets every block exactly once.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int i, int grid) {
  const int q = grid / kXcds, r = grid % kXcds;
  const int x = i % kXcds, k = i / kXcds;
  return x * q + min(x, r) + k;
}

// ------------------------------------------------------------- tile kernels
template <int LMAX>
struct Theta {
  double mu[LMAX], w[LMAX], lg[LMAX];
};

// What one iteration launch needs of a graph, in registers.
struct Ctx {
  gptr<const TileDesc> tiles;
  gptr<const int32_t> vid;
  gptr<const uint32_t> mask;
  gptr<const ChunkHdr> chdr;
  gptr<const int32_t> svid;
  gptr<const uint32_t> smask, smask_hi;
  gptr<const int32_t> hood_ptr;
  gptr<const VertexRec> vr;  // intensities and labels
  gptr<int32_t> xw;          // labels written this iteration: xw[4 v] (x[(t + 1) & 1] of vertex v)
  int par;                   // label buffer read this iteration (t & 1)
  gptr<double> ring;
  gptr<const GraphState> st;
  int H, W, L, P, t, ntiles, nchunks;
  int rule;
  gptr<const uint64_t> lastbits;
  gptr<double> em, eg;
  gptr<int32_t> ea;
  double beta, tol, tie_eps;
};

constexpr int kRuleOwner = PMRF_SCATTER_OWNER, kRuleLast = PMRF_SCATTER_LAST, kRuleMin = PMRF_SCATTER_MIN;

// Whether element e (processing order) decides its vertex's label, for the
// rules other than the owner's (whose flag is the element's own adjacency bit).
__device__ __forceinline__ bool decides(const Ctx &c, int e) {
  return c.rule == kRuleLast && ((c.lastbits[e >> 6] >> (e & 63)) & 1);
}
// Rule MIN: the element's minimum energy, arg-minimum and gap, for the vertex pass.
__device__ __forceinline__ void record_elem(const Ctx &c, int e, double m, int a, double gap) {
  c.em[e] = m;
  c.ea[e] = a;
  c.eg[e] = gap;
}

// Label (read buffer) and intensity of vertex v: one 16-byte load.
__device__ __forceinline__ void vrec_load(const Ctx &c, unsigned v, int &x, double &y) {
  const v4i q = *(gptr<const v4i>)(c.vr + v);
  y = __longlong_as_double(((long long)q.y << 32) | (unsigned)q.x);
  x = c.par ? q.w : q.z;
}
__device__ __forceinline__ void vrec_store_label(const Ctx &c, int v, int a) { c.xw[4 * (size_t)v] = a; }

__device__ __forceinline__ TileDesc load_tile(gptr<const TileDesc> p) {
  TileDesc td;
  td.start_mask = p->start_mask;
  td.elem_start = p->elem_start;
  td.hood_start = p->hood_start;
  td.mask_start = p->mask_start;
  td.nelem = p->nelem;
  td.kind = p->kind;
  td.words = p->words;
  return td;
}

// Energies of one element under every label; returns min, argmin, gap and
// y - mu of the argmin label.
template <int LMAX>
__device__ __forceinline__ void element_energy(const Theta<LMAX> &th, int L, double beta, double yv, int deg,
                                               const int *cnt, double &m, int &a, double &gap, double &dsel) {
  m = 0.0;
  a = 0;
  double second = INFINITY;
  dsel = 0.0;
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    if (l < L) {
      double d = yv - th.mu[l];
      double en = (d * d) * th.w[l] + th.lg[l];
      en = en + beta * (double)(deg - cnt[l]);
      if (l == 0) {
        m = en;
        dsel = d;
      } else if (en < m) {
        second = m;
        m = en;
        a = l;
        dsel = d;
      } else if (en < second) {
        second = en;
      }
    }
  }
  gap = second - m;
}

// Convergence window of one neighbourhood: |S - S^{t-w}| < tol for w = 1..W.
__device__ __forceinline__ bool hood_converged(const Ctx &c, int h, double S) {
  const int slots = c.W + 1;
  c.ring[(size_t)(c.t % slots) * c.H + h] = S;
  if (c.t < c.W) return false;
  bool conv = true;
  for (int w = 1; w <= c.W; ++w) {
    double prev = c.ring[(size_t)((c.t - w) % slots) * c.H + h];
    if (!(fabs(S - prev) < c.tol)) conv = false;
  }
  return conv;
}

// Per-lane data of one packet, loaded ahead of its computation.
struct Stream {
  int v;
  uint64_t am;
};
struct Gather {
  int xv;
  double yv;
};

__device__ __forceinline__ Stream load_stream(const Ctx &c, const TileDesc &td, int lane) {
  Stream r{0, 0};
  if (td.kind != kLarge && lane < td.nelem) {
    r.v = c.vid[td.elem_start + lane];
    if (td.words == 1)
      r.am = c.mask[td.mask_start + lane];
    else
      r.am = (uint64_t)c.mask[td.mask_start + 2 * lane] | ((uint64_t)c.mask[td.mask_start + 2 * lane + 1] << 32);
  }
  return r;
}

__device__ __forceinline__ Gather load_gather(const Ctx &c, const TileDesc &td, const Stream &st, int lane) {
  Gather r{0, 0.0};
  if (td.kind != kLarge && lane < td.nelem) {
    vrec_load(c, (unsigned)st.v, r.xv, r.yv);
  }
  return r;
}

// Element pass of a packet of whole neighbourhoods of at most 64 members
// (kinds SMALL, MID): minimum energies into mb[e - gstart].
template <int LMAX>
__device__ __forceinline__ void elem_pass(const Ctx &c, const TileDesc &td, const Stream &sd, const Gather &gd,
                                          int gstart, const Theta<LMAX> &th, LaneStats<LMAX> &ls, double *mb,
                                          int lane) {
  const bool valid = lane < td.nelem;
  const int e = td.elem_start + lane;
  const int v = sd.v, xv = gd.xv;
  const uint64_t am = sd.am;
  const double yv = gd.yv;
  if (valid && (unsigned)xv >= (unsigned)c.L) ls.err |= 1;
  uint64_t planes[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < c.P) planes[k] = __ballot(valid && ((xv >> k) & 1));
  const uint64_t below = (2ull << lane) - 1ull;  // lanes 0..lane
  const int base = 63 - __clzll(td.start_mask & below);
  const uint64_t self = 1ull << (lane - base);
  const bool owner = valid && (c.rule == kRuleOwner ? (am & self) != 0 : decides(c, e));
  const uint64_t nbr = am & ~self;
  const int deg = __popcll(nbr);
  int cnt[LMAX];
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    uint64_t eq = ~0ull;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < c.P) {
        uint64_t pk = planes[k] >> base;
        eq &= ((l >> k) & 1) ? pk : ~pk;
      }
    cnt[l] = __popcll(nbr & eq);
  }
  double m, gap, dsel;
  int a;
  element_energy<LMAX>(th, c.L, c.beta, yv, deg, cnt, m, a, gap, dsel);
  if (owner) {
    vrec_store_label(c, v, a);
    ls.add_owner(a, dsel);
    if (gap < c.tie_eps) ls.ties += 1;
  }
  if (c.rule == kRuleMin && valid) record_elem(c, e, m, a, gap);
  if (valid) mb[e - gstart] = m;
}

// Neighbourhood pass: neighbourhoods [h0, h1) whose elements start at gstart,
// one lane each: member-order sum, convergence window, energy total.
template <int LMAX>
__device__ __forceinline__ void hood_pass(const Ctx &c, int h0, int h1, int gstart, LaneStats<LMAX> &ls,
                                          const double *mb, int lane) {
  wave_lds_sync();
  const int slots = c.W + 1;
  const bool window = c.t >= c.W;
  for (int hb = h0; hb < h1; hb += 64) {
    const int h = hb + lane;
    const bool act = h < h1;
    int o = 0, s = 0;
    double prev[kMaxWindow];
    if (act) {
      const int p0 = c.hood_ptr[h];
      o = p0 - gstart;
      s = c.hood_ptr[h + 1] - p0;
      if (window) {
#pragma unroll
        for (int w = 1; w <= kMaxWindow; ++w)
          if (w <= c.W) prev[w - 1] = c.ring[(size_t)((c.t - w) % slots) * c.H + h];
      }
    }
    double S = 0.0;
    for (int k = 0; __ballot(k < s); k += 4) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (k + i < s) S = S + mb[o + k + i];
    }
    if (act) {
      c.ring[(size_t)(c.t % slots) * c.H + h] = S;
      bool conv = window;
      if (window) {
#pragma unroll
        for (int w = 1; w <= kMaxWindow; ++w)
          if (w <= c.W && !(fabs(S - prev[w - 1]) < c.tol)) conv = false;
      }
      if (!conv) ls.nonconv += 1;
      ls.T = ls.T + S;
    }
  }
  wave_lds_sync();
}

// One neighbourhood of 65..1024 members, in chunks of 64 (kind LARGE).
template <int LMAX>
__device__ void do_large(const Ctx &c, const TileDesc &td, const Theta<LMAX> &th, LaneStats<LMAX> &ls, double *mb,
                         uint64_t *pl /* 4 x 16 words */, int lane) {
  const int s = td.nelem;
  const int W = td.words;
  const int chunks = (s + 63) >> 6;
  wave_lds_sync();
  for (int ch = 0; ch < chunks; ++ch) {
    const int jj = ch * 64 + lane;
    int xv = 0;
    const bool valid = jj < s;
    if (valid) {
      double unused;
      vrec_load(c, (unsigned)c.vid[td.elem_start + jj], xv, unused);
      if ((unsigned)xv >= (unsigned)c.L) ls.err |= 1;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < c.P) {
        uint64_t b = __ballot(valid && ((xv >> k) & 1));
        if (lane == 0) pl[k * 16 + ch] = b;
      }
  }
  wave_lds_sync();
  double S = 0.0;  // lane 0 accumulates in member order
  for (int ch = 0; ch < chunks; ++ch) {
    const int jj = ch * 64 + lane;
    const bool valid = jj < s;
    int v = 0;
    double yv = 0.0;
    int cnt[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) cnt[l] = 0;
    int deg = 0;
    bool owner = false;
    if (valid) {
      v = c.vid[td.elem_start + jj];
      int unused;
      vrec_load(c, (unsigned)v, unused, yv);
      gptr<const uint32_t> mw = c.mask + td.mask_start + (size_t)jj * W;
      for (int wi = 0; wi < W; ++wi) {
        uint32_t word = mw[wi];
        if (wi == (jj >> 5)) {
          const uint32_t selfb = 1u << (jj & 31);
          owner = c.rule == kRuleOwner ? (word & selfb) != 0 : decides(c, td.elem_start + jj);
          word &= ~selfb;
        }
        deg += __popc(word);
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
          uint32_t eq = ~0u;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < c.P) {
              uint32_t pk = (uint32_t)(pl[k * 16 + (wi >> 1)] >> ((wi & 1) * 32));
              eq &= ((l >> k) & 1) ? pk : ~pk;
            }
          cnt[l] += __popc(word & eq);
        }
      }
    }
    double m, gap, dsel;
    int a;
    element_energy<LMAX>(th, c.L, c.beta, yv, deg, cnt, m, a, gap, dsel);
    if (owner) {
      vrec_store_label(c, v, a);
      ls.add_owner(a, dsel);
      if (gap < c.tie_eps) ls.ties += 1;
    }
    if (c.rule == kRuleMin && valid) record_elem(c, td.elem_start + jj, m, a, gap);
    mb[lane] = valid ? m : 0.0;
    wave_lds_sync();
    if (lane == 0) {
      const int lim = min(64, s - ch * 64);
      for (int k = 0; k < lim; ++k) S = S + mb[k];
    }
    wave_lds_sync();
  }
  if (lane == 0) {
    if (!hood_converged(c, td.hood_start, S)) ls.nonconv += 1;
    ls.T = ls.T + S;
  }
}

// Neighbourhood pass over [h0, h1) with the first 64 neighbourhoods' offsets
// and window values already loaded, used by the chunk fast path.
constexpr int kPreWindow = 4;  // window values prefetched (larger windows take the plain pass)
struct HoodPre {
  int p0, p1;  // hood_ptr[h], hood_ptr[h + 1] as loaded (the size is formed where it is used)
  double prev[kPreWindow];
};


__device__ __forceinline__ int bcast(int v, int lane_src) { return __builtin_amdgcn_readlane(v, lane_src); }

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ---------------------------------------------------------------- lean path
// Per-wave LDS: 512 minima, 64 label-plane words (LARGE packets), and an owner
// list of kOwnCap entries (y - mu_a as double, a as int).
constexpr int kOwnCap = 128;
constexpr int kWaveLds = kGroupTiles * 64 + 64 + kOwnCap + kOwnCap / 2;  // in doubles
static_assert(kGroupTiles * 64 + 64 + 7 <= kWaveLds, "neighbourhood sums read up to 7 minima past 64 members");
static_assert(kGroupTiles * 64 >= 8 * 64, "record rows pass eight values through the minima buffer");

template <int LMAX>
struct ChunkStats {
  double s1[LMAX], s2[LMAX];  // per lane: sums of (y - mu_a), (y - mu_a)^2 of the owners it took
  int cnt[LMAX];
  double T;                   // per lane: sum of the neighbourhood totals it took
  int ties, nonconv, err;     // uniform across the wave
  __device__ void clear() {
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
      s1[l] = 0.0;
      s2[l] = 0.0;
      cnt[l] = 0;
    }
    T = 0.0;
    ties = nonconv = err = 0;
  }
  // owner entries k (in list order) go to lane k % 64, in order
  __device__ void take_owners(const double *od, const int *oa, int count, int lane) {
    for (int k0 = 0; k0 < count; k0 += 64) {
      const int k = k0 + lane;
      if (k < count) {
        const double d = od[k];
        const int a = oa[k];
        const double d2 = d * d;
#pragma unroll
        for (int l = 0; l < LMAX; ++l)
          if (a == l) {
            cnt[l] += 1;
            s1[l] = s1[l] + d;
            s2[l] = s2[l] + d2;
          }
      }
    }
  }
  // Value v of a lane's statistics: for label l = v / 3 its owner count
  // (v % 3 == 0), sum of y - mu (1) and of its square (2); v = 3 LMAX is the
  // sum of neighbourhood totals.
  static constexpr int kValues = 3 * LMAX + 1;
  __device__ __forceinline__ double value(int v) const {
    if (v == 3 * LMAX) return T;
    const int l = v / 3;
    return v % 3 == 0 ? (double)cnt[l] : v % 3 == 1 ? s1[l] : s2[l];
  }
  // Record row of the chunk (LDS), in a fixed order: eight values at a time
  // pass through the wave's scratch buf (>= 8 * 64 doubles) transposed;
  // lane 8 v + q adds lanes 8 q .. 8 q + 7 of value v in lane order, and the
  // eight lanes of value v combine with pair, quad and half-row moves.  Lane
  // 8 v writes value v.  The caller has synchronised buf.
  __device__ void store(double *row, double *buf, int L, int lane) {
#pragma unroll
    for (int v0 = 0; v0 < kValues; v0 += 8) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (v0 + i < kValues) buf[i * 64 + lane] = value(v0 + i);
      wave_lds_sync();
      const int vi = lane >> 3, q = lane & 7;
      const double *src = buf + vi * 64 + q * 8;
      double p = 0.0;
      if (v0 + vi < kValues) {
        double r[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) r[i] = src[i];
#pragma unroll
        for (int i = 0; i < 8; ++i) p = p + r[i];
      }
      p = p + dpp_f64<kDppSwap1, 0xf>(p);
      p = p + dpp_f64<kDppSwap2, 0xf>(p);
      p = p + dpp_f64<kDppHalfMirror, 0xf>(p);
      const int v = v0 + vi;
      if (q == 0 && v < kValues) {
        const int l = v / 3;
        if (v == 3 * LMAX) row[3 * L] = p;
        else if (l < L) row[v] = p;
      }
      wave_lds_sync();  // buf is rewritten by the next eight values
    }
    const int e = __popcll(__ballot(err != 0));
    if (lane == 0) {
      row[3 * L + 1] = (double)ties;
      row[3 * L + 2] = (double)nonconv;
      row[3 * L + 3] = (double)e;
    }
  }
};

// Whether the slot path requests the second adjacency words of MID packets
// with the gathers (more registers) or when the packet is computed (one more
// wait per MID packet).  Two-label kernels keep their register budget.
template <int LMAX>
constexpr bool kPrefetchHi = LMAX >= 4;

// Element pass of one SMALL or MID packet on the slot layout.  sv is the slot
// word (member vertex in bits 0..25, the member's index j inside its
// neighbourhood in bits 26..31, all ones for an unused slot), so the lane of
// the neighbourhood's first member is lane - j.  eoff: the packet's first
// element relative to the chunk; am: the element's first adjacency word; the
// second word of a MID packet is prefetched (ah) or read here.
template <int LMAX>
__device__ __forceinline__ void slot_elem(const Ctx &c, int e0, int eoff, bool mid, int ti, uint32_t sv, uint32_t am,
                                          uint32_t ah, int xv, double yv, const Theta<LMAX> &th,
                                          ChunkStats<LMAX> &cs, double *mb, double *od, int *oa, int &ocount,
                                          int lane) {
  constexpr int PMAX = LMAX <= 2 ? 1 : LMAX <= 4 ? 2 : LMAX <= 8 ? 3 : 4;  // label bit planes
  const bool valid = sv != kSlotEmpty;
  const int v = (int)(sv & kSlotVidMask);
  const int j = (int)(sv >> kSlotJShift);
  const int base = lane - j;
  if (valid && (unsigned)xv >= (unsigned)c.L) cs.err |= 1;
  // all PMAX planes: for valid labels (below L) the planes past the graph's
  // own count are zero, and an invalid label fails the run anyway.  Plane bits
  // of empty slots are never read: they are reached only through adjacency
  // bits, which name members of the same neighbourhood.
  uint64_t planes[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) planes[k] = __ballot((xv >> k) & 1);
  int deg, cnt[LMAX];
  uint32_t own;  // the element's own bit: set for the owner element of its vertex
  if (!mid) {
    const uint32_t self = 1u << (j & 31);  // j < 32 in a SMALL packet (empty slots carry 63)
    own = am & self;
    const uint32_t nbr = am & ~self;
    deg = __popc(nbr);
    if constexpr (LMAX == 2) {  // neighbours with label 1; the rest have label 0
      cnt[1] = __popc(nbr & (uint32_t)(planes[0] >> base));
      cnt[0] = deg - cnt[1];
    } else {
#pragma unroll
      for (int l = 0; l < LMAX; ++l) {
        uint32_t eq = ~0u;
#pragma unroll
        for (int k = 0; k < PMAX; ++k)
        {
          const uint32_t pk = (uint32_t)(planes[k] >> base);
          eq &= ((l >> k) & 1) ? pk : ~pk;
        }
        cnt[l] = __popc(nbr & eq);
      }
    }
  } else {
    const uint32_t hi = kPrefetchHi<LMAX> ? ah : c.smask_hi[(size_t)ti * kWave + lane];
    const uint64_t a64 = (uint64_t)am | ((uint64_t)hi << 32);
    const uint64_t self = 1ull << j;
    own = (a64 & self) != 0;
    const uint64_t nbr = a64 & ~self;
    deg = __popcll(nbr);
    if constexpr (LMAX == 2) {
      cnt[1] = __popcll(nbr & (planes[0] >> base));
      cnt[0] = deg - cnt[1];
    } else {
#pragma unroll
      for (int l = 0; l < LMAX; ++l) {
        uint64_t eq = ~0ull;
#pragma unroll
        for (int k = 0; k < PMAX; ++k)
        {
          const uint64_t pk = planes[k] >> base;
          eq &= ((l >> k) & 1) ? pk : ~pk;
        }
        cnt[l] = __popcll(nbr & eq);
      }
    }
  }
  // empty slots have no adjacency bits; e0 + lane is the element's index
  const bool owner = c.rule == kRuleOwner ? own != 0 : valid && decides(c, e0 + lane);
  double m, gap, dsel;
  int a;
  if constexpr (LMAX == 2) {
    const double d0 = yv - th.mu[0], d1 = yv - th.mu[1];
    double e0 = (d0 * d0) * th.w[0] + th.lg[0];
    double e1 = (d1 * d1) * th.w[1] + th.lg[1];
    e0 = e0 + c.beta * (double)(deg - cnt[0]);
    e1 = e1 + c.beta * (double)(deg - cnt[1]);
    const bool one = e1 < e0;
    a = one ? 1 : 0;
    m = one ? e1 : e0;
    gap = fabs(e1 - e0);  // the runner-up minus the minimum
    dsel = one ? d1 : d0;
  } else {
    element_energy<LMAX>(th, c.L, c.beta, yv, deg, cnt, m, a, gap, dsel);
  }
  if (c.rule == kRuleMin && valid) record_elem(c, e0 + lane, m, a, gap);
  const uint64_t ob = __ballot(owner);
  if (ob) {
    const int idx = ocount + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ob >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)ob, 0u));
    if (owner) {
      vrec_store_label(c, v, a);
      od[idx] = dsel;
      oa[idx] = a;
    }
    ocount += __popcll(ob);
    cs.ties += __popcll(ob & __ballot(gap < c.tie_eps));
  }
  if (valid) mb[eoff + lane] = m;
}

// Neighbourhood pass of the lean path: lane per neighbourhood, offsets and
// window values of the first 64 already loaded.
template <int LMAX>
__device__ __forceinline__ void lean_hoods(const Ctx &c, int h0, int h1, int gstart, const HoodPre &pre,
                                           ChunkStats<LMAX> &cs, const double *mb, int lane) {
  const int slots = c.W + 1;
  const bool window = c.t >= c.W;
  for (int hb = h0; hb < h1; hb += 64) {
    const int h = hb + lane;
    const bool act = h < h1;
    int o = 0, s = 0;
    double prev[kPreWindow];
    if (hb == h0) {
      o = pre.p0 - gstart;
      s = act ? pre.p1 - pre.p0 : 0;
#pragma unroll
      for (int w = 0; w < kPreWindow; ++w) prev[w] = pre.prev[w];
    } else if (act) {
      const int p0 = c.hood_ptr[h];
      o = p0 - gstart;
      s = c.hood_ptr[h + 1] - p0;
      if (window)
#pragma unroll
        for (int w = 1; w <= kPreWindow; ++w)
          if (w <= c.W) prev[w - 1] = c.ring[(size_t)((c.t - w) % slots) * c.H + h];
    }
    // eight minima per step, requested together; a lane whose neighbourhood
    // has ended keeps its sum.  The reads past a neighbourhood stay inside the
    // wave's LDS region: o < kGroupTiles * 64 and k + 7 < 64 + 7 (no
    // neighbourhood on this path has more than 64 members).
    if (!act) o = 0;
    double S = 0.0;
    for (int k = 0; __ballot(k < s); k += 8) {
      double m8[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) m8[i] = mb[o + k + i];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double S1 = S + m8[i];
        S = k + i < s ? S1 : S;
      }
    }
    bool conv = true;
    if (act) {
      c.ring[(size_t)(c.t % slots) * c.H + h] = S;
      conv = window;
      if (window)
#pragma unroll
        for (int w = 1; w <= kPreWindow; ++w)
          if (w <= c.W && !(fabs(S - prev[w - 1]) < c.tol)) conv = false;
      cs.T = cs.T + S;
    }
    cs.nonconv += __popcll(__ballot(act && !conv));
  }
}

// Run state and parameters of iteration c.t (uniform scalar loads); every slot
// holds kMaxLabels >= LMAX entries.
template <int LMAX>
__device__ __forceinline__ int load_theta(const Ctx &c, Theta<LMAX> &th) {
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    th.mu[l] = c.st->th[c.t & 1][l].mu;
    th.w[l] = c.st->th[c.t & 1][l].w;
    th.lg[l] = c.st->th[c.t & 1][l].lg;
  }
  return c.st->done;
}

// ------------------------------------------------------------- LDS staging
// A slot-kernel block stages the intensities (double) and current labels
// (byte) of its member vertex range [lo, lo + span) in LDS with coalesced
// loads when the range holds at most kStageCap vertices (the neighbourhoods of
// a run of consecutive cliques of an image graph cover a few rows of regions),
// and its elements then read LDS instead of gathering from memory one
// vertex per lane.  A wider range gathers from memory as before.  The range of
// each superchunk comes with the graph's device layout.
constexpr int kStageCap = 3072;
constexpr int kStageDoubles = kStageCap + kStageCap / 8;  // LDS of the staged range, in doubles
constexpr int kStagePerThread = 3;                         // entries a thread requests together

struct Stage {
  int lo, span;
  bool on;  // uniform across the block
};

// The member range of chunks [c0, c1) (whole superchunks): scalar loads.
__device__ __forceinline__ Stage block_stage(const GraphDev &G, int c0, int c1) {
  const int sc = G.sc;
  const int s0 = c0 / sc, s1 = max(s0 + 1, (c1 + sc - 1) / sc);
  gptr<const int32_t> r = gbl(G.srange);
  int lo = r[2 * s0], hi = r[2 * s0 + 1];
  for (int sp = s0 + 1; sp < s1; ++sp) {
    lo = min(lo, r[2 * sp]);
    hi = max(hi, r[2 * sp + 1]);
  }
  Stage sg;
  sg.lo = lo;
  sg.span = hi - lo;
  sg.on = sg.span > 0 && sg.span <= kStageCap;
  return sg;
}

// Staging of entries [i0, i0 + blockDim.x * kStagePerThread): requested into
// registers (every lane loads; lanes past the range repeat its last entry) ...
struct StageIn {
  double y[kStagePerThread];
  int x[kStagePerThread];
};
__device__ __forceinline__ void stage_issue(const Ctx &c, const Stage &sg, int i0, StageIn &si) {
#pragma unroll
  for (int k = 0; k < kStagePerThread; ++k) {
    const int i = min(i0 + k * (int)blockDim.x + (int)threadIdx.x, sg.span - 1);
    vrec_load(c, (unsigned)(sg.lo + i), si.x[k], si.y[k]);
  }
}
// ... and written to LDS once they arrive.
__device__ __forceinline__ void stage_commit(const Stage &sg, int i0, const StageIn &si, double *sy, uint8_t *sx) {
#pragma unroll
  for (int k = 0; k < kStagePerThread; ++k) {
    const int i = i0 + k * (int)blockDim.x + (int)threadIdx.x;
    if (i < sg.span) {
      sy[i] = si.y[k];
      sx[i] = (uint8_t)si.x[k];
    }
  }
}
// The whole range, first part already requested in si (the caller synchronises).
__device__ __forceinline__ void stage_rest(const Ctx &c, const Stage &sg, StageIn &si, double *sy, uint8_t *sx) {
  const int step = (int)blockDim.x * kStagePerThread;
  stage_commit(sg, 0, si, sy, sx);
  for (int i0 = step; i0 < sg.span; i0 += step) {
    stage_issue(c, sg, i0, si);
    stage_commit(sg, i0, si, sy, sx);
  }
}

// A chunk's loads on the slot layout, requested by chunk_issue and consumed by
// chunk_run.
struct ChunkIn {
  int v[kChunkTiles];
  uint32_t am[kChunkTiles];
  uint32_t hw;  // header: dword k in lane k
  int xv[kChunkTiles];
  double yv[kChunkTiles];
  uint32_t ah[kChunkTiles];
};

constexpr int kHdrDw = sizeof(ChunkHdr) / 4;
constexpr int kDwElem = offsetof(ChunkHdr, elem_start) / 4, kDwHood = offsetof(ChunkHdr, hood_start) / 4,
              kDwHend = offsetof(ChunkHdr, hood_end) / 4, kDwFlags = offsetof(ChunkHdr, flags) / 4,
              kDwOff = offsetof(ChunkHdr, elem_off) / 4;
__device__ __forceinline__ uint32_t hdr_field(uint32_t hw, int k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)hw, k);
}

// Chunk on the slot layout, first half: the chunk's member ids and adjacency
// words are requested from the chunk index alone, together with its header;
// then the label and intensity gathers.  Nothing here writes, and nothing
// waits for more than the slot words each gather needs.
template <int LMAX>
__device__ __forceinline__ void chunk_stream(const Ctx &c, int ck, ChunkIn &in, int lane) {
  const int tb = ck * kChunkTiles;
  // The slot arrays are padded to whole chunks, so every packet slot of the
  // chunk can be read; chunk bases are uniform, each load is base + lane * 4 +
  // an immediate.
  const gptr<const int32_t> svb = c.svid + (size_t)tb * kWave;
  const gptr<const uint32_t> smb = c.smask + (size_t)tb * kWave;
  const unsigned ul = (unsigned)lane;
#pragma unroll
  for (int i = 0; i < kChunkTiles; ++i) {
    in.v[i] = svb[i * kWave + ul];
    in.am[i] = smb[i * kWave + ul];
  }
  // the header: dword k in lane k (one load), fields read out with readlane
  // once it has arrived
  in.hw = lane < kHdrDw ? gptr<const uint32_t>(c.chdr + ck)[lane] : 0u;
}

// The label and intensity gathers of a chunk whose slot words chunk_stream
// requested (each waits only for its own packet's slot words).
template <int LMAX>
__device__ __forceinline__ void chunk_gather(const Ctx &c, int ck, ChunkIn &in, int lane, const Stage &sg,
                                             const double *sy, const uint8_t *sx) {
  const int tb = ck * kChunkTiles;
  const unsigned ul = (unsigned)lane;
  const int flags = kPrefetchHi<LMAX> ? (int)hdr_field(in.hw, kDwFlags) : 0;
#pragma unroll
  for (int i = 0; i < kChunkTiles; ++i) {
    // an empty slot reads vertex 0 (staged: the range's first entry); nothing
    // of an empty slot is used
    const bool valid = (uint32_t)in.v[i] != kSlotEmpty;
    if (sg.on) {
      const int li = valid ? (int)((uint32_t)in.v[i] & kSlotVidMask) - sg.lo : 0;
      in.xv[i] = sx[li];
      in.yv[i] = sy[li];
    } else {
      const unsigned vv = valid ? (uint32_t)in.v[i] & kSlotVidMask : 0u;
      vrec_load(c, vv, in.xv[i], in.yv[i]);
    }
    in.ah[i] = 0;
    if (kPrefetchHi<LMAX> && ((flags >> (kHdrMidShift + i)) & 1))
      in.ah[i] = (c.smask_hi + (size_t)tb * kWave)[i * kWave + ul];
  }
}

// Offsets and window values of the chunk's first 64 neighbourhoods [h0, hend),
// lane h - h0 (requested before the element passes, used after them).
__device__ __forceinline__ HoodPre load_pre(const Ctx &c, int h0, int hend, int lane) {
  HoodPre pre{0, 0, {}};
  const int h = h0 + lane;
  if (h < hend) {
    pre.p0 = c.hood_ptr[h];
    pre.p1 = c.hood_ptr[h + 1];
    if (c.t >= c.W) {
      const int slots = c.W + 1;
#pragma unroll
      for (int w = 1; w <= kPreWindow; ++w)
        if (w <= c.W) pre.prev[w - 1] = c.ring[(size_t)((c.t - w) % slots) * c.H + h];
    }
  }
  return pre;
}


// Second half: the offsets and window values of the chunk's first 64
// neighbourhoods are requested, then the element passes, the owner list, the
// neighbourhood pass and the chunk's record row.
template <int LMAX>
__device__ __forceinline__ void chunk_run(const Ctx &c, int ck, const ChunkIn &in, const Theta<LMAX> &th, double *row,
                                          double *mb, double *od, int *oa, int lane) {
  const int tb = ck * kChunkTiles;
  const int nt = min(kChunkTiles, c.ntiles - tb);
  const int flags = (int)hdr_field(in.hw, kDwFlags);
  const int gstart = (int)hdr_field(in.hw, kDwElem), h0 = (int)hdr_field(in.hw, kDwHood),
            hend = (int)hdr_field(in.hw, kDwHend);
  const HoodPre pre = load_pre(c, h0, hend, lane);
  ChunkStats<LMAX> cs;
  cs.clear();
  int ocount = 0;
#pragma unroll
  for (int i = 0; i < kChunkTiles; ++i)
    if (i < nt) {
      if (ocount > kOwnCap - 64) {
        wave_lds_sync();
        cs.take_owners(od, oa, ocount, lane);
        ocount = 0;
        wave_lds_sync();
      }
      const int eoff = (int)((hdr_field(in.hw, kDwOff + i / 2) >> (16 * (i & 1))) & 0xffffu);
      slot_elem<LMAX>(c, gstart + eoff, eoff, (flags >> (kHdrMidShift + i)) & 1, tb + i, (uint32_t)in.v[i], in.am[i],
                      in.ah[i], in.xv[i], in.yv[i], th, cs, mb, od, oa, ocount, lane);
    }
  wave_lds_sync();
  cs.take_owners(od, oa, ocount, lane);
  lean_hoods<LMAX>(c, h0, hend, gstart, pre, cs, mb, lane);
  wave_lds_sync();
  cs.store(row, mb, c.L, lane);  // the minima are no longer needed
}

// One statistics chunk: packets [ck * kChunkTiles, min(ntiles, (ck + 1) * kChunkTiles)).
//
// Chunks without a LARGE packet (window <= 4) take the slot layout, where the
// wave waits for memory twice per chunk (chunk_slots).  The others go packet by
// packet over the element arrays.  Which path a chunk takes depends only on the
// graph and the window length, never on the launch shape, so results stay
// independent of it (the two paths add the owner statistics in different lane
// orders).
template <int LMAX>
__device__ void chunk_packets(const Ctx &c, int ck, const Theta<LMAX> &th, double *part, double *mb, uint64_t *pl,
                              int lane) {
  LaneStats<LMAX> ls;
  ls.clear();
  const int tb = ck * kChunkTiles, te = min(c.ntiles, tb + kChunkTiles);
  const int nt = te - tb;
  // lane i < nt holds packet i's descriptor; lane nt the next chunk's first
  TileDesc mine{};
  if (lane <= nt && tb + lane < c.ntiles) mine = load_tile(c.tiles + tb + lane);
  const bool any_large = __ballot(lane < nt && mine.kind == kLarge) != 0;
  const int hend = te < c.ntiles ? bcast(mine.hood_start, nt) : c.H;
  (void)any_large;
  {
    int g0 = tb;  // first packet of the pending neighbourhood group
    int gstart = 0, ghood = 0;
    for (int i = 0; i < nt; ++i) {
      const int ti = tb + i;
      const TileDesc t = load_tile(c.tiles + ti);
      if (t.kind == kLarge) {
        if (ti > g0) hood_pass<LMAX>(c, ghood, t.hood_start, gstart, ls, mb, lane);
        do_large<LMAX>(c, t, th, ls, mb, pl, lane);
        g0 = ti + 1;
      } else {
        if (ti == g0) {
          gstart = t.elem_start;
          ghood = t.hood_start;
        }
        const Stream sd = load_stream(c, t, lane);
        elem_pass<LMAX>(c, t, sd, load_gather(c, t, sd, lane), gstart, th, ls, mb, lane);
      }
    }
    if (te > g0) hood_pass<LMAX>(c, ghood, hend, gstart, ls, mb, lane);
  }
  ls.store(part, 1, c.L, lane);
}

// ------------------------------------------------------------------ kernels
__global__ void k_write_desc(DescPack pack, GraphDev *dst) {
  int i = threadIdx.x;
  if (i < pack.count) dst[pack.first + i] = pack.d[i];
}

// The run state of one graph from the caller's starting parameters.
__device__ void setup_graph(const GraphDev &G) {
  GraphState *st = G.st;
  st->done = 0;
  st->stop[0] = 0;
  st->stop[1] = 0;
  st->status = 0;
  st->iters = 0;
  st->map_conv = -1;
  st->em_conv = -1;
  st->ties_total = 0;
  bool ok = true;
  for (int l = 0; l < G.L; ++l) {
    double mu = G.in_mu[l], sigma = G.in_sigma[l];
    if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(mu)) ok = false;
    st->th[0][l].mu = mu;
    st->th[0][l].sigma = sigma;
  }
  if (!ok) {
    st->status = PMRF_EBADPARAM;
    st->done = 1;
    st->stop[0] = 1;
    return;
  }
  for (int l = 0; l < G.L; ++l) set_label_theta(st->th[0], l, st->th[0][l].mu, st->th[0][l].sigma);
}

// The workspace vertex records from the caller's intensities and starting
// labels (label buffer 0): block b of the graph's nb vertex blocks.
__device__ void vr_init_part(const GraphDev &G, int b, int nb) {
  const int stride = nb * blockDim.x;
  for (int v = b * blockDim.x + threadIdx.x; v < G.n; v += stride) {
    VertexRec r;
    r.y = G.y[v];
    r.x[0] = G.x0[v];
    r.x[1] = 0;
    G.vr[v] = r;
  }
}

// Set up the state of every graph from the caller's starting parameters.
__global__ void k_setup(const GraphDev *graphs, int B) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= B) return;
  setup_graph(graphs[g]);
}

// The vertex records of every graph, once per run.
__global__ void k_vr_init(const GraphDev *graphs, int B) {
  const GraphDev &G = graphs[find_graph(graphs, B, blockIdx.x, kGridVertex)];
  vr_init_part(G, blockIdx.x - G.vblock0, G.vnblocks);
}

// A single graph's start in one launch: its descriptor (a kernel argument)
// to device memory for the later kernels, its run state, its vertex records.
__global__ void k_start1(const GraphDev g1, GraphDev *dst) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *dst = g1;
    setup_graph(g1);
  }
  vr_init_part(g1, blockIdx.x, gridDim.x);
}

// Graph of every slot-kernel block, written once per run (batches only):
// blocks [block0, block0 + nblocks) of graph g map to g, so a block finds its
// descriptor with one load instead of a search over the graphs.
__global__ void k_block_graph(const GraphDev *graphs, int32_t *table) {
  const GraphDev &G = graphs[blockIdx.x];
  for (int i = threadIdx.x; i < G.nblocks; i += blockDim.x) table[G.block0 + i] = (int32_t)blockIdx.x;
}

// Parameter update from the starting labels (used when init_from_labels is
// set): pass 0 sums y per label (mean), pass 1 sums (y - mean) and (y - mean)^2.
// Block b covers vertices [b*1024, b*1024 + 1024), thread t the vertices
// t, t+256, ... of that range; one record per block.
__global__ __launch_bounds__(256) void k_mstep_init(const GraphDev *graphs, int B, int pass) {
  __shared__ double part[4][kRecMax];
  const int g = find_graph(graphs, B, blockIdx.x, kGridVertex);
  const GraphDev &G = graphs[g];
  gptr<const GraphState> st = gbl((const GraphState *)G.st);
  if (!G.init_from_labels || st->done) return;
  const int L = G.L, words = rec_words(L);
  const int b = blockIdx.x - G.vblock0;
  const int v0 = b * kVertPerBlock, v1 = min(G.n, v0 + kVertPerBlock);
  gptr<const int32_t> x = gbl((const int32_t *)G.x0);
  gptr<const double> y = gbl(G.y);
  LaneStats<kMaxLabels> ls;
  ls.clear();
  double c[kMaxLabels];
  for (int l = 0; l < kMaxLabels; ++l) c[l] = (pass == 0 || l >= L) ? 0.0 : st->th[0][l].mu;
  for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    int xv = x[v];
    if ((unsigned)xv >= (unsigned)L) {
      ls.err |= 1;
      continue;
    }
    double cv = 0.0;
    for (int l = 0; l < L; ++l)
      if (l == xv) cv = c[l];
    ls.add_owner(xv, y[v] - cv);
  }
  const int wave = wave_id(), lane = threadIdx.x & 63;
  ls.store(&part[wave][0], 1, L, lane);
  __syncthreads();
  if (threadIdx.x >= 64) return;
  // the four waves in order
  if (lane < words) {
    const int w = lane;
    double acc = 0.0;
    for (int k = 0; k < 4; ++k) acc = acc + part[k][w];
    gbl(G.rec)[(size_t)w * G.vnblocks + b] = acc;
  }
}

// Scatter rule MIN, after iteration t's element kernels: vertex v takes the
// label of its element with the smallest minimum energy, the first in
// canonical neighbourhood order on ties (elements listed in that order); a
// near tie is a gap below tie_eps at that element or another element of v
// within tie_eps of the minimum at a different label.  The new label goes to
// label buffer (t + 1) & 1, and the vertex's share of the parameter update
// (y - mu_a of iteration t) and its near tie to the record of its vertex
// block (records nsuper + block; thread i takes vertices i, i + 256, ... in
// order, the four waves add in order).
template <int LMAX>
__global__ __launch_bounds__(256) void k_decide(const GraphDev *graphs, int B, int t) {
  __shared__ double part[4][kRecMax];
  const GraphDev &G = graphs[find_graph(graphs, B, blockIdx.x, kGridVertex)];
  if (G.rule != kRuleMin) return;
  gptr<const GraphState> st = gbl((const GraphState *)G.st);
  if (t >= G.max_iters || st->done) return;
  const int L = G.L, words = rec_words(L);
  const int b = blockIdx.x - G.vblock0;
  const int v0 = b * kVertPerBlock, v1 = min(G.n, v0 + kVertPerBlock);
  gptr<const int32_t> optr = gbl(G.occ_ptr), occ = gbl(G.occ), ea = gbl((const int32_t *)G.ea);
  gptr<const double> em = gbl((const double *)G.em), eg = gbl((const double *)G.eg);
  gptr<VertexRec> vr = gbl(G.vr);
  double mu[LMAX];
#pragma unroll
  for (int l = 0; l < LMAX; ++l) mu[l] = l < L ? st->th[t & 1][l].mu : 0.0;
  LaneStats<LMAX> ls;
  ls.clear();
  for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    const int o0 = optr[v], o1 = optr[v + 1];
    int best = occ[o0];
    double mbest = em[best];
    for (int o = o0 + 1; o < o1; ++o) {
      const int e = occ[o];
      const double m = em[e];
      if (m < mbest) {
        mbest = m;
        best = e;
      }
    }
    const int a = ea[best];
    bool tie = eg[best] < G.tie_eps;
    for (int o = o0; o < o1; ++o) {
      const int e = occ[o];
      if (e != best && em[e] - mbest < G.tie_eps && ea[e] != a) tie = true;
    }
    vr[v].x[(t + 1) & 1] = a;
    double cm = 0.0;
#pragma unroll
    for (int l = 0; l < LMAX; ++l)
      if (l == a) cm = mu[l];
    ls.add_owner(a, vr[v].y - cm);
    if (tie) ls.ties += 1;
  }
  const int wave = wave_id(), lane = threadIdx.x & 63;
  ls.store(&part[wave][0], 1, L, lane);
  __syncthreads();
  if (threadIdx.x < words) {
    const int w = threadIdx.x;
    double acc = 0.0;
    for (int k = 0; k < 4; ++k) acc = acc + part[k][w];
    gbl(G.rec)[(size_t)(t & 1) * G.rec_stride + (size_t)w * G.nrec + G.nsuper + b] = acc;
  }
}

// LDS of the parameter update.
struct FoldLds {
  double tot[kRecMax];
  double scr[kFoldGroup * kFoldLanes];
};

__global__ __launch_bounds__(kFoldThreads) void k_fin_init(const GraphDev *graphs, int B, int pass) {
  __shared__ FoldLds sh;
  const GraphDev &G = graphs[blockIdx.x];
  GraphState *st = G.st;
  if (!G.init_from_labels || st->done) return;
  fold_all(gbl((const double *)G.rec), G.vnblocks, rec_words(G.L), sh.scr, sh.tot, blockDim.x >> 6, wave_id(),
           threadIdx.x & 63);
  if (threadIdx.x != 0) return;
  if (sh.tot[3 * G.L + 3] != 0.0) {
    st->status = PMRF_EBADLABEL;
    st->done = 1;
    st->stop[0] = 1;
    return;
  }
  update_theta(st->th[0], sh.tot, G.L, G.sigma_min, pass == 0);
}

// What the parameter update of iteration tp = t - 1 reads of the run state
// besides the records, requested before the fold: whether the run had stopped
// before tp, the running counters, and in lane l label l's parameters of tp
// and the energy total of iteration tp - l - 1 (thist holds max(1, max_iters)
// entries; used where tp >= l + 1).
struct FoldPrev {
  int done;
  int map_conv, em_conv;
  long long ties_total;
  double mu, sg, wl, lg;
  double hist;
};

__device__ __forceinline__ FoldPrev fold_prev(const GraphDev &G, int t, int done, int lane) {
  gptr<const GraphState> st = gbl((const GraphState *)G.st);
  gptr<const double> thist = gbl((const double *)G.thist);
  const int tp = t - 1;
  FoldPrev p;
  p.done = done;
  p.ties_total = st->ties_total;
  p.map_conv = st->map_conv;
  p.em_conv = st->em_conv;
  const int ll = lane < kMaxLabels ? lane : 0;
  p.mu = st->th[tp & 1][ll].mu;
  p.sg = st->th[tp & 1][ll].sigma;
  p.wl = st->th[tp & 1][ll].w;
  p.lg = st->th[tp & 1][ll].lg;
  p.hist = thist[min(max(0, tp - lane - 1), max(0, G.max_iters - 1))];
  return p;
}

// Parameter update ("Update Parameters") and convergence check of iteration
// tp = t - 1, by one wave, from the record totals tot[]: lane l < L gets label
// l's parameters of iteration t in (p.mu, p.sg, p.wl, p.lg); with `write`, the
// parameters and the results of tp (energy total, near ties, convergence,
// iteration count, early exit, errors) go to the run state (one block per
// graph writes).  Returns whether the run stops before iteration t: it had
// stopped before tp, a starting label was out of range, or every neighbourhood
// converged with early exit on.
__device__ __forceinline__ bool finish_iteration(const GraphDev &G, int t, const double *tot, FoldPrev &p, bool write,
                                                 int lane) {
  const int L = G.L, W = G.W, tp = t - 1;
  gptr<GraphState> st = gbl(G.st);
  if (p.done) return true;
  if (tot[3 * L + 3] != 0.0) {
    if (write && lane == 0) {
      st->status = PMRF_EBADLABEL;
      st->done = 1;
    }
    return true;
  }
  const double T = tot[3 * L];
  const long long ties = (long long)tot[3 * L + 1];
  const long long nonconv = (long long)tot[3 * L + 2];
  // the energy total has converged if it moved less than tol against each of
  // the previous W totals
  const bool em_ok = __ballot(lane < W && !(fabs(T - p.hist) < G.tol)) == 0;
  if (lane < L) {
    next_label_theta(tot[3 * lane], tot[3 * lane + 1], tot[3 * lane + 2], G.sigma_min, false, p.mu, p.sg, p.wl, p.lg);
    if (write) {
      st->th[t & 1][lane].mu = p.mu;
      st->th[t & 1][lane].sigma = p.sg;
      st->th[t & 1][lane].w = p.wl;
      st->th[t & 1][lane].lg = p.lg;
    }
  }
  const bool stop = G.early_exit && nonconv == 0 && tp >= W;
  if (write && lane == 0) {
    gbl(G.thist)[tp] = T;
    if (G.out_trace) gbl(G.out_trace)[tp] = T;
    if (G.out_stats) {
      gbl(G.out_stats)[2 * tp] = ties;
      gbl(G.out_stats)[2 * tp + 1] = nonconv;
    }
    st->ties_total = p.ties_total + ties;
    if (nonconv == 0 && tp >= W && p.map_conv < 0) st->map_conv = tp;
    if (tp >= W && p.em_conv < 0 && em_ok) st->em_conv = tp;
    st->iters = t;
    if (stop) st->done = 1;
  }
  return stop;
}

// The parameter update of iteration t - 1 of one graph, by one block: fold the
// records of t - 1 and finish the iteration in wave 0.  Every value the update
// reads is requested before the fold.
__device__ __forceinline__ void fold_iteration(const GraphDev &G, int t, FoldLds &sh, int nw, int wave, int lane) {
  const int tp = t - 1;
  FoldPrev p = fold_prev(G, t, gbl((const GraphState *)G.st)->done, lane);
  // a graph whose run has ended (tp >= max_iters, in a batch of mixed run
  // lengths) folds but stores nothing; testing it after the fold lets every
  // load above be requested at once
  fold_all(gbl((const double *)G.rec) + (size_t)(tp & 1) * G.rec_stride, G.nrec, rec_words(G.L), sh.scr, sh.tot,
           nw, wave, lane);
  if (tp >= G.max_iters || wave != 0) return;
  (void)finish_iteration(G, t, sh.tot, p, true, lane);
}

// The parameter update of iteration t - 1 (one block per graph; SINGLE: the
// one graph's descriptor g1 travels in the kernel arguments).
template <bool SINGLE>
__global__ __launch_bounds__(kFoldThreads) void k_fold(const GraphDev *graphs, const GraphDev g1, int B, int t) {
  __shared__ FoldLds sh;
  if constexpr (SINGLE)
    fold_iteration(g1, t, sh, blockDim.x >> 6, wave_id(), threadIdx.x & 63);
  else
    fold_iteration(graphs[blockIdx.x], t, sh, blockDim.x >> 6, wave_id(), threadIdx.x & 63);
}

// Registers of one iteration launch for a graph.
// ANY: the graph's scatter rule is read from its descriptor; otherwise the
// launch is compiled for the owner rule (every rule test folds away).
template <bool ANY = false>
__device__ __forceinline__ Ctx make_ctx(const GraphDev &G, int t) {
  Ctx c;
  c.tiles = gbl(G.tiles);
  c.vid = gbl(G.vid);
  c.mask = gbl(G.mask);
  c.chdr = gbl(G.chdr);
  c.svid = gbl(G.svid);
  c.smask = gbl(G.smask);
  c.smask_hi = gbl(G.smask_hi);
  c.st = gbl((const GraphState *)G.st);
  c.hood_ptr = gbl(G.hood_ptr);
  c.vr = gbl((const VertexRec *)G.vr);
  c.par = t & 1;
  c.xw = gbl(reinterpret_cast<int32_t *>(G.vr)) + 2 + ((t + 1) & 1);
  c.ring = gbl(G.ring);
  c.H = G.H;
  c.W = G.W;
  c.L = G.L;
  c.P = G.P;
  c.t = t;
  c.ntiles = G.ntiles;
  c.nchunks = G.nchunks;
  c.beta = G.beta;
  c.tol = G.tol;
  c.tie_eps = G.tie_eps;
  c.rule = ANY ? G.rule : kRuleOwner;
  c.lastbits = gbl(G.lastbits);
  c.em = gbl(G.em);
  c.eg = gbl(G.eg);
  c.ea = gbl(G.ea);
  return c;
}

// The block's records: superchunk s of chunks [c0, c1) (c0 a superchunk
// boundary) gets its chunk rows added in chunk order; an empty graph's one
// block writes record 0 (zeros).  The caller has synchronised the block.
template <int LMAX>
__device__ __forceinline__ void store_records(const GraphDev &G, int c0, int c1, int t,
                                              double (*part)[rec_words(LMAX)]) {
  const int words = rec_words(G.L), sc = G.sc;
  const int s0 = c0 / sc, ns = max(1, (c1 - c0 + sc - 1) / sc);
  gptr<double> rec = gbl(G.rec) + (size_t)(t & 1) * G.rec_stride;
  for (int i = threadIdx.x; i < ns * words; i += blockDim.x) {
    const int r = i / words, w = i - r * words;
    const int k1 = min((r + 1) * sc, c1 - c0);
    double out = 0.0;
    for (int k = r * sc; k < k1; ++k) out = out + part[k][w];
    rec[(size_t)w * G.nrec + s0 + r] = out;
  }
}

// One EM iteration over every graph of the launch.  A block takes chunks
// [c0, c1) of a graph (whole superchunks: one on the packet path and for a
// single graph, up to 16 chunks' worth in a batch); its waves take the chunks
// in turn, leave each chunk's statistics in LDS, and the block adds them in
// chunk order into one record per superchunk (buffer t & 1).  PACKET: the
// superchunk holds a LARGE packet (or the window is longer than kPreWindow)
// and goes packet by packet over the element arrays; otherwise every chunk
// takes the slot layout.
template <int LMAX, bool PACKET, bool SINGLE = false, bool ANY = false>
__device__ __forceinline__ void iter_superchunk(const GraphDev &G, int c0, int c1, int t,
                                                double (*part)[rec_words(LMAX)], double *mb, uint64_t *pl, double *od,
                                                int *oa, int nw, int wave, int lane) {
  // A graph whose run has ended (a batch mixes run lengths) computes and
  // writes nothing; the test joins the run state's done flag instead of
  // returning first, so the chunk's loads need not wait for it (they only read).
  const bool ended = t >= G.max_iters;
  const Ctx c = make_ctx<ANY>(G, t);
  Theta<LMAX> th;
  const int done_flag = load_theta<LMAX>(c, th);  // scalar loads, waited for with the chunk's
  if constexpr (!PACKET) {
    // single graph: the slot path's descriptor fields (kernel arguments)
    // arrive in one batch of scalar loads, before the first branch
    // (otherwise each branch waits for the fields it tests before the next
    // ones are even requested).  (A batch looks its descriptor up in memory;
    // pinning it there costs registers.)
    if constexpr (SINGLE)
      asm volatile("" ::"s"(c.chdr), "s"(c.svid), "s"(c.smask), "s"(c.st), "s"(c.hood_ptr), "s"(c.vr), "s"(c.xw),
                   "s"(c.ring), "s"(c.H), "s"(c.W), "s"(c.L), "s"(c.ntiles), "s"(c.nchunks), "s"(nw));
    // (no staging here: a barrier at the start of every block and the
    // staged range's LDS cost more than the gathers they save where blocks
    // run in many rounds; the fused single-graph launch stages)
    const Stage sg{0, 0, false};
    // nothing is written once the run has ended or is done (the run state's
    // done flag is read with the parameters, before the chunk's loads wait)
    const bool skip = ended || done_flag != 0;
    for (int ck = c0 + wave; ck < c1; ck += nw) {
      ChunkIn in;
      chunk_stream<LMAX>(c, ck, in, lane);
      chunk_gather<LMAX>(c, ck, in, lane, sg, nullptr, nullptr);
      if (!skip) chunk_run<LMAX>(c, ck, in, th, part[ck - c0], mb, od, oa, lane);
    }
  } else {
    if (!(done_flag != 0 || ended))
      for (int ck = c0 + wave; ck < c1; ck += nw) chunk_packets<LMAX>(c, ck, th, part[ck - c0], mb, pl, lane);
  }
  const bool done = done_flag != 0 || ended;
  __syncthreads();
  if (!done) store_records<LMAX>(G, c0, c1, t, part);
}

// Chunks of slot-kernel block b of a graph, and of packet-kernel block i.
__device__ __forceinline__ int slot_c0(const GraphDev &G, int b) { return b * G.bc; }
__device__ __forceinline__ int slot_c1(const GraphDev &G, int b) { return min(G.slot_end, (b + 1) * G.bc); }
__device__ __forceinline__ int packet_c0(const GraphDev &G, int i) { return (G.nslot + i) * G.sc; }
__device__ __forceinline__ int packet_c1(const GraphDev &G, int i) { return min(G.nchunks, (G.nslot + i + 1) * G.sc); }

// Element v of a row of nrec doubles, or 0.0 when v >= nrec: a raw buffer
// load, whose range check returns zero past the row's end (no memory is read
// there).  The resource's last dword is the gfx9 raw-buffer format.
__device__ __forceinline__ double row_load(const double *row, int nrec, int v) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(row), (short)0, nrec * 8, 0x00020000);
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v * 8, 0, 0));
}

// LDS of the fused launch: the record totals, the parameters of the iteration
// and the stop flag, handed from wave 0 to the block.
template <int LMAX>
struct FusedLds {
  double tot[kRecMax];
  double mu[LMAX], w[LMAX], lg[LMAX];
  int stop;
};

// Iteration t >= 1 of a single graph whose superchunks all take the slot
// kernel and number at most kFoldLanes (one record per virtual thread of the
// fold): the parameter update of iteration t - 1 happens here instead of in a
// launch of its own.  Every block folds the records of t - 1 in the fold
// kernel's order (so every block derives the same bits, and the same bits as
// k_fold) and computes the parameters of iteration t in wave 0; the block that
// plays superchunk 0 also stores them with the results of t - 1 in the run
// state, as k_fold would.  Records of t - 1 (virtual wave q by wave q), the run
// state and the first chunk's loads are all requested before the fold waits,
// so the fold overlaps the chunk's trip to memory.  The launch reads the stop
// flag of t - 1 and its superchunk-0 block writes that of t (the other slot).
// The block has at least kFoldLanes / 64 waves (wave q plays virtual wave q)
// and the graph at least one chunk.
// scr: at least rec_words(L) * kFoldLanes doubles of LDS (the waves' minima
// buffers, unused until the fold is over).
template <int LMAX>
__device__ __forceinline__ void iter_superchunk_fused(const GraphDev &G, int b, int t,
                                                      double (*part)[rec_words(LMAX)], double *sy, uint8_t *sx,
                                                      double *scr, double *mb, double *od, int *oa,
                                                      FusedLds<LMAX> &fl, int nw, int wave, int lane) {
  // one superchunk per block (bc == sc, every superchunk on the slot kernel)
  constexpr int WORDS = rec_words(LMAX);
  static_assert(WORDS <= kFoldGroup, "the fused fold takes one pass of words");
  const int tp = t - 1, R = G.nrec, words = rec_words(G.L);
  gptr<GraphState> st = gbl(G.st);
  const bool writer = b == 0;
  // this wave's virtual fold thread: at most one record
  // (range-checked loads: a lane past the records, a word past the label
  // count and every lane of a wave that plays no virtual wave read 0.0, with
  // no branch or select the compiler could turn into a wait)
  double rv[WORDS];
  {
    const double *rec = G.rec + (size_t)(tp & 1) * G.rec_stride;
    const int nrec = wave < kFoldLanes / 64 ? R : 0;
    const int v = wave * 64 + lane;
#pragma unroll
    for (int j = 0; j < WORDS; ++j) rv[j] = row_load(rec + (size_t)j * R, j < words ? nrec : 0, v);
  }
  FoldPrev pv = fold_prev(G, t, st->stop[tp & 1], lane);  // used by wave 0
  const Ctx c = make_ctx(G, t);
  const int c0 = slot_c0(G, b), c1 = slot_c1(G, b);
  const int ck0 = c0 + wave;
  const Stage sg = block_stage(G, c0, c1);
  // requested unconditionally (a wave without a chunk of its own requests the
  // superchunk's last one and drops it), so no branch joins the loads in
  // flight during the fold
  ChunkIn in;
  const int ckl = min(ck0, c1 - 1);
  chunk_stream<LMAX>(c, ckl, in, lane);
  StageIn si;
  if (sg.on) stage_issue(c, sg, 0, si);
  if (wave < kFoldLanes / 64) {
    const int v = wave * 64 + lane;
#pragma unroll
    for (int j = 0; j < WORDS; ++j) scr[fold_slot(j, v)] = rv[j];  // words >= L's are zero and never read
  }
  if (sg.on) stage_rest(c, sg, si, sy, sx);
  __syncthreads();
  // stage 2: one row of 64 virtual lanes per wave (16 * words <= 256 lanes),
  // then the update in wave 0
  fold_stage2(scr, words, fl.tot, nw, wave, lane);
  __syncthreads();
  if (wave == 0) {
    const bool stop = finish_iteration(G, t, fl.tot, pv, writer, lane);
    if (lane < LMAX) {
      const bool ok = lane < G.L;
      fl.mu[lane] = ok ? pv.mu : 0.0;
      fl.w[lane] = ok ? pv.wl : 0.0;
      fl.lg[lane] = ok ? pv.lg : 0.0;
    }
    if (lane == 0) {
      fl.stop = stop ? 1 : 0;
      if (writer) st->stop[t & 1] = stop ? 1 : 0;
    }
  }
  __syncthreads();
  // the parameters are uniform: scalar registers
  Theta<LMAX> th;
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    th.mu[l] = uniform_f64(fl.mu[l]);
    th.w[l] = uniform_f64(fl.w[l]);
    th.lg[l] = uniform_f64(fl.lg[l]);
  }
  const bool stop = __builtin_amdgcn_readfirstlane(fl.stop) != 0;
  chunk_gather<LMAX>(c, ckl, in, lane, sg, sy, sx);
  if (!stop && ck0 < c1) chunk_run<LMAX>(c, ck0, in, th, part[ck0 - c0], mb, od, oa, lane);
  for (int ck = ck0 + nw; ck < c1; ck += nw) {
    chunk_stream<LMAX>(c, ck, in, lane);
    chunk_gather<LMAX>(c, ck, in, lane, sg, sy, sx);
    if (!stop) chunk_run<LMAX>(c, ck, in, th, part[ck - c0], mb, od, oa, lane);
  }
  __syncthreads();
  if (!stop) store_records<LMAX>(G, c0, c1, t, part);
}

// PERSIST = false: block b works on superchunk b.  PERSIST = true: a grid sized
// to the machine whose blocks walk all superchunks.  SINGLE: one graph, whose
// descriptor g1 travels in the kernel arguments (its fields are then at hand
// without a dependent load); otherwise each block looks its graph up in
// graphs[0 .. B).  FUSED (single graph, t >= 1, not persistent): the launch
// also does the parameter update of iteration t - 1 (iter_superchunk_fused).
// Not persistent and not fused (and not the batched two-label kernel, whose
// registers are budgeted for five waves per SIMD), the launch also takes the
// superchunks that hold a LARGE packet: workgroups [0, npk) play packet blocks
// 0 .. npk - 1 (first, so the longest blocks start first), [npk, npk_pad)
// return at once, and the slot blocks follow; npk_pad is a multiple of the XCD
// count, so the slot blocks keep their XCD placement.
template <int LMAX, bool PERSIST, bool SINGLE, bool FUSED = false, bool ANY = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(LMAX <= 2 ? (SINGLE ? PMRF_ITER_WAVES_PER_EU : PMRF_BATCH_WAVES_PER_EU) : 1, 8))) void k_iter(
    const GraphDev *__restrict__ graphs, const int32_t *__restrict__ block_graph, const GraphDev g1, int B,
    int nsuper_total, int t, int npk, int npk_pad) {
  static_assert(!FUSED || (SINGLE && !PERSIST), "the fused launch is for one graph, one block per superchunk");
  // dynamic LDS: one region of kWaveLds doubles per wave, after (fused
  // launch) the staged range (kStageCap doubles, then kStageCap bytes)
  extern __shared__ double smem[];
  __shared__ double part[kMaxSuperChunks][rec_words(LMAX)];
  const int nw = blockDim.x >> 6, wave = wave_id(), lane = threadIdx.x & 63;
  double *sy = smem;
  uint8_t *sx = reinterpret_cast<uint8_t *>(smem + kStageCap);
  double *wbase = FUSED ? smem + kStageDoubles : smem;
  double *mb = wbase + wave * kWaveLds;
  uint64_t *pl = reinterpret_cast<uint64_t *>(mb + kGroupTiles * 64);
  double *od = mb + kGroupTiles * 64 + 64;
  int *oa = reinterpret_cast<int *>(od + kOwnCap);
  if constexpr (FUSED) {
    __shared__ FusedLds<LMAX> fl;
    iter_superchunk_fused<LMAX>(g1, xcd_block(blockIdx.x, gridDim.x), t, part, sy, sx, wbase, mb, od, oa, fl, nw,
                                wave, lane);
  } else if constexpr (!PERSIST) {
    if constexpr (SINGLE || LMAX > 2) {
      if ((int)blockIdx.x < npk_pad) {
        if ((int)blockIdx.x < npk) {
          const GraphDev &G = graphs[find_graph(graphs, B, blockIdx.x, kGridPacket)];
          const int i = blockIdx.x - G.pblock0;
          iter_superchunk<LMAX, true, false, ANY>(G, packet_c0(G, i), packet_c1(G, i), t, part, mb, pl, od, oa, nw,
                                                  wave, lane);
        }
        return;
      }
    }
    const int pad = SINGLE || LMAX > 2 ? npk_pad : 0;
    const int blk = xcd_block(blockIdx.x - pad, gridDim.x - pad);
    if constexpr (SINGLE) {
      iter_superchunk<LMAX, false, true, ANY>(g1, slot_c0(g1, blk), slot_c1(g1, blk), t, part, mb, pl, od, oa, nw,
                                         wave, lane);
    } else {
      const GraphDev &G = graphs[block_graph[blk]];
      const int b = blk - G.block0;
      iter_superchunk<LMAX, false, false, ANY>(G, slot_c0(G, b), slot_c1(G, b), t, part, mb, pl, od, oa, nw, wave,
                                               lane);
    }
  } else {
    for (int sc = blockIdx.x; sc < nsuper_total; sc += gridDim.x) {
      if constexpr (SINGLE) {
        iter_superchunk<LMAX, false, true>(g1, slot_c0(g1, sc), slot_c1(g1, sc), t, part, mb, pl, od, oa, nw,
                                           wave, lane);
      } else {
        const GraphDev &G = graphs[block_graph[sc]];
        const int b = sc - G.block0;
        iter_superchunk<LMAX, false>(G, slot_c0(G, b), slot_c1(G, b), t, part, mb, pl, od, oa, nw, wave, lane);
      }
      __syncthreads();  // part[] is reused by the next superchunk
    }
  }
}

// The superchunks that hold a LARGE packet: block i of a graph works on its
// superchunk nslot + i, packet by packet.
template <int LMAX, bool ANY = false>
__global__ __launch_bounds__(1024) void k_iter_packets(const GraphDev *__restrict__ graphs, int B, int t) {
  extern __shared__ double smem[];
  __shared__ double part[kMaxSuperChunks][rec_words(LMAX)];
  const int nw = blockDim.x >> 6, wave = wave_id(), lane = threadIdx.x & 63;
  double *mb = smem + wave * kWaveLds;
  uint64_t *pl = reinterpret_cast<uint64_t *>(mb + kGroupTiles * 64);
  double *od = mb + kGroupTiles * 64 + 64;
  int *oa = reinterpret_cast<int *>(od + kOwnCap);
  const GraphDev &G = graphs[find_graph(graphs, B, blockIdx.x, kGridPacket)];
  const int i = blockIdx.x - G.pblock0;
  iter_superchunk<LMAX, true, false, ANY>(G, packet_c0(G, i), packet_c1(G, i), t, part, mb, pl, od, oa, nw, wave,
                                          lane);
}


// Copy results to the caller's buffers.
__global__ void k_final(const GraphDev *graphs, int B) {
  const int g = find_graph(graphs, B, blockIdx.x, kGridVertex);
  const GraphDev &G = graphs[g];
  GraphState *st = G.st;
  const int b = blockIdx.x - G.vblock0;
  const int iters = st->iters;
  const int stride = G.vnblocks * blockDim.x;
  for (int v = b * blockDim.x + threadIdx.x; v < G.n; v += stride) G.x0[v] = G.vr[v].x[iters & 1];
  if (G.out_S && iters > 0) {
    const double *src = G.ring + (size_t)((iters - 1) % (G.W + 1)) * G.H;
    for (int h = b * blockDim.x + threadIdx.x; h < G.H; h += stride) G.out_S[G.perm[h]] = src[h];
  }
  if (b == 0 && threadIdx.x == 0) {
    for (int l = 0; l < G.L; ++l) {
      G.out_mu[l] = st->th[iters & 1][l].mu;
      G.out_sigma[l] = st->th[iters & 1][l].sigma;
    }
    int64_t *c = G.out_ctr;
    c[PMRF_CTR_STATUS] = st->status;
    c[PMRF_CTR_ITERS] = iters;
    c[PMRF_CTR_MAP_CONV] = st->map_conv;
    c[PMRF_CTR_EM_CONV] = st->em_conv;
    c[PMRF_CTR_NEAR_TIES] = st->ties_total;
    c[PMRF_CTR_EVALS] = G.M * (int64_t)G.L * (int64_t)iters;
    c[6] = 0;
    c[7] = 0;
  }
}

// A fused single-graph run of T >= 1 iterations ends in one launch: block 0
// folds the records of iteration T - 1 and then writes the parameters and
// counters; every block copies its share of the labels and neighbourhood
// sums.  Which label buffer is final follows from the stop flag the last
// iteration launch wrote (it cannot change in this launch): set, the run had
// stopped before iteration T - 1 and its iteration count is already in the
// state; clear, iteration T - 1 ran, so T iterations did.
__global__ __launch_bounds__(kFoldThreads) void k_finish1(const GraphDev g1, int T) {
  __shared__ FoldLds sh;
  const GraphDev &G = g1;
  GraphState *st = G.st;
  const int iters = st->stop[(T - 1) & 1] ? st->iters : T;
  const int stride = gridDim.x * blockDim.x;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < G.n; v += stride) G.x0[v] = G.vr[v].x[iters & 1];
  if (G.out_S && iters > 0) {
    const double *src = G.ring + (size_t)((iters - 1) % (G.W + 1)) * G.H;
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < G.H; h += stride) G.out_S[G.perm[h]] = src[h];
  }
  if (blockIdx.x != 0) return;
  fold_iteration(G, T, sh, blockDim.x >> 6, wave_id(), threadIdx.x & 63);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int l = 0; l < G.L; ++l) {
      G.out_mu[l] = st->th[iters & 1][l].mu;
      G.out_sigma[l] = st->th[iters & 1][l].sigma;
    }
    int64_t *c = G.out_ctr;
    c[PMRF_CTR_STATUS] = st->status;
    c[PMRF_CTR_ITERS] = iters;
    c[PMRF_CTR_MAP_CONV] = st->map_conv;
    c[PMRF_CTR_EM_CONV] = st->em_conv;
    c[PMRF_CTR_NEAR_TIES] = st->ties_total;
    c[PMRF_CTR_EVALS] = G.M * (int64_t)G.L * (int64_t)iters;
    c[6] = 0;
    c[7] = 0;
  }
}

// ------------------------------------------------------------------- host side
std::mutex g_launch_mu;
pmrf_launch g_launch{0, 0, 0, 0};

// While profiling is on, each EM iteration's work kernels are launched with a
// start/stop event pair that the runtime stamps with the kernels' own dispatch
// begin and end times (hipExtLaunchKernel), so no marker packet sits between
// the stamps and the kernel.
struct Profiler {
  bool on = false;
  size_t used = 0;
  std::vector<hipEvent_t> start, stop;
} g_prof;

// events for the next iteration (nullptr pair when profiling is off)
hipError_t prof_pair(hipEvent_t *a, hipEvent_t *b) {
  *a = *b = nullptr;
  if (!g_prof.on) return hipSuccess;
  if (g_prof.used == g_prof.start.size()) {
    hipEvent_t x, y;
    hipError_t e = hipEventCreate(&x);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&y);
    if (e != hipSuccess) return e;
    g_prof.start.push_back(x);
    g_prof.stop.push_back(y);
  }
  *a = g_prof.start[g_prof.used];
  *b = g_prof.stop[g_prof.used];
  ++g_prof.used;
  return hipSuccess;
}

constexpr int kModeGraph = 1, kModePersistent = 2, kModeDirect = 3;
constexpr int kFusedMaxLabels = 4;  // fused launches exist for LMAX = 2 and 4

struct LaunchShape {
  int mode, waves_per_block, tiles_per_wave, blocks_per_cu;
  bool automatic;  // mode 0: graph replay from an argument set's second run on
};

LaunchShape resolve_shape() {
  std::lock_guard<std::mutex> lk(g_launch_mu);
  LaunchShape s{g_launch.mode > 0 ? g_launch.mode : kModeGraph,
                g_launch.waves_per_block,  // 0: automatic (run_items)
                g_launch.tiles_per_wave > 0 ? g_launch.tiles_per_wave : 1,
                g_launch.blocks_per_cu > 0 ? g_launch.blocks_per_cu : 5, g_launch.mode == 0};
  return s;
}

// Instantiated HIP graphs of recent argument sets (most recent first).  In
// the automatic mode an argument set runs as direct launches the first time it
// is seen and is captured on its second run, so one-off sets (a serving step,
// whose trace offsets and starting flags change every call) never pay a
// capture; the keys seen once are remembered in a bounded list.
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec;
  hipEvent_t done;  // recorded after each replay: the entry is idle once it completes
};
constexpr size_t kGraphCacheSize = 128;
constexpr size_t kSeenKeys = 1024;
std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;
std::list<std::string> g_seen;  // keys run once as direct launches (most recent first)
std::map<int, hipStream_t> g_capture_streams;
int64_t g_captures = 0, g_replays = 0, g_direct = 0;

hipStream_t capture_stream(int dev) {
  auto it = g_capture_streams.find(dev);
  if (it != g_capture_streams.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  g_capture_streams[dev] = s;
  return s;
}

struct WsPlan {
  int64_t desc_off = 0;
  int64_t block_graph_off = 0, slot_blocks = 0;  // int32 graph of every slot-kernel block
  std::vector<int64_t> state_off, vr_off, ring_off, thist_off, rec_off, elem_off;
  int64_t total = 0;
};

pmrf_status check_params(const pmrf_em_params *p) {
  if (!p) return fail(PMRF_EINVAL, "params is NULL");
  if (p->L < 2) return fail(PMRF_EINVAL, "L must be >= 2");
  if (p->L > kMaxLabels) return fail(PMRF_EUNSUPPORTED, "L above 16 is not supported");
  if (!(p->beta >= 0.0) || !std::isfinite(p->beta)) return fail(PMRF_EINVAL, "beta must be finite and >= 0");
  if (p->max_iters < 0) return fail(PMRF_EINVAL, "max_iters must be >= 0");
  if (p->conv_window < 1 || p->conv_window > kMaxWindow) return fail(PMRF_EINVAL, "conv_window must be in 1..8");
  if (!(p->conv_tol >= 0.0)) return fail(PMRF_EINVAL, "conv_tol must be >= 0");
  if (!(p->sigma_min > 0.0) || !std::isfinite(p->sigma_min)) return fail(PMRF_EINVAL, "sigma_min must be > 0");
  if (!(p->tie_eps >= 0.0)) return fail(PMRF_EINVAL, "tie_eps must be >= 0");
  if (p->early_exit != 0 && p->early_exit != 1) return fail(PMRF_EINVAL, "early_exit must be 0 or 1");
  if (p->init_from_labels != 0 && p->init_from_labels != 1) return fail(PMRF_EINVAL, "init_from_labels must be 0 or 1");
  if (p->scatter_rule < PMRF_SCATTER_OWNER || p->scatter_rule > PMRF_SCATTER_MIN)
    return fail(PMRF_EINVAL, "scatter_rule must be 0 (owner), 1 (last) or 2 (min)");
  return PMRF_OK;
}

pmrf_status check_item(const pmrf_em_item &it, int idx) {
  std::string where = idx >= 0 ? " (item " + std::to_string(idx) + ")" : "";
  if (!it.hoods) return fail(PMRF_EINVAL, "hoods is NULL" + where);
  pmrf_status s = check_params(&it.params);
  if (s != PMRF_OK) return fail(s, std::string(pmrf_last_error()) + where);
  if (!it.d_hoodbuf || !it.d_y || !it.d_labels || !it.d_mu || !it.d_sigma || !it.d_counters)
    return fail(PMRF_EINVAL, "a required device pointer is NULL" + where);
  return PMRF_OK;
}

int64_t n_chunks(const pmrf_hoods *h) { return (h->ntiles + kChunkTiles - 1) / kChunkTiles; }
int64_t vert_blocks(const pmrf_hoods *h) { return std::max<int64_t>(1, ((int64_t)h->n + kVertPerBlock - 1) / kVertPerBlock); }
int32_t superchunk_chunks(const pmrf_hoods *h) { return superchunk_chunks_of(n_chunks(h)); }
int64_t n_super(const pmrf_hoods *h) {
  const int64_t sc = superchunk_chunks(h);
  return std::max<int64_t>(1, (n_chunks(h) + sc - 1) / sc);
}
// Statistics records per iteration: one per superchunk, and under rule MIN
// one more per vertex block (the vertex pass adds the parameter update's sums).
int64_t n_records(const pmrf_hoods *h, const pmrf_em_params &p) {
  return n_super(h) + (p.scatter_rule == PMRF_SCATTER_MIN ? vert_blocks(h) : 0);
}
int64_t max_records(const pmrf_hoods *h, const pmrf_em_params &p) {
  return std::max<int64_t>(n_records(h, p), vert_blocks(h));
}

// Superchunks of a graph that take the slot kernel: those before the first
// LARGE packet (all of them when there is none), none when the window is
// longer than kPreWindow; the rest take the packet path.
int32_t slot_supers(const pmrf_hoods *h, const pmrf_em_params &params) {
  const int64_t per_super = (int64_t)kChunkTiles * superchunk_chunks(h);
  int32_t nslot = h->slot_tiles == h->ntiles ? (int32_t)n_super(h) : (int32_t)(h->slot_tiles / per_super);
  if (params.conv_window > kPreWindow) nslot = 0;
  return nslot;
}

// How a graph's chunks are cut for one run: superchunks (records) of sc
// chunks, which depend on the graph alone; slot-kernel blocks of bc chunks (a
// single graph: one superchunk per block; a batch: 16 chunks per block, so
// every block of the launch costs about the same and the blocks dealt to each
// XCD carry equal work); packet-kernel blocks of one superchunk each.
struct GraphSplit {
  int32_t sc, bc, nsuper, nslot, slot_end, nblocks, pnblocks;
};

GraphSplit split_graph(const pmrf_hoods *h, const pmrf_em_params &params, int B) {
  GraphSplit g;
  g.sc = superchunk_chunks(h);
  g.bc = B == 1 ? g.sc : kMaxSuperChunks;
  g.nsuper = (int32_t)n_super(h);
  g.nslot = slot_supers(h, params);
  g.slot_end = (int32_t)std::min<int64_t>(n_chunks(h), (int64_t)g.nslot * g.sc);
  g.nblocks = g.nslot == 0 ? 0 : std::max(1, (g.slot_end + g.bc - 1) / g.bc);  // an empty graph keeps one block
  g.pnblocks = g.nsuper - g.nslot;
  return g;
}

WsPlan plan_workspace(int B, const pmrf_em_item *items) {
  WsPlan p;
  int64_t off = 0;
  p.desc_off = off;
  off += align_up((int64_t)B * (int64_t)sizeof(GraphDev), 256);
  for (int i = 0; i < B; ++i) p.slot_blocks += split_graph(items[i].hoods, items[i].params, B).nblocks;
  p.block_graph_off = off;
  off += align_up(std::max<int64_t>(1, p.slot_blocks) * 4, 256);
  for (int i = 0; i < B; ++i) {
    const pmrf_hoods *h = items[i].hoods;
    p.state_off.push_back(off);
    off += align_up(sizeof(GraphState), 256);
    p.vr_off.push_back(off);
    off += align_up((int64_t)h->n * (int64_t)sizeof(VertexRec), 256);
    p.ring_off.push_back(off);
    off += align_up((int64_t)(items[i].params.conv_window + 1) * h->H * 8, 256);
    p.thist_off.push_back(off);
    off += align_up((int64_t)std::max(1, items[i].params.max_iters) * 8, 256);
    p.rec_off.push_back(off);
    off += align_up(2 * max_records(h, items[i].params) * rec_words(items[i].params.L) * 8, 256);  // two record buffers
    p.elem_off.push_back(off);  // rule MIN: per element minimum, gap (doubles) and label (int32)
    if (items[i].params.scatter_rule == PMRF_SCATTER_MIN) off += align_up(std::max<int64_t>(1, h->M) * 20, 256);
  }
  p.total = std::max<int64_t>(off, 256);
  return p;
}

int lmax_for(int L) { return L <= 2 ? 2 : L <= 4 ? 4 : L <= 8 ? 8 : 16; }

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(PMRF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// no_alloc: enqueue the kernels directly, never capturing a HIP graph and
// never creating timing events (the allocation-free entry point).
pmrf_status run_items(int B, const pmrf_em_item *items, void *d_ws, int64_t ws_bytes, hipStream_t stream,
                      bool no_alloc = false) {
  WsPlan plan = plan_workspace(B, items);
  if (!d_ws) return fail(PMRF_EINVAL, "workspace is NULL");
  if (ws_bytes < plan.total) return fail(PMRF_ENOMEM, "workspace smaller than the required size");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(PMRF_EINVAL, "workspace must be 256-byte aligned");
  LaunchShape shape = resolve_shape();
  // automatic block size: one wave per chunk of a superchunk for a single
  // graph, four waves for a batch
  if (shape.waves_per_block <= 0) shape.waves_per_block = B == 1 ? superchunk_chunks(items[0].hoods) : 4;
  const int threads = shape.waves_per_block * kWave;
  char *ws = static_cast<char *>(d_ws);
  std::vector<GraphDev> desc(B);
  int blocks_iter = 0, blocks_pk = 0, blocks_vert = 0, max_iters = 0, Lmax = 2;
  for (int i = 0; i < B; ++i) {
    const pmrf_em_item &it = items[i];
    const pmrf_hoods *h = it.hoods;
    GraphDev &G = desc[i];
    const char *hb = static_cast<const char *>(it.d_hoodbuf);
    G.tiles = reinterpret_cast<const TileDesc *>(hb + h->layout.tiles_off);
    G.vid = reinterpret_cast<const int32_t *>(hb + h->layout.vid_off);
    G.mask = reinterpret_cast<const uint32_t *>(hb + h->layout.mask_off);
    G.chdr = reinterpret_cast<const ChunkHdr *>(hb + h->layout.chdr_off);
    G.svid = reinterpret_cast<const int32_t *>(hb + h->layout.svid_off);
    G.smask = reinterpret_cast<const uint32_t *>(hb + h->layout.smask_off);
    G.smask_hi = reinterpret_cast<const uint32_t *>(hb + h->layout.smaskhi_off);
    G.hood_ptr = reinterpret_cast<const int32_t *>(hb + h->layout.hptr_off);
    G.y = it.d_y;
    G.x0 = it.d_labels;
    G.vr = reinterpret_cast<VertexRec *>(ws + plan.vr_off[i]);
    G.ring = reinterpret_cast<double *>(ws + plan.ring_off[i]);
    G.thist = reinterpret_cast<double *>(ws + plan.thist_off[i]);
    G.st = reinterpret_cast<GraphState *>(ws + plan.state_off[i]);
    G.rec = reinterpret_cast<double *>(ws + plan.rec_off[i]);
    G.in_mu = it.d_mu;
    G.in_sigma = it.d_sigma;
    G.out_mu = it.d_mu;
    G.out_sigma = it.d_sigma;
    G.out_S = it.d_hood_energy;
    G.out_trace = it.d_trace;
    G.out_stats = it.d_iter_stats;
    G.out_ctr = it.d_counters;
    G.M = h->M;
    G.rec_stride = max_records(h, it.params) * rec_words(it.params.L);
    G.nrec = (int32_t)n_records(h, it.params);
    G.rule = it.params.scatter_rule;
    G.lastbits = reinterpret_cast<const uint64_t *>(hb + h->layout.lastbits_off);
    G.occ_ptr = reinterpret_cast<const int32_t *>(hb + h->layout.occptr_off);
    G.occ = reinterpret_cast<const int32_t *>(hb + h->layout.occ_off);
    if (G.rule == PMRF_SCATTER_MIN) {
      const int64_t Mp = std::max<int64_t>(1, h->M);
      G.em = reinterpret_cast<double *>(ws + plan.elem_off[i]);
      G.eg = G.em + Mp;
      G.ea = reinterpret_cast<int32_t *>(G.eg + Mp);
    } else {
      G.em = G.eg = nullptr;
      G.ea = nullptr;
    }
    G.n = h->n;
    G.H = (int32_t)h->H;
    G.ntiles = (int32_t)h->ntiles;
    G.L = it.params.L;
    G.P = it.params.L <= 2 ? 1 : it.params.L <= 4 ? 2 : it.params.L <= 8 ? 3 : 4;
    G.W = it.params.conv_window;
    G.max_iters = it.params.max_iters;
    G.early_exit = it.params.early_exit;
    G.init_from_labels = it.params.init_from_labels;
    G.beta = it.params.beta;
    G.tol = it.params.conv_tol;
    G.sigma_min = it.params.sigma_min;
    G.tie_eps = it.params.tie_eps;
    G.block0 = blocks_iter;
    G.nchunks = (int32_t)n_chunks(h);
    const GraphSplit sp = split_graph(h, it.params, B);
    G.nsuper = sp.nsuper;
    G.sc = sp.sc;
    G.bc = sp.bc;
    G.nslot = sp.nslot;
    G.slot_end = sp.slot_end;
    G.nblocks = sp.nblocks;
    blocks_iter += G.nblocks;
    G.pblock0 = blocks_pk;
    G.pnblocks = sp.pnblocks;
    blocks_pk += G.pnblocks;
    G.perm = reinterpret_cast<const int32_t *>(hb + h->layout.perm_off);
    G.srange = reinterpret_cast<const int32_t *>(hb + h->layout.srange_off);
    G.vblock0 = blocks_vert;
    G.vnblocks = (int32_t)vert_blocks(h);
    blocks_vert += G.vnblocks;
    max_iters = std::max(max_iters, G.max_iters);
    Lmax = std::max(Lmax, G.L);
  }
  GraphDev *d_desc = reinterpret_cast<GraphDev *>(ws + plan.desc_off);
  int32_t *block_graph = reinterpret_cast<int32_t *>(ws + plan.block_graph_off);
  if (blocks_iter != plan.slot_blocks) return fail(PMRF_EDEVICE, "internal: slot block count differs from the plan");
  bool any_init = false, any_min = false, any_rule = false;
  for (int i = 0; i < B; ++i) {
    any_init |= desc[i].init_from_labels != 0;
    any_min |= desc[i].rule == PMRF_SCATTER_MIN;
    any_rule |= desc[i].rule != PMRF_SCATTER_OWNER;
  }
  const int lm = lmax_for(Lmax);
  // One launch per EM iteration for a single graph whose superchunks all take
  // the slot kernel and whose records fit one fold pass per block (the blocks
  // of iteration t fold the records of t - 1 themselves); otherwise a fold
  // launch follows every iteration launch.  The fold order is the same either
  // way, so this changes speed only.
  // runs with a scatter rule other than the owner's use the launches compiled
  // for any rule: one block per superchunk group, a fold launch per iteration
  const bool persist = shape.mode == kModePersistent && !any_rule;
  const bool fused = B == 1 && blocks_pk == 0 && !persist && lm <= kFusedMaxLabels && !any_rule &&
                     desc[0].nsuper <= kFoldLanes && desc[0].nslot == desc[0].nsuper && desc[0].nchunks >= 1 &&
                     shape.waves_per_block >= kFoldLanes / 64;
  // a fused run ends with the last fold and the result copies in one launch
  const bool fused_finish = fused && max_iters >= 1;
  // dynamic LDS of the slot kernel: the staged range, then the waves' regions
  // (which hold the fused fold's partials before any chunk is computed); of
  // the packet path: the waves' regions
  const size_t lds_pk = (size_t)(kWaveLds * shape.waves_per_block) * 8;
  const size_t lds_fused = (size_t)kStageDoubles * 8 + std::max(lds_pk, (size_t)rec_words(lm) * kFoldLanes * 8);
  const bool events = g_prof.on && !no_alloc;
  // grid of the iteration kernel: one block per superchunk, or in persistent
  // mode a machine-sized grid whose blocks walk the superchunks
  int grid_iter = blocks_iter;
  if (persist) {
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    grid_iter = std::max(1, std::min(blocks_iter, cus * shape.blocks_per_cu));
  }
  // not persistent: the packet superchunks ride in the iteration launch
  // (their blocks first), so they run beside the slot blocks (the batched
  // two-label kernel excepted)
  const bool merge_pk = !persist && blocks_pk > 0 && blocks_iter > 0 && (B == 1 || lm > 2);
  const int npk = merge_pk ? blocks_pk : 0;
  const int npk_pad = merge_pk ? (blocks_pk + kXcds - 1) / kXcds * kXcds : 0;
  if (merge_pk) grid_iter = blocks_iter + npk_pad;

  // Everything the run enqueues; descriptors travel as kernel arguments, so no
  // host buffer must outlive the call and the sequence can be captured.
  auto enqueue = [&](hipStream_t s) -> pmrf_status {
    const GraphDev *gd = d_desc;
    if (B == 1) {
      hipLaunchKernelGGL(k_start1, dim3(blocks_vert), dim3(256), 0, s, desc[0], d_desc);
      HIP_TRY(hipGetLastError());
    } else {
      for (int first = 0; first < B; first += kDescPerPack) {
        DescPack pack{};
        pack.first = first;
        pack.count = std::min(kDescPerPack, B - first);
        for (int k = 0; k < pack.count; ++k) pack.d[k] = desc[first + k];
        hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, s, pack, d_desc);
        HIP_TRY(hipGetLastError());
      }
      hipLaunchKernelGGL(k_setup, dim3((B + 63) / 64), dim3(64), 0, s, gd, B);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(k_vr_init, dim3(blocks_vert), dim3(256), 0, s, gd, B);
      HIP_TRY(hipGetLastError());
    }
    if (B > 1 && blocks_iter > 0) {
      hipLaunchKernelGGL(k_block_graph, dim3(B), dim3(256), 0, s, gd, block_graph);
      HIP_TRY(hipGetLastError());
    }
    if (any_init) {
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_mstep_init, dim3(blocks_vert), dim3(256), 0, s, gd, B, pass);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_fin_init, dim3(B), dim3(kFoldThreads), 0, s, gd, B, pass);
        HIP_TRY(hipGetLastError());
      }
    }
    for (int t = 0; t < max_iters; ++t) {
      // the iteration's first kernel carries the start event, its last the stop event
      hipEvent_t ev0 = nullptr, ev1 = nullptr;
      if (events && (blocks_iter > 0 || blocks_pk > 0)) HIP_TRY(prof_pair(&ev0, &ev1));
      hipEvent_t slot_start = ev0, slot_stop = blocks_pk > 0 && !merge_pk ? nullptr : ev1;
      hipEvent_t pk_start = blocks_iter > 0 ? nullptr : ev0, pk_stop = ev1;
// plain launches unless the iteration is being timed (graph capture never is)
#define PMRF_LAUNCH(KERNEL, GRID, LDS, START, STOP, ...)                                                     \
  do {                                                                                                        \
    if ((START) || (STOP))                                                                                    \
      hipExtLaunchKernelGGL(KERNEL, GRID, dim3(threads), LDS, s, START, STOP, 0, __VA_ARGS__);                \
    else                                                                                                      \
      hipLaunchKernelGGL(KERNEL, GRID, dim3(threads), LDS, s, __VA_ARGS__);                                   \
  } while (0)
#define PMRF_LAUNCH_LDS(KERNEL, GRID, ...) PMRF_LAUNCH(KERNEL, GRID, lds_pk, __VA_ARGS__)
#define PMRF_LAUNCH_ITER(LM)                                                                                  \
  do {                                                                                                        \
    if (any_rule && B == 1)                                                                                   \
      PMRF_LAUNCH_LDS((k_iter<LM, false, true, false, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, \
                      desc[0], B, blocks_iter, t, npk, npk_pad);                                                            \
    else if (any_rule)                                                                                        \
      PMRF_LAUNCH_LDS((k_iter<LM, false, false, false, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, \
                      desc[0], B, blocks_iter, t, npk, npk_pad);                                                            \
    else if (fused && t > 0)                                                                                  \
      PMRF_LAUNCH((k_iter<LM, false, true, true>), dim3(grid_iter), lds_fused, slot_start, slot_stop, gd, block_graph, \
                  desc[0], B, blocks_iter, t, npk, npk_pad);                                                                \
    else if (persist && B == 1)                                                                               \
      PMRF_LAUNCH_LDS((k_iter<LM, true, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,           \
                  blocks_iter, t, npk, npk_pad);                                                                            \
    else if (persist)                                                                                         \
      PMRF_LAUNCH_LDS((k_iter<LM, true, false>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,          \
                  blocks_iter, t, npk, npk_pad);                                                                            \
    else if (B == 1)                                                                                          \
      PMRF_LAUNCH_LDS((k_iter<LM, false, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,          \
                  blocks_iter, t, npk, npk_pad);                                                                            \
    else                                                                                                      \
      PMRF_LAUNCH_LDS((k_iter<LM, false, false>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,         \
                  blocks_iter, t, npk, npk_pad);                                                                            \
  } while (0)
#define PMRF_LAUNCH_ITER_UNFUSED(LM)                                                                          \
  do {                                                                                                        \
    if (any_rule && B == 1)                                                                                   \
      PMRF_LAUNCH_LDS((k_iter<LM, false, true, false, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, \
                      desc[0], B, blocks_iter, t, npk, npk_pad);                                                            \
    else if (any_rule)                                                                                        \
      PMRF_LAUNCH_LDS((k_iter<LM, false, false, false, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, \
                      desc[0], B, blocks_iter, t, npk, npk_pad);                                                            \
    else if (persist && B == 1)                                                                               \
      PMRF_LAUNCH_LDS((k_iter<LM, true, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,           \
                  blocks_iter, t, npk, npk_pad);                                                                            \
    else if (persist)                                                                                         \
      PMRF_LAUNCH_LDS((k_iter<LM, true, false>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,          \
                  blocks_iter, t, npk, npk_pad);                                                                            \
    else if (B == 1)                                                                                          \
      PMRF_LAUNCH_LDS((k_iter<LM, false, true>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,          \
                  blocks_iter, t, npk, npk_pad);                                                                            \
    else                                                                                                      \
      PMRF_LAUNCH_LDS((k_iter<LM, false, false>), dim3(grid_iter), slot_start, slot_stop, gd, block_graph, desc[0], B,         \
                  blocks_iter, t, npk, npk_pad);                                                                            \
  } while (0)
#define PMRF_LAUNCH_PK(LM)                                                                                      \
  do {                                                                                                          \
    if (any_rule)                                                                                               \
      PMRF_LAUNCH((k_iter_packets<LM, true>), dim3(blocks_pk), lds_pk, pk_start, pk_stop, gd, B, t);           \
    else                                                                                                        \
      PMRF_LAUNCH((k_iter_packets<LM, false>), dim3(blocks_pk), lds_pk, pk_start, pk_stop, gd, B, t);          \
  } while (0)
      if (blocks_iter > 0) {
        switch (lm) {
          case 2: PMRF_LAUNCH_ITER(2); break;
          case 4: PMRF_LAUNCH_ITER(4); break;
          case 8: PMRF_LAUNCH_ITER_UNFUSED(8); break;
          default: PMRF_LAUNCH_ITER_UNFUSED(16); break;
        }
        HIP_TRY(hipGetLastError());
      }
      if (blocks_pk > 0 && !merge_pk) {
        switch (lm) {
          case 2: PMRF_LAUNCH_PK(2); break;
          case 4: PMRF_LAUNCH_PK(4); break;
          case 8: PMRF_LAUNCH_PK(8); break;
          default: PMRF_LAUNCH_PK(16); break;
        }
      }
#undef PMRF_LAUNCH_ITER
#undef PMRF_LAUNCH_ITER_UNFUSED
#undef PMRF_LAUNCH_PK
#undef PMRF_LAUNCH_LDS
#undef PMRF_LAUNCH
      HIP_TRY(hipGetLastError());
      // rule MIN: the vertex pass decides the labels of iteration t
      if (any_min) {
        switch (lm) {
          case 2: hipLaunchKernelGGL(k_decide<2>, dim3(blocks_vert), dim3(256), 0, s, gd, B, t); break;
          case 4: hipLaunchKernelGGL(k_decide<4>, dim3(blocks_vert), dim3(256), 0, s, gd, B, t); break;
          case 8: hipLaunchKernelGGL(k_decide<8>, dim3(blocks_vert), dim3(256), 0, s, gd, B, t); break;
          default: hipLaunchKernelGGL(k_decide<16>, dim3(blocks_vert), dim3(256), 0, s, gd, B, t); break;
        }
        HIP_TRY(hipGetLastError());
      }
      // the parameter update of iteration t: here, or (fused) inside the next
      // iteration launch and after the last one
      if (!fused || (t + 1 == max_iters && !fused_finish)) {
        if (B == 1)
          hipLaunchKernelGGL((k_fold<true>), dim3(B), dim3(kFoldThreads), 0, s, gd, desc[0], B, t + 1);
        else
          hipLaunchKernelGGL((k_fold<false>), dim3(B), dim3(kFoldThreads), 0, s, gd, desc[0], B, t + 1);
        HIP_TRY(hipGetLastError());
      }
    }
    if (fused_finish)
      hipLaunchKernelGGL(k_finish1, dim3(blocks_vert), dim3(kFoldThreads), 0, s, desc[0], max_iters);
    else
      hipLaunchKernelGGL(k_final, dim3(blocks_vert), dim3(256), 0, s, gd, B);
    HIP_TRY(hipGetLastError());
    return PMRF_OK;
  };

  // Direct launches when asked for, or while kernel timing is on (the timing
  // events sit between launches); otherwise one cached HIP graph per distinct
  // argument set, replayed on the caller's stream.
  if (no_alloc || shape.mode == kModeDirect || events) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    ++g_direct;
    return enqueue(stream);
  }
  std::string key;
  auto put = [&](const void *p, size_t n) { key.append(static_cast<const char *>(p), n); };
  put(&B, sizeof B);
  put(&max_iters, sizeof max_iters);
  put(&lm, sizeof lm);
  put(&blocks_iter, sizeof blocks_iter);
  put(&blocks_pk, sizeof blocks_pk);
  put(&grid_iter, sizeof grid_iter);
  put(&blocks_vert, sizeof blocks_vert);
  put(&threads, sizeof threads);
  put(&lds_pk, sizeof lds_pk);
  put(&any_init, sizeof any_init);
  put(&d_desc, sizeof d_desc);
  put(desc.data(), desc.size() * sizeof(GraphDev));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  put(&dev, sizeof dev);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  GraphEntry *entry = nullptr;
  for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
    if (it->key == key) {
      g_graphs.splice(g_graphs.begin(), g_graphs, it);
      entry = &g_graphs.front();
      break;
    }
  if (!entry && shape.automatic) {
    // automatic mode: the first run of an argument set is direct
    auto seen = std::find(g_seen.begin(), g_seen.end(), key);
    if (seen == g_seen.end()) {
      g_seen.push_front(key);
      if (g_seen.size() > kSeenKeys) g_seen.pop_back();
      ++g_direct;
      return enqueue(stream);
    }
    g_seen.erase(seen);
  }
  if (!entry) {
    ++g_captures;
    hipStream_t cap = capture_stream(dev);
    if (!cap) return fail(PMRF_EDEVICE, "could not create the capture stream");
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    pmrf_status st = enqueue(cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    if (st != PMRF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(PMRF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(PMRF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    hipEvent_t done = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    if (g_graphs.size() >= kGraphCacheSize) {
      GraphEntry &old = g_graphs.back();
      (void)hipEventSynchronize(old.done);
      (void)hipGraphExecDestroy(old.exec);
      (void)hipEventDestroy(old.done);
      g_graphs.pop_back();
    }
    g_graphs.push_front(GraphEntry{key, exec, done});
    entry = &g_graphs.front();
  }
  ++g_replays;
  HIP_TRY(hipGraphLaunch(entry->exec, stream));
  HIP_TRY(hipEventRecord(entry->done, stream));
  return PMRF_OK;
}

}  // namespace

// ---------------------------------------------------------------------- ABI
extern "C" pmrf_status pmrf_em_workspace_bytes(const pmrf_hoods *hoods, const pmrf_em_params *params,
                                               int64_t *bytes) {
  clear_error();
  if (!hoods || !bytes) return fail(PMRF_EINVAL, "NULL argument");
  pmrf_status s = check_params(params);
  if (s != PMRF_OK) return s;
  pmrf_em_item it{};
  it.hoods = hoods;
  it.params = *params;
  *bytes = plan_workspace(1, &it).total;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_em_run(const pmrf_hoods *hoods, const void *d_hoodbuf, const double *d_y,
                                   int32_t *d_labels, double *d_mu, double *d_sigma, double *d_hood_energy,
                                   double *d_trace, int64_t *d_iter_stats, int64_t *d_counters, void *d_ws,
                                   int64_t ws_bytes, const pmrf_em_params *params, void *hip_stream) {
  clear_error();
  if (!params) return fail(PMRF_EINVAL, "params is NULL");
  pmrf_em_item it{hoods, d_hoodbuf, d_y, d_labels, d_mu, d_sigma, d_hood_energy, d_trace, d_iter_stats, d_counters,
                  *params};
  pmrf_status s = check_item(it, -1);
  if (s != PMRF_OK) return s;
  return run_items(1, &it, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
}

// ------------------------------------------------- allocation-free entry point
namespace {
// Workspace of pmrf_em_run_noalloc: one array per GPU the library runs on,
// held until the process ends.  In host code the name `scratch` is only a
// host-side stand-in; kernels get its device address, looked up once per
// device (with that device current) and kept in g_scratch_ptr.
constexpr int64_t kScratchBytes = PMRF_NOALLOC_WS_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

pmrf_status scratch_address(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return PMRF_OK;
  }
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(PMRF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return PMRF_OK;
}

}  // namespace

extern "C" pmrf_status pmrf_em_run_noalloc(const pmrf_hoods *hoods, const void *d_hoodbuf, const double *d_y,
                                           int32_t *d_labels, double *d_mu, double *d_sigma, double *d_hood_energy,
                                           double *d_trace, int64_t *d_iter_stats, int64_t *d_counters,
                                           const pmrf_em_params *params, void *hip_stream) {
  clear_error();
  if (!params) return fail(PMRF_EINVAL, "params is NULL");
  pmrf_em_item it{hoods, d_hoodbuf, d_y, d_labels, d_mu, d_sigma, d_hood_energy, d_trace, d_iter_stats, d_counters,
                  *params};
  pmrf_status s = check_item(it, -1);
  if (s != PMRF_OK) return s;
  // the size check needs no device, so an oversized request fails before any HIP call
  const int64_t need = plan_workspace(1, &it).total;
  if (need > kScratchBytes)
    return fail(PMRF_ENOMEM, "the run needs " + std::to_string(need) + " bytes of workspace; the static workspace holds " +
                                 std::to_string(kScratchBytes));
  void *ws = nullptr;
  s = scratch_address(&ws);
  if (s != PMRF_OK) return s;
  return run_items(1, &it, ws, kScratchBytes, static_cast<hipStream_t>(hip_stream), true);
}

extern "C" pmrf_status pmrf_em_batch_workspace_bytes(int32_t B, const pmrf_em_item *items, int64_t *bytes) {
  clear_error();
  if (B < 1 || !items || !bytes) return fail(PMRF_EINVAL, "bad batch arguments");
  for (int i = 0; i < B; ++i) {
    if (!items[i].hoods) return fail(PMRF_EINVAL, "hoods is NULL (item " + std::to_string(i) + ")");
    pmrf_status s = check_params(&items[i].params);
    if (s != PMRF_OK) return s;
  }
  *bytes = plan_workspace(B, items).total;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_em_batch(int32_t B, const pmrf_em_item *items, void *d_ws, int64_t ws_bytes,
                                     void *hip_stream) {
  clear_error();
  if (B < 1 || !items) return fail(PMRF_EINVAL, "bad batch arguments");
  for (int i = 0; i < B; ++i) {
    pmrf_status s = check_item(items[i], i);
    if (s != PMRF_OK) return s;
  }
  return run_items(B, items, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
}

extern "C" pmrf_status pmrf_set_launch(const pmrf_launch *l) {
  clear_error();
  if (!l) return fail(PMRF_EINVAL, "launch is NULL");
  if (l->mode < 0 || l->mode > 3) return fail(PMRF_EINVAL, "mode must be 0..3");
  if (l->waves_per_block < 0 || l->waves_per_block > 16) return fail(PMRF_EINVAL, "waves_per_block must be 0..16");
  if (l->tiles_per_wave < 0 || l->tiles_per_wave > 4096) return fail(PMRF_EINVAL, "tiles_per_wave must be 0..4096");
  if (l->blocks_per_cu < 0 || l->blocks_per_cu > 32) return fail(PMRF_EINVAL, "blocks_per_cu must be 0..32");
  std::lock_guard<std::mutex> lk(g_launch_mu);
  g_launch = *l;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_get_launch(pmrf_launch *l) {
  clear_error();
  if (!l) return fail(PMRF_EINVAL, "launch is NULL");
  std::lock_guard<std::mutex> lk(g_launch_mu);
  *l = g_launch;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_launch_stats(int64_t *captures, int64_t *replays, int64_t *direct) {
  clear_error();
  if (!captures || !replays || !direct) return fail(PMRF_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_graph_mu);
  *captures = g_captures;
  *replays = g_replays;
  *direct = g_direct;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_profile_begin(void) {
  clear_error();
  g_prof.on = true;
  g_prof.used = 0;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_profile_end(double *total_ms, int64_t *launches) {
  clear_error();
  if (!total_ms || !launches) return fail(PMRF_EINVAL, "NULL argument");
  g_prof.on = false;
  double sum = 0.0;
  if (g_prof.used) HIP_TRY(hipEventSynchronize(g_prof.stop[g_prof.used - 1]));
  for (size_t i = 0; i < g_prof.used; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, g_prof.start[i], g_prof.stop[i]));
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)g_prof.used;
  g_prof.used = 0;
  return PMRF_OK;
}
