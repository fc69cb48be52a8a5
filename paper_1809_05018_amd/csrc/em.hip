// EM optimisation of DPP-PMRF on gfx950 (Alg. 2, EM loop; Sec. 3.2.2 "EM
// Parameter Estimation").
//
// One launch per EM iteration.  Each wave takes 64-lane work packets of whole
// neighbourhoods and, per element (neighbourhood h, member v, every label l):
//   - gathers y_v and the current labels of the packet (label bit planes from
//     __ballot, so every lane sees its neighbourhood's labels without LDS);
//   - counts in-neighbourhood neighbours per label with popcounts of its
//     adjacency bit mask against the planes (the Potts term);
//   - forms the Gaussian energy for each label, keeps the minimum, the lowest
//     arg-minimum and the gap to the runner-up (the paper's SortByKey +
//     ReduceByKey<Min>, done in registers: no replicated arrays exist);
//   - sums the minima of each neighbourhood in member order through LDS (the
//     paper's ReduceByKey<Add>) and checks the neighbourhood's convergence
//     window;
//   - the owner element of each vertex writes the vertex's new label (the
//     paper's Scatter, without write conflicts) and adds its intensity to the
//     per-label statistics of the parameter update.
// Every cross-lane and cross-block sum of the M-step and of the total energy is
// an integer sum of fixed-point limbs, so the result is independent of the
// launch shape and of how graphs are batched.  The last block of a graph to
// finish turns the sums into the next parameters (mean, standard deviation)
// and the per-iteration records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "pmrf_internal.h"

using namespace pmrf;

namespace {

// ------------------------------------------------------------ device records
// accumulator words of one graph (int64):
//   per label l: [9l] count, [9l+1 .. 9l+4] sum of (y - c_l) limbs,
//                [9l+5 .. 9l+8] sum of (y - c_l)^2 limbs   (c_l = current mean)
//   [9L .. 9L+3] total energy limbs, [9L+4] near ties, [9L+5] neighbourhoods not
//   converged, [9L+6] error bits (1: label out of range, 2: value out of range)
constexpr int kAccWords = 9 * kMaxLabels + 7;
__host__ __device__ constexpr int acc_t(int L) { return 9 * L; }
__host__ __device__ constexpr int acc_ties(int L) { return 9 * L + 4; }
__host__ __device__ constexpr int acc_nonconv(int L) { return 9 * L + 5; }
__host__ __device__ constexpr int acc_err(int L) { return 9 * L + 6; }
__host__ __device__ constexpr int acc_words(int L) { return 9 * L + 7; }

struct GraphState {
  double mu[kMaxLabels], sigma[kMaxLabels], w[kMaxLabels], lg[kMaxLabels];
  unsigned long long acc[kAccWords];
  unsigned int arrivals;  // blocks of the current launch that have finished
  int32_t done;           // 1: no further iterations (early exit or error)
  int32_t status;
  int32_t iters;
  int32_t map_conv, em_conv;
  int64_t ties_total;
};

struct GraphDev {
  const TileDesc *tiles;
  const int32_t *vid;
  const uint32_t *mask;
  const double *y;
  int32_t *x0;  // caller labels (even iterations read here)
  int32_t *x1;  // workspace labels (odd iterations read here)
  double *ring; // (W+1) x H neighbourhood sums
  double *thist;
  GraphState *st;
  const double *in_mu, *in_sigma;
  double *out_mu, *out_sigma, *out_S, *out_trace;
  int64_t *out_stats, *out_ctr;
  int64_t M;
  int32_t n, H, ntiles, L, P, W, max_iters, early_exit, init_from_labels;
  double beta, tol, sigma_min, tie_eps;
  int32_t block0, nblocks;    // blocks of this graph in an iteration launch
  int32_t vblock0, vnblocks;  // blocks of this graph in a vertex-parallel launch
  int32_t tiles_per_block;
};

constexpr int kDescPerPack = 12;
struct DescPack {
  GraphDev d[kDescPerPack];
  int32_t first, count;
};

// -------------------------------------------------------- fixed-point sums
// A value t is accumulated as round(|t| * 2^64) split into four base-2^32 limbs,
// each added (with the sign of t) into its own int64 word; the words are
// combined exactly at the end.  Integer addition is associative, so the sum
// does not depend on order or grouping.
__device__ __forceinline__ void fx_add(unsigned long long *acc, double t, int &err) {
  double v = fabs(t) * 0x1p64;
  if (!(v < 0x1p126)) {  // also rejects NaN
    err |= 2;
    return;
  }
  double a3 = floor(v * 0x1p-96);
  v = v - a3 * 0x1p96;
  double a2 = floor(v * 0x1p-64);
  v = v - a2 * 0x1p64;
  double a1 = floor(v * 0x1p-32);
  v = v - a1 * 0x1p32;
  double a0 = rint(v);
  long long s = t < 0.0 ? -1 : 1;
  if (a0 != 0.0) atomicAdd(acc + 0, (unsigned long long)(s * (long long)a0));
  if (a1 != 0.0) atomicAdd(acc + 1, (unsigned long long)(s * (long long)a1));
  if (a2 != 0.0) atomicAdd(acc + 2, (unsigned long long)(s * (long long)a2));
  if (a3 != 0.0) atomicAdd(acc + 3, (unsigned long long)(s * (long long)a3));
}

__device__ double fx_value(const unsigned long long *a) {
  unsigned long long w0 = 0, w1 = 0, w2 = 0;
  auto add3 = [&](unsigned long long x0, unsigned long long x1, unsigned long long x2) {
    unsigned long long s0 = w0 + x0;
    unsigned long long c0 = s0 < x0;
    unsigned long long t1 = w1 + x1;
    unsigned long long c1 = t1 < x1;
    unsigned long long s1 = t1 + c0;
    c1 += s1 < t1;
    w2 = w2 + x2 + c1;
    w0 = s0;
    w1 = s1;
  };
  for (int k = 0; k < 4; ++k) {
    long long v = (long long)a[k];
    unsigned long long sx = v < 0 ? ~0ull : 0ull;
    unsigned long long u = (unsigned long long)v;
    unsigned long long hi = (unsigned long long)(v >> 32);
    if (k == 0) add3(u, sx, sx);
    else if (k == 1) add3(u << 32, hi, sx);
    else if (k == 2) add3(0, u, sx);
    else add3(0, u << 32, hi);
  }
  bool neg = (long long)w2 < 0;
  if (neg) {
    w0 = ~w0;
    w1 = ~w1;
    w2 = ~w2;
    w0 += 1;
    unsigned long long c = w0 == 0;
    w1 += c;
    c = c && w1 == 0;
    w2 += c;
  }
  double r = ((double)w2 * 0x1p128 + (double)w1 * 0x1p64) + (double)w0;
  r *= 0x1p-64;
  return neg ? -r : r;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void block_acc_flush(unsigned long long *lacc, unsigned long long *gacc, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) {
    unsigned long long v = lacc[i];
    if (v) __hip_atomic_fetch_add(gacc + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Parameters for the next iteration from the exact per-label sums
// ("Update Parameters"): mu = c + D1, sigma^2 = D2 - D1^2 with
// D1 = sum(y - c)/n, D2 = sum((y - c)^2)/n, c = the mean used this iteration
// (pass 0 of the starting update uses c = 0 and keeps sigma).  A label with no
// vertex keeps its parameters.  Updated in place, one label at a time.
__device__ void set_label_theta(GraphState *st, int l, double mu, double sigma) {
  st->mu[l] = mu;
  st->sigma[l] = sigma;
  st->w[l] = 1.0 / (2.0 * sigma * sigma);
  st->lg[l] = log(sigma);
}

__device__ __forceinline__ unsigned long long acc_load(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void acc_store(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ double fx_load_value(unsigned long long *p) {
  unsigned long long a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = acc_load(p + k);
  return fx_value(a);
}

__device__ void update_theta(GraphState *st, int L, double sigma_min, bool mean_only) {
  for (int l = 0; l < L; ++l) {
    long long cnt = (long long)acc_load(st->acc + 9 * l);
    if (cnt <= 0) continue;
    double nd = (double)cnt;
    double d1 = fx_load_value(st->acc + 9 * l + 1) / nd;
    if (mean_only) {
      set_label_theta(st, l, d1, st->sigma[l]);
      continue;
    }
    double d2 = fx_load_value(st->acc + 9 * l + 5) / nd;
    double var = d2 - d1 * d1;
    double sg = sqrt(var > 0.0 ? var : 0.0);
    set_label_theta(st, l, st->mu[l] + d1, sg < sigma_min ? sigma_min : sg);
  }
}

__device__ void clear_acc(GraphState *st, int L) {
  for (int i = 0; i < acc_words(L); ++i) acc_store(st->acc + i, 0ull);
  __hip_atomic_store(&st->arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __threadfence();
}

// Graph owning a block: the last graph whose first block is <= block.
__device__ __forceinline__ int find_graph(const GraphDev *graphs, int B, int block, bool vertex_launch) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    int first = vertex_launch ? graphs[mid].vblock0 : graphs[mid].block0;
    if (first <= block) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------- tile kernels
template <int LMAX>
struct Theta {
  double mu[LMAX], w[LMAX], lg[LMAX];
};

// Energies of one element under every label; returns min, argmin, gap.
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

// Owner-element work: label write, parameter statistics, near-tie flag.
__device__ __forceinline__ void owner_update(unsigned long long *lacc, int32_t *xw, int v, int a, double dsel,
                                             int &err) {
  xw[v] = a;
  atomicAdd(lacc + 9 * a, 1ull);
  fx_add(lacc + 9 * a + 1, dsel, err);
  fx_add(lacc + 9 * a + 5, dsel * dsel, err);
}

// Neighbourhood total: convergence window and energy total.
__device__ __forceinline__ bool hood_done(const GraphDev &G, int t, int h, double S, unsigned long long *lacc,
                                          int &err) {
  const int slots = G.W + 1;
  G.ring[(size_t)(t % slots) * G.H + h] = S;
  bool conv = t >= G.W;
  if (conv) {
    for (int w = 1; w <= G.W; ++w) {
      double prev = G.ring[(size_t)((t - w) % slots) * G.H + h];
      if (!(fabs(S - prev) < G.tol)) conv = false;
    }
  }
  fx_add(lacc + acc_t(G.L), S, err);
  return conv;
}

// Packets of whole neighbourhoods of at most 64 members (kinds SMALL, MID).
template <int LMAX>
__device__ void do_packed(const GraphDev &G, const TileDesc &td, int t, const int32_t *__restrict__ xr,
                          int32_t *__restrict__ xw, const Theta<LMAX> &th, unsigned long long *lacc, double *mb,
                          int lane, int &err) {
  const bool valid = lane < td.nelem;
  int v = 0, xv = 0;
  double yv = 0.0;
  uint64_t am = 0;
  if (valid) {
    const int e = td.elem_start + lane;
    v = G.vid[e];
    xv = xr[v];
    yv = G.y[v];
    if (td.words == 1) {
      am = G.mask[td.mask_start + lane];
    } else {
      const uint32_t *mw = G.mask + td.mask_start + 2 * lane;
      am = (uint64_t)mw[0] | ((uint64_t)mw[1] << 32);
    }
    if ((unsigned)xv >= (unsigned)G.L) err |= 1;
  }
  uint64_t planes[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < G.P) planes[k] = __ballot(valid && ((xv >> k) & 1));
  const uint64_t below = (2ull << lane) - 1ull;  // lanes 0..lane
  const uint64_t sm = td.start_mask;
  const int base = 63 - __clzll(sm & below);
  const uint64_t after = sm & ~below;
  const int end = after ? (__ffsll((long long)after) - 1) : td.nelem;
  const int j = lane - base;
  const int s = end - base;
  const uint64_t self = 1ull << j;
  const bool owner = valid && (am & self);
  const uint64_t nbr = am & ~self;
  const int deg = __popcll(nbr);
  int cnt[LMAX];
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    uint64_t eq = ~0ull;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < G.P) {
        uint64_t pk = planes[k] >> base;
        eq &= ((l >> k) & 1) ? pk : ~pk;
      }
    cnt[l] = __popcll(nbr & eq);
  }
  double m, gap, dsel;
  int a;
  element_energy<LMAX>(th, G.L, G.beta, yv, deg, cnt, m, a, gap, dsel);
  if (owner) owner_update(lacc, xw, v, a, dsel, err);
  const uint64_t ties = __ballot(owner && gap < G.tie_eps);
  mb[lane] = valid ? m : 0.0;
  wave_sync_lds();
  bool leader = valid && j == 0;
  bool conv = true;
  if (leader) {
    double S = 0.0;
    for (int k = 0; k < s; ++k) S = S + mb[base + k];
    const int h = td.hood_start + __popcll(sm & below) - 1;
    conv = hood_done(G, t, h, S, lacc, err);
  }
  const uint64_t nonconv = __ballot(leader && !conv);
  if (lane == 0) {
    if (ties) atomicAdd(lacc + acc_ties(G.L), (unsigned long long)__popcll(ties));
    if (nonconv) atomicAdd(lacc + acc_nonconv(G.L), (unsigned long long)__popcll(nonconv));
  }
  wave_sync_lds();
}

// One neighbourhood of 65..1024 members, in chunks of 64 (kind LARGE).
template <int LMAX>
__device__ void do_large(const GraphDev &G, const TileDesc &td, int t, const int32_t *__restrict__ xr,
                         int32_t *__restrict__ xw, const Theta<LMAX> &th, unsigned long long *lacc, double *mb,
                         uint64_t *pl /* 4 x 16 words */, int lane, int &err) {
  const int s = td.nelem;
  const int W = td.words;
  const int chunks = (s + 63) >> 6;
  for (int c = 0; c < chunks; ++c) {
    const int jj = c * 64 + lane;
    int xv = 0;
    const bool valid = jj < s;
    if (valid) {
      xv = xr[G.vid[td.elem_start + jj]];
      if ((unsigned)xv >= (unsigned)G.L) err |= 1;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < G.P) {
        uint64_t b = __ballot(valid && ((xv >> k) & 1));
        if (lane == 0) pl[k * 16 + c] = b;
      }
  }
  wave_sync_lds();
  double S = 0.0;  // lane 0 accumulates in member order
  unsigned long long ties = 0;
  for (int c = 0; c < chunks; ++c) {
    const int jj = c * 64 + lane;
    const bool valid = jj < s;
    int v = 0;
    double yv = 0.0;
    int cnt[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) cnt[l] = 0;
    int deg = 0;
    bool owner = false;
    if (valid) {
      v = G.vid[td.elem_start + jj];
      yv = G.y[v];
      const uint32_t *mw = G.mask + td.mask_start + (size_t)jj * W;
      for (int wi = 0; wi < W; ++wi) {
        uint32_t word = mw[wi];
        if (wi == (jj >> 5)) {
          const uint32_t selfb = 1u << (jj & 31);
          owner = (word & selfb) != 0;
          word &= ~selfb;
        }
        deg += __popc(word);
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
          uint32_t eq = ~0u;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < G.P) {
              uint32_t pk = (uint32_t)(pl[k * 16 + (wi >> 1)] >> ((wi & 1) * 32));
              eq &= ((l >> k) & 1) ? pk : ~pk;
            }
          cnt[l] += __popc(word & eq);
        }
      }
    }
    double m, gap, dsel;
    int a;
    element_energy<LMAX>(th, G.L, G.beta, yv, deg, cnt, m, a, gap, dsel);
    if (owner) owner_update(lacc, xw, v, a, dsel, err);
    ties += __popcll(__ballot(owner && gap < G.tie_eps));
    mb[lane] = valid ? m : 0.0;
    wave_sync_lds();
    if (lane == 0) {
      const int lim = min(64, s - c * 64);
      for (int k = 0; k < lim; ++k) S = S + mb[k];
    }
    wave_sync_lds();
  }
  if (lane == 0) {
    bool conv = hood_done(G, t, td.hood_start, S, lacc, err);
    if (ties) atomicAdd(lacc + acc_ties(G.L), ties);
    if (!conv) atomicAdd(lacc + acc_nonconv(G.L), 1ull);
  }
}

// The last block of a graph: fold the sums into the next parameters and the
// per-iteration records; clear the sums for the next launch.
__device__ void finalize_iteration(const GraphDev &G, int t) {
  GraphState *st = G.st;
  const int L = G.L;
  unsigned long long errbits = acc_load(st->acc + acc_err(L));
  if (errbits) {
    st->status = (errbits & 1) ? PMRF_EBADLABEL : PMRF_ERANGE;
    st->done = 1;
  } else {
    double T = fx_load_value(st->acc + acc_t(L));
    long long ties = (long long)acc_load(st->acc + acc_ties(L));
    long long nonconv = (long long)acc_load(st->acc + acc_nonconv(L));
    G.thist[t] = T;
    if (G.out_trace) G.out_trace[t] = T;
    if (G.out_stats) {
      G.out_stats[2 * t] = ties;
      G.out_stats[2 * t + 1] = nonconv;
    }
    st->ties_total += ties;
    if (nonconv == 0 && t >= G.W && st->map_conv < 0) st->map_conv = t;
    if (t >= G.W && st->em_conv < 0) {
      bool ok = true;
      for (int w = 1; w <= G.W; ++w)
        if (!(fabs(T - G.thist[t - w]) < G.tol)) ok = false;
      if (ok) st->em_conv = t;
    }
    update_theta(st, L, G.sigma_min, false);
    st->iters = t + 1;
    if (G.early_exit && nonconv == 0 && t >= G.W) st->done = 1;
  }
  clear_acc(st, L);
}

// ------------------------------------------------------------------ kernels
__global__ void k_write_desc(DescPack pack, GraphDev *dst) {
  int i = threadIdx.x;
  if (i < pack.count) dst[pack.first + i] = pack.d[i];
}

// Set up the state of every graph from the caller's starting parameters.
__global__ void k_setup(const GraphDev *graphs, int B) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= B) return;
  const GraphDev &G = graphs[g];
  GraphState *st = G.st;
  st->done = 0;
  st->status = 0;
  st->iters = 0;
  st->map_conv = -1;
  st->em_conv = -1;
  st->ties_total = 0;
  st->arrivals = 0u;
  for (int i = 0; i < kAccWords; ++i) st->acc[i] = 0ull;
  bool ok = true;
  for (int l = 0; l < G.L; ++l) {
    double mu = G.in_mu[l], sigma = G.in_sigma[l];
    if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(mu)) ok = false;
    st->mu[l] = mu;
    st->sigma[l] = sigma;
  }
  if (!ok) {
    st->status = PMRF_EBADPARAM;
    st->done = 1;
    return;
  }
  for (int l = 0; l < G.L; ++l) set_label_theta(st, l, st->mu[l], st->sigma[l]);
}

// Parameter update from the starting labels (used when init_from_labels is
// set): pass 0 sums y per label (mean), pass 1 sums (y - mean) and (y - mean)^2.
__global__ void k_mstep_init(const GraphDev *graphs, int B, int pass) {
  __shared__ unsigned long long lacc[kAccWords];
  __shared__ int last;
  const int g = find_graph(graphs, B, blockIdx.x, true);
  const GraphDev &G = graphs[g];
  GraphState *st = G.st;
  if (!G.init_from_labels || st->done) return;
  const int words = acc_words(G.L);
  for (int i = threadIdx.x; i < words; i += blockDim.x) lacc[i] = 0ull;
  __syncthreads();
  int err = 0;
  const int b = blockIdx.x - G.vblock0;
  const int per = (G.n + G.vnblocks - 1) / G.vnblocks;
  const int v0 = b * per, v1 = min(G.n, v0 + per);
  for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    int x = G.x0[v];
    if ((unsigned)x >= (unsigned)G.L) {
      err |= 1;
      continue;
    }
    double d = G.y[v] - (pass == 0 ? 0.0 : st->mu[x]);
    atomicAdd(lacc + 9 * x, 1ull);
    fx_add(lacc + 9 * x + 1, d, err);
    if (pass == 1) fx_add(lacc + 9 * x + 5, d * d, err);
  }
  if (err) atomicOr(lacc + acc_err(G.L), (unsigned long long)err);
  __syncthreads();
  block_acc_flush(lacc, st->acc, words);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&st->arrivals, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
           (unsigned)(G.vnblocks - 1);
  __syncthreads();
  if (!last || threadIdx.x != 0) return;
  __threadfence();
  unsigned long long errbits = acc_load(st->acc + acc_err(G.L));
  if (errbits) {
    st->status = (errbits & 1) ? PMRF_EBADLABEL : PMRF_ERANGE;
    st->done = 1;
  } else {
    update_theta(st, G.L, G.sigma_min, pass == 0);
  }
  clear_acc(st, G.L);
}

// One EM iteration over every graph of the launch.
template <int LMAX>
__global__ __launch_bounds__(1024) void k_iter(const GraphDev *__restrict__ graphs, int B, int t) {
  __shared__ unsigned long long lacc[acc_words(LMAX)];
  __shared__ double mbuf[16][64];
  __shared__ uint64_t planes[16][64];
  __shared__ int last;
  const int g = find_graph(graphs, B, blockIdx.x, false);
  const GraphDev &G = graphs[g];
  GraphState *st = G.st;
  if (t >= G.max_iters || st->done) return;
  const int words = acc_words(G.L);
  for (int i = threadIdx.x; i < words; i += blockDim.x) lacc[i] = 0ull;
  Theta<LMAX> th;
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    th.mu[l] = l < G.L ? st->mu[l] : 0.0;
    th.w[l] = l < G.L ? st->w[l] : 0.0;
    th.lg[l] = l < G.L ? st->lg[l] : 0.0;
  }
  __syncthreads();
  const int32_t *xr = (t & 1) ? G.x1 : G.x0;
  int32_t *xw = (t & 1) ? G.x0 : G.x1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int b = blockIdx.x - G.block0;
  const int t0 = b * G.tiles_per_block;
  const int t1 = min(G.ntiles, t0 + G.tiles_per_block);
  int err = 0;
  for (int ti = t0 + wave; ti < t1; ti += nw) {
    const TileDesc td = G.tiles[ti];
    if (td.kind == kLarge)
      do_large<LMAX>(G, td, t, xr, xw, th, lacc, mbuf[wave], planes[wave], lane, err);
    else
      do_packed<LMAX>(G, td, t, xr, xw, th, lacc, mbuf[wave], lane, err);
  }
  if (err) atomicOr(lacc + acc_err(G.L), (unsigned long long)err);
  __syncthreads();
  block_acc_flush(lacc, st->acc, words);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&st->arrivals, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
           (unsigned)(G.nblocks - 1);
  __syncthreads();
  if (!last || threadIdx.x != 0) return;
  __threadfence();
  finalize_iteration(G, t);
}

// Copy results to the caller's buffers.
__global__ void k_final(const GraphDev *graphs, int B) {
  const int g = find_graph(graphs, B, blockIdx.x, true);
  const GraphDev &G = graphs[g];
  GraphState *st = G.st;
  const int b = blockIdx.x - G.vblock0;
  const int iters = st->iters;
  const int stride = G.vnblocks * blockDim.x;
  if (iters & 1)  // final labels sit in the workspace buffer
    for (int v = b * blockDim.x + threadIdx.x; v < G.n; v += stride) G.x0[v] = G.x1[v];
  if (G.out_S && iters > 0) {
    const double *src = G.ring + (size_t)((iters - 1) % (G.W + 1)) * G.H;
    for (int h = b * blockDim.x + threadIdx.x; h < G.H; h += stride) G.out_S[h] = src[h];
  }
  if (b == 0 && threadIdx.x == 0) {
    for (int l = 0; l < G.L; ++l) {
      G.out_mu[l] = st->mu[l];
      G.out_sigma[l] = st->sigma[l];
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

struct LaunchShape {
  int waves_per_block, tiles_per_wave;
};

LaunchShape resolve_shape() {
  std::lock_guard<std::mutex> lk(g_launch_mu);
  LaunchShape s{g_launch.waves_per_block > 0 ? g_launch.waves_per_block : 4,
                g_launch.tiles_per_wave > 0 ? g_launch.tiles_per_wave : 8};
  return s;
}

struct WsPlan {
  int64_t desc_off = 0;
  std::vector<int64_t> state_off, x1_off, ring_off, thist_off;
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

WsPlan plan_workspace(int B, const pmrf_em_item *items) {
  WsPlan p;
  int64_t off = 0;
  p.desc_off = off;
  off += align_up((int64_t)B * (int64_t)sizeof(GraphDev), 256);
  for (int i = 0; i < B; ++i) {
    const pmrf_hoods *h = items[i].hoods;
    p.state_off.push_back(off);
    off += align_up(sizeof(GraphState), 256);
    p.x1_off.push_back(off);
    off += align_up((int64_t)h->n * 4, 256);
    p.ring_off.push_back(off);
    off += align_up((int64_t)(items[i].params.conv_window + 1) * h->H * 8, 256);
    p.thist_off.push_back(off);
    off += align_up((int64_t)std::max(1, items[i].params.max_iters) * 8, 256);
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

pmrf_status run_items(int B, const pmrf_em_item *items, void *d_ws, int64_t ws_bytes, hipStream_t stream) {
  WsPlan plan = plan_workspace(B, items);
  if (!d_ws) return fail(PMRF_EINVAL, "workspace is NULL");
  if (ws_bytes < plan.total) return fail(PMRF_ENOMEM, "workspace smaller than the required size");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(PMRF_EINVAL, "workspace must be 256-byte aligned");
  const LaunchShape shape = resolve_shape();
  const int tpb = shape.waves_per_block * shape.tiles_per_wave;
  const int threads = shape.waves_per_block * kWave;
  char *ws = static_cast<char *>(d_ws);
  std::vector<GraphDev> desc(B);
  int blocks_iter = 0, blocks_vert = 0, max_iters = 0, Lmax = 2;
  for (int i = 0; i < B; ++i) {
    const pmrf_em_item &it = items[i];
    const pmrf_hoods *h = it.hoods;
    GraphDev &G = desc[i];
    const char *hb = static_cast<const char *>(it.d_hoodbuf);
    G.tiles = reinterpret_cast<const TileDesc *>(hb + h->layout.tiles_off);
    G.vid = reinterpret_cast<const int32_t *>(hb + h->layout.vid_off);
    G.mask = reinterpret_cast<const uint32_t *>(hb + h->layout.mask_off);
    G.y = it.d_y;
    G.x0 = it.d_labels;
    G.x1 = reinterpret_cast<int32_t *>(ws + plan.x1_off[i]);
    G.ring = reinterpret_cast<double *>(ws + plan.ring_off[i]);
    G.thist = reinterpret_cast<double *>(ws + plan.thist_off[i]);
    G.st = reinterpret_cast<GraphState *>(ws + plan.state_off[i]);
    G.in_mu = it.d_mu;
    G.in_sigma = it.d_sigma;
    G.out_mu = it.d_mu;
    G.out_sigma = it.d_sigma;
    G.out_S = it.d_hood_energy;
    G.out_trace = it.d_trace;
    G.out_stats = it.d_iter_stats;
    G.out_ctr = it.d_counters;
    G.M = h->M;
    G.n = h->n;
    G.H = (int32_t)h->H;
    G.ntiles = (int32_t)h->tiles.size();
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
    G.tiles_per_block = tpb;
    G.block0 = blocks_iter;
    G.nblocks = std::max(1, (G.ntiles + tpb - 1) / tpb);
    blocks_iter += G.nblocks;
    G.vblock0 = blocks_vert;
    G.vnblocks = std::max(1, std::min(1024, (G.n + 1023) / 1024));
    blocks_vert += G.vnblocks;
    max_iters = std::max(max_iters, G.max_iters);
    Lmax = std::max(Lmax, G.L);
  }
  GraphDev *d_desc = reinterpret_cast<GraphDev *>(ws + plan.desc_off);
  // descriptors travel as kernel arguments, so no host buffer must outlive the call
  for (int first = 0; first < B; first += kDescPerPack) {
    DescPack pack{};
    pack.first = first;
    pack.count = std::min(kDescPerPack, B - first);
    for (int k = 0; k < pack.count; ++k) pack.d[k] = desc[first + k];
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, stream, pack, d_desc);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_setup, dim3((B + 63) / 64), dim3(64), 0, stream, (const GraphDev *)d_desc, B);
  HIP_TRY(hipGetLastError());
  bool any_init = false;
  for (int i = 0; i < B; ++i) any_init |= desc[i].init_from_labels != 0;
  if (any_init) {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_mstep_init, dim3(blocks_vert), dim3(256), 0, stream, (const GraphDev *)d_desc, B, pass);
      HIP_TRY(hipGetLastError());
    }
  }
  const int lm = lmax_for(Lmax);
  for (int t = 0; t < max_iters; ++t) {
    switch (lm) {
      case 2: hipLaunchKernelGGL(k_iter<2>, dim3(blocks_iter), dim3(threads), 0, stream, (const GraphDev *)d_desc, B, t); break;
      case 4: hipLaunchKernelGGL(k_iter<4>, dim3(blocks_iter), dim3(threads), 0, stream, (const GraphDev *)d_desc, B, t); break;
      case 8: hipLaunchKernelGGL(k_iter<8>, dim3(blocks_iter), dim3(threads), 0, stream, (const GraphDev *)d_desc, B, t); break;
      default: hipLaunchKernelGGL(k_iter<16>, dim3(blocks_iter), dim3(threads), 0, stream, (const GraphDev *)d_desc, B, t); break;
    }
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_final, dim3(blocks_vert), dim3(256), 0, stream, (const GraphDev *)d_desc, B);
  HIP_TRY(hipGetLastError());
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
  if (l->mode < 0 || l->mode > 2) return fail(PMRF_EINVAL, "mode must be 0, 1 or 2");
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
