// Host side of the neighbourhood construction (Sec. 3.2.1 maximal cliques,
// Sec. 3.1 and Sec. 3.2.2 "Construction of Neighborhoods": clique plus 1-ring,
// duplicates removed, members ordered by vertex id) and the device layout the
// EM kernels stream.
//
// The paper builds neighbourhoods with data-parallel primitives on the device
// (a Map counting neighbours, a Scan, a Map writing them, then SortByKey and
// Unique).  Here they are built once per graph on the host, outside the timed
// EM loop, and uploaded as wave-sized work packets with one in-neighbourhood
// adjacency bit mask per element.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>

#include "pmrf_internal.h"

using namespace pmrf;

namespace {

// ---------------------------------------------------------------- validation
pmrf_status validate_csr(int32_t n, const int32_t *rp, const int32_t *ci) {
  if (n < 0) return fail(PMRF_EINVAL, "n must be >= 0");
  if (!rp) return fail(PMRF_EINVAL, "row_ptr is NULL");
  if (rp[0] != 0) return fail(PMRF_EINVAL, "row_ptr[0] must be 0");
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) return fail(PMRF_EINVAL, "row_ptr must be non-decreasing (row " + std::to_string(v) + ")");
  if (rp[n] > 0 && !ci) return fail(PMRF_EINVAL, "col_idx is NULL");
  for (int32_t v = 0; v < n; ++v) {
    for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
      int32_t u = ci[k];
      if (u < 0 || u >= n) return fail(PMRF_EINVAL, "col_idx out of range in row " + std::to_string(v));
      if (u == v) return fail(PMRF_EINVAL, "self loop at vertex " + std::to_string(v));
      if (k > rp[v] && ci[k - 1] >= u)
        return fail(PMRF_EINVAL, "row " + std::to_string(v) + " is not strictly ascending");
    }
  }
  for (int32_t v = 0; v < n; ++v)
    for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
      int32_t u = ci[k];
      if (!std::binary_search(ci + rp[u], ci + rp[u + 1], v))
        return fail(PMRF_EINVAL, "edge " + std::to_string(v) + "-" + std::to_string(u) + " is missing its reverse");
    }
  return PMRF_OK;
}

// ------------------------------------------------ maximal clique enumeration
// Bron-Kerbosch with Tomita pivoting, run from each vertex in a degeneracy
// ordering (Eppstein, Loffler, Strash 2010): candidates are the later
// neighbours, exclusions the earlier ones.
struct Mce {
  int32_t n;
  const int32_t *rp, *ci;
  std::vector<int32_t> out_vid;
  std::vector<int64_t> out_ptr{0};
  std::vector<int32_t> R;

  bool adjacent(int32_t a, int32_t b) const { return std::binary_search(ci + rp[a], ci + rp[a + 1], b); }

  static void intersect_row(const std::vector<int32_t> &S, const int32_t *row, int32_t len, std::vector<int32_t> &out) {
    out.clear();
    int32_t i = 0, j = 0, ns = (int32_t)S.size();
    while (i < ns && j < len) {
      if (S[i] < row[j]) ++i;
      else if (S[i] > row[j]) ++j;
      else { out.push_back(S[i]); ++i; ++j; }
    }
  }

  void expand(std::vector<int32_t> &P, std::vector<int32_t> &X) {
    if (P.empty() && X.empty()) {
      std::vector<int32_t> c(R);
      std::sort(c.begin(), c.end());
      out_vid.insert(out_vid.end(), c.begin(), c.end());
      out_ptr.push_back((int64_t)out_vid.size());
      return;
    }
    // pivot: vertex of P u X with the most neighbours in P
    int32_t pivot = -1, best = -1;
    for (const std::vector<int32_t> *S : {&P, &X})
      for (int32_t u : *S) {
        int32_t cnt = 0;
        const int32_t *row = ci + rp[u];
        int32_t len = rp[u + 1] - rp[u];
        int32_t i = 0, j = 0;
        while (i < (int32_t)P.size() && j < len) {
          if (P[i] < row[j]) ++i;
          else if (P[i] > row[j]) ++j;
          else { ++cnt; ++i; ++j; }
        }
        if (cnt > best) { best = cnt; pivot = u; }
      }
    std::vector<int32_t> cand;
    for (int32_t v : P)
      if (!adjacent(pivot, v)) cand.push_back(v);
    std::vector<int32_t> P2, X2;
    for (int32_t v : cand) {
      intersect_row(P, ci + rp[v], rp[v + 1] - rp[v], P2);
      intersect_row(X, ci + rp[v], rp[v + 1] - rp[v], X2);
      R.push_back(v);
      std::vector<int32_t> P3(P2), X3(X2);
      expand(P3, X3);
      R.pop_back();
      P.erase(std::lower_bound(P.begin(), P.end(), v));
      X.insert(std::lower_bound(X.begin(), X.end(), v), v);
    }
  }

  void run() {
    // degeneracy ordering by repeated removal of a minimum-degree vertex
    std::vector<int32_t> deg(n), order;
    order.reserve(n);
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; ++v) { deg[v] = rp[v + 1] - rp[v]; maxd = std::max(maxd, deg[v]); }
    std::vector<std::vector<int32_t>> bucket(maxd + 1);
    for (int32_t v = 0; v < n; ++v) bucket[deg[v]].push_back(v);
    std::vector<char> removed(n, 0);
    int32_t d = 0;
    for (int32_t done = 0; done < n;) {
      d = std::max(0, d - 1);
      while (d <= maxd && bucket[d].empty()) ++d;
      int32_t v = bucket[d].back();
      bucket[d].pop_back();
      if (removed[v] || deg[v] != d) continue;  // stale bucket entry
      removed[v] = 1;
      order.push_back(v);
      ++done;
      for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
        int32_t u = ci[k];
        if (!removed[u]) bucket[--deg[u]].push_back(u);
      }
    }
    std::vector<int32_t> pos(n);
    for (int32_t i = 0; i < n; ++i) pos[order[i]] = i;
    std::vector<int32_t> P, X;
    for (int32_t v : order) {
      P.clear();
      X.clear();
      for (int32_t k = rp[v]; k < rp[v + 1]; ++k) (pos[ci[k]] > pos[v] ? P : X).push_back(ci[k]);
      R.assign(1, v);
      expand(P, X);
    }
  }
};

}  // namespace

// -------------------------------------------------------------------- build
extern "C" pmrf_status pmrf_build_neighborhoods(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t k,
                                                pmrf_hoods **out) {
  clear_error();
  if (!out) return fail(PMRF_EINVAL, "out is NULL");
  if (k < 1) return fail(PMRF_EINVAL, "k must be >= 1");
  if (k > kMaxHoodRadius) return fail(PMRF_EUNSUPPORTED, "k above " + std::to_string(kMaxHoodRadius) + " is not supported");
  pmrf_status st = validate_csr(n, row_ptr, col_idx);
  if (st != PMRF_OK) return st;
  if (n > kMaxSlotVertices)
    return fail(PMRF_EUNSUPPORTED, "more than " + std::to_string(kMaxSlotVertices) + " vertices in one graph");
  pmrf_hoods *hd = nullptr;
  try {
    hd = new pmrf_hoods();
    hd->n = n;
    Mce mce{n, row_ptr, col_idx, {}, {0}, {}};
    mce.run();
    // canonical order: lexicographic over ascending cliques
    int64_t H = (int64_t)mce.out_ptr.size() - 1;
    std::vector<int64_t> idx(H);
    for (int64_t h = 0; h < H; ++h) idx[h] = h;
    const int32_t *cv = mce.out_vid.data();
    const int64_t *cp = mce.out_ptr.data();
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      return std::lexicographical_compare(cv + cp[a], cv + cp[a + 1], cv + cp[b], cv + cp[b + 1]);
    });
    hd->H = H;
    hd->clique_ptr.assign(1, 0);
    for (int64_t h = 0; h < H; ++h) {
      int64_t a = idx[h];
      hd->clique_vid.insert(hd->clique_vid.end(), cv + cp[a], cv + cp[a + 1]);
      hd->clique_ptr.push_back((int64_t)hd->clique_vid.size());
    }
    // k-neighbourhood = the clique and every vertex within k edges of a member
    // (rings added one hop at a time from the previous ring), ascending, each
    // vertex once; the search stops early once a neighbourhood outgrows the
    // supported size
    std::vector<int64_t> stamp(n, -1);
    hd->k = k;
    hd->hood_ptr.assign(1, 0);
    for (int64_t h = 0; h < H; ++h) {
      size_t start = hd->hood_vid.size();
      for (int64_t q = hd->clique_ptr[h]; q < hd->clique_ptr[h + 1]; ++q) {
        int32_t c = hd->clique_vid[q];
        if (stamp[c] != h) { stamp[c] = h; hd->hood_vid.push_back(c); }
      }
      size_t ring0 = start, ring1 = hd->hood_vid.size();
      for (int32_t depth = 1; depth <= k && ring1 - start <= (size_t)kMaxHood; ++depth) {
        for (size_t f = ring0; f < ring1; ++f) {
          const int32_t c = hd->hood_vid[f];
          for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
            int32_t u = col_idx[e];
            if (stamp[u] != h) { stamp[u] = h; hd->hood_vid.push_back(u); }
          }
        }
        ring0 = ring1;
        ring1 = hd->hood_vid.size();
      }
      std::sort(hd->hood_vid.begin() + start, hd->hood_vid.end());
      int64_t s = (int64_t)(hd->hood_vid.size() - start);
      hd->max_hood = std::max<int32_t>(hd->max_hood, (int32_t)std::min<int64_t>(s, INT32_MAX));
      hd->hood_ptr.push_back((int64_t)hd->hood_vid.size());
      if (hd->max_hood > kMaxHood) break;
    }
    hd->M = (int64_t)hd->hood_vid.size();
    if (hd->max_hood > kMaxHood) {
      int mh = hd->max_hood;
      delete hd;
      return fail(PMRF_EUNSUPPORTED, "a neighbourhood has " + std::to_string(mh) + " members (limit 1024)");
    }
    if (hd->M >= (int64_t(1) << 31) / 2) {
      delete hd;
      return fail(PMRF_EUNSUPPORTED, "more than 2^30 neighbourhood elements in one graph");
    }
    // owner element: the vertex's place in the first clique holding it
    hd->owner.assign(n, -1);
    for (int64_t h = 0; h < H; ++h)
      for (int64_t q = hd->clique_ptr[h]; q < hd->clique_ptr[h + 1]; ++q) {
        int32_t v = hd->clique_vid[q];
        if (hd->owner[v] >= 0) continue;
        auto b = hd->hood_vid.begin() + hd->hood_ptr[h], e = hd->hood_vid.begin() + hd->hood_ptr[h + 1];
        hd->owner[v] = hd->hood_ptr[h] + (std::lower_bound(b, e, v) - b);
      }
    // processing order: neighbourhoods of at most 64 members first, then the
    // larger ones, each group in canonical order; the device arrays follow it
    // (perm maps a processing index to the canonical one)
    hd->perm.clear();
    for (int64_t h = 0; h < H; ++h)
      if (hd->hood_ptr[h + 1] - hd->hood_ptr[h] <= kWave) hd->perm.push_back((int32_t)h);
    for (int64_t h = 0; h < H; ++h)
      if (hd->hood_ptr[h + 1] - hd->hood_ptr[h] > kWave) hd->perm.push_back((int32_t)h);
    hd->hood_ptr32.assign(1, 0);
    hd->dev_vid.clear();
    hd->dev_vid.reserve((size_t)hd->M);
    for (int64_t hp = 0; hp < H; ++hp) {
      const int64_t h = hd->perm[hp];
      hd->dev_vid.insert(hd->dev_vid.end(), hd->hood_vid.begin() + hd->hood_ptr[h],
                         hd->hood_vid.begin() + hd->hood_ptr[h + 1]);
      hd->hood_ptr32.push_back((int32_t)hd->dev_vid.size());
    }
    // the elements of each vertex (processing-order indices) in canonical
    // neighbourhood order, and the element in its last canonical neighbourhood
    {
      std::vector<int32_t> inv(H);
      for (int64_t hp = 0; hp < H; ++hp) inv[hd->perm[hp]] = (int32_t)hp;
      hd->occ_ptr.assign((size_t)n + 1, 0);
      for (int64_t e = 0; e < hd->M; ++e) hd->occ_ptr[hd->hood_vid[e] + 1]++;
      for (int32_t v = 0; v < n; ++v) hd->occ_ptr[v + 1] += hd->occ_ptr[v];
      hd->occ.assign((size_t)std::max<int64_t>(1, hd->M), 0);
      std::vector<int32_t> fill(hd->occ_ptr.begin(), hd->occ_ptr.end() - 1);
      hd->lastbits.assign((size_t)(hd->M / 64 + 2), 0ull);
      for (int64_t h = 0; h < H; ++h) {
        const int64_t pe = hd->hood_ptr32[inv[h]];
        for (int64_t e = hd->hood_ptr[h]; e < hd->hood_ptr[h + 1]; ++e)
          hd->occ[fill[hd->hood_vid[e]]++] = (int32_t)(pe + (e - hd->hood_ptr[h]));
      }
      for (int32_t v = 0; v < n; ++v) {
        const int32_t e = hd->occ[hd->occ_ptr[v + 1] - 1];
        hd->lastbits[e >> 6] |= 1ull << (e & 63);
      }
    }
    // work packets, in processing order: next-fit over the neighbourhoods of
    // at most 64 members (one joins the open packet while its lanes hold it,
    // else opens a new one); a packet holding a neighbourhood above 32 members
    // is MID (two adjacency words per element), else SMALL (one).  A LARGE
    // neighbourhood takes a packet of its own.
    std::vector<int32_t> tile_of((size_t)H), pos_of((size_t)H);
    bool open = false;
    for (int64_t hp = 0; hp < H; ++hp) {
      const int32_t s = (int32_t)(hd->hood_ptr[hd->perm[hp] + 1] - hd->hood_ptr[hd->perm[hp]]);
      if (s <= kWave) {
        if (!open || hd->tiles.back().nelem + s > kWave) {
          TileDesc t{};
          t.elem_start = hd->hood_ptr32[hp];
          t.hood_start = (int32_t)hp;
          t.kind = kSmall;
          t.words = 1;
          hd->tiles.push_back(t);
          open = true;
        }
        TileDesc &t = hd->tiles.back();
        pos_of[hp] = t.nelem;
        t.start_mask |= uint64_t(1) << t.nelem;
        t.nelem = (int16_t)(t.nelem + s);
        if (s > 32) {
          t.kind = kMid;
          t.words = 2;
        }
      } else {
        open = false;
        TileDesc t{};
        t.elem_start = hd->hood_ptr32[hp];
        t.hood_start = (int32_t)hp;
        t.kind = kLarge;
        t.words = (uint8_t)((s + 31) / 32);
        t.start_mask = 1;
        t.nelem = (int16_t)s;
        hd->tiles.push_back(t);
        pos_of[hp] = 0;
      }
      tile_of[hp] = (int32_t)hd->tiles.size() - 1;
    }
    int64_t words_total = 0;
    for (TileDesc &t : hd->tiles) {
      t.mask_start = (int32_t)words_total;
      words_total += (int64_t)t.nelem * t.words;
    }
    // adjacency words: bit p of an element's words marks member p of its
    // neighbourhood as a neighbour, its own bit marks the owner element
    hd->mask.assign((size_t)words_total, 0u);
    std::vector<int32_t> loc(n, -1);
    for (int64_t hp = 0; hp < H; ++hp) {
      const int64_t h = hd->perm[hp];
      const int64_t o = hd->hood_ptr[h];  // canonical element offset (owner indices are canonical)
      const int32_t s = (int32_t)(hd->hood_ptr[h + 1] - o);
      const TileDesc &t = hd->tiles[tile_of[hp]];
      const int words = t.words;
      for (int32_t j = 0; j < s; ++j) loc[hd->hood_vid[o + j]] = j;
      const size_t base = (size_t)t.mask_start + (size_t)pos_of[hp] * words;
      for (int32_t j = 0; j < s; ++j) {
        int32_t v = hd->hood_vid[o + j];
        uint32_t *w = hd->mask.data() + base + (size_t)j * words;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
          int32_t p = loc[col_idx[e]];
          if (p >= 0) { w[p >> 5] |= 1u << (p & 31); hd->A++; }
        }
        if (hd->owner[v] == o + j) w[j >> 5] |= 1u << (j & 31);
      }
      for (int32_t j = 0; j < s; ++j) loc[hd->hood_vid[o + j]] = -1;
    }
    hd->slot_tiles = 0;
    while (hd->slot_tiles < (int64_t)hd->tiles.size() && hd->tiles[hd->slot_tiles].kind != kLarge) ++hd->slot_tiles;
    // slot layout and chunk headers: packet t's elements in slots [64 t, 64 t + 64)
    const int64_t ntiles = (int64_t)hd->tiles.size();
    const int64_t nchunks = (ntiles + kChunkTiles - 1) / kChunkTiles;
    bool any_mid = false;
    for (const TileDesc &t : hd->tiles) any_mid |= t.kind == kMid;
    // padded to whole chunks (empty slots), so a chunk's loads need no bounds,
    // and to at least one chunk (an empty graph's one block reads chunk 0)
    const int64_t chunks_alloc = std::max<int64_t>(1, nchunks);
    const size_t slots = (size_t)(chunks_alloc * kChunkTiles) * kWave;
    hd->svid.assign(slots, (int32_t)kSlotEmpty);
    hd->smask.assign(slots, 0u);
    hd->smask_hi.assign(any_mid ? slots : 0, 0u);
    hd->chdr.assign((size_t)chunks_alloc, ChunkHdr{});
    for (int64_t ti = 0; ti < ntiles; ++ti) {
      const TileDesc &t = hd->tiles[ti];
      if (t.kind == kLarge) continue;
      int first = 0;  // lane of the current neighbourhood's first member
      for (int k = 0; k < t.nelem; ++k) {
        if ((t.start_mask >> k) & 1) first = k;
        hd->svid[ti * kWave + k] = (int32_t)((uint32_t)hd->dev_vid[t.elem_start + k] |
                                             ((uint32_t)(k - first) << kSlotJShift));
        hd->smask[ti * kWave + k] = hd->mask[t.mask_start + (size_t)k * t.words];
        if (t.kind == kMid) hd->smask_hi[ti * kWave + k] = hd->mask[t.mask_start + (size_t)k * t.words + 1];
      }
    }
    for (int64_t ck = 0; ck < nchunks; ++ck) {
      ChunkHdr &c = hd->chdr[ck];
      const int64_t tb = ck * kChunkTiles, te = std::min(ntiles, tb + kChunkTiles);
      c.elem_start = hd->tiles[tb].elem_start;
      c.hood_start = hd->tiles[tb].hood_start;
      c.hood_end = te < ntiles ? hd->tiles[te].hood_start : (int32_t)hd->H;
      for (int64_t ti = tb; ti < te; ++ti) {
        const TileDesc &t = hd->tiles[ti];
        const int i = (int)(ti - tb);
        if (t.kind == kLarge) c.flags |= kHdrLarge;
        if (t.kind == kMid) c.flags |= 1 << (kHdrMidShift + i);
        // offsets of a chunk without LARGE packets stay below 8 * 64
        c.elem_off[i] = (uint16_t)std::min<int64_t>(t.elem_start - c.elem_start, 0xffff);
      }
    }
    // member vertex range of each superchunk's slot-layout packets
    {
      const int64_t sc = superchunk_chunks_of(nchunks);
      const int64_t nsuper = std::max<int64_t>(1, (nchunks + sc - 1) / sc);
      hd->srange.assign((size_t)(2 * nsuper), 0);
      for (int64_t sp = 0; sp < nsuper; ++sp) {
        int32_t lo = INT32_MAX, hi = INT32_MIN;
        const size_t s0 = (size_t)(sp * sc * kChunkTiles) * kWave;
        const size_t s1 = std::min(hd->svid.size(), (size_t)((sp + 1) * sc * kChunkTiles) * kWave);
        for (size_t k = s0; k < s1; ++k) {
          const uint32_t w = (uint32_t)hd->svid[k];
          if (w == kSlotEmpty) continue;
          const int32_t v = (int32_t)(w & kSlotVidMask);
          lo = std::min(lo, v);
          hi = std::max(hi, v + 1);
        }
        if (lo > hi) lo = hi = 0;
        hd->srange[2 * sp] = lo;
        hd->srange[2 * sp + 1] = hi;
      }
    }
    LayoutSizes z{};
    z.ntiles = ntiles;
    z.H = hd->H;
    z.M = hd->M;
    z.mask_words = (int64_t)hd->mask.size();
    z.nchdr = (int64_t)hd->chdr.size();
    z.slots = (int64_t)hd->svid.size();
    z.slots_hi = (int64_t)hd->smask_hi.size();
    z.nsrange = (int64_t)hd->srange.size();
    z.nlastbits = (int64_t)hd->lastbits.size();
    z.nocc_ptr = (int64_t)hd->occ_ptr.size();
    z.nocc = (int64_t)hd->occ.size();
    hd->layout = layout_of(z);
    hd->ntiles = ntiles;
  } catch (const std::bad_alloc &) {
    delete hd;
    return fail(PMRF_ENOMEM, "host allocation failed while building neighbourhoods");
  }
  *out = hd;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_hoods_get_info(const pmrf_hoods *h, pmrf_hoods_info *info) {
  clear_error();
  if (!h || !info) return fail(PMRF_EINVAL, "NULL argument");
  info->n = h->n;
  info->H = h->H;
  info->M = h->M;
  info->A = h->A;
  info->max_hood = h->max_hood;
  info->tiles = h->ntiles;
  info->device_bytes = h->layout.total;
  return PMRF_OK;
}

pmrf_hoods::~pmrf_hoods() {
  for (void *p : {dev_layout, dev_clique_ptr, dev_clique_vid, dev_hood_ptr, dev_hood_vid, dev_owner})
    if (p) (void)hipFree(p);
}

namespace {

// int32 device array -> host int64 (or int32) array
hipError_t fetch_widened(int64_t *dst, const void *src, int64_t count) {
  if (count <= 0 || !dst) return hipSuccess;
  std::vector<int32_t> tmp((size_t)count);
  hipError_t e = hipMemcpy(tmp.data(), src, (size_t)count * 4, hipMemcpyDeviceToHost);
  for (int64_t i = 0; i < count; ++i) dst[i] = tmp[(size_t)i];
  return e;
}

hipError_t fetch(int32_t *dst, const void *src, int64_t count) {
  if (count <= 0 || !dst) return hipSuccess;
  return hipMemcpy(dst, src, (size_t)count * 4, hipMemcpyDeviceToHost);
}

// exports of a neighbourhood structure built on the device
pmrf_status export_device(const pmrf_hoods *h, int64_t *hood_ptr, int32_t *hood_vid, int64_t *clique_ptr,
                          int32_t *clique_vid, int64_t *owner) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(PMRF_EDEVICE, "no current HIP device");
  if (cur != h->device && hipSetDevice(h->device) != hipSuccess) return fail(PMRF_EDEVICE, "hipSetDevice failed");
  hipError_t e = fetch_widened(hood_ptr, h->dev_hood_ptr, h->H + 1);
  if (e == hipSuccess) e = fetch(hood_vid, h->dev_hood_vid, h->M);
  if (e == hipSuccess) e = fetch_widened(clique_ptr, h->dev_clique_ptr, h->H + 1);
  if (e == hipSuccess) e = fetch(clique_vid, h->dev_clique_vid, h->dev_clique_total);
  if (e == hipSuccess) e = fetch_widened(owner, h->dev_owner, h->n);
  if (cur != h->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return fail(PMRF_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  return PMRF_OK;
}

}  // namespace

extern "C" pmrf_status pmrf_hoods_export(const pmrf_hoods *h, int64_t *hood_ptr, int32_t *hood_vid,
                                         int64_t *clique_ptr, int32_t *clique_vid, int64_t *owner) {
  clear_error();
  if (!h) return fail(PMRF_EINVAL, "hoods is NULL");
  if (h->on_device) return export_device(h, hood_ptr, hood_vid, clique_ptr, clique_vid, owner);
  if (hood_ptr) std::memcpy(hood_ptr, h->hood_ptr.data(), h->hood_ptr.size() * sizeof(int64_t));
  if (hood_vid && h->M) std::memcpy(hood_vid, h->hood_vid.data(), (size_t)h->M * sizeof(int32_t));
  if (clique_ptr) std::memcpy(clique_ptr, h->clique_ptr.data(), h->clique_ptr.size() * sizeof(int64_t));
  if (clique_vid && !h->clique_vid.empty())
    std::memcpy(clique_vid, h->clique_vid.data(), h->clique_vid.size() * sizeof(int32_t));
  if (owner && h->n) std::memcpy(owner, h->owner.data(), (size_t)h->n * sizeof(int64_t));
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_hoods_device_buffer(const pmrf_hoods *h, void **d_layout, int64_t *held_bytes) {
  clear_error();
  if (!h) return fail(PMRF_EINVAL, "hoods is NULL");
  if (d_layout) *d_layout = h->on_device ? h->dev_layout : nullptr;
  if (held_bytes)
    *held_bytes = h->on_device ? h->layout.total + 4 * (2 * (h->H + 1) + h->dev_clique_total + h->M + h->n) : 0;
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_hoods_upload(const pmrf_hoods *h, void *d_buf, int64_t bytes, void *stream) {
  clear_error();
  if (!h || !d_buf) return fail(PMRF_EINVAL, "NULL argument");
  if (bytes < h->layout.total) return fail(PMRF_ENOMEM, "device buffer smaller than info.device_bytes");
  if (reinterpret_cast<uintptr_t>(d_buf) % 256) return fail(PMRF_EINVAL, "device buffer must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(d_buf);
  hipError_t e = hipSuccess;
  if (h->on_device) {
    e = hipMemcpyAsync(base, h->dev_layout, (size_t)h->layout.total, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(PMRF_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    return PMRF_OK;
  }
  if (!h->tiles.empty())
    e = hipMemcpyAsync(base + h->layout.tiles_off, h->tiles.data(), h->tiles.size() * sizeof(TileDesc),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + h->layout.hptr_off, h->hood_ptr32.data(), h->hood_ptr32.size() * 4,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && h->M)
    e = hipMemcpyAsync(base + h->layout.vid_off, h->dev_vid.data(), (size_t)h->M * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->mask.empty())
    e = hipMemcpyAsync(base + h->layout.mask_off, h->mask.data(), h->mask.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->chdr.empty())
    e = hipMemcpyAsync(base + h->layout.chdr_off, h->chdr.data(), h->chdr.size() * sizeof(ChunkHdr),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->svid.empty())
    e = hipMemcpyAsync(base + h->layout.svid_off, h->svid.data(), h->svid.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->smask.empty())
    e = hipMemcpyAsync(base + h->layout.smask_off, h->smask.data(), h->smask.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->perm.empty())
    e = hipMemcpyAsync(base + h->layout.perm_off, h->perm.data(), h->perm.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->lastbits.empty())
    e = hipMemcpyAsync(base + h->layout.lastbits_off, h->lastbits.data(), h->lastbits.size() * 8, hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess && !h->occ_ptr.empty())
    e = hipMemcpyAsync(base + h->layout.occptr_off, h->occ_ptr.data(), h->occ_ptr.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->occ.empty())
    e = hipMemcpyAsync(base + h->layout.occ_off, h->occ.data(), h->occ.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->srange.empty())
    e = hipMemcpyAsync(base + h->layout.srange_off, h->srange.data(), h->srange.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !h->smask_hi.empty())
    e = hipMemcpyAsync(base + h->layout.smaskhi_off, h->smask_hi.data(), h->smask_hi.size() * 4,
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(PMRF_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_replicate_hood_array(int64_t H, const int64_t *hood_ptr, int32_t L, int32_t *test_label,
                                                 int64_t *old_index, int32_t *hood_id) {
  clear_error();
  if (H < 0 || !hood_ptr || !test_label || !old_index || !hood_id) return fail(PMRF_EINVAL, "NULL argument");
  if (L < 1) return fail(PMRF_EINVAL, "L must be >= 1");
  int64_t k = 0;
  for (int64_t h = 0; h < H; ++h) {
    int64_t s = hood_ptr[h + 1] - hood_ptr[h];
    for (int32_t l = 0; l < L; ++l)
      for (int64_t j = 0; j < s; ++j, ++k) {
        test_label[k] = l;
        old_index[k] = hood_ptr[h] + j;
        hood_id[k] = (int32_t)h;
      }
  }
  return PMRF_OK;
}

extern "C" pmrf_status pmrf_replicate_indices(const pmrf_hoods *h, int32_t L, int32_t *test_label, int64_t *old_index,
                                              int32_t *hood_id) {
  if (!h) {
    clear_error();
    return fail(PMRF_EINVAL, "hoods is NULL");
  }
  if (!h->on_device) return pmrf_replicate_hood_array(h->H, h->hood_ptr.data(), L, test_label, old_index, hood_id);
  std::vector<int64_t> hp((size_t)h->H + 1);
  clear_error();
  pmrf_status st = export_device(h, hp.data(), nullptr, nullptr, nullptr, nullptr);
  if (st != PMRF_OK) return st;
  return pmrf_replicate_hood_array(h->H, hp.data(), L, test_label, old_index, hood_id);
}

extern "C" void pmrf_hoods_free(pmrf_hoods *h) { delete h; }
