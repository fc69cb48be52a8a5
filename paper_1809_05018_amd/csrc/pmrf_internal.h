// Internal data layout shared by the host builder and the HIP kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pmrf.h"

namespace pmrf {

constexpr int kWave = 64;
constexpr int kMaxLabels = 16;
constexpr int kMaxHood = 1024;
constexpr int kMaxHoodRadius = 8;  // k of the k-neighbourhoods
constexpr int kMaxWindow = 8;

// Work packet kinds.  SMALL and MID tiles pack whole neighbourhoods of at most
// 64 members into the 64 lanes of one wave (next-fit in processing order); a
// tile holding one of 33..64 members is MID (two 32-bit adjacency words per
// element, for every element of the tile), else SMALL (one word).  A LARGE
// tile holds one neighbourhood of 65..1024 members processed in 64-element
// pieces (ceil(s/32) words per element).
enum TileKind : uint8_t { kSmall = 0, kMid = 1, kLarge = 2 };

// One wave-sized work packet.  Elements of the packet are contiguous in the
// element arrays; neighbourhoods inside it are consecutive in processing order.
struct TileDesc {
  uint64_t start_mask;  // bit i set: lane i starts a neighbourhood (SMALL/MID); 1 for LARGE
  int32_t elem_start;   // first element
  int32_t hood_start;   // processing index of the first neighbourhood
  int32_t mask_start;   // first adjacency word
  int16_t nelem;        // elements in the packet (<= 64, or the neighbourhood size for LARGE)
  uint8_t kind;         // TileKind
  uint8_t words;        // adjacency words per element
};
static_assert(sizeof(TileDesc) == 24, "TileDesc layout");

#ifndef PMRF_CHUNK_TILES
#define PMRF_CHUNK_TILES 10
#endif
constexpr int kChunkTiles = PMRF_CHUNK_TILES;  // packets per statistics chunk (part of the result's definition)
static_assert(kChunkTiles >= 8 && kChunkTiles <= 23, "chunk header layout; record rows use 8 packets of LDS");

// Header of one chunk of kChunkTiles consecutive packets, for the slot layout:
// packet t owns slots [64 t, 64 t + 64) of the slot arrays (member id, low and
// high adjacency word; unused slots hold id -1), so a wave can request a
// chunk's element data knowing only the chunk index.  Chunks with a LARGE
// packet are processed from the element arrays instead.
struct ChunkHdr {
  int32_t elem_start;                // first element of the chunk (element arrays)
  int32_t hood_start, hood_end;      // the chunk holds neighbourhoods [hood_start, hood_end)
  int32_t flags;                     // bit 0: a LARGE packet; bit 8 + i: packet i is MID (two words)
  uint16_t elem_off[kChunkTiles];    // first element of packet i, relative to elem_start
};
static_assert(sizeof(ChunkHdr) % 4 == 0 && sizeof(ChunkHdr) <= 64 * 4, "ChunkHdr: one dword per lane");
constexpr int kHdrLarge = 1;
// slot word: member vertex (bits 0..25) and the member's index inside its
// neighbourhood (bits 26..31); an unused slot holds all ones
constexpr uint32_t kSlotEmpty = 0xffffffffu;
constexpr int kSlotJShift = 26;
constexpr uint32_t kSlotVidMask = (1u << kSlotJShift) - 1u;
constexpr int32_t kMaxSlotVertices = (1 << kSlotJShift) - 1;
constexpr int kHdrMidShift = 8;

// Chunks per superchunk (one statistics record): 4, 8 or 16, the smallest
// that keeps a graph at or below kMaxRecordsPerPass records.  A function of
// the graph alone, so it belongs to the result's definition.
constexpr int kMaxRecordsPerPass = 256;
constexpr int kMaxSuperChunks = 16;
inline int32_t superchunk_chunks_of(int64_t nchunks) {
  return nchunks <= 4 * kMaxRecordsPerPass ? 4 : nchunks <= 8 * kMaxRecordsPerPass ? 8 : kMaxSuperChunks;
}

// Offsets (bytes) of the arrays inside the uploaded device buffer.
struct DeviceLayout {
  int64_t tiles_off, hptr_off, vid_off, mask_off;
  int64_t chdr_off, svid_off, smask_off, smaskhi_off;  // slot layout
  int64_t perm_off;                                     // processing index -> canonical neighbourhood
  int64_t srange_off;                                   // member vertex range of each superchunk
  int64_t lastbits_off;                                 // element holds the last occurrence of its vertex
  int64_t occptr_off, occ_off;                          // each vertex's elements, canonical hood order
  int64_t total;
};

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Entry counts of the device arrays; both builders place them with layout_of.
struct LayoutSizes {
  int64_t ntiles, H, M, mask_words, nchdr, slots, slots_hi, nsrange, nlastbits, nocc_ptr, nocc;
};

inline DeviceLayout layout_of(const LayoutSizes &z) {
  DeviceLayout L{};
  L.tiles_off = 0;
  L.hptr_off = align_up(z.ntiles * (int64_t)sizeof(TileDesc), 256);
  L.vid_off = L.hptr_off + align_up((z.H + 1) * 4, 256);
  L.mask_off = L.vid_off + align_up(z.M * 4, 256);
  L.chdr_off = L.mask_off + align_up(z.mask_words * 4, 256);
  L.svid_off = L.chdr_off + align_up(z.nchdr * (int64_t)sizeof(ChunkHdr), 256);
  L.smask_off = L.svid_off + align_up(z.slots * 4, 256);
  L.smaskhi_off = L.smask_off + align_up(z.slots * 4, 256);
  L.perm_off = L.smaskhi_off + align_up(z.slots_hi * 4, 256);
  L.srange_off = L.perm_off + align_up(z.H * 4, 256);
  L.lastbits_off = L.srange_off + align_up(z.nsrange * 4, 256);
  L.occptr_off = L.lastbits_off + align_up(z.nlastbits * 8, 256);
  L.occ_off = L.occptr_off + align_up(z.nocc_ptr * 4, 256);
  L.total = L.occ_off + align_up(z.nocc * 4, 256);
  if (L.total == 0) L.total = 256;
  return L;
}

}  // namespace pmrf

// Host object behind the opaque pmrf_hoods handle.  The host builder fills
// the vectors below; the device builder leaves them empty and keeps the
// layout and the canonical arrays in device memory it owns (dev_*).
struct pmrf_hoods {
  ~pmrf_hoods();
  int32_t n = 0;
  int32_t k = 1;  // neighbourhood radius
  int64_t H = 0, M = 0, A = 0;
  int32_t max_hood = 0;
  std::vector<int64_t> clique_ptr;
  std::vector<int32_t> clique_vid;
  std::vector<int64_t> hood_ptr;
  std::vector<int32_t> hood_vid;
  // device arrays use the processing order: neighbourhoods of at most 64
  // members first, then the larger ones, each group in canonical order
  std::vector<int32_t> perm;        // processing index -> canonical index
  std::vector<int32_t> hood_ptr32;  // element offsets in processing order
  std::vector<int32_t> dev_vid;     // members in processing order
  std::vector<int64_t> owner;  // element owning each vertex
  // device layout, built once
  std::vector<pmrf::TileDesc> tiles;
  int64_t slot_tiles = 0;  // leading packets without a LARGE one (all LARGE packets come last)
  std::vector<uint32_t> mask;  // adjacency words (bit j' = in-hood neighbour j'; own bit = owner flag)
  std::vector<pmrf::ChunkHdr> chdr;               // one per chunk of packets
  std::vector<int32_t> svid;                      // slot layout: member id (-1: unused slot)
  std::vector<uint32_t> smask, smask_hi;          // slot layout: adjacency words 0 and 1 (the latter only if MID packets exist)
  // per superchunk s: [srange[2 s], srange[2 s + 1]) holds the member vertices
  // of its slot-layout packets (empty range where it has none)
  std::vector<int32_t> srange;
  // scatter rules other than the owner's: bit e of lastbits is set when
  // element e (processing order) holds its vertex in the vertex's last
  // neighbourhood in canonical order; occ[occ_ptr[v] .. occ_ptr[v + 1]) are
  // the elements holding v, in canonical neighbourhood order
  std::vector<uint64_t> lastbits;
  std::vector<int32_t> occ_ptr, occ;
  int64_t ntiles = 0;  // packets of the layout
  pmrf::DeviceLayout layout{};
  // built on the device: the layout (layout.total bytes) and the canonical
  // arrays as int32 (clique_ptr and hood_ptr H + 1, clique members, hood
  // members M, owner n), all on device `device`
  bool on_device = false;
  int device = -1;
  void *dev_layout = nullptr;
  void *dev_clique_ptr = nullptr, *dev_clique_vid = nullptr, *dev_hood_ptr = nullptr, *dev_hood_vid = nullptr,
       *dev_owner = nullptr;
  int64_t dev_clique_total = 0;
};

namespace pmrf {
// error state (abi.cpp)
pmrf_status fail(pmrf_status code, const std::string &msg);
void clear_error();
}  // namespace pmrf
