// Host-side channel layout: validation, canonicalisation and the
// destination-sorted entry arrays (the paper's "target layer", Optimized GPU
// algorithm step 1).  Pure host C++; no HIP calls.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "ephbte.h"

namespace ephbte {

// Packed per-entry key: partner state in the high 29 bits, mode in the low 3.
inline uint32_t pack_pnu(int32_t partner, int32_t mode) {
    return (static_cast<uint32_t>(partner) << 3) | static_cast<uint32_t>(mode);
}

struct HostLayout {
    int32_t S = 0;
    int64_t n_input = 0;              // channels the caller passed
    int64_t n_channels = 0;           // channels kept by the selection
    int64_t E = 0;                    // entries = 2 * n_channels
    int32_t n_modes = 0;
    int32_t nq[3] = {0, 0, 0};        // q grid
    std::vector<int64_t> row_ptr;     // [S+1] entries of destination d: [row_ptr[d], row_ptr[d+1])
    std::vector<uint32_t> pnu;        // [E] partner << 3 | mode, ascending inside a destination
    std::vector<int32_t> ent_chan;    // [E] caller channel index of the entry
    std::vector<uint32_t> kq;         // [S] k coordinates in q-grid units, 10 bits each (k0,k1,k2)
    std::vector<int32_t> pmin, pmax;  // [S] smallest / largest partner of each destination
    std::vector<int32_t> dropped;     // caller indices of the channels the selection removed
    // field term: [S][3][2] state of the same band one k step up / down along
    // each axis (periodic), -1 if not in the list; empty when some (k, band)
    // is held by two states
    std::vector<int32_t> nbr;
};

// Validates the problem, applies the channel selection of opts (may be NULL:
// keep every channel) and builds the layout.  On failure returns the status
// and fills *err with a description.
ephbte_status build_host_layout(const ephbte_problem *p, const ephbte_build_opts *opts,
                                HostLayout *out, std::string *err);

// Work-split of the destination segments into chunks of at most
// chunk_entries entries (each destination gets at least one chunk, possibly
// empty).  chunk_beg has n_chunks+1 boundaries; dest_chunk has S+1.
struct ChunkTable {
    std::vector<int64_t> chunk_beg;   // n_chunks + 1 (the last is the end of the last segment)
    std::vector<int64_t> chunk_end;   // n_chunks
    std::vector<int32_t> chunk_dest;
    std::vector<int32_t> dest_chunk;
    int64_t n_chunks = 0;
    bool one_per_dest = true;
};
ChunkTable make_chunks(const std::vector<int64_t> &row_ptr, int64_t chunk_entries);

// The same split over per-destination segments [seg_beg[d], seg_end[d]) that
// need not be contiguous with each other (the upper part p > d of each row).
ChunkTable make_chunks_seg(const std::vector<int64_t> &seg_beg, const std::vector<int64_t> &seg_end,
                           int64_t chunk_entries);

// Workgroup tiles: runs of consecutive chunks [c0, c1).  When the partners of
// all their destinations lie in [p_lo, p_hi] with at most lds_states states,
// the tile stages those partners in LDS (lds = 1); a chunk whose destination's
// partners span more than lds_states states goes to a global-memory tile.
// Each tile holds at most target_entries entries (at least one chunk).
struct Tile {
    int64_t c0, c1;        // chunks [c0, c1)
    int32_t p_lo, p_hi;    // LDS window of partner states (inclusive; at least one state
                           // when lds = 1, see make_tiles)
    int32_t lds;           // 1: partners staged in LDS, 0: read from global memory,
                           // 2: staged in LDS with the records in q order (pair records,
                           // see order_pair_tiles)
    int32_t pad;
};
std::vector<Tile> make_tiles(const ChunkTable &ct, const std::vector<int64_t> &row_ptr,
                             const std::vector<int32_t> &pmin, const std::vector<int32_t> &pmax,
                             int32_t lds_states, int64_t target_entries);

// Batch tiles: up to dmax consecutive destinations whose partner ranges
// span at most window_cap states (a single destination may exceed it), cut
// into n_sub partner sub-tiles of pt states from p_lo.  Every destination x
// of a tile owns n_sub + 1 slots of the sub-tile offset array, from
// off_base + (x - d0) (n_sub + 1): slot k is the first entry of x whose
// partner is >= p_lo + k pt (so sub-tile k is [slot k, slot k+1)).  The
// offsets themselves are searched on the device; *slots receives their count.
struct BTile {
    int32_t d0, d1, p_lo, n_sub;
    int64_t off_base;
};
std::vector<BTile> make_btiles(const std::vector<int32_t> &pmin, const std::vector<int32_t> &pmax,
                               int32_t pt, int32_t dmax, int32_t window_cap, int64_t *slots);

// Phonon-side layout: the channels grouped by the phonon they exchange.  A
// channel (i, j, nu) emits or absorbs phonon (nu, q) with q = k_j - k_i in one
// orientation and (nu, -q) in the other, so each channel belongs to one
// unordered pair {q, -q}; its canonical member qc is the smaller linear index
// of the two.  Channels are grouped into pair records (a, b) oriented so that
// k_b - k_a = qc, one slot per mode, and the records are bucketed by qc.
// Inside a bucket they are ordered by (min(a, b), max(a, b)), which does not
// depend on how the build is split over threads.
struct PhononLayout {
    int64_t n_pairs = 0;
    std::vector<uint32_t> pa, pb;       // [n_pairs]
    std::vector<int32_t> slot_chan;     // [n_modes][n_pairs]: caller channel, -1 if the pair has no such mode
    std::vector<int64_t> bucket_beg;    // [n_buckets + 1] pair ranges
    std::vector<int32_t> bucket_q;      // [n_buckets] qc
    std::vector<int32_t> bucket_qm;     // [n_buckets] linear index of -qc (= qc when q = -q)
    std::vector<uint32_t> bucket_modes; // [n_buckets] bit nu: the bucket holds a channel of mode nu
    std::vector<int32_t> q_bucket;      // [Nq]: 2 b + side of the bucket b holding q (side 1: q = -qc), -1 if none
};
// Channels of elastic modes are kept (the collision integral depends on their
// N); the phonon-side kernels skip those modes.
PhononLayout build_phonon_layout(const HostLayout &L);

// Pair records of the single-copy pass.  Row d holds the pairs (d, p) with
// p > d in partner order, each with one |g|^2 slot per mode (the caller's
// channel of that mode, -1 when the pair has none), so that every channel of
// a pair is evaluated from one partner gather and the partner side of the
// pair is one sum.
struct PairRows {
    int64_t n_pairs = 0;
    int64_t n_filled = 0;               // slots holding a channel
    std::vector<int64_t> row_ptr;       // [S + 1]
    std::vector<uint32_t> partner;      // [n_pairs]
    std::vector<int32_t> slot_chan;     // [n_modes][n_pairs]
};
PairRows build_pair_rows(const HostLayout &L);

// Table row of the difference q = k_p - k_d, as the pair pass computes it:
// with the padded box, (key_p - key_d) + qoff over the states' packed box
// coordinates; otherwise the linear index of q on the q grid (keys are the
// packed grid coordinates, 10 bits an axis).
struct RowKey {
    const uint32_t *key = nullptr;   // [S]
    bool padq = false;
    int32_t qoff = 0;
    int32_t n[3] = {1, 1, 1};
    int32_t shift = 0;               // order_pair_tiles sorts by row >> shift first
};
int64_t row_of(const RowKey &k, int32_t d, int32_t p);

// Pair records in q order.  Inside every LDS tile (lds = 1) of the pair
// pass, the records are sorted by (table row of k_p - k_d >> rk.shift,
// destination, partner), so that the lanes of a batch read few rows of the
// {hw, N} table (2^shift neighbouring rows form one group, inside which the
// records of a destination are consecutive, and so are their channels when
// the caller lists the channels by state pair),
// and the tile's records are cut into chunks_per_tile equal chunks (a
// multiple of it when a chunk would exceed max_chunk records).  The window
// of such a tile must hold its destinations too (p_lo <= every destination
// with records).  A record's word is then (partner - p_lo) << 16 |
// (destination - p_lo); elsewhere it stays the absolute partner.  A tile
// whose window exceeds 65536 states keeps destination order.  The chunk
// table is renumbered: destinations of a q-ordered tile own no chunk of
// their own (their dest_chunk ranges cover only q-ordered chunks, which
// carry no row partials).
struct PairOrder {
    ChunkTable chunks;
    std::vector<Tile> tiles;          // c0, c1 renumbered; lds = 2 for q-ordered tiles
    std::vector<uint32_t> perm;       // [n_pairs] new position -> record in destination order
    std::vector<uint32_t> word;       // [n_pairs] stream word of the record at that position
};
PairOrder order_pair_tiles(const ChunkTable &pc, const std::vector<Tile> &tiles,
                           const std::vector<uint32_t> &partner, const RowKey &rk, int chunks_per_tile,
                           int64_t max_chunk);

// Runs fn(t, begin, end) over [0, n) split into contiguous ranges on up to
// `threads` host threads (deterministic partition).
void parallel_ranges(int64_t n, int threads,
                     const std::function<void(int, int64_t, int64_t)> &fn);
int host_threads();

}  // namespace ephbte
