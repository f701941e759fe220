// host_logic.hpp -- the library's host-only logic: checks of the public
// structures, the serving footprint, the byte layout of a serving batch and
// the row copies that pack events into it and results out of it.
//
// Nothing here touches HIP, so the same source builds into the library and,
// with the address / undefined-behaviour / thread sanitizers, into a plain
// CPU test program.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/ktf.h"

namespace ktf {

// Bounds on sizes the checks accept: every index and byte count derived
// from them stays far inside int64 / size_t.
constexpr int64_t kMaxPitch = int64_t(1) << 40;
constexpr int64_t kMaxEventSeeds = INT32_MAX;
constexpr int64_t kMaxEventHits = INT32_MAX;

// The building's candidate rows are split into region_count regions, each
// with its own row counter (spreading same-address atomics).  Two launches
// reserve rows: the seed fit (blocks of 256 seeds, one row each) and the
// merge (blocks of merge_seeds seeds, up to max_cands rows each); block b of
// a launch of G blocks reserves in region b * regions / G, so a region
// serves at most ceil(G / regions) blocks of either.
constexpr int kMaxRegions = 64;
constexpr int kMergeThreads = 256;
// lanes per seed in the merge, and seeds per merge block
constexpr int merge_lanes(int max_cands) { return max_cands <= 4 ? 1 : (max_cands <= 10 ? 2 : 4); }
constexpr int merge_seeds(int lps) { return kMergeThreads / lps; }
inline int64_t seed_blocks(int64_t n_seeds) { return n_seeds > 0 ? (n_seeds + 255) / 256 : 1; }
inline int64_t merge_blocks(int64_t n_seeds, int max_cands) {
  const int64_t sb = merge_seeds(merge_lanes(max_cands));
  return n_seeds > 0 ? (n_seeds + sb - 1) / sb : 1;
}
// at most kMaxRegions regions, as many as spread the merge's blocks evenly
// (each region then serves ceil(blocks / regions) of them with little
// rounding: the merge reserves nearly all rows)
inline int region_count(int64_t n_seeds, int max_cands) {
  const int64_t g = merge_blocks(n_seeds, max_cands);
  const int64_t per = (g + kMaxRegions - 1) / kMaxRegions;
  return (int)((g + per - 1) / per);
}
// rows per region, a multiple of 256 (the row-kernel block)
inline int64_t region_rows(int64_t n_seeds, int max_cands) {
  const int64_t nr = region_count(n_seeds, max_cands);
  const int64_t per_merge = (merge_blocks(n_seeds, max_cands) + nr - 1) / nr *
                            merge_seeds(merge_lanes(max_cands)) * max_cands;
  const int64_t per_seed = (seed_blocks(n_seeds) + nr - 1) / nr * 256;
  const int64_t r = per_merge > per_seed ? per_merge : per_seed;
  return (r + 255) / 256 * 256;
}

// nullptr when the argument is valid, else why it is not
const char* check_config(const ktf_config* cfg);
const char* check_fit_in(const ktf_fit_in* in, const ktf_fit_out* out);
// an event batch for ktf_build (with n_layers and max_cands of the context)
const char* check_event_batch(const ktf_event_batch* ev, int n_layers, int max_cands);
// one host event for ktf_submit
const char* check_event_host(const ktf_event_host* ev, int n_layers);

// device bytes an event holds while in flight: inputs, outputs and its
// share of the lane workspace (candidates, records, bins)
size_t footprint_of(const ktf_config& cfg, int64_t n, int64_t nh, ktf_precision prec);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of a batch's packed inputs (all 256-byte aligned): seed
// offsets [E+1], hit offsets [E*L+1] (int64), hits [3][H], states [6][N],
// covariances [21][N] (values of ts bytes), seed hits [NSL][N] (int32),
// charges [N] (int8).  N and H are at least 1 so that every array has an
// address.
struct InLayout {
  size_t soff, hoff, hits, state, cov, sh, q, total;
};
InLayout in_layout(int E, int L, int NSL, int64_t N, int64_t H, size_t ts);

// Byte offsets of a batch's outputs: the part the host reads (hit indices
// [L][N], the final fit's state [6][N], cov [21][N], chi2, count, status)
// comes first and ends at `host`; the building's own fit outputs follow.
struct OutLayout {
  size_t hit, f_state, f_cov, f_chi2, f_nu, f_st, host;
  size_t b_state, b_cov, b_chi2, b_nh, b_st, total;
};
OutLayout out_layout(int L, int64_t N, size_t ts);

// A copy of n elements of `size` bytes.
struct RowCopy {
  const void* src;
  void* dst;
  int64_t n;
  int size;
};
// Runs the copies; above 4 MB in total they are cut into pieces of at most
// 256K elements and spread over four host threads.
void run_copies(const std::vector<RowCopy>& rows);

// One event's host arrays in its precision (ts bytes per value).
struct EventRows {
  int64_t n_seeds, n_hits;
  const int64_t* hit_off;  // [L+1], from 0
  const void* hits;        // [3][n_hits]
  const void* state;       // [6][n_seeds]
  const void* cov;         // [21][n_seeds]
  const int8_t* q;         // [n_seeds]
  const int32_t* seed_hit; // [NSL][n_seeds]
};
// One event's result arrays (sized for its n_seeds), in its precision.
struct ResultRows {
  int32_t* hit;     // [L][n]
  void* state;      // [6][n]
  void* cov;        // [21][n]
  double* chi2;     // [n]
  int32_t* n_hits;  // [n]
  uint32_t* status; // [n]
};

// Seed offsets [E+1] and hit offsets [E*L+1] of the events packed in order.
void batch_offsets(const std::vector<EventRows>& ev, int L, std::vector<int64_t>& seed_off,
                   std::vector<int64_t>& hit_off);
// The copies that fill staging (laid out by `in` for N = seed_off[E] and
// H = hit_off[E*L], each at least 1) with the offsets and every event's rows.
void pack_rows(const std::vector<EventRows>& ev, int L, int NSL, size_t ts, const std::vector<int64_t>& seed_off,
               const std::vector<int64_t>& hit_off, char* staging, const InLayout& in, std::vector<RowCopy>& out);
// The copies from a batch's host outputs (laid out by `ol` for N, at least
// 1) into each event's result arrays, events in batch order.
void unpack_rows(const std::vector<int64_t>& n_seeds, const std::vector<ResultRows>& res, int L, size_t ts,
                 int64_t N, const char* staging, const OutLayout& ol, std::vector<RowCopy>& out);

}  // namespace ktf
