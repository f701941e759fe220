// build.hip -- combinatorial track building with the clone engine (gfx950).
//
// Building (Sec. 3) extends every seed layer by layer.  The hits of each
// (event, layer) are first placed in z x phi bins so that a candidate only
// scores the hits near its prediction (the paper's fix for the "nHits"
// problem: hits sorted in phi per bin and layer with phi bins as a fast
// look-up).  Then, per layer, the clone engine (Sec. 3.1):
//   score   one lane per live candidate: propagate to the layer, scan the
//           bins inside a window that no compatible hit can lie outside of,
//           keep the candidate's best records (a bookkeeping list) -- no
//           candidate is copied here;
//   merge   a lane group per seed: merge the candidates' sorted record
//           lists to the best max_cands by the ranking (more hits, lower chi2, lower
//           parent rank, lower hit index, a missed layer last);
//   clone   applying each kept record's update to its parent's propagated
//           state (the child) is folded into the next layer's score, which
//           needs the child anyway; of the last layer's children only the
//           one the final choice takes is made;
//   final   one lane per seed: the best survivor or ended candidate, hit
//           indices recovered by walking the per-layer (parent, hit) records.
//
// Layout: candidates live in dense rows (one structure-of-arrays row per
// field), split into 64 regions with a row counter each; a seed's candidates
// are contiguous and in rank order.  Positions are kept in double, momentum
// and covariance in the storage precision.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "ctx.hpp"
#include "host_logic.hpp"
#include "kf_math.hpp"

namespace ktf {

constexpr double kPi = 3.14159265358979323846;

// Candidate rows are split into NR <= kMaxRegions regions of RS rows, each
// with its own row counter (kCtrStride ints apart, one 128-byte line each),
// so that row reservations spread over many addresses: same-address
// atomics serialise in the memory system.
constexpr int kCtrStride = 32;

template <typename T> struct BuildNewton;
template <> struct BuildNewton<double> { static constexpr int n = 3; };
template <> struct BuildNewton<float> { static constexpr int n = 2; };

struct BuildArgs {
  BuildGeom g;
  int32_t n_events;
  int32_t n_groups;        // n_events * n_layers
  int32_t bin_l0;          // first layer binned (the seed layers' bins are not searched by a build)
  int32_t off16;           // the bin offsets are 16-bit (a build whose groups all fit one binning block)
  int32_t n_bins;          // n_zbins * n_phibins
  int64_t n_seeds, sp;     // seeds, seed pitch
  int64_t S;               // candidate rows = NR * RS
  int64_t RS;              // rows per region
  int NR;                  // regions in use
  int64_t n_hits;          // total hits
  int64_t max_group;       // most hits in one (event, layer)
  int64_t hp;              // hit pitch
  const int64_t* seed_off; // device [n_events+1]
  const int64_t* hit_off;  // device [n_groups+1]
  const void* hits;        // [3][hp]
  const void* seed_state;  // [6][sp]
  const void* seed_cov;    // [21][sp]
  const int8_t* q;         // [sp]
  const int32_t* seed_hit; // [nsl][sp]
  // seed order: building works on the seeds of each event sorted by their
  // predicted phi bin at the first building layer (neighbouring rows then
  // search neighbouring hit bins); the seed arrays above are copies in that
  // order, the caller's are src_*, and the outputs go back through order
  const void* src_state;   // [6][sp] as the caller gave them
  const void* src_cov;     // [21][sp]
  const int8_t* src_q;     // [sp]
  const int32_t* src_seed_hit; // [nsl][sp]
  int32_t* skey;           // [sp]: sort key of each (caller's) seed
  int32_t* order;          // [sp]: the caller's index of the seed at each sorted place
  int32_t* rank;           // [sp]: the sorted place of each caller's seed
  int32_t n_keys;          // values of the sort key
  int32_t seed_order;      // 1: seeds sorted and window boxes staged in LDS, 0: the caller's order
  int32_t* u_hit;          // caller's outputs: [L][sp]
  void* u_state;           // [6][sp]
  void* u_cov;             // [21][sp]
  double* u_chi2;
  int32_t* u_nhits;
  uint32_t* u_status;
  int32_t* u_hist;         // optional [L][max_cands][2][sp]
  int32_t* u_count;        // optional [L][sp]
  // binning
  int32_t* bin_off;        // [n_groups][n_bins+1]
  int32_t* bin_cur;        // [n_groups][n_bins]
  int32_t* hit_bin;        // [n_hits]
  int32_t* perm;           // [n_hits]: local index of the hit at each binned position (binning alone; null when building: the records hold it)
  int32_t* perm_raw;       // [n_hits]: the same before ordering within bins
  int32_t* sev;            // [sp]: event of each seed
  int32_t* cinfo[2];       // [S]: event << 1 | (charge > 0) of each dense candidate row
  int32_t* cstart[2];      // [sp]: first dense row of each seed's candidates
  int32_t* sel_parent;     // [S]: per child row, its parent's row
  int32_t* sel_hit;        // [S]: per child row, the hit it takes as its position among the binned records (-1: missed layer)
  double* sel_chi2;        // [S]: per child row, its chi2 total
  unsigned* ccount;        // [n_layers][kMaxRegions][kCtrStride]: rows used per region after each layer
  void* hb;                // [n_hits] BinHit<TS>: binned coordinates and local index
  // candidates (double buffered), propagated parents, records
  double* cpos[2];
  void* cmom[2];
  void* ccov[2];
  double* cchi2[2];
  uint32_t* cmeta[2];      // nh | nm << 8 | status << 16
  double* ppos[2];         // propagated candidates, by layer parity
  void* pmom[2];
  void* pcov[2];
  double* rchi;            // [max_cands][S]
  int32_t* rhit;           // [max_cands][S]: the hit's index within its (event, layer)
  int32_t* rpos;           // [max_cands][S]: the hit's position among the binned records
  int32_t* rcount;         // [S]: records, -1 ended (no reach), -2 ended (missed too often)
  int32_t* hist;           // [L][max_cands][2][sp]: (parent rank, hit index)
  int32_t* count;          // [L][sp]
  // best ended candidate per seed
  double* bpos;
  void* bmom;
  void* bcov;
  double* bchi2;
  uint32_t* bmeta;
  int32_t* bend;           // end layer, -1 = none
  int32_t* brank;
  // outputs
  int32_t* o_hit;          // [L][sp]
  void* o_state;
  void* o_cov;
  double* o_chi2;
  int32_t* o_nhits;
  uint32_t* o_status;
};

__device__ __forceinline__ int find_event(const int64_t* off, int n, int64_t j) {
  int lo = 0, hi = n;  // off[lo] <= j < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid; else hi = mid;
  }
  return lo;
}

// a candidate row's event and charge, so that scoring reads neither the
// seed's event nor its charge through the seed index
__device__ __forceinline__ int32_t pack_info(int e, int8_t q) { return (e << 1) | (q > 0 ? 1 : 0); }
__device__ __forceinline__ int info_event(int32_t i) { return i >> 1; }
__device__ __forceinline__ double info_charge(int32_t i) { return (i & 1) ? 1.0 : -1.0; }

__device__ __forceinline__ uint32_t pack_meta(int nh, int nm, uint32_t st) {
  return (uint32_t)nh | ((uint32_t)nm << 8) | (st << 16);
}
__device__ __forceinline__ int meta_nh(uint32_t m) { return (int)(m & 0xffu); }
__device__ __forceinline__ int meta_nm(uint32_t m) { return (int)((m >> 8) & 0xffu); }
__device__ __forceinline__ uint32_t meta_st(uint32_t m) { return m >> 16; }

// bin of a hit: zbin = floor((z + zh) nz / (2 zh)) clamped, phibin =
// floor((atan2(y, x) + pi) nphi / (2 pi)) mod nphi; same arithmetic order in
// double as the definition, no contraction.
// A binned hit as the window scan reads it: its coordinates and its index
// within the group in one record (one 16-byte load in float, two in
// double), so a window's run of hits is one run of records.
template <typename TS> struct BinHit;
template <> struct __align__(16) BinHit<float> {
  float x, y, z;
  int32_t id;
};
template <> struct __align__(16) BinHit<double> {
  double x, y, z;
  int32_t id, pad;
};

// The phi bin in double, for the rare hits near a bin edge, and the eta
// row: out of line, so that callers keep only the registers of the common
// path (a z row from a float phi estimate).
__device__ __attribute__((noinline)) int phi_bin_near_edge(double x, double y, int nphi) {
#pragma clang fp contract(off)
  const double phi = atan2(y, x);
  const double pf = floor((phi + kPi) * nphi / (2.0 * kPi));
  return pf == pf ? (int)pf : 0;  // a coordinate that is not a number: bin 0
}
__device__ __attribute__((noinline)) double z_row_near_edge(double z, double zh, int nz) {
#pragma clang fp contract(off)
  return floor((z + zh) * nz / (2.0 * zh));
}
__device__ __attribute__((noinline)) double eta_row_of(double x, double y, double z, double eta_max, int nz) {
#pragma clang fp contract(off)
  const double eta = asinh(z / sqrt(x * x + y * y));
  return floor((eta + eta_max) * nz / (2.0 * eta_max));
}

// bin of a hit: its row is the z bin, zbin = floor((z + zh) nz / (2 zh))
// clamped, or (eta rows) the eta bin, floor((asinh(z / rho) + eta_max) nz /
// (2 eta_max)) clamped; the phi bin as below

__device__ __forceinline__ int hit_bin_of(double x, double y, double z, const BuildGeom& g) {
#pragma clang fp contract(off)
  const double zh = g.z_half;
  const int nz = g.n_zbins, nphi = g.n_phibins;
  double zf;
  if (g.eta_rows) {
    zf = eta_row_of(x, y, z, g.eta_max, nz);
  } else {
    // the z row from a float estimate u of its position in rows, unless
    // that lies within m = 2e-6 (nz + |u|) of a row edge: rounding the
    // coordinate, the sum, the scale and the product to float moves u by
    // at most 2^-24 (1.5 nz + 3 |u|) for a position inside the table, well
    // below m, so away from an edge it floors to the row of the double
    // form, which decides the rest (a position beyond the table clamps to
    // the same end row either way; not a number goes to the double form)
    const float uz = ((float)z + (float)zh) * ((float)nz / (float)(2.0 * zh));
    const float flz = floorf(uz), frz = uz - flz, mz = 2e-6f * ((float)nz + fabsf(uz));
    if (frz > mz && frz < 1.0f - mz) {
      zf = (double)flz;
    } else {
      zf = z_row_near_edge(z, zh, nz);
    }
  }
  // (not a number: the first row, as a number below the range)
  const int zb = zf >= 0.0 ? (zf > nz - 1 ? nz - 1 : (int)zf) : 0;
  // the phi bin from a float estimate of its position, unless that lies
  // within 1e-5 rad of a bin edge: the float angle's error (coordinates
  // rounded to float, atan2f, the sum and the scale) is below 2e-6 rad, so
  // away from an edge it floors to the same bin as the double form, which
  // decides the rest
  const float uf = (atan2f((float)y, (float)x) + (float)kPi) * ((float)nphi / (float)(2.0 * kPi));
  const float mf = 1e-5f * ((float)nphi / (float)(2.0 * kPi));
  const float fl = floorf(uf);
  const float fr = uf - fl;
  int pb;
  if (fr > mf && fr < 1.0f - mf) {
    pb = (int)fl;
  } else {
    pb = phi_bin_near_edge(x, y, nphi);
  }
  pb = ((pb % nphi) + nphi) % nphi;
  return zb * nphi + pb;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename TS>
__global__ void bin_count_kernel(BuildArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_hits) return;
  const int g = find_event(a.hit_off, a.n_groups, j);
  if (g % a.g.n_layers < a.bin_l0) return;
  const TS* h = static_cast<const TS*>(a.hits);
  const int b = hit_bin_of((double)h[j], (double)h[a.hp + j], (double)h[2 * a.hp + j], a.g);
  a.hit_bin[j] = b;
  atomicAdd(&a.bin_cur[(int64_t)g * a.n_bins + b], 1);
}

// one block per (event, layer): exclusive scan of the bin counts into the CSR
// offsets, and the cursor reset to each bin's start.  The block walks the
// bins in coalesced chunks of 1024; each chunk is scanned with wave
// shuffles, the wave totals through LDS, and a running carry.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void bin_scan_kernel(BuildArgs a) {
  __shared__ int32_t wsum[kScanThreads / 64];
  const int g = blockIdx.x;
  if (g % a.g.n_layers < a.bin_l0) return;  // the whole block
  const int nb = a.n_bins;
  int32_t* cnt = a.bin_cur + (int64_t)g * nb;
  int32_t* off = a.bin_off + (int64_t)g * (nb + 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int nw = kScanThreads / 64;
  int32_t carry = 0;
  for (int base = 0; base < nb; base += kScanThreads) {
    const int b = base + threadIdx.x;
    const int32_t v = b < nb ? cnt[b] : 0;
    int32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
      int32_t t = lane < nw ? wsum[lane] : 0;
#pragma unroll
      for (int d = 1; d < nw; d <<= 1) {
        const int32_t y = __shfl_up(t, d, 64);
        if (lane >= d) t += y;
      }
      if (lane < nw) wsum[lane] = t;
    }
    __syncthreads();
    const int32_t excl = carry + (wave > 0 ? wsum[wave - 1] : 0) + x - v;
    if (b < nb) {
      off[b] = excl;
      cnt[b] = excl;
    }
    carry += wsum[nw - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[nb] = carry;
}

__global__ void bin_scatter_kernel(BuildArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_hits) return;
  const int g = find_event(a.hit_off, a.n_groups, j);
  if (g % a.g.n_layers < a.bin_l0) return;
  const int b = a.hit_bin[j];
  const int32_t pos = atomicAdd(&a.bin_cur[(int64_t)g * a.n_bins + b], 1);
  a.perm_raw[a.hit_off[g] + pos] = (int32_t)(j - a.hit_off[g]);
}

// one lane per hit: its place within its bin is the number of the bin's
// hits with a smaller original index (the scatter's atomics left the bin in
// arrival order), which orders every bin by original index; the hit's
// coordinates are copied to that binned position
template <typename TS>
__global__ void bin_rank_kernel(BuildArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_hits) return;
  const int g = find_event(a.hit_off, a.n_groups, j);
  if (g % a.g.n_layers < a.bin_l0) return;
  const int b = a.hit_bin[j];
  const int32_t* off = a.bin_off + (int64_t)g * (a.n_bins + 1);
  const int64_t base = a.hit_off[g];
  const int32_t lo = off[b], hi = off[b + 1];
  const int32_t jl = (int32_t)(j - base);
  int32_t rank = 0;
  for (int32_t k = lo; k < hi; ++k) rank += a.perm_raw[base + k] < jl ? 1 : 0;
  const int64_t dst = base + lo + rank;
  if (a.perm) a.perm[dst] = jl;
  const TS* h = static_cast<const TS*>(a.hits);
  BinHit<TS> r;
  r.x = h[j];
  r.y = h[a.hp + j];
  r.z = h[2 * a.hp + j];
  r.id = jl;
  static_cast<BinHit<TS>*>(a.hb)[dst] = r;
}

constexpr int kBinThreads = 1024;
constexpr int kLdsBins = 32768;

// One block per (event, layer) group of at most kPackMaxHits hits (the
// usual case) with the whole bin table in LDS: count the hits per bin,
// scan the counts into the CSR offsets, scatter the hits through a cursor,
// then order every bin by original index (a hit's place is the number of
// its bin's hits with a smaller index) and copy the coordinates into binned
// order.  Counts, offsets and cursors are 16-bit halves of 32-bit LDS words
// (64 KB for 32,768 bins) and the unordered scatter stays in LDS as 16-bit
// local indices, so ordering each bin by original index reads LDS only.
// Larger groups or bin tables take the multi-kernel path above, whose
// kernels spread every phase over all hits (one block per group would
// leave a batch of few heavy events with few blocks).  Each
// thread takes its hits kBinBatch at a time with their loads issued
// together, so a phase costs one memory round trip per batch.
constexpr int kPackMaxHits = 32768;
constexpr int kBinBatch = 8;
// MB batches of BB x kBinThreads hits: a group of at most MB x BB x 1024
// hits.  The LDS holds the bin table (one word per two bins) and the
// unordered scatter (one 16-bit index per hit), sized by the host for the
// launch's bins and largest group, so that a layer of a few thousand hits
// over 32,768 bins (78 KB) lets two blocks share a CU; batches of four
// keep the registers within the eight waves per SIMD that two blocks need.
template <int BB> struct BinWaves { static constexpr int v = BB == 4 ? 8 : 4; };
// 16-bit offsets: a group's row of n_bins + 1 rounded up to 16 bytes, so
// that the binning block writes it in whole 16-byte stores (within the
// 32-bit row's bytes for n_bins >= 8, which the host requires)
__host__ __device__ inline int64_t off16_pitch(int nb) { return ((int64_t)nb + 8) & ~int64_t(7); }
inline size_t bin_lds_bytes(int n_bins, int64_t max_group) {
  return (size_t)((n_bins + 1) >> 1) * 4 + (size_t)((max_group + 1) & ~int64_t(1)) * 2;
}
template <typename TS, int MB, int BB>
__global__ __launch_bounds__(kBinThreads) __attribute__((amdgpu_waves_per_eu(BinWaves<BB>::v)))
void bin_group16_kernel(BuildArgs a) {
  extern __shared__ __align__(16) uint32_t bin_lds[];
  __shared__ int32_t wsum[kBinThreads / 64];
  const int g = blockIdx.x;
  if (g % a.g.n_layers < a.bin_l0) return;  // the whole block
  const int nb = a.n_bins, nwords = (nb + 1) >> 1;
  uint32_t* cnt = bin_lds;  // bin b in half b & 1 of word b >> 1
  uint16_t* permr = reinterpret_cast<uint16_t*>(bin_lds + nwords);
  const int tid = threadIdx.x;
  const int64_t base = a.hit_off[g];
  const int32_t n = (int32_t)(a.hit_off[g + 1] - base);
  int32_t* off = a.bin_off + (int64_t)g * (nb + 1);
  const TS* h = static_cast<const TS*>(a.hits);
  // cleared in 16-byte words (the table starts 16-byte aligned), then the
  // last few words one by one
  for (int q = tid; q < (nwords >> 2); q += kBinThreads) reinterpret_cast<uint4*>(cnt)[q] = make_uint4(0u, 0u, 0u, 0u);
  if (tid < (nwords & 3)) cnt[(nwords & ~3) + tid] = 0;
  __syncthreads();
  // count; each hit's bin (below 32,768) stays in a 16-bit half of a
  // register for the scatter and the ordering, whose place then replaces it
  uint32_t bk[MB][BB / 2];
#pragma unroll
  for (int bi = 0; bi < MB; ++bi) {
    const int32_t j0 = bi * BB * kBinThreads;
#pragma unroll
    for (int u = 0; u < BB / 2; ++u) bk[bi][u] = 0;
    if (j0 >= n) continue;
    TS x[BB], y[BB], z[BB];
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t j = j0 + u * kBinThreads + tid;
      x[u] = y[u] = z[u] = TS(0);
      if (j < n) {
        x[u] = h[base + j];
        y[u] = h[a.hp + base + j];
        z[u] = h[2 * a.hp + base + j];
      }
    }
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t j = j0 + u * kBinThreads + tid;
      if (j < n) {
        const int b = hit_bin_of((double)x[u], (double)y[u], (double)z[u], a.g);
        bk[bi][u >> 1] |= (uint32_t)b << ((u & 1) * 16);
        atomicAdd(&cnt[b >> 1], 1u << ((b & 1) * 16));
      }
    }
  }
  __syncthreads();
  // exclusive scan: each thread a contiguous run of words, then the block.
  // A thread walks its run from a lane-dependent start, wrapping round, so
  // that the lanes of a wave (runs 16 words apart) touch distinct LDS banks
  // at each step, where a common start would put 16 of them on one bank;
  // the sum from that start to the run's end gives the prefix at the start,
  // and the prefix restarts at the run's first word
  const int per = (nwords + kBinThreads - 1) / kBinThreads;
  const int w0 = min(nwords, tid * per), len = min(nwords, w0 + per) - w0;
  const int rot = per > 0 ? ((((tid >> 1) & 15) ^ ((tid >> 5) & 1)) % per) : 0;
  // a run of the usual 16 words (32,768 bins over 1,024 threads) is read
  // once into registers, its loads issued together; any other run length
  // takes the loops below
  constexpr int kRun = 16;
  const bool full = per == kRun && len == kRun;
  uint32_t rv[kRun];
  int32_t sum = 0, upper = 0;
  if (full) {
#pragma unroll
    for (int k = 0; k < kRun; ++k) rv[k] = cnt[w0 + ((k + rot) & (kRun - 1))];
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      const int32_t c = (int32_t)((rv[k] & 0xffffu) + (rv[k] >> 16));
      sum += c;
      upper += k < kRun - rot ? c : 0;  // words from the start to the run's end
    }
  } else {
    for (int k = 0; k < per; ++k) {
      const int m = k + rot < per ? k + rot : k + rot - per;
      if (m < len) {
        const uint32_t v = cnt[w0 + m];
        const int32_t c = (int32_t)((v & 0xffffu) + (v >> 16));
        sum += c;
        upper += m >= rot ? c : 0;
      }
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
  int32_t x = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int32_t first = x - sum;
  for (int w = 0; w < wave; ++w) first += wsum[w];
  int32_t run = first + (sum - upper);
  if (full) {
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      if (k == ((kRun - rot) & (kRun - 1))) run = first;  // the run's first word
      const uint32_t lo = rv[k] & 0xffffu;
      cnt[w0 + ((k + rot) & (kRun - 1))] = (uint32_t)run | ((uint32_t)(run + (int32_t)lo) << 16);
      run += (int32_t)(lo + (rv[k] >> 16));
    }
  } else {
    for (int k = 0; k < per; ++k) {
      const int m = k + rot < per ? k + rot : k + rot - per;
      if (m == 0) run = first;
      if (m < len) {
        const uint32_t v = cnt[w0 + m];
        const uint32_t lo = v & 0xffffu;
        cnt[w0 + m] = (uint32_t)run | ((uint32_t)(run + (int32_t)lo) << 16);
        run += (int32_t)(lo + (v >> 16));
      }
    }
  }
  __syncthreads();
  if (a.off16) {
    // the offsets (at most 32,768) in half the bytes, for the build's own
    // use: a word of the table is the two 16-bit offsets of its bins in
    // order, so the row is the table itself, then n (in the high half of
    // the last word already, for an odd bin count) and padding
    const int64_t pitch = off16_pitch(nb);
    uint4* row = reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(a.bin_off) + (int64_t)g * pitch);
    const uint32_t tail = (uint32_t)n * 0x10001u;
    for (int q = tid; q < (int)(pitch >> 3); q += kBinThreads) {
      const int w = 4 * q;
      uint4 v;
      if (w + 3 < nwords) {  // one 16-byte LDS read: consecutive lanes, no bank shared
        v = *reinterpret_cast<const uint4*>(cnt + w);
      } else {
        v.x = w < nwords ? cnt[w] : tail;
        v.y = w + 1 < nwords ? cnt[w + 1] : tail;
        v.z = w + 2 < nwords ? cnt[w + 2] : tail;
        v.w = w + 3 < nwords ? cnt[w + 3] : tail;
      }
      row[q] = v;
    }
  } else {
    for (int b = tid; b < nb; b += kBinThreads) off[b] = (int32_t)((cnt[b >> 1] >> ((b & 1) * 16)) & 0xffffu);
    if (tid == 0) off[nb] = n;
  }
  __syncthreads();
  // scatter through the cursors (a bin's cursor ends at the next offset)
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t j = bi * BB * kBinThreads + u * kBinThreads + tid;
      if (j < n) {
        const int b = (int)((bk[bi][u >> 1] >> ((u & 1) * 16)) & 0xffffu);
        const int sh = (b & 1) * 16;
        const uint32_t pos = (atomicAdd(&cnt[b >> 1], 1u << sh) >> sh) & 0xffffu;
        permr[pos] = (uint16_t)j;
      }
    }
  __syncthreads();
  // order every bin by original index: a hit's place is the number of its
  // bin's hits with a smaller index; the places stay in registers until all
  // are taken, then the permutation goes to LDS and out in coalesced rows
  // (scattered 4-byte stores would each cost HBM a line)
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t j = bi * BB * kBinThreads + u * kBinThreads + tid;
      if (j < n) {
        const int sh = (u & 1) * 16;
        const int b = (int)((bk[bi][u >> 1] >> sh) & 0xffffu);
        const int32_t hi = (int32_t)((cnt[b >> 1] >> ((b & 1) * 16)) & 0xffffu);
        const int32_t lo = b > 0 ? (int32_t)((cnt[(b - 1) >> 1] >> (((b - 1) & 1) * 16)) & 0xffffu) : 0;
        int32_t rank = 0;
        for (int32_t k = lo; k < hi; ++k) rank += permr[k] < j ? 1 : 0;
        bk[bi][u >> 1] = (bk[bi][u >> 1] & (0xffff0000u >> sh)) | ((uint32_t)(lo + rank) << sh);
      }
    }
  __syncthreads();  // every place is taken; the unordered scatter is done with
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t j = bi * BB * kBinThreads + u * kBinThreads + tid;
      if (j < n) permr[(bk[bi][u >> 1] >> ((u & 1) * 16)) & 0xffffu] = (uint16_t)j;
    }
  __syncthreads();
  BinHit<TS>* o = static_cast<BinHit<TS>*>(a.hb);
  for (int32_t i0 = 0; i0 < n; i0 += BB * kBinThreads) {
    int32_t jj[BB];
    TS x[BB], y[BB], z[BB];
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t i = i0 + u * kBinThreads + tid;
      jj[u] = i < n ? (int32_t)permr[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t i = i0 + u * kBinThreads + tid;
      x[u] = y[u] = z[u] = TS(0);
      if (i < n) {
        x[u] = h[base + jj[u]];
        y[u] = h[a.hp + base + jj[u]];
        z[u] = h[2 * a.hp + base + jj[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int32_t i = i0 + u * kBinThreads + tid;
      if (i < n) {
        const int64_t d = base + i;
        if (a.perm) a.perm[d] = jj[u];
        BinHit<TS> r;
        r.x = x[u];
        r.y = y[u];
        r.z = z[u];
        r.id = jj[u];
        o[d] = r;
      }
    }
  }
}

// ------------------------------------------------------------ seed order
// Workgroups are dealt to the chip's eight XCDs in turn, each XCD with its
// own L2.  A kernel whose neighbouring blocks share data (one event's seed
// rows) maps block b to a logical block so that every XCD takes one
// contiguous eighth of the logical blocks; the grid is rounded up to a
// multiple of eight and the logical blocks beyond nb do nothing.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t nb) {
  const int64_t per = (nb + kXcds - 1) / kXcds;
  return (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}
static inline unsigned xcd_grid(int64_t nb) { return (unsigned)((nb + kXcds - 1) / kXcds * kXcds); }

// Sort key of every seed (the caller's order): where the seed's helix
// meets the first building layer (or the seed itself, if it does not reach
// it), as a cell of 256 (phi) x 32 (z) over the layer, the cells numbered
// along a Z-order (Morton) curve so that seeds close in the order are close
// in both phi and z.
template <typename TS, typename TP>
__global__ void seed_key_kernel(BuildArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  const TS* st = static_cast<const TS*>(a.src_state);
  TrackState<TP> x, xo;
#pragma unroll
  for (int c = 0; c < 3; ++c) x.pos[c] = (double)st[c * a.sp + s];
#pragma unroll
  for (int c = 0; c < 3; ++c) x.mom[c] = (TP)st[(c + 3) * a.sp + s];
  const TP k = (TP)(kCLight * (a.src_q[s] > 0 ? 1.0 : -1.0) * a.g.bz);
  Jac<TP> F;
  const int lb = a.g.n_seed_layers < a.g.n_layers ? a.g.n_seed_layers : a.g.n_layers - 1;
  double px = x.pos[0], py = x.pos[1], pz = x.pos[2];
  if (propagate<TP, BuildNewton<TP>::n>(x, k, a.g.radii[lb], false, xo, F)) {
    px = xo.pos[0];
    py = xo.pos[1];
    pz = xo.pos[2];
  }
  // clamped before the conversion (a position that is not a number: cell 0)
  const int cp = (int)fminf(255.0f, fmaxf(0.0f, (atan2f((float)py, (float)px) + (float)kPi) *
                                                     (float)(256.0 / (2.0 * kPi))));
  const int cz = (int)fmin(31.0, fmax(0.0, floor((pz + a.g.z_half) * (32.0 / (2.0 * a.g.z_half)))));
  int key = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) key |= (((cz >> b) & 1) << (2 * b)) | (((cp >> b) & 1) << (2 * b + 1));
  key |= (cp >> 5) << 10;
  a.skey[s] = key;
}

// One block per event: its seeds' sorted places by a counting sort on the
// key (the order within a key is whatever the atomics give: rows may land
// anywhere, a seed's result does not depend on its row).
constexpr int kOrderThreads = 1024;
constexpr int kMaxKeys = 8192;
__global__ __launch_bounds__(kOrderThreads) void seed_order_kernel(BuildArgs a) {
  __shared__ int32_t cnt[kMaxKeys];
  __shared__ int32_t wsum[kOrderThreads / 64];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int64_t lo = a.seed_off[e], hi = a.seed_off[e + 1];
  const int nk = a.n_keys;
  for (int b = tid; b < nk; b += kOrderThreads) cnt[b] = 0;
  __syncthreads();
  for (int64_t i = lo + tid; i < hi; i += kOrderThreads) atomicAdd(&cnt[a.skey[i]], 1);
  __syncthreads();
  // exclusive scan: each thread a contiguous run of keys, then the block
  const int per = (nk + kOrderThreads - 1) / kOrderThreads;
  const int b0 = min(nk, tid * per), b1 = min(nk, b0 + per);
  int32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += cnt[b];
  const int lane = tid & 63, wave = tid >> 6;
  int32_t x = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int32_t run = x - sum;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  for (int b = b0; b < b1; ++b) {
    const int32_t v = cnt[b];
    cnt[b] = run;
    run += v;
  }
  __syncthreads();
  for (int64_t i = lo + tid; i < hi; i += kOrderThreads) {
    const int32_t pos = atomicAdd(&cnt[a.skey[i]], 1);
    a.order[lo + pos] = (int32_t)i;
    a.rank[i] = (int32_t)(lo + pos);
  }
}

// the seed inputs in sorted order (reads within each event's rows, which
// stay in one XCD's L2)
template <typename TS>
__global__ void seed_gather_kernel(BuildArgs a) {
  const int64_t i = xcd_block((a.n_seeds + blockDim.x - 1) / blockDim.x) * blockDim.x + threadIdx.x;
  if (i >= a.n_seeds) return;
  const int64_t s = a.order[i];
  const TS* st = static_cast<const TS*>(a.src_state);
  const TS* cv = static_cast<const TS*>(a.src_cov);
  TS* dst = static_cast<TS*>(const_cast<void*>(a.seed_state));
  TS* dcv = static_cast<TS*>(const_cast<void*>(a.seed_cov));
#pragma unroll
  for (int c = 0; c < 6; ++c) dst[c * a.sp + i] = st[c * a.sp + s];
#pragma unroll
  for (int c = 0; c < 21; ++c) dcv[c * a.sp + i] = cv[c * a.sp + s];
  const_cast<int8_t*>(a.q)[i] = a.src_q[s];
  for (int l = 0; l < a.g.n_seed_layers; ++l)
    const_cast<int32_t*>(a.seed_hit)[l * a.sp + i] = a.src_seed_hit[l * a.sp + s];
}

// the outputs back to the caller's order: one lane per caller seed, so the
// writes are coalesced and the reads stay within the event's sorted rows
template <typename TS>
__global__ void seed_scatter_kernel(BuildArgs a) {
  const int64_t s = xcd_block((a.n_seeds + blockDim.x - 1) / blockDim.x) * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  const int64_t i = a.rank[s], sp = a.sp;
  const int L = a.g.n_layers, NC = a.g.max_cands;
  for (int l = 0; l < L; ++l) a.u_hit[l * sp + s] = a.o_hit[l * sp + i];
  const TS* st = static_cast<const TS*>(a.o_state);
  const TS* cv = static_cast<const TS*>(a.o_cov);
  TS* ust = static_cast<TS*>(a.u_state);
  TS* ucv = static_cast<TS*>(a.u_cov);
#pragma unroll
  for (int c = 0; c < 6; ++c) ust[c * sp + s] = st[c * sp + i];
#pragma unroll
  for (int c = 0; c < 21; ++c) ucv[c * sp + s] = cv[c * sp + i];
  a.u_chi2[s] = a.o_chi2[i];
  a.u_nhits[s] = a.o_nhits[i];
  a.u_status[s] = a.o_status[i];
  if (a.u_count)
    for (int l = 0; l < L; ++l) a.u_count[l * sp + s] = a.count[l * sp + i];
  if (a.u_hist)
    for (int64_t r = 0; r < (int64_t)L * NC * 2; ++r) a.u_hist[r * sp + s] = a.hist[r * sp + i];
}

// event of every seed, once per build
// each seed's event; and the per-region row counters cleared for the
// layers to come (the seed kernel, next, counts its rows there)
__global__ void seed_event_kernel(BuildArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < a.n_seeds) a.sev[s] = find_event(a.seed_off, a.n_events, s);
  const int64_t nctr = (int64_t)a.g.n_layers * kMaxRegions * kCtrStride;
  for (int64_t i = s; i < nctr; i += (int64_t)gridDim.x * blockDim.x) a.ccount[i] = 0u;
}

// ------------------------------------------------------------- candidates
template <typename TS, typename TP>
__device__ __forceinline__ void load_cand(const double* pos, const void* mom, const void* cov,
                                          int64_t S, int64_t slot, TrackState<TP>& x, TP P[21]) {
  const TS* m = static_cast<const TS*>(mom);
  const TS* c = static_cast<const TS*>(cov);
#pragma unroll
  for (int k = 0; k < 3; ++k) x.pos[k] = pos[k * S + slot];
#pragma unroll
  for (int k = 0; k < 3; ++k) x.mom[k] = (TP)m[k * S + slot];
#pragma unroll
  for (int k = 0; k < 21; ++k) P[k] = (TP)c[k * S + slot];
}

template <typename TS, typename TP>
__device__ __forceinline__ void store_cand(double* pos, void* mom, void* cov, int64_t S, int64_t slot,
                                           const TrackState<TP>& x, const TP P[21]) {
  TS* m = static_cast<TS*>(mom);
  TS* c = static_cast<TS*>(cov);
#pragma unroll
  for (int k = 0; k < 3; ++k) pos[k * S + slot] = x.pos[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k * S + slot] = (TS)x.mom[k];
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k * S + slot] = (TS)P[k];
}

// A store that nothing reads back within the launch or the next one (the
// propagated state, read a layer later) carries the non-temporal hint, so
// that it does not evict the hit bins and offsets that a launch's
// candidates search over and over from L2.  Data that the next kernel
// reads right away (the merge's child rows, the score kernel's record
// lists) goes through the caches with plain accesses.
template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

template <typename TS, typename TP>
__device__ __forceinline__ void store_cand_nt(double* pos, void* mom, void* cov, int64_t S,
                                              int64_t slot, const TrackState<TP>& x, const TP P[21]) {
  TS* m = static_cast<TS*>(mom);
  TS* c = static_cast<TS*>(cov);
#pragma unroll
  for (int k = 0; k < 3; ++k) st_nt(pos + k * S + slot, x.pos[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) st_nt(m + k * S + slot, (TS)x.mom[k]);
#pragma unroll
  for (int k = 0; k < 21; ++k) st_nt(c + k * S + slot, (TS)P[k]);
}

__device__ __forceinline__ HitRes hit_res(const BuildArgs& a) {
  return HitRes{a.g.hr.sr2, a.g.hr.srphi2, a.g.hr.sz2};
}

// Candidates are stored densely per layer: the live candidates of a layer
// occupy rows 0 .. n-1 of the current buffer, each seed's candidates are
// contiguous (cstart[s] .. cstart[s] + count - 1, in rank order), and every
// per-candidate field is its own row.  So neighbouring lanes always touch
// neighbouring rows, whatever the rank.  Rows are reserved with one atomic
// per block (a block prefix sum of the threads' counts; same-address atomics
// serialise in L2, so a batch of many seeds wants as few of them as
// possible).  The placement of a seed's range depends on scheduling; the
// per-seed arithmetic and results do not.  Every thread of the block calls
// this; wtot is LDS scratch of (blockDim / 64 + 1) ints.  Returns the
// thread's first row.
__device__ __forceinline__ int64_t block_reserve(unsigned* counter, int n, int* wtot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = n;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wtot[wave] = x;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < nw; ++w) {
    const int t = wtot[w];
    before += w < wave ? t : 0;
    total += t;
  }
  if (threadIdx.x == 0) wtot[nw] = total > 0 ? (int)atomicAdd(counter, (unsigned)total) : 0;
  __syncthreads();
  return (int64_t)(unsigned)wtot[nw] + before + (x - n);
}

// Region of this block in a launch that reserves rows (seed fit, merge):
// contiguous ranges of at most ceil(gridDim / NR) blocks share a region, so
// a region holds the candidates of neighbouring seeds (one or two events),
// and blocks in flight together still spread their row reservations over
// several counters.
__device__ __forceinline__ int block_region(const BuildArgs& a) {
  return (int)(((int64_t)blockIdx.x * a.NR) / gridDim.x);
}

__device__ __forceinline__ unsigned* region_ctr(const BuildArgs& a, int l, int r) {
  return a.ccount + ((int64_t)l * kMaxRegions + r) * kCtrStride;
}

// The row kernel (score) runs one lane per live candidate row after
// layer l.  A launch has NR * k blocks: block b takes region b % NR
// and, within it, the kRowChunks chunks b / NR + j k
// (j = 0 .. kRowChunks - 1) of blockDim rows, each while it holds live
// rows.  Consecutive blocks take the same chunk of consecutive regions, so
// the rows in flight together belong to seeds close in index (same events,
// same bins in cache), and a region's empty tail costs kRowChunks times
// fewer blocks.  The chunks are written out rather than looped over: a loop
// around the row body costs the row kernels registers.
constexpr int kRowChunks = 4;
#define ROW_CHUNK(J, CALL)                                                              \
  if (l0_ + (J) * step_ < n_) {                                                         \
    const int64_t c = r_ * rs_ + l0_ + (J) * step_;                                     \
    CALL;                                                                               \
  }
#define ROW_CHUNKS(a, l, CALL)                                                          \
  do {                                                                                  \
    const unsigned nr_ = (unsigned)(a).NR;                                              \
    const int r_ = (int)(blockIdx.x % nr_);                                             \
    const int64_t n_ = *region_ctr(a, l, r_);                                           \
    const int64_t rs_ = (a).RS;                                                         \
    const int64_t step_ = (int64_t)(gridDim.x / nr_) * blockDim.x;                      \
    const int64_t l0_ = (int64_t)(blockIdx.x / nr_) * blockDim.x + threadIdx.x;         \
    static_assert(kRowChunks == 4, "ROW_CHUNKS writes out four chunks");                \
    ROW_CHUNK(0, CALL) ROW_CHUNK(1, CALL) ROW_CHUNK(2, CALL) ROW_CHUNK(3, CALL)         \
  } while (0)

// seed phase: fit each seed over the seed layers with its own hits.  MAT:
// the material of the layer being left goes onto a copy of the state, so
// that a seed that cannot reach the next layer ends with its filtered state.
// Held to two waves per SIMD (the double form with material needs more
// registers than that allows without heavy spills, and runs at one).
template <typename TS, typename TP, bool MAT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MAT && sizeof(TP) == 8 ? 1 : 2)))
void build_seed_kernel(BuildArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = s < a.n_seeds;
  const int L = a.g.n_layers, NSL = a.g.n_seed_layers;
  TrackState<TP> x;
  TP P[21];
  double chi2 = 0.0;
  int nh = 0;
  uint32_t status = 0;
  int reached = 0;
  if (valid) {
    const int e = a.sev[s];
    const TS* st = static_cast<const TS*>(a.seed_state);
    const TS* cv = static_cast<const TS*>(a.seed_cov);
#pragma unroll
    for (int c = 0; c < 3; ++c) x.pos[c] = (double)st[c * a.sp + s];
#pragma unroll
    for (int c = 0; c < 3; ++c) x.mom[c] = (TP)st[(c + 3) * a.sp + s];
#pragma unroll
    for (int c = 0; c < 21; ++c) P[c] = (TP)cv[c * a.sp + s];
    const TP k = (TP)(kCLight * (a.q[s] > 0 ? 1.0 : -1.0) * a.g.bz);
    const HitRes hr = hit_res(a);
    const TS* hits = static_cast<const TS*>(a.hits);
    // a seed layer's hit is loaded while the layer before is fitted (the
    // indices do not depend on the fit); an index outside the layer's hit
    // list counts as no hit
    auto load_hit = [&](int l, int32_t& h, double m[3]) {
      const int g = e * L + l;
      const int32_t h0 = a.seed_hit[l * a.sp + s];
      const int64_t lo = a.hit_off[g];
      h = (h0 >= 0 && h0 < a.hit_off[g + 1] - lo) ? h0 : -1;
      m[0] = m[1] = m[2] = 0.0;
      if (h >= 0) {
        const int64_t hi = lo + h;
        m[0] = (double)hits[hi];
        m[1] = (double)hits[a.hp + hi];
        m[2] = (double)hits[2 * a.hp + hi];
      }
    };
    int32_t h_next;
    double m_next[3];
    load_hit(0, h_next, m_next);
    for (int l = 0; l < NSL; ++l) {
      const int32_t h = h_next;
      const double m[3] = {m_next[0], m_next[1], m_next[2]};
      if (l + 1 < NSL) load_hit(l + 1, h_next, m_next);
      TrackState<TP> xp;
      Jac<TP> F;
      TP Pp[21];
      if constexpr (MAT) {
        TrackState<TP> xm = x;
        TP Pm[21];
#pragma unroll
        for (int c = 0; c < 21; ++c) Pm[c] = P[c];
        if (l > 0 && a.g.mat.x0[l - 1] > 0.0)
          apply_material(a.g.mat.x0[l - 1], a.g.mat.eloss, a.g.mat.mass, xm, Pm);
        if (!propagate<TP, BuildNewton<TP>::n>(xm, k, a.g.radii[l], l == 0, xp, F)) {
          status |= kNoReach;
          break;
        }
        cov_propagate(Pm, F, Pp);
      } else {
        if (!propagate<TP, BuildNewton<TP>::n>(x, k, a.g.radii[l], l == 0, xp, F)) {
          status |= kNoReach;
          break;
        }
        cov_propagate(P, F, Pp);
      }
      reached = l + 1;
      int32_t used = -1;
      x = xp;
#pragma unroll
      for (int c = 0; c < 21; ++c) P[c] = Pp[c];
      if (h >= 0) {
        Residual R;
        if (residual(x, P, m, hr, R)) {
          apply_update(x, P, R, x, P);  // in place
          chi2 += R.chi2;
          ++nh;
          used = h;
        } else {
          status |= kSNotPD;
        }
      }
      st_nt(a.hist + ((int64_t)l * a.g.max_cands + 0) * 2 * a.sp + 0 * a.sp + s, (int32_t)0);
      st_nt(a.hist + ((int64_t)l * a.g.max_cands + 0) * 2 * a.sp + 1 * a.sp + s, (int32_t)used);
    }
    for (int l = 0; l < NSL; ++l) a.count[(int64_t)l * a.sp + s] = l < reached ? 1 : 0;
    if (reached < NSL) {  // the seed itself ended: it is the best ended candidate
      store_cand<TS, TP>(a.bpos, a.bmom, a.bcov, a.sp, s, x, P);
      a.bchi2[s] = chi2;
      a.bmeta[s] = pack_meta(nh, 0, status);
      a.bend[s] = reached;
      a.brank[s] = 0;
    } else {
      a.bend[s] = -1;
    }
  }
  __shared__ int wtot[256 / 64 + 1];
  const int alive = valid && reached == NSL ? 1 : 0;
  const int reg = block_region(a);
  const int64_t row = reg * a.RS + block_reserve(region_ctr(a, NSL - 1, reg), alive, wtot);
  if (alive) {
    a.cstart[0][s] = (int32_t)row;
    store_cand<TS, TP>(a.cpos[0], a.cmom[0], a.ccov[0], a.S, row, x, P);
    a.cchi2[0][row] = chi2;
    a.cmeta[0][row] = pack_meta(nh, 0, status);
    a.cinfo[0][row] = pack_info(a.sev[s], a.q[s]);
  }
}

// A group's CSR bin offsets, 32- or 16-bit (the same for the whole launch)
struct BinOffsets {
  const int32_t* o32;
  const uint16_t* o16;  // null: 32-bit
  __device__ __forceinline__ int32_t operator[](int i) const { return o16 ? (int32_t)o16[i] : o32[i]; }
};

// ---------------------------------------------------------------- scoring
// A wave's LDS area for staging its window box: 8 reduction words, the
// box's offsets (rows x (bins + 1)), the start of each row's hits and
// their total, then the hits (about 5.4 KB per wave in float, 6.9 KB in
// double).
template <typename TS> struct StageArea {
  static constexpr int offs = 512, rows = 64;
  static constexpr int hits = sizeof(TS) == 4 ? 192 : 96;
  static constexpr size_t bytes = (size_t)(8 + offs + rows + 8) * 4 + (size_t)hits * sizeof(BinHit<TS>);
};

// LDS written by some lanes of a wave and read by others: the wave's LDS
// operations are processed in order, so the compiler must only keep them
// in program order
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}


// A child of layer l (row c of the buffer `to`): its parent's propagated
// state on layer l with the Kalman update of the hit it took (a missed layer
// keeps the propagated state); returns its meta word.
template <typename TS, typename TP>
__device__ __forceinline__ uint32_t make_child(const BuildArgs& a, int l, int from, int64_t c,
                                               TrackState<TP>& x, TP P[21]) {
  const int64_t p = a.sel_parent[c];
  const int32_t h = a.sel_hit[c];
  const uint32_t pm = a.cmeta[from][p];
  load_cand<TS, TP>(a.ppos[l & 1], a.pmom[l & 1], a.pcov[l & 1], a.S, p, x, P);
  int cnh = meta_nh(pm), cnm = meta_nm(pm);
  if (h >= 0) {
    // the hit's binned record: its coordinates in one load
    const BinHit<TS> r = static_cast<const BinHit<TS>*>(a.hb)[h];
    const double m[3] = {(double)r.x, (double)r.y, (double)r.z};
    Residual R;
    residual(x, P, m, hit_res(a), R);  // scored positive definite already
    apply_update(x, P, R, x, P);       // in place
    ++cnh;
  } else {
    ++cnm;
  }
  return pack_meta(cnh, cnm, meta_st(pm));
}

// One lane per live candidate (dense row c of the current buffer).  MAT:
// the layers carry material.  CHILD: the candidates are the children kept
// on layer l - 1, made here from their parents' propagated states (their
// state is stored only if they end here, for the best-ended choice);
// otherwise they are stored (the seeds' fits).
// (The child variants are held to three waves per SIMD: left alone they
// take a few registers over that budget and run at two, which costs more
// than the few registers the cap spills in double.)
template <typename TS, typename TP, bool MAT, bool CHILD, bool STAGE>
__device__ __forceinline__ void score_row(const BuildArgs& a, int l, int cur, int64_t c) {
  const int32_t info = a.cinfo[cur][c];
  const int L = a.g.n_layers, NC = a.g.max_cands;
  const int64_t S = a.S;
  const int e = info_event(info);
  TrackState<TP> x;
  TP P[21];
  uint32_t meta;
  double pchi2;
  if constexpr (CHILD) {
    meta = make_child<TS, TP>(a, l - 1, cur ^ 1, c, x, P);
    pchi2 = a.sel_chi2[c];
    // plain stores: the merge reads these right after, from the caches
    a.cmeta[cur][c] = meta;
    a.cchi2[cur][c] = pchi2;
  } else {
    load_cand<TS, TP>(a.cpos[cur], a.cmom[cur], a.ccov[cur], S, c, x, P);
    meta = a.cmeta[cur][c];
    pchi2 = a.cchi2[cur][c];
  }
  // an ended child keeps its filtered state for the best-ended choice
  auto store_ended = [&]() {
    if constexpr (CHILD) {
      TrackState<TP> xc;
      TP Pc[21];
      make_child<TS, TP>(a, l - 1, cur ^ 1, c, xc, Pc);
      store_cand<TS, TP>(a.cpos[cur], a.cmom[cur], a.ccov[cur], S, c, xc, Pc);
    }
  };
  const TP k = (TP)(kCLight * info_charge(info) * a.g.bz);
  TrackState<TP> xp;
  Jac<TP> F;
  // the material of the layer being left
  if constexpr (MAT) {
    if (a.g.mat.x0[l - 1] > 0.0) apply_material(a.g.mat.x0[l - 1], a.g.mat.eloss, a.g.mat.mass, x, P);
  }
  if (!propagate<TP, BuildNewton<TP>::n>(x, k, a.g.radii[l], false, xp, F)) {
    a.rcount[c] = -1;
    store_ended();
    return;
  }
  TP Pp[21];
  cov_propagate(P, F, Pp);
  store_cand_nt<TS, TP>(a.ppos[l & 1], a.pmom[l & 1], a.pcov[l & 1], S, c, xp, Pp);

  // search window: for any unit vector u, chi2 < cut implies
  // |u.d| < sqrt(cut u^T S u) (Cauchy-Schwarz in the S^-1 metric); with u
  // the tangent and z, and the hit covariance bounded by its largest
  // transverse variance, no compatible hit lies outside (5% margin; hits
  // are taken to lie within 1% of the layer radius)
  const double cut = a.g.chi2_cut;
  const double rho = sqrt(xp.pos[0] * xp.pos[0] + xp.pos[1] * xp.pos[1]);
  const double irho = 1.0 / rho;  // one division for the window's three
  const double tx = -xp.pos[1] * irho, ty = xp.pos[0] * irho;
  const double ptt = tx * tx * (double)Pp[pidx(0, 0)] + 2.0 * tx * ty * (double)Pp[pidx(0, 1)] +
                     ty * ty * (double)Pp[pidx(1, 1)];
  const double vmax = fmax(a.g.hr.sr2, a.g.hr.srphi2);
  const double bt = 1.05 * sqrt(cut * (fmax(ptt, 0.0) + vmax)) + 1e-7;
  const double bzw = 1.05 * sqrt(cut * (fmax((double)Pp[pidx(2, 2)], 0.0) + a.g.hr.sz2)) + 1e-7;
  const int nz = a.g.n_zbins, nphi = a.g.n_phibins;
  const double zh = a.g.z_half;
  const double zp = xp.pos[2];
  int zlo, zhi;
  if (a.g.eta_rows) {
    // the window's z range at hit radii within 1% of the layer's: asinh(z /
    // rho) grows with z and, for z of one sign, with 1 / rho, so its least
    // and greatest values over that box are at its corners; 1e-9 covers the
    // rounding of asinh between this bound and the binning
    const double z0 = zp - bzw, z1 = zp + bzw, ra = 0.99 * rho, rb = 1.01 * rho;
    const double e0 = asinh(z0 / (z0 >= 0.0 ? rb : ra)) - 1e-9;
    const double e1 = asinh(z1 / (z1 >= 0.0 ? ra : rb)) + 1e-9;
    const double em = a.g.eta_max;
    zlo = (int)fmax(-1.0, floor((e0 + em) * a.g.row_scale));
    zhi = (int)fmin((double)nz, floor((e1 + em) * a.g.row_scale));
  } else {
    // (the scale rounded once instead of a division: a few ulp of a row,
    // far inside the window's 5% margin)
    zlo = (int)fmax(-1.0, floor((zp - bzw + zh) * a.g.row_scale));
    zhi = (int)fmin((double)nz, floor((zp + bzw + zh) * a.g.row_scale));
  }
  zlo = max(0, min(nz - 1, zlo));
  zhi = max(0, min(nz - 1, zhi));
  const double sphi = bt * irho * (1.0 / 0.99);
  int plo = 0, phi_hi = nphi - 1;
  bool full_phi = true;
  if (sphi < 0.5) {
    // asin(x) <= 1.1 x for x <= 0.5; the window centre in float (an error
    // of a few 1e-7 rad, covered by the 1e-5 added)
    const double dphi = 1.1 * sphi + 1e-5;
    const double php = (double)atan2f((float)xp.pos[1], (float)xp.pos[0]);
    plo = (int)floor((php - dphi + kPi) * a.g.phi_scale);
    phi_hi = (int)floor((php + dphi + kPi) * a.g.phi_scale);
    full_phi = (phi_hi - plo + 1) >= nphi;
  }
  const int g = e * L + l;
  const BinOffsets off{a.bin_off + (int64_t)g * (a.n_bins + 1),
                       a.off16 ? reinterpret_cast<const uint16_t*>(a.bin_off) + (int64_t)g * off16_pitch(a.n_bins) : nullptr};
  const int64_t base = a.hit_off[g];
  const BinHit<TS>* hb = static_cast<const BinHit<TS>*>(a.hb);
  const HitRes hr = hit_res(a);
  // the candidate's sorted record list lives in LDS while the window is
  // scanned (rows [k][blockDim] of the dynamic shared memory: chi2 totals,
  // hit indices, binned positions) and goes to its record rows once
  // complete; records rank by (chi2 total, hit index)
  extern __shared__ double rec_lds[];
  const int t = threadIdx.x, B = blockDim.x;
  double* lc = rec_lds;
  int32_t* lh = reinterpret_cast<int32_t*>(rec_lds + NC * B);
  int32_t* lp = lh + NC * B;
  int nrec = 0;
  auto rec_less = [](double c1, int32_t h1, double c2, int32_t h2) {
    return c1 < c2 || (c1 == c2 && (uint32_t)h1 < (uint32_t)h2);
  };
  auto insert = [&](double c2, int32_t hid, int32_t hpos) {
    if (nrec == NC && !rec_less(c2, hid, lc[(NC - 1) * B + t], lh[(NC - 1) * B + t])) return;
    int pos = nrec < NC ? nrec : NC - 1;
    while (pos > 0 && rec_less(c2, hid, lc[(pos - 1) * B + t], lh[(pos - 1) * B + t])) {
      lc[pos * B + t] = lc[(pos - 1) * B + t];
      lh[pos * B + t] = lh[(pos - 1) * B + t];
      lp[pos * B + t] = lp[(pos - 1) * B + t];
      --pos;
    }
    lc[pos * B + t] = c2;
    lh[pos * B + t] = hid;
    lp[pos * B + t] = hpos;
    if (nrec < NC) ++nrec;
  };
  // each hit's loads are issued before it is scored; score(m0, m1, m2,
  // hit index, binned position)
  auto scan_range = [&](int32_t j0, int32_t j1, auto&& score) {
    if constexpr (sizeof(TS) == 4) {
      // two hits per step, their loads issued together (in double the
      // second hit's registers would spill)
      for (int32_t j = j0; j < j1; j += 2) {
        const int64_t h0 = base + j, h1 = base + (j + 1 < j1 ? j + 1 : j);
        const BinHit<TS> r0 = hb[h0], r1 = hb[h1];
        score((double)r0.x, (double)r0.y, (double)r0.z, r0.id, (int32_t)h0);
        if (j + 1 < j1) score((double)r1.x, (double)r1.y, (double)r1.z, r1.id, (int32_t)h1);
      }
    } else {
      for (int32_t j = j0; j < j1; ++j) {
        const BinHit<TS> r = hb[base + j];
        score(r.x, r.y, r.z, r.id, (int32_t)(base + j));
      }
    }
  };
  // up to two contiguous runs of phi bins (wrap-around), the same in every
  // z row of the window
  int lo0 = 0, hi0 = nphi - 1, lo1 = 0, hi1 = -1;
  if (!full_phi) {
    lo0 = ((plo % nphi) + nphi) % nphi;
    const int a1 = lo0 + (phi_hi - plo);
    if (a1 < nphi) {
      hi0 = a1;
    } else {
      hi0 = nphi - 1;
      hi1 = a1 - nphi;
    }
  }
  // Staging (seed order on): the wave's candidates come from neighbouring
  // seeds, so the union of their windows is a small box of bins; the wave
  // copies the box's offsets and binned hits into its own LDS area once,
  // and every lane scans its window there.  The wave works alone (its LDS
  // operations are in order; no barrier), with the lanes that reached this
  // point (the others ended).  A box that wraps in phi, spans two events
  // or exceeds the area falls back to the global scan below.
  bool staged = false;
  int32_t* s_off = nullptr;
  int32_t* s_row = nullptr;
  BinHit<TS>* s_hit = nullptr;
  int s_z0 = 0, s_p0 = 0, s_per = 0;
  if constexpr (STAGE) {
    char* wa = reinterpret_cast<char*>(rec_lds + NC * B) + (size_t)NC * B * 2 * sizeof(int32_t) +
               (size_t)(threadIdx.x >> 6) * StageArea<TS>::bytes;
    int32_t* red = reinterpret_cast<int32_t*>(wa);
    s_off = red + 8;
    s_row = s_off + StageArea<TS>::offs;
    s_hit = reinterpret_cast<BinHit<TS>*>(s_row + StageArea<TS>::rows + 8);
    const uint64_t act = __ballot(1);
    const int nact = __popcll(act);
    const int rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    if (rk == 0) {
      red[0] = INT32_MAX;
      red[1] = INT32_MIN;
      red[2] = INT32_MAX;
      red[3] = INT32_MIN;
      red[4] = INT32_MAX;
      red[5] = INT32_MIN;
    }
    wave_sync();
    atomicMin(&red[0], zlo);
    atomicMax(&red[1], zhi);
    atomicMin(&red[2], full_phi ? -1 : plo);
    atomicMax(&red[3], full_phi ? nphi : phi_hi);
    atomicMin(&red[4], g);
    atomicMax(&red[5], g);
    wave_sync();
    const int z0 = red[0], z1 = red[1], p0 = red[2], p1 = red[3];
    const int nrows = z1 - z0 + 1, per = p1 - p0 + 2;  // a row: the box's bins and the end of the last
    staged = red[4] == red[5] && p0 >= 0 && p1 < nphi && nrows <= StageArea<TS>::rows &&
             nrows * per <= StageArea<TS>::offs;
    if (staged) {
      for (int i = rk; i < nrows * per; i += nact) {
        const int r = i / per;
        s_off[i] = off[(z0 + r) * nphi + p0 + (i - r * per)];
      }
      wave_sync();
      if (rk == 0) {  // where each row's hits start in the area, and their total
        int tot = 0;
        for (int r = 0; r < nrows; ++r) {
          s_row[r] = tot;
          tot += s_off[r * per + per - 1] - s_off[r * per];
        }
        s_row[nrows] = tot;
      }
      wave_sync();
      staged = s_row[nrows] <= StageArea<TS>::hits;
      if (staged) {
        for (int r = 0; r < nrows; ++r) {
          const int32_t g0 = s_off[r * per], n = s_off[r * per + per - 1] - g0, b = s_row[r];
          for (int j = rk; j < n; j += nact) s_hit[b + j] = hb[base + g0 + j];
        }
        wave_sync();
      }
    }
    s_z0 = z0;
    s_p0 = p0;
    s_per = per;
  }
  auto scan_window = [&](auto&& score) {
    if constexpr (STAGE) {
      if (staged) {  // the lane's window lies in the box: one run per row
        for (int zb = zlo; zb <= zhi; ++zb) {
          const int32_t* ro = s_off + (zb - s_z0) * s_per;
          const int32_t j0 = ro[lo0 - s_p0], j1 = ro[hi0 + 1 - s_p0];
          const int32_t sh = s_row[zb - s_z0] - ro[0];  // area place of the row's hit j: sh + j
          for (int32_t j = j0; j < j1; ++j) {
            const BinHit<TS> r = s_hit[sh + j];
            score((double)r.x, (double)r.y, (double)r.z, r.id, (int32_t)(base + j));
          }
        }
        return;
      }
    }
    // the next row's first run is looked up while this row's hits are scored
    int32_t nj0 = off[zlo * nphi + lo0], nj1 = off[zlo * nphi + hi0 + 1];
    for (int zb = zlo; zb <= zhi; ++zb) {
      const int32_t j0 = nj0, j1 = nj1;
      if (zb < zhi) {
        nj0 = off[(zb + 1) * nphi + lo0];
        nj1 = off[(zb + 1) * nphi + hi0 + 1];
      }
      scan_range(j0, j1, score);
      if (hi1 >= lo1) scan_range(off[zb * nphi + lo1], off[zb * nphi + hi1 + 1], score);
    }
  };
  if (hr.sr2 == hr.srphi2) {
    // equal radial and tangential resolutions: the hit covariance is
    // diag(sr^2, sr^2, sz^2) wherever the hit lies in phi, so S and its
    // inverse belong to the candidate and each hit costs only its residual
    // and the quadratic form (the per-hit form below rounds V's transverse
    // terms differently, by an ulp of sr^2)
    const double Sc[6] = {(double)Pp[pidx(0, 0)] + hr.sr2, (double)Pp[pidx(0, 1)],
                          (double)Pp[pidx(0, 2)], (double)Pp[pidx(1, 1)] + hr.sr2,
                          (double)Pp[pidx(1, 2)], (double)Pp[pidx(2, 2)] + hr.sz2};
    double Si[6];
    const double p0 = xp.pos[0], p1 = xp.pos[1], p2 = xp.pos[2];
    if (sym3_inverse(Sc, Si)) {
      scan_window([&](double m0, double m1, double m2, int32_t hid, int32_t hpos) {
        const double r[3] = {m0 - p0, m1 - p1, m2 - p2};
        const double c2 = quad3(Si, r);
        if (c2 < cut) insert(pchi2 + c2, hid, hpos);
      });
    }
  } else {
    scan_window([&](double m0, double m1, double m2, int32_t hid, int32_t hpos) {
      const double m[3] = {m0, m1, m2};
      Residual R;
      if (residual(xp, Pp, m, hr, R) && R.chi2 < cut) insert(pchi2 + R.chi2, hid, hpos);
    });
  }
  if (nrec == 0) {
    if (meta_nm(meta) < a.g.max_missed) {
      lc[t] = pchi2;
      lh[t] = -1;
      lp[t] = -1;
      nrec = 1;
    } else {
      a.rcount[c] = -2;
      store_ended();
      return;
    }
  }
  // the record list and its count go out with plain stores: the merge
  // reads them right after this launch, while they are still in the caches
  for (int k = 0; k < nrec; ++k) {
    a.rchi[(int64_t)k * S + c] = lc[k * B + t];
    a.rhit[(int64_t)k * S + c] = lh[k * B + t];
    a.rpos[(int64_t)k * S + c] = lp[k * B + t];
  }
  a.rcount[c] = (int32_t)nrec;
}

template <typename TS, typename TP, bool MAT, bool CHILD, bool STAGE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CHILD ? 3 : 1)))
void build_score_kernel(BuildArgs a, int l, int cur) {
  ROW_CHUNKS(a, l - 1, (score_row<TS, TP, MAT, CHILD, STAGE>(a, l, cur, c)));
}

// ----------------------------------------------------------------- select
// final-choice key: more hits, lower chi2, earlier end, lower rank
__device__ __forceinline__ bool final_less(int nh1, double c1, int e1, int r1, int nh2, double c2,
                                           int e2, int r2) {
  if (nh1 != nh2) return nh1 > nh2;
  if (c1 != c2) return c1 < c2;
  if (e1 != e2) return e1 < e2;
  return r1 < r2;
}

// LPS lanes per seed (1, 2 or 4, inside one quad): lane q owns the seed's
// parents q, q + LPS, ... (PPL = ceil(max_cands / LPS) slots) and holds each
// one's record-list head (chi2, hit) in registers, with the next three
// records prefetched in the same pass of independent loads.  The max_cands
// best heads by the ranking (more hits, lower chi2, lower parent, lower hit;
// a missed layer counts no hit) are taken one at a time: each lane's best
// slot, then the group's best by DPP exchanges, so the dependent chain per
// pick stays in registers.  Parents that ended this layer compete for the
// seed's best ended candidate the same way.  The kept records become the
// seed's children: contiguous rows of the next buffer, in pick order,
// reserved for the whole block at once.
//
// Fewer lanes per seed issue fewer instructions per seed (a lane-local
// compare costs less than an exchange, and a group's lanes all execute
// every pick) but hold more parents' heads in registers.

// a record-list head as ranked by the merge: key = 0 for none, else the hit
// count it gives plus one; pj = parent << 16 | records in its list << 8 |
// this record's place in the list
__device__ __forceinline__ int mpj(int parent, int count, int rec) { return (parent << 16) | (count << 8) | rec; }
__device__ __forceinline__ int mpj_parent(int pj) { return pj >> 16; }
__device__ __forceinline__ int mpj_count(int pj) { return (pj >> 8) & 0xff; }
__device__ __forceinline__ int mpj_rec(int pj) { return pj & 0xff; }

struct MHead {
  int key;
  double c;
  int pj;
  int hit;  // index within the (event, layer), -1: missed layer
  int pos;  // binned position, -1: missed layer
};

// all terms evaluated (no short circuit), so that the choice compiles to
// compares and selects rather than branches
__device__ __forceinline__ bool mhead_better(const MHead& x, const MHead& y) {
  const bool gt = x.key > y.key, eq = x.key == y.key;
  const bool cl = x.c < y.c, ce = x.c == y.c;
  const bool pl = x.pj < y.pj;  // the parent decides: parents differ, and they are the top bits
  return gt | (eq & (cl | (ce & pl)));
}

// w = the better of w and h
__device__ __forceinline__ void mhead_take(MHead& w, const MHead& h) {
  const bool b = mhead_better(h, w);
  w.key = b ? h.key : w.key;
  w.c = b ? h.c : w.c;
  w.pj = b ? h.pj : w.pj;
  w.hit = b ? h.hit : w.hit;
  w.pos = b ? h.pos : w.pos;
}

// w = the better of w and h where h's parent is known to come after w's
// (a lane's own slots, taken in order): a tie in hits and chi2 keeps w
__device__ __forceinline__ void mhead_take_later(MHead& w, const MHead& h) {
  const bool b = (h.key > w.key) | ((h.key == w.key) & (h.c < w.c));
  w.key = b ? h.key : w.key;
  w.c = b ? h.c : w.c;
  w.pj = b ? h.pj : w.pj;
  w.hit = b ? h.hit : w.hit;
  w.pos = b ? h.pos : w.pos;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ void dpp_take(MHead& h) {
  const int64_t cb = __double_as_longlong(h.c);
  const MHead o{dpp_i<CTRL>(h.key),
                __longlong_as_double(((int64_t)dpp_i<CTRL>((int)(cb >> 32)) << 32) |
                                     (uint32_t)dpp_i<CTRL>((int)cb)),
                dpp_i<CTRL>(h.pj), dpp_i<CTRL>(h.hit), dpp_i<CTRL>(h.pos)};
  mhead_take(h, o);
}

// best of the seed's LPS lanes; every one ends with the same head (a strict
// total order: parents are distinct)
template <int LPS>
__device__ __forceinline__ void group_best(MHead& h) {
  if constexpr (LPS >= 2) dpp_take<0xB1>(h);  // lanes q ^ 1
  if constexpr (LPS == 4) dpp_take<0x4E>(h);  // lanes q ^ 2
}

// the sum over the group's lanes, in every one of them
template <int LPS>
__device__ __forceinline__ int group_sum(int v) {
  if constexpr (LPS >= 2) v += dpp_i<0xB1>(v);  // lanes q ^ 1
  if constexpr (LPS == 4) v += dpp_i<0x4E>(v);  // lanes q ^ 2
  return v;
}

// the value of the group's first lane
template <int LPS>
__device__ __forceinline__ int group_first(int v) {
  if constexpr (LPS == 4) return dpp_i<0x00>(v);  // quad lanes 0,0,0,0
  if constexpr (LPS == 2) return dpp_i<0xA0>(v);  // quad lanes 0,0,2,2
  return v;
}

template <typename TS, int LPS, int PPL>
__global__ __launch_bounds__(kMergeThreads) void build_merge_kernel(BuildArgs a, int l, int cur) {
  constexpr int SB = merge_seeds(LPS);
  __shared__ int wtot[kMergeThreads / 64 + 1];
  const int NC = a.g.max_cands;
  const int tid = threadIdx.x;
  const int q = tid % LPS, ls = tid / LPS;
  const int64_t sp = a.sp, S = a.S;
  const int64_t s = (int64_t)blockIdx.x * SB + ls;
  const bool real = s < a.n_seeds;
  int nlive = 0;
  int64_t pbase = 0;
  int32_t info = 0;
  if (real) {  // cstart is only meaningful for a seed with candidates
    nlive = a.count[(int64_t)(l - 1) * sp + s];
    pbase = a.cstart[cur][s];
    const int e = a.sev[s];
    info = pack_info(e, a.q[s]);
  }
  // Each parent's head record sits in registers; the records behind it, up
  // to PF of them, wait in LDS rows [PF][PPL][threads] (one column per
  // thread: conflict-free however the lanes index them), so that taking a
  // head replaces only that head's registers instead of shifting a queue
  // through every slot.  Records beyond PF are read from their rows, rarely.
  constexpr int PF = 1;
  __shared__ double qc_s[PF * PPL][kMergeThreads];
  __shared__ int qh_s[PF * PPL][kMergeThreads];
  __shared__ int qp_s[PF * PPL][kMergeThreads];
  int rc[PPL], nh[PPL], hd[PPL], hh[PPL], hp[PPL];
  double pchi[PPL], hc[PPL];
#pragma unroll
  for (int u = 0; u < PPL; ++u) {
    const int j = q + LPS * u;
    const int64_t p = pbase + j;
    rc[u] = 0;
    nh[u] = 0;
    hd[u] = 0;
    pchi[u] = 0.0;
    hc[u] = 0.0;
    hh[u] = -1;
    hp[u] = -1;
    if (j < nlive) {  // record 0 is read with the count and used only if rc > 0
      rc[u] = a.rcount[p];
      nh[u] = meta_nh(a.cmeta[cur][p]);
      pchi[u] = a.cchi2[cur][p];
      hc[u] = a.rchi[p];
      hh[u] = a.rhit[p];
      hp[u] = a.rpos[p];
    }
  }
#pragma unroll
  for (int u = 0; u < PPL; ++u) {
    const int64_t p = pbase + q + LPS * u;
#pragma unroll
    for (int v = 0; v < PF; ++v) {
      if (v + 1 < rc[u]) {
        const int64_t ri = (int64_t)(v + 1) * S + p;
        qc_s[v * PPL + u][tid] = a.rchi[ri];
        qh_s[v * PPL + u][tid] = a.rhit[ri];
        qp_s[v * PPL + u][tid] = a.rpos[ri];
      }
    }
  }
  // best ended parent (the same in all the seed's lanes)
  MHead eb{0, 0.0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < PPL; ++u) {
    const int j = q + LPS * u;
    const MHead h{(j < nlive && rc[u] <= 0) ? nh[u] + 1 : 0, pchi[u], mpj(j, 0, 0), 0, 0};
    if (u == 0)
      eb = h;
    else
      mhead_take_later(eb, h);
  }
  group_best<LPS>(eb);
  if (eb.key > 0) {
    const int e_nh = eb.key - 1, ej = mpj_parent(eb.pj);
    const int be = a.bend[s];
    if (be < 0 || final_less(e_nh, eb.c, l, ej, meta_nh(a.bmeta[s]), a.bchi2[s], be, a.brank[s])) {
      // the seed's lanes copy the ended candidate in chunks of five
      // elements, a chunk's loads before its stores (a load issued after a
      // store waits for it: the memory counter counts both); float elements
      // go through double exactly
      const int64_t pe = pbase + ej;
      const TS* mo = static_cast<const TS*>(a.cmom[cur]);
      const TS* co = static_cast<const TS*>(a.ccov[cur]);
      TS* bm = static_cast<TS*>(a.bmom);
      TS* bc = static_cast<TS*>(a.bcov);
      constexpr int NE = (27 + LPS - 1) / LPS, CH = 5;
#pragma unroll
      for (int i0 = 0; i0 < NE; i0 += CH) {
        double ev[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int e = q + LPS * (i0 + i);
          ev[i] = 0.0;
          if (e < 3)
            ev[i] = a.cpos[cur][e * S + pe];
          else if (e < 6)
            ev[i] = (double)mo[(e - 3) * S + pe];
          else if (e < 27)
            ev[i] = (double)co[(e - 6) * S + pe];
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int e = q + LPS * (i0 + i);
          if (e < 3)
            a.bpos[e * sp + s] = ev[i];
          else if (e < 6)
            bm[(e - 3) * sp + s] = (TS)ev[i];
          else if (e < 27)
            bc[(e - 6) * sp + s] = (TS)ev[i];
        }
      }
      if (q == 0) {
        const uint32_t m = a.cmeta[cur][pe];
        a.bchi2[s] = eb.c;
        a.bmeta[s] = pack_meta(e_nh, meta_nm(m), meta_st(m) | (a.rcount[pe] == -1 ? kNoReach : 0u));
        a.bend[s] = l;
        a.brank[s] = ej;
      }
    }
  }
  // k-way merge of the parents' lists.  A list's records all give the same
  // hit count (a missed-layer record is a list of its own), so a head's
  // key stays fixed until its list runs out.
  int hk[PPL];
#pragma unroll
  for (int u = 0; u < PPL; ++u) hk[u] = rc[u] > 0 ? nh[u] + (hh[u] >= 0 ? 1 : 0) + 1 : 0;
  // the seed keeps min(max_cands, records of all its parents) children: its
  // rows of the next buffer are reserved before the picks, which then go
  // straight to them
  int nrec_lane = 0;
#pragma unroll
  for (int u = 0; u < PPL; ++u) nrec_lane += rc[u] > 0 ? rc[u] : 0;
  const int nsel = min(NC, group_sum<LPS>(nrec_lane));
  const int reg = block_region(a);
  const int local = (int)block_reserve(region_ctr(a, l, reg), q == 0 ? nsel : 0, wtot);
  const int64_t first = reg * a.RS + group_first<LPS>(local);
  // every load issued so far is complete before the picks: otherwise the
  // wait for the heads' loads sits at the top of the pick loop, and with the
  // stores of each pick in flight it would wait for those every time (the
  // seed's count and first row are stored after the picks, so that this
  // wait does not include them)
  __builtin_amdgcn_s_waitcnt(0);
  for (int k = 0; k < nsel; ++k) {
    MHead w{hk[0], hc[0], mpj(q, rc[0], hd[0]), hh[0], hp[0]};
#pragma unroll
    for (int u = 1; u < PPL; ++u) {
      mhead_take_later(w, MHead{hk[u], hc[u], mpj(q + LPS * u, rc[u], hd[u]), hh[u], hp[u]});
    }
    group_best<LPS>(w);
    // the seed's k-th child: its parent, hit and chi2 total (the history
    // is read only by the backtrack: non-temporal)
    if constexpr (LPS == 1) {
      st_nt(a.hist + ((int64_t)l * NC + k) * 2 * sp + 0 * sp + s, (int32_t)mpj_parent(w.pj));
      st_nt(a.hist + ((int64_t)l * NC + k) * 2 * sp + 1 * sp + s, (int32_t)w.hit);
      a.sel_parent[first + k] = (int32_t)(pbase + mpj_parent(w.pj));
      a.sel_hit[first + k] = w.pos;
      a.sel_chi2[first + k] = w.c;
      a.cinfo[cur ^ 1][first + k] = info;
    } else if (q < 2) {
      // the seed's first two lanes share the stores: one instruction writes
      // the parent from one lane and the hit from the other
      const bool p0 = q == 0;
      st_nt(a.hist + (((int64_t)l * NC + k) * 2 + q) * sp + s, p0 ? (int32_t)mpj_parent(w.pj) : (int32_t)w.hit);
      int32_t* sel = p0 ? a.sel_parent : a.sel_hit;
      sel[first + k] = p0 ? (int32_t)(pbase + mpj_parent(w.pj)) : w.pos;
      if (p0)
        a.cinfo[cur ^ 1][first + k] = info;
      else
        a.sel_chi2[first + k] = w.c;
    }
    // the owner lane replaces the taken head by the next record of its list
    // (selects, not branches).  A record beyond the LDS ones is loaded in a
    // branch of its own that also consumes it, rarely: a load whose value
    // is used after the branch would make every pick wait on the memory
    // counter, which on this chip also counts the stores above, so each pick
    // would wait for the previous pick's child to be written.
    const int wj = mpj_parent(w.pj);
    const int us = wj / LPS;               // the winner's slot in its owner lane
    const int nx = mpj_rec(w.pj) + 1;      // the next record of its list
    const bool more = nx < mpj_count(w.pj);
    const int vq = nx - 1 < PF ? nx - 1 : PF - 1;
    double ncv = qc_s[vq * PPL + us][tid];
    int nhv = qh_s[vq * PPL + us][tid];
    int npv = qp_s[vq * PPL + us][tid];
    const bool far = more && nx > PF && wj % LPS == q;
    if (__any(far)) {
      if (far) {
        const int64_t fr = (int64_t)nx * S + pbase + wj;
        ncv = a.rchi[fr];
        nhv = a.rhit[fr];
        npv = a.rpos[fr];
      }
      // the loaded values go into the heads here, inside the branch
#pragma unroll
      for (int u = 0; u < PPL; ++u) {
        const bool adv = far && wj == q + LPS * u;
        hc[u] = adv ? ncv : hc[u];
        hh[u] = adv ? nhv : hh[u];
        hp[u] = adv ? npv : hp[u];
      }
    }
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
      const bool adv = wj == q + LPS * u;
      const bool lds = adv && !far;
      hd[u] = adv ? nx : hd[u];
      hc[u] = lds ? ncv : hc[u];
      hh[u] = lds ? nhv : hh[u];
      hp[u] = lds ? npv : hp[u];
      hk[u] = adv && !more ? 0 : hk[u];
    }
  }
  if (real && q == 0) {
    a.count[(int64_t)l * sp + s] = nsel;
    if (nsel > 0) a.cstart[cur ^ 1][s] = (int32_t)first;
  }
}
// ------------------------------------------------------------------ final
// The seed's final choice: the best survivor or the best ended candidate.
// LAZY: the survivors are the last layer's children, not yet made, ranked
// from their records (the parent's hits plus the one taken, the chi2
// total); otherwise (no building layer) they are the stored seed fits.
struct FinalChoice {
  bool from_ended;
  int end_layer, rank;
  int64_t base;  // the seed's first survivor row
};

template <bool LAZY>
__device__ __forceinline__ FinalChoice final_choice(const BuildArgs& a, int cur, int64_t s) {
  const int L = a.g.n_layers;
  // the seed's own words first, all in one round trip: its survivors and
  // its best ended candidate
  const int nalive = a.count[(int64_t)(L - 1) * a.sp + s];
  const int64_t cst = a.cstart[cur][s];
  const int be = a.bend[s];
  const int e_nh = meta_nh(a.bmeta[s]);
  const double e_c2 = a.bchi2[s];
  const int e_rank = a.brank[s];
  FinalChoice f{false, L, -1, nalive > 0 ? cst : 0};
  // The survivors are in rank order, and the rank order (more hits, then
  // lower chi2, then the pick order) is the final key among candidates that
  // all end on the last layer: the best survivor is the first.
  int bnh = 0;
  double bc2 = 0.0;
  if (nalive > 0) {
    f.rank = 0;
    if constexpr (LAZY) {
      bnh = meta_nh(a.cmeta[cur ^ 1][a.sel_parent[f.base]]) + (a.sel_hit[f.base] >= 0 ? 1 : 0);
      bc2 = a.sel_chi2[f.base];
    } else {
      bnh = meta_nh(a.cmeta[cur][f.base]);
      bc2 = a.cchi2[cur][f.base];
    }
  }
  if (be >= 0 && (f.rank < 0 || final_less(e_nh, e_c2, be, e_rank, bnh, bc2, L, f.rank))) {
    f.from_ended = true;
    f.end_layer = be;
    f.rank = e_rank;
  }
  return f;
}

// One lane per seed: the chosen candidate's hits, walking the (parent, hit)
// records back from its end layer.  A kernel of its own: the walk is a
// chain of dependent loads, which wants many waves in flight, while making
// the chosen child needs the registers of a Kalman update.
template <typename TS, bool LAZY>
__global__ __launch_bounds__(256) void build_backtrack_kernel(BuildArgs a, int cur) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  const int L = a.g.n_layers, NC = a.g.max_cands;
  const FinalChoice f = final_choice<LAZY>(a, cur, s);
  for (int l = L - 1; l >= f.end_layer; --l) st_nt(a.o_hit + (int64_t)l * a.sp + s, (int32_t)-1);
  // The walk is a chain of dependent loads; each layer's record is loaded
  // before the layer above it is stored, so that waiting for the load does
  // not also wait for that store (the memory counter counts both).
  int r = f.rank;
  int l = f.end_layer - 1;
  int hit = -1, nr = -1;
  if (l >= 0 && r >= 0 && r < NC) {
    const int64_t hb = ((int64_t)l * NC + r) * 2 * a.sp;
    hit = a.hist[hb + a.sp + s];
    nr = a.hist[hb + s];
  }
  for (; l >= 0; --l) {
    // the record of layer l (hit, parent rank nr) is in flight or done;
    // issue layer l - 1's before storing layer l's hit
    const bool rec = r >= 0 && r < NC;
    const int h_l = rec ? hit : -1;
    r = rec ? nr : -1;
    if (l > 0 && r >= 0 && r < NC) {
      const int64_t hb = ((int64_t)(l - 1) * NC + r) * 2 * a.sp;
      hit = a.hist[hb + a.sp + s];
      nr = a.hist[hb + s];
    }
    st_nt(a.o_hit + (int64_t)l * a.sp + s, (int32_t)h_l);
  }
}

// One lane per seed: the chosen candidate's state, covariance, chi2, hit
// count and status (LAZY: the chosen child is made here, the only one of
// the last layer's children that is).
template <typename TS, typename TP, bool LAZY>
__global__ __launch_bounds__(256) void build_final_kernel(BuildArgs a, int cur) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  const int L = a.g.n_layers;
  const FinalChoice f = final_choice<LAZY>(a, cur, s);
  TrackState<TP> x;
  TP P[21];
  uint32_t meta;
  double c2;
  if (f.from_ended) {
    load_cand<TS, TP>(a.bpos, a.bmom, a.bcov, a.sp, s, x, P);
    meta = a.bmeta[s];
    c2 = a.bchi2[s];
  } else if constexpr (LAZY) {
    meta = make_child<TS, TP>(a, L - 1, cur ^ 1, f.base + f.rank, x, P);
    c2 = a.sel_chi2[f.base + f.rank];
  } else {
    load_cand<TS, TP>(a.cpos[cur], a.cmom[cur], a.ccov[cur], a.S, f.base + f.rank, x, P);
    meta = a.cmeta[cur][f.base + f.rank];
    c2 = a.cchi2[cur][f.base + f.rank];
  }
  // the results are not read again by the build: non-temporal
  TS* so = static_cast<TS*>(a.o_state);
  TS* co = static_cast<TS*>(a.o_cov);
#pragma unroll
  for (int c = 0; c < 3; ++c) st_nt(so + c * a.sp + s, (TS)x.pos[c]);
#pragma unroll
  for (int c = 0; c < 3; ++c) st_nt(so + (c + 3) * a.sp + s, (TS)x.mom[c]);
#pragma unroll
  for (int c = 0; c < 21; ++c) st_nt(co + c * a.sp + s, (TS)P[c]);
  uint32_t st = meta_st(meta);
  if (!finite_state(x, P)) st |= kNonFinite;
  a.o_chi2[s] = c2;
  a.o_nhits[s] = meta_nh(meta);
  a.o_status[s] = st;
}

// -------------------------------------------------------------- host side
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename TS, typename TP, bool STAGE>
static void launch_score(const BuildArgs& a, int l, int cur, bool child, dim3 rows, size_t lds, hipStream_t st) {
  const dim3 blk(256);
  if (a.g.mat.on && child)
    hipLaunchKernelGGL((build_score_kernel<TS, TP, true, true, STAGE>), rows, blk, lds, st, a, l, cur);
  else if (a.g.mat.on)
    hipLaunchKernelGGL((build_score_kernel<TS, TP, true, false, STAGE>), rows, blk, lds, st, a, l, cur);
  else if (child)
    hipLaunchKernelGGL((build_score_kernel<TS, TP, false, true, STAGE>), rows, blk, lds, st, a, l, cur);
  else
    hipLaunchKernelGGL((build_score_kernel<TS, TP, false, false, STAGE>), rows, blk, lds, st, a, l, cur);
}

template <typename TS, int LPS, int PPL>
static void launch_merge_as(const BuildArgs& a, int l, int cur, hipStream_t st) {
  const dim3 grid(nblk(a.n_seeds, merge_seeds(LPS))), block(kMergeThreads);
  hipLaunchKernelGGL((build_merge_kernel<TS, LPS, PPL>), grid, block, 0, st, a, l, cur);
}

// parents per lane: max_cands over the lanes per seed, rounded up
template <typename TS>
static void launch_merge(const BuildArgs& a, int l, int cur, hipStream_t st) {
  const int nc = a.g.max_cands, lps = merge_lanes(nc), ppl = (nc + lps - 1) / lps;
  if (lps == 1) {
    if (ppl <= 2)
      launch_merge_as<TS, 1, 2>(a, l, cur, st);
    else
      launch_merge_as<TS, 1, 4>(a, l, cur, st);
  } else if (lps == 2) {
    if (ppl <= 3)
      launch_merge_as<TS, 2, 3>(a, l, cur, st);
    else
      launch_merge_as<TS, 2, 5>(a, l, cur, st);
  } else {
    launch_merge_as<TS, 4, 4>(a, l, cur, st);
  }
}

// a launch with more than 64 KB of dynamic LDS first raises the kernel's
// limit to what it asks for
template <typename... P, typename... A>
static hipError_t launch_dyn_lds(void (*k)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t st, A&&... args) {
  if (lds > 65536) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, grid, block, lds, st, std::forward<A>(args)...);
  return hipGetLastError();
}

template <typename TS, typename TP>
static hipError_t run_build(const BuildArgs& a, bool bins_only, hipStream_t st) {
  const int bs = 256;
  const int64_t nbins_all = (int64_t)a.n_groups * a.n_bins;
  if (nbins_all > 0 && a.n_bins <= kLdsBins && a.max_group <= kPackMaxHits) {
    const size_t lds = bin_lds_bytes(a.n_bins, a.max_group);
    hipError_t e = hipSuccess;
    if (a.max_group <= 2 * 4 * kBinThreads)
      e = launch_dyn_lds(bin_group16_kernel<TS, 2, 4>, dim3(a.n_groups), dim3(kBinThreads), lds, st, a);
    else if (a.max_group <= 2 * kBinBatch * kBinThreads)
      e = launch_dyn_lds(bin_group16_kernel<TS, 2, kBinBatch>, dim3(a.n_groups), dim3(kBinThreads), lds, st, a);
    else
      e = launch_dyn_lds(bin_group16_kernel<TS, 4, kBinBatch>, dim3(a.n_groups), dim3(kBinThreads), lds, st, a);
    if (e != hipSuccess) return e;
  } else if (nbins_all > 0) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(nbins_all, bs)), dim3(bs), 0, st, a.bin_cur, nbins_all, 0);
    if (a.n_hits > 0)
      hipLaunchKernelGGL((bin_count_kernel<TS>), dim3(nblk(a.n_hits, bs)), dim3(bs), 0, st, a);
    hipLaunchKernelGGL(bin_scan_kernel, dim3(a.n_groups), dim3(kScanThreads), 0, st, a);
    if (a.n_hits > 0)
      hipLaunchKernelGGL(bin_scatter_kernel, dim3(nblk(a.n_hits, bs)), dim3(bs), 0, st, a);
    if (a.n_hits > 0)
      hipLaunchKernelGGL((bin_rank_kernel<TS>), dim3(nblk(a.n_hits, bs)), dim3(bs), 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || bins_only || a.n_seeds == 0) return e;
  if (a.seed_order) {  // the seeds of each event in order of their predicted cell
    hipLaunchKernelGGL((seed_key_kernel<TS, TP>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a);
    hipLaunchKernelGGL(seed_order_kernel, dim3(a.n_events), dim3(kOrderThreads), 0, st, a);
    hipLaunchKernelGGL((seed_gather_kernel<TS>), dim3(xcd_grid(nblk(a.n_seeds, bs))), dim3(bs), 0, st, a);
  }
  hipLaunchKernelGGL(seed_event_kernel, dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a);
  if (a.g.mat.on)
    hipLaunchKernelGGL((build_seed_kernel<TS, TP, true>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a);
  else
    hipLaunchKernelGGL((build_seed_kernel<TS, TP, false>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a);
  int cur = 0;
  // the score kernel's record lists in LDS: max_cands chi2 totals and hit
  // indices per thread
  const size_t rec_lds = (size_t)a.g.max_cands * bs * (sizeof(double) + 2 * sizeof(int32_t)) +
                         (a.seed_order ? (size_t)(bs / 64) * StageArea<TS>::bytes : 0);
  const dim3 rows((unsigned)(a.NR * ((a.RS / bs + kRowChunks - 1) / kRowChunks)));
  for (int l = a.g.n_seed_layers; l < a.g.n_layers; ++l) {
    const bool child = l > a.g.n_seed_layers;  // candidates kept on layer l - 1, not yet made
    if (a.seed_order)
      launch_score<TS, TP, true>(a, l, cur, child, rows, rec_lds, st);
    else
      launch_score<TS, TP, false>(a, l, cur, child, rows, rec_lds, st);
    launch_merge<TS>(a, l, cur, st);
    cur ^= 1;
  }
  if (a.g.n_layers > a.g.n_seed_layers) {  // the last layer's children are made for the chosen one only
    hipLaunchKernelGGL((build_backtrack_kernel<TS, true>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a, cur);
    hipLaunchKernelGGL((build_final_kernel<TS, TP, true>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a, cur);
  } else {
    hipLaunchKernelGGL((build_backtrack_kernel<TS, false>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a, cur);
    hipLaunchKernelGGL((build_final_kernel<TS, TP, false>), dim3(nblk(a.n_seeds, bs)), dim3(bs), 0, st, a, cur);
  }
  if (a.seed_order)
    hipLaunchKernelGGL((seed_scatter_kernel<TS>), dim3(xcd_grid(nblk(a.n_seeds, bs))), dim3(bs), 0, st, a);
  return hipGetLastError();
}

static int validate_batch(ktf_ctx* c, const ktf_event_batch* ev) {
  if (const char* why = check_event_batch(ev, c->cfg.n_layers, c->cfg.max_cands))
    return fail(c, KTF_EINVAL, "ktf_build: %s", why);
  // seed_pitch * max_cands < 2^31 here, so the row count cannot overflow
  const int64_t n = ev->seed_off[ev->n_events];
  if (region_rows(n, c->cfg.max_cands) * region_count(n, c->cfg.max_cands) > INT32_MAX)
    return fail(c, KTF_EINVAL, "ktf_build: more than 2^31 candidate rows");
  return KTF_OK;
}

// Fills the workspace part of BuildArgs; allocates (grows) context buffers.
static int prepare(ktf_ctx* c, const ktf_event_batch* ev, bool bins_only, BuildArgs& a, hipStream_t st) {
  const ktf_config& cfg = c->cfg;
  const int L = cfg.n_layers;
  memset(&a, 0, sizeof a);
  a.g.n_layers = L;
  a.g.eta_rows = cfg.n_etabins > 0 ? 1 : 0;
  a.g.eta_max = cfg.eta_max;
  a.g.n_zbins = cfg.n_etabins > 0 ? cfg.n_etabins : cfg.n_zbins;
  a.g.n_phibins = cfg.n_phibins;
  a.g.max_cands = cfg.max_cands;
  a.g.max_missed = cfg.max_missed;
  a.g.n_seed_layers = cfg.n_seed_layers;
  a.g.bz = cfg.bz;
  a.g.z_half = cfg.z_half;
  a.g.row_scale = a.g.n_zbins / (2.0 * (a.g.eta_rows ? a.g.eta_max : a.g.z_half));
  a.g.phi_scale = a.g.n_phibins / (2.0 * kPi);
  a.g.chi2_cut = cfg.chi2_cut;
  a.g.hr.sr2 = cfg.sigma_r * cfg.sigma_r;
  a.g.hr.srphi2 = cfg.sigma_rphi * cfg.sigma_rphi;
  a.g.hr.sz2 = cfg.sigma_z * cfg.sigma_z;
  for (int l = 0; l < L; ++l) a.g.radii[l] = c->radii[l];
  a.g.mat = material_of(c);
  a.n_events = ev->n_events;
  a.n_groups = ev->n_events * L;
  a.bin_l0 = bins_only ? 0 : cfg.n_seed_layers;
  a.n_bins = a.g.n_zbins * cfg.n_phibins;
  a.n_seeds = ev->seed_off[ev->n_events];
  a.sp = ev->seed_pitch;
  a.RS = region_rows(a.n_seeds, cfg.max_cands);
  a.NR = region_count(a.n_seeds, cfg.max_cands);
  a.S = a.RS * a.NR;
  a.n_hits = ev->hit_off[a.n_groups];
  a.max_group = 0;
  for (int g = 0; g < a.n_groups; ++g)
    a.max_group = std::max<int64_t>(a.max_group, ev->hit_off[g + 1] - ev->hit_off[g]);
  // a build binned by the one-block kernel (every group within its limits,
  // as run_build decides) keeps its offsets in 16 bits; ktf_bin_hits hands
  // the caller 32-bit ones
  a.off16 = !bins_only && a.n_bins >= 8 && a.n_bins <= kLdsBins && a.max_group <= kPackMaxHits ? 1 : 0;
  a.hp = ev->hit_pitch;
  a.hits = ev->hits;
  a.seed_state = ev->seed_state;
  a.seed_cov = ev->seed_cov;
  a.q = ev->charge;
  a.seed_hit = ev->seed_hit;
  const size_t ts = ev->prec == KTF_FP64 ? 8 : 4;
  hipError_t e;
  // offsets to the device through pinned staging
  const size_t n_off = (size_t)(ev->n_events + 1) + (size_t)(a.n_groups + 1);
  const size_t off_bytes = n_off * sizeof(int64_t);
  if (c->h_pinned_bytes < off_bytes) {
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    c->h_pinned = nullptr;
    c->h_pinned_bytes = 0;
    if ((e = hipHostMalloc(&c->h_pinned, off_bytes * 2, 0)) != hipSuccess) return hip_fail(c, e, "pinned staging");
    c->h_pinned_bytes = off_bytes * 2;
  }
  // calls on one context share the workspace and the staging buffer: wait
  // until the previous call's work (on whatever stream) has finished
  if (c->build_done) {
    if ((e = hipEventSynchronize(c->build_done)) != hipSuccess) return hip_fail(c, e, "previous build");
  }
  int64_t* hp = static_cast<int64_t*>(c->h_pinned);
  memcpy(hp, ev->seed_off, sizeof(int64_t) * (ev->n_events + 1));
  memcpy(hp + ev->n_events + 1, ev->hit_off, sizeof(int64_t) * (a.n_groups + 1));
  if ((e = c->b_stage.ensure(off_bytes)) != hipSuccess) return hip_fail(c, e, "workspace");
  if ((e = hipMemcpyAsync(c->b_stage.p, hp, off_bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(c, e, "offsets copy");
  a.seed_off = static_cast<const int64_t*>(c->b_stage.p);
  a.hit_off = a.seed_off + ev->n_events + 1;

  const int64_t nb = a.n_bins;
  const int64_t nhits = std::max<int64_t>(a.n_hits, 1);
  if ((e = c->b_off.ensure(sizeof(int32_t) * ((size_t)a.n_groups * (nb + 1) + (size_t)a.n_groups * nb))) != hipSuccess)
    return hip_fail(c, e, "bin workspace");
  a.bin_off = static_cast<int32_t*>(c->b_off.p);
  a.bin_cur = a.bin_off + (size_t)a.n_groups * (nb + 1);
  if ((e = c->b_perm.ensure(sizeof(int32_t) * 3 * (size_t)nhits)) != hipSuccess) return hip_fail(c, e, "bin workspace");
  a.perm = static_cast<int32_t*>(c->b_perm.p);
  a.hit_bin = a.perm + nhits;
  a.perm_raw = a.hit_bin + nhits;
  const size_t rec = ts == 4 ? sizeof(BinHit<float>) : sizeof(BinHit<double>);
  if ((e = c->b_binned.ensure(rec * (size_t)nhits)) != hipSuccess) return hip_fail(c, e, "bin workspace");
  a.hb = c->b_binned.p;
  if (bins_only) return KTF_OK;
  a.perm = nullptr;  // building reads the local indices from the records

  const int64_t S = std::max<int64_t>(a.S, 1);
  const size_t cand_bytes = (size_t)S * (3 * 8 + 24 * ts + 8 + 4);
  for (int b = 0; b < 2; ++b) {
    if ((e = c->b_cand[b].ensure(cand_bytes)) != hipSuccess) return hip_fail(c, e, "candidate workspace");
    char* p = static_cast<char*>(c->b_cand[b].p);
    a.cpos[b] = reinterpret_cast<double*>(p);
    p += (size_t)S * 3 * 8;
    a.cchi2[b] = reinterpret_cast<double*>(p);
    p += (size_t)S * 8;
    a.cmom[b] = p;
    p += (size_t)S * 3 * ts;
    a.ccov[b] = p;
    p += (size_t)S * 21 * ts;
    a.cmeta[b] = reinterpret_cast<uint32_t*>(p);
  }
  if ((e = c->b_prop.ensure(2 * (size_t)S * (3 * 8 + 24 * ts + 8) + 8)) != hipSuccess)
    return hip_fail(c, e, "workspace");
  {
    char* p = static_cast<char*>(c->b_prop.p);
    for (int b = 0; b < 2; ++b) {
      a.ppos[b] = reinterpret_cast<double*>(p);
      p += (size_t)S * 3 * 8;
      a.pmom[b] = p;
      p += (size_t)S * 3 * ts;
      a.pcov[b] = p;
      p += (size_t)S * 21 * ts;
    }
    p = reinterpret_cast<char*>(((uintptr_t)p + 7) & ~(uintptr_t)7);
    a.sel_chi2 = reinterpret_cast<double*>(p);
  }
  const int NC = cfg.max_cands;
  if ((e = c->b_rec.ensure((size_t)S * (NC * 16 + 4))) != hipSuccess) return hip_fail(c, e, "record workspace");
  {
    char* p = static_cast<char*>(c->b_rec.p);
    a.rchi = reinterpret_cast<double*>(p);
    p += (size_t)S * NC * 8;
    a.rhit = reinterpret_cast<int32_t*>(p);
    p += (size_t)S * NC * 4;
    a.rpos = reinterpret_cast<int32_t*>(p);
    p += (size_t)S * NC * 4;
    a.rcount = reinterpret_cast<int32_t*>(p);
  }
  const int64_t sp = std::max<int64_t>(a.sp, 1);
  if ((e = c->b_best.ensure((size_t)sp * (3 * 8 + 24 * ts + 8 + 4 + 4 + 4 + 4))) != hipSuccess)
    return hip_fail(c, e, "workspace");
  {
    char* p = static_cast<char*>(c->b_best.p);
    a.bpos = reinterpret_cast<double*>(p);
    p += (size_t)sp * 3 * 8;
    a.bchi2 = reinterpret_cast<double*>(p);
    p += (size_t)sp * 8;
    a.bmom = p;
    p += (size_t)sp * 3 * ts;
    a.bcov = p;
    p += (size_t)sp * 21 * ts;
    a.bmeta = reinterpret_cast<uint32_t*>(p);
    p += (size_t)sp * 4;
    a.bend = reinterpret_cast<int32_t*>(p);
    p += (size_t)sp * 4;
    a.brank = reinterpret_cast<int32_t*>(p);
    p += (size_t)sp * 4;
    a.sev = reinterpret_cast<int32_t*>(p);
  }
  a.seed_order = cfg.seed_order != 0 ? 1 : 0;
  if (a.seed_order) {
    // the seeds in sorted order (inputs and outputs), the key and the order
    const size_t NSL = (size_t)cfg.n_seed_layers;
    const size_t sort_bytes = (size_t)sp * (27 * ts + 1 + 4 * NSL + 4 + 4) + (size_t)sp * (4 * L + 27 * ts + 8 + 4 + 4 + 4) + 16 * 256;  // 15 pieces, each rounded up to 256 bytes
    if ((e = c->b_sort.ensure(sort_bytes)) != hipSuccess) return hip_fail(c, e, "seed order workspace");
    char* p = static_cast<char*>(c->b_sort.p);
    auto take = [&](size_t bytes) {
      char* r = p;
      p += (bytes + 255) / 256 * 256;
      return r;
    };
    a.src_state = a.seed_state;
    a.src_cov = a.seed_cov;
    a.src_q = a.q;
    a.src_seed_hit = a.seed_hit;
    a.seed_state = take((size_t)sp * 6 * ts);
    a.seed_cov = take((size_t)sp * 21 * ts);
    a.seed_hit = reinterpret_cast<int32_t*>(take((size_t)sp * 4 * NSL));
    a.skey = reinterpret_cast<int32_t*>(take((size_t)sp * 4));
    a.order = reinterpret_cast<int32_t*>(take((size_t)sp * 4));
    a.rank = reinterpret_cast<int32_t*>(take((size_t)sp * 4));
    a.o_hit = reinterpret_cast<int32_t*>(take((size_t)sp * 4 * L));
    a.o_state = take((size_t)sp * 6 * ts);
    a.o_cov = take((size_t)sp * 21 * ts);
    a.o_chi2 = reinterpret_cast<double*>(take((size_t)sp * 8));
    a.o_nhits = reinterpret_cast<int32_t*>(take((size_t)sp * 4));
    a.o_status = reinterpret_cast<uint32_t*>(take((size_t)sp * 4));
    a.q = reinterpret_cast<int8_t*>(take((size_t)sp));
    a.n_keys = kMaxKeys;
  }
  const size_t ctr_at = ((size_t)S * 4 + (size_t)sp * 2 + kCtrStride - 1) / kCtrStride * kCtrStride;
  if ((e = c->b_list.ensure((ctr_at + (size_t)L * kMaxRegions * kCtrStride) * 4)) != hipSuccess)
    return hip_fail(c, e, "list workspace");
  {
    int32_t* p = static_cast<int32_t*>(c->b_list.p);
    a.cinfo[0] = p;
    a.cinfo[1] = p + S;
    a.sel_parent = p + 2 * S;
    a.sel_hit = p + 3 * S;
    a.cstart[0] = p + 4 * S;
    a.cstart[1] = p + 4 * S + sp;
    a.ccount = reinterpret_cast<unsigned*>(p + ctr_at);
  }
  return KTF_OK;
}

static hipError_t record_done(ktf_ctx* c, hipStream_t st) {
  if (!c->build_done) {
    hipError_t e = hipEventCreateWithFlags(&c->build_done, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(c->build_done, st);
}

int build_impl(ktf_ctx* c, const ktf_event_batch* ev, ktf_build_out* out, hipStream_t st) {
  int rc = validate_batch(c, ev);
  if (rc) return rc;
  if (!out->hit_idx || !out->state || !out->cov || !out->chi2 || !out->n_hits || !out->status)
    return fail(c, KTF_EINVAL, "ktf_build: null output");
  BuildArgs a;
  if ((rc = prepare(c, ev, false, a, st))) return rc;
  const int L = c->cfg.n_layers, NC = c->cfg.max_cands;
  const int64_t sp = std::max<int64_t>(a.sp, 1);
  hipError_t e;
  // with the seed order on, the (parent, hit) records and the counts per
  // layer are kept in sorted order and copied to the caller's arrays at the
  // end if asked for; otherwise the caller's arrays are used directly
  if (out->cand_hist && !a.seed_order) {
    a.hist = out->cand_hist;
  } else {
    if ((e = c->b_hist.ensure(sizeof(int32_t) * (size_t)L * NC * 2 * sp)) != hipSuccess)
      return hip_fail(c, e, "history workspace");
    a.hist = static_cast<int32_t*>(c->b_hist.p);
  }
  if (out->cand_count && !a.seed_order) {
    a.count = out->cand_count;
  } else {
    if ((e = c->b_misc.ensure(sizeof(int32_t) * (size_t)L * sp)) != hipSuccess)
      return hip_fail(c, e, "count workspace");
    a.count = static_cast<int32_t*>(c->b_misc.p);
  }
  a.u_hist = a.seed_order ? out->cand_hist : nullptr;
  a.u_count = a.seed_order ? out->cand_count : nullptr;
  // the caller's copy of the (parent, hit) records reads -1 for unused
  // ranks; otherwise they are only ever read along written paths
  if (out->cand_hist) {
    const int64_t nh = (int64_t)L * NC * 2 * sp;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(nh, 256)), dim3(256), 0, st, a.hist, nh, -1);
  }
  // every count the build reads is written first (the seed fit's layers
  // for every seed, then each merge's layer), so only a caller's array,
  // pitch padding included, is cleared
  if (out->cand_count)
    hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk((int64_t)L * sp, 256)), dim3(256), 0, st, a.count,
                       (int64_t)L * sp, 0);
  a.u_hit = out->hit_idx;
  a.u_state = out->state;
  a.u_cov = out->cov;
  a.u_chi2 = out->chi2;
  a.u_nhits = out->n_hits;
  a.u_status = out->status;
  if (!a.seed_order) {  // the kernels write the caller's outputs directly
    a.o_hit = out->hit_idx;
    a.o_state = out->state;
    a.o_cov = out->cov;
    a.o_chi2 = out->chi2;
    a.o_nhits = out->n_hits;
    a.o_status = out->status;
  }
  e = ev->prec == KTF_FP64 ? run_build<double, double>(a, false, st) : run_build<float, float>(a, false, st);
  if (e == hipSuccess) e = record_done(c, st);
  return e == hipSuccess ? KTF_OK : hip_fail(c, e, "build launch");
}

int bin_impl(ktf_ctx* c, const ktf_event_batch* ev, int32_t* offsets, int32_t* perm, hipStream_t st) {
  int rc = validate_batch(c, ev);
  if (rc) return rc;
  BuildArgs a;
  if ((rc = prepare(c, ev, true, a, st))) return rc;
  hipError_t e = ev->prec == KTF_FP64 ? run_build<double, double>(a, true, st) : run_build<float, float>(a, true, st);
  if (e != hipSuccess) return hip_fail(c, e, "binning launch");
  const size_t ob = sizeof(int32_t) * (size_t)a.n_groups * (a.n_bins + 1);
  if ((e = hipMemcpyAsync(offsets, a.bin_off, ob, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(c, e, "copy offsets");
  if (a.n_hits > 0 &&
      (e = hipMemcpyAsync(perm, a.perm, sizeof(int32_t) * (size_t)a.n_hits, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(c, e, "copy perm");
  if ((e = record_done(c, st)) != hipSuccess) return hip_fail(c, e, "event record");
  return KTF_OK;
}

}  // namespace ktf

extern "C" int ktf_build(ktf_ctx* c, const ktf_event_batch* ev, ktf_build_out* out, void* st) {
  if (!c || !ev || !out) return KTF_EINVAL;
  return ktf::build_impl(c, ev, out, static_cast<hipStream_t>(st));
}

extern "C" int ktf_bin_hits(ktf_ctx* c, const ktf_event_batch* ev, int32_t* offsets, int32_t* perm,
                            void* st) {
  if (!c || !ev || !offsets || !perm) return KTF_EINVAL;
  return ktf::bin_impl(c, ev, offsets, perm, static_cast<hipStream_t>(st));
}
