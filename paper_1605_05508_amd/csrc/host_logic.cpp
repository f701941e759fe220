// host_logic.cpp -- host-only logic of the library (no HIP): argument
// checks, serving footprint, batch layouts and row copies.
#include "host_logic.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

namespace ktf {

// The precision field as the integer a C caller stored: a C++ load of an
// enum holding a value outside its enumerators is undefined.
static int prec_value(const ktf_precision& p) {
  static_assert(sizeof(ktf_precision) == sizeof(int), "enum size");
  int v;
  std::memcpy(&v, &p, sizeof v);
  return v;
}

const char* check_config(const ktf_config* cfg) {
  if (!cfg) return "null config";
  if (cfg->n_layers < 1 || cfg->n_layers > KTF_MAX_LAYERS) return "n_layers outside 1..KTF_MAX_LAYERS";
  if (!cfg->layer_r) return "null layer_r";
  for (int l = 0; l < cfg->n_layers; ++l)
    if (!(cfg->layer_r[l] > 0.0) || !std::isfinite(cfg->layer_r[l]) ||
        (l > 0 && !(cfg->layer_r[l] > cfg->layer_r[l - 1])))
      return "layer radii must be finite, positive and increasing";
  if (!std::isfinite(cfg->bz)) return "bz not finite";
  if (!(cfg->sigma_r > 0.0) || !(cfg->sigma_rphi > 0.0) || !(cfg->sigma_z > 0.0) || !std::isfinite(cfg->sigma_r) ||
      !std::isfinite(cfg->sigma_rphi) || !std::isfinite(cfg->sigma_z))
    return "hit resolutions must be finite and positive";
  if (cfg->max_cands < 1 || cfg->max_cands > KTF_MAX_CANDS) return "max_cands outside 1..KTF_MAX_CANDS";
  if (cfg->max_missed < 0) return "max_missed < 0";
  if (cfg->n_seed_layers < 1 || cfg->n_seed_layers > cfg->n_layers) return "n_seed_layers outside 1..n_layers";
  if (cfg->n_zbins < 1 || cfg->n_phibins < 1) return "bin counts must be positive";
  if (!(cfg->z_half > 0.0) || !std::isfinite(cfg->z_half)) return "z_half must be finite and positive";
  if (cfg->n_etabins < 0) return "n_etabins < 0";
  if (cfg->n_etabins > 0 && !(cfg->eta_max > 0.0 && std::isfinite(cfg->eta_max)))
    return "eta_max must be finite and positive with eta bins";
  const int64_t rows = cfg->n_etabins > 0 ? cfg->n_etabins : cfg->n_zbins;
  if (rows * (int64_t)cfg->n_phibins > INT32_MAX / 2) return "too many bins";
  if (cfg->layer_x0) {
    bool material = false;
    for (int l = 0; l < cfg->n_layers; ++l) {
      if (!(cfg->layer_x0[l] >= 0.0) || !std::isfinite(cfg->layer_x0[l]))
        return "layer_x0 must be finite and non-negative";
      material = material || cfg->layer_x0[l] > 0.0;
    }
    if (material && (!(cfg->mass > 0.0) || !(cfg->eloss_per_x0 >= 0.0) || !std::isfinite(cfg->mass) ||
                     !std::isfinite(cfg->eloss_per_x0)))
      return "material needs a finite positive mass and a finite non-negative energy loss";
  }
  return nullptr;
}

const char* check_fit_in(const ktf_fit_in* in, const ktf_fit_out* out) {
  if (!in || !out) return "null argument";
  if (in->n < 0 || in->pitch < in->n) return "need 0 <= n <= pitch";
  if (in->pitch > kMaxPitch) return "pitch above 2^40";
  const int prec = prec_value(in->prec);
  if (prec != KTF_FP64 && prec != KTF_FP32_BULK && prec != KTF_FP32_PROP) return "unknown precision";
  if (in->n_passes < 0 || in->n_passes > KTF_MAX_PASSES) return "n_passes outside 0..KTF_MAX_PASSES";
  if (in->n_passes > 1 && prec == KTF_FP32_BULK)
    return "the iterated refit needs a double covariance (KTF_FP64 or KTF_FP32_PROP)";
  if (in->n > 0 && (!in->seed_state || !in->seed_cov || !in->charge || !in->hits || !out->state || !out->cov ||
                    !out->chi2 || !out->n_upd || !out->status))
    return "null buffer";
  return nullptr;
}

const char* check_event_batch(const ktf_event_batch* ev, int L, int max_cands) {
  if (!ev || ev->n_events < 0 || !ev->seed_off || !ev->hit_off) return "bad event batch";
  const int prec = prec_value(ev->prec);
  if (prec != KTF_FP64 && prec != KTF_FP32_BULK) return "unknown precision";
  if (ev->seed_off[0] != 0 || ev->hit_off[0] != 0) return "offsets must start at 0";
  for (int e = 0; e < ev->n_events; ++e)
    if (ev->seed_off[e + 1] < ev->seed_off[e]) return "seed_off not monotone";
  const int64_t G = (int64_t)ev->n_events * L;
  for (int64_t g = 0; g < G; ++g) {
    if (ev->hit_off[g + 1] < ev->hit_off[g]) return "hit_off not monotone";
    if (ev->hit_off[g + 1] - ev->hit_off[g] > INT32_MAX) return "too many hits in one layer";
  }
  const int64_t ns = ev->seed_off[ev->n_events];
  const int64_t nh = ev->hit_off[G];
  if (ev->seed_pitch < ns || ev->hit_pitch < nh) return "pitch < size";
  if (ev->seed_pitch > kMaxPitch || ev->hit_pitch > kMaxPitch) return "pitch above 2^40";
  if (nh > INT32_MAX) return "more than 2^31 hits in one batch";
  if (ev->seed_pitch > INT32_MAX / max_cands) return "more than 2^31 candidate rows";
  if (ns > 0 && (!ev->seed_state || !ev->seed_cov || !ev->charge || !ev->seed_hit)) return "null seed buffer";
  if (nh > 0 && !ev->hits) return "null hits";
  return nullptr;
}

const char* check_event_host(const ktf_event_host* ev, int L) {
  if (!ev || !ev->hit_off) return "bad event";
  if (ev->n_seeds < 0 || ev->n_seeds > kMaxEventSeeds) return "n_seeds outside 0..2^31-1";
  const int prec = prec_value(ev->prec);
  if (prec != KTF_FP64 && prec != KTF_FP32_BULK) return "unknown precision";
  if (ev->hit_off[0] != 0) return "hit_off[0] != 0";
  for (int l = 0; l < L; ++l)
    if (ev->hit_off[l + 1] < ev->hit_off[l]) return "hit_off not monotone";
  if (ev->hit_off[L] > kMaxEventHits) return "more than 2^31-1 hits";
  const int64_t n = ev->n_seeds, nh = ev->hit_off[L];
  if ((n > 0 && (!ev->seed_state || !ev->seed_cov || !ev->charge || !ev->seed_hit)) || (nh > 0 && !ev->hits))
    return "null buffer";
  return nullptr;
}

size_t footprint_of(const ktf_config& cfg, int64_t n, int64_t nh, ktf_precision prec) {
  const size_t ts = prec == KTF_FP64 ? 8 : 4;
  const size_t L = cfg.n_layers, NC = cfg.max_cands;
  const size_t per_seed_in = 27 * ts + 1 + 4 * cfg.n_seed_layers;
  // candidate rows (the building's regions); per row: two candidate
  // buffers, two propagated-state buffers, records, the row lists (info x2,
  // parent, hit) and the child chi2
  const size_t per_row = 2 * (24 + 24 * ts + 12) + 2 * (24 + 24 * ts) + 16 * NC + 4 + 16 + 8;
  const size_t rows = (size_t)region_count(n, cfg.max_cands) * (size_t)region_rows(n, cfg.max_cands);
  const size_t per_seed_ws = L * NC * 8 + L * 4 + (24 + 24 * ts + 20) + 8;
  const size_t per_seed_fit = L * (3 * ts + 1) + 27 * ts + 16 + L * 4;
  const size_t counters = L * kMaxRegions * 128;
  const size_t bin_rows = cfg.n_etabins > 0 ? (size_t)cfg.n_etabins : (size_t)cfg.n_zbins;
  const size_t bins = L * (bin_rows * cfg.n_phibins * 8 + 8);
  return rows * per_row + (size_t)n * (per_seed_in + per_seed_ws + per_seed_fit) + (size_t)nh * (3 * ts * 2 + 8) +
         counters + bins;
}

InLayout in_layout(int E, int L, int NSL, int64_t N, int64_t H, size_t ts) {
  InLayout o;
  o.soff = 0;
  o.hoff = align256(o.soff + sizeof(int64_t) * (size_t)(E + 1));
  o.hits = align256(o.hoff + sizeof(int64_t) * ((size_t)E * L + 1));
  o.state = align256(o.hits + ts * 3 * (size_t)H);
  o.cov = align256(o.state + ts * 6 * (size_t)N);
  o.sh = align256(o.cov + ts * 21 * (size_t)N);
  o.q = align256(o.sh + sizeof(int32_t) * (size_t)NSL * N);
  o.total = align256(o.q + (size_t)N);
  return o;
}

OutLayout out_layout(int L, int64_t N, size_t ts) {
  OutLayout o;
  o.hit = 0;
  o.f_state = align256(o.hit + sizeof(int32_t) * (size_t)L * N);
  o.f_cov = align256(o.f_state + ts * 6 * (size_t)N);
  o.f_chi2 = align256(o.f_cov + ts * 21 * (size_t)N);
  o.f_nu = align256(o.f_chi2 + sizeof(double) * (size_t)N);
  o.f_st = align256(o.f_nu + sizeof(int32_t) * (size_t)N);
  o.host = align256(o.f_st + sizeof(uint32_t) * (size_t)N);
  o.b_state = o.host;
  o.b_cov = align256(o.b_state + ts * 6 * (size_t)N);
  o.b_chi2 = align256(o.b_cov + ts * 21 * (size_t)N);
  o.b_nh = align256(o.b_chi2 + sizeof(double) * (size_t)N);
  o.b_st = align256(o.b_nh + sizeof(int32_t) * (size_t)N);
  o.total = align256(o.b_st + sizeof(uint32_t) * (size_t)N);
  return o;
}

static void run_copy(const RowCopy& t) {
  if (t.n > 0) memcpy(t.dst, t.src, (size_t)t.n * t.size);
}

void run_copies(const std::vector<RowCopy>& rows) {
  size_t bytes = 0;
  for (const RowCopy& t : rows) bytes += (size_t)t.n * t.size;
  const int nt = bytes > ((size_t)4 << 20) ? 4 : 1;
  if (nt == 1) {
    for (const RowCopy& t : rows) run_copy(t);
    return;
  }
  // rows cut into pieces of at most 256K elements, dealt round robin
  std::vector<RowCopy> tasks;
  constexpr int64_t kPiece = 256 * 1024;
  for (const RowCopy& t : rows)
    for (int64_t o = 0; o < t.n; o += kPiece)
      tasks.push_back({static_cast<const char*>(t.src) + o * t.size, static_cast<char*>(t.dst) + o * t.size,
                       std::min(kPiece, t.n - o), t.size});
  std::vector<std::thread> th;
  for (int w = 1; w < nt; ++w)
    th.emplace_back([&tasks, w, nt] {
      for (size_t i = w; i < tasks.size(); i += nt) run_copy(tasks[i]);
    });
  for (size_t i = 0; i < tasks.size(); i += nt) run_copy(tasks[i]);
  for (std::thread& x : th) x.join();
}

void batch_offsets(const std::vector<EventRows>& ev, int L, std::vector<int64_t>& seed_off,
                   std::vector<int64_t>& hit_off) {
  const size_t E = ev.size();
  seed_off.assign(E + 1, 0);
  hit_off.assign(E * L + 1, 0);
  int64_t hb = 0;
  for (size_t e = 0; e < E; ++e) {
    seed_off[e + 1] = seed_off[e] + ev[e].n_seeds;
    for (int l = 0; l < L; ++l) hit_off[e * L + l] = hb + ev[e].hit_off[l];
    hb += ev[e].n_hits;
  }
  hit_off[E * L] = hb;
}

void pack_rows(const std::vector<EventRows>& ev, int L, int NSL, size_t ts, const std::vector<int64_t>& seed_off,
               const std::vector<int64_t>& hit_off, char* P, const InLayout& in, std::vector<RowCopy>& out) {
  const int E = (int)ev.size();
  const int64_t N = std::max<int64_t>(seed_off[E], 1), H = std::max<int64_t>(hit_off[(size_t)E * L], 1);
  const int sz = (int)ts;
  out.push_back({seed_off.data(), P + in.soff, E + 1, 8});
  out.push_back({hit_off.data(), P + in.hoff, (int64_t)E * L + 1, 8});
  char* hh = P + in.hits;
  char* st = P + in.state;
  char* cv = P + in.cov;
  int32_t* sh = reinterpret_cast<int32_t*>(P + in.sh);
  int8_t* qq = reinterpret_cast<int8_t*>(P + in.q);
  int64_t sb = 0, hb = 0;
  for (const EventRows& r : ev) {
    const int64_t n = r.n_seeds, nh = r.n_hits;
    const char* eh = static_cast<const char*>(r.hits);
    const char* es = static_cast<const char*>(r.state);
    const char* ec = static_cast<const char*>(r.cov);
    // rows of the event into rows of the batch
    for (int k = 0; k < 3; ++k) out.push_back({eh + ts * (k * nh), hh + ts * (k * H + hb), nh, sz});
    for (int k = 0; k < 6; ++k) out.push_back({es + ts * (k * n), st + ts * (k * N + sb), n, sz});
    for (int k = 0; k < 21; ++k) out.push_back({ec + ts * (k * n), cv + ts * (k * N + sb), n, sz});
    for (int k = 0; k < NSL; ++k) out.push_back({r.seed_hit + k * n, sh + k * N + sb, n, 4});
    out.push_back({r.q, qq + sb, n, 1});
    sb += n;
    hb += nh;
  }
}

void unpack_rows(const std::vector<int64_t>& n_seeds, const std::vector<ResultRows>& res, int L, size_t ts,
                 int64_t N, const char* O, const OutLayout& ol, std::vector<RowCopy>& out) {
  const int sz = (int)ts;
  const int32_t* hit = reinterpret_cast<const int32_t*>(O + ol.hit);
  const char* st = O + ol.f_state;
  const char* cv = O + ol.f_cov;
  const double* c2 = reinterpret_cast<const double*>(O + ol.f_chi2);
  const int32_t* nu = reinterpret_cast<const int32_t*>(O + ol.f_nu);
  const uint32_t* ss = reinterpret_cast<const uint32_t*>(O + ol.f_st);
  int64_t sb = 0;
  for (size_t e = 0; e < res.size(); ++e) {
    const int64_t n = n_seeds[e];
    const ResultRows& r = res[e];
    char* rs = static_cast<char*>(r.state);
    char* rc = static_cast<char*>(r.cov);
    for (int l = 0; l < L; ++l) out.push_back({hit + l * N + sb, r.hit + l * n, n, 4});
    for (int k = 0; k < 6; ++k) out.push_back({st + ts * (k * N + sb), rs + ts * (k * n), n, sz});
    for (int k = 0; k < 21; ++k) out.push_back({cv + ts * (k * N + sb), rc + ts * (k * n), n, sz});
    out.push_back({c2 + sb, r.chi2, n, 8});
    out.push_back({nu + sb, r.n_hits, n, 4});
    out.push_back({ss + sb, r.status, n, 4});
    sb += n;
  }
}

}  // namespace ktf
