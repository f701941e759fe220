// serve.hip -- continuous-batching request loop: events arrive on the host,
// are admitted onto the device as stream lanes and HBM budget free up, run
// building + final fit there, and are collected by ticket.
//
// The paper's pipeline per event is seeding -> building -> fitting (Sec. 2);
// here seeds come with the event, building and the final fit run on the
// GPU.  Each lane owns a stream and a private workspace (a sub-context), so
// batches on different lanes overlap on the device while new arrivals wait
// only for a free lane and budget, not for the whole queue to drain.
// Per-seed arithmetic never mixes seeds or events, so an event's result is
// identical whichever batch it runs in.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>

#include "ctx.hpp"
#include "kf_math.hpp"

namespace ktf {

constexpr int kLanes = 4;                 // streams with their own workspace
constexpr size_t kPoolEvents = 16;        // collected events kept for reuse
constexpr size_t kPoolEventBytes = 64ull << 20;  // ... each holding at most this much host memory
constexpr int64_t kMaxBatchSeeds = 131072;  // bound on one batch's work (latency)

// A host buffer that keeps its pages between events: grown geometrically
// and never zero-filled, so a reused event neither allocates nor faults.
template <typename T>
struct HostBuf {
  std::unique_ptr<T[]> p;
  size_t cap = 0;
  T* get(size_t n) {
    if (n > cap) {
      const size_t c = std::max(n, cap + cap / 2);
      p.reset(new T[c]);
      cap = c;
    }
    return p.get();
  }
  T* data() const { return p.get(); }
  size_t bytes() const { return cap * sizeof(T); }
};

// An event's host copies.  Coordinates, states and covariances are kept in
// the event's own precision (float for KTF_FP32_BULK, double for KTF_FP64),
// as bytes: a batch holds events of one precision, so every copy between an
// event and a batch is a plain row copy.
struct ServeEvent {
  uint64_t ticket = 0;
  int64_t n_seeds = 0, n_hits = 0;
  ktf_precision prec = KTF_FP32_BULK;
  size_t ts = 4;                 // bytes of one value: 8 for KTF_FP64, else 4
  std::vector<int64_t> hit_off;  // [L+1]
  HostBuf<unsigned char> hits;   // [3][n_hits] values
  HostBuf<unsigned char> state;  // [6][n]
  HostBuf<unsigned char> cov;    // [21][n]
  HostBuf<int8_t> q;
  HostBuf<int32_t> seed_hit;     // [nsl][n]
  size_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool done = false;
  int error = 0;
  bool fail_injected = false;    // ktf_debug_fail_next_event: fail at launch
  bool solo = false;             // run in a batch of its own (after a batch failed)
  // results
  HostBuf<int32_t> r_hit;        // [L][n]
  HostBuf<unsigned char> r_state, r_cov;  // [6][n], [21][n] values
  HostBuf<double> r_chi2;
  HostBuf<int32_t> r_nh;
  HostBuf<uint32_t> r_st;
  size_t held_bytes() const {
    return hits.bytes() + state.bytes() + cov.bytes() + q.bytes() + seed_hit.bytes() + r_hit.bytes() +
           r_state.bytes() + r_cov.bytes() + r_chi2.bytes() + r_nh.bytes() + r_st.bytes();
  }
};

struct Lane {
  hipStream_t stream = nullptr;
  ktf_ctx* sub = nullptr;        // private workspace for build and fit
  DevBuf in, out, fitin;
  void* pin_in = nullptr;
  size_t pin_in_bytes = 0;
  void* pin_out = nullptr;
  size_t pin_out_bytes = 0;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<ServeEvent*> batch;
  ktf_precision prec = KTF_FP32_BULK;
  int64_t N = 0;
  std::vector<int64_t> seed_off;
};

struct ServeState {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<ServeEvent*> queue;
  std::map<uint64_t, ServeEvent*> tickets;
  // collected events kept for reuse with their host buffers (at most
  // kPoolEvents of them)
  std::vector<ServeEvent*> pool;
  Lane lanes[kLanes];
  uint64_t next_ticket = 1;
  size_t inflight_bytes = 0;
  int64_t n_inflight = 0, n_done = 0;
  bool stop = false;
  bool fail_next = false;  // ktf_debug_fail_next_event armed
  std::string error;
  std::thread th;
};

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// device bytes an event holds while in flight: inputs, outputs and its
// share of the lane workspace (candidates, records, bins)
static size_t footprint_of(const ktf_config& cfg, int64_t n, int64_t nh, ktf_precision prec) {
  const size_t ts = prec == KTF_FP64 ? 8 : 4;
  const size_t L = cfg.n_layers, NC = cfg.max_cands;
  const size_t per_seed_in = 27 * ts + 1 + 4 * cfg.n_seed_layers;
  // candidate rows: max_cands per seed plus the slack of the 64 row regions
  // per row: two candidate buffers, two propagated-state buffers, records,
  // the row lists (seed x2, parent, hit) and the child chi2
  const size_t per_row = 2 * (24 + 24 * ts + 12) + 2 * (24 + 24 * ts) + 16 * NC + 4 + 16 + 8;
  const size_t rows = (size_t)n * NC + 64 * 257;
  const size_t per_seed_ws = L * NC * 8 + L * 4 + (24 + 24 * ts + 20) + 8;
  const size_t per_seed_fit = L * (3 * ts + 1) + 27 * ts + 16 + L * 4;
  const size_t bin_rows = cfg.n_etabins > 0 ? (size_t)cfg.n_etabins : (size_t)cfg.n_zbins;
  const size_t bins = L * (bin_rows * cfg.n_phibins * 8 + 8);
  return rows * per_row + (size_t)n * (per_seed_in + per_seed_ws + per_seed_fit) +
         (size_t)nh * (3 * ts * 2 + 8) + bins;
}

// --------------------------------------------------------------- kernels
// fit inputs from the built tracks: the hit coordinates each seed took on
// each layer, and a valid flag
template <typename TS>
__global__ void gather_fit_inputs(int64_t N, int L, int E, const int64_t* seed_off,
                                  const int64_t* hit_off, const TS* hits, int64_t hp,
                                  const int32_t* hit_idx, TS* fh, uint8_t* valid) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  int lo = 0, hi = E;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seed_off[mid] <= s) lo = mid; else hi = mid;
  }
  const int e = lo;
  for (int l = 0; l < L; ++l) {
    const int32_t h = hit_idx[(int64_t)l * N + s];
    TS x = TS(0), y = TS(0), z = TS(0);
    if (h >= 0) {
      const int64_t j = hit_off[(int64_t)e * L + l] + h;
      x = hits[j];
      y = hits[hp + j];
      z = hits[2 * hp + j];
    }
    fh[((int64_t)l * 3 + 0) * N + s] = x;
    fh[((int64_t)l * 3 + 1) * N + s] = y;
    fh[((int64_t)l * 3 + 2) * N + s] = z;
    valid[(int64_t)l * N + s] = h >= 0 ? 1 : 0;
  }
}

__global__ void or_status(int64_t N, uint32_t* a, const uint32_t* b) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < N) a[s] |= b[s];
}

// ------------------------------------------------------------- batching
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// pinned staging of a lane, grown geometrically like the device buffers
// (pinning host memory takes milliseconds)
static hipError_t ensure_pinned(void** p, size_t* have, size_t want) {
  if (*have >= want) return hipSuccess;
  size_t b = std::max(want + want / 4, 2 * *have);
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipHostMalloc(p, b, 0);
  if (e != hipSuccess && b > want + want / 4) {  // the doubling does not fit: the request alone
    (void)hipGetLastError();
    b = want + want / 4;
    e = hipHostMalloc(p, b, 0);
  }
  if (e == hipSuccess) *have = b;
  return e;
}

// Row copies between an event's host arrays and a batch's pinned staging.
// A large batch's rows take a millisecond or more on one core, on the
// path of every event in it, so above a few MB they are spread over a few
// host threads.
struct RowCopy {
  const void* src;
  void* dst;
  int64_t n;     // elements
  int size;      // bytes per element
};

static void run_copy(const RowCopy& t) { memcpy(t.dst, t.src, (size_t)t.n * t.size); }

static void run_copies(const std::vector<RowCopy>& rows) {
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

// Byte offsets of a batch's outputs in the lane's output buffer: the part
// the host reads (hit indices and the final fit's results) comes first and
// is the only part copied back; the building's own fit outputs follow.
struct OutLayout {
  size_t hit, f_state, f_cov, f_chi2, f_nu, f_st, host;
  size_t b_state, b_cov, b_chi2, b_nh, b_st, total;
};

template <typename TS>
static OutLayout out_layout(int L, int64_t Np) {
  OutLayout o;
  o.hit = 0;
  o.f_state = align256(o.hit + sizeof(int32_t) * L * Np);
  o.f_cov = align256(o.f_state + sizeof(TS) * 6 * Np);
  o.f_chi2 = align256(o.f_cov + sizeof(TS) * 21 * Np);
  o.f_nu = align256(o.f_chi2 + sizeof(double) * Np);
  o.f_st = align256(o.f_nu + sizeof(int32_t) * Np);
  o.host = align256(o.f_st + sizeof(uint32_t) * Np);
  o.b_state = o.host;
  o.b_cov = align256(o.b_state + sizeof(TS) * 6 * Np);
  o.b_chi2 = align256(o.b_cov + sizeof(TS) * 21 * Np);
  o.b_nh = align256(o.b_chi2 + sizeof(double) * Np);
  o.b_st = align256(o.b_nh + sizeof(int32_t) * Np);
  o.total = align256(o.b_st + sizeof(uint32_t) * Np);
  return o;
}

template <typename TS>
static int launch_batch_t(ktf_ctx* c, Lane& ln) {
  const ktf_config& cfg = c->cfg;
  const int L = cfg.n_layers, NSL = cfg.n_seed_layers;
  const int E = (int)ln.batch.size();
  int64_t N = 0, H = 0;
  for (ServeEvent* ev : ln.batch) {
    // a failure forced from the host for tests of isolation: before any
    // device work of the batch is enqueued, as a launch failure would be
    if (ev->fail_injected) return fail(c, KTF_EDEVICE, "serve: injected failure (ktf_debug_fail_next_event)");
    N += ev->n_seeds;
    H += ev->n_hits;
  }
  ln.N = N;
  const int64_t Np = std::max<int64_t>(N, 1), Hp = std::max<int64_t>(H, 1);
  // packed inputs: offsets, hits [3][H], state [6][N], cov [21][N], seed_hit, q
  std::vector<int64_t> hoff((size_t)E * L + 1);
  ln.seed_off.assign(E + 1, 0);
  {
    int64_t hb = 0;
    for (int e = 0; e < E; ++e) {
      ServeEvent* ev = ln.batch[e];
      ln.seed_off[e + 1] = ln.seed_off[e] + ev->n_seeds;
      for (int l = 0; l < L; ++l) hoff[(size_t)e * L + l] = hb + ev->hit_off[l];
      hb += ev->n_hits;
    }
    hoff[(size_t)E * L] = hb;
  }
  size_t o_soff = 0;
  size_t o_hoff = align256(o_soff + sizeof(int64_t) * (E + 1));
  size_t o_hits = align256(o_hoff + sizeof(int64_t) * hoff.size());
  size_t o_state = align256(o_hits + sizeof(TS) * 3 * Hp);
  size_t o_cov = align256(o_state + sizeof(TS) * 6 * Np);
  size_t o_sh = align256(o_cov + sizeof(TS) * 21 * Np);
  size_t o_q = align256(o_sh + sizeof(int32_t) * NSL * Np);
  size_t in_bytes = align256(o_q + Np);
  hipError_t e;
  if ((e = ensure_pinned(&ln.pin_in, &ln.pin_in_bytes, in_bytes)) != hipSuccess) return hip_fail(c, e, "serve staging");
  if ((e = ln.in.ensure(in_bytes)) != hipSuccess) return hip_fail(c, e, "serve inputs");
  char* P = static_cast<char*>(ln.pin_in);
  memcpy(P + o_soff, ln.seed_off.data(), sizeof(int64_t) * (E + 1));
  memcpy(P + o_hoff, hoff.data(), sizeof(int64_t) * hoff.size());
  {
    TS* hh = reinterpret_cast<TS*>(P + o_hits);
    TS* st = reinterpret_cast<TS*>(P + o_state);
    TS* cv = reinterpret_cast<TS*>(P + o_cov);
    int32_t* sh = reinterpret_cast<int32_t*>(P + o_sh);
    int8_t* qq = reinterpret_cast<int8_t*>(P + o_q);
    int64_t sb = 0, hb = 0;
    std::vector<RowCopy> tasks;
    for (ServeEvent* ev : ln.batch) {
      const int64_t n = ev->n_seeds, nh = ev->n_hits;
      // rows of the event into rows of the batch
      const TS* eh = reinterpret_cast<const TS*>(ev->hits.data());
      const TS* es = reinterpret_cast<const TS*>(ev->state.data());
      const TS* ec = reinterpret_cast<const TS*>(ev->cov.data());
      for (int k = 0; k < 3; ++k) tasks.push_back({eh + k * nh, hh + k * H + hb, nh, (int)sizeof(TS)});
      for (int k = 0; k < 6; ++k) tasks.push_back({es + k * n, st + k * N + sb, n, (int)sizeof(TS)});
      for (int k = 0; k < 21; ++k) tasks.push_back({ec + k * n, cv + k * N + sb, n, (int)sizeof(TS)});
      for (int k = 0; k < NSL; ++k) tasks.push_back({ev->seed_hit.data() + k * n, sh + k * N + sb, n, 4});
      tasks.push_back({ev->q.data(), qq + sb, n, 1});
      sb += n;
      hb += nh;
    }
    run_copies(tasks);
  }
  if ((e = hipMemcpyAsync(ln.in.p, P, in_bytes, hipMemcpyHostToDevice, ln.stream)) != hipSuccess)
    return hip_fail(c, e, "serve H2D");
  char* D = static_cast<char*>(ln.in.p);

  // outputs of building and fit: what goes back to the host first (hit
  // indices, the fit's results), then the building's own fit outputs
  const OutLayout ol = out_layout<TS>(L, Np);
  const size_t b_hit = ol.hit, f_state = ol.f_state, f_cov = ol.f_cov, f_chi2 = ol.f_chi2, f_nu = ol.f_nu,
               f_st = ol.f_st, b_state = ol.b_state, b_cov = ol.b_cov, b_chi2 = ol.b_chi2, b_nh = ol.b_nh,
               b_st = ol.b_st, out_bytes = ol.total;
  if ((e = ln.out.ensure(out_bytes)) != hipSuccess) return hip_fail(c, e, "serve outputs");
  char* O = static_cast<char*>(ln.out.p);
  ktf_event_batch bt;
  bt.n_events = E;
  bt.seed_off = ln.seed_off.data();
  bt.hit_off = hoff.data();
  bt.hit_pitch = H;
  bt.hits = D + o_hits;
  bt.seed_pitch = N;
  bt.seed_state = D + o_state;
  bt.seed_cov = D + o_cov;
  bt.charge = reinterpret_cast<const int8_t*>(D + o_q);
  bt.seed_hit = reinterpret_cast<const int32_t*>(D + o_sh);
  bt.prec = sizeof(TS) == 8 ? KTF_FP64 : KTF_FP32_BULK;
  ktf_build_out bo;
  memset(&bo, 0, sizeof bo);
  bo.hit_idx = reinterpret_cast<int32_t*>(O + b_hit);
  bo.state = O + b_state;
  bo.cov = O + b_cov;
  bo.chi2 = reinterpret_cast<double*>(O + b_chi2);
  bo.n_hits = reinterpret_cast<int32_t*>(O + b_nh);
  bo.status = reinterpret_cast<uint32_t*>(O + b_st);
  int rc = build_impl(ln.sub, &bt, &bo, ln.stream);
  if (rc) return fail(c, rc, "serve build: %s", ln.sub->last_error.c_str());

  // final fit over the hits each seed took
  size_t fin_h = 0;
  size_t fin_v = align256(fin_h + sizeof(TS) * (size_t)L * 3 * Np);
  size_t fin_bytes = align256(fin_v + (size_t)L * Np);
  if ((e = ln.fitin.ensure(fin_bytes)) != hipSuccess) return hip_fail(c, e, "serve fit inputs");
  char* FI = static_cast<char*>(ln.fitin.p);
  if (N > 0) {
    hipLaunchKernelGGL((gather_fit_inputs<TS>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, ln.stream, N,
                       L, E, reinterpret_cast<const int64_t*>(D + o_soff),
                       reinterpret_cast<const int64_t*>(D + o_hoff), reinterpret_cast<const TS*>(D + o_hits),
                       H, bo.hit_idx, reinterpret_cast<TS*>(FI + fin_h), reinterpret_cast<uint8_t*>(FI + fin_v));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "serve gather");
    ktf_fit_in fi{N, N, bt.prec, D + o_state, D + o_cov, bt.charge, FI + fin_h,
                  reinterpret_cast<const uint8_t*>(FI + fin_v), 1};  // one pass
    ktf_fit_out fo{O + f_state, O + f_cov, reinterpret_cast<double*>(O + f_chi2),
                   reinterpret_cast<int32_t*>(O + f_nu), reinterpret_cast<uint32_t*>(O + f_st)};
    rc = ktf_fit(ln.sub, &fi, &fo, KTF_FIT_FUSED, ln.stream);
    if (rc) return fail(c, rc, "serve fit: %s", ln.sub->last_error.c_str());
    hipLaunchKernelGGL(or_status, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, ln.stream, N,
                       reinterpret_cast<uint32_t*>(O + f_st), bo.status);
  }
  // results back: hit indices and the fit's outputs
  if ((e = ensure_pinned(&ln.pin_out, &ln.pin_out_bytes, ol.host)) != hipSuccess) return hip_fail(c, e, "serve staging");
  if ((e = hipMemcpyAsync(ln.pin_out, O, ol.host, hipMemcpyDeviceToHost, ln.stream)) != hipSuccess)
    return hip_fail(c, e, "serve D2H");
  if ((e = hipEventRecord(ln.done, ln.stream)) != hipSuccess) return hip_fail(c, e, "serve event");
  // remember the layout for unpacking
  ln.busy = true;
  return KTF_OK;
}

template <typename TS>
static void unpack_batch_t(ktf_ctx* c, Lane& ln) {
  const int L = c->cfg.n_layers;
  const int64_t N = ln.N, Np = std::max<int64_t>(N, 1);
  const OutLayout ol = out_layout<TS>(L, Np);
  const char* O = static_cast<const char*>(ln.pin_out);
  const int32_t* hit = reinterpret_cast<const int32_t*>(O + ol.hit);
  const TS* st = reinterpret_cast<const TS*>(O + ol.f_state);
  const TS* cv = reinterpret_cast<const TS*>(O + ol.f_cov);
  const double* c2 = reinterpret_cast<const double*>(O + ol.f_chi2);
  const int32_t* nu = reinterpret_cast<const int32_t*>(O + ol.f_nu);
  const uint32_t* ss = reinterpret_cast<const uint32_t*>(O + ol.f_st);
  int64_t sb = 0;
  std::vector<RowCopy> tasks;
  for (ServeEvent* ev : ln.batch) {
    const int64_t n = ev->n_seeds;
    int32_t* r_hit = ev->r_hit.get((size_t)L * n);
    TS* r_state = reinterpret_cast<TS*>(ev->r_state.get(sizeof(TS) * 6 * n));
    TS* r_cov = reinterpret_cast<TS*>(ev->r_cov.get(sizeof(TS) * 21 * n));
    for (int l = 0; l < L; ++l) tasks.push_back({hit + l * N + sb, r_hit + l * n, n, 4});
    for (int k = 0; k < 6; ++k) tasks.push_back({st + k * N + sb, r_state + k * n, n, (int)sizeof(TS)});
    for (int k = 0; k < 21; ++k) tasks.push_back({cv + k * N + sb, r_cov + k * n, n, (int)sizeof(TS)});
    tasks.push_back({c2 + sb, ev->r_chi2.get(n), n, 8});
    tasks.push_back({nu + sb, ev->r_nh.get(n), n, 4});
    tasks.push_back({ss + sb, ev->r_st.get(n), n, 4});
    sb += n;
  }
  run_copies(tasks);
}

static void scheduler(ktf_ctx* c) {
  ServeState* S = c->serve;
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    bool progressed = false;
    // retire finished batches
    for (Lane& ln : S->lanes) {
      if (!ln.busy) continue;
      hipError_t q = hipEventQuery(ln.done);
      if (q == hipErrorNotReady) continue;
      if (q == hipSuccess) {
        // the lane and its events' result buffers belong to this thread
        // until the events are marked done: submissions and polls go on
        lk.unlock();
        if (ln.prec == KTF_FP64) unpack_batch_t<double>(c, ln); else unpack_batch_t<float>(c, ln);
        lk.lock();
      }
      const double t = now_s();  // the results can be collected from here on
      for (ServeEvent* ev : ln.batch) {
        ev->done = true;
        ev->error = q == hipSuccess ? 0 : KTF_EDEVICE;
        ev->t_done = t;
        S->inflight_bytes -= ev->footprint;
        --S->n_inflight;
        ++S->n_done;
      }
      ln.batch.clear();
      ln.busy = false;
      progressed = true;
    }
    // admit queued events onto idle lanes, oldest first
    for (Lane& ln : S->lanes) {
      if (ln.busy || S->queue.empty()) continue;
      const ktf_precision prec = S->queue.front()->prec;
      int64_t seeds = 0;
      while (!S->queue.empty()) {
        ServeEvent* ev = S->queue.front();
        if (ev->prec != prec) break;
        if (!ln.batch.empty() && (ev->solo || ln.batch.front()->solo)) break;
        if (S->n_inflight >= c->cfg.max_inflight) break;
        if (S->inflight_bytes + ev->footprint > c->cfg.hbm_budget_bytes) break;
        if (!ln.batch.empty() && seeds + ev->n_seeds > kMaxBatchSeeds) break;
        S->queue.pop_front();
        ev->t_admit = now_s();
        S->inflight_bytes += ev->footprint;
        ++S->n_inflight;
        seeds += ev->n_seeds;
        ln.batch.push_back(ev);
      }
      if (ln.batch.empty()) break;  // budget or slots exhausted
      ln.prec = prec;
      lk.unlock();
      int rc = prec == KTF_FP64 ? launch_batch_t<double>(c, ln) : launch_batch_t<float>(c, ln);
      lk.lock();
      // a failed launch may have enqueued part of the batch's copies: the
      // lane's staging is reused only once they are done
      if (rc) (void)hipStreamSynchronize(ln.stream);
      if (rc && ln.batch.size() > 1) {
        // one event must not fail the others: every event of the batch goes
        // back to the front of the queue (in order) to run alone
        for (auto it = ln.batch.rbegin(); it != ln.batch.rend(); ++it) {
          ServeEvent* ev = *it;
          ev->solo = true;
          S->inflight_bytes -= ev->footprint;
          --S->n_inflight;
          S->queue.push_front(ev);
        }
        ln.batch.clear();
        ln.busy = false;
      } else if (rc) {  // fail this event, keep serving
        for (ServeEvent* ev : ln.batch) {
          ev->done = true;
          ev->error = rc;
          ev->t_done = now_s();
          S->inflight_bytes -= ev->footprint;
          --S->n_inflight;
          ++S->n_done;
        }
        ln.batch.clear();
        ln.busy = false;
      }
      progressed = true;
    }
    if (progressed) {
      S->cv.notify_all();
      continue;
    }
    bool any_busy = false;
    for (Lane& ln : S->lanes) any_busy |= ln.busy;
    // poll the device briskly while work is in flight; otherwise sleep
    // until a submission arrives
    if (any_busy)
      S->cv.wait_for(lk, std::chrono::microseconds(50));
    else
      S->cv.wait_for(lk, std::chrono::milliseconds(20));
  }
}

// The serving state is created by the first ktf_submit on a context; the
// context's serve_mu makes concurrent first submissions create it once.
static int ensure_serving(ktf_ctx* c) {
  std::lock_guard<std::mutex> g(c->serve_mu);
  if (c->serve) return KTF_OK;
  ServeState* S = new ServeState();
  for (Lane& ln : S->lanes) {
    hipError_t e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ln.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      delete S;
      return hip_fail(c, e, "serve lanes");
    }
    ktf_config cfg = c->cfg;
    if (ktf_create(&cfg, &ln.sub) != KTF_OK) {
      delete S;
      return fail(c, KTF_EDEVICE, "serve: sub-context");
    }
  }
  c->serve = S;
  S->th = std::thread(scheduler, c);
  return KTF_OK;
}

void serve_shutdown(ktf_ctx* c) {
  std::lock_guard<std::mutex> g(c->serve_mu);
  ServeState* S = c->serve;
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  for (Lane& ln : S->lanes) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    ln.in.release();
    ln.out.release();
    ln.fitin.release();
    if (ln.pin_in) (void)hipHostFree(ln.pin_in);
    if (ln.pin_out) (void)hipHostFree(ln.pin_out);
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
    if (ln.sub) ktf_destroy(ln.sub);
  }
  for (auto& kv : S->tickets) delete kv.second;
  for (ServeEvent* e : S->pool) delete e;
  delete S;
  c->serve = nullptr;
}

}  // namespace ktf

using namespace ktf;

extern "C" {

double ktf_now(void) { return now_s(); }

int ktf_submit(ktf_ctx* c, const ktf_event_host* ev, uint64_t* ticket) {
  const double t_entry = now_s();  // latency counts the copy-in below
  if (!c || !ev || !ticket) return KTF_EINVAL;
  const ktf_config& cfg = c->cfg;
  const int L = cfg.n_layers, NSL = cfg.n_seed_layers;
  if (ev->n_seeds < 0 || !ev->hit_off || (ev->prec != KTF_FP64 && ev->prec != KTF_FP32_BULK))
    return fail(c, KTF_EINVAL, "ktf_submit: bad event");
  if (ev->hit_off[0] != 0) return fail(c, KTF_EINVAL, "ktf_submit: hit_off[0] != 0");
  for (int l = 0; l < L; ++l)
    if (ev->hit_off[l + 1] < ev->hit_off[l]) return fail(c, KTF_EINVAL, "ktf_submit: hit_off not monotone");
  const int64_t n = ev->n_seeds, nh = ev->hit_off[L];
  if ((n > 0 && (!ev->seed_state || !ev->seed_cov || !ev->charge || !ev->seed_hit)) || (nh > 0 && !ev->hits))
    return fail(c, KTF_EINVAL, "ktf_submit: null buffer");
  const size_t fp = footprint_of(cfg, n, nh, ev->prec);
  const size_t ts = ev->prec == KTF_FP64 ? 8 : 4;
  if (fp > cfg.hbm_budget_bytes)
    return fail(c, KTF_ENOMEM, "ktf_submit: event needs %zu bytes, budget %llu", fp,
                (unsigned long long)cfg.hbm_budget_bytes);
  int rc = ensure_serving(c);
  if (rc) return rc;
  ServeState* S = c->serve;
  ServeEvent* e = nullptr;
  {
    // a collected event whose buffers already hold this one's hits, else
    // the largest one kept
    std::lock_guard<std::mutex> g(S->mu);
    const size_t need = (size_t)(3 * nh);
    int fit = -1, big = -1;
    for (int i = 0; i < (int)S->pool.size(); ++i) {
      const size_t cap = S->pool[i]->hits.cap;
      if (cap >= need && (fit < 0 || cap < S->pool[fit]->hits.cap)) fit = i;
      if (big < 0 || cap > S->pool[big]->hits.cap) big = i;
    }
    const int pick = fit >= 0 ? fit : big;
    if (pick >= 0) {
      e = S->pool[pick];
      S->pool[pick] = S->pool.back();
      S->pool.pop_back();
    }
  }
  if (!e) e = new ServeEvent();
  e->done = false;
  e->error = 0;
  e->t_admit = e->t_done = 0;
  e->solo = false;
  e->n_seeds = n;
  e->n_hits = nh;
  e->prec = ev->prec;
  e->ts = ts;
  e->hit_off.assign(ev->hit_off, ev->hit_off + L + 1);
  run_copies({{ev->hits, e->hits.get(ts * 3 * nh), 3 * nh, (int)ts},
              {ev->seed_state, e->state.get(ts * 6 * n), 6 * n, (int)ts},
              {ev->seed_cov, e->cov.get(ts * 21 * n), 21 * n, (int)ts},
              {ev->charge, e->q.get(n), n, 1},
              {ev->seed_hit, e->seed_hit.get((size_t)NSL * n), (int64_t)NSL * n, 4}});
  e->footprint = fp;
  e->t_submit = t_entry;
  {
    std::lock_guard<std::mutex> g(S->mu);
    e->fail_injected = S->fail_next;
    S->fail_next = false;
    e->ticket = S->next_ticket++;
    S->tickets[e->ticket] = e;
    S->queue.push_back(e);
  }
  S->cv.notify_all();
  *ticket = e->ticket;
  return KTF_OK;
}

int ktf_poll(ktf_ctx* c, uint64_t ticket, ktf_result_host* out) {
  if (!c || !out) return KTF_EINVAL;
  ServeState* S = c->serve;
  if (!S) return fail(c, KTF_ENOTFOUND, "ktf_poll: unknown ticket");
  ServeEvent* e;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(c, KTF_ENOTFOUND, "ktf_poll: unknown ticket");
    e = it->second;
    if (!e->done) return KTF_EAGAIN;
    S->tickets.erase(it);
    --S->n_done;
  }
  const int rc = e->error;
  if (rc == 0) {
    const int L = c->cfg.n_layers;
    const int64_t n = e->n_seeds;
    if (out->hit_idx) memcpy(out->hit_idx, e->r_hit.data(), sizeof(int32_t) * L * n);
    if (out->state) memcpy(out->state, e->r_state.data(), e->ts * 6 * n);
    if (out->cov) memcpy(out->cov, e->r_cov.data(), e->ts * 21 * n);
    if (out->chi2) memcpy(out->chi2, e->r_chi2.data(), sizeof(double) * n);
    if (out->n_hits) memcpy(out->n_hits, e->r_nh.data(), sizeof(int32_t) * n);
    if (out->status) memcpy(out->status, e->r_st.data(), sizeof(uint32_t) * n);
  }
  out->t_submit = e->t_submit;
  out->t_admit = e->t_admit;
  out->t_done = e->t_done;
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->pool.size() < kPoolEvents && e->held_bytes() <= kPoolEventBytes) {
      S->pool.push_back(e);
      e = nullptr;
    }
  }
  delete e;
  return rc ? fail(c, rc, "ktf_poll: event failed on the device") : KTF_OK;
}

int ktf_debug_fail_next_event(ktf_ctx* c) {
  if (!c) return KTF_EINVAL;
  int rc = ensure_serving(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->serve->mu);
  c->serve->fail_next = true;
  return KTF_OK;
}

int ktf_serving_stats(ktf_ctx* c, int64_t* queued, int64_t* inflight, int64_t* done) {
  if (!c) return KTF_EINVAL;
  ServeState* S = c->serve;
  int64_t q = 0, f = 0, d = 0;
  if (S) {
    std::lock_guard<std::mutex> g(S->mu);
    q = (int64_t)S->queue.size();
    f = S->n_inflight;
    d = S->n_done;
  }
  if (queued) *queued = q;
  if (inflight) *inflight = f;
  if (done) *done = d;
  return KTF_OK;
}

}  // extern "C"
