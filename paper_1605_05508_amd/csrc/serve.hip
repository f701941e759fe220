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
#include "host_logic.hpp"
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
  std::vector<EventRows> rows;
  rows.reserve(E);
  for (ServeEvent* ev : ln.batch)
    rows.push_back({ev->n_seeds, ev->n_hits, ev->hit_off.data(), ev->hits.data(), ev->state.data(), ev->cov.data(),
                    ev->q.data(), ev->seed_hit.data()});
  std::vector<int64_t> hoff;
  batch_offsets(rows, L, ln.seed_off, hoff);
  const InLayout il = in_layout(E, L, NSL, Np, Hp, sizeof(TS));
  const size_t o_soff = il.soff, o_hoff = il.hoff, o_hits = il.hits, o_state = il.state, o_cov = il.cov,
               o_sh = il.sh, o_q = il.q, in_bytes = il.total;
  hipError_t e;
  if ((e = ensure_pinned(&ln.pin_in, &ln.pin_in_bytes, in_bytes)) != hipSuccess) return hip_fail(c, e, "serve staging");
  if ((e = ln.in.ensure(in_bytes)) != hipSuccess) return hip_fail(c, e, "serve inputs");
  char* P = static_cast<char*>(ln.pin_in);
  {
    std::vector<RowCopy> tasks;
    pack_rows(rows, L, NSL, sizeof(TS), ln.seed_off, hoff, P, il, tasks);
    run_copies(tasks);
  }
  if ((e = hipMemcpyAsync(ln.in.p, P, in_bytes, hipMemcpyHostToDevice, ln.stream)) != hipSuccess)
    return hip_fail(c, e, "serve H2D");
  char* D = static_cast<char*>(ln.in.p);

  // outputs of building and fit: what goes back to the host first (hit
  // indices, the fit's results), then the building's own fit outputs
  const OutLayout ol = out_layout(L, Np, sizeof(TS));
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
  std::vector<int64_t> ns;
  std::vector<ResultRows> res;
  for (ServeEvent* ev : ln.batch) {
    const int64_t n = ev->n_seeds;
    ns.push_back(n);
    res.push_back({ev->r_hit.get((size_t)L * n), ev->r_state.get(sizeof(TS) * 6 * n),
                   ev->r_cov.get(sizeof(TS) * 21 * n), ev->r_chi2.get(n), ev->r_nh.get(n), ev->r_st.get(n)});
  }
  std::vector<RowCopy> tasks;
  unpack_rows(ns, res, L, sizeof(TS), Np, static_cast<const char*>(ln.pin_out), out_layout(L, Np, sizeof(TS)), tasks);
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
  if (const char* why = check_event_host(ev, L)) return fail(c, KTF_EINVAL, "ktf_submit: %s", why);
  const int64_t n = ev->n_seeds, nh = ev->hit_off[L];
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
    const size_t need = ts * 3 * (size_t)nh;
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
