// Self-checking CPU program over the library's host-only logic
// (csrc/host_logic.cpp), built with the address, undefined-behaviour or
// thread sanitizer by tests/test_host_sanitizers.py.  No GPU and no HIP.
//
//  - argument checks: valid inputs pass, each single defect is refused, and
//    random inputs with extreme values run without undefined behaviour;
//  - serving batches: random mixes of events (empty ones included, both
//    value sizes) are packed into staging of exactly the layout's size and
//    every row lands where the batch layout says; results are unpacked from
//    a host output block of exactly its size into per-event arrays of
//    exactly their size, and read back;
//  - row copies above 4 MB take the threaded path.
// Prints "host logic OK" and returns 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <random>
#include <vector>

#include "../../paper_1605_05508_amd/csrc/host_logic.hpp"

using namespace ktf;

static int g_fail = 0;
#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                        \
    }                                                                  \
  } while (0)

static ktf_config good_config(std::vector<double>& radii) {
  radii.clear();
  for (int l = 0; l < 10; ++l) radii.push_back(4.0 + 4.0 * l);
  ktf_config c;
  std::memset(&c, 0, sizeof c);
  c.n_layers = 10;
  c.layer_r = radii.data();
  c.bz = 3.8;
  c.sigma_r = c.sigma_rphi = 0.01;
  c.sigma_z = 0.1;
  c.max_cands = 10;
  c.max_missed = 1;
  c.n_seed_layers = 3;
  c.n_zbins = 64;
  c.n_phibins = 512;
  c.z_half = 100.0;
  c.hbm_budget_bytes = 1ull << 30;
  c.eta_max = 1.2;
  return c;
}

static void check_configs(std::mt19937_64& rng) {
  std::vector<double> radii;
  ktf_config c = good_config(radii);
  CHECK(check_config(&c) == nullptr);
  CHECK(check_config(nullptr) != nullptr);
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  // one defect at a time
  struct Mut {
    void (*f)(ktf_config&, std::vector<double>&);
  };
  const Mut muts[] = {
      {[](ktf_config& x, std::vector<double>&) { x.n_layers = 0; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_layers = KTF_MAX_LAYERS + 1; }},
      {[](ktf_config& x, std::vector<double>&) { x.layer_r = nullptr; }},
      {[](ktf_config& x, std::vector<double>& r) { r[3] = r[2]; }},
      {[](ktf_config& x, std::vector<double>& r) { r[0] = -1.0; }},
      {[](ktf_config& x, std::vector<double>& r) { r[9] = std::numeric_limits<double>::infinity(); }},
      {[](ktf_config& x, std::vector<double>&) { x.sigma_r = 0.0; }},
      {[](ktf_config& x, std::vector<double>&) { x.sigma_z = std::numeric_limits<double>::quiet_NaN(); }},
      {[](ktf_config& x, std::vector<double>&) { x.bz = std::numeric_limits<double>::infinity(); }},
      {[](ktf_config& x, std::vector<double>&) { x.max_cands = 0; }},
      {[](ktf_config& x, std::vector<double>&) { x.max_cands = KTF_MAX_CANDS + 1; }},
      {[](ktf_config& x, std::vector<double>&) { x.max_missed = -1; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_seed_layers = 11; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_zbins = 0; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_phibins = INT32_MAX; }},
      {[](ktf_config& x, std::vector<double>&) { x.z_half = 0.0; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_etabins = -1; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_etabins = 21; x.eta_max = 0.0; }},
      {[](ktf_config& x, std::vector<double>&) { x.n_etabins = INT32_MAX; }},
  };
  for (const Mut& m : muts) {
    ktf_config x = good_config(radii);
    m.f(x, radii);
    CHECK(check_config(&x) != nullptr);
  }
  // material
  std::vector<double> x0(10, 0.02);
  c = good_config(radii);
  c.layer_x0 = x0.data();
  c.mass = 0.1396;
  c.eloss_per_x0 = 0.0;
  CHECK(check_config(&c) == nullptr);
  c.mass = 0.0;
  CHECK(check_config(&c) != nullptr);
  x0[4] = nan;
  c.mass = 0.1396;
  CHECK(check_config(&c) != nullptr);
  // random extreme values: no undefined behaviour, accepted or not
  const int32_t ints[] = {INT32_MIN, -1, 0, 1, 2, 3, 16, 17, 32, 33, 512, 1 << 20, INT32_MAX};
  const double dbls[] = {-inf, -1.0, 0.0, 1e-300, 0.5, 1.2, 3.8, 100.0, 1e300, inf, nan};
  for (int it = 0; it < 20000; ++it) {
    ktf_config x = good_config(radii);
    auto I = [&] { return ints[rng() % (sizeof ints / sizeof *ints)]; };
    auto D = [&] { return dbls[rng() % (sizeof dbls / sizeof *dbls)]; };
    switch (rng() % 6) {
      case 0: x.n_layers = I() % 40; break;
      case 1: x.n_zbins = I(); x.n_phibins = I(); break;
      case 2: x.n_etabins = I(); x.eta_max = D(); x.n_phibins = I(); break;
      case 3: x.max_cands = I(); x.n_seed_layers = I(); x.max_missed = I(); break;
      case 4: x.sigma_r = D(); x.sigma_rphi = D(); x.sigma_z = D(); x.z_half = D(); x.bz = D(); break;
      default: radii[rng() % 10] = D(); break;
    }
    (void)check_config(&x);
  }
}

static void check_fits(std::mt19937_64& rng) {
  char dummy[64];
  void* p = dummy;
  ktf_fit_in in{100, 128, KTF_FP32_BULK, p, p, reinterpret_cast<const int8_t*>(p), p,
                reinterpret_cast<const uint8_t*>(p), 1};
  ktf_fit_out out{p, p, reinterpret_cast<double*>(p), reinterpret_cast<int32_t*>(p),
                  reinterpret_cast<uint32_t*>(p)};
  CHECK(check_fit_in(&in, &out) == nullptr);
  ktf_fit_in x = in;
  x.pitch = 99;
  CHECK(check_fit_in(&x, &out) != nullptr);
  x = in;
  x.n_passes = 3;
  CHECK(check_fit_in(&x, &out) != nullptr);  // the refit needs a double covariance
  x.prec = KTF_FP32_PROP;
  CHECK(check_fit_in(&x, &out) == nullptr);
  x = in;
  x.prec = (ktf_precision)7;
  CHECK(check_fit_in(&x, &out) != nullptr);
  x = in;
  x.pitch = std::numeric_limits<int64_t>::max();
  CHECK(check_fit_in(&x, &out) != nullptr);
  x = in;
  x.hits = nullptr;
  CHECK(check_fit_in(&x, &out) != nullptr);
  x.n = 0;
  CHECK(check_fit_in(&x, &out) == nullptr);  // nothing to read
  CHECK(check_fit_in(nullptr, &out) != nullptr);
  const int64_t big[] = {std::numeric_limits<int64_t>::min(), -1, 0, 1, INT32_MAX, int64_t(1) << 40,
                         (int64_t(1) << 40) + 1, std::numeric_limits<int64_t>::max()};
  for (int it = 0; it < 5000; ++it) {
    x = in;
    x.n = big[rng() % 8];
    x.pitch = big[rng() % 8];
    x.n_passes = (int32_t)(rng() % 40) - 5;
    const char* why = check_fit_in(&x, &out);
    if (!why) CHECK(x.n >= 0 && x.n <= x.pitch && x.pitch <= kMaxPitch);
  }
}

static void check_batches(std::mt19937_64& rng) {
  const int L = 6;
  std::vector<int64_t> so{0, 10, 10, 25}, ho(3 * L + 1);
  for (int g = 0; g <= 3 * L; ++g) ho[g] = 7 * g;
  char dummy[64];
  ktf_event_batch b{3, so.data(), ho.data(), 7 * 3 * L, dummy, 25, dummy, dummy,
                    reinterpret_cast<const int8_t*>(dummy), reinterpret_cast<const int32_t*>(dummy), KTF_FP64};
  CHECK(check_event_batch(&b, L, 10) == nullptr);
  ktf_event_batch x = b;
  x.seed_pitch = 24;
  CHECK(check_event_batch(&x, L, 10) != nullptr);
  x = b;
  x.seed_pitch = std::numeric_limits<int64_t>::max();  // seed_pitch * max_cands must not be evaluated
  CHECK(check_event_batch(&x, L, 16) != nullptr);
  x = b;
  x.seed_pitch = INT32_MAX / 10 + 1;
  CHECK(check_event_batch(&x, L, 10) != nullptr);
  x.seed_pitch = INT32_MAX / 10;
  CHECK(check_event_batch(&x, L, 10) == nullptr);
  x = b;
  x.prec = KTF_FP32_PROP;
  CHECK(check_event_batch(&x, L, 10) != nullptr);
  std::vector<int64_t> so2 = so;
  so2[2] = 9;
  x = b;
  x.seed_off = so2.data();
  CHECK(check_event_batch(&x, L, 10) != nullptr);
  std::vector<int64_t> ho2 = ho;
  ho2[5] = ho2[4] + (int64_t)INT32_MAX + 1;
  for (int g = 6; g <= 3 * L; ++g) ho2[g] = ho2[5] + g;
  x = b;
  x.hit_off = ho2.data();
  x.hit_pitch = ho2[3 * L];
  CHECK(check_event_batch(&x, L, 10) != nullptr);
  // random offsets with extreme steps
  for (int it = 0; it < 5000; ++it) {
    std::vector<int64_t> s(4), h(3 * L + 1);
    const int64_t steps[] = {0, 1, 5, INT32_MAX, (int64_t)INT32_MAX + 1, int64_t(1) << 40, int64_t(1) << 61, -3};
    // offsets as a caller may pass them, kept below 2^62 so that building
    // them here does not overflow
    auto step = [&](int64_t prev) {
      const int64_t d = steps[rng() % 8];
      return prev > (int64_t(1) << 62) - d ? prev : prev + d;
    };
    for (int e = 1; e < 4; ++e) s[e] = step(s[e - 1]);
    for (int g = 1; g <= 3 * L; ++g) h[g] = step(h[g - 1]);
    x = b;
    x.seed_off = s.data();
    x.hit_off = h.data();
    x.seed_pitch = s[3] + steps[rng() % 3];
    x.hit_pitch = h[3 * L] + steps[rng() % 3];
    (void)check_event_batch(&x, L, 1 + (int)(rng() % 16));
  }
  // host events
  std::vector<int64_t> eh{0, 3, 3, 9, 12, 12, 20};
  ktf_event_host ev{5, eh.data(), dummy, dummy, dummy, reinterpret_cast<const int8_t*>(dummy),
                    reinterpret_cast<const int32_t*>(dummy), KTF_FP32_BULK};
  CHECK(check_event_host(&ev, L) == nullptr);
  ktf_event_host y = ev;
  y.n_seeds = (int64_t)INT32_MAX + 1;
  CHECK(check_event_host(&y, L) != nullptr);
  y = ev;
  y.hits = nullptr;
  CHECK(check_event_host(&y, L) != nullptr);
  std::vector<int64_t> eh2 = eh;
  eh2[6] = (int64_t)INT32_MAX + 5;
  y = ev;
  y.hit_off = eh2.data();
  CHECK(check_event_host(&y, L) != nullptr);
  // footprints grow with the event and stay finite at the largest accepted sizes
  std::vector<double> radii;
  ktf_config c = good_config(radii);
  const size_t f1 = footprint_of(c, 1000, 6000, KTF_FP32_BULK), f2 = footprint_of(c, 2000, 6000, KTF_FP32_BULK);
  CHECK(f2 > f1 && footprint_of(c, 1000, 6000, KTF_FP64) > f1);
  c.max_cands = KTF_MAX_CANDS;
  c.n_layers = KTF_MAX_LAYERS;
  const size_t fmax = footprint_of(c, kMaxEventSeeds, kMaxEventHits, KTF_FP64);
  CHECK(fmax > footprint_of(c, kMaxEventSeeds / 2, kMaxEventHits, KTF_FP64));
}

// The building's row regions: for random and edge seed counts, walk the
// blocks of both launches that reserve rows (seed fit: 256 seeds, one row
// each; merge: merge_seeds seeds, up to max_cands rows each) through the
// block-to-region map b * regions / blocks and check that no region is
// asked for more rows than it has, that the regions are few for small
// events and that the slack over n * max_cands stays bounded.
static void check_regions(std::mt19937_64& rng) {
  std::vector<int64_t> ns = {0, 1, 255, 256, 257, 300, 4095, 20000, 50000, 500000, 1000003};
  for (int i = 0; i < 60; ++i) ns.push_back(1 + (int64_t)(rng() % 3000000));
  for (int64_t n : ns) {
    for (int nc = 1; nc <= KTF_MAX_CANDS; ++nc) {
      const int nr = region_count(n, nc);
      const int64_t rs = region_rows(n, nc);
      CHECK(nr >= 1 && nr <= kMaxRegions && rs % 256 == 0 && rs > 0);
      const int64_t sb = merge_seeds(merge_lanes(nc));
      struct Launch {
        int64_t per_block, rows_per_seed;
      } launches[2] = {{256, 1}, {sb, nc}};
      for (const Launch& ln : launches) {
        const int64_t G = n > 0 ? (n + ln.per_block - 1) / ln.per_block : 1;
        std::vector<int64_t> used(nr, 0);
        for (int64_t b = 0; b < G; ++b) {
          const int64_t seeds = std::min<int64_t>(ln.per_block, std::max<int64_t>(n - b * ln.per_block, 0));
          const int64_t r = b * nr / G;
          CHECK(r >= 0 && r < nr);
          if (r >= 0 && r < nr) used[r] += seeds * ln.rows_per_seed;
        }
        for (int r = 0; r < nr; ++r) CHECK(used[r] <= rs);
      }
      // never more regions than merge blocks: one for an event of one block
      CHECK(nr <= merge_blocks(n, nc));
      if (n <= sb) CHECK(nr == 1);
      // slack: at most one block of either launch per region, plus rounding
      CHECK(nr * rs <= n * nc + (int64_t)nr * (sb * nc + 256 + 255));
    }
  }
}

// pattern value of (event, array, row, element) so that every packed or
// unpacked element can be checked where it lands
static uint64_t pat(int e, int arr, int row, int64_t i) {
  return ((uint64_t)(e + 1) << 48) ^ ((uint64_t)(arr + 1) << 40) ^ ((uint64_t)(row + 1) << 32) ^ (uint64_t)i;
}

template <typename T>
static T as(uint64_t v) {
  return (T)(v & 0xffffff);  // exact in float and double
}

template <typename T>
static void check_pack_unpack(std::mt19937_64& rng, int E, int L, int NSL) {
  const size_t ts = sizeof(T);
  struct Ev {
    int64_t n, nh;
    std::vector<int64_t> off;
    std::unique_ptr<T[]> hits, state, cov;
    std::unique_ptr<int8_t[]> q;
    std::unique_ptr<int32_t[]> sh;
  };
  std::vector<Ev> evs(E);
  std::vector<EventRows> rows;
  for (int e = 0; e < E; ++e) {
    Ev& v = evs[e];
    v.n = rng() % 4 == 0 ? 0 : (int64_t)(rng() % 300);
    v.off.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) v.off[l + 1] = v.off[l] + (rng() % 3 == 0 ? 0 : (int64_t)(rng() % 80));
    v.nh = v.off[L];
    // exact-size heap arrays: any access past them is a sanitizer report
    v.hits.reset(v.nh ? new T[3 * v.nh] : nullptr);
    v.state.reset(v.n ? new T[6 * v.n] : nullptr);
    v.cov.reset(v.n ? new T[21 * v.n] : nullptr);
    v.q.reset(v.n ? new int8_t[v.n] : nullptr);
    v.sh.reset(v.n ? new int32_t[NSL * v.n] : nullptr);
    for (int k = 0; k < 3; ++k)
      for (int64_t i = 0; i < v.nh; ++i) v.hits[k * v.nh + i] = as<T>(pat(e, 0, k, i));
    for (int k = 0; k < 6; ++k)
      for (int64_t i = 0; i < v.n; ++i) v.state[k * v.n + i] = as<T>(pat(e, 1, k, i));
    for (int k = 0; k < 21; ++k)
      for (int64_t i = 0; i < v.n; ++i) v.cov[k * v.n + i] = as<T>(pat(e, 2, k, i));
    for (int64_t i = 0; i < v.n; ++i) v.q[i] = (int8_t)(pat(e, 3, 0, i) & 0x7f);
    for (int k = 0; k < NSL; ++k)
      for (int64_t i = 0; i < v.n; ++i) v.sh[k * v.n + i] = (int32_t)(pat(e, 4, k, i) & 0x7fffffff);
    rows.push_back({v.n, v.nh, v.off.data(), v.hits.get(), v.state.get(), v.cov.get(), v.q.get(), v.sh.get()});
  }
  std::vector<int64_t> so, ho;
  batch_offsets(rows, L, so, ho);
  const int64_t N = so[E], H = ho[(size_t)E * L];
  const int64_t Np = std::max<int64_t>(N, 1), Hp = std::max<int64_t>(H, 1);
  const InLayout il = in_layout(E, L, NSL, Np, Hp, ts);
  CHECK(il.total % 256 == 0 && il.soff < il.hoff && il.hoff < il.hits && il.hits < il.state && il.state < il.cov &&
        il.cov < il.sh && il.sh < il.q && il.q < il.total);
  std::unique_ptr<char[]> P(new char[il.total]);
  std::vector<RowCopy> tasks;
  pack_rows(rows, L, NSL, ts, so, ho, P.get(), il, tasks);
  run_copies(tasks);
  const int64_t* pso = reinterpret_cast<const int64_t*>(P.get() + il.soff);
  const int64_t* pho = reinterpret_cast<const int64_t*>(P.get() + il.hoff);
  for (int e = 0; e <= E; ++e) CHECK(pso[e] == so[e]);
  for (size_t g = 0; g < ho.size(); ++g) CHECK(pho[g] == ho[g]);
  const T* ph = reinterpret_cast<const T*>(P.get() + il.hits);
  const T* ps = reinterpret_cast<const T*>(P.get() + il.state);
  const T* pc = reinterpret_cast<const T*>(P.get() + il.cov);
  const int32_t* psh = reinterpret_cast<const int32_t*>(P.get() + il.sh);
  const int8_t* pq = reinterpret_cast<const int8_t*>(P.get() + il.q);
  for (int e = 0; e < E; ++e) {
    const Ev& v = evs[e];
    const int64_t s0 = so[e], h0 = ho[(size_t)e * L];
    for (int l = 0; l < L; ++l) CHECK(ho[(size_t)e * L + l] - h0 == v.off[l]);
    for (int k = 0; k < 3; ++k)
      for (int64_t i = 0; i < v.nh; ++i) CHECK(ph[k * Hp + h0 + i] == as<T>(pat(e, 0, k, i)));
    for (int k = 0; k < 6; ++k)
      for (int64_t i = 0; i < v.n; ++i) CHECK(ps[k * Np + s0 + i] == as<T>(pat(e, 1, k, i)));
    for (int k = 0; k < 21; ++k)
      for (int64_t i = 0; i < v.n; ++i) CHECK(pc[k * Np + s0 + i] == as<T>(pat(e, 2, k, i)));
    for (int k = 0; k < NSL; ++k)
      for (int64_t i = 0; i < v.n; ++i) CHECK(psh[k * Np + s0 + i] == (int32_t)(pat(e, 4, k, i) & 0x7fffffff));
    for (int64_t i = 0; i < v.n; ++i) CHECK(pq[i + s0] == (int8_t)(pat(e, 3, 0, i) & 0x7f));
  }
  // results: a host output block of exactly `host` bytes, filled by batch row
  const OutLayout ol = out_layout(L, Np, ts);
  CHECK(ol.host <= ol.total && ol.total % 256 == 0);
  std::unique_ptr<char[]> O(new char[ol.host]);
  int32_t* oh = reinterpret_cast<int32_t*>(O.get() + ol.hit);
  T* os = reinterpret_cast<T*>(O.get() + ol.f_state);
  T* oc = reinterpret_cast<T*>(O.get() + ol.f_cov);
  double* o2 = reinterpret_cast<double*>(O.get() + ol.f_chi2);
  int32_t* onu = reinterpret_cast<int32_t*>(O.get() + ol.f_nu);
  uint32_t* ost = reinterpret_cast<uint32_t*>(O.get() + ol.f_st);
  for (int64_t s = 0; s < N; ++s) {
    for (int l = 0; l < L; ++l) oh[l * Np + s] = (int32_t)(7 * s + l);
    for (int k = 0; k < 6; ++k) os[k * Np + s] = as<T>(pat(0, 5, k, s));
    for (int k = 0; k < 21; ++k) oc[k * Np + s] = as<T>(pat(0, 6, k, s));
    o2[s] = 0.5 * (double)s;
    onu[s] = (int32_t)(s % 17);
    ost[s] = (uint32_t)(s * 3);
  }
  struct Res {
    std::unique_ptr<int32_t[]> hit, nh;
    std::unique_ptr<T[]> st, cv;
    std::unique_ptr<double[]> c2;
    std::unique_ptr<uint32_t[]> ss;
  };
  std::vector<Res> rr(E);
  std::vector<ResultRows> res;
  std::vector<int64_t> ns;
  for (int e = 0; e < E; ++e) {
    const int64_t n = evs[e].n;
    Res& r = rr[e];
    r.hit.reset(n ? new int32_t[L * n] : nullptr);
    r.st.reset(n ? new T[6 * n] : nullptr);
    r.cv.reset(n ? new T[21 * n] : nullptr);
    r.c2.reset(n ? new double[n] : nullptr);
    r.nh.reset(n ? new int32_t[n] : nullptr);
    r.ss.reset(n ? new uint32_t[n] : nullptr);
    res.push_back({r.hit.get(), r.st.get(), r.cv.get(), r.c2.get(), r.nh.get(), r.ss.get()});
    ns.push_back(n);
  }
  tasks.clear();
  unpack_rows(ns, res, L, ts, Np, O.get(), ol, tasks);
  run_copies(tasks);
  for (int e = 0; e < E; ++e) {
    const int64_t n = ns[e], s0 = so[e];
    const Res& r = rr[e];
    for (int64_t i = 0; i < n; ++i) {
      const int64_t s = s0 + i;
      for (int l = 0; l < L; ++l) CHECK(r.hit[l * n + i] == (int32_t)(7 * s + l));
      for (int k = 0; k < 6; ++k) CHECK(r.st[k * n + i] == as<T>(pat(0, 5, k, s)));
      for (int k = 0; k < 21; ++k) CHECK(r.cv[k * n + i] == as<T>(pat(0, 6, k, s)));
      CHECK(r.c2[i] == 0.5 * (double)s && r.nh[i] == (int32_t)(s % 17) && r.ss[i] == (uint32_t)(s * 3));
    }
  }
}

static void check_threaded_copies(std::mt19937_64& rng) {
  // about 12 MB in rows of uneven length: above 4 MB the copies are split
  // into 256K-element pieces over four threads
  std::vector<std::vector<float>> src, dst;
  std::vector<RowCopy> rows;
  for (int r = 0; r < 9; ++r) {
    const size_t n = 100000 + (size_t)(rng() % 400000);
    src.emplace_back(n);
    dst.emplace_back(n, -1.0f);
    for (size_t i = 0; i < n; ++i) src.back()[i] = (float)(r * 1000003 + i);
  }
  for (int r = 0; r < 9; ++r) rows.push_back({src[r].data(), dst[r].data(), (int64_t)src[r].size(), 4});
  rows.push_back({nullptr, nullptr, 0, 4});  // an empty row copies nothing
  run_copies(rows);
  for (int r = 0; r < 9; ++r) CHECK(src[r] == dst[r]);
}

int main() {
  std::mt19937_64 rng(20160518);
  check_configs(rng);
  check_fits(rng);
  check_batches(rng);
  check_regions(rng);
  for (int it = 0; it < 40; ++it) {
    const int E = 1 + (int)(rng() % 9), L = 1 + (int)(rng() % 17), NSL = 1 + (int)(rng() % L);
    if (it % 2)
      check_pack_unpack<float>(rng, E, L, NSL);
    else
      check_pack_unpack<double>(rng, E, L, NSL);
  }
  check_pack_unpack<float>(rng, 3, 17, 3);
  check_threaded_copies(rng);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host logic OK\n");
  return 0;
}
