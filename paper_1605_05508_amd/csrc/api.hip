// api.hip -- C-ABI entry points: context, fitting, launch-shape tuning.
#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstring>

#include "ctx.hpp"
#include "host_logic.hpp"

namespace ktf {

int fail(ktf_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->set_error(buf);
  return code;
}

int hip_fail(ktf_ctx* c, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(c, KTF_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(c, KTF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

FitArgs make_fit_args(ktf_ctx* c, const ktf_fit_in* in, ktf_fit_out* out) {
  FitArgs a{};
  a.n = in->n;
  a.pitch = in->pitch;
  a.state = in->seed_state;
  a.cov = in->seed_cov;
  a.q = in->charge;
  a.hits = in->hits;
  a.valid = in->hit_valid;
  a.state_o = out->state;
  a.cov_o = out->cov;
  a.chi2 = out->chi2;
  a.nupd = out->n_upd;
  a.status = out->status;
  a.n_layers = c->cfg.n_layers;
  a.n_passes = in->n_passes > 1 ? in->n_passes : 1;
  a.bz = c->cfg.bz;
  a.hr.sr2 = c->cfg.sigma_r * c->cfg.sigma_r;
  a.hr.srphi2 = c->cfg.sigma_rphi * c->cfg.sigma_rphi;
  a.hr.sz2 = c->cfg.sigma_z * c->cfg.sigma_z;
  for (int l = 0; l < c->cfg.n_layers; ++l) a.radii[l] = c->radii[l];
  a.mat = material_of(c);
  return a;
}

static int size_class(int64_t n) {
  int k = 0;
  while ((int64_t(1) << (k + 1)) <= n && k < 62) ++k;
  return k;
}

int check_fit_args(ktf_ctx* c, const ktf_fit_in* in, const ktf_fit_out* out) {
  if (const char* why = check_fit_in(in, out)) return fail(c, KTF_EINVAL, "ktf_fit: %s", why);
  return KTF_OK;
}

// blocks per CU for the persistent kernel, from the occupancy calculator
int persistent_blocks(ktf_ctx* c, ktf_precision prec, int bs, int waves, int tpl);

// the launch shape the tuner chose for (prec, size class of n); false (and
// the arguments unchanged) when none was tuned
bool tuned_launch(ktf_ctx* c, ktf_precision prec, int64_t n, int& bs, int& waves, int& tpl, bool& persistent) {
  auto it = c->tuned.find({(int)prec, size_class(n)});
  if (it == c->tuned.end()) return false;
  bs = it->second.block;
  waves = it->second.waves;
  tpl = it->second.tpl;
  persistent = it->second.persistent;
  return true;
}

// device address of the allocation-free entry point's scratch (noalloc.hip)
hipError_t noalloc_init(int device);

static int run_fit(ktf_ctx* c, FitArgs a, ktf_precision prec, ktf_fit_mode mode, int bs, int waves, int tpl,
                   bool persistent, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (mode == KTF_FIT_SWEEP || mode == KTF_FIT_SWEEP_GRAPH) {
    if ((e = c->fit_lend.ensure((size_t)a.pitch)) != hipSuccess) return hip_fail(c, e, "sweep workspace");
    a.lend = static_cast<uint8_t*>(c->fit_lend.p);
    if (prec == KTF_FP32_BULK) {
      if ((e = c->fit_pos.ensure((size_t)a.pitch * 3 * sizeof(double))) != hipSuccess)
        return hip_fail(c, e, "sweep workspace");
      a.pos_ws = static_cast<double*>(c->fit_pos.p);
    }
    if (mode == KTF_FIT_SWEEP) {
      for (int l = 0; l < a.n_layers && e == hipSuccess; ++l) e = launch_fit_layer(a, prec, l, st);
      return e == hipSuccess ? KTF_OK : hip_fail(c, e, "fit layer launch");
    }
    // graph: capture the per-layer launches once per argument set, replay
    SweepGraph& g = c->sweep;
    if (!g.valid || g.prec != prec || memcmp(&g.args, &a, sizeof a) != 0) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
      g.exec = nullptr;
      g.graph = nullptr;
      g.valid = false;
      e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
      for (int l = 0; l < a.n_layers && e == hipSuccess; ++l)
        e = launch_fit_layer(a, prec, l, c->capture_stream);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(c->capture_stream, &graph);
      if (e == hipSuccess) e = e2;
      if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(c, e, "sweep graph capture");
      }
      e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(c, e, "sweep graph instantiate");
      }
      g.graph = graph;
      g.args = a;
      g.prec = prec;
      g.valid = true;
    }
    e = hipGraphLaunch(g.exec, st);
    return e == hipSuccess ? KTF_OK : hip_fail(c, e, "sweep graph launch");
  }
  int pblocks = 0;
  if (persistent) {
    if ((e = c->counters.ensure(64 * sizeof(unsigned long long))) != hipSuccess)
      return hip_fail(c, e, "counters");
    a.counters = static_cast<unsigned long long*>(c->counters.p);
    const int tile = a.mat.on ? bs : bs * tpl;
    a.tile_count = (a.n + tile - 1) / tile;
    pblocks = persistent_blocks(c, prec, bs, waves, tpl) * c->n_cu;
    if (pblocks <= 0) pblocks = c->n_cu;
    if ((e = launch_fill_u64(a.counters, 1, 0ull, st)) != hipSuccess) return hip_fail(c, e, "fill");
  }
  e = launch_fit_fused(a, prec, bs, waves, tpl, persistent, pblocks, st);
  return e == hipSuccess ? KTF_OK : hip_fail(c, e, "fit launch");
}

}  // namespace ktf

using namespace ktf;

extern "C" {

int ktf_create(const ktf_config* cfg, ktf_ctx** out) {
  if (!cfg || !out) return KTF_EINVAL;
  *out = nullptr;
  if (check_config(cfg)) return KTF_EINVAL;
  bool material = false;
  if (cfg->layer_x0)
    for (int l = 0; l < cfg->n_layers; ++l) material = material || cfg->layer_x0[l] > 0.0;
  ktf_ctx* c = new ktf_ctx();
  c->cfg = *cfg;
  c->radii.assign(cfg->layer_r, cfg->layer_r + cfg->n_layers);
  c->cfg.layer_r = c->radii.data();
  if (material) c->x0.assign(cfg->layer_x0, cfg->layer_x0 + cfg->n_layers);
  c->cfg.layer_x0 = material ? c->x0.data() : nullptr;
  hipError_t e = hipGetDevice(&c->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, c->device);
  if (e == hipSuccess) {
    c->n_cu = prop.multiProcessorCount;
    c->gcn_arch = prop.gcnArchName;
    e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
  }
  if (e == hipSuccess) e = noalloc_init(c->device);
  if (e != hipSuccess) {
    delete c;
    return KTF_EDEVICE;
  }
  *out = c;
  return KTF_OK;
}

int ktf_destroy(ktf_ctx* c) {
  if (!c) return KTF_OK;
  serve_shutdown(c);
  (void)hipDeviceSynchronize();
  if (c->sweep.exec) (void)hipGraphExecDestroy(c->sweep.exec);
  if (c->sweep.graph) (void)hipGraphDestroy(c->sweep.graph);
  c->fit_lend.release();
  c->fit_pos.release();
  c->counters.release();
  for (DevBuf* b : {&c->b_off, &c->b_perm, &c->b_binned, &c->b_cand[0], &c->b_cand[1], &c->b_prop,
                    &c->b_rec, &c->b_hist, &c->b_best, &c->b_misc, &c->b_stage, &c->b_list, &c->b_sort})
    b->release();
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  if (c->build_done) (void)hipEventDestroy(c->build_done);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  delete c;
  return KTF_OK;
}

size_t ktf_config_bytes(void) { return sizeof(ktf_config); }

const char* ktf_last_error(const ktf_ctx* c) {
  if (!c) return "";
  return c->last_error.c_str();
}

int ktf_fit(ktf_ctx* c, const ktf_fit_in* in, ktf_fit_out* out, ktf_fit_mode mode,
            void* hip_stream) {
  int rc = check_fit_args(c, in, out);
  if (rc) return rc;
  if (in->n == 0) return KTF_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  FitArgs a = make_fit_args(c, in, out);
  int bs = 256, waves = 1, tpl = 1;
  bool persistent = false;
  switch (mode) {
    case KTF_FIT_AUTO: (void)tuned_launch(c, in->prec, in->n, bs, waves, tpl, persistent); break;
    case KTF_FIT_FUSED: break;
    case KTF_FIT_PERSISTENT: persistent = true; break;
    case KTF_FIT_SWEEP:
    case KTF_FIT_SWEEP_GRAPH:
      if (in->prec == KTF_FP32_PROP)
        return fail(c, KTF_EINVAL, "ktf_fit: KTF_FP32_PROP keeps the covariance in registers; use a fused mode");
      if (in->n_passes > 1)
        return fail(c, KTF_EINVAL, "ktf_fit: the iterated refit runs in the fused modes");
      break;
    default: return fail(c, KTF_EINVAL, "ktf_fit: unknown mode %d", (int)mode);
  }
  return run_fit(c, a, in->prec, mode, bs, waves, tpl, persistent, st);
}

int ktf_autotune_fit(ktf_ctx* c, const ktf_fit_in* in, ktf_fit_out* out, void* hip_stream) {
  int rc = check_fit_args(c, in, out);
  if (rc) return rc;
  if (in->n == 0) return KTF_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  FitArgs a = make_fit_args(c, in, out);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(c, KTF_EDEVICE, "autotune: event create");
  // every shape is timed in two rounds (the first may still run while the
  // clocks ramp up) and keeps its faster round
  TunedShape best;
  best.ms = 1e30f;
  // two tracks per lane only for one pass without material
  const int ntpl = (a.mat.on || a.n_passes > 1) ? 1 : kTplChoices;
  for (int round = 0; round < 2 && rc == 0; ++round) {
    int t = 0;
    for (int bs : kBlockSizes) {
      for (int w = 0; w < 2 * kWaveChoices * ntpl && rc == 0; ++w, ++t) {
        const int pers = w & 1, waves = 1 + (w / 2) % kWaveChoices, tpl = 1 + w / (2 * kWaveChoices);
        rc = run_fit(c, a, in->prec, KTF_FIT_FUSED, bs, waves, tpl, pers != 0, st);  // warm-up
        if (rc) break;
        float tot = 0.f;
        const int reps = 3;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && rc == 0; ++r)
          rc = run_fit(c, a, in->prec, KTF_FIT_FUSED, bs, waves, tpl, pers != 0, st);
        (void)hipEventRecord(e1, st);
        if (rc) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(c, KTF_EDEVICE, "autotune: sync");
          break;
        }
        (void)hipEventElapsedTime(&tot, e0, e1);
        const float ms = tot / reps;
        if (round == 0)
          best.trials.push_back(LaunchTrial{bs, waves, pers != 0, tpl, ms});
        else
          best.trials[t].ms = std::min(best.trials[t].ms, ms);
      }
      if (rc) break;
    }
  }
  for (const LaunchTrial& tr : best.trials) {
    if (tr.ms < best.ms) {
      best.ms = tr.ms;
      best.block = tr.block;
      best.waves = tr.waves;
      best.tpl = tr.tpl;
      best.persistent = tr.persistent;
      best.persistent_blocks = tr.persistent ? persistent_blocks(c, in->prec, tr.block, tr.waves, tr.tpl) : 0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  c->tuned[{(int)in->prec, size_class(in->n)}] = best;
  return KTF_OK;
}

int ktf_tuned_shape(ktf_ctx* c, ktf_precision prec, int64_t n, char* buf, size_t len) {
  if (!c || !buf || len == 0) return KTF_EINVAL;
  auto it = c->tuned.find({(int)prec, size_class(n)});
  if (it == c->tuned.end()) {
    snprintf(buf, len, "{\"block\": 256, \"waves_per_simd\": 1, \"tracks_per_lane\": 1, \"persistent\": false, \"tuned\": false}");
  } else {
    const TunedShape& t = it->second;
    std::string s = "{\"block\": " + std::to_string(t.block) + ", \"waves_per_simd\": " +
                    std::to_string(t.waves) + ", \"tracks_per_lane\": " + std::to_string(t.tpl) +
                    ", \"persistent\": " + (t.persistent ? "true" : "false") +
                    ", \"blocks_per_cu\": " + std::to_string(t.persistent_blocks);
    char num[32];
    snprintf(num, sizeof num, "%.6f", t.ms);
    s += std::string(", \"ms\": ") + num + ", \"tuned\": true, \"trials\": [";
    for (size_t i = 0; i < t.trials.size(); ++i) {
      snprintf(num, sizeof num, "%.6f", t.trials[i].ms);
      s += std::string(i ? ", " : "") + "[" + std::to_string(t.trials[i].block) + ", " +
           std::to_string(t.trials[i].waves) + ", " + (t.trials[i].persistent ? "1" : "0") + ", " +
           std::to_string(t.trials[i].tpl) + ", " + num + "]";
    }
    s += "]}";
    snprintf(buf, len, "%s", s.c_str());
  }
  return KTF_OK;
}

}  // extern "C"
