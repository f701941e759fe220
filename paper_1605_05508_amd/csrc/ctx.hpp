// ctx.hpp -- library context (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ktf_internal.hpp"

namespace ktf {

// grow-only device buffer owned by the context.  A regrowth frees and
// reallocates, which waits for the device, so it grows geometrically (to
// at least twice its size): a workload that varies regrows a few times,
// not at every new maximum.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    const size_t b = std::max(want + want / 4, 2 * bytes);
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess && b > want + want / 4) {  // the doubling does not fit: the request alone
      (void)hipGetLastError();
      e = hipMalloc(&p, want + want / 4);
      if (e == hipSuccess) bytes = want + want / 4;
      return e;
    }
    if (e == hipSuccess) bytes = b;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct LaunchTrial {
  int block;
  int waves;
  bool persistent;
  int tpl;
  float ms;
};

struct TunedShape {
  int block = 256;
  int waves = 1;  // waves per SIMD the registers must allow (1: compiler's choice)
  int tpl = 1;    // tracks per lane
  bool persistent = false;
  int persistent_blocks = 0;
  float ms = 0.f;
  std::vector<LaunchTrial> trials;  // every shape timed, in trial order
};

struct SweepGraph {
  bool valid = false;
  FitArgs args{};
  ktf_precision prec = KTF_FP64;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct ServeEvent;  // serving.cpp
struct ServeState;

}  // namespace ktf

struct ktf_ctx {
  ktf_config cfg{};
  std::vector<double> radii;
  std::vector<double> x0;  // per-layer material thickness (radiation lengths), empty = none
  int device = 0;
  int n_cu = 0;
  std::string gcn_arch;
  std::string last_error;
  std::mutex err_mu;

  // fit workspace
  ktf::DevBuf fit_lend, fit_pos, counters;
  std::map<std::pair<int, int>, ktf::TunedShape> tuned;  // (prec, size class) -> shape
  ktf::SweepGraph sweep;
  hipStream_t capture_stream = nullptr;

  // build workspace
  ktf::DevBuf b_off, b_perm, b_binned, b_cand[2], b_prop, b_rec, b_hist, b_best, b_misc, b_stage, b_list, b_sort;
  hipEvent_t build_done = nullptr;  // last ktf_build / ktf_bin_hits work on the workspace
  void* h_pinned = nullptr;
  size_t h_pinned_bytes = 0;

  // serving
  ktf::ServeState* serve = nullptr;  // owned; freed by serve_shutdown
  std::mutex serve_mu;               // guards the creation and shutdown of serve

  void set_error(const std::string& s) {
    std::lock_guard<std::mutex> g(err_mu);
    last_error = s;
  }
};

namespace ktf {
int fail(ktf_ctx* c, int code, const char* fmt, ...);
int hip_fail(ktf_ctx* c, hipError_t e, const char* what);
FitArgs make_fit_args(ktf_ctx* c, const ktf_fit_in* in, ktf_fit_out* out);
int build_impl(ktf_ctx* c, const ktf_event_batch* ev, ktf_build_out* out, hipStream_t st);
int bin_impl(ktf_ctx* c, const ktf_event_batch* ev, int32_t* offsets, int32_t* perm,
             hipStream_t st);
void serve_shutdown(ktf_ctx* c);

// the context's layer material as kernels take it
inline MaterialD material_of(const ktf_ctx* c) {
  MaterialD m{};
  m.on = c->x0.empty() ? 0 : 1;
  for (size_t l = 0; l < c->x0.size(); ++l) m.x0[l] = c->x0[l];
  m.eloss = c->cfg.eloss_per_x0;
  m.mass = c->cfg.mass;
  return m;
}
}  // namespace ktf
