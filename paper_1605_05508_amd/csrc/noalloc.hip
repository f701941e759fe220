// noalloc.hip -- the fit without any device allocation, for callers that
// cannot allocate (code under graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The fit modes that need scratch memory take it from one file-scope device
// array instead of the context's grow-only workspace:
//   persistent  the tile counter the blocks pull work from (256 bytes);
//   sweep       per track the end layer (1 byte) and, with float storage,
//               the position carried in double between layers (24 bytes).
// The fused modes need no scratch.  Every GPU keeps its own copy of the
// array, whose device address is looked up once per device when a context
// is created there; every call on that GPU shares it, so calls that overlap
// in time on one GPU race (order them on one stream, or synchronize).
#include <mutex>

#include "ctx.hpp"

namespace ktf {

constexpr size_t kScratchCounterBytes = 256;

// The scratch array.  In host code its name is only a stand-in for the
// symbol: the device address comes from hipGetSymbolAddress (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[KTF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Called by ktf_create with the context's device current.
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// scratch bytes a sweep over tracks of this pitch needs
static size_t sweep_bytes(int64_t pitch, ktf_precision prec) {
  size_t b = kScratchCounterBytes + round256((size_t)pitch);
  if (prec == KTF_FP32_BULK) b += (size_t)pitch * 3 * sizeof(double);
  return b;
}

int persistent_blocks(ktf_ctx* c, ktf_precision prec, int bs, int waves, int tpl);
int check_fit_args(ktf_ctx* c, const ktf_fit_in* in, const ktf_fit_out* out);
bool tuned_launch(ktf_ctx* c, ktf_precision prec, int64_t n, int& bs, int& waves, int& tpl, bool& persistent);

static int fit_noalloc(ktf_ctx* c, const ktf_fit_in* in, ktf_fit_out* out, ktf_fit_mode mode,
                       hipStream_t st) {
  int rc = check_fit_args(c, in, out);
  if (rc) return rc;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(c, e, "ktf_fit_noalloc: current device");
  if (dev != c->device)
    return fail(c, KTF_EINVAL, "ktf_fit_noalloc: the current device (%d) is not the context's (%d)", dev,
                c->device);
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr(dev));
  if (!base) return fail(c, KTF_EDEVICE, "ktf_fit_noalloc: no scratch address for device %d", dev);
  if (in->n == 0) return KTF_OK;
  FitArgs a = make_fit_args(c, in, out);
  int bs = 256, waves = 1, tpl = 1;
  bool persistent = false;
  switch (mode) {
    case KTF_FIT_AUTO: (void)tuned_launch(c, in->prec, in->n, bs, waves, tpl, persistent); break;
    case KTF_FIT_FUSED: break;
    case KTF_FIT_PERSISTENT: persistent = true; break;
    case KTF_FIT_SWEEP: {
      if (in->prec == KTF_FP32_PROP)
        return fail(c, KTF_EINVAL, "ktf_fit_noalloc: KTF_FP32_PROP keeps the covariance in registers; use a fused mode");
      if (in->n_passes > 1) return fail(c, KTF_EINVAL, "ktf_fit_noalloc: the iterated refit runs in the fused modes");
      const size_t need = sweep_bytes(in->pitch, in->prec);
      if (need > (size_t)KTF_NOALLOC_SCRATCH_BYTES)
        return fail(c, KTF_EINVAL,
                    "ktf_fit_noalloc: a sweep over pitch %lld needs %zu scratch bytes, more than the %zu available",
                    (long long)in->pitch, need, (size_t)KTF_NOALLOC_SCRATCH_BYTES);
      a.lend = base + kScratchCounterBytes;
      if (in->prec == KTF_FP32_BULK)
        a.pos_ws = reinterpret_cast<double*>(base + kScratchCounterBytes + round256((size_t)in->pitch));
      for (int l = 0; l < a.n_layers && e == hipSuccess; ++l) e = launch_fit_layer(a, in->prec, l, st);
      return e == hipSuccess ? KTF_OK : hip_fail(c, e, "ktf_fit_noalloc: layer launch");
    }
    case KTF_FIT_SWEEP_GRAPH:
      return fail(c, KTF_EINVAL, "ktf_fit_noalloc: building a graph allocates; use KTF_FIT_SWEEP");
    default: return fail(c, KTF_EINVAL, "ktf_fit_noalloc: unknown mode %d", (int)mode);
  }
  int pblocks = 0;
  if (persistent && in->n_passes <= 1) {
    a.counters = reinterpret_cast<unsigned long long*>(base);
    const int tile = a.mat.on ? bs : bs * tpl;
    a.tile_count = (a.n + tile - 1) / tile;
    pblocks = persistent_blocks(c, in->prec, bs, waves, tpl) * c->n_cu;
    if (pblocks <= 0) pblocks = c->n_cu;
    // a fill kernel, not a memset: a caller may capture this call in a graph
    if ((e = launch_fill_u64(a.counters, 1, 0ull, st)) != hipSuccess)
      return hip_fail(c, e, "ktf_fit_noalloc: counter reset");
  }
  e = launch_fit_fused(a, in->prec, bs, waves, tpl, persistent && in->n_passes <= 1, pblocks, st);
  return e == hipSuccess ? KTF_OK : hip_fail(c, e, "ktf_fit_noalloc: launch");
}

}  // namespace ktf

extern "C" int ktf_fit_noalloc(ktf_ctx* c, const ktf_fit_in* in, ktf_fit_out* out, ktf_fit_mode mode,
                               void* hip_stream) {
  if (!c || !in || !out) return KTF_EINVAL;
  return ktf::fit_noalloc(c, in, out, mode, static_cast<hipStream_t>(hip_stream));
}
