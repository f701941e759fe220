// ktf_internal.hpp -- kernel argument blocks and launchers shared by the
// library's translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ktf.h"

namespace ktf {

struct HitResD {
  double sr2, srphi2, sz2;
};

// Arguments of the fit kernels (passed by value in the kernarg segment).
// layer material (see ktf_config): thickness per layer, energy loss, mass
struct MaterialD {
  double x0[KTF_MAX_LAYERS];
  double eloss, mass;
  int32_t on;
};

struct FitArgs {
  int64_t n, pitch;
  const void* state;
  const void* cov;
  const int8_t* q;
  const void* hits;
  const uint8_t* valid;
  void* state_o;
  void* cov_o;
  double* chi2;
  int32_t* nupd;
  uint32_t* status;
  uint8_t* lend;        // sweep: per-track end layer (workspace)
  double* pos_ws;       // sweep, float storage: positions in double between layers [3][pitch]
  unsigned long long* counters;  // persistent: tile counters
  int64_t tile_count;   // persistent: number of tiles
  int32_t n_layers;
  int32_t n_passes;     // fused fits: passes of the iterated refit, >= 1
  double bz;
  HitResD hr;
  double radii[KTF_MAX_LAYERS];
  MaterialD mat;
};

// launch shapes of the fused fit
constexpr int kBlockSizes[4] = {64, 128, 256, 512};
constexpr int kWaveChoices = 3;  // register budgets tried: 1 (compiler's), 2 and 3 waves per SIMD
constexpr int kTplChoices = 2;   // tracks per lane tried: 1 and 2

// waves: 1, 2 or 3, the waves per SIMD the fused kernel's registers must
// allow; tpl: tracks per lane, 1 or 2 (2 only for one pass without material)
hipError_t launch_fit_fused(const FitArgs& a, ktf_precision prec, int bs, int waves, int tpl, bool persistent,
                            int persistent_blocks, hipStream_t st);
hipError_t launch_fit_layer(const FitArgs& a, ktf_precision prec, int layer, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);

// ------------------------------------------------------------------ build
struct BuildGeom {
  // n_zbins: rows of bins per layer, z bins, or eta bins when eta_rows
  int32_t n_layers, n_zbins, n_phibins, max_cands, max_missed, n_seed_layers;
  int32_t eta_rows;  // 1: rows are eta bins over |eta| < eta_max
  double bz, z_half, chi2_cut, eta_max;
  // rows per unit of the row coordinate (z, or eta when eta_rows) and phi
  // bins per radian, n_zbins / (2 z_half or 2 eta_max) and n_phibins /
  // (2 pi), for the search windows, whose bounds need only be conservative
  double row_scale, phi_scale;
  HitResD hr;
  double radii[KTF_MAX_LAYERS];
  MaterialD mat;
};

}  // namespace ktf
