// fit.hip -- batched Kalman-filter track fit kernels for gfx950.
//
// One track per lane.  Inputs and outputs are structure-of-arrays with a
// common pitch, so lane i of a wave touches element i of every row and each
// row access is one coalesced 256-byte (float) or 512-byte (double) wave
// transaction.  The fit of a track is the Kalman filter of Sec. 2 run over
// its layers: propagate to the next cylinder, update with the hit there.
//
// Variants:
//  fused       all layers of a track in registers, read the seed and the
//              hits once, write the result once (the arithmetic-bound design)
//  persistent  the fused body in a fixed grid of blocks that pull tiles of
//              tracks from a device counter until the tiles run out, which
//              evens out tracks with very different hit counts
//  layer       one layer of every track per launch; the state and covariance
//              round-trip HBM between launches (the memory-bound design used
//              for per-layer graph sweeps)
#include "kf_math.hpp"
#include "ctx.hpp"

namespace ktf {

template <typename T> struct NewtonIters;
template <> struct NewtonIters<double> { static constexpr int n = 3; };
template <> struct NewtonIters<float> { static constexpr int n = 2; };

// One pass of the filter over a track's layers from the start state (x, P):
// x and P end as the filtered state at the last layer reached (layer `at`,
// -1 if none).  Storage type TS,
// propagation type TP (state, path solve, transport, Jacobian), covariance
// type TC (registers, F P F^T and update).  MAT: the layers carry material,
// applied to a copy of the state when it leaves a layer (the filtered state
// stays the result if the next layer is missed).
template <typename TS, typename TP, typename TC, bool MAT>
__device__ __forceinline__ void fit_pass(const FitArgs& a, int64_t i, uint32_t vmask, TP k,
                                         TrackState<TP>& x, TC P[21], double& chi2, int32_t& nupd,
                                         uint32_t& status, int& at) {
  const int64_t p = a.pitch;
  const int lend = vmask ? 32 - __builtin_clz(vmask) : 1;
  const HitRes hr{a.hr.sr2, a.hr.srphi2, a.hr.sz2};
  chi2 = 0.0;
  nupd = 0;
  status = 0;
  at = -1;
  const TS* hits = static_cast<const TS*>(a.hits);
  // the next layer's hit is loaded one layer ahead so that its latency
  // hides behind the current layer's arithmetic
  TS hn0 = TS(0), hn1 = TS(0), hn2 = TS(0);
  if (vmask & 1u) {
    hn0 = hits[i];
    hn1 = hits[p + i];
    hn2 = hits[2 * p + i];
  }
  for (int l = 0; l < lend; ++l) {
    const double m[3] = {(double)hn0, (double)hn1, (double)hn2};
    if (l + 1 < lend && ((vmask >> (l + 1)) & 1u)) {
      const TS* h = hits + (int64_t)(l + 1) * 3 * p;
      hn0 = h[i];
      hn1 = h[p + i];
      hn2 = h[2 * p + i];
    }
    TrackState<TP> xp;
    Jac<TP> F;
    TC Pp[21];
    if constexpr (MAT) {
      TrackState<TP> xm = x;
      TC Pm[21];
#pragma unroll
      for (int c = 0; c < 21; ++c) Pm[c] = P[c];
      if (l > 0 && a.mat.x0[l - 1] > 0.0) apply_material(a.mat.x0[l - 1], a.mat.eloss, a.mat.mass, xm, Pm);
      if (!propagate<TP, NewtonIters<TP>::n>(xm, k, a.radii[l], l == 0, xp, F)) {
        status |= kNoReach;
        break;
      }
      cov_propagate(Pm, F, Pp);
    } else {
      if (!propagate<TP, NewtonIters<TP>::n>(x, k, a.radii[l], l == 0, xp, F)) {
        status |= kNoReach;
        break;
      }
      cov_propagate(P, F, Pp);
    }
    at = l;
    // the update works in place on the propagated state, so that a layer
    // without an update needs no per-lane selection of the result
    if ((vmask >> l) & 1u) {
      Residual R;
      if (residual(xp, Pp, m, hr, R)) {
        apply_update(xp, Pp, R, xp, Pp);
        chi2 += R.chi2;
        ++nupd;
      } else {
        status |= kSNotPD;
      }
    }
    x = xp;
#pragma unroll
    for (int c = 0; c < 21; ++c) P[c] = Pp[c];
    if (!finite_state(x, P)) {
      status |= kNonFinite;
      break;
    }
  }
}

// The state on layer `from` carried back to layer 0 along its helix: the
// same helix travelled with reversed momentum and charge, one layer at a
// time, giving back the mean energy lost when leaving each crossed layer.
template <typename TP, bool MAT>
__device__ __forceinline__ bool carry_back(const FitArgs& a, TP k, int from, TrackState<TP>& x) {
  for (int l = from - 1; l >= 0; --l) {
    TrackState<TP> xr = x, xo;
#pragma unroll
    for (int c = 0; c < 3; ++c) xr.mom[c] = -x.mom[c];
    Jac<TP> F;
    if (!propagate<TP, NewtonIters<TP>::n>(xr, -k, a.radii[l], true, xo, F)) return false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x.pos[c] = xo.pos[c];
      x.mom[c] = -xo.mom[c];
    }
    if constexpr (MAT) {
      if (a.mat.x0[l] > 0.0 && a.mat.eloss > 0.0) undo_energy_loss(a.mat.x0[l], a.mat.eloss, a.mat.mass, x);
    }
  }
  return true;
}

// The fit of one track: one pass, or (REFIT) an iterated refit over
// a.n_passes passes: each further pass refits from the previous pass's
// result carried back to layer 0, with the seed covariance.  A pass that
// sets a status bit the pass before did not is dropped and ends the refit,
// as does a result that is non-finite or cannot be carried back; the kept
// pass's result stays in the outputs.  The single pass is its own
// instantiation so that it keeps its register allocation.
template <typename TS, typename TP, typename TC, bool MAT, bool REFIT>
__device__ __forceinline__ void fit_one_track(const FitArgs& a, int64_t i) {
  const int64_t p = a.pitch;
  const TS* st = static_cast<const TS*>(a.state);
  const TS* cv = static_cast<const TS*>(a.cov);
  TrackState<TP> x;
  TC P[21];
#pragma unroll
  for (int c = 0; c < 3; ++c) x.pos[c] = (double)st[c * p + i];
#pragma unroll
  for (int c = 0; c < 3; ++c) x.mom[c] = (TP)st[(c + 3) * p + i];
#pragma unroll
  for (int c = 0; c < 21; ++c) P[c] = (TC)cv[c * p + i];
  const TP k = (TP)(kCLight * (double)a.q[i] * a.bz);
  uint32_t vmask = 0;
  for (int l = 0; l < a.n_layers; ++l)
    if (a.valid == nullptr || a.valid[l * p + i]) vmask |= 1u << l;
  TS* so = static_cast<TS*>(a.state_o);
  TS* co = static_cast<TS*>(a.cov_o);
  uint32_t kept = 0;
  const int npass = REFIT ? a.n_passes : 1;
  for (int pass = 0; pass < npass; ++pass) {
    if (pass > 0) {  // the seed covariance again
#pragma unroll
      for (int c = 0; c < 21; ++c) P[c] = (TC)cv[c * p + i];
    }
    double chi2;
    int32_t nupd;
    uint32_t status;
    int at;
    fit_pass<TS, TP, TC, MAT>(a, i, vmask, k, x, P, chi2, nupd, status, at);
    if (pass > 0 && status != 0 && kept == 0) break;
    // the results are written once and not read back by the kernel: the
    // non-temporal hint leaves the caches to the inputs (0.285 -> 0.272 ms
    // for 1e6 tracks x 10 layers in float propagation)
#pragma unroll
    for (int c = 0; c < 3; ++c) __builtin_nontemporal_store((TS)x.pos[c], so + c * p + i);
#pragma unroll
    for (int c = 0; c < 3; ++c) __builtin_nontemporal_store((TS)x.mom[c], so + (c + 3) * p + i);
#pragma unroll
    for (int c = 0; c < 21; ++c) __builtin_nontemporal_store((TS)P[c], co + c * p + i);
    __builtin_nontemporal_store(chi2, a.chi2 + i);
    __builtin_nontemporal_store(nupd, a.nupd + i);
    __builtin_nontemporal_store(status, a.status + i);
    kept = status;
    if constexpr (!REFIT) break;
    if (pass + 1 >= npass || (status & kNonFinite) || at < 0 || !carry_back<TP, MAT>(a, k, at, x)) break;
  }
}

// Two tracks per lane (register tiling): the lane fits tracks i and i + BS
// (so that each row access of the wave stays one coalesced transaction),
// layer by layer, the two tracks' work on a layer side by side, so that one
// track's arithmetic can cover the other's latencies.  One pass, no
// material: the same arithmetic per track as fit_pass, whose results it
// reproduces bit for bit.
template <typename TS, typename TP, typename TC, int TPL>
__device__ __forceinline__ void fit_tile(const FitArgs& a, int64_t i0, int64_t stride) {
  const int64_t p = a.pitch;
  const HitRes hr{a.hr.sr2, a.hr.srphi2, a.hr.sz2};
  const TS* st = static_cast<const TS*>(a.state);
  const TS* cv = static_cast<const TS*>(a.cov);
  const TS* hits = static_cast<const TS*>(a.hits);
  TrackState<TP> x[TPL];
  TC P[TPL][21];
  TP k[TPL];
  uint32_t vmask[TPL], status[TPL];
  int lend[TPL];
  double chi2[TPL];
  int32_t nupd[TPL];
  bool live[TPL];
  int lmax = 0;
#pragma unroll
  for (int j = 0; j < TPL; ++j) {
    const int64_t i = i0 + j * stride;
    live[j] = i < a.n;
    const int64_t ic = live[j] ? i : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) x[j].pos[c] = (double)st[c * p + ic];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[j].mom[c] = (TP)st[(c + 3) * p + ic];
#pragma unroll
    for (int c = 0; c < 21; ++c) P[j][c] = (TC)cv[c * p + ic];
    k[j] = (TP)(kCLight * (double)a.q[ic] * a.bz);
    vmask[j] = 0;
    for (int l = 0; l < a.n_layers; ++l)
      if (a.valid == nullptr || a.valid[l * p + ic]) vmask[j] |= 1u << l;
    lend[j] = live[j] ? (vmask[j] ? 32 - __builtin_clz(vmask[j]) : 1) : 0;
    lmax = lend[j] > lmax ? lend[j] : lmax;
    chi2[j] = 0.0;
    nupd[j] = 0;
    status[j] = 0;
  }
  for (int l = 0; l < lmax; ++l) {
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
      if (!live[j] || l >= lend[j]) continue;
      const int64_t i = i0 + j * stride;
      double m[3] = {0.0, 0.0, 0.0};
      const bool has = (vmask[j] >> l) & 1u;
      if (has) {
        const TS* h = hits + (int64_t)l * 3 * p;
        m[0] = (double)h[i];
        m[1] = (double)h[p + i];
        m[2] = (double)h[2 * p + i];
      }
      TrackState<TP> xp;
      Jac<TP> F;
      if (!propagate<TP, NewtonIters<TP>::n>(x[j], k[j], a.radii[l], l == 0, xp, F)) {
        status[j] |= kNoReach;
        live[j] = false;
        continue;
      }
      TC Pp[21];
      cov_propagate(P[j], F, Pp);
      if (has) {
        Residual R;
        if (residual(xp, Pp, m, hr, R)) {
          apply_update(xp, Pp, R, xp, Pp);
          chi2[j] += R.chi2;
          ++nupd[j];
        } else {
          status[j] |= kSNotPD;
        }
      }
      x[j] = xp;
#pragma unroll
      for (int c = 0; c < 21; ++c) P[j][c] = Pp[c];
      if (!finite_state(x[j], P[j])) {
        status[j] |= kNonFinite;
        live[j] = false;
      }
    }
  }
  TS* so = static_cast<TS*>(a.state_o);
  TS* co = static_cast<TS*>(a.cov_o);
#pragma unroll
  for (int j = 0; j < TPL; ++j) {
    const int64_t i = i0 + j * stride;
    if (i >= a.n) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) __builtin_nontemporal_store((TS)x[j].pos[c], so + c * p + i);
#pragma unroll
    for (int c = 0; c < 3; ++c) __builtin_nontemporal_store((TS)x[j].mom[c], so + (c + 3) * p + i);
#pragma unroll
    for (int c = 0; c < 21; ++c) __builtin_nontemporal_store((TS)P[j][c], co + c * p + i);
    __builtin_nontemporal_store(chi2[j], a.chi2 + i);
    __builtin_nontemporal_store(nupd[j], a.nupd + i);
    __builtin_nontemporal_store(status[j], a.status + i);
  }
}

// W: the waves per SIMD the register allocation must allow (1 leaves it to
// the compiler; more trades registers, and maybe spills, for latency
// hiding); TPL: tracks per lane (2: fit_tile, one pass without material)
template <typename TS, typename TP, typename TC, int BS, int W, bool MAT, bool REFIT = false, int TPL = 1>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(W))) void fit_fused_kernel(FitArgs a) {
  if constexpr (TPL == 1) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i < a.n) fit_one_track<TS, TP, TC, MAT, REFIT>(a, i);
  } else {
    fit_tile<TS, TP, TC, TPL>(a, (int64_t)blockIdx.x * BS * TPL + threadIdx.x, BS);
  }
}

// Persistent blocks: every block loops taking the next tile of BS * TPL
// tracks from counters[0]; all waves leave once the tile index passes
// tile_count.
template <typename TS, typename TP, typename TC, int BS, int W, bool MAT, int TPL = 1>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(W))) void fit_persistent_kernel(FitArgs a) {
  __shared__ long long tile;
  for (;;) {
    if (threadIdx.x == 0) tile = (long long)atomicAdd(&a.counters[0], 1ull);
    __syncthreads();
    const long long t = tile;
    __syncthreads();
    if (t >= a.tile_count) break;
    if constexpr (TPL == 1) {
      const int64_t i = t * BS + threadIdx.x;
      if (i < a.n) fit_one_track<TS, TP, TC, MAT, false>(a, i);
    } else {
      fit_tile<TS, TP, TC, TPL>(a, t * BS * TPL + threadIdx.x, BS);
    }
  }
}

// One layer of every track.  Layer 0 reads the seed and initialises the
// outputs and the per-track end layer; later layers work in place on the
// outputs.  A track that has stopped (NO_REACH / NONFINITE) or is past its
// last hit is left untouched.
// Three waves per SIMD fit without spills in both precisions (this kernel
// is bound by HBM latency, so occupancy matters).
template <typename TS, typename TP, int BS, bool MAT>
// The state, covariance and carried position are touched once per launch:
// their loads and stores carry the non-temporal hint (ten layers of 1e6
// tracks: 0.641 -> 0.627-0.635 ms in paired runs, the same within the
// spread under the profiler).
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void fit_layer_kernel(FitArgs a, int l) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= a.n) return;
  const int64_t p = a.pitch;
  int lend;
  uint32_t status;
  double chi2;
  int32_t nupd;
  const TS* st;
  const TS* cv;
  if (l == 0) {
    uint32_t vmask = 0;
    for (int ll = 0; ll < a.n_layers; ++ll)
      if (a.valid == nullptr || a.valid[ll * p + i]) vmask |= 1u << ll;
    lend = vmask ? 32 - __builtin_clz(vmask) : 1;
    a.lend[i] = (uint8_t)lend;
    status = 0;
    chi2 = 0.0;
    nupd = 0;
    st = static_cast<const TS*>(a.state);
    cv = static_cast<const TS*>(a.cov);
  } else {
    lend = a.lend[i];
    status = a.status[i];
    if (l >= lend || (status & (kNoReach | kNonFinite))) return;
    chi2 = a.chi2[i];
    nupd = a.nupd[i];
    st = static_cast<const TS*>(a.state_o);
    cv = static_cast<const TS*>(a.cov_o);
  }
  TrackState<TP> x;
  TP P[21];
  if (l == 0 || a.pos_ws == nullptr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) x.pos[c] = (double)__builtin_nontemporal_load(st + c * p + i);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) x.pos[c] = __builtin_nontemporal_load(a.pos_ws + c * p + i);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) x.mom[c] = (TP)__builtin_nontemporal_load(st + (c + 3) * p + i);
#pragma unroll
  for (int c = 0; c < 21; ++c) P[c] = (TP)__builtin_nontemporal_load(cv + c * p + i);
  const TP k = (TP)(kCLight * (double)a.q[i] * a.bz);
  const HitRes hr{a.hr.sr2, a.hr.srphi2, a.hr.sz2};
  // the material of the layer being left; the stored (filtered) state stays
  // the result if the next layer is missed
  if constexpr (MAT) {
    if (l > 0 && a.mat.x0[l - 1] > 0.0) apply_material(a.mat.x0[l - 1], a.mat.eloss, a.mat.mass, x, P);
  }
  TrackState<TP> xp;
  Jac<TP> F;
  if (!propagate<TP, NewtonIters<TP>::n>(x, k, a.radii[l], l == 0, xp, F)) {
    status |= kNoReach;
    if (l > 0) {
      // the track ends with the layer before: its position, carried in
      // double between layers, becomes the stored one now
      if (a.pos_ws != nullptr) {
        TS* so = static_cast<TS*>(a.state_o);
#pragma unroll
        for (int c = 0; c < 3; ++c) so[c * p + i] = (TS)x.pos[c];
      }
      a.status[i] = status;
      return;
    }
  } else {
    TP Pp[21];
    cov_propagate(P, F, Pp);
    if (a.valid == nullptr || a.valid[l * p + i]) {
      const TS* h = static_cast<const TS*>(a.hits) + (int64_t)l * 3 * p;
      const double m[3] = {(double)h[i], (double)h[p + i], (double)h[2 * p + i]};
      Residual R;
      if (residual(xp, Pp, m, hr, R)) {
        apply_update(xp, Pp, R, xp, Pp);  // in place
        chi2 += R.chi2;
        ++nupd;
      } else {
        status |= kSNotPD;
      }
    }
    x = xp;
#pragma unroll
    for (int c = 0; c < 21; ++c) P[c] = Pp[c];
    if (!finite_state(x, P)) status |= kNonFinite;
  }
  TS* so = static_cast<TS*>(a.state_o);
  TS* co = static_cast<TS*>(a.cov_o);
  // float storage: positions are carried in double between layers and
  // stored in the storage type only where the track ends (its last layer
  // with a hit, or a layer it cannot leave: not reaching the next one is
  // handled above, a state that is not finite stops it here)
  const bool last = a.pos_ws == nullptr || l + 1 >= lend || (status & (kNoReach | kNonFinite));
  if (a.pos_ws != nullptr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(x.pos[c], a.pos_ws + c * p + i);
  }
  if (last) {
#pragma unroll
    for (int c = 0; c < 3; ++c) so[c * p + i] = (TS)x.pos[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) __builtin_nontemporal_store((TS)x.mom[c], so + (c + 3) * p + i);
#pragma unroll
  for (int c = 0; c < 21; ++c) __builtin_nontemporal_store((TS)P[c], co + c * p + i);
  a.chi2[i] = chi2;
  a.nupd[i] = nupd;
  a.status[i] = status;
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, p, n, v);
  return hipGetLastError();
}

template <typename TS, typename TP, typename TC, int BS, int W, bool MAT, int TPL>
static hipError_t launch_fused_m(const FitArgs& a, bool persistent, int pblocks, hipStream_t st) {
  if (persistent) {
    hipLaunchKernelGGL((fit_persistent_kernel<TS, TP, TC, BS, W, MAT, TPL>), dim3(pblocks), dim3(BS), 0, st, a);
  } else {
    const int64_t nb = (a.n + BS * TPL - 1) / (BS * TPL);
    hipLaunchKernelGGL((fit_fused_kernel<TS, TP, TC, BS, W, MAT, false, TPL>), dim3((unsigned)nb), dim3(BS), 0, st, a);
  }
  return hipGetLastError();
}

// two tracks per lane only without material (the material fit keeps its
// own single-track kernels)
template <typename TS, typename TP, typename TC, int BS, int W>
static hipError_t launch_fused_bs(const FitArgs& a, int tpl, bool persistent, int pblocks, hipStream_t st) {
  if (a.mat.on) return launch_fused_m<TS, TP, TC, BS, W, true, 1>(a, persistent, pblocks, st);
  return tpl == 2 ? launch_fused_m<TS, TP, TC, BS, W, false, 2>(a, persistent, pblocks, st)
                  : launch_fused_m<TS, TP, TC, BS, W, false, 1>(a, persistent, pblocks, st);
}

// the iterated refit: one launch shape (256 threads, the compiler's
// register allocation, plain grid)
template <typename TS, typename TP, typename TC>
static hipError_t launch_refit(const FitArgs& a, hipStream_t st) {
  constexpr int BS = 256;
  const unsigned nb = (unsigned)((a.n + BS - 1) / BS);
  if (a.mat.on)
    hipLaunchKernelGGL((fit_fused_kernel<TS, TP, TC, BS, 1, true, true>), dim3(nb), dim3(BS), 0, st, a);
  else
    hipLaunchKernelGGL((fit_fused_kernel<TS, TP, TC, BS, 1, false, true>), dim3(nb), dim3(BS), 0, st, a);
  return hipGetLastError();
}

template <typename TS, typename TP, typename TC, int W>
static hipError_t launch_fused_w(const FitArgs& a, int bs, int tpl, bool persistent, int pblocks, hipStream_t st) {
  switch (bs) {
    case 64: return launch_fused_bs<TS, TP, TC, 64, W>(a, tpl, persistent, pblocks, st);
    case 128: return launch_fused_bs<TS, TP, TC, 128, W>(a, tpl, persistent, pblocks, st);
    case 256: return launch_fused_bs<TS, TP, TC, 256, W>(a, tpl, persistent, pblocks, st);
    case 512: return launch_fused_bs<TS, TP, TC, 512, W>(a, tpl, persistent, pblocks, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename TS, typename TP, typename TC>
static hipError_t launch_fused_t(const FitArgs& a, int bs, int waves, int tpl, bool persistent, int pblocks,
                                 hipStream_t st) {
  switch (waves) {
    case 1: return launch_fused_w<TS, TP, TC, 1>(a, bs, tpl, persistent, pblocks, st);
    case 2: return launch_fused_w<TS, TP, TC, 2>(a, bs, tpl, persistent, pblocks, st);
    case 3: return launch_fused_w<TS, TP, TC, 3>(a, bs, tpl, persistent, pblocks, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fit_fused(const FitArgs& a, ktf_precision prec, int bs, int waves, int tpl, bool persistent,
                            int persistent_blocks, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n_passes > 1) {  // a double covariance (checked at the boundary)
    if (prec == KTF_FP64) return launch_refit<double, double, double>(a, st);
    return launch_refit<float, float, double>(a, st);
  }
  if (prec == KTF_FP64)
    return launch_fused_t<double, double, double>(a, bs, waves, tpl, persistent, persistent_blocks, st);
  if (prec == KTF_FP32_PROP)
    return launch_fused_t<float, float, double>(a, bs, waves, tpl, persistent, persistent_blocks, st);
  return launch_fused_t<float, float, float>(a, bs, waves, tpl, persistent, persistent_blocks, st);
}

hipError_t launch_fit_layer(const FitArgs& a, ktf_precision prec, int layer, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  constexpr int BS = 256;
  const unsigned nb = (unsigned)((a.n + BS - 1) / BS);
  if (prec == KTF_FP64 && a.mat.on)
    hipLaunchKernelGGL((fit_layer_kernel<double, double, BS, true>), dim3(nb), dim3(BS), 0, st, a, layer);
  else if (prec == KTF_FP64)
    hipLaunchKernelGGL((fit_layer_kernel<double, double, BS, false>), dim3(nb), dim3(BS), 0, st, a, layer);
  else if (a.mat.on)
    hipLaunchKernelGGL((fit_layer_kernel<float, float, BS, true>), dim3(nb), dim3(BS), 0, st, a, layer);
  else
    hipLaunchKernelGGL((fit_layer_kernel<float, float, BS, false>), dim3(nb), dim3(BS), 0, st, a, layer);
  return hipGetLastError();
}

}  // namespace ktf

namespace ktf {

template <typename TS, typename TP, typename TC, int W, bool MAT, int TPL>
static int occ_blocks_w(int bs) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (bs) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_persistent_kernel<TS, TP, TC, 64, W, MAT, TPL>, 64, 0); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_persistent_kernel<TS, TP, TC, 128, W, MAT, TPL>, 128, 0); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_persistent_kernel<TS, TP, TC, 256, W, MAT, TPL>, 256, 0); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_persistent_kernel<TS, TP, TC, 512, W, MAT, TPL>, 512, 0); break;
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

template <typename TS, typename TP, typename TC, bool MAT, int TPL>
static int occ_blocks(int bs, int waves) {
  switch (waves) {
    case 1: return occ_blocks_w<TS, TP, TC, 1, MAT, TPL>(bs);
    case 2: return occ_blocks_w<TS, TP, TC, 2, MAT, TPL>(bs);
    case 3: return occ_blocks_w<TS, TP, TC, 3, MAT, TPL>(bs);
    default: return 0;
  }
}

template <bool MAT, int TPL>
static int persistent_blocks_m(ktf_precision prec, int bs, int waves) {
  if (prec == KTF_FP64) return occ_blocks<double, double, double, MAT, TPL>(bs, waves);
  if (prec == KTF_FP32_PROP) return occ_blocks<float, float, double, MAT, TPL>(bs, waves);
  return occ_blocks<float, float, float, MAT, TPL>(bs, waves);
}

int persistent_blocks(ktf_ctx* c, ktf_precision prec, int bs, int waves, int tpl) {
  if (!c->x0.empty()) return persistent_blocks_m<true, 1>(prec, bs, waves);
  return tpl == 2 ? persistent_blocks_m<false, 2>(prec, bs, waves) : persistent_blocks_m<false, 1>(prec, bs, waves);
}

}  // namespace ktf
