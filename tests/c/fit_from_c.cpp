// fit_from_c.cpp -- the fit driven through the C-ABI from a plain host
// program, with device memory from the HIP runtime and no Python or torch.
//
// usage: fit_from_c <input> <output> <mode>
//   input  (little-endian): int32 n, L; double bz, sigma_r, sigma_rphi,
//          sigma_z, z_half; double radii[L]; double state[6][n],
//          cov[21][n], hits[L][3][n]; int8 q[n]; uint8 valid[L][n]
//   output: double state[6][n], cov[21][n], chi2[n]; int32 n_upd[n];
//           uint32 status[n]
//   mode   ktf_fit_mode as an integer
// Exits 0 on success; prints the library's message and exits 1 otherwise.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/ktf.h"

static void die(const char* what) {
  std::fprintf(stderr, "fit_from_c: %s\n", what);
  std::exit(1);
}

template <typename T>
static void read_n(FILE* f, T* p, size_t n) {
  if (std::fread(p, sizeof(T), n, f) != n) die("short input");
}

template <typename T>
static T* to_device(const std::vector<T>& h) {
  T* d = nullptr;
  if (hipMalloc(&d, h.size() * sizeof(T) + 1) != hipSuccess) die("hipMalloc");
  if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    die("hipMemcpy");
  return d;
}

int main(int argc, char** argv) {
  if (argc != 4) die("usage: fit_from_c <input> <output> <mode>");
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) die("cannot open input");
  int32_t n, L;
  double g[5];
  read_n(f, &n, 1);
  read_n(f, &L, 1);
  read_n(f, g, 5);
  std::vector<double> radii(L), state(6 * (size_t)n), cov(21 * (size_t)n), hits((size_t)L * 3 * n);
  std::vector<int8_t> q(n);
  std::vector<uint8_t> valid((size_t)L * n);
  read_n(f, radii.data(), radii.size());
  read_n(f, state.data(), state.size());
  read_n(f, cov.data(), cov.size());
  read_n(f, hits.data(), hits.size());
  read_n(f, q.data(), q.size());
  read_n(f, valid.data(), valid.size());
  std::fclose(f);

  if (ktf_config_bytes() != sizeof(ktf_config)) die("ktf_config differs between this program and the library");
  ktf_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  cfg.n_layers = L;
  cfg.layer_r = radii.data();
  cfg.bz = g[0];
  cfg.sigma_r = g[1];
  cfg.sigma_rphi = g[2];
  cfg.sigma_z = g[3];
  cfg.z_half = g[4];
  cfg.n_zbins = 64;
  cfg.n_phibins = 512;
  cfg.max_cands = 10;
  cfg.max_missed = 1;
  cfg.n_seed_layers = L < 3 ? L : 3;
  cfg.chi2_cut = 30.0;
  cfg.hbm_budget_bytes = 1ull << 30;
  cfg.max_inflight = 4;
  cfg.layer_x0 = nullptr;
  cfg.mass = 0.13957;
  ktf_ctx* ctx = nullptr;
  if (ktf_create(&cfg, &ctx) != KTF_OK) die("ktf_create");

  ktf_fit_in in;
  std::memset(&in, 0, sizeof in);
  in.n = n;
  in.pitch = n;
  in.prec = KTF_FP64;
  in.seed_state = to_device(state);
  in.seed_cov = to_device(cov);
  in.charge = to_device(q);
  in.hits = to_device(hits);
  in.hit_valid = to_device(valid);
  in.n_passes = 1;
  std::vector<double> o_state(6 * (size_t)n), o_cov(21 * (size_t)n), o_chi2(n);
  std::vector<int32_t> o_nupd(n);
  std::vector<uint32_t> o_status(n);
  ktf_fit_out out;
  out.state = to_device(o_state);
  out.cov = to_device(o_cov);
  out.chi2 = to_device(o_chi2);
  out.n_upd = to_device(o_nupd);
  out.status = to_device(o_status);

  hipStream_t st;
  if (hipStreamCreate(&st) != hipSuccess) die("hipStreamCreate");
  if (ktf_fit(ctx, &in, &out, (ktf_fit_mode)std::atoi(argv[3]), st) != KTF_OK) {
    std::fprintf(stderr, "fit_from_c: ktf_fit: %s\n", ktf_last_error(ctx));
    return 1;
  }
  if (hipStreamSynchronize(st) != hipSuccess) die("hipStreamSynchronize");
  auto back = [](void* d, void* h, size_t bytes) {
    if (hipMemcpy(h, d, bytes, hipMemcpyDeviceToHost) != hipSuccess) die("hipMemcpy back");
  };
  back(out.state, o_state.data(), o_state.size() * 8);
  back(out.cov, o_cov.data(), o_cov.size() * 8);
  back(out.chi2, o_chi2.data(), o_chi2.size() * 8);
  back(out.n_upd, o_nupd.data(), o_nupd.size() * 4);
  back(out.status, o_status.data(), o_status.size() * 4);

  FILE* o = std::fopen(argv[2], "wb");
  if (!o) die("cannot open output");
  std::fwrite(o_state.data(), 8, o_state.size(), o);
  std::fwrite(o_cov.data(), 8, o_cov.size(), o);
  std::fwrite(o_chi2.data(), 8, o_chi2.size(), o);
  std::fwrite(o_nupd.data(), 4, o_nupd.size(), o);
  std::fwrite(o_status.data(), 4, o_status.size(), o);
  std::fclose(o);

  for (const void* p : {in.seed_state, in.seed_cov, (const void*)in.charge, in.hits, (const void*)in.hit_valid})
    (void)hipFree(const_cast<void*>(p));
  for (void* p : {out.state, out.cov, (void*)out.chi2, (void*)out.n_upd, (void*)out.status}) (void)hipFree(p);
  (void)hipStreamDestroy(st);
  ktf_destroy(ctx);
  return 0;
}
