// serve.hip -- continuous-batching request loop.
#include <chrono>

#include "ctx.hpp"

namespace ktf {
struct ServeState {};
void serve_shutdown(ktf_ctx* c) {
  delete c->serve;
  c->serve = nullptr;
}
}  // namespace ktf

extern "C" {
double ktf_now(void) {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}
int ktf_submit(ktf_ctx* c, const ktf_event_host*, uint64_t*) {
  return ktf::fail(c, KTF_EINVAL, "ktf_submit: not available in this build");
}
int ktf_poll(ktf_ctx* c, uint64_t, ktf_result_host*) {
  return ktf::fail(c, KTF_EINVAL, "ktf_poll: not available in this build");
}
int ktf_serving_stats(ktf_ctx* c, int64_t* q, int64_t* f, int64_t* d) {
  if (!c) return KTF_EINVAL;
  if (q) *q = 0;
  if (f) *f = 0;
  if (d) *d = 0;
  return KTF_OK;
}
}
