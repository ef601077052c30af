// Serving loop entry points (placeholder until the batching engine lands).
#include "gym_internal.hpp"

using namespace gym;

extern "C" {

int gym_serve_start(const gym_serve_opts* opts, gym_server** out) {
  (void)opts;
  if (out) *out = nullptr;
  return fail(GYM_E_UNSUPPORTED, "serving loop not built yet");
}

int gym_serve_submit(gym_server* srv, const gym_request* req, uint64_t* id) {
  (void)srv;
  (void)req;
  (void)id;
  return fail(GYM_E_UNSUPPORTED, "serving loop not built yet");
}

int gym_serve_poll(gym_server* srv, uint64_t id, gym_result* res, double* x_host) {
  (void)srv;
  (void)id;
  (void)res;
  (void)x_host;
  return fail(GYM_E_UNSUPPORTED, "serving loop not built yet");
}

int gym_serve_stop(gym_server* srv) {
  (void)srv;
  return fail(GYM_E_UNSUPPORTED, "serving loop not built yet");
}

}  // extern "C"
