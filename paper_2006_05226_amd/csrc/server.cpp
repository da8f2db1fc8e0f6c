// Serving loop (continuous batching of excitation solves).
#include "drivers.h"

extern "C" {
mlcc_status mlcc_server_create(mlcc_context *, const mlcc_server_opts *, mlcc_server **) {
  return MLCC_E_ARG;
}
mlcc_status mlcc_server_destroy(mlcc_server *) { return MLCC_E_ARG; }
mlcc_status mlcc_submit(mlcc_server *, const mlcc_problem_desc *, int32_t,
                        const mlcc_solver_opts *, const mlcc_solver_opts *, uint64_t *) {
  return MLCC_E_ARG;
}
mlcc_status mlcc_poll(mlcc_server *, uint64_t, mlcc_result *) { return MLCC_E_ARG; }
uint64_t mlcc_request_footprint(const mlcc_problem_desc *, int32_t, const mlcc_solver_opts *) {
  return 0;
}
}
