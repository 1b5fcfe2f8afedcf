// Request loop with continuous batching (filled in below).
#include "internal.hpp"

extern "C" {
int shapley_server_create(shapley_server_t* out, size_t hbm_budget, void* stream) {
  (void)out; (void)hbm_budget; (void)stream;
  shp::set_last_error("server not available");
  return SHAPLEY_EINVAL;
}
int shapley_server_submit(shapley_server_t srv, shapley_game_t g, const shapley_solve_opts* o,
                          uint64_t* ticket) {
  (void)srv; (void)g; (void)o; (void)ticket;
  return SHAPLEY_EINVAL;
}
int shapley_server_wait(shapley_server_t srv, uint64_t ticket, int32_t max_steps, shapley_stats* st) {
  (void)srv; (void)ticket; (void)max_steps; (void)st;
  return SHAPLEY_EINVAL;
}
int shapley_server_poll(shapley_server_t srv, uint64_t ticket, shapley_stats* st) {
  (void)srv; (void)ticket; (void)st;
  return SHAPLEY_EINVAL;
}
int shapley_server_step(shapley_server_t srv, int32_t* active) {
  (void)srv; (void)active;
  return SHAPLEY_EINVAL;
}
void shapley_server_destroy(shapley_server_t srv) { (void)srv; }
}
