// Batched multi-query BFS, continuous-batching server and launch-shape tuner.
#include "bfs_internal.h"

using namespace bfsi;

extern "C" {

int bfs_run_batch(int32_t count, bfs_graph_t* const* graphs, const int32_t* roots,
                  int32_t* const* parents, int32_t* const* levels, void* hip_stream) {
  (void)count; (void)graphs; (void)roots; (void)parents; (void)levels; (void)hip_stream;
  return fail(BFS_ERR_UNSUPPORTED, "not built yet");
}

int bfs_server_create(const bfs_server_config_t* cfg, bfs_server_t** out) {
  (void)cfg; (void)out;
  return fail(BFS_ERR_UNSUPPORTED, "not built yet");
}
int bfs_server_submit(bfs_server_t* s, bfs_graph_t* g, int32_t root, int32_t* parent,
                      int32_t* level, uint64_t* ticket) {
  (void)s; (void)g; (void)root; (void)parent; (void)level; (void)ticket;
  return fail(BFS_ERR_UNSUPPORTED, "not built yet");
}
int bfs_server_poll(bfs_server_t* s, uint64_t ticket, bfs_result_t* out) {
  (void)s; (void)ticket; (void)out;
  return fail(BFS_ERR_UNSUPPORTED, "not built yet");
}
int bfs_server_wait(bfs_server_t* s, uint64_t ticket, double timeout_s, bfs_result_t* out) {
  (void)s; (void)ticket; (void)timeout_s; (void)out;
  return fail(BFS_ERR_UNSUPPORTED, "not built yet");
}
int bfs_server_drain(bfs_server_t* s) { (void)s; return fail(BFS_ERR_UNSUPPORTED, "not built yet"); }
int bfs_server_destroy(bfs_server_t* s) { (void)s; return fail(BFS_ERR_UNSUPPORTED, "not built yet"); }
int bfs_tune(bfs_graph_t* g, const char* cache_path) {
  (void)g; (void)cache_path;
  return fail(BFS_ERR_UNSUPPORTED, "not built yet");
}

}  // extern "C"
