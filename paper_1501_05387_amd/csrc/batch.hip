// batch.hip -- many sources on one graph.
#include "engine.h"

namespace gfr {

void run_bfs_batch(Ctx &c, Graph &g, const int32_t *sources, int32_t k, int32_t *depth, hipStream_t s)
{
    for (int32_t i = 0; i < k; ++i) run_bfs(c, g, sources[i], depth + (size_t)i * g.n, s);
}

void run_sssp_batch(Ctx &c, Graph &g, const int32_t *sources, int32_t k, uint32_t *dist, hipStream_t s)
{
    for (int32_t i = 0; i < k; ++i) run_sssp(c, g, sources[i], dist + (size_t)i * g.n, s);
}

}  // namespace gfr
