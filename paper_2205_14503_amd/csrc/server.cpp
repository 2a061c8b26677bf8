// Continuous-batching query server (see steiner.h).
#include "engine.h"

using namespace stn;

struct steiner_server {
    steiner_graph *g = nullptr;
};

extern "C" int steiner_server_create(steiner_graph *g, uint64_t, uint32_t, const steiner_options *,
                                     steiner_server **out) {
    (void)g;
    (void)out;
    return fail(STEINER_EINVAL, "server not built");
}
extern "C" int steiner_server_submit(steiner_server *, const uint32_t *, uint32_t, uint64_t *) {
    return fail(STEINER_EINVAL, "server not built");
}
extern "C" int steiner_server_wait(steiner_server *, uint64_t, int64_t, steiner_result **) {
    return fail(STEINER_EINVAL, "server not built");
}
extern "C" uint64_t steiner_server_query_bytes(const steiner_server *, uint32_t) { return 0; }
extern "C" int steiner_server_destroy(steiner_server *) { return STEINER_OK; }
