// Serving loop (continuous batching); filled in below the stub.
#include "mmpm_internal.hpp"

namespace mm {
struct Server {};
Server *server_start(mm_ctx &, size_t, uint32_t) { throw Error(MM_ESTATE, "serving not built yet"); }
void server_stop(Server *s) { delete s; }
}  // namespace mm

extern "C" {
int mm_server_start(mm_ctx *, size_t, uint32_t, mm_server **) { return MM_ESTATE; }
int mm_submit(mm_server *, int, const uint32_t *, uint64_t *) { return MM_ESTATE; }
int mm_poll(mm_server *, uint64_t, uint32_t *) { return MM_ESTATE; }
int mm_server_stats(mm_server *, double *, double *, double *, uint64_t *) { return MM_ESTATE; }
int mm_server_stop(mm_server *) { return MM_ESTATE; }
int mm_server_replay(mm_server *, const int *, const uint32_t *, const int64_t *, size_t, uint32_t *, double *)
{
    return MM_ESTATE;
}
}
