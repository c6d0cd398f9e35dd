// server.cpp -- continuous batching over a caller-provided device arena.
#include "host.h"

extern "C" {
int mhs_server_create(void*, size_t, int32_t, uint32_t, void*, mhs_server**) { return mhsk::set_error(MHS_EINVAL, "not built"); }
int mhs_server_submit(mhs_server*, const mhs_instance*, uint64_t) { return MHS_EINVAL; }
int mhs_server_poll(mhs_server*, int32_t, uint64_t*, mhs_result**, int32_t*) { return MHS_EINVAL; }
int mhs_server_pending(const mhs_server*, int32_t*, int32_t*) { return MHS_EINVAL; }
int mhs_server_arena_used(const mhs_server*, size_t*) { return MHS_EINVAL; }
void mhs_server_destroy(mhs_server*) {}
}
