#include "serve.h"

namespace cnnsns {

cnnsns_server server_create(int64_t, int32_t, int32_t, int32_t, const cnnsns_cnn*)
{
    fail(CNNSNS_EINVAL, "server_create: serving loop not available in this build");
}
uint64_t server_submit(cnnsns_server, cnnsns_mesh, const float*, int64_t, const double*, const double*,
                       const int32_t*, int32_t*, int32_t*)
{
    fail(CNNSNS_EINVAL, "submit: serving loop not available in this build");
}
bool server_poll(cnnsns_server, uint64_t, double*)
{
    fail(CNNSNS_EINVAL, "poll: serving loop not available in this build");
}
void server_wait(cnnsns_server, uint64_t, double*)
{
    fail(CNNSNS_EINVAL, "wait: serving loop not available in this build");
}
void server_destroy(cnnsns_server s)
{
    if (s) fail(CNNSNS_EINVAL, "server_destroy: serving loop not available in this build");
}

}  // namespace cnnsns
