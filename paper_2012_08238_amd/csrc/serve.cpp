// Serving loop (placeholder until the scheduler lands).
#include "common.hpp"
#include "internal.hpp"

using namespace sfft;

extern "C" {
sfft_status sfft_server_create(sfft_server_t* out, size_t, int32_t, int32_t) {
    if (out) *out = nullptr;
    return set_error(SFFT_E_UNSUPPORTED, "server not built yet");
}
sfft_status sfft_server_submit(sfft_server_t, const sfft_params*, const void*, int64_t*, void*, double*, uint64_t*) {
    return set_error(SFFT_E_UNSUPPORTED, "server not built yet");
}
sfft_status sfft_server_poll(sfft_server_t, uint64_t, int32_t*, double*, int32_t*) {
    return set_error(SFFT_E_UNSUPPORTED, "server not built yet");
}
sfft_status sfft_server_wait(sfft_server_t, uint64_t, double*, int32_t*) {
    return set_error(SFFT_E_UNSUPPORTED, "server not built yet");
}
sfft_status sfft_server_stats_get(sfft_server_t, sfft_server_stats*) {
    return set_error(SFFT_E_UNSUPPORTED, "server not built yet");
}
sfft_status sfft_server_destroy(sfft_server_t) { return set_error(SFFT_E_UNSUPPORTED, "server not built yet"); }
}
