// Serving entry points (request loop with continuous batching).
#include "../../include/ed.h"
#include "host.h"

struct ed_server {
    ed_ctx* ctx;
};

int ed_serve_open(ed_ctx*, uint64_t, uint32_t, ed_server** out) {
    if (out) *out = nullptr;
    ed::set_error("ed_serve_open: not available in this build");
    return ED_EINVAL;
}
int ed_serve_submit(ed_server*, const uint8_t*, uint64_t, const uint8_t*, uint64_t, uint64_t) { return ED_EINVAL; }
int ed_serve_poll(ed_server*, ed_result*, uint32_t, uint32_t* got) {
    if (got) *got = 0;
    return ED_EINVAL;
}
int ed_serve_drain(ed_server*) { return ED_EINVAL; }
int ed_serve_close(ed_server*) { return ED_EINVAL; }
