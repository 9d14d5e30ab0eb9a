// Serving entry points (placeholder until the scheduler lands).
#include "serve.h"

extern "C" {
hz_status hz_serve_start(hz_ctx*, int32_t) { return HZ_ERR_STATE; }
hz_status hz_serve_submit(hz_ctx*, const hz_request*, uint64_t*) { return HZ_ERR_STATE; }
hz_status hz_serve_poll(hz_ctx*, uint64_t, int*) { return HZ_ERR_STATE; }
hz_status hz_serve_wait(hz_ctx*, uint64_t, int32_t*) { return HZ_ERR_STATE; }
hz_status hz_serve_stats_get(hz_ctx*, hz_serve_stats*) { return HZ_ERR_STATE; }
hz_status hz_serve_stop(hz_ctx*) { return HZ_ERR_STATE; }
}
