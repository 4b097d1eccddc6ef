// emt_host.h -- host-side pieces of a context that the serving loop uses:
// a call split into an enqueue half and a completion half, and the device
// footprint of a batch for admission by HBM budget.
#ifndef EMT_HOST_H
#define EMT_HOST_H

#include <cstddef>
#include <cstdint>

#include "emt.h"

namespace emt {

// Check, size and stage the views and enqueue the first attempt on the
// context's stream. The views and their grains must stay valid until
// finish_views returns. One batch per context at a time.
int begin_views(emt_ctx *ctx, const emt_view_in *views, uint32_t n_views);
// True once the enqueued batch has finished on the device (or none is pending).
bool views_ready(emt_ctx *ctx);
// Wait for the batch, re-run it if a capacity overflowed, and fill out[]
// exactly as emt_track_views does.
int finish_views(emt_ctx *ctx, emt_view_out *out);
// Device bytes the context's buffers need for a batch of these sizes.
size_t batch_bytes(const emt_ctx *ctx, unsigned long long n_total, uint32_t n_views,
                   uint32_t max_n);
// Device bytes the context holds now.
size_t held_bytes(const emt_ctx *ctx);

}  // namespace emt

#endif
