// Library-internal controls of a context, used by the server.
#pragma once

#include "../../include/soap_dp.h"

namespace soapdp {

// A frozen context serves calls only from what it already holds: a call
// that would grow its workspace, task buffers or stream set is refused with
// SOAP_DP_ENOMEM instead of synchronising the device and reallocating, and
// batched calls are enqueued directly rather than captured into graphs.
// The server freezes each slot's context once it is reserved and warmed
// up, so that no worker thread ever synchronises the whole device, frees
// memory or captures a graph while other slots' work runs.
void ctx_set_frozen(soap_dp_ctx *ctx, bool frozen);

// soap_dp_reserve for calls with this scoring only: the workspace covers the
// length classes those calls can populate (soap_dp_reserve, which does not
// know the scoring, covers every class kind).
int ctx_reserve_for(soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                    uint32_t flags, const soap_dp_scoring *sc);

}  // namespace soapdp
