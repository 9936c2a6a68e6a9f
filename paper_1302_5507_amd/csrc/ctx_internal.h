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

}  // namespace soapdp
