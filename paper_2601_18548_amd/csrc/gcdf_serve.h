// Serving loop interface (continuous batching of gcdf_request).
#pragma once
#include "gcdf.h"
#include "gcdf_internal.h"

namespace gcdf {

struct Server;

gcdf_status server_start(gcdf_ctx* ctx, size_t mem_budget, int slots, Server** out);
void server_stop(Server* s);
gcdf_status server_submit(Server* s, const gcdf_request* req, uint64_t* ticket);
gcdf_status server_poll(Server* s, uint64_t ticket);

// Shared with gcdf_api.cpp.
gcdf_status set_error(gcdf_status st, const char* msg);
const DevNet& ctx_net(const gcdf_ctx* ctx);
int ctx_num_cu(const gcdf_ctx* ctx);
int ctx_device(const gcdf_ctx* ctx);

}  // namespace gcdf
