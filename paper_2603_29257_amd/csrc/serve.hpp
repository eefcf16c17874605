// Serving loop (continuous batching) behind risp_submit / risp_poll.
#pragma once

#include "common.hpp"

struct risp_ctx;

namespace risp {

struct Server;
int64_t job_footprint(const risp_system* sys, const risp_params* prm, const risp_dav_opts* opts);
Server* ensure_server(risp_ctx* ctx);
void stop_server(risp_ctx* ctx);
uint64_t submit_job(risp_ctx* ctx, const risp_system* sys, const risp_params* prm, const risp_dav_opts* opts);
risp_status poll_job(risp_ctx* ctx, uint64_t id, risp_result* out);
void serve_stats(risp_ctx* ctx, risp_serve_stats* st);

}  // namespace risp
