// Continuous-batching serving loop behind risp_submit / risp_poll.
//
// A scheduler thread per context admits queued jobs first-fit in arrival order while their
// estimated device footprint fits the budget and a slot is free, builds their factors on a stream of
// their own, and then runs ticks: every active job's pending sigma block is launched on its stream
// (optionally captured as one fork-join hipGraph per tick), the blocks run concurrently, and each
// job's Davidson subspace step follows. A job's arithmetic depends only on its own inputs (own
// factors, workspaces and stream; fixed reduction orders), so its result is the same alone and in a
// mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>

#include "davidson.hpp"
#include "factors.hpp"
#include "serve.hpp"

namespace risp {

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct Job {
  uint64_t id = 0;
  std::vector<double> coords, radius, C, e;
  std::vector<int32_t> Z;
  std::vector<risp_shell> shells;
  risp_system sys{};
  risp_params prm{};
  risp_dav_opts opts{};
  int64_t footprint = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<risp_factors> F;
  std::unique_ptr<DavidsonRun> run;
  int stage = 0;  // 0: main stage, 1: FP32 correction stage
  DavResult main_res;
  double t_sigma = 0.0;
  bool sigma_pending = false;
  Timer sigma_timer;
  // result
  risp_status status = RISP_PENDING;
  std::string message;
  std::vector<double> energies;
  std::vector<float> vectors;
  risp_dav_info info{};
  double t_submit = 0, t_admit = -1, t_first_sigma = -1, t_done = -1;

  // every device allocation of the job is released here, on the scheduler thread: a Job object that
  // still held device memory when risp_poll destroys it would call hipFree from the polling thread
  // while the scheduler thread may be capturing a graph on its streams
  void release_device() {
    run.reset();
    main_res = DavResult();
    F.reset();
    if (stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
      stream = nullptr;
    }
  }
  ~Job() { release_device(); }
};

struct Server {
  risp_ctx* ctx = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::unique_ptr<Job>> queue;
  // resident jobs: only the scheduler thread changes the vector, under mu (serve_stats reads its size)
  std::vector<std::unique_ptr<Job>> active;
  std::map<uint64_t, std::unique_ptr<Job>> done;
  std::set<uint64_t> inflight;  // queued or active ids (guarded by mu)
  uint64_t next_id = 1;
  int64_t budget = 0, used = 0;
  int max_active = 8;
  bool use_graphs = true;
  bool stop = false;
  std::thread thread;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::atomic<int64_t> ticks{0}, graph_ticks{0};  // written by the scheduler, read by serve_stats

  void loop();
  void admit(Job& j);
  void tick();
  void finish(std::unique_ptr<Job> j);
};

// ---------------------------------------------------------------------------------------------
// footprint model
// ---------------------------------------------------------------------------------------------
int64_t job_footprint(const risp_system* sys, const risp_params* prm, const risp_dav_opts* opts) {
  int heavy = 0;
  for (int a = 0; a < sys->natm; ++a) heavy += (sys->Z[a] != 1 || prm->h_in_aux) ? 1 : 0;
  const int64_t nao = sys->nao, nocc = sys->nocc, nvir = sys->nmo - sys->nocc;
  const int64_t ov = nocc * nvir;
  const int64_t nJ = 4 * (int64_t)heavy;
  const int64_t nblocks = (prm->rsh_mode == RISP_RSH_SPLIT && prm->c_x != 0.0 && prm->beta != 0.0) ? 2 : 1;
  const int64_t nK = (prm->c_x != 0.0 || prm->beta != 0.0) ? heavy * nblocks : 0;
  const int64_t esz = prm->precision == RISP_FP64 ? 8 : (prm->precision == RISP_FP32 ? 4 : 2);
  // stored factors (+ for BF16 factors the FP32 copy of T_ia and the BF16 remainders of T_ij and
  // T_ab), orbital gaps and the FP64 diagonal of A
  const int64_t store = esz * (nJ * ov + nK * (nocc * nocc + nvir * nvir)) +
                        (prm->precision == RISP_BF16 ? 4 * nJ * ov + 2 * nK * (nocc * nocc + nvir * nvir) : 0) +
                        ov * (8 + 4 + 8);
  const int64_t per_func = nao * nao * 8;
  const int64_t max_f = std::max<int64_t>(3, std::min<int64_t>(256, (16ll << 30) / std::max<int64_t>(per_func, 1)));
  const int64_t build = 2 * nJ * ov * 8 + max_f * per_func + max_f * nocc * nao * 8 + 2 * nJ * nJ * 8 +
                        nK * (nocc * nocc + nvir * nvir) * 16 + nao * sys->nmo * 8 * 2;
  const int nstates = opts ? opts->nstates : 15;
  const int64_t block = std::min<int64_t>(64, opts && opts->block > 0 ? opts->block : std::min(2 * nstates, 30));
  const int64_t max_space = opts && opts->max_space > 0 ? opts->max_space : std::max<int64_t>(8 * block, nstates + 2 * block);
  const int64_t cap = max_space + block;
  const int64_t vsz = prm->precision == RISP_FP64 ? 8 : 4;
  const int64_t csz = std::max<int64_t>(esz, prm->precision == RISP_BF16 ? 4 : esz);
  // sigma workspaces (see ensure_workspace): exchange intermediate per auxiliary chunk (at most 4 GiB
  // plus one function), window block, exchange accumulator, split-K partial sums, BF16 copies of X, Y
  const int64_t acc = prm->precision == RISP_FP64 ? 8 : 4;
  const int64_t blk_ov = block * nocc * nvir;
  const int64_t mt = std::min<int64_t>(std::max<int64_t>(nK, 1) * blk_ov * csz, (4ll << 30) + blk_ov * csz);
  // padded X and Yt of the skinny Coulomb passes take 4 bytes per element for FP32 products
  const int64_t sig = mt + blk_ov * csz + blk_ov * acc + std::max(1024 * nJ * block * acc, 4 * blk_ov * acc) +
                      block * (ov + 8) * 4 + nJ * block * acc + 64 * (nJ + 32) * 4;
  const bool spill = opts && (opts->flags & RISP_DAV_SPILL);
  // V, W (unless spilled); Ritz vectors, residuals and two correction buffers (FP64); the thick
  // restart's two staging copies of 2 block rows; split-K partial sums; the subspace matrices; and
  // for BF16 jobs with a correction pass the main stage's Ritz vectors, which seed the FP32 stage
  const bool corr = prm->precision == RISP_BF16 && opts && opts->correction_pass;
  const int64_t dav = (spill ? 0 : 2 * cap * ov * vsz) + 4 * block * ov * 8 + 4 * block * ov * vsz +
                      512 * cap * block * 8 + 4 * cap * cap * 8 + (corr ? block * ov * 8 : 0);
  return store + std::max(build, sig + dav) + (64ll << 20);
}

// ---------------------------------------------------------------------------------------------
// scheduler
// ---------------------------------------------------------------------------------------------
void Server::admit(Job& j) {
  j.t_admit = now_s(t0);
  RISP_HIP(hipStreamCreateWithFlags(&j.stream, hipStreamNonBlocking));
  j.F = std::make_unique<risp_factors>();
  Timer tb;
  build_factors(ctx, &j.sys, &j.prm, j.F.get(), j.stream);
  j.F->t_build = tb.sec();
  DavOptions o;
  o.nstates = j.opts.nstates;
  o.block = j.opts.block;
  o.max_space = j.opts.max_space;
  o.max_iter = j.opts.max_iter > 0 ? j.opts.max_iter : 200;
  o.tol = j.opts.tol;
  o.max_corr = j.opts.ncorr > 0 ? j.opts.ncorr : j.opts.nstates;
  o.spill = (j.opts.flags & RISP_DAV_SPILL) != 0;
  o.olsen = (j.opts.flags & RISP_DAV_OLSEN) != 0;
  if (j.prm.precision == RISP_BF16) {
    if (j.opts.correction_pass) o.tol = std::max(o.tol, j.opts.bf16_tol > 0.0 ? j.opts.bf16_tol : kBf16StageTol);
    o.stall_iters = 2;
    o.stall_below = 10.0 * (j.opts.bf16_tol > 0.0 ? j.opts.bf16_tol : kBf16StageTol);
  }
  j.run = std::make_unique<DavidsonRun>(j.F.get(), o, j.stream);
  j.stage = 0;
}

void Server::finish(std::unique_ptr<Job> j) {
  const int64_t fp = j->footprint;
  j->release_device();
  j->t_done = now_s(t0);
  std::lock_guard<std::mutex> lk(mu);
  used -= fp;
  inflight.erase(j->id);
  done[j->id] = std::move(j);
  cv.notify_all();
}

// copy the final results of a finished run to the host side of the job
static void collect(Job& j, DavResult& fin, DavResult* corr) {
  const int64_t ov = (int64_t)j.F->nocc * j.F->nvir;
  const int ns = std::min<int>(j.opts.nstates, (int)fin.energies.size());
  j.energies.assign(fin.energies.begin(), fin.energies.begin() + ns);
  std::vector<double> h((size_t)ns * ov);
  if (ns > 0) {
    RISP_HIP(hipMemcpyAsync(h.data(), fin.X.get(), h.size() * 8, hipMemcpyDeviceToHost, j.stream));
    RISP_HIP(hipStreamSynchronize(j.stream));
  }
  j.vectors.resize(h.size());
  for (size_t t = 0; t < h.size(); ++t) j.vectors[t] = (float)h[t];
  DavResult& m = j.main_res;
  std::memset(&j.info, 0, sizeof(j.info));
  j.info.iters = m.iters;
  j.info.restarts = m.restarts + (corr ? corr->restarts : 0);
  j.info.sigma_vectors = m.sigma_vectors;
  j.info.converged = fin.converged ? 1 : 0;
  j.info.correction_iters = corr ? corr->iters : 0;
  j.info.correction_vectors = corr ? corr->sigma_vectors : 0;
  j.info.t_build = j.F->t_build;
  j.info.sigma_flops = m.sigma_flops;
  j.info.sigma_flops_correct = corr ? corr->sigma_flops : 0.0;
  j.info.t_subspace = m.t_subspace;
  j.info.hbm_bytes = j.F->bytes();
  std::vector<double> hist = m.resid_hist;
  if (corr) hist.insert(hist.end(), corr->resid_hist.begin(), corr->resid_hist.end());
  for (size_t k = 0; k < std::min<size_t>(256, hist.size()); ++k) j.info.resid_hist[k] = hist[k];
  j.status = fin.converged ? RISP_OK : RISP_E_NOTCONV;
  if (!fin.converged) j.message = "Davidson did not converge within max_iter";
}

void Server::tick() {
  ++ticks;
  // launch every pending sigma block; each job on its own stream
  std::vector<Job*> launched;
  std::vector<DavidsonRun::Request> reqs;
  for (auto& jp : active) {
    Job& j = *jp;
    DavidsonRun::Request rq;
    if (!j.run || !j.run->next(rq)) continue;
    launched.push_back(&j);
    reqs.push_back(rq);
  }
  if (launched.empty()) return;
  // workspaces sized before any capture (their first allocation synchronises)
  for (size_t k = 0; k < launched.size(); ++k) sigma_prepare(launched[k]->F.get(), reqs[k].n, launched[k]->stage == 1);
  bool graphed = false;
  if (use_graphs && launched.size() > 1) {
    // fork-join capture: the tick stream forks to every job stream and joins them again
    hipStream_t ts = ctx->serve_stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins(launched.size(), nullptr);
    RISP_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (auto& ev : joins) RISP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const bool prof = ctx->profiling;
    ctx->profiling = false;  // no event records inside the captured graph
    RISP_HIP(hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal));
    try {
      RISP_HIP(hipEventRecord(fork, ts));
      for (size_t k = 0; k < launched.size(); ++k) {
        Job& j = *launched[k];
        RISP_HIP(hipStreamWaitEvent(j.stream, fork, 0));
        sigma(j.F.get(), reqs[k].n, reqs[k].X, reqs[k].S, j.stage == 1, j.stream,
              j.stage == 1 && j.run->bf16_basis());
        RISP_HIP(hipEventRecord(joins[k], j.stream));
        RISP_HIP(hipStreamWaitEvent(ts, joins[k], 0));
      }
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(ts, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      ctx->profiling = prof;
      throw;
    }
    ctx->profiling = prof;
    RISP_HIP(hipStreamEndCapture(ts, &graph));
    RISP_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    for (Job* j : launched) {
      j->sigma_timer = Timer();
      if (j->t_first_sigma < 0) j->t_first_sigma = now_s(t0);
    }
    RISP_HIP(hipGraphLaunch(exec, ts));
    RISP_HIP(hipStreamSynchronize(ts));
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(fork);
    for (auto& ev : joins) (void)hipEventDestroy(ev);
    graphed = true;
    ++graph_ticks;
  } else {
    for (size_t k = 0; k < launched.size(); ++k) {
      Job& j = *launched[k];
      j.sigma_timer = Timer();
      if (j.t_first_sigma < 0) j.t_first_sigma = now_s(t0);
      sigma(j.F.get(), reqs[k].n, reqs[k].X, reqs[k].S, j.stage == 1, j.stream,
            j.stage == 1 && j.run->bf16_basis());
    }
  }
  // subspace steps
  for (Job* jp : launched) {
    Job& j = *jp;
    if (!graphed) RISP_HIP(hipStreamSynchronize(j.stream));
    j.t_sigma += j.sigma_timer.sec();
    j.run->complete();
  }
}

void Server::loop() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    std::vector<std::unique_ptr<Job>> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      if (stop && queue.empty() && active.empty()) return;
      // first-fit admission in arrival order
      for (auto it = queue.begin(); it != queue.end();) {
        if ((int)(active.size() + admitted.size()) >= max_active) break;
        if (used + (*it)->footprint <= budget) {
          used += (*it)->footprint;
          admitted.push_back(std::move(*it));
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
    }
    for (auto& j : admitted) {
      try {
        admit(*j);
        std::lock_guard<std::mutex> lk(mu);
        active.push_back(std::move(j));
      } catch (const std::exception& ex) {
        j->status = dynamic_cast<const Error*>(&ex) ? static_cast<const Error&>(ex).code : RISP_E_HIP;
        j->message = ex.what();
        finish(std::move(j));
      }
    }
    try {
      tick();
    } catch (const std::exception& ex) {
      // a failure inside a tick cannot be attributed safely: fail every active job
      for (auto& j : active) {
        j->status = dynamic_cast<const Error*>(&ex) ? static_cast<const Error&>(ex).code : RISP_E_HIP;
        j->message = ex.what();
      }
      std::vector<std::unique_ptr<Job>> failed;
      {
        std::lock_guard<std::mutex> lk(mu);
        failed.swap(active);
      }
      for (auto& j : failed) finish(std::move(j));
      continue;
    }
    // retire finished runs; start the FP32 correction stage where it applies
    for (auto it = active.begin(); it != active.end();) {
      Job& j = **it;
      if (!j.run->done()) {
        ++it;
        continue;
      }
      try {
        if (j.stage == 0) {
          j.main_res = std::move(j.run->result());
          j.main_res.t_sigma = j.t_sigma;
          j.t_sigma = 0.0;
          if (j.prm.precision == RISP_BF16 && j.opts.correction_pass && j.main_res.krows > 0) {
            DavOptions oc;
            oc.nstates = j.opts.nstates;
            oc.block = j.opts.block;
            oc.max_corr = j.opts.correction_ncorr > 0 ? j.opts.correction_ncorr : j.opts.nstates;
            oc.spill = (j.opts.flags & RISP_DAV_SPILL) != 0;
            oc.olsen = (j.opts.flags & RISP_DAV_OLSEN) != 0;
            oc.bf16_basis = (j.opts.flags & RISP_DAV_FP32_BASIS) == 0;
            oc.max_space = j.opts.max_space;
            oc.tol = j.opts.tol;
            oc.x0_dev = j.main_res.X.as<double>();
            oc.nx0 = j.main_res.krows;
            oc.max_iter = 1 + (j.opts.correction_steps > 0 ? j.opts.correction_steps : 16);
            // the finished main-stage run goes first, so the job never holds two runs' buffers
            // (main_res.X, already moved out of it, seeds the correction run)
            j.run.reset();
            j.run = std::make_unique<DavidsonRun>(j.F.get(), oc, j.stream);
            j.stage = 1;
            ++it;
            continue;
          }
          collect(j, j.main_res, nullptr);
          j.info.t_sigma = j.main_res.t_sigma;
        } else {
          DavResult& rc = j.run->result();
          collect(j, rc, &rc);
          j.info.t_sigma = j.main_res.t_sigma;
          j.info.t_sigma_correct = j.t_sigma;
        }
      } catch (const std::exception& ex) {
        j.status = dynamic_cast<const Error*>(&ex) ? static_cast<const Error&>(ex).code : RISP_E_HIP;
        j.message = ex.what();
      }
      std::unique_ptr<Job> fin;
      {
        std::lock_guard<std::mutex> lk(mu);
        fin = std::move(*it);
        it = active.erase(it);
      }
      finish(std::move(fin));
    }
  }
}

// ---------------------------------------------------------------------------------------------
// entry points used by the ABI
// ---------------------------------------------------------------------------------------------
Server* ensure_server(risp_ctx* ctx) {
  if (!ctx->server) {
    auto* sv = new Server();
    sv->ctx = ctx;
    size_t fr = 0, tot = 0;
    RISP_HIP(hipMemGetInfo(&fr, &tot));
    sv->budget = ctx->serve_budget > 0 ? ctx->serve_budget : (int64_t)(0.85 * (double)fr);
    sv->max_active = ctx->serve_max_active > 0 ? ctx->serve_max_active : 8;
    sv->use_graphs = ctx->serve_graphs != 0;
    if (!ctx->serve_stream) RISP_HIP(hipStreamCreateWithFlags(&ctx->serve_stream, hipStreamNonBlocking));
    ctx->server = sv;
    sv->thread = std::thread([sv] { sv->loop(); });
  }
  return ctx->server;
}

void stop_server(risp_ctx* ctx) {
  Server* sv = ctx->server;
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (auto& j : sv->queue) {  // queued jobs are dropped
      j->status = RISP_E_STATE;
      j->message = "context destroyed before admission";
    }
    sv->queue.clear();
    sv->cv.notify_all();
  }
  if (sv->thread.joinable()) sv->thread.join();
  delete sv;
  ctx->server = nullptr;
  if (ctx->serve_stream) {
    (void)hipStreamDestroy(ctx->serve_stream);
    ctx->serve_stream = nullptr;
  }
}

uint64_t submit_job(risp_ctx* ctx, const risp_system* sys, const risp_params* prm, const risp_dav_opts* opts) {
  validate_system(sys);
  RISP_CHECK(prm && opts, RISP_E_ARG, "params and options are required");
  RISP_CHECK(opts->nstates > 0, RISP_E_ARG, "nstates must be positive");
  RISP_CHECK(opts->nx0 == 0, RISP_E_ARG, "initial vectors are not supported for served jobs");
  RISP_CHECK(opts->ncorr >= 0 && opts->correction_ncorr >= 0, RISP_E_ARG, "ncorr must be non-negative");
  RISP_CHECK(prm->j_mode == RISP_J_MO, RISP_E_ARG,
             "served jobs use the stored-factor Coulomb route (j_mode RISP_J_MO)");
  Server* sv = ensure_server(ctx);
  auto j = std::make_unique<Job>();
  j->coords.assign(sys->coords, sys->coords + 3 * (size_t)sys->natm);
  j->radius.assign(sys->aux_radius, sys->aux_radius + sys->natm);
  j->Z.assign(sys->Z, sys->Z + sys->natm);
  j->shells.assign(sys->shells, sys->shells + sys->nshell);
  j->C.assign(sys->mo_coeff, sys->mo_coeff + (size_t)sys->nao * sys->nmo);
  j->e.assign(sys->mo_energy, sys->mo_energy + sys->nmo);
  j->sys = *sys;
  j->sys.coords = j->coords.data();
  j->sys.aux_radius = j->radius.data();
  j->sys.Z = j->Z.data();
  j->sys.shells = j->shells.data();
  j->sys.mo_coeff = j->C.data();
  j->sys.mo_energy = j->e.data();
  j->prm = *prm;
  j->opts = *opts;
  j->opts.x0 = nullptr;
  j->footprint = job_footprint(sys, prm, opts);
  std::lock_guard<std::mutex> lk(sv->mu);
  RISP_CHECK(j->footprint <= sv->budget, RISP_E_NOMEM,
             "job needs " + std::to_string(j->footprint) + " bytes, more than the serving budget " +
                 std::to_string(sv->budget));
  j->id = sv->next_id++;
  j->t_submit = now_s(sv->t0);
  const uint64_t id = j->id;
  sv->inflight.insert(id);
  sv->queue.push_back(std::move(j));
  sv->cv.notify_all();
  return id;
}

risp_status poll_job(risp_ctx* ctx, uint64_t id, risp_result* out) {
  Server* sv = ctx->server;
  RISP_CHECK(sv != nullptr, RISP_E_NOTFOUND, "no job with this id");
  std::unique_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(id);
    if (it == sv->done.end()) {
      if (sv->inflight.count(id)) return RISP_PENDING;
      throw Error(RISP_E_NOTFOUND, "no job with this id (unknown or already polled)");
    }
    j = std::move(it->second);
    sv->done.erase(it);
  }
  out->status = j->status;
  out->nstates = (int32_t)j->energies.size();
  if (out->energies) std::copy(j->energies.begin(), j->energies.end(), out->energies);
  if (out->vectors) std::copy(j->vectors.begin(), j->vectors.end(), out->vectors);
  out->info = j->info;
  out->t_submit = j->t_submit;
  out->t_admit = j->t_admit;
  out->t_first_sigma = j->t_first_sigma;
  out->t_done = j->t_done;
  std::snprintf(out->message, sizeof(out->message), "%s", j->message.c_str());
  return RISP_OK;
}

void serve_stats(risp_ctx* ctx, risp_serve_stats* st) {
  std::memset(st, 0, sizeof(*st));
  Server* sv = ctx->server;
  if (!sv) return;
  std::lock_guard<std::mutex> lk(sv->mu);
  st->queued = (int32_t)sv->queue.size();
  st->active = (int32_t)sv->active.size();
  st->done = (int32_t)sv->done.size();
  st->budget_bytes = sv->budget;
  st->used_bytes = sv->used;
  st->ticks = sv->ticks;
  st->graph_ticks = sv->graph_ticks;
}

}  // namespace risp
