// Continuous-batching solve server.
//
// Gauge fields stay resident on the device, each with its own HIP stream, its
// own slot engine (engine.hip) and its own worker thread.  Requests (one
// field, one mass per right-hand side, 1..n right-hand sides) enter a FIFO
// queue.  A field's worker admits the right-hand sides of its field's
// requests into free engine slots as soon as earlier ones finish -- a request
// does not wait for a batch to drain -- and drives its engine phase by phase
// (restart phase, then one Arnoldi step, each a fused multi-RHS launch
// sequence replayed as a hipGraph).  Because every field advances on its own
// thread and stream, a small lattice's requests proceed at its own step rate
// instead of waiting on the largest field's steps, and the fields' work
// overlaps on the device.  Each field's slot pool is sized once from the HBM
// budget; a right-hand side is admitted only into a reserved slot, so the
// workspace never exceeds the budget.  Completion times give per-request
// latency; the statistics report p50/p99 beside throughput.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dd_internal.h"
#include "engine.h"
#include "serve_core.h"

struct dd_server {
    dd_server_config cfg{};
    int device = 0;
    struct Field {
        dd_ctx *ctx = nullptr;
        hipStream_t stream = nullptr;
        std::unique_ptr<dd::Engine> eng;
        size_t workspace = 0;
        std::vector<std::pair<long, int>> slot_owner; // (request, rhs) per slot
    };
    std::vector<Field> fields;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    dd::ServeQueue q; // requests, admission order, completion accounting (under mu)
    std::vector<std::thread> workers; // one per field
    std::atomic<bool> stop{false};
    bool started = false;
    size_t used = 0;
    std::string err;
    int fatal = DD_OK;
    double busy_s = 0;
};

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// One pass of field fi's worker: admit its queued right-hand sides, run one
// engine iteration if any slot is busy, harvest finished right-hand sides.
dd::Status work_once(dd_server *s, int fi, bool &did_work)
{
    did_work = false;
    dd_server::Field &f = s->fields[fi];
    std::vector<dd::ServeAdmit> adm;
    const size_t vstride = (size_t)f.ctx->g.V * 24;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->q.admit(
            fi, [&](int k) { return f.eng->slot(k).state == dd::SLOT_FREE; }, f.slot_owner, vstride, now_s(), adm);
    }
    for (auto &a : adm) DD_TRY(f.eng->admit(a.slot, a.b, nullptr, a.m0, a.req, a.rhs));
    if (f.eng->busy_slots() == 0) return dd::Status::ok();
    did_work = true;
    dd::TraceRange tr("serve_step");
    const double t0 = now_s();
    DD_TRY(f.eng->launch_restart());
    DD_TRY(f.eng->finish_restart());
    if (f.eng->busy_slots()) DD_TRY(f.eng->launch_step());
    DD_TRY(f.eng->finish_step());
    // harvest finished right-hand sides
    std::vector<dd::ServeDone> fin;
    for (int r = 0; r < f.eng->width(); ++r) {
        dd::SlotState &st = f.eng->slot(r);
        if (st.state != dd::SLOT_DONE) continue;
        const long req = f.slot_owner[r].first;
        const int rhs = f.slot_owner[r].second;
        double *xdst = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            xdst = s->q.result(req, rhs, vstride);
        }
        if (xdst) DD_TRY(f.eng->extract(r, xdst));
        fin.push_back({req, rhs, st.info});
        f.eng->release(r);
        f.slot_owner[r] = {0, 0};
    }
    if (!fin.empty()) DD_HIP_TRY(hipStreamSynchronize(f.stream));
    const double t1 = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    s->busy_s += t1 - t0;
    s->q.finish(fin, t1);
    if (!fin.empty()) s->cv_done.notify_all();
    return dd::Status::ok();
}

void worker_main(dd_server *s, int fi)
{
    if (hipSetDevice(s->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->fatal = DD_HIP_ERROR;
        s->err = "server: hipSetDevice failed in a worker";
        s->cv_done.notify_all();
        return;
    }
    while (!s->stop.load()) {
        bool did = false;
        dd::Status st = work_once(s, fi, did);
        if (!st.good()) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->fatal = st.code;
            s->err = "server: " + st.msg;
            s->q.fail_all(st.code);
            s->stop.store(true);
            s->cv_done.notify_all();
            s->cv_work.notify_all();
            return;
        }
        if (!did) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2),
                                [&] { return s->stop.load() || !s->q.queue.empty(); });
        }
    }
}

} // namespace

extern "C" {

void dd_server_default_config(dd_server_config *c)
{
    if (!c) return;
    c->hbm_budget_bytes = (size_t)200 << 30;
    c->max_width = 12;
    c->m = 20;
    c->tol = 1e-10;
    c->max_restarts = 100;
    c->ncy = 12;
    c->nmr = 4;
    c->sap_prec = DD_F32;
    c->sap_eo = 0;
    c->use_graphs = 1;
    c->sap_half_fields = 0;
}

dd_status dd_server_create(const dd_server_config *cfg, dd_server **out)
{
    if (!out) return DD_INVALID_ARG;
    *out = nullptr;
    dd_server_config c;
    dd_server_default_config(&c);
    if (cfg) c = *cfg;
    if (c.max_width < 1 || c.max_width > dd::ENGINE_MAXW || c.m < 1 || c.m > dd::ENGINE_MAXM || !(c.tol > 0) ||
        c.ncy < 0 || c.nmr < 0 || c.max_restarts < 0 || (c.sap_prec != DD_F64 && c.sap_prec != DD_F32 && c.sap_prec != DD_F16))
        return DD_INVALID_ARG;
    dd_server *s = nullptr;
    try {
        s = new dd_server();
    } catch (...) {
        return DD_OOM;
    }
    s->cfg = c;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return DD_HIP_ERROR;
    }
    *out = s;
    return DD_OK;
}

const char *dd_server_last_error(const dd_server *s) { return s ? s->err.c_str() : ""; }

dd_status dd_server_add_field(dd_server *s, const int dims[4], const int bcs[4], const double *U_host, double csw,
                              int width, int *field_id)
{
    if (!s || !field_id) return DD_INVALID_ARG;
    if (s->started) {
        s->err = "server: fields must be added before the first submit";
        return DD_INVALID_ARG;
    }
    dd_server::Field f;
    if (hipStreamCreateWithFlags(&f.stream, hipStreamNonBlocking) != hipSuccess) {
        s->err = "server: stream creation failed";
        return DD_HIP_ERROR;
    }
    dd_status st = dd_create(dims, nullptr, bcs, f.stream, &f.ctx);
    if (st != DD_OK) {
        s->err = std::string("server: ") + dd_last_error(nullptr);
        (void)hipStreamDestroy(f.stream);
        return st;
    }
    st = dd_set_gauge(f.ctx, U_host, csw);
    if (st == DD_OK) st = dd_set_sap_half_fields(f.ctx, s->cfg.sap_half_fields);
    if (st != DD_OK) {
        s->err = std::string("server: ") + dd_last_error(f.ctx);
        dd_destroy(f.ctx);
        (void)hipStreamDestroy(f.stream);
        return st;
    }
    const size_t per_slot = dd::Engine::bytes_per_slot(f.ctx->g, s->cfg.m, s->cfg.sap_prec);
    const size_t left = s->cfg.hbm_budget_bytes > s->used ? s->cfg.hbm_budget_bytes - s->used : 0;
    int w = width > 0 ? width : s->cfg.max_width;
    w = std::min<long>(w, (long)(left / per_slot));
    if (w < 1) {
        s->err = "server: HBM budget leaves no slot for this field";
        dd_destroy(f.ctx);
        (void)hipStreamDestroy(f.stream);
        return DD_OOM;
    }
    dd::EngineParams ep;
    ep.width = w;
    ep.m = s->cfg.m;
    ep.ncy = s->cfg.ncy;
    ep.nmr = s->cfg.nmr;
    ep.sap_prec = s->cfg.sap_prec;
    ep.sap_eo = s->cfg.sap_eo != 0;
    ep.tol = s->cfg.tol;
    ep.max_restarts = s->cfg.max_restarts;
    ep.graphs = s->cfg.use_graphs != 0;
    f.eng.reset(new dd::Engine());
    dd::Status es = f.eng->init(f.ctx, ep);
    if (!es.good()) {
        s->err = "server: " + es.msg;
        f.eng.reset();
        dd_destroy(f.ctx);
        (void)hipStreamDestroy(f.stream);
        return es.code;
    }
    f.workspace = per_slot * w;
    f.slot_owner.assign(w, {0, 0});
    s->used += f.workspace;
    *field_id = (int)s->fields.size();
    s->fields.push_back(std::move(f));
    return DD_OK;
}

dd_status dd_server_field_info(const dd_server *s, int field_id, int *width, size_t *workspace_bytes)
{
    if (!s || field_id < 0 || field_id >= (int)s->fields.size()) return DD_INVALID_ARG;
    if (width) *width = s->fields[field_id].eng->width();
    if (workspace_bytes) *workspace_bytes = s->fields[field_id].workspace;
    return DD_OK;
}

dd_status dd_server_submit(dd_server *s, int field_id, int nrhs, const double *m0, const double *b, double *x,
                           long *request_id)
{
    if (!s || !m0 || !b || !x || !request_id || nrhs < 1) return DD_INVALID_ARG;
    if (field_id < 0 || field_id >= (int)s->fields.size()) {
        s->err = "server: unknown field";
        return DD_INVALID_ARG;
    }
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(m0[r])) {
            s->err = "server: non-finite mass";
            return DD_INVALID_ARG;
        }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != DD_OK) return (dd_status)s->fatal;
    if (!s->started) {
        s->started = true;
        try {
            for (int fi = 0; fi < (int)s->fields.size(); ++fi) s->workers.emplace_back(worker_main, s, fi);
        } catch (...) {
            s->err = "server: could not start the worker threads";
            s->stop.store(true);
            return DD_HIP_ERROR;
        }
    }
    *request_id = s->q.submit(field_id, nrhs, m0, b, x, now_s());
    s->cv_work.notify_all();
    return DD_OK;
}

namespace {
// Hand a finished request's results to the caller and forget it (the caller
// holds s->mu).
dd_status deliver(dd_server *s, long request_id, dd_solve_info *info, double *latency_ms)
{
    return (dd_status)s->q.take(request_id, info, latency_ms);
}
} // namespace

dd_status dd_server_poll(dd_server *s, long request_id, int *done, dd_solve_info *info, double *latency_ms)
{
    if (!s || !done) return DD_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->q.reqs.find(request_id);
    if (it == s->q.reqs.end()) return DD_INVALID_ARG;
    *done = it->second.complete ? 1 : 0;
    if (it->second.complete) return deliver(s, request_id, info, latency_ms);
    return DD_OK;
}

dd_status dd_server_wait(dd_server *s, long request_id, dd_solve_info *info, double *latency_ms)
{
    if (!s) return DD_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->q.reqs.find(request_id);
    if (it == s->q.reqs.end()) return DD_INVALID_ARG;
    // an element reference survives the rehash that a concurrent submit may
    // cause; an iterator does not
    const dd::ServeRequest &r = it->second;
    s->cv_done.wait(lk, [&] { return r.complete; });
    return deliver(s, request_id, info, latency_ms);
}

dd_status dd_server_get_stats(dd_server *s, dd_server_stats *out)
{
    if (!s || !out) return DD_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    const dd::ServeQueue &q = s->q;
    out->requests_done = (long)q.latencies_ms.size();
    out->rhs_done = q.rhs_done;
    out->iterations = q.iterations;
    out->p50_ms = dd::ServeQueue::percentile(q.latencies_ms, 0.50);
    out->p99_ms = dd::ServeQueue::percentile(q.latencies_ms, 0.99);
    double sum = 0;
    for (double l : q.latencies_ms) sum += l;
    out->mean_ms = q.latencies_ms.empty() ? 0 : sum / q.latencies_ms.size();
    out->wall_s = q.t_first < 0 ? 0 : q.t_last - q.t_first;
    out->rhs_per_s = out->wall_s > 0 ? q.rhs_done / out->wall_s : 0;
    out->busy_s = s->busy_s;
    out->workspace_bytes = s->used;
    return DD_OK;
}

dd_status dd_server_destroy(dd_server *s)
{
    if (!s) return DD_INVALID_ARG;
    s->stop.store(true);
    s->cv_work.notify_all();
    for (auto &w : s->workers)
        if (w.joinable()) w.join();
    (void)hipSetDevice(s->device);
    for (auto &f : s->fields) {
        f.eng.reset();
        if (f.ctx) dd_destroy(f.ctx);
        if (f.stream) (void)hipStreamDestroy(f.stream);
    }
    delete s;
    return DD_OK;
}

} // extern "C"
