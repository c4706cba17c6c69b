// The serving scheduler's bookkeeping, apart from the engines that do the
// work: the FIFO of requests, the admission of their right-hand sides into
// the free slots of their field's executor, and the completion accounting
// (latency, throughput).  Host-only C++ with no GPU types, so that the
// server (server.hip, slot engines on the GPU) and a host test (a CPU
// executor) drive the same code.  The caller serialises every call (the
// server holds its mutex).
#pragma once

#include <algorithm>
#include <cstddef>
#include <deque>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/ddsap.h"

namespace dd {

struct ServeRequest {
    long id = 0;
    int field = 0;
    int nrhs = 0;
    std::vector<double> m0;
    const double *b = nullptr; // nrhs canonical right-hand sides, rhs stride vstride
    double *x = nullptr;       // their solutions
    int next_rhs = 0;          // next right-hand side to admit
    int done_rhs = 0;
    std::vector<dd_solve_info> info;
    double t_submit = 0, t_admit = -1, t_done = 0;
    bool complete = false;
    int status = DD_OK;
};

// One right-hand side placed into a slot by admit().
struct ServeAdmit {
    int slot;
    long req;
    int rhs;
    const double *b;
    double m0;
};

// One finished right-hand side reported to finish().
struct ServeDone {
    long req;
    int rhs;
    dd_solve_info info;
};

class ServeQueue {
  public:
    std::deque<long> queue; // requests with right-hand sides not yet admitted, FIFO
    std::unordered_map<long, ServeRequest> reqs;
    std::vector<double> latencies_ms;
    long rhs_done = 0, iterations = 0;
    double t_first = -1, t_last = 0;

    long submit(int field, int nrhs, const double *m0, const double *b, double *x, double now)
    {
        ServeRequest r;
        r.id = next_id_++;
        r.field = field;
        r.nrhs = nrhs;
        r.m0.assign(m0, m0 + nrhs);
        r.b = b;
        r.x = x;
        r.info.assign(nrhs, dd_solve_info{});
        r.t_submit = now;
        if (t_first < 0) t_first = now;
        queue.push_back(r.id);
        const long id = r.id;
        reqs.emplace(id, std::move(r));
        return id;
    }

    // FIFO admission of field fi's queued right-hand sides into its free
    // slots: slot k is taken when the executor has it free (is_free(k)) and
    // no admission holds it yet (owner[k].first == 0).  A request's
    // right-hand sides go in order, and a later request of the field is
    // admitted only after every right-hand side of the earlier ones.
    template <class IsFree>
    void admit(int fi, IsFree is_free, std::vector<std::pair<long, int>> &owner, size_t vstride, double now,
               std::vector<ServeAdmit> &out)
    {
        for (auto it = queue.begin(); it != queue.end();) {
            auto found = reqs.find(*it);
            if (found == reqs.end()) { // forgotten (cannot happen while queued; kept safe)
                it = queue.erase(it);
                continue;
            }
            ServeRequest &r = found->second;
            if (r.field != fi) {
                ++it;
                continue;
            }
            bool full = false;
            while (r.next_rhs < r.nrhs) {
                int slot = -1;
                for (int k = 0; k < (int)owner.size() && slot < 0; ++k)
                    if (is_free(k) && owner[k].first == 0) slot = k;
                if (slot < 0) {
                    full = true;
                    break;
                }
                owner[slot] = {r.id, r.next_rhs};
                out.push_back({slot, r.id, r.next_rhs, r.b + r.next_rhs * vstride, r.m0[r.next_rhs]});
                if (r.t_admit < 0) r.t_admit = now;
                ++r.next_rhs;
            }
            if (r.next_rhs == r.nrhs) it = queue.erase(it);
            else ++it;
            if (full) break; // FIFO: no later request of this field overtakes
        }
    }

    // Where right-hand side rhs of request req goes (nullptr once the
    // request has been delivered and forgotten).
    double *result(long req, int rhs, size_t vstride)
    {
        auto it = reqs.find(req);
        return it == reqs.end() ? nullptr : it->second.x + (size_t)rhs * vstride;
    }

    // Account finished right-hand sides; returns whether any request completed.
    bool finish(const std::vector<ServeDone> &done, double now)
    {
        bool any = false;
        for (const ServeDone &d : done) {
            auto it = reqs.find(d.req);
            if (it == reqs.end()) continue;
            ServeRequest &r = it->second;
            r.info[d.rhs] = d.info;
            if (d.info.status != DD_OK && r.status == DD_OK) r.status = d.info.status;
            iterations += d.info.iterations;
            ++rhs_done;
            if (++r.done_rhs == r.nrhs) {
                r.complete = true;
                r.t_done = now;
                latencies_ms.push_back((r.t_done - r.t_submit) * 1e3);
                t_last = now;
                any = true;
            }
        }
        return any;
    }

    // Hand over completed request id (info: nrhs entries, may be NULL;
    // latency_ms may be NULL) and forget it; returns its status
    // (DD_INVALID_ARG for an unknown id).
    int take(long id, dd_solve_info *info, double *latency_ms)
    {
        auto it = reqs.find(id);
        if (it == reqs.end()) return DD_INVALID_ARG;
        const ServeRequest &r = it->second;
        if (info) std::copy(r.info.begin(), r.info.end(), info);
        if (latency_ms) *latency_ms = (r.t_done - r.t_submit) * 1e3;
        const int st = r.status;
        reqs.erase(it);
        return st;
    }

    // A fatal error: every request not yet complete completes with code.
    void fail_all(int code)
    {
        for (auto &kv : reqs)
            if (!kv.second.complete) {
                kv.second.complete = true;
                kv.second.status = code;
            }
        queue.clear();
    }

    // q-quantile of the completed requests' latencies (linear interpolation).
    static double percentile(std::vector<double> v, double q)
    {
        if (v.empty()) return 0.0;
        std::sort(v.begin(), v.end());
        const double pos = q * (v.size() - 1);
        const size_t lo = (size_t)pos;
        const size_t hi = std::min(lo + 1, v.size() - 1);
        const double f = pos - lo;
        return v[lo] * (1 - f) + v[hi] * f;
    }

  private:
    long next_id_ = 1;
};

} // namespace dd
