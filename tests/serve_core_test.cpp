// Host test of the serving scheduler's bookkeeping (serve_core.h) with a CPU
// executor in place of the GPU slot engines.  The executor solves every
// admitted right-hand side with the FP64 oracle's SAP-preconditioned FGMRES
// at once, then holds the slot busy for as many scheduler steps as the solve
// took Arnoldi steps, so right-hand sides finish out of order and new ones
// are admitted into the slots that free up, as with the slot engines.
//
// Usage: serve_core_test DIR MODE
//   DIR/spec.txt   L0 L1 L2 L3 nfields width nreq fail_field fail_step
//                  then per field: csw; then per request: field nrhs step
//   DIR/U.bin      nfields gauge fields, canonical order, complex128
//   DIR/b.bin      the right-hand sides of all requests in order
//   DIR/m0.bin     their masses
//   MODE           "steps": one thread; request i is submitted at scheduler
//                  step `step`; every step runs one pass per field
//                  "threads": one worker thread per field and a submitting
//                  thread, as in the server
// Writes DIR/x.bin (the solutions) and prints a log, one event a line:
//   admit STEP FIELD SLOT REQ RHS
//   pass STEP FIELD FREE QUEUED      (after admission: free slots, rhs waiting)
//   done STEP FIELD SLOT REQ RHS ITERS
//   complete REQ STATUS LATENCY_MS RHS_ITERS...
//   stats P50 P99 RHS_DONE ITERATIONS
#include <atomic>
#include <chrono>
#include <complex>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../paper_1710_07041_amd/csrc/serve_core.h"

typedef std::complex<double> cd;

// The oracle's C interface (double complex arrays are layout-compatible with
// std::complex<double>).
extern "C" {
typedef struct {
    int iterations, restarts, precond_calls, status;
    double rel_residual;
} or_info;
void or_clover_field(const int L[4], const cd *U, double csw, cd *C);
int or_fgmres(const int L[4], const int B[4], const int bcs[4], const cd *U, const cd *C, double m0,
              const cd *b, cd *x, int m, double tol, int max_restarts, int ncy, int nmr, void *pre,
              void *pre_user, or_info *info);
}

namespace {

const int BLK[4] = {4, 4, 4, 4};
const int BCS[4] = {1, 1, 1, -1};

enum { FREE, BUSY, DONE };

// One field's stand-in for the slot engine.
struct Executor {
    int L[4];
    long V = 0;
    const cd *U = nullptr;
    std::vector<cd> C;
    struct Slot {
        int state = FREE;
        int left = 0;
        std::vector<cd> x;
        dd_solve_info info{};
    };
    std::vector<Slot> slots;

    void admit(int k, const double *b, double m0)
    {
        Slot &s = slots[k];
        if (s.state != FREE) {
            std::fprintf(stderr, "slot %d admitted while not free\n", k);
            std::exit(3);
        }
        s.x.assign(V * 12, cd(0, 0));
        or_info oi{};
        or_fgmres(L, BLK, BCS, U, C.data(), m0, (const cd *)b, s.x.data(), 10, 1e-10, 50, 2, 4, nullptr,
                  nullptr, &oi);
        s.info.status = oi.status == 0 ? DD_OK : DD_NOT_CONVERGED;
        s.info.iterations = oi.iterations;
        s.info.restarts = oi.restarts;
        s.info.sap_calls = oi.precond_calls;
        s.info.rel_residual = oi.rel_residual;
        s.left = oi.iterations > 0 ? oi.iterations : 1;
        s.state = BUSY;
    }
    int busy() const
    {
        int n = 0;
        for (const Slot &s : slots) n += s.state == BUSY;
        return n;
    }
    // one Arnoldi step of every busy slot
    void step()
    {
        for (Slot &s : slots)
            if (s.state == BUSY && --s.left == 0) s.state = DONE;
    }
};

struct World {
    std::vector<Executor> ex;
    std::vector<std::vector<std::pair<long, int>>> owner;
    dd::ServeQueue q;
    std::mutex mu;
    std::condition_variable cv_done;
    size_t vstride = 0;
    int fail_field = -1, fail_step = -1;
    bool failed = false;
};

// One scheduler pass of field fi (the server's work_once with the executor
// in place of the engine).  Returns false once the field has failed.
bool pass(World &w, int fi, long step, double now)
{
    Executor &e = w.ex[fi];
    auto &own = w.owner[fi];
    std::vector<dd::ServeAdmit> adm;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        w.q.admit(fi, [&](int k) { return e.slots[k].state == FREE; }, own, w.vstride, now, adm);
        int nfree = 0;
        for (int k = 0; k < (int)own.size(); ++k) nfree += e.slots[k].state == FREE && own[k].first == 0;
        long waiting = 0;
        for (long id : w.q.queue) {
            const dd::ServeRequest &r = w.q.reqs.at(id);
            if (r.field == fi) waiting += r.nrhs - r.next_rhs;
        }
        for (const dd::ServeAdmit &a : adm)
            std::printf("admit %ld %d %d %ld %d\n", step, fi, a.slot, a.req, a.rhs);
        std::printf("pass %ld %d %d %ld\n", step, fi, nfree, waiting);
    }
    for (const dd::ServeAdmit &a : adm) e.admit(a.slot, a.b, a.m0);
    if (fi == w.fail_field && step >= w.fail_step && e.busy()) {
        std::lock_guard<std::mutex> lk(w.mu);
        w.q.fail_all(DD_HIP_ERROR);
        w.failed = true;
        w.cv_done.notify_all();
        return false;
    }
    if (!e.busy()) return true;
    e.step();
    std::vector<dd::ServeDone> fin;
    for (int k = 0; k < (int)e.slots.size(); ++k) {
        Executor::Slot &s = e.slots[k];
        if (s.state != DONE) continue;
        std::lock_guard<std::mutex> lk(w.mu);
        double *dst = w.q.result(own[k].first, own[k].second, w.vstride);
        if (dst) std::copy(s.x.begin(), s.x.end(), (cd *)dst);
        std::printf("done %ld %d %d %ld %d %d\n", step, fi, k, own[k].first, own[k].second, s.info.iterations);
        fin.push_back({own[k].first, own[k].second, s.info});
        s.state = FREE;
        own[k] = {0, 0};
    }
    std::lock_guard<std::mutex> lk(w.mu);
    if (w.q.finish(fin, now)) w.cv_done.notify_all();
    return true;
}

template <class T> std::vector<T> read_bin(const std::string &path)
{
    std::ifstream f(path, std::ios::binary | std::ios::ate);
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path.c_str());
        std::exit(2);
    }
    const size_t n = (size_t)f.tellg() / sizeof(T);
    std::vector<T> v(n);
    f.seekg(0);
    f.read((char *)v.data(), n * sizeof(T));
    return v;
}

double wall()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

} // namespace

int main(int argc, char **argv)
{
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s DIR steps|threads\n", argv[0]);
        return 2;
    }
    const std::string dir = argv[1], mode = argv[2];
    std::ifstream spec(dir + "/spec.txt");
    int L[4], nf, width, nreq;
    World w;
    spec >> L[0] >> L[1] >> L[2] >> L[3] >> nf >> width >> nreq >> w.fail_field >> w.fail_step;
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    w.vstride = (size_t)V * 24;
    std::vector<double> csw(nf);
    for (double &c : csw) spec >> c;
    std::vector<int> rf(nreq), rn(nreq), rstep(nreq);
    for (int i = 0; i < nreq; ++i) spec >> rf[i] >> rn[i] >> rstep[i];
    if (!spec) {
        std::fprintf(stderr, "bad spec\n");
        return 2;
    }
    const std::vector<cd> U = read_bin<cd>(dir + "/U.bin");
    const std::vector<double> b = read_bin<double>(dir + "/b.bin");
    const std::vector<double> m0 = read_bin<double>(dir + "/m0.bin");
    long tot = 0;
    for (int n : rn) tot += n;
    if ((long)U.size() != nf * V * 36 || (long)b.size() != tot * (long)w.vstride || (long)m0.size() != tot) {
        std::fprintf(stderr, "input sizes do not match the spec\n");
        return 2;
    }
    std::vector<double> x(b.size(), 0.0);
    w.ex.resize(nf);
    w.owner.assign(nf, std::vector<std::pair<long, int>>(width, {0, 0}));
    for (int f = 0; f < nf; ++f) {
        Executor &e = w.ex[f];
        std::copy(L, L + 4, e.L);
        e.V = V;
        e.U = U.data() + f * V * 36;
        e.C.resize(V * 144);
        or_clover_field(L, e.U, csw[f], e.C.data());
        e.slots.resize(width);
    }
    std::vector<long> id(nreq);
    std::vector<long> off(nreq);
    for (int i = 0, o = 0; i < nreq; o += rn[i], ++i) off[i] = o;
    auto submit = [&](int i, double now) {
        std::lock_guard<std::mutex> lk(w.mu);
        id[i] = w.q.submit(rf[i], rn[i], m0.data() + off[i], b.data() + off[i] * w.vstride,
                           x.data() + off[i] * w.vstride, now);
    };

    if (mode == "steps") {
        int submitted = 0;
        for (long step = 0; step < 100000; ++step) {
            for (int i = 0; i < nreq; ++i)
                if (rstep[i] == step) submit(i, (double)step), ++submitted;
            bool alive = true;
            for (int f = 0; f < nf && alive; ++f) alive = pass(w, f, step, (double)step);
            if (!alive) break;
            bool all = submitted == nreq;
            for (int i = 0; i < nreq && all; ++i) all = w.q.reqs.at(id[i]).complete;
            if (all) break;
        }
    } else if (mode == "threads") {
        std::atomic<bool> stop{false};
        std::vector<std::thread> workers;
        for (int f = 0; f < nf; ++f)
            workers.emplace_back([&, f] {
                for (long step = 0; !stop.load(); ++step) {
                    if (!pass(w, f, step, wall())) return;
                    std::this_thread::yield();
                }
            });
        for (int i = 0; i < nreq; ++i) {
            submit(i, wall());
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
        {
            std::unique_lock<std::mutex> lk(w.mu);
            w.cv_done.wait(lk, [&] {
                for (int i = 0; i < nreq; ++i)
                    if (!w.q.reqs.at(id[i]).complete) return false;
                return true;
            });
        }
        stop.store(true);
        for (auto &t : workers) t.join();
    } else {
        std::fprintf(stderr, "unknown mode %s\n", mode.c_str());
        return 2;
    }

    for (int i = 0; i < nreq; ++i) {
        if (!w.q.reqs.at(id[i]).complete) {
            std::fprintf(stderr, "request %ld never completed\n", id[i]);
            return 1;
        }
        std::vector<dd_solve_info> info(rn[i]);
        double lat = 0;
        const int st = w.q.take(id[i], info.data(), &lat);
        std::printf("complete %ld %d %.6f", id[i], st, lat);
        for (const dd_solve_info &in : info) std::printf(" %d", in.iterations);
        std::printf("\n");
    }
    std::printf("stats %.6f %.6f %ld %ld\n", dd::ServeQueue::percentile(w.q.latencies_ms, 0.5),
                dd::ServeQueue::percentile(w.q.latencies_ms, 0.99), w.q.rhs_done, w.q.iterations);
    if (!w.q.reqs.empty()) {
        std::fprintf(stderr, "requests left after delivery\n");
        return 1;
    }
    std::ofstream xo(dir + "/x.bin", std::ios::binary);
    xo.write((const char *)x.data(), x.size() * sizeof(double));
    return 0;
}
