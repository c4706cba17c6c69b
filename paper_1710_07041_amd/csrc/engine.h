// Batched SAP-preconditioned FGMRES engine with independent slots (engine.hip).
#pragma once

#include <complex>
#include <memory>
#include <vector>

#include "dd_internal.h"

namespace dd {

constexpr int ENGINE_MAXW = 16; // slots per engine (right-hand sides fused per launch)
constexpr int ENGINE_MAXM = 32; // largest Krylov dimension

struct EngineParams {
    int width = 1;
    int m = 20;
    int ncy = 12;
    int nmr = 4;
    int sap_prec = DD_F32;
    bool sap_eo = false; // even-odd preconditioned block solves
    double tol = 1e-10;
    int max_restarts = 100;
    bool graphs = false; // capture the Arnoldi step as hipGraphs (needs a non-null stream)
    bool amg = false;    // precondition with the two-grid method of dd_amg_setup (FP32/FP64 smoother)
};

enum SlotStateKind { SLOT_FREE = 0, SLOT_RESTART = 1, SLOT_CYCLE = 2, SLOT_DONE = 3 };

struct SlotState {
    int state = SLOT_FREE;
    int j = 0;         // Arnoldi steps in the current cycle
    int cycle_len = 0; // length of a cycle that just ended (combine pending)
    bool need_bnorm = false;
    double bnorm = 0, m0 = 0;
    double beta0 = 0;     // |r| at the start of the cycle
    double beta_prev = 0; // last subdiagonal entry, against the not yet reorthogonalised p_j
    // H: unrotated Hessenberg matrix ((m+1) x m, row stride m); R, g, cs, sn:
    // its Givens QR and the rotated right-hand side, rebuilt by qr()
    std::vector<std::complex<double>> H, R, g, sn;
    std::vector<double> cs;
    // QR of the leading (n+1) x n block; returns the residual estimate |g[n]|
    double qr(int m, int n);
    // y = R^-1 g over n columns (ENGINE_MAXM entries, the rest zero)
    void solve_y(int m, int n, std::complex<double> *y) const;
    // whether the QR factor of the leading n columns has a zero on its
    // diagonal (the projected least-squares problem has no unique solution)
    bool singular(int m, int n) const;
    dd_solve_info info{};
    // initial guess known to be zero (none given, or all entries zero as the
    // packing pass found): the first residual is b, with no operator call
    bool x0_zero = false;
    bool x0_check = false; // the packing pass's nonzero flag is still on the device
    long owner = 0;        // caller's tag (request id) and right-hand-side index
    int owner_rhs = 0;
};

class Engine {
  public:
    Engine();
    ~Engine();
    Status init(dd_ctx *ctx, const EngineParams &p);
    void set_params(const EngineParams &p);
    // Place right-hand side b (canonical FP64, device) with initial guess x0
    // (canonical FP64 device, or nullptr for zero) into free slot r.
    Status admit(int r, const double *b_canon, const double *x0_canon, double m0, long owner, int owner_rhs);
    // One restart phase then one Arnoldi step for every busy slot (synchronises).
    Status iterate();
    // The same, split so that several engines can overlap on the device.
    Status launch_restart();
    Status finish_restart();
    Status launch_step();
    Status finish_step();
    // Copy slot r's solution to a canonical FP64 device buffer (async).
    Status extract(int r, double *x_canon);
    void release(int r);
    int free_slot() const;
    int busy_slots() const;
    int width() const;
    const EngineParams &params() const;
    SlotState &slot(int r);
    dd_ctx *ctx() const;
    static size_t bytes_per_slot(const GeomHost &g, int m, int sap_prec);
    // (re)size the two-grid preconditioner's workspace for the context's setup
    Status prepare_amg();

  private:
    struct Impl;
    std::unique_ptr<Impl> d;
};

} // namespace dd
