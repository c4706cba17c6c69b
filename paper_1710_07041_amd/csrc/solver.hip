// SAP-preconditioned flexible GMRES(m) (Saad, SIAM J. Sci. Comput. 14 (1993)
// 461) with an FP64 outer iteration and an FP32 / FP16-storage smoother -- the
// mixed-precision structure of the paper's solver (Sec. 3.1: mixed precision,
// some data structures in half precision; the Schwarz method as the
// fine-grid smoother).  Flexible GMRES is required because SAP with MR block
// solves is not a linear map of its input.
//
// Device side, per Arnoldi step j (every right-hand side in lock step):
//   lp   = v_j in the smoother precision (FP16: scaled so max|lp| = 1)
//   z_j  = SAP(lp)                (FP32 storage for the basis Z; FP16 unscaled)
//   w    = D z_j                  (FP64 operator reading the stored z_j, so the
//                                  Arnoldi relation D Z = V H holds exactly)
//   classical Gram-Schmidt with one re-orthogonalisation (CGS2) in three
//   fused passes over V:
//     (1) h1 = V^+ w
//     (2) w' = w - V h1, h2 = V^+ w', |w'|^2, max|w'|
//     (3) w'' = w' - V h2, v_{j+1} = w''/h, lp copy,  h^2 = |w'|^2 - |h2|^2
//   All reductions are two-stage with a fixed summation order (bitwise
//   reproducible); one small device-to-host copy per step feeds the host-side
//   Givens rotations and the stopping test.  Restarts recompute the true
//   residual b - D x in FP64 on the device; the solve stops only on it.
// Right-hand sides that have converged are masked at the restart boundary
// (zero basis vectors); one that finishes its cycle early rides along in the
// fused launches until the restart, its extra columns never read.
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

namespace {

constexpr int TPB = 256;
constexpr int MAXM = 32;          // largest Krylov dimension supported
constexpr int KMAX = MAXM + 1 + 2; // reduction slots: dots + |w|^2 + max|w|

typedef cx<double> C64;

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum a per-thread value over the workgroup (fixed order) and have thread 0
// write it.  red: 4 doubles of LDS.
__device__ __forceinline__ double wg_sum(double v, double *red)
{
    v = wave_sum_d(v);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}
__device__ __forceinline__ double wg_max(double v, double *red)
{
    v = wave_max_d(v);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Pass 1: partial[g][r][i] = sum over this workgroup's blocks of <V_i, w>
template <int NV>
__global__ __launch_bounds__(TPB) void k_dots(const double2 *__restrict__ V, long vstride, int nv,
                                              const double2 *__restrict__ w, double2 *__restrict__ partial,
                                              int nblocks, int nrhs, int K)
{
    __shared__ double red[4];
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    C64 acc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = mk(0.0, 0.0);
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 wc = ldc<double>(w + base + c * BS);
            // unconditional loads keep all NV in flight; slots i >= nv
            // re-read the last vector and are never written out
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : nv - 1;
                cmacc(acc[i], ldc<double>(V + ii * vstride + base + c * BS), wc);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) { // nv is uniform over the workgroup
            double re = wg_sum(acc[i].re, red);
            double im = wg_sum(acc[i].im, red);
            if (s == 0) partial[((long)g * nrhs + r) * K + i] = make_double2(re, im);
        }
    }
}

// Pass 2: w' = w - sum_i h[r][i] V_i ; partial <V_i, w'>, |w'|^2 (slot nv),
// max|w'| (slot nv+1, in .x).  nv may be 0 (plain norm + max).
template <int NV>
__global__ __launch_bounds__(TPB) void k_update_dots(const double2 *__restrict__ V, long vstride, int nv,
                                                     const double2 *__restrict__ h, double2 *__restrict__ w,
                                                     double2 *__restrict__ partial, int nblocks, int nrhs, int K,
                                                     int hK)
{
    __shared__ double red[4];
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    C64 hc[NV > 0 ? NV : 1], acc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        acc[i] = mk(0.0, 0.0);
        hc[i] = i < nv ? ldc<double>(h + (long)r * hK + i) : mk(0.0, 0.0);
    }
    double n2 = 0.0, mx = 0.0;
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 vv[NV > 0 ? NV : 1];
            C64 wc = ldc<double>(w + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : nv - 1; // hc[i] = 0 beyond nv
                vv[i] = ldc<double>(V + ii * vstride + base + c * BS);
                wc = wc - hc[i] * vv[i];
            }
            stc(w + base + c * BS, wc);
#pragma unroll
            for (int i = 0; i < NV; ++i) cmacc(acc[i], vv[i], wc);
            n2 = fma(wc.re, wc.re, fma(wc.im, wc.im, n2));
            mx = fmax(mx, fmax(fabs(wc.re), fabs(wc.im)));
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) { // nv is uniform over the workgroup
            double re = wg_sum(acc[i].re, red);
            double im = wg_sum(acc[i].im, red);
            if (s == 0) partial[((long)g * nrhs + r) * K + i] = make_double2(re, im);
        }
    }
    double tn = wg_sum(n2, red);
    double tm = wg_max(mx, red);
    if (s == 0) {
        partial[((long)g * nrhs + r) * K + nv] = make_double2(tn, 0.0);
        partial[((long)g * nrhs + r) * K + nv + 1] = make_double2(tm, 0.0);
    }
}

// Per right-hand side normalisation constants, computed identically by every
// thread from the reduced pass-2 results:  h = sqrt(|w'|^2 - |h2|^2).
struct NormInfo {
    double inv;   // 1/h (0 when masked or h == 0)
    double scale; // factor applied to the smoother input copy
};
__device__ __forceinline__ NormInfo norm_info(const double2 *res, int K, int nv, int r, const int *active,
                                              bool fp16_scale)
{
    NormInfo ni{0.0, 0.0};
    if (!active[r]) return ni;
    const double2 *row = res + (long)r * K;
    double h2 = row[nv].x;
    for (int i = 0; i < nv; ++i) h2 -= row[i].x * row[i].x + row[i].y * row[i].y;
    double hn = sqrt(fmax(h2, 0.0));
    if (hn == 0.0) return ni;
    ni.inv = 1.0 / hn;
    // max|v| <= (max|w'| + |h2|-sized correction) / h ; 1.0625 leaves head room
    double mxv = row[nv + 1].x * ni.inv * 1.0625;
    ni.scale = fp16_scale ? (mxv > 0.0 ? 1.0 / mxv : 1.0) : 1.0;
    return ni;
}

// Pass 3: w'' = w' - sum_i h2[r][i] V_i ; vnext = w'' / h ; lp = scale * vnext
template <int NV, typename SL>
__global__ __launch_bounds__(TPB) void k_update_normalize(const double2 *__restrict__ V, long vstride, int nv,
                                                          const double2 *__restrict__ res, int K,
                                                          const double2 *__restrict__ w, double2 *__restrict__ vnext,
                                                          vec2_t<SL> *__restrict__ lp, double *__restrict__ scl,
                                                          const int *__restrict__ active, int fp16_scale,
                                                          int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    NormInfo ni = norm_info(res, K, nv, r, active, fp16_scale != 0);
    if (g == 0 && s == 0 && scl) scl[r] = ni.scale;
    C64 hc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hc[i] = i < nv ? ldc<double>(res + (long)r * K + i) : mk(0.0, 0.0);
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 wc = ldc<double>(w + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : nv - 1; // hc[i] = 0 beyond nv
                wc = wc - hc[i] * ldc<double>(V + ii * vstride + base + c * BS);
            }
            C64 v = ni.inv * wc;
            stc(vnext + base + c * BS, v);
            if (lp) stc(lp + base + c * BS, ni.scale * v);
        }
    }
}

// Deterministic second stage: out[r][k] = sum_g partial[g][r][k] (slot
// kmax_slot uses max instead of sum).
__global__ __launch_bounds__(TPB) void k_reduce(const double2 *__restrict__ partial, double2 *__restrict__ out, int G,
                                                int nrhs, int K, int kmax_slot)
{
    __shared__ double red[4];
    const int r = blockIdx.y, k = blockIdx.x, s = threadIdx.x;
    bool is_max = (k == kmax_slot);
    double re = 0.0, im = 0.0;
    for (int g = s; g < G; g += TPB) {
        double2 v = partial[((long)g * nrhs + r) * K + k];
        if (is_max) re = fmax(re, v.x);
        else {
            re += v.x;
            im += v.y;
        }
    }
    double tre = is_max ? wg_max(re, red) : wg_sum(re, red);
    double tim = is_max ? 0.0 : wg_sum(im, red);
    if (s == 0) out[(long)r * K + k] = make_double2(tre, tim);
}

// x += sum_i y[r][i] Z_i   (Z in FP64 or FP32)
template <int NV, typename SZ>
__global__ __launch_bounds__(TPB) void k_combine(double2 *__restrict__ x, const vec2_t<SZ> *__restrict__ Z, long zstride,
                                                 int nv, const double2 *__restrict__ y, const int *__restrict__ len,
                                                 int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    // columns beyond this right-hand side's cycle length are never read (a
    // dropped column may hold non-finite values)
    nv = nv < len[r] ? nv : len[r];
    if (nv == 0) return;
    C64 yc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) yc[i] = i < nv ? ldc<double>(y + (long)r * MAXM + i) : mk(0.0, 0.0);
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 xc = ldc<double>(x + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : nv - 1; // yc[i] = 0 beyond nv
                cmac(xc, yc[i], ldc<double>(Z + ii * zstride + base + c * BS));
            }
            stc(x + base + c * BS, xc);
        }
    }
}

// out = in / scl[r]  (FP16 smoother output -> FP32 basis vector)
__global__ __launch_bounds__(TPB) void k_unscale(const __half2 *__restrict__ in, float2 *__restrict__ out,
                                                 const double *__restrict__ scl, int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    double sc = scl[r];
    float f = sc != 0.0 ? (float)(1.0 / sc) : 0.0f;
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) stc(out + base + c * BS, f * ldc<float>(in + base + c * BS));
    }
}

} // namespace

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct SolverWork {
    int nrhs = 0, m = 0, zprec = -1;
    long vlen = 0; // complex entries of one vector (all rhs)
    DevBuf V, Z, w, xb, bb, lp, sapout, partial, res, res2, y, scl, active;
    double2 *h_res = nullptr;  // pinned: results of the last reduction
    double2 *h_res2 = nullptr; // pinned
    double2 *h_y = nullptr;    // pinned
    int *h_active = nullptr;   // pinned
    int G = 0;
    ~SolverWork()
    {
        if (h_res) (void)hipHostFree(h_res);
        if (h_res2) (void)hipHostFree(h_res2);
        if (h_y) (void)hipHostFree(h_y);
        if (h_active) (void)hipHostFree(h_active);
    }
};

void free_solver_work(dd_ctx *ctx) { ctx->work.reset(); }

void SolverWorkDeleter::operator()(SolverWork *w) const { delete w; }

namespace {

int pick_bucket(int nv)
{
    static const int b[] = {0, 1, 2, 3, 4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24, 28, 33};
    for (int v : b)
        if (nv <= v) return v;
    return 33;
}

struct Launch {
    dd_ctx *ctx;
    SolverWork *W;
    dim3 grid() const { return dim3(W->G, W->nrhs); }
};

#define DD_BUCKETS(X) X(0) X(1) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(28) X(33)

double vec64_bytes(const Launch &L) { return (double)L.W->vlen * 16.0; }

Status dots(const Launch &L, const double2 *V, int nv, const double2 *w)
{
    SolverWork *W = L.W;
    int K = KMAX;
    ProfScope ps(L.ctx->prof, L.ctx->stream, K_CGS_DOTS, vec64_bytes(L) * (nv + 1), 8.0 * W->vlen * nv);
    switch (pick_bucket(nv)) {
#define C(N) case N: k_dots<N><<<L.grid(), TPB, 0, L.ctx->stream>>>(V, W->vlen, nv, w, W->partial.as<double2>(), L.ctx->g.nblocks, W->nrhs, K); break;
        DD_BUCKETS(C)
#undef C
    }
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status update_dots(const Launch &L, const double2 *V, int nv, const double2 *h, double2 *w)
{
    SolverWork *W = L.W;
    ProfScope ps(L.ctx->prof, L.ctx->stream, K_CGS_UPDATE, vec64_bytes(L) * (nv + 2), 16.0 * W->vlen * nv + 4.0 * W->vlen);
    switch (pick_bucket(nv)) {
#define C(N) case N: k_update_dots<N><<<L.grid(), TPB, 0, L.ctx->stream>>>(V, W->vlen, nv, h, w, W->partial.as<double2>(), L.ctx->g.nblocks, W->nrhs, KMAX, KMAX); break;
        DD_BUCKETS(C)
#undef C
    }
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

template <typename SL>
Status update_normalize_t(const Launch &L, const double2 *V, int nv, const double2 *res, const double2 *w,
                          double2 *vnext, void *lp, bool fp16)
{
    SolverWork *W = L.W;
    ProfScope ps(L.ctx->prof, L.ctx->stream, K_CGS_NORMALIZE,
                 vec64_bytes(L) * (nv + 2) + (lp ? (double)W->vlen * 2 * sizeof(SL) : 0.0), 8.0 * W->vlen * (nv + 1));
    switch (pick_bucket(nv)) {
#define C(N) case N: k_update_normalize<N, SL><<<L.grid(), TPB, 0, L.ctx->stream>>>(V, W->vlen, nv, res, KMAX, w, vnext, static_cast<vec2_t<SL> *>(lp), W->scl.as<double>(), W->active.as<int>(), fp16 ? 1 : 0, L.ctx->g.nblocks, W->nrhs); break;
        DD_BUCKETS(C)
#undef C
    }
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status update_normalize(const Launch &L, const double2 *V, int nv, const double2 *res, const double2 *w,
                        double2 *vnext, int sap_prec)
{
    SolverWork *W = L.W;
    if (sap_prec == DD_F64) return update_normalize_t<double>(L, V, nv, res, w, vnext, nullptr, false);
    if (sap_prec == DD_F32) return update_normalize_t<float>(L, V, nv, res, w, vnext, W->lp.p, false);
    return update_normalize_t<__half>(L, V, nv, res, w, vnext, W->lp.p, true);
}

Status reduce(const Launch &L, int nslots, int kmax_slot, double2 *out)
{
    dim3 grid(nslots, L.W->nrhs);
    ProfScope ps(L.ctx->prof, L.ctx->stream, K_REDUCE, (double)L.W->G * L.W->nrhs * nslots * 16.0, 0.0);
    k_reduce<<<grid, TPB, 0, L.ctx->stream>>>(L.W->partial.as<double2>(), out, L.W->G, L.W->nrhs, KMAX, kmax_slot);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status combine(const Launch &L, double2 *x, int nv)
{
    SolverWork *W = L.W;
    const double2 *y = W->y.as<double2>();
    ProfScope ps(L.ctx->prof, L.ctx->stream, K_COMBINE,
                 vec64_bytes(L) * 2 + (double)W->vlen * 2 * real_bytes(W->zprec) * nv, 8.0 * W->vlen * nv);
    if (W->zprec == DD_F64) {
        switch (pick_bucket(nv)) {
#define C(N) case N: k_combine<N, double><<<L.grid(), TPB, 0, L.ctx->stream>>>(x, W->Z.as<double2>(), W->vlen, nv, y, W->active.as<int>(), L.ctx->g.nblocks, W->nrhs); break;
            DD_BUCKETS(C)
#undef C
        }
    } else {
        switch (pick_bucket(nv)) {
#define C(N) case N: k_combine<N, float><<<L.grid(), TPB, 0, L.ctx->stream>>>(x, W->Z.as<float2>(), W->vlen, nv, y, W->active.as<int>(), L.ctx->g.nblocks, W->nrhs); break;
            DD_BUCKETS(C)
#undef C
        }
    }
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status alloc_base(dd_ctx *ctx, SolverWork *W, int nrhs, int m, int zprec);

Status prepare(dd_ctx *ctx, int nrhs, int m, int sap_prec)
{
    auto &Wp = ctx->work;
    int zprec = sap_prec == DD_F64 ? DD_F64 : DD_F32;
    if (!(Wp && Wp->nrhs == nrhs && Wp->m >= m && Wp->zprec == zprec)) {
        Wp.reset(new SolverWork());
        DD_TRY(alloc_base(ctx, Wp.get(), nrhs, m, zprec));
    }
    // buffers that only some smoother precisions need; a workspace reused from
    // a solve in another precision may lack them
    SolverWork *W = Wp.get();
    if (sap_prec != DD_F64 && !W->lp.p) DD_TRY(W->lp.alloc((size_t)W->vlen * 2 * real_bytes(DD_F32)));
    if (sap_prec == DD_F16 && !W->sapout.p) DD_TRY(W->sapout.alloc((size_t)W->vlen * 2 * real_bytes(DD_F16)));
    return Status::ok();
}

Status alloc_base(dd_ctx *ctx, SolverWork *W, int nrhs, int m, int zprec)
{
    W->nrhs = nrhs;
    W->m = m;
    W->zprec = zprec;
    W->vlen = (long)ctx->g.nblocks * nrhs * 12 * BS;
    W->G = ctx->g.nblocks < 1024 ? ctx->g.nblocks : 1024;
    size_t v64 = (size_t)W->vlen * 16;
    DD_TRY(W->V.alloc(v64 * (m + 1)));
    DD_TRY(W->Z.alloc((size_t)W->vlen * 2 * real_bytes(zprec) * m));
    DD_TRY(W->w.alloc(v64));
    DD_TRY(W->xb.alloc(v64));
    DD_TRY(W->bb.alloc(v64));
    DD_TRY(W->partial.alloc((size_t)W->G * nrhs * KMAX * 16));
    DD_TRY(W->res.alloc((size_t)nrhs * KMAX * 16));
    DD_TRY(W->res2.alloc((size_t)nrhs * KMAX * 16));
    DD_TRY(W->y.alloc((size_t)nrhs * MAXM * 16));
    DD_TRY(W->scl.alloc((size_t)nrhs * 8));
    DD_TRY(W->active.alloc((size_t)nrhs * 4));
    DD_HIP_TRY(hipHostMalloc((void **)&W->h_res, (size_t)nrhs * KMAX * 16, hipHostMallocDefault));
    DD_HIP_TRY(hipHostMalloc((void **)&W->h_res2, (size_t)nrhs * KMAX * 16, hipHostMallocDefault));
    DD_HIP_TRY(hipHostMalloc((void **)&W->h_y, (size_t)nrhs * MAXM * 16, hipHostMallocDefault));
    DD_HIP_TRY(hipHostMalloc((void **)&W->h_active, (size_t)nrhs * 4, hipHostMallocDefault));
    return Status::ok();
}

typedef std::complex<double> Z64;

// LAPACK zlartg semantics: [c s; -conj(s) c] [f; g] = [r; 0], c >= 0 real
void givens(Z64 f, Z64 g, double &c, Z64 &s, Z64 &r)
{
    double af = std::abs(f), ag = std::abs(g);
    if (ag == 0.0) {
        c = 1.0;
        s = 0.0;
        r = f;
    } else if (af == 0.0) {
        c = 0.0;
        s = std::conj(g) / ag;
        r = ag;
    } else {
        double nrm = std::hypot(af, ag);
        Z64 ph = f / af;
        c = af / nrm;
        s = ph * std::conj(g) / nrm;
        r = ph * nrm;
    }
}

struct RhsState {
    std::vector<Z64> H; // (m+1) x m, row-major H[i*m + j]
    std::vector<Z64> g, sn;
    std::vector<double> cs;
    double bnorm = 0;
    int jlen = 0;         // Arnoldi steps in the current cycle
    bool in_cycle = false; // still extending the current cycle
    bool done = false;
    dd_solve_info info{};
};

} // namespace

Status solve(dd_ctx *ctx, const double *m0, const double *b, double *x, int nrhs, const dd_params &p,
             dd_solve_info *info_out)
{
    const int m = p.m;
    DD_TRY(prepare(ctx, nrhs, m, p.sap_prec));
    SolverWork *W = ctx->work.get();
    Launch L{ctx, W};
    hipStream_t st = ctx->stream;
    const long vlen = W->vlen;
    double2 *V = W->V.as<double2>();
    double2 *w = W->w.as<double2>();
    double2 *xb = W->xb.as<double2>();
    double2 *bb = W->bb.as<double2>();
    const size_t zbytes_vec = (size_t)vlen * 2 * real_bytes(W->zprec);
    auto Zj = [&](int j) { return static_cast<char *>(W->Z.p) + (size_t)j * zbytes_vec; };

    DD_TRY(pack_spinor(ctx, b, bb, DD_F64, nrhs));
    DD_TRY(pack_spinor(ctx, x, xb, DD_F64, nrhs));

    std::vector<RhsState> R(nrhs);
    for (auto &rs : R) {
        rs.H.assign((size_t)(m + 1) * m, 0.0);
        rs.g.assign(m + 1, 0.0);
        rs.sn.assign(m, 0.0);
        rs.cs.assign(m, 0.0);
        rs.info.status = DD_NOT_CONVERGED;
    }
    // |b|
    DD_HIP_TRY(hipMemcpyAsync(w, bb, (size_t)vlen * 16, hipMemcpyDeviceToDevice, st));
    DD_TRY(update_dots(L, V, 0, nullptr, w));
    DD_TRY(reduce(L, 2, 1, W->res.as<double2>()));
    DD_HIP_TRY(hipMemcpyAsync(W->h_res, W->res.p, (size_t)nrhs * KMAX * 16, hipMemcpyDeviceToHost, st));
    DD_HIP_TRY(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) {
        double n2 = W->h_res[(size_t)r * KMAX + 0].x;
        if (!std::isfinite(n2)) return Status{DD_NAN, "right-hand side holds NaN or Inf"};
        R[r].bnorm = std::sqrt(n2);
    }

    int sap_prec = p.sap_prec;
    for (int cycle = 0;; ++cycle) {
        // true residual r = b - D x (FP64), its norm and max
        DD_TRY(launch_dslash(ctx, m0, nrhs, xb, DD_F64, w, DD_F64, DD_F64, reinterpret_cast<const double *>(bb)));
        DD_TRY(update_dots(L, V, 0, nullptr, w));
        DD_TRY(reduce(L, 2, 1, W->res.as<double2>()));
        DD_HIP_TRY(hipMemcpyAsync(W->h_res, W->res.p, (size_t)nrhs * KMAX * 16, hipMemcpyDeviceToHost, st));
        DD_HIP_TRY(hipStreamSynchronize(st));
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            RhsState &rs = R[r];
            W->h_active[r] = 0;
            if (rs.done) continue;
            double beta = std::sqrt(W->h_res[(size_t)r * KMAX].x);
            if (!std::isfinite(beta)) {
                rs.done = true;
                rs.info.status = DD_NAN;
                rs.info.rel_residual = beta;
                continue;
            }
            rs.info.rel_residual = rs.bnorm > 0 ? beta / rs.bnorm : 0.0;
            if (rs.bnorm == 0.0 || beta / rs.bnorm <= p.tol) {
                rs.done = true;
                rs.info.status = DD_OK;
                continue;
            }
            if (cycle == p.max_restarts) {
                rs.done = true;
                rs.info.status = DD_NOT_CONVERGED;
                continue;
            }
            rs.info.restarts++;
            std::fill(rs.g.begin(), rs.g.end(), Z64(0.0));
            rs.g[0] = beta;
            rs.jlen = 0;
            rs.in_cycle = true;
            W->h_active[r] = 1;
            any = true;
        }
        if (!any) break;
        DD_HIP_TRY(hipMemcpyAsync(W->active.p, W->h_active, (size_t)nrhs * 4, hipMemcpyHostToDevice, st));
        // v_0 = r / beta (+ smoother-precision copy)
        DD_TRY(update_normalize(L, V, 0, W->res.as<double2>(), w, V, sap_prec));

        for (int j = 0; j < m; ++j) {
            double2 *vj = V + (long)j * vlen;
            // z_j = SAP(v_j)
            if (sap_prec == DD_F64) {
                DD_TRY(run_sap(ctx, m0, nrhs, vj, Zj(j), p.ncy, p.nmr, DD_F64));
            } else if (sap_prec == DD_F32) {
                DD_TRY(run_sap(ctx, m0, nrhs, W->lp.p, Zj(j), p.ncy, p.nmr, DD_F32));
            } else {
                DD_TRY(run_sap(ctx, m0, nrhs, W->lp.p, W->sapout.p, p.ncy, p.nmr, DD_F16));
                ProfScope ps(ctx->prof, st, K_CONVERT, (double)vlen * 12.0, 2.0 * vlen);
                k_unscale<<<L.grid(), TPB, 0, st>>>(W->sapout.as<__half2>(), reinterpret_cast<float2 *>(Zj(j)),
                                                    W->scl.as<double>(), ctx->g.nblocks, nrhs);
                DD_HIP_TRY(hipGetLastError());
            }
            // w = D z_j (FP64)
            DD_TRY(launch_dslash(ctx, m0, nrhs, Zj(j), W->zprec, w, DD_F64, DD_F64, nullptr));
            const int nv = j + 1;
            DD_TRY(dots(L, V, nv, w));
            DD_TRY(reduce(L, nv, -1, W->res.as<double2>()));
            DD_TRY(update_dots(L, V, nv, W->res.as<double2>(), w));
            DD_TRY(reduce(L, nv + 2, nv + 1, W->res2.as<double2>()));
            DD_TRY(update_normalize(L, V, nv, W->res2.as<double2>(), w, V + (long)nv * vlen, sap_prec));
            DD_HIP_TRY(hipMemcpyAsync(W->h_res, W->res.p, (size_t)nrhs * KMAX * 16, hipMemcpyDeviceToHost, st));
            DD_HIP_TRY(hipMemcpyAsync(W->h_res2, W->res2.p, (size_t)nrhs * KMAX * 16, hipMemcpyDeviceToHost, st));
            DD_HIP_TRY(hipStreamSynchronize(st));
            bool cont = false, broken = false;
            for (int r = 0; r < nrhs; ++r) {
                RhsState &rs = R[r];
                if (!rs.in_cycle) continue;
                const double2 *h1 = W->h_res + (size_t)r * KMAX;
                const double2 *h2 = W->h_res2 + (size_t)r * KMAX;
                double hh = h2[nv].x;
                for (int i = 0; i < nv; ++i) {
                    Z64 hij = Z64(h1[i].x, h1[i].y) + Z64(h2[i].x, h2[i].y);
                    rs.H[(size_t)i * m + j] = hij;
                    hh -= h2[i].x * h2[i].x + h2[i].y * h2[i].y;
                }
                double hn = std::sqrt(std::max(hh, 0.0));
                rs.H[(size_t)(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    Z64 a = rs.H[(size_t)i * m + j], c = rs.H[(size_t)(i + 1) * m + j];
                    rs.H[(size_t)i * m + j] = rs.cs[i] * a + rs.sn[i] * c;
                    rs.H[(size_t)(i + 1) * m + j] = -std::conj(rs.sn[i]) * a + rs.cs[i] * c;
                }
                Z64 rr;
                givens(rs.H[(size_t)j * m + j], rs.H[(size_t)(j + 1) * m + j], rs.cs[j], rs.sn[j], rr);
                rs.H[(size_t)j * m + j] = rr;
                rs.H[(size_t)(j + 1) * m + j] = 0.0;
                rs.g[j + 1] = -std::conj(rs.sn[j]) * rs.g[j];
                rs.g[j] = rs.cs[j] * rs.g[j];
                rs.info.iterations++;
                rs.info.sap_calls++;
                rs.jlen = j + 1;
                bool finite = std::isfinite(hn) && std::isfinite(std::abs(rr));
                if (!finite || hn == 0.0 || std::abs(rs.g[j + 1]) / rs.bnorm <= p.tol) {
                    rs.in_cycle = false;
                    W->h_active[r] = 0;
                    if (!finite) {
                        // drop the broken column; the restart recomputes the true residual
                        rs.jlen = j;
                        broken = true;
                    }
                } else {
                    cont = true;
                }
            }
            if (broken) {
                // a non-finite column (FP16 range exceeded in the smoother):
                // close the cycle for everyone and continue in FP32
                for (auto &rs : R) rs.in_cycle = false;
                if (sap_prec == DD_F16) sap_prec = DD_F32;
                break;
            }
            if (!cont) break;
            // A right-hand side that left its cycle keeps riding along in the
            // fused launches until the restart: its columns are never read
            // again (the host skips it, combine stops at its cycle length).
            DD_HIP_TRY(hipMemcpyAsync(W->active.p, W->h_active, (size_t)nrhs * 4, hipMemcpyHostToDevice, st));
        }
        // y = R^{-1} g per right-hand side, x += Z y
        int maxlen = 0;
        for (int r = 0; r < nrhs; ++r) {
            RhsState &rs = R[r];
            Z64 *y = reinterpret_cast<Z64 *>(W->h_y + (size_t)r * MAXM);
            for (int i = 0; i < MAXM; ++i) y[i] = 0.0;
            if (rs.done) continue;
            for (int i = rs.jlen - 1; i >= 0; --i) {
                Z64 acc = rs.g[i];
                for (int k = i + 1; k < rs.jlen; ++k) acc -= rs.H[(size_t)i * m + k] * y[k];
                y[i] = acc / rs.H[(size_t)i * m + i];
            }
            maxlen = std::max(maxlen, rs.jlen);
        }
        if (maxlen > 0) {
            // the mask buffer carries the per right-hand-side cycle lengths here
            for (int r = 0; r < nrhs; ++r) W->h_active[r] = R[r].done ? 0 : R[r].jlen;
            DD_HIP_TRY(hipMemcpyAsync(W->active.p, W->h_active, (size_t)nrhs * 4, hipMemcpyHostToDevice, st));
            DD_HIP_TRY(hipMemcpyAsync(W->y.p, W->h_y, (size_t)nrhs * MAXM * 16, hipMemcpyHostToDevice, st));
            DD_TRY(combine(L, xb, maxlen));
        }
    }
    DD_TRY(unpack_spinor(ctx, xb, x, DD_F64, nrhs));
    DD_HIP_TRY(hipStreamSynchronize(st));
    Status out = Status::ok();
    for (int r = 0; r < nrhs; ++r) {
        if (info_out) info_out[r] = R[r].info;
        if (R[r].info.status != DD_OK && out.good())
            out = Status{(dd_status)R[r].info.status, "right-hand side " + std::to_string(r) + " did not converge"};
    }
    return out;
}

} // namespace dd
