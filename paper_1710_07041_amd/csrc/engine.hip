// Batched SAP-preconditioned FGMRES engine with independent slots.
//
// Flexible GMRES (Saad, SIAM J. Sci. Comput. 14 (1993) 461) with an FP64
// outer iteration and the red-black Schwarz smoother in FP64, FP32 or FP16
// storage -- the mixed-precision structure of the paper's solver (Sec. 3.1:
// a low-precision smoother with part of its data in 16-bit floating point,
// and the Schwarz method as the fine-grid smoother).  Flexible GMRES is needed because SAP with MR
// block solves is not a linear map of its input.
//
// One engine serves `width` right-hand-side slots of one lattice.  Every slot
// runs its own FGMRES(m): its own mass, restart count, Arnoldi index j and
// Hessenberg matrix.  The device work of one Arnoldi step is fused over all
// slots that are inside a cycle:
//   z_j   = SAP(v_j)          (one multi-RHS SAP launch per colour sweep; the
//                              smoother writes straight into slot r's Z[j_r])
//   w     = D z_j             (FP64 operator reading the stored z_j, so the
//                              Arnoldi relation D Z = V H holds exactly)
//   CGS2 with the reorthogonalisation of v_j delayed into step j+1 (the
//   low-synchronisation "DCGS2" arrangement: Swirydowicz, Langou, Ananthan,
//   Yang, Thomas, Numer. Linear Algebra Appl. 28 (2021) e2343), two passes
//   over V per step instead of three.  V[j] holds p_j, the once-orthogonalised
//   and normalised vector of the previous step, and V[0..j-1] the final basis:
//     (A) c = V[0..j-1]^+ p_j, |p_j|^2, s = V[0..j-1]^+ w, <p_j, w>, |w|^2
//     (B) v_j = (p_j - V c)/alpha (written over p_j),
//         w'  = w - V[0..j-1] s - h_jj v_j,  p_{j+1} = w'/beta,
//         smoother-precision copy of p_{j+1}
//   with alpha^2 = |p_j|^2 - |c|^2, h_jj = (<p_j, w> - c^+ s)/alpha and
//   beta^2 = |w|^2 - |s|^2 - |h_jj|^2.  Since p_j = V c + alpha v_j, the
//   Hessenberg column j-1 (whose last entry was beta_{j-1} against p_j) is
//   finished at step j: h_{i,j-1} += beta_{j-1} c_i, h_{j,j-1} = beta_{j-1}
//   alpha.  The stopping estimate of step j uses column j as it stands; its
//   correction is of the size of the rounding error of once-orthogonalised
//   Gram-Schmidt and only the FP64 true residual stops a slot.  The smoother
//   sees p_j rather than v_j, which flexible GMRES allows (z_j is any vector;
//   the Arnoldi relation D Z = V H is kept exactly).
// Per-slot data (masses, basis indices, masks, offsets) live in device
// memory, so the launch sequence of a step has fixed arguments and is
// captured once per CGS bucket as a hipGraph and replayed.  Reductions are
// two-stage with a fixed summation order; one small device-to-host copy per
// phase feeds the host-side Givens rotations and stopping tests.  Restarts
// recompute the true residual b - D x in FP64; a slot stops only on it.
//
// A slot whose cycle ends early rides along in the fused launches until its
// restart: its masked writes are skipped and its columns are never read.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstddef>
#include <cstring>
#include <map>
#include <vector>

#include "dd_device.h"
#include "dd_internal.h"
#include "engine.h"

namespace dd {

namespace {

constexpr int TPB = 256;
// Reduction slots per rhs.  The lagged dot pass stores <V_i, w> in slot 2i
// and <V_i, p> in slot 2i+1; the single-target passes use slots 0..nv-1.
constexpr int KMAX = 2 * (ENGINE_MAXM + 1) + 2;
constexpr int K_NORM = KMAX - 2;       // |w|^2
constexpr int K_MAX = KMAX - 1;        // max|w|
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
// workgroup sum / max in a fixed order (result valid in every thread)
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

__device__ __forceinline__ int slot_nv(const int *nv_dev, int nvmax, int r) { return nv_dev ? nv_dev[r] : nvmax; }

// Restart pass: w' = w - sum_{i<nv_r} h[r][i] V_i ; partial <V_i, w'>, |w'|^2,
// max|w'| (with nv = 0: |w|^2 and max|w| of the restart residual and of b).
template <int NV>
__global__ __launch_bounds__(TPB) void k_update_dots(const double2 *__restrict__ V, long vstride, int nvmax,
                                                     const int *__restrict__ nv_dev, const double2 *__restrict__ h,
                                                     double2 *__restrict__ w, double2 *__restrict__ partial,
                                                     int nblocks, int nrhs)
{
    __shared__ double red[4];
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    const int nv = slot_nv(nv_dev, nvmax, r);
    C64 hc[NV > 0 ? NV : 1], acc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        acc[i] = mk(0.0, 0.0);
        hc[i] = i < nv ? ldc<double>(h + (long)r * KMAX + i) : mk(0.0, 0.0);
    }
    double n2 = 0.0, mx = 0.0;
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 vv[NV > 0 ? NV : 1];
            C64 wc = ldc<double>(w + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : (nv > 0 ? nv - 1 : 0); // hc[i] = 0 beyond nv
                vv[i] = ldc_stream<double>(V + ii * vstride + base + c * BS);
                wc = wc - hc[i] * vv[i];
            }
            if (NV > 0) stc(w + base + c * BS, wc);
#pragma unroll
            for (int i = 0; i < NV; ++i) cmacc(acc[i], vv[i], wc);
            n2 = fma(wc.re, wc.re, fma(wc.im, wc.im, n2));
            mx = fmax(mx, fmax(fabs(wc.re), fabs(wc.im)));
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) {
            double re = wg_sum(acc[i].re, red);
            double im = wg_sum(acc[i].im, red);
            if (s == 0) partial[((long)g * nrhs + r) * KMAX + i] = make_double2(re, im);
        }
    }
    double tn = wg_sum(n2, red);
    double tm = wg_max(mx, red);
    if (s == 0) {
        partial[((long)g * nrhs + r) * KMAX + K_NORM] = make_double2(tn, 0.0);
        partial[((long)g * nrhs + r) * KMAX + K_MAX] = make_double2(tm, 0.0);
    }
}

// Normalisation constants of slot r from the reduced pass-2 results.
struct NormInfo {
    double inv;   // 1/h (0 when h == 0)
    double scale; // factor applied to the smoother-precision copy
};
__device__ __forceinline__ NormInfo norm_info(const double2 *res, int nv, int r, bool fp16_scale)
{
    NormInfo ni{0.0, 0.0};
    const double2 *row = res + (long)r * KMAX;
    double h2 = row[K_NORM].x;
    for (int i = 0; i < nv; ++i) h2 -= row[i].x * row[i].x + row[i].y * row[i].y;
    double hn = sqrt(fmax(h2, 0.0));
    if (hn == 0.0) return ni;
    ni.inv = 1.0 / hn;
    // max|v| <= (max|w'| + a correction of the size of |h2|) / h; 1.0625 is head room
    double mxv = row[K_MAX].x * ni.inv * 1.0625;
    ni.scale = fp16_scale ? (mxv > 0.0 ? 1.0 / mxv : 1.0) : 1.0;
    return ni;
}

// Restart normalisation: w'' = w' - sum_{i<nv_r} h2[r][i] V_i ; V[dst_r] = w''/h ;
// lp = scale * V[dst_r].
// Slots with active[r] == 0 write nothing.
template <int NV, typename SL>
__global__ __launch_bounds__(TPB) void k_update_normalize(const double2 *__restrict__ V, long vstride, int nvmax,
                                                          const int *__restrict__ nv_dev,
                                                          const int *__restrict__ dst_dev,
                                                          const double2 *__restrict__ res,
                                                          const double2 *__restrict__ w, double2 *__restrict__ Vout,
                                                          vec2_t<SL> *__restrict__ lp, double *__restrict__ scl,
                                                          const int *__restrict__ active, int fp16_scale,
                                                          int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    if (!active[r]) return;
    const int nv = slot_nv(nv_dev, nvmax, r);
    const int dst = dst_dev ? dst_dev[r] : nvmax;
    NormInfo ni = norm_info(res, nv, r, fp16_scale != 0);
    if (g == 0 && s == 0 && scl) scl[r] = ni.scale;
    C64 hc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hc[i] = i < nv ? ldc<double>(res + (long)r * KMAX + i) : mk(0.0, 0.0);
    double2 *vnext = Vout + dst * vstride;
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 wc = ldc<double>(w + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : (nv > 0 ? nv - 1 : 0);
                wc = wc - hc[i] * ldc_stream<double>(V + ii * vstride + base + c * BS);
            }
            C64 v = ni.inv * wc;
            stc_stream(vnext + base + c * BS, v);
            if (lp) stc(lp + base + c * BS, ni.scale * v);
        }
    }
}

// Lagged pass (A) of step j = nv_r - 1 (from 12 to 18 vectors the kernel is
// pinned to two waves per SIMD: left to itself the compiler picks a
// three-wave schedule for some of these sizes that keeps fewer loads in
// flight and runs up to 1.6x slower).  For i < j the partial sums of
// <V_i, w> (slot 2i) and <V_i, p> (slot 2i+1) with p = V[j]; <p, w> in slot
// 2j, |p|^2 in slot 2j+1, |w|^2 in K_NORM.  Inactive slots write nothing.
template <int NV>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(NV >= 12 && NV < 20 ? 2 : 1, NV >= 12 && NV < 20 ? 2 : 8))) void k_dots_lag(const double2 *__restrict__ V, long vstride,
                                                  const int *__restrict__ nv_dev, const double2 *__restrict__ w,
                                                  double2 *__restrict__ partial, const int *__restrict__ active,
                                                  int nblocks, int nrhs)
{
    __shared__ double red[4];
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    if (!active[r]) return;
    const int j = nv_dev[r] - 1;
    C64 sw[NV > 0 ? NV : 1], sp[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) sw[i] = sp[i] = mk(0.0, 0.0);
    C64 pw = mk(0.0, 0.0);
    double pp = 0.0, ww = 0.0;
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            const C64 wc = ldc<double>(w + base + c * BS);
            const C64 pc = ldc_stream<double>(V + j * vstride + base + c * BS);
            // unconditional loads keep every vector in flight; i >= j re-reads
            // a valid vector whose sums are never stored
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < j ? i : (j > 0 ? j - 1 : 0);
                const C64 v = ldc_stream<double>(V + ii * vstride + base + c * BS);
                cmacc(sw[i], v, wc);
                cmacc(sp[i], v, pc);
            }
            cmacc(pw, pc, wc);
            pp = fma(pc.re, pc.re, fma(pc.im, pc.im, pp));
            ww = fma(wc.re, wc.re, fma(wc.im, wc.im, ww));
        }
    }
    double2 *out = partial + ((long)g * nrhs + r) * KMAX;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < j) { // uniform over the workgroup
            const double a = wg_sum(sw[i].re, red), b = wg_sum(sw[i].im, red);
            const double c = wg_sum(sp[i].re, red), d = wg_sum(sp[i].im, red);
            if (s == 0) {
                out[2 * i] = make_double2(a, b);
                out[2 * i + 1] = make_double2(c, d);
            }
        }
    }
    const double a = wg_sum(pw.re, red), b = wg_sum(pw.im, red);
    const double tp = wg_sum(pp, red), tw = wg_sum(ww, red);
    if (s == 0) {
        out[2 * j] = make_double2(a, b);
        out[2 * j + 1] = make_double2(tp, 0.0);
        out[K_NORM] = make_double2(tw, 0.0);
    }
}

// Coefficients of the lagged update of slot r at step j from the reduced
// pass-A sums (the same arithmetic runs on the host for the Hessenberg matrix).
struct LagCoef {
    double inv_alpha; // 1/alpha (0 when p_j lies in span V[0..j-1])
    double inv_beta;  // 1/beta (0 on breakdown)
    C64 hjj;          // <v_j, w>
};
__device__ __forceinline__ LagCoef lag_coef(const double2 *row, int j)
{
    LagCoef L{1.0, 0.0, mk(row[2 * j].x, row[2 * j].y)};
    double w2 = row[K_NORM].x;
    if (j > 0) {
        double a2 = row[2 * j + 1].x;
        C64 cs = mk(0.0, 0.0); // c^+ s
        for (int i = 0; i < j; ++i) {
            const C64 c = mk(row[2 * i + 1].x, row[2 * i + 1].y), sv = mk(row[2 * i].x, row[2 * i].y);
            a2 -= c.re * c.re + c.im * c.im;
            cmacc(cs, c, sv);
            w2 -= sv.re * sv.re + sv.im * sv.im;
        }
        const double al = sqrt(fmax(a2, 0.0));
        L.inv_alpha = al > 0.0 ? 1.0 / al : 0.0;
        L.hjj = L.inv_alpha * (L.hjj - cs);
    }
    w2 -= L.hjj.re * L.hjj.re + L.hjj.im * L.hjj.im;
    const double be = sqrt(fmax(w2, 0.0));
    L.inv_beta = be > 0.0 ? 1.0 / be : 0.0;
    return L;
}

// Lagged pass (B) of step j: V[j] = v_j = (p_j - sum_{i<j} c_i V_i)/alpha
// (j > 0), V[j+1] = p_{j+1} = (w - sum_{i<j} s_i V_i - h_jj v_j)/beta, and
// lp = lsc * p_{j+1} in the smoother precision SL (lp == nullptr: none;
// scl[r] = lsc when scl is given).  With want_max, max|p_{j+1}| goes to
// partial slot K_MAX.  Inactive slots write nothing.
template <int NV, typename SL>
__global__ __launch_bounds__(TPB) void k_update_lag(double2 *__restrict__ V, long vstride,
                                                    const int *__restrict__ nv_dev, const double2 *__restrict__ res,
                                                    const double2 *__restrict__ w, vec2_t<SL> *__restrict__ lp,
                                                    double lsc, double *__restrict__ scl,
                                                    double2 *__restrict__ partial, int want_max,
                                                    const int *__restrict__ active, int nblocks, int nrhs)
{
    __shared__ double red[4];
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    if (!active[r]) return;
    if (scl && g == 0 && s == 0) scl[r] = lsc;
    const int j = nv_dev[r] - 1;
    const double2 *row = res + (long)r * KMAX;
    const LagCoef L = lag_coef(row, j);
    C64 cf[NV > 0 ? NV : 1], sf[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        cf[i] = i < j ? ldc<double>(row + 2 * i + 1) : mk(0.0, 0.0);
        sf[i] = i < j ? ldc<double>(row + 2 * i) : mk(0.0, 0.0);
    }
    double2 *vj = V + j * vstride;
    double2 *pn = V + (j + 1) * vstride;
    double mx = 0.0;
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 wc = ldc<double>(w + base + c * BS);
            C64 pc = ldc_stream<double>(vj + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < j ? i : (j > 0 ? j - 1 : 0); // cf[i] = sf[i] = 0 beyond j
                const C64 v = ldc_stream<double>(V + ii * vstride + base + c * BS);
                pc = pc - cf[i] * v;
                wc = wc - sf[i] * v;
            }
            const C64 v = L.inv_alpha * pc;
            if (j > 0) stc_stream(vj + base + c * BS, v);
            wc = wc - L.hjj * v;
            const C64 q = L.inv_beta * wc;
            stc_stream(pn + base + c * BS, q);
            if (lp) stc(lp + base + c * BS, lsc * q);
            mx = fmax(mx, fmax(fabs(q.re), fabs(q.im)));
        }
    }
    if (want_max) {
        const double tm = wg_max(mx, red);
        if (s == 0) partial[((long)g * nrhs + r) * KMAX + K_MAX] = make_double2(tm, 0.0);
    }
}

// Second stage of every reduction: out[r][k] = sum_g partial[g][r][k]
// (slot K_MAX takes the maximum); fixed order.
// The grid covers slots 0..nlead-1 and then K_NORM, K_MAX.
__global__ __launch_bounds__(TPB) void k_reduce(const double2 *__restrict__ partial, double2 *__restrict__ out, int G,
                                                int nrhs, int nlead)
{
    __shared__ double red[4];
    const int r = blockIdx.y, s = threadIdx.x;
    const int k = (int)blockIdx.x < nlead ? (int)blockIdx.x : K_NORM + ((int)blockIdx.x - nlead);
    const bool is_max = (k == K_MAX);
    double re = 0.0, im = 0.0;
    for (int g = s; g < G; g += TPB) {
        double2 v = partial[((long)g * nrhs + r) * KMAX + k];
        if (is_max) re = fmax(re, v.x);
        else {
            re += v.x;
            im += v.y;
        }
    }
    double tre = is_max ? wg_max(re, red) : wg_sum(re, red);
    double tim = is_max ? 0.0 : wg_sum(im, red);
    if (s == 0) out[(long)r * KMAX + k] = make_double2(tre, tim);
}

// x_r += sum_{i < len_r} y[r][i] Z_i  (Z in FP64 or FP32)
template <int NV, typename SZ>
__global__ __launch_bounds__(TPB) void k_combine(double2 *__restrict__ x, const vec2_t<SZ> *__restrict__ Z, long zstride,
                                                 int nvmax, const double2 *__restrict__ y, const int *__restrict__ len,
                                                 int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    const int nv = nvmax < len[r] ? nvmax : len[r];
    if (nv <= 0) return;
    C64 yc[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) yc[i] = i < nv ? ldc<double>(y + (long)r * ENGINE_MAXM + i) : mk(0.0, 0.0);
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            C64 xc = ldc<double>(x + base + c * BS);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int ii = i < nv ? i : nv - 1; // yc[i] = 0 beyond nv
                cmac(xc, yc[i], ldc_stream<double>(Z + ii * zstride + base + c * BS));
            }
            stc(x + base + c * BS, xc);
        }
    }
}

// FP16 smoother output -> FP32 basis vector: Z[off_r] = out / scale_r
// Test hook: an FP16 infinity in the first entry of every active slot's
// smoother output, as if FP16's range had been exceeded.
__global__ void k_poison_half(__half2 *__restrict__ p, const int *__restrict__ active, int nrhs)
{
    const int r = threadIdx.x;
    if (r < nrhs && active[r]) p[(long)r * 12 * BS] = __halves2half2(__ushort_as_half(0x7C00), __ushort_as_half(0x7C00));
}

__global__ __launch_bounds__(TPB) void k_unscale(const __half2 *__restrict__ in, float2 *__restrict__ Z,
                                                 const long *__restrict__ zoff, const double *__restrict__ scl,
                                                 const int *__restrict__ active, int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    if (!active[r]) return;
    const double sc = scl[r];
    const float f = sc != 0.0 ? (float)(1.0 / sc) : 0.0f;
    float2 *out = Z + zoff[r];
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) stc(out + base + c * BS, f * ldc<float>(in + base + c * BS));
    }
}

// out_r[out_off_r] = in_r[in_off_r] for active slots (identity preconditioner)
template <typename S>
__global__ __launch_bounds__(TPB) void k_slot_copy(const vec2_t<S> *__restrict__ in, const long *__restrict__ in_off,
                                                   vec2_t<S> *__restrict__ out, const long *__restrict__ out_off,
                                                   const int *__restrict__ active, int nblocks, int nrhs)
{
    const int g = blockIdx.x, G = gridDim.x, r = blockIdx.y, s = threadIdx.x;
    if (!active[r]) return;
    const vec2_t<S> *src = in + (in_off ? in_off[r] : 0);
    vec2_t<S> *dst = out + (out_off ? out_off[r] : 0);
    for (int b = g; b < nblocks; b += G) {
        const long base = ((long)b * nrhs + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) dst[base + c * BS] = src[base + c * BS];
    }
}

int pick_bucket(int nv)
{
    static const int b[] = {0, 1, 2, 3, 4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24, 28, 33};
    for (int v : b)
        if (nv <= v) return v;
    return 33;
}
#define DD_BUCKETS(X) X(0) X(1) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(28) X(33)

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

} // namespace

// per-slot arrays shared by host (pinned) and device, one upload per phase
struct SlotArrays {
    int active[ENGINE_MAXW];
    int nv[ENGINE_MAXW];
    int dst[ENGINE_MAXW];
    int len[ENGINE_MAXW];
    double m0[ENGINE_MAXW];
    long eta_off[ENGINE_MAXW];
    long psi_off[ENGINE_MAXW];
    long in_off[ENGINE_MAXW];
};

struct Engine::Impl {
    dd_ctx *ctx = nullptr;
    EngineParams P{};
    int W = 0;
    int zprec = DD_F32;
    int sap_prec = DD_F32;
    long vlen = 0; // complex entries of one width-wide vector
    int G = 0;
    DevBuf V, Z, w, xb, bb, lp, sapout, sapscr, partial, res, res2, resb, y, scl, slots;
    DevBuf xnz;           // per slot: the packed initial guess has a nonzero entry
    int *h_xnz = nullptr; // its host copy (pinned)
    std::unique_ptr<AmgWork, AmgWorkDeleter> amgw; // the two-grid preconditioner's workspace
    SlotArrays *h_slots[3] = {nullptr, nullptr, nullptr}; // ring of pinned staging buffers
    int ring = 0;
    double2 *h_res = nullptr, *h_resb = nullptr, *h_y = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<SlotState> S;
    std::map<int, hipGraphExec_t> graphs;
    bool restart_pending = false, step_pending = false, bnorm_pending = false;

    ~Impl()
    {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto p : h_slots)
            if (p) (void)hipHostFree(p);
        if (h_res) (void)hipHostFree(h_res);
        if (h_resb) (void)hipHostFree(h_resb);
        if (h_y) (void)hipHostFree(h_y);
        if (h_xnz) (void)hipHostFree(h_xnz);
        if (ev) (void)hipEventDestroy(ev);
    }

    hipStream_t st() const { return ctx->stream; }
    dim3 grid() const { return dim3(G, W); }
    SlotArrays *dev_slots() const { return slots.as<SlotArrays>(); }
    const int *d_active() const { return dev_slots()->active; }
    const int *d_nv() const { return dev_slots()->nv; }
    const int *d_dst() const { return dev_slots()->dst; }
    const int *d_len() const { return dev_slots()->len; }
    const double *d_m0() const { return dev_slots()->m0; }
    const long *d_eta_off() const { return dev_slots()->eta_off; }
    const long *d_psi_off() const { return dev_slots()->psi_off; }
    const long *d_in_off() const { return dev_slots()->in_off; }
    double vec64() const { return (double)vlen * 16.0; }

    SlotArrays &stage()
    {
        ring = (ring + 1) % 3;
        return *h_slots[ring];
    }
    Status upload(const SlotArrays &h)
    {
        DD_HIP_TRY(hipMemcpyAsync(slots.p, &h, sizeof(SlotArrays), hipMemcpyHostToDevice, st()));
        return Status::ok();
    }
    void fill_common(SlotArrays &h)
    {
        for (int r = 0; r < ENGINE_MAXW; ++r) {
            h.m0[r] = r < W ? S[r].m0 : 0.0;
            h.len[r] = 0;
        }
    }

    // ---- launch helpers -------------------------------------------------
    // lagged pass A over V[0..j] and w (nb >= every active slot's j)
    Status dots_lag(const double2 *wv, int nb)
    {
        ProfScope ps(ctx->prof, st(), K_CGS_DOTS, vec64() * (nb + 2), 16.0 * vlen * (nb + 1));
        switch (pick_bucket(nb)) {
#define C(N) case N: k_dots_lag<N><<<grid(), TPB, 0, st()>>>(V.as<double2>(), vlen, d_nv(), wv, partial.as<double2>(), d_active(), ctx->g.nblocks, W); break;
            DD_BUCKETS(C)
#undef C
        }
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }
    // lagged pass B: v_j over p_j, p_{j+1}, smoother-precision copy
    template <typename SL>
    Status update_lag_t(int nb, void *lpp, bool want_max, double lsc = 1.0, double *sclp = nullptr)
    {
        ProfScope ps(ctx->prof, st(), K_CGS_UPDATE,
                     vec64() * (nb + 4) + (lpp ? (double)vlen * 2 * sizeof(SL) : 0.0), 16.0 * vlen * (nb + 1));
        switch (pick_bucket(nb)) {
#define C(N) case N: k_update_lag<N, SL><<<grid(), TPB, 0, st()>>>(V.as<double2>(), vlen, d_nv(), res.as<double2>(), w.as<double2>(), static_cast<vec2_t<SL> *>(lpp), lsc, sclp, partial.as<double2>(), want_max ? 1 : 0, d_active(), ctx->g.nblocks, W); break;
            DD_BUCKETS(C)
#undef C
        }
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }
    Status update_lag(int nb)
    {
        if (sap_prec == DD_F64) return update_lag_t<double>(nb, nullptr, false);
        if (sap_prec == DD_F32) return update_lag_t<float>(nb, lp.p, false);
        // FP16: p_{j+1} has unit 2-norm up to rounding (beta is its norm), so
        // max|p_{j+1}| <= 1 and the fixed scale sqrt(24 V)/8 keeps the copy
        // inside FP16's range (at most 4.1e4 for 2^32 sites) while its RMS
        // entry, 1/8, sits far above the subnormals; the pass writes the
        // copy itself
        return update_lag_t<__half>(nb, lp.p, false, std::sqrt(24.0 * (double)ctx->g.V) / 8.0, scl.as<double>());
    }
    // nvmax == 0: plain |w|^2 and max|w| (no vectors, w untouched)
    Status update_dots(double2 *wv, int nvmax, const double2 *h)
    {
        ProfScope ps(ctx->prof, st(), K_CGS_NORMALIZE, vec64() * (nvmax + (nvmax > 0 ? 2 : 1)),
                     16.0 * vlen * nvmax + 4.0 * vlen);
        const int *nvp = nvmax > 0 ? d_nv() : nullptr;
        switch (pick_bucket(nvmax)) {
#define C(N) case N: k_update_dots<N><<<grid(), TPB, 0, st()>>>(V.as<double2>(), vlen, nvmax == 0 ? 0 : N, nvp, h, wv, partial.as<double2>(), ctx->g.nblocks, W); break;
            DD_BUCKETS(C)
#undef C
        }
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }
    template <typename SL> Status normalize_t(int nvmax, const double2 *r2, const double2 *wv, void *lpp, bool fp16)
    {
        ProfScope ps(ctx->prof, st(), K_CGS_NORMALIZE, vec64() * (nvmax + 2) + (lpp ? (double)vlen * 2 * sizeof(SL) : 0.0),
                     8.0 * vlen * (nvmax + 1));
        const int *nvp = nvmax > 0 ? d_nv() : nullptr;
        switch (pick_bucket(nvmax)) {
#define C(N) case N: k_update_normalize<N, SL><<<grid(), TPB, 0, st()>>>(V.as<double2>(), vlen, nvmax == 0 ? 0 : N, nvp, d_dst(), r2, wv, V.as<double2>(), static_cast<vec2_t<SL> *>(lpp), scl.as<double>(), d_active(), fp16 ? 1 : 0, ctx->g.nblocks, W); break;
            DD_BUCKETS(C)
#undef C
        }
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }
    Status normalize(int nvmax, const double2 *r2, const double2 *wv)
    {
        if (sap_prec == DD_F64) return normalize_t<double>(nvmax, r2, wv, nullptr, false);
        if (sap_prec == DD_F32) return normalize_t<float>(nvmax, r2, wv, lp.p, false);
        return normalize_t<__half>(nvmax, r2, wv, lp.p, true);
    }
    // slots 0..nlead-1, K_NORM and K_MAX
    Status reduce(double2 *out, int nlead)
    {
        ProfScope ps(ctx->prof, st(), K_REDUCE, (double)G * W * (nlead + 2) * 16.0, 0.0);
        k_reduce<<<dim3(nlead + 2, W), TPB, 0, st()>>>(partial.as<double2>(), out, G, W, nlead);
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }
    Status combine(int nvmax)
    {
        ProfScope ps(ctx->prof, st(), K_COMBINE, vec64() * 2 + (double)vlen * 2 * real_bytes(zprec) * nvmax,
                     8.0 * vlen * nvmax);
        const double2 *yp = y.as<double2>();
        if (zprec == DD_F64) {
            switch (pick_bucket(nvmax)) {
#define C(N) case N: k_combine<N, double><<<grid(), TPB, 0, st()>>>(xb.as<double2>(), Z.as<double2>(), vlen, nvmax, yp, d_len(), ctx->g.nblocks, W); break;
                DD_BUCKETS(C)
#undef C
            }
        } else {
            switch (pick_bucket(nvmax)) {
#define C(N) case N: k_combine<N, float><<<grid(), TPB, 0, st()>>>(xb.as<double2>(), Z.as<float2>(), vlen, nvmax, yp, d_len(), ctx->g.nblocks, W); break;
                DD_BUCKETS(C)
#undef C
            }
        }
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }

    // The fixed launch sequence of one Arnoldi step (captured into a graph);
    // nb >= the Arnoldi index j of every active slot.
    Status step_sequence(int nb)
    {
        SapSlots ss;
        ss.m0_dev = d_m0();
        ss.active = d_active(); // done or empty slots cost no smoother work
        ss.scratch = sapscr.p;
        if (P.amg) {
            // two-grid preconditioner: coarse correction, then post-smoothing
            if (sap_prec == DD_F64)
                DD_TRY(run_two_grid(ctx, *amgw, W, V.p, d_eta_off(), DD_F64, Z.p, d_psi_off(), d_m0(), d_active()));
            else
                DD_TRY(run_two_grid(ctx, *amgw, W, lp.p, nullptr, DD_F32, Z.p, d_psi_off(), d_m0(), d_active()));
        } else if (P.ncy == 0) {
            // no smoother: z_j = v_j (the smoother-precision copy, or V itself in FP64)
            ProfScope ps(ctx->prof, st(), K_CONVERT, (double)vlen * 2 * 2 * real_bytes(zprec), 0.0);
            if (sap_prec == DD_F64)
                k_slot_copy<double><<<grid(), TPB, 0, st()>>>(V.as<double2>(), d_eta_off(), Z.as<double2>(), d_psi_off(), d_active(), ctx->g.nblocks, W);
            else if (sap_prec == DD_F32)
                k_slot_copy<float><<<grid(), TPB, 0, st()>>>(lp.as<float2>(), nullptr, Z.as<float2>(), d_psi_off(), d_active(), ctx->g.nblocks, W);
            else
                k_unscale<<<grid(), TPB, 0, st()>>>(lp.as<__half2>(), Z.as<float2>(), d_psi_off(), scl.as<double>(), d_active(), ctx->g.nblocks, W);
            DD_HIP_TRY(hipGetLastError());
        } else if (sap_prec == DD_F64) {
            ss.eta_off = d_eta_off();
            ss.psi_off = d_psi_off();
            DD_TRY(run_sap(ctx, nullptr, W, V.p, Z.p, P.ncy, P.nmr, DD_F64, &ss, P.sap_eo));
        } else if (sap_prec == DD_F32) {
            ss.psi_off = d_psi_off();
            DD_TRY(run_sap(ctx, nullptr, W, lp.p, Z.p, P.ncy, P.nmr, DD_F32, &ss, P.sap_eo));
        } else {
            DD_TRY(run_sap(ctx, nullptr, W, lp.p, sapout.p, P.ncy, P.nmr, DD_F16, &ss, P.sap_eo));
            if (ctx->debug_poison_half != 0) {
                k_poison_half<<<1, 64, 0, st()>>>(sapout.as<__half2>(), d_active(), W);
                DD_HIP_TRY(hipGetLastError());
                if (ctx->debug_poison_half > 0) --ctx->debug_poison_half;
            }
            ProfScope ps(ctx->prof, st(), K_CONVERT, (double)vlen * 12.0, 2.0 * vlen);
            k_unscale<<<grid(), TPB, 0, st()>>>(sapout.as<__half2>(), Z.as<float2>(), d_psi_off(), scl.as<double>(),
                                                d_active(), ctx->g.nblocks, W);
            DD_HIP_TRY(hipGetLastError());
        }
        DD_TRY(launch_dslash(ctx, nullptr, W, Z.p, zprec, w.p, DD_F64, DD_F64, nullptr, d_m0(), d_in_off(), d_active()));
        DD_TRY(dots_lag(w.as<double2>(), nb));
        DD_TRY(reduce(res.as<double2>(), std::min(2 * nb + 2, K_NORM)));
        DD_TRY(update_lag(nb));
        return Status::ok();
    }
};

double SlotState::qr(int m, int n)
{
    // R = Q^+ H over the leading (n+1) x n block of the unrotated H; g = Q^+ beta0 e_1
    R = H;
    std::fill(g.begin(), g.end(), Z64(0.0));
    g[0] = beta0;
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < k; ++i) {
            Z64 a = R[(size_t)i * m + k], c = R[(size_t)(i + 1) * m + k];
            R[(size_t)i * m + k] = cs[i] * a + sn[i] * c;
            R[(size_t)(i + 1) * m + k] = -std::conj(sn[i]) * a + cs[i] * c;
        }
        Z64 rr;
        givens(R[(size_t)k * m + k], R[(size_t)(k + 1) * m + k], cs[k], sn[k], rr);
        R[(size_t)k * m + k] = rr;
        R[(size_t)(k + 1) * m + k] = 0.0;
        g[k + 1] = -std::conj(sn[k]) * g[k];
        g[k] = cs[k] * g[k];
    }
    return std::abs(g[n]);
}

bool SlotState::singular(int m, int n) const
{
    for (int k = 0; k < n; ++k)
        if (R[(size_t)k * m + k] == Z64(0.0)) return true;
    return false;
}

void SlotState::solve_y(int m, int n, std::complex<double> *y) const
{
    for (int i = 0; i < ENGINE_MAXM; ++i) y[i] = 0.0;
    for (int i = n - 1; i >= 0; --i) {
        Z64 acc = g[i];
        for (int k = i + 1; k < n; ++k) acc -= R[(size_t)i * m + k] * y[k];
        y[i] = acc / R[(size_t)i * m + i];
    }
}

Engine::Engine() : d(new Impl()) {}
Engine::~Engine()
{
    if (d && d->ctx) (void)hipStreamSynchronize(d->ctx->stream);
}

size_t Engine::bytes_per_slot(const GeomHost &g, int m, int sap_prec)
{
    size_t v = (size_t)g.V * 12 * 16; // one FP64 vector
    size_t zb = (size_t)g.V * 12 * 2 * real_bytes(sap_prec == DD_F64 ? DD_F64 : DD_F32);
    size_t lpb = sap_prec == DD_F64 ? 0 : (size_t)g.V * 12 * 2 * real_bytes(DD_F32);
    size_t so = sap_prec == DD_F16 ? (size_t)g.V * 12 * 4 : 0;
    // the smoother's scratch (face buffers, carried residual) takes two
    // vectors of Z's precision
    return v * (m + 1 + 3) + zb * (m + 2) + lpb + so;
}

int Engine::width() const { return d->W; }
const EngineParams &Engine::params() const { return d->P; }

Status Engine::prepare_amg()
{
    Impl &e = *d;
    if (!e.ctx->amg) return Status{DD_INVALID_ARG, "the two-grid preconditioner needs dd_amg_setup first"};
    if (e.P.sap_prec == DD_F16) return Status{DD_INVALID_ARG, "the two-grid preconditioner smooths in FP32 or FP64"};
    if (!e.amgw) e.amgw.reset(amg_work_new());
    return amg_reserve(e.ctx, *e.amgw, e.W, e.zprec, 0);
}
SlotState &Engine::slot(int r) { return d->S[r]; }
dd_ctx *Engine::ctx() const { return d->ctx; }

Status Engine::init(dd_ctx *ctx, const EngineParams &p)
{
    Impl &e = *d;
    if (p.width < 1 || p.width > ENGINE_MAXW || p.m < 1 || p.m > ENGINE_MAXM)
        return Status{DD_INVALID_ARG, "engine: width or Krylov dimension out of range"};
    e.ctx = ctx;
    e.P = p;
    e.W = p.width;
    e.sap_prec = p.sap_prec;
    e.zprec = p.sap_prec == DD_F64 ? DD_F64 : DD_F32;
    e.vlen = (long)ctx->g.nblocks * e.W * 12 * BS;
    e.G = ctx->g.nblocks < 1024 ? ctx->g.nblocks : 1024;
    const size_t v64 = (size_t)e.vlen * 16;
    DD_TRY(e.V.alloc(v64 * (p.m + 1)));
    DD_TRY(e.Z.alloc((size_t)e.vlen * 2 * real_bytes(e.zprec) * p.m));
    DD_TRY(e.w.alloc(v64));
    DD_TRY(e.xb.alloc(v64));
    DD_TRY(e.bb.alloc(v64));
    if (p.sap_prec != DD_F64) DD_TRY(e.lp.alloc((size_t)e.vlen * 2 * real_bytes(DD_F32))); // room for an FP32 fallback
    if (p.sap_prec == DD_F16) DD_TRY(e.sapout.alloc((size_t)e.vlen * 2 * real_bytes(DD_F16)));
    // smoother scratch, sized for FP32 so that an FP16 engine can fall back
    DD_TRY(e.sapscr.alloc(sap_scratch_bytes(ctx->g, e.zprec, e.W)));
    DD_TRY(e.partial.alloc((size_t)e.G * e.W * KMAX * 16));
    DD_TRY(e.res.alloc((size_t)e.W * KMAX * 16));
    DD_TRY(e.res2.alloc((size_t)e.W * KMAX * 16));
    DD_TRY(e.resb.alloc((size_t)e.W * KMAX * 16));
    DD_TRY(e.y.alloc((size_t)e.W * ENGINE_MAXM * 16));
    DD_TRY(e.scl.alloc((size_t)e.W * 8));
    DD_TRY(e.slots.alloc(sizeof(SlotArrays)));
    if (p.amg) DD_TRY(prepare_amg());
    for (auto &hs : e.h_slots) {
        DD_HIP_TRY(hipHostMalloc((void **)&hs, sizeof(SlotArrays), hipHostMallocDefault));
        std::memset(hs, 0, sizeof(SlotArrays));
    }
    DD_HIP_TRY(hipHostMalloc((void **)&e.h_res, (size_t)e.W * KMAX * 16, hipHostMallocDefault));
    DD_HIP_TRY(hipHostMalloc((void **)&e.h_resb, (size_t)e.W * KMAX * 16, hipHostMallocDefault));
    DD_HIP_TRY(hipHostMalloc((void **)&e.h_y, (size_t)e.W * ENGINE_MAXM * 16, hipHostMallocDefault));
    DD_TRY(e.xnz.alloc((size_t)e.W * sizeof(int)));
    DD_HIP_TRY(hipHostMalloc((void **)&e.h_xnz, (size_t)e.W * sizeof(int), hipHostMallocDefault));
    DD_HIP_TRY(hipEventCreateWithFlags(&e.ev, hipEventDisableTiming));
    e.S.assign(e.W, SlotState{});
    for (auto &s : e.S) {
        s.H.assign((size_t)(p.m + 1) * p.m, 0.0);
        s.R.assign((size_t)(p.m + 1) * p.m, 0.0);
        s.g.assign(p.m + 1, 0.0);
        s.sn.assign(p.m, 0.0);
        s.cs.assign(p.m, 0.0);
    }
    return Status::ok();
}

int Engine::free_slot() const
{
    for (int r = 0; r < d->W; ++r)
        if (d->S[r].state == SLOT_FREE) return r;
    return -1;
}

int Engine::busy_slots() const
{
    int n = 0;
    for (auto &s : d->S) n += s.state == SLOT_RESTART || s.state == SLOT_CYCLE;
    return n;
}

Status Engine::admit(int r, const double *b_canon, const double *x0_canon, double m0, long owner, int owner_rhs)
{
    Impl &e = *d;
    if (r < 0 || r >= e.W || e.S[r].state != SLOT_FREE) return Status{DD_INVALID_ARG, "engine: slot not free"};
    DD_TRY(pack_slot(e.ctx, e.st(), b_canon, e.bb.p, e.W, r));
    SlotState &s0 = e.S[r];
    if (x0_canon) {
        // the packing pass also finds whether x0 has a nonzero entry (the
        // flag is cleared first; admission is never inside a captured graph)
        int *flag = e.xnz.as<int>() + r;
        DD_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), e.st()));
        DD_TRY(pack_slot(e.ctx, e.st(), x0_canon, e.xb.p, e.W, r, flag));
        s0.x0_zero = false;
        s0.x0_check = true;
    } else {
        s0.x0_zero = true;
        s0.x0_check = false;
        // x0 = 0: clear slot r's chunk in every block (strided 2D clear,
        // never inside a captured graph)
        const size_t chunk = (size_t)12 * BS * 16;
        DD_HIP_TRY(hipMemset2DAsync(static_cast<char *>(e.xb.p) + (size_t)r * chunk, chunk * e.W, 0, chunk,
                                    e.ctx->g.nblocks, e.st()));
    }
    SlotState &s = e.S[r];
    s.state = SLOT_RESTART;
    s.need_bnorm = true;
    s.j = 0;
    s.m0 = m0;
    s.bnorm = 0;
    s.info = dd_solve_info{};
    s.info.status = DD_NOT_CONVERGED;
    s.owner = owner;
    s.owner_rhs = owner_rhs;
    return Status::ok();
}

Status Engine::extract(int r, double *x_canon)
{
    Impl &e = *d;
    if (r < 0 || r >= e.W) return Status{DD_INVALID_ARG, "engine: bad slot"};
    return unpack_slot(e.ctx, e.st(), e.xb.p, x_canon, e.W, r);
}

void Engine::release(int r)
{
    if (r >= 0 && r < d->W) d->S[r].state = SLOT_FREE;
}

// ---- restart phase ----------------------------------------------------------
Status Engine::launch_restart()
{
    Impl &e = *d;
    e.restart_pending = false;
    e.bnorm_pending = false;
    bool any = false, bn = false;
    for (auto &s : e.S) {
        any |= s.state == SLOT_RESTART;
        bn |= s.state == SLOT_RESTART && s.need_bnorm;
    }
    if (!any) return Status::ok();
    // whether freshly packed initial guesses were zero (one small copy and
    // a wait, on the first restart of a slot given an x0 only)
    bool check = false;
    for (auto &s : e.S) check |= s.state == SLOT_RESTART && s.x0_check;
    if (check) {
        DD_HIP_TRY(hipMemcpyAsync(e.h_xnz, e.xnz.p, (size_t)e.W * sizeof(int), hipMemcpyDeviceToHost, e.st()));
        DD_HIP_TRY(hipStreamSynchronize(e.st()));
        for (int r = 0; r < e.W; ++r)
            if (e.S[r].state == SLOT_RESTART && e.S[r].x0_check) {
                e.S[r].x0_zero = e.h_xnz[r] == 0;
                e.S[r].x0_check = false;
            }
    }
    bool from_zero = true;
    for (auto &s : e.S)
        if (s.state == SLOT_RESTART) from_zero &= s.need_bnorm && s.x0_zero;
    SlotArrays &h = e.stage();
    e.fill_common(h);
    for (int r = 0; r < ENGINE_MAXW; ++r) {
        const bool act = r < e.W && e.S[r].state == SLOT_RESTART;
        h.active[r] = act ? 1 : 0;
        h.nv[r] = 0;
        h.dst[r] = 0;
        h.eta_off[r] = h.psi_off[r] = h.in_off[r] = 0;
    }
    DD_TRY(e.upload(h));
    if (from_zero) {
        // every restarting slot starts from x0 = 0: r = b, so |r| = |b| and
        // v_0 = b/|b| without an operator application
        DD_TRY(e.update_dots(e.bb.as<double2>(), 0, nullptr));
        DD_TRY(e.reduce(e.res.as<double2>(), 0));
        DD_TRY(e.normalize(0, e.res.as<double2>(), e.bb.as<double2>()));
        DD_HIP_TRY(hipMemcpyAsync(e.h_res, e.res.p, (size_t)e.W * KMAX * 16, hipMemcpyDeviceToHost, e.st()));
        DD_HIP_TRY(hipMemcpyAsync(e.h_resb, e.res.p, (size_t)e.W * KMAX * 16, hipMemcpyDeviceToHost, e.st()));
        e.bnorm_pending = true;
        DD_HIP_TRY(hipEventRecord(e.ev, e.st()));
        e.restart_pending = true;
        return Status::ok();
    }
    if (bn) {
        // |b| of newly admitted slots
        DD_TRY(e.update_dots(e.bb.as<double2>(), 0, nullptr));
        DD_TRY(e.reduce(e.resb.as<double2>(), 0));
        DD_HIP_TRY(hipMemcpyAsync(e.h_resb, e.resb.p, (size_t)e.W * KMAX * 16, hipMemcpyDeviceToHost, e.st()));
        e.bnorm_pending = true;
    }
    // true residual r = b - D x (FP64) for every slot; |r|, max|r|; v_0 for restarting slots
    DD_TRY(launch_dslash(e.ctx, nullptr, e.W, e.xb.p, DD_F64, e.w.p, DD_F64, DD_F64, e.bb.as<double>(), e.d_m0()));
    DD_TRY(e.update_dots(e.w.as<double2>(), 0, nullptr));
    DD_TRY(e.reduce(e.res.as<double2>(), 0));
    DD_TRY(e.normalize(0, e.res.as<double2>(), e.w.as<double2>()));
    DD_HIP_TRY(hipMemcpyAsync(e.h_res, e.res.p, (size_t)e.W * KMAX * 16, hipMemcpyDeviceToHost, e.st()));
    DD_HIP_TRY(hipEventRecord(e.ev, e.st()));
    e.restart_pending = true;
    return Status::ok();
}

Status Engine::finish_restart()
{
    Impl &e = *d;
    if (!e.restart_pending) return Status::ok();
    e.restart_pending = false;
    DD_HIP_TRY(hipEventSynchronize(e.ev));
    for (int r = 0; r < e.W; ++r) {
        SlotState &s = e.S[r];
        if (s.state != SLOT_RESTART) continue;
        if (s.need_bnorm && e.bnorm_pending) {
            double n2 = e.h_resb[(size_t)r * KMAX + K_NORM].x;
            s.need_bnorm = false;
            s.bnorm = std::sqrt(n2);
            if (!std::isfinite(n2)) {
                s.state = SLOT_DONE;
                s.info.status = DD_NAN;
                s.info.rel_residual = n2;
                continue;
            }
        }
        const double beta = std::sqrt(e.h_res[(size_t)r * KMAX + K_NORM].x);
        if (!std::isfinite(beta)) {
            s.state = SLOT_DONE;
            s.info.status = DD_NAN;
            s.info.rel_residual = beta;
            continue;
        }
        s.info.rel_residual = s.bnorm > 0 ? beta / s.bnorm : 0.0;
        if (s.bnorm == 0.0 || beta / s.bnorm <= e.P.tol) {
            s.state = SLOT_DONE;
            s.info.status = DD_OK;
            continue;
        }
        if (s.info.restarts >= e.P.max_restarts) {
            s.state = SLOT_DONE;
            s.info.status = DD_NOT_CONVERGED;
            continue;
        }
        s.info.restarts++;
        s.beta0 = beta;
        s.beta_prev = 0.0;
        s.j = 0;
        s.state = SLOT_CYCLE;
    }
    return Status::ok();
}

// ---- Arnoldi step phase -------------------------------------------------------
Status Engine::launch_step()
{
    Impl &e = *d;
    e.step_pending = false;
    int jmax = -1;
    for (auto &s : e.S)
        if (s.state == SLOT_CYCLE) jmax = std::max(jmax, s.j);
    if (jmax < 0) return Status::ok();
    SlotArrays &h = e.stage();
    e.fill_common(h);
    for (int r = 0; r < ENGINE_MAXW; ++r) {
        const bool act = r < e.W && e.S[r].state == SLOT_CYCLE;
        const int j = act ? e.S[r].j : 0;
        h.active[r] = act ? 1 : 0;
        h.nv[r] = act ? j + 1 : 1;
        h.dst[r] = act ? j + 1 : 0;
        h.eta_off[r] = (e.sap_prec == DD_F64) ? (long)j * e.vlen : 0;
        h.psi_off[r] = (long)j * e.vlen;
        h.in_off[r] = (long)j * e.vlen;
    }
    DD_TRY(e.upload(h));
    const int bucket = pick_bucket(jmax);
    const bool use_graph = e.P.graphs && !e.ctx->prof.on && e.ctx->debug_poison_half == 0;
    if (use_graph) {
        // the kernels' arguments also depend on the link format
        const int key = ((bucket * 4 + e.sap_prec) * 2 + (e.ctx->link_r12 ? 1 : 0)) * 2 + (e.ctx->sap_half_fields ? 1 : 0);
        auto it = e.graphs.find(key);
        if (it == e.graphs.end()) {
            hipGraph_t g = nullptr;
            DD_HIP_TRY(hipStreamBeginCapture(e.st(), hipStreamCaptureModeThreadLocal));
            Status cs = e.step_sequence(bucket);
            hipError_t ce = hipStreamEndCapture(e.st(), &g);
            if (!cs.good()) {
                if (g) (void)hipGraphDestroy(g);
                return cs;
            }
            if (ce != hipSuccess) return Status{DD_HIP_ERROR, std::string("graph capture: ") + hipGetErrorString(ce)};
            hipGraphExec_t ex = nullptr;
            hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) return Status{DD_HIP_ERROR, std::string("graph instantiate: ") + hipGetErrorString(ie)};
            it = e.graphs.emplace(key, ex).first;
        }
        DD_HIP_TRY(hipGraphLaunch(it->second, e.st()));
    } else {
        DD_TRY(e.step_sequence(bucket));
    }
    DD_HIP_TRY(hipMemcpyAsync(e.h_res, e.res.p, (size_t)e.W * KMAX * 16, hipMemcpyDeviceToHost, e.st()));
    DD_HIP_TRY(hipEventRecord(e.ev, e.st()));
    e.step_pending = true;
    return Status::ok();
}

Status Engine::finish_step()
{
    Impl &e = *d;
    if (!e.step_pending) return Status::ok();
    e.step_pending = false;
    DD_HIP_TRY(hipEventSynchronize(e.ev));
    const int m = e.P.m;
    bool broken = false, any_end = false;
    int maxlen = 0;
    for (int r = 0; r < e.W; ++r) {
        SlotState &s = e.S[r];
        Z64 *yr = reinterpret_cast<Z64 *>(e.h_y + (size_t)r * ENGINE_MAXM);
        if (s.state != SLOT_CYCLE) continue;
        const int j = s.j;
        const double2 *row = e.h_res + (size_t)r * KMAX;
        auto sv = [&](int i) { return Z64(row[2 * i].x, row[2 * i].y); };
        auto cv = [&](int i) { return Z64(row[2 * i + 1].x, row[2 * i + 1].y); };
        // finish column j-1: p_j = V c + alpha v_j
        double alpha = 1.0, w2 = row[K_NORM].x;
        Z64 hjj = sv(j);
        bool ok_prev = true;
        if (j > 0) {
            double a2 = row[2 * j + 1].x;
            Z64 cs(0.0);
            for (int i = 0; i < j; ++i) {
                a2 -= std::norm(cv(i));
                cs += std::conj(cv(i)) * sv(i);
                w2 -= std::norm(sv(i));
            }
            ok_prev = std::isfinite(a2);
            alpha = std::sqrt(std::max(a2, 0.0));
            if (ok_prev) {
                for (int i = 0; i < j; ++i) s.H[(size_t)i * m + j - 1] += s.beta_prev * cv(i);
                s.H[(size_t)j * m + j - 1] = s.beta_prev * alpha;
            }
            hjj = alpha > 0.0 ? (hjj - cs) / alpha : Z64(0.0);
        }
        // column j as it stands
        for (int i = 0; i < j; ++i) s.H[(size_t)i * m + j] = sv(i);
        s.H[(size_t)j * m + j] = hjj;
        w2 -= std::norm(hjj);
        const bool ok_cur = std::isfinite(w2);
        const double beta = std::sqrt(std::max(w2, 0.0));
        s.H[(size_t)(j + 1) * m + j] = beta;
        s.beta_prev = beta;
        s.info.iterations++;
        s.info.sap_calls++;
        int ncols = j + 1;
        bool end = false;
        if (!ok_prev) { // cannot happen with finite data; drop both columns
            ncols = j - 1;
            broken = end = true;
        } else if (j > 0 && alpha == 0.0) { // p_j in span V: column j-1 ended the space
            ncols = j;
            end = true;
        } else if (!ok_cur) { // drop the broken column; the restart recomputes the true residual
            ncols = j;
            broken = end = true;
        }
        const double est = s.qr(m, ncols);
        if (beta == 0.0 || !(est / s.bnorm > e.P.tol) || ncols == m) end = true;
        s.j = ncols;
        if (end && s.singular(m, ncols)) {
            // the Krylov space closed (beta = 0, or p_j in the span of V) on a
            // singular projection of D: no correction from this space
            // minimises the residual uniquely, and restarting would rebuild
            // the same space.  Arnoldi breakdown without convergence; x keeps
            // the last iterate, rel_residual its true residual.
            s.state = SLOT_DONE;
            s.info.status = DD_BREAKDOWN;
            s.cycle_len = 0;
            continue;
        }
        if (end) {
            // end of this slot's cycle: y = R^-1 g, then x += Z y
            s.solve_y(m, ncols, yr);
            s.state = SLOT_RESTART;
            s.cycle_len = ncols;
            any_end = true;
            maxlen = std::max(maxlen, ncols);
        }
    }
    if (broken && e.sap_prec == DD_F16) {
        // FP16 range exceeded in the smoother: every slot restarts in FP32
        e.sap_prec = DD_F32;
        for (int r = 0; r < e.W; ++r) {
            SlotState &s = e.S[r];
            if (s.state != SLOT_CYCLE) continue;
            Z64 *yr = reinterpret_cast<Z64 *>(e.h_y + (size_t)r * ENGINE_MAXM);
            const int len = s.j;
            (void)s.qr(m, len);
            s.solve_y(m, len, yr);
            s.state = SLOT_RESTART;
            s.cycle_len = len;
            any_end = true;
            maxlen = std::max(maxlen, len);
        }
    }
    if (any_end && maxlen > 0) {
        SlotArrays &h = e.stage();
        e.fill_common(h);
        for (int r = 0; r < ENGINE_MAXW; ++r) {
            const bool ended = r < e.W && e.S[r].state == SLOT_RESTART && e.S[r].cycle_len > 0;
            h.len[r] = ended ? e.S[r].cycle_len : 0;
            h.active[r] = 0;
            h.nv[r] = 1;
            h.dst[r] = 0;
            h.eta_off[r] = h.psi_off[r] = h.in_off[r] = 0;
        }
        for (int r = 0; r < e.W; ++r) e.S[r].cycle_len = 0;
        DD_TRY(e.upload(h));
        DD_HIP_TRY(hipMemcpyAsync(e.y.p, e.h_y, (size_t)e.W * ENGINE_MAXM * 16, hipMemcpyHostToDevice, e.st()));
        DD_TRY(e.combine(maxlen));
    }
    return Status::ok();
}

Status Engine::iterate()
{
    {
        TraceRange tr("restart");
        DD_TRY(launch_restart());
        DD_TRY(finish_restart());
    }
    TraceRange tr("arnoldi_step");
    DD_TRY(launch_step());
    DD_TRY(finish_step());
    return Status::ok();
}

// ---------------------------------------------------------------------------
// dd_solve: every right-hand side admitted at once into one engine
// ---------------------------------------------------------------------------
Status solve(dd_ctx *ctx, const double *m0, const double *b, double *x, int nrhs, const dd_params &p,
             dd_solve_info *info_out)
{
    EngineParams ep;
    ep.width = nrhs;
    ep.m = p.m;
    ep.ncy = p.ncy;
    ep.nmr = p.nmr;
    ep.sap_prec = p.sap_prec;
    ep.sap_eo = p.sap_eo != 0;
    ep.tol = p.tol;
    ep.max_restarts = p.max_restarts;
    ep.graphs = false;
    // reuse the context's engine when the shape matches
    ep.amg = p.amg != 0;
    Engine *eng = ctx->engine.get();
    if (!eng || eng->width() != nrhs || eng->params().m != p.m || eng->params().sap_prec != p.sap_prec ||
        eng->params().amg != ep.amg) {
        ctx->engine.reset();
        std::unique_ptr<Engine, EngineDeleter> ne(new Engine());
        DD_TRY(ne->init(ctx, ep));
        ctx->engine = std::move(ne);
        eng = ctx->engine.get();
    } else {
        eng->set_params(ep);
    }
    if (ep.amg) DD_TRY(eng->prepare_amg()); // sizes follow the latest dd_amg_setup
    const size_t vstride = (size_t)ctx->g.V * 12 * 2; // doubles per canonical rhs
    for (int r = 0; r < nrhs; ++r) DD_TRY(eng->admit(r, b + r * vstride, x + r * vstride, m0[r], 0, r));
    for (int guard = 0; eng->busy_slots() > 0; ++guard) {
        if (guard > (p.max_restarts + 2) * (p.m + 2) + 8)
            return Status{DD_HIP_ERROR, "dd_solve: engine made no progress"};
        DD_TRY(eng->iterate());
    }
    Status out = Status::ok();
    for (int r = 0; r < nrhs; ++r) {
        DD_TRY(eng->extract(r, x + r * vstride));
        SlotState &s = eng->slot(r);
        if (info_out) info_out[r] = s.info;
        if (s.info.status != DD_OK && out.good())
            out = Status{(dd_status)s.info.status, "right-hand side " + std::to_string(r) + " did not converge"};
        eng->release(r);
    }
    DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
    return out;
}

void Engine::set_params(const EngineParams &p)
{
    // tolerance, restarts and the smoother's cycles and form may change between solves; the
    // shape (width, m, precision) may not
    d->P.tol = p.tol;
    d->P.max_restarts = p.max_restarts;
    d->P.ncy = p.ncy;
    d->P.nmr = p.nmr;
    d->P.sap_eo = p.sap_eo;
    d->P.graphs = p.graphs;
    for (auto &kv : d->graphs) (void)hipGraphExecDestroy(kv.second);
    d->graphs.clear();
    d->sap_prec = p.sap_prec;
}

void EngineDeleter::operator()(Engine *e) const { delete e; }

} // namespace dd
