// Field ingest (setup, once per resident gauge field): canonical -> blocked
// layout transforms for links, clover and spinors, precision conversion, and
// the clover term built on the device in FP64.
//
// Clover construction.  With F_munu = Q_munu - Q_munu^+ (Q the four-leaf
// clover of plaquettes at x; the (nu,mu) leaves are the adjoints of the
// (mu,nu) leaves) the term -(csw/32) sum_{mu,nu} g_mu g_nu (x) (Q_munu - Q_numu)
// equals -(csw/16) sum_{mu<nu} g_mu g_nu (x) F_munu.  In the chiral basis
// g_mu g_nu is block diagonal, so C splits into two 6x6 Hermitian halves:
//   half 0 (spins 0,1) = -i (csw/16) sum_m sigma_m (x) (B_m - E_m)
//   half 1 (spins 2,3) = -i (csw/16) sum_m sigma_m (x) (B_m + E_m)
// with B = (F_yz, F_zx, F_xy) and E_k = F_kt.  This is the form evaluated
// below; it is derived here from the gamma algebra, not taken from the CPU
// reference code.
#include <algorithm>
#include <vector>

#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

namespace {

constexpr int TPB = 256;
// largest deviation from SU(3) at which gauge compression is enabled: the
// rebuilt third row then differs from the stored one by about this much
constexpr double SU3_TOL = 1e-13;

struct CanonGeom {
    int L[4];
    int nb[4];
};

// canonical site index of (block b, block-local site s)
__device__ __forceinline__ long canon_site(const CanonGeom &g, int b, int s)
{
    int bc0 = b % g.nb[0];
    int t = b / g.nb[0];
    int bc1 = t % g.nb[1];
    t /= g.nb[1];
    int bc2 = t % g.nb[2];
    int bc3 = t / g.nb[2];
    int x = bc0 * 4 + (s & 3), y = bc1 * 4 + ((s >> 2) & 3), z = bc2 * 4 + ((s >> 4) & 3), w = bc3 * 4 + (s >> 6);
    return x + (long)g.L[0] * (y + (long)g.L[1] * (z + (long)g.L[2] * w));
}

__device__ __forceinline__ long shift_site(const CanonGeom &g, long site, int mu, int step)
{
    long stride = 1;
    for (int k = 0; k < mu; ++k) stride *= g.L[k];
    int c = (int)((site / stride) % g.L[mu]);
    int n = c + step;
    if (n >= g.L[mu]) n -= g.L[mu];
    if (n < 0) n += g.L[mu];
    return site + (long)(n - c) * stride;
}

typedef cx<double> C64;

__device__ __forceinline__ void load_link(const double2 *U, long site, int mu, C64 out[9])
{
    const double2 *p = U + (site * 4 + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) out[e] = ldc<double>(p + e);
}

// c = a^(da) * b^(db)
__device__ __forceinline__ void mm(const C64 *a, bool da, const C64 *b, bool db, C64 *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            C64 acc = mk(0.0, 0.0);
            for (int k = 0; k < 3; ++k) {
                C64 x = da ? conjx(a[k * 3 + i]) : a[i * 3 + k];
                C64 y = db ? conjx(b[j * 3 + k]) : b[k * 3 + j];
                acc = acc + x * y;
            }
            c[i * 3 + j] = acc;
        }
}

// acc += a^(da) b^(db) c^(dc) d^(dd)
__device__ void add_leaf(const C64 *a, bool da, const C64 *b, bool db, const C64 *c, bool dc, const C64 *d, bool dd,
                         C64 *acc)
{
    C64 t1[9], t2[9], t3[9];
    mm(a, da, b, db, t1);
    mm(t1, false, c, dc, t2);
    mm(t2, false, d, dd, t3);
    for (int i = 0; i < 9; ++i) acc[i] = acc[i] + t3[i];
}

// F = Q_munu - Q_munu^+ at site x
__device__ void field_strength(const CanonGeom &g, const double2 *U, long x, int mu, int nu, C64 F[9])
{
    long xpm = shift_site(g, x, mu, 1), xpn = shift_site(g, x, nu, 1);
    long xmm = shift_site(g, x, mu, -1), xmn = shift_site(g, x, nu, -1);
    long xmm_pn = shift_site(g, xmm, nu, 1), xmm_mn = shift_site(g, xmm, nu, -1), xmn_pm = shift_site(g, xmn, mu, 1);
    C64 Q[9];
    for (int i = 0; i < 9; ++i) Q[i] = mk(0.0, 0.0);
    C64 a[9], b[9], c[9], d[9];
    // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    load_link(U, x, mu, a); load_link(U, xpm, nu, b); load_link(U, xpn, mu, c); load_link(U, x, nu, d);
    add_leaf(a, false, b, false, c, true, d, true, Q);
    // U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    load_link(U, x, nu, a); load_link(U, xmm_pn, mu, b); load_link(U, xmm, nu, c); load_link(U, xmm, mu, d);
    add_leaf(a, false, b, true, c, true, d, false, Q);
    // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    load_link(U, xmm, mu, a); load_link(U, xmm_mn, nu, b); load_link(U, xmm_mn, mu, c); load_link(U, xmn, nu, d);
    add_leaf(a, true, b, true, c, false, d, false, Q);
    // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    load_link(U, xmn, nu, a); load_link(U, xmn, mu, b); load_link(U, xmn_pm, nu, c); load_link(U, x, mu, d);
    add_leaf(a, true, b, false, c, false, d, true, Q);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i * 3 + j] = Q[i * 3 + j] - conjx(Q[j * 3 + i]);
}

__global__ __launch_bounds__(TPB) void k_clover_build(const double2 *__restrict__ U, double2 *__restrict__ out,
                                                      CanonGeom g, double csw, int nblocks)
{
    int b = blockIdx.x;
    int s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    // F for the six planes
    C64 Fxy[9], Fxz[9], Fyz[9], Fxt[9], Fyt[9], Fzt[9];
    field_strength(g, U, x, 0, 1, Fxy);
    field_strength(g, U, x, 0, 2, Fxz);
    field_strength(g, U, x, 1, 2, Fyz);
    field_strength(g, U, x, 0, 3, Fxt);
    field_strength(g, U, x, 1, 3, Fyt);
    field_strength(g, U, x, 2, 3, Fzt);
    const double k = csw / 16.0;
    for (int half = 0; half < 2; ++half) {
        double sg = half == 0 ? -1.0 : 1.0; // X_m = B_m - E_m (half 0), B_m + E_m (half 1)
        C64 Xx[9], Xy[9], Xz[9];
        for (int i = 0; i < 9; ++i) {
            Xx[i] = Fyz[i] + sg * Fxt[i];
            Xy[i] = (-1.0) * Fxz[i] + sg * Fyt[i];
            Xz[i] = Fxy[i] + sg * Fzt[i];
        }
        // M = -i k [[Xz, Xx - i Xy], [Xx + i Xy, -Xz]]
        C64 M[36];
        for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) {
                int e = a * 3 + bb;
                C64 m00 = Xz[e], m01 = Xx[e] - ti(Xy[e]), m10 = Xx[e] + ti(Xy[e]), m11 = (-1.0) * Xz[e];
                M[(0 + a) * 6 + 0 + bb] = k * tmi(m00);
                M[(0 + a) * 6 + 3 + bb] = k * tmi(m01);
                M[(3 + a) * 6 + 0 + bb] = k * tmi(m10);
                M[(3 + a) * 6 + 3 + bb] = k * tmi(m11);
            }
        double2 *o = out + ((long)b * 36 + half * 18) * BS + s;
        for (int p = 0; p < 3; ++p) o[(long)p * BS] = make_double2(M[(2 * p) * 7].re, M[(2 * p + 1) * 7].re);
        int e = 3;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                o[(long)e * BS] = make_double2(M[i * 6 + j].re, M[i * 6 + j].im);
                ++e;
            }
    }
}

// canonical C[s][k][i][j] (full Hermitian halves) -> packed blocked FP64
__global__ __launch_bounds__(TPB) void k_clover_pack(const double2 *__restrict__ C, double2 *__restrict__ out,
                                                     CanonGeom g, int nblocks)
{
    int b = blockIdx.x, s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    for (int half = 0; half < 2; ++half) {
        const double2 *c = C + (x * 2 + half) * 36;
        double2 *o = out + ((long)b * 36 + half * 18) * BS + s;
        for (int p = 0; p < 3; ++p) o[(long)p * BS] = make_double2(c[(2 * p) * 7].x, c[(2 * p + 1) * 7].x);
        int e = 3;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                o[(long)e * BS] = c[i * 6 + j];
                ++e;
            }
    }
}

template <typename S>
__global__ __launch_bounds__(TPB) void k_links_pack(const double2 *__restrict__ U, vec2_t<S> *__restrict__ out,
                                                    CanonGeom g, int nblocks)
{
    int b = blockIdx.x, s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    for (int mu = 0; mu < 4; ++mu)
        for (int e = 0; e < 9; ++e) stc(out + (((long)b * 4 + mu) * 9 + e) * BS + s, ldc<double>(U + (x * 4 + mu) * 9 + e));
}

// Largest deviation of a link from SU(3) in each block: max over the block's
// sites and directions of max_ij |(U U^+ - 1)_ij| and |det U - 1| (FP64).
__global__ __launch_bounds__(TPB) void k_su3_deviation(const double2 *__restrict__ U, double *__restrict__ out,
                                                       CanonGeom g, int nblocks)
{
    __shared__ double red[TPB / 64];
    const int b = blockIdx.x, s = threadIdx.x;
    if (b >= nblocks) return; // uniform over the workgroup
    const long x = canon_site(g, b, s);
    double dev = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
        cx<double> u[9];
        for (int e = 0; e < 9; ++e) u[e] = ldc<double>(U + (x * 4 + mu) * 9 + e);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                cx<double> m = mk(i == j ? -1.0 : 0.0, 0.0);
                for (int k = 0; k < 3; ++k) cmacc(m, u[j * 3 + k], u[i * 3 + k]); // += u_ik conj(u_jk)
                dev = fmax(dev, fmax(fabs(m.re), fabs(m.im)));
            }
        const cx<double> det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                               u[2] * (u[3] * u[7] - u[4] * u[6]);
        dev = fmax(dev, hypot(det.re - 1.0, det.im));
    }
    for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
    if ((s & 63) == 0) red[s >> 6] = dev;
    __syncthreads();
    if (s == 0) {
        double m = red[0];
        for (int w = 1; w < TPB / 64; ++w) m = fmax(m, red[w]);
        out[b] = isfinite(m) ? m : 1e300;
    }
}

// elementwise complex conversion FP64 -> S (round to nearest even)
template <typename S>
__global__ __launch_bounds__(TPB) void k_convert_from64(const double2 *__restrict__ in, vec2_t<S> *__restrict__ out,
                                                        long n)
{
    long i = (long)blockIdx.x * TPB + threadIdx.x;
    if (i < n) stc(out + i, ldc<double>(in + i));
}

// canonical spinors [rhs][site][12] (FP64) <-> blocked (precision S)
template <typename S>
__global__ __launch_bounds__(TPB) void k_spinor_pack(const double2 *__restrict__ in, vec2_t<S> *__restrict__ out,
                                                     CanonGeom g, int nblocks, int nrhs, long V)
{
    int b = blockIdx.x / nrhs, r = blockIdx.x % nrhs, s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    const double2 *src = in + ((long)r * V + x) * 12;
    vec2_t<S> *dst = out + ((long)b * nrhs + r) * 12 * BS + s;
    for (int c = 0; c < 12; ++c) stc(dst + (long)c * BS, ldc<double>(src + c));
}

template <typename S>
__global__ __launch_bounds__(TPB) void k_spinor_unpack(const vec2_t<S> *__restrict__ in, double2 *__restrict__ out,
                                                       CanonGeom g, int nblocks, int nrhs, long V)
{
    int b = blockIdx.x / nrhs, r = blockIdx.x % nrhs, s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    const vec2_t<S> *src = in + ((long)b * nrhs + r) * 12 * BS + s;
    double2 *dst = out + ((long)r * V + x) * 12;
    for (int c = 0; c < 12; ++c) stc(dst + c, ldc<double>(src + (long)c * BS));
}

// one canonical FP64 right-hand side <-> slot `slot` of a width-wide blocked buffer
__global__ __launch_bounds__(TPB) void k_slot_pack(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                   CanonGeom g, int nblocks, int width, int slot,
                                                   int *__restrict__ nonzero)
{
    int b = blockIdx.x, s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    double2 *dst = out + ((long)b * width + slot) * 12 * BS + s;
    bool nz = false;
    for (int c = 0; c < 12; ++c) {
        const double2 v = in[x * 12 + c];
        nz |= v.x != 0.0 || v.y != 0.0; // NaN counts as nonzero
        dst[(long)c * BS] = v;
    }
    if (nonzero && __any(nz) && (threadIdx.x % 64) == 0) atomicOr(nonzero, 1);
}
__global__ __launch_bounds__(TPB) void k_slot_unpack(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                     CanonGeom g, int nblocks, int width, int slot)
{
    int b = blockIdx.x, s = threadIdx.x;
    if (b >= nblocks) return;
    long x = canon_site(g, b, s);
    const double2 *src = in + ((long)b * width + slot) * 12 * BS + s;
    for (int c = 0; c < 12; ++c) out[x * 12 + c] = src[(long)c * BS];
}

__global__ __launch_bounds__(TPB) void k_nonfinite(const double *__restrict__ p, long n, int *flag)
{
    long i = (long)blockIdx.x * TPB + threadIdx.x;
    long stride = (long)gridDim.x * TPB;
    int bad = 0;
    for (; i < n; i += stride) bad |= !isfinite(p[i]);
    if (__any(bad) && (threadIdx.x % 64) == 0) atomicOr(flag, 1);
}

CanonGeom canon_geom(const GeomHost &g)
{
    CanonGeom c;
    for (int i = 0; i < 4; ++i) {
        c.L[i] = g.L[i];
        c.nb[i] = g.nb[i];
    }
    return c;
}

Status convert_field(hipStream_t st, const double2 *src, void *dst, int prec, long ncomplex)
{
    int grid = (int)((ncomplex + TPB - 1) / TPB);
    if (prec == DD_F32)
        k_convert_from64<float><<<grid, TPB, 0, st>>>(src, static_cast<float2 *>(dst), ncomplex);
    else
        k_convert_from64<__half><<<grid, TPB, 0, st>>>(src, static_cast<__half2 *>(dst), ncomplex);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace

Status build_fields(dd_ctx *ctx, const double *U_dev, double csw)
{
    const GeomHost &g = ctx->g;
    CanonGeom cg = canon_geom(g);
    long nl = (long)g.nblocks * 4 * 9 * BS; // complex entries of the link field
    long nc = (long)g.nblocks * 36 * BS;    // complex slots of the clover field
    for (int p = 0; p < 3; ++p) {
        DD_TRY(ctx->links[p].alloc(nl * 2 * real_bytes(p)));
        DD_TRY(ctx->clover[p].alloc(nc * 2 * real_bytes(p)));
    }
    const double2 *U = reinterpret_cast<const double2 *>(U_dev);
    k_links_pack<double><<<g.nblocks, TPB, 0, ctx->stream>>>(U, ctx->links[DD_F64].as<double2>(), cg, g.nblocks);
    k_links_pack<float><<<g.nblocks, TPB, 0, ctx->stream>>>(U, ctx->links[DD_F32].as<float2>(), cg, g.nblocks);
    k_links_pack<__half><<<g.nblocks, TPB, 0, ctx->stream>>>(U, ctx->links[DD_F16].as<__half2>(), cg, g.nblocks);
    DD_HIP_TRY(hipGetLastError());
    k_clover_build<<<g.nblocks, TPB, 0, ctx->stream>>>(U, ctx->clover[DD_F64].as<double2>(), cg, csw, g.nblocks);
    DD_HIP_TRY(hipGetLastError());
    DD_TRY(convert_field(ctx->stream, ctx->clover[DD_F64].as<double2>(), ctx->clover[DD_F32].p, DD_F32, nc));
    DD_TRY(convert_field(ctx->stream, ctx->clover[DD_F64].as<double2>(), ctx->clover[DD_F16].p, DD_F16, nc));
    // gauge compression applies when every link is SU(3) to FP64 rounding
    DevBuf dev;
    DD_TRY(dev.alloc((size_t)g.nblocks * sizeof(double)));
    k_su3_deviation<<<g.nblocks, TPB, 0, ctx->stream>>>(U, dev.as<double>(), cg, g.nblocks);
    DD_HIP_TRY(hipGetLastError());
    std::vector<double> hdev(g.nblocks);
    DD_HIP_TRY(hipMemcpyAsync(hdev.data(), dev.p, hdev.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
    double worst = 0.0;
    for (double d : hdev) worst = std::max(worst, d);
    ctx->link_su3 = worst <= SU3_TOL;
    ctx->link_r12 = ctx->link_su3;
    return Status::ok();
}

Status set_clover_canon(dd_ctx *ctx, const double *C_dev)
{
    const GeomHost &g = ctx->g;
    long nc = (long)g.nblocks * 36 * BS;
    k_clover_pack<<<g.nblocks, TPB, 0, ctx->stream>>>(reinterpret_cast<const double2 *>(C_dev),
                                                      ctx->clover[DD_F64].as<double2>(), canon_geom(g), g.nblocks);
    DD_HIP_TRY(hipGetLastError());
    DD_TRY(convert_field(ctx->stream, ctx->clover[DD_F64].as<double2>(), ctx->clover[DD_F32].p, DD_F32, nc));
    DD_TRY(convert_field(ctx->stream, ctx->clover[DD_F64].as<double2>(), ctx->clover[DD_F16].p, DD_F16, nc));
    return Status::ok();
}

Status pack_spinor(dd_ctx *ctx, const double *canon, void *blocked, int prec, int nrhs)
{
    const GeomHost &g = ctx->g;
    ProfScope ps(ctx->prof, ctx->stream, K_PACK, (double)g.V * nrhs * 24.0 * (8 + real_bytes(prec)), 0.0);
    CanonGeom cg = canon_geom(g);
    int grid = g.nblocks * nrhs;
    const double2 *in = reinterpret_cast<const double2 *>(canon);
    if (prec == DD_F64)
        k_spinor_pack<double><<<grid, TPB, 0, ctx->stream>>>(in, static_cast<double2 *>(blocked), cg, g.nblocks, nrhs, g.V);
    else if (prec == DD_F32)
        k_spinor_pack<float><<<grid, TPB, 0, ctx->stream>>>(in, static_cast<float2 *>(blocked), cg, g.nblocks, nrhs, g.V);
    else
        k_spinor_pack<__half><<<grid, TPB, 0, ctx->stream>>>(in, static_cast<__half2 *>(blocked), cg, g.nblocks, nrhs, g.V);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status unpack_spinor(dd_ctx *ctx, const void *blocked, double *canon, int prec, int nrhs)
{
    const GeomHost &g = ctx->g;
    ProfScope ps(ctx->prof, ctx->stream, K_PACK, (double)g.V * nrhs * 24.0 * (8 + real_bytes(prec)), 0.0);
    CanonGeom cg = canon_geom(g);
    int grid = g.nblocks * nrhs;
    double2 *out = reinterpret_cast<double2 *>(canon);
    if (prec == DD_F64)
        k_spinor_unpack<double><<<grid, TPB, 0, ctx->stream>>>(static_cast<const double2 *>(blocked), out, cg, g.nblocks, nrhs, g.V);
    else if (prec == DD_F32)
        k_spinor_unpack<float><<<grid, TPB, 0, ctx->stream>>>(static_cast<const float2 *>(blocked), out, cg, g.nblocks, nrhs, g.V);
    else
        k_spinor_unpack<__half><<<grid, TPB, 0, ctx->stream>>>(static_cast<const __half2 *>(blocked), out, cg, g.nblocks, nrhs, g.V);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status pack_slot(dd_ctx *ctx, hipStream_t st, const double *canon, void *blocked, int width, int slot, int *nonzero)
{
    const GeomHost &g = ctx->g;
    ProfScope ps(ctx->prof, st, K_PACK, (double)g.V * 24.0 * 16, 0.0);
    k_slot_pack<<<g.nblocks, TPB, 0, st>>>(reinterpret_cast<const double2 *>(canon), static_cast<double2 *>(blocked),
                                           canon_geom(g), g.nblocks, width, slot, nonzero);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status unpack_slot(dd_ctx *ctx, hipStream_t st, const void *blocked, double *canon, int width, int slot)
{
    const GeomHost &g = ctx->g;
    ProfScope ps(ctx->prof, st, K_PACK, (double)g.V * 24.0 * 16, 0.0);
    k_slot_unpack<<<g.nblocks, TPB, 0, st>>>(static_cast<const double2 *>(blocked), reinterpret_cast<double2 *>(canon),
                                             canon_geom(g), g.nblocks, width, slot);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

Status any_nonfinite(dd_ctx *ctx, const double *p, size_t n, bool &bad)
{
    DevBuf flag;
    DD_TRY(flag.alloc(sizeof(int)));
    DD_HIP_TRY(hipMemsetAsync(flag.p, 0, sizeof(int), ctx->stream));
    long blocks = (long)((n + TPB - 1) / TPB);
    int grid = (int)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
    k_nonfinite<<<grid, TPB, 0, ctx->stream>>>(p, (long)n, flag.as<int>());
    DD_HIP_TRY(hipGetLastError());
    int h = 0;
    DD_HIP_TRY(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
    bad = h != 0;
    return Status::ok();
}

} // namespace dd
