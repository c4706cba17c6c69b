// Device-side building blocks shared by the HIP kernels of libddsap:
// complex arithmetic, precision-generic loads/stores, the chiral-basis spin
// projectors, SU(3) and clover matrix-vector products, and the blocked
// lattice geometry.
//
// Blocked layout (all precisions, complex numbers stored as (re, im) pairs):
//   Schwarz block b (4x4x4x4 sites), block-local site s = lx + 4 ly + 16 lz + 64 lt
//   spinor : ((b*nrhs + r)*12 + c)*256 + s          c = spin*3 + colour
//   links  : ((b*4 + mu)*9 + row*3 + col)*256 + s   U_mu(x)
//   clover : (b*36 + e)*256 + s                     e < 18: chiral half 0, else half 1;
//            per half: slots 0-2 hold the six real diagonal entries in pairs,
//            slots 3-17 the upper triangle (0,1),(0,2),..,(4,5) row by row.
// Site-innermost storage makes every component load of a 64-lane wavefront
// one contiguous segment.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

constexpr int BS = 256;   // sites per Schwarz block
constexpr int BEXT = 4;   // block extent per direction
constexpr int MAXRHS = 16;

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename A>
struct alignas(2 * sizeof(A)) cx {
    A re, im;
};

template <typename A> __device__ __forceinline__ cx<A> mk(A r, A i) { return {r, i}; }
template <typename A> __device__ __forceinline__ cx<A> operator+(cx<A> a, cx<A> b) { return {a.re + b.re, a.im + b.im}; }
template <typename A> __device__ __forceinline__ cx<A> operator-(cx<A> a, cx<A> b) { return {a.re - b.re, a.im - b.im}; }
template <typename A> __device__ __forceinline__ cx<A> operator*(cx<A> a, cx<A> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename A> __device__ __forceinline__ cx<A> operator*(A s, cx<A> a) { return {s * a.re, s * a.im}; }
template <typename A> __device__ __forceinline__ cx<A> conjx(cx<A> a) { return {a.re, -a.im}; }
// i*a and -i*a
template <typename A> __device__ __forceinline__ cx<A> ti(cx<A> a) { return {-a.im, a.re}; }
template <typename A> __device__ __forceinline__ cx<A> tmi(cx<A> a) { return {a.im, -a.re}; }
// acc += a*b ; acc += conj(a)*b
template <typename A> __device__ __forceinline__ void cmac(cx<A> &acc, cx<A> a, cx<A> b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
template <typename A> __device__ __forceinline__ void cmacc(cx<A> &acc, cx<A> a, cx<A> b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

// ---------------------------------------------------------------------------
// storage types: a complex number is one 2-vector of the storage scalar
// ---------------------------------------------------------------------------
template <typename S> struct st2;
template <> struct st2<double> { using T = double2; };
template <> struct st2<float> { using T = float2; };
template <> struct st2<__half> { using T = __half2; };
template <typename S> using vec2_t = typename st2<S>::T;

template <typename A> __device__ __forceinline__ cx<A> ldc(const double2 *p)
{
    double2 v = *p;
    return {(A)v.x, (A)v.y};
}
template <typename A> __device__ __forceinline__ cx<A> ldc(const float2 *p)
{
    float2 v = *p;
    return {(A)v.x, (A)v.y};
}
template <typename A> __device__ __forceinline__ cx<A> ldc(const __half2 *p)
{
    float2 v = __half22float2(*p);
    return {(A)v.x, (A)v.y};
}
template <typename A> __device__ __forceinline__ void stc(double2 *p, cx<A> a) { *p = make_double2((double)a.re, (double)a.im); }
template <typename A> __device__ __forceinline__ void stc(float2 *p, cx<A> a) { *p = make_float2((float)a.re, (float)a.im); }
// round to nearest even (hardware conversion)
template <typename A> __device__ __forceinline__ void stc(__half2 *p, cx<A> a)
{
    *p = __floats2half2_rn((float)a.re, (float)a.im);
}

// Streaming (nontemporal) forms for data touched once per launch (clover
// terms, outputs): they keep the L2 for the spinor neighbours that are reused.
template <typename T> __device__ __forceinline__ T ld_stream(const T *p)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    T t;
    if constexpr (sizeof(T) == 4) {
        unsigned v = __builtin_nontemporal_load(reinterpret_cast<const unsigned *>(p));
        __builtin_memcpy(&t, &v, 4);
    } else if constexpr (sizeof(T) == 8) {
        u2 v = __builtin_nontemporal_load(reinterpret_cast<const u2 *>(p));
        __builtin_memcpy(&t, &v, 8);
    } else {
        static_assert(sizeof(T) == 16, "2-vector storage of 4, 8 or 16 bytes");
        u4 v = __builtin_nontemporal_load(reinterpret_cast<const u4 *>(p));
        __builtin_memcpy(&t, &v, 16);
    }
    return t;
}
template <typename T> __device__ __forceinline__ void st_stream(T *p, T t)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) {
        unsigned v;
        __builtin_memcpy(&v, &t, 4);
        __builtin_nontemporal_store(v, reinterpret_cast<unsigned *>(p));
    } else if constexpr (sizeof(T) == 8) {
        u2 v;
        __builtin_memcpy(&v, &t, 8);
        __builtin_nontemporal_store(v, reinterpret_cast<u2 *>(p));
    } else {
        static_assert(sizeof(T) == 16, "2-vector storage of 4, 8 or 16 bytes");
        u4 v;
        __builtin_memcpy(&v, &t, 16);
        __builtin_nontemporal_store(v, reinterpret_cast<u4 *>(p));
    }
}
template <typename A, typename T> __device__ __forceinline__ cx<A> ldc_stream(const T *p)
{
    T v = ld_stream(p);
    return ldc<A>(&v);
}
template <typename A, typename T> __device__ __forceinline__ void stc_stream(T *p, cx<A> a)
{
    T v;
    stc(&v, a);
    st_stream(p, v);
}

// ---------------------------------------------------------------------------
// Links.  One link is nine complex entries U[3 row + col], BS apart in the
// blocked layout.  With r12 (gauge compression, "reconstruct-12") only the
// first two rows are read and the third is the complex conjugate of their
// cross product, which is exact for SU(3) matrices (orthonormal rows,
// determinant 1); the context enables it only for fields that are SU(3) to
// FP64 rounding.
template <typename A> __device__ __forceinline__ void su3_third_row(cx<A> U[9])
{
    U[6] = conjx(U[1] * U[5] - U[2] * U[4]);
    U[7] = conjx(U[2] * U[3] - U[0] * U[5]);
    U[8] = conjx(U[0] * U[4] - U[1] * U[3]);
}
// The four links of a site (u: entry 0 of link mu = 0; links mu are 9 BS
// apart), times k: all loads are issued before any third row is rebuilt, so
// they are in flight together.
template <typename A, bool NT = false, typename T>
__device__ __forceinline__ void load_links4(const T *u, bool r12, A k, cx<A> U[4][9])
{
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int e = 0; e < 6; ++e)
            U[mu][e] = NT ? ldc_stream<A>(u + (mu * 9 + e) * BS) : ldc<A>(u + (mu * 9 + e) * BS);
    if (r12) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) su3_third_row(U[mu]);
    } else {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int e = 6; e < 9; ++e)
                U[mu][e] = NT ? ldc_stream<A>(u + (mu * 9 + e) * BS) : ldc<A>(u + (mu * 9 + e) * BS);
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int e = 0; e < 9; ++e) U[mu][e] = k * U[mu][e];
}

template <typename A, bool NT = false, typename T>
__device__ __forceinline__ void load_link(const T *u, bool r12, cx<A> U[9])
{
#pragma unroll
    for (int e = 0; e < 6; ++e) U[e] = NT ? ldc_stream<A>(u + e * BS) : ldc<A>(u + e * BS);
    if (r12) {
        su3_third_row(U);
    } else {
#pragma unroll
        for (int e = 6; e < 9; ++e) U[e] = NT ? ldc_stream<A>(u + e * BS) : ldc<A>(u + e * BS);
    }
}

// ---------------------------------------------------------------------------
// chiral-basis spin projection.  g_mu = [[0, A_mu], [A_mu^+, 0]] with
// A_k = -i sigma_k (k = x, y, z) and A_t = 1.  For psi = (u, l) (upper spins
// 0-1, lower spins 2-3):
//   (1 - g_mu) psi = (h, -A^+ h),  h = u - A l
//   (1 + g_mu) psi = (h,  A^+ h),  h = u + A l
// so a hop needs the colour matrix on the two-spin h only.
// ---------------------------------------------------------------------------
template <int MU, typename A>
__device__ __forceinline__ void proj_minus(const cx<A> p[12], cx<A> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<A> u0 = p[c], u1 = p[3 + c], l0 = p[6 + c], l1 = p[9 + c];
        if (MU == 0) { h[c] = u0 + ti(l1); h[3 + c] = u1 + ti(l0); }
        if (MU == 1) { h[c] = u0 + l1;     h[3 + c] = u1 - l0; }
        if (MU == 2) { h[c] = u0 + ti(l0); h[3 + c] = u1 - ti(l1); }
        if (MU == 3) { h[c] = u0 - l0;     h[3 + c] = u1 - l1; }
    }
}
template <int MU, typename A>
__device__ __forceinline__ void proj_plus(const cx<A> p[12], cx<A> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<A> u0 = p[c], u1 = p[3 + c], l0 = p[6 + c], l1 = p[9 + c];
        if (MU == 0) { h[c] = u0 - ti(l1); h[3 + c] = u1 - ti(l0); }
        if (MU == 1) { h[c] = u0 - l1;     h[3 + c] = u1 + l0; }
        if (MU == 2) { h[c] = u0 - ti(l0); h[3 + c] = u1 + ti(l1); }
        if (MU == 3) { h[c] = u0 + l0;     h[3 + c] = u1 + l1; }
    }
}
// acc += k * (h, -A^+ h)
template <int MU, typename A>
__device__ __forceinline__ void recon_minus(cx<A> acc[12], const cx<A> h[6], A k)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<A> h0 = k * h[c], h1 = k * h[3 + c];
        acc[c] = acc[c] + h0;
        acc[3 + c] = acc[3 + c] + h1;
        if (MU == 0) { acc[6 + c] = acc[6 + c] + tmi(h1); acc[9 + c] = acc[9 + c] + tmi(h0); }
        if (MU == 1) { acc[6 + c] = acc[6 + c] - h1;      acc[9 + c] = acc[9 + c] + h0; }
        if (MU == 2) { acc[6 + c] = acc[6 + c] + tmi(h0); acc[9 + c] = acc[9 + c] + ti(h1); }
        if (MU == 3) { acc[6 + c] = acc[6 + c] - h0;      acc[9 + c] = acc[9 + c] - h1; }
    }
}
// acc += k * (h, A^+ h)
template <int MU, typename A>
__device__ __forceinline__ void recon_plus(cx<A> acc[12], const cx<A> h[6], A k)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<A> h0 = k * h[c], h1 = k * h[3 + c];
        acc[c] = acc[c] + h0;
        acc[3 + c] = acc[3 + c] + h1;
        if (MU == 0) { acc[6 + c] = acc[6 + c] + ti(h1);  acc[9 + c] = acc[9 + c] + ti(h0); }
        if (MU == 1) { acc[6 + c] = acc[6 + c] + h1;      acc[9 + c] = acc[9 + c] - h0; }
        if (MU == 2) { acc[6 + c] = acc[6 + c] + ti(h0);  acc[9 + c] = acc[9 + c] + tmi(h1); }
        if (MU == 3) { acc[6 + c] = acc[6 + c] + h0;      acc[9 + c] = acc[9 + c] + h1; }
    }
}

// acc += (h, -A^+ h) and acc += (h, A^+ h) without a scale factor
template <int MU, typename A>
__device__ __forceinline__ void recon_minus1(cx<A> acc[12], const cx<A> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<A> h0 = h[c], h1 = h[3 + c];
        acc[c] = acc[c] + h0;
        acc[3 + c] = acc[3 + c] + h1;
        if (MU == 0) { acc[6 + c] = acc[6 + c] + tmi(h1); acc[9 + c] = acc[9 + c] + tmi(h0); }
        if (MU == 1) { acc[6 + c] = acc[6 + c] - h1;      acc[9 + c] = acc[9 + c] + h0; }
        if (MU == 2) { acc[6 + c] = acc[6 + c] + tmi(h0); acc[9 + c] = acc[9 + c] + ti(h1); }
        if (MU == 3) { acc[6 + c] = acc[6 + c] - h0;      acc[9 + c] = acc[9 + c] - h1; }
    }
}
template <int MU, typename A>
__device__ __forceinline__ void recon_plus1(cx<A> acc[12], const cx<A> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<A> h0 = h[c], h1 = h[3 + c];
        acc[c] = acc[c] + h0;
        acc[3 + c] = acc[3 + c] + h1;
        if (MU == 0) { acc[6 + c] = acc[6 + c] + ti(h1);  acc[9 + c] = acc[9 + c] + ti(h0); }
        if (MU == 1) { acc[6 + c] = acc[6 + c] + h1;      acc[9 + c] = acc[9 + c] - h0; }
        if (MU == 2) { acc[6 + c] = acc[6 + c] + ti(h0);  acc[9 + c] = acc[9 + c] + tmi(h1); }
        if (MU == 3) { acc[6 + c] = acc[6 + c] + h0;      acc[9 + c] = acc[9 + c] + h1; }
    }
}

// out = U h (two spins), U row-major 3x3
template <typename A>
__device__ __forceinline__ void su3_mul(const cx<A> U[9], const cx<A> h[6], cx<A> out[6])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<A> acc = U[a * 3] * h[s * 3];
            cmac(acc, U[a * 3 + 1], h[s * 3 + 1]);
            cmac(acc, U[a * 3 + 2], h[s * 3 + 2]);
            out[s * 3 + a] = acc;
        }
}
// out = U^+ h
template <typename A>
__device__ __forceinline__ void su3_mul_adj(const cx<A> U[9], const cx<A> h[6], cx<A> out[6])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<A> acc = conjx(U[a]) * h[s * 3];
            cmacc(acc, U[3 + a], h[s * 3 + 1]);
            cmacc(acc, U[6 + a], h[s * 3 + 2]);
            out[s * 3 + a] = acc;
        }
}

// acc += (diag + C_k) p for one packed Hermitian 6x6 chiral half (18 slots);
// p and acc point at that half's six components
template <typename A>
__device__ __forceinline__ void clover_half_mac(const cx<A> c[18], A diag, const cx<A> x[6], cx<A> acc[6])
{
    A d[6] = {c[0].re, c[0].im, c[1].re, c[1].im, c[2].re, c[2].im};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const A di = d[i] + diag;
        acc[i].re = fma(di, x[i].re, acc[i].re);
        acc[i].im = fma(di, x[i].im, acc[i].im);
    }
    int e = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            cmac(acc[i], c[e], x[j]);
            cmacc(acc[j], c[e], x[i]);
            ++e;
        }
}

// acc += (diag + C) p, C = two packed Hermitian 6x6 halves (36 slots)
template <typename A>
__device__ __forceinline__ void clover_mac(const cx<A> cl[36], A diag, const cx<A> p[12], cx<A> acc[12])
{
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const cx<A> *c = cl + 18 * k;
        const cx<A> *x = p + 6 * k;
        A d[6] = {c[0].re, c[0].im, c[1].re, c[1].im, c[2].re, c[2].im};
        cx<A> y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) y[i] = (d[i] + diag) * x[i];
        int e = 3;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j) {
                cmac(y[i], c[e], x[j]);
                cmacc(y[j], c[e], x[i]);
                ++e;
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[6 * k + i] = acc[6 * k + i] + y[i];
    }
}

// ---------------------------------------------------------------------------
// geometry of the blocked lattice
// ---------------------------------------------------------------------------
struct Geom {
    int nb[4];      // blocks per direction
    int bstride[4]; // block-id stride per direction
    int nblocks;
    int bcs[4];     // fermion boundary sign per direction
};

__device__ __forceinline__ void block_coords(const Geom &g, int b, int bc[4])
{
    bc[0] = b % g.nb[0];
    int t = b / g.nb[0];
    bc[1] = t % g.nb[1];
    t /= g.nb[1];
    bc[2] = t % g.nb[2];
    bc[3] = t / g.nb[2];
}

// Neighbour of (block b, site s) one step in +mu (DIR = +1) or -mu (DIR = -1).
// Returns the neighbour's block and site and the boundary sign (+1/-1) that
// multiplies the hop.  inblk tells whether the neighbour lies in block b.
template <int MU, int DIR>
__device__ __forceinline__ void neighbour(const Geom &g, int b, const int bc[4], int s, int &bn, int &sn, int &sign,
                                          bool &inblk)
{
    constexpr int st = 1 << (2 * MU);
    int l = (s >> (2 * MU)) & 3;
    sign = 1;
    if (DIR > 0) {
        if (l < 3) { bn = b; sn = s + st; inblk = true; return; }
        sn = s - 3 * st;
        if (bc[MU] + 1 == g.nb[MU]) {
            bn = b - (g.nb[MU] - 1) * g.bstride[MU];
            sign = g.bcs[MU];
        } else {
            bn = b + g.bstride[MU];
        }
    } else {
        if (l > 0) { bn = b; sn = s - st; inblk = true; return; }
        sn = s + 3 * st;
        if (bc[MU] == 0) {
            bn = b + (g.nb[MU] - 1) * g.bstride[MU];
            sign = g.bcs[MU];
        } else {
            bn = b - g.bstride[MU];
        }
    }
    inblk = (bn == b); // only when the block spans the whole direction
}

// Same as neighbour<MU, DIR> with a run-time direction (mu, dir = +1/-1).
__device__ __forceinline__ void neighbour_rt(const Geom &g, int b, const int bc[4], int s, int mu, int dir, int &bn,
                                             int &sn, int &sign, bool &inblk)
{
    const int st = 1 << (2 * mu);
    const int l = (s >> (2 * mu)) & 3;
    sign = 1;
    if (dir > 0) {
        if (l < 3) { bn = b; sn = s + st; inblk = true; return; }
        sn = s - 3 * st;
        if (bc[mu] + 1 == g.nb[mu]) {
            bn = b - (g.nb[mu] - 1) * g.bstride[mu];
            sign = g.bcs[mu];
        } else {
            bn = b + g.bstride[mu];
        }
    } else {
        if (l > 0) { bn = b; sn = s - st; inblk = true; return; }
        sn = s + 3 * st;
        if (bc[mu] == 0) {
            bn = b + (g.nb[mu] - 1) * g.bstride[mu];
            sign = g.bcs[mu];
        } else {
            bn = b - g.bstride[mu];
        }
    }
    inblk = (bn == b);
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Remap so that XCD k runs a contiguous range of logical tiles: neighbouring
// tiles then share an L2.
__device__ __forceinline__ int xcd_remap(int i, int n)
{
    constexpr int NX = 8;
    int base = n / NX, extra = n % NX;
    int x = i % NX, loc = i / NX;
    return x * base + (x < extra ? x : extra) + loc;
}

} // namespace dd
