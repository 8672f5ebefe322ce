// device_math.h -- gfx950 device building blocks: complex 3x3 algebra,
// Philox4x32-10, and the tiled link storage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"
#include "log_table.h"

namespace su3hb {

// ---------------------------------------------------------------------------
// complex numbers and 3x3 complex matrices in T = float or double

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmake(T r, T i) { return cx<T>{r, i}; }

// a += b * c
template <typename T>
__device__ __forceinline__ void cfma(cx<T> &a, const cx<T> &b, const cx<T> &c)
{
    a.re = fma(b.re, c.re, fma(-b.im, c.im, a.re));
    a.im = fma(b.re, c.im, fma(b.im, c.re, a.im));
}

// a += b * conj(c)
template <typename T>
__device__ __forceinline__ void cfma_nc(cx<T> &a, const cx<T> &b, const cx<T> &c)
{
    a.re = fma(b.re, c.re, fma(b.im, c.im, a.re));
    a.im = fma(b.im, c.re, fma(-b.re, c.im, a.im));
}

// a += conj(b) * c
template <typename T>
__device__ __forceinline__ void cfma_cn(cx<T> &a, const cx<T> &b, const cx<T> &c)
{
    a.re = fma(b.re, c.re, fma(b.im, c.im, a.re));
    a.im = fma(b.re, c.im, fma(-b.im, c.re, a.im));
}

template <typename T>
struct mat3 {
    cx<T> e[3][3];
};

template <typename T>
__device__ __forceinline__ void set_zero(mat3<T> &m)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.e[i][j] = cx<T>{T(0), T(0)};
}

// c = a * b
template <typename T>
__device__ __forceinline__ mat3<T> mul_nn(const mat3<T> &a, const mat3<T> &b)
{
    mat3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s{T(0), T(0)};
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma(s, a.e[i][k], b.e[k][j]);
            c.e[i][j] = s;
        }
    return c;
}

// c = a * b^dagger
template <typename T>
__device__ __forceinline__ mat3<T> mul_na(const mat3<T> &a, const mat3<T> &b)
{
    mat3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s{T(0), T(0)};
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_nc(s, a.e[i][k], b.e[j][k]);
            c.e[i][j] = s;
        }
    return c;
}

// acc += a * b^dagger
template <typename T>
__device__ __forceinline__ void acc_na(mat3<T> &acc, const mat3<T> &a, const mat3<T> &b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_nc(acc.e[i][j], a.e[i][k], b.e[j][k]);
}

// acc += a^dagger * b
template <typename T>
__device__ __forceinline__ void acc_an(mat3<T> &acc, const mat3<T> &a, const mat3<T> &b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_cn(acc.e[i][j], a.e[k][i], b.e[k][j]);
}

template <typename T>
__device__ __forceinline__ void scale(mat3<T> &m, T s)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            m.e[i][j].re *= s;
            m.e[i][j].im *= s;
        }
}

template <typename D, typename S>
__device__ __forceinline__ mat3<D> widen(const mat3<S> &m)
{
    mat3<D> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = cx<D>{D(m.e[i][j].re), D(m.e[i][j].im)};
    return r;
}

// Re Tr(a * b) = sum_ij Re(a_ij b_ji)
template <typename T>
__device__ __forceinline__ T re_tr_nn(const mat3<T> &a, const mat3<T> &b)
{
    T s = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s = fma(a.e[i][j].re, b.e[j][i].re, fma(-a.e[i][j].im, b.e[j][i].im, s));
    return s;
}

// Re Tr(a * b^dagger) = sum_ij Re(a_ij conj(b_ij))
template <typename T>
__device__ __forceinline__ T re_tr_na(const mat3<T> &a, const mat3<T> &b)
{
    T s = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s = fma(a.e[i][j].re, b.e[i][j].re, fma(a.e[i][j].im, b.e[i][j].im, s));
    return s;
}

// row 2 = conj(row 0 x row 1): completes an SU(3) matrix from its first two rows
template <typename T>
__device__ __forceinline__ void third_row(mat3<T> &u)
{
    const cx<T> *a = u.e[0], *b = u.e[1];
    cx<T> c0{T(0), T(0)}, c1{T(0), T(0)}, c2{T(0), T(0)};
    cfma(c0, a[1], b[2]);
    cfma(c0, cx<T>{-a[2].re, -a[2].im}, b[1]);
    cfma(c1, a[2], b[0]);
    cfma(c1, cx<T>{-a[0].re, -a[0].im}, b[2]);
    cfma(c2, a[0], b[1]);
    cfma(c2, cx<T>{-a[1].re, -a[1].im}, b[0]);
    u.e[2][0] = cx<T>{c0.re, -c0.im};
    u.e[2][1] = cx<T>{c1.re, -c1.im};
    u.e[2][2] = cx<T>{c2.re, -c2.im};
}

// 1/sqrt(x) for x >= 2^-1000: the hardware reciprocal square-root estimate
// refined by two Newton steps y <- y + (y/2)(1 - x y^2), each of which about
// doubles the number of correct bits; within about an ulp.
__device__ __forceinline__ double rsqrt_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// sqrt(t) for t >= 0 in T: FP64 through rsqrt_refined (t below 2^-1000,
// including 0, takes the library square root), FP32 the library one.
template <typename T>
__device__ __forceinline__ T sqrt_nonneg(T t);
template <>
__device__ __forceinline__ double sqrt_nonneg<double>(double t)
{
    return t >= 0x1p-1000 ? t * rsqrt_refined(t) : sqrt(t);
}
template <>
__device__ __forceinline__ float sqrt_nonneg<float>(float t)
{
    return sqrtf(t);
}

// Gram-Schmidt on rows 0 and 1, then row 2 = conj(row0 x row1): det = 1.
// The row norms are near 1 (links are unitary to rounding before the update
// rotates them), inside the range of rsqrt_refined.
__device__ __forceinline__ void reunitarize(mat3<double> &u)
{
    double n0 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) n0 = fma(u.e[0][c].re, u.e[0][c].re, fma(u.e[0][c].im, u.e[0][c].im, n0));
    n0 = rsqrt_refined(n0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u.e[0][c].re *= n0;
        u.e[0][c].im *= n0;
    }
    cx<double> d{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) cfma_cn(d, u.e[0][c], u.e[1][c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) cfma(u.e[1][c], cx<double>{-d.re, -d.im}, u.e[0][c]);
    double n1 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) n1 = fma(u.e[1][c].re, u.e[1][c].re, fma(u.e[1][c].im, u.e[1][c].im, n1));
    n1 = rsqrt_refined(n1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u.e[1][c].re *= n1;
        u.e[1][c].im *= n1;
    }
    third_row(u);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies with the key bumped by a Weyl sequence between rounds.

// a ^ b ^ c in one gfx950 three-input bit operation (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32 -> 64-bit product gives both halves (a single mad_u64_u32)
        const uint64_t p0 = uint64_t(0xD2511F53u) * c.x, p1 = uint64_t(0xCD9E8D57u) * c.z;
        const uint32_t lo0 = uint32_t(p0), hi0 = uint32_t(p0 >> 32);
        const uint32_t lo1 = uint32_t(p1), hi1 = uint32_t(p1 >> 32);
        c = make_uint4(xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0);
    }
    return c;
}

// 32-bit word -> uniform double (r + 1) / 2^32 in (0, 1], exact (one FMA)
__host__ __device__ __forceinline__ double u01(uint32_t r) { return fma(double(r), 0x1p-32, 0x1p-32); }

// ---------------------------------------------------------------------------
// Elementary functions of a uniform u in (0, 1] (a Philox word (r+1)/2^32,
// so u has at most 32 significant bits), written for this range only: a
// few FP64 operations instead of the general library routines, which handle
// every argument.  Each is a short series after a reduction to a small argument.

// ln u to about one ulp, table-driven (the reduction of P. T. P. Tang, ACM
// TOMS 16, 1990): u = 2^e m with m in [3/4, 3/2) (exact); the 7 leading
// fraction bits of m pick the entry j of tbl (log_table.h, 128 entries, in
// LDS in the kernels) with c_j near 1 over the bin's midpoint and t_j + tl_j
// = -ln c_j; r = m c_j - 1 in one rounding (|r| <= 2^-7; r = m - 1 exactly
// in the two bins next to m = 1, c_j = 1); ln(1 + r) = r - r^2/2 + ... -
// r^8/8 (the first omitted term is below 2^-59 relative); and
// ln u = (e ln2_hi + t_j) + (e ln2_lo + tl_j + ln(1 + r)), where ln2_hi is
// ln 2 with its last 11 mantissa bits cleared, so e ln2_hi is exact.
__host__ __device__ __forceinline__ double log_unit(double u, const LogEntry *tbl)
{
    int e = 0;
    double m = frexp(u, &e);  // u = m 2^e, m in [1/2, 1)
    if (m < 0.75) {           // m in [3/4, 3/2)
        m *= 2.0;
        e -= 1;
    }
    uint64_t bits;
    __builtin_memcpy(&bits, &m, sizeof bits);
    const LogEntry &t = tbl[uint32_t(bits >> 45) & 127u];
    const double r = fma(m, t.c, -1.0);
    double p = -1.0 / 8;
    p = fma(p, r, 1.0 / 7);
    p = fma(p, r, -1.0 / 6);
    p = fma(p, r, 1.0 / 5);
    p = fma(p, r, -1.0 / 4);
    p = fma(p, r, 1.0 / 3);
    p = fma(p, r, -1.0 / 2);
    const double lp = fma(r * r, p, r);  // ln(1 + r)
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
    const double de = double(e);
    return fma(de, kLn2Hi, t.t) + (fma(de, kLn2Lo, t.tl) + lp);
}

// cos^2(2 pi u): with t = 4u = k + f (k = nearest integer, |f| <= 1/2, both
// exact), 2 pi u = (pi/2)(k + f), so cos^2(2 pi u) = (1 + cos(pi f))/2 for
// even k and (1 - cos(pi f))/2 for odd k.  cos(pi f) = sum_n c_n f^(2n),
// c_n = (-1)^n pi^(2n)/(2n)!, through n = 11 (the next term is below 1e-19).
__host__ __device__ __forceinline__ double cos2_turn(double u)
{
    const double t = 4.0 * u;
    const double k = rint(t);
    const double f = t - k;
    const double w = f * f;
    double c = -0x1.52ae4120fde27p-34;
    c = fma(c, w, 0x1.ef6e308d6d1c4p-29);
    c = fma(c, w, -0x1.2a0c591af8314p-23);
    c = fma(c, w, 0x1.20c62c2f2d7f5p-18);
    c = fma(c, w, -0x1.b6e24f44b128fp-14);
    c = fma(c, w, 0x1.f9d38a3763cc3p-10);
    c = fma(c, w, -0x1.a6d1f2a204a8cp-6);
    c = fma(c, w, 0x1.e1f506891babbp-3);
    c = fma(c, w, -0x1.55d3c7e3cbffap+0);
    c = fma(c, w, 0x1.03c1f081b5ac4p+2);
    c = fma(c, w, -0x1.3bd3cc9be45dep+2);
    c = fma(c, w, 1.0);  // cos(pi f)
    const bool odd = (int64_t(k) & 1) != 0;
    return 0.5 + (odd ? -0.5 : 0.5) * c;
}

// sin(2 pi u) and cos(2 pi u) in T (float or double): with t = 4u = k + f as
// above, 2 pi u = (pi/2) k + x, x = (pi/2) f in [-pi/4, pi/4]; sin x and
// cos x from their Taylor series in f (float: through f^9 and f^10, double:
// through f^17 and f^18, each next term below the precision's half ulp),
// then rotated by the quarter turns k mod 4.
template <typename T>
__host__ __device__ __forceinline__ void sincos_turn(double u, T *sn, T *cs);

template <>
__host__ __device__ __forceinline__ void sincos_turn<float>(double u, float *sn, float *cs)
{
    const double t = 4.0 * u;
    const double k = rint(t);
    const float f = float(t - k);
    const float w = f * f;
    // sin((pi/2) f) / f = sum_n (-1)^n (pi/2)^(2n+1) w^n / (2n+1)!,
    // cos((pi/2) f) = sum_n (-1)^n (pi/2)^(2n) w^n / (2n)!
    float sp = 0x1.507834p-13f;
    sp = fmaf(sp, w, -0x1.32d2ccp-8f);
    sp = fmaf(sp, w, 0x1.466bc6p-4f);
    sp = fmaf(sp, w, -0x1.4abbcep-1f);
    sp = fmaf(sp, w, 0x1.921fb6p+0f);
    float cp = -0x1.a6d1f2p-16f;
    cp = fmaf(cp, w, 0x1.e1f506p-11f);
    cp = fmaf(cp, w, -0x1.55d3c8p-6f);
    cp = fmaf(cp, w, 0x1.03c1f0p-2f);
    cp = fmaf(cp, w, -0x1.3bd3ccp+0f);
    cp = fmaf(cp, w, 1.0f);
    const float S = sp * f, C = cp;
    const int q = int(int64_t(k) & 3);
    *sn = q == 0 ? S : q == 1 ? C : q == 2 ? -S : -C;
    *cs = q == 0 ? C : q == 1 ? -S : q == 2 ? -C : S;
}

template <>
__host__ __device__ __forceinline__ void sincos_turn<double>(double u, double *sn, double *cs)
{
    const double t = 4.0 * u;
    const double k = rint(t);
    const double f = t - k;
    const double w = f * f;
    double sp = -0x1.8a404211f9547p-45;
    sp = fma(sp, w, 0x1.aaec32af93359p-38);
    sp = fma(sp, w, -0x1.6fadb9f155744p-31);
    sp = fma(sp, w, 0x1.e8f434d018d63p-25);
    sp = fma(sp, w, -0x1.e3074fde8871fp-19);
    sp = fma(sp, w, 0x1.50783487ee782p-13);
    sp = fma(sp, w, -0x1.32d2cce62bd86p-8);
    sp = fma(sp, w, 0x1.466bc6775aae2p-4);
    sp = fma(sp, w, -0x1.4abbce625be53p-1);
    sp = fma(sp, w, 0x1.921fb54442d18p+0);
    double cp = -0x1.2a0c591af8314p-41;
    cp = fma(cp, w, 0x1.20c62c2f2d7f5p-34);
    cp = fma(cp, w, -0x1.b6e24f44b128fp-28);
    cp = fma(cp, w, 0x1.f9d38a3763cc3p-22);
    cp = fma(cp, w, -0x1.a6d1f2a204a8cp-16);
    cp = fma(cp, w, 0x1.e1f506891babbp-11);
    cp = fma(cp, w, -0x1.55d3c7e3cbffap-6);
    cp = fma(cp, w, 0x1.03c1f081b5ac4p-2);
    cp = fma(cp, w, -0x1.3bd3cc9be45dep+0);
    cp = fma(cp, w, 1.0);
    const double S = sp * f, C = cp;
    const int q = int(int64_t(k) & 3);
    *sn = q == 0 ? S : q == 1 ? C : q == 2 ? -S : -C;
    *cs = q == 0 ? C : q == 1 ? -S : q == 2 ? -C : S;
}

constexpr uint32_t kTagUpdate = 0;
constexpr uint32_t kTagStart = 1;

// ---------------------------------------------------------------------------
// Link storage.  Per replica the links form slabs [layer][mu][parity], each
// holding the links of one direction and parity, ordered by the half-lattice
// index h and cut into tiles of kTile consecutive h.  A tile stores 16-byte
// packets: packet 0 of its kTile links, then packet 1, and so on, so a wave
// reads each packet of 64 consecutive links as 1 KB in one piece and a whole
// link of 64 consecutive h from one contiguous stretch of memory:
//   FP64: one complex element (double2) per packet, NE packets;
//   FP32: two complex elements (float4) per packet; 18-real storage ends the
//         tile with the odd element of its links as float2.
// Every access goes through a LinkRef (slab base, h).

template <int PREC>
struct Store;

template <>
struct Store<kFP64_18> {
    using real = double;
    static constexpr int NE = 9;
};
template <>
struct Store<kFP32_18> {
    using real = float;
    static constexpr int NE = 9;
};
template <>
struct Store<kFP32_12> {
    using real = float;
    static constexpr int NE = 6;
};
template <>
struct Store<kFP64_12> {
    using real = double;
    static constexpr int NE = 6;
};

struct LinkRef {
    char *slab;   // first byte of the (layer, direction, parity) slab
    uint32_t h;   // half-lattice index of the link
};

// Bytes of one stored link and the address of packet 0 of link h: tile
// h / kTile, lane h % kTile inside it.
template <int PREC>
constexpr size_t link_store_bytes()
{
    return size_t(Store<PREC>::NE) * 2 * sizeof(typename Store<PREC>::real);
}

template <int PREC>
__device__ __forceinline__ char *tile_of(const LinkRef &r)
{
    return r.slab + size_t(r.h / kTile) * (kTile * link_store_bytes<PREC>());
}

template <int PREC>
__device__ __forceinline__ char *packet_ptr(const LinkRef &r, int j)
{
    return tile_of<PREC>(r) + (size_t(j) * kTile + r.h % kTile) * 16;
}

// the odd element of FP32 18-real storage, after the tile's four packets
template <int PREC>
__device__ __forceinline__ char *tail_ptr(const LinkRef &r)
{
    return tile_of<PREC>(r) + size_t(Store<PREC>::NE / 2) * kTile * 16 + size_t(r.h % kTile) * 8;
}

typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float4 __attribute__((ext_vector_type(4)));
typedef float nt_float2 __attribute__((ext_vector_type(2)));

// A packet read with the normal or (NT) the non-temporal cache policy.
template <typename V, bool NT>
__device__ __forceinline__ V read_packet(const char *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    else return *reinterpret_cast<const V *>(p);
}

// complex element e of a link
template <int PREC, bool NT = false>
__device__ __forceinline__ cx<typename Store<PREC>::real> load_elem(const LinkRef &r, int e)
{
    using R = typename Store<PREC>::real;
    if constexpr (sizeof(R) == 8) {
        const nt_double2 v = read_packet<nt_double2, NT>(packet_ptr<PREC>(r, e));
        return cx<R>{v.x, v.y};
    } else {
        constexpr int NP = Store<PREC>::NE / 2;
        if (e >= 2 * NP) {
            const nt_float2 v = read_packet<nt_float2, NT>(tail_ptr<PREC>(r));
            return cx<R>{v.x, v.y};
        }
        const nt_float2 v = read_packet<nt_float2, NT>(packet_ptr<PREC>(r, e >> 1) + (e & 1) * 8);
        return cx<R>{v.x, v.y};
    }
}

// The NE stored elements of a link (row 2 of 12-real storage left unset);
// NT: the non-temporal policy, for a link no other thread of the launch
// reads.
template <int PREC, bool NT = false>
__device__ __forceinline__ mat3<typename Store<PREC>::real> load_stored(const LinkRef &r)
{
    using R = typename Store<PREC>::real;
    constexpr int NE = Store<PREC>::NE;
    mat3<R> m;
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int e = 0; e < NE; ++e) m.e[e / 3][e % 3] = load_elem<PREC, NT>(r, e);
    } else {
        constexpr int NP = NE / 2;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const nt_float4 v = read_packet<nt_float4, NT>(packet_ptr<PREC>(r, j));
            m.e[(2 * j) / 3][(2 * j) % 3] = cx<R>{v.x, v.y};
            m.e[(2 * j + 1) / 3][(2 * j + 1) % 3] = cx<R>{v.z, v.w};
        }
        if constexpr (NE & 1) m.e[2][2] = load_elem<PREC, NT>(r, NE - 1);
    }
    return m;
}

// A whole link.
template <int PREC, bool NT = false>
__device__ __forceinline__ mat3<typename Store<PREC>::real> load_link(const LinkRef &r)
{
    mat3<typename Store<PREC>::real> m = load_stored<PREC, NT>(r);
    if constexpr (Store<PREC>::NE == 6) third_row(m);
    return m;
}

// A slice writes each link once and reads it back only in later slices, so
// the stores take the non-temporal policy and leave L2 to the neighbour
// lines that other threads of the slice read again.

template <int PREC>
__device__ __forceinline__ void store_link(const LinkRef &r, const mat3<double> &m)
{
    using R = typename Store<PREC>::real;
    constexpr int NE = Store<PREC>::NE;
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int e = 0; e < NE; ++e)
            __builtin_nontemporal_store(nt_double2{m.e[e / 3][e % 3].re, m.e[e / 3][e % 3].im},
                                        reinterpret_cast<nt_double2 *>(packet_ptr<PREC>(r, e)));
    } else {
        constexpr int NP = NE / 2;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const cx<double> a = m.e[(2 * j) / 3][(2 * j) % 3], b = m.e[(2 * j + 1) / 3][(2 * j + 1) % 3];
            __builtin_nontemporal_store(nt_float4{float(a.re), float(a.im), float(b.re), float(b.im)},
                                        reinterpret_cast<nt_float4 *>(packet_ptr<PREC>(r, j)));
        }
        if constexpr (NE & 1)
            __builtin_nontemporal_store(nt_float2{float(m.e[2][2].re), float(m.e[2][2].im)},
                                        reinterpret_cast<nt_float2 *>(tail_ptr<PREC>(r)));
    }
}

// The matrix a link reads back as after store_link<PREC>(m), in the storage
// precision: rounded, with row 2 rebuilt for 12-real storage.
template <int PREC>
__device__ __forceinline__ mat3<typename Store<PREC>::real> stored_form_r(const mat3<double> &m)
{
    using R = typename Store<PREC>::real;
    mat3<R> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = cx<R>{R(m.e[i][j].re), R(m.e[i][j].im)};
    if constexpr (Store<PREC>::NE == 6) third_row(r);
    return r;
}

// Rows 0 and 1 of a link (row 2 left unset): the first six stored elements
// of every storage form.
template <int PREC>
__device__ __forceinline__ mat3<typename Store<PREC>::real> load_rows01(const LinkRef &r)
{
    using R = typename Store<PREC>::real;
    mat3<R> m;
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int e = 0; e < 6; ++e) m.e[e / 3][e % 3] = load_elem<PREC>(r, e);
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const nt_float4 v = read_packet<nt_float4, false>(packet_ptr<PREC>(r, j));
            m.e[(2 * j) / 3][(2 * j) % 3] = cx<R>{v.x, v.y};
            m.e[(2 * j + 1) / 3][(2 * j + 1) % 3] = cx<R>{v.z, v.w};
        }
    }
    return m;
}

// A neighbour link read from global memory or from a wave's staging area in
// LDS.  The staging area holds the stored elements of nslot consecutive
// links of one slab, element-major (element e of slot i at e * nslot + i);
// the link is taken from there when stg is set and slot < nslot, else from
// global memory.  Both give the same bits.
template <int PREC>
struct LinkSrc {
    LinkRef ref;
    const cx<typename Store<PREC>::real> *stg;
    uint32_t slot, nslot;
    bool rows;  // from global memory: read rows 0 and 1 and rebuild row 2 as their cross product
};

template <int PREC>
__device__ __forceinline__ LinkSrc<PREC> from_global(const LinkRef &r, bool rows = false)
{
    return LinkSrc<PREC>{r, nullptr, 0u, 0u, rows};
}

template <int PREC>
__device__ __forceinline__ bool staged(const LinkSrc<PREC> &s)
{
    return s.stg != nullptr && s.slot < s.nslot;
}

template <int PREC>
__device__ __forceinline__ mat3<typename Store<PREC>::real> stored_from_lds(const LinkSrc<PREC> &s)
{
    mat3<typename Store<PREC>::real> m;
#pragma unroll
    for (int e = 0; e < Store<PREC>::NE; ++e) m.e[e / 3][e % 3] = s.stg[e * s.nslot + s.slot];
    return m;
}

template <int PREC>
__device__ __forceinline__ mat3<typename Store<PREC>::real> fetch_link(const LinkSrc<PREC> &s)
{
    if (staged(s)) {
        // the same values as from global memory: row 2 rebuilt wherever the
        // global read would rebuild it
        mat3<typename Store<PREC>::real> m = stored_from_lds(s);
        if (Store<PREC>::NE == 6 || s.rows) third_row(m);
        return m;
    }
    if (s.rows) {
        mat3<typename Store<PREC>::real> m = load_rows01<PREC>(s.ref);
        third_row(m);
        return m;
    }
    return load_link<PREC>(s.ref);
}

template <int PREC>
__device__ __forceinline__ mat3<typename Store<PREC>::real> fetch_rows01(const LinkSrc<PREC> &s)
{
    if (staged(s)) return stored_from_lds(s);
    return load_rows01<PREC>(s.ref);
}

// Both staples of plane (mu, nu), with F1 = U_nu(x+mu), F2 = U_mu(x+nu),
// F3 = U_nu(x), B1 = U_nu(x+mu-nu), B2 = U_mu(x-nu), B3 = U_nu(x-nu):
// acc += wf F1 (F3 F2)^dag + wb (B2 B1)^dag B3.  Every product of SU(3)
// matrices is in SU(3), so only its rows 0 and 1 are multiplied out and row
// 2 is conj(row0 x row1); then F3, F1 and B2 are needed only as their rows 0
// and 1 (6 of 9 packets in 18-real storage):
//   M = F3 F2 (rows 0, 1 from F3's rows 0, 1), Q = F1 M^dag (rows 0, 1 from
//   F1's rows 0, 1): the forward staple F1 (F3 F2)^dag = Q;
//   N = B2 B1 (rows 0, 1 from B2's rows 0, 1), R = N^dag B3: the backward
//   staple (B2 B1)^dag B3 = R;
// acc += wf Q + wb R.  Every link a slice reads is still read whole by one of
// its two readers (F3 of x is B1 of x - mu + nu, F1 of x is B3 of
// x + mu + nu, F2 of x is B2 of x + 2 nu).  The loads come in partner pairs
// (F3 with B1, F2 with B2, F1 with B3), so the second read of a line comes
// while the first has it in L2.  CLASSES (the fused measurement on two
// layers): the unweighted Q and R are also added to class sums cf and cb in
// LDS (cls, element-major with the given stride, thread slot t).
template <int PREC, bool CLASSES = false>
__device__ __forceinline__ void acc_plane_staples(mat3<typename Store<PREC>::real> &acc, const LinkRef &f1,
                                                  const LinkSrc<PREC> &f2, const LinkRef &f3, const LinkRef &b1,
                                                  const LinkSrc<PREC> &b2, const LinkRef &b3,
                                                  typename Store<PREC>::real wf, typename Store<PREC>::real wb,
                                                  cx<typename Store<PREC>::real> *cls = nullptr,
                                                  uint32_t stride = 0, uint32_t t = 0, int cf = 0, int cb = 0)
{
    using R = typename Store<PREC>::real;
    const mat3<R> m3 = load_rows01<PREC>(f3);
    const mat3<R> mb1 = load_link<PREC>(b1);
    mat3<R> M;
    {
        const mat3<R> m2 = fetch_link<PREC>(f2);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                cx<R> s{R(0), R(0)};
#pragma unroll
                for (int k = 0; k < 3; ++k) cfma(s, m3.e[j][k], m2.e[k][i]);
                M.e[j][i] = s;
            }
        third_row(M);
    }
    mat3<R> N;
    {
        const mat3<R> mb2 = fetch_rows01<PREC>(b2);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                cx<R> s{R(0), R(0)};
#pragma unroll
                for (int k = 0; k < 3; ++k) cfma(s, mb2.e[j][k], mb1.e[k][i]);
                N.e[j][i] = s;
            }
        third_row(N);
    }
    const mat3<R> m1 = load_rows01<PREC>(f1);
    const mat3<R> mb3 = load_link<PREC>(b3);
    mat3<R> Q, Rb;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<R> q{R(0), R(0)}, b{R(0), R(0)};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cfma_nc(q, m1.e[r][k], M.e[j][k]);   // (F1 M^dag)_rj
                cfma_cn(b, N.e[k][r], mb3.e[k][j]);  // (N^dag B3)_rj
            }
            Q.e[r][j] = q;
            Rb.e[r][j] = b;
        }
    third_row(Q);
    third_row(Rb);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            acc.e[i][j].re = fma(wf, Q.e[i][j].re, fma(wb, Rb.e[i][j].re, acc.e[i][j].re));
            acc.e[i][j].im = fma(wf, Q.e[i][j].im, fma(wb, Rb.e[i][j].im, acc.e[i][j].im));
        }
    if constexpr (CLASSES) {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            cx<R> &fe = cls[(cf * 9 + e) * stride + t];
            fe.re += Q.e[e / 3][e % 3].re;
            fe.im += Q.e[e / 3][e % 3].im;
            cx<R> &be = cls[(cb * 9 + e) * stride + t];
            be.re += Rb.e[e / 3][e % 3].re;
            be.im += Rb.e[e / 3][e % 3].im;
        }
    }
}

}  // namespace su3hb
