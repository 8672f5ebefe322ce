// device_math.h -- gfx950 device building blocks: complex 3x3 algebra,
// Philox4x32-10, and the structure-of-arrays link storage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

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

// Gram-Schmidt on rows 0 and 1, then row 2 = conj(row0 x row1): det = 1.
__device__ __forceinline__ void reunitarize(mat3<double> &u)
{
    double n0 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) n0 = fma(u.e[0][c].re, u.e[0][c].re, fma(u.e[0][c].im, u.e[0][c].im, n0));
    n0 = 1.0 / sqrt(n0);
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
    n1 = 1.0 / sqrt(n1);
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

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// 32-bit word -> uniform double (r + 1) / 2^32 in (0, 1]
__device__ __forceinline__ double u01(uint32_t r) { return (double(r) + 1.0) * 0x1p-32; }

constexpr uint32_t kTagUpdate = 0;
constexpr uint32_t kTagStart = 1;

// ---------------------------------------------------------------------------
// Link storage: per replica [layer][mu][parity][element][Vh] with one complex
// element per entry (double2 or float2), so each element of a matrix is a
// contiguous, fully coalesced array over the half-lattice index h.

template <int PREC>
struct Store;

template <>
struct Store<kFP64_18> {
    using real = double;
    using elem = double2;
    static constexpr int NE = 9;
};
template <>
struct Store<kFP32_18> {
    using real = float;
    using elem = float2;
    static constexpr int NE = 9;
};
template <>
struct Store<kFP32_12> {
    using real = float;
    using elem = float2;
    static constexpr int NE = 6;
};

template <int PREC>
__device__ __forceinline__ mat3<typename Store<PREC>::real> load_link(
    const typename Store<PREC>::elem *__restrict__ p, uint32_t Vh)
{
    using R = typename Store<PREC>::real;
    mat3<R> m;
    constexpr int NE = Store<PREC>::NE;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const auto v = p[(size_t)e * Vh];
        m.e[e / 3][e % 3] = cx<R>{v.x, v.y};
    }
    if constexpr (NE == 6) third_row(m);
    return m;
}

template <int PREC>
__device__ __forceinline__ void store_link(typename Store<PREC>::elem *__restrict__ p, uint32_t Vh,
                                           const mat3<double> &m)
{
    using E = typename Store<PREC>::elem;
    using R = typename Store<PREC>::real;
    constexpr int NE = Store<PREC>::NE;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        E v;
        v.x = R(m.e[e / 3][e % 3].re);
        v.y = R(m.e[e / 3][e % 3].im);
        p[(size_t)e * Vh] = v;
    }
}


// The FP64 matrix a link reads back as after store_link<PREC>(m): rounded to
// the storage precision, with row 2 rebuilt for 12-real storage.
template <int PREC>
__device__ __forceinline__ mat3<double> stored_form(const mat3<double> &m)
{
    using R = typename Store<PREC>::real;
    if constexpr (Store<PREC>::NE == 9 && sizeof(R) == sizeof(double)) {
        return m;
    } else {
        mat3<R> r;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) r.e[i][j] = cx<R>{R(m.e[i][j].re), R(m.e[i][j].im)};
        if constexpr (Store<PREC>::NE == 6) third_row(r);
        return widen<double>(r);
    }
}

// Row i of a stored link (12-real storage: row 2 is rebuilt from rows 0, 1).
template <int PREC>
__device__ __forceinline__ void load_link_row(const typename Store<PREC>::elem *__restrict__ p, uint32_t Vh, int i,
                                              cx<typename Store<PREC>::real> r[3])
{
    using R = typename Store<PREC>::real;
    if (Store<PREC>::NE == 6 && i == 2) {
        cx<R> a[3], b[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const auto v = p[size_t(c) * Vh];
            const auto w = p[size_t(3 + c) * Vh];
            a[c] = cx<R>{v.x, v.y};
            b[c] = cx<R>{w.x, w.y};
        }
        cx<R> c0{R(0), R(0)}, c1{R(0), R(0)}, c2{R(0), R(0)};
        cfma(c0, a[1], b[2]);
        cfma(c0, cx<R>{-a[2].re, -a[2].im}, b[1]);
        cfma(c1, a[2], b[0]);
        cfma(c1, cx<R>{-a[0].re, -a[0].im}, b[2]);
        cfma(c2, a[0], b[1]);
        cfma(c2, cx<R>{-a[1].re, -a[1].im}, b[0]);
        r[0] = cx<R>{c0.re, -c0.im};
        r[1] = cx<R>{c1.re, -c1.im};
        r[2] = cx<R>{c2.re, -c2.im};
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const auto v = p[size_t(3 * i + c) * Vh];
            r[c] = cx<R>{v.x, v.y};
        }
    }
}

// acc += w * u1 u2^dag u3^dag, streaming u1 row by row (u2, u3 held whole).
template <int PREC>
__device__ __forceinline__ void acc_forward_staple(mat3<typename Store<PREC>::real> &acc,
                                                   const typename Store<PREC>::elem *__restrict__ p1,
                                                   const mat3<typename Store<PREC>::real> &u2,
                                                   const mat3<typename Store<PREC>::real> &u3,
                                                   uint32_t Vh, typename Store<PREC>::real w)
{
    using R = typename Store<PREC>::real;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        cx<R> r1[3];
        load_link_row<PREC>(p1, Vh, i, r1);
        cx<R> t[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<R> s{R(0), R(0)};
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_nc(s, r1[k], u2.e[j][k]);
            t[j] = cx<R>{w * s.re, w * s.im};
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma_nc(acc.e[i][j], t[k], u3.e[j][k]);
    }
}

// acc += w * (u1 u2)^dag u3, streaming rows of u1 and u3 together (u2 whole):
// (t^dag u3)_ij = sum_k conj(t_ki) u3_kj with t_k. = u1_k. u2.
template <int PREC>
__device__ __forceinline__ void acc_backward_staple(mat3<typename Store<PREC>::real> &acc,
                                                    const typename Store<PREC>::elem *__restrict__ p1,
                                                    const mat3<typename Store<PREC>::real> &u2,
                                                    const typename Store<PREC>::elem *__restrict__ p3,
                                                    uint32_t Vh, typename Store<PREC>::real w)
{
    using R = typename Store<PREC>::real;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cx<R> r1[3], r3[3];
        load_link_row<PREC>(p1, Vh, k, r1);
        load_link_row<PREC>(p3, Vh, k, r3);
        cx<R> t[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cx<R> s{R(0), R(0)};
#pragma unroll
            for (int m = 0; m < 3; ++m) cfma(s, r1[m], u2.e[m][i]);
            t[i] = cx<R>{w * s.re, w * s.im};
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) cfma_cn(acc.e[i][j], t[i], r3[j]);
    }
}

}  // namespace su3hb
