// aux.hip -- plaquette measurement (paper Sec. 2.4 measurement step) with
// FP64 accumulation, start configurations (Sec. 2.3 istart), conversion
// between the canonical FP64 layout and the internal storage, SU(3) input
// validation, and small counter kernels.
#include "geometry.h"
#include "kernels.h"

namespace su3hb {

// ---------------------------------------------------------------------------
// plaquettes

// Reduce NV doubles over the block; thread 0 returns the sums.  Fixed order
// for a fixed block size, so repeated measurements agree bit for bit.
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV])
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off);
    __shared__ double s[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) s[wave][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 1; w < nw; ++w)
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] += s[w][i];
    }
}

// Plane k of D(D-1)/2 as (mu, nu), mu < nu, in the order (0,1), (0,2), ...
template <int D>
__device__ __forceinline__ void plane_dirs(int k, int &mu, int &nu)
{
    mu = 0;
    nu = 1;
#pragma unroll
    for (int m = 0, c = 0; m < D; ++m)
#pragma unroll
        for (int n = m + 1; n < D; ++n, ++c)
            if (c == k) {
                mu = m;
                nu = n;
            }
}

// One thread per (site, plane) item (`spt` items per thread, strided by the
// block size; items plane-major, so a wave reads consecutive sites):
// (1/3) Re Tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag] = (1/3) Re Tr(T1 T2^dag)
// with T1 = U_mu(x) U_nu(x+mu), T2 = U_nu(x) U_mu(x+nu); products in FP64.
// Partial sums per block: [spacelike, timelike, layer0, layer1, beta-weighted].
template <int D, int PREC>
__global__ void __launch_bounds__(256) plaquette_kernel(PlaqArgs a)
{
    constexpr int NPL = D * (D - 1) / 2;
    const uint32_t lb = blockIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (lb < a.total_blocks) {
        const int r = a.nrep == 1 ? 0 : find_replica(a.reps, a.nrep, lb, kPlaquetteBlocks);
        const RepDesc &rep = a.reps[r];
        const uint32_t glued = rep.nlat == 2 ? rep.glued : 0u;
        const double beta0 = a.use_rep_beta ? rep.beta0 : a.beta0;
        const double beta1 = a.use_rep_beta ? rep.beta1 : a.beta1;
        void *links = const_cast<void *>(a.links);
        // items can outnumber links ((D-1)/2 per link): 64-bit item index
        const uint32_t nsite = rep.nlat * rep.V;
        const uint64_t nitem = uint64_t(nsite) * uint64_t(NPL);
        const uint64_t first = uint64_t(lb - rep.plq_block0) * blockDim.x * rep.plq_spt + threadIdx.x;
        for (uint32_t j = 0; j < rep.plq_spt; ++j) {
            const uint64_t it = first + uint64_t(j) * blockDim.x;
            if (it >= nitem) break;
            const int k = int(it / nsite);
            const uint32_t lt = uint32_t(it - uint64_t(k) * nsite);
            const uint32_t layer = lt >= rep.V ? 1u : 0u;
            const uint32_t rem = lt - layer * rep.V;
            const int p = rem >= rep.Vh ? 1 : 0;
            const uint32_t h = rem - uint32_t(p) * rep.Vh;
            Site<D> x;
            x.from_half(rep, h, p, layer);
            const int q = 1 - p;
            int mu, nu;
            plane_dirs<D>(k, mu, nu);
            const Step fm = step_fwd<D>(rep, x, mu, glued);
            const Step fn = step_fwd<D>(rep, x, nu, glued);
            const uint32_t s_pm = x.s + uint32_t(fm.ds), l_pm = layer ^ fm.flip;
            const uint32_t s_pn = x.s + uint32_t(fn.ds), l_pn = layer ^ fn.flip;
            const mat3<double> t1 =
                mul_nn(widen<double>(load_link<PREC>(link_ref<D, PREC>(links, rep, layer, mu, p, x.s))),
                       widen<double>(load_link<PREC>(link_ref<D, PREC>(links, rep, l_pm, nu, q, s_pm))));
            const mat3<double> t2 =
                mul_nn(widen<double>(load_link<PREC>(link_ref<D, PREC>(links, rep, layer, nu, p, x.s))),
                       widen<double>(load_link<PREC>(link_ref<D, PREC>(links, rep, l_pn, mu, q, s_pn))));
            const double P = re_tr_na(t1, t2) * (1.0 / 3.0);
            if (nu == D - 1) v[1] += P; else v[0] += P;
            if (layer == 0) v[2] += P; else v[3] += P;
            const uint32_t tags = layer + l_pm + l_pn + layer;
            v[4] += (tags == 0 ? beta0 : beta1) * P;
        }
    }
    block_sum<5>(v);
    if (threadIdx.x == 0 && lb < a.total_blocks)
#pragma unroll
        for (int i = 0; i < 5; ++i) a.partials[size_t(lb) * 5 + i] = v[i];
}

// Fused measurement: meas[mu][b][c] holds the block sums of (1/3) Re Tr U_p
// over the planes (nu, mu), nu < mu, written by the parity-1 update slices,
// in nc classes: nc = 1 for one layer; nc = 3 for two layers (0: base site in
// layer 0 and all links in layer 0, 1: base in layer 0 otherwise, 2: base in
// layer 1).  One block adds them up in a fixed order.
__global__ void __launch_bounds__(1024) measure_finalize_kernel(const double *meas, int D, uint32_t nblocks, int nc,
                                                                 double V, int nlat, double beta0, double beta1,
                                                                 double *out, double *series, uint32_t *cursor)
{
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // [spacelike, timelike] x class
    const uint32_t bd = blockDim.x;
    for (int mu = 1; mu < D; ++mu) {
        for (int c = 0; c < nc; ++c) {
            // eight independent partial sums (fixed assignment, so the result
            // is reproducible) keep eight loads in flight per thread
            const double *m = meas + size_t(mu) * nblocks * nc + c;
            double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            uint32_t b = threadIdx.x;
            for (; b + 7 * bd < nblocks; b += 8 * bd) {
#pragma unroll
                for (int k = 0; k < 8; ++k) s[k] += m[size_t(b + k * bd) * nc];
            }
            for (; b < nblocks; b += bd) s[0] += m[size_t(b) * nc];
            v[(mu == D - 1 ? 3 : 0) + c] += ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] += __shfl_xor(v[i], off);
    __shared__ double sh[16][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i) sh[wave][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x >> 6); ++w)
#pragma unroll
            for (int i = 0; i < 6; ++i) v[i] += sh[w][i];
        const double nV = double(nlat) * V;
        const double nspace = nV * (D - 1) * (D - 2) / 2.0, ntime = nV * (D - 1);
        const double nlayer = V * D * (D - 1) / 2.0;
        const double nan = __builtin_nan("");
        const double space = v[0] + v[1] + v[2], time = v[3] + v[4] + v[5];
        const double t0 = v[0] + v[3], t1 = v[1] + v[4], t2 = v[2] + v[5];
        double o[6];
        o[0] = (space + time) / (nspace + ntime);
        o[1] = nspace > 0 ? space / nspace : nan;
        o[2] = time / ntime;
        o[3] = (t0 + t1) / nlayer;
        o[4] = nlat == 2 ? t2 / nlayer : nan;
        o[5] = beta0 * t0 + beta1 * (t1 + t2);
        for (int i = 0; i < 6; ++i) out[i] = o[i];
        if (series) {
            const uint32_t k = atomicAdd(cursor, 1u);
            for (int i = 0; i < 6; ++i) series[size_t(k) * 6 + i] = o[i];
        }
    }
}

hipError_t launch_measure_finalize(hipStream_t st, const double *meas, int D, uint32_t nblocks, int nc, double V,
                                   int nlat, double beta0, double beta1, double *out, double *series,
                                   uint32_t *cursor)
{
    if (nc != 1 && nc != 3) return hipErrorInvalidValue;
    hipLaunchKernelGGL(measure_finalize_kernel, dim3(1), dim3(1024), 0, st, meas, D, nblocks, nc, V, nlat, beta0,
                       beta1, out, series, cursor);
    return hipGetLastError();
}

// One block per replica: fixed-order sum of its block partials, normalised.
__global__ void __launch_bounds__(256) plaquette_finalize_kernel(const RepDesc *reps, int D,
                                                                  const double *partials, double *out,
                                                                  double *series, uint32_t *cursor)
{
    const RepDesc &rep = reps[blockIdx.x];
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < rep.plq_blocks; b += blockDim.x)
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] += partials[size_t(rep.plq_block0 + b) * 5 + i];
    block_sum<5>(v);
    if (threadIdx.x == 0) {
        const double nV = double(rep.nlat) * double(rep.V);
        const double nspace = nV * (D - 1) * (D - 2) / 2.0;
        const double ntime = nV * (D - 1);
        const double nlayer = double(rep.V) * D * (D - 1) / 2.0;
        const double nan = __builtin_nan("");
        double o[6];
        o[0] = (v[0] + v[1]) / (nspace + ntime);
        o[1] = nspace > 0 ? v[0] / nspace : nan;
        o[2] = v[1] / ntime;
        o[3] = v[2] / nlayer;
        o[4] = rep.nlat == 2 ? v[3] / nlayer : nan;
        o[5] = v[4];
        for (int i = 0; i < 6; ++i) out[size_t(blockIdx.x) * 6 + i] = o[i];
        if (series) {
            const uint32_t k = atomicAdd(cursor, 1u);
            for (int i = 0; i < 6; ++i) series[size_t(k) * 6 + i] = o[i];
        }
    }
}

template <int D, int PREC>
static hipError_t launch_plaquette_t(dim3 g, dim3 b, hipStream_t st, const PlaqArgs &a)
{
    hipLaunchKernelGGL((plaquette_kernel<D, PREC>), g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_plaquette(int D, int prec, dim3 g, dim3 b, hipStream_t st, const PlaqArgs &a)
{
#define SU3HB_CASE(DD)                                                            \
    case DD:                                                                      \
        switch (prec) {                                                           \
        case kFP64_18: return launch_plaquette_t<DD, kFP64_18>(g, b, st, a);      \
        case kFP32_18: return launch_plaquette_t<DD, kFP32_18>(g, b, st, a);      \
        case kFP32_12: return launch_plaquette_t<DD, kFP32_12>(g, b, st, a);      \
        case kFP64_12: return launch_plaquette_t<DD, kFP64_12>(g, b, st, a);      \
        default: return hipErrorInvalidValue;                                     \
        }
    switch (D) {
        SU3HB_CASE(2)
        SU3HB_CASE(3)
        SU3HB_CASE(4)
        SU3HB_CASE(5)
        SU3HB_CASE(6)
    default: return hipErrorInvalidValue;
    }
#undef SU3HB_CASE
}

hipError_t launch_plaquette_finalize(hipStream_t st, const RepDesc *reps, int nrep, int D,
                                     const double *partials, double *out, double *series,
                                     uint32_t *series_cursor)
{
    hipLaunchKernelGGL(plaquette_finalize_kernel, dim3(nrep), dim3(256), 0, st, reps, D, partials, out,
                       series, series_cursor);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// start configurations

// Haar SU(3): two rows of complex Gaussians (Box-Muller on three Philox
// blocks of the start stream), Gram-Schmidt and the cross product.
template <int D, int PREC>
__global__ void __launch_bounds__(256) start_kernel(void *links, const RepDesc *reps, int r,
                                                     uint32_t nthreads, int mode)
{
    const uint32_t lt = blockIdx.x * blockDim.x + threadIdx.x;
    if (lt >= nthreads) return;
    const RepDesc &rep = reps[r];
    const uint32_t h = lt % rep.Vh;
    const uint32_t t2 = lt / rep.Vh;
    const int p = int(t2 & 1u);
    const uint32_t t3 = t2 >> 1;
    const int mu = int(t3 % uint32_t(D));
    const uint32_t layer = t3 / uint32_t(D);
    Site<D> x;
    x.from_half(rep, h, p, layer);
    mat3<double> u;
    if (mode == 1) {
        set_zero(u);
        u.e[0][0].re = u.e[1][1].re = u.e[2][2].re = 1.0;
    } else {
        const uint32_t lid = ((rep.lat2test ? 0u : layer * rep.V) + x.s) * uint32_t(D) + uint32_t(mu);
        double uu[12];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint4 w = philox4x32_10(make_uint4(lid, 0u, uint32_t(j), kTagStart), rep.key0, rep.key1);
            uu[4 * j + 0] = u01(w.x);
            uu[4 * j + 1] = u01(w.y);
            uu[4 * j + 2] = u01(w.z);
            uu[4 * j + 3] = u01(w.w);
        }
        double g[12];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double rho = sqrt(-2.0 * log(uu[2 * k]));
            double sn, cs;
            sincospi(2.0 * uu[2 * k + 1], &sn, &cs);  // sin, cos of 2 pi u
            g[2 * k] = rho * cs;
            g[2 * k + 1] = rho * sn;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u.e[0][c] = cx<double>{g[2 * c], g[2 * c + 1]};
            u.e[1][c] = cx<double>{g[6 + 2 * c], g[7 + 2 * c]};
        }
        reunitarize(u);
    }
    store_link<PREC>(link_ref<D, PREC>(links, rep, layer, mu, p, x.s), u);
}

// ---------------------------------------------------------------------------
// canonical <-> internal

template <int D>
__device__ __forceinline__ void site_from_number(const RepDesc &rep, uint32_t s, Site<D> &x, int &p)
{
    int sum = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        x.x[i] = int((s / rep.stride[i]) % uint32_t(rep.n[i]));
        sum += x.x[i];
    }
    x.s = s;
    x.set_edges(rep);
    p = sum & 1;
}

template <int D, int PREC>
__global__ void __launch_bounds__(256) pack_kernel(const void *links, const RepDesc *reps, int r, uint64_t c0,
                                                    uint32_t count, double *dst)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const RepDesc &rep = reps[r];
    const uint64_t f = c0 + t;
    const uint32_t layer = uint32_t(f / rep.V);
    const uint32_t s = uint32_t(f - uint64_t(layer) * rep.V);
    Site<D> x;
    int p;
    site_from_number<D>(rep, s, x, p);
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const mat3<double> u = widen<double>(
            load_link<PREC>(link_ref<D, PREC>(const_cast<void *>(links), rep, layer, mu, p, s)));
        double *o = dst + (size_t(t) * D + mu) * 18;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            o[2 * e] = u.e[e / 3][e % 3].re;
            o[2 * e + 1] = u.e[e / 3][e % 3].im;
        }
    }
}

template <int D, int PREC>
__global__ void __launch_bounds__(256) unpack_kernel(void *links, const RepDesc *reps, int r, uint64_t c0,
                                                      uint32_t count, const double *src)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const RepDesc &rep = reps[r];
    const uint64_t f = c0 + t;
    const uint32_t layer = uint32_t(f / rep.V);
    const uint32_t s = uint32_t(f - uint64_t(layer) * rep.V);
    Site<D> x;
    int p;
    site_from_number<D>(rep, s, x, p);
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double *in = src + (size_t(t) * D + mu) * 18;
        mat3<double> u;
#pragma unroll
        for (int e = 0; e < 9; ++e) u.e[e / 3][e % 3] = cx<double>{in[2 * e], in[2 * e + 1]};
        store_link<PREC>(link_ref<D, PREC>(links, rep, layer, mu, p, s), u);
    }
}

#define SU3HB_DISPATCH(KERNEL, ...)                                                        \
    switch (D) {                                                                            \
    case 2: SU3HB_PREC(KERNEL, 2, __VA_ARGS__)                                             \
    case 3: SU3HB_PREC(KERNEL, 3, __VA_ARGS__)                                             \
    case 4: SU3HB_PREC(KERNEL, 4, __VA_ARGS__)                                             \
    case 5: SU3HB_PREC(KERNEL, 5, __VA_ARGS__)                                             \
    case 6: SU3HB_PREC(KERNEL, 6, __VA_ARGS__)                                             \
    default: return hipErrorInvalidValue;                                                  \
    }
#define SU3HB_PREC(KERNEL, DD, ...)                                                        \
    switch (prec) {                                                                        \
    case kFP64_18: hipLaunchKernelGGL((KERNEL<DD, kFP64_18>), __VA_ARGS__); break;         \
    case kFP32_18: hipLaunchKernelGGL((KERNEL<DD, kFP32_18>), __VA_ARGS__); break;         \
    case kFP32_12: hipLaunchKernelGGL((KERNEL<DD, kFP32_12>), __VA_ARGS__); break;         \
    case kFP64_12: hipLaunchKernelGGL((KERNEL<DD, kFP64_12>), __VA_ARGS__); break;         \
    default: return hipErrorInvalidValue;                                                  \
    }                                                                                      \
    break;

hipError_t launch_start(int D, int prec, hipStream_t st, void *links, const RepDesc *reps, int r,
                        uint32_t nthreads, int mode)
{
    if (nthreads == 0) return hipSuccess;
    const dim3 g((nthreads + 255) / 256), b(256);
    SU3HB_DISPATCH(start_kernel, g, b, 0, st, links, reps, r, nthreads, mode)
    return hipGetLastError();
}

hipError_t launch_pack(int D, int prec, hipStream_t st, const void *links, const RepDesc *reps, int r,
                       uint64_t c0, uint32_t count, double *dst)
{
    if (count == 0) return hipSuccess;
    const dim3 g((count + 255) / 256), b(256);
    SU3HB_DISPATCH(pack_kernel, g, b, 0, st, links, reps, r, c0, count, dst)
    return hipGetLastError();
}

hipError_t launch_unpack(int D, int prec, hipStream_t st, void *links, const RepDesc *reps, int r,
                         uint64_t c0, uint32_t count, const double *src)
{
    if (count == 0) return hipSuccess;
    const dim3 g((count + 255) / 256), b(256);
    SU3HB_DISPATCH(unpack_kernel, g, b, 0, st, links, reps, r, c0, count, src)
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// validation of canonical input

__global__ void __launch_bounds__(256) validate_kernel(const double *src, uint64_t nmat,
                                                        unsigned long long *maxdef)
{
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double d = 0.0;
    if (t < nmat) {
        const double *in = src + t * 18;
        mat3<double> u;
        bool finite = true;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            u.e[e / 3][e % 3] = cx<double>{in[2 * e], in[2 * e + 1]};
            finite = finite && isfinite(in[2 * e]) && isfinite(in[2 * e + 1]);
        }
        if (!finite) {
            d = __builtin_inf();
        } else {
            const mat3<double> uu = mul_na(u, u);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double re = uu.e[i][j].re - (i == j ? 1.0 : 0.0);
                    d = fmax(d, fmax(fabs(re), fabs(uu.e[i][j].im)));
                }
            // det via the first row and the cofactors
            cx<double> m0{0, 0}, m1{0, 0}, m2{0, 0};
            cfma(m0, u.e[1][1], u.e[2][2]);
            cfma(m0, cx<double>{-u.e[1][2].re, -u.e[1][2].im}, u.e[2][1]);
            cfma(m1, u.e[1][2], u.e[2][0]);
            cfma(m1, cx<double>{-u.e[1][0].re, -u.e[1][0].im}, u.e[2][2]);
            cfma(m2, u.e[1][0], u.e[2][1]);
            cfma(m2, cx<double>{-u.e[1][1].re, -u.e[1][1].im}, u.e[2][0]);
            cx<double> det{0, 0};
            cfma(det, u.e[0][0], m0);
            cfma(det, u.e[0][1], m1);
            cfma(det, u.e[0][2], m2);
            d = fmax(d, sqrt((det.re - 1.0) * (det.re - 1.0) + det.im * det.im));
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off));
    if ((threadIdx.x & 63) == 0) atomicMax(maxdef, (unsigned long long)__double_as_longlong(d));
}

hipError_t launch_validate(hipStream_t st, const double *src, uint64_t nmat, unsigned long long *maxdef)
{
    if (nmat == 0) return hipSuccess;
    hipLaunchKernelGGL(validate_kernel, dim3(uint32_t((nmat + 255) / 256)), dim3(256), 0, st, src, nmat,
                       maxdef);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// statistics and counters

__global__ void stats_zero_kernel(StatSlot *slots)
{
    StatSlot &s = slots[threadIdx.x];
    for (int i = 0; i < 3; ++i) {
        s.attempts[i] = 0;
        s.accepts[i] = 0;
    }
    s.updates = 0;
    s.dtrace = 0.0;
}

__global__ void stats_reduce_kernel(const StatSlot *slots, StatSlot *out)
{
    __shared__ unsigned long long si[kStatSlots][7];
    __shared__ double sd[kStatSlots];
    const int t = threadIdx.x;
    for (int i = 0; i < 3; ++i) {
        si[t][i] = slots[t].attempts[i];
        si[t][3 + i] = slots[t].accepts[i];
    }
    si[t][6] = slots[t].updates;
    sd[t] = slots[t].dtrace;
    __syncthreads();
    for (int w = kStatSlots / 2; w > 0; w >>= 1) {
        if (t < w) {
            for (int i = 0; i < 7; ++i) si[t][i] += si[t + w][i];
            sd[t] += sd[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int i = 0; i < 3; ++i) {
            out->attempts[i] = si[0][i];
            out->accepts[i] = si[0][3 + i];
        }
        out->updates = si[0][6];
        out->dtrace = sd[0];
    }
}

__global__ void counter_add_kernel(uint32_t *ctr, uint32_t add)
{
    if (threadIdx.x == 0) atomicAdd(ctr, add);
}

__global__ void counter_set_kernel(uint32_t *ctr, uint32_t value)
{
    if (threadIdx.x == 0) atomicExch(ctr, value);
}

__global__ void u32_zero_kernel(uint32_t *p, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}

__global__ void u64_zero_kernel(unsigned long long *p, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) atomicExch(&p[t], 0ull);
}

// One replica descriptor, passed by value, written to device memory (so a
// captured graph carries the descriptor in its kernel arguments).
__global__ void rep_set_kernel(RepDesc r, RepDesc *dst)
{
    if (threadIdx.x == 0) *dst = r;
}

hipError_t launch_rep_set(hipStream_t st, const RepDesc &r, RepDesc *dst)
{
    hipLaunchKernelGGL(rep_set_kernel, dim3(1), dim3(64), 0, st, r, dst);
    return hipGetLastError();
}

hipError_t launch_stats_zero(hipStream_t st, StatSlot *slots)
{
    hipLaunchKernelGGL(stats_zero_kernel, dim3(1), dim3(kStatSlots), 0, st, slots);
    return hipGetLastError();
}

hipError_t launch_stats_reduce(hipStream_t st, const StatSlot *slots, StatSlot *out)
{
    hipLaunchKernelGGL(stats_reduce_kernel, dim3(1), dim3(kStatSlots), 0, st, slots, out);
    return hipGetLastError();
}

hipError_t launch_counter_add(hipStream_t st, uint32_t *ctr, uint32_t add)
{
    hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, st, ctr, add);
    return hipGetLastError();
}

hipError_t launch_counter_set(hipStream_t st, uint32_t *ctr, uint32_t value)
{
    hipLaunchKernelGGL(counter_set_kernel, dim3(1), dim3(64), 0, st, ctr, value);
    return hipGetLastError();
}

hipError_t launch_u32_zero(hipStream_t st, uint32_t *p, int n)
{
    hipLaunchKernelGGL(u32_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_u64_zero(hipStream_t st, unsigned long long *p, int n)
{
    hipLaunchKernelGGL(u64_zero_kernel, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace su3hb
