// update.hip -- the checkerboard slice update: for one colour p and one
// direction mu, every link U_mu(x) with parity(x) = p in every layer of every
// replica receives one Cabibbo-Marinari heatbath update (paper Sec. 1, 2.1):
//   staple A (beta-weighted, Sec. 2.2 tag rule) -> W = U A ->
//   SU(2) subgroups (0,1), (0,2), (1,2): project W, Kennedy-Pendleton draw of
//   x0 in multi-hit form (at most n_hit proposals; none accepted keeps the
//   link), random direction, U <- R U, W <- R W ->
//   Gram-Schmidt reunitarisation -> store,
// accumulating the change of sum_p beta_p Re Tr U_p / 3 and the counters.
// The links of one slice are independent (Sec. 2), so one thread owns one
// link and the slice is one launch.

#include "geometry.h"
#include "kernels.h"

namespace su3hb {

// 1/k for the norm k = sqrt(k2) of a projected SU(2) block; false for a
// degenerate projection (k <= 1e-300), which no hit accepts.  Norms from
// 2^-500 up take rsqrt_refined; smaller ones the exact square root, so the
// degenerate test is the one of the definition.
__device__ __forceinline__ bool inv_norm(double k2, double &ik)
{
    if (k2 >= 0x1p-1000) {
        ik = rsqrt_refined(k2);
        return true;
    }
    const double k = sqrt(k2);
    if (!(k > 1e-300)) return false;
    ik = 1.0 / k;
    return true;
}

// The logarithm table of log_unit, copied into LDS by every update kernel
// before its first draw (fill_log_table: all threads of the block).
__shared__ LogEntry s_log_table[128];

__device__ __forceinline__ void fill_log_table()
{
    for (uint32_t i = threadIdx.x; i < 128u; i += blockDim.x) s_log_table[i] = kLogTable[i];
    __syncthreads();
}

// U <- R_IJ(r) U and W <- R_IJ(r) W: the 2x2 matrix r mixes rows I and J.
template <typename H, int I, int J>
__device__ __forceinline__ void rotate_rows(mat3<H> &U, mat3<H> &W, const cx<H> &r00, const cx<H> &r01,
                                            const cx<H> &r10, const cx<H> &r11)
{
    const H z = H(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<H> ui = U.e[I][c], uj = U.e[J][c];
        cx<H> ni{z, z}, nj{z, z};
        cfma(ni, r00, ui); cfma(ni, r01, uj);
        cfma(nj, r10, ui); cfma(nj, r11, uj);
        U.e[I][c] = ni;
        U.e[J][c] = nj;
        const cx<H> wi = W.e[I][c], wj = W.e[J][c];
        cx<H> mi{z, z}, mj{z, z};
        cfma(mi, r00, wi); cfma(mi, r01, wj);
        cfma(mj, r10, wi); cfma(mj, r11, wj);
        W.e[I][c] = mi;
        W.e[J][c] = mj;
    }
}

// One SU(2)-subgroup heatbath on rows (I, J) of U (and W = U A), with U, W
// and the rotation in H (double for FP64 storage, float for FP32 storage).
// The quaternion components of the block are formed in H (the precision W
// is held in) and widened; the norm k, alpha and the Kennedy-Pendleton draw
// and acceptance test are FP64 in every mode.
template <typename H, int I, int J, int SUB>
__device__ __forceinline__ void su2_heatbath(mat3<H> &U, mat3<H> &W, uint32_t lid, uint32_t sweep, int nhit,
                                             uint32_t k0, uint32_t k1, int &attempts, int &accepts)
{
    // quaternion part a0 + i a.sigma of the 2x2 block (I, J) of W
    const double a0 = double(H(0.5) * (W.e[I][I].re + W.e[J][J].re));
    const double a1 = double(H(0.5) * (W.e[I][J].im + W.e[J][I].im));
    const double a2 = double(H(0.5) * (W.e[I][J].re - W.e[J][I].re));
    const double a3 = double(H(0.5) * (W.e[I][I].im - W.e[J][J].im));
    // alpha = 2k/3; the draw multiplies by 1/alpha = 1.5/k, computed once
    double ik;
    if (!inv_norm(fma(a0, a0, fma(a1, a1, fma(a2, a2, a3 * a3))), ik)) return;  // degenerate: every hit rejected
    const double inv_alpha = 1.5 * ik;

    // multi-hit Kennedy-Pendleton: delta = 1 - x0 ~ sqrt(delta) exp(-alpha delta),
    // accepted with probability sqrt(1 - delta/2)
    int hit = 0;
    bool ok = false;
    double delta = 0.0;
    for (; hit < nhit; ++hit) {
        const uint4 r = philox4x32_10(
            make_uint4(lid, sweep, (uint32_t(SUB) << 16) | (uint32_t(hit) << 1), kTagUpdate), k0, k1);
        ++attempts;
        const double c2 = cos2_turn(u01(r.y));  // cos^2(2 pi u)
        delta = -(log_unit(u01(r.x), s_log_table) + c2 * log_unit(u01(r.z), s_log_table)) * inv_alpha;
        const double r4 = u01(r.w);
        if (r4 * r4 <= 1.0 - 0.5 * delta) {
            ok = true;
            break;
        }
    }
    if (!ok) return;
    ++accepts;
    const double x0d = 1.0 - delta;

    // (x1, x2, x3) uniform on the sphere of radius sqrt(1 - x0^2)
    const uint4 q = philox4x32_10(
        make_uint4(lid, sweep, (uint32_t(SUB) << 16) | (uint32_t(hit) << 1) | 1u, kTagUpdate), k0, k1);
    const H x0 = H(x0d);
    const H rad = sqrt_nonneg<H>(H(fmax(0.0, 1.0 - x0d * x0d)));
    const H cth = H(2.0 * u01(q.x) - 1.0);
    const H sth = sqrt_nonneg<H>(max(H(0), H(1) - cth * cth));
    H sph, cph;
    sincos_turn<H>(u01(q.y), &sph, &cph);  // phi = 2 pi u
    const H x1 = rad * sth * cph, x2 = rad * sth * sph, x3 = rad * cth;

    // r = X V^dag, X = [[x0 + i x3, x2 + i x1], [-x2 + i x1, x0 - i x3]],
    // V^dag = [[a0 - i a3, -a2 - i a1], [a2 - i a1, a0 + i a3]] / k
    const H b0 = H(a0 * ik), b1 = H(a1 * ik), b2 = H(a2 * ik), b3 = H(a3 * ik);
    const cx<H> X00{x0, x3}, X01{x2, x1}, X10{-x2, x1}, X11{x0, -x3};
    const cx<H> V00{b0, -b3}, V01{-b2, -b1}, V10{b2, -b1}, V11{b0, b3};
    const H z = H(0);
    cx<H> r00{z, z}, r01{z, z}, r10{z, z}, r11{z, z};
    cfma(r00, X00, V00); cfma(r00, X01, V10);
    cfma(r01, X00, V01); cfma(r01, X01, V11);
    cfma(r10, X10, V00); cfma(r10, X11, V10);
    cfma(r11, X10, V01); cfma(r11, X11, V11);

    rotate_rows<H, I, J>(U, W, r00, r01, r10, r11);
}

// Overrelaxation on rows (I, J): the reflection that keeps Re Tr(U A).  With
// the block of W = U A equal to k V (V in SU(2)) the block becomes k V^dag:
// U <- R_IJ(r) U with r = V^dag V^dag.  The projection is FP64 as in the
// heatbath; the rotation is in H.  No random numbers.
template <typename H, int I, int J>
__device__ __forceinline__ void su2_reflect(mat3<H> &U, mat3<H> &W, int &attempts, int &accepts)
{
    const double a0 = double(H(0.5) * (W.e[I][I].re + W.e[J][J].re));
    const double a1 = double(H(0.5) * (W.e[I][J].im + W.e[J][I].im));
    const double a2 = double(H(0.5) * (W.e[I][J].re - W.e[J][I].re));
    const double a3 = double(H(0.5) * (W.e[I][I].im - W.e[J][J].im));
    double ik;
    if (!inv_norm(fma(a0, a0, fma(a1, a1, fma(a2, a2, a3 * a3))), ik)) return;  // degenerate: no reflection
    ++attempts;
    ++accepts;
    const double b0 = a0 * ik, b1 = a1 * ik, b2 = a2 * ik, b3 = a3 * ik;
    // V^dag = [[b0 - i b3, -b2 - i b1], [b2 - i b1, b0 + i b3]], r = V^dag V^dag
    const cx<double> V00{b0, -b3}, V01{-b2, -b1}, V10{b2, -b1}, V11{b0, b3};
    cx<double> q00{0.0, 0.0}, q01{0.0, 0.0}, q10{0.0, 0.0}, q11{0.0, 0.0};
    cfma(q00, V00, V00); cfma(q00, V01, V10);
    cfma(q01, V00, V01); cfma(q01, V01, V11);
    cfma(q10, V10, V00); cfma(q10, V11, V10);
    cfma(q11, V10, V01); cfma(q11, V11, V11);
    rotate_rows<H, I, J>(U, W, cx<H>{H(q00.re), H(q00.im)}, cx<H>{H(q01.re), H(q01.im)},
                         cx<H>{H(q10.re), H(q10.im)}, cx<H>{H(q11.re), H(q11.im)});
}

// Update one link.  On a single-layer lattice every plaquette carries beta0,
// so the staple is summed unweighted and scaled once; on two layers each
// staple gets the beta of its plaquette (tag rule).
//
// Fused measurement (single layer, parity 1, a.meas set): in slice (1, mu)
// the staple terms of the planes (nu, mu) with nu < mu contain only links
// that are final for this sweep once U_mu(x) is updated (directions below mu
// finished their parity-1 slice, even-site U_mu finished in parity 0), and
// every plaquette of such a plane holds exactly one odd-site U_mu link.  So
// (1/3) Re Tr(U'_mu(x) A_{nu<mu}(x)) summed over the parity-1 slices counts
// every plaquette of the end-of-sweep configuration exactly once.
//
// Two layers (NC = 3, a kernel instantiated for measured parity-1 slices of
// two-layer lattices): the unweighted forward and backward terms of the
// planes nu < mu go to three classes, by the layer of the plaquette's base
// site and its tag sum: 0 = base in layer 0 with all links in layer 0 (beta0),
// 1 = base in layer 0 otherwise (beta1), 2 = base in layer 1 (beta1), so that
// the layer averages and the beta-weighted sum follow from the class sums.
template <int D, int PREC, int NC>
__device__ __forceinline__ void update_link(const UpdateArgs &a, const RepDesc &rep, uint32_t lt,
                                            uint32_t sweep, int att[3], int acc[3], double &dtrace,
                                            double *plaq, const cx<typename Store<PREC>::real> *stg,
                                            int32_t stg_lo)
{
    using R = typename Store<PREC>::real;
    const int p = a.parity, q = 1 - a.parity, mu = a.mu;
    const uint32_t Vh = rep.Vh;
    uint32_t layer = 0, h = lt;
    if (h >= Vh) {
        layer = 1;
        h -= Vh;
    }
    Site<D> x;
    // FP32-12 on single-layer lattices, the kernel bound by its vector ALU
    // work, takes the multipliers; the others keep the division, which holds
    // their register counts (FP32-18 and the two-layer FP32-12 measurement
    // sit at the 128 registers of 4 waves per SIMD)
    x.template from_half<PREC == kFP32_12 && NC == 1>(rep, h, p, layer);
    const bool single = rep.nlat == 1;
    const uint32_t glued = single ? 0u : rep.glued;
    const double beta0 = a.use_rep_beta ? rep.beta0 : a.beta0;
    const double beta1 = a.use_rep_beta ? rep.beta1 : a.beta1;
    const bool measure = a.meas != nullptr && p == 1 && (NC == 3 || single);

    // staple sum A = sum_{nu != mu} beta_f U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    //                             + beta_b U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
    const Step fm = step_fwd<D>(rep, x, mu, glued);
    const uint32_t s_pm = x.s + uint32_t(fm.ds), l_pm = layer ^ fm.flip;
    // the unweighted sum of the planes nu < mu (NC = 1), or its NC class
    // sums, waits in this thread's slots of dynamic LDS (element-major, sized
    // by the launch when measuring)
    extern __shared__ char s_dyn[];
    cx<R> *alow = reinterpret_cast<cx<R> *>(s_dyn);
    const uint32_t bd = blockDim.x, tid = threadIdx.x;
    if constexpr (NC == 3) {
        if (measure) {
#pragma unroll
            for (int e = 0; e < 27; ++e) alow[e * bd + tid] = cx<R>{R(0), R(0)};
        }
    }
    mat3<R> A;
    set_zero(A);
#pragma unroll
    for (int nu = 0; nu < D; ++nu) {
        if (nu == mu) {
            if constexpr (NC == 1) {
                if (measure) {
#pragma unroll
                    for (int e = 0; e < 9; ++e) alow[e * bd + tid] = A.e[e / 3][e % 3];
                }
            }
            continue;
        }
        const Step fn = step_fwd<D>(rep, x, nu, glued);
        const Step bn = step_bwd<D>(rep, x, nu, glued);
        const uint32_t s_pn = x.s + uint32_t(fn.ds), l_pn = layer ^ fn.flip;
        const uint32_t s_mn = x.s + uint32_t(bn.ds), l_mn = layer ^ bn.flip;
        const uint32_t s_pmmn = s_pm + uint32_t(bn.ds), l_pmmn = l_pm ^ bn.flip;

        const uint32_t tags_f = layer + l_pm + l_pn + layer;
        const uint32_t tags_b = l_mn + l_pmmn + layer + l_mn;
        // U_mu(x + nu) and U_mu(x - nu): from the wave's staging area for
        // nu = 0, 1 when the launch stages (single-layer lattices only).
        // A parity-q U_mu link is read by six threads (F2 of x - nu, B2 of
        // x + nu); one whole read suffices: the first plane other than mu
        // (nu = 0, or 1 when mu = 0) reads F2 whole, the others read rows 0
        // and 1 like B2.
        const bool f2_rows = nu >= 2 || (nu == 1 && mu != 0);
        LinkSrc<PREC> f2 = from_global<PREC>(link_ref<D, PREC>(a.links, rep, l_pn, mu, q, s_pn), f2_rows);
        LinkSrc<PREC> b2 = from_global<PREC>(link_ref<D, PREC>(a.links, rep, l_mn, mu, q, s_mn));
        if (nu < 2 && stg != nullptr) {
            const uint32_t nslot = 64u + 2u * a.stage_r;
            f2.stg = stg;
            f2.slot = uint32_t(int32_t(s_pn >> 1) - stg_lo);
            f2.nslot = nslot;
            b2.stg = stg;
            b2.slot = uint32_t(int32_t(s_mn >> 1) - stg_lo);
            b2.nslot = nslot;
        }
        if constexpr (NC == 3) {
            if (measure && nu < mu) {
                const int cf = layer == 0 ? (tags_f == 0 ? 0 : 1) : 2;
                const int cb = l_mn == 0 ? (tags_b == 0 ? 0 : 1) : 2;
                acc_plane_staples<PREC, true>(A, link_ref<D, PREC>(a.links, rep, l_pm, nu, q, s_pm), f2,
                                              link_ref<D, PREC>(a.links, rep, layer, nu, p, x.s),
                                              link_ref<D, PREC>(a.links, rep, l_pmmn, nu, p, s_pmmn), b2,
                                              link_ref<D, PREC>(a.links, rep, l_mn, nu, q, s_mn),
                                              single ? R(1) : R(tags_f == 0 ? beta0 : beta1),
                                              single ? R(1) : R(tags_b == 0 ? beta0 : beta1), alow, bd, tid,
                                              cf, cb);
                continue;
            }
        }
        acc_plane_staples<PREC>(A, link_ref<D, PREC>(a.links, rep, l_pm, nu, q, s_pm), f2,
                                link_ref<D, PREC>(a.links, rep, layer, nu, p, x.s),
                                link_ref<D, PREC>(a.links, rep, l_pmmn, nu, p, s_pmmn), b2,
                                link_ref<D, PREC>(a.links, rep, l_mn, nu, q, s_mn),
                                single ? R(1) : R(tags_f == 0 ? beta0 : beta1),
                                single ? R(1) : R(tags_b == 0 ? beta0 : beta1));
    }
    if (single) scale(A, R(beta0));

    // heatbath in the storage precision (FP64 for the draw, see su2_heatbath)
    const LinkRef uptr = link_ref<D, PREC>(a.links, rep, layer, mu, p, x.s);
    mat3<R> U = load_link<PREC, true>(uptr);   // no other thread of the slice reads U
    mat3<R> W = mul_nn(U, A);   // A is not needed past this point
    const double tr_old = double(W.e[0][0].re) + double(W.e[1][1].re) + double(W.e[2][2].re);

    const uint32_t lid = ((rep.lat2test ? 0u : layer * rep.V) + x.s) * uint32_t(D) + uint32_t(mu);
    if (a.nhit > 0) {
        su2_heatbath<R, 0, 1, 0>(U, W, lid, sweep, a.nhit, rep.key0, rep.key1, att[0], acc[0]);
        su2_heatbath<R, 0, 2, 1>(U, W, lid, sweep, a.nhit, rep.key0, rep.key1, att[1], acc[1]);
        su2_heatbath<R, 1, 2, 2>(U, W, lid, sweep, a.nhit, rep.key0, rep.key1, att[2], acc[2]);
    } else {  // n_hit 0: overrelaxation sweep
        su2_reflect<R, 0, 1>(U, W, att[0], acc[0]);
        su2_reflect<R, 0, 2>(U, W, att[1], acc[1]);
        su2_reflect<R, 1, 2>(U, W, att[2], acc[2]);
    }
    // W was rotated with U, so Re Tr W is now Re Tr(U' A)
    dtrace += (double(W.e[0][0].re) + double(W.e[1][1].re) + double(W.e[2][2].re) - tr_old) * (1.0 / 3.0);
    // reunitarisation in FP64 in every mode
    mat3<double> Ud = widen<double>(U);
    reunitarize(Ud);
    if (measure) {
        // the link as it will be read back, times the snapshot staple: each
        // link's trace in the storage precision, the sums in FP64
        const mat3<R> Us = stored_form_r<PREC>(Ud);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            mat3<R> M;
#pragma unroll
            for (int e = 0; e < 9; ++e) M.e[e / 3][e % 3] = alow[(c * 9 + e) * bd + tid];
            plaq[c] += double(re_tr_nn(Us, M)) * (1.0 / 3.0);
        }
    }
    store_link<PREC>(uptr, Ud);
}

// Sum the per-thread counters over the block and add them to one slot; with
// a fused measurement also store the block's NC plaquette class sums (plain
// stores, one group per (direction, block), added up later in a fixed order).
template <int NC>
__device__ __forceinline__ void flush_stats(const UpdateArgs &a, uint32_t lb, int att[3], int acc[3], int upd,
                                            double dtrace, double *plaq)
{
    int v[7] = {att[0], att[1], att[2], acc[0], acc[1], acc[2], upd};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < 7; ++i) v[i] += __shfl_xor(v[i], off);
        dtrace += __shfl_xor(dtrace, off);
#pragma unroll
        for (int c = 0; c < NC; ++c) plaq[c] += __shfl_xor(plaq[c], off);
    }
    __shared__ int s_int[kPersistentThreads / 64][7];
    __shared__ double s_dbl[kPersistentThreads / 64][1 + NC];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 7; ++i) s_int[wave][i] = v[i];
        s_dbl[wave][0] = dtrace;
#pragma unroll
        for (int c = 0; c < NC; ++c) s_dbl[wave][1 + c] = plaq[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 1; w < nw; ++w) {
#pragma unroll
            for (int i = 0; i < 7; ++i) v[i] += s_int[w][i];
            dtrace += s_dbl[w][0];
#pragma unroll
            for (int c = 0; c < NC; ++c) plaq[c] += s_dbl[w][1 + c];
        }
        StatSlot *sl = &a.stats[lb % kStatSlots];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            atomicAdd(&sl->attempts[i], (unsigned long long)v[i]);
            atomicAdd(&sl->accepts[i], (unsigned long long)v[3 + i]);
        }
        atomicAdd(&sl->updates, (unsigned long long)v[6]);
        unsafeAtomicAdd(&sl->dtrace, dtrace);
        if (a.meas != nullptr && a.parity == 1 && lb < a.total_blocks)
#pragma unroll
            for (int c = 0; c < NC; ++c) a.meas[(size_t(a.mu) * a.total_blocks + lb) * NC + c] = plaq[c];
    }
    __syncthreads();  // the shared arrays are reused by the next block in a persistent loop
}

// Update the links of logical block lb (replica found by binary search),
// adding to the thread's counters; lt_override >= 0 gives the thread's link
// directly (order 3).
// Staging of the U_mu neighbours along directions 0 and 1 (launches with
// a.stage, single-layer lattices, launch orders that give every wave 64
// consecutive half-lattice indices hw .. hw + 63).  A step along direction
// 0 moves h by at most n_0/2 - 1 (the wrap stays in the row), one along
// direction 1 by exactly n_0/2 unless it wraps, so the parity-q U_mu links
// that the wave's planes nu = 0, 1 read lie in h = hw - R .. hw + 63 + R,
// R = n_0/2, except after a wrap along direction 1.  Every lane of the wave
// (also lanes past the end of the lattice) copies its share of that range
// into the wave's staging area once; the staple then reads those links from
// LDS and the few outside the range from global memory.  The slice does not
// write these links (it writes parity p), so both give the same values.
// Returns the wave's staging area; stg_lo = hw - R.
template <int D, int PREC>
__device__ __forceinline__ const cx<typename Store<PREC>::real> *stage_wave(const UpdateArgs &a, const RepDesc &rep,
                                                                           uint32_t lt, int32_t &stg_lo)
{
    using R = typename Store<PREC>::real;
    constexpr int NE = Store<PREC>::NE;
    extern __shared__ char s_dyn[];
    const uint32_t lane = threadIdx.x & 63u, nslot = 64u + 2u * a.stage_r;
    // the staging areas follow the staple snapshots of a measuring launch
    const uint32_t snap = (a.meas != nullptr && a.parity == 1) ? blockDim.x * 9u * uint32_t(a.meas_classes) : 0u;
    cx<R> *stg = reinterpret_cast<cx<R> *>(s_dyn) + snap + size_t(threadIdx.x >> 6) * nslot * NE;
    stg_lo = int32_t(lt - lane) - int32_t(a.stage_r);
    const int q = 1 - a.parity;
    for (uint32_t slot = lane; slot < nslot; slot += 64u) {
        const int32_t h = stg_lo + int32_t(slot);
        if (h >= 0 && uint32_t(h) < rep.Vh) {
            const mat3<R> m = load_stored<PREC>(link_ref<D, PREC>(a.links, rep, 0u, a.mu, q, 2u * uint32_t(h)));
#pragma unroll
            for (int e = 0; e < NE; ++e) stg[e * nslot + slot] = m.e[e / 3][e % 3];
        }
    }
    // the wave's LDS operations complete in order: after the stores, any lane
    // of the wave reads what the others wrote
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return stg;
}

template <int D, int PREC, int NC>
__device__ __forceinline__ void block_links(const UpdateArgs &a, uint32_t lb, uint32_t sweep, int att[3], int acc[3],
                                            int &upd, double &dtrace, double *plaq, int64_t lt_override = -1)
{
    if (lb < a.total_blocks) {
        const int kind = a.persistent ? kPersistentBlocks : kUpdateBlocks;
        const int r = a.nrep == 1 ? 0 : find_replica(a.reps, a.nrep, lb, kind);
        const RepDesc &rep = a.reps[r];
        const uint32_t lt = lt_override >= 0 ? uint32_t(lt_override)
                                             : (lb - first_block(rep, kind)) * blockDim.x + threadIdx.x;
        const cx<typename Store<PREC>::real> *stg = nullptr;
        int32_t stg_lo = 0;
        if constexpr (NC == 1) {
            if (a.stage) stg = stage_wave<D, PREC>(a, rep, lt, stg_lo);
        }
        if (lt < rep.nlat * rep.Vh) {
            update_link<D, PREC, NC>(a, rep, lt, sweep, att, acc, dtrace, plaq, stg, stg_lo);
            ++upd;
        }
    }
}

// One logical block of a per-slice launch, its counters flushed at the end.
template <int D, int PREC, int NC>
__device__ __forceinline__ void process_block(const UpdateArgs &a, uint32_t lb, uint32_t sweep,
                                              int64_t lt_override = -1)
{
    int att[3] = {0, 0, 0}, acc[3] = {0, 0, 0}, upd = 0;
    double dtrace = 0.0, plaq[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) plaq[c] = 0.0;
    block_links<D, PREC, NC>(a, lb, sweep, att, acc, upd, dtrace, plaq, lt_override);
    flush_stats<NC>(a, lb, att, acc, upd, dtrace, plaq);
}

// Logical block of hardware block b.  Hardware blocks are dealt round-robin
// to the 8 XCDs.  Order 1 gives each XCD a contiguous run of logical blocks;
// order 2 gives XCD k the slab k of the last direction and walks it with
// that direction fastest, then the blocks of an (x_{D-2}, x_{D-1}) plane,
// then x_{D-2}, so the neighbours of a block along the two slowest
// directions are fetched by blocks that run next to it on the same L2.
__device__ __forceinline__ uint32_t logical_block(const UpdateArgs &a, uint32_t b)
{
    if (a.order == 1) {
        const uint32_t per = gridDim.x >> 3;
        return (b & 7u) * per + (b >> 3);
    }
    if (a.order == 2) {
        const uint32_t k = b & 7u, e = b >> 3;
        const uint32_t xl = e % a.slab, t = e / a.slab;
        const uint32_t c = t % a.cp, x2 = t / a.cp;
        return (x2 + a.n2 * (k * a.slab + xl)) * a.cp + c;
    }
    if (a.order == 4) {
        // as order 2 with the block's chunk of the plane slowest and x_{D-2}
        // in the middle: neighbours along x_{D-2} are one slab apart
        const uint32_t k = b & 7u, e = b >> 3;
        const uint32_t xl = e % a.slab, t = e / a.slab;
        const uint32_t x2 = t % a.n2, c = t / a.n2;
        return (x2 + a.n2 * (k * a.slab + xl)) * a.cp + c;
    }
    return b;
}

// Orders 3, 5 and 6: a block is tile2 x tile3 waves stacked along x_{D-2} and x_{D-1},
// each wave 64 consecutive half-sites of its (x_{D-2}, x_{D-1}) plane, so the
// neighbours along the two slowest directions are loaded by sibling waves at
// nearly the same time.  Blocks walk XCD slabs as in order 2.  Returns the
// half-lattice index of the calling thread's link.
__device__ __forceinline__ uint32_t link_of_thread_3d(const UpdateArgs &a, uint32_t b)
{
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t w2 = w % a.tile2, w3 = w / a.tile2;
    const uint32_t k = b & 7u, e = b >> 3;
    const uint32_t xl = e % a.slab, t = e / a.slab;
    // order 5 walks the x_{D-2} tiles before the chunks of the plane
    const uint32_t nt2 = a.n2 / a.tile2;
    const uint32_t c = a.order == 5 ? t / nt2 : t % a.cp, x2t = a.order == 5 ? t % nt2 : t / a.cp;
    const uint32_t x2 = x2t * a.tile2 + w2;
    const uint32_t x3 = (k * a.slab + xl) * a.tile3 + w3;
    return (x2 + a.n2 * x3) * a.plane + c * 64u + lane;
}

// Order 7 (D = 4): each wave covers a 4D tile, 8 consecutive half-sites
// along x_0 (16 sites) by 2 x 2 x 2 along x_1, x_2, x_3, so that most partner
// links along every direction are loaded by lanes of the same wave (8 lanes
// read one 128-byte line of each packet); the waves of a block stack along
// x_2.  XCD k owns slab k of x_3 and walks it x_3 fastest, then x_2, x_1 and
// the x_0 groups.  Returns the half-lattice index of the calling thread's
// link.
__device__ __forceinline__ uint32_t link_of_thread_4d(const UpdateArgs &a, uint32_t b)
{
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t k = b & 7u, e = b >> 3;
    const uint32_t e3 = e % a.slab, t = e / a.slab;
    const uint32_t nb2 = a.n2 / (2u * nw);
    const uint32_t e2 = t % nb2, t2 = t / nb2;
    const uint32_t nb1 = a.n1 / 2u;
    const uint32_t e1 = t2 % nb1, e0 = t2 / nb1;
    const uint32_t x3 = (k * a.slab + e3) * 2u + (lane >> 5);
    const uint32_t x2 = (e2 * nw + w) * 2u + ((lane >> 4) & 1u);
    const uint32_t x1 = e1 * 2u + ((lane >> 3) & 1u);
    const uint32_t hx = e0 * 8u + (lane & 7u);
    return hx + a.n0h * (x1 + a.n1 * (x2 + a.n2 * x3));
}

// Hardware block b with the walk of every XCD reversed (a.reverse): XCD
// b mod 8 keeps its blocks but takes them last to first.  Alternate slices
// walk back and forth, so a slice starts on the links its predecessor read
// last, while they are still in the last-level cache.
__device__ __forceinline__ uint32_t walk_block(const UpdateArgs &a)
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    if (!a.reverse) return b;
    if ((G & 7u) == 0u) return (b & 7u) | ((G / 8u - 1u - (b >> 3)) << 3);
    return G - 1u - b;
}

template <int D, int PREC, int WAVES, int NC = 1>
__global__ void __launch_bounds__(256, WAVES) update_kernel(UpdateArgs a)
{
    fill_log_table();
    // the launch order only decides which link a thread takes; the update
    // itself is one inlined body for every order
    const uint32_t b = walk_block(a);
    uint32_t lb = b;
    int64_t lt = -1;
    if (a.order == 3 || a.order == 5 || a.order == 6)
        lt = int64_t(link_of_thread_3d(a, b));
    else if (a.order == 7)
        lt = int64_t(link_of_thread_4d(a, b));
    else
        lb = logical_block(a, b);
    process_block<D, PREC, NC>(a, lb, *a.sweep, lt);
}

// Grid barrier of a persistent launch (all blocks resident: cooperative
// launch).  Each block's first thread arrives on one of the leaf counters
// with release semantics; the last arrival of a leaf adds to the top
// counter; everybody waits for the top counter to reach its target for
// generation gen and then acquires.  Counters only grow within a launch, so
// no reset is needed between generations.  A wait that exceeds the spin
// limit, or sees the abort flag, raises the flag and returns false so that
// every block leaves the kernel.
__device__ __forceinline__ bool grid_barrier(uint32_t *bar, uint32_t gen)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t G = gridDim.x, L = G < kBarrierLeaves ? G : kBarrierLeaves, leaf = blockIdx.x % L;
        const uint32_t members = (G - leaf + L - 1) / L;
        const uint32_t old =
            __hip_atomic_fetch_add(bar + leaf * 32u, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == (gen + 1u) * members)
            __hip_atomic_fetch_add(bar + kBarrierTop, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = (gen + 1u) * L;
        int ok = 1;
        uint32_t spins = 0;
        while (__hip_atomic_load(bar + kBarrierTop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(bar + kBarrierFlag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                ++spins > kBarrierSpinLimit) {
                atomicOr(bar + kBarrierFlag, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// XCD of the calling wave (hardware register XCC_ID, 4 bits).
__device__ __forceinline__ uint32_t xcc_id()
{
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kBarrierXcds - 1u);
}

// Wait until *w reaches target (agent-scope loads); false when the abort
// flag is seen (checked every 64 polls) or the spin limit is passed, after
// raising the flag so that every block leaves the kernel.
__device__ __forceinline__ bool wait_word(uint32_t *bar, const uint32_t *w, uint32_t target)
{
    uint32_t spins = 0;
    while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        ++spins;
        if (spins > kBarrierSpinLimit ||
            ((spins & 63u) == 0u &&
             __hip_atomic_load(bar + kBarrierFlag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
            atomicOr(bar + kBarrierFlag, 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Slice barrier of a persistent launch, with one L2 writeback and one L2
// invalidation per XCD instead of one per block.  The XCD's L2 is shared by
// all its blocks but not kept coherent with the other XCDs, so a block's
// stores reach the other XCDs only through a writeback of its XCD's L2, and
// a block sees the other XCDs' stores only after its XCD's L2 has dropped
// its stale lines.  Every wave first waits for its own stores to complete
// into L2; each block then arrives on its XCD's counter; the last arrival
// of an XCD (members: blocks on that XCD, counted at the start) writes the
// L2 back (agent release), arrives on the XCD top counter and waits for the
// release word, which the last XCD sets; it then invalidates the L2 (agent
// acquire) and sets its XCD's go word, on which the other blocks of the XCD
// wait before they drop their compute unit's L1 lines.
__device__ __forceinline__ bool xcd_barrier(uint32_t *bar, uint32_t gen, uint32_t x, uint32_t members,
                                            uint32_t nxcd)
{
    __shared__ int s_ok;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok;
        const uint32_t old =
            __hip_atomic_fetch_add(bar + kBarrierXcdArrive + 32u * x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == (gen + 1u) * members) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t t =
                __hip_atomic_fetch_add(bar + kBarrierXcdTop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t + 1u == (gen + 1u) * nxcd)
                __hip_atomic_store(bar + kBarrierXcdRelease, gen + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = wait_word(bar, bar + kBarrierXcdRelease, gen + 1u);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(bar + kBarrierXcdGo + 32u * x, gen + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = wait_word(bar, bar + kBarrierXcdGo + 32u * x, gen + 1u);
            asm volatile("buffer_inv sc0" ::: "memory");
        }
        s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return s_ok != 0;
}

// Persistent form for batches: every resident block (as many per CU as fit)
// stays for n_sweeps sweeps, loops over the logical blocks of every slice and meets the others
// at a grid barrier between slices (the next slice reads links this one
// wrote).  Blocks are dealt round-robin to the 8 XCDs, so the blocks of XCD k
// walk the k-th eighth of the logical blocks together, keeping neighbouring
// links on one L2.  The sweep number is the counter's value at entry plus
// the local sweep index; the counter itself is advanced once, by the host,
// after the launch.
template <int D, int PREC, int THREADS>
__global__ void __launch_bounds__(THREADS, persistent_waves(PREC)) update_persistent_kernel(UpdateArgs a, int n_sweeps)
{
    fill_log_table();
    // count the blocks of every XCD, then one grid-wide barrier (per-block
    // cache maintenance) before the counts are read
    __shared__ uint32_t s_members, s_nxcd;
    const uint32_t x = xcc_id();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(a.barrier + kBarrierXcdMembers + 32u * x, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(a.barrier, 0)) return;
    if (threadIdx.x == 0) {
        uint32_t n = 0;
        for (uint32_t k = 0; k < kBarrierXcds; ++k)
            n += __hip_atomic_load(a.barrier + kBarrierXcdMembers + 32u * k, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) != 0u ? 1u : 0u;
        s_members = __hip_atomic_load(a.barrier + kBarrierXcdMembers + 32u * x, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
        s_nxcd = n;
    }
    __syncthreads();
    const uint32_t members = s_members, nxcd = s_nxcd;
    const uint32_t sweep0 = *a.sweep;
    const uint32_t G = gridDim.x, T = a.total_blocks;
    uint32_t first = blockIdx.x, last = T, step = G;
    if (G % 8 == 0 && G >= 8) {
        const uint32_t chunk = (T + 7) / 8, k = blockIdx.x & 7u;
        first = k * chunk + (blockIdx.x >> 3);
        last = min(T, (k + 1) * chunk);
        step = G / 8;
    }
    uint32_t gen = 0;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        for (int p = 0; p < 2; ++p) {
            for (int mu = 0; mu < D; ++mu) {
                UpdateArgs b = a;
                b.parity = p;
                b.mu = mu;
                // the waves of the block run freely over the slice; counters
                // are flushed once per slice, next to the barrier's own sync
                int att[3] = {0, 0, 0}, acc[3] = {0, 0, 0}, upd = 0;
                double dtrace = 0.0, plaq[1] = {0.0};
                // alternate slices walk the block's share backwards, so a
                // slice starts on the links its predecessor read last
                const uint32_t n = first < last ? (last - first + step - 1) / step : 0u;
                const bool back = ((p * D + mu) & 1) != 0;
                for (uint32_t j = 0; j < n; ++j) {
                    const uint32_t lb = first + (back ? n - 1u - j : j) * step;
                    block_links<D, PREC, 1>(b, lb, sweep0 + uint32_t(sw), att, acc, upd, dtrace, plaq);
                }
                flush_stats<1>(b, blockIdx.x, att, acc, upd, dtrace, plaq);
                if (!xcd_barrier(a.barrier, gen++, x, members, nxcd)) return;
            }
        }
    }
}

// Dynamic LDS of an update launch: one staple snapshot per thread when the
// launch measures plaquettes (parity-1 slices with a measurement buffer).
template <int PREC>
static size_t update_lds_bytes(dim3 block, const UpdateArgs &a)
{
    using R = typename Store<PREC>::real;
    const size_t snap = (a.meas != nullptr && a.parity == 1) ? size_t(block.x) * 9 * a.meas_classes * sizeof(cx<R>) : 0;
    if (!a.stage) return snap;
    // the staging areas follow the snapshots
    return snap + size_t(block.x / 64u) * (64u + 2u * a.stage_r) * Store<PREC>::NE * sizeof(cx<R>);
}

// The kernel a slice launch uses: the class-splitting form for measured
// parity-1 slices of two-layer lattices, else the form built for `waves`.
template <int D, int PREC>
static const void *update_fn(int waves, const UpdateArgs &a)
{
    if (a.meas != nullptr && a.parity == 1 && a.meas_classes == 3)
        return reinterpret_cast<const void *>(&update_kernel<D, PREC, kDefaultWaves, 3>);
    // parity-0 slices of a measured sweep measure nothing and use this kernel
    if (a.meas != nullptr && a.meas_classes != 1 && a.meas_classes != 3) return nullptr;
    if constexpr (D == 4) {
        if (waves == 3) return reinterpret_cast<const void *>(&update_kernel<D, PREC, 3>);
        if constexpr (PREC == kFP32_18 || PREC == kFP32_12)
            if (waves == 4) return reinterpret_cast<const void *>(&update_kernel<D, PREC, 4>);
    }
    if (waves != kDefaultWaves) return nullptr;
    return reinterpret_cast<const void *>(&update_kernel<D, PREC, kDefaultWaves>);
}

// Per-block LDS limit of the current device (queried once per device).
static size_t lds_limit()
{
    static size_t cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
        cached[dev] = size_t(v);
    }
    return cached[dev];
}

template <int D, int PREC>
static hipError_t update_lds_t(int waves, dim3 block, const UpdateArgs &a, size_t *need, size_t *limit)
{
    const void *fn = update_fn<D, PREC>(waves, a);
    if (!fn) return hipErrorInvalidValue;
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return e;
    *need = attr.sharedSizeBytes + update_lds_bytes<PREC>(block, a);
    *limit = lds_limit();
    return hipSuccess;
}

template <int D, int PREC>
static hipError_t launch_update_t(int waves, dim3 grid, dim3 block, hipStream_t st, const UpdateArgs &a)
{
    const void *fn = update_fn<D, PREC>(waves, a);
    if (!fn) return hipErrorInvalidValue;
    UpdateArgs args = a;
    void *params[] = {&args};
    return hipLaunchKernel(fn, grid, block, params, update_lds_bytes<PREC>(block, a), st);
}

template <int D>
static hipError_t launch_update_d(int prec, int waves, dim3 grid, dim3 block, hipStream_t st,
                                  const UpdateArgs &a)
{
    switch (prec) {
    case kFP64_18: return launch_update_t<D, kFP64_18>(waves, grid, block, st, a);
    case kFP32_18: return launch_update_t<D, kFP32_18>(waves, grid, block, st, a);
    case kFP32_12: return launch_update_t<D, kFP32_12>(waves, grid, block, st, a);
    case kFP64_12: return launch_update_t<D, kFP64_12>(waves, grid, block, st, a);
    default: return hipErrorInvalidValue;
    }
}

template <int D>
static hipError_t update_lds_d(int prec, int waves, dim3 block, const UpdateArgs &a, size_t *need, size_t *limit)
{
    switch (prec) {
    case kFP64_18: return update_lds_t<D, kFP64_18>(waves, block, a, need, limit);
    case kFP32_18: return update_lds_t<D, kFP32_18>(waves, block, a, need, limit);
    case kFP32_12: return update_lds_t<D, kFP32_12>(waves, block, a, need, limit);
    case kFP64_12: return update_lds_t<D, kFP64_12>(waves, block, a, need, limit);
    default: return hipErrorInvalidValue;
    }
}

hipError_t update_lds(int D, int prec, int waves, dim3 block, const UpdateArgs &a, size_t *need, size_t *limit)
{
    switch (D) {
    case 2: return update_lds_d<2>(prec, waves, block, a, need, limit);
    case 3: return update_lds_d<3>(prec, waves, block, a, need, limit);
    case 4: return update_lds_d<4>(prec, waves, block, a, need, limit);
    case 5: return update_lds_d<5>(prec, waves, block, a, need, limit);
    case 6: return update_lds_d<6>(prec, waves, block, a, need, limit);
    default: return hipErrorInvalidValue;
    }
}

static const void *persistent_fn(int D, int prec)
{
#define SU3HB_K(DD, PP) reinterpret_cast<const void *>(&update_persistent_kernel<DD, PP, kPersistentThreads>)
#define SU3HB_P(DD)                                        \
    case DD:                                               \
        switch (prec) {                                    \
        case kFP64_18: return SU3HB_K(DD, kFP64_18);       \
        case kFP32_18: return SU3HB_K(DD, kFP32_18);       \
        case kFP32_12: return SU3HB_K(DD, kFP32_12);       \
        case kFP64_12: return SU3HB_K(DD, kFP64_12);       \
        default: return nullptr;                           \
        }
    switch (D) {
        SU3HB_P(2)
        SU3HB_P(3)
        SU3HB_P(4)
        SU3HB_P(5)
        SU3HB_P(6)
    default: return nullptr;
    }
#undef SU3HB_P
#undef SU3HB_K
}

hipError_t persistent_max_blocks(int D, int prec, int *blocks_per_cu)
{
    const void *fn = persistent_fn(D, prec);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, kPersistentThreads, 0);
}

hipError_t launch_update_persistent(int D, int prec, int blocks, hipStream_t st, const UpdateArgs &a, int n_sweeps)
{
    const void *fn = persistent_fn(D, prec);
    if (!fn || a.barrier == nullptr || !a.persistent) return hipErrorInvalidValue;
    UpdateArgs args = a;
    int ns = n_sweeps;
    void *params[] = {&args, &ns};
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kPersistentThreads), params, 0, st);
}

hipError_t launch_update(int D, int prec, int waves, dim3 grid, dim3 block, hipStream_t st,
                         const UpdateArgs &a)
{
    switch (D) {
    case 2: return launch_update_d<2>(prec, waves, grid, block, st, a);
    case 3: return launch_update_d<3>(prec, waves, grid, block, st, a);
    case 4: return launch_update_d<4>(prec, waves, grid, block, st, a);
    case 5: return launch_update_d<5>(prec, waves, grid, block, st, a);
    case 6: return launch_update_d<6>(prec, waves, grid, block, st, a);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace su3hb
