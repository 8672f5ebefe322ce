// geometry.h -- per-thread lattice geometry for the kernels: coordinates of a
// checkerboard site from its half-lattice index, neighbour site numbers with
// periodic wrap or the layer flip of the double-layered torus, link pointers.
#pragma once

#include "device_math.h"

namespace su3hb {

// Block partitions of the replicas: per-slice update launches, plaquette
// launches, persistent launches.
enum BlockKind { kUpdateBlocks = 0, kPlaquetteBlocks = 1, kPersistentBlocks = 2 };

__device__ __forceinline__ uint32_t first_block(const RepDesc &r, int kind)
{
    return kind == kPlaquetteBlocks ? r.plq_block0 : kind == kPersistentBlocks ? r.pers_block0 : r.upd_block0;
}

// Find the replica owning logical block lb: largest r with first[r] <= lb.
// The block index and the table are uniform, so this runs on scalar units.
__device__ __forceinline__ int find_replica(const RepDesc *__restrict__ reps, int nrep, uint32_t lb, int kind)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const uint32_t first = first_block(reps[mid], kind);
        if (first <= lb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// x / d for x < 2^31 by the multiplier of d (div_magic).
__device__ __forceinline__ uint32_t div_by(uint32_t x, DivMagic dm)
{
    return uint32_t((uint64_t(x) * dm.m) >> dm.s);
}

// A site of parity p given by its half index h (site number s = 2h + b).
// Eq. (i_s) with direction 0 fastest: since n0 is even, sites 2h and 2h+1
// share x1..x_{D-1} and have opposite parity, so h indexes each checkerboard.
template <int D>
struct Site {
    int x[D];
    uint32_t s;
    uint32_t layer;

    // MAGIC: the divisions by the extents use the replica's multipliers (a
    // 64-bit product and a shift each instead of the compiler's expansion of
    // a division by a run-time value, about 16 vector instructions); exact
    // because h < 2^31.
    template <bool MAGIC = false>
    __device__ __forceinline__ void from_half(const RepDesc &rep, uint32_t h, int p, uint32_t lay)
    {
        const uint32_t nh0 = uint32_t(rep.n[0]) >> 1;
        uint32_t rest = MAGIC ? div_by(h, rep.div[0]) : h / nh0;
        const uint32_t hx = h - rest * nh0;
        int psum = p;
#pragma unroll
        for (int i = 1; i < D; ++i) {
            if (i < D - 1) {
                const uint32_t q = MAGIC ? div_by(rest, rep.div[i]) : rest / uint32_t(rep.n[i]);
                x[i] = int(rest - q * uint32_t(rep.n[i]));
                rest = q;
            } else {
                x[i] = int(rest);
            }
            psum += x[i];
        }
        x[0] = int(2 * hx) + (psum & 1);
        s = 2 * h + uint32_t(psum & 1);
        layer = lay;
        set_edges(rep);
    }

    // bit i of hi (lo): x_i is the last (first) coordinate of direction i.
    // Steps along a run-time direction read these bits instead of indexing
    // the coordinate array, which would move it to scratch memory.
    uint32_t hi, lo;

    __device__ __forceinline__ void set_edges(const RepDesc &rep)
    {
        hi = 0;
        lo = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            hi |= uint32_t(x[i] == rep.n[i] - 1) << i;
            lo |= uint32_t(x[i] == 0) << i;
        }
    }
};

// Site-number offset and layer of one step along +dir or -dir.
struct Step {
    int32_t ds;       // change of the site number
    uint32_t flip;    // 1 if the step changes layer
};

template <int D>
__device__ __forceinline__ Step step_fwd(const RepDesc &rep, const Site<D> &x, int dir, uint32_t glued)
{
    const bool wrap = (x.hi >> dir) & 1u;
    Step st;
    st.ds = wrap ? -int32_t((rep.n[dir] - 1) * rep.stride[dir]) : int32_t(rep.stride[dir]);
    st.flip = wrap ? ((glued >> dir) & 1u) : 0u;
    return st;
}

template <int D>
__device__ __forceinline__ Step step_bwd(const RepDesc &rep, const Site<D> &x, int dir, uint32_t glued)
{
    const bool wrap = (x.lo >> dir) & 1u;
    Step st;
    st.ds = wrap ? int32_t((rep.n[dir] - 1) * rep.stride[dir]) : -int32_t(rep.stride[dir]);
    st.flip = wrap ? ((glued >> dir) & 1u) : 0u;
    return st;
}

// Reference to link (layer, dir) at the site with number s and parity par:
// its slab (Vhp links, whole tiles) and its half-lattice index s / 2.
template <int D, int PREC>
__device__ __forceinline__ LinkRef link_ref(void *links, const RepDesc &rep, uint32_t layer, int dir, int par,
                                            uint32_t s)
{
    constexpr size_t kElemBytes = sizeof(typename Store<PREC>::real) * 2;
    constexpr int NE = Store<PREC>::NE;
    const size_t slab = size_t((layer * D + uint32_t(dir)) * 2u + uint32_t(par)) * NE * rep.Vhp;
    return LinkRef{reinterpret_cast<char *>(links) + (rep.elem_offset + slab) * kElemBytes, s >> 1};
}

}  // namespace su3hb
