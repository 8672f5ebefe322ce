// layout.h -- descriptors shared by the host side and the kernels of the GPU
// library: storage modes, the per-replica descriptor and kernel arguments.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace su3hb {

constexpr int kFP64_18 = 0;
constexpr int kFP32_18 = 1;
constexpr int kFP32_12 = 2;
constexpr int kFP64_12 = 3;

constexpr int kMaxD = 6;          // kernels are instantiated for D = 2 .. 6
constexpr int kStatSlots = 256;   // spread of the per-block statistics atomics

inline constexpr int elems_per_link(int prec) { return (prec == kFP32_12 || prec == kFP64_12) ? 6 : 9; }
inline constexpr int bytes_per_elem(int prec) { return (prec == kFP64_18 || prec == kFP64_12) ? 16 : 8; }
inline constexpr bool is_fp32(int prec) { return prec == kFP32_18 || prec == kFP32_12; }
inline constexpr int bytes_per_link(int prec) { return elems_per_link(prec) * bytes_per_elem(prec); }

// Links are stored in tiles of kTile consecutive half-lattice sites (one
// wave); a slab of Vh links takes Vhp = Vh rounded up to whole tiles.
constexpr uint32_t kTile = 64;
inline constexpr uint32_t padded_half(uint32_t Vh) { return (Vh + kTile - 1) / kTile * kTile; }

// Division by an invariant integer (T. Granlund and P. L. Montgomery, PLDI
// 1994): for d >= 1 and 0 <= x < 2^31, x / d = (x m) >> s with
// l = ceil(log2 d), s = 31 + l and m = ceil(2^s / d), which is below 2^32
// (so m d - 2^s < d <= 2^l, the condition of their Theorem 4.2).
struct DivMagic {
    uint32_t m, s;
};

inline DivMagic div_magic(uint32_t d)
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint32_t s = 31u + l;
    return DivMagic{uint32_t(((uint64_t(1) << s) + d - 1u) / d), s};
}

// One lattice ("replica").  A single lattice is a batch of one.  Its links
// start `elem_offset` complex elements into the batch's link buffer and are
// laid out as [layer][mu][parity][tile][packet][kTile].
struct RepDesc {
    uint64_t elem_offset;
    int32_t n[kMaxD];        // extents
    uint32_t stride[kMaxD];  // site-number strides: 1, n0, n0 n1, ...
    uint32_t V;              // sites per layer
    uint32_t Vh;             // V / 2
    uint32_t Vhp;            // Vh rounded up to a multiple of kTile (links per slab in memory)
    uint32_t nlat;           // 1 or 2
    uint32_t glued;          // dlt mask (only with nlat == 2)
    uint32_t lat2test;
    uint32_t key0, key1;     // Philox key (seed)
    double beta0, beta1;     // couplings used when the batch carries them
    uint32_t upd_block0;     // first block of this replica in an update launch
    uint32_t upd_blocks;     // blocks of this replica in an update launch
    uint32_t plq_block0;     // first block in a plaquette launch
    uint32_t plq_blocks;
    uint32_t plq_spt;        // plaquettes per thread in the plaquette launch
    uint32_t pers_block0;    // first block in a persistent launch (kPersistentThreads links per block)
    uint32_t pers_blocks;
    DivMagic div[kMaxD - 1];  // division by n0 / 2 (entry 0) and by n_i (entry i, 0 < i < D - 1)
};

// Persistent batch launches: blocks of kPersistentThreads, as many per CU as
// the kernel's registers allow (2 waves per SIMD for FP64 links, 3 for
// FP32), slices separated by a grid barrier on a small array of counters
// (kBarrierWords words, each counter on its own 128-byte line): the start
// barrier's kBarrierLeaves leaf counters and top counter, an abort flag, and
// for the slice barriers per-XCD member counts, arrival counters and go
// words, a top counter of the XCDs and a release word.
constexpr int kPersistentThreads = 256;
inline constexpr int persistent_waves(int prec) { return (prec == kFP32_18 || prec == kFP32_12) ? 3 : 2; }
constexpr int kBarrierWords = 4096;
constexpr uint32_t kBarrierLeaves = 16;
constexpr uint32_t kBarrierTop = 1024;
constexpr uint32_t kBarrierFlag = 1536;
constexpr uint32_t kBarrierXcds = 16;            // XCC ids are 4 bits
constexpr uint32_t kBarrierXcdMembers = 2048;    // + 32 x: blocks on XCD x
constexpr uint32_t kBarrierXcdArrive = 2560;     // + 32 x
constexpr uint32_t kBarrierXcdGo = 3072;         // + 32 x
constexpr uint32_t kBarrierXcdTop = 3584;
constexpr uint32_t kBarrierXcdRelease = 3712;
constexpr uint32_t kBarrierSpinLimit = 1u << 22;

// Statistics slot, padded to its own 128-byte line.
struct alignas(128) StatSlot {
    unsigned long long attempts[3];
    unsigned long long accepts[3];
    unsigned long long updates;
    double dtrace;
};

struct UpdateArgs {
    void *links;                 // base of the link buffer
    const RepDesc *reps;         // device array
    int nrep;
    int parity;                  // checkerboard colour being updated
    int mu;                      // direction being updated
    int nhit;                    // KP proposals per subgroup, at most; 0: overrelaxation
    int use_rep_beta;            // 1: couplings from RepDesc; 0: from beta0/beta1
    int order;                   // 0 hardware, 1 XCD-contiguous, 2 and 4 XCD slabs, 3, 5 and 6 XCD slabs of 3D blocks,
                                 // 7 XCD slabs of 4D wave tiles
    int reverse;                 // 1: each XCD walks its blocks last to first (alternate slices)
    uint32_t slab;               // orders 2, 3: tiles of the last direction per XCD
    uint32_t cp;                 // orders 2, 3: blocks (order 3: waves) per (x_{D-2}, x_{D-1}) plane
    uint32_t n2;                 // orders 2, 3: extent of direction D-2
    uint32_t plane;              // order 3: half-sites of one (x_{D-2}, x_{D-1}) plane
    uint32_t tile2, tile3;       // order 3: waves of a block along x_{D-2} and x_{D-1}
    uint32_t n0h, n1;            // order 7: n_0 / 2 and n_1
    int stage;                   // 1: each wave stages the U_mu links its planes nu = 0, 1 read in LDS
    uint32_t stage_r;            // staging halo: n_0 / 2 half-sites before and after a wave's 64
    double beta0, beta1;
    const uint32_t *sweep;       // device sweep counter
    StatSlot *stats;             // kStatSlots slots
    uint32_t total_blocks;       // real blocks (grid may be padded to 8)
    double *meas;                // fused plaquettes: [mu][total_blocks][meas_classes] partial sums, or null
    int meas_classes;            // 1: one lattice layer; 3: two layers (classes by base layer and tags)
    int persistent;              // 1: logical blocks of the persistent partition
    uint32_t *barrier;           // persistent launches: kBarrierWords counters, zeroed before the launch
};

struct PlaqArgs {
    const void *links;
    const RepDesc *reps;
    int nrep;
    double beta0, beta1;
    int use_rep_beta;
    double *partials;            // [block][5]
    uint32_t total_blocks;
};

constexpr int kDefaultWaves = 2;  // update kernels for D = 4 also exist for 3 (and, FP32, 4) waves/SIMD

}  // namespace su3hb
