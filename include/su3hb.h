/*
 * su3hb.h -- C ABI of libsu3hb.so: checkerboard Cabibbo-Marinari SU(3)
 * heatbath with FHKP SU(2) updates in multi-hit form, for the Wilson action on
 * a D-dimensional torus or a double-layered torus, on one AMD MI355X (gfx950).
 *
 * Method: B. A. Berg, "Fortran MPI Checkerboard Code for SU(3) Lattice Gauge
 * Theory I" (arXiv:0904.0642).  Section, equation and table numbers below
 * refer to that paper.
 *
 * Conventions shared by every call:
 *   - All functions return SU3HB_OK (0) or a negative su3hb_status.  They never
 *     abort.  su3hb_last_error() returns a thread-local message describing the
 *     last failure of the calling thread.
 *   - Sites are numbered as in eq. (i_s) of Sec. 2 but 0-based, direction 0
 *     fastest; the colour of eq. (i_c) is the parity (sum of coordinates) mod 2.
 *   - The canonical host layout of the links (get/set) is FP64
 *     [layer][site][mu][row][col][re,im], i.e. 18 doubles per SU(3) matrix,
 *     nlat * V * D * 18 doubles in total (V = product of the extents).
 *   - Device work is issued on the stream given at creation (NULL = the null
 *     stream).  Calls marked "asynchronous" return before the GPU finishes;
 *     calls that return host data synchronise that stream.
 *   - A handle must not be used from two threads at once.
 */
#ifndef SU3HB_H
#define SU3HB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SU3HB_MAX_D 8           /* parameter structs hold up to 8 extents     */
#define SU3HB_GPU_MIN_D 2       /* the GPU kernels are built for D = 2 .. 6   */
#define SU3HB_GPU_MAX_D 6

typedef enum su3hb_status {
    SU3HB_OK = 0,
    SU3HB_EINVAL = -1,      /* invalid argument (message says which)          */
    SU3HB_ENOMEM = -2,      /* device or host allocation failed               */
    SU3HB_EHIP = -3,        /* a HIP runtime call failed                      */
    SU3HB_ENOTSU3 = -4,     /* set_links input is not in SU(3) (or not finite)*/
    SU3HB_EUNSUPPORTED = -5 /* valid request the GPU build does not cover     */
} su3hb_status;

/* Link storage.  The Kennedy-Pendleton draw and acceptance test,
 * reunitarisation and every accumulation run in FP64 in all modes; FP32
 * modes store the links and form the staple products, W = U A, the random
 * direction and the SU(2) rotations in FP32.  12-real storage keeps rows 0
 * and 1 and rebuilds row 2 = conj(row0 x row1) on load. */
typedef enum su3hb_precision {
    SU3HB_FP64_18 = 0,  /* 144 bytes per link */
    SU3HB_FP32_18 = 1,  /*  72 bytes per link */
    SU3HB_FP32_12 = 2,  /*  48 bytes per link */
    SU3HB_FP64_12 = 3   /*  96 bytes per link, FP64 arithmetic throughout */
} su3hb_precision;

/* Start configuration (istart of mc.par, Sec. 2.3). */
typedef enum su3hb_start {
    SU3HB_START_NONE = 0, /* leave the links unset (call su3hb_set_links) */
    SU3HB_COLD = 1,       /* ordered start: every link is the unit matrix  */
    SU3HB_HOT = 2         /* disordered start: Haar-random SU(3) links drawn
                             from the seeded Philox stream                 */
} su3hb_start;

/* Lattice parameters (latmpi.par / mc.par of Sec. 2.3, given at run time). */
typedef struct su3hb_params {
    int nd;                        /* dimension D; 2 .. SU3HB_GPU_MAX_D       */
    int extents[SU3HB_MAX_D];      /* n^1 .. n^D, each even and >= 2 (Sec. 2) */
    int nlat;                      /* 1 = torus, 2 = double-layered torus     */
    unsigned dlt_mask;             /* nlat = 2: bit d set = direction d glued
                                      to the other layer (Sec. 2.2 glues every
                                      direction or the spatial ones only); 0 =
                                      two independent tori.  Must be 0 if
                                      nlat=1.                                  */
    int lat2test;                  /* nlat = 2 only: both layers draw the same
                                      random numbers (Sec. 3.4)               */
    int precision;                 /* su3hb_precision                          */
    int start;                     /* su3hb_start                              */
    uint64_t seed;                 /* Philox key                               */
    void *device_links;            /* NULL: the library allocates the links;
                                      else a device buffer it borrows (e.g. a
                                      torch tensor) that must outlive the
                                      handle and hold su3hb_links_bytes()     */
    size_t device_bytes;           /* size of device_links                     */
    void *hip_stream;              /* hipStream_t for all work; NULL = null    */
} su3hb_params;

/* Counters of su3hb_sweep (over the sweeps of that call). */
typedef struct su3hb_stats {
    uint64_t attempts[3];   /* KP proposals per SU(2) subgroup (0,1),(0,2),(1,2) */
    uint64_t accepts[3];    /* subgroup updates that accepted a proposal          */
    uint64_t link_updates;  /* SU(3) link updates performed                       */
    double dtrace;          /* change of sum_p beta_p (1/3) Re Tr U_p, accumulated
                               link by link during the update (Sec. 2.1 keeps the
                               total action on record this way)                  */
} su3hb_stats;

typedef struct su3hb_lattice su3hb_lattice;

/* Bytes of device memory the links of `p` occupy: nlat*D*2 slabs of V/2
 * links, each slab rounded up to whole tiles of 64 links, times the bytes of
 * one link (144, 96, 72 or 48).  The layout inside is the library's own;
 * su3hb_get_links / su3hb_set_links convert to and from the canonical
 * order. */
int su3hb_links_bytes(const su3hb_params *p, size_t *bytes);

/* Validate `p`, allocate or adopt the link buffer, and write the start
 * configuration (Sec. 2.4, initialisation step).  Errors: SU3HB_EINVAL for
 * odd or < 2 extents (Sec. 2: checkerboard needs even extensions), nd out of
 * range, nlat not 1 or 2 (Sec. 2.3), dlt_mask or lat2test without nlat = 2,
 * too small device buffer, more than 2^32 links (the Philox counter holds a
 * 32-bit link id).  On error *out is NULL. */
int su3hb_init_lattice(su3hb_lattice **out, const su3hb_params *p);

/* Release the handle and the memory the library owns (not borrowed links). */
void su3hb_free(su3hb_lattice *lat);

/* n_sweeps sweeps (Sec. 2.1): for parity 0 then 1, for mu = 0..D-1, every
 * link U_mu(x) of that parity in every layer gets one CM update: staple sum,
 * SU(2) subgroups (0,1),(0,2),(1,2) by FHKP with at most n_hit proposals each
 * (Sec. 2.1, multi-hit; a subgroup with no accepted proposal keeps the link),
 * then reunitarisation.  beta0/beta1 are the couplings of the two tori
 * (Sec. 2.2 tag rule: a plaquette with every link in layer 0 uses beta0,
 * otherwise beta1); pass beta1 = beta0 for a plain torus.  Wilson beta = 6/g^2.
 * n_hit >= 1 and < 32768.  Asynchronous if stats is NULL; otherwise
 * synchronises and fills *stats for these sweeps. */
int su3hb_sweep(su3hb_lattice *lat, double beta0, double beta1, int n_hit, int n_sweeps,
                su3hb_stats *stats);

/* n_sweeps overrelaxation sweeps: the order of su3hb_sweep, each link gets,
 * per SU(2) subgroup (0,1),(0,2),(1,2), the reflection that keeps its local
 * action Re Tr(U A) unchanged: with the subgroup block of W = U A equal to
 * k V, V in SU(2), the block becomes k V^dag (U <- R U, r = V^dag V^dag),
 * then reunitarisation.  Sec. 1 of the paper names overrelaxation moves as
 * an addition the code could take in; interleaved with heatbath sweeps they
 * leave the Boltzmann distribution invariant.  No random numbers are drawn;
 * the sweep counter advances by n_sweeps.  stats: attempts and accepts both
 * count the reflections (subgroups with k > 1e-300), dtrace is the change of
 * the action (zero up to rounding).  Errors and synchronisation as
 * su3hb_sweep. */
int su3hb_overrelax(su3hb_lattice *lat, double beta0, double beta1, int n_sweeps, su3hb_stats *stats);

/* As su3hb_sweep, measuring the plaquettes after every sweep (Sec. 2.4,
 * measurement step) into series[6*i .. 6*i+5] for sweep i (the layout of
 * su3hb_plaquette).  Synchronises once at the end. */
int su3hb_sweep_measure(su3hb_lattice *lat, double beta0, double beta1, int n_hit, int n_sweeps,
                        double *series, su3hb_stats *stats);

/* Plaquette measurement (Sec. 2.4): out[0] mean of (1/3) Re Tr U_p over all
 * nlat*V*D(D-1)/2 plaquettes; out[1] spacelike (planes without direction D-1),
 * out[2] timelike (planes containing it), out[3] layer 0, out[4] layer 1 (by
 * base site; NaN when absent; out[1] NaN for D = 2); out[5] the weighted sum
 * sum_p beta_p (1/3) Re Tr U_p for the given couplings.  All in FP64.
 * Synchronises. */
int su3hb_plaquette(su3hb_lattice *lat, double beta0, double beta1, double out[6]);

/* Copy the links to host memory in the canonical FP64 layout, the paper's
 * own array of links indexed by site number and direction (the A(n_s, nd)
 * link arrays of Sec. 2) with the 18 reals of the 3x3 complex matrix
 * innermost and the layer outermost; n must equal nlat*V*D*18.  FP32 modes
 * are widened; 12-real links get their third row rebuilt.  Synchronises. */
int su3hb_get_links(const su3hb_lattice *lat, double *host, size_t n);

/* Replace the links from host memory in the canonical layout (as
 * su3hb_get_links: the A(n_s, nd) arrays of Sec. 2).  Every matrix
 * is checked on the GPU first: a NaN/Inf entry, or max|U U^dag - 1| or
 * |det U - 1| above 1e-10 (FP64 modes) / 1e-6 (FP32 modes) returns SU3HB_ENOTSU3
 * and leaves the lattice unchanged.  Synchronises. */
int su3hb_set_links(su3hb_lattice *lat, const double *host, size_t n);

/* Seed and sweep counter: with the links they are the whole Markov-chain
 * state, so get_links + get_state ... set_links + set_state resumes a run
 * exactly (the random numbers are a function of seed, sweep and link).  The
 * seed plays the part of the seed pair iseed1, iseed2 of mc.par (Sec. 2.3);
 * the sweep counter stands for the position of the paper's sequential
 * generator, which a counter-based generator does not have.  The
 * sweep index of the Philox counter is 32 bits: set_state rejects sweep >=
 * 2^32 and a sweep call that would pass 2^32 returns SU3HB_EINVAL. */
int su3hb_get_state(const su3hb_lattice *lat, uint64_t *seed, uint64_t *sweep);
int su3hb_set_state(su3hb_lattice *lat, uint64_t seed, uint64_t sweep);

/* Launch shape of the update kernel.  block: threads per block (64, 128 or
 * 256).  order: 0 = hardware block order; 1 = each XCD gets a contiguous run
 * of blocks; 2 = each of the 8 XCDs gets a slab of the last direction and
 * walks it with that direction fastest (one single-layer lattice whose last
 * extent is a multiple of 8 and whose blocks tile an (x_{D-2}, x_{D-1})
 * plane); 3 = as 2, with the waves of a block stacked along the two slowest
 * directions (2 x 2 waves for 256 threads, 1 x 2 for 128; needs planes of a
 * multiple of 64 half-sites); 4 = as 2, walking the block's chunk of the
 * plane slowest and x_{D-2} in the middle; 5 = as 3, walking the x_{D-2}
 * tiles before the chunks of the plane; 6 = as 3, with all waves of a block
 * along x_{D-2}; 7 (D = 4) = each wave covers a 4D tile of 8 half-sites along
 * x_0 by 2 x 2 x 2 along x_1, x_2, x_3, the waves of a block stacked along
 * x_2, each XCD walking one x_3 slab (n_0/2 a multiple of 8, n_2 of twice
 * the waves per block, n_3 of 16).  Where an order does not apply a lower one
 * that does is used (4 and 2 fall back to 1; 3, 5 and 6 to 2 or 1; 7 to 1).
 * Adding 8 to an order makes every second slice of a sweep walk each XCD's
 * blocks last to first, so a slice starts on the links the slice before it
 * read last.  Adding 16 makes every wave copy the U_mu links that the
 * staples of its planes nu = 0, 1 read (Sec. 2.1, the staple sum) into LDS
 * once, n_0/2 half-sites on either side of its own 64, and read them from
 * there (single-layer lattices outside batches, orders 0 to 6; ignored
 * elsewhere).  waves: minimum waves per SIMD the kernel is compiled for: 2;
 * 3 for D = 4; 4 for D = 4 with FP32 links.  Results are bit-identical for
 * every shape.  get_launch reports the order in effect (with the 8 and 16).
 * A shape whose LDS (staple snapshots of a measured slice plus staging
 * areas) exceeds the device's per-block limit returns SU3HB_EUNSUPPORTED
 * and leaves the launch shape as it was. */
int su3hb_set_launch(su3hb_lattice *lat, int block, int order, int waves);
int su3hb_get_launch(const su3hb_lattice *lat, int *block, int *order, int *waves);

/* Time the candidate launch shapes on this lattice for about budget_ms (two
 * passes, each shape keeping its faster one) and
 * keep the fastest (cached per precision, D and extents for the process).
 * The links and the sweep counter are restored afterwards.  Synchronises. */
int su3hb_autotune(su3hb_lattice *lat, int budget_ms);

/* As su3hb_sweep (measure != 0: plus plaquettes into series as in
 * su3hb_sweep_measure; n_hit = 0: overrelaxation sweeps as in
 * su3hb_overrelax), launched kernel by kernel with a HIP event pair
 * around every launch on the lattice's stream.  timing[0] = summed update
 * kernel time (ms), timing[1] = number of update launches, timing[2] =
 * summed plaquette kernel time (ms), timing[3] = number of plaquette
 * launches.  Synchronises. */
int su3hb_sweep_timed(su3hb_lattice *lat, double beta0, double beta1, int n_hit, int n_sweeps,
                      int measure, double *series, double timing[4]);

/* ------------------------------------------------------------------------ */
/* Batches: many independent periodic lattices of one dimension D, each with
 * its own extents, coupling and seed, updated together.  (Not in the paper;
 * the paper's own parallelism is sublattices of one lattice, Sec. 2.3.)      */

typedef struct su3hb_replica_desc {
    int extents[SU3HB_MAX_D];   /* even, >= 2 */
    double beta;
    uint64_t seed;
    int start;                  /* SU3HB_COLD or SU3HB_HOT */
} su3hb_replica_desc;

typedef struct su3hb_lattice su3hb_batch;

/* Create n replicas of dimension nd in one device allocation.  Errors as for
 * su3hb_init_lattice. */
int su3hb_batch_create(su3hb_batch **out, int nd, const su3hb_replica_desc *reps, int n,
                       int precision, void *hip_stream);

/* n_sweeps sweeps of every replica at its own beta.  mode 0: one launch per
 * checkerboard slice covering all replicas; mode 1: one persistent
 * cooperative launch (256-thread blocks, as many per compute unit as fit) that loops over
 * sweeps and slices with a grid barrier between slices, in launches of at
 * most 65536 sweeps.  Both give bit-identical links.  Mode 1 returns after
 * the work has finished (it synchronises the stream); if a grid barrier
 * waits past its spin limit every block leaves the kernel and the call
 * returns SU3HB_EHIP with the links not valid.  stats as in su3hb_sweep,
 * summed over replicas. */
int su3hb_batch_sweep(su3hb_batch *b, int n_hit, int n_sweeps, int mode, su3hb_stats *stats);

/* Per-replica plaquette: out[6*r .. 6*r+5] as in su3hb_plaquette. */
int su3hb_batch_plaquette(su3hb_batch *b, double *out, size_t n);

/* Links of one replica in the canonical layout (n = V_r * D * 18). */
int su3hb_batch_get_links(su3hb_batch *b, int replica, double *host, size_t n);
int su3hb_batch_set_links(su3hb_batch *b, int replica, const double *host, size_t n);

void su3hb_batch_free(su3hb_batch *b);

/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): su3hb_sweep_measure
 * without a handle and without any device or host allocation.
 *
 * n_sweeps sweeps of the lattice described by p, in the order and with the
 * random numbers of su3hb_sweep (sweep indices sweep0 .. sweep0+n_sweeps-1,
 * key p->seed), on the links at p->device_links (caller-owned device memory
 * of p->device_bytes bytes in the library's layout, e.g. the buffer a handle
 * created with su3hb_init_lattice on borrowed memory works on; p->start is
 * ignored), issued on p->hip_stream.  series: NULL, or caller-owned DEVICE
 * memory of 6 * n_sweeps doubles that receives, per sweep, the plaquettes in
 * the layout of su3hb_plaquette.  The call only enqueues kernels (no memset,
 * no copy, no synchronisation) and returns before the GPU finishes, so it can
 * be captured into a graph.
 *
 * The kernels' counters, statistics and partial sums live in one static
 * device array of 8 MiB per GPU, held until the process ends and shared by
 * every call on that GPU: calls that overlap on one GPU (two streams, two
 * threads) race.  Each call clears what must start at zero.  With series
 * non-NULL the measurement needs D * ceil(nlat * V / 512) * (1 or 3)
 * partial sums (3 for two layers) in that array, at most (8 MiB - 33 KiB) / 8;
 * a larger lattice returns SU3HB_EINVAL (64^4 fits; 128^4 does not).  Other
 * errors as su3hb_init_lattice and su3hb_sweep, all reported before any
 * device work; the links are left unchanged then. */
int su3hb_sweep_measure_static(const su3hb_params *p, double beta0, double beta1, int n_hit, int n_sweeps,
                               uint64_t sweep0, double *series);

/* Thread-local description of the last error ("" if none). */
const char *su3hb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SU3HB_H */
