// capi.cpp -- the extern "C" boundary of libsu3hb.so (declared in
// include/su3hb.h): argument checks, device memory, the sweep driver
// (parity outer, direction inner; one launch per slice, replayed from a
// captured HIP graph), measurement, canonical get/set, autotuning and batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "su3hb.h"
#include "kernels.h"
#include "layout.h"

using namespace su3hb;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(SU3HB_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                 \
    } while (0)

constexpr int kPlaqBlock = 256;
constexpr uint32_t kSeriesCap = 4096;
constexpr size_t kStageBytes = size_t(256) << 20;

// A captured sweep, keyed by its couplings, kind (n_hit; 0 = overrelaxation)
// and measurement.  A few are kept so that heatbath and overrelaxation sweeps
// can alternate without capturing again.
struct GraphCache {
    bool valid = false;
    double b0 = 0, b1 = 0;
    int nhit = 0, measure = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};
constexpr int kGraphSlots = 4;

}  // namespace

struct su3hb_lattice {
    int device = 0;
    int nd = 0, prec = 0, nrep = 0;
    bool batch = false;
    std::vector<RepDesc> reps;
    RepDesc *d_reps = nullptr;
    void *links = nullptr;
    size_t links_bytes = 0;
    bool owns_links = false;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    uint32_t *d_sweep = nullptr;
    uint64_t sweep = 0;
    uint64_t seed = 0;
    StatSlot *d_stats = nullptr;
    StatSlot *d_stats_out = nullptr;
    double *d_partials = nullptr;
    double *d_meas = nullptr;     // fused measurement partials, [D][update blocks]
    size_t meas_cap = 0;
    double *d_plaq = nullptr;
    double *d_series = nullptr;
    uint32_t *d_cursor = nullptr;
    unsigned long long *d_maxdef = nullptr;
    double *d_stage = nullptr;
    uint32_t *d_bar = nullptr;    // grid-barrier counters of persistent launches
    int block = 256, order = 1, waves = kDefaultWaves;
    uint32_t upd_blocks = 0, plq_blocks = 0, pers_blocks = 0;
    bool use_graph = true;
    GraphCache graphs[kGraphSlots];
    uint64_t graph_tick = 0;
    std::vector<hipEvent_t> events;
    int num_cus = 0;
};

namespace {

std::mutex g_tune_mu;
struct Shape {
    int block, order, waves;
};
std::map<std::string, Shape> g_tune_cache;

void drop_slot(GraphCache &g)
{
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
    g = GraphCache{};
}

void drop_graph(su3hb_lattice *L)
{
    for (auto &g : L->graphs) drop_slot(g);
}

// Block tables and offsets of every replica for the current launch shape.
void layout_reps(su3hb_lattice *L)
{
    uint64_t off = 0;
    uint32_t ub = 0, pb = 0, sb = 0;
    const int NE = elems_per_link(L->prec);
    for (auto &r : L->reps) {
        r.elem_offset = off;
        off += uint64_t(r.nlat) * L->nd * NE * 2 * r.Vhp;
        r.upd_block0 = ub;
        r.upd_blocks = (r.nlat * r.Vh + L->block - 1) / L->block;
        ub += r.upd_blocks;
        // one plaquette thread item per (site, plane); a few items per thread
        // keep the partial sums to about 4096 blocks per lattice for the
        // finalize pass
        const uint64_t nitem = uint64_t(r.nlat) * r.V * uint64_t(L->nd * (L->nd - 1) / 2);
        r.plq_spt = uint32_t(std::min<uint64_t>(16, std::max<uint64_t>(1, nitem / (uint64_t(kPlaqBlock) * 4096u))));
        r.plq_block0 = pb;
        const uint64_t per_block = uint64_t(kPlaqBlock) * r.plq_spt;
        r.plq_blocks = uint32_t((nitem + per_block - 1) / per_block);
        pb += r.plq_blocks;
        r.pers_block0 = sb;
        r.pers_blocks = (r.nlat * r.Vh + kPersistentThreads - 1) / kPersistentThreads;
        sb += r.pers_blocks;
    }
    L->upd_blocks = ub;
    L->plq_blocks = pb;
    L->pers_blocks = sb;
}

int upload_reps(su3hb_lattice *L)
{
    HIPCHK(hipMemcpyAsync(L->d_reps, L->reps.data(), sizeof(RepDesc) * L->reps.size(), hipMemcpyHostToDevice,
                          L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    return SU3HB_OK;
}

int check_extents(int nd, const int *ext, uint64_t *V)
{
    if (nd < SU3HB_GPU_MIN_D || nd > SU3HB_GPU_MAX_D)
        return fail(SU3HB_EINVAL, "nd = %d outside %d..%d", nd, SU3HB_GPU_MIN_D, SU3HB_GPU_MAX_D);
    uint64_t v = 1;
    for (int i = 0; i < nd; ++i) {
        if (ext[i] < 2 || (ext[i] & 1))
            return fail(SU3HB_EINVAL, "extent %d of direction %d must be even and >= 2", ext[i], i);
        v *= uint64_t(ext[i]);
        if (v > (uint64_t(1) << 32)) return fail(SU3HB_EINVAL, "lattice volume exceeds 2^32 sites");
    }
    *V = v;
    return SU3HB_OK;
}

RepDesc make_rep(int nd, const int *ext, int nlat, unsigned glued, int lat2test, uint64_t seed, double b0,
                 double b1)
{
    RepDesc r;
    std::memset(&r, 0, sizeof r);
    uint32_t st = 1;
    for (int i = 0; i < nd; ++i) {
        r.n[i] = ext[i];
        r.stride[i] = st;
        st *= uint32_t(ext[i]);
    }
    for (int i = 0; i + 1 < nd; ++i) r.div[i] = div_magic(i == 0 ? uint32_t(ext[0]) / 2u : uint32_t(ext[i]));
    r.V = st;
    r.Vh = st / 2;
    r.Vhp = padded_half(r.Vh);
    r.nlat = uint32_t(nlat);
    r.glued = glued;
    r.lat2test = uint32_t(lat2test);
    r.key0 = uint32_t(seed);
    r.key1 = uint32_t(seed >> 32);
    r.beta0 = b0;
    r.beta1 = b1;
    return r;
}

int alloc_common(su3hb_lattice *L)
{
    hipDeviceProp_t prop;
    HIPCHK(hipGetDevice(&L->device));
    HIPCHK(hipGetDeviceProperties(&prop, L->device));
    L->num_cus = prop.multiProcessorCount;
    HIPCHK(hipStreamCreateWithFlags(&L->cap, hipStreamNonBlocking));
    HIPCHK(hipMalloc(&L->d_reps, sizeof(RepDesc) * L->reps.size()));
    HIPCHK(hipMalloc(&L->d_sweep, sizeof(uint32_t)));
    HIPCHK(hipMalloc(&L->d_stats, sizeof(StatSlot) * kStatSlots));
    HIPCHK(hipMalloc(&L->d_stats_out, sizeof(StatSlot)));
    HIPCHK(hipMalloc(&L->d_plaq, sizeof(double) * 6 * L->reps.size()));
    HIPCHK(hipMalloc(&L->d_series, sizeof(double) * 6 * kSeriesCap));
    HIPCHK(hipMalloc(&L->d_cursor, sizeof(uint32_t)));
    HIPCHK(hipMalloc(&L->d_maxdef, sizeof(unsigned long long)));
    HIPCHK(hipMalloc(&L->d_bar, sizeof(uint32_t) * kBarrierWords));
    layout_reps(L);
    HIPCHK(hipMalloc(&L->d_partials, sizeof(double) * 5 * L->plq_blocks));
    int rc = upload_reps(L);
    if (rc) return rc;
    HIPCHK(launch_counter_set(L->stream, L->d_sweep, 0));
    HIPCHK(launch_counter_set(L->stream, L->d_cursor, 0));
    HIPCHK(launch_stats_zero(L->stream, L->d_stats));
    return SU3HB_OK;
}

int adopt_or_alloc_links(su3hb_lattice *L, void *borrowed, size_t borrowed_bytes)
{
    uint64_t elems = 0;
    for (auto &r : L->reps) elems += uint64_t(r.nlat) * L->nd * elems_per_link(L->prec) * 2 * r.Vhp;
    L->links_bytes = size_t(elems) * bytes_per_elem(L->prec);
    if (borrowed) {
        if (borrowed_bytes < L->links_bytes)
            return fail(SU3HB_EINVAL, "device buffer holds %zu bytes, the links need %zu", borrowed_bytes,
                        L->links_bytes);
        if (reinterpret_cast<uintptr_t>(borrowed) % 16)
            return fail(SU3HB_EINVAL, "device buffer must be 16-byte aligned");
        L->links = borrowed;
        L->owns_links = false;
    } else {
        hipError_t e = hipMalloc(&L->links, L->links_bytes);
        if (e != hipSuccess)
            return fail(SU3HB_ENOMEM, "hipMalloc of %zu bytes for the links failed: %s", L->links_bytes,
                        hipGetErrorString(e));
        L->owns_links = true;
    }
    return SU3HB_OK;
}

void destroy(su3hb_lattice *L)
{
    if (!L) return;
    hipSetDevice(L->device);
    hipStreamSynchronize(L->stream);   // also the null stream: nothing may still run on this memory
    drop_graph(L);
    for (auto e : L->events) hipEventDestroy(e);
    if (L->owns_links && L->links) hipFree(L->links);
    hipFree(L->d_reps);
    hipFree(L->d_sweep);
    hipFree(L->d_stats);
    hipFree(L->d_stats_out);
    hipFree(L->d_partials);
    hipFree(L->d_meas);
    hipFree(L->d_plaq);
    hipFree(L->d_series);
    hipFree(L->d_cursor);
    hipFree(L->d_maxdef);
    hipFree(L->d_stage);
    hipFree(L->d_bar);
    if (L->cap) hipStreamDestroy(L->cap);
    delete L;
}

int start_replica(su3hb_lattice *L, int r, int mode)
{
    if (mode == SU3HB_START_NONE) return SU3HB_OK;
    const RepDesc &rep = L->reps[r];
    const uint32_t nthreads = rep.nlat * uint32_t(L->nd) * rep.V;
    HIPCHK(launch_start(L->nd, L->prec, L->stream, L->links, L->d_reps, r, nthreads, mode));
    return SU3HB_OK;
}

// Order 2 (XCD slabs of the last direction) needs one single-layer lattice,
// a last extent divisible by 8 and blocks that tile an (x_{D-2}, x_{D-1}) plane.
bool slab_order_ok(const su3hb_lattice *L, int block)
{
    if (L->batch || L->nrep != 1 || L->nd < 3) return false;
    const RepDesc &r = L->reps[0];
    if (r.nlat != 1) return false;
    const uint32_t nl = uint32_t(r.n[L->nd - 1]), n2 = uint32_t(r.n[L->nd - 2]);
    if (nl % 8) return false;
    const uint32_t plane = r.Vh / (nl * n2);
    return plane % uint32_t(block) == 0;
}

// Orders 3, 5 and 6 (3D blocks: tile2 x tile3 waves along x_{D-2}, x_{D-1})
// need one single-layer lattice whose (x_{D-2}, x_{D-1}) planes hold a
// multiple of 64 half-sites, n_{D-2} divisible by tile2 and n_{D-1} by
// 8 tile3.  Order 6 puts all waves of a block along x_{D-2}.
bool is_cube_order(int o) { return o == 3 || o == 5 || o == 6; }

void cube_tiles(int block, int order, uint32_t *t2, uint32_t *t3)
{
    *t2 = order == 6 ? uint32_t(block) / 64u : block == 256 ? 2u : 1u;
    *t3 = uint32_t(block) / 64u / *t2;
}

bool cube_order_ok(const su3hb_lattice *L, int block, int order)
{
    if (L->batch || L->nrep != 1 || L->nd < 3) return false;
    const RepDesc &r = L->reps[0];
    if (r.nlat != 1) return false;
    const uint32_t nl = uint32_t(r.n[L->nd - 1]), n2 = uint32_t(r.n[L->nd - 2]);
    const uint32_t plane = r.Vh / (nl * n2);
    uint32_t t2, t3;
    cube_tiles(block, order, &t2, &t3);
    return plane % 64u == 0 && n2 % t2 == 0 && nl % (8u * t3) == 0;
}

// Order 7 (4D wave tiles, D = 4): one single-layer lattice with n_0/2 a
// multiple of 8, n_2 of twice the waves per block and n_3 of 16 (one x_3 slab
// of whole tiles per XCD).
bool tile4_order_ok(const su3hb_lattice *L, int block)
{
    if (L->batch || L->nrep != 1 || L->nd != 4) return false;
    const RepDesc &r = L->reps[0];
    if (r.nlat != 1) return false;
    const uint32_t nw = uint32_t(block) / 64u;
    return (uint32_t(r.n[0]) / 2u) % 8u == 0 && uint32_t(r.n[2]) % (2u * nw) == 0 && uint32_t(r.n[3]) % 16u == 0;
}

// Flag added to an order: alternate slices walk every XCD's blocks backwards.
constexpr int kOrderReverse = 8;
// Flag added to an order: every wave stages the U_mu links that its planes
// nu = 0, 1 read in LDS (single-layer lattices outside batches, orders 0 to
// 6, which give each wave 64 consecutive half-lattice indices).
constexpr int kOrderStage = 16;

// Block order in effect, without the flags.
int base_order(const su3hb_lattice *L)
{
    const int o = L->order & ~(kOrderReverse | kOrderStage);
    if (o == 7 && !tile4_order_ok(L, L->block)) return 1;
    if (is_cube_order(o) && !cube_order_ok(L, L->block, o)) return slab_order_ok(L, L->block) ? 2 : 1;
    if ((o == 2 || o == 4) && !slab_order_ok(L, L->block)) return 1;
    return o;
}

bool stage_applies(const su3hb_lattice *L)
{
    return (L->order & kOrderStage) && !L->batch && L->nrep == 1 && L->reps[0].nlat == 1 && base_order(L) != 7;
}

int effective_order(const su3hb_lattice *L)
{
    return base_order(L) | (L->order & kOrderReverse) | (stage_applies(L) ? kOrderStage : 0);
}

UpdateArgs update_args(const su3hb_lattice *L, double b0, double b1, int nhit)
{
    UpdateArgs a;
    std::memset(&a, 0, sizeof a);
    a.links = L->links;
    a.reps = L->d_reps;
    a.nrep = L->nrep;
    a.nhit = nhit;
    a.use_rep_beta = L->batch ? 1 : 0;
    a.order = base_order(L);
    if (a.order == 7) {
        const RepDesc &r = L->reps[0];
        a.n0h = uint32_t(r.n[0]) / 2u;
        a.n1 = uint32_t(r.n[1]);
        a.n2 = uint32_t(r.n[2]);
        a.slab = uint32_t(r.n[3]) / 16u;
    } else if (a.order >= 2) {
        const RepDesc &r = L->reps[0];
        const uint32_t nl = uint32_t(r.n[L->nd - 1]), n2 = uint32_t(r.n[L->nd - 2]);
        a.n2 = n2;
        a.plane = r.Vh / (nl * n2);
        if (a.order == 2 || a.order == 4) {
            a.slab = nl / 8;
            a.cp = a.plane / uint32_t(L->block);
        } else {
            cube_tiles(L->block, a.order, &a.tile2, &a.tile3);
            a.slab = nl / (8u * a.tile3);
            a.cp = a.plane / 64u;
        }
    }
    if (stage_applies(L)) {
        a.stage = 1;
        a.stage_r = uint32_t(L->reps[0].n[0]) / 2u;
    }
    a.beta0 = b0;
    a.beta1 = b1;
    a.meas_classes = 1;
    a.sweep = L->d_sweep;
    a.stats = L->d_stats;
    a.total_blocks = L->upd_blocks;
    return a;
}

dim3 update_grid(const su3hb_lattice *L)
{
    uint32_t g = L->upd_blocks;
    if (base_order(L) == 1) g = (g + 7) / 8 * 8;
    return dim3(g);
}

int enqueue_plaquette(su3hb_lattice *L, hipStream_t st, double b0, double b1, double *series)
{
    PlaqArgs pa;
    std::memset(&pa, 0, sizeof pa);
    pa.links = L->links;
    pa.reps = L->d_reps;
    pa.nrep = L->nrep;
    pa.beta0 = b0;
    pa.beta1 = b1;
    pa.use_rep_beta = L->batch ? 1 : 0;
    pa.partials = L->d_partials;
    pa.total_blocks = L->plq_blocks;
    HIPCHK(launch_plaquette(L->nd, L->prec, dim3(L->plq_blocks), dim3(kPlaqBlock), st, pa));
    HIPCHK(launch_plaquette_finalize(st, L->d_reps, L->nrep, L->nd, L->d_partials, L->d_plaq, series,
                                     L->d_cursor));
    return SU3HB_OK;
}

// The plaquettes of a single-layer lattice are measured inside the parity-1
// update slices (see update.hip); two layers and batches use the plaquette
// kernel after the sweep.
// Single lattices (one or two layers) measure inside the parity-1 update
// slices; batches use the plaquette kernel.
bool fused_measure(const su3hb_lattice *L) { return !L->batch; }

// Measurement classes: one layer 1; two layers 3 (by base layer and tags).
int meas_classes(const su3hb_lattice *L) { return L->reps[0].nlat == 2 ? 3 : 1; }

int ensure_meas(su3hb_lattice *L)
{
    const size_t need = size_t(L->nd) * L->upd_blocks * size_t(meas_classes(L));
    if (need <= L->meas_cap) return SU3HB_OK;
    // captured sweeps hold the old buffer's address
    HIPCHK(hipStreamSynchronize(L->stream));
    drop_graph(L);
    hipFree(L->d_meas);
    L->d_meas = nullptr;
    L->meas_cap = 0;
    hipError_t e = hipMalloc(&L->d_meas, sizeof(double) * need);
    if (e != hipSuccess) return fail(SU3HB_ENOMEM, "measurement buffer: %s", hipGetErrorString(e));
    L->meas_cap = need;
    return SU3HB_OK;
}

// One sweep: parity 0 then 1, directions 0..D-1 inside, then the counter and
// (measure != 0) the plaquettes into the series.  `timed` (optional) records
// an event pair around every update launch and the plaquette launch.
int enqueue_sweep(su3hb_lattice *L, hipStream_t st, double b0, double b1, int nhit, int measure,
                  std::vector<int> *timed = nullptr, size_t *ev = nullptr)
{
    UpdateArgs a = update_args(L, b0, b1, nhit);
    const bool fused = measure && fused_measure(L);
    if (fused) {
        a.meas = L->d_meas;
        a.meas_classes = meas_classes(L);
    }
    const dim3 grid = update_grid(L), block(L->block);
    {
        // the largest LDS request of the sweep (a measured parity-1 slice)
        // must fit one block's share of the compute unit
        UpdateArgs m = a;
        m.parity = 1;
        size_t need = 0, limit = 0;
        HIPCHK(update_lds(L->nd, L->prec, L->waves, block, m, &need, &limit));
        if (limit == 0 || need > limit)
            return fail(SU3HB_EUNSUPPORTED, "update launch needs %zu bytes of LDS per block, the device allows %zu",
                        need, limit);
    }
    for (int p = 0; p < 2; ++p)
        for (int mu = 0; mu < L->nd; ++mu) {
            a.parity = p;
            a.mu = mu;
            a.reverse = (L->order & kOrderReverse) && ((p * L->nd + mu) & 1) ? 1 : 0;
            if (timed) HIPCHK(hipEventRecord(L->events[(*ev)++], st));
            HIPCHK(launch_update(L->nd, L->prec, L->waves, grid, block, st, a));
            if (timed) {
                HIPCHK(hipEventRecord(L->events[(*ev)++], st));
                timed->push_back(0);
            }
        }
    HIPCHK(launch_counter_add(st, L->d_sweep, 1));
    if (!measure) return SU3HB_OK;
    if (fused) {
        if (timed) HIPCHK(hipEventRecord(L->events[(*ev)++], st));
        HIPCHK(launch_measure_finalize(st, L->d_meas, L->nd, L->upd_blocks, meas_classes(L), double(L->reps[0].V),
                                       int(L->reps[0].nlat), b0, b1, L->d_plaq, L->d_series, L->d_cursor));
        if (timed) {
            HIPCHK(hipEventRecord(L->events[(*ev)++], st));
            timed->push_back(1);
        }
        return SU3HB_OK;
    }
    if (timed) HIPCHK(hipEventRecord(L->events[(*ev)++], st));
    PlaqArgs pa;
    std::memset(&pa, 0, sizeof pa);
    pa.links = L->links;
    pa.reps = L->d_reps;
    pa.nrep = L->nrep;
    pa.beta0 = b0;
    pa.beta1 = b1;
    pa.use_rep_beta = L->batch ? 1 : 0;
    pa.partials = L->d_partials;
    pa.total_blocks = L->plq_blocks;
    HIPCHK(launch_plaquette(L->nd, L->prec, dim3(L->plq_blocks), dim3(kPlaqBlock), st, pa));
    if (timed) {
        HIPCHK(hipEventRecord(L->events[(*ev)++], st));
        timed->push_back(1);
    }
    HIPCHK(launch_plaquette_finalize(st, L->d_reps, L->nrep, L->nd, L->d_partials, L->d_plaq, L->d_series,
                                     L->d_cursor));
    return SU3HB_OK;
}

int get_graph(su3hb_lattice *L, double b0, double b1, int nhit, int measure, hipGraphExec_t *out)
{
    GraphCache *slot = nullptr;
    for (auto &g : L->graphs)
        if (g.valid && g.b0 == b0 && g.b1 == b1 && g.nhit == nhit && g.measure == measure) {
            g.used = ++L->graph_tick;
            *out = g.exec;
            return SU3HB_OK;
        }
    // an empty slot, else the least recently used one
    for (auto &g : L->graphs)
        if (!slot || !g.valid || (slot->valid && g.used < slot->used)) {
            slot = &g;
            if (!g.valid) break;
        }
    drop_slot(*slot);
    HIPCHK(hipStreamBeginCapture(L->cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_sweep(L, L->cap, b0, b1, nhit, measure);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(L->cap, &graph);
    if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(SU3HB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return fail(SU3HB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    slot->valid = true;
    slot->b0 = b0;
    slot->b1 = b1;
    slot->nhit = nhit;
    slot->measure = measure;
    slot->graph = graph;
    slot->exec = exec;
    slot->used = ++L->graph_tick;
    *out = exec;
    return SU3HB_OK;
}

// The device counter (the Philox sweep word) is 32 bits: refuse to wrap it.
int check_sweep_room(const su3hb_lattice *L, int n)
{
    if (L->sweep + uint64_t(n < 0 ? 0 : n) > (uint64_t(1) << 32))
        return fail(SU3HB_EINVAL, "sweep %llu + %d passes 2^32: the Philox counter holds a 32-bit sweep index",
                    (unsigned long long)L->sweep, n);
    return SU3HB_OK;
}

int run_sweeps(su3hb_lattice *L, double b0, double b1, int nhit, int n, int measure)
{
    if (n <= 0) return SU3HB_OK;
    if (int rc = check_sweep_room(L, n)) return rc;
    if (measure && fused_measure(L)) {
        int rc = ensure_meas(L);
        if (rc) return rc;
    }
    if (L->use_graph) {
        hipGraphExec_t exec = nullptr;
        int rc = get_graph(L, b0, b1, nhit, measure, &exec);
        if (rc) return rc;
        for (int i = 0; i < n; ++i) HIPCHK(hipGraphLaunch(exec, L->stream));
    } else {
        for (int i = 0; i < n; ++i) {
            int rc = enqueue_sweep(L, L->stream, b0, b1, nhit, measure);
            if (rc) return rc;
        }
    }
    L->sweep += uint64_t(n);
    return SU3HB_OK;
}

int read_stats(su3hb_lattice *L, su3hb_stats *out)
{
    StatSlot s;
    HIPCHK(launch_stats_reduce(L->stream, L->d_stats, L->d_stats_out));
    HIPCHK(hipMemcpyAsync(&s, L->d_stats_out, sizeof s, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    for (int i = 0; i < 3; ++i) {
        out->attempts[i] = s.attempts[i];
        out->accepts[i] = s.accepts[i];
    }
    out->link_updates = s.updates;
    out->dtrace = s.dtrace;
    return SU3HB_OK;
}

int check_sweep_args(double b0, double b1, int nhit, int n)
{
    if (!std::isfinite(b0) || !std::isfinite(b1)) return fail(SU3HB_EINVAL, "beta must be finite");
    if (nhit < 1 || nhit > 32767) return fail(SU3HB_EINVAL, "n_hit = %d outside 1..32767", nhit);
    if (n < 0) return fail(SU3HB_EINVAL, "n_sweeps = %d is negative", n);
    return SU3HB_OK;
}

int ensure_stage(su3hb_lattice *L)
{
    if (!L->d_stage) {
        hipError_t e = hipMalloc(&L->d_stage, kStageBytes);
        if (e != hipSuccess) return fail(SU3HB_ENOMEM, "staging buffer: %s", hipGetErrorString(e));
    }
    return SU3HB_OK;
}

int get_replica_links(su3hb_lattice *L, int r, double *host, size_t n)
{
    const RepDesc &rep = L->reps[r];
    const uint64_t nsites = uint64_t(rep.nlat) * rep.V;
    const size_t per_site = size_t(L->nd) * 18;
    if (!host) return fail(SU3HB_EINVAL, "host buffer is NULL");
    if (n != nsites * per_site)
        return fail(SU3HB_EINVAL, "n = %zu, expected nlat*V*D*18 = %zu", n, size_t(nsites * per_site));
    int rc = ensure_stage(L);
    if (rc) return rc;
    const uint64_t chunk = kStageBytes / (per_site * sizeof(double));
    for (uint64_t c0 = 0; c0 < nsites; c0 += chunk) {
        const uint32_t cnt = uint32_t(std::min<uint64_t>(chunk, nsites - c0));
        HIPCHK(launch_pack(L->nd, L->prec, L->stream, L->links, L->d_reps, r, c0, cnt, L->d_stage));
        HIPCHK(hipMemcpyAsync(host + c0 * per_site, L->d_stage, size_t(cnt) * per_site * sizeof(double),
                              hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    return SU3HB_OK;
}

int set_replica_links(su3hb_lattice *L, int r, const double *host, size_t n)
{
    const RepDesc &rep = L->reps[r];
    const uint64_t nsites = uint64_t(rep.nlat) * rep.V;
    const size_t per_site = size_t(L->nd) * 18;
    if (!host) return fail(SU3HB_EINVAL, "host buffer is NULL");
    if (n != nsites * per_site)
        return fail(SU3HB_EINVAL, "n = %zu, expected nlat*V*D*18 = %zu", n, size_t(nsites * per_site));
    int rc = ensure_stage(L);
    if (rc) return rc;
    const double tol = is_fp32(L->prec) ? 1e-6 : 1e-10;
    const uint64_t chunk = kStageBytes / (per_site * sizeof(double));
    const bool single = nsites <= chunk;
    // pass 1: validate every matrix on the GPU before anything is written
    HIPCHK(launch_u64_zero(L->stream, L->d_maxdef, 1));
    for (uint64_t c0 = 0; c0 < nsites; c0 += chunk) {
        const uint32_t cnt = uint32_t(std::min<uint64_t>(chunk, nsites - c0));
        HIPCHK(hipMemcpyAsync(L->d_stage, host + c0 * per_site, size_t(cnt) * per_site * sizeof(double),
                              hipMemcpyHostToDevice, L->stream));
        HIPCHK(launch_validate(L->stream, L->d_stage, uint64_t(cnt) * L->nd, L->d_maxdef));
        if (!single) HIPCHK(hipStreamSynchronize(L->stream));
    }
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, L->d_maxdef, sizeof bits, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    double maxdef;
    std::memcpy(&maxdef, &bits, sizeof maxdef);
    if (!(maxdef <= tol))
        return fail(SU3HB_ENOTSU3, "input is not SU(3): max defect %.3g exceeds %.1g", maxdef, tol);
    // pass 2: convert into the internal storage
    for (uint64_t c0 = 0; c0 < nsites; c0 += chunk) {
        const uint32_t cnt = uint32_t(std::min<uint64_t>(chunk, nsites - c0));
        if (!single)
            HIPCHK(hipMemcpyAsync(L->d_stage, host + c0 * per_site, size_t(cnt) * per_site * sizeof(double),
                                  hipMemcpyHostToDevice, L->stream));
        HIPCHK(launch_unpack(L->nd, L->prec, L->stream, L->links, L->d_reps, r, c0, cnt, L->d_stage));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    return SU3HB_OK;
}

std::string tune_key(const su3hb_lattice *L)
{
    std::string k = std::to_string(L->prec) + ":" + std::to_string(L->nd);
    for (auto &r : L->reps) {
        k += "|";
        for (int i = 0; i < L->nd; ++i) k += std::to_string(r.n[i]) + ",";
        k += std::to_string(r.nlat);
    }
    return k;
}

int apply_launch(su3hb_lattice *L, int block, int order, int waves)
{
    if (block != 64 && block != 128 && block != 256)
        return fail(SU3HB_EINVAL, "block = %d, expected 64, 128 or 256", block);
    if (order < 0 || (order & ~(kOrderReverse | kOrderStage)) > 7)
        return fail(SU3HB_EINVAL, "order = %d, expected 0 .. 7, optionally + %d and + %d", order, kOrderReverse,
                    kOrderStage);
    if (waves != 2 && !(waves == 3 && L->nd == 4) && !(waves == 4 && L->nd == 4 && is_fp32(L->prec)))
        return fail(SU3HB_EINVAL, "waves = %d: 2, or 3 for D = 4, or 4 for D = 4 with FP32 links", waves);
    HIPCHK(hipStreamSynchronize(L->stream));
    drop_graph(L);
    const int old_block = L->block, old_order = L->order, old_waves = L->waves;
    L->block = block;
    L->order = order;
    L->waves = waves;
    layout_reps(L);
    // a measured parity-1 slice asks for the most LDS: staple snapshots and,
    // when staging, the staging areas
    size_t need = 0, limit = 0;
    UpdateArgs m = update_args(L, 6.0, 6.0, 8);
    m.parity = 1;
    if (fused_measure(L)) {
        m.meas = reinterpret_cast<double *>(uintptr_t(256));  // only tested for null
        m.meas_classes = meas_classes(L);
    }
    const hipError_t e = update_lds(L->nd, L->prec, L->waves, dim3(block), m, &need, &limit);
    if (e != hipSuccess || limit == 0 || need > limit) {
        L->block = old_block;
        L->order = old_order;
        L->waves = old_waves;
        layout_reps(L);
        if (e != hipSuccess) return fail(SU3HB_EHIP, "LDS query: %s", hipGetErrorString(e));
        return fail(SU3HB_EUNSUPPORTED, "launch (%d, %d, %d) needs %zu bytes of LDS per block, the device allows %zu",
                    block, order, waves, need, limit);
    }
    return upload_reps(L);
}

int ensure_events(su3hb_lattice *L, size_t n)
{
    while (L->events.size() < n) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        L->events.push_back(e);
    }
    return SU3HB_OK;
}

// ---------------------------------------------------------------------------
// Scratch of su3hb_sweep_measure_static: a file-scope device array, so that
// call allocates nothing.  Each GPU holds its own copy until the process
// ends; every call on a GPU shares it (calls that overlap on one GPU race).
// Layout (byte offsets): the replica descriptor, the sweep counter, the
// series cursor, the last plaquettes, the statistics slots, then the fused
// measurement's per-block partial sums.
constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr size_t kScrRep = 0, kScrSweep = 256, kScrCursor = 512, kScrPlaq = 768, kScrStats = 1024;
constexpr size_t kScrMeas = kScrStats + sizeof(StatSlot) * kStatSlots;
constexpr size_t kScratchMeasDoubles = (kScratchBytes - kScrMeas) / sizeof(double);
static_assert(sizeof(RepDesc) <= kScrSweep - kScrRep, "replica descriptor overflows its scratch slot");
static_assert(kScrMeas % 256 == 0, "partial sums start on a 256-byte boundary");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  The host-side name `scratch` is not a
// device address and is never passed to a kernel.
int scratch_base(unsigned char **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SU3HB_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SU3HB_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SU3HB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

const char *su3hb_last_error(void) { return g_err.c_str(); }

int su3hb_links_bytes(const su3hb_params *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SU3HB_EINVAL, "NULL argument");
    uint64_t V;
    int rc = check_extents(p->nd, p->extents, &V);
    if (rc) return rc;
    if (p->nlat != 1 && p->nlat != 2) return fail(SU3HB_EINVAL, "nlat = %d, expected 1 or 2", p->nlat);
    if (p->precision < 0 || p->precision > 3) return fail(SU3HB_EINVAL, "unknown precision %d", p->precision);
    // two slabs (parities) of whole tiles per layer and direction
    *bytes = size_t(p->nlat) * p->nd * 2 * size_t(padded_half(uint32_t(V / 2))) * size_t(bytes_per_link(p->precision));
    return SU3HB_OK;
}

int su3hb_init_lattice(su3hb_lattice **out, const su3hb_params *p)
{
    if (!out) return fail(SU3HB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(SU3HB_EINVAL, "params is NULL");
    uint64_t V;
    int rc = check_extents(p->nd, p->extents, &V);
    if (rc) return rc;
    if (p->nlat != 1 && p->nlat != 2) return fail(SU3HB_EINVAL, "nlat = %d, expected 1 or 2", p->nlat);
    if (p->nlat == 1 && (p->dlt_mask != 0 || p->lat2test))
        return fail(SU3HB_EINVAL, "dlt_mask and lat2test need nlat = 2");
    if (p->dlt_mask >> p->nd) return fail(SU3HB_EINVAL, "dlt_mask has bits beyond direction %d", p->nd - 1);
    if (p->precision < 0 || p->precision > 3) return fail(SU3HB_EINVAL, "unknown precision %d", p->precision);
    if (p->start < 0 || p->start > 2) return fail(SU3HB_EINVAL, "unknown start %d", p->start);
    if (double(p->nlat) * double(V) * p->nd > 4294967295.0)
        return fail(SU3HB_EINVAL, "more than 2^32 links: the Philox counter holds a 32-bit link id");

    su3hb_lattice *L = new su3hb_lattice;
    L->nd = p->nd;
    L->prec = p->precision;
    L->nrep = 1;
    L->batch = false;
    L->seed = p->seed;
    L->stream = reinterpret_cast<hipStream_t>(p->hip_stream);
    L->reps.push_back(make_rep(p->nd, p->extents, p->nlat, p->nlat == 2 ? p->dlt_mask : 0u, p->lat2test,
                               p->seed, 0.0, 0.0));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(L));
        if (it != g_tune_cache.end()) {
            L->block = it->second.block;
            L->order = it->second.order;
            L->waves = it->second.waves;
        }
    }
    rc = adopt_or_alloc_links(L, p->device_links, p->device_bytes);
    if (!rc) rc = alloc_common(L);
    if (!rc) rc = start_replica(L, 0, p->start);
    if (!rc) {
        hipError_t e = hipStreamSynchronize(L->stream);
        if (e != hipSuccess) rc = fail(SU3HB_EHIP, "init: %s", hipGetErrorString(e));
    }
    if (rc) {
        destroy(L);
        return rc;
    }
    *out = L;
    return SU3HB_OK;
}

void su3hb_free(su3hb_lattice *lat) { destroy(lat); }

int su3hb_sweep(su3hb_lattice *L, double beta0, double beta1, int n_hit, int n_sweeps, su3hb_stats *stats)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    int rc = check_sweep_args(beta0, beta1, n_hit, n_sweeps);
    if (rc) return rc;
    HIPCHK(hipSetDevice(L->device));
    if (stats) HIPCHK(launch_stats_zero(L->stream, L->d_stats));
    rc = run_sweeps(L, beta0, beta1, n_hit, n_sweeps, 0);
    if (rc) return rc;
    if (stats) return read_stats(L, stats);
    return SU3HB_OK;
}

int su3hb_overrelax(su3hb_lattice *L, double beta0, double beta1, int n_sweeps, su3hb_stats *stats)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    int rc = check_sweep_args(beta0, beta1, 1, n_sweeps);
    if (rc) return rc;
    HIPCHK(hipSetDevice(L->device));
    if (stats) HIPCHK(launch_stats_zero(L->stream, L->d_stats));
    rc = run_sweeps(L, beta0, beta1, 0, n_sweeps, 0);  // n_hit 0: overrelaxation
    if (rc) return rc;
    if (stats) return read_stats(L, stats);
    return SU3HB_OK;
}

int su3hb_sweep_measure(su3hb_lattice *L, double beta0, double beta1, int n_hit, int n_sweeps, double *series,
                        su3hb_stats *stats)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (L->batch) return fail(SU3HB_EINVAL, "use su3hb_batch_plaquette for batches");
    if (!series && n_sweeps > 0) return fail(SU3HB_EINVAL, "series is NULL");
    int rc = check_sweep_args(beta0, beta1, n_hit, n_sweeps);
    if (rc) return rc;
    HIPCHK(hipSetDevice(L->device));
    if (stats) HIPCHK(launch_stats_zero(L->stream, L->d_stats));
    for (int done = 0; done < n_sweeps;) {
        const int chunk = std::min<int>(int(kSeriesCap), n_sweeps - done);
        HIPCHK(launch_counter_set(L->stream, L->d_cursor, 0));
        rc = run_sweeps(L, beta0, beta1, n_hit, chunk, 1);
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(series + size_t(done) * 6, L->d_series, sizeof(double) * 6 * chunk,
                              hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
        done += chunk;
    }
    if (stats) return read_stats(L, stats);
    return SU3HB_OK;
}

int su3hb_plaquette(su3hb_lattice *L, double beta0, double beta1, double out[6])
{
    if (!L || !out) return fail(SU3HB_EINVAL, "NULL argument");
    if (L->batch) return fail(SU3HB_EINVAL, "use su3hb_batch_plaquette for batches");
    HIPCHK(hipSetDevice(L->device));
    int rc = enqueue_plaquette(L, L->stream, beta0, beta1, nullptr);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(out, L->d_plaq, sizeof(double) * 6, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    return SU3HB_OK;
}

int su3hb_get_links(const su3hb_lattice *Lc, double *host, size_t n)
{
    su3hb_lattice *L = const_cast<su3hb_lattice *>(Lc);
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (L->batch) return fail(SU3HB_EINVAL, "use su3hb_batch_get_links for batches");
    HIPCHK(hipSetDevice(L->device));
    return get_replica_links(L, 0, host, n);
}

int su3hb_set_links(su3hb_lattice *L, const double *host, size_t n)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (L->batch) return fail(SU3HB_EINVAL, "use su3hb_batch_set_links for batches");
    HIPCHK(hipSetDevice(L->device));
    return set_replica_links(L, 0, host, n);
}

int su3hb_get_state(const su3hb_lattice *L, uint64_t *seed, uint64_t *sweep)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (seed) *seed = L->seed;
    if (sweep) *sweep = L->sweep;
    return SU3HB_OK;
}

int su3hb_set_state(su3hb_lattice *L, uint64_t seed, uint64_t sweep)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (L->batch) return fail(SU3HB_EINVAL, "batches keep one seed per replica");
    if (sweep >= (uint64_t(1) << 32))
        return fail(SU3HB_EINVAL, "sweep = %llu: the Philox counter holds a 32-bit sweep index",
                    (unsigned long long)sweep);
    HIPCHK(hipSetDevice(L->device));
    L->seed = seed;
    L->reps[0].key0 = uint32_t(seed);
    L->reps[0].key1 = uint32_t(seed >> 32);
    int rc = upload_reps(L);
    if (rc) return rc;
    L->sweep = sweep;
    HIPCHK(launch_counter_set(L->stream, L->d_sweep, uint32_t(sweep)));
    HIPCHK(hipStreamSynchronize(L->stream));
    return SU3HB_OK;
}

int su3hb_set_launch(su3hb_lattice *L, int block, int order, int waves)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    HIPCHK(hipSetDevice(L->device));
    return apply_launch(L, block, order, waves);
}

int su3hb_get_launch(const su3hb_lattice *L, int *block, int *order, int *waves)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (block) *block = L->block;
    if (order) *order = effective_order(L);
    if (waves) *waves = L->waves;
    return SU3HB_OK;
}

int su3hb_autotune(su3hb_lattice *L, int budget_ms)
{
    if (!L) return fail(SU3HB_EINVAL, "lattice is NULL");
    if (budget_ms < 1) return fail(SU3HB_EINVAL, "budget_ms must be positive");
    HIPCHK(hipSetDevice(L->device));
    const std::string key = tune_key(L);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end())
            return apply_launch(L, it->second.block, it->second.order, it->second.waves);
    }
    // keep the state: links, sweep counter and statistics are restored below
    void *backup = nullptr;
    hipError_t e = hipMalloc(&backup, L->links_bytes);
    if (e != hipSuccess) return fail(SU3HB_ENOMEM, "autotune backup: %s", hipGetErrorString(e));
    struct Free {
        void *p;
        ~Free() { hipFree(p); }
    } guard{backup};
    HIPCHK(hipMemcpyAsync(backup, L->links, L->links_bytes, hipMemcpyDeviceToDevice, L->stream));
    const uint64_t sweep0 = L->sweep;
    // candidate shapes: every block size and order, both occupancy targets for
    // D = 4; orders 2 to 6 only where they apply (otherwise they would repeat
    // another order), orders 3, 5 and 6 only with more than one wave per block
    std::vector<Shape> cands;
    for (int waves : {2, 3, 4}) {
        if (waves >= 3 && L->nd != 4) continue;
        if (waves == 4 && !is_fp32(L->prec)) continue;
        for (int block : {256, 128, 64})
            for (int order : {0, 1, 2, 3, 4, 5, 6, 7}) {
                if ((order == 2 || order == 4) && !slab_order_ok(L, block)) continue;
                if (order == 7 && !tile4_order_ok(L, block)) continue;
                if (is_cube_order(order) && (block == 64 || !cube_order_ok(L, block, order))) continue;
                cands.push_back(Shape{block, order, waves});
                cands.push_back(Shape{block, order | kOrderReverse, waves});
                if (order != 7 && !L->batch && L->reps[0].nlat == 1) {
                    cands.push_back(Shape{block, order | kOrderStage, waves});
                    cands.push_back(Shape{block, order | kOrderReverse | kOrderStage, waves});
                }
            }
    }
    const double b = L->batch ? 0.0 : 6.0;
    // single lattices are timed with the fused measurement (its parity-1
    // slices hold the staple snapshots in LDS, which decides the occupancy
    // of some shapes); the series cursor is reset before every timed batch of
    // at most 64 sweeps and after the tuning
    const int meas = fused_measure(L) ? 1 : 0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // two passes over the candidates, each keeping its faster pass, so that a
    // slow moment of the machine does not decide the choice
    std::vector<float> per(cands.size(), 1e30f);
    size_t best_i = 0;
    const bool graph = L->use_graph;
    L->use_graph = false;
    int rc = SU3HB_OK;
    // time candidate i: its launch, a warm-up sweep, then timed batches of
    // at least min_reps sweeps, doubling until a batch takes target_ms (at
    // most 64 sweeps); ms per sweep, or a negative value for a shape whose
    // LDS does not fit (not a candidate)
    auto time_cand = [&](size_t i, int min_reps, double target_ms, float *out) -> int {
        int r = apply_launch(L, cands[i].block, cands[i].order, cands[i].waves);
        if (r == SU3HB_EUNSUPPORTED) {
            *out = -1.f;
            return SU3HB_OK;
        }
        if (r) return r;
        if (meas && (r = ensure_meas(L)) != SU3HB_OK) return r;
        if (hipSuccess != launch_counter_set(L->stream, L->d_cursor, 0)) return fail(SU3HB_EHIP, "cursor");
        if ((r = enqueue_sweep(L, L->stream, b, b, 8, meas)) != SU3HB_OK) return r;  // warm-up
        int reps = min_reps;
        float ms = 0.f;
        for (;;) {
            if (hipSuccess != launch_counter_set(L->stream, L->d_cursor, 0)) return fail(SU3HB_EHIP, "cursor");
            if (hipEventRecord(e0, L->stream) != hipSuccess) return fail(SU3HB_EHIP, "event");
            for (int k = 0; k < reps; ++k)
                if ((r = enqueue_sweep(L, L->stream, b, b, 8, meas)) != SU3HB_OK) return r;
            if (hipEventRecord(e1, L->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(SU3HB_EHIP, "event");
            hipEventElapsedTime(&ms, e0, e1);
            if (ms >= target_ms || reps >= 64) break;
            reps *= 2;
        }
        *out = ms / float(reps);
        return SU3HB_OK;
    };
    // two passes over every candidate with about a quarter of the budget each
    for (int pass = 0; pass < 2 && !rc; ++pass)
        for (size_t i = 0; i < cands.size() && !rc; ++i) {
            float t = 0.f;
            rc = time_cand(i, 1, double(budget_ms) / (4.0 * double(cands.size())), &t);
            if (!rc && t >= 0.f) per[i] = std::min(per[i], t);
        }
    // the six fastest again, in three interleaved rounds of at least two
    // sweeps each, with the other half of the budget: single sweeps of
    // shapes within a per cent of each other do not order them reliably
    std::vector<size_t> rank(cands.size());
    for (size_t i = 0; i < rank.size(); ++i) rank[i] = i;
    const size_t K = std::min<size_t>(6, rank.size());
    std::partial_sort(rank.begin(), rank.begin() + K, rank.end(), [&](size_t x, size_t y) { return per[x] < per[y]; });
    std::vector<float> fin(K, 1e30f);
    for (int round = 0; round < 3 && !rc; ++round)
        for (size_t k = 0; k < K && !rc; ++k) {
            if (per[rank[k]] >= 1e30f) continue;
            float t = 0.f;
            rc = time_cand(rank[k], 2, double(budget_ms) / (6.0 * double(K)), &t);
            if (!rc && t >= 0.f) fin[k] = std::min(fin[k], t);
        }
    {
        size_t bk = 0;
        for (size_t k = 1; k < K; ++k)
            if (fin[k] < fin[bk]) bk = k;
        best_i = rank[bk];
    }
    L->use_graph = graph;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    HIPCHK(hipMemcpyAsync(L->links, backup, L->links_bytes, hipMemcpyDeviceToDevice, L->stream));
    HIPCHK(launch_counter_set(L->stream, L->d_sweep, uint32_t(sweep0)));
    HIPCHK(launch_counter_set(L->stream, L->d_cursor, 0));
    HIPCHK(launch_stats_zero(L->stream, L->d_stats));
    HIPCHK(hipStreamSynchronize(L->stream));
    L->sweep = sweep0;
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = cands[best_i];
    }
    return apply_launch(L, cands[best_i].block, cands[best_i].order, cands[best_i].waves);
}

int su3hb_sweep_timed(su3hb_lattice *L, double beta0, double beta1, int n_hit, int n_sweeps, int measure,
                      double *series, double timing[4])
{
    if (!L || !timing) return fail(SU3HB_EINVAL, "NULL argument");
    if (L->batch && measure) return fail(SU3HB_EINVAL, "batches measure with su3hb_batch_plaquette");
    if (measure && !series && n_sweeps > 0) return fail(SU3HB_EINVAL, "series is NULL");
    if (measure && n_sweeps > int(kSeriesCap))
        return fail(SU3HB_EINVAL, "at most %u measured sweeps per call", kSeriesCap);
    int rc = check_sweep_args(beta0, beta1, n_hit == 0 ? 1 : n_hit, n_sweeps);  // 0: overrelaxation
    if (!rc) rc = check_sweep_room(L, n_sweeps);
    if (rc) return rc;
    HIPCHK(hipSetDevice(L->device));
    if (measure && fused_measure(L)) {
        rc = ensure_meas(L);
        if (rc) return rc;
    }
    const size_t launches = size_t(n_sweeps) * (size_t(2 * L->nd) + (measure ? 1 : 0));
    rc = ensure_events(L, 2 * launches);
    if (rc) return rc;
    if (measure) HIPCHK(launch_counter_set(L->stream, L->d_cursor, 0));
    size_t ev = 0;
    std::vector<int> kinds;
    kinds.reserve(launches);
    for (int sw = 0; sw < n_sweeps; ++sw) {
        rc = enqueue_sweep(L, L->stream, beta0, beta1, n_hit, measure, &kinds, &ev);
        if (rc) return rc;
    }
    L->sweep += uint64_t(n_sweeps);
    HIPCHK(hipStreamSynchronize(L->stream));
    double t_upd = 0, t_plq = 0, n_upd = 0, n_plq = 0;
    for (size_t i = 0; i < kinds.size(); ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, L->events[2 * i], L->events[2 * i + 1]));
        if (kinds[i]) {
            t_plq += ms;
            n_plq += 1;
        } else {
            t_upd += ms;
            n_upd += 1;
        }
    }
    timing[0] = t_upd;
    timing[1] = n_upd;
    timing[2] = t_plq;
    timing[3] = n_plq;
    if (measure && n_sweeps > 0) {
        HIPCHK(hipMemcpyAsync(series, L->d_series, sizeof(double) * 6 * n_sweeps, hipMemcpyDeviceToHost,
                              L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    return SU3HB_OK;
}

// ---------------------------------------------------------------------------
// batches

int su3hb_batch_create(su3hb_batch **out, int nd, const su3hb_replica_desc *reps, int n, int precision,
                       void *hip_stream)
{
    if (!out) return fail(SU3HB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!reps || n < 1) return fail(SU3HB_EINVAL, "need at least one replica");
    if (precision < 0 || precision > 3) return fail(SU3HB_EINVAL, "unknown precision %d", precision);
    for (int r = 0; r < n; ++r) {
        uint64_t V;
        int rc = check_extents(nd, reps[r].extents, &V);
        if (rc) return fail(rc, "replica %d: %s", r, g_err.c_str());
        if (!std::isfinite(reps[r].beta)) return fail(SU3HB_EINVAL, "replica %d: beta not finite", r);
        if (reps[r].start < 0 || reps[r].start > 2) return fail(SU3HB_EINVAL, "replica %d: bad start", r);
        // each replica numbers its links from 0 in the Philox counter (32 bits)
        if (V * uint64_t(nd) > uint64_t(0xFFFFFFFFu))
            return fail(SU3HB_EINVAL, "replica %d: more than 2^32 links: the Philox counter holds a 32-bit link id", r);
    }
    su3hb_lattice *L = new su3hb_lattice;
    L->nd = nd;
    L->prec = precision;
    L->nrep = n;
    L->batch = true;
    L->stream = reinterpret_cast<hipStream_t>(hip_stream);
    for (int r = 0; r < n; ++r)
        L->reps.push_back(make_rep(nd, reps[r].extents, 1, 0u, 0, reps[r].seed, reps[r].beta, reps[r].beta));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(L));
        if (it != g_tune_cache.end()) {
            L->block = it->second.block;
            L->order = it->second.order;
            L->waves = it->second.waves;
        }
    }
    int rc = adopt_or_alloc_links(L, nullptr, 0);
    if (!rc) rc = alloc_common(L);
    for (int r = 0; r < n && !rc; ++r) rc = start_replica(L, r, reps[r].start);
    if (!rc) {
        hipError_t e = hipStreamSynchronize(L->stream);
        if (e != hipSuccess) rc = fail(SU3HB_EHIP, "batch init: %s", hipGetErrorString(e));
    }
    if (rc) {
        destroy(L);
        return rc;
    }
    *out = L;
    return SU3HB_OK;
}

int su3hb_batch_sweep(su3hb_batch *L, int n_hit, int n_sweeps, int mode, su3hb_stats *stats)
{
    if (!L || !L->batch) return fail(SU3HB_EINVAL, "not a batch");
    int rc = check_sweep_args(0.0, 0.0, n_hit, n_sweeps);
    if (rc) return rc;
    if (mode != 0 && mode != 1) return fail(SU3HB_EINVAL, "mode = %d, expected 0 or 1", mode);
    HIPCHK(hipSetDevice(L->device));
    if (stats) HIPCHK(launch_stats_zero(L->stream, L->d_stats));
    if (mode == 0) {
        rc = run_sweeps(L, 0.0, 0.0, n_hit, n_sweeps, 0);
        if (rc) return rc;
    } else if (n_sweeps > 0) {
        // one resident block per CU (as many as fit), slices separated by a
        // grid barrier; a barrier that gives up raises a flag checked below
        if (int rc2 = check_sweep_room(L, n_sweeps)) return rc2;
        int per_cu = 0;
        HIPCHK(persistent_max_blocks(L->nd, L->prec, &per_cu));
        if (per_cu < 1) return fail(SU3HB_EUNSUPPORTED, "persistent kernel cannot be resident");
        const int blocks = int(std::min<uint64_t>(uint64_t(per_cu) * L->num_cus, L->pers_blocks));
        UpdateArgs a = update_args(L, 0.0, 0.0, n_hit);
        a.order = 0;
        a.persistent = 1;
        a.barrier = L->d_bar;
        a.total_blocks = L->pers_blocks;
        // bounded sweeps per launch keep the barrier counters far from overflow
        constexpr int kChunk = 1 << 16;
        for (int done = 0; done < n_sweeps;) {
            const int n = std::min(kChunk, n_sweeps - done);
            HIPCHK(launch_u32_zero(L->stream, L->d_bar, kBarrierWords));
            HIPCHK(launch_update_persistent(L->nd, L->prec, blocks, L->stream, a, n));
            HIPCHK(launch_counter_add(L->stream, L->d_sweep, uint32_t(n)));
            done += n;
        }
        L->sweep += uint64_t(n_sweeps);
        uint32_t flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, L->d_bar + kBarrierFlag, sizeof flag, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
        if (flag) return fail(SU3HB_EHIP, "persistent sweep: a grid barrier timed out; the links are not valid");
    }
    if (stats) return read_stats(L, stats);
    return SU3HB_OK;
}

int su3hb_batch_plaquette(su3hb_batch *L, double *out, size_t n)
{
    if (!L || !L->batch || !out) return fail(SU3HB_EINVAL, "bad arguments");
    if (n != size_t(L->nrep) * 6) return fail(SU3HB_EINVAL, "n = %zu, expected 6 per replica", n);
    HIPCHK(hipSetDevice(L->device));
    int rc = enqueue_plaquette(L, L->stream, 0.0, 0.0, nullptr);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(out, L->d_plaq, sizeof(double) * n, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    return SU3HB_OK;
}

int su3hb_batch_get_links(su3hb_batch *L, int replica, double *host, size_t n)
{
    if (!L || !L->batch) return fail(SU3HB_EINVAL, "not a batch");
    if (replica < 0 || replica >= L->nrep) return fail(SU3HB_EINVAL, "replica %d out of range", replica);
    HIPCHK(hipSetDevice(L->device));
    return get_replica_links(L, replica, host, n);
}

int su3hb_batch_set_links(su3hb_batch *L, int replica, const double *host, size_t n)
{
    if (!L || !L->batch) return fail(SU3HB_EINVAL, "not a batch");
    if (replica < 0 || replica >= L->nrep) return fail(SU3HB_EINVAL, "replica %d out of range", replica);
    HIPCHK(hipSetDevice(L->device));
    return set_replica_links(L, replica, host, n);
}

void su3hb_batch_free(su3hb_batch *b) { destroy(b); }

// ---------------------------------------------------------------------------
// measured sweeps that allocate nothing

int su3hb_sweep_measure_static(const su3hb_params *p, double beta0, double beta1, int n_hit, int n_sweeps,
                               uint64_t sweep0, double *series)
{
    // every check comes before the first device call
    if (!p) return fail(SU3HB_EINVAL, "params is NULL");
    uint64_t V;
    int rc = check_extents(p->nd, p->extents, &V);
    if (rc) return rc;
    if (p->nlat != 1 && p->nlat != 2) return fail(SU3HB_EINVAL, "nlat = %d, expected 1 or 2", p->nlat);
    if (p->nlat == 1 && (p->dlt_mask != 0 || p->lat2test))
        return fail(SU3HB_EINVAL, "dlt_mask and lat2test need nlat = 2");
    if (p->dlt_mask >> p->nd) return fail(SU3HB_EINVAL, "dlt_mask has bits beyond direction %d", p->nd - 1);
    if (p->precision < 0 || p->precision > 3) return fail(SU3HB_EINVAL, "unknown precision %d", p->precision);
    if (double(p->nlat) * double(V) * p->nd > 4294967295.0)
        return fail(SU3HB_EINVAL, "more than 2^32 links: the Philox counter holds a 32-bit link id");
    rc = check_sweep_args(beta0, beta1, n_hit, n_sweeps);
    if (rc) return rc;
    if (sweep0 + uint64_t(n_sweeps) > (uint64_t(1) << 32))
        return fail(SU3HB_EINVAL, "sweep %llu + %d passes 2^32: the Philox counter holds a 32-bit sweep index",
                    (unsigned long long)sweep0, n_sweeps);
    if (!p->device_links) return fail(SU3HB_EINVAL, "device_links is NULL: the links are the caller's");
    if (reinterpret_cast<uintptr_t>(p->device_links) % 16)
        return fail(SU3HB_EINVAL, "device buffer must be 16-byte aligned");
    const size_t need_links = size_t(p->nlat) * p->nd * 2 * size_t(padded_half(uint32_t(V / 2))) *
                              size_t(bytes_per_link(p->precision));
    if (p->device_bytes < need_links)
        return fail(SU3HB_EINVAL, "device buffer holds %zu bytes, the links need %zu", p->device_bytes, need_links);

    // launch shape: 256-thread blocks, each XCD a contiguous run of blocks,
    // 2 waves per SIMD (links are bit-identical for every shape)
    constexpr int kBlock = 256;
    RepDesc rep = make_rep(p->nd, p->extents, p->nlat, p->nlat == 2 ? p->dlt_mask : 0u, p->lat2test, p->seed,
                           0.0, 0.0);
    rep.upd_block0 = 0;
    rep.upd_blocks = (rep.nlat * rep.Vh + kBlock - 1) / kBlock;
    const int nc = p->nlat == 2 ? 3 : 1;
    const size_t meas_doubles = size_t(p->nd) * rep.upd_blocks * size_t(nc);
    if (series && meas_doubles > kScratchMeasDoubles)
        return fail(SU3HB_EINVAL,
                    "lattice too large for the static scratch: the measurement needs %zu partial sums, the scratch "
                    "holds %zu (%zu bytes)",
                    meas_doubles, kScratchMeasDoubles, kScratchBytes);
    if (n_sweeps == 0) return SU3HB_OK;

    unsigned char *base = nullptr;
    rc = scratch_base(&base);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(p->hip_stream);
    RepDesc *d_rep = reinterpret_cast<RepDesc *>(base + kScrRep);
    uint32_t *d_sweep = reinterpret_cast<uint32_t *>(base + kScrSweep);
    uint32_t *d_cursor = reinterpret_cast<uint32_t *>(base + kScrCursor);
    double *d_plaq = reinterpret_cast<double *>(base + kScrPlaq);
    StatSlot *d_stats = reinterpret_cast<StatSlot *>(base + kScrStats);
    double *d_meas = reinterpret_cast<double *>(base + kScrMeas);

    UpdateArgs a;
    std::memset(&a, 0, sizeof a);
    a.links = p->device_links;
    a.reps = d_rep;
    a.nrep = 1;
    a.nhit = n_hit;
    a.order = 1;
    a.beta0 = beta0;
    a.beta1 = beta1;
    a.meas_classes = nc;
    a.sweep = d_sweep;
    a.stats = d_stats;
    a.total_blocks = rep.upd_blocks;
    a.meas = series ? d_meas : nullptr;
    const dim3 grid((rep.upd_blocks + 7) / 8 * 8), block(kBlock);
    {
        UpdateArgs m = a;
        m.parity = 1;
        size_t need = 0, limit = 0;
        HIPCHK(update_lds(p->nd, p->precision, kDefaultWaves, block, m, &need, &limit));
        if (limit == 0 || need > limit)
            return fail(SU3HB_EUNSUPPORTED, "update launch needs %zu bytes of LDS per block, the device allows %zu",
                        need, limit);
    }
    // set-up: no memset nodes (kernels clear what must start at zero)
    HIPCHK(launch_rep_set(st, rep, d_rep));
    HIPCHK(launch_counter_set(st, d_sweep, uint32_t(sweep0)));
    HIPCHK(launch_counter_set(st, d_cursor, 0));
    HIPCHK(launch_stats_zero(st, d_stats));
    for (int sw = 0; sw < n_sweeps; ++sw) {
        for (int par = 0; par < 2; ++par)
            for (int mu = 0; mu < p->nd; ++mu) {
                a.parity = par;
                a.mu = mu;
                HIPCHK(launch_update(p->nd, p->precision, kDefaultWaves, grid, block, st, a));
            }
        HIPCHK(launch_counter_add(st, d_sweep, 1));
        if (series)
            HIPCHK(launch_measure_finalize(st, d_meas, p->nd, rep.upd_blocks, nc, double(rep.V), int(rep.nlat), beta0,
                                           beta1, d_plaq, series, d_cursor));
    }
    return SU3HB_OK;
}

}  // extern "C"
