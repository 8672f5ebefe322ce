/*
 * su3_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, sequential FP64 CPU reference of the checkerboard
 * Cabibbo-Marinari (CM) SU(3) heatbath with FHKP SU(2) updates in multi-hit
 * accept/reject form, for the Wilson action on a D-dimensional torus or a
 * double-layered torus (B. A. Berg, "Fortran MPI Checkerboard Code for SU(3)
 * Lattice Gauge Theory I", arXiv:0904.0642).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source, header, table or
 * helper with the GPU library: geometry, SU(3) algebra, the SU(2) heatbath and
 * the Philox generator are all written out again here.
 *
 * Paper passages followed (section / equation / table of the paper):
 *   - site number and coordinates: Sec. 2, eqs. (i_s), (xD), (x^i); we use
 *     0-based site numbers and 0-based directions, direction 0 fastest.
 *   - checkerboard colour: Sec. 2, eq. (i_c); parity p = (sum_i x^i) mod 2.
 *   - CM updating with FHKP SU(2) heatbath, multi-hit form: Sec. 1 and
 *     Sec. 2.1 (finite number of hits, old link kept when none is accepted).
 *   - sweep = every SU(3) matrix updated once in sequential order: Sec. 2.1.
 *   - double-layered torus and the beta0/beta1 plaquette tags: Sec. 2.2.
 *   - plaquette measurement, spacelike/timelike split: Sec. 2.4 (measurement
 *     step) and the mptime/mpspace counts of the latmpi.par example, Sec. 2.3.
 *   - ordered (cold) and disordered (hot) starts: Sec. 2.3, istart of mc.par.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   R-ORDER  sweep order: parity 0 then 1; inside, directions 0..D-1; inside,
 *            layers, then sites in increasing site number.
 *   R-SUB    SU(2) subgroups (0,1), (0,2), (1,2) in that order, each applied
 *            by left multiplication U <- R U, with W = U A.
 *   R-BETA   beta is the standard SU(3) Wilson beta = 6/g^2: the weight of a
 *            link is exp((1/3) Re Tr(U A)) with beta folded into the staple A.
 *   R-HIT    multi-hit per SU(2) subgroup: up to n_hit Kennedy-Pendleton
 *            proposals; if none is accepted that subgroup leaves U unchanged.
 *   R-REUNIT Gram-Schmidt reunitarisation after every link update.
 *   R-DLT    nlat = 2: crossing the boundary of a glued direction moves to the
 *            same coordinates in the other layer.
 *   R-TAG    a link's tag is the layer of its base site; a plaquette uses
 *            beta0 if its four tags add to zero, beta1 otherwise.
 *   R-DEGEN  a projected SU(2) norm k <= 1e-300 rejects every hit.
 *   R-RNG    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
 *            64-bit seed, counter (link id, sweep, (sub<<16)|(hit<<1)|blk,
 *            stream tag); 32-bit words map to uniforms (r+1)/2^32 in (0,1].
 *   R-OR     overrelaxation, which Sec. 1 names as a move the code could
 *            take in: per SU(2) subgroup, in the CM order, the reflection
 *            that keeps Re Tr(U A) fixed.  With the subgroup block of W = U A
 *            equal to k V (V in SU(2)), the block becomes k V^dag, i.e.
 *            U <- R(r) U with r = V^dag V^dag; no random numbers; a sweep
 *            with n_hit = 0 is an overrelaxation sweep.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 8
#define OR_TWO_PI 6.283185307179586476925286766559

enum { OR_TAG_UPDATE = 0, OR_TAG_START = 1 };

typedef double complex cplx;
typedef struct { cplx m[3][3]; } su3;

typedef struct {
    int nd;
    int n[OR_MAXD];
    long stride[OR_MAXD]; /* n_a of eq. (i_s): product of the extents below */
    int nlat;
    unsigned dlt_mask;
    int lat2test;
    long V;               /* sites per layer */
    su3 *U;               /* U[((layer * V + site) * nd + mu)] */
    uint32_t key[2];
    uint32_t sweep;
    int nthreads;
} olat;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon et al., SC'11.               */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {           /* Weyl sequence bump of the key */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A 32-bit word r becomes the uniform (r + 1) / 2^32, which lies in (0, 1]. */
double or_uniform(uint32_t r) { return ((double)r + 1.0) * 0x1p-32; }

static void draw4(const uint32_t key[2], uint32_t w0, uint32_t w1, uint32_t w2,
                  uint32_t w3, double u[4])
{
    uint32_t ctr[4] = {w0, w1, w2, w3}, r[4];
    or_philox4x32_10(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = or_uniform(r[i]);
}

static uint32_t hit_word(int sub, int hit, int blk)
{
    return ((uint32_t)sub << 16) | ((uint32_t)hit << 1) | (uint32_t)blk;
}

/* ------------------------------------------------------------------------ */
/* SU(3) algebra on 3x3 complex matrices.                                    */
/* ------------------------------------------------------------------------ */

static su3 mat_mul(const su3 *a, const su3 *b)             /* a b */
{
    su3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a->m[i][k] * b->m[k][j];
            c.m[i][j] = s;
        }
    return c;
}

static su3 mat_adj(const su3 *a)                            /* a^dagger */
{
    su3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.m[i][j] = conj(a->m[j][i]);
    return c;
}

static double re_trace(const su3 *a)
{
    return creal(a->m[0][0] + a->m[1][1] + a->m[2][2]);
}

/* Gram-Schmidt on rows 0 and 1; row 2 = conj(row0 x row1), so det = 1. */
static void reunitarize(su3 *u)
{
    double n0 = 0;
    for (int c = 0; c < 3; ++c) n0 += creal(u->m[0][c] * conj(u->m[0][c]));
    n0 = 1.0 / sqrt(n0);
    for (int c = 0; c < 3; ++c) u->m[0][c] *= n0;

    cplx d = 0;
    for (int c = 0; c < 3; ++c) d += conj(u->m[0][c]) * u->m[1][c];
    for (int c = 0; c < 3; ++c) u->m[1][c] -= d * u->m[0][c];

    double n1 = 0;
    for (int c = 0; c < 3; ++c) n1 += creal(u->m[1][c] * conj(u->m[1][c]));
    n1 = 1.0 / sqrt(n1);
    for (int c = 0; c < 3; ++c) u->m[1][c] *= n1;

    const cplx *a = u->m[0], *b = u->m[1];
    u->m[2][0] = conj(a[1] * b[2] - a[2] * b[1]);
    u->m[2][1] = conj(a[2] * b[0] - a[0] * b[2]);
    u->m[2][2] = conj(a[0] * b[1] - a[1] * b[0]);
}

void or_reunitarize(double *u18) { reunitarize((su3 *)u18); }

/* ------------------------------------------------------------------------ */
/* Geometry: eq. (i_s) 0-based, eq. (i_c), the double-layered torus.         */
/* ------------------------------------------------------------------------ */

static int coord(const olat *L, long s, int i) { return (int)((s / L->stride[i]) % L->n[i]); }

static int parity_of(const olat *L, long s)
{
    int sum = 0;
    for (int i = 0; i < L->nd; ++i) sum += coord(L, s, i);
    return sum & 1;
}

/* Neighbour of (layer, s) one step along +/- dir.  A step across the boundary
 * wraps periodically; with two layers and dir glued it also moves to the
 * other layer (reading R-DLT). */
static void neighbor(const olat *L, int layer, long s, int dir, int sgn, int *lo, long *so)
{
    int x = coord(L, s, dir);
    int xn = x + sgn, wrapped = 0;
    if (xn == L->n[dir]) { xn = 0; wrapped = 1; }
    if (xn < 0) { xn = L->n[dir] - 1; wrapped = 1; }
    *so = s + (long)(xn - x) * L->stride[dir];
    *lo = (wrapped && L->nlat == 2 && ((L->dlt_mask >> dir) & 1u)) ? 1 - layer : layer;
}

static su3 *link_at(const olat *L, int layer, long s, int mu)
{
    return &L->U[((long)layer * L->V + s) * L->nd + mu];
}

/* Link id entering the Philox counter; lat2test drops the layer so both
 * layers draw identical random numbers (Sec. 3.4, lat2test). */
static uint32_t link_id(const olat *L, int layer, long s, int mu)
{
    long base = L->lat2test ? 0 : (long)layer * L->V;
    return (uint32_t)((base + s) * L->nd + mu);
}

/* ------------------------------------------------------------------------ */
/* Staple: the sum over nu != mu of the two plaquette complements of U_mu(x),
 * each weighted with the beta of its plaquette (Sec. 2.2 tag rule). */
static void staple(const olat *L, int layer, long s, int mu, double beta0, double beta1, su3 *A)
{
    memset(A, 0, sizeof *A);
    int l_xpmu; long s_xpmu;
    neighbor(L, layer, s, mu, +1, &l_xpmu, &s_xpmu);
    for (int nu = 0; nu < L->nd; ++nu) {
        if (nu == mu) continue;
        int l_xpnu, l_xmnu, l_xpmu_mnu; long s_xpnu, s_xmnu, s_xpmu_mnu;
        neighbor(L, layer, s, nu, +1, &l_xpnu, &s_xpnu);
        neighbor(L, layer, s, nu, -1, &l_xmnu, &s_xmnu);
        neighbor(L, l_xpmu, s_xpmu, nu, -1, &l_xpmu_mnu, &s_xpmu_mnu);

        /* forward: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
        su3 a = *link_at(L, l_xpmu, s_xpmu, nu);
        su3 b = mat_adj(link_at(L, l_xpnu, s_xpnu, mu));
        su3 c = mat_adj(link_at(L, layer, s, nu));
        su3 ab = mat_mul(&a, &b);
        su3 f = mat_mul(&ab, &c);
        int tags = layer + l_xpmu + l_xpnu + layer;
        double bf = tags == 0 ? beta0 : beta1;

        /* backward: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) */
        su3 d = mat_adj(link_at(L, l_xpmu_mnu, s_xpmu_mnu, nu));
        su3 e = mat_adj(link_at(L, l_xmnu, s_xmnu, mu));
        su3 g = *link_at(L, l_xmnu, s_xmnu, nu);
        su3 de = mat_mul(&d, &e);
        su3 bk = mat_mul(&de, &g);
        int tagb = l_xmnu + l_xpmu_mnu + layer + l_xmnu;
        double bb = tagb == 0 ? beta0 : beta1;

        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A->m[i][j] += bf * f.m[i][j] + bb * bk.m[i][j];
    }
}

/* ------------------------------------------------------------------------ */
/* FHKP (Kennedy-Pendleton) SU(2) heatbath in multi-hit form: sample
 * x0 with density ~ sqrt(1 - x0^2) exp(alpha x0).  delta = 1 - x0 is proposed
 * from the Gamma(3/2) density ~ sqrt(delta) exp(-alpha delta) and accepted
 * with probability sqrt(1 - delta/2).  Returns the accepted hit or -1. */
static int kp_multihit(double alpha, int nhit, const uint32_t key[2], uint32_t lid,
                       uint32_t sweep, int sub, double *x0, uint64_t *attempts, double *margin)
{
    for (int hit = 0; hit < nhit; ++hit) {
        double r[4];
        draw4(key, lid, sweep, hit_word(sub, hit, 0), OR_TAG_UPDATE, r);
        ++*attempts;
        double c = cos(OR_TWO_PI * r[1]);
        double delta = -(log(r[0]) + c * c * log(r[2])) / alpha;
        /* distance of this proposal from the accept/reject threshold (only
         * observed, for the rounding study of Sec. 3) */
        if (margin && fabs(r[3] * r[3] - (1.0 - 0.5 * delta)) < *margin)
            *margin = fabs(r[3] * r[3] - (1.0 - 0.5 * delta));
        if (r[3] * r[3] <= 1.0 - 0.5 * delta) {
            *x0 = 1.0 - delta;
            return hit;
        }
    }
    return -1;
}

int or_kp_draw(double alpha, int nhit, uint64_t seed, uint32_t lid, uint32_t sweep, int sub,
               double *x0, uint64_t *attempts)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    return kp_multihit(alpha, nhit, key, lid, sweep, sub, x0, attempts, NULL);
}

static const int SUB_I[3] = {0, 0, 1};
static const int SUB_J[3] = {1, 2, 2};

/* One CM update of the link matrix u for the staple a: the three SU(2)
 * subgroups in turn, then reunitarisation.  Counts proposals and accepts. */
static void cm_update(su3 *u, const su3 *a, int nhit, const uint32_t key[2], uint32_t lid,
                      uint32_t sweep, uint64_t attempts[3], uint64_t accepts[3], double *margin)
{
    for (int sub = 0; sub < 3; ++sub) {
        int i = SUB_I[sub], j = SUB_J[sub];
        su3 w = mat_mul(u, a);
        /* quaternion part of the 2x2 block (i,j) of W: a0 + i a.sigma */
        double a0 = creal(w.m[i][i] + w.m[j][j]) / 2;
        double a1 = cimag(w.m[i][j] + w.m[j][i]) / 2;
        double a2 = creal(w.m[i][j] - w.m[j][i]) / 2;
        double a3 = cimag(w.m[i][i] - w.m[j][j]) / 2;
        double k = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
        if (!(k > 1e-300)) continue;                   /* reading R-DEGEN */
        double alpha = 2.0 * k / 3.0;

        double x0;
        int hit = kp_multihit(alpha, nhit, key, lid, sweep, sub, &x0, &attempts[sub], margin);
        if (hit < 0) continue;                          /* keep the link */
        ++accepts[sub];

        /* direction of (x1,x2,x3): uniform on the sphere of radius sqrt(1-x0^2) */
        double r[4];
        draw4(key, lid, sweep, hit_word(sub, hit, 1), OR_TAG_UPDATE, r);
        double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
        double cth = 2.0 * r[0] - 1.0;
        double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
        double phi = OR_TWO_PI * r[1];
        double x1 = rad * sth * cos(phi), x2 = rad * sth * sin(phi), x3 = rad * cth;

        /* X = x0 + i x.sigma, V^dag = (a0 - i a.sigma)/k, r = X V^dag */
        cplx X[2][2] = {{x0 + I * x3, x2 + I * x1}, {-x2 + I * x1, x0 - I * x3}};
        cplx Vd[2][2] = {{(a0 - I * a3) / k, (-a2 - I * a1) / k},
                         {(a2 - I * a1) / k, (a0 + I * a3) / k}};
        cplx R[2][2];
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) R[p][q] = X[p][0] * Vd[0][q] + X[p][1] * Vd[1][q];

        /* U <- R_ij(r) U: mixes rows i and j */
        for (int c = 0; c < 3; ++c) {
            cplx ui = u->m[i][c], uj = u->m[j][c];
            u->m[i][c] = R[0][0] * ui + R[0][1] * uj;
            u->m[j][c] = R[1][0] * ui + R[1][1] * uj;
        }
    }
    reunitarize(u);
}

/* Overrelaxation (reading R-OR): per SU(2) subgroup, the block k V of
 * W = U A becomes k V^dag, which leaves Re Tr(U A) unchanged, by U <- R U with
 * r = V^dag V^dag; then reunitarisation.  A degenerate projection (k <= 1e-300)
 * leaves the subgroup alone.  attempts and accepts count the reflections. */
static void cm_reflect(su3 *u, const su3 *a, uint64_t attempts[3], uint64_t accepts[3])
{
    for (int sub = 0; sub < 3; ++sub) {
        int i = SUB_I[sub], j = SUB_J[sub];
        su3 w = mat_mul(u, a);
        double a0 = creal(w.m[i][i] + w.m[j][j]) / 2;
        double a1 = cimag(w.m[i][j] + w.m[j][i]) / 2;
        double a2 = creal(w.m[i][j] - w.m[j][i]) / 2;
        double a3 = cimag(w.m[i][i] - w.m[j][j]) / 2;
        double k = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
        if (!(k > 1e-300)) continue;
        ++attempts[sub];
        ++accepts[sub];
        cplx Vd[2][2] = {{(a0 - I * a3) / k, (-a2 - I * a1) / k},
                         {(a2 - I * a1) / k, (a0 + I * a3) / k}};
        cplx R[2][2];
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) R[p][q] = Vd[p][0] * Vd[0][q] + Vd[p][1] * Vd[1][q];
        for (int c = 0; c < 3; ++c) {
            cplx ui = u->m[i][c], uj = u->m[j][c];
            u->m[i][c] = R[0][0] * ui + R[0][1] * uj;
            u->m[j][c] = R[1][0] * ui + R[1][1] * uj;
        }
    }
    reunitarize(u);
}

/* Test hook: one overrelaxation step of the matrix u18 for the staple a18. */
void or_reflect_matrix(double *u18, const double *a18)
{
    uint64_t at[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
    cm_reflect((su3 *)u18, (const su3 *)a18, at, ac);
}

/* Test hook: CM-update one matrix u18 for the staple a18. */
void or_cm_update_matrix(double *u18, const double *a18, int nhit, uint64_t seed, uint32_t lid,
                         uint32_t sweep, uint64_t attempts[3], uint64_t accepts[3])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    cm_update((su3 *)u18, (const su3 *)a18, nhit, key, lid, sweep, attempts, accepts, NULL);
}

/* ------------------------------------------------------------------------ */
/* Lattice object.                                                           */
/* ------------------------------------------------------------------------ */

void or_destroy(void *h)
{
    olat *L = (olat *)h;
    if (!L) return;
    free(L->U);
    free(L);
}

void *or_create(int nd, const int *n, int nlat, unsigned dlt_mask, int lat2test, uint64_t seed)
{
    if (nd < 2 || nd > OR_MAXD || (nlat != 1 && nlat != 2)) return NULL;
    if (nlat == 1 && (dlt_mask != 0 || lat2test)) return NULL;
    olat *L = (olat *)calloc(1, sizeof *L);
    if (!L) return NULL;
    L->nd = nd;
    L->V = 1;
    for (int i = 0; i < nd; ++i) {
        if (n[i] < 2 || (n[i] & 1)) { free(L); return NULL; }  /* even extents, Sec. 2 */
        L->n[i] = n[i];
        L->stride[i] = L->V;
        L->V *= n[i];
    }
    if ((double)nlat * (double)L->V * nd >= 4294967296.0) { free(L); return NULL; }
    L->nlat = nlat;
    L->dlt_mask = dlt_mask;
    L->lat2test = lat2test;
    L->key[0] = (uint32_t)seed;
    L->key[1] = (uint32_t)(seed >> 32);
    L->nthreads = 1;
    L->U = (su3 *)malloc(sizeof(su3) * (size_t)nlat * (size_t)L->V * (size_t)nd);
    if (!L->U) { free(L); return NULL; }
    return L;
}

void or_set_threads(void *h, int nthreads) { ((olat *)h)->nthreads = nthreads < 1 ? 1 : nthreads; }
long or_volume(void *h) { return ((olat *)h)->V; }
uint32_t or_get_sweep(void *h) { return ((olat *)h)->sweep; }
void or_set_sweep(void *h, uint32_t sweep) { ((olat *)h)->sweep = sweep; }

long or_site_index(void *h, const int *x)
{
    const olat *L = (const olat *)h;
    long s = 0;
    for (int i = 0; i < L->nd; ++i) s += (long)x[i] * L->stride[i];
    return s;
}

void or_site_coords(void *h, long s, int *x)
{
    const olat *L = (const olat *)h;
    for (int i = 0; i < L->nd; ++i) x[i] = coord(L, s, i);
}

int or_parity(void *h, long s) { return parity_of((const olat *)h, s); }

void or_neighbor(void *h, int layer, long s, int dir, int sgn, int *layer_out, long *site_out)
{
    neighbor((const olat *)h, layer, s, dir, sgn, layer_out, site_out);
}

/* Ordered start (istart = 1): every matrix is the identity. */
void or_cold_start(void *h)
{
    olat *L = (olat *)h;
    long nl = (long)L->nlat * L->V * L->nd;
    for (long i = 0; i < nl; ++i) {
        memset(&L->U[i], 0, sizeof(su3));
        L->U[i].m[0][0] = L->U[i].m[1][1] = L->U[i].m[2][2] = 1;
    }
}

/* Disordered start (istart = 2): Haar-random SU(3).  Two rows of complex
 * Gaussians (Box-Muller on the start stream), then Gram-Schmidt and the
 * cross product. */
void or_hot_start(void *h)
{
    olat *L = (olat *)h;
    for (int layer = 0; layer < L->nlat; ++layer)
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(L->nthreads)
#endif
        for (long s = 0; s < L->V; ++s)
            for (int mu = 0; mu < L->nd; ++mu) {
                uint32_t lid = link_id(L, layer, s, mu);
                double u[12], g[12];
                for (int j = 0; j < 3; ++j) draw4(L->key, lid, 0, (uint32_t)j, OR_TAG_START, &u[4 * j]);
                for (int q = 0; q < 6; ++q) {
                    double rho = sqrt(-2.0 * log(u[2 * q]));
                    double th = OR_TWO_PI * u[2 * q + 1];
                    g[2 * q] = rho * cos(th);
                    g[2 * q + 1] = rho * sin(th);
                }
                su3 *U = link_at(L, layer, s, mu);
                for (int c = 0; c < 3; ++c) {
                    U->m[0][c] = g[2 * c] + I * g[2 * c + 1];
                    U->m[1][c] = g[6 + 2 * c] + I * g[6 + 2 * c + 1];
                    U->m[2][c] = 0;
                }
                reunitarize(U);
            }
}

/* Canonical layout: [layer][site][mu][3][3][re,im], FP64. */
int or_get_links(void *h, double *out, size_t n)
{
    olat *L = (olat *)h;
    size_t need = (size_t)L->nlat * (size_t)L->V * (size_t)L->nd * 18;
    if (n != need) return -1;
    memcpy(out, L->U, need * sizeof(double));
    return 0;
}

int or_set_links(void *h, const double *in, size_t n)
{
    olat *L = (olat *)h;
    size_t need = (size_t)L->nlat * (size_t)L->V * (size_t)L->nd * 18;
    if (n != need) return -1;
    memcpy(L->U, in, need * sizeof(double));
    return 0;
}

void or_staple(void *h, int layer, long s, int mu, double beta0, double beta1, double *a18)
{
    staple((const olat *)h, layer, s, mu, beta0, beta1, (su3 *)a18);
}

/* Update one link in place; returns (1/3) Re Tr((U' - U) A), the change of
 * the beta-weighted trace sum sum_p beta_p Re Tr U_p / 3. */
static double update_link(olat *L, int layer, long s, int mu, double beta0, double beta1,
                          int nhit, uint64_t attempts[3], uint64_t accepts[3])
{
    su3 A;
    staple(L, layer, s, mu, beta0, beta1, &A);
    su3 *U = link_at(L, layer, s, mu);
    su3 old = *U;
    if (nhit == 0)
        cm_reflect(U, &A, attempts, accepts);   /* overrelaxation, reading R-OR */
    else
        cm_update(U, &A, nhit, L->key, link_id(L, layer, s, mu), L->sweep, attempts, accepts, NULL);
    su3 d;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) d.m[i][j] = U->m[i][j] - old.m[i][j];
    su3 dA = mat_mul(&d, &A);
    return re_trace(&dA) / 3.0;
}

double or_update_link(void *h, int layer, long s, int mu, double beta0, double beta1, int nhit)
{
    uint64_t at[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
    return update_link((olat *)h, layer, s, mu, beta0, beta1, nhit, at, ac);
}

/* Smallest |R4^2 - (1 - delta/2)| over the Kennedy-Pendleton proposals that
 * the update of link (layer, s, mu) evaluates in the current configuration:
 * how close its accept/reject decisions come to the threshold (Sec. 3 notes
 * that rounding differences between platforms eventually flip such
 * decisions).  The lattice is left unchanged. */
double or_link_margin(void *h, int layer, long s, int mu, double beta0, double beta1, int nhit)
{
    olat *L = (olat *)h;
    su3 A;
    staple(L, layer, s, mu, beta0, beta1, &A);
    su3 u = *link_at(L, layer, s, mu);
    uint64_t at[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
    double margin = INFINITY;
    cm_update(&u, &A, nhit, L->key, link_id(L, layer, s, mu), L->sweep, at, ac, &margin);
    return margin;
}

/* One checkerboard slice: every link U_mu(x) with parity(x) = p, in every
 * layer.  `order` (optional, length V) permutes the site loop; the sites of a
 * slice are independent, so the result does not depend on it (Sec. 2). */
static double update_slice(olat *L, int p, int mu, double beta0, double beta1, int nhit,
                           const long *order, uint64_t attempts[3], uint64_t accepts[3])
{
    double dtrace = 0;
    for (int layer = 0; layer < L->nlat; ++layer) {
        uint64_t a0 = 0, a1 = 0, a2 = 0, c0 = 0, c1 = 0, c2 = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(L->nthreads) \
        reduction(+ : dtrace, a0, a1, a2, c0, c1, c2)
#endif
        for (long i = 0; i < L->V; ++i) {
            long s = order ? order[i] : i;
            if (parity_of(L, s) != p) continue;
            uint64_t at[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
            dtrace += update_link(L, layer, s, mu, beta0, beta1, nhit, at, ac);
            a0 += at[0]; a1 += at[1]; a2 += at[2];
            c0 += ac[0]; c1 += ac[1]; c2 += ac[2];
        }
        attempts[0] += a0; attempts[1] += a1; attempts[2] += a2;
        accepts[0] += c0; accepts[1] += c1; accepts[2] += c2;
    }
    return dtrace;
}

double or_update_slice(void *h, int p, int mu, double beta0, double beta1, int nhit,
                       const long *order)
{
    uint64_t at[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
    return update_slice((olat *)h, p, mu, beta0, beta1, nhit, order, at, ac);
}

/* stats (may be NULL): [attempts x3, accepts x3, dtrace] as doubles.
 * nhit = 0 makes every sweep an overrelaxation sweep (reading R-OR); every
 * sweep, of either kind, advances the sweep counter. */
void or_sweep(void *h, double beta0, double beta1, int nhit, int nsweeps, double *stats)
{
    olat *L = (olat *)h;
    uint64_t at[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
    double dtrace = 0;
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int p = 0; p < 2; ++p)
            for (int mu = 0; mu < L->nd; ++mu)
                dtrace += update_slice(L, p, mu, beta0, beta1, nhit, NULL, at, ac);
        L->sweep += 1;
    }
    if (stats) {
        for (int i = 0; i < 3; ++i) {
            stats[i] = (double)at[i];
            stats[3 + i] = (double)ac[i];
        }
        stats[6] = dtrace;
    }
}

/* Plaquette measurement.  out[0] total <P> = <(1/3) Re Tr U_p> over
 * N_p = nlat V D(D-1)/2 plaquettes; out[1] spacelike (planes without the
 * last direction); out[2] timelike (planes containing it); out[3], out[4]
 * per layer of the base site; out[5] = sum_p beta_p Re Tr U_p / 3 for the
 * given betas (tag rule).  Empty categories give NaN. */
void or_plaquette(void *h, double beta0, double beta1, double out[6])
{
    const olat *L = (const olat *)h;
    int D = L->nd;
    double space = 0, time = 0, lay[2] = {0, 0}, weighted = 0;
    for (int layer = 0; layer < L->nlat; ++layer)
        for (long s = 0; s < L->V; ++s)
            for (int mu = 0; mu < D; ++mu)
                for (int nu = mu + 1; nu < D; ++nu) {
                    int l1, l2; long s1, s2;
                    neighbor(L, layer, s, mu, +1, &l1, &s1);
                    neighbor(L, layer, s, nu, +1, &l2, &s2);
                    su3 a = mat_mul(link_at(L, layer, s, mu), link_at(L, l1, s1, nu));
                    su3 b = mat_adj(link_at(L, l2, s2, mu));
                    su3 c = mat_adj(link_at(L, layer, s, nu));
                    su3 ab = mat_mul(&a, &b);
                    su3 pl = mat_mul(&ab, &c);
                    double P = re_trace(&pl) / 3.0;
                    if (nu == D - 1) time += P; else space += P;
                    lay[layer] += P;
                    int tags = layer + l1 + l2 + layer;
                    weighted += (tags == 0 ? beta0 : beta1) * P;
                }
    double nV = (double)L->nlat * (double)L->V;
    double np = nV * D * (D - 1) / 2.0;
    double nspace = nV * (D - 1) * (D - 2) / 2.0;
    double ntime = nV * (D - 1);
    out[0] = (space + time) / np;
    out[1] = nspace > 0 ? space / nspace : NAN;
    out[2] = time / ntime;
    out[3] = lay[0] / ((double)L->V * D * (D - 1) / 2.0);
    out[4] = L->nlat == 2 ? lay[1] / ((double)L->V * D * (D - 1) / 2.0) : NAN;
    out[5] = weighted;
}

/* Test hook: read or write one link (18 doubles) without copying the lattice. */
void or_get_link(void *h, int layer, long s, int mu, double *out18)
{
    memcpy(out18, link_at((const olat *)h, layer, s, mu), sizeof(su3));
}

void or_put_link(void *h, int layer, long s, int mu, const double *in18)
{
    memcpy(link_at((const olat *)h, layer, s, mu), in18, sizeof(su3));
}
