/*
 * FP64 CPU oracle for one time step of the hybrid chemotaxis model of
 * Bruna, Maini & Robinson, "Particle-based simulations of reaction-diffusion
 * processes with Aboria" (arXiv:1805.11007).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source with the GPU library and includes none of its headers.
 *
 * Every function below cites the part of the paper it follows.  Where the
 * paper is silent or garbled the reading taken is stated next to the code.
 * Each function is pinned by the CPU tests (closed forms, invariants,
 * library routines, brute force); the coupled multi-step trajectory has no
 * printed values in the paper and is parity unpinned beyond the per-step
 * pins and the diffusion / drift laws.
 *
 * State of one instance: positions X (N x dim, float64), species s (uint8),
 * stable ids (uint32), chemical c on the node grid (x fastest), a step
 * counter.  Node gradients g are derived from c when needed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_SPECIES 8

/* Parameters of one instance.  Layout mirrored by oracle/__init__.py. */
typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t periodic;     /* 1: torus [0,L)^d ; 0: reflecting walls [0,L]^d */
    double L;
    int32_t grid_n;       /* nodes per axis */
    int32_t n_sub;        /* PDE substeps per time step (>= 1) */
    double dt, k, D_c, gamma;
    int32_t n_species;
    int32_t mode;         /* 0: all-pairs neighbour search ; 1: cell list */
    double diam[ORC_MAX_SPECIES], D[ORC_MAX_SPECIES], chi[ORC_MAX_SPECIES];
    double source[ORC_MAX_SPECIES], uptake[ORC_MAX_SPECIES];
    /* type switching (eq. Chemo_reactions): species s becomes react_to[s]
     * at rate react_rate[s] + react_rate_c[s] * c(X); react_to < 0: none */
    int32_t react_to[ORC_MAX_SPECIES];
    double react_rate[ORC_MAX_SPECIES], react_rate_c[ORC_MAX_SPECIES];
    uint64_t seed;        /* Philox key = (lo32(seed), hi32(seed) ^ inst) */
    uint32_t inst;
    double chi_scale;     /* per-instance multiplier of chi */
    int32_t deposit_kernel;  /* 0: particle-in-cell ; 1: Gaussian kernel density */
    double kde_radius;    /* kernel truncation radius in units of the bandwidth */
    int32_t potential;    /* 0: harmonic ; 1: exponential ; 2: hard spheres */
    int32_t tamed;        /* 1: tamed Euler drift for the pair forces (eq. sde_ETamed) */
    double pot_range;     /* exponential potential cut at pot_range * d_ij */
} orc_params;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Noise.  The paper draws xi_i ~ N(0, I) per agent and step (eq. sde_EM)
 * from per-agent std:: generators (Sect. 3.2).  The oracle replaces them by
 * the counter-based generator Philox4x32-10 of Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a
 * multiply/xor S-box on a 4x32-bit counter under a 2x32-bit key that is
 * advanced by the Weyl constants between rounds.
 * ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    for (int64_t i = 0; i < n; ++i) orc_philox(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* 24-bit uniform strictly inside (0,1): the top 24 bits of a word with the
 * lowest kept bit forced to one, times 2^-24 (exact in float32 and float64). */
static double orc_uniform(uint32_t w) {
    return (double)((w >> 8) | 1u) * (1.0 / 16777216.0);
}

/* Standard normals for agent `id` at step `step` of instance `inst`
 * (counter = (step, id, inst, 0)), by the Box-Muller transform (1958):
 * xi0, xi1 from (u0, u1); xi2 from (u2, u3).  Only the first `dim` are used. */
static void orc_normals_one(const orc_params *p, uint32_t step, uint32_t id, double xi[3]) {
    uint32_t ctr[4] = {step, id, p->inst, 0u};
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32) ^ p->inst};
    uint32_t w[4];
    orc_philox(ctr, key, w);
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = orc_uniform(w[0]), u1 = orc_uniform(w[1]);
    double u2 = orc_uniform(w[2]), u3 = orc_uniform(w[3]);
    double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
    xi[0] = r0 * cos(two_pi * u1);
    xi[1] = r0 * sin(two_pi * u1);
    xi[2] = r1 * cos(two_pi * u3);
}

void orc_normals(const orc_params *p, uint32_t step, int64_t n, const uint32_t *ids, double *xi) {
    for (int64_t i = 0; i < n; ++i) {
        double t[3];
        orc_normals_one(p, step, ids[i], t);
        for (int a = 0; a < p->dim; ++a) xi[i * p->dim + a] = t[a];
    }
}

/* ------------------------------------------------------------------------
 * Pairs.  The interaction loop of Sect. 3.2 visits every j within the
 * cutoff of i through the shortest (periodic-aware) vector dx = x_j - x_i.
 * Contact distance of a pair: mean of the two diameters (Sect. 2.2, the
 * hard-sphere overlap rule).  Neighbours are the j != i with |dx| < d_ij.
 * ------------------------------------------------------------------------ */
static double orc_min_image(double dx, double L) {
    if (dx > 0.5 * L) dx -= L;
    else if (dx < -0.5 * L) dx += L;
    return dx;
}

static double orc_contact(const orc_params *p, int si, int sj) {
    return 0.5 * (p->diam[si] + p->diam[sj]);
}

/* Interaction range of a pair: the contact distance, or pot_range times it
 * for the exponential potential (which has no natural end). */
static double orc_pair_cut(const orc_params *p, int si, int sj) {
    const double d = orc_contact(p, si, sj);
    return p->potential == 1 ? p->pot_range * d : d;
}

static double orc_max_cutoff(const orc_params *p) {
    double m = 0.0;
    for (int s = 0; s < p->n_species; ++s) if (p->diam[s] > m) m = p->diam[s];
    return p->potential == 1 ? p->pot_range * m : m;
}

/* Pair force on i from j at distance r > 0 inside the range, as the factor g
 * of F_i -= g (X_j - X_i):
 *   harmonic    u = (k/2)(d - r)^2 :  g = k (d - r) / r;
 *   exponential u = k exp(-r/d)    :  g = (k/d) exp(-r/d) / r (the soft
 *               potential of Sect. 4 with length scale d = the contact
 *               distance and strength k);
 *   hard spheres have no force (overlaps are corrected after the step). */
static double orc_pair_g(const orc_params *p, double dij, double r) {
    if (p->potential == 0) return p->k * (dij - r) / r;
    if (p->potential == 1) return (p->k / dij) * exp(-r / dij) / r;
    return 0.0;
}

/* A plain uniform-bin index of the agents, used only to enumerate
 * candidate pairs faster than all-pairs in mode 1.  The accepted
 * neighbours are the same set as all-pairs and are summed in the same
 * (ascending j) order, so both modes give identical floating-point
 * results. */
typedef struct {
    int nb;              /* bins per axis (>= 3) */
    double side;
    int64_t *start;      /* nb^dim + 1 */
    int64_t *order;      /* agents sorted by bin */
} orc_bins;

static int orc_bin_coord(double x, double side, int nb) {
    int b = (int)floor(x / side);
    if (b < 0) b = 0;
    if (b > nb - 1) b = nb - 1;
    return b;
}

static int orc_bins_build(orc_bins *B, int dim, int periodic, double L, double cutoff,
                          int64_t n, const double *X) {
    int nb = (int)floor(L / cutoff);
    if (nb < 3) return 0;
    /* keep the bin table modest; wider bins only add candidates */
    while ((dim == 3 && (int64_t)nb * nb * nb > (1 << 25)) || (dim == 2 && nb > 4096)) nb /= 2;
    (void)periodic;
    B->nb = nb;
    B->side = L / nb;
    int64_t nbins = 1;
    for (int a = 0; a < dim; ++a) nbins *= nb;
    B->start = (int64_t *)calloc((size_t)nbins + 1, sizeof(int64_t));
    B->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *bin = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = 0;
        for (int a = dim - 1; a >= 0; --a) b = b * nb + orc_bin_coord(X[i * dim + a], B->side, nb);
        bin[i] = b;
        B->start[b + 1]++;
    }
    for (int64_t b = 0; b < nbins; ++b) B->start[b + 1] += B->start[b];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nbins);
    memcpy(fill, B->start, sizeof(int64_t) * (size_t)nbins);
    for (int64_t i = 0; i < n; ++i) B->order[fill[bin[i]]++] = i;
    free(fill);
    free(bin);
    return 1;
}

static void orc_bins_free(orc_bins *B) {
    free(B->start);
    free(B->order);
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Candidate indices j (j != i) for agent i, ascending.  Mode 0 returns all
 * agents; mode 1 returns the agents of the 3^dim bins around i. */
typedef struct { int64_t *v; int64_t n, cap; } orc_list;

static void list_push(orc_list *l, int64_t j) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 256;
        l->v = (int64_t *)realloc(l->v, sizeof(int64_t) * (size_t)l->cap);
    }
    l->v[l->n++] = j;
}

static void orc_candidates(int dim, int periodic, int64_t n, const double *X, const orc_bins *B,
                           int64_t i, orc_list *out) {
    out->n = 0;
    if (!B) {
        for (int64_t j = 0; j < n; ++j) if (j != i) list_push(out, j);
        return;
    }
    int nb = B->nb, c[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) c[a] = orc_bin_coord(X[i * dim + a], B->side, nb);
    int off[3];
    int lim2 = dim == 3 ? 1 : 0;
    for (off[2] = -lim2; off[2] <= lim2; ++off[2])
        for (off[1] = -1; off[1] <= 1; ++off[1])
            for (off[0] = -1; off[0] <= 1; ++off[0]) {
                int64_t b = 0;
                int skip = 0;
                for (int a = dim - 1; a >= 0; --a) {
                    int q = c[a] + off[a];
                    if (periodic) q = (q + nb) % nb;
                    else if (q < 0 || q >= nb) { skip = 1; break; }
                    b = b * nb + q;
                }
                if (skip) continue;
                for (int64_t t = B->start[b]; t < B->start[b + 1]; ++t)
                    if (B->order[t] != i) list_push(out, B->order[t]);
            }
    if (out->n > 1) qsort(out->v, (size_t)out->n, sizeof(int64_t), cmp_i64);
}

/* Pair repulsion for every agent: F_i = -sum_j g(r) dx over neighbours
 * (r inside the pair's range) with r > 0 (the r > 0 guard of the
 * interaction loop in Sect. 3.2), dx = X_j - X_i; unit mobility, F = -grad_i
 * u (eqs. sde_alpha, sde_beta) with the potential of orc_pair_g. */
void orc_forces(const orc_params *p, int64_t n, const double *X, const uint8_t *sp, double *F) {
    const int dim = p->dim;
    orc_bins B;
    int use_bins = p->mode == 1 && n > 0 &&
                   orc_bins_build(&B, dim, p->periodic, p->L, orc_max_cutoff(p), n, X);
#pragma omp parallel
    {
        orc_list cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            double f[3] = {0, 0, 0};
            orc_candidates(dim, p->periodic, n, X, use_bins ? &B : NULL, i, &cand);
            for (int64_t t = 0; t < cand.n; ++t) {
                int64_t j = cand.v[t];
                double dx[3], r2 = 0.0;
                for (int a = 0; a < dim; ++a) {
                    dx[a] = X[j * dim + a] - X[i * dim + a];
                    if (p->periodic) dx[a] = orc_min_image(dx[a], p->L);
                    r2 += dx[a] * dx[a];
                }
                const double cut = orc_pair_cut(p, sp[i], sp[j]);
                if (!(r2 < cut * cut)) continue;
                double r = sqrt(r2);
                if (r > 0.0) {
                    const double g = orc_pair_g(p, orc_contact(p, sp[i], sp[j]), r);
                    for (int a = 0; a < dim; ++a) f[a] -= g * dx[a];
                }
            }
            for (int a = 0; a < dim; ++a) F[i * dim + a] = f[a];
        }
        free(cand.v);
    }
    if (use_bins) orc_bins_free(&B);
}

/* Forces on a subset of agents only (sampled checks at large N). */
void orc_forces_subset(const orc_params *p, int64_t n, const double *X, const uint8_t *sp,
                       int64_t m, const int64_t *which, double *F) {
    const int dim = p->dim;
    orc_bins B;
    int use_bins = p->mode == 1 && n > 0 &&
                   orc_bins_build(&B, dim, p->periodic, p->L, orc_max_cutoff(p), n, X);
#pragma omp parallel
    {
        orc_list cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < m; ++q) {
            int64_t i = which[q];
            double f[3] = {0, 0, 0};
            orc_candidates(dim, p->periodic, n, X, use_bins ? &B : NULL, i, &cand);
            for (int64_t t = 0; t < cand.n; ++t) {
                int64_t j = cand.v[t];
                double dx[3], r2 = 0.0;
                for (int a = 0; a < dim; ++a) {
                    dx[a] = X[j * dim + a] - X[i * dim + a];
                    if (p->periodic) dx[a] = orc_min_image(dx[a], p->L);
                    r2 += dx[a] * dx[a];
                }
                const double cut = orc_pair_cut(p, sp[i], sp[j]);
                if (!(r2 < cut * cut)) continue;
                double r = sqrt(r2);
                if (r > 0.0) {
                    const double g = orc_pair_g(p, orc_contact(p, sp[i], sp[j]), r);
                    for (int a = 0; a < dim; ++a) f[a] -= g * dx[a];
                }
            }
            for (int a = 0; a < dim; ++a) F[q * dim + a] = f[a];
        }
        free(cand.v);
    }
    if (use_bins) orc_bins_free(&B);
}

/* 64-bit mixing function "splitmix64" (Steele, Lea & Flood, OOPSLA 2014). */
static uint64_t orc_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_hash_id(uint32_t id) { return orc_splitmix64((uint64_t)id); }

/* Neighbour sets decided in float32, as the float32 GPU state decides them:
 * dx = x_j - x_i (float32), minimum image by +-L when |dx| > L/2,
 * r2 = fma(dx2, dx2, fma(dx1, dx1, dx0*dx0)), every product and fused
 * multiply-add rounded to float32 once (C99 fmaf); neighbour iff
 * r2 < cut2[s_i][s_j] (a float32 table of the squared contact distances).  Output per agent: the neighbour count and the
 * wrap-around sum of splitmix64(id_j) over its neighbours. */
void orc_neighbours_f32(int dim, int periodic, float L, int64_t n, const float *X,
                        const uint8_t *sp, const uint32_t *ids, const float *cut2, int n_species,
                        int mode, uint32_t *count, uint64_t *hash) {
    double *Xd = (double *)malloc(sizeof(double) * (size_t)(n * dim > 0 ? n * dim : 1));
    for (int64_t t = 0; t < n * dim; ++t) Xd[t] = (double)X[t];
    float maxc2 = 0.0f;
    for (int t = 0; t < n_species * n_species; ++t) if (cut2[t] > maxc2) maxc2 = cut2[t];
    orc_bins B;
    /* bins slightly wider than the cutoff so that float32 rounding can never
     * hide a pair from the candidate enumeration */
    double cutoff = sqrt((double)maxc2) * 1.0001 + 1e-6 * (double)L;
    int use_bins = mode == 1 && n > 0 && orc_bins_build(&B, dim, periodic, (double)L, cutoff, n, Xd);
    const float halfL = 0.5f * L;
#pragma omp parallel
    {
        orc_list cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t cnt = 0;
            uint64_t h = 0;
            orc_candidates(dim, periodic, n, Xd, use_bins ? &B : NULL, i, &cand);
            for (int64_t t = 0; t < cand.n; ++t) {
                int64_t j = cand.v[t];
                volatile float dx[3];
                for (int a = 0; a < dim; ++a) {
                    float d = X[j * dim + a] - X[i * dim + a];
                    if (periodic) {
                        if (d > halfL) d = d - L;
                        else if (d < -halfL) d = d + L;
                    }
                    dx[a] = d;
                }
                volatile float x2 = dx[0] * dx[0];
                volatile float r2 = fmaf(dx[1], dx[1], x2);
                if (dim == 3) r2 = fmaf(dx[2], dx[2], r2);
                if (r2 < cut2[sp[i] * n_species + sp[j]]) {
                    cnt++;
                    h += orc_splitmix64((uint64_t)ids[j]);
                }
            }
            count[i] = cnt;
            hash[i] = h;
        }
        free(cand.v);
    }
    if (use_bins) orc_bins_free(&B);
    free(Xd);
}

/* ------------------------------------------------------------------------
 * Chemical grid (Sect. 2.3 and 3.5): N_c nodes per axis, x fastest.
 * Reading of the node placement (the listing never defines the spacing):
 *   periodic  h = L / N_c, nodes at i*h, i = 0..N_c-1
 *   walls     h = L / (N_c - 1), nodes at i*h on both walls; a node on a
 *             wall carries half the cell volume along that axis.
 * ------------------------------------------------------------------------ */
static double orc_h(const orc_params *p) {
    return p->periodic ? p->L / p->grid_n : p->L / (p->grid_n - 1);
}

static int64_t orc_nodes(const orc_params *p) {
    int64_t g = 1;
    for (int a = 0; a < p->dim; ++a) g *= p->grid_n;
    return g;
}

/* Neighbouring node index along axis a at offset +-1: periodic wrap, or the
 * mirror image across a wall (ghost c_{-1} = c_1, c_{N} = c_{N-2}), which
 * is the second-order no-flux closure. */
static int orc_nbr(const orc_params *p, int i, int off) {
    int n = p->grid_n, q = i + off;
    if (p->periodic) return (q + n) % n;
    if (q < 0) return 1;
    if (q > n - 1) return n - 2;
    return q;
}

static void orc_unflat(const orc_params *p, int64_t l, int c[3]) {
    int n = p->grid_n;
    c[0] = (int)(l % n);
    c[1] = (int)((l / n) % n);
    c[2] = p->dim == 3 ? (int)(l / ((int64_t)n * n)) : 0;
}

static int64_t orc_flat(const orc_params *p, const int c[3]) {
    int64_t n = p->grid_n;
    return c[0] + n * (c[1] + (p->dim == 3 ? n * c[2] : 0));
}

/* Node gradient of c by second-order central differences (the first
 * derivative matrices of Sect. 3.5 with the centred scheme stated there).
 * g is dim x G (component-major). */
void orc_gradient(const orc_params *p, const double *c, double *g) {
    const int64_t G = orc_nodes(p);
    const double h = orc_h(p);
#pragma omp parallel for
    for (int64_t l = 0; l < G; ++l) {
        int ci[3];
        orc_unflat(p, l, ci);
        for (int a = 0; a < p->dim; ++a) {
            int cp[3] = {ci[0], ci[1], ci[2]}, cm[3] = {ci[0], ci[1], ci[2]};
            cp[a] = orc_nbr(p, ci[a], +1);
            cm[a] = orc_nbr(p, ci[a], -1);
            g[a * G + l] = (c[orc_flat(p, cp)] - c[orc_flat(p, cm)]) / (2.0 * h);
        }
    }
}

/* Lower corner index and fractional offset of x along one axis.  Shared by
 * interpolation and deposit (the two are each other's transpose). */
static void orc_cell(const orc_params *p, double x, int *i0, int *i1, double *t) {
    const double h = orc_h(p);
    const int n = p->grid_n;
    double s = x / h;
    int i = (int)floor(s);
    int top = p->periodic ? n - 1 : n - 2;
    if (i > top) i = top;
    if (i < 0) i = 0;
    *i0 = i;
    *t = s - i;
    *i1 = p->periodic ? (i + 1) % n : i + 1;
}

/* Multilinear (bilinear in 2D, trilinear in 3D) interpolation of a node
 * field f at x: the grid-to-particle matching of Sect. 2.3 with linear
 * interpolation. */
static double orc_interp_one(const orc_params *p, const double *f, const double *x) {
    int i0[3] = {0, 0, 0}, i1[3] = {0, 0, 0};
    double t[3] = {0, 0, 0};
    for (int a = 0; a < p->dim; ++a) orc_cell(p, x[a], &i0[a], &i1[a], &t[a]);
    double v = 0.0;
    int ncorner = 1 << p->dim;
    for (int m = 0; m < ncorner; ++m) {
        int c[3] = {0, 0, 0};
        double w = 1.0;
        for (int a = 0; a < p->dim; ++a) {
            int up = (m >> a) & 1;
            c[a] = up ? i1[a] : i0[a];
            w *= up ? t[a] : 1.0 - t[a];
        }
        v += w * f[orc_flat(p, c)];
    }
    return v;
}

void orc_interp(const orc_params *p, const double *f, int64_t n, const double *X, double *out) {
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) out[i] = orc_interp_one(p, f, X + i * p->dim);
}

/* Particle-in-cell deposit with piecewise-linear weights (Sect. 2.3: the
 * delta mass at X_i shared among the 2^dim surrounding nodes in proportion
 * to distance).  S_src gets source_s * W, S_upt gets uptake_s * W. */
void orc_deposit(const orc_params *p, int64_t n, const double *X, const uint8_t *sp,
                 double *S_src, double *S_upt) {
    const int64_t G = orc_nodes(p);
    memset(S_src, 0, sizeof(double) * (size_t)G);
    memset(S_upt, 0, sizeof(double) * (size_t)G);
    for (int64_t i = 0; i < n; ++i) {
        int i0[3] = {0, 0, 0}, i1[3] = {0, 0, 0};
        double t[3] = {0, 0, 0};
        for (int a = 0; a < p->dim; ++a) orc_cell(p, X[i * p->dim + a], &i0[a], &i1[a], &t[a]);
        int ncorner = 1 << p->dim;
        for (int m = 0; m < ncorner; ++m) {
            int c[3] = {0, 0, 0};
            double w = 1.0;
            for (int a = 0; a < p->dim; ++a) {
                int up = (m >> a) & 1;
                c[a] = up ? i1[a] : i0[a];
                w *= up ? t[a] : 1.0 - t[a];
            }
            int64_t l = orc_flat(p, c);
            S_src[l] += p->source[sp[i]] * w;
            S_upt[l] += p->uptake[sp[i]] * w;
        }
    }
}

/* Gaussian kernel density estimate at every node (Sect. 2.3 and the
 * density loop of Sect. 3.5): rho_s(p_l) = sum over agents i of species s
 * within distance kde_radius * eps_s of p_l of
 *   K_eps(p_l - X_i) = (2 pi eps^2)^(-dim/2) exp(-|p_l - X_i|^2 / (2 eps^2)),
 * with the bandwidth eps_s = the species' diameter (the cell size).  Distances
 * are minimum-image on the torus; with walls there is no image (kernel mass
 * beyond a wall is lost, as in the paper's loop).  sigma = sum_s source_s
 * rho_s and upsilon = sum_s uptake_s rho_s are densities (no control
 * volume).  Readings: the 2D kernel of the paper taken to dim dimensions;
 * a per-species bandwidth; the truncation radius is a parameter. */
static void orc_kde_node(const orc_params *p, int64_t n, const double *X, const uint8_t *sp,
                         int64_t l, double *sigma, double *ups) {
    const double h = orc_h(p);
    const double PI = 3.14159265358979323846;
    int ci[3];
    orc_unflat(p, l, ci);
    double s_acc = 0.0, u_acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int s = sp[i];
        const double eps = p->diam[s];
        double r2 = 0.0;
        for (int a = 0; a < p->dim; ++a) {
            double dx = ci[a] * h - X[i * p->dim + a];
            if (p->periodic) dx = orc_min_image(dx, p->L);
            r2 += dx * dx;
        }
        const double R = p->kde_radius * eps;
        if (!(r2 < R * R)) continue;
        const double K = pow(2.0 * PI * eps * eps, -0.5 * p->dim) * exp(-r2 / (2.0 * eps * eps));
        s_acc += p->source[s] * K;
        u_acc += p->uptake[s] * K;
    }
    *sigma = s_acc;
    *ups = u_acc;
}

void orc_deposit_kde(const orc_params *p, int64_t n, const double *X, const uint8_t *sp,
                     double *sigma, double *ups) {
    const int64_t G = orc_nodes(p);
#pragma omp parallel for
    for (int64_t l = 0; l < G; ++l) orc_kde_node(p, n, X, sp, l, &sigma[l], &ups[l]);
}

/* The same densities at m given nodes only (sampled checks of large grids). */
void orc_deposit_kde_at(const orc_params *p, int64_t n, const double *X, const uint8_t *sp,
                        int64_t m, const int64_t *nodes, double *sigma, double *ups) {
#pragma omp parallel for
    for (int64_t k = 0; k < m; ++k) orc_kde_node(p, n, X, sp, nodes[k], &sigma[k], &ups[k]);
}

/* Control volume of node l in units of h^dim: 1, or 1/2 per wall axis. */
static double orc_volume(const orc_params *p, int64_t l) {
    if (p->periodic) return 1.0;
    int c[3];
    orc_unflat(p, l, c);
    double v = 1.0;
    for (int a = 0; a < p->dim; ++a)
        if (c[a] == 0 || c[a] == p->grid_n - 1) v *= 0.5;
    return v;
}

/* One forward-Euler update of eq. pde_c with second-order centred
 * differences (Sect. 3.5), repeated n_sub times with dt' = dt / n_sub:
 *   c <- c + dt' [ D_c Lap_h c + sigma - upsilon * c - gamma c ]
 * sigma = S_src / (h^d v_l) and upsilon = S_upt / (h^d v_l) are the number
 * densities of the deposited measures (eq. random_measure), held fixed over
 * the substeps.  Reading: the printed update matrix I - dt D^2 has the sign
 * of an implicit step while the text states forward Euler; forward Euler
 * with +dt D_c Lap_h is taken. */
void orc_pde_density(const orc_params *p, double *c, const double *sigma, const double *ups);

void orc_pde(const orc_params *p, double *c, const double *S_src, const double *S_upt) {
    const int64_t G = orc_nodes(p);
    const double h = orc_h(p);
    double hd = 1.0;
    for (int a = 0; a < p->dim; ++a) hd *= h;
    double *sigma = (double *)malloc(sizeof(double) * (size_t)G);
    double *ups = (double *)malloc(sizeof(double) * (size_t)G);
    for (int64_t l = 0; l < G; ++l) {
        const double vol = hd * orc_volume(p, l);
        sigma[l] = S_src[l] / vol;
        ups[l] = S_upt[l] / vol;
    }
    orc_pde_density(p, c, sigma, ups);
    free(sigma);
    free(ups);
}

/* The update above with the source and uptake densities given per node. */
void orc_pde_density(const orc_params *p, double *c, const double *sigma_in,
                     const double *ups_in) {
    const int64_t G = orc_nodes(p);
    const double h = orc_h(p);
    const double dts = p->dt / p->n_sub;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)G);
    for (int sub = 0; sub < p->n_sub; ++sub) {
#pragma omp parallel for
        for (int64_t l = 0; l < G; ++l) {
            int ci[3];
            orc_unflat(p, l, ci);
            double lap = 0.0;
            for (int a = 0; a < p->dim; ++a) {
                int cp[3] = {ci[0], ci[1], ci[2]}, cm[3] = {ci[0], ci[1], ci[2]};
                cp[a] = orc_nbr(p, ci[a], +1);
                cm[a] = orc_nbr(p, ci[a], -1);
                lap += (c[orc_flat(p, cp)] - 2.0 * c[l] + c[orc_flat(p, cm)]) / (h * h);
            }
            const double sigma = sigma_in[l], ups = ups_in[l];
            tmp[l] = c[l] + dts * (p->D_c * lap + sigma - ups * c[l] - p->gamma * c[l]);
        }
        memcpy(c, tmp, sizeof(double) * (size_t)G);
    }
    free(tmp);
}

/* Boundary closure of a new position (Sect. 2, periodic or no-flux).
 * Periodic: x - L floor(x/L), and x == L (possible after rounding) -> 0.
 * Walls: one specular reflection (x < 0 -> -x, x > L -> 2L - x, the
 * reflection listing of Sect. 3.2 written for [0, L]), then clamp. */
static double orc_boundary(const orc_params *p, double x) {
    const double L = p->L;
    if (p->periodic) {
        x = x - L * floor(x / L);
        if (x >= L) x -= L;
        return x;
    }
    if (x < 0.0) x = -x;
    else if (x > L) x = 2.0 * L - x;
    if (x < 0.0) x = 0.0;
    if (x > L) x = L;
    return x;
}

/* Pieces of the particle update, exposed for per-stage tests. */
void orc_drift(const orc_params *p, const double *c, int64_t n, const double *X,
               const uint8_t *sp, double *drift) {
    const int64_t G = orc_nodes(p);
    double *g = (double *)malloc(sizeof(double) * (size_t)(G * p->dim));
    orc_gradient(p, c, g);
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) {
        double chi = p->chi[sp[i]] * p->chi_scale;
        for (int a = 0; a < p->dim; ++a)
            drift[i * p->dim + a] = chi == 0.0 ? 0.0 : chi * orc_interp_one(p, g + a * G, X + i * p->dim);
    }
    free(g);
}

/* One time step of the hybrid model in the order of the listings of
 * Sect. 3 (Lie splitting): node gradient of c^n; drift chi grad c at X^n;
 * pair forces at X^n; Euler-Maruyama update (eq. sde_EM, with the drift of
 * eq. sde_beta for chemotactic species) with the species held at the start
 * of the step; type switching; boundary closure; deposit of the new
 * positions with the new types; PDE update of c (eq. pde_c); step + 1.
 * X, sp, c are updated in place; `ids` are the stable agent ids. */
/* Hard-sphere overlap correction (Sect. 2.2): at the updated positions,
 * every pair closer than its contact distance d_ij = (eps_i + eps_j)/2 is
 * pushed apart along the line of centres by twice the penetration
 * d_p = d_ij - r, agent i taking the share D_i / (D_i + D_j) (a pair of
 * immobile agents does not move).  All corrections are computed from the
 * same positions and summed per agent, then the boundary closure is
 * applied again.  Reading: the text's share D_i / (D_i + D_j) is taken; the
 * printed loop divides by the sum of the two species' coefficients, which
 * equals it only for unlike pairs. */
static double orc_boundary(const orc_params *p, double x);

void orc_hs_correct(const orc_params *p, int64_t n, double *X, const uint8_t *sp) {
    const int dim = p->dim;
    double *Y = (double *)malloc(sizeof(double) * (size_t)(n * dim > 0 ? n * dim : 1));
    memcpy(Y, X, sizeof(double) * (size_t)(n * dim));
    orc_bins B;
    int use_bins = p->mode == 1 && n > 0 &&
                   orc_bins_build(&B, dim, p->periodic, p->L, orc_max_cutoff(p), n, Y);
#pragma omp parallel
    {
        orc_list cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            double corr[3] = {0, 0, 0};
            orc_candidates(dim, p->periodic, n, Y, use_bins ? &B : NULL, i, &cand);
            for (int64_t t = 0; t < cand.n; ++t) {
                int64_t j = cand.v[t];
                double dx[3], r2 = 0.0;
                for (int a = 0; a < dim; ++a) {
                    dx[a] = Y[j * dim + a] - Y[i * dim + a];
                    if (p->periodic) dx[a] = orc_min_image(dx[a], p->L);
                    r2 += dx[a] * dx[a];
                }
                const double dij = orc_contact(p, sp[i], sp[j]);
                if (!(r2 < dij * dij)) continue;
                const double r = sqrt(r2), Ds = p->D[sp[i]] + p->D[sp[j]];
                if (!(r > 0.0) || !(Ds > 0.0)) continue;
                const double share = 2.0 * (dij - r) * p->D[sp[i]] / Ds;
                for (int a = 0; a < dim; ++a) corr[a] -= share * dx[a] / r;
            }
            for (int a = 0; a < dim; ++a)
                X[i * dim + a] = orc_boundary(p, Y[i * dim + a] + corr[a]);
        }
        free(cand.v);
    }
    if (use_bins) orc_bins_free(&B);
    free(Y);
}

/* Fixed-step type switching (Sect. 2.1 and the reaction listing of
 * Sect. 3.4): during [t, t + dt) agent i of species s switches to
 * react_to[s] iff zeta < (react_rate[s] + react_rate_c[s] c(X_i)) dt, with
 * zeta the 24-bit uniform of word 0 of the agent's Philox block with
 * counter word 3 = 1 (the switching stream), and c(X_i) the multilinear
 * interpolation of c^n at X^n.  new_sp receives the species after the step. */
void orc_react(const orc_params *p, int64_t n, const double *X, const uint8_t *sp,
               const uint32_t *ids, const double *c, uint32_t step, uint8_t *new_sp) {
    for (int64_t i = 0; i < n; ++i) {
        int s = sp[i];
        new_sp[i] = (uint8_t)s;
        if (p->react_to[s] < 0) continue;
        double rate = p->react_rate[s];
        if (p->react_rate_c[s] != 0.0) rate += p->react_rate_c[s] * orc_interp_one(p, c, X + i * p->dim);
        uint32_t ctr[4] = {step, ids[i], p->inst, 1u};
        uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32) ^ p->inst};
        uint32_t w[4];
        orc_philox(ctr, key, w);
        if (orc_uniform(w[0]) < rate * p->dt) new_sp[i] = (uint8_t)p->react_to[s];
    }
}

void orc_step(const orc_params *p, int64_t n, double *X, uint8_t *sp, const uint32_t *ids,
              double *c, uint32_t *step) {
    const int dim = p->dim;
    const int64_t G = orc_nodes(p);
    double *F = (double *)malloc(sizeof(double) * (size_t)(n * dim > 0 ? n * dim : 1));
    double *drift = (double *)malloc(sizeof(double) * (size_t)(n * dim > 0 ? n * dim : 1));
    uint8_t *nsp = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    orc_forces(p, n, X, sp, F);
    if (p->tamed) {
        /* tamed Euler (eq. sde_ETamed): the pair drift f becomes
         * f / (1 + |f| dt), so its step is below one in length */
        for (int64_t i = 0; i < n; ++i) {
            double nf = 0.0;
            for (int a = 0; a < dim; ++a) nf += F[i * dim + a] * F[i * dim + a];
            nf = sqrt(nf);
            for (int a = 0; a < dim; ++a) F[i * dim + a] /= 1.0 + nf * p->dt;
        }
    }
    orc_drift(p, c, n, X, sp, drift);
    orc_react(p, n, X, sp, ids, c, *step, nsp);
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) {
        double xi[3];
        orc_normals_one(p, *step, ids[i], xi);
        double amp = sqrt(2.0 * p->D[sp[i]] * p->dt);
        for (int a = 0; a < dim; ++a) {
            double x = X[i * dim + a] + p->dt * (F[i * dim + a] + drift[i * dim + a]) + amp * xi[a];
            X[i * dim + a] = orc_boundary(p, x);
        }
    }
    memcpy(sp, nsp, (size_t)n);  /* overlap correction and deposit see the switched types */
    if (p->potential == 2) orc_hs_correct(p, n, X, sp);
    double *Ss = (double *)malloc(sizeof(double) * (size_t)G);
    double *Su = (double *)malloc(sizeof(double) * (size_t)G);
    if (p->deposit_kernel == 1) {
        orc_deposit_kde(p, n, X, sp, Ss, Su);
        orc_pde_density(p, c, Ss, Su);
    } else {
        orc_deposit(p, n, X, sp, Ss, Su);
        orc_pde(p, c, Ss, Su);
    }
    *step += 1;
    free(Ss);
    free(Su);
    free(F);
    free(drift);
    free(nsp);
}

void orc_run(const orc_params *p, int64_t n, double *X, uint8_t *sp, const uint32_t *ids,
             double *c, uint32_t *step, int n_steps) {
    for (int s = 0; s < n_steps; ++s) orc_step(p, n, X, sp, ids, c, step);
}

/* ------------------------------------------------------------------------
 * Density-mismatch loss (used to check the reverse mode).  The paper
 * analyses its runs through histograms of the cell positions (Sect. 4); the
 * loss below uses a smooth version of such a histogram:
 *   rho   = cloud-in-cell histogram of the positions on a periodic grid of
 *           m nodes per axis (spacing L/m, node i at i L/m), divided by n;
 *   rho_s = separable periodic Gaussian smoothing, taps exp(-k^2 / 2 s^2)
 *           for |k| <= round(3 s), normalised to sum 1;
 *   loss  = sum (rho_s - target)^2.
 * grad (n x dim, may be NULL) receives d loss / d X.
 * ------------------------------------------------------------------------ */
static void orc_smooth_axis(int dim, int m, const double *taps, int R, int axis, const double *in,
                            double *out) {
    int64_t H = 1, stride = 1;
    for (int a = 0; a < dim; ++a) H *= m;
    for (int a = 0; a < axis; ++a) stride *= m;
    for (int64_t l = 0; l < H; ++l) {
        int i = (int)((l / stride) % m);
        int64_t base = l - (int64_t)i * stride;
        double s = 0.0;
        for (int q = -R; q <= R; ++q) {
            int ii = ((i + q) % m + m) % m;
            s += taps[q + R] * in[base + (int64_t)ii * stride];
        }
        out[l] = s;
    }
}

double orc_density_loss(int dim, double L, int64_t n, const double *X, int m, double sigma,
                        const double *target, double *grad) {
    int64_t H = 1;
    for (int a = 0; a < dim; ++a) H *= m;
    const double hh = L / m;
    int R = (int)floor(3.0 * sigma + 0.5);
    double *taps = (double *)malloc(sizeof(double) * (size_t)(2 * R + 1));
    double tot = 0.0;
    for (int k = -R; k <= R; ++k) tot += (taps[k + R] = exp(-0.5 * k * k / (sigma * sigma)));
    for (int k = 0; k <= 2 * R; ++k) taps[k] /= tot;
    double *rho = (double *)calloc((size_t)H, sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)H);
    for (int64_t i = 0; i < n; ++i) {
        int i0[3] = {0, 0, 0}, i1[3] = {0, 0, 0};
        double t[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            double s = X[i * dim + a] / hh;
            int c = (int)floor(s);
            if (c > m - 1) c = m - 1;
            if (c < 0) c = 0;
            i0[a] = c;
            t[a] = s - c;
            i1[a] = (c + 1) % m;
        }
        for (int mm = 0; mm < (1 << dim); ++mm) {
            double w = 1.0;
            int64_t idx = 0, stride = 1;
            for (int a = 0; a < dim; ++a) {
                int up = (mm >> a) & 1;
                w *= up ? t[a] : 1.0 - t[a];
                idx += (up ? i1[a] : i0[a]) * stride;
                stride *= m;
            }
            rho[idx] += w / (double)n;
        }
    }
    for (int a = 0; a < dim; ++a) {
        orc_smooth_axis(dim, m, taps, R, a, rho, tmp);
        memcpy(rho, tmp, sizeof(double) * (size_t)H);
    }
    double loss = 0.0;
    for (int64_t l = 0; l < H; ++l) {
        double d = rho[l] - target[l];
        loss += d * d;
        rho[l] = 2.0 * d;  /* reuse as dloss / drho_s */
    }
    if (grad) {
        for (int a = 0; a < dim; ++a) {
            orc_smooth_axis(dim, m, taps, R, a, rho, tmp);
            memcpy(rho, tmp, sizeof(double) * (size_t)H);
        }
        for (int64_t i = 0; i < n; ++i) {
            int i0[3] = {0, 0, 0}, i1[3] = {0, 0, 0};
            double t[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) {
                double s = X[i * dim + a] / hh;
                int c = (int)floor(s);
                if (c > m - 1) c = m - 1;
                if (c < 0) c = 0;
                i0[a] = c;
                t[a] = s - c;
                i1[a] = (c + 1) % m;
            }
            double g[3] = {0, 0, 0};
            for (int mm = 0; mm < (1 << dim); ++mm) {
                double w[3], dw[3];
                int64_t idx = 0, stride = 1;
                for (int a = 0; a < dim; ++a) {
                    int up = (mm >> a) & 1;
                    w[a] = up ? t[a] : 1.0 - t[a];
                    dw[a] = (up ? 1.0 : -1.0) / hh;
                    idx += (up ? i1[a] : i0[a]) * stride;
                    stride *= m;
                }
                for (int b = 0; b < dim; ++b) {
                    double d = dw[b];
                    for (int a = 0; a < dim; ++a)
                        if (a != b) d *= w[a];
                    g[b] += rho[idx] * d;
                }
            }
            for (int b = 0; b < dim; ++b) grad[i * dim + b] = g[b] / (double)n;
        }
    }
    free(taps);
    free(rho);
    free(tmp);
    return loss;
}

/* The smoothed histogram rho_s of the loss above, e.g. to build a target
 * from a reference run (same steps as the loss). */
void orc_density_hist(int dim, double L, int64_t n, const double *X, int m, double sigma,
                      double *out) {
    int64_t H = 1;
    for (int a = 0; a < dim; ++a) H *= m;
    const double hh = L / m;
    int R = (int)floor(3.0 * sigma + 0.5);
    double *taps = (double *)malloc(sizeof(double) * (size_t)(2 * R + 1));
    double tot = 0.0;
    for (int k = -R; k <= R; ++k) tot += (taps[k + R] = exp(-0.5 * k * k / (sigma * sigma)));
    for (int k = 0; k <= 2 * R; ++k) taps[k] /= tot;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)H);
    memset(out, 0, sizeof(double) * (size_t)H);
    for (int64_t i = 0; i < n; ++i) {
        int i0[3] = {0, 0, 0}, i1[3] = {0, 0, 0};
        double t[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            double s = X[i * dim + a] / hh;
            int c = (int)floor(s);
            if (c > m - 1) c = m - 1;
            if (c < 0) c = 0;
            i0[a] = c;
            t[a] = s - c;
            i1[a] = (c + 1) % m;
        }
        for (int mm = 0; mm < (1 << dim); ++mm) {
            double w = 1.0;
            int64_t idx = 0, stride = 1;
            for (int a = 0; a < dim; ++a) {
                int up = (mm >> a) & 1;
                w *= up ? t[a] : 1.0 - t[a];
                idx += (up ? i1[a] : i0[a]) * stride;
                stride *= m;
            }
            out[idx] += w / (double)n;
        }
    }
    for (int a = 0; a < dim; ++a) {
        orc_smooth_axis(dim, m, taps, R, a, out, tmp);
        memcpy(out, tmp, sizeof(double) * (size_t)H);
    }
    free(taps);
    free(tmp);
}

/* Ensemble statistics in the style of the experiment of Sect. 4 (Fig. 1):
 * per-species position histograms over all realisations, hist_n bins per
 * axis on [0, L].  The bin of a coordinate is floor(x * s) clamped to
 * [0, hist_n - 1] with s = float32(hist_n / L), formed in float32 arithmetic
 * on float32 positions (an integer decided by floating point is decided in
 * the precision of the positions).  counts: n_species x hist_n^dim (x
 * fastest); totals: agents of each species. */
void orc_species_hist(int dim, double L, int64_t n, const float *X, const uint8_t *sp,
                      int n_species, int hist_n, uint32_t *counts, uint32_t *totals) {
    int64_t H = 1;
    for (int a = 0; a < dim; ++a) H *= hist_n;
    memset(counts, 0, sizeof(uint32_t) * (size_t)(H * n_species));
    memset(totals, 0, sizeof(uint32_t) * (size_t)n_species);
    const float s = (float)((double)hist_n / L);
    for (int64_t i = 0; i < n; ++i) {
        int64_t idx = 0, stride = 1;
        for (int a = 0; a < dim; ++a) {
            const float v = X[i * dim + a] * s;
            int b = (int)floorf(v);
            if (b < 0) b = 0;
            if (b > hist_n - 1) b = hist_n - 1;
            idx += b * stride;
            stride *= hist_n;
        }
        counts[(int64_t)sp[i] * H + idx] += 1;
        totals[sp[i]] += 1;
    }
}
