/* Driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host only).  It compiles the oracle's single
 * source file into this program and calls every exported function on small
 * inputs: 2D and 3D, torus and walls, all-pairs and cell-list search, every
 * pair potential, tamed Euler, type switching, both deposits, the loss and
 * the ensemble histograms, plus the edge cases one agent and agents piled
 * on one point and on the walls.  A memory or undefined-behaviour error
 * aborts the run with a sanitizer report; success prints "ok". */
#include "../../oracle/oracle.c"

#include <stdio.h>

static uint64_t rng_state = 12345;
static double urand(void) {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static orc_params base_params(int dim, int periodic, int grid_n) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.dim = dim;
    p.periodic = periodic;
    p.L = 1.0;
    p.grid_n = grid_n;
    p.n_sub = 2;
    p.dt = 1e-5;
    p.k = 100.0;
    p.D_c = 1.0;
    p.gamma = 0.1;
    p.n_species = 2;
    p.mode = 1;
    for (int s = 0; s < ORC_MAX_SPECIES; ++s) p.react_to[s] = -1;
    p.diam[0] = 0.03; p.D[0] = 1.0; p.chi[0] = 0.0; p.source[0] = 1.0; p.uptake[0] = 0.0;
    p.diam[1] = 0.05; p.D[1] = 0.5; p.chi[1] = 2.0; p.source[1] = 0.0; p.uptake[1] = 1.0;
    p.react_to[0] = 1;
    p.react_rate[0] = 50.0;
    p.react_to[1] = 0;
    p.react_rate_c[1] = 20.0;
    p.seed = 0x123456789abcdefull;
    p.inst = 3;
    p.chi_scale = 1.0;
    p.kde_radius = 3.0;
    p.pot_range = 3.0;
    return p;
}

static void fill_state(const orc_params *p, int64_t n, double *X, uint8_t *sp, uint32_t *ids,
                       double *c, int pile) {
    const int64_t G = orc_nodes(p);
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < p->dim; ++a) {
            double x = urand();
            if (pile == 1 && i % 3 == 0) x = 0.5;            /* coincident agents */
            if (pile == 2 && i % 4 == 0) x = (i % 8) ? 0.0 : 1.0;  /* on the walls */
            if (p->periodic && x >= 1.0) x = 0.0;
            X[i * p->dim + a] = x;
        }
        sp[i] = (uint8_t)(i % 2);
        ids[i] = (uint32_t)i;
    }
    for (int64_t l = 0; l < G; ++l) c[l] = 1.0 + urand();
}

static void exercise(int dim, int periodic, int grid_n, int64_t n, int mode, int potential,
                     int tamed, int kde, int pile) {
    orc_params p = base_params(dim, periodic, grid_n);
    p.mode = mode;
    p.potential = potential;
    p.tamed = tamed;
    p.deposit_kernel = kde;
    const int64_t G = orc_nodes(&p);
    const int64_t nd = n * dim > 0 ? n * dim : 1;
    double *X = calloc((size_t)nd, sizeof(double));
    double *F = calloc((size_t)nd, sizeof(double));
    double *D = calloc((size_t)nd, sizeof(double));
    double *xi = calloc((size_t)(n > 0 ? 3 * n : 1), sizeof(double));
    uint8_t *sp = calloc((size_t)(n > 0 ? n : 1), 1);
    uint8_t *nsp = calloc((size_t)(n > 0 ? n : 1), 1);
    uint32_t *ids = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    double *c = calloc((size_t)G, sizeof(double));
    double *g = calloc((size_t)(G * dim), sizeof(double));
    double *Ss = calloc((size_t)G, sizeof(double));
    double *Su = calloc((size_t)G, sizeof(double));
    fill_state(&p, n, X, sp, ids, c, pile);

    orc_normals(&p, 7, n, ids, xi);
    orc_forces(&p, n, X, sp, F);
    int64_t which[3] = {0, n / 2, n - 1};
    double F3[9];
    if (n > 0) orc_forces_subset(&p, n, X, sp, 3, which, F3);
    orc_gradient(&p, c, g);
    orc_interp(&p, c, n, X, D);
    orc_drift(&p, c, n, X, sp, D);
    orc_deposit(&p, n, X, sp, Ss, Su);
    orc_pde(&p, c, Ss, Su);
    orc_deposit_kde(&p, n, X, sp, Ss, Su);
    int64_t nodes[2] = {0, G - 1};
    double s2[2], u2[2];
    orc_deposit_kde_at(&p, n, X, sp, 2, nodes, s2, u2);
    orc_pde_density(&p, c, Ss, Su);
    orc_react(&p, n, X, sp, ids, c, 3, nsp);
    double *Y = calloc((size_t)nd, sizeof(double));
    memcpy(Y, X, sizeof(double) * (size_t)nd);
    orc_hs_correct(&p, n, Y, sp);
    free(Y);

    float *Xf = calloc((size_t)nd, sizeof(float));
    for (int64_t t = 0; t < n * dim; ++t) Xf[t] = (float)X[t];
    float cut2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const double m = 0.5 * (p.diam[a] + p.diam[b]);
            cut2[a * 2 + b] = (float)(m * m);
        }
    uint32_t *cnt = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    uint64_t *hs = calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    orc_neighbours_f32(dim, periodic, 1.0f, n, Xf, sp, ids, cut2, 2, mode, cnt, hs);
    uint32_t counts[2 * 7 * 7 * 7], totals[2];
    orc_species_hist(dim, 1.0, n, Xf, sp, 2, 7, counts, totals);

    uint32_t step = 0;
    orc_step(&p, n, X, sp, ids, c, &step);
    orc_run(&p, n, X, sp, ids, c, &step, 3);

    if (periodic) {
        const int m = 16;
        int64_t H = 1;
        for (int a = 0; a < dim; ++a) H *= m;
        double *tgt = calloc((size_t)H, sizeof(double));
        double *rho = calloc((size_t)H, sizeof(double));
        double *grad = calloc((size_t)nd, sizeof(double));
        for (int64_t l = 0; l < H; ++l) tgt[l] = urand() / (double)H;
        (void)orc_density_loss(dim, 1.0, n, X, m, 2.0, tgt, grad);
        (void)orc_density_loss(dim, 1.0, n, X, m, 1.5, tgt, NULL);
        orc_density_hist(dim, 1.0, n, X, m, 2.0, rho);
        free(tgt);
        free(rho);
        free(grad);
    }
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, w[4];
    orc_philox(ctr, key, w);
    orc_philox_batch(1, ctr, key, w);
    (void)orc_hash_id(42);

    free(X); free(F); free(D); free(xi); free(sp); free(nsp); free(ids); free(c); free(g);
    free(Ss); free(Su); free(Xf); free(cnt); free(hs);
}

int main(void) {
    for (int dim = 2; dim <= 3; ++dim)
        for (int periodic = 0; periodic <= 1; ++periodic)
            for (int mode = 0; mode <= 1; ++mode) {
                const int gn = dim == 2 ? 17 : 9;
                exercise(dim, periodic, gn, 300, mode, 0, 0, 0, 0);
                exercise(dim, periodic, gn, 300, mode, 1, 1, 1, 0);
                exercise(dim, periodic, gn, 200, mode, 2, 0, 0, 1);
                exercise(dim, periodic, gn, 200, mode, 0, 1, 1, 2);
                exercise(dim, periodic, 3, 1, mode, 0, 0, 0, 0);
                exercise(dim, periodic, 4, 2, mode, 2, 0, 1, 1);
            }
    printf("ok\n");
    return 0;
}
