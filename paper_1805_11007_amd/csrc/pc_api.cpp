// C ABI of the hybrid chemotaxis step (declared in include/pc.h): parameter
// validation, workspace layout, kernel sequencing, HIP-graph replay and the
// checkpoint / debug entry points.  Device work is enqueued on the caller's
// stream; the library allocates no device memory.
#include <math.h>
#include <cmath>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pc.h"
#include "pc_internal.h"
#include "pc_kde.h"

using namespace pc;

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_OK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(PC_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

namespace {

struct Derived {
    int dim, periodic, ns, ni;
    int64_t n_total;
    int nb, stencil;
    double bin_side, cutoff, h;
    int64_t bins_per_inst, bins_total, nodes_per_inst, nodes_total;
    int n_sub, block, has_uptake, has_react, kde, potential, tamed;
    double kde_radius, pot_range, contact_max;
    uint32_t warn;
    int slab_ok;           // the node slabs of the owner-computes deposit fit
    SlabShape slab;
};

// A species switches when react_to >= 0 and one of its rates is > 0.
// Agents per chemical node below which the deposit skips LDS aggregation.
constexpr double kDepositSparse = 0.2;
// Agents below which it skips it too: the aggregating deposit runs 1024
// agents per work-group and needs about one work-group per compute unit
// (measured: direct atomics are faster on 100k, 50k and 1k agents).
constexpr int64_t kDepositAggMinAgents = 256 * 1024;
// Instances from which a batch whose per-instance deposit sums fit in LDS
// runs deposit + PDE as one work-group per instance.
constexpr int kFusedMinInstances = 64;
// Agents above which a slab of the owner-computes deposit is handed to the
// agent-parallel pass (8 per thread of its 256-thread work-group).
constexpr uint32_t kSlabSplitDefault = 2048;

static bool reacts(const pc_species_t &s) {
    return s.react_to >= 0 && (s.react_rate > 0 || s.react_rate_c > 0);
}

struct Layout {
    size_t P[3], I[3], count, start, tile_sum, tile_cnt, c[2], S_src, S_upt, slab_cnt,
        slab_tab, inst, species_id, step, flags, seg_x, seg_c, lamX[2], lamY, lamC[2], aSrc, aUpt, lamG, csub, dth;
    size_t total;
};

size_t take(size_t &cur, size_t bytes) {
    const size_t o = (cur + 255) & ~(size_t)255;
    cur = o + bytes;
    return o;
}

int derive(const pc_config *cfg, const pc_species_t *sp, int ns, const pc_instance *in, int ni,
           Derived &d) {
    if (!cfg || !sp || !in) return fail(PC_EINVAL, "null argument");
    if (cfg->dim != 2 && cfg->dim != 3) return fail(PC_EINVAL, "dim must be 2 or 3");
    if (!(cfg->L > 0)) return fail(PC_EINVAL, "L must be > 0");
    if (cfg->grid_n < 3) return fail(PC_EINVAL, "grid_n must be >= 3");
    if (!(cfg->dt > 0)) return fail(PC_EINVAL, "dt must be > 0");
    if (!(cfg->k_rep >= 0) || !(cfg->D_c >= 0) || !(cfg->gamma >= 0))
        return fail(PC_EINVAL, "k_rep, D_c and gamma must be >= 0");
    if (ns < 1 || ns > PC_MAX_SPECIES) return fail(PC_EINVAL, "1..8 species supported");
    if (ni < 1 || ni >= (1 << 24)) return fail(PC_EINVAL, "instance count out of range");
    if (cfg->bin_order != 0) return fail(PC_ENOTSUP, "only row-major bin order is built");
    if (cfg->deposit_mode < 0 || cfg->deposit_mode > 4)
        return fail(PC_EINVAL, "deposit_mode must be 0 .. 4");
    if (cfg->slab_split < 0) return fail(PC_EINVAL, "slab_split must be >= 0");
    if (cfg->block != 0 && cfg->block != 64 && cfg->block != 128 && cfg->block != 256 &&
        cfg->block != 512 && cfg->block != 1024)
        return fail(PC_EINVAL, "block must be 0, 64, 128, 256, 512 or 1024");
    d.dim = cfg->dim;
    d.periodic = cfg->periodic ? 1 : 0;
    d.ns = ns;
    d.ni = ni;
    d.cutoff = 0;
    d.has_uptake = 0;
    d.has_react = 0;
    if (cfg->potential < 0 || cfg->potential > 2) return fail(PC_EINVAL, "potential must be 0..2");
    if (cfg->tamed != 0 && cfg->tamed != 1) return fail(PC_EINVAL, "tamed must be 0 or 1");
    if (!(cfg->pot_range >= 0) || !std::isfinite(cfg->pot_range))
        return fail(PC_EINVAL, "pot_range must be finite and >= 0");
    d.potential = cfg->potential;
    d.tamed = cfg->tamed;
    d.pot_range = cfg->pot_range > 0 ? cfg->pot_range : 3.0;
    if (d.potential == 1 && d.pot_range < 1.0)
        return fail(PC_EINVAL, "pot_range must be >= 1 (the neighbour cut is >= the diameter)");
    for (int s = 0; s < ns; ++s) {
        if (!(sp[s].diameter > 0)) return fail(PC_EINVAL, "diameter must be > 0");
        if (!(sp[s].D >= 0)) return fail(PC_EINVAL, "D must be >= 0");
        if (!(sp[s].source >= 0) || !(sp[s].uptake >= 0))
            return fail(PC_EINVAL, "source and uptake must be >= 0");
        if (!(sp[s].react_rate >= 0) || !(sp[s].react_rate_c >= 0) ||
            !std::isfinite(sp[s].react_rate) || !std::isfinite(sp[s].react_rate_c))
            return fail(PC_EINVAL, "switching rates must be finite and >= 0");
        if (reacts(sp[s])) {
            if (sp[s].react_to >= ns) return fail(PC_EINVAL, "react_to >= n_species");
            if (sp[s].react_to == s) return fail(PC_EINVAL, "a species cannot switch to itself");
            d.has_react = 1;
        }
        if (sp[s].diameter > d.cutoff) d.cutoff = sp[s].diameter;
        if (sp[s].uptake > 0) d.has_uptake = 1;
    }
    d.n_total = 0;
    for (int k = 0; k < ni; ++k) {
        if (in[k].n_agents < 1) return fail(PC_EINVAL, "every instance needs >= 1 agent");
        d.n_total += in[k].n_agents;
    }
    if (d.n_total >= (int64_t)1 << 31) return fail(PC_EINVAL, "too many agents");
    d.contact_max = d.cutoff;
    if (d.potential == 1) d.cutoff *= d.pot_range;  // neighbour range of the exponential
    if (d.cutoff >= cfg->L / 2) return fail(PC_EINVAL, "interaction range must be < L/2");
    if (cfg->deposit_kernel != 0 && cfg->deposit_kernel != 1)
        return fail(PC_EINVAL, "deposit_kernel must be 0 or 1");
    d.kde = cfg->deposit_kernel;
    d.kde_radius = cfg->kde_radius > 0 ? cfg->kde_radius : 3.0;
    if (!(cfg->kde_radius >= 0) || !std::isfinite(cfg->kde_radius))
        return fail(PC_EINVAL, "kde_radius must be finite and >= 0");
    if (d.kde) {
        if (cfg->deposit_mode == 3 || cfg->deposit_mode == 4)
            return fail(PC_EINVAL, "deposit_modes 3 and 4 are particle-in-cell paths");
        if (d.kde_radius * d.contact_max >= cfg->L / 2)
            return fail(PC_EINVAL, "kde_radius * diameter must be < L/2");
        if (d.potential == 2)
            return fail(PC_ENOTSUP, "hard spheres with the kernel density deposit are not built");
    }

    // Bins: side >= cutoff (1 + 1e-4) so float32 rounding of the bin index
    // can never separate a pair closer than the cutoff by two bins.  A side
    // >= 2 cutoff allows the 2^dim stencil chosen by the half-bin side.
    const double margin = 1.0 + 1e-4;
    auto bins_for = [&](double side) { return (int)floor(cfg->L / side); };
    int nb;
    if (cfg->bin_size > 0) {
        nb = bins_for(cfg->bin_size);
        if (nb < 3) return fail(PC_EINVAL, "fewer than 3 bins per axis");
        if (cfg->L / nb < d.cutoff * margin)
            return fail(PC_EINVAL, "bin side must exceed the largest diameter");
    } else {
        nb = bins_for(d.cutoff * margin);
        int64_t b3 = 1;
        for (int a = 0; a < d.dim; ++a) b3 *= nb;
        // the 3^dim stencil at side ~cutoff tests the fewest candidates; only
        // when its bin table dwarfs the agents and nodes use side >= 2 cutoff
        int64_t g3 = 1;
        for (int a = 0; a < d.dim; ++a) g3 *= cfg->grid_n;
        if ((int64_t)b3 * ni > 16 * (d.n_total + g3 * ni)) {
            const int nb2 = bins_for(2 * d.cutoff * margin);
            if (nb2 >= 3) nb = nb2;
        }
        if (nb < 3) return fail(PC_EINVAL, "fewer than 3 bins per axis (cutoff too large)");
    }
    d.nb = nb;
    d.bin_side = cfg->L / nb;
    d.stencil = d.bin_side >= 2 * d.cutoff * margin ? 2 : 3;
    d.bins_per_inst = 1;
    for (int a = 0; a < d.dim; ++a) d.bins_per_inst *= nb;
    d.bins_total = d.bins_per_inst * ni;
    if (d.bins_total >= ((int64_t)1 << 31)) return fail(PC_EINVAL, "too many bins");

    d.h = d.periodic ? cfg->L / cfg->grid_n : cfg->L / (cfg->grid_n - 1);
    d.nodes_per_inst = 1;
    for (int a = 0; a < d.dim; ++a) d.nodes_per_inst *= cfg->grid_n;
    d.nodes_total = d.nodes_per_inst * ni;
    if (d.nodes_total >= ((int64_t)1 << 31)) return fail(PC_EINVAL, "too many grid nodes");
    const double r = cfg->D_c * cfg->dt / (d.h * d.h);
    const double lim = 1.0 / (2 * d.dim);
    if (cfg->pde_substeps > 0) {
        d.n_sub = cfg->pde_substeps;
        if (r / d.n_sub > lim) return fail(PC_EUNSTABLE, "D_c dt'/h^2 above 1/(2 dim)");
    } else {
        d.n_sub = (int)ceil(r / (0.9 * lim));
        if (d.n_sub < 1) d.n_sub = 1;
    }
    d.block = cfg->block ? cfg->block : 128;
    d.warn = 0;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            const double dij = 0.5 * (sp[a].diameter + sp[b].diameter);
            if (sqrt(2.0 * (sp[a].D + sp[b].D) * cfg->dt) >= dij) d.warn |= PC_WARN_DT_RULE;
        }
    d.slab_ok = chem_slab_shape(d.dim, cfg->grid_n, d.h / d.bin_side, d.ni, d.slab) ? 1 : 0;
    return PC_OK;
}

Layout layout(const Derived &d, int seg_steps) {
    Layout L;
    memset(&L, 0, sizeof(L));
    size_t cur = 0;
    const size_t N = (size_t)d.n_total;
    for (int k = 0; k < 3; ++k) L.P[k] = take(cur, 16 * N);
    for (int k = 0; k < 3; ++k) L.I[k] = take(cur, 4 * N);
    L.count = take(cur, 4 * ((size_t)d.bins_total + 1));
    L.start = take(cur, 4 * ((size_t)d.bins_total + 1));
    L.tile_sum = take(cur, 4 * (((size_t)d.bins_total + 1 + kScanTile - 1) / kScanTile));
    L.tile_cnt = take(cur, 4 * kTileReps * (((size_t)d.bins_total + kScanTile) / kScanTile));
    L.c[0] = take(cur, 4 * (size_t)d.nodes_total);
    L.c[1] = take(cur, 4 * (size_t)d.nodes_total);
    L.S_src = take(cur, 8 * (size_t)d.nodes_total);
    L.S_upt = take(cur, d.has_uptake ? 8 * (size_t)d.nodes_total : 8);
    if (d.slab_ok) {
        L.slab_cnt = take(cur, 4 * (size_t)d.slab.nslabs);
        L.slab_tab = take(cur, 4 * (size_t)d.slab.nslabs * chem_slab_table_words());
    }
    L.inst = take(cur, sizeof(InstInfo) * (size_t)d.ni);
    L.species_id = take(cur, N);
    L.step = take(cur, 4);
    L.flags = take(cur, 4);
    if (seg_steps > 0) {
        const size_t G = (size_t)d.nodes_total, XD = N * d.dim;
        L.seg_x = take(cur, 4 * ((size_t)seg_steps + 1) * XD);
        L.seg_c = take(cur, 4 * (size_t)seg_steps * G);
        L.lamX[0] = take(cur, 4 * XD);
        L.lamX[1] = take(cur, 4 * XD);
        L.lamY = take(cur, 16 * N);
        L.lamC[0] = take(cur, 4 * G);
        L.lamC[1] = take(cur, 4 * G);
        L.aSrc = take(cur, 4 * G);
        L.aUpt = take(cur, 4 * G);
        L.lamG = take(cur, 4 * G * d.dim);
        L.csub = take(cur, 4 * G * d.n_sub);
        L.dth = take(cur, 8 * 3 * (size_t)d.ni);
    }
    L.total = take(cur, 0) + 256;
    return L;
}

}  // namespace

struct pc_sim {
    Derived d;
    Layout lay;
    pc_config cfg;
    std::vector<pc_species_t> species;
    std::vector<pc_instance> inst_cfg;
    std::vector<InstInfo> inst_host;
    StepParams sp;
    PdeParams pp;
    Buffers b;
    hipStream_t stream;
    hipStream_t cap_stream;
    int device;
    int cur_c;                // which c buffer holds the field
    uint32_t host_step;
    uint32_t warn_bits;
    int use_graph;
    hipGraphExec_t graph[2];  // two-step graphs, by starting field buffer
    int seg_steps;
    uint32_t flags_host;
    // Pipeline state.  A step is: [bin] scan scatter [stable] update deposit pde.
    // binned:  count/bin hold the cell-list counts of the positions in P[0]
    // sorted:  P[sorted_src] / start hold the cell-sorted current positions
    int binned, sorted, sorted_src;
    int chem_fused;           // deposit + PDE in one per-instance kernel (k_chem_inst)
    int slab;                 // owner-computes deposit by node slabs (k_chem_slabs) from
                              // the sorted X^{n+1}: the step sorts after the update
    uint32_t slab_split;      // agents above which a slab is handed to k_slab_assist
};

static void fill_params(pc_sim *s) {
    const Derived &d = s->d;
    const pc_config &c = s->cfg;
    StepParams &p = s->sp;
    memset(&p, 0, sizeof(p));
    p.dim = d.dim;
    p.periodic = d.periodic;
    p.n_species = d.ns;
    p.n_inst = d.ni;
    p.nb = d.nb;
    p.stencil = d.stencil;
    p.bin_order = 0;
    // Row order changes only the float summation order of a lane's forces;
    // deterministic mode keeps the fixed order, so that an agent's bits do
    // not depend on which path its wave takes.
    p.sort_rows = c.deterministic ? 0 : 1;
    p.grid_n = c.grid_n;
    p.n_total = (int32_t)d.n_total;
    p.nodes_per_inst = (int32_t)d.nodes_per_inst;
    p.bins_per_inst = (int32_t)d.bins_per_inst;
    p.has_uptake = d.has_uptake;
    p.L = (float)c.L;
    p.halfL = (float)(0.5 * c.L);
    p.inv_bin = (float)(d.nb / c.L);
    p.bin_w = (float)c.L / (float)d.nb;
    p.h = (float)d.h;
    p.inv_h = (float)(1.0 / d.h);
    p.inv_2h = (float)(0.5 / d.h);
    p.inv_h2 = (float)(1.0 / (d.h * d.h));
    p.dt = (float)c.dt;
    p.k = (float)c.k_rep;
    // Tile totals gathered by the histogram spare the scan a pass over every
    // bin count.  With many tiles each has one counter, used where bins far
    // outnumber agents (else waves would queue on few counters); a grid of
    // few tiles has kTileReps counters per tile, one picked by each wave.
    {
        const int64_t T = (d.bins_total + kScanTile) / kScanTile;
        p.tile_reps = T <= kTileRepsMaxTiles ? kTileReps : 1;
        p.tile_totals = (T <= kTileRepsMaxTiles || d.bins_total + 1 >= 8 * d.n_total) ? 1 : 0;
    }
    // the factor k (d / r - 1) reaches this only for r < 1e-10 d; it keeps
    // the factor finite at r = 0, where it multiplies dx = 0
    p.fcap = (float)std::min(1e10 * c.k_rep * d.contact_max, 1e38);
    p.cell_top = (float)(d.periodic ? c.grid_n - 1 : c.grid_n - 2);
    for (int a = 0; a < d.ns; ++a) {
        for (int b = 0; b < d.ns; ++b) {
            const double m = 0.5 * (s->species[a].diameter + s->species[b].diameter);
            const double range = d.potential == 1 ? d.pot_range * m : m;
            p.cut2[a * d.ns + b] = (float)(range * range);
            p.dij[a * d.ns + b] = (float)m;
            const double Ds = s->species[a].D + s->species[b].D;
            p.hs_share[a * d.ns + b] = Ds > 0 ? (float)(2.0 * s->species[a].D / Ds) : 0.0f;
        }
        p.amp[a] = (float)sqrt(2.0 * s->species[a].D * c.dt);
        p.chi[a] = (float)s->species[a].chi;
        p.src_fx[a] = (float)(s->species[a].source * 4294967296.0);
        p.upt_fx[a] = (float)(s->species[a].uptake * 4294967296.0);
        // probability threshold rate*dt rounded up to float: for a float
        // uniform u, u < float threshold exactly when u < the double product
        const pc_species_t &sa = s->species[a];
        p.react_to[a] = reacts(sa) ? sa.react_to : -1;
        const double pr = sa.react_rate * c.dt;
        float f = (float)pr;
        if ((double)f < pr) f = std::nextafter(f, INFINITY);
        p.react_p[a] = reacts(sa) ? f : 0.0f;
        p.react_cdt[a] = reacts(sa) ? (float)(sa.react_rate_c * c.dt) : 0.0f;
        const double e = sa.diameter, R = d.kde_radius * e;
        p.kde_R2[a] = (float)(R * R);
        p.kde_norm[a] = (float)pow(2.0 * M_PI * e * e, -0.5 * d.dim);
        p.kde_l2e[a] = (float)(1.4426950408889634 / (2.0 * e * e));
        p.src_f[a] = (float)sa.source;
        p.upt_f[a] = (float)sa.uptake;
    }
    p.kde = d.kde;
    // bins scanned around a node: a hair wider than the largest radius, so
    // that float32 rounding of the bin range never drops a candidate
    p.kde_R = (float)(d.kde_radius * d.contact_max * (1.0 + 1e-4));
    p.potential = d.potential;
    p.tamed = d.tamed;
    p.has_react = d.has_react;
    // LDS aggregation pays where a work-group's agents share nodes and the
    // work-groups fill the chip; with fewer agents than kDepositSparse per
    // node most corners are distinct
    p.deposit_agg = c.deposit_mode == 1 ? 1
                    : c.deposit_mode == 2 ? 0
                    : (d.n_total >= kDepositAggMinAgents &&
                               (double)d.n_total >= kDepositSparse * (double)d.nodes_total
                           ? 1
                           : 0);
    PdeParams &q = s->pp;
    memset(&q, 0, sizeof(q));
    q.dim = d.dim;
    q.periodic = d.periodic;
    q.grid_n = c.grid_n;
    q.nodes_per_inst = (int32_t)d.nodes_per_inst;
    q.n_nodes_total = d.nodes_total;
    q.dts = (float)(c.dt / d.n_sub);
    q.D_c = (float)c.D_c;
    q.gamma = (float)c.gamma;
    q.inv_h2 = (float)(1.0 / (d.h * d.h));
    double hd = 1.0;
    for (int a = 0; a < d.dim; ++a) hd *= d.h;
    q.fx_to_density = (float)(1.0 / (4294967296.0 * hd));
    q.inv_hd = (float)(1.0 / hd);
    q.has_uptake = d.has_uptake;
    q.kde = d.kde;
    // the 3D kernel density deposit scatters from the agents into pairs
    // that must start each step at zero (enqueue_kde picks the same path)
    q.kde_clear = d.kde && d.dim == 3 && !c.deterministic ? 1 : 0;
}

static void carve(pc_sim *s, char *ws) {
    const Layout &L = s->lay;
    Buffers &b = s->b;
    memset(&b, 0, sizeof(b));
    for (int k = 0; k < 3; ++k) {
        b.P[k] = (float4 *)(ws + L.P[k]);
        b.I[k] = (uint32_t *)(ws + L.I[k]);
    }
    b.count = (uint32_t *)(ws + L.count);
    b.start = (uint32_t *)(ws + L.start);
    b.tile_sum = (uint32_t *)(ws + L.tile_sum);
    b.tile_cnt = (uint32_t *)(ws + L.tile_cnt);
    b.c[0] = (float *)(ws + L.c[0]);
    b.c[1] = (float *)(ws + L.c[1]);
    b.S_src = (unsigned long long *)(ws + L.S_src);
    b.S_upt = (unsigned long long *)(ws + L.S_upt);
    if (s->d.slab_ok) {
        b.slab_cnt = (uint32_t *)(ws + L.slab_cnt);
        b.slab_tab = (uint32_t *)(ws + L.slab_tab);
    }
    b.inst = (InstInfo *)(ws + L.inst);
    b.species_id = (uint8_t *)(ws + L.species_id);
    b.step = (uint32_t *)(ws + L.step);
    b.flags = (uint32_t *)(ws + L.flags);
    if (s->seg_steps > 0) {
        b.seg_x = (float *)(ws + L.seg_x);
        b.seg_c = (float *)(ws + L.seg_c);
        b.lamX[0] = (float *)(ws + L.lamX[0]);
        b.lamX[1] = (float *)(ws + L.lamX[1]);
        b.lamY = (float4 *)(ws + L.lamY);
        b.lamC[0] = (float *)(ws + L.lamC[0]);
        b.lamC[1] = (float *)(ws + L.lamC[1]);
        b.aSrc = (float *)(ws + L.aSrc);
        b.aUpt = (float *)(ws + L.aUpt);
        b.lamG = (float *)(ws + L.lamG);
        b.csub = (float *)(ws + L.csub);
        b.dth = (double *)(ws + L.dth);
    }
}

// Clear a histogram that no scan consumed: the bin counts and the tile totals.
static void zero_counts(pc_sim *s, hipStream_t st) {
    launch_zero_u32(s->b.count, s->d.bins_total + 1, st);
    launch_zero_u32(s->b.tile_cnt, (int64_t)kTileReps * ((s->d.bins_total + kScanTile) / kScanTile),
                    st);
}

// Cell-sort the current positions (scan of the counts, scatter, optional
// id-stable order) unless already done.
static void ensure_sorted(pc_sim *s, hipStream_t st) {
    if (s->sorted) return;
    const int blk = s->d.block;
    if (!s->binned) launch_bin(s->sp, s->b, 0, blk, st);
    launch_scan(s->sp, s->b, s->d.bins_total, st);
    s->binned = 0;
    launch_scatter(s->sp, s->b, 0, 1, blk, st);
    s->sorted_src = 1;
    if (s->cfg.deterministic) {
        launch_stable(s->sp, s->b, 1, 2, blk, st);
        s->sorted_src = 2;
    }
    s->sorted = 1;
}

// Kernel density deposit from the sorted X^{n+1}.  In 3D the agent-side
// scatter (~17 nodes per agent at radius 3 bandwidths) beats the node-side
// gather, whose lanes idle beside a collapsed cluster: 0.19 vs 0.74 ms on
// 1M agents in 8 blobs.  In 2D a ball holds ~66 nodes per agent and the
// gather wins (0.031 vs 0.22 ms on 100k agents).  Deterministic mode keeps
// the gather, which sums in a fixed order.
static void enqueue_kde(pc_sim *s, hipStream_t st) {
    if (s->d.dim == 3 && !s->cfg.deterministic)
        launch_kde_scatter(s->sp, s->b, s->sorted_src, st);
    else
        launch_kde(s->sp, s->b, s->sorted_src, st);
}

// PDE substeps of a step after the deposit; the last one clears the deposits
// and advances the step counter.
static void enqueue_pde(pc_sim *s, hipStream_t st) {
    for (int k = 0; k < s->d.n_sub; ++k) {
        launch_pde(s->pp, s->b, s->cur_c, 1 - s->cur_c, k == s->d.n_sub - 1 ? 1 : 0, st);
        s->cur_c = 1 - s->cur_c;
    }
}

// Kernel sequence of one step (kernels only, so it can be graph-captured).
static void enqueue_chem(pc_sim *s, hipStream_t st) {
    if (s->chem_fused) {
        launch_chem_inst(s->sp, s->pp, s->b, 0, s->cur_c, s->d.n_sub, st);
        s->cur_c = (s->cur_c + s->d.n_sub) & 1;
    } else {
        launch_deposit(s->sp, s->b, 0, st);
        enqueue_pde(s, st);
    }
}

// Owner-computes deposit by node slabs from the sorted X^{n+1}; with one PDE
// substep the same kernel updates the field (and advances the step counter),
// otherwise it stores the deposits for the substeps.
static void enqueue_slabs(pc_sim *s, hipStream_t st, int classify = 1) {
    const int fuse = s->d.n_sub == 1 ? 1 : 0;
    launch_chem_slabs(s->sp, s->pp, s->b, s->d.slab, s->slab_split, s->sorted_src, s->cur_c,
                      fuse, st, classify);
    if (fuse) s->cur_c = 1 - s->cur_c;
    else enqueue_pde(s, st);
}

static void enqueue_step(pc_sim *s, hipStream_t st) {
    ensure_sorted(s, st);
    launch_update(s->sp, s->b, s->sorted_src, 0, s->cur_c, s->d.block, st);
    if (s->d.potential == 2) {
        // overlaps are found on the cell list of the updated positions; the
        // corrected positions go back to P[0] with their bins counted
        s->binned = 1;
        s->sorted = 0;
        ensure_sorted(s, st);
        launch_overlap(s->sp, s->b, s->sorted_src, 0, s->d.block, st);
        s->binned = 1;
        s->sorted = 0;
    }
    if (s->d.kde) {
        // the density gather needs the cell list of X^{n+1}: sort now, and
        // the next step starts from the sorted state
        s->binned = 1;
        s->sorted = 0;
        ensure_sorted(s, st);
        enqueue_kde(s, st);
        enqueue_pde(s, st);
        return;
    }
    if (s->slab) {
        // the slab deposit gathers through the cell list of X^{n+1}; the
        // scatter's grid also classifies the slabs, which needs only the
        // bin starts of the scan
        const int blk = s->d.block;
        launch_scan(s->sp, s->b, s->d.bins_total, st);
        s->binned = 0;
        launch_scatter_classify(s->sp, s->pp, s->b, s->d.slab, s->slab_split, 0, 1, st);
        s->sorted_src = 1;
        if (s->cfg.deterministic) {
            launch_stable(s->sp, s->b, 1, 2, blk, st);
            s->sorted_src = 2;
        }
        s->sorted = 1;
        enqueue_slabs(s, st, 0);
        return;
    }
    enqueue_chem(s, st);
    s->binned = 1;
    s->sorted = 0;
}

// The state a step leaves: binned (counts of X^{n+1} kept for the next
// step's scan), or sorted already when the deposit gathers per node.
static int is_steady(const pc_sim *s) {
    return (s->d.kde || s->slab) ? (s->sorted && !s->binned) : (s->binned && !s->sorted);
}

static int common_create(const pc_config *cfg, const pc_species_t *species, int n_species,
                         const pc_instance *inst, int n_inst, void *workspace_dev,
                         size_t workspace_bytes, const float *x0_dev, const uint8_t *species0_dev,
                         const float *c0_dev, void *hip_stream, int seg_steps, pc_sim **out) {
    if (!out) return fail(PC_EINVAL, "out is null");
    *out = nullptr;
    Derived d;
    int rc = derive(cfg, species, n_species, inst, n_inst, d);
    if (rc) return rc;
    if (!workspace_dev || !x0_dev || !species0_dev || !c0_dev)
        return fail(PC_EINVAL, "null device pointer");
    if (((uintptr_t)workspace_dev) & 255) return fail(PC_EINVAL, "workspace not 256-byte aligned");
    Layout L = layout(d, seg_steps);
    if (workspace_bytes < L.total)
        return fail(PC_ENOSPACE, "workspace too small: need " + std::to_string(L.total) +
                                     " bytes, got " + std::to_string(workspace_bytes));
    pc_sim *s = new (std::nothrow) pc_sim();
    if (!s) return fail(PC_EINVAL, "host allocation failed");
    s->d = d;
    s->lay = L;
    s->cfg = *cfg;
    s->species.assign(species, species + n_species);
    s->inst_cfg.assign(inst, inst + n_inst);
    s->seg_steps = seg_steps;
    s->stream = (hipStream_t)hip_stream;
    s->cap_stream = nullptr;
    s->graph[0] = s->graph[1] = nullptr;
    s->cur_c = 0;
    s->host_step = 0;
    s->warn_bits = d.warn;
    s->use_graph = 0;
    s->flags_host = 0;
    s->binned = 0;
    s->sorted = 0;
    s->sorted_src = 1;
    (void)hipGetDevice(&s->device);
    fill_params(s);
    {
        int max_lds = 65536;
        if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                  s->device) != hipSuccess)
            max_lds = 65536;
        // dynamic LDS of k_chem_inst plus room for its static species table
        const bool fits = chem_inst_lds_bytes(s->pp) + 4096 <= (size_t)max_lds;
        if (cfg->deposit_mode == 3 && !fits) {
            delete s;
            return fail(PC_EINVAL, "deposit_mode 3: an instance's deposit sums exceed the LDS");
        }
        s->chem_fused = !d.kde && (cfg->deposit_mode == 3 ||
                                   (cfg->deposit_mode == 0 && fits && d.ni >= kFusedMinInstances));
        // the slab deposit: its LDS sums and run table must fit, and the
        // bins per cell must leave a slab few enough runs
        const size_t slab_lds = d.slab_ok ? d.slab.lds_bytes * (d.has_uptake ? 2 : 1) : 0;
        const bool slab_ok = !d.kde && !s->chem_fused && slab_lds > 0 &&
                             slab_lds + 12288 <= (size_t)max_lds;
        if (cfg->deposit_mode == 4 && !slab_ok) {
            delete s;
            return fail(PC_EINVAL, "deposit_mode 4: the node slabs do not fit this grid");
        }
        s->slab = slab_ok && (cfg->deposit_mode == 4 || (cfg->deposit_mode == 0 && d.dim == 3));
        s->slab_split = cfg->slab_split > 0 ? (uint32_t)cfg->slab_split : kSlabSplitDefault;
        if (s->slab) chem_slab_assist_grid(s->sp, s->d.slab);
    }
    carve(s, (char *)workspace_dev);
    s->inst_host.resize(n_inst);
    uint32_t abase = 0;
    for (int k = 0; k < n_inst; ++k) {
        InstInfo &ii = s->inst_host[k];
        ii.agent_base = abase;
        ii.n_agents = (uint32_t)inst[k].n_agents;
        ii.bin_base = (uint32_t)(d.bins_per_inst * k);
        ii.node_base = (uint32_t)(d.nodes_per_inst * k);
        const uint32_t stream = inst[k].stream < 0 ? (uint32_t)k : (uint32_t)inst[k].stream;
        ii.key0 = (uint32_t)inst[k].seed;
        ii.key1 = (uint32_t)(inst[k].seed >> 32) ^ stream;
        ii.chi_scale = (float)inst[k].chi_scale;
        ii.stream = stream;
        abase += (uint32_t)inst[k].n_agents;
    }
    hipStream_t st = s->stream;
    auto bail = [&](int code) {
        delete s;
        return code;
    };
    hipError_t e;
#define CK(x)                                                                                \
    do {                                                                                     \
        e = (x);                                                                             \
        if (e != hipSuccess) {                                                               \
            fail(PC_EHIP, std::string(#x " failed: ") + hipGetErrorString(e));               \
            return bail(PC_EHIP);                                                            \
        }                                                                                    \
    } while (0)
    CK(hipMemcpyAsync(s->b.inst, s->inst_host.data(), sizeof(InstInfo) * n_inst,
                      hipMemcpyHostToDevice, st));
    CK(hipMemsetAsync(s->b.count, 0, 4 * ((size_t)d.bins_total + 1), st));
    CK(hipMemsetAsync(s->b.tile_cnt, 0,
                      4 * kTileReps * (((size_t)d.bins_total + kScanTile) / kScanTile), st));
    CK(hipMemsetAsync(s->b.S_src, 0, 8 * (size_t)d.nodes_total, st));
    if (d.has_uptake) CK(hipMemsetAsync(s->b.S_upt, 0, 8 * (size_t)d.nodes_total, st));
    CK(hipMemsetAsync(s->b.step, 0, 4, st));
    CK(hipMemsetAsync(s->b.flags, 0, 4, st));
    launch_init_agents(s->sp, s->b, x0_dev, species0_dev, 1, st);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(s->b.c[0], c0_dev, 4 * (size_t)d.nodes_total, hipMemcpyDeviceToDevice, st));
    launch_bin(s->sp, s->b, 0, d.block, st);
    s->binned = 1;
    CK(hipStreamSynchronize(st));
    uint32_t fl = 0;
    CK(hipMemcpy(&fl, s->b.flags, 4, hipMemcpyDeviceToHost));
    if (fl & FLAG_BAD_SPECIES) {
        fail(PC_EINVAL, "species index >= n_species in species0");
        return bail(PC_EINVAL);
    }
#undef CK
    *out = s;
    return PC_OK;
}

extern "C" {

size_t pc_workspace_bytes(const pc_config *cfg, const pc_species_t *species, int n_species,
                          const pc_instance *inst, int n_inst) {
    Derived d;
    if (derive(cfg, species, n_species, inst, n_inst, d)) return 0;
    return layout(d, 0).total;
}

size_t pc_workspace_bytes_adjoint(const pc_config *cfg, const pc_species_t *species,
                                  int n_species, const pc_instance *inst, int n_inst,
                                  int seg_steps) {
    Derived d;
    if (seg_steps < 1) return 0;
    if (derive(cfg, species, n_species, inst, n_inst, d)) return 0;
    return layout(d, seg_steps).total;
}

int pc_create(const pc_config *cfg, const pc_species_t *species, int n_species,
              const pc_instance *inst, int n_inst, void *workspace_dev, size_t workspace_bytes,
              const float *x0_dev, const uint8_t *species0_dev, const float *c0_dev,
              void *hip_stream, pc_sim **out) {
    // A workspace sized by pc_workspace_bytes_adjoint enables the adjoint.
    int seg = 0;
    Derived d;
    if (derive(cfg, species, n_species, inst, n_inst, d) == PC_OK) {
        const size_t base = layout(d, 0).total;
        if (workspace_bytes > base) {
            // largest segment length that fits
            int lo = 0, hi = 1 << 16;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (layout(d, mid).total <= workspace_bytes) lo = mid;
                else hi = mid - 1;
            }
            seg = lo;
        }
    }
    return common_create(cfg, species, n_species, inst, n_inst, workspace_dev, workspace_bytes,
                         x0_dev, species0_dev, c0_dev, hip_stream, seg, out);
}

int pc_use_graph(pc_sim *s, int on) {
    if (!s) return fail(PC_EINVAL, "null handle");
    s->use_graph = on ? 1 : 0;
    return PC_OK;
}

static int capture_graph(pc_sim *s, int slot) {
    if (!s->cap_stream) HIP_OK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    const int saved_c = s->cur_c;
    HIP_OK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    enqueue_step(s, s->cap_stream);
    enqueue_step(s, s->cap_stream);
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    // capture runs nothing: a steady step leaves the state flags steady, and
    // two steps flip the field buffer 2 * n_sub times
    s->cur_c = saved_c;
    if (e != hipSuccess) return fail(PC_EHIP, std::string("capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&s->graph[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PC_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
    return PC_OK;
}

int pc_step(pc_sim *s, int n_steps) {
    if (!s) return fail(PC_EINVAL, "null handle");
    if (n_steps < 0) return fail(PC_EINVAL, "n_steps < 0");
    int left = n_steps;
    if (s->use_graph) {
        while (left > 0 && !is_steady(s)) {
            enqueue_step(s, s->stream);
            --left;
            s->host_step += 1;
        }
        if (left >= 2) {
            const int slot = s->cur_c;
            if (!s->graph[slot]) {
                int rc = capture_graph(s, slot);
                if (rc) return rc;
            }
            while (left >= 2) {
                HIP_OK(hipGraphLaunch(s->graph[slot], s->stream));
                left -= 2;
                s->host_step += 2;
            }
        }
    }
    while (left > 0) {
        enqueue_step(s, s->stream);
        --left;
        s->host_step += 1;
    }
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_profile_steps(pc_sim *s, int n_steps, double *stage_ms) {
    if (!s || !stage_ms || n_steps < 1) return fail(PC_EINVAL, "bad argument");
    hipStream_t st = s->stream;
    const int blk = s->d.block;
    // the events are destroyed on every return path
    struct Events {
        hipEvent_t e[2][PC_N_STAGES] = {};
        ~Events() {
            for (auto &row : e)
                for (hipEvent_t ev : row)
                    if (ev) (void)hipEventDestroy(ev);
        }
    } ev;
    hipEvent_t *e0 = ev.e[0], *e1 = ev.e[1];
    for (int k = 0; k < PC_N_STAGES; ++k) {
        HIP_OK(hipEventCreate(&e0[k]));
        HIP_OK(hipEventCreate(&e1[k]));
    }
    double acc[PC_N_STAGES] = {0};
    // with the per-node density gather a step starts sorted; the sort of
    // the initial state belongs to no step
    if (s->d.kde || s->slab) ensure_sorted(s, st);
    for (int t = 0; t < n_steps; ++t) {
        bool ran[PC_N_STAGES] = {false};
#define PC_STAGE(K, BODY)                              \
    do {                                               \
        HIP_OK(hipEventRecord(e0[K], st));             \
        BODY;                                          \
        HIP_OK(hipEventRecord(e1[K], st));             \
        ran[K] = true;                                 \
    } while (0)
        // with_classify: the scatter's grid also classifies the slabs, as
        // in the step (its time is then the scatter's); returns through
        // classified whether it did
        bool classified = false;
        auto sort_stages = [&](bool with_classify = false) -> int {
            classified = false;
            if (s->sorted) return PC_OK;
            if (!s->binned) {
                PC_STAGE(PC_STAGE_BIN, launch_bin(s->sp, s->b, 0, blk, st));
                s->binned = 1;
            }
            PC_STAGE(PC_STAGE_SCAN, launch_scan(s->sp, s->b, s->d.bins_total, st));
            s->binned = 0;
            if (with_classify) {
                PC_STAGE(PC_STAGE_SCATTER,
                         launch_scatter_classify(s->sp, s->pp, s->b, s->d.slab, s->slab_split, 0,
                                                 1, st));
                classified = true;
            } else {
                PC_STAGE(PC_STAGE_SCATTER, launch_scatter(s->sp, s->b, 0, 1, blk, st));
            }
            s->sorted_src = 1;
            if (s->cfg.deterministic) {
                PC_STAGE(PC_STAGE_STABLE, launch_stable(s->sp, s->b, 1, 2, blk, st));
                s->sorted_src = 2;
            }
            s->sorted = 1;
            return PC_OK;
        };
        int rc = sort_stages();
        if (rc) return rc;
        PC_STAGE(PC_STAGE_UPDATE, launch_update(s->sp, s->b, s->sorted_src, 0, s->cur_c, blk, st));
        s->binned = 1;
        s->sorted = 0;
        if (s->d.potential == 2) {
            rc = sort_stages();
            if (rc) return rc;
            PC_STAGE(PC_STAGE_OVERLAP, launch_overlap(s->sp, s->b, s->sorted_src, 0, blk, st));
            s->binned = 1;
            s->sorted = 0;
        }
        if (s->d.kde) {
            rc = sort_stages();
            if (rc) return rc;
            PC_STAGE(PC_STAGE_DEPOSIT, enqueue_kde(s, st));
            PC_STAGE(PC_STAGE_PDE, enqueue_pde(s, st));
        } else if (s->slab) {
            rc = sort_stages(true);
            if (rc) return rc;
            const int cls = classified ? 0 : 1;
            if (s->d.n_sub == 1) {
                // deposit and PDE in one pass: its time is reported under
                // the deposit
                PC_STAGE(PC_STAGE_DEPOSIT, enqueue_slabs(s, st, cls));
            } else {
                PC_STAGE(PC_STAGE_DEPOSIT, launch_chem_slabs(s->sp, s->pp, s->b, s->d.slab,
                                                             s->slab_split, s->sorted_src,
                                                             s->cur_c, 0, st, cls));
                PC_STAGE(PC_STAGE_PDE, enqueue_pde(s, st));
            }
        } else if (s->chem_fused) {
            // one kernel for both: its time is reported under the deposit
            PC_STAGE(PC_STAGE_DEPOSIT, enqueue_chem(s, st));
        } else {
            PC_STAGE(PC_STAGE_DEPOSIT, launch_deposit(s->sp, s->b, 0, st));
            PC_STAGE(PC_STAGE_PDE, enqueue_pde(s, st));
        }
#undef PC_STAGE
        s->host_step += 1;
        HIP_OK(hipStreamSynchronize(st));
        for (int k = 0; k < PC_N_STAGES; ++k) {
            if (!ran[k]) continue;
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, e0[k], e1[k]));
            acc[k] += ms;
        }
    }
    for (int k = 0; k < PC_N_STAGES; ++k) stage_ms[k] = acc[k] / n_steps;
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_positions(pc_sim *s, float *out_dev) {
    if (!s || !out_dev) return fail(PC_EINVAL, "null argument");
    launch_positions(s->sp, s->b, 0, out_dev, s->stream);
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_field(pc_sim *s, float *out_dev) {
    if (!s || !out_dev) return fail(PC_EINVAL, "null argument");
    HIP_OK(hipMemcpyAsync(out_dev, s->b.c[s->cur_c], 4 * (size_t)s->d.nodes_total,
                          hipMemcpyDeviceToDevice, s->stream));
    return PC_OK;
}

int pc_species(pc_sim *s, uint8_t *out_dev) {
    if (!s || !out_dev) return fail(PC_EINVAL, "null argument");
    launch_species(s->sp, s->b, 0, out_dev, s->stream);
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_get_state(pc_sim *s, float *x_dev, float *c_dev, uint32_t *step) {
    if (!s) return fail(PC_EINVAL, "null handle");
    if (x_dev) {
        int rc = pc_positions(s, x_dev);
        if (rc) return rc;
    }
    if (c_dev) {
        int rc = pc_field(s, c_dev);
        if (rc) return rc;
    }
    if (step) *step = s->host_step;
    return PC_OK;
}

int pc_set_state(pc_sim *s, const float *x_dev, const float *c_dev, uint32_t step) {
    if (!s) return fail(PC_EINVAL, "null handle");
    if (x_dev) {
        if (s->binned) zero_counts(s, s->stream);
        launch_init_agents(s->sp, s->b, x_dev, s->b.species_id, 0, s->stream);
        launch_bin(s->sp, s->b, 0, s->d.block, s->stream);
        s->binned = 1;
        s->sorted = 0;
    }
    if (c_dev)
        HIP_OK(hipMemcpyAsync(s->b.c[s->cur_c], c_dev, 4 * (size_t)s->d.nodes_total,
                              hipMemcpyDeviceToDevice, s->stream));
    launch_set_u32(s->b.step, step, s->stream);
    s->host_step = step;
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_set_species(pc_sim *s, const uint8_t *species_dev) {
    if (!s || !species_dev) return fail(PC_EINVAL, "null argument");
    HIP_OK(hipMemcpyAsync(s->b.species_id, species_dev, (size_t)s->d.n_total,
                          hipMemcpyDeviceToDevice, s->stream));
    launch_apply_species(s->sp, s->b, 0, s->b.species_id, s->stream);
    // a sorted copy made before this call holds the old species
    s->sorted = 0;
    HIP_OK(hipGetLastError());
    return PC_OK;
}

static int read_flags(pc_sim *s) {
    HIP_OK(hipStreamSynchronize(s->stream));
    uint32_t fl = 0;
    HIP_OK(hipMemcpy(&fl, s->b.flags, 4, hipMemcpyDeviceToHost));
    s->flags_host |= fl;
    if (fl & FLAG_WARN_POSITIVITY) s->warn_bits |= PC_WARN_POSITIVITY;
    if (fl & FLAG_WARN_CLAMPED) s->warn_bits |= PC_WARN_CLAMPED;
    if (fl & FLAG_WARN_REACTION) s->warn_bits |= PC_WARN_REACTION;
    return PC_OK;
}

int pc_sync(pc_sim *s) {
    if (!s) return fail(PC_EINVAL, "null handle");
    int rc = read_flags(s);
    if (rc) return rc;
    if (s->flags_host & FLAG_NONFINITE) {
        s->flags_host &= ~FLAG_NONFINITE;
        uint32_t zero = 0;
        HIP_OK(hipMemcpy(s->b.flags, &zero, 4, hipMemcpyHostToDevice));
        return fail(PC_ENONFINITE, "a non-finite value reached the state");
    }
    if (s->flags_host & FLAG_BAD_SPECIES) {
        s->flags_host &= ~FLAG_BAD_SPECIES;
        uint32_t zero = 0;
        HIP_OK(hipMemcpy(s->b.flags, &zero, 4, hipMemcpyHostToDevice));
        return fail(PC_EINVAL, "a species index >= n_species was replaced by 0");
    }
    if (s->flags_host & FLAG_INTERNAL) {
        s->flags_host &= ~FLAG_INTERNAL;
        uint32_t zero = 0;
        HIP_OK(hipMemcpy(s->b.flags, &zero, 4, hipMemcpyHostToDevice));
        return fail(PC_EHIP, "internal: a kernel's bound check failed (deposit slab runs)");
    }
    return PC_OK;
}

int pc_warnings(pc_sim *s, uint32_t *bits) {
    if (!s || !bits) return fail(PC_EINVAL, "null argument");
    int rc = read_flags(s);
    if (rc) return rc;
    *bits = s->warn_bits;
    return PC_OK;
}

int pc_info(pc_sim *s, pc_info_t *info) {
    if (!s || !info) return fail(PC_EINVAL, "null argument");
    info->n_total = (int32_t)s->d.n_total;
    info->n_inst = s->d.ni;
    info->bins_per_axis = s->d.nb;
    info->stencil = s->d.stencil;
    info->n_bins_total = s->d.bins_total;
    info->n_nodes_total = s->d.nodes_total;
    info->pde_substeps = s->d.n_sub;
    info->block = s->d.block;
    info->bin_side = s->d.bin_side;
    info->workspace_bytes = s->lay.total;
    info->deposit_path = s->d.kde ? 4 : s->slab ? 5 : s->chem_fused ? 3 : (s->sp.deposit_agg ? 1 : 2);
    info->reserved = 0;
    return PC_OK;
}

int pc_destroy(pc_sim *s) {
    if (!s) return PC_OK;
    for (int k = 0; k < 2; ++k)
        if (s->graph[k]) (void)hipGraphExecDestroy(s->graph[k]);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    delete s;
    return PC_OK;
}

const char *pc_strerror(int code) {
    switch (code) {
        case PC_OK: return "ok";
        case PC_EINVAL: return "invalid argument";
        case PC_EUNSTABLE: return "explicit PDE step above the stability limit";
        case PC_ENOSPACE: return "workspace too small";
        case PC_EHIP: return "HIP runtime error";
        case PC_ENONFINITE: return "non-finite value in the state";
        case PC_ENOTSUP: return "not supported";
        default: return "unknown error";
    }
}

const char *pc_last_error(void) { return g_err.c_str(); }

int pc_debug_neighbours(pc_sim *s, uint32_t *count_dev, uint64_t *hash_dev) {
    if (!s || !count_dev || !hash_dev) return fail(PC_EINVAL, "null argument");
    ensure_sorted(s, s->stream);
    launch_debug_pairs(s->sp, s->b, s->sorted_src, count_dev, (unsigned long long *)hash_dev, nullptr,
                       s->d.block, s->stream);
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_debug_forces(pc_sim *s, float *F_dev) {
    if (!s || !F_dev) return fail(PC_EINVAL, "null argument");
    ensure_sorted(s, s->stream);
    launch_debug_pairs(s->sp, s->b, s->sorted_src, nullptr, nullptr, F_dev, s->d.block, s->stream);
    HIP_OK(hipGetLastError());
    return PC_OK;
}

// Load positions (id order, device) into P[0] without touching the field.
static void load_positions(pc_sim *s, const float *x, hipStream_t st) {
    if (s->binned) zero_counts(s, st);
    launch_init_agents(s->sp, s->b, x, s->b.species_id, 0, st);
    s->binned = 0;
    s->sorted = 0;
}

int pc_adjoint_segment(pc_sim *s, const float *lamX_in_dev, const float *lamC_in_dev,
                       int n_steps, float *lamX_out_dev, float *lamC_out_dev,
                       double *dtheta_out) {
    if (!s || !lamX_in_dev || !lamC_in_dev || !lamX_out_dev || !lamC_out_dev || !dtheta_out)
        return fail(PC_EINVAL, "null argument");
    if (s->seg_steps < 1) return fail(PC_ENOTSUP, "workspace holds no adjoint segment");
    if (n_steps < 1 || n_steps > s->seg_steps)
        return fail(PC_EINVAL, "n_steps must be in [1, segment capacity]");
    if (s->d.has_react) return fail(PC_ENOTSUP, "reverse mode over type switches is not built");
    if (s->d.kde) return fail(PC_ENOTSUP, "reverse mode of the kernel density deposit is not built");
    if (s->d.potential != 0 || s->d.tamed)
        return fail(PC_ENOTSUP, "reverse mode is built for the untamed harmonic potential only");
    hipStream_t st = s->stream;
    const Buffers &b = s->b;
    const size_t XD = (size_t)s->d.n_total * s->d.dim;
    const int64_t G = s->d.nodes_total;
    const uint32_t t0 = s->host_step;
    const int ns = s->d.n_sub;
    // 1) recompute the forward segment, keeping X^t (t = 0..n) and c^t (t < n)
    for (int t = 0; t < n_steps; ++t) {
        launch_positions(s->sp, b, 0, b.seg_x + t * XD, st);
        HIP_OK(hipMemcpyAsync(b.seg_c + t * G, b.c[s->cur_c], 4 * G, hipMemcpyDeviceToDevice, st));
        enqueue_step(s, st);
        s->host_step += 1;
    }
    launch_positions(s->sp, b, 0, b.seg_x + (size_t)n_steps * XD, st);
    // 2) reverse sweep
    HIP_OK(hipMemcpyAsync(b.lamX[0], lamX_in_dev, 4 * XD, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(b.lamC[0], lamC_in_dev, 4 * G, hipMemcpyDeviceToDevice, st));
    launch_zero_f64(b.dth, 3 * (int64_t)s->d.ni, st);
    int cx = 0, cc = 0;
    for (int t = n_steps - 1; t >= 0; --t) {
        // deposit of X^{t+1}
        load_positions(s, b.seg_x + (size_t)(t + 1) * XD, st);
        launch_deposit(s->sp, b, 0, st);
        // forward PDE substeps from c^t (inputs of the reversed substeps)
        HIP_OK(hipMemcpyAsync(b.csub, b.seg_c + t * G, 4 * G, hipMemcpyDeviceToDevice, st));
        for (int m = 1; m < ns; ++m)
            launch_pde_ptr(s->pp, b.csub + (m - 1) * G, b.csub + m * G, b.S_src, b.S_upt, 0,
                           b.flags, st);
        // reversed substeps: lamC[cc] -> ... -> mu^(0)
        for (int m = ns; m >= 1; --m) {
            launch_adj_pde(s->pp, b.lamC[cc], b.lamC[1 - cc], b.csub + (m - 1) * G, b, b.aSrc,
                           b.aUpt, m == ns ? 1 : 0, m == 1 ? 1 : 0, st);
            cc = 1 - cc;
        }
        // agents at X^t, cell-sorted
        load_positions(s, b.seg_x + (size_t)t * XD, st);
        ensure_sorted(s, st);
        launch_zero_f32(b.lamG, G * s->d.dim, st);
        AdjArgs A;
        A.xnext = b.seg_x + (size_t)(t + 1) * XD;
        A.lamX_in = b.lamX[cx];
        A.aSrc = b.aSrc;
        A.aUpt = b.aUpt;
        A.lamY = b.lamY;
        A.lamX_out = b.lamX[1 - cx];
        A.lamG = b.lamG;
        A.dth = b.dth;
        A.nodes_total = G;
        A.step = t0 + (uint32_t)t;
        launch_adj_agent(s->sp, A, b, s->sorted_src, b.seg_c + t * G, st);
        launch_adj_pair(s->sp, b, s->sorted_src, b.lamY, b.lamX[1 - cx], st);
        launch_adj_grad(s->pp, s->sp.inv_2h, b.lamC[cc], b.lamG, b.lamC[1 - cc], st);
        cc = 1 - cc;
        cx = 1 - cx;
    }
    HIP_OK(hipMemcpyAsync(lamX_out_dev, b.lamX[cx], 4 * XD, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(lamC_out_dev, b.lamC[cc], 4 * G, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(dtheta_out, b.dth, 8 * 3 * (size_t)s->d.ni, hipMemcpyDeviceToHost, st));
    // 3) leave the state as it was at the start of the segment
    int rc = pc_set_state(s, b.seg_x, b.seg_c, t0);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_ensemble_stats(pc_sim *s, int hist_n, uint32_t *counts_dev, uint32_t *totals_dev,
                      float *c_mean_dev) {
    if (!s || !counts_dev || !totals_dev) return fail(PC_EINVAL, "null argument");
    if (hist_n < 1) return fail(PC_EINVAL, "hist_n must be >= 1");
    int64_t H = 1;
    for (int a = 0; a < s->d.dim; ++a) {
        H *= hist_n;
        if (H * s->d.ns >= ((int64_t)1 << 31)) return fail(PC_EINVAL, "hist_n too large");
    }
    const float scale = (float)((double)hist_n / s->cfg.L);
    launch_species_hist(s->sp, s->b, 0, hist_n, scale, counts_dev, totals_dev, s->stream);
    if (c_mean_dev)
        launch_field_mean(s->b.c[s->cur_c], s->d.ni, s->d.nodes_per_inst, c_mean_dev, s->stream);
    HIP_OK(hipGetLastError());
    return PC_OK;
}

size_t pc_density_loss_work_bytes(pc_sim *s, int hist_n) {
    if (!s || hist_n < 2) return 0;
    size_t H = 1;
    for (int a = 0; a < s->d.dim; ++a) H *= (size_t)hist_n;
    const size_t HN = H * (size_t)s->d.ni;
    return 8 * HN + 4 * HN * 2 + 8 * (size_t)s->d.ni + 1024;
}

static int density_common(pc_sim *s, const float *target_dev, int hist_n, double sigma_bins,
                          void *work_dev, size_t work_bytes, double *loss_out, float *dLdX_dev,
                          float *rho_out) {
    if (!s->d.periodic) return fail(PC_ENOTSUP, "the density loss is defined on the torus");
    if (hist_n < 2) return fail(PC_EINVAL, "hist_n must be >= 2");
    const int R = (int)floor(3.0 * sigma_bins + 0.5);
    if (!(sigma_bins > 0) || 2 * R + 1 > 65 || 2 * R + 1 > hist_n)
        return fail(PC_EINVAL, "sigma_bins out of range");
    if (work_bytes < pc_density_loss_work_bytes(s, hist_n) || ((uintptr_t)work_dev & 255))
        return fail(PC_ENOSPACE, "loss work buffer too small or misaligned");
    LossArgs a;
    memset(&a, 0, sizeof(a));
    a.m = hist_n;
    a.dim = s->d.dim;
    a.radius = R;
    a.n_taps = 2 * R + 1;
    a.L = (float)s->cfg.L;
    a.inv_hh = (float)(hist_n / s->cfg.L);
    a.H = 1;
    for (int k = 0; k < a.dim; ++k) a.H *= hist_n;
    double tot = 0.0, w[65];
    for (int k = -R; k <= R; ++k) tot += (w[k + R] = exp(-0.5 * k * k / (sigma_bins * sigma_bins)));
    for (int k = 0; k < a.n_taps; ++k) a.taps[k] = (float)(w[k] / tot);
    const size_t HN = (size_t)a.H * s->d.ni;
    char *wp = (char *)work_dev;
    unsigned long long *hist = (unsigned long long *)wp;
    float *b0 = (float *)(wp + 8 * HN);
    float *b1 = b0 + HN;
    double *loss = (double *)(((uintptr_t)(b1 + HN) + 255) & ~(uintptr_t)255);
    launch_loss(a, s->sp, s->b, s->d.ni, target_dev, hist, b0, b1, loss, dLdX_dev, rho_out,
                s->stream);
    if (loss_out)
        HIP_OK(hipMemcpyAsync(loss_out, loss, 8 * (size_t)s->d.ni, hipMemcpyDeviceToHost,
                              s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    HIP_OK(hipGetLastError());
    return PC_OK;
}

int pc_density_loss(pc_sim *s, const float *target_dev, int hist_n, double sigma_bins,
                    void *work_dev, size_t work_bytes, double *loss_out, float *dLdX_dev) {
    if (!s || !target_dev || !work_dev || !loss_out) return fail(PC_EINVAL, "null argument");
    return density_common(s, target_dev, hist_n, sigma_bins, work_dev, work_bytes, loss_out,
                          dLdX_dev, nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Static scratch of pc_density_loss_noalloc: the loss histogram, two
// smoothing buffers and the per-instance sums in a file-scope device array,
// so that the call needs no caller buffer and allocates nothing.  Each GPU
// holds its own copy for the life of the process; its address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is ever handed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kLossScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

int loss_scratch(int device, void **out) {
    if (device < 0 || device >= kMaxScratchDevices)
        return fail(PC_EINVAL, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = -1;
        HIP_OK(hipGetDevice(&prev));
        if (prev != device) HIP_OK(hipSetDevice(device));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !ptr)
            return fail(PC_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                     hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return PC_OK;
}
}  // namespace

extern "C" {

int pc_density_loss_noalloc(pc_sim *s, const float *target_dev, int hist_n, double sigma_bins,
                            double *loss_out, float *dLdX_dev) {
    if (!s || !target_dev || !loss_out) return fail(PC_EINVAL, "null argument");
    const size_t need = pc_density_loss_work_bytes(s, hist_n);
    if (need == 0) return fail(PC_EINVAL, "hist_n must be >= 2");
    if (need > kLossScratchBytes)
        return fail(PC_ENOSPACE, "n_inst * hist_n^dim exceeds the 4 MiB static loss scratch");
    void *ws = nullptr;
    const int rc = loss_scratch(s->device, &ws);
    if (rc) return rc;
    return density_common(s, target_dev, hist_n, sigma_bins, ws, kLossScratchBytes, loss_out,
                          dLdX_dev, nullptr);
}

int pc_density_hist(pc_sim *s, int hist_n, double sigma_bins, void *work_dev, size_t work_bytes,
                    float *rho_out_dev) {
    if (!s || !work_dev || !rho_out_dev) return fail(PC_EINVAL, "null argument");
    return density_common(s, nullptr, hist_n, sigma_bins, work_dev, work_bytes, nullptr,
                          nullptr, rho_out_dev);
}

}  // extern "C"
